// dk_theta.hip -- level kernel of eq. (FullyDiscreteDK) with an implicit weight b0 > 0.
//
// One step solves (I - tau b0/2 Lap_h) rho^m = (I + tau b1/2 Lap_h) rho^{m-1} + noise term
// (b1 = 1 - b0).  Writing d for the increment of the explicit scheme (b0 = 0), the same step is
// rho^m = rho^{m-1} + S d with S = (I - tau b0/2 Lap_h)^{-1}: the right-hand side minus
// (I - tau b0/2 Lap_h) rho^{m-1} is exactly d.  So a step computes d with the per-cell arithmetic
// of the other kernels, filters it with S -- diagonal in the discrete Fourier basis, with
// eigenvalue 1 / (1 + 2 b0 mu (sin^2(pi kx/n) + sin^2(pi ky/n))) from a host table -- and adds
// the filtered increment with the compensated sum of the FP32 kernels (FP64: plain sum).
// Pairs are NN-coupled (Sec. 3.2): the coarse grid takes the same scheme every 4 fine steps
// with the restricted noise (the sum over the 2 x 2 block and the 4 steps, kept in registers
// by the thread that owns the block, in state precision).
//
// Layout: one block per sample (blocks stride over the batch), n <= 64.  LDS holds the state,
// one direction of the step's normals (binary32, exact) and a complex work array.  The 2-D
// transform runs one row (or column) per group of n lanes with the butterflies across lanes by
// shuffles: rows forward, then per column the forward transform, the multiplier and the inverse
// without leaving registers, then rows inverse -- four barriers per filter.  Decimation in time
// from bit-reversed input for the forward transforms and in frequency to bit-reversed output
// for the inverse ones, so each pass reads or writes its own row or column in permuted order
// and no separate reordering is needed.  The coarse step reuses the work array (its transform
// and its restricted noise sums use disjoint parts of it).  A thread owns 2 x 2 cell blocks (two
// generator calls per step).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "dk_rng.h"
#include "dk_theta.h"

namespace dk {

namespace {
template <int N>
struct TG {
    static constexpr int NC = N / 2;
    static constexpr int NB = NC * NC;                                // 2 x 2 blocks
    static constexpr int THREADS = N >= 64 ? 512 : (N >= 32 ? 256 : 64);
    static constexpr int SLOTS = (NB + THREADS - 1) / THREADS;
};

template <typename Real>
__device__ __forceinline__ Real tpsq(Real x) { return sqrt(x > Real(0) ? x : Real(0)); }

template <typename V>
__device__ __forceinline__ int t_after(int t, V v)
{
    asm volatile("" : "+v"(t) : "v"(v));
    return t;
}

__device__ __forceinline__ double t_wave_sum(double v)
{
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Radix-2 transform of M points held one per lane, in groups of M lanes (M <= 64), butterflies
// across lanes by shuffles.  Forward: decimation in time, input in bit-reversed order, output in
// natural order.  Inverse (unnormalised, conjugate twiddles): decimation in frequency, input in
// natural order, output in bit-reversed order.  l is the lane's index in its group;
// tw[k] = exp(-2 pi i k / NT), k < NT/2, M <= NT.
template <typename Real, int M, int NT, bool INVERSE>
__device__ __forceinline__ void lane_fft(Real& xr, Real& xi, int l, const Real* tw)
{
#pragma clang fp contract(off)
    if constexpr (!INVERSE) {
#pragma unroll
        for (int h = 1; h < M; h <<= 1) {
            const Real pr = __shfl_xor(xr, h, 64), pi = __shfl_xor(xi, h, 64);
            const int k = (l & (h - 1)) * (NT / (2 * h));
            const Real wr = tw[2 * k], wi = tw[2 * k + 1];
            if ((l & h) == 0) {            // x[i] + w x[i + h]
                xr = xr + (wr * pr - wi * pi);
                xi = xi + (wr * pi + wi * pr);
            } else {                       // x[i] - w x[i + h]
                const Real tr = wr * xr - wi * xi, ti = wr * xi + wi * xr;
                xr = pr - tr;
                xi = pi - ti;
            }
        }
    } else {
#pragma unroll
        for (int h = M / 2; h >= 1; h >>= 1) {
            const Real pr = __shfl_xor(xr, h, 64), pi = __shfl_xor(xi, h, 64);
            const int k = (l & (h - 1)) * (NT / (2 * h));
            const Real wr = tw[2 * k], wi = -tw[2 * k + 1];
            if ((l & h) == 0) {            // u + v
                xr = xr + pr;
                xi = xi + pi;
            } else {                       // (u - v) conj(w)
                const Real dr = pr - xr, di = pi - xi;
                xr = dr * wr - di * wi;
                xi = dr * wi + di * wr;
            }
        }
    }
}

// re <- (1/M^2) F^-1 (sol .* F re) for a real M x M array in LDS (natural order, [y][x]); im is
// scratch.  Rows, then columns (forward transform, the multiplier and the inverse in registers),
// then rows again: four barriers.  Every lane takes part in every shuffle; lanes past the last
// row or column compute on zeros and store nothing.
template <typename Real, int M, int NT, int THREADS>
__device__ void filter2d(Real* re, Real* im, const Real* sol, const Real* tw, int t)
{
#pragma clang fp contract(off)
    constexpr int PER = 64 / M;                       // rows (columns) per wavefront
    constexpr int LOG = __builtin_ctz(M);
    const int lane = t & 63, l = lane & (M - 1), g = lane / M, w = t >> 6;
    const int rl = (int)(__builtin_bitreverse32((uint32_t)l) >> (32 - LOG));
    constexpr int WAVES = THREADS / 64;
    __syncthreads();
    // rows: input at bit-reversed x, output natural kx
    for (int r0 = w * PER; r0 < M; r0 += WAVES * PER) {
        const int row = r0 + g;
        Real xr = row < M ? re[row * M + rl] : Real(0), xi = Real(0);
        lane_fft<Real, M, NT, false>(xr, xi, l, tw);
        if (row < M) { re[row * M + l] = xr; im[row * M + l] = xi; }
    }
    __syncthreads();
    // columns: forward from bit-reversed ky, multiplier, inverse to bit-reversed y
    for (int c0 = w * PER; c0 < M; c0 += WAVES * PER) {
        const int col = c0 + g;
        Real xr = Real(0), xi = Real(0);
        if (col < M) { xr = re[rl * M + col]; xi = im[rl * M + col]; }
        lane_fft<Real, M, NT, false>(xr, xi, l, tw);
        if (col < M) {
            const Real sv = sol[l * M + col];
            xr = xr * sv;
            xi = xi * sv;
        }
        lane_fft<Real, M, NT, true>(xr, xi, l, tw);
        if (col < M) { re[rl * M + col] = xr; im[rl * M + col] = xi; }
    }
    __syncthreads();
    // rows: inverse from natural kx to bit-reversed x; real part, scaled
    for (int r0 = w * PER; r0 < M; r0 += WAVES * PER) {
        const int row = r0 + g;
        Real xr = Real(0), xi = Real(0);
        if (row < M) { xr = re[row * M + l]; xi = im[row * M + l]; }
        lane_fft<Real, M, NT, true>(xr, xi, l, tw);
        if (row < M) re[row * M + rl] = xr * (Real(1) / Real(M * M));
    }
    __syncthreads();
}
}  // namespace

template <typename Real, int N, bool PAIR>
__global__ void __launch_bounds__(TG<N>::THREADS) theta_kernel(const ThetaArgs A)
{
#pragma clang fp contract(off)
    constexpr int THREADS = TG<N>::THREADS, NC = TG<N>::NC, NB = TG<N>::NB, SLOTS = TG<N>::SLOTS;
    constexpr int NN = N * N, NCC = NC * NC;
    constexpr bool KAHAN = sizeof(Real) == 4;
    __shared__ Real rho[NN];
    __shared__ float zr[NN];
    __shared__ Real wre[NN], wim[NN];
    __shared__ Real rhoc[PAIR ? NCC : 1];
    __shared__ double red[THREADS / 64];
    Real* zc0 = wre + NCC;                     // coarse step: restricted sums beside the coarse transform
    Real* zc1 = wre + 2 * NCC;
    const int t = threadIdx.x;
    const Real a = (Real)A.a, kf = (Real)A.kf, kc = (Real)A.kc;
    const Real* r0f = (const Real*)A.rho0_f;
    const Real* r0c = (const Real*)A.rho0_c;
    const Real* tw = (const Real*)A.tw;
    const Real* solf = (const Real*)A.sol_f;
    const Real* solc = (const Real*)A.sol_c;

    for (uint64_t si = blockIdx.x; si < A.count; si += gridDim.x) {
        const NoiseKey key = make_key(A.seed, A.tag, A.level_id, A.first + si);
        Real cmp[SLOTS][4], Z[SLOTS][2], cmpc[SLOTS];
#pragma unroll
        for (int k = 0; k < SLOTS; ++k) {
            const int bq = t + k * THREADS;
            cmp[k][0] = cmp[k][1] = cmp[k][2] = cmp[k][3] = Real(0);
            Z[k][0] = Z[k][1] = Real(0);
            cmpc[k] = Real(0);
            if (bq < NB) {
                const int bx = bq % NC, by = bq / NC;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int c = (2 * by + (q >> 1)) * N + 2 * bx + (q & 1);
                    rho[c] = r0f[c];
                }
                if (PAIR) rhoc[bq] = r0c[bq];
            }
        }
        __syncthreads();

        for (int m = 0; m < A.steps; ++m) {
            int tq = t;
            float z1[SLOTS][4];
            Real dv[SLOTS][4];
            // normals of the 2 x 2 blocks; direction 0 to LDS
#pragma unroll
            for (int k = 0; k < SLOTS; ++k) {
                const int bq = tq + k * THREADS;
                if (bq >= NB) continue;
                const int bx = bq % NC, by = bq / NC;
                float w0[4], w1[4];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    float a0, a1, b0, b1;
                    site_pair_normals(key, (uint32_t)(bx + NC * (2 * by + r)), (uint32_t)m, a0, a1, b0, b1);
                    w0[2 * r] = a0; w1[2 * r] = a1; w0[2 * r + 1] = b0; w1[2 * r + 1] = b1;
                }
                if constexpr (PAIR) {
                    Z[k][0] += ((Real)w0[0] + (Real)w0[1]) + ((Real)w0[2] + (Real)w0[3]);
                    Z[k][1] += ((Real)w1[0] + (Real)w1[1]) + ((Real)w1[2] + (Real)w1[3]);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    zr[(2 * by + (q >> 1)) * N + 2 * bx + (q & 1)] = w0[q];
                    z1[k][q] = w1[q];
                }
                tq = t_after(tq, w1[3]);
            }
            __syncthreads();
            tq = t;
            // x-divergence of sqrt(rho+) z (central difference)
#pragma unroll
            for (int k = 0; k < SLOTS; ++k) {
                const int bq = tq + k * THREADS;
                if (bq >= NB) continue;
                const int bx = bq % NC, by = bq / NC;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int x = 2 * bx + (q & 1), y = 2 * by + (q >> 1), c = y * N + x;
                    const int cl = x == 0 ? c + N - 1 : c - 1, cr = x == N - 1 ? c + 1 - N : c + 1;
                    dv[k][q] = tpsq(rho[cr]) * (Real)zr[cr] - tpsq(rho[cl]) * (Real)zr[cl];
                }
                tq = t_after(tq, dv[k][3]);
            }
            __syncthreads();
            tq = t;
#pragma unroll
            for (int k = 0; k < SLOTS; ++k) {
                const int bq = tq + k * THREADS;
                if (bq >= NB) continue;
                const int bx = bq % NC, by = bq / NC;
#pragma unroll
                for (int q = 0; q < 4; ++q) zr[(2 * by + (q >> 1)) * N + 2 * bx + (q & 1)] = z1[k][q];
            }
            __syncthreads();
            tq = t;
            // the explicit increment d, written to bit-reversed positions of the work array
#pragma unroll
            for (int k = 0; k < SLOTS; ++k) {
                const int bq = tq + k * THREADS;
                if (bq >= NB) continue;
                const int bx = bq % NC, by = bq / NC;
                Real dlast = Real(0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int x = 2 * bx + (q & 1), y = 2 * by + (q >> 1), c = y * N + x;
                    const int cl = x == 0 ? c + N - 1 : c - 1, cr = x == N - 1 ? c + 1 - N : c + 1;
                    const int cu = y == 0 ? c + NN - N : c - N, cd = y == N - 1 ? c + N - NN : c + N;
                    const Real rv = rho[c];
                    const Real dy = tpsq(rho[cd]) * (Real)zr[cd] - tpsq(rho[cu]) * (Real)zr[cu];
                    const Real lap = fma(Real(-4), rv, (rho[cl] + rho[cr]) + (rho[cu] + rho[cd]));
                    const Real d = fma(kf, dv[k][q] + dy, a * lap);
                    wre[c] = d;
                    dlast = d;
                }
                tq = t_after(tq, dlast);
            }
            filter2d<Real, N, N, THREADS>(wre, wim, solf, tw, t);
            // rho += S d (own cells only: every read of rho this step is behind a barrier)
            tq = t;
#pragma unroll
            for (int k = 0; k < SLOTS; ++k) {
                const int bq = tq + k * THREADS;
                if (bq >= NB) continue;
                const int bx = bq % NC, by = bq / NC;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int x = 2 * bx + (q & 1), y = 2 * by + (q >> 1), c = y * N + x;
                    const Real u = wre[c];
                    const Real rv = rho[c];
                    if constexpr (KAHAN) {
                        const Real yk = u - cmp[k][q];
                        const Real tv = rv + yk;
                        cmp[k][q] = (tv - rv) - yk;
                        rho[c] = tv;
                    } else {
                        rho[c] = rv + u;
                    }
                }
            }
            if constexpr (PAIR) {
                if ((m & 3) == 3) {
                    __syncthreads();          // the work array is read above
#pragma unroll
                    for (int k = 0; k < SLOTS; ++k) {
                        const int bq = t + k * THREADS;
                        if (bq < NB) {
                            zc0[bq] = Z[k][0];
                            zc1[bq] = Z[k][1];
                        }
                        Z[k][0] = Z[k][1] = Real(0);
                    }
                    __syncthreads();
#pragma unroll
                    for (int k = 0; k < SLOTS; ++k) {
                        const int c = t + k * THREADS;
                        if (c >= NCC) continue;
                        const int x = c % NC, y = c / NC;
                        const int cl = x == 0 ? c + NC - 1 : c - 1, cr = x == NC - 1 ? c + 1 - NC : c + 1;
                        const int cu = y == 0 ? c + NCC - NC : c - NC, cd = y == NC - 1 ? c + NC - NCC : c + NC;
                        const Real rv = rhoc[c];
                        const Real dx = tpsq(rhoc[cr]) * zc0[cr] - tpsq(rhoc[cl]) * zc0[cl];
                        const Real dy = tpsq(rhoc[cd]) * zc1[cd] - tpsq(rhoc[cu]) * zc1[cu];
                        const Real lap = fma(Real(-4), rv, (rhoc[cl] + rhoc[cr]) + (rhoc[cu] + rhoc[cd]));
                        const Real d = fma(kc, dx + dy, a * lap);
                        wre[c] = d;
                    }
                    filter2d<Real, NC, N, THREADS>(wre, wim, solc, tw, t);
#pragma unroll
                    for (int k = 0; k < SLOTS; ++k) {
                        const int c = t + k * THREADS;
                        if (c >= NCC) continue;
                        const int x = c % NC, y = c / NC;
                        const Real u = wre[c];
                        const Real rv = rhoc[c];
                        if constexpr (KAHAN) {
                            const Real yk = u - cmpc[k];
                            const Real tv = rv + yk;
                            cmpc[k] = (tv - rv) - yk;
                            rhoc[c] = tv;
                        } else {
                            rhoc[c] = rv + u;
                        }
                    }
                }
            }
            __syncthreads();
        }

        // observables of eq. (eqn_MLMCLevels): FP64 inner products, ordered block reduction
        for (int j = 0; j < A.n_obs; ++j) {
            for (int slot = 0; slot < (PAIR ? 2 : 1); ++slot) {
                double acc = 0.0;
                if (slot == 0) {
                    const double* ph = A.phi_f + (size_t)j * NN;
                    for (int c = t; c < NN; c += THREADS) acc = fma((double)rho[c], ph[c], acc);
                } else {
                    const double* ph = A.phi_c + (size_t)j * NCC;
                    for (int c = t; c < NCC; c += THREADS) acc = fma((double)rhoc[c], ph[c], acc);
                }
                acc = t_wave_sum(acc);
                if ((t & 63) == 0) red[t >> 6] = acc;
                __syncthreads();
                if (t == 0) {
                    double L = 0.0;
                    for (int w = 0; w < THREADS / 64; ++w) L += red[w];
                    const double* ob = (slot == 0 ? A.obs_f : A.obs_c) + 3 * j;
                    const double X = ob[0] * ((slot == 0 ? A.h2f : A.h2c) * L - ob[1]);
                    A.out[(si * A.n_obs + j) * 2 + slot] = ob[2] != 0.0 ? X * X : X;
                    if (!PAIR) A.out[(si * A.n_obs + j) * 2 + 1] = 0.0;
                }
                __syncthreads();
            }
        }
    }
}

bool theta_supported(int n, bool pair) { return (n == 4 && !pair) || n == 8 || n == 16 || n == 32 || n == 64; }

int theta_grid(int n, int precision, uint64_t count)
{
    const size_t e = precision == DK_PREC_F64 ? 8 : 4;
    const size_t lds = (size_t)n * n * (3 * e + 4) + (size_t)(n / 2) * (n / 2) * e + 64;
    const int threads = n >= 64 ? 512 : (n >= 32 ? 256 : 64);
    const size_t per_cu = std::max<size_t>(1, std::min<size_t>((160u * 1024u) / lds, 2048u / threads));
    const uint64_t cap = 256ull * per_cu * 4ull;
    return (int)std::max<uint64_t>(1, std::min<uint64_t>(count, cap));
}

template <typename Real, bool PAIR>
static hipError_t launch_n(const ThetaArgs& A, int grid, hipStream_t s)
{
    switch (A.n) {
    case 4: if constexpr (!PAIR) { hipLaunchKernelGGL((theta_kernel<Real, 4, false>), dim3(grid), dim3(TG<4>::THREADS), 0, s, A); break; } return hipErrorInvalidValue;
    case 8: hipLaunchKernelGGL((theta_kernel<Real, 8, PAIR>), dim3(grid), dim3(TG<8>::THREADS), 0, s, A); break;
    case 16: hipLaunchKernelGGL((theta_kernel<Real, 16, PAIR>), dim3(grid), dim3(TG<16>::THREADS), 0, s, A); break;
    case 32: hipLaunchKernelGGL((theta_kernel<Real, 32, PAIR>), dim3(grid), dim3(TG<32>::THREADS), 0, s, A); break;
    case 64: hipLaunchKernelGGL((theta_kernel<Real, 64, PAIR>), dim3(grid), dim3(TG<64>::THREADS), 0, s, A); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_theta(const ThetaArgs& A, int precision, bool pair, int grid, hipStream_t s)
{
    if (!theta_supported(A.n, pair) || grid < 1 || (pair && A.steps % 4 != 0) || !A.tw || !A.sol_f || (pair && !A.sol_c))
        return hipErrorInvalidValue;
    if (precision == DK_PREC_F64) return pair ? launch_n<double, true>(A, grid, s) : launch_n<double, false>(A, grid, s);
    return pair ? launch_n<float, true>(A, grid, s) : launch_n<float, false>(A, grid, s);
}

}  // namespace dk
