// dk_fourier.hip -- level kernel of the Fourier coupling (Sec. 3.1): h_{l-1} = 3 h_l and
// tau_{l-1} = 9 tau_l, grids n_l = n_0 3^l up to 108 x 108.
//
// The fine level runs the scheme of eq. (FullyDiscreteDK) with the nodal noise of every other
// level (the same generator and counters): in the orthonormal Fourier basis of the grid
// functions its coefficients are exactly the family of complex Brownian increments of
// Sec. 3.1.  The coarse level reuses the coefficients of the frequencies it resolves, summed
// over its 9 fine steps; in real space that is the fine normals summed over the coarse step,
// projected onto the coarse frequencies and read at the coarse nodes, i.e. the separable map
// S -> K S K^T with the [nc][nf] kernel K built on the host (a sum of cosines; on the coarse
// Nyquist frequency the two fine aliases enter with weight 2^{-1/2} each, which makes the
// coarse noise real with the coarse level's own law).  The projected sums have unit variance
// per coarse node, so the coarse noise coefficient is kc = kf h_f / h_c.
//
// Layout: one block per sample (blocks stride over the batch).  The fine state lives in LDS
// (state type), with one direction of the step's normals beside it (binary32: the normals
// are binary32 values, so this loses nothing); a thread owns horizontal site pairs (one
// generator call each) and keeps their compensation terms and, for pairs, their running
// noise sums in registers.  A fine step is: normals -> x-divergence -> y normals ->
// y-divergence, Laplacian and update -> store, with a barrier between phases.  At the end of
// each coarse step the sums go to a per-block scratch area (L2), K is applied along x and
// then along y, and the coarse step runs on the coarse state in LDS with the projected sums
// in the normals' LDS area.  FP32 states use the compensated increment of the other kernels;
// FP64 states add the increment directly.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "dk_fourier.h"
#include "dk_rng.h"

namespace dk {

namespace {
template <int NF>
struct FG {
    static constexpr int NC = NF / 3;
    static constexpr int THREADS = NF >= 108 ? 1024 : (NF >= 72 ? 512 : (NF >= 36 ? 256 : (NF >= 24 ? 128 : 64)));
    static constexpr int NPR = NF / 2;            // site pairs per row
    static constexpr int NPAIRS = NF * NF / 2;
    static constexpr int SLOTS = (NPAIRS + THREADS - 1) / THREADS;
    static constexpr int NCC = NC * NC;
    static constexpr int CSLOTS = (NCC + THREADS - 1) / THREADS;
};

template <typename Real>
__device__ __forceinline__ Real psqr(Real x) { return sqrt(x > Real(0) ? x : Real(0)); }

// t, made to depend on v: the next slot's addresses (and loads) wait for this slot's result,
// so the compiler does not issue the loads of every slot at once and run out of registers
template <typename V>
__device__ __forceinline__ int after(int t, V v)
{
    asm volatile("" : "+v"(t) : "v"(v));
    return t;
}

template <int THREADS>
__device__ __forceinline__ int opaque_tid(int t)
{
    asm volatile("" : "+v"(t));
    __builtin_assume(t >= 0 && t < THREADS);
    return t;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
}  // namespace

template <typename Real, int NF, bool PAIR>
__global__ void __launch_bounds__(FG<NF>::THREADS) fourier_kernel(const FourierArgs A)
{
#pragma clang fp contract(off)
    constexpr int THREADS = FG<NF>::THREADS, NPAIRS = FG<NF>::NPAIRS, SLOTS = FG<NF>::SLOTS;
    constexpr int NC = FG<NF>::NC, NCC = FG<NF>::NCC, CSLOTS = FG<NF>::CSLOTS;
    constexpr bool KAHAN = sizeof(Real) == 4;
    constexpr int NN = NF * NF;
    static_assert(!PAIR || (NF % 3 == 0 && NC % 2 == 0), "pairs need n = 3 n_c with n_c even");
    static_assert(!PAIR || 2 * NCC * sizeof(Real) <= NN * sizeof(float), "projected sums must fit the normals' area");
    __shared__ Real rho[NN];
    __shared__ float zr[NN];                       // one direction of the normals; coarse step: Real zc[2][NCC]
    __shared__ Real rhoc[PAIR ? NCC : 1];
    __shared__ double red[THREADS / 64];
    Real* zc = reinterpret_cast<Real*>(zr);
    const int t = threadIdx.x;
    auto opaque = [](int v) { return opaque_tid<THREADS>(v); };
    const Real a = (Real)A.a, kf = (Real)A.kf, kc = (Real)A.kc;
    const Real* r0f = (const Real*)A.rho0_f;
    const Real* r0c = (const Real*)A.rho0_c;
    const Real* K = (const Real*)A.K;
    Real* gS = PAIR ? (Real*)A.scratch + (size_t)blockIdx.x * (2 * NN + 2 * NF * NC) : nullptr;
    Real* gT = PAIR ? gS + 2 * NN : nullptr;

    for (uint64_t si = blockIdx.x; si < A.count; si += gridDim.x) {
        const NoiseKey key = make_key(A.seed, A.tag, A.level_id, A.first + si);
        Real cmp[SLOTS][2], S[SLOTS][4], cmpc[CSLOTS];
#pragma unroll
        for (int k = 0; k < SLOTS; ++k) {
            const int p = t + k * THREADS;
            cmp[k][0] = cmp[k][1] = Real(0);
            S[k][0] = S[k][1] = S[k][2] = S[k][3] = Real(0);
            if (p < NPAIRS) {
                rho[2 * p] = r0f[2 * p];
                rho[2 * p + 1] = r0f[2 * p + 1];
            }
        }
        if constexpr (PAIR) {
#pragma unroll
            for (int k = 0; k < CSLOTS; ++k) {
                const int c = t + k * THREADS;
                cmpc[k] = Real(0);
                if (c < NCC) rhoc[c] = r0c[c];
            }
        }
        __syncthreads();

        for (int m = 0; m < A.steps; ++m) {
            // the thread index is made opaque in every phase: otherwise the compiler computes the
            // cell and neighbour addresses of all slots once and keeps them in registers across
            // the phases (and the steps)
            int tq = opaque(t);
            float z1[SLOTS][2];
            Real dv[SLOTS][2];
            // normals of the step (site pair p = cells 2p, 2p + 1); direction 0 to LDS
#pragma unroll
            for (int k = 0; k < SLOTS; ++k) {
                const int p = tq + k * THREADS;
                if (p >= NPAIRS) continue;
                float a0, a1, b0, b1;
                site_pair_normals(key, (uint32_t)p, (uint32_t)m, a0, a1, b0, b1);
                zr[2 * p] = a0;
                zr[2 * p + 1] = b0;
                z1[k][0] = a1;
                z1[k][1] = b1;
                if constexpr (PAIR) {
                    S[k][0] += (Real)a0;
                    S[k][1] += (Real)b0;
                    S[k][2] += (Real)a1;
                    S[k][3] += (Real)b1;
                }
                tq = after(tq, b1);     // one generator call at a time
            }
            __syncthreads();
            // x-divergence of sqrt(rho+) z: central difference
            tq = opaque(t);
#pragma unroll
            for (int k = 0; k < SLOTS; ++k) {
                const int p = tq + k * THREADS;
                if (p >= NPAIRS) continue;
                const int c = 2 * p, x = c % NF;
                const int cl = x == 0 ? c + NF - 1 : c - 1;
                const int cr = x + 2 == NF ? c + 2 - NF : c + 2;
                dv[k][0] = psqr(rho[c + 1]) * (Real)zr[c + 1] - psqr(rho[cl]) * (Real)zr[cl];
                dv[k][1] = psqr(rho[cr]) * (Real)zr[cr] - psqr(rho[c]) * (Real)zr[c];
                tq = after(tq, dv[k][1]);
            }
            __syncthreads();
            tq = opaque(t);
#pragma unroll
            for (int k = 0; k < SLOTS; ++k) {
                const int p = tq + k * THREADS;
                if (p >= NPAIRS) continue;
                zr[2 * p] = z1[k][0];
                zr[2 * p + 1] = z1[k][1];
            }
            __syncthreads();
            // y-divergence, Laplacian and the update (new values kept in dv)
            tq = opaque(t);
#pragma unroll
            for (int k = 0; k < SLOTS; ++k) {
                const int p = tq + k * THREADS;
                if (p >= NPAIRS) continue;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int c = 2 * p + q, x = c % NF, y = c / NF;
                    const int cl = x == 0 ? c + NF - 1 : c - 1, cr = x == NF - 1 ? c + 1 - NF : c + 1;
                    const int cu = y == 0 ? c + NN - NF : c - NF, cd = y == NF - 1 ? c + NF - NN : c + NF;
                    const Real rv = rho[c];
                    const Real dy = psqr(rho[cd]) * (Real)zr[cd] - psqr(rho[cu]) * (Real)zr[cu];
                    const Real lap = fma(Real(-4), rv, (rho[cl] + rho[cr]) + (rho[cu] + rho[cd]));
                    const Real d = fma(kf, dv[k][q] + dy, a * lap);
                    if constexpr (KAHAN) {
                        const Real yk = d - cmp[k][q];
                        const Real tv = rv + yk;
                        cmp[k][q] = (tv - rv) - yk;
                        dv[k][q] = tv;
                    } else {
                        dv[k][q] = rv + d;
                    }
                }
                tq = after(tq, dv[k][1]);
            }
            __syncthreads();
            tq = opaque(t);
#pragma unroll
            for (int k = 0; k < SLOTS; ++k) {
                const int p = tq + k * THREADS;
                if (p >= NPAIRS) continue;
                rho[2 * p] = dv[k][0];
                rho[2 * p + 1] = dv[k][1];
            }
            if constexpr (PAIR) {
                if (m % 9 == 8) {
                    // the coarse step: sums of the 9 fine steps -> scratch [r][y][x]
#pragma unroll
                    for (int k = 0; k < SLOTS; ++k) {
                        const int p = tq + k * THREADS;
                        if (p < NPAIRS) {
                            gS[2 * p] = S[k][0];
                            gS[2 * p + 1] = S[k][1];
                            gS[NN + 2 * p] = S[k][2];
                            gS[NN + 2 * p + 1] = S[k][3];
                        }
                        S[k][0] = S[k][1] = S[k][2] = S[k][3] = Real(0);
                    }
                    __syncthreads();
                    // along x: T_r[y][ic] = sum_x K[ic][x] S_r[y][x]
                    for (int o = tq; o < 2 * NF * NC; o += THREADS) {
                        const int r = o / (NF * NC), rem = o - r * NF * NC, y = rem / NC, ic = rem - y * NC;
                        const Real* srow = gS + r * NN + y * NF;
                        const Real* krow = K + ic * NF;
                        Real acc = Real(0);
#pragma unroll 4
                        for (int x = 0; x < NF; ++x) acc = fma(krow[x], srow[x], acc);
                        gT[o] = acc;
                    }
                    __syncthreads();
                    // along y: Zc_r[jc][ic] = sum_y K[jc][y] T_r[y][ic]  (into the normals' LDS area)
                    for (int o = tq; o < 2 * NCC; o += THREADS) {
                        const int r = o / NCC, rem = o - r * NCC, jc = rem / NC, ic = rem - jc * NC;
                        const Real* col = gT + r * NF * NC + ic;
                        const Real* krow = K + jc * NF;
                        Real acc = Real(0);
#pragma unroll 4
                        for (int y = 0; y < NF; ++y) acc = fma(krow[y], col[y * NC], acc);
                        zc[o] = acc;
                    }
                    __syncthreads();
                    Real nvc[CSLOTS];
#pragma unroll
                    for (int k = 0; k < CSLOTS; ++k) {
                        const int c = tq + k * THREADS;
                        nvc[k] = Real(0);
                        if (c >= NCC) continue;
                        const int x = c % NC, y = c / NC;
                        const int cl = x == 0 ? c + NC - 1 : c - 1, cr = x == NC - 1 ? c + 1 - NC : c + 1;
                        const int cu = y == 0 ? c + NCC - NC : c - NC, cd = y == NC - 1 ? c + NC - NCC : c + NC;
                        const Real rv = rhoc[c];
                        const Real dx = psqr(rhoc[cr]) * zc[cr] - psqr(rhoc[cl]) * zc[cl];
                        const Real dy = psqr(rhoc[cd]) * zc[NCC + cd] - psqr(rhoc[cu]) * zc[NCC + cu];
                        const Real lap = fma(Real(-4), rv, (rhoc[cl] + rhoc[cr]) + (rhoc[cu] + rhoc[cd]));
                        const Real d = fma(kc, dx + dy, a * lap);
                        if constexpr (KAHAN) {
                            const Real yk = d - cmpc[k];
                            const Real tv = rv + yk;
                            cmpc[k] = (tv - rv) - yk;
                            nvc[k] = tv;
                        } else {
                            nvc[k] = rv + d;
                        }
                        tq = after(tq, nvc[k]);
                    }
                    __syncthreads();
#pragma unroll
                    for (int k = 0; k < CSLOTS; ++k) {
                        const int c = tq + k * THREADS;
                        if (c < NCC) rhoc[c] = nvc[k];
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
                acc = wave_sum(acc);
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

bool fourier_supported(int nf, bool pair)
{
    switch (nf) {
    case 4: case 8: return !pair;
    case 12: case 24: case 36: case 72: case 108: return true;
    default: return false;
    }
}

template <int NF>
static size_t lds_bytes(int precision)
{
    const size_t e = precision == DK_PREC_F64 ? 8 : 4;
    return NF * NF * (e + 4) + (NF / 3) * (NF / 3) * e + 8 * (FG<NF>::THREADS / 64);
}

int fourier_grid(int nf, int precision, uint64_t count)
{
    int threads = 64;
    size_t lds = 0;
    switch (nf) {
    case 4: threads = FG<4>::THREADS; lds = lds_bytes<4>(precision); break;
    case 8: threads = FG<8>::THREADS; lds = lds_bytes<8>(precision); break;
    case 12: threads = FG<12>::THREADS; lds = lds_bytes<12>(precision); break;
    case 24: threads = FG<24>::THREADS; lds = lds_bytes<24>(precision); break;
    case 36: threads = FG<36>::THREADS; lds = lds_bytes<36>(precision); break;
    case 72: threads = FG<72>::THREADS; lds = lds_bytes<72>(precision); break;
    default: threads = FG<108>::THREADS; lds = lds_bytes<108>(precision); break;
    }
    // resident blocks per CU (160 KB of LDS, 2048 threads), 256 CUs, a few waves of blocks
    const size_t per_cu = std::max<size_t>(1, std::min<size_t>((160u * 1024u) / lds, 2048u / threads));
    const uint64_t cap = 256ull * per_cu * 4ull;
    return (int)std::max<uint64_t>(1, std::min<uint64_t>(count, cap));
}

size_t fourier_scratch_elems(int nf) { return 2 * (size_t)nf * nf + 2 * (size_t)nf * (nf / 3); }

template <typename Real, bool PAIR>
static hipError_t launch_nf(const FourierArgs& A, int grid, hipStream_t s)
{
    switch (A.nf) {
    case 4: if constexpr (!PAIR) { hipLaunchKernelGGL((fourier_kernel<Real, 4, false>), dim3(grid), dim3(FG<4>::THREADS), 0, s, A); break; } return hipErrorInvalidValue;
    case 8: if constexpr (!PAIR) { hipLaunchKernelGGL((fourier_kernel<Real, 8, false>), dim3(grid), dim3(FG<8>::THREADS), 0, s, A); break; } return hipErrorInvalidValue;
    case 12: hipLaunchKernelGGL((fourier_kernel<Real, 12, PAIR>), dim3(grid), dim3(FG<12>::THREADS), 0, s, A); break;
    case 24: hipLaunchKernelGGL((fourier_kernel<Real, 24, PAIR>), dim3(grid), dim3(FG<24>::THREADS), 0, s, A); break;
    case 36: hipLaunchKernelGGL((fourier_kernel<Real, 36, PAIR>), dim3(grid), dim3(FG<36>::THREADS), 0, s, A); break;
    case 72: hipLaunchKernelGGL((fourier_kernel<Real, 72, PAIR>), dim3(grid), dim3(FG<72>::THREADS), 0, s, A); break;
    case 108: hipLaunchKernelGGL((fourier_kernel<Real, 108, PAIR>), dim3(grid), dim3(FG<108>::THREADS), 0, s, A); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fourier(const FourierArgs& A, int precision, bool pair, int grid, hipStream_t s)
{
    if (!fourier_supported(A.nf, pair) || grid < 1 || (pair && (A.steps % 9 != 0 || !A.K || !A.scratch)))
        return hipErrorInvalidValue;
    if (precision == DK_PREC_F64)
        return pair ? launch_nf<double, true>(A, grid, s) : launch_nf<double, false>(A, grid, s);
    return pair ? launch_nf<float, true>(A, grid, s) : launch_nf<float, false>(A, grid, s);
}

}  // namespace dk
