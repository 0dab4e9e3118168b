// dk_level.h -- device building blocks of the resident level kernel, shared by the per-level
// kernel (one launch per batch of one level) and the persistent round kernel (all levels of an
// Algorithm-1 round in one launch).
//
// Resident level kernel (grids up to 128 x 128): every sample (or NN-coupled pair) lives in
// the VGPRs of a group of lanes for its whole time horizon.  A lane owns C consecutive
// columns and R consecutive rows of the fine grid (and the matching (C/2) x (R/2) block of
// the coarse grid, so every fine site of a coarse cell's right-most 2x2 block B-> is local).
// Per fine step:
//   1. the lane draws the normals of its first and last row and publishes those rows'
//      density and y-noise to LDS (the only LDS traffic; double-buffered by step parity, so
//      one barrier per step suffices);
//   2. after the barrier it reads the rows above and below its block;
//   3. it sweeps its rows top to bottom: Philox + Box--Muller for the next row, the x-halo
//      (one column each side) from the neighbouring lanes by ds_bpermute, then the explicit
//      EM update of eq. (FullyDiscreteDK) with b0 = 0, b1 = 1:
//         rho' = rho + (mu/2) (sum of 4 neighbours - 4 rho) + kappa div(sqrt(rho^+) w)
//      where w are the unit normals and kappa = N^{-1/2} h^{-d/2} sigma / (2h) (central) or
//      N^{-1/2} h^{-d/2} sigma / h (staggered), sigma the increment's standard deviation.
//   The fine normals of each coarse cell are summed over its 2x2 block and the 4 fine steps
//   of one coarse step (NN coupling, Sec. 3.2); every 4th fine step the coarse grid takes one
//   EM step with those sums (sigma = 2^{-d/2} sqrt(tau_f)).
// At the final time each lane forms (rho, I_h phi_j) over its cells in FP64, the sample's
// lanes combine them with wavefront shuffles (and LDS across wavefronts), and the first lane
// applies centring, scaling and psi (eq. eqn_MLMCLevels).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "dk_internal.h"
#include "dk_rng.h"

namespace dk {

// ---------------------------------------------------------------------------------------
// Lane exchange
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ float lane_get(int addr, float v)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double lane_get(int addr, double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(b & 0xFFFFFFFFll));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename Real>
__device__ __forceinline__ Real pos_sqrt(Real x) { return x > Real(0) ? sqrt(x) : Real(0); }
// [x]^+ as a signed integer maximum of the bits: a negative binary32 (and -0) has a negative bit
// pattern and becomes +0, a positive one is kept; one instruction, where fmaxf in IEEE mode
// adds a NaN-quieting step (the state is finite, so the two agree)
__device__ __forceinline__ float pos_part_f32(float x) { return __int_as_float(max(__float_as_int(x), 0)); }
template <>
__device__ __forceinline__ float pos_sqrt<float>(float x) { return __builtin_amdgcn_sqrtf(pos_part_f32(x)); }

// ---------------------------------------------------------------------------------------
// Noise sources for one tile step: row(i, w0, w1) yields the unit noise of the tile's row i
// (both directions); it is called exactly once per row and step.
// ---------------------------------------------------------------------------------------
template <typename Real, int R, int C, bool PAIR>
struct FineNoise {
    NoiseKey key;
    uint32_t step;
    uint32_t pair_base;      // site-pair index of the tile's row 0, first column pair
    uint32_t pairs_per_row;  // n / 2
    Real (*Z)[C / 2 > 0 ? C / 2 : 1][2];
    Real (*pend)[C / 2 > 0 ? C / 2 : 1][2];   // row sums waiting for the other row of their coarse cell

    // order in which tile_step draws the rows: 0, R-1, then 1 .. R-2
    static constexpr int gen(int i) { return i == 0 ? 0 : (i == R - 1 ? 1 : i + 1); }

    template <int I>
    __device__ __forceinline__ void row(Real (&w0)[C], Real (&w1)[C])
    {
#pragma unroll
        for (int cp = 0; cp < C / 2; ++cp) {
            float a0, a1, b0, b1;
            uint32_t idx = pair_base + (uint32_t)I * pairs_per_row + cp;
            // The counter word and the parts of Philox's first round that depend only on it are
            // invariant over time steps; hoisting them out of the step loop would keep three
            // words per row live across the whole path.  Recompute them every step instead.
            asm volatile("" : "+v"(idx));
            site_pair_normals(key, idx, step, a0, a1, b0, b1);
            w0[2 * cp] = a0;
            w1[2 * cp] = a1;
            w0[2 * cp + 1] = b0;
            w1[2 * cp + 1] = b1;
            if constexpr (PAIR) {
                // each coarse cell adds (even-row sum + odd-row sum) once per fine step, whatever the
                // order in which the two rows are drawn
                const Real s0 = Real(a0) + Real(b0), s1 = Real(a1) + Real(b1);
                constexpr int partner = (I % 2 == 0) ? I + 1 : I - 1;
                if constexpr (gen(partner) < gen(I)) {
                    constexpr int ev = (I % 2 == 0) ? I : partner;
                    const Real e0 = (I == ev) ? s0 : pend[partner][cp][0];
                    const Real e1 = (I == ev) ? s1 : pend[partner][cp][1];
                    const Real o0 = (I == ev) ? pend[partner][cp][0] : s0;
                    const Real o1 = (I == ev) ? pend[partner][cp][1] : s1;
                    Z[I / 2][cp][0] += e0 + o0;
                    Z[I / 2][cp][1] += e1 + o1;
                } else {
                    pend[I][cp][0] = s0;
                    pend[I][cp][1] = s1;
                }
            }
        }
    }
};

template <typename Real, int R, int C>
struct CoarseNoise {
    Real (*Z)[C][2];
    template <int I>
    __device__ __forceinline__ void row(Real (&w0)[C], Real (&w1)[C])
    {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            w0[c] = Z[I][c][0];
            w1[c] = Z[I][c][1];
        }
    }
};

template <typename Real, int C>
struct NoNoise {
    template <int I>
    __device__ __forceinline__ void row(Real (&w0)[C], Real (&w1)[C])
    {
#pragma unroll
        for (int c = 0; c < C; ++c) { w0[c] = Real(0); w1[c] = Real(0); }
    }
};

// compile-time row loop
template <int I, int N>
struct RowLoop {
    template <class F>
    __device__ __forceinline__ static void run(F&& f)
    {
        if constexpr (I < N) {
            f(std::integral_constant<int, I>{});
            RowLoop<I + 1, N>::run(f);
        }
    }
};

// ---------------------------------------------------------------------------------------
// One EM step of an R x C tile held in registers.
//   halo: this sample's LDS area, [G][2 (top,bottom)][2 (rho, w1)][NN]
//   g, G: row group of the lane and number of groups; cl: column lane; NN: grid width
// ---------------------------------------------------------------------------------------
// Synchronisation of the lanes of one sample around the LDS halo exchange.  A sample spread over
// several wavefronts needs the block barrier.  A sample inside one wavefront does not: the LDS
// serves one wavefront's requests in issue order, so it is enough that the compiler keeps this
// wavefront's LDS accesses on their side of this point.
template <bool WAVE_LOCAL>
__device__ __forceinline__ void sample_sync()
{
    if constexpr (WAVE_LOCAL) asm volatile("" ::: "memory");
    else __syncthreads();
}

// Issue priority of a wavefront by its progress through one step: 3 from the start of the step
// (the halo barrier) through row 1, then 2, 1, 0 over the remaining rows.  The SIMD's arbiter
// otherwise favours the oldest wavefront, which runs ahead and waits at the next barrier while the
// last ones finish with few wavefronts left to hide their latencies; ranking by progress keeps the
// wavefronts of a sample level.
template <bool ON, int LEVEL>
__device__ __forceinline__ void progress_prio()
{
    if constexpr (ON) __builtin_amdgcn_s_setprio(LEVEL);
}

constexpr int row_prio(int i, int R) { return i < 2 ? 3 : 2 - (i - 2) * 3 / (R - 2); }

template <typename Real, int R, int C, int FLUX, bool NOISE, bool COMP, bool ONE_BARRIER, bool WAVE_LOCAL, class Noise>
__device__ __forceinline__ void tile_step(Real (&rho)[R][C], Real (&cmp)[R][C], Noise& noise, const Real a, const Real kappa,
                                          Real* __restrict__ halo, const int g, const int G, const int cl,
                                          const int NN, const int addr_l, const int addr_r)
{
    // Every rounding step of the update is written out (fma where intended), so a cell's value
    // does not depend on how the compiler schedules a particular tile shape.
#pragma clang fp contract(off)
    constexpr bool BALANCE = !WAVE_LOCAL;
    progress_prio<BALANCE, 3>();
    Real w0_first[C], w1_first[C], w0_last[C], w1_last[C];
    if constexpr (NOISE) {
        noise.template row<0>(w0_first, w1_first);
        if constexpr (R > 1) noise.template row<R - 1>(w0_last, w1_last);
    }
    Real* top = halo + (g * 2 + 0) * 2 * NN + C * cl;
    Real* bot = halo + (g * 2 + 1) * 2 * NN + C * cl;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        top[c] = rho[0][c];
        bot[c] = rho[R - 1][c];
        if constexpr (NOISE) {
            top[NN + c] = w1_first[c];
            bot[NN + c] = (R > 1) ? w1_last[c] : w1_first[c];
        }
    }
    sample_sync<WAVE_LOCAL>();
    const int gu = g == 0 ? G - 1 : g - 1;
    const int gd = g == G - 1 ? 0 : g + 1;
    const Real* above = halo + (gu * 2 + 1) * 2 * NN + C * cl;
    const Real* below = halo + (gd * 2 + 0) * 2 * NN + C * cl;
    Real rho_up[C], rho_dn[C], w1_up[C], w1_dn[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        rho_up[c] = above[c];
        rho_dn[c] = below[c];
        if constexpr (NOISE) {
            w1_up[c] = above[NN + c];
            w1_dn[c] = below[NN + c];
        }
    }
    // With a double-buffered halo (alternating by step) the next step writes the other buffer,
    // and its barrier orders those writes after every lane's reads of this one.
    if constexpr (!ONE_BARRIER) sample_sync<WAVE_LOCAL>();

    Real rprev[C];     // old density of row i-1
    Real F1prev[C];    // y-flux of row i-1 (central) / of edge (i-1, i) (staggered)
    Real F1cur[C];     // central: y-flux of row i (carried from the previous iteration)
    Real w0c[C], w1c[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        rprev[c] = rho_up[c];
        if constexpr (NOISE) {
            if constexpr (FLUX == DK_FLUX_CENTRAL) {
                F1prev[c] = pos_sqrt(rho_up[c]) * w1_up[c];
                F1cur[c] = pos_sqrt(rho[0][c]) * w1_first[c];
            } else {
                F1prev[c] = pos_sqrt(Real(0.5) * (rho_up[c] + rho[0][c])) * w1_up[c];
            }
            w0c[c] = w0_first[c];
            w1c[c] = w1_first[c];
        }
    }

    RowLoop<0, R>::run([&](auto Ic) {
        constexpr int i = decltype(Ic)::value;
        if constexpr (i >= 2 && row_prio(i, R) != row_prio(i - 1, R)) progress_prio<BALANCE, row_prio(i, R)>();
        Real rnext[C];
#pragma unroll
        for (int c = 0; c < C; ++c) rnext[c] = (i + 1 < R) ? rho[(i + 1 < R) ? i + 1 : 0][c] : rho_dn[c];
        Real w0n[C], w1n[C];
        if constexpr (NOISE) {
            if constexpr (i + 1 <= R - 2) {
                noise.template row<(i + 1 <= R - 2) ? i + 1 : 0>(w0n, w1n);
            } else if constexpr (i + 1 == R - 1) {
#pragma unroll
                for (int c = 0; c < C; ++c) { w0n[c] = w0_last[c]; w1n[c] = w1_last[c]; }
            } else {
#pragma unroll
                for (int c = 0; c < C; ++c) { w0n[c] = Real(0); w1n[c] = w1_dn[c]; }
            }
        }
        // x-halo of the density
        const Real rl = lane_get(addr_l, rho[i][C - 1]);
        const Real rr = lane_get(addr_r, rho[i][0]);
        Real F0[C], F1n[C];
        Real F0l = Real(0), F0r = Real(0);
        if constexpr (NOISE) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if constexpr (FLUX == DK_FLUX_CENTRAL) {
                    F0[c] = pos_sqrt(rho[i][c]) * w0c[c];
                    F1n[c] = pos_sqrt(rnext[c]) * w1n[c];
                } else {
                    const Real right = (c + 1 < C) ? rho[i][(c + 1 < C) ? c + 1 : 0] : rr;
                    F0[c] = pos_sqrt(Real(0.5) * (rho[i][c] + right)) * w0c[c];
                    F1n[c] = pos_sqrt(Real(0.5) * (rho[i][c] + rnext[c])) * w1c[c];   // edge (i, i+1)
                }
            }
            F0l = lane_get(addr_l, F0[C - 1]);
            if constexpr (FLUX == DK_FLUX_CENTRAL) F0r = lane_get(addr_r, F0[0]);
        }
        Real rnew[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const Real left = (c > 0) ? rho[i][(c > 0) ? c - 1 : 0] : rl;
            const Real right = (c + 1 < C) ? rho[i][(c + 1 < C) ? c + 1 : 0] : rr;
            const Real lap = fma(Real(-4), rho[i][c], (left + right) + (rprev[c] + rnext[c]));
            Real d = a * lap;
            if constexpr (NOISE) {
                Real div;
                if constexpr (FLUX == DK_FLUX_CENTRAL) {
                    const Real fl = (c > 0) ? F0[(c > 0) ? c - 1 : 0] : F0l;
                    const Real fr = (c + 1 < C) ? F0[(c + 1 < C) ? c + 1 : 0] : F0r;
                    div = (fr - fl) + (F1n[c] - F1prev[c]);
                } else {
                    const Real fl = (c > 0) ? F0[(c > 0) ? c - 1 : 0] : F0l;
                    div = (F0[c] - fl) + (F1n[c] - F1prev[c]);
                }
                d = fma(kappa, div, d);
            }
            if constexpr (COMP) {
                // compensated (Kahan) accumulation of the increment: the rounding error of the
                // FP32 state is carried in cmp and fed back the next step
                const Real y = d - cmp[i][c];
                const Real t = rho[i][c] + y;
                cmp[i][c] = (t - rho[i][c]) - y;
                rnew[c] = t;
            } else {
                rnew[c] = rho[i][c] + d;
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            rprev[c] = rho[i][c];
            rho[i][c] = rnew[c];
            if constexpr (NOISE) {
                if constexpr (FLUX == DK_FLUX_CENTRAL) {
                    F1prev[c] = F1cur[c];
                    F1cur[c] = F1n[c];
                } else {
                    F1prev[c] = F1n[c];
                }
                w0c[c] = w0n[c];
                w1c[c] = w1n[c];
            }
        }
    });
}

// ---------------------------------------------------------------------------------------
// Segmented sum over the TS lanes of one sample (TS a power of two); result valid in the
// sample's first lane.  red: LDS scratch of one double per wavefront of the block.
// ---------------------------------------------------------------------------------------
template <int TS>
__device__ __forceinline__ double sample_sum(double v, double* red, int tid)
{
    constexpr int W = TS < 64 ? TS : 64;
#pragma unroll
    for (int off = W / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if constexpr (TS > 64) {
        constexpr int NW = TS / 64;
        const int wave = tid >> 6;
        if ((tid & 63) == 0) red[wave] = v;
        __syncthreads();
        double s = 0.0;
        if ((tid % TS) == 0) {
            const int w0 = wave;   // first wavefront of this sample
            for (int w = 0; w < NW; ++w) s += red[w0 + w];
        }
        __syncthreads();
        return s;
    }
    return v;
}

template <typename Real, int R, int C, int TS>
__device__ __forceinline__ void observe(const Real (&rho)[R][C], const double* __restrict__ phi, const double* obs,
                                        int n_obs, int NN, int row0, int col0, double h2, double* red, int tid,
                                        double* dst, bool write)
{
    for (int j = 0; j < n_obs; ++j) {
        const double* ph = phi + (size_t)j * NN * NN;
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int c = 0; c < C; ++c) acc = fma((double)rho[i][c], ph[(row0 + i) * NN + col0 + c], acc);
        const double L = sample_sum<TS>(acc, red, tid);
        if (write) {
            const double scale = obs[3 * j + 0], centre = obs[3 * j + 1];
            const double X = scale * (h2 * L - centre);
            dst[2 * j] = (obs[3 * j + 2] != 0.0) ? X * X : X;
        }
    }
}

// ---------------------------------------------------------------------------------------
// LDS elements one sample needs: the fine halo rows double-buffered by step parity, then the
// coarse halo rows.
// ---------------------------------------------------------------------------------------
template <int NF, int R, bool PAIR>
constexpr int halo_elems()
{
    return 2 * (NF / R) * 4 * NF + (PAIR ? (NF / R) * 4 * (NF / 2) : 0);
}

// ---------------------------------------------------------------------------------------
// One block-iteration of the resident level kernel: the block's SPW samples (local indices
// local0 + s, s < SPW; those at or beyond A.count run but write nothing) advanced over the
// whole time horizon, then reduced to their observables.
//   halo: LDS, SPW * halo_elems<NF, R, PAIR>() elements;  red: LDS, one double per wavefront;
//   tid: the lane's index in the block (threadIdx.x).
// ---------------------------------------------------------------------------------------
template <typename Real, int NF, int R, int C, bool PAIR, int FLUX, bool NOISE, int SPW>
__device__ __forceinline__ void level_body(const LevelArgs& A, uint64_t local0, Real* halo, double* red, const int tid)
{
    constexpr int NPL = NF / C;            // lanes per row group
    constexpr int G = NF / R;              // row groups
    constexpr int TS = NPL * G;            // lanes per sample
    constexpr int NC = NF / 2;
    constexpr int RC = PAIR ? R / 2 : 1;
    constexpr int CCc = PAIR ? C / 2 : 1;
    static_assert(NPL <= 64 && (64 % NPL) == 0, "a row group must sit inside one wavefront");
    static_assert(!PAIR || (R % 2 == 0 && C % 2 == 0), "pairs need even tiles");
    static_assert(TS <= 64 || TS % 64 == 0, "sample lanes");

    constexpr int HALO = halo_elems<NF, R, PAIR>();
    constexpr bool WL = TS <= 64;     // the sample's lanes lie inside one wavefront

    const int sw = tid / TS;
    const int t = tid % TS;
    const int cl = t % NPL;
    const int g = t / NPL;
    const uint64_t local = local0 + (uint64_t)sw;
    const bool active = local < A.count;
    const uint64_t sample = A.first + (active ? local : 0);
    const int lane = tid & 63;
    const int addr_l = (lane - cl + (cl + NPL - 1) % NPL) * 4;
    const int addr_r = (lane - cl + (cl + 1) % NPL) * 4;
    const int row0 = R * g, col0 = C * cl;

    // FP32 states carry a Kahan compensation term per cell; FP64 states do not need one
    constexpr bool COMP = std::is_same<Real, float>::value && NOISE;
    Real rho[R][C], rho_cmp[R][C];
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int c = 0; c < C; ++c) rho_cmp[i][c] = Real(0);
    {
        const Real* r0 = (const Real*)A.rho0_f;
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int c = 0; c < C; ++c) rho[i][c] = r0[(row0 + i) * NF + col0 + c];
    }
    Real rhoc[RC][CCc], rhoc_cmp[RC][CCc];
    Real Z[RC][CCc][2];
    if constexpr (PAIR) {
        const Real* r0 = (const Real*)A.rho0_c;
#pragma unroll
        for (int i = 0; i < RC; ++i)
#pragma unroll
            for (int c = 0; c < CCc; ++c) {
                rhoc[i][c] = r0[(RC * g + i) * NC + CCc * cl + c];
                rhoc_cmp[i][c] = Real(0);
                Z[i][c][0] = Real(0);
                Z[i][c][1] = Real(0);
            }
    }

    Real pend[R][C / 2 > 0 ? C / 2 : 1][2];
    const NoiseKey key = make_key(A.seed, A.tag, A.level_id, sample);
    const Real a = (Real)A.a, kf = (Real)A.kf, kc = (Real)A.kc;
    Real* my_halo = halo + sw * HALO;

    // Time loop.  For pairs the fine steps are grouped by coarse step (M_f = 4 M_c); the loops
    // are kept rolled so that the compiler does not interleave the (state-independent) noise
    // of several steps, which would multiply the live registers.
    auto fine_step = [&](int m) {
        if constexpr (NOISE) {
            FineNoise<Real, R, C, PAIR> fn{key, (uint32_t)m, (uint32_t)(col0 / 2 + row0 * (NF / 2)),
                                           (uint32_t)(NF / 2), PAIR ? (Real(*)[C / 2 > 0 ? C / 2 : 1][2])Z : nullptr,
                                           pend};
            tile_step<Real, R, C, FLUX, true, COMP, true, WL>(rho, rho_cmp, fn, a, kf, my_halo + (m & 1) * G * 4 * NF, g, G,
                                                          cl, NF, addr_l, addr_r);
        } else {
            NoNoise<Real, C> nn;
            tile_step<Real, R, C, FLUX, false, false, true, WL>(rho, rho_cmp, nn, a, Real(0), my_halo + (m & 1) * G * 4 * NF, g,
                                                            G, cl, NF, addr_l, addr_r);
        }
    };
    if constexpr (PAIR) {
        const int Mc = A.steps / 4;
#pragma unroll 1
        for (int mc = 0; mc < Mc; ++mc) {
#pragma unroll 1
            for (int j = 0; j < 4; ++j) fine_step(4 * mc + j);
            CoarseNoise<Real, RC, CCc> cn{Z};
            tile_step<Real, RC, CCc, FLUX, NOISE, COMP, false, WL>(rhoc, rhoc_cmp, cn, a, kc, my_halo + 2 * G * 4 * NF, g, G,
                                                                 cl, NC, addr_l, addr_r);
#pragma unroll
            for (int i = 0; i < RC; ++i)
#pragma unroll
                for (int c = 0; c < CCc; ++c) { Z[i][c][0] = Real(0); Z[i][c][1] = Real(0); }
        }
    } else {
        // grouped by four steps like the pairs' loop: the flat loop of single steps compiles to a
        // schedule that runs 5 % slower on MI355X (same steps in the same order)
        const int M4 = A.steps / 4;
#pragma unroll 1
        for (int mq = 0; mq < M4; ++mq) {
#pragma unroll 1
            for (int j = 0; j < 4; ++j) fine_step(4 * mq + j);
        }
#pragma unroll 1
        for (int m = 4 * M4; m < A.steps; ++m) fine_step(m);
    }

    double* dst = A.out + (size_t)(active ? local : 0) * A.n_obs * 2;
    const bool writer = active && t == 0;
    observe<Real, R, C, TS>(rho, A.phi_f, A.obs_f, A.n_obs, NF, row0, col0, A.h2f, red, tid, dst, writer);
    if constexpr (PAIR) {
        observe<Real, RC, CCc, TS>(rhoc, A.phi_c, A.obs_c, A.n_obs, NC, RC * g, CCc * cl, A.h2c, red, tid, dst + 1,
                                   writer);
    } else {
        if (writer)
            for (int j = 0; j < A.n_obs; ++j) dst[2 * j + 1] = 0.0;
    }
    if (A.field_f && active) {
        Real* f = (Real*)A.field_f + (size_t)local * NF * NF;
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int c = 0; c < C; ++c) f[(row0 + i) * NF + col0 + c] = rho[i][c];
    }
    if constexpr (PAIR) {
        if (A.field_c && active) {
            Real* f = (Real*)A.field_c + (size_t)local * NC * NC;
#pragma unroll
            for (int i = 0; i < RC; ++i)
#pragma unroll
                for (int c = 0; c < CCc; ++c) f[(RC * g + i) * NC + CCc * cl + c] = rhoc[i][c];
        }
    }
}

// Lanes per sample (TS) and samples per block (SPW) of a tile shape with C = 2 columns and R rows
// per lane: about 256 lanes per block, or X times as many samples (X = 4: 1024-lane blocks).
template <int NF, int R, int X = 1>
struct ShapeOf {
    static constexpr int C = 2;
    static constexpr int TS = (NF / C) * (NF / R);
    static constexpr int SPW = (TS >= 256 ? 1 : 256 / TS) * X;
};

// Neumaier's compensated summation step: s + c accumulates x.
__device__ __forceinline__ void neumaier(double& s, double& c, double x)
{
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

}  // namespace dk
