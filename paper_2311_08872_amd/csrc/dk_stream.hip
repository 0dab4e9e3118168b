// dk_stream.hip -- the level kernel for grids that do not fit on chip (n >= 256; any multiple
// of 64 works), with the state in HBM and temporal blocking of depth D in {1, 2, 4, 8}.
//
// One launch advances a batch of samples by up to D fine steps.  Each block owns a 64 x 64 fine
// tile of one sample and loads it with a halo of H = max(D, 2) cells (H is even so that
// the 2 x 2 blocks below line up with the coarse cells and with the horizontal site pairs that
// share a generator call).  The noise of the halo is regenerated from the counter-based
// generator (it is a pure function of site and step), so no noise is exchanged; the valid
// region shrinks by one cell per step.  The state is double-buffered in HBM (read buffer / write
// buffer alternate by launch), so neighbouring tiles never read cells another block is writing.
//
// Coupled pairs: the coarse grid takes one step per 4 fine steps with the restricted noise, the
// sum of the fine noise over the coarse cell's 2 x 2 fine sites and those 4 steps.  At D = 4 a
// launch covers exactly one coarse step and takes it at its end, in the same kernel (the coarse
// halo's sums come from the fine halo).  At the other depths each block keeps the sums of its
// own coarse cells in an HBM buffer (loaded when a launch continues a group of 4 steps, stored
// at its end; D = 8 stores two groups) and a separate coarse kernel takes the coarse step once
// a group is complete.
//
// The per-cell arithmetic (explicit FMAs, Kahan-compensated increment, coarse-noise sums added
// as (even-row block sum + odd-row block sum)) is the same operation sequence as the resident
// kernel, so every depth produces bit-identical fields.
//
// Lane work: a block of 512 threads (640 at D = 8) owns the (32 + H)^2 2x2 blocks of the extended
// tile, up to three per thread, and keeps their cells in registers for the whole launch; LDS only
// passes the cells and fluxes that neighbouring blocks read (two barriers per fine step).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dk_stream.h"
#include "dk_rng.h"

namespace dk {

namespace {
constexpr int TT = 64;               // fine tile interior

template <int D>
struct Geo {
    // 3 blocks per thread at every depth (448 threads would idle fewer slots at D <= 4 but hold 14
    // wavefronts per compute unit instead of 16)
    static constexpr int THREADS = D == 8 ? 640 : 512;
    static constexpr int HH = D < 2 ? 2 : D;                  // halo width
    static constexpr int EXT = TT + 2 * HH;                   // extended tile side
    static constexpr int NBS = EXT / 2;                       // 2x2 blocks per side
    static constexpr int NBLK = NBS * NBS;
    static constexpr int BPT = (NBLK + THREADS - 1) / THREADS;
    // LDS planes hold the extended tile with one pad row above and below and two pad columns on
    // each side: the neighbour reads of the outermost blocks stay inside the plane, and every
    // block's first cell is even (8-byte aligned pairs)
    static constexpr int P = EXT + 4;                         // row pitch
    static constexpr int PLANE = P * (EXT + 2);
    // register budget: two blocks per compute unit at D <= 4; at D = 8 the LDS planes admit one
    static constexpr int WAVES_PER_SIMD = D == 8 ? 3 : 4;
};

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
// sqrt([x]^+) with [x]^+ as a signed integer maximum of the bits (negative values and -0 become
// +0), the same as the resident kernel's, one instruction shorter than fmaxf in IEEE mode
__device__ __forceinline__ float psq(float x) { return __builtin_amdgcn_sqrtf(__int_as_float(max(__float_as_int(x), 0))); }
__device__ __forceinline__ float2 lds2(const float* p) { return *(const float2*)p; }
__device__ __forceinline__ void lds2(float* p, float x, float y) { *(float2*)p = make_float2(x, y); }

// One cell's explicit EM update with the Kahan-compensated increment: the operation sequence of
// the resident kernel (lap = fma(-4, rho, (left + right) + (up + down)), d = fma(kappa, div,
// a lap), compensation fed back), so both give bit-identical fields.
__device__ __forceinline__ void em_cell(float& r, float& cm, float l, float rt, float u, float dn, float div, float a,
                                        float kappa)
{
#pragma clang fp contract(off)
    const float lap = fmaf(-4.0f, r, (l + rt) + (u + dn));
    const float d = fmaf(kappa, div, a * lap);
    const float y = d - cm;
    const float tv = r + y;
    cm = (tv - r) - y;
    r = tv;
}
}  // namespace

// Lane work: the threads own the 2x2 blocks of the extended tile (thread t holds blocks t,
// t + THREADS, t + 2 THREADS in row-major block order) and keep their cells' density and
// compensation in registers for all D steps.  A block is one generator call per row (the row's
// horizontal site pair) and its coarse cell's noise sum.  LDS only carries what the neighbouring
// blocks read: each step a block publishes its density and fluxes, and after one barrier reads
// the adjacent cells of the blocks around it.  A block takes part in step j while it meets that
// step's region: blocks at block distance L from the extended tile's edge hold cells at distances
// 2L and 2L + 1, the fluxes are needed at distance >= j and the updates at distance >= j + 1.
// Cells a block computes outside those regions hold values no valid cell reads.
template <int FLUX, bool PAIR, int D>
__global__ void __launch_bounds__(Geo<D>::THREADS, Geo<D>::WAVES_PER_SIMD) stream_kernel(const StreamArgs A)
{
#pragma clang fp contract(off)
    constexpr int THREADS = Geo<D>::THREADS;
    constexpr int HH = Geo<D>::HH, EXT = Geo<D>::EXT, NBS = Geo<D>::NBS, NBLK = Geo<D>::NBLK, BPT = Geo<D>::BPT;
    constexpr int P = Geo<D>::P, PLANE = Geo<D>::PLANE;
    constexpr bool FUSED = PAIR && D == 4;     // coarse step taken by this kernel
    constexpr bool SPLIT = PAIR && D != 4;     // noise sums kept in HBM, coarse step by its own kernel
    constexpr int HB = HH / 2;                 // first block of the tile interior
    static_assert(PLANE < (1 << 13) && NBS / 2 + 1 < (1 << 6), "block descriptor fields");
    __shared__ __align__(16) float sr[PLANE];
    __shared__ __align__(16) float sf0[PLANE];
    __shared__ __align__(16) float sf1[PLANE];
    const int n = A.n;
    const int tiles_x = n / TT;
    // Workgroups are handed to the 8 compute dies in turn by their index; this numbering gives each
    // die a contiguous run of (sample, tile-row-major) tiles, so that the left and right neighbours
    // whose columns a tile's halo reads sit in the same die's L2 (numbering by tile index would put
    // them on other dies and fetch every horizontal halo line from HBM a second time).
    const unsigned total = gridDim.x, per = total / 8u, rem = total % 8u;
    const unsigned die = blockIdx.x % 8u, kd = blockIdx.x / 8u;
    const unsigned lin = (die < rem ? die * (per + 1u) : rem * (per + 1u) + (die - rem) * per) + kd;
    const int tile = (int)(lin % (unsigned)(tiles_x * tiles_x));
    const int sidx = (int)(lin / (unsigned)(tiles_x * tiles_x));
    const int tx0 = (tile % tiles_x) * TT, ty0 = (tile / tiles_x) * TT;
    const int cx0 = tx0 / 2, cy0 = ty0 / 2;
    const int nc = n / 2;
    const uint64_t sample = A.first + sidx;
    const size_t nn = (size_t)n * n;
    // per-sample bases; cells are addressed by 32-bit byte offsets from them (4 n^2 < 2^32 for the
    // grids up to 4096^2 that the library accepts)
    const char* rin = (const char*)(A.rho_in + sidx * nn);
    const char* cin = (const char*)(A.cmp_in + sidx * nn);
    char* rout = (char*)(A.rho_out + sidx * nn);
    char* cout = (char*)(A.cmp_out + sidx * nn);
    auto at = [n](int y, int x) { return 4u * ((uint32_t)y * (uint32_t)n + (uint32_t)x); };
    const int t = threadIdx.x;
    const NoiseKey key = make_key(A.seed, A.tag, A.level_id, sample);
    const uint32_t ppr = (uint32_t)(n / 2);
    // (split pairs) block (bx, by) of the interior <-> coarse cell (cx0 + bx - HB, cy0 + by - HB)
    auto zslot = [&](int bx, int by, int group) -> float2* {
        return (float2*)A.z + group * A.zgroup + ((size_t)sidx * nc + (cy0 + by - HB)) * nc + (cx0 + bx - HB);
    };

    // zero the pad cells (read only by the outermost blocks, whose results are never used)
    for (int i = t; i < 2 * P + 4 * EXT; i += THREADS) {
        const int e = i - 2 * P;   // side pads: 4 per row, 2 on the left and 2 on the right
        const int c = i < 2 * P ? (i < P ? i : PLANE - 2 * P + i) : (1 + e / 4) * P + ((e & 3) < 2 ? (e & 3) : P - 4 + (e & 3));
        sr[c] = 0.f;
        sf0[c] = 0.f;
        sf1[c] = 0.f;
    }

    // Per block: the two rows of its density and compensation, its noise sums, and two descriptor
    // words: its first cell's LDS index | (1 + block distance to the edge) << 13 (0: no block), and
    // the generator index of its upper site pair | a flag for the wrap of its lower row.
    float r[BPT][4], cm[BPT][4], Z[BPT][2];
    uint32_t binf[BPT], bidx[BPT];
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int b = t + k * THREADS;
        binf[k] = 0u;
        bidx[k] = 0u;
        Z[k][0] = 0.f;
        Z[k][1] = 0.f;
#pragma unroll
        for (int q = 0; q < 4; ++q) { r[k][q] = 0.f; cm[k][q] = 0.f; }
        if (b < NBLK) {
            const int bx = b % NBS, by = b / NBS;
            const int lay = min(min(bx, NBS - 1 - bx), min(by, NBS - 1 - by));
            binf[k] = (uint32_t)((2 * by + 1) * P + 2 * bx + 2) | ((uint32_t)(lay + 1) << 13);
            const int gy = wrapi(ty0 + 2 * by - HH, n);
            const int gy1 = gy + 1 == n ? 0 : gy + 1;
            const int gx = wrapi(tx0 + 2 * bx - HH, n);   // even
            bidx[k] = ((uint32_t)(gx / 2) + ppr * (uint32_t)gy) | ((uint32_t)(gy == n - 1) << 31);
            const float2 r0 = *(const float2*)(rin + at(gy, gx));
            const float2 r1 = *(const float2*)(rin + at(gy1, gx));
            const float2 c0 = *(const float2*)(cin + at(gy, gx));
            const float2 c1 = *(const float2*)(cin + at(gy1, gx));
            r[k][0] = r0.x; r[k][1] = r0.y; r[k][2] = r1.x; r[k][3] = r1.y;
            cm[k][0] = c0.x; cm[k][1] = c0.y; cm[k][2] = c1.x; cm[k][3] = c1.y;
            if constexpr (SPLIT) {
                if (A.z_load && lay >= HB) {
                    const float2 zz = *zslot(bx, by, 0);
                    Z[k][0] = zz.x;
                    Z[k][1] = zz.y;
                }
            }
        }
    }
    const uint32_t wrap_back = ppr * (uint32_t)(n - 1);   // lower row index of a block on the last row: gx / 2

    // the unit normals of block k at step m, added to its coarse cell's sums as (upper row sum +
    // lower row sum)
    auto draw = [&](int k, uint32_t m, float (&w0)[4], float (&w1)[4]) {
        const uint32_t idx0 = bidx[k] & 0x7FFFFFFFu;
        const uint32_t idx1 = (bidx[k] >> 31) ? idx0 - wrap_back : idx0 + ppr;
        site_pair_normals(key, idx0, m, w0[0], w1[0], w0[1], w1[1]);
        site_pair_normals(key, idx1, m, w0[2], w1[2], w0[3], w1[3]);
        if constexpr (PAIR) {
            Z[k][0] += (w0[0] + w0[1]) + (w0[2] + w0[3]);
            Z[k][1] += (w1[0] + w1[1]) + (w1[2] + w1[3]);
        }
    };

    const float a = A.a, kappa = A.kf;
    for (int j = 0; j < A.ksteps; ++j) {
        const uint32_t m = (uint32_t)(A.m0 + j);
        const uint32_t lo_flux = (uint32_t)(j >> 1) + 1u;         // 1 + least block distance of the flux region
        const uint32_t lo_upd = (uint32_t)((j + 1) >> 1) + 1u;    // ... of the update region
        float f0k[BPT][4], f1k[BPT][4];
        if constexpr (FLUX == DK_FLUX_CENTRAL) {
            // publish density and node fluxes sqrt(rho^+) w
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                if ((binf[k] >> 13) < lo_flux) continue;
                const int c0 = (int)(binf[k] & 0x1FFFu);
                float w0[4], w1[4];
                draw(k, m, w0, w1);
                float (&f0)[4] = f0k[k];
                float (&f1)[4] = f1k[k];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float sq = psq(r[k][q]);
                    f0[q] = sq * w0[q];
                    f1[q] = sq * w1[q];
                }
                lds2(sr + c0, r[k][0], r[k][1]);
                lds2(sr + c0 + P, r[k][2], r[k][3]);
                lds2(sf0 + c0, f0[0], f0[1]);
                lds2(sf0 + c0 + P, f0[2], f0[3]);
                lds2(sf1 + c0, f1[0], f1[1]);
                lds2(sf1 + c0 + P, f1[2], f1[3]);
            }
        } else {
            // publish density; the edge fluxes need the right and lower neighbours' densities
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                if ((binf[k] >> 13) < lo_flux) continue;
                const int c0 = (int)(binf[k] & 0x1FFFu);
                lds2(sr + c0, r[k][0], r[k][1]);
                lds2(sr + c0 + P, r[k][2], r[k][3]);
            }
        }
        __syncthreads();
        if constexpr (FLUX == DK_FLUX_CENTRAL) {
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                if ((binf[k] >> 13) < lo_upd) continue;
                const int c0 = (int)(binf[k] & 0x1FFFu);
                const float2 up = lds2(sr + c0 - P), dn = lds2(sr + c0 + 2 * P);
                const float l0 = lds2(sr + c0 - 2).y, l1 = lds2(sr + c0 + P - 2).y;
                const float r0 = lds2(sr + c0 + 2).x, r1 = lds2(sr + c0 + P + 2).x;
                const float2 f0a = make_float2(f0k[k][0], f0k[k][1]), f0b = make_float2(f0k[k][2], f0k[k][3]);
                const float fl0 = lds2(sf0 + c0 - 2).y, fl1 = lds2(sf0 + c0 + P - 2).y;
                const float fr0 = lds2(sf0 + c0 + 2).x, fr1 = lds2(sf0 + c0 + P + 2).x;
                const float2 f1u = lds2(sf1 + c0 - P), f1a = make_float2(f1k[k][0], f1k[k][1]),
                             f1b = make_float2(f1k[k][2], f1k[k][3]), f1d = lds2(sf1 + c0 + 2 * P);
                const float o0 = r[k][0], o1 = r[k][1], o2 = r[k][2], o3 = r[k][3];
                // div = (right x-flux - left x-flux) + (lower y-flux - upper y-flux)
                em_cell(r[k][0], cm[k][0], l0, o1, up.x, o2, (f0a.y - fl0) + (f1b.x - f1u.x), a, kappa);
                em_cell(r[k][1], cm[k][1], o0, r0, up.y, o3, (fr0 - f0a.x) + (f1b.y - f1u.y), a, kappa);
                em_cell(r[k][2], cm[k][2], l1, o3, o0, dn.x, (f0b.y - fl1) + (f1d.x - f1a.x), a, kappa);
                em_cell(r[k][3], cm[k][3], o2, r1, o1, dn.y, (fr1 - f0b.x) + (f1d.y - f1a.y), a, kappa);
            }
        } else {
            // edge fluxes psq((rho + right) / 2) w0 and psq((rho + lower) / 2) w1; the Laplacian
            // is formed here, where the neighbours' densities are read
            float lap4[BPT][4];
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                if ((binf[k] >> 13) < lo_flux) continue;
                const int c0 = (int)(binf[k] & 0x1FFFu);
                float w0[4], w1[4];
                draw(k, m, w0, w1);
                const float2 up = lds2(sr + c0 - P), dn = lds2(sr + c0 + 2 * P);
                const float l0 = lds2(sr + c0 - 2).y, l1 = lds2(sr + c0 + P - 2).y;
                const float r0 = lds2(sr + c0 + 2).x, r1 = lds2(sr + c0 + P + 2).x;
                const float o0 = r[k][0], o1 = r[k][1], o2 = r[k][2], o3 = r[k][3];
                const float f0[4] = {psq(0.5f * (o0 + o1)) * w0[0], psq(0.5f * (o1 + r0)) * w0[1],
                                     psq(0.5f * (o2 + o3)) * w0[2], psq(0.5f * (o3 + r1)) * w0[3]};
                const float f1[4] = {psq(0.5f * (o0 + o2)) * w1[0], psq(0.5f * (o1 + o3)) * w1[1],
                                     psq(0.5f * (o2 + dn.x)) * w1[2], psq(0.5f * (o3 + dn.y)) * w1[3]};
                lds2(sf0 + c0, f0[0], f0[1]);
                lds2(sf0 + c0 + P, f0[2], f0[3]);
                lds2(sf1 + c0, f1[0], f1[1]);
                lds2(sf1 + c0 + P, f1[2], f1[3]);
                lap4[k][0] = fmaf(-4.0f, o0, (l0 + o1) + (up.x + o2));
                lap4[k][1] = fmaf(-4.0f, o1, (o0 + r0) + (up.y + o3));
                lap4[k][2] = fmaf(-4.0f, o2, (l1 + o3) + (o0 + dn.x));
                lap4[k][3] = fmaf(-4.0f, o3, (o2 + r1) + (o1 + dn.y));
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                if ((binf[k] >> 13) < lo_upd) continue;
                const int c0 = (int)(binf[k] & 0x1FFFu);
                const float2 f0a = lds2(sf0 + c0), f0b = lds2(sf0 + c0 + P);
                const float fl0 = lds2(sf0 + c0 - 2).y, fl1 = lds2(sf0 + c0 + P - 2).y;
                const float2 f1u = lds2(sf1 + c0 - P), f1a = lds2(sf1 + c0), f1b = lds2(sf1 + c0 + P);
                const float div[4] = {(f0a.x - fl0) + (f1a.x - f1u.x), (f0a.y - f0a.x) + (f1a.y - f1u.y),
                                      (f0b.x - fl1) + (f1b.x - f1a.x), (f0b.y - f0b.x) + (f1b.y - f1a.y)};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float d = fmaf(kappa, div[q], a * lap4[k][q]);
                    const float y = d - cm[k][q];
                    const float tv = r[k][q] + y;
                    cm[k][q] = (tv - r[k][q]) - y;
                    r[k][q] = tv;
                }
            }
        }
        if constexpr (SPLIT) {
            // a group of 4 fine steps is complete (D = 8: two per launch), or the launch ends
            if ((D == 8 && j == 3) || j == A.ksteps - 1) {
#pragma unroll
                for (int k = 0; k < BPT; ++k) {
                    const int b = t + k * THREADS;
                    if ((binf[k] >> 13) > (uint32_t)HB)
                        *zslot(b % NBS, b / NBS, D == 8 ? (j >> 2) : 0) = make_float2(Z[k][0], Z[k][1]);
                    Z[k][0] = 0.f;
                    Z[k][1] = 0.f;
                }
            }
        }
        // Central fluxes: the next step's writes must wait for this step's reads.  Edge fluxes
        // need no barrier here: the next density writes follow the flux barrier above, after the
        // last density read, and the next flux writes follow the next step's first barrier.
        if constexpr (FLUX == DK_FLUX_CENTRAL) __syncthreads();
    }
    // write back the interior blocks
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        if ((binf[k] >> 13) <= (uint32_t)HB) continue;
        const int b = t + k * THREADS;
        const int bx = b % NBS, by = b / NBS;
        const uint32_t g0 = at(ty0 + 2 * by - HH, tx0 + 2 * bx - HH), g1 = g0 + 4u * (uint32_t)n;
        *(float2*)(rout + g0) = make_float2(r[k][0], r[k][1]);
        *(float2*)(rout + g1) = make_float2(r[k][2], r[k][3]);
        *(float2*)(cout + g0) = make_float2(cm[k][0], cm[k][1]);
        *(float2*)(cout + g1) = make_float2(cm[k][2], cm[k][3]);
    }
    if constexpr (FUSED) {
        if (!A.do_coarse) return;
        // One coarse EM step with the restricted noise Z.  The block at (bx, by), block distance >= 1
        // from the edge, holds the coarse cell (cx0 + bx - HB, cy0 + by - HB): together the coarse
        // tile and a ring of one cell.  Its coarse density and fluxes go to the LDS slot of its
        // first fine cell, so coarse neighbours sit two fine cells (two rows) apart.
        const size_t ncc = (size_t)nc * nc;
        const float* rcin = A.rhoc_in + sidx * ncc;
        const float* ccin = A.cmpc_in + sidx * ncc;
        float* rcout = A.rhoc_out + sidx * ncc;
        float* ccout = A.cmpc_out + sidx * ncc;
        const float kc = A.kc;
        // central fluxes: the last fine step's closing barrier already ordered its reads
        if constexpr (FLUX != DK_FLUX_CENTRAL) __syncthreads();
        float rc[BPT];
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            rc[k] = 0.f;
            if ((binf[k] >> 13) < 2u) continue;
            const int b = t + k * THREADS;
            const int bx = b % NBS, by = b / NBS;
            const int c0 = (int)(binf[k] & 0x1FFFu);
            rc[k] = rcin[(size_t)wrapi(cy0 + by - HB, nc) * nc + wrapi(cx0 + bx - HB, nc)];
            sr[c0] = rc[k];
            if constexpr (FLUX == DK_FLUX_CENTRAL) {
                const float sq = psq(rc[k]);
                sf0[c0] = sq * Z[k][0];
                sf1[c0] = sq * Z[k][1];
            }
        }
        __syncthreads();
        if constexpr (FLUX != DK_FLUX_CENTRAL) {
            // edge fluxes (the ring's outer ones read cells that are not coarse; no update reads them)
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                if ((binf[k] >> 13) < 2u) continue;
                const int c0 = (int)(binf[k] & 0x1FFFu);
                sf0[c0] = psq(0.5f * (rc[k] + sr[c0 + 2])) * Z[k][0];
                sf1[c0] = psq(0.5f * (rc[k] + sr[c0 + 2 * P])) * Z[k][1];
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            if ((binf[k] >> 13) <= (uint32_t)HB) continue;
            const int b = t + k * THREADS;
            const int bx = b % NBS, by = b / NBS;
            const int c0 = (int)(binf[k] & 0x1FFFu);
            const size_t g = (size_t)(cy0 + by - HB) * nc + (cx0 + bx - HB);
            float div;
            if constexpr (FLUX == DK_FLUX_CENTRAL) div = (sf0[c0 + 2] - sf0[c0 - 2]) + (sf1[c0 + 2 * P] - sf1[c0 - 2 * P]);
            else div = (sf0[c0] - sf0[c0 - 2]) + (sf1[c0] - sf1[c0 - 2 * P]);
            float rv = rc[k], cmv = ccin[g];
            em_cell(rv, cmv, sr[c0 - 2], sr[c0 + 2], sr[c0 - 2 * P], sr[c0 + 2 * P], div, a, kc);
            rcout[g] = rv;
            ccout[g] = cmv;
        }
    }
}

// One coarse EM step of a batch of coarse grids from completed restricted-noise sums z
// ([count][nc][nc] pairs, as stored by the split-depth pair kernels): a thread per coarse cell,
// the operation sequence of the fused coarse step, so both give bit-identical coarse fields.
template <int FLUX>
__global__ void __launch_bounds__(256) stream_coarse_kernel(const int nc, const size_t total, const float a,
                                                            const float kc, const float* __restrict__ rin,
                                                            const float* __restrict__ cin,
                                                            const float2* __restrict__ z, float* __restrict__ rout,
                                                            float* __restrict__ cout)
{
#pragma clang fp contract(off)
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const size_t ncc = (size_t)nc * nc;
    const size_t base = i - i % ncc;
    const int c = (int)(i % ncc);
    const int x = c % nc, y = c / nc;
    const int xm = x == 0 ? nc - 1 : x - 1, xp = x == nc - 1 ? 0 : x + 1;
    const int ym = y == 0 ? nc - 1 : y - 1, yp = y == nc - 1 ? 0 : y + 1;
    const float* r = rin + base;
    const float2* zz = z + base;
    const int cl = y * nc + xm, cr = y * nc + xp, cu = ym * nc + x, cd = yp * nc + x;
    const float rv = r[c], rl = r[cl], rr = r[cr], ru = r[cu], rd = r[cd];
    const float lap = fmaf(-4.0f, rv, (rl + rr) + (ru + rd));
    float div;
    if (FLUX == DK_FLUX_CENTRAL) {
        div = (psq(rr) * zz[cr].x - psq(rl) * zz[cl].x) + (psq(rd) * zz[cd].y - psq(ru) * zz[cu].y);
    } else {
        const float f0 = psq(0.5f * (rv + rr)) * zz[c].x, f0m = psq(0.5f * (rl + rv)) * zz[cl].x;
        const float f1 = psq(0.5f * (rv + rd)) * zz[c].y, f1m = psq(0.5f * (ru + rv)) * zz[cu].y;
        div = (f0 - f0m) + (f1 - f1m);
    }
    const float d = fmaf(kc, div, a * lap);
    const float y2 = d - cin[i];
    const float tv = rv + y2;
    rout[i] = tv;
    cout[i] = (tv - rv) - y2;
}

// state initialisation: rho = rho0 table, compensation 0
__global__ void stream_init_kernel(const float* __restrict__ rho0, size_t nn, int count, float* __restrict__ rho,
                                   float* __restrict__ cmp)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn * (size_t)count) return;
    rho[i] = rho0[i % nn];
    cmp[i] = 0.f;
}

// copy the coarse state when a launch does no coarse step (keeps the read/write buffers in step)
__global__ void stream_copy_kernel(const float* __restrict__ a, const float* __restrict__ b, size_t total,
                                   float* __restrict__ a2, float* __restrict__ b2)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    a2[i] = a[i];
    b2[i] = b[i];
}

// observables of final fields: one block per sample; out[s][j][slot]
__global__ void __launch_bounds__(256) stream_observe_kernel(const float* __restrict__ rho, int n, int count,
                                                             const double* __restrict__ phi, const double* __restrict__ obs,
                                                             int n_obs, double h2, double* __restrict__ out, int slot)
{
    const int s = blockIdx.x;
    if (s >= count) return;
    const size_t nn = (size_t)n * n;
    const float* r = rho + s * nn;
    __shared__ double red[4];
    for (int j = 0; j < n_obs; ++j) {
        const double* ph = phi + j * nn;
        double acc = 0.0;
        for (size_t i = threadIdx.x; i < nn; i += 256) acc = fma((double)r[i], ph[i], acc);
        for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            const double L = (red[0] + red[1]) + (red[2] + red[3]);
            const double X = obs[3 * j] * (h2 * L - obs[3 * j + 1]);
            out[((size_t)s * n_obs + j) * 2 + slot] = obs[3 * j + 2] != 0.0 ? X * X : X;
        }
        __syncthreads();
    }
}

__global__ void zero_slot_kernel(double* out, int count, int n_obs, int slot)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count * n_obs) return;
    out[(size_t)i * 2 + slot] = 0.0;
}

// Noise-free FP32 step of a batch of fields (the scheme without noise, i.e. the discrete mean
// field of many initial data at once).  A thread owns 4 consecutive columns and marches down a
// strip of HRY rows, keeping the rows above, at and below in registers, so every row is read
// from memory once per strip plus the two halo rows (18 reads per 16 rows) instead of once per
// neighbouring row: consecutive blocks are spread over the XCDs, whose L2s do not share lines,
// so re-reads of a neighbour's rows would otherwise come from HBM.  The two outer neighbours of
// the 4 columns are scalar loads that hit the lines of the adjacent threads.
constexpr int HRY = 16;

__global__ void __launch_bounds__(256) heat_f32_kernel(const float* __restrict__ in, float* __restrict__ out, int n,
                                                       size_t total, float a)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int q = n / 4;
    const int strips = (n + HRY - 1) / HRY;
    const int x0 = (int)(i % q) * 4;
    const size_t rest = i / q;
    const int strip = (int)(rest % strips);
    const size_t b = rest / strips;
    const size_t nn = (size_t)n * n;
    const float* f = in + b * nn;
    float* g = out + b * nn;
    const int y0 = strip * HRY, y1 = y0 + HRY < n ? y0 + HRY : n;
    const int xl = x0 == 0 ? n - 1 : x0 - 1, xr = x0 + 4 == n ? 0 : x0 + 4;
    float4 u = *(const float4*)(f + (size_t)(y0 == 0 ? n - 1 : y0 - 1) * n + x0);
    float4 c = *(const float4*)(f + (size_t)y0 * n + x0);
#pragma unroll 4
    for (int y = y0; y < y1; ++y) {
        const int yp = y == n - 1 ? 0 : y + 1;
        const float4 d = *(const float4*)(f + (size_t)yp * n + x0);
        const float l = f[(size_t)y * n + xl];
        const float rr = f[(size_t)y * n + xr];
        float4 o;
        o.x = c.x + a * fmaf(-4.0f, c.x, (l + c.y) + (u.x + d.x));
        o.y = c.y + a * fmaf(-4.0f, c.y, (c.x + c.z) + (u.y + d.y));
        o.z = c.z + a * fmaf(-4.0f, c.z, (c.y + c.w) + (u.z + d.z));
        o.w = c.w + a * fmaf(-4.0f, c.w, (c.z + rr) + (u.w + d.w));
        *(float4*)(g + (size_t)y * n + x0) = o;
        u = c;
        c = d;
    }
}

hipError_t launch_heat_f32(const float* in, float* out, int n, int batch, float a, hipStream_t s)
{
    const size_t total = (size_t)(n / 4) * ((n + HRY - 1) / HRY) * batch;
    hipLaunchKernelGGL(heat_f32_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, in, out, n, total, a);
    return hipGetLastError();
}

bool stream_supported(int nf) { return nf >= 64 && nf % TT == 0; }

template <int FLUX, bool PAIR>
static hipError_t launch_depth(const StreamArgs& A, int depth, dim3 grid, hipStream_t s)
{
    switch (depth) {
    case 1: hipLaunchKernelGGL((stream_kernel<FLUX, PAIR, 1>), grid, dim3(Geo<1>::THREADS), 0, s, A); break;
    case 2: hipLaunchKernelGGL((stream_kernel<FLUX, PAIR, 2>), grid, dim3(Geo<2>::THREADS), 0, s, A); break;
    case 4: hipLaunchKernelGGL((stream_kernel<FLUX, PAIR, 4>), grid, dim3(Geo<4>::THREADS), 0, s, A); break;
    case 8: hipLaunchKernelGGL((stream_kernel<FLUX, PAIR, 8>), grid, dim3(Geo<8>::THREADS), 0, s, A); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool stream_depth_supported(int depth) { return depth == 1 || depth == 2 || depth == 4 || depth == 8; }

hipError_t launch_stream_step(const StreamArgs& A, bool pair, int flux, int depth, hipStream_t s)
{
    if (A.ksteps < 1 || A.ksteps > depth || (pair && depth != 4 && !A.z)) return hipErrorInvalidValue;
    const uint64_t blocks = (uint64_t)(A.n / TT) * (A.n / TT) * (uint64_t)A.count;
    if (blocks == 0 || blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks);
    if (pair) {
        if (flux == DK_FLUX_CENTRAL) return launch_depth<DK_FLUX_CENTRAL, true>(A, depth, grid, s);
        return launch_depth<DK_FLUX_STAGGERED, true>(A, depth, grid, s);
    }
    if (flux == DK_FLUX_CENTRAL) return launch_depth<DK_FLUX_CENTRAL, false>(A, depth, grid, s);
    return launch_depth<DK_FLUX_STAGGERED, false>(A, depth, grid, s);
}

hipError_t launch_stream_coarse(int nc, int count, float a, float kc, int flux, const float* rho_in, const float* cmp_in,
                                const float* z, float* rho_out, float* cmp_out, hipStream_t s)
{
    const size_t total = (size_t)nc * nc * count;
    const dim3 grid((unsigned)((total + 255) / 256));
    if (flux == DK_FLUX_CENTRAL)
        hipLaunchKernelGGL((stream_coarse_kernel<DK_FLUX_CENTRAL>), grid, dim3(256), 0, s, nc, total, a, kc, rho_in,
                           cmp_in, (const float2*)z, rho_out, cmp_out);
    else
        hipLaunchKernelGGL((stream_coarse_kernel<DK_FLUX_STAGGERED>), grid, dim3(256), 0, s, nc, total, a, kc, rho_in,
                           cmp_in, (const float2*)z, rho_out, cmp_out);
    return hipGetLastError();
}

hipError_t launch_stream_init(const float* rho0, int n, int count, float* rho, float* cmp, hipStream_t s)
{
    const size_t total = (size_t)n * n * count;
    hipLaunchKernelGGL(stream_init_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, rho0, (size_t)n * n,
                       count, rho, cmp);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const float* a, const float* b, size_t total, float* a2, float* b2, hipStream_t s)
{
    hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a, b, total, a2, b2);
    return hipGetLastError();
}

hipError_t launch_stream_observe(const float* rho, int n, int count, const double* phi, const double* obs, int n_obs,
                                 double h2, double* out, int slot, hipStream_t s)
{
    hipLaunchKernelGGL(stream_observe_kernel, dim3(count), dim3(256), 0, s, rho, n, count, phi, obs, n_obs, h2, out, slot);
    return hipGetLastError();
}

hipError_t launch_zero_slot(double* out, int count, int n_obs, int slot, hipStream_t s)
{
    const int total = count * n_obs;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_slot_kernel, dim3((total + 255) / 256), dim3(256), 0, s, out, count, n_obs, slot);
    return hipGetLastError();
}

}  // namespace dk
