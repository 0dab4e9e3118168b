// dk_stream.hip -- the level kernel for grids that do not fit on chip (n >= 256; any multiple
// of 64 works), with the state in HBM and temporal blocking of depth D in {1, 2, 4, 8}.
//
// One launch advances a batch of samples by up to D fine steps.  Each block owns a 64 x 64 fine
// tile of one sample and loads it with a halo of H = max(D, 2) cells into LDS (H is even so that
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
// tile, up to three per thread (thread t owns blocks t, t + 512, t + 1024); each 2x2 block is two
// generator calls per step (one per horizontal site pair) and holds its coarse cell's noise sum in
// registers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dk_stream.h"
#include "dk_rng.h"

namespace dk {

namespace {
constexpr int TT = 64;               // fine tile interior
constexpr int CT = TT / 2;           // coarse tile interior (32)
constexpr int CEXT = CT + 2;         // coarse tile with a 1-cell halo (34), fused coarse step

template <int D>
struct Geo {
    // 3 blocks per thread at every depth (448 threads would idle fewer slots at D <= 4 but hold 14
    // wavefronts per compute unit instead of 16, and ran 19 % slower)
    static constexpr int THREADS = D == 8 ? 640 : 512;
    static constexpr int HH = D < 2 ? 2 : D;                  // halo width
    static constexpr int EXT = TT + 2 * HH;                   // extended tile side
    static constexpr int NBS = EXT / 2;                       // 2x2 blocks per side
    static constexpr int NBLK = NBS * NBS;
    static constexpr int BPT = (NBLK + THREADS - 1) / THREADS;
    static constexpr int NCELL = EXT * EXT;
    static constexpr int CPT = (NCELL + THREADS - 1) / THREADS;   // cells per thread, row-major deal
};

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
// sqrt([x]^+) with [x]^+ as a signed integer maximum of the bits (negative values and -0 become
// +0), the same as the resident kernel's, one instruction shorter than fmaxf in IEEE mode
__device__ __forceinline__ float psq(float x) { return __builtin_amdgcn_sqrtf(__int_as_float(max(__float_as_int(x), 0))); }
}  // namespace

template <int FLUX, bool PAIR, int D>
__global__ void __launch_bounds__(Geo<D>::THREADS, 4) stream_kernel(const StreamArgs A)
{
#pragma clang fp contract(off)
    constexpr int THREADS = Geo<D>::THREADS;
    constexpr int HH = Geo<D>::HH, EXT = Geo<D>::EXT, NBS = Geo<D>::NBS, NBLK = Geo<D>::NBLK, BPT = Geo<D>::BPT;
    constexpr int NCELL = Geo<D>::NCELL, CPT = Geo<D>::CPT;
    constexpr bool FUSED = PAIR && D == 4;     // coarse step taken by this kernel
    constexpr bool SPLIT = PAIR && D != 4;     // noise sums kept in HBM, coarse step by its own kernel
    constexpr int HB = HH / 2;                 // first block of the tile interior
    __shared__ float sr[EXT * EXT];
    __shared__ float sf0[EXT * EXT];
    __shared__ float sf1[EXT * EXT];
    const int n = A.n;
    const int tiles_x = n / TT;
    // Workgroups are handed to the 8 compute dies in turn by their index; this numbering gives each
    // die a contiguous run of (sample, tile-row-major) tiles, so that the left and right neighbours
    // whose columns a tile's halo reads sit in the same die's L2 (numbering by tile index would put
    // them on other dies and fetch every horizontal halo line from HBM a second time).
    const unsigned total = gridDim.x, per = total / 8u, rem = total % 8u;
    const unsigned die = blockIdx.x % 8u, k = blockIdx.x / 8u;
    const unsigned lin = (die < rem ? die * (per + 1u) : rem * (per + 1u) + (die - rem) * per) + k;
    const int tile = (int)(lin % (unsigned)(tiles_x * tiles_x));
    const int sidx = (int)(lin / (unsigned)(tiles_x * tiles_x));
    const int tx0 = (tile % tiles_x) * TT, ty0 = (tile / tiles_x) * TT;
    const int cx0 = tx0 / 2, cy0 = ty0 / 2;
    const int nc = n / 2;
    const uint64_t sample = A.first + sidx;
    const size_t nn = (size_t)n * n;
    const float* rin = A.rho_in + sidx * nn;
    const float* cin = A.cmp_in + sidx * nn;
    float* rout = A.rho_out + sidx * nn;
    float* cout = A.cmp_out + sidx * nn;
    const int t = threadIdx.x;
    const NoiseKey key = make_key(A.seed, A.tag, A.level_id, sample);
    const uint32_t ppr = (uint32_t)(n / 2);
    // (split pairs) block (bx, by) of the interior <-> coarse cell (cx0 + bx - HB, cy0 + by - HB)
    auto zslot = [&](int bx, int by, int group) -> float2* {
        return (float2*)A.z + group * A.zgroup + ((size_t)sidx * nc + (cy0 + by - HB)) * nc + (cx0 + bx - HB);
    };
    auto interior = [&](int bx, int by) { return bx >= HB && bx < HB + CT && by >= HB && by < HB + CT; };

    // Two deals of the extended tile to the threads: 2x2 blocks (b = t + k THREADS) for the noise,
    // whose generator calls cover horizontal site pairs and whose restriction sums 2x2 cells, and
    // single cells in row-major order (i = t + k THREADS) for the update, so that the lanes of a
    // wavefront read and write consecutive LDS words (no bank conflicts) and the halo's shrinking
    // update region is shared out cell by cell.
    float cmp[CPT], Z[BPT][2];
    // load the extended tile (and, continuing a group, the running noise sums)
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int i = t + k * THREADS;
        cmp[k] = 0.f;
        if (i < NCELL) {
            const int ex = i % EXT, ey = i / EXT;
            const int gx = wrapi(tx0 + ex - HH, n), gy = wrapi(ty0 + ey - HH, n);
            sr[i] = rin[(size_t)gy * n + gx];
            cmp[k] = cin[(size_t)gy * n + gx];
        }
    }
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int b = t + k * THREADS;
        Z[k][0] = 0.f;
        Z[k][1] = 0.f;
        if constexpr (SPLIT) {
            const int bx = b % NBS, by = b / NBS;
            if (b < NBLK && A.z_load && interior(bx, by)) {
                const float2 zz = *zslot(bx, by, 0);
                Z[k][0] = zz.x;
                Z[k][1] = zz.y;
            }
        }
    }
    // Per-launch constants of the two deals, so that no step repeats the index arithmetic: for each
    // cell slot its distance to the extended tile's edge, four to a register (the update region of
    // step j is the cells at distance > j; 0 marks a slot past the tile); for each 2x2 block slot
    // its first cell's LDS index, 1 + its distance in blocks to the edge (0 marks a slot past the
    // tile) and whether it is in the last block column / row, and the generator index of its
    // upper site pair with a flag for the wrap of its lower row.
    uint32_t clay[(CPT + 3) / 4];
#pragma unroll
    for (int q = 0; q < (CPT + 3) / 4; ++q) clay[q] = 0u;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int i = t + k * THREADS;
        if (i < NCELL) {
            const int ex = i % EXT, ey = i / EXT;
            const int lay = min(min(ex, EXT - 1 - ex), min(ey, EXT - 1 - ey));
            clay[k / 4] |= (uint32_t)lay << (8 * (k % 4));
        }
    }
    uint32_t binf[BPT], bidx[BPT];
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int b = t + k * THREADS;
        binf[k] = 0u;
        bidx[k] = 0u;
        if (b < NBLK) {
            const int bx = b % NBS, by = b / NBS;
            const int lay = min(min(bx, NBS - 1 - bx), min(by, NBS - 1 - by));
            binf[k] = (uint32_t)(2 * by * EXT + 2 * bx) | ((uint32_t)(lay + 1) << 13) |
                      ((uint32_t)(bx == NBS - 1) << 19) | ((uint32_t)(by == NBS - 1) << 20);
            const int gy = wrapi(ty0 + 2 * by - HH, n);
            const int gx = wrapi(tx0 + 2 * bx - HH, n);   // even
            bidx[k] = ((uint32_t)(gx / 2) + ppr * (uint32_t)gy) | ((uint32_t)(gy == n - 1) << 31);
        }
    }
    const uint32_t wrap_back = ppr * (uint32_t)(n - 1);   // lower row index of a block on the last row: gx / 2
    __syncthreads();

    const float a = A.a, kappa = A.kf;
    for (int j = 0; j < A.ksteps; ++j) {
        const uint32_t m = (uint32_t)(A.m0 + j);
        // noise is needed on the flux region [j, EXT - j) and, for the fused coarse step, on the
        // blocks whose coarse cell is in the coarse tile plus its halo (ext [2, EXT - 2))
        const int lo = FUSED ? (j < 2 ? j : 2) : j;
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const uint32_t lay1 = (binf[k] >> 13) & 0x3Fu;          // 1 + distance in blocks; 0: no block
            if (lay1 <= (uint32_t)(lo >> 1)) continue;             // the block misses [lo, EXT - lo)
            const int c0 = (int)(binf[k] & 0x1FFFu);
            float w0[4], w1[4];
            const uint32_t idx0 = bidx[k] & 0x7FFFFFFFu;
            const uint32_t idx1 = (bidx[k] >> 31) ? idx0 - wrap_back : idx0 + ppr;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                float a0, a1, b0, b1;
                site_pair_normals(key, r == 0 ? idx0 : idx1, m, a0, a1, b0, b1);
                w0[2 * r] = a0; w1[2 * r] = a1; w0[2 * r + 1] = b0; w1[2 * r + 1] = b1;
            }
            if constexpr (FUSED) {
                if (lay1 >= 2u) {
                    Z[k][0] += (w0[0] + w0[1]) + (w0[2] + w0[3]);
                    Z[k][1] += (w1[0] + w1[1]) + (w1[2] + w1[3]);
                }
            } else if constexpr (SPLIT) {
                Z[k][0] += (w0[0] + w0[1]) + (w0[2] + w0[3]);
                Z[k][1] += (w1[0] + w1[1]) + (w1[2] + w1[3]);
            }
            // fluxes of all 4 cells: those outside this step's region get values no valid update reads
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c = c0 + (q & 1) + (q >> 1) * EXT;
                const float rv = sr[c];
                if (FLUX == DK_FLUX_CENTRAL) {
                    const float sq = psq(rv);
                    sf0[c] = sq * w0[q];
                    sf1[c] = sq * w1[q];
                } else {
                    const bool last_x = (q & 1) && ((binf[k] >> 19) & 1u), last_y = (q >> 1) && ((binf[k] >> 20) & 1u);
                    const float rx = sr[last_x ? c : c + 1];
                    const float ry = sr[last_y ? c : c + EXT];
                    sf0[c] = psq(0.5f * (rv + rx)) * w0[q];
                    sf1[c] = psq(0.5f * (rv + ry)) * w1[q];
                }
            }
        }
        if constexpr (SPLIT) {
            // a group of 4 fine steps is complete (D = 8: two per launch), or the launch ends
            if ((D == 8 && j == 3) || j == A.ksteps - 1) {
#pragma unroll
                for (int k = 0; k < BPT; ++k) {
                    const int b = t + k * THREADS;
                    const int bx = b % NBS, by = b / NBS;
                    if (((binf[k] >> 13) & 0x3Fu) > (uint32_t)HB) *zslot(bx, by, D == 8 ? (j >> 2) : 0) = make_float2(Z[k][0], Z[k][1]);
                    Z[k][0] = 0.f;
                    Z[k][1] = 0.f;
                }
            }
        }
        __syncthreads();
        // update region [j + 1, EXT - j - 1), one cell per deal slot
        float nv[CPT];
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int i = t + k * THREADS;
            nv[k] = 0.f;
            if (((clay[k / 4] >> (8 * (k % 4))) & 0xFFu) <= (uint32_t)j) continue;
            const int c = i;
            const float rv = sr[c];
            const float lap = fmaf(-4.0f, rv, (sr[c - 1] + sr[c + 1]) + (sr[c - EXT] + sr[c + EXT]));
            float div;
            if (FLUX == DK_FLUX_CENTRAL) div = (sf0[c + 1] - sf0[c - 1]) + (sf1[c + EXT] - sf1[c - EXT]);
            else div = (sf0[c] - sf0[c - 1]) + (sf1[c] - sf1[c - EXT]);
            const float d = fmaf(kappa, div, a * lap);
            const float y = d - cmp[k];
            const float tv = rv + y;
            cmp[k] = (tv - rv) - y;
            nv[k] = tv;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int i = t + k * THREADS;
            if (((clay[k / 4] >> (8 * (k % 4))) & 0xFFu) <= (uint32_t)j) continue;
            sr[i] = nv[k];
        }
        __syncthreads();
    }
    // write back the interior
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int i = t + k * THREADS;
        if (i >= NCELL) continue;
        const int ex = i % EXT, ey = i / EXT;
        if (ex < HH || ex >= EXT - HH || ey < HH || ey >= EXT - HH) continue;
        const size_t g = (size_t)(ty0 + ey - HH) * n + (tx0 + ex - HH);
        rout[g] = sr[i];
        cout[g] = cmp[k];
    }
    if constexpr (FUSED) {
        if (!A.do_coarse) return;
        // one coarse EM step with the restricted noise Z (coarse tile + 1 halo cell), reusing LDS
        const size_t ncc = (size_t)nc * nc;
        const float* rcin = A.rhoc_in + sidx * ncc;
        const float* ccin = A.cmpc_in + sidx * ncc;
        float* rcout = A.rhoc_out + sidx * ncc;
        float* ccout = A.cmpc_out + sidx * ncc;
        __syncthreads();
        float* scr = sr;                 // [CEXT][CEXT]
        float* scf0 = sf0;
        float* scf1 = sf1;
        for (int c = t; c < CEXT * CEXT; c += THREADS) {
            const int ex = c % CEXT, ey = c / CEXT;
            scr[c] = rcin[(size_t)wrapi(cy0 + ey - 1, nc) * nc + wrapi(cx0 + ex - 1, nc)];
        }
        __syncthreads();
        // fluxes of the coarse cells in the halo region: block (bx, by) <-> coarse ext (bx - 1, by - 1)
        const float kc = A.kc;
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const int b = t + k * THREADS;
            if (b >= NBLK) continue;
            const int bx = b % NBS, by = b / NBS;
            if (bx < 1 || bx >= NBS - 1 || by < 1 || by >= NBS - 1) continue;
            const int ex = bx - 1, ey = by - 1;
            const int c = ey * CEXT + ex;
            const float rv = scr[c];
            if (FLUX == DK_FLUX_CENTRAL) {
                const float sq = psq(rv);
                scf0[c] = sq * Z[k][0];
                scf1[c] = sq * Z[k][1];
            } else {
                const float rx = ex + 1 < CEXT ? scr[c + 1] : rv;
                const float ry = ey + 1 < CEXT ? scr[c + CEXT] : rv;
                scf0[c] = psq(0.5f * (rv + rx)) * Z[k][0];
                scf1[c] = psq(0.5f * (rv + ry)) * Z[k][1];
            }
        }
        __syncthreads();
        for (int c = t; c < CT * CT; c += THREADS) {
            const int ix = c % CT, iy = c / CT;
            const int e = (iy + 1) * CEXT + (ix + 1);
            const size_t g = (size_t)(cy0 + iy) * nc + (cx0 + ix);
            const float rv = scr[e];
            const float lap = fmaf(-4.0f, rv, (scr[e - 1] + scr[e + 1]) + (scr[e - CEXT] + scr[e + CEXT]));
            float div;
            if (FLUX == DK_FLUX_CENTRAL) div = (scf0[e + 1] - scf0[e - 1]) + (scf1[e + CEXT] - scf1[e - CEXT]);
            else div = (scf0[e] - scf0[e - 1]) + (scf1[e] - scf1[e - CEXT]);
            const float d = fmaf(kc, div, a * lap);
            const float cm = ccin[g];
            const float y = d - cm;
            const float tv = rv + y;
            rcout[g] = tv;
            ccout[g] = (tv - rv) - y;
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
