// dk_kernels.hip -- gfx950 kernels of the MLMC Dean--Kawasaki hot path: the resident level
// kernel (grids up to 128 x 128; its building blocks and the scheme it implements are described
// in dk_level.h), the ordered moment reduction, field evaluation, the noise dump and the FP64
// noise-free stepping of large grids.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "dk_internal.h"
#include "dk_level.h"
#include "dk_rng.h"

namespace dk {

// ---------------------------------------------------------------------------------------
// The resident level kernel: one block-iteration per block.
// ---------------------------------------------------------------------------------------
template <typename Real, int NF, int R, int C, bool PAIR, int FLUX, bool NOISE, int SPW>
__global__ void __launch_bounds__(SPW * (NF / C) * (NF / R))
level_kernel(const LevelArgs A)
{
    constexpr int TS = (NF / C) * (NF / R);
    __shared__ Real halo[SPW * halo_elems<NF, R, PAIR>()];
    __shared__ double red[(SPW * TS + 63) / 64];
    level_body<Real, NF, R, C, PAIR, FLUX, NOISE, SPW>(A, (uint64_t)blockIdx.x * SPW, halo, red, (int)threadIdx.x);
}

// ---------------------------------------------------------------------------------------
// Tile shapes.  A lane owns C = 2 columns and R rows; a sample uses (NF/2) x (NF/R) lanes and a
// block holds SPW samples (about 256 lanes, or four times as many samples in 1024-lane blocks).
// Several (R, SPW) per grid size are compiled for the FP32 noisy kernels; the host picks one by
// timing them (autotuning).  The other variants (FP64 state, noise-free mean field) use the
// first shape.
// ---------------------------------------------------------------------------------------
// rows per lane of shape variant v for grid size nf (0 = no such variant); variant 0 is the
// default (8 rows: the fastest measured on MI355X for every grid size of the hierarchy)
int shape_rows(int nf, int v)
{
    switch (nf) {
        case 4: return v == 0 ? 4 : 0;
        case 8: { const int r[] = {8, 2, 4, 8}; return v < 4 ? r[v] : 0; }
        case 16: { const int r[] = {8, 4, 2, 8}; return v < 4 ? r[v] : 0; }
        case 32: { const int r[] = {8, 4, 16, 8}; return v < 4 ? r[v] : 0; }
        case 64: { const int r[] = {8, 16, 8}; return v < 3 ? r[v] : 0; }
        case 128: { const int r[] = {8, 16}; return v < 2 ? r[v] : 0; }
        default: return 0;
    }
}

// samples per block of shape variant v (0 = no such variant): the last variant of 8^2 .. 64^2
// is the default shape with four times the samples per block
int shape_spw(int nf, int v)
{
    const int r = shape_rows(nf, v);
    if (r == 0) return 0;
    const int ts = (nf / 2) * (nf / r);
    const int base = ts >= 256 ? 1 : 256 / ts;
    const bool wide = (nf == 8 || nf == 16 || nf == 32) ? v == 3 : (nf == 64 ? v == 2 : false);
    return wide ? 4 * base : base;
}

template <typename Real, int NF, int R, bool PAIR, int FLUX, bool NOISE, int X = 1>
static hipError_t launch_R(const LevelArgs& A, hipStream_t s)
{
    using S = ShapeOf<NF, R, X>;
    const uint64_t blocks = (A.count + S::SPW - 1) / S::SPW;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL((level_kernel<Real, NF, R, S::C, PAIR, FLUX, NOISE, S::SPW>), dim3((unsigned)blocks),
                       dim3(S::SPW * S::TS), 0, s, A);
    return hipGetLastError();
}

template <typename Real, int NF, bool PAIR, int FLUX, bool NOISE>
static hipError_t launch_variants(const LevelArgs& A, int v, hipStream_t s)
{
    constexpr bool TUNED = std::is_same<Real, float>::value && NOISE;
    if (!TUNED) v = 0;
    if constexpr (NF == 4) {
        // 4 x 4 (the level 0 of the paper's own hierarchy): 2 lanes per sample, 4 rows each
        return launch_R<Real, 4, 4, PAIR, FLUX, NOISE>(A, s);
    } else if constexpr (NF == 8) {
        if constexpr (TUNED) {
            if (v == 1) return launch_R<Real, 8, 2, PAIR, FLUX, NOISE>(A, s);
            if (v == 2) return launch_R<Real, 8, 4, PAIR, FLUX, NOISE>(A, s);
            if (v == 3) return launch_R<Real, 8, 8, PAIR, FLUX, NOISE, 4>(A, s);
        }
        return launch_R<Real, 8, 8, PAIR, FLUX, NOISE>(A, s);
    } else if constexpr (NF == 16) {
        if constexpr (TUNED) {
            if (v == 1) return launch_R<Real, 16, 4, PAIR, FLUX, NOISE>(A, s);
            if (v == 2) return launch_R<Real, 16, 2, PAIR, FLUX, NOISE>(A, s);
            if (v == 3) return launch_R<Real, 16, 8, PAIR, FLUX, NOISE, 4>(A, s);
        }
        return launch_R<Real, 16, 8, PAIR, FLUX, NOISE>(A, s);
    } else if constexpr (NF == 32) {
        if constexpr (TUNED) {
            if (v == 1) return launch_R<Real, 32, 4, PAIR, FLUX, NOISE>(A, s);
            if (v == 2) return launch_R<Real, 32, 16, PAIR, FLUX, NOISE>(A, s);
            if (v == 3) return launch_R<Real, 32, 8, PAIR, FLUX, NOISE, 4>(A, s);
        }
        return launch_R<Real, 32, 8, PAIR, FLUX, NOISE>(A, s);
    } else if constexpr (NF == 64) {
        if constexpr (TUNED) {
            if (v == 1) return launch_R<Real, 64, 16, PAIR, FLUX, NOISE>(A, s);
            if (v == 2) return launch_R<Real, 64, 8, PAIR, FLUX, NOISE, 4>(A, s);
        }
        return launch_R<Real, 64, 8, PAIR, FLUX, NOISE>(A, s);
    } else {
        if constexpr (TUNED) {
            if (v == 1) return launch_R<Real, 128, 16, PAIR, FLUX, NOISE>(A, s);
            return launch_R<Real, 128, 8, PAIR, FLUX, NOISE>(A, s);
        } else {
            // FP64 states: 8-row groups would need more LDS than a CU has
            return launch_R<Real, 128, 16, PAIR, FLUX, NOISE>(A, s);
        }
    }
}

template <typename Real, bool PAIR, int FLUX, bool NOISE>
static hipError_t launch_nf(const LevelArgs& A, int v, hipStream_t s)
{
    switch (A.nf) {
        case 4: return launch_variants<Real, 4, PAIR, FLUX, NOISE>(A, v, s);
        case 8: return launch_variants<Real, 8, PAIR, FLUX, NOISE>(A, v, s);
        case 16: return launch_variants<Real, 16, PAIR, FLUX, NOISE>(A, v, s);
        case 32: return launch_variants<Real, 32, PAIR, FLUX, NOISE>(A, v, s);
        case 64: return launch_variants<Real, 64, PAIR, FLUX, NOISE>(A, v, s);
        case 128: return launch_variants<Real, 128, PAIR, FLUX, NOISE>(A, v, s);
        default: return hipErrorInvalidValue;
    }
}

bool level_supported(int nf) { return nf == 4 || nf == 8 || nf == 16 || nf == 32 || nf == 64 || nf == 128; }

hipError_t launch_level(const LevelKind& k, const LevelArgs& A, hipStream_t s)
{
    const int v = k.shape;
    if (!k.noise) {
        // noise-free FP64 mean field, single path
        return launch_nf<double, false, DK_FLUX_CENTRAL, false>(A, 0, s);
    }
    const bool f64 = k.precision == DK_PREC_F64;
    const bool stag = k.flux == DK_FLUX_STAGGERED;
    if (!f64 && !stag) return k.pair ? launch_nf<float, true, DK_FLUX_CENTRAL, true>(A, v, s)
                                     : launch_nf<float, false, DK_FLUX_CENTRAL, true>(A, v, s);
    if (!f64 && stag) return k.pair ? launch_nf<float, true, DK_FLUX_STAGGERED, true>(A, v, s)
                                    : launch_nf<float, false, DK_FLUX_STAGGERED, true>(A, v, s);
    if (f64 && !stag) return k.pair ? launch_nf<double, true, DK_FLUX_CENTRAL, true>(A, 0, s)
                                    : launch_nf<double, false, DK_FLUX_CENTRAL, true>(A, 0, s);
    return k.pair ? launch_nf<double, true, DK_FLUX_STAGGERED, true>(A, 0, s)
                  : launch_nf<double, false, DK_FLUX_STAGGERED, true>(A, 0, s);
}

// ---------------------------------------------------------------------------------------
// Ordered compensated moment sums.  One block per observable; thread k reduces a contiguous
// slice of samples in index order with Neumaier's compensated summation, then the slices
// are merged in a fixed pairwise tree.  The result depends only on (count, data).
// ---------------------------------------------------------------------------------------

constexpr int MOM_THREADS = 256;

__global__ void __launch_bounds__(MOM_THREADS) moments_kernel(const double* __restrict__ ps, uint64_t count, int n_obs,
                                                             double* __restrict__ out)
{
    const int j = blockIdx.x;
    const int t = threadIdx.x;
    const uint64_t per = (count + MOM_THREADS - 1) / MOM_THREADS;
    const uint64_t b = per * t, e = (b + per < count) ? b + per : count;
    double s[DK_NMOM], c[DK_NMOM];
#pragma unroll
    for (int k = 0; k < DK_NMOM; ++k) { s[k] = 0.0; c[k] = 0.0; }
    for (uint64_t i = b; i < e; ++i) {
        const double pf = ps[(i * n_obs + j) * 2 + 0];
        const double pc = ps[(i * n_obs + j) * 2 + 1];
        const double y = pf - pc;
        neumaier(s[DK_MOM_Y], c[DK_MOM_Y], y);
        neumaier(s[DK_MOM_Y2], c[DK_MOM_Y2], y * y);
        neumaier(s[DK_MOM_PF], c[DK_MOM_PF], pf);
        neumaier(s[DK_MOM_PF2], c[DK_MOM_PF2], pf * pf);
        neumaier(s[DK_MOM_PC], c[DK_MOM_PC], pc);
        neumaier(s[DK_MOM_PC2], c[DK_MOM_PC2], pc * pc);
    }
    __shared__ double sh[MOM_THREADS][2 * DK_NMOM];
#pragma unroll
    for (int k = 0; k < DK_NMOM; ++k) { sh[t][2 * k] = s[k]; sh[t][2 * k + 1] = c[k]; }
    __syncthreads();
    for (int w = MOM_THREADS / 2; w >= 1; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int k = 0; k < DK_NMOM; ++k) {
                double ss = sh[t][2 * k], cc = sh[t][2 * k + 1];
                neumaier(ss, cc, sh[t + w][2 * k]);
                cc += sh[t + w][2 * k + 1];
                sh[t][2 * k] = ss;
                sh[t][2 * k + 1] = cc;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
#pragma unroll
        for (int k = 0; k < DK_NMOM; ++k) {
            out[(j * DK_NMOM + k) * 2 + 0] = sh[0][2 * k];
            out[(j * DK_NMOM + k) * 2 + 1] = sh[0][2 * k + 1];
        }
    }
}

hipError_t launch_moments(const double* per_sample, uint64_t count, int n_obs, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(moments_kernel, dim3(n_obs), dim3(MOM_THREADS), 0, s, per_sample, count, n_obs, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Field evaluation (I_h of an analytic field), FP64.
// ---------------------------------------------------------------------------------------
__global__ void field_eval_kernel(const FieldDev f, double box, int n, void* out, int as_double)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    const int ix = idx % n, iy = idx / n;
    const double h = box / n;
    const double x = ix * h, y = iy * h;
    const double two_pi = 6.28318530717958647692;
    double v = f.c0;
    if (f.kind == DK_FIELD_MODES || f.kind == DK_FIELD_CLIPPED) {
        for (int k = 0; k < f.n_modes; ++k) v += f.amp[k] * cos(two_pi * (f.kx[k] * x + f.ky[k] * y) / box + f.phase[k]);
        if (f.kind == DK_FIELD_CLIPPED) v = fmax(v, 0.0) + f.floor_add;
    } else if (f.kind == DK_FIELD_BUMP) {
        double dx = fmod(fabs(x - f.bump_cx), box);
        dx = fmin(dx, box - dx);
        double dy = fmod(fabs(y - f.bump_cy), box);
        dy = fmin(dy, box - dy);
        v += f.bump_amp * exp(-(dx * dx + dy * dy) / (2.0 * f.bump_sigma * f.bump_sigma));
    } else {
        const double sx = sin(x - f.es_x0), sy = sin(y - f.es_y0);
        v = f.es_scale * (f.es_a + f.es_b * exp(-(sx * sx + sy * sy) / (2.0 * f.es_s)));
    }
    if (as_double) ((double*)out)[idx] = v;
    else ((float*)out)[idx] = (float)v;
}

hipError_t launch_field_eval(const FieldDev& f, double box, int n, void* out, bool as_double, hipStream_t s)
{
    const int total = n * n;
    hipLaunchKernelGGL(field_eval_kernel, dim3((total + 255) / 256), dim3(256), 0, s, f, box, n, out, (int)as_double);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Noise dump: out[sample][step][y][x][r] (one thread per site pair and step)
// ---------------------------------------------------------------------------------------
__global__ void noise_dump_kernel(uint64_t seed, uint32_t tag, int level, int n, uint64_t first_sample,
                                  uint32_t n_samples, int first_step, int n_steps, float* out)
{
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t pairs = (uint64_t)(n / 2) * n;
    const uint64_t total = pairs * n_steps * n_samples;
    if (idx >= total) return;
    const uint64_t p = idx % pairs;
    const uint64_t ms = (idx / pairs) % n_steps;
    const uint64_t si = idx / (pairs * n_steps);
    const NoiseKey key = make_key(seed, tag, level, first_sample + si);
    float a0, a1, b0, b1;
    site_pair_normals(key, (uint32_t)p, (uint32_t)(first_step + ms), a0, a1, b0, b1);
    const uint64_t y = p / (n / 2), x = 2 * (p % (n / 2));
    float* o = out + (((si * n_steps + ms) * n + y) * n + x) * 2;
    o[0] = a0;
    o[1] = a1;
    o[2] = b0;
    o[3] = b1;
}

hipError_t launch_noise_dump(uint64_t seed, uint32_t tag, int level, int n, uint64_t first_sample, uint32_t n_samples,
                             int first_step, int n_steps, float* out, hipStream_t s)
{
    const uint64_t total = (uint64_t)(n / 2) * n * n_steps * n_samples;
    if (total == 0) return hipSuccess;
    const uint64_t blocks = (total + 255) / 256;
    if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(noise_dump_kernel, dim3((unsigned)blocks), dim3(256), 0, s, seed, tag, level, n, first_sample,
                       n_samples, first_step, n_steps, out);
    return hipGetLastError();
}

__global__ void gauss_kernel(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b, uint64_t count,
                             float* __restrict__ z0, float* __restrict__ z1)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float u, v;
    box_muller(a[i], b[i], u, v);
    z0[i] = u;
    z1[i] = v;
}

hipError_t launch_gauss(const uint32_t* a, const uint32_t* b, uint64_t count, float* z0, float* z1, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    const uint64_t blocks = (count + 255) / 256;
    if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gauss_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, b, count, z0, z1);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Streaming noise-free FP64 step for large grids (one launch per step) and inner products.
// ---------------------------------------------------------------------------------------
__global__ void heat_step_kernel(const double* __restrict__ in, double* __restrict__ out, int n, double a)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= n) return;
    const int xm = x == 0 ? n - 1 : x - 1, xp = x == n - 1 ? 0 : x + 1;
    const int ym = y == 0 ? n - 1 : y - 1, yp = y == n - 1 ? 0 : y + 1;
    const double c = in[(size_t)y * n + x];
    const double lap = (in[(size_t)y * n + xm] + in[(size_t)y * n + xp]) + (in[(size_t)ym * n + x] + in[(size_t)yp * n + x]) - 4.0 * c;
    out[(size_t)y * n + x] = c + a * lap;
}

hipError_t launch_meanfield_stream(int n, double a, int steps, double* buf0, double* buf1, double** result, hipStream_t s)
{
    double* in = buf0;
    double* out = buf1;
    const dim3 grid((n + 255) / 256, n);
    for (int m = 0; m < steps; ++m) {
        hipLaunchKernelGGL(heat_step_kernel, grid, dim3(256), 0, s, in, out, n, a);
        double* t = in; in = out; out = t;
    }
    *result = in;
    return hipGetLastError();
}

__global__ void inner_kernel(const double* __restrict__ rho, int n, const double* __restrict__ phi, double h2,
                             double* __restrict__ out)
{
    const int j = blockIdx.x;
    const double* ph = phi + (size_t)j * n * n;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n * n; i += blockDim.x) acc = fma(rho[i], ph[i], acc);
    __shared__ double sh[256];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = h2 * sh[0];
}

hipError_t launch_inner_products(const double* rho, int n, const double* phi, int n_obs, double h2, double* out,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(inner_kernel, dim3(n_obs), dim3(256), 0, s, rho, n, phi, h2, out);
    return hipGetLastError();
}

}  // namespace dk
