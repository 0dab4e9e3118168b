// dk_cnn.hip -- the control-variate network on gfx950: forward, backward and Adam.
//
// Network (coarse final field -> prediction of the level correction Y):
//   conv 3x3 1->16 (circular) + ReLU, conv 3x3 16->16 + ReLU, conv 3x3 16->16 + ReLU,
//   global average pool, dense 16->64 + ReLU, dense 64->1.
// Parameters are FP32 masters, flat in the order W1 b1 W2 b2 W3 b3 U1 c1 U2 c2 with conv
// weights [o][c][ky][kx] and dense weights [out][in] (5953 values).
//
// The two 16->16 convolutions run as implicit GEMMs on v_mfma_f32_16x16x32_bf16: activations are
// BF16, pixel-major with the 16 channels contiguous ([pixel][16]); one wavefront computes a tile
// of 16 pixels x 16 output channels, K = 9 neighbour positions x 16 channels = 144, padded to 160
// (5 MFMAs).  The same kernel computes the input gradient (neighbours mirrored, weights stored
// [c][pos][o]).  Weight gradients are a second GEMM reducing over pixels (32 per MFMA) into
// per-wavefront partials that are summed in a fixed order.  The 1->16 convolution, pooling and
// the dense head are small and run on the vector ALU in FP32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dk_cnn.h"

namespace dk {
namespace cnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ int shifted_pixel(int P, int n, int dy, int dx)
{
    const int nn = n * n;
    const int b = P / nn;
    const int r = P - b * nn;
    const int y = r / n, x = r - (r / n) * n;
    int yy = y + dy, xx = x + dx;
    yy = yy < 0 ? yy + n : (yy >= n ? yy - n : yy);
    xx = xx < 0 ? xx + n : (xx >= n ? xx - n : xx);
    return b * nn + yy * n + xx;
}

// ---------------------------------------------------------------------------------------
// conv 1->16 (FP32 in, BF16 out), ReLU.  One thread per pixel.
// ---------------------------------------------------------------------------------------
__global__ void conv1_fwd(const float* __restrict__ x, const float* __restrict__ prm, uint16_t* __restrict__ a1, int n,
                          int npix)
{
    const int P = blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= npix) return;
    float v[9];
#pragma unroll
    for (int pos = 0; pos < 9; ++pos) v[pos] = x[shifted_pixel(P, n, pos / 3 - 1, pos % 3 - 1)];
    uint16_t o16[16];
#pragma unroll
    for (int o = 0; o < 16; ++o) {
        float s = prm[OFF_B1 + o];
#pragma unroll
        for (int pos = 0; pos < 9; ++pos) s = fmaf(prm[OFF_W1 + o * 9 + pos], v[pos], s);
        o16[o] = f2bf(fmaxf(s, 0.0f));
    }
    uint4* dst = (uint4*)(a1 + (size_t)P * 16);
    dst[0] = make_uint4(o16[0] | (o16[1] << 16), o16[2] | (o16[3] << 16), o16[4] | (o16[5] << 16), o16[6] | (o16[7] << 16));
    dst[1] = make_uint4(o16[8] | (o16[9] << 16), o16[10] | (o16[11] << 16), o16[12] | (o16[13] << 16),
                        o16[14] | (o16[15] << 16));
}

// ---------------------------------------------------------------------------------------
// Implicit-GEMM 3x3 16->16 convolution on MFMA.
//   MODE 0 (forward):        out[p][o] = ReLU(b[o] + sum_{pos,c} W[o][c][pos] in[p + d(pos)][c])
//   MODE 1 (input gradient): out[p][c] = mask(p,c) sum_{pos,o} W[o][c][pos] in[p - d(pos)][o]
// Wk: BF16 [16][160], row j holds the B-matrix column j: k = pos*16 + (c or o), zero-padded.
// One wavefront per 16-pixel tile, 4 wavefronts per block.
// ---------------------------------------------------------------------------------------
template <int MODE>
__global__ void __launch_bounds__(256) conv_gemm(const uint16_t* __restrict__ in, const uint16_t* __restrict__ Wk,
                                                 const float* __restrict__ bias, const uint16_t* __restrict__ mask,
                                                 uint16_t* __restrict__ out, int n, int npix)
{
    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile * 16 >= npix) return;
    const int i = lane & 15;
    const int kg = lane >> 4;
    const int P = tile * 16 + i;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        const int pos = 2 * s + (kg >> 1);
        uint4 av = make_uint4(0, 0, 0, 0);
        if (pos < 9) {
            int dy = pos / 3 - 1, dx = pos % 3 - 1;
            if (MODE == 1) { dy = -dy; dx = -dx; }
            const int q = shifted_pixel(P, n, dy, dx);
            av = *(const uint4*)(in + (size_t)q * 16 + 8 * (kg & 1));
        }
        const uint4 bv = *(const uint4*)(Wk + i * 160 + 32 * s + 8 * kg);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv),
                                                       acc, 0, 0, 0);
    }
    // D[row][col]: col = lane & 15 (output channel), rows 4 kg .. 4 kg + 3 (pixels of the tile)
    const int ch = lane & 15;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int Pr = tile * 16 + 4 * kg + r;
        float v = acc[r];
        if (MODE == 0) {
            v = fmaxf(v + bias[ch], 0.0f);
        } else {
            if (bf2f(mask[(size_t)Pr * 16 + ch]) <= 0.0f) v = 0.0f;
        }
        out[(size_t)Pr * 16 + ch] = f2bf(v);
    }
}

// ---------------------------------------------------------------------------------------
// Weight gradient of a 16->16 conv: dW[o][c][pos] = sum_p dz[p][o] x[p + d(pos)][c].
// GEMM with the reduction over pixels, 32 per MFMA; each wavefront reduces a pixel range into
// 9 accumulators (one per neighbour position) and writes a partial [9][16][16].
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) conv_dw(const uint16_t* __restrict__ x, const uint16_t* __restrict__ dz,
                                               float* __restrict__ partial, int n, int npix, int pix_per_wave)
{
    const int lane = threadIdx.x & 63;
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int p0 = w * pix_per_wave;
    if (p0 >= npix) return;
    const int p1 = min(npix, p0 + pix_per_wave);
    const int j = lane & 15;
    const int kg = lane >> 4;
    floatx4 acc[9];
#pragma unroll
    for (int pos = 0; pos < 9; ++pos) acc[pos] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int c0 = p0; c0 < p1; c0 += 32) {
        uint16_t a[8];
        int pix[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int P = c0 + 8 * kg + t;
            pix[t] = P;
            a[t] = P < p1 ? dz[(size_t)P * 16 + j] : (uint16_t)0;   // A[o = j][pixel]
        }
        const uint4 av = make_uint4(a[0] | (a[1] << 16), a[2] | (a[3] << 16), a[4] | (a[5] << 16), a[6] | (a[7] << 16));
        const bf16x8 A = __builtin_bit_cast(bf16x8, av);
#pragma unroll
        for (int pos = 0; pos < 9; ++pos) {
            uint16_t b[8];
#pragma unroll
            for (int t = 0; t < 8; ++t)
                b[t] = pix[t] < p1 ? x[(size_t)shifted_pixel(pix[t], n, pos / 3 - 1, pos % 3 - 1) * 16 + j] : (uint16_t)0;
            const uint4 bv = make_uint4(b[0] | (b[1] << 16), b[2] | (b[3] << 16), b[4] | (b[5] << 16), b[6] | (b[7] << 16));
            acc[pos] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, __builtin_bit_cast(bf16x8, bv), acc[pos], 0, 0, 0);
        }
    }
    // D[o][c]: c = lane & 15, o = 4 kg + r
#pragma unroll
    for (int pos = 0; pos < 9; ++pos)
#pragma unroll
        for (int r = 0; r < 4; ++r) partial[((size_t)w * 9 + pos) * 256 + (4 * kg + r) * 16 + j] = acc[pos][r];
}

// Sum partials [nw][9][16][16] in wavefront order into dW[o][c][pos] of the flat gradient.
__global__ void reduce_dw(const float* __restrict__ partial, int nw, float* __restrict__ grad, int off)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;   // over 9*256
    if (t >= 9 * 256) return;
    const int pos = t / 256, oc = t % 256, o = oc / 16, c = oc % 16;
    float s = 0.f;
    for (int w = 0; w < nw; ++w) s += partial[(size_t)w * 9 * 256 + t];
    grad[off + o * 144 + c * 9 + pos] = s;
}

// Column sums of a [rows][cols] matrix in row order (deterministic), into dst[cols].
__global__ void colsum(const float* __restrict__ m, int rows, int cols, float* __restrict__ dst)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int r = 0; r < rows; ++r) s += m[(size_t)r * cols + c];
    dst[c] = s;
}

// Per-block partial sums of dz (BF16 [npix][16]) over pixels: out[block][16] (bias gradients)
__global__ void bias_partial(const uint16_t* __restrict__ dz, int npix, int pix_per_block, float* __restrict__ out)
{
    __shared__ float sh[256];
    const int c = threadIdx.x & 15, lane16 = threadIdx.x >> 4;
    const int p0 = blockIdx.x * pix_per_block, p1 = min(npix, p0 + pix_per_block);
    float s = 0.f;
    for (int p = p0 + lane16; p < p1; p += 16) s += bf2f(dz[(size_t)p * 16 + c]);
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < 16) {
        float t = 0.f;
        for (int k = 0; k < 16; ++k) t += sh[k * 16 + threadIdx.x];
        out[blockIdx.x * 16 + threadIdx.x] = t;
    }
}

// conv1 weight/bias gradient partials: per block, thread t < 144 -> (o, pos), t in [144,160) -> db1
__global__ void conv1_dw(const float* __restrict__ x, const uint16_t* __restrict__ dz1, int n, int npix,
                         int pix_per_block, float* __restrict__ out /* [blocks][160] */)
{
    const int t = threadIdx.x;
    if (t >= 160) return;
    const int p0 = blockIdx.x * pix_per_block, p1 = min(npix, p0 + pix_per_block);
    float s = 0.f;
    if (t < 144) {
        const int o = t / 9, pos = t % 9;
        for (int p = p0; p < p1; ++p) s += bf2f(dz1[(size_t)p * 16 + o]) * x[shifted_pixel(p, n, pos / 3 - 1, pos % 3 - 1)];
    } else {
        const int o = t - 144;
        for (int p = p0; p < p1; ++p) s += bf2f(dz1[(size_t)p * 16 + o]);
    }
    out[blockIdx.x * 160 + t] = s;
}

// ---------------------------------------------------------------------------------------
// Pooling and dense head (FP32).
// ---------------------------------------------------------------------------------------
__global__ void pool(const uint16_t* __restrict__ a3, int nn, int batch, float* __restrict__ g)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;   // (sample, channel)
    if (t >= batch * 16) return;
    const int b = t / 16, c = t % 16;
    float s = 0.f;
    for (int p = 0; p < nn; ++p) s += bf2f(a3[((size_t)b * nn + p) * 16 + c]);
    g[t] = s / (float)nn;
}

__global__ void head_fwd(const float* __restrict__ g, const float* __restrict__ prm, int batch, float* __restrict__ h1,
                         float* __restrict__ r)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    float gi[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) gi[c] = g[b * 16 + c];
    float out = prm[OFF_C2];
    for (int k = 0; k < 64; ++k) {
        float s = prm[OFF_C1 + k];
#pragma unroll
        for (int c = 0; c < 16; ++c) s = fmaf(prm[OFF_U1 + k * 16 + c], gi[c], s);
        if (h1) h1[b * 64 + k] = s;
        out = fmaf(prm[OFF_U2 + k], fmaxf(s, 0.f), out);
    }
    r[b] = out;
}

// Per-sample head backward: gradient contributions [batch][GH] with GH = 64 (U2) + 1 (c2) +
// 1024 (U1) + 64 (c1); dg [batch][16]; loss terms (r - y)^2 [batch].
constexpr int GH = 64 + 1 + 1024 + 64;
__global__ void head_bwd(const float* __restrict__ g, const float* __restrict__ h1, const float* __restrict__ r,
                         const float* __restrict__ y, const float* __restrict__ prm, int batch, float* __restrict__ contrib,
                         float* __restrict__ dg, float* __restrict__ sq)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const float e = r[b] - y[b];
    sq[b] = e * e;
    const float dr = 2.0f * e / (float)batch;
    float* cb = contrib + (size_t)b * GH;
    float dgi[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) dgi[c] = 0.f;
    for (int k = 0; k < 64; ++k) {
        const float hk = h1[b * 64 + k];
        const float a4 = fmaxf(hk, 0.f);
        cb[k] = dr * a4;                                       // dU2
        const float dh = hk > 0.f ? dr * prm[OFF_U2 + k] : 0.f;
        cb[65 + 1024 + k] = dh;                                // dc1
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            cb[65 + k * 16 + c] = dh * g[b * 16 + c];          // dU1
            dgi[c] = fmaf(prm[OFF_U1 + k * 16 + c], dh, dgi[c]);
        }
    }
    cb[64] = dr;                                               // dc2
#pragma unroll
    for (int c = 0; c < 16; ++c) dg[b * 16 + c] = dgi[c];
}

// scatter the head gradient sums [GH] into the flat gradient
__global__ void head_scatter(const float* __restrict__ sums, float* __restrict__ grad)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= GH) return;
    if (t < 64) grad[OFF_U2 + t] = sums[t];
    else if (t == 64) grad[OFF_C2] = sums[t];
    else if (t < 65 + 1024) grad[OFF_U1 + (t - 65)] = sums[t];
    else grad[OFF_C1 + (t - 65 - 1024)] = sums[t];
}

// dz3[p][c] = dg[b][c] / nn * (a3[p][c] > 0)
__global__ void pool_bwd(const float* __restrict__ dg, const uint16_t* __restrict__ a3, int nn, int npix,
                         uint16_t* __restrict__ dz3)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npix * 16) return;
    const int p = t / 16, c = t % 16, b = p / nn;
    const float v = bf2f(a3[t]) > 0.f ? dg[b * 16 + c] / (float)nn : 0.f;
    dz3[t] = f2bf(v);
}

// place per-block partial sums [blocks][cols] into the gradient at off (after colsum)
__global__ void copy_to(const float* __restrict__ src, int n, float* __restrict__ dst, int off)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) dst[off + t] = src[t];
}

// conv1 partial layout [144 W1 (o*9+pos) | 16 b1] -> grad
__global__ void conv1_scatter(const float* __restrict__ sums, float* __restrict__ grad)
{
    const int t = threadIdx.x;
    if (t < 144) grad[OFF_W1 + t] = sums[t];
    else if (t < 160) grad[OFF_B1 + t - 144] = sums[t];
}

// Adam (Kingma & Ba) with bias correction; t is the 1-based step.
__global__ void adam(float* __restrict__ p, const float* __restrict__ gr, float* __restrict__ m, float* __restrict__ v,
                     int n, float lr, float b1, float b2, float eps, int t)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = gr[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float mh = mk / (1.f - powf(b1, (float)t));
    const float vh = vk / (1.f - powf(b2, (float)t));
    p[k] -= lr * mh / (sqrtf(vh) + eps);
}

// BF16 GEMM layouts of a 16->16 conv: fwd[o][pos*16+c], bwd[c][pos*16+o] (rows of 160)
__global__ void pack_weights(const float* __restrict__ prm, int off, uint16_t* __restrict__ fwd, uint16_t* __restrict__ bwd)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;   // 16 * 160
    if (t >= 16 * 160) return;
    const int row = t / 160, k = t % 160;
    if (k >= 144) { fwd[t] = 0; bwd[t] = 0; return; }
    const int pos = k / 16, col = k % 16;
    fwd[t] = f2bf(prm[off + row * 144 + col * 9 + pos]);   // W[o=row][c=col][pos]
    bwd[t] = f2bf(prm[off + col * 144 + row * 9 + pos]);   // W[o=col][c=row][pos]
}

// x = scale (rho - rho_bar) (FP32 or FP64 fields; rho_bar FP64 [nn])
__global__ void normalize_fields(const void* __restrict__ rho, int is_double, const double* __restrict__ rbar, int nn,
                                 size_t total, double scale, float* __restrict__ x)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const double v = is_double ? ((const double*)rho)[t] : (double)((const float*)rho)[t];
    x[t] = (float)(scale * (v - rbar[t % nn]));
}

// Y = P_f - P_c of observable j as float targets
__global__ void extract_y_kernel(const double* __restrict__ ps, int nobs, int j, int count, float* __restrict__ y)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    y[i] = (float)(ps[((size_t)i * nobs + j) * 2] - ps[((size_t)i * nobs + j) * 2 + 1]);
}

// Z_i = (Y_i - r_i) + (1/k) sum_{j<k} r'_{k i + j}, written as (Z, 0) pairs for the moment kernel
__global__ void combine_cv_kernel(const double* __restrict__ ps, int nobs, int jobs, const float* __restrict__ r,
                                  const float* __restrict__ rco, int k, int count, double* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const double y = ps[((size_t)i * nobs + jobs) * 2] - ps[((size_t)i * nobs + jobs) * 2 + 1];
    double m = 0.0;
    for (int t = 0; t < k; ++t) m += (double)rco[(size_t)i * k + t];
    out[2 * (size_t)i] = (y - (double)r[i]) + m / (double)k;
    out[2 * (size_t)i + 1] = 0.0;
}

hipError_t extract_y(const double* ps, int nobs, int j, int count, float* y, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(extract_y_kernel, dim3((count + 255) / 256), dim3(256), 0, s, ps, nobs, j, count, y);
    return hipGetLastError();
}

hipError_t combine_cv(const double* ps, int nobs, int j, const float* r, const float* rco, int k, int count, double* out,
                      hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(combine_cv_kernel, dim3((count + 255) / 256), dim3(256), 0, s, ps, nobs, j, r, rco, k, count, out);
    return hipGetLastError();
}

// sum of W.sq into acc[0] (ordered, one thread)
__global__ void sum_into(const float* __restrict__ v, int n, double* __restrict__ acc)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += (double)v[i];
    acc[0] += s;
}

hipError_t accumulate_sq(const Workspace& W, int batch, double* acc, hipStream_t s)
{
    hipLaunchKernelGGL(sum_into, dim3(1), dim3(64), 0, s, W.sq, batch, acc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Host-side launch sequences
// ---------------------------------------------------------------------------------------
static inline unsigned blocks_for(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t Workspace::reserve(int n_, int batch_)
{
    if (n_ == n && batch_ <= batch) return hipSuccess;
    release();
    n = n_;
    batch = batch_;
    const size_t npix = (size_t)batch * n * n;
    hipError_t e;
#define ALLOC(ptr, bytes) if ((e = hipMalloc((void**)&ptr, bytes)) != hipSuccess) return e
    ALLOC(a1, npix * 16 * 2);
    ALLOC(a2, npix * 16 * 2);
    ALLOC(a3, npix * 16 * 2);
    ALLOC(dz, npix * 16 * 2);
    ALLOC(dz2, npix * 16 * 2);
    ALLOC(g, (size_t)batch * 16 * 4);
    ALLOC(h1, (size_t)batch * 64 * 4);
    ALLOC(dg, (size_t)batch * 16 * 4);
    ALLOC(sq, (size_t)batch * 4);
    ALLOC(contrib, (size_t)batch * GH * 4);
    ALLOC(hsum, (size_t)GH * 4);
    nwaves = (int)((npix + kPixPerWave - 1) / kPixPerWave);
    ALLOC(partial, (size_t)nwaves * 9 * 256 * 4);
    nblk = (int)((npix + kPixPerBlock - 1) / kPixPerBlock);
    ALLOC(bpart, (size_t)nblk * 160 * 4);
    ALLOC(bsum, 160 * 4);
    ALLOC(wt2, 16 * 160 * 2);
    ALLOC(wb2, 16 * 160 * 2);
    ALLOC(wt3, 16 * 160 * 2);
    ALLOC(wb3, 16 * 160 * 2);
#undef ALLOC
    return hipSuccess;
}

void Workspace::release()
{
    void* ptrs[] = {a1, a2, a3, dz, dz2, g, h1, dg, sq, contrib, hsum, partial, bpart, bsum, wt2, wb2, wt3, wb3};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    a1 = a2 = a3 = dz = dz2 = nullptr;
    g = h1 = dg = sq = contrib = hsum = partial = bpart = bsum = nullptr;
    wt2 = wb2 = wt3 = wb3 = nullptr;
    n = batch = 0;
}

hipError_t pack(Workspace& W, const float* prm, hipStream_t s)
{
    hipLaunchKernelGGL(pack_weights, dim3(blocks_for(16 * 160, 256)), dim3(256), 0, s, prm, OFF_W2, W.wt2, W.wb2);
    hipLaunchKernelGGL(pack_weights, dim3(blocks_for(16 * 160, 256)), dim3(256), 0, s, prm, OFF_W3, W.wt3, W.wb3);
    return hipGetLastError();
}

hipError_t forward(Workspace& W, const float* prm, const float* x, int batch, float* r, hipStream_t s)
{
    const int n = W.n;
    const int npix = batch * n * n;
    hipLaunchKernelGGL(conv1_fwd, dim3(blocks_for(npix, 256)), dim3(256), 0, s, x, prm, W.a1, n, npix);
    const unsigned gb = blocks_for((size_t)npix / 16, 4);
    hipLaunchKernelGGL(conv_gemm<0>, dim3(gb), dim3(256), 0, s, W.a1, W.wt2, prm + OFF_B2, (const uint16_t*)nullptr, W.a2,
                       n, npix);
    hipLaunchKernelGGL(conv_gemm<0>, dim3(gb), dim3(256), 0, s, W.a2, W.wt3, prm + OFF_B3, (const uint16_t*)nullptr, W.a3,
                       n, npix);
    hipLaunchKernelGGL(pool, dim3(blocks_for((size_t)batch * 16, 256)), dim3(256), 0, s, W.a3, n * n, batch, W.g);
    hipLaunchKernelGGL(head_fwd, dim3(blocks_for(batch, 128)), dim3(128), 0, s, W.g, prm, batch, W.h1, r);
    return hipGetLastError();
}

hipError_t backward(Workspace& W, const float* prm, const float* x, const float* r, const float* y, int batch, float* grad,
                    hipStream_t s)
{
    const int n = W.n;
    const int nn = n * n;
    const int npix = batch * nn;
    hipLaunchKernelGGL(head_bwd, dim3(blocks_for(batch, 128)), dim3(128), 0, s, W.g, W.h1, r, y, prm, batch, W.contrib,
                       W.dg, W.sq);
    hipLaunchKernelGGL(colsum, dim3(blocks_for(GH, 256)), dim3(256), 0, s, W.contrib, batch, GH, W.hsum);
    hipLaunchKernelGGL(head_scatter, dim3(blocks_for(GH, 256)), dim3(256), 0, s, W.hsum, grad);
    // conv3
    hipLaunchKernelGGL(pool_bwd, dim3(blocks_for((size_t)npix * 16, 256)), dim3(256), 0, s, W.dg, W.a3, nn, npix, W.dz);
    const int nwaves = (npix + kPixPerWave - 1) / kPixPerWave;
    const int nblk = (npix + kPixPerBlock - 1) / kPixPerBlock;
    const unsigned gb = blocks_for((size_t)npix / 16, 4);
    hipLaunchKernelGGL(conv_dw, dim3(blocks_for(nwaves, 4)), dim3(256), 0, s, W.a2, W.dz, W.partial, n, npix, kPixPerWave);
    hipLaunchKernelGGL(reduce_dw, dim3(blocks_for(9 * 256, 256)), dim3(256), 0, s, W.partial, nwaves, grad, OFF_W3);
    hipLaunchKernelGGL(bias_partial, dim3(nblk), dim3(256), 0, s, W.dz, npix, kPixPerBlock, W.bpart);
    hipLaunchKernelGGL(colsum, dim3(1), dim3(64), 0, s, W.bpart, nblk, 16, W.bsum);
    hipLaunchKernelGGL(copy_to, dim3(1), dim3(64), 0, s, W.bsum, 16, grad, OFF_B3);
    hipLaunchKernelGGL(conv_gemm<1>, dim3(gb), dim3(256), 0, s, W.dz, W.wb3, (const float*)nullptr, W.a2, W.dz2, n, npix);
    // conv2 (dz2 holds the gradient at conv2's output, masked)
    hipLaunchKernelGGL(conv_dw, dim3(blocks_for(nwaves, 4)), dim3(256), 0, s, W.a1, W.dz2, W.partial, n, npix, kPixPerWave);
    hipLaunchKernelGGL(reduce_dw, dim3(blocks_for(9 * 256, 256)), dim3(256), 0, s, W.partial, nwaves, grad, OFF_W2);
    hipLaunchKernelGGL(bias_partial, dim3(nblk), dim3(256), 0, s, W.dz2, npix, kPixPerBlock, W.bpart);
    hipLaunchKernelGGL(colsum, dim3(1), dim3(64), 0, s, W.bpart, nblk, 16, W.bsum);
    hipLaunchKernelGGL(copy_to, dim3(1), dim3(64), 0, s, W.bsum, 16, grad, OFF_B2);
    hipLaunchKernelGGL(conv_gemm<1>, dim3(gb), dim3(256), 0, s, W.dz2, W.wb2, (const float*)nullptr, W.a1, W.dz, n, npix);
    // conv1 (dz holds the gradient at conv1's output, masked)
    hipLaunchKernelGGL(conv1_dw, dim3(nblk), dim3(256), 0, s, x, W.dz, n, npix, kPixPerBlock, W.bpart);
    hipLaunchKernelGGL(colsum, dim3(1), dim3(256), 0, s, W.bpart, nblk, 160, W.bsum);
    hipLaunchKernelGGL(conv1_scatter, dim3(1), dim3(256), 0, s, W.bsum, grad);
    return hipGetLastError();
}

hipError_t adam_update(float* prm, const float* grad, float* m, float* v, float lr, int t, hipStream_t s)
{
    hipLaunchKernelGGL(adam, dim3(blocks_for(NPARAM, 256)), dim3(256), 0, s, prm, grad, m, v, NPARAM, lr, 0.9f, 0.999f,
                       1e-8f, t);
    return hipGetLastError();
}

hipError_t normalize(const void* rho, bool is_double, const double* rbar, int nn, size_t total, double scale, float* x,
                     hipStream_t s)
{
    hipLaunchKernelGGL(normalize_fields, dim3(blocks_for(total, 256)), dim3(256), 0, s, rho, (int)is_double, rbar, nn, total,
                       scale, x);
    return hipGetLastError();
}

}  // namespace cnn
}  // namespace dk
