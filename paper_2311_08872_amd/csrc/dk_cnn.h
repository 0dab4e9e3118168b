// dk_cnn.h -- launch interface of the control-variate network kernels (dk_cnn.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dk {
namespace cnn {

// flat FP32 parameter vector: W1 b1 W2 b2 W3 b3 U1 c1 U2 c2
constexpr int OFF_W1 = 0;      // [16][1][3][3]
constexpr int OFF_B1 = 144;
constexpr int OFF_W2 = 160;    // [16][16][3][3]
constexpr int OFF_B2 = 2464;
constexpr int OFF_W3 = 2480;
constexpr int OFF_B3 = 4784;
constexpr int OFF_U1 = 4800;   // [64][16]
constexpr int OFF_C1 = 5824;
constexpr int OFF_U2 = 5888;   // [1][64]
constexpr int OFF_C2 = 5952;
constexpr int NPARAM = 5953;

constexpr int kPixPerWave = 2048;   // pixels reduced by one wavefront in the weight-gradient GEMM
constexpr int kPixPerBlock = 1024;  // pixels per block in the bias / first-layer gradients

// Activation and gradient buffers for a batch of n x n inputs.
struct Workspace {
    int n = 0, batch = 0, nwaves = 0, nblk = 0;
    uint16_t *a1 = nullptr, *a2 = nullptr, *a3 = nullptr, *dz = nullptr, *dz2 = nullptr;   // BF16 [pixels][16]
    float *g = nullptr, *h1 = nullptr, *dg = nullptr, *sq = nullptr, *contrib = nullptr, *hsum = nullptr;
    float *partial = nullptr, *bpart = nullptr, *bsum = nullptr;
    uint16_t *wt2 = nullptr, *wb2 = nullptr, *wt3 = nullptr, *wb3 = nullptr;   // BF16 GEMM weights
    hipError_t reserve(int n, int batch);
    void release();
    ~Workspace() { release(); }
};

// BF16 GEMM weight layouts from the FP32 parameters (call after every parameter change).
hipError_t pack(Workspace& W, const float* prm, hipStream_t s);
// r[batch] = network(x[batch][n][n]); keeps the activations for backward().
hipError_t forward(Workspace& W, const float* prm, const float* x, int batch, float* r, hipStream_t s);
// grad[NPARAM] of mean_b (r_b - y_b)^2 after forward(); per-sample squared errors in W.sq.
hipError_t backward(Workspace& W, const float* prm, const float* x, const float* r, const float* y, int batch, float* grad,
                    hipStream_t s);
hipError_t adam_update(float* prm, const float* grad, float* m, float* v, float lr, int t, hipStream_t s);
// x = scale (rho - rho_bar), rho FP32 or FP64 fields [count][nn], rho_bar FP64 [nn]
hipError_t normalize(const void* rho, bool is_double, const double* rbar, int nn, size_t total, double scale, float* x,
                     hipStream_t s);

hipError_t extract_y(const double* ps, int nobs, int j, int count, float* y, hipStream_t s);
hipError_t combine_cv(const double* ps, int nobs, int j, const float* r, const float* rco, int k, int count, double* out,
                      hipStream_t s);
hipError_t accumulate_sq(const Workspace& W, int batch, double* acc, hipStream_t s);

}  // namespace cnn
}  // namespace dk
