// dk_stream.h -- launch interface of the HBM-streaming kernels (grids that do not fit on chip)
// and of the noise-free FP32 stencil.
#pragma once
#include "dk_internal.h"

namespace dk {

// Streaming level kernel (state in HBM, temporal blocking of depth 1, 2, 4 or 8 fine steps,
// 64 x 64 tiles), FP32 state.
struct StreamArgs {
    int n;                  // fine grid points per axis (a multiple of 64)
    int level_id;
    uint32_t tag;
    uint64_t seed;
    uint64_t first;         // first sample of the batch
    int count;              // samples in the batch (grid.y)
    int m0;                 // first fine step of this launch
    int ksteps;             // fine steps of this launch (1 .. depth; pairs: the launch ends on a step
                            // that a group of 4 ends on, or continues it at the next launch)
    int do_coarse;          // depth-4 pairs: 1 = take the coarse step after the fine steps
    int z_load;             // other pairs: 1 = the launch continues a group, load the running sums
    float* z;               // other pairs: restricted-noise sums, [groups][count][n/2][n/2] float pairs
    size_t zgroup;          // float pairs per group
    float a, kf, kc;
    const float *rho_in, *cmp_in;      // [count][n][n]
    float *rho_out, *cmp_out;
    const float *rhoc_in, *cmpc_in;    // [count][n/2][n/2]
    float *rhoc_out, *cmpc_out;
};
bool stream_supported(int nf);
hipError_t launch_heat_f32(const float* in, float* out, int n, int batch, float a, hipStream_t s);
bool stream_depth_supported(int depth);
hipError_t launch_stream_step(const StreamArgs& A, bool pair, int flux, int depth, hipStream_t s);
hipError_t launch_stream_coarse(int nc, int count, float a, float kc, int flux, const float* rho_in, const float* cmp_in,
                                const float* z, float* rho_out, float* cmp_out, hipStream_t s);
hipError_t launch_stream_init(const float* rho0, int n, int count, float* rho, float* cmp, hipStream_t s);
hipError_t launch_stream_copy(const float* a, const float* b, size_t total, float* a2, float* b2, hipStream_t s);
hipError_t launch_stream_observe(const float* rho, int n, int count, const double* phi, const double* obs, int n_obs,
                                 double h2, double* out, int slot, hipStream_t s);
hipError_t launch_zero_slot(double* out, int count, int n_obs, int slot, hipStream_t s);

}  // namespace dk
