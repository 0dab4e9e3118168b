// dk_internal.h -- launch interface between the host driver and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dk_mlmc.h"

namespace dk {

// One batch of samples of one level (single paths or NN-coupled pairs).
struct LevelArgs {
    int nf;                 // fine grid points per axis
    int level_id;           // level number in the noise counter
    uint32_t tag;           // noise stream tag
    uint64_t seed;
    uint64_t first;         // first sample index
    uint64_t count;         // samples in this batch
    int steps;              // fine steps M_l
    double a;               // mu / 2 (both grids)
    double kf;              // fine noise coefficient
    double kc;              // coarse noise coefficient (per unit of the restricted sum)
    double h2f, h2c;        // h^d on the fine and coarse grid
    const void* rho0_f;     // I_h rho0 on the fine grid [nf*nf], element type = state type
    const void* rho0_c;     // on the coarse grid [nf*nf/4]
    const double* phi_f;    // I_h phi_j on the fine grid [n_obs][nf*nf]
    const double* phi_c;    // [n_obs][nf*nf/4]
    const double* obs_f;    // per observable: {scale, centre (0 if uncentred), psi} x n_obs, fine
    const double* obs_c;    // same for the coarse level
    int n_obs;
    double* out;            // [count][n_obs][2] (P_fine, P_coarse)
    void* field_f;          // optional final fine fields [count][nf*nf]
    void* field_c;          // optional final coarse fields [count][nf*nf/4]
};

// Kernel selection flags
struct LevelKind {
    int precision;          // DK_PREC_*
    bool pair;              // coupled fine/coarse pair
    int flux;               // DK_FLUX_*
    bool noise;             // false: noise-free mean-field run
    int shape = 0;          // tile-shape variant (FP32 noisy kernels; see shape_rows)
};

// Returns hipSuccess, or hipErrorInvalidValue when no kernel exists for the size.
hipError_t launch_level(const LevelKind& k, const LevelArgs& a, hipStream_t s);
bool level_supported(int nf);
// rows per lane of tile-shape variant v for grid size nf, 0 if the variant does not exist
int shape_rows(int nf, int v);

// Ordered, compensated per-observable moment sums of a per-sample buffer.
// out: device [n_obs][DK_NMOM][2] (sum, compensation).
hipError_t launch_moments(const double* per_sample, uint64_t count, int n_obs, double* out,
                          hipStream_t s);

// Analytic field on the n x n grid (FP64 evaluation), stored as float or double.
struct FieldDev {
    int kind, n_modes;
    double c0, floor_add, bump_amp, bump_sigma, bump_cx, bump_cy;
    double es_a, es_b, es_s, es_x0, es_y0, es_scale;
    double amp[DK_MAX_MODES], kx[DK_MAX_MODES], ky[DK_MAX_MODES], phase[DK_MAX_MODES];
};
hipError_t launch_field_eval(const FieldDev& f, double box, int n, void* out, bool as_double,
                             hipStream_t s);

hipError_t launch_noise_dump(uint64_t seed, uint32_t tag, int level, int n, uint64_t first_sample,
                             uint32_t n_samples, int first_step, int n_steps, float* out,
                             hipStream_t s);

// Streaming level kernel (state in HBM, 4-step temporal blocking, 64 x 64 tiles), FP32 state.
struct StreamArgs {
    int n;                  // fine grid points per axis (a multiple of 64)
    int level_id;
    uint32_t tag;
    uint64_t seed;
    uint64_t first;         // first sample of the batch
    int count;              // samples in the batch (grid.y)
    int m0;                 // first fine step of this launch
    int ksteps;             // fine steps of this launch (4 for pairs)
    int do_coarse;          // pairs: 1 = take the coarse step after the fine steps
    float a, kf, kc;
    const float *rho_in, *cmp_in;      // [count][n][n]
    float *rho_out, *cmp_out;
    const float *rhoc_in, *cmpc_in;    // [count][n/2][n/2]
    float *rhoc_out, *cmpc_out;
};
bool stream_supported(int nf);
hipError_t launch_heat_f32(const float* in, float* out, int n, int batch, float a, hipStream_t s);
hipError_t launch_stream_step(const StreamArgs& A, bool pair, int flux, hipStream_t s);
hipError_t launch_stream_init(const float* rho0, int n, int count, float* rho, float* cmp, hipStream_t s);
hipError_t launch_stream_copy(const float* a, const float* b, size_t total, float* a2, float* b2, hipStream_t s);
hipError_t launch_stream_observe(const float* rho, int n, int count, const double* phi, const double* obs, int n_obs,
                                 double h2, double* out, int slot, hipStream_t s);
hipError_t launch_zero_slot(double* out, int count, int n_obs, int slot, hipStream_t s);

// Persistent round kernel: all resident levels of one Algorithm-1 round in one launch.
struct RoundLevel {
    LevelArgs A;            // the level's tables and coefficients (first, count, out unused)
    int kind;               // round_kind(nf, pair)
    int spw;                // samples per block-iteration, round_spw_of(nf)
};
struct RoundTask {
    uint32_t level;         // index into RoundArgs::levels
    uint32_t pad;
    uint64_t first;         // first sample index (absolute) of the task
    uint64_t count;         // samples of the task
};
struct RoundArgs {
    const RoundLevel* levels;   // device
    const RoundTask* tasks;     // device, in the order they are handed out
    const uint32_t* ntasks;     // device scalar
    uint32_t* head;             // device queue counter (reset by the launch)
    double* task_mom;           // device [ntasks][n_obs][DK_NMOM][2] (sum, compensation)
    double* scratch;            // device [grid][scratch_stride] per-sample values of a block-iteration
    uint64_t scratch_stride;    // doubles per block, >= 256 * n_obs * 2
    int n_obs;
};
int round_kind(int nf, bool pair);
int round_spw_of(int nf);
int round_blocks_per_cu(int flux);
int round_max_obs();
// Resets the queue counter, then launches `grid` blocks of the round kernel.
hipError_t launch_round(const RoundArgs& P, int flux, int grid, hipStream_t s);

// Noise-free FP64 stepping for grids that do not fit on chip: one launch per step.
hipError_t launch_meanfield_stream(int n, double a, int steps, double* buf0, double* buf1,
                                   double** result, hipStream_t s);
hipError_t launch_inner_products(const double* rho, int n, const double* phi, int n_obs, double h2,
                                 double* out, hipStream_t s);

}  // namespace dk
