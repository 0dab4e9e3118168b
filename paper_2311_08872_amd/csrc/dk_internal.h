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
// samples per block of tile-shape variant v for grid size nf, 0 if the variant does not exist
int shape_spw(int nf, int v);

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
hipError_t launch_gauss(const uint32_t* a, const uint32_t* b, uint64_t count, float* z0, float* z1, hipStream_t s);

// Noise-free FP64 stepping for grids that do not fit on chip: one launch per step.
hipError_t launch_meanfield_stream(int n, double a, int steps, double* buf0, double* buf1,
                                   double** result, hipStream_t s);
hipError_t launch_inner_products(const double* rho, int n, const double* phi, int n_obs, double h2,
                                 double* out, hipStream_t s);

// Host side of the allocation-free level batch (dk_arena.cpp): samples [first, first + count) of
// resident level `level` (a pair for level >= 1) with every device buffer, the level tables and
// the centring run included, carved from `arena` (device, arena_bytes, 256-byte aligned); returns a
// dk status (DK_EINVAL when the tables and one chunk of per-sample values do not fit).
int level_pair_arena(const dk_problem* p, int level, uint64_t first, uint64_t count, uint32_t tag, dk_moments* sums_out,
                     double* per_sample_out, void* arena, size_t arena_bytes, hipStream_t s);
// Sets the calling thread's dk_last_error() text and returns code.
int set_error(int code, const char* msg);

}  // namespace dk
