// dk_fourier.h -- launch interface of the Fourier-coupled level kernel (Sec. 3.1).
#pragma once
#include "dk_internal.h"

namespace dk {

// One batch of samples of one level of a Fourier-coupled hierarchy (n_l = n_0 3^l): single
// paths, or pairs (fine n, coarse n/3, 9 fine steps per coarse step).
struct FourierArgs {
    int nf;                 // fine grid points per axis
    int level_id;           // level number in the noise counter
    uint32_t tag;
    uint64_t seed;
    uint64_t first;         // first sample index
    uint64_t count;         // samples in this batch
    int steps;              // fine steps M_l (a multiple of 9 for pairs)
    int n_obs;
    double a;               // mu / 2 (both grids)
    double kf;              // fine noise coefficient per unit of the central difference of sqrt(rho+) z
    double kc;              // coarse coefficient per unit of the projected, summed normals
    double h2f, h2c;        // h^2 of the fine and coarse grid
    const void* rho0_f;     // I_h rho0 [nf*nf], state type
    const void* rho0_c;     // [nc*nc]
    const double* phi_f;    // I_h phi_j [n_obs][nf*nf]
    const double* phi_c;    // [n_obs][nc*nc]
    const double* obs_f;    // per observable {scale, centre, psi}, fine
    const double* obs_c;    // coarse
    const void* K;          // pairs: restriction kernel [nc][nf], state type
    void* scratch;          // pairs: per block [2 nf^2 + 2 nf nc] state-type elements
    double* out;            // [count][n_obs][2] (P_fine, P_coarse)
};

// Grid sizes with a compiled kernel (pairs need n divisible by 3 with n/3 even).
bool fourier_supported(int nf, bool pair);
// Blocks of one launch for `count` samples (each block strides over samples).
int fourier_grid(int nf, int precision, uint64_t count);
// State-type elements of pair scratch per block.
size_t fourier_scratch_elems(int nf);
hipError_t launch_fourier(const FourierArgs& A, int precision, bool pair, int grid, hipStream_t s);

}  // namespace dk
