// dk_theta.h -- launch interface of the general-weight (b0 > 0) level kernel.
#pragma once
#include "dk_internal.h"

namespace dk {

// One batch of samples of one level of eq. (FullyDiscreteDK) with b0 > 0: single paths, or NN
// pairs (fine n, coarse n/2, 4 fine steps per coarse step).
struct ThetaArgs {
    int n;                  // fine grid points per axis (4 .. 64, a power of two)
    int level_id;
    uint32_t tag;
    uint64_t seed;
    uint64_t first;
    uint64_t count;
    int steps;              // fine steps (a multiple of 4 for pairs)
    int n_obs;
    double a;               // mu / 2
    double kf, kc;          // noise coefficients (fine; coarse per unit of the restricted sum)
    double h2f, h2c;
    const void* rho0_f;     // I_h rho0, state type
    const void* rho0_c;
    const double* phi_f;
    const double* phi_c;
    const double* obs_f;
    const double* obs_c;
    const void* tw;         // exp(-2 pi i k / n), k < n/2: [n/2][2] (re, im), state type
    const void* sol_f;      // 1 / (1 + 2 b0 mu (sin^2(pi kx/n) + sin^2(pi ky/n))) [n][n], state type
    const void* sol_c;      // the same on the coarse grid [n/2][n/2]
    double* out;            // [count][n_obs][2]
};

bool theta_supported(int n, bool pair);
int theta_grid(int n, int precision, uint64_t count);
hipError_t launch_theta(const ThetaArgs& A, int precision, bool pair, int grid, hipStream_t s);

}  // namespace dk
