/*
 * dk_mlmc.h -- C ABI of the MI355X (gfx950) MLMC Dean--Kawasaki hot path.
 *
 * Method: Cornalba & Fischer, "Multilevel Monte Carlo methods for the Dean--Kawasaki
 * equation from Fluctuating Hydrodynamics" (arXiv 2311.08872).
 *
 *   discrete model     Definition "def_discrete_DK", eq. (FullyDiscreteDK), explicit
 *                      Euler--Maruyama (b0 = 0, b1 = 1, Sec. 7) or any b0 in (0, 1]
 *                      (dk_problem.b0), V = 0, d = 2
 *   operators          5-point Laplacian and central divergence (Sec. 7, "Differential
 *                      operators"); DK_FLUX_STAGGERED selects a forward difference of edge
 *                      fluxes with the edge-averaged density under the square root
 *   level hierarchy    h_l = box / (n0 2^l) (box / (n0 3^l) for the Fourier coupling),
 *                      tau_l = mu h_l^2 (eq. cfl_preserved), M_l = T / tau_l steps
 *   coupling           NN ("Right-Most Nearest Neighbours"), Sec. 3.2: coarse Brownian
 *                      increments are 2^{-d/2} times the sum of the fine increments over the
 *                      2x2 right-most block and over the 4 fine steps of one coarse step;
 *                      or Fourier, Sec. 3.1 (h_{l-1} = 3 h_l; DK_COUPLING_FOURIER below)
 *   observables        P_l of eq. (eqn_MLMCLevels): psi( s ((rho_l^T, I_h phi)_h - c_l) ),
 *                      c_l = (rho_bar_l^T, I_h phi)_h from the discrete mean field (Sec. 3)
 *   estimator          eq. (MLMCEstimator) and Algorithm 1 (Sec. 7) with eq. (opt_M_ell)
 *                      and eq. (convergence_criterion)
 *
 * Noise: Philox4x32-10 (Salmon et al., SC'11) keyed by the problem seed, with counter
 *   (site pair a + (n/2) y, fine step m, sample bits 0..31,
 *    tag << 24 | level << 16 | sample bits 32..47),
 * followed by a Box--Muller transform evaluated as a fixed sequence of correctly rounded
 * binary32 operations; words (0,1) give the two directions of site (2a, y), words (2,3)
 * those of site (2a + 1, y).  The normals are therefore a pure function of
 * (seed, tag, level, sample, site, step) and do not depend on launch shape or batching.
 *
 * Conventions for every entry point:
 *   - all structs are caller-owned and only read during the call;
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream); device outputs are
 *     written stream-ordered; host outputs are complete when the call returns;
 *   - return value: 0 = success, > 0 = warning with a valid result, < 0 = error (outputs
 *     unspecified, inputs untouched); dk_last_error() describes the last error of the
 *     calling thread;
 *   - no C++ exception crosses this interface.
 */
#ifndef DK_MLMC_H
#define DK_MLMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define DK_OK 0
#define DK_WARN_NOT_CONVERGED 1   /* Algorithm 1 reached the last level without passing the bias test */
#define DK_EINVAL (-1)            /* invalid argument or problem */
#define DK_ENOMEM (-2)            /* device or host allocation failed */
#define DK_EDEVICE (-3)           /* HIP runtime error */
#define DK_ENUMERIC (-4)          /* non-finite sample values */
#define DK_EUNSUPPORTED (-5)      /* valid request outside what this build implements */

/* ---- enums ---- */
#define DK_FIELD_MODES 0      /* c0 + sum amp cos(2 pi (kx x + ky y)/box + phase)            */
#define DK_FIELD_CLIPPED 1    /* max(0, c0 + sum modes) + floor_add                            */
#define DK_FIELD_BUMP 2       /* c0 + bump_amp exp(-|x - c|_per^2 / (2 sigma^2))               */
#define DK_FIELD_EXPSIN2 3    /* es_scale (es_a + es_b exp(-(sin^2(x-x0) + sin^2(y-y0))/(2 es_s))) */

#define DK_PSI_ID 0
#define DK_PSI_SQUARE 1

#define DK_FLUX_CENTRAL 0     /* central divergence of node fluxes (the paper's Sec. 7) */
#define DK_FLUX_STAGGERED 1   /* forward divergence of edge fluxes                      */

#define DK_STEPS_EXACT 0      /* EINVAL unless T / tau_0 is an integer            */
#define DK_STEPS_ROUND_T 1    /* M_0 = round(T / tau_0); effective T = M_0 tau_0   */

#define DK_PREC_F32 0         /* FP32 density state (default) */
#define DK_PREC_F64 1         /* FP64 density state           */

#define DK_TAG_MLMC 0         /* noise stream tags */
#define DK_TAG_MC 1
#define DK_TAG_CV_TRAIN 2     /* training pairs of the control variate              */
#define DK_TAG_CV_COARSE 3    /* independent coarse-only paths of the control variate */

#define DK_COST_CELLS 0       /* dk_mlmc_opts.cost_model: cell updates per sample (deterministic) */
#define DK_COST_MEASURED 1    /*                          measured kernel seconds per sample      */

#define DK_CNN_NPARAM 5953    /* parameters of the control-variate network */

#define DK_MAX_OBS 64
#define DK_MAX_LEVELS 12
#define DK_MAX_MODES 64

/* Level coupling (Sec. 3).  NN: right-most nearest neighbours, h_{l-1} = 2 h_l, tau_{l-1} =
 * 4 tau_l (Sec. 3.2; every kernel).  FOURIER: h_{l-1} = 3 h_l, tau_{l-1} = 9 tau_l (Sec. 3.1):
 * grids n_l = n0 3^l with n0 in {4, 8} up to 108 x 108 (FP32 or FP64 state, central flux);
 * the fine level runs the same nodal noise as every level, the coarse level the fine normals
 * summed over its 9 fine steps and projected onto the coarse frequencies (on the coarse
 * Nyquist frequency the two fine aliases enter with weight 2^{-1/2}), read at the coarse
 * nodes.  Pair cost: n^2 M (1 + 1/81) cell updates; the bias test of Algorithm 1 uses ratio
 * 3 in place of 2. */
#define DK_COUPLING_NN 0
#define DK_COUPLING_FOURIER 1

/* Grid points.  VERTEX: x_i = i h on [0, box), so a coarse point is the fine point (2a, 2b)
 * and the NN block B->(x) = {x + h v, v in {0,1}^2} lies to its right (Sec. 3.2).  CELL:
 * x_i = (i + 1/2) h, the symmetric variant of the NN coupling that the remark after Sec. 3.2
 * describes (coupling unchanged, every coarse point the centre of its 2 x 2 fine block).  Only
 * the sampling of rho0 and phi changes; NN coupling only. */
#define DK_GRID_VERTEX 0
#define DK_GRID_CELL 1

/* ---- problem statement (Sec. 2, Sec. 3, Sec. 7) ---- */
typedef struct { double amp, kx, ky, phase; } dk_mode;

typedef struct {
    int32_t kind;             /* DK_FIELD_*                                */
    int32_t n_modes;          /* <= DK_MAX_MODES                           */
    double c0;
    const dk_mode* modes;     /* host array [n_modes]                      */
    double floor_add;
    double bump_amp, bump_sigma, bump_cx, bump_cy;
    double es_a, es_b, es_s, es_x0, es_y0, es_scale;
} dk_field;

typedef struct {
    dk_field phi;             /* test function phi, evaluated at grid points (I_h)       */
    int32_t centre;           /* 1: subtract (rho_bar_l^T, I_h phi)_h (discrete mean field) */
    int32_t scale_sqrtN;      /* 1: multiply by N^{1/2}                                   */
    int32_t psi;              /* DK_PSI_ID or DK_PSI_SQUARE                              */
    int32_t reserved;
} dk_obs;

typedef struct {
    int32_t d;                /* must be 2                                                 */
    int32_t n0;               /* points per axis on level 0 (even, >= 4)                  */
    int32_t levels;           /* number of levels L_max + 1 (<= DK_MAX_LEVELS)            */
    int32_t steps_policy;     /* DK_STEPS_*                                                */
    double box;               /* torus side length                                          */
    double mu;                /* tau_l / h_l^2, 0 < mu <= 1/d (explicit stability)          */
    double T;                 /* final time                                                 */
    double N;                 /* particle number, > 0                                       */
    int32_t flux;             /* DK_FLUX_*                                                  */
    int32_t precision;        /* DK_PREC_*                                                  */
    int32_t n_obs;            /* 1 .. DK_MAX_OBS                                            */
    int32_t primary_obs;      /* observable that drives Algorithm 1                         */
    const dk_obs* obs;        /* host array [n_obs]                                         */
    dk_field rho0;            /* initial mean-field profile; rho^0 = I_h rho0 on every level */
    uint64_t seed;            /* Philox key                                                 */
    int32_t coupling;         /* DK_COUPLING_NN (default) or DK_COUPLING_FOURIER           */
    int32_t grid;             /* DK_GRID_VERTEX (default) or DK_GRID_CELL                  */
    double b0;                /* implicit weight of eq. (FullyDiscreteDK), b1 = 1 - b0, in
                                 [0, 1]; 0 (default) is the explicit scheme of Sec. 7.  b0 > 0:
                                 NN coupling, central flux, grids up to 64 x 64, stable for
                                 mu (1 - 2 b0) <= 1/2 (any mu once b0 >= 1/2); each step
                                 filters the explicit increment with (I - tau b0/2 Lap_h)^{-1}
                                 by an FFT per step and grid (Appendix A, operator A_h)     */
} dk_problem;

/* ---- per-level moment sums ---- */
#define DK_MOM_Y 0     /* sum of Y = P_fine - P_coarse (P_coarse = 0 on level 0 / plain MC) */
#define DK_MOM_Y2 1
#define DK_MOM_PF 2
#define DK_MOM_PF2 3
#define DK_MOM_PC 4
#define DK_MOM_PC2 5
#define DK_NMOM 6

typedef struct {
    uint64_t count;
    double sum[DK_NMOM];      /* compensated sums: value = sum + comp */
    double comp[DK_NMOM];
} dk_moments;

/* Sample mean and unbiased sample variance (denominator count - 1; 0 when count = 1) of one
 * quantity of a moment record, from its compensated sums: q = 0 for Y = P_fine - P_coarse, 1 for
 * P_fine, 2 for P_coarse (the estimates of eq. (MLMCEstimator) and the V_l of eq. (opt_M_ell)).
 * Host arithmetic only.  DK_EINVAL for NULL pointers, q outside 0..2 or a record without samples. */
int dk_moments_mean_var(const dk_moments* m, int32_t q, double* mean, double* var);

typedef struct {
    int32_t m_pilot;          /* pilot samples per level (Algorithm 1's M-bar); default 1000     */
    int32_t L_start;          /* first L (default 2)                                             */
    double alpha;             /* weak order in the bias test (default 2)                          */
    int32_t max_rounds;       /* safety cap on Algorithm-1 rounds (default 1000)                  */
    int32_t plain_mc_level;   /* >= 0: run plain MC on this level instead of MLMC                 */
    uint64_t max_samples;     /* cap on total samples of one level (0 = none)                     */
    const float* cv_params;   /* host [levels][DK_CNN_NPARAM] network parameters, or NULL         */
    uint32_t cv_level_mask;   /* bit l set: level l >= 1 uses the learned control variate         */
    int32_t cv_ratio;         /* independent coarse-only paths per pair (default 4)               */
    int32_t round_mode;       /* 0: levels one after another (per-launch timing);
                                 1: each round's levels concurrently, one stream per level;
                                 2: as 1, captured into a hipGraph launched once per round;
                                 3: persistent: the round's resident FP32 levels in one launch of
                                    one 1024-lane block per compute unit pulling (level, sample
                                    range) tasks, finest level first, from a device counter; the
                                    launch is a hipGraph captured once per context and replayed
                                    (rounds above about 2e12 cell updates take one launch per
                                    2e12).  Other levels run as in mode 0; FP64 problems run as
                                    in mode 1.
                                 Modes 0-2 give identical results; mode 3 uses 8 rows per lane and
                                 sums moments per task, so its results agree with mode 0's to
                                 rounding (per-sample paths are the same).                         */
    int32_t cost_model;       /* DK_COST_CELLS (0, default): C_l = fine + coarse cell updates per
                                 sample, so the M_l are a function of the samples alone;
                                 DK_COST_MEASURED (1): C_l = measured kernel seconds per sample of
                                 level l (HIP events of the previous rounds; levels not yet run use
                                 the cell count scaled by the last measured level's time per cell
                                 update).  Faster levels then get more samples; the M_l depend on
                                 timings.  Rounds whose kernels are not timed per level (the
                                 persistent round, round_mode 3) keep the cell model.            */
    const char* checkpoint_path; /* NULL, or a file for Algorithm-1 checkpoints: after every round
                                 the state (levels, samples done and targeted, compensated sums) is
                                 written to path.tmp and renamed over path.  A run that finds the
                                 file resumes after its last round and gives bit-identical results
                                 to an uninterrupted run; a file of another run (problem, eps or
                                 options differ) gives DK_EINVAL.  MLMC only (not plain MC).      */
} dk_mlmc_opts;

typedef struct {
    double estimate[DK_MAX_OBS];   /* MLMC (or MC) estimate of E[P_L] per observable           */
    double var_est[DK_MAX_OBS];    /* estimator variance sum_l V_l / M_l per observable        */
    double bias_est;               /* bias estimate of the primary observable (remainder term) */
    double rmse_est;               /* sqrt(var_est[primary] + bias_est^2)                      */
    int32_t L;                     /* finest level used                                         */
    int32_t converged;             /* 1 if the bias test passed                                 */
    int32_t rounds;                /* Algorithm-1 rounds                                        */
    int32_t reserved;
    uint64_t M[DK_MAX_LEVELS];     /* samples per level                                          */
    double Yhat[DK_MAX_LEVELS];    /* mean of Y_l, primary observable                            */
    double Vhat[DK_MAX_LEVELS];    /* unbiased variance of Y_l, primary observable               */
    double cost[DK_MAX_LEVELS];    /* C_l used by the last round: cell updates per sample, or
                                      seconds per sample with DK_COST_MEASURED                   */
    double cell_updates;           /* total fine + coarse cell updates performed                 */
    double wall_s;                 /* host wall time of the call                                 */
} dk_mlmc_result;

typedef struct dk_context dk_context;

/* Create a context on HIP device `device` (owns device workspace, per-problem level tables,
 * cached centring constants and tuning choices).  One context per host thread. */
int dk_context_create(dk_context** out, int device);
void dk_context_destroy(dk_context* ctx);

/* One batch of level-l samples [first_sample, first_sample + n_samples) of the MLMC hierarchy:
 * l = 0: single level-0 paths (Y = P_0); l >= 1: NN-coupled pairs (fine l, coarse l-1),
 * Y = P_l - P_{l-1} (Sec. 3.2, eq. MLMCEstimator).  stream_tag selects an independent noise
 * stream (DK_TAG_MLMC for the estimator).
 *   sums_out        host, caller-owned [n_obs]; receives the moment sums of this batch.
 *   per_sample_out  optional DEVICE pointer [n_samples][n_obs][2] of doubles
 *                   (P_fine, P_coarse), or NULL.
 * Samples of any batch split give the same per-sample values. */
int dk_mlmc_level_pair(dk_context* ctx, const dk_problem* problem, int32_t level,
                       uint64_t first_sample, uint64_t n_samples, uint32_t stream_tag,
                       dk_moments* sums_out, double* per_sample_out, void* stream);

/* Allocation-free variant of dk_mlmc_level_pair, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments and results without the context: runs on the current device and calls no hipMalloc,
 * hipFree or other allocating routine.  Its workspace (level tables, the centring run, one chunk of
 * per-sample values, chunk moments) is a fixed 32 MiB device array that each GPU the library runs
 * on holds until the process ends; calls on one GPU share it, so calls that overlap on one GPU
 * (other host threads, or other streams still running an earlier call) race.  Every table is
 * rebuilt on each call (no cache; the noise-free centring run adds about one sample's time).
 * Resident levels only (grids up to 128 x 128), explicit NN scheme; the default tile shape.
 * Per-sample values equal dk_mlmc_level_pair's; moment sums may be grouped in other chunks
 * (rounding-level differences).  Errors: as dk_mlmc_level_pair, plus DK_EINVAL when the level's
 * tables and one chunk of per-sample values do not fit the 32 MiB (e.g. 128 x 128 with more than
 * about 190 observables, never within DK_MAX_OBS) and DK_EUNSUPPORTED for streamed grids, the
 * Fourier coupling or b0 > 0. */
int dk_mlmc_level_pair_noalloc(const dk_problem* problem, int32_t level, uint64_t first_sample,
                               uint64_t n_samples, uint32_t stream_tag, dk_moments* sums_out,
                               double* per_sample_out, void* stream);

/* Plain (single-level) Monte Carlo batch on level l (the baseline of Sec. 7): uncoupled
 * paths with the DK_TAG_MC stream; per_sample_out as above with P_coarse = 0. */
int dk_mc_level(dk_context* ctx, const dk_problem* problem, int32_t level,
                uint64_t first_sample, uint64_t n_samples,
                dk_moments* sums_out, double* per_sample_out, void* stream);

/* One round of Algorithm 1 (Sec. 7) without the algorithm around it: samples
 * [first[l], first[l] + count[l]) of every level l <= L (level 0 single paths, l >= 1 pairs
 * coupled by the NN restriction of Sec. 3.2) from noise stream `tag` (0-255), run as
 * round_mode (0-3, as in dk_mlmc_opts) would run them.  first, count: host [L + 1]; sample
 * indices < 2^48; count[l] = 0 skips level l.  sums_out: host [(L + 1) * n_obs], moments per
 * level and observable (zero where count is 0).  For callers that drive their own estimator
 * loop; results do not depend on round_mode except as stated for mode 3.  Errors: DK_EINVAL
 * for bad arguments; device errors as for dk_mlmc_level_pair. */
int dk_mlmc_round(dk_context* ctx, const dk_problem* problem, int32_t L, const uint64_t* first, const uint64_t* count,
                  uint32_t tag, int32_t round_mode, dk_moments* sums_out, void* stream);

/* Algorithm 1 of Sec. 7 to RMSE eps on the GPU (or plain MC when opts->plain_mc_level >= 0).
 * opts may be NULL (defaults).  level_moments: optional host array [levels][n_obs].
 * Returns DK_WARN_NOT_CONVERGED when the last level is reached without passing the bias test. */
int dk_mlmc_estimate(dk_context* ctx, const dk_problem* problem, double eps,
                     const dk_mlmc_opts* opts, dk_mlmc_result* out,
                     dk_moments* level_moments, void* stream);

/* Centring constants c_{l,j} = (rho_bar_l^M, I_h phi_j)_h of the discrete mean field
 * (noise-free FP64 run of the scheme from I_h rho0, Sec. 3).  centre_out: host [n_obs];
 * rho_out: optional DEVICE pointer [n_l * n_l] doubles (x fastest) for the final field. */
int dk_meanfield(dk_context* ctx, const dk_problem* problem, int32_t level,
                 double* centre_out, double* rho_out, void* stream);

/* The standard normals of the generator: out (DEVICE, floats) [n_samples][n_steps][n][n][2],
 * indexed [sample][step][y][x][direction], for samples first_sample.. and steps
 * first_step.. of an n x n grid (n even) on level `level` with the given tag. */
int dk_noise_dump(dk_context* ctx, uint64_t seed, uint32_t tag, int32_t level, int32_t n,
                  uint64_t first_sample, uint32_t n_samples, int32_t first_step,
                  int32_t n_steps, float* out, void* stream);

/* The generator's Gaussian transform alone (Box-Muller, Sec. 7's standard normals; the fixed
 * binary32 sequence documented with the generator): for i < count, (z0[i], z1[i]) are the two
 * normals of the Philox output words (a[i], b[i]), a the radius word and b the angle word, as
 * used for every site.  a, b, z0, z1: DEVICE arrays of count elements.  For parity checks of
 * the transform over chosen words (e.g. every radius word); DK_EINVAL on NULL arrays. */
int dk_gauss_transform(dk_context* ctx, const uint32_t* a, const uint32_t* b, uint64_t count,
                       float* z0, float* z1, void* stream);

/* Final density fields of a batch (for field-level checks): rho_f_out [n_samples][n_l^2] and,
 * for coupled pairs, rho_c_out [n_samples][n_{l-1}^2], DEVICE, element type float for
 * DK_PREC_F32 and double for DK_PREC_F64.  coupled = 0 runs uncoupled level-l paths. */
int dk_level_fields(dk_context* ctx, const dk_problem* problem, int32_t level, int32_t coupled,
                    uint64_t first_sample, uint64_t n_samples, uint32_t stream_tag,
                    double* per_sample_out, void* rho_f_out, void* rho_c_out, void* stream);

/* Host-only Algorithm 1 (Sec. 7) over a caller-supplied level sampler; no GPU is touched.
 * The sampler adds `count` samples of level l starting at sample index `first` and writes
 * sum Y and sum Y^2 (primary observable) into sums[0], sums[1]; it returns 0 or an error
 * code, which aborts the run.  cost[l] is C_l.  result->M, Yhat, Vhat, L, converged,
 * rounds, estimate[0], var_est[0], bias_est and rmse_est are filled. */
typedef int (*dk_level_sampler)(void* user, int32_t level, uint64_t first, uint64_t count,
                                double* sums);
int dk_alg1_host(double eps, int32_t L_max, const double* cost, const dk_mlmc_opts* opts,
                 dk_level_sampler sampler, void* user, dk_mlmc_result* out);

/* ---- learned control variate (an extension of the method; plain MLMC stays the fallback) ----
 * For a level l >= 1 with network r (coarse final field -> prediction of Y_l), each MLMC sample
 * of level l is Z = (Y_l - r(x_c)) + (1/k) sum_{j<k} r(x'_j) with x_c the pair's normalised coarse
 * field and x'_j from k independent level-(l-1) paths (stream DK_TAG_CV_COARSE, sample indices
 * k i + j).  E[Z] = E[Y_l] for any fixed r, so the estimator stays unbiased; its variance is
 * Var(Y - r) + Var(r)/k.  Inputs are x = N^{1/2} h_c (rho_c^T - rho_bar_c^T).
 * The network: conv3x3 1->16, 16->16, 16->16 (circular, ReLU), global mean, dense 16->64 (ReLU),
 * dense 64->1; parameters flat FP32 in the order W1 b1 W2 b2 W3 b3 U1 c1 U2 c2 with conv weights
 * [out][in][ky][kx] and dense weights [out][in].  The 16->16 layers run on BF16 MFMA with FP32
 * accumulation; the rest in FP32. */

/* Seeded He initialisation of the network parameters (host only). */
int dk_cnn_init(uint64_t seed, float* params_out);

/* r[b] = network(x[b]) for x DEVICE [batch][n][n] floats (n a multiple of 4), r DEVICE [batch]. */
int dk_cnn_forward(dk_context* ctx, const float* params, int32_t n, int32_t batch, const float* x, float* r,
                   void* stream);

/* Mean squared error of the network on (x, y) (DEVICE [batch][n][n], [batch]) and its gradient
 * with respect to the parameters (host [DK_CNN_NPARAM]). */
int dk_cnn_loss_grad(dk_context* ctx, const float* params, int32_t n, int32_t batch, const float* x, const float* y,
                     float* grad_out, double* loss_out, void* stream);

/* Train the network for level `level` >= 1 with Adam on n_train coupled pairs drawn from the
 * DK_TAG_CV_TRAIN stream (targets Y of the primary observable, standardised internally; the
 * scaling is folded into the last layer).  params_inout: host [DK_CNN_NPARAM], the initial values
 * on entry.  loss_hist: optional host [epochs] (mean squared error on the standardised targets).
 * val_out: optional host [3] = {Var(Y), Var(Y - r), Var(r)} on n_val further training-stream
 * pairs (0 = skip). */
int dk_cv_train(dk_context* ctx, const dk_problem* problem, int32_t level, uint64_t n_train, int32_t epochs,
                int32_t batch, double lr, uint64_t n_val, float* params_inout, double* loss_hist, double* val_out,
                void* stream);

/* Per-kernel timing of a context, measured with HIP events around every level-kernel launch
 * on the caller's stream (for profiling and roofline reports).  One record per
 * (level, coupled) pair that ran since the last reset.  The persistent round kernel
 * (round_mode 3) has the record with level = -1 (its launches, samples, time and cell updates
 * over all levels); the per-level records of its samples carry samples and cell updates with
 * no launches or time. */
typedef struct {
    int32_t level;            /* fine level                                  */
    int32_t coupled;          /* 1 for NN-coupled pairs                      */
    uint64_t launches;        /* kernel launches                             */
    uint64_t samples;         /* samples (or pairs) computed                 */
    double kernel_ms;         /* summed event time of the launches           */
    double cell_updates;      /* fine + coarse cell updates                  */
    int32_t rows;             /* rows per lane of the tile shape used; -D for  */
                              /* the streaming kernel at temporal depth D      */
    int32_t reserved;
} dk_kernel_stats;

/* Copies up to max records into out and returns the number of records (>= 0). */
int dk_context_stats(dk_context* ctx, dk_kernel_stats* out, int32_t max);
/* Clears the records; also drops cached level tables and tuning choices when drop_tables != 0. */
int dk_context_reset(dk_context* ctx, int32_t drop_tables);

/* Tile shapes of the resident kernel: a lane owns 2 columns and R rows of an n x n grid, and a
 * block holds S samples (about 256 lanes, or four times as many samples in 1024-lane blocks).
 * dk_shape_rows(n, v) gives R of variant v and dk_shape_spw(n, v) its S (both 0 if the variant
 * does not exist).  By default the
 * context times the variants on a short batch the first time a large job (>= 1e11 cell updates)
 * runs a grid size, and keeps the fastest; dk_context_set_shape forces variant v for grid size
 * n (v < 0 restores the automatic choice).  Per-sample fields do not depend on the shape; the
 * observables' FP64 lane reduction order does (last-bit differences). */
int dk_context_set_shape(dk_context* ctx, int32_t n, int32_t variant);
int dk_shape_rows(int32_t n, int32_t variant);
int dk_shape_spw(int32_t n, int32_t variant);

/* The autotuner's tile-shape and streaming-depth choices of the context (and those loaded) as
 * JSON text:
 *   {"format": "dk-tile-shapes-1", "arch": "gfx950",
 *    "shapes": [{"n": 128, "pair": 1, "flux": 0, "rows": 8, "spw": 1}, {"n": 1024, "pair": 1,
 *               "flux": 0, "depth": 4}, ...]}
 * ("spw" may be left out of a shape entry: it then names the ~256-lane shape with that R)
 * Writes at most cap bytes including the terminating NUL into buf (buf may be NULL when cap is
 * 0) and returns the text's full length without the NUL, or a negative error code. */
int dk_context_tuning_json(dk_context* ctx, char* buf, uint64_t cap);
/* Loads choices in that format; listed shapes replace the context's choices and are used
 * without timing.  DK_EINVAL if the text lacks the format tag, names another architecture,
 * lists a row count (and samples per block) that no compiled shape of that grid has, or a depth
 * other than 1, 2, 4, 8.
 * With the environment variable DK_TUNE_CACHE set to a file path, every context loads that file
 * when it is created (if it exists and is valid) and rewrites it whenever the autotuner makes a
 * new choice. */
int dk_context_load_tuning_json(dk_context* ctx, const char* json);

/* Grids larger than 128 x 128 (multiples of 64) run on the streaming kernel: the FP32 state
 * stays in HBM (double-buffered), each launch advances 64 x 64 tiles with a halo of max(D, 2)
 * cells by D fine steps (temporal depth D in {1, 2, 4, 8}), regenerating the halo's noise.  For
 * pairs the coarse step (Sec. 4, one per 4 fine steps) is fused into the launch at D = 4; at the
 * other depths the restricted-noise sums go through HBM and a coarse kernel takes the step.  Its
 * fields are bit-identical to the resident kernel's at every depth.  dk_context_set_streaming(ctx,
 * 1) routes every level of size >= 64 through it (for comparison); field output is not
 * available there. */
int dk_context_set_streaming(dk_context* ctx, int32_t on);
/* Temporal depth of the streaming kernel: 1, 2, 4 or 8 forces it for every streamed level; 0
 * (the default) times the four depths on a short batch (16 fine steps, up to 64 samples) the
 * first time a job of >= 1e11 cell updates runs a grid size, keeps the fastest (listed in the
 * tuning JSON as {"n": .., "pair": .., "flux": .., "depth": D}) and uses depth 4 for smaller
 * jobs.  DK_EINVAL for other values.  The depth changes no result. */
int dk_context_set_stream_depth(dk_context* ctx, int32_t depth);

/* Largest work of one sampling launch, in fine + coarse cell updates (default 2e12, about 5 s
 * on MI355X; 0 restores the default, values below 1e6 are raised to 1e6).  Longer levels are
 * split into more launches and persistent rounds into more segments (graph replays); moment
 * sums are then grouped differently (rounding-level differences only). */
int dk_context_set_launch_cap(dk_context* ctx, double cells);

/* Noise-free scheme (rho <- rho + (mu/2) Lap_h rho, the discrete mean-field dynamics of Sec. 3)
 * for `steps` steps on a batch of FP32 fields rho (DEVICE [batch][n][n], updated in place;
 * work: DEVICE scratch of the same size).  n a multiple of 4.  kernel_ms (optional) receives
 * the event time of the steps.  Memory-bound: 8 B of HBM traffic per cell update. */
int dk_heat_steps(dk_context* ctx, int32_t n, int32_t batch, int32_t steps, double mu, float* rho, float* work,
                  double* kernel_ms, void* stream);

/* Description of the last error on the calling thread (static storage, never NULL). */
const char* dk_last_error(void);

/* Library version string. */
const char* dk_version(void);

/* sizeof of dk_mode, dk_field, dk_obs, dk_problem, dk_moments, dk_mlmc_opts, dk_mlmc_result,
 * dk_kernel_stats (in that order) into out[0..n); returns the number of entries (bindings
 * use it to check their struct layouts). */
int dk_abi_sizes(int32_t* out, int32_t n);

#ifdef __cplusplus
}
#endif
#endif /* DK_MLMC_H */
