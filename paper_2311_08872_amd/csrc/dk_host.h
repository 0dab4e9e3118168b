// dk_host.h -- declarations shared by the host-side sources of the library (not part of the
// C ABI): error reporting, problem geometry and validation, device buffers and level tables, the
// context behind the opaque dk_context handle, and the level drivers, rounds, Algorithm 1 and
// samplers that the C ABI calls.
//
//   dk_host_common.cpp  errors, compensated sums, problem hashing and validation, field tables
//   dk_levels.cpp       level tables and centring, one level's batches (resident, streamed,
//                       Fourier-coupled, semi-implicit)
//   dk_tuning.cpp       tile-shape choice and its JSON cache
//   dk_rounds.cpp       whole Algorithm-1 rounds (concurrent streams, hipGraph, persistent kernel)
//   dk_alg1.cpp         Algorithm 1 of Sec. 7 and its checkpoints
//   dk_samplers.cpp     the GPU samplers Algorithm 1 drives, the learned control variate
//   dk_arena.cpp        the allocation-free level batch
//   dk_api.cpp          the C ABI: argument checks and dispatch
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "dk_cnn.h"
#include "dk_fourier.h"
#include "dk_internal.h"
#include "dk_round.h"
#include "dk_stream.h"
#include "dk_theta.h"

namespace dkh {

// Records the message returned by dk_last_error (per thread) and returns code.
int fail(int code, const char* fmt, ...);
const char* last_error();

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return ::dkh::fail(DK_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Compensated (Neumaier) accumulation on the host, used to merge ordered partial sums.
void nadd(double& s, double& c, double x);
void merge_moments(dk_moments& dst, const double* part /* [DK_NMOM][2] */, uint64_t count);
double mom_value(const dk_moments& m, int k);

// Problem geometry and validation.
uint64_t problem_hash(const dk_problem* p);
int validate(const dk_problem* p);
long steps0_of(const dk_problem* p);            // steps on level 0, or a negative error code
bool fourier(const dk_problem* p);
bool implicit(const dk_problem* p);
int level_ratio(const dk_problem* p);           // h_{l-1} / h_l: 2 (NN coupling) or 3 (Fourier)
int level_n(const dk_problem* p, int l);
long level_steps(const dk_problem* p, long steps0, int l);
double pair_factor(const dk_problem* p);        // coarse work of a pair relative to its fine work
dk::FieldDev to_dev_on(const dk_problem* p, const dk_field& f, int n);

// device buffer owned by the context
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ~DevBuf() { if (p) (void)hipFree(p); }
    int ensure(size_t n)
    {
        if (n <= bytes) return DK_OK;
        if (p) { (void)hipFree(p); p = nullptr; bytes = 0; }
        if (hipMalloc(&p, n) != hipSuccess) return fail(DK_ENOMEM, "hipMalloc(%zu) failed", n);
        bytes = n;
        return DK_OK;
    }
};

struct LevelTables {
    int n = 0;
    double h = 0, tau = 0;
    long steps = 0;
    DevBuf rho0;      // state type
    DevBuf phi;       // double [n_obs][n*n]
    DevBuf obs;       // double [n_obs][3] {scale, centre, psi}
    std::vector<double> centre;   // c_{l,j} (0 where not centred)
    bool have_centre = false;
    DevBuf rbar;                  // FP64 discrete mean field at the final time [n*n]
    bool have_rbar = false;
    DevBuf fourier_K;             // Fourier pairs with this fine level: projection kernel [n/3][n], state type
    DevBuf theta_tw, theta_sol;   // b0 > 0: twiddles exp(-2 pi i k/n) [n/2][2] and the solve multipliers [n][n]
};

struct ProblemTables {
    std::vector<std::unique_ptr<LevelTables>> level;
};

constexpr double kMaxCellsPerLaunch = 2e12;   // default cap: about 5 s of kernel time per launch

struct KStat {
    uint64_t launches = 0, samples = 0;
    double ms = 0, cells = 0;
    int rows = 0;
};

}  // namespace dkh

struct dk_context {
    int device = 0;
    std::map<std::pair<int, int>, dkh::KStat> stats;
    std::map<int, int> forced_shape;          // grid size -> tile-shape variant
    bool force_stream = false;                // run every level with the streaming kernel
    int stream_depth = 0;                     // forced temporal depth of the streaming kernel (0: automatic)
    std::map<long, int> tuned_depth;          // (nf, pair, flux) -> streaming depth chosen by timing
    double max_launch_cells = dkh::kMaxCellsPerLaunch;   // work cap of one sampling launch
    // concurrent rounds: one stream per level, fork/join events, per-level buffers
    hipStream_t lvl_stream[DK_MAX_LEVELS] = {};
    hipEvent_t fork_ev = nullptr, join_ev[DK_MAX_LEVELS] = {};
    dkh::DevBuf rnd_ps[DK_MAX_LEVELS], rnd_mom[DK_MAX_LEVELS];
    hipEvent_t rnd_t0 = nullptr, rnd_t1 = nullptr;
    hipStream_t cap_stream = nullptr;         // private stream that round graphs are captured on
    double round_ms = 0;
    uint64_t round_graphs = 0;
    // persistent rounds: device tables, the queue counter, per-task moments, per-block scratch,
    // pinned staging, and the captured graph (reset + round kernel) replayed for every segment
    dkh::DevBuf pr_levels, pr_tasks, pr_ntasks, pr_head, pr_task_mom, pr_scratch;
    void* pr_host = nullptr;
    size_t pr_host_bytes = 0;
    hipGraph_t pr_graph = nullptr;
    hipGraphExec_t pr_exec = nullptr;
    dk::RoundArgs pr_args{};
    int pr_flux = -1, pr_grid = 0;
    hipEvent_t pr_t0 = nullptr, pr_t1 = nullptr;
    std::map<long, int> tuned;                // (nf, pair, flux) -> variant chosen by timing
    std::vector<std::pair<int, double>> tune_log;   // (variant, ms) of the last tuning
    std::vector<hipEvent_t> ev_pool;
    dkh::DevBuf per_sample;     // chunk buffer of per-sample outputs
    dkh::DevBuf moments;        // [chunks][n_obs][DK_NMOM][2]
    dkh::DevBuf mf0, mf1;       // mean-field streaming buffers
    dkh::DevBuf scratch_c;      // inner products
    dkh::DevBuf st_f[2][2], st_c[2][2];   // streaming state: [buffer][rho, cmp] fine / coarse
    dkh::DevBuf st_z;                     // streaming pairs: restricted-noise sums of split depths
    dkh::DevBuf fourier_scratch;          // Fourier pairs: per-block sums and half-projected sums
    std::vector<double> host_mom;
    // learned control variate
    dk::cnn::Workspace cnn;
    dkh::DevBuf cv_prm, cv_grad, cv_m, cv_v, cv_loss;
    dkh::DevBuf cv_fields, cv_x, cv_r, cv_y, cv_ps, cv_ps2, cv_z, cv_fields2, cv_x2, cv_r2;
    std::map<uint64_t, std::unique_ptr<dkh::ProblemTables>> problems;
};

namespace dkh {

// Level tables, centring constants and the batching of one level (dk_levels.cpp).
double noise_coeff(const dk_problem* p, double h, double sigma);
int ensure_level(dk_context* ctx, const dk_problem* p, int level, LevelTables** out, hipStream_t s);
int compute_centre(dk_context* ctx, const dk_problem* p, int level, LevelTables& T, hipStream_t s, double* rho_out);
uint64_t chunk_size(int n_obs, double cells_per_sample, double max_cells);
int run_level(dk_context* ctx, const dk_problem* p, int level, bool pair, uint64_t first, uint64_t count,
              uint32_t tag, dk_moments* sums_out, double* per_sample_out, void* field_f, void* field_c,
              hipStream_t s, double* cell_updates);
int level_args(dk_context* ctx, const dk_problem* p, int l, bool pair, uint32_t tag, hipStream_t s, dk::LevelArgs* out,
               double* cells_per_sample);

// Tile shapes (dk_tuning.cpp).
std::string tuning_json(const dk_context* ctx);
int load_tuning_json(dk_context* ctx, const std::string& text);
void save_tuning_cache(const dk_context* ctx);
int choose_shape(dk_context* ctx, const dk_problem* p, bool pair, const dk::LevelArgs& A, uint64_t count,
                 double cells_per_sample, hipStream_t s, int* variant);

// Whole rounds (dk_rounds.cpp); sums [(L+1) * n_obs].
int run_round(dk_context* ctx, const dk_problem* p, int L, const uint64_t* first, const uint64_t* count, uint32_t tag,
              int mode, std::vector<dk_moments>& sums, hipStream_t s, double* cell_updates);
bool round_eligible(const dk_problem* p, int l, bool force_stream);
int run_round_persistent(dk_context* ctx, const dk_problem* p, int L, const uint64_t* first, const uint64_t* count,
                         uint32_t tag, std::vector<dk_moments>& sums, hipStream_t s, double* cell_updates);

// Algorithm 1 (dk_alg1.cpp).
dk_mlmc_opts default_opts();
struct CkptHooks {
    uint64_t key = 0;                                         // identifies the run
    std::function<void(std::vector<double>&)> save;           // extra sampler state
    std::function<int(const std::vector<double>&)> load;
};

struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void bytes(const void* p, size_t n)
    {
        const unsigned char* c = (const unsigned char*)p;
        for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
    }
    template <class T> void val(const T& v) { bytes(&v, sizeof(v)); }
};

// optional: all levels of one round at once; sums [L+1][2]
typedef int (*round_sampler)(void* user, int L, const uint64_t* first, const uint64_t* count, double* sums);

// measure(L, C): optional; with DK_COST_MEASURED it replaces C[0..L] by measured costs after a round
typedef std::function<void(int, std::vector<double>&)> cost_measure;

int alg1_core(double eps, int L_max, const double* cost, const dk_mlmc_opts& o, dk_level_sampler sampler, void* user,
              dk_mlmc_result* out, round_sampler rsampler = nullptr, const CkptHooks* ck = nullptr,
              const cost_measure* measure = nullptr, double ratio = 2.0);

// Samplers and the learned control variate (dk_samplers.cpp).
int ensure_rbar(dk_context* ctx, const dk_problem* p, int level, LevelTables** out, hipStream_t s);
int cnn_forward_batched(dk_context* ctx, const float* prm, int n, uint64_t count, const float* x, float* r, hipStream_t s);
int run_cv_level(dk_context* ctx, const dk_problem* p, int level, uint64_t first, uint64_t count, const float* prm_host,
                 int kappa, dk_moments* sums_out, dk_moments& zsum, hipStream_t s, double* cell_updates);
struct GpuSampler {
    dk_context* ctx = nullptr;
    const dk_problem* p = nullptr;
    hipStream_t s = nullptr;
    uint32_t tag = DK_TAG_MLMC;
    bool plain_mc = false;
    std::vector<dk_moments> mom;   // [levels][n_obs]
    std::vector<dk_moments> tmp;
    double cell_updates = 0;
    const float* cv_params = nullptr;   // [levels][NPARAM]
    uint32_t cv_mask = 0;
    int cv_ratio = 4;
    std::vector<dk_moments> zmom;       // [levels] moments of the control-variate samples
    int round_mode = 0;                 // 0: level after level, 1: concurrent streams, 2: hipGraph per round,
                                        // 3: persistent round kernel (graph replayed per segment)
};
int gpu_sample(void* user, int32_t level, uint64_t first, uint64_t count, double* sums);
int gpu_round(void* user, int L, const uint64_t* first, const uint64_t* count, double* sums);
double level_cost(const dk_problem* p, long steps0, int level, bool pair);

}  // namespace dkh
