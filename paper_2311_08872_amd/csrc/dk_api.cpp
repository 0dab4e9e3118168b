// dk_api.cpp -- host side of the C ABI: validation, level tables, batching into chunks,
// the ordered moment reduction, Algorithm 1 of Sec. 7 and plain Monte Carlo.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "dk_cnn.h"
#include "dk_fourier.h"
#include "dk_theta.h"
#include "dk_internal.h"
#include "dk_round.h"
#include "dk_stream.h"
#include <fstream>
#include <random>
#include <regex>
#include <sstream>

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(DK_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

// ------------------------------------------------------------------------------------------
// Compensated accumulation on the host (Neumaier), used to merge ordered partial sums.
// ------------------------------------------------------------------------------------------
void nadd(double& s, double& c, double x)
{
    const double t = s + x;
    if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

void merge_moments(dk_moments& dst, const double* part /* [DK_NMOM][2] */, uint64_t count)
{
    dst.count += count;
    for (int k = 0; k < DK_NMOM; ++k) {
        nadd(dst.sum[k], dst.comp[k], part[2 * k]);
        dst.comp[k] += part[2 * k + 1];
    }
}

double mom_value(const dk_moments& m, int k) { return m.sum[k] + m.comp[k]; }

// ------------------------------------------------------------------------------------------
// Problem hashing (FNV-1a over every field that changes results)
// ------------------------------------------------------------------------------------------
struct Hasher {
    uint64_t h = 1469598103934665603ull;
    void bytes(const void* p, size_t n)
    {
        const unsigned char* b = (const unsigned char*)p;
        for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
    }
    template <class T> void val(const T& v) { bytes(&v, sizeof(T)); }
    void field(const dk_field& f)
    {
        val(f.kind); val(f.n_modes); val(f.c0); val(f.floor_add);
        val(f.bump_amp); val(f.bump_sigma); val(f.bump_cx); val(f.bump_cy);
        val(f.es_a); val(f.es_b); val(f.es_s); val(f.es_x0); val(f.es_y0); val(f.es_scale);
        for (int k = 0; k < f.n_modes; ++k) val(f.modes[k]);
    }
};

uint64_t problem_hash(const dk_problem* p)
{
    Hasher H;
    H.val(p->d); H.val(p->n0); H.val(p->levels); H.val(p->steps_policy); H.val(p->box); H.val(p->mu);
    H.val(p->T); H.val(p->N); H.val(p->flux); H.val(p->precision); H.val(p->n_obs); H.val(p->coupling);
    H.val(p->grid); H.val(p->b0);
    H.field(p->rho0);
    for (int j = 0; j < p->n_obs; ++j) {
        H.field(p->obs[j].phi); H.val(p->obs[j].centre); H.val(p->obs[j].scale_sqrtN); H.val(p->obs[j].psi);
    }
    return H.h;
}

int validate_field(const dk_field& f, const char* what)
{
    if (f.kind < DK_FIELD_MODES || f.kind > DK_FIELD_EXPSIN2) return fail(DK_EINVAL, "%s: unknown field kind %d", what, f.kind);
    if (f.n_modes < 0 || f.n_modes > DK_MAX_MODES) return fail(DK_EINVAL, "%s: n_modes %d outside [0, %d]", what, f.n_modes, DK_MAX_MODES);
    if (f.n_modes > 0 && !f.modes) return fail(DK_EINVAL, "%s: modes is NULL", what);
    if (f.kind == DK_FIELD_BUMP && !(f.bump_sigma > 0)) return fail(DK_EINVAL, "%s: bump_sigma must be > 0", what);
    if (f.kind == DK_FIELD_EXPSIN2 && !(f.es_s > 0)) return fail(DK_EINVAL, "%s: es_s must be > 0", what);
    return DK_OK;
}

// steps on level 0, or a negative error code
long steps0_of(const dk_problem* p)
{
    const double h0 = p->box / p->n0;
    const double tau0 = p->mu * h0 * h0;
    const double r = p->T / tau0;
    const long m = std::lround(r);
    if (m < 1) return fail(DK_EINVAL, "T / tau_0 = %g gives no time step", r);
    if (p->steps_policy == DK_STEPS_EXACT && std::fabs(r - (double)m) > 1e-9 * std::max(1.0, r))
        return fail(DK_EINVAL, "T / tau_0 = %.12g is not an integer (use DK_STEPS_ROUND_T)", r);
    return m;
}

bool fourier(const dk_problem* p) { return p->coupling == DK_COUPLING_FOURIER; }
bool implicit(const dk_problem* p) { return p->b0 > 0.0; }
// h_{l-1} / h_l: 2 (NN coupling) or 3 (Fourier coupling)
int level_ratio(const dk_problem* p) { return fourier(p) ? 3 : 2; }
long ipow(long b, int e)
{
    long r = 1;
    while (e-- > 0) r *= b;
    return r;
}
int level_n(const dk_problem* p, int l) { return (int)(p->n0 * ipow(level_ratio(p), l)); }
long level_steps(const dk_problem* p, long steps0, int l) { return steps0 * ipow(level_ratio(p), 2 * l); }
// coarse work of a pair relative to its fine work: ratio^{-(d+2)}
double pair_factor(const dk_problem* p) { return fourier(p) ? 1.0 + 1.0 / 81.0 : 1.0 + 1.0 / 16.0; }

int validate(const dk_problem* p)
{
    if (!p) return fail(DK_EINVAL, "problem is NULL");
    if (p->d != 2) return fail(DK_EUNSUPPORTED, "d = %d: only d = 2 is implemented", p->d);
    if (p->n0 < 4 || (p->n0 & 1)) return fail(DK_EINVAL, "n0 = %d must be even and >= 4", p->n0);
    if (p->levels < 1 || p->levels > DK_MAX_LEVELS) return fail(DK_EINVAL, "levels = %d outside [1, %d]", p->levels, DK_MAX_LEVELS);
    if (!(p->box > 0)) return fail(DK_EINVAL, "box must be > 0");
    if (!(p->b0 >= 0.0 && p->b0 <= 1.0)) return fail(DK_EINVAL, "b0 = %g outside [0, 1]", p->b0);
    // |(1 - 2 b1 mu s)/(1 + 2 b0 mu s)| <= 1 for s in [0, 2]: mu (1 - 2 b0) <= 1/2
    if (!(p->mu > 0) || p->mu * (1.0 - 2.0 * p->b0) > 0.5 + 1e-12)
        return fail(DK_EINVAL, "mu = %g with b0 = %g: the scheme is unstable (mu (1 - 2 b0) must be <= 1/d)", p->mu, p->b0);
    if (!(p->T > 0)) return fail(DK_EINVAL, "T must be > 0");
    if (!(p->N > 0)) return fail(DK_EINVAL, "N must be > 0");
    if (p->flux != DK_FLUX_CENTRAL && p->flux != DK_FLUX_STAGGERED) return fail(DK_EINVAL, "unknown flux %d", p->flux);
    if (p->precision != DK_PREC_F32 && p->precision != DK_PREC_F64) return fail(DK_EINVAL, "unknown precision %d", p->precision);
    if (p->steps_policy != DK_STEPS_EXACT && p->steps_policy != DK_STEPS_ROUND_T) return fail(DK_EINVAL, "unknown steps_policy");
    if (p->n_obs < 1 || p->n_obs > DK_MAX_OBS) return fail(DK_EINVAL, "n_obs = %d outside [1, %d]", p->n_obs, DK_MAX_OBS);
    if (!p->obs) return fail(DK_EINVAL, "obs is NULL");
    if (p->primary_obs < 0 || p->primary_obs >= p->n_obs) return fail(DK_EINVAL, "primary_obs out of range");
    int rc = validate_field(p->rho0, "rho0");
    if (rc) return rc;
    for (int j = 0; j < p->n_obs; ++j) {
        rc = validate_field(p->obs[j].phi, "obs.phi");
        if (rc) return rc;
        if (p->obs[j].psi != DK_PSI_ID && p->obs[j].psi != DK_PSI_SQUARE) return fail(DK_EINVAL, "obs %d: unknown psi", j);
    }
    if (p->coupling != DK_COUPLING_NN && p->coupling != DK_COUPLING_FOURIER)
        return fail(DK_EINVAL, "unknown coupling %d", p->coupling);
    if (p->grid != DK_GRID_VERTEX && p->grid != DK_GRID_CELL) return fail(DK_EINVAL, "unknown grid %d", p->grid);
    if (fourier(p) && p->grid != DK_GRID_VERTEX)
        return fail(DK_EUNSUPPORTED, "the Fourier coupling is set up on the vertex grid");
    if (implicit(p)) {
        if (fourier(p)) return fail(DK_EUNSUPPORTED, "b0 > 0 runs with the NN coupling");
        if (p->flux != DK_FLUX_CENTRAL) return fail(DK_EUNSUPPORTED, "b0 > 0 runs the central flux only");
        for (int l = 0; l < p->levels; ++l)
            if (!dk::theta_supported(p->n0 << l, l >= 1))
                return fail(DK_EUNSUPPORTED, "b0 > 0: no kernel for the %d x %d grid of level %d (powers of two up to 64)",
                            p->n0 << l, p->n0 << l, l);
    }
    if (fourier(p)) {
        if (p->flux != DK_FLUX_CENTRAL) return fail(DK_EUNSUPPORTED, "the Fourier coupling runs the central flux only");
        if (p->levels > 6) return fail(DK_EINVAL, "levels = %d: the Fourier hierarchy has at most 6 levels", p->levels);
        for (int l = 0; l < p->levels; ++l)
            if (!dk::fourier_supported(level_n(p, l), l >= 1))
                return fail(DK_EUNSUPPORTED, "Fourier coupling: no kernel for the %d x %d grid of level %d (n0 = 4 or 8, "
                                             "at most 108 x 108)", level_n(p, l), level_n(p, l), l);
    }
    const long m0 = steps0_of(p);
    if (m0 < 0) return (int)m0;
    const long mtop = level_steps(p, m0, p->levels - 1);
    if (mtop > (1l << 30)) return fail(DK_EINVAL, "too many time steps (%ld) on the finest level", mtop);
    if (!fourier(p) && (long)p->n0 << (p->levels - 1) > 4096) return fail(DK_EINVAL, "finest grid larger than 4096");
    return DK_OK;
}

dk::FieldDev to_dev(const dk_field& f)
{
    dk::FieldDev d;
    std::memset(&d, 0, sizeof(d));
    d.kind = f.kind; d.n_modes = f.n_modes; d.c0 = f.c0; d.floor_add = f.floor_add;
    d.bump_amp = f.bump_amp; d.bump_sigma = f.bump_sigma; d.bump_cx = f.bump_cx; d.bump_cy = f.bump_cy;
    d.es_a = f.es_a; d.es_b = f.es_b; d.es_s = f.es_s; d.es_x0 = f.es_x0; d.es_y0 = f.es_y0; d.es_scale = f.es_scale;
    for (int k = 0; k < f.n_modes; ++k) {
        d.amp[k] = f.modes[k].amp; d.kx[k] = f.modes[k].kx; d.ky[k] = f.modes[k].ky; d.phase[k] = f.modes[k].phase;
    }
    return d;
}

// I_h f on the problem's grid for an n x n level: on cell centres the field is sampled at
// (i + 1/2) h, which for every field kind is the same field with shifted parameters (a phase
// for cosine modes, the centre for the bump and the sin^2 datum) sampled at i h.
dk::FieldDev to_dev_on(const dk_problem* p, const dk_field& f, int n)
{
    dk::FieldDev d = to_dev(f);
    if (p->grid != DK_GRID_CELL) return d;
    const double delta = 0.5 * p->box / n;
    const double two_pi = 6.28318530717958647692;
    for (int k = 0; k < d.n_modes; ++k) d.phase[k] += two_pi * (d.kx[k] + d.ky[k]) * delta / p->box;
    d.bump_cx -= delta;
    d.bump_cy -= delta;
    d.es_x0 -= delta;
    d.es_y0 -= delta;
    return d;
}

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

}  // namespace

constexpr double kMaxCellsPerLaunch = 2e12;   // default cap: about 5 s of kernel time per launch

struct KStat {
    uint64_t launches = 0, samples = 0;
    double ms = 0, cells = 0;
    int rows = 0;
};

struct dk_context {
    int device = 0;
    std::map<std::pair<int, int>, KStat> stats;
    std::map<int, int> forced_shape;          // grid size -> tile-shape variant
    bool force_stream = false;                // run every level with the streaming kernel
    int stream_depth = 0;                     // forced temporal depth of the streaming kernel (0: automatic)
    std::map<long, int> tuned_depth;          // (nf, pair, flux) -> streaming depth chosen by timing
    double max_launch_cells = kMaxCellsPerLaunch;   // work cap of one sampling launch
    // concurrent rounds: one stream per level, fork/join events, per-level buffers
    hipStream_t lvl_stream[DK_MAX_LEVELS] = {};
    hipEvent_t fork_ev = nullptr, join_ev[DK_MAX_LEVELS] = {};
    DevBuf rnd_ps[DK_MAX_LEVELS], rnd_mom[DK_MAX_LEVELS];
    hipEvent_t rnd_t0 = nullptr, rnd_t1 = nullptr;
    hipStream_t cap_stream = nullptr;         // private stream that round graphs are captured on
    double round_ms = 0;
    uint64_t round_graphs = 0;
    // persistent rounds: device tables, the queue counter, per-task moments, per-block scratch,
    // pinned staging, and the captured graph (reset + round kernel) replayed for every segment
    DevBuf pr_levels, pr_tasks, pr_ntasks, pr_head, pr_task_mom, pr_scratch;
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
    DevBuf per_sample;     // chunk buffer of per-sample outputs
    DevBuf moments;        // [chunks][n_obs][DK_NMOM][2]
    DevBuf mf0, mf1;       // mean-field streaming buffers
    DevBuf scratch_c;      // inner products
    DevBuf st_f[2][2], st_c[2][2];   // streaming state: [buffer][rho, cmp] fine / coarse
    DevBuf st_z;                     // streaming pairs: restricted-noise sums of split depths
    DevBuf fourier_scratch;          // Fourier pairs: per-block sums and half-projected sums
    std::vector<double> host_mom;
    // learned control variate
    dk::cnn::Workspace cnn;
    DevBuf cv_prm, cv_grad, cv_m, cv_v, cv_loss;
    DevBuf cv_fields, cv_x, cv_r, cv_y, cv_ps, cv_ps2, cv_z, cv_fields2, cv_x2, cv_r2;
    std::map<uint64_t, std::unique_ptr<ProblemTables>> problems;
};

namespace {

double noise_coeff(const dk_problem* p, double h, double sigma)
{
    // N^{-1/2} h^{-d/2} sigma / (2h) (central) or N^{-1/2} h^{-d/2} sigma / h (staggered), d = 2
    const double base = sigma / (std::sqrt(p->N) * h * h);
    return p->flux == DK_FLUX_CENTRAL ? 0.5 * base : base;
}

int ensure_level(dk_context* ctx, const dk_problem* p, int level, LevelTables** out, hipStream_t s);

// Noise-free scheme with weight b0 to step M, in FP64 on the host: every Fourier mode is
// multiplied by g^M, g = (1 - 2 b1 mu s)/(1 + 2 b0 mu s), s = sin^2(pi kx/n) + sin^2(pi ky/n)
// (Appendix A, operator A_h); separable DFTs, n <= 64.
void theta_meanfield_host(int n, double mu, double b0, long M, std::vector<double>& rho)
{
    typedef std::complex<double> cd;
    const double pi = 3.14159265358979323846;
    std::vector<cd> W((size_t)n * n), X((size_t)n * n), Y((size_t)n * n);
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) W[(size_t)j * n + k] = std::polar(1.0, -2.0 * pi * (double)((j * k) % n) / n);
    // forward: Y = W rho W^T  (rho indexed [y][x])
    for (int y = 0; y < n; ++y)
        for (int kx = 0; kx < n; ++kx) {
            cd acc = 0.0;
            for (int x = 0; x < n; ++x) acc += W[(size_t)kx * n + x] * rho[(size_t)y * n + x];
            X[(size_t)y * n + kx] = acc;
        }
    for (int ky = 0; ky < n; ++ky)
        for (int kx = 0; kx < n; ++kx) {
            cd acc = 0.0;
            for (int y = 0; y < n; ++y) acc += W[(size_t)ky * n + y] * X[(size_t)y * n + kx];
            const double sx = std::sin(pi * kx / n), sy = std::sin(pi * ky / n), ss = sx * sx + sy * sy;
            const double g = (1.0 - 2.0 * (1.0 - b0) * mu * ss) / (1.0 + 2.0 * b0 * mu * ss);
            Y[(size_t)ky * n + kx] = acc * std::pow(g, (double)M);
        }
    // inverse: conj(W) on both sides, 1/n^2
    for (int y = 0; y < n; ++y)
        for (int kx = 0; kx < n; ++kx) {
            cd acc = 0.0;
            for (int ky = 0; ky < n; ++ky) acc += std::conj(W[(size_t)y * n + ky]) * Y[(size_t)ky * n + kx];
            X[(size_t)y * n + kx] = acc;
        }
    for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) {
            cd acc = 0.0;
            for (int kx = 0; kx < n; ++kx) acc += std::conj(W[(size_t)x * n + kx]) * X[(size_t)y * n + kx];
            rho[(size_t)y * n + x] = acc.real() / ((double)n * n);
        }
}

int compute_centre(dk_context* ctx, const dk_problem* p, int level, LevelTables& T, hipStream_t s, double* rho_out)
{
    const int n = T.n;
    const int nobs = p->n_obs;
    std::vector<double> c(nobs, 0.0);
    const double a = 0.5 * p->mu;
    if (implicit(p)) {
        DevBuf r0;
        int rc = r0.ensure(sizeof(double) * n * n);
        if (rc) return rc;
        HIP_TRY(dk::launch_field_eval(to_dev_on(p, p->rho0, n), p->box, n, r0.p, true, s));
        std::vector<double> rho((size_t)n * n), phi((size_t)nobs * n * n);
        HIP_TRY(hipMemcpyAsync(rho.data(), r0.p, sizeof(double) * n * n, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(phi.data(), T.phi.p, sizeof(double) * nobs * n * n, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        theta_meanfield_host(n, p->mu, p->b0, T.steps, rho);
        for (int j = 0; j < nobs; ++j) {
            double acc = 0.0;
            for (size_t i = 0; i < (size_t)n * n; ++i) acc += rho[i] * phi[(size_t)j * n * n + i];
            c[j] = T.h * T.h * acc;
        }
        if (rho_out) {
            HIP_TRY(hipMemcpyAsync(rho_out, rho.data(), sizeof(double) * n * n, hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
        T.centre = c;
        T.have_centre = true;
        return DK_OK;
    }
    if (dk::level_supported(n)) {
        // FP64 rho0 for the noise-free resident kernel
        DevBuf r0;
        int rc = r0.ensure(sizeof(double) * n * n);
        if (rc) return rc;
        HIP_TRY(dk::launch_field_eval(to_dev_on(p, p->rho0, n), p->box, n, r0.p, true, s));
        rc = ctx->per_sample.ensure(sizeof(double) * 2 * nobs);
        if (rc) return rc;
        std::vector<double> obs_host(3 * nobs);
        for (int j = 0; j < nobs; ++j) { obs_host[3 * j] = 1.0; obs_host[3 * j + 1] = 0.0; obs_host[3 * j + 2] = 0.0; }
        DevBuf obs_unit;
        rc = obs_unit.ensure(sizeof(double) * 3 * nobs);
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(obs_unit.p, obs_host.data(), sizeof(double) * 3 * nobs, hipMemcpyHostToDevice, s));
        dk::LevelArgs A{};
        A.nf = n; A.level_id = level; A.tag = 0; A.seed = 0; A.first = 0; A.count = 1; A.steps = (int)T.steps;
        A.a = a; A.kf = 0; A.kc = 0; A.h2f = T.h * T.h; A.h2c = 0;
        A.rho0_f = r0.p; A.rho0_c = nullptr; A.phi_f = (const double*)T.phi.p; A.phi_c = nullptr;
        A.obs_f = (const double*)obs_unit.p; A.obs_c = nullptr; A.n_obs = nobs;
        A.out = (double*)ctx->per_sample.p; A.field_f = rho_out; A.field_c = nullptr;
        dk::LevelKind K{DK_PREC_F64, false, DK_FLUX_CENTRAL, false};
        HIP_TRY(dk::launch_level(K, A, s));
        std::vector<double> res(2 * nobs);
        HIP_TRY(hipMemcpyAsync(res.data(), ctx->per_sample.p, sizeof(double) * 2 * nobs, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int j = 0; j < nobs; ++j) c[j] = res[2 * j];
    } else {
        int rc = ctx->mf0.ensure(sizeof(double) * n * n);
        if (rc) return rc;
        rc = ctx->mf1.ensure(sizeof(double) * n * n);
        if (rc) return rc;
        rc = ctx->scratch_c.ensure(sizeof(double) * nobs);
        if (rc) return rc;
        HIP_TRY(dk::launch_field_eval(to_dev_on(p, p->rho0, n), p->box, n, ctx->mf0.p, true, s));
        double* res = nullptr;
        HIP_TRY(dk::launch_meanfield_stream(n, a, (int)T.steps, (double*)ctx->mf0.p, (double*)ctx->mf1.p, &res, s));
        HIP_TRY(dk::launch_inner_products(res, n, (const double*)T.phi.p, nobs, T.h * T.h, (double*)ctx->scratch_c.p, s));
        HIP_TRY(hipMemcpyAsync(c.data(), ctx->scratch_c.p, sizeof(double) * nobs, hipMemcpyDeviceToHost, s));
        if (rho_out) HIP_TRY(hipMemcpyAsync(rho_out, res, sizeof(double) * n * n, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    T.centre = c;
    T.have_centre = true;
    return DK_OK;
}

int ensure_level(dk_context* ctx, const dk_problem* p, int level, LevelTables** out, hipStream_t s)
{
    const uint64_t key = problem_hash(p);
    auto& slot = ctx->problems[key];
    if (!slot) slot.reset(new ProblemTables());
    ProblemTables& PT = *slot;
    if ((int)PT.level.size() < p->levels) PT.level.resize(p->levels);
    if (level < 0 || level >= p->levels) return fail(DK_EINVAL, "level %d outside [0, %d)", level, p->levels);
    if (PT.level[level]) { *out = PT.level[level].get(); return DK_OK; }
    std::unique_ptr<LevelTables> T(new LevelTables());
    const int n = level_n(p, level);
    T->n = n;
    T->h = p->box / n;
    T->tau = p->mu * T->h * T->h;
    T->steps = level_steps(p, steps0_of(p), level);
    const bool f64 = p->precision == DK_PREC_F64;
    const int nobs = p->n_obs;
    int rc = T->rho0.ensure((f64 ? 8 : 4) * (size_t)n * n);
    if (rc) return rc;
    HIP_TRY(dk::launch_field_eval(to_dev_on(p, p->rho0, n), p->box, n, T->rho0.p, f64, s));
    rc = T->phi.ensure(sizeof(double) * (size_t)nobs * n * n);
    if (rc) return rc;
    for (int j = 0; j < nobs; ++j)
        HIP_TRY(dk::launch_field_eval(to_dev_on(p, p->obs[j].phi, n), p->box, n, (double*)T->phi.p + (size_t)j * n * n, true, s));
    bool any_centre = false;
    for (int j = 0; j < nobs; ++j) any_centre |= p->obs[j].centre != 0;
    if (any_centre) {
        rc = compute_centre(ctx, p, level, *T, s, nullptr);
        if (rc) return rc;
    } else {
        T->centre.assign(nobs, 0.0);
    }
    std::vector<double> obs_host(3 * nobs);
    for (int j = 0; j < nobs; ++j) {
        obs_host[3 * j + 0] = p->obs[j].scale_sqrtN ? std::sqrt(p->N) : 1.0;
        obs_host[3 * j + 1] = p->obs[j].centre ? T->centre[j] : 0.0;
        obs_host[3 * j + 2] = p->obs[j].psi == DK_PSI_SQUARE ? 1.0 : 0.0;
    }
    rc = T->obs.ensure(sizeof(double) * 3 * nobs);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(T->obs.p, obs_host.data(), sizeof(double) * 3 * nobs, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    PT.level[level] = std::move(T);
    *out = PT.level[level].get();
    return DK_OK;
}

constexpr uint64_t kMaxChunk = 1ull << 22;
constexpr size_t kChunkBytes = 256ull << 20;

// Samples per launch: bounded by the per-sample output buffer and by the work of one launch
// (long levels are split so that no launch runs for more than a few seconds).
uint64_t chunk_size(int n_obs, double cells_per_sample, double max_cells)
{
    uint64_t c = kChunkBytes / (16ull * n_obs);
    c = std::min<uint64_t>(c, kMaxChunk);
    const double by_work = std::floor(max_cells / std::max(cells_per_sample, 1.0));
    if (by_work < (double)c) c = std::max<uint64_t>(256, (uint64_t)by_work);
    return c;
}

// ------------------------------------------------------------------------------------------
// Tile-shape choices as JSON text:
//   {"format": "dk-tile-shapes-1", "arch": "gfx950",
//    "shapes": [{"n": 128, "pair": 1, "flux": 0, "rows": 8, "spw": 1}, ...]}
// ("spw", samples per block, may be left out: then the shape with that R and ~256-lane blocks)
// ------------------------------------------------------------------------------------------
std::string device_arch(int device)
{
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, device) != hipSuccess) return "unknown";
    std::string a = pr.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

std::string tuning_json(const dk_context* ctx)
{
    std::ostringstream o;
    o << "{\"format\": \"dk-tile-shapes-1\", \"arch\": \"" << device_arch(ctx->device) << "\", \"shapes\": [";
    bool first = true;
    for (const auto& kv : ctx->tuned) {
        const int nf = (int)(kv.first >> 8), pair = (int)((kv.first >> 4) & 0xF), flux = (int)(kv.first & 0xF);
        o << (first ? "" : ", ") << "{\"n\": " << nf << ", \"pair\": " << pair << ", \"flux\": " << flux
          << ", \"rows\": " << dk::shape_rows(nf, kv.second) << ", \"spw\": " << dk::shape_spw(nf, kv.second) << "}";
        first = false;
    }
    for (const auto& kv : ctx->tuned_depth) {
        const int nf = (int)(kv.first >> 8), pair = (int)((kv.first >> 4) & 0xF), flux = (int)(kv.first & 0xF);
        o << (first ? "" : ", ") << "{\"n\": " << nf << ", \"pair\": " << pair << ", \"flux\": " << flux
          << ", \"depth\": " << kv.second << "}";
        first = false;
    }
    o << "]}";
    return o.str();
}

int load_tuning_json(dk_context* ctx, const std::string& text)
{
    static const std::regex fmt("\"format\"\\s*:\\s*\"dk-tile-shapes-1\"");
    static const std::regex arch("\"arch\"\\s*:\\s*\"([^\"]*)\"");
    static const std::regex entry("\\{\\s*\"n\"\\s*:\\s*(\\d+)\\s*,\\s*\"pair\"\\s*:\\s*(\\d+)\\s*,\\s*\"flux\"\\s*:\\s*(\\d+)"
                                  "\\s*,\\s*\"rows\"\\s*:\\s*(\\d+)(?:\\s*,\\s*\"spw\"\\s*:\\s*(\\d+))?\\s*\\}");
    if (!std::regex_search(text, fmt)) return fail(DK_EINVAL, "tuning JSON: missing \"format\": \"dk-tile-shapes-1\"");
    std::smatch m;
    if (!std::regex_search(text, m, arch)) return fail(DK_EINVAL, "tuning JSON: missing \"arch\"");
    const std::string dev = device_arch(ctx->device);
    if (m[1].str() != dev) return fail(DK_EINVAL, "tuning JSON is for %s, the device is %s", m[1].str().c_str(), dev.c_str());
    static const std::regex dentry("\\{\\s*\"n\"\\s*:\\s*(\\d+)\\s*,\\s*\"pair\"\\s*:\\s*(\\d+)\\s*,\\s*\"flux\"\\s*:\\s*(\\d+)"
                                   "\\s*,\\s*\"depth\"\\s*:\\s*(\\d+)\\s*\\}");
    std::map<long, int> got, gotd;
    for (auto it = std::sregex_iterator(text.begin(), text.end(), dentry); it != std::sregex_iterator(); ++it) {
        const int nf = std::stoi((*it)[1]), pair = std::stoi((*it)[2]), flux = std::stoi((*it)[3]);
        const int depth = std::stoi((*it)[4]);
        if (pair > 1 || (flux != DK_FLUX_CENTRAL && flux != DK_FLUX_STAGGERED) || !dk::stream_supported(nf) ||
            !dk::stream_depth_supported(depth))
            return fail(DK_EINVAL, "tuning JSON: bad streaming entry for n = %d", nf);
        gotd[((long)nf << 8) | ((long)pair << 4) | (long)flux] = depth;
    }
    for (auto it = std::sregex_iterator(text.begin(), text.end(), entry); it != std::sregex_iterator(); ++it) {
        const int nf = std::stoi((*it)[1]), pair = std::stoi((*it)[2]), flux = std::stoi((*it)[3]);
        const int rows = std::stoi((*it)[4]);
        if (pair > 1 || (flux != DK_FLUX_CENTRAL && flux != DK_FLUX_STAGGERED))
            return fail(DK_EINVAL, "tuning JSON: bad entry for n = %d", nf);
        int v = 0;
        while (dk::shape_rows(nf, v) > 0 && dk::shape_rows(nf, v) != rows) ++v;
        if (dk::shape_rows(nf, v) == 0) return fail(DK_EINVAL, "tuning JSON: no %d-row shape for n = %d", rows, nf);
        if ((*it)[5].matched) {
            const int spw = std::stoi((*it)[5]);
            while (dk::shape_rows(nf, v) > 0 && !(dk::shape_rows(nf, v) == rows && dk::shape_spw(nf, v) == spw)) ++v;
            if (dk::shape_rows(nf, v) == 0)
                return fail(DK_EINVAL, "tuning JSON: no %d-row shape with %d samples per block for n = %d", rows, spw, nf);
        }
        got[((long)nf << 8) | ((long)pair << 4) | (long)flux] = v;
    }
    for (const auto& kv : got) ctx->tuned[kv.first] = kv.second;
    for (const auto& kv : gotd) ctx->tuned_depth[kv.first] = kv.second;
    return DK_OK;
}

// DK_TUNE_CACHE: the file the context loads when created and rewrites after every new choice
void save_tuning_cache(const dk_context* ctx)
{
    const char* path = std::getenv("DK_TUNE_CACHE");
    if (!path || !*path) return;
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return;
        f << tuning_json(ctx) << "\n";
    }
    std::rename(tmp.c_str(), path);
}

// Tile-shape choice for the FP32 noisy kernels: a forced variant, a cached choice, or the
// fastest variant on a short tuning batch (same tables, at most 2048 fine steps, samples from
// the requested range; the outputs are discarded).  Small jobs use the default shape.
int choose_shape(dk_context* ctx, const dk_problem* p, bool pair, const dk::LevelArgs& A, uint64_t count,
                 double cells_per_sample, hipStream_t s, int* variant)
{
    *variant = 0;
    const int nf = A.nf;
    auto f = ctx->forced_shape.find(nf);
    if (f != ctx->forced_shape.end() && f->second >= 0) {
        if (dk::shape_rows(nf, f->second) == 0) return fail(DK_EINVAL, "no tile-shape variant %d for n = %d", f->second, nf);
        *variant = f->second;
        return DK_OK;
    }
    if (p->precision != DK_PREC_F32) return DK_OK;
    const long key = ((long)nf << 8) | ((long)pair << 4) | (long)p->flux;
    auto t = ctx->tuned.find(key);
    if (t != ctx->tuned.end()) { *variant = t->second; return DK_OK; }
    if ((double)count * cells_per_sample < 1e11) return DK_OK;
    int nvar = 0;
    while (dk::shape_rows(nf, nvar) > 0) ++nvar;
    if (nvar < 2) { ctx->tuned[key] = 0; save_tuning_cache(ctx); return DK_OK; }
    // The batch resembles a production launch: the level's own horizon (capped at 2048 steps;
    // a much shorter one favours shapes whose per-sample setup is cheaper, not their time loop)
    // and about one full round of blocks (256 CUs) of the larger grids.
    dk::LevelArgs T = A;
    T.count = std::min<uint64_t>(count, nf <= 32 ? 8192 : (nf == 64 ? 1024 : 256));
    T.steps = std::min(A.steps, 2048);
    T.field_f = nullptr;
    T.field_c = nullptr;
    int rc = ctx->per_sample.ensure(sizeof(double) * 2 * A.n_obs * T.count);
    if (rc) return rc;
    T.out = (double*)ctx->per_sample.p;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    ctx->tune_log.clear();
    double best = 1e300;
    int bestv = 0;
    for (int v = 0; v < nvar; ++v) {
        dk::LevelKind K{p->precision, pair, p->flux, true, v};
        HIP_TRY(dk::launch_level(K, T, s));   // warm-up
        HIP_TRY(hipEventRecord(e0, s));
        HIP_TRY(dk::launch_level(K, T, s));
        HIP_TRY(dk::launch_level(K, T, s));
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        ctx->tune_log.push_back(std::make_pair(v, (double)ms));
        if (ms < best) { best = ms; bestv = v; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->tuned[key] = bestv;
    save_tuning_cache(ctx);
    if (std::getenv("DK_LOG")) {
        std::fprintf(stderr, "[dk] tuned n=%d pair=%d flux=%d:", nf, (int)pair, p->flux);
        for (auto& kv : ctx->tune_log)
            std::fprintf(stderr, " R=%d/S=%d %.3f ms", dk::shape_rows(nf, kv.first), dk::shape_spw(nf, kv.first), kv.second);
        std::fprintf(stderr, " -> R=%d/S=%d\n", dk::shape_rows(nf, bestv), dk::shape_spw(nf, bestv));
        std::fflush(stderr);
    }
    *variant = bestv;
    return DK_OK;
}

// Grids beyond the resident kernel: state in HBM, batches of samples, launches of `depth` fine
// steps (the last one shorter if the step count is not a multiple), coarse steps fused into the
// depth-4 launches or taken by the coarse kernel after each group of 4, then the observables.
// The depth is forced (dk_context_set_stream_depth), cached, or chosen by timing the four depths
// on a short batch the first time a large job runs a grid size.
int stream_pass(dk_context* ctx, const dk_problem* p, bool pair, int depth, const dk::LevelArgs& A, uint64_t first,
                int c, int steps, size_t zgroup, hipStream_t s, int* cur_f, int* cur_c)
{
    const int nf = A.nf, nc = nf / 2;
    HIP_TRY(dk::launch_stream_init((const float*)A.rho0_f, nf, c, (float*)ctx->st_f[0][0].p, (float*)ctx->st_f[0][1].p, s));
    if (pair)
        HIP_TRY(dk::launch_stream_init((const float*)A.rho0_c, nc, c, (float*)ctx->st_c[0][0].p, (float*)ctx->st_c[0][1].p, s));
    dk::StreamArgs S{};
    S.n = nf; S.level_id = A.level_id; S.tag = A.tag; S.seed = A.seed; S.first = first; S.count = c;
    S.a = (float)A.a; S.kf = (float)A.kf; S.kc = (float)A.kc;
    S.z = pair && depth != 4 ? (float*)ctx->st_z.p : nullptr;
    S.zgroup = zgroup;
    int cf = 0, cc = 0;
    for (int m0 = 0; m0 < steps; m0 += depth) {
        S.m0 = m0;
        S.ksteps = std::min(depth, steps - m0);
        S.do_coarse = pair && depth == 4 ? 1 : 0;
        S.z_load = pair && depth != 4 && m0 % 4 != 0 ? 1 : 0;
        S.rho_in = (const float*)ctx->st_f[cf][0].p; S.cmp_in = (const float*)ctx->st_f[cf][1].p;
        S.rho_out = (float*)ctx->st_f[1 - cf][0].p; S.cmp_out = (float*)ctx->st_f[1 - cf][1].p;
        if (pair) {
            S.rhoc_in = (const float*)ctx->st_c[cc][0].p; S.cmpc_in = (const float*)ctx->st_c[cc][1].p;
            S.rhoc_out = (float*)ctx->st_c[1 - cc][0].p; S.cmpc_out = (float*)ctx->st_c[1 - cc][1].p;
        }
        HIP_TRY(dk::launch_stream_step(S, pair, p->flux, depth, s));
        cf = 1 - cf;
        if (!pair) continue;
        if (depth == 4) { cc = 1 - cc; continue; }
        const int groups = depth == 8 ? S.ksteps / 4 : ((m0 + S.ksteps) % 4 == 0 ? 1 : 0);
        for (int g = 0; g < groups; ++g) {
            HIP_TRY(dk::launch_stream_coarse(nc, c, S.a, S.kc, p->flux, (const float*)ctx->st_c[cc][0].p,
                                             (const float*)ctx->st_c[cc][1].p, (const float*)ctx->st_z.p + 2 * g * zgroup,
                                             (float*)ctx->st_c[1 - cc][0].p, (float*)ctx->st_c[1 - cc][1].p, s));
            cc = 1 - cc;
        }
    }
    *cur_f = cf;
    *cur_c = cc;
    return DK_OK;
}

int run_stream(dk_context* ctx, const dk_problem* p, int level, bool pair, uint64_t first, uint64_t count, uint32_t tag,
               const dk::LevelArgs& A, dk_moments* sums_out, double* per_sample_out, hipStream_t s,
               double* cell_updates, uint64_t nchunks_unused, uint64_t ch_unused, size_t mom_stride)
{
    const int nf = A.nf, nc = nf / 2;
    const int nobs = p->n_obs;
    const size_t nn = (size_t)nf * nf, ncc = (size_t)nc * nc;
    // state [buffer][rho, cmp] fine and coarse, and two groups of restricted-noise sums
    const size_t per_sample_bytes = 2 * 2 * 4 * (nn + (pair ? ncc : 0)) + (pair ? 2 * 8 * ncc : 0);
    uint64_t B = std::max<uint64_t>(1, (4ull << 30) / per_sample_bytes);
    B = std::min<uint64_t>({B, count, 4096ull});
    int rc;
    for (int b = 0; b < 2; ++b)
        for (int k = 0; k < 2; ++k) {
            if ((rc = ctx->st_f[b][k].ensure(4 * nn * B))) return rc;
            if (pair && (rc = ctx->st_c[b][k].ensure(4 * ncc * B))) return rc;
        }
    const size_t zgroup = ncc * B;
    if (pair && (rc = ctx->st_z.ensure(2 * 8 * zgroup))) return rc;
    const uint64_t nbatch = (count + B - 1) / B;
    if (!per_sample_out && (rc = ctx->per_sample.ensure(sizeof(double) * 2 * nobs * B))) return rc;
    if ((rc = ctx->moments.ensure(sizeof(double) * mom_stride * nbatch))) return rc;
    while (ctx->ev_pool.size() < 2 * nbatch) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        ctx->ev_pool.push_back(e);
    }
    const bool log = std::getenv("DK_LOG") != nullptr;
    const int steps = A.steps;
    const double cells_per_sample = (double)nn * (double)steps * (pair ? 1.0 + 1.0 / 16.0 : 1.0);
    int depth = ctx->stream_depth;
    if (depth == 0) {
        const long key = ((long)nf << 8) | ((long)pair << 4) | (long)p->flux;
        auto t = ctx->tuned_depth.find(key);
        if (t != ctx->tuned_depth.end()) {
            depth = t->second;
        } else if ((double)count * cells_per_sample < 1e11) {
            depth = 4;
        } else {
            // time each depth on 16 fine steps of a short batch (outputs discarded)
            const int tc = (int)std::min<uint64_t>(B, 64);
            const int ts = std::min(steps, 16);
            hipEvent_t e0 = ctx->ev_pool[0], e1 = ctx->ev_pool[1];
            double best = 1e300;
            int cf, cc;
            ctx->tune_log.clear();
            for (int d : {1, 2, 4, 8}) {
                if ((rc = stream_pass(ctx, p, pair, d, A, first, tc, ts, zgroup, s, &cf, &cc))) return rc;   // warm-up
                HIP_TRY(hipEventRecord(e0, s));
                if ((rc = stream_pass(ctx, p, pair, d, A, first, tc, ts, zgroup, s, &cf, &cc))) return rc;
                HIP_TRY(hipEventRecord(e1, s));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                ctx->tune_log.push_back(std::make_pair(d, (double)ms));
                if (ms < best) { best = ms; depth = d; }
            }
            ctx->tuned_depth[key] = depth;
            save_tuning_cache(ctx);
            if (log) {
                std::fprintf(stderr, "[dk] tuned streaming depth n=%d pair=%d flux=%d:", nf, (int)pair, p->flux);
                for (auto& kv : ctx->tune_log) std::fprintf(stderr, " D=%d %.3f ms", kv.first, kv.second);
                std::fprintf(stderr, " -> D=%d\n", depth);
                std::fflush(stderr);
            }
        }
    }
    for (uint64_t bi = 0; bi < nbatch; ++bi) {
        const uint64_t b0 = bi * B;
        const int c = (int)std::min<uint64_t>(B, count - b0);
        double* out = per_sample_out ? per_sample_out + b0 * nobs * 2 : (double*)ctx->per_sample.p;
        HIP_TRY(hipEventRecord(ctx->ev_pool[2 * bi], s));
        int cur = 0, curc = 0;
        if ((rc = stream_pass(ctx, p, pair, depth, A, first + b0, c, steps, zgroup, s, &cur, &curc))) return rc;
        HIP_TRY(dk::launch_stream_observe((const float*)ctx->st_f[cur][0].p, nf, c, A.phi_f, A.obs_f, nobs, A.h2f, out, 0, s));
        if (pair)
            HIP_TRY(dk::launch_stream_observe((const float*)ctx->st_c[curc][0].p, nc, c, A.phi_c, A.obs_c, nobs, A.h2c, out, 1, s));
        else
            HIP_TRY(dk::launch_zero_slot(out, c, nobs, 1, s));
        HIP_TRY(hipEventRecord(ctx->ev_pool[2 * bi + 1], s));
        HIP_TRY(dk::launch_moments(out, (uint64_t)c, nobs, (double*)ctx->moments.p + bi * mom_stride, s));
        if (log && nbatch > 1) {
            HIP_TRY(hipEventSynchronize(ctx->ev_pool[2 * bi + 1]));
            std::fprintf(stderr, "[dk] level %d%s (streamed %dx%d) batch %llu/%llu (%d samples)\n", level, pair ? " pair" : "",
                         nf, nf, (unsigned long long)(bi + 1), (unsigned long long)nbatch, c);
            std::fflush(stderr);
        }
    }
    ctx->host_mom.resize(mom_stride * nbatch);
    HIP_TRY(hipMemcpyAsync(ctx->host_mom.data(), ctx->moments.p, sizeof(double) * mom_stride * nbatch,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    {
        KStat& st = ctx->stats[std::make_pair(level, pair ? 1 : 0)];
        for (uint64_t k = 0; k < nbatch; ++k) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ctx->ev_pool[2 * k], ctx->ev_pool[2 * k + 1]));
            st.ms += ms;
        }
        st.launches += nbatch;
        st.samples += count;
        st.cells += cells_per_sample * (double)count;
        st.rows = -depth;   // streamed, temporal depth |rows|
    }
    for (uint64_t k = 0; k < nbatch; ++k) {
        const uint64_t c = std::min(B, count - k * B);
        for (int j = 0; j < nobs; ++j) merge_moments(sums_out[j], &ctx->host_mom[k * mom_stride + j * DK_NMOM * 2], c);
    }
    for (int j = 0; j < nobs; ++j)
        for (int m = 0; m < DK_NMOM; ++m)
            if (!std::isfinite(mom_value(sums_out[j], m))) return fail(DK_ENUMERIC, "non-finite sample values on level %d", level);
    if (cell_updates) *cell_updates += cells_per_sample * (double)count;
    return DK_OK;
}

// Levels of a Fourier-coupled hierarchy (Sec. 3.1): the projection kernel of the pair, then
// chunks of samples with blocks striding over each chunk, the moments in chunk order.
int run_fourier(dk_context* ctx, const dk_problem* p, int level, bool pair, uint64_t first, uint64_t count,
                const dk::LevelArgs& A, LevelTables* Tf, LevelTables* Tc, dk_moments* sums_out, double* per_sample_out,
                hipStream_t s, double* cell_updates, uint64_t nchunks, uint64_t ch, size_t mom_stride)
{
    const int nf = A.nf, nc = nf / 3, nobs = p->n_obs;
    const bool f64 = p->precision == DK_PREC_F64;
    const size_t esize = f64 ? 8 : 4;
    int rc;
    if (pair && !Tf->fourier_K.p) {
        // K[ic][i] = (1/nf) [1 + 2 sum_{k=1}^{nc/2-1} cos(2 pi k d / nf) + sqrt(2) cos(pi nc d / nf)], d = 3 ic - i:
        // projection onto the coarse frequencies (weight 2^{-1/2} on +-nc/2) read at coarse node ic
        std::vector<double> K((size_t)nc * nf);
        const double pi = 3.14159265358979323846;
        for (int ic = 0; ic < nc; ++ic)
            for (int i = 0; i < nf; ++i) {
                const double d = (double)(3 * ic - i);
                double v = 1.0;
                for (int k = 1; k < nc / 2; ++k) v += 2.0 * std::cos(2.0 * pi * k * d / nf);
                v += std::sqrt(2.0) * std::cos(pi * nc * d / nf);
                K[(size_t)ic * nf + i] = v / nf;
            }
        if ((rc = Tf->fourier_K.ensure(esize * K.size()))) return rc;
        std::vector<float> Kf(K.begin(), K.end());
        if (f64) HIP_TRY(hipMemcpyAsync(Tf->fourier_K.p, K.data(), 8 * K.size(), hipMemcpyHostToDevice, s));
        else HIP_TRY(hipMemcpyAsync(Tf->fourier_K.p, Kf.data(), 4 * Kf.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    dk::FourierArgs F{};
    F.nf = nf; F.level_id = level; F.tag = A.tag; F.seed = A.seed; F.steps = A.steps; F.n_obs = nobs;
    F.a = A.a; F.kf = A.kf;
    // projected sums have unit variance per coarse node: kc = kf h_f / h_c
    F.kc = pair ? noise_coeff(p, Tc->h, std::sqrt(Tf->tau) * Tc->h / Tf->h) : 0.0;
    F.h2f = A.h2f; F.h2c = A.h2c;
    F.rho0_f = A.rho0_f; F.rho0_c = A.rho0_c; F.phi_f = A.phi_f; F.phi_c = A.phi_c; F.obs_f = A.obs_f; F.obs_c = A.obs_c;
    F.K = pair ? Tf->fourier_K.p : nullptr;
    const int grid = dk::fourier_grid(nf, p->precision, ch);
    if (pair && (rc = ctx->fourier_scratch.ensure(esize * dk::fourier_scratch_elems(nf) * (size_t)grid))) return rc;
    F.scratch = pair ? ctx->fourier_scratch.p : nullptr;
    while (ctx->ev_pool.size() < 2 * nchunks) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        ctx->ev_pool.push_back(e);
    }
    const bool log = std::getenv("DK_LOG") != nullptr;
    for (uint64_t k = 0; k < nchunks; ++k) {
        const uint64_t b = k * ch;
        const uint64_t c = std::min(ch, count - b);
        F.first = first + b;
        F.count = c;
        F.out = per_sample_out ? per_sample_out + b * nobs * 2 : (double*)ctx->per_sample.p;
        HIP_TRY(hipEventRecord(ctx->ev_pool[2 * k], s));
        HIP_TRY(dk::launch_fourier(F, p->precision, pair, std::min(grid, dk::fourier_grid(nf, p->precision, c)), s));
        HIP_TRY(hipEventRecord(ctx->ev_pool[2 * k + 1], s));
        HIP_TRY(dk::launch_moments(F.out, c, nobs, (double*)ctx->moments.p + k * mom_stride, s));
        if (log && nchunks > 1) {
            HIP_TRY(hipEventSynchronize(ctx->ev_pool[2 * k + 1]));
            std::fprintf(stderr, "[dk] Fourier level %d%s launch %llu/%llu (%llu samples)\n", level, pair ? " pair" : "",
                         (unsigned long long)(k + 1), (unsigned long long)nchunks, (unsigned long long)c);
            std::fflush(stderr);
        }
    }
    ctx->host_mom.resize(mom_stride * nchunks);
    HIP_TRY(hipMemcpyAsync(ctx->host_mom.data(), ctx->moments.p, sizeof(double) * mom_stride * nchunks,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double per = (double)nf * nf * (double)A.steps * (pair ? pair_factor(p) : 1.0);
    {
        KStat& st = ctx->stats[std::make_pair(level, pair ? 1 : 0)];
        for (uint64_t k = 0; k < nchunks; ++k) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ctx->ev_pool[2 * k], ctx->ev_pool[2 * k + 1]));
            st.ms += ms;
        }
        st.launches += nchunks;
        st.samples += count;
        st.rows = 0;   // Fourier kernel: the fine state in LDS, no tile shapes
        st.cells += per * (double)count;
    }
    for (uint64_t k = 0; k < nchunks; ++k) {
        const uint64_t c = std::min(ch, count - k * ch);
        for (int j = 0; j < nobs; ++j) merge_moments(sums_out[j], &ctx->host_mom[k * mom_stride + j * DK_NMOM * 2], c);
    }
    for (int j = 0; j < nobs; ++j)
        for (int m = 0; m < DK_NMOM; ++m)
            if (!std::isfinite(mom_value(sums_out[j], m))) return fail(DK_ENUMERIC, "non-finite sample values on level %d", level);
    if (cell_updates) *cell_updates += per * (double)count;
    return DK_OK;
}

// Levels with b0 > 0: per-level tables (twiddles, solve multipliers), then chunks of samples
// with blocks striding over each chunk, the moments in chunk order.
int theta_tables(const dk_problem* p, LevelTables* T, hipStream_t s)
{
    if (T->theta_tw.p) return DK_OK;
    const int n = T->n;
    const bool f64 = p->precision == DK_PREC_F64;
    const size_t esize = f64 ? 8 : 4;
    const double pi = 3.14159265358979323846;
    std::vector<double> tw(n), sol((size_t)n * n);
    for (int k = 0; k < n / 2; ++k) {
        tw[2 * k] = std::cos(2.0 * pi * k / n);
        tw[2 * k + 1] = -std::sin(2.0 * pi * k / n);
    }
    for (int ky = 0; ky < n; ++ky)
        for (int kx = 0; kx < n; ++kx) {
            const double sx = std::sin(pi * kx / n), sy = std::sin(pi * ky / n);
            sol[(size_t)ky * n + kx] = 1.0 / (1.0 + 2.0 * p->b0 * p->mu * (sx * sx + sy * sy));
        }
    int rc;
    if ((rc = T->theta_tw.ensure(esize * tw.size())) || (rc = T->theta_sol.ensure(esize * sol.size()))) return rc;
    std::vector<float> twf(tw.begin(), tw.end()), solf(sol.begin(), sol.end());
    HIP_TRY(hipMemcpyAsync(T->theta_tw.p, f64 ? (const void*)tw.data() : (const void*)twf.data(), esize * tw.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(T->theta_sol.p, f64 ? (const void*)sol.data() : (const void*)solf.data(), esize * sol.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return DK_OK;
}

int run_theta(dk_context* ctx, const dk_problem* p, int level, bool pair, uint64_t first, uint64_t count,
              const dk::LevelArgs& A, LevelTables* Tf, LevelTables* Tc, dk_moments* sums_out, double* per_sample_out,
              hipStream_t s, double* cell_updates, uint64_t nchunks, uint64_t ch, size_t mom_stride)
{
    const int nf = A.nf, nobs = p->n_obs;
    int rc;
    if ((rc = theta_tables(p, Tf, s))) return rc;
    if (pair && (rc = theta_tables(p, Tc, s))) return rc;
    dk::ThetaArgs F{};
    F.n = nf; F.level_id = level; F.tag = A.tag; F.seed = A.seed; F.steps = A.steps; F.n_obs = nobs;
    F.a = A.a; F.kf = A.kf; F.kc = A.kc;
    F.h2f = A.h2f; F.h2c = A.h2c;
    F.rho0_f = A.rho0_f; F.rho0_c = A.rho0_c; F.phi_f = A.phi_f; F.phi_c = A.phi_c; F.obs_f = A.obs_f; F.obs_c = A.obs_c;
    F.tw = Tf->theta_tw.p;
    F.sol_f = Tf->theta_sol.p;
    F.sol_c = pair ? Tc->theta_sol.p : nullptr;
    while (ctx->ev_pool.size() < 2 * nchunks) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        ctx->ev_pool.push_back(e);
    }
    const bool log = std::getenv("DK_LOG") != nullptr;
    for (uint64_t k = 0; k < nchunks; ++k) {
        const uint64_t b = k * ch;
        const uint64_t c = std::min(ch, count - b);
        F.first = first + b;
        F.count = c;
        F.out = per_sample_out ? per_sample_out + b * nobs * 2 : (double*)ctx->per_sample.p;
        HIP_TRY(hipEventRecord(ctx->ev_pool[2 * k], s));
        HIP_TRY(dk::launch_theta(F, p->precision, pair, dk::theta_grid(nf, p->precision, c), s));
        HIP_TRY(hipEventRecord(ctx->ev_pool[2 * k + 1], s));
        HIP_TRY(dk::launch_moments(F.out, c, nobs, (double*)ctx->moments.p + k * mom_stride, s));
        if (log && nchunks > 1) {
            HIP_TRY(hipEventSynchronize(ctx->ev_pool[2 * k + 1]));
            std::fprintf(stderr, "[dk] b0 = %g level %d%s launch %llu/%llu (%llu samples)\n", p->b0, level, pair ? " pair" : "",
                         (unsigned long long)(k + 1), (unsigned long long)nchunks, (unsigned long long)c);
            std::fflush(stderr);
        }
    }
    ctx->host_mom.resize(mom_stride * nchunks);
    HIP_TRY(hipMemcpyAsync(ctx->host_mom.data(), ctx->moments.p, sizeof(double) * mom_stride * nchunks,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double per = (double)nf * nf * (double)A.steps * (pair ? pair_factor(p) : 1.0);
    {
        KStat& st = ctx->stats[std::make_pair(level, pair ? 1 : 0)];
        for (uint64_t k = 0; k < nchunks; ++k) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ctx->ev_pool[2 * k], ctx->ev_pool[2 * k + 1]));
            st.ms += ms;
        }
        st.launches += nchunks;
        st.samples += count;
        st.rows = 0;   // b0 > 0 kernel: the state in LDS, no tile shapes
        st.cells += per * (double)count;
    }
    for (uint64_t k = 0; k < nchunks; ++k) {
        const uint64_t c = std::min(ch, count - k * ch);
        for (int j = 0; j < nobs; ++j) merge_moments(sums_out[j], &ctx->host_mom[k * mom_stride + j * DK_NMOM * 2], c);
    }
    for (int j = 0; j < nobs; ++j)
        for (int m = 0; m < DK_NMOM; ++m)
            if (!std::isfinite(mom_value(sums_out[j], m))) return fail(DK_ENUMERIC, "non-finite sample values on level %d", level);
    if (cell_updates) *cell_updates += per * (double)count;
    return DK_OK;
}

// Run samples [first, first+count) of level `level` (coupled pair if `pair`), reduce the
// per-sample values in chunk order and return per-observable moments.
int run_level(dk_context* ctx, const dk_problem* p, int level, bool pair, uint64_t first, uint64_t count,
              uint32_t tag, dk_moments* sums_out, double* per_sample_out, void* field_f, void* field_c,
              hipStream_t s, double* cell_updates)
{
    int rc = validate(p);
    if (rc) return rc;
    if (pair && level < 1) return fail(DK_EINVAL, "a coupled pair needs level >= 1");
    if (level < 0 || level >= p->levels) return fail(DK_EINVAL, "level %d outside [0, %d)", level, p->levels);
    if (count > 0 && first + count < first) return fail(DK_EINVAL, "sample range overflows");
    if (first + count > (1ull << 48)) return fail(DK_EINVAL, "sample index beyond 2^48");
    const int nf = level_n(p, level);
    const bool four = fourier(p), theta = implicit(p);
    const bool stream = !four && !theta && (!dk::level_supported(nf) || (ctx->force_stream && dk::stream_supported(nf)));
    if (four && (field_f || field_c)) return fail(DK_EUNSUPPORTED, "field output is not available for the Fourier coupling");
    if (theta && (field_f || field_c)) return fail(DK_EUNSUPPORTED, "field output is not available for b0 > 0");
    if (stream) {
        if (!dk::stream_supported(nf))
            return fail(DK_EUNSUPPORTED, "grid %d x %d: neither the resident nor the streaming kernel supports it", nf, nf);
        if (p->precision != DK_PREC_F32) return fail(DK_EUNSUPPORTED, "the streaming kernel has an FP32 state only");
        if (field_f || field_c) return fail(DK_EUNSUPPORTED, "field output is not available for streamed grids");
    }
    LevelTables* Tf = nullptr;
    LevelTables* Tc = nullptr;
    rc = ensure_level(ctx, p, level, &Tf, s);
    if (rc) return rc;
    if (pair) {
        rc = ensure_level(ctx, p, level - 1, &Tc, s);
        if (rc) return rc;
    }
    const int nobs = p->n_obs;
    for (int j = 0; j < nobs; ++j) std::memset(&sums_out[j], 0, sizeof(dk_moments));
    if (count == 0) return DK_OK;
    const double cells_per_sample = (double)nf * nf * (double)Tf->steps * (pair ? pair_factor(p) : 1.0);
    const uint64_t ch = chunk_size(nobs, cells_per_sample, ctx->max_launch_cells);
    const bool log = std::getenv("DK_LOG") != nullptr;
    const uint64_t nchunks = (count + ch - 1) / ch;
    if (!per_sample_out) {
        rc = ctx->per_sample.ensure(sizeof(double) * 2 * nobs * std::min<uint64_t>(ch, count));
        if (rc) return rc;
    }
    const size_t mom_stride = (size_t)nobs * DK_NMOM * 2;
    rc = ctx->moments.ensure(sizeof(double) * mom_stride * nchunks);
    if (rc) return rc;

    dk::LevelArgs A{};
    A.nf = nf;
    A.level_id = level;
    A.tag = tag;
    A.seed = p->seed;
    A.steps = (int)Tf->steps;
    A.a = 0.5 * p->mu;
    const double sig_f = std::sqrt(Tf->tau);
    A.kf = noise_coeff(p, Tf->h, sig_f);
    A.kc = pair ? noise_coeff(p, Tc->h, 0.5 * sig_f) : 0.0;   // 2^{-d/2} sqrt(tau_f) per unit of the restricted sum
    A.h2f = Tf->h * Tf->h;
    A.h2c = pair ? Tc->h * Tc->h : 0.0;
    A.rho0_f = Tf->rho0.p;
    A.rho0_c = pair ? Tc->rho0.p : nullptr;
    A.phi_f = (const double*)Tf->phi.p;
    A.phi_c = pair ? (const double*)Tc->phi.p : nullptr;
    A.obs_f = (const double*)Tf->obs.p;
    A.obs_c = pair ? (const double*)Tc->obs.p : nullptr;
    A.n_obs = nobs;
    if (stream)
        return run_stream(ctx, p, level, pair, first, count, tag, A, sums_out, per_sample_out, s, cell_updates, nchunks, ch,
                          mom_stride);
    if (four)
        return run_fourier(ctx, p, level, pair, first, count, A, Tf, Tc, sums_out, per_sample_out, s, cell_updates, nchunks,
                           ch, mom_stride);
    if (theta)
        return run_theta(ctx, p, level, pair, first, count, A, Tf, Tc, sums_out, per_sample_out, s, cell_updates, nchunks,
                         ch, mom_stride);
    int variant = 0;
    rc = choose_shape(ctx, p, pair, A, count, (double)nf * nf * (double)Tf->steps * (pair ? 1.0 + 1.0 / 16.0 : 1.0), s,
                      &variant);
    if (rc) return rc;
    dk::LevelKind K{p->precision, pair, p->flux, true, variant};
    const size_t esize = p->precision == DK_PREC_F64 ? 8 : 4;
    while (ctx->ev_pool.size() < 2 * nchunks) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        ctx->ev_pool.push_back(e);
    }
    for (uint64_t k = 0; k < nchunks; ++k) {
        const uint64_t b = k * ch;
        const uint64_t c = std::min(ch, count - b);
        A.first = first + b;
        A.count = c;
        A.out = per_sample_out ? per_sample_out + b * nobs * 2 : (double*)ctx->per_sample.p;
        A.field_f = field_f ? (char*)field_f + b * esize * nf * nf : nullptr;
        A.field_c = (field_c && pair) ? (char*)field_c + b * esize * (nf / 2) * (nf / 2) : nullptr;
        HIP_TRY(hipEventRecord(ctx->ev_pool[2 * k], s));
        HIP_TRY(dk::launch_level(K, A, s));
        HIP_TRY(hipEventRecord(ctx->ev_pool[2 * k + 1], s));
        HIP_TRY(dk::launch_moments(A.out, c, nobs, (double*)ctx->moments.p + k * mom_stride, s));
        if (log && nchunks > 1) {
            // progress of long levels (waits for this launch)
            HIP_TRY(hipEventSynchronize(ctx->ev_pool[2 * k + 1]));
            std::fprintf(stderr, "[dk] level %d%s launch %llu/%llu (%llu samples)\n", level, pair ? " pair" : "",
                         (unsigned long long)(k + 1), (unsigned long long)nchunks, (unsigned long long)c);
            std::fflush(stderr);
        }
    }
    ctx->host_mom.resize(mom_stride * nchunks);
    HIP_TRY(hipMemcpyAsync(ctx->host_mom.data(), ctx->moments.p, sizeof(double) * mom_stride * nchunks,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    {
        KStat& st = ctx->stats[std::make_pair(level, pair ? 1 : 0)];
        for (uint64_t k = 0; k < nchunks; ++k) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ctx->ev_pool[2 * k], ctx->ev_pool[2 * k + 1]));
            st.ms += ms;
        }
        st.launches += nchunks;
        st.samples += count;
        st.rows = p->precision == DK_PREC_F32 ? dk::shape_rows(nf, variant) : (nf == 128 ? 16 : dk::shape_rows(nf, 0));
        st.cells += (double)nf * nf * (double)Tf->steps * (pair ? 1.0 + 1.0 / 16.0 : 1.0) * (double)count;
    }
    for (uint64_t k = 0; k < nchunks; ++k) {
        const uint64_t c = std::min(ch, count - k * ch);
        for (int j = 0; j < nobs; ++j) merge_moments(sums_out[j], &ctx->host_mom[k * mom_stride + j * DK_NMOM * 2], c);
    }
    for (int j = 0; j < nobs; ++j)
        for (int m = 0; m < DK_NMOM; ++m)
            if (!std::isfinite(mom_value(sums_out[j], m))) return fail(DK_ENUMERIC, "non-finite sample values on level %d", level);
    if (cell_updates) {
        const double per = (double)nf * nf * (double)Tf->steps * (pair ? 1.0 + 1.0 / 16.0 : 1.0);
        *cell_updates += per * (double)count;
    }
    return DK_OK;
}

// Tables and coefficients of level l (a pair with level l-1 if `pair`) for the level kernels;
// first, count and the output pointers are left to the caller.
int level_args(dk_context* ctx, const dk_problem* p, int l, bool pair, uint32_t tag, hipStream_t s, dk::LevelArgs* out,
               double* cells_per_sample)
{
    if (fourier(p) || implicit(p)) return fail(DK_EUNSUPPORTED, "the Fourier coupling and b0 > 0 run level by level");
    const int nf = level_n(p, l);
    LevelTables *Tf = nullptr, *Tc = nullptr;
    int rc = ensure_level(ctx, p, l, &Tf, s);
    if (rc) return rc;
    if (pair && (rc = ensure_level(ctx, p, l - 1, &Tc, s))) return rc;
    *cells_per_sample = (double)nf * nf * (double)Tf->steps * (pair ? 1.0 + 1.0 / 16.0 : 1.0);
    dk::LevelArgs A{};
    A.nf = nf; A.level_id = l; A.tag = tag; A.seed = p->seed; A.steps = (int)Tf->steps; A.a = 0.5 * p->mu;
    const double sig_f = std::sqrt(Tf->tau);
    A.kf = noise_coeff(p, Tf->h, sig_f);
    A.kc = pair ? noise_coeff(p, Tc->h, 0.5 * sig_f) : 0.0;
    A.h2f = Tf->h * Tf->h;
    A.h2c = pair ? Tc->h * Tc->h : 0.0;
    A.rho0_f = Tf->rho0.p;
    A.rho0_c = pair ? Tc->rho0.p : nullptr;
    A.phi_f = (const double*)Tf->phi.p;
    A.phi_c = pair ? (const double*)Tc->phi.p : nullptr;
    A.obs_f = (const double*)Tf->obs.p;
    A.obs_c = pair ? (const double*)Tc->obs.p : nullptr;
    A.n_obs = p->n_obs;
    *out = A;
    return DK_OK;
}

// ------------------------------------------------------------------------------------------
// One Algorithm-1 round of resident levels at once: every level's batches go to its own
// stream (forked from and joined to the caller's stream), so levels of very different size
// fill the GPU together; mode 2 captures the whole round into a hipGraph and launches it once.
// The per-sample values and the chunking are those of run_level, so results are identical.
// ------------------------------------------------------------------------------------------
struct RoundJob {
    int level = 0;
    bool pair = false;
    uint64_t first = 0, count = 0, ch = 0, nchunks = 0;
    dk::LevelArgs A{};
    dk::LevelKind K{};
    double cells_per_sample = 0;
};

int run_round(dk_context* ctx, const dk_problem* p, int L, const uint64_t* first, const uint64_t* count, uint32_t tag,
              int mode, std::vector<dk_moments>& sums /* [(L+1) * n_obs] */, hipStream_t s, double* cell_updates)
{
    const int nobs = p->n_obs;
    const size_t mom_stride = (size_t)nobs * DK_NMOM * 2;
    std::vector<RoundJob> jobs;
    for (int l = 0; l <= L; ++l) {
        for (int j = 0; j < nobs; ++j) std::memset(&sums[(size_t)l * nobs + j], 0, sizeof(dk_moments));
        if (count[l] == 0) continue;
        RoundJob J;
        J.level = l;
        J.pair = l >= 1;
        J.first = first[l];
        J.count = count[l];
        int rc = level_args(ctx, p, l, J.pair, tag, s, &J.A, &J.cells_per_sample);
        if (rc) return rc;
        J.ch = chunk_size(nobs, J.cells_per_sample, ctx->max_launch_cells);
        J.nchunks = (J.count + J.ch - 1) / J.ch;
        dk::LevelArgs& A = J.A;
        int variant = 0;
        if ((rc = choose_shape(ctx, p, J.pair, A, J.count, J.cells_per_sample, s, &variant))) return rc;
        J.K = dk::LevelKind{p->precision, J.pair, p->flux, true, variant};
        if ((rc = ctx->rnd_ps[l].ensure(sizeof(double) * 2 * nobs * std::min(J.ch, J.count)))) return rc;
        if ((rc = ctx->rnd_mom[l].ensure(sizeof(double) * mom_stride * J.nchunks))) return rc;
        if (!ctx->lvl_stream[l]) {
            HIP_TRY(hipStreamCreateWithFlags(&ctx->lvl_stream[l], hipStreamNonBlocking));
            HIP_TRY(hipEventCreateWithFlags(&ctx->join_ev[l], hipEventDisableTiming));
        }
        jobs.push_back(J);
    }
    if (jobs.empty()) return DK_OK;
    if (!ctx->fork_ev) {
        HIP_TRY(hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
        HIP_TRY(hipEventCreate(&ctx->rnd_t0));
        HIP_TRY(hipEventCreate(&ctx->rnd_t1));
    }
    if (mode == 2 && !ctx->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    // the caller's stream may be the null stream, which cannot be captured: graphs are captured
    // on a private stream and launched on the caller's
    const hipStream_t o = mode == 2 ? ctx->cap_stream : s;
    auto enqueue = [&]() -> int {
        HIP_TRY(hipEventRecord(ctx->fork_ev, o));
        for (RoundJob& J : jobs) {
            hipStream_t ls = ctx->lvl_stream[J.level];
            HIP_TRY(hipStreamWaitEvent(ls, ctx->fork_ev, 0));
            for (uint64_t k = 0; k < J.nchunks; ++k) {
                dk::LevelArgs A = J.A;
                const uint64_t b = k * J.ch;
                A.first = J.first + b;
                A.count = std::min(J.ch, J.count - b);
                A.out = (double*)ctx->rnd_ps[J.level].p;
                A.field_f = nullptr;
                A.field_c = nullptr;
                HIP_TRY(dk::launch_level(J.K, A, ls));
                HIP_TRY(dk::launch_moments(A.out, A.count, nobs, (double*)ctx->rnd_mom[J.level].p + k * mom_stride, ls));
            }
            HIP_TRY(hipEventRecord(ctx->join_ev[J.level], ls));
            HIP_TRY(hipStreamWaitEvent(o, ctx->join_ev[J.level], 0));
        }
        return DK_OK;
    };
    HIP_TRY(hipEventRecord(ctx->rnd_t0, s));
    if (mode == 2) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        HIP_TRY(hipStreamBeginCapture(o, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue();
        hipGraph_t g2 = nullptr;
        const hipError_t ec = hipStreamEndCapture(o, &g2);
        if (rc) { if (g2) (void)hipGraphDestroy(g2); return rc; }
        if (ec != hipSuccess) return fail(DK_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ec));
        graph = g2;
        HIP_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        HIP_TRY(hipGraphLaunch(exec, s));
        HIP_TRY(hipEventRecord(ctx->rnd_t1, s));
        HIP_TRY(hipStreamSynchronize(s));
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        ctx->round_graphs += 1;
    } else {
        const int rc = enqueue();
        if (rc) return rc;
        HIP_TRY(hipEventRecord(ctx->rnd_t1, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->rnd_t0, ctx->rnd_t1));
    ctx->round_ms += ms;
    std::vector<double> h;
    for (RoundJob& J : jobs) {
        h.resize(mom_stride * J.nchunks);
        HIP_TRY(hipMemcpy(h.data(), ctx->rnd_mom[J.level].p, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
        for (uint64_t k = 0; k < J.nchunks; ++k) {
            const uint64_t c = std::min(J.ch, J.count - k * J.ch);
            for (int j = 0; j < nobs; ++j)
                merge_moments(sums[(size_t)J.level * nobs + j], &h[k * mom_stride + j * DK_NMOM * 2], c);
        }
        for (int j = 0; j < nobs; ++j)
            for (int m = 0; m < DK_NMOM; ++m)
                if (!std::isfinite(mom_value(sums[(size_t)J.level * nobs + j], m)))
                    return fail(DK_ENUMERIC, "non-finite sample values on level %d", J.level);
        KStat& st = ctx->stats[std::make_pair(J.level, J.pair ? 1 : 0)];
        st.launches += J.nchunks;
        st.samples += J.count;
        st.cells += J.cells_per_sample * (double)J.count;
        st.rows = dk::shape_rows(J.A.nf, J.K.shape);
        if (cell_updates) *cell_updates += J.cells_per_sample * (double)J.count;
    }
    return DK_OK;
}

// ------------------------------------------------------------------------------------------
// One Algorithm-1 round of resident FP32 levels in one persistent launch (round_mode 3).
// Tasks: for each level, from the finest down, contiguous sample ranges of whole
// block-iterations sized to about 1/8 of a block's share of one launch; segments: consecutive
// tasks of at most the context's launch cap in cell updates (one launch each, so no launch runs for more
// than a few seconds).  Every segment replays the same captured graph (queue reset + round
// kernel) after its task list has been uploaded; the graph is captured again only when a
// device buffer it points to had to grow.  Task moments are merged per level in task order.
// ------------------------------------------------------------------------------------------
bool round_eligible(const dk_problem* p, int l, bool force_stream)
{
    const int nf = level_n(p, l);
    return !fourier(p) && !implicit(p) && p->precision == DK_PREC_F32 && p->n_obs <= dk::round_max_obs() && !force_stream &&
           dk::round_kind(nf, l >= 1) >= 0;
}

int run_round_persistent(dk_context* ctx, const dk_problem* p, int L, const uint64_t* first, const uint64_t* count,
                         uint32_t tag, std::vector<dk_moments>& sums /* [(L+1) * n_obs] */, hipStream_t s,
                         double* cell_updates)
{
    const int nobs = p->n_obs;
    const size_t nmom = (size_t)nobs * DK_NMOM;
    std::vector<dk::RoundLevel> lv(L + 1);
    std::vector<double> cps(L + 1, 0.0);
    double total = 0;
    for (int l = 0; l <= L; ++l) {
        for (int j = 0; j < nobs; ++j) std::memset(&sums[(size_t)l * nobs + j], 0, sizeof(dk_moments));
        std::memset(&lv[l], 0, sizeof(dk::RoundLevel));
        lv[l].kind = -1;
        if (count[l] == 0) continue;
        if (!round_eligible(p, l, ctx->force_stream)) return fail(DK_EUNSUPPORTED, "level %d cannot join a persistent round", l);
        int rc = level_args(ctx, p, l, l >= 1, tag, s, &lv[l].A, &cps[l]);
        if (rc) return rc;
        lv[l].kind = dk::round_kind(lv[l].A.nf, l >= 1);
        lv[l].spw = dk::round_spw_of(lv[l].A.nf);
        total += cps[l] * (double)count[l];
    }
    if (total == 0) return DK_OK;
    if (ctx->pr_grid == 0) {
        int cus = 0;
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
        ctx->pr_grid = std::max(1, cus) * dk::round_blocks_per_cu(p->flux);
        HIP_TRY(hipEventCreate(&ctx->pr_t0));
        HIP_TRY(hipEventCreate(&ctx->pr_t1));
    }
    const int grid = ctx->pr_grid;
    // tasks, finest level first
    const double cap = ctx->max_launch_cells;
    const double per_task = std::min(total, cap) / (8.0 * grid);
    std::vector<dk::RoundTask> tasks;
    std::vector<double> work;
    for (int l = L; l >= 0; --l) {
        if (count[l] == 0) continue;
        const uint64_t spw = (uint64_t)lv[l].spw;
        const uint64_t iters = std::max<uint64_t>(1, (uint64_t)std::floor(per_task / (cps[l] * (double)spw)));
        const uint64_t chunk = iters * spw;
        for (uint64_t b = 0; b < count[l]; b += chunk) {
            dk::RoundTask t{};
            t.level = (uint32_t)l;
            t.first = first[l] + b;
            t.count = std::min(chunk, count[l] - b);
            tasks.push_back(t);
            work.push_back(cps[l] * (double)t.count);
        }
    }
    // segments
    std::vector<size_t> seg = {0};
    double acc = 0;
    for (size_t t = 0; t < tasks.size(); ++t) {
        if (acc > 0 && acc + work[t] > cap) { seg.push_back(t); acc = 0; }
        acc += work[t];
    }
    seg.push_back(tasks.size());
    size_t max_seg = 0;
    for (size_t k = 0; k + 1 < seg.size(); ++k) max_seg = std::max(max_seg, seg[k + 1] - seg[k]);
    // buffers; the graph is captured again when any of them moved
    const uint64_t stride = 256ull * nobs * 2;
    const void* before[6] = {ctx->pr_levels.p, ctx->pr_tasks.p, ctx->pr_ntasks.p, ctx->pr_head.p, ctx->pr_task_mom.p,
                             ctx->pr_scratch.p};
    int rc;
    if ((rc = ctx->pr_levels.ensure(sizeof(dk::RoundLevel) * DK_MAX_LEVELS))) return rc;
    if ((rc = ctx->pr_tasks.ensure(sizeof(dk::RoundTask) * max_seg))) return rc;
    if ((rc = ctx->pr_ntasks.ensure(sizeof(uint32_t)))) return rc;
    if ((rc = ctx->pr_head.ensure(sizeof(uint32_t)))) return rc;
    if ((rc = ctx->pr_task_mom.ensure(sizeof(double) * 2 * nmom * max_seg))) return rc;
    if ((rc = ctx->pr_scratch.ensure(sizeof(double) * stride * grid))) return rc;
    const size_t host_bytes = sizeof(dk::RoundLevel) * DK_MAX_LEVELS + sizeof(dk::RoundTask) * max_seg + 64 +
                              sizeof(double) * 2 * nmom * max_seg;
    if (host_bytes > ctx->pr_host_bytes) {
        if (ctx->pr_host) { (void)hipHostFree(ctx->pr_host); ctx->pr_host = nullptr; ctx->pr_host_bytes = 0; }
        if (hipHostMalloc(&ctx->pr_host, host_bytes, hipHostMallocDefault) != hipSuccess)
            return fail(DK_ENOMEM, "hipHostMalloc(%zu) failed", host_bytes);
        ctx->pr_host_bytes = host_bytes;
    }
    const void* after[6] = {ctx->pr_levels.p, ctx->pr_tasks.p, ctx->pr_ntasks.p, ctx->pr_head.p, ctx->pr_task_mom.p,
                            ctx->pr_scratch.p};
    bool moved = std::memcmp(before, after, sizeof(before)) != 0;
    if (!ctx->pr_exec || moved || ctx->pr_flux != p->flux || ctx->pr_args.n_obs != nobs) {
        if (ctx->pr_exec) { (void)hipGraphExecDestroy(ctx->pr_exec); ctx->pr_exec = nullptr; }
        if (ctx->pr_graph) { (void)hipGraphDestroy(ctx->pr_graph); ctx->pr_graph = nullptr; }
        dk::RoundArgs P{};
        P.levels = (const dk::RoundLevel*)ctx->pr_levels.p;
        P.tasks = (const dk::RoundTask*)ctx->pr_tasks.p;
        P.ntasks = (const uint32_t*)ctx->pr_ntasks.p;
        P.head = (uint32_t*)ctx->pr_head.p;
        P.task_mom = (double*)ctx->pr_task_mom.p;
        P.scratch = (double*)ctx->pr_scratch.p;
        P.scratch_stride = stride;
        P.n_obs = nobs;
        if (!ctx->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
        const hipError_t el = dk::launch_round(P, p->flux, grid, ctx->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &g);
        if (el != hipSuccess) { if (g) (void)hipGraphDestroy(g); return fail(DK_EDEVICE, "round launch: %s", hipGetErrorString(el)); }
        if (ec != hipSuccess) return fail(DK_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ec));
        ctx->pr_graph = g;
        HIP_TRY(hipGraphInstantiate(&ctx->pr_exec, g, nullptr, nullptr, 0));
        ctx->pr_args = P;
        ctx->pr_flux = p->flux;
    }
    char* hb = (char*)ctx->pr_host;
    dk::RoundLevel* h_lv = (dk::RoundLevel*)hb;
    dk::RoundTask* h_tasks = (dk::RoundTask*)(hb + sizeof(dk::RoundLevel) * DK_MAX_LEVELS);
    uint32_t* h_nt = (uint32_t*)((char*)h_tasks + sizeof(dk::RoundTask) * max_seg);
    double* h_mom = (double*)((char*)h_nt + 64);
    for (int l = 0; l <= L; ++l) h_lv[l] = lv[l];
    HIP_TRY(hipMemcpyAsync(ctx->pr_levels.p, h_lv, sizeof(dk::RoundLevel) * (L + 1), hipMemcpyHostToDevice, s));
    const bool log = std::getenv("DK_LOG") != nullptr;
    KStat& rs = ctx->stats[std::make_pair(-1, 0)];
    rs.rows = 8;
    for (size_t k = 0; k + 1 < seg.size(); ++k) {
        const size_t t0 = seg[k], t1 = seg[k + 1], nt = t1 - t0;
        std::memcpy(h_tasks, &tasks[t0], sizeof(dk::RoundTask) * nt);
        *h_nt = (uint32_t)nt;
        HIP_TRY(hipMemcpyAsync(ctx->pr_tasks.p, h_tasks, sizeof(dk::RoundTask) * nt, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(ctx->pr_ntasks.p, h_nt, sizeof(uint32_t), hipMemcpyHostToDevice, s));
        HIP_TRY(hipEventRecord(ctx->pr_t0, s));
        HIP_TRY(hipGraphLaunch(ctx->pr_exec, s));
        HIP_TRY(hipEventRecord(ctx->pr_t1, s));
        HIP_TRY(hipMemcpyAsync(h_mom, ctx->pr_task_mom.p, sizeof(double) * 2 * nmom * nt, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ctx->pr_t0, ctx->pr_t1));
        double seg_cells = 0;
        uint64_t seg_samples = 0;
        for (size_t t = t0; t < t1; ++t) {
            const dk::RoundTask& T = tasks[t];
            for (int j = 0; j < nobs; ++j)
                merge_moments(sums[(size_t)T.level * nobs + j], &h_mom[((t - t0) * nobs + j) * DK_NMOM * 2], T.count);
            KStat& st = ctx->stats[std::make_pair((int)T.level, T.level >= 1 ? 1 : 0)];
            st.samples += T.count;
            st.cells += work[t];
            st.rows = 8;
            seg_cells += work[t];
            seg_samples += T.count;
        }
        rs.launches += 1;
        rs.samples += seg_samples;
        rs.cells += seg_cells;
        rs.ms += ms;
        ctx->round_ms += ms;
        ctx->round_graphs += 1;
        if (cell_updates) *cell_updates += seg_cells;
        if (log) {
            std::fprintf(stderr, "[dk] persistent round segment %zu/%zu: %zu tasks, %.3g cell updates, %.1f ms (%.3g /s)\n",
                         k + 1, seg.size() - 1, nt, seg_cells, ms, seg_cells / (ms * 1e-3));
            std::fflush(stderr);
        }
    }
    for (int l = 0; l <= L; ++l)
        for (int j = 0; j < nobs && count[l] > 0; ++j)
            for (int m = 0; m < DK_NMOM; ++m)
                if (!std::isfinite(mom_value(sums[(size_t)l * nobs + j], m)))
                    return fail(DK_ENUMERIC, "non-finite sample values on level %d", l);
    return DK_OK;
}

// ------------------------------------------------------------------------------------------
// Algorithm 1 (Sec. 7), independent of how samples are produced.
// ------------------------------------------------------------------------------------------
dk_mlmc_opts default_opts()
{
    dk_mlmc_opts o;
    std::memset(&o, 0, sizeof(o));
    o.m_pilot = 1000;
    o.L_start = 2;
    o.alpha = 2.0;
    o.max_rounds = 1000;
    o.plain_mc_level = -1;
    o.max_samples = 0;
    return o;
}

double bias_remainder(const std::vector<double>& Y, int L, double alpha, double ratio)
{
    // eq. (convergence_criterion) with the refinement ratio h_{l-1}/h_l (2 in the paper)
    double r = 0.0;
    for (int j = 0; j <= std::min(2, L); ++j) r = std::max(r, std::pow(ratio, -j * alpha) * std::fabs(Y[L - j]));
    return r / (std::pow(ratio, alpha) - 1.0);
}

// ------------------------------------------------------------------------------------------
// Algorithm-1 checkpoints: after every completed round the state (level, round count, samples
// done and targeted, compensated sums, and whatever the sampler adds) is written as text, doubles
// as their bit patterns, to path.tmp and renamed over path.  A run that finds the file resumes
// from it; since the sample ranges of every round follow from that state and the noise is a pure
// function of the sample index, the resumed run reproduces the uninterrupted one bit for bit.
// ------------------------------------------------------------------------------------------
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

uint64_t alg1_key(double eps, int L_max, const double* cost, const dk_mlmc_opts& o)
{
    Fnv f;
    f.val(eps); f.val(L_max);
    for (int l = 0; l <= L_max; ++l) f.val(cost[l]);
    f.val(o.m_pilot); f.val(o.L_start); f.val(o.alpha); f.val(o.max_samples); f.val(o.cost_model);
    return f.h;
}

std::string hex_bits(double v)
{
    uint64_t b;
    std::memcpy(&b, &v, 8);
    char buf[24];
    std::snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)b);
    return buf;
}

double from_bits(const std::string& t)
{
    const uint64_t b = std::strtoull(t.c_str(), nullptr, 16);
    double v;
    std::memcpy(&v, &b, 8);
    return v;
}

struct Alg1State {
    int L = 0, rounds = 0;
    std::vector<uint64_t> done, target;
    std::vector<double> s1, c1, s2, c2, extra;
};

int write_checkpoint(const char* path, uint64_t key, const Alg1State& S)
{
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return fail(DK_EINVAL, "cannot write checkpoint %s", tmp.c_str());
        char k[24];
        std::snprintf(k, sizeof(k), "%016llx", (unsigned long long)key);
        f << "dk-alg1-checkpoint 1\nkey " << k << "\nL " << S.L << " rounds " << S.rounds << " levels "
          << S.done.size() << "\n";
        for (size_t l = 0; l < S.done.size(); ++l)
            f << S.done[l] << " " << S.target[l] << " " << hex_bits(S.s1[l]) << " " << hex_bits(S.c1[l]) << " "
              << hex_bits(S.s2[l]) << " " << hex_bits(S.c2[l]) << "\n";
        f << "extra " << S.extra.size();
        for (double v : S.extra) f << " " << hex_bits(v);
        f << "\nend\n";
        if (!f) return fail(DK_EINVAL, "cannot write checkpoint %s", tmp.c_str());
    }
    if (std::rename(tmp.c_str(), path) != 0) return fail(DK_EINVAL, "cannot rename checkpoint to %s", path);
    return DK_OK;
}

// 1: state loaded; 0: no file; < 0: error (unreadable, another run's file, wrong shape)
int read_checkpoint(const char* path, uint64_t key, int levels, Alg1State& S)
{
    std::ifstream f(path);
    if (!f) return 0;
    std::string w, k;
    int version = 0;
    size_t nl = 0;
    if (!(f >> w >> version) || w != "dk-alg1-checkpoint" || version != 1)
        return fail(DK_EINVAL, "%s is not an Algorithm-1 checkpoint", path);
    char want[24];
    std::snprintf(want, sizeof(want), "%016llx", (unsigned long long)key);
    if (!(f >> w >> k) || w != "key") return fail(DK_EINVAL, "checkpoint %s: no key", path);
    if (k != want) return fail(DK_EINVAL, "checkpoint %s belongs to another run (problem, eps or options differ)", path);
    std::string wl, wr, wv;
    if (!(f >> wl >> S.L >> wr >> S.rounds >> wv >> nl) || wl != "L" || wr != "rounds" || wv != "levels" ||
        (int)nl != levels || S.L < 0 || S.L >= levels || S.rounds < 0)
        return fail(DK_EINVAL, "checkpoint %s: bad header", path);
    S.done.assign(nl, 0); S.target.assign(nl, 0);
    S.s1.assign(nl, 0); S.c1.assign(nl, 0); S.s2.assign(nl, 0); S.c2.assign(nl, 0);
    for (size_t l = 0; l < nl; ++l) {
        std::string a, b, c, d;
        if (!(f >> S.done[l] >> S.target[l] >> a >> b >> c >> d)) return fail(DK_EINVAL, "checkpoint %s: bad level line", path);
        S.s1[l] = from_bits(a); S.c1[l] = from_bits(b); S.s2[l] = from_bits(c); S.c2[l] = from_bits(d);
    }
    size_t ne = 0;
    if (!(f >> w >> ne) || w != "extra" || ne > (1u << 24)) return fail(DK_EINVAL, "checkpoint %s: bad extra", path);
    S.extra.resize(ne);
    for (size_t i = 0; i < ne; ++i) {
        if (!(f >> w)) return fail(DK_EINVAL, "checkpoint %s: truncated", path);
        S.extra[i] = from_bits(w);
    }
    if (!(f >> w) || w != "end") return fail(DK_EINVAL, "checkpoint %s: truncated", path);
    return 1;
}

// optional: all levels of one round at once; sums [L+1][2]
typedef int (*round_sampler)(void* user, int L, const uint64_t* first, const uint64_t* count, double* sums);

// measure(L, C): optional; with DK_COST_MEASURED it replaces C[0..L] by measured costs after a round
typedef std::function<void(int, std::vector<double>&)> cost_measure;

int alg1_core(double eps, int L_max, const double* cost, const dk_mlmc_opts& o, dk_level_sampler sampler, void* user,
              dk_mlmc_result* out, round_sampler rsampler = nullptr, const CkptHooks* ck = nullptr,
              const cost_measure* measure = nullptr, double ratio = 2.0)
{
    if (!(eps > 0)) return fail(DK_EINVAL, "eps must be > 0");
    if (L_max < 0 || L_max >= DK_MAX_LEVELS) return fail(DK_EINVAL, "L_max out of range");
    if (o.m_pilot < 2) return fail(DK_EINVAL, "m_pilot must be >= 2");
    for (int l = 0; l <= L_max; ++l)
        if (!(cost[l] > 0)) return fail(DK_EINVAL, "cost[%d] must be > 0", l);
    if (o.cost_model != DK_COST_CELLS && o.cost_model != DK_COST_MEASURED)
        return fail(DK_EINVAL, "cost_model must be DK_COST_CELLS or DK_COST_MEASURED");
    std::vector<double> C(cost, cost + L_max + 1);   // costs in use (measured ones replace these)
    int L = std::min(std::max(o.L_start, 0), L_max);
    std::vector<uint64_t> done(L_max + 1, 0), target(L_max + 1, 0);
    std::vector<double> s1(L_max + 1, 0), c1(L_max + 1, 0), s2(L_max + 1, 0), c2(L_max + 1, 0);
    for (int l = 0; l <= L; ++l) target[l] = (uint64_t)o.m_pilot;
    std::vector<double> Y(L_max + 1, 0), V(L_max + 1, 0);
    auto stats = [&](int upto) {
        for (int l = 0; l <= upto; ++l) {
            const double n = (double)done[l];
            const double m1 = (s1[l] + c1[l]) / n;
            Y[l] = m1;
            V[l] = done[l] > 1 ? std::max(0.0, ((s2[l] + c2[l]) - n * m1 * m1) / (n - 1.0)) : 0.0;
        }
    };
    int rounds = 0;
    bool conv = false;
    const char* ckpath = o.checkpoint_path && *o.checkpoint_path ? o.checkpoint_path : nullptr;
    const uint64_t ckkey = alg1_key(eps, L_max, cost, o) ^ (ck ? ck->key * 0x9E3779B97F4A7C15ull : 0);
    if (ckpath) {
        Alg1State S;
        const int rc = read_checkpoint(ckpath, ckkey, L_max + 1, S);
        if (rc < 0) return rc;
        if (rc == 1) {
            L = S.L; rounds = S.rounds; done = S.done; target = S.target;
            s1 = S.s1; c1 = S.c1; s2 = S.s2; c2 = S.c2;
            if (ck && ck->load) {
                const int lr = ck->load(S.extra);
                if (lr < 0) return lr;
            }
            if (std::getenv("DK_LOG")) {
                std::fprintf(stderr, "[dk] resumed from %s after round %d (L=%d)\n", ckpath, rounds, L);
                std::fflush(stderr);
            }
        }
    }
    for (;;) {
        bool need = false;
        for (int l = 0; l <= L; ++l) need |= target[l] > done[l];
        if (!need) {
            stats(L);
            if (L >= 2 || L == L_max) {
                if (bias_remainder(Y, L, o.alpha, ratio) < eps / std::sqrt(2.0)) { conv = true; break; }
            }
            if (L == L_max) { conv = false; break; }
            L += 1;
            target[L] = (uint64_t)o.m_pilot;
            continue;
        }
        if (rounds >= o.max_rounds) return fail(DK_EINVAL, "Algorithm 1 exceeded max_rounds = %d", o.max_rounds);
        ++rounds;
        if (rsampler) {
            std::vector<uint64_t> f(L + 1), c(L + 1);
            std::vector<double> sums(2 * (L + 1), 0.0);
            for (int l = 0; l <= L; ++l) {
                f[l] = done[l];
                c[l] = target[l] > done[l] ? target[l] - done[l] : 0;
            }
            const int rc = rsampler(user, L, f.data(), c.data(), sums.data());
            if (rc < 0) return rc;
            for (int l = 0; l <= L; ++l) {
                if (c[l] == 0) continue;
                if (!std::isfinite(sums[2 * l]) || !std::isfinite(sums[2 * l + 1]))
                    return fail(DK_ENUMERIC, "non-finite sums on level %d", l);
                nadd(s1[l], c1[l], sums[2 * l]);
                nadd(s2[l], c2[l], sums[2 * l + 1]);
                done[l] += c[l];
            }
        } else {
            for (int l = 0; l <= L; ++l) {
                if (target[l] <= done[l]) continue;
                const uint64_t extra = target[l] - done[l];
                double sums[2] = {0, 0};
                const int rc = sampler(user, l, done[l], extra, sums);
                if (rc < 0) return rc;
                if (!std::isfinite(sums[0]) || !std::isfinite(sums[1])) return fail(DK_ENUMERIC, "non-finite sums on level %d", l);
                nadd(s1[l], c1[l], sums[0]);
                nadd(s2[l], c2[l], sums[1]);
                done[l] += extra;
            }
        }
        stats(L);
        if (std::getenv("DK_LOG")) {
            std::fprintf(stderr, "[dk] round %d L=%d", rounds, L);
            for (int l = 0; l <= L; ++l) std::fprintf(stderr, " | l%d M=%llu Y=%.4g V=%.4g", l, (unsigned long long)done[l], Y[l], V[l]);
            std::fprintf(stderr, "\n");
            std::fflush(stderr);
        }
        if (o.cost_model == DK_COST_MEASURED && measure && *measure) (*measure)(L, C);
        double acc = 0.0;
        for (int l = 0; l <= L; ++l) acc += std::sqrt(V[l] * C[l]);
        for (int l = 0; l <= L; ++l) {
            const double m = std::ceil(2.0 / (eps * eps) * std::sqrt(V[l] / C[l]) * acc);
            uint64_t mi = m > 1.8e19 ? (uint64_t)1.8e19 : (uint64_t)m;
            if (o.max_samples && mi > o.max_samples) mi = o.max_samples;
            target[l] = std::max(done[l], mi);
        }
        if (ckpath) {
            Alg1State S;
            S.L = L; S.rounds = rounds; S.done = done; S.target = target;
            S.s1 = s1; S.c1 = c1; S.s2 = s2; S.c2 = c2;
            if (ck && ck->save) ck->save(S.extra);
            const int rc = write_checkpoint(ckpath, ckkey, S);
            if (rc < 0) return rc;
        }
    }
    stats(L);
    std::memset(out, 0, sizeof(*out));
    double est = 0.0, var = 0.0;
    for (int l = 0; l <= L; ++l) {
        out->M[l] = done[l];
        out->Yhat[l] = Y[l];
        out->Vhat[l] = V[l];
        out->cost[l] = C[l];
        est += Y[l];
        var += V[l] / (double)done[l];
    }
    out->estimate[0] = est;
    out->var_est[0] = var;
    out->L = L;
    out->converged = conv ? 1 : 0;
    out->rounds = rounds;
    out->bias_est = bias_remainder(Y, L, o.alpha, ratio);
    out->rmse_est = std::sqrt(var + out->bias_est * out->bias_est);
    return conv ? DK_OK : DK_WARN_NOT_CONVERGED;
}

// ------------------------------------------------------------------------------------------
// Learned control variate
// ------------------------------------------------------------------------------------------
int ensure_rbar(dk_context* ctx, const dk_problem* p, int level, LevelTables** out, hipStream_t s)
{
    LevelTables* T = nullptr;
    int rc = ensure_level(ctx, p, level, &T, s);
    if (rc) return rc;
    if (!T->have_rbar) {
        rc = T->rbar.ensure(sizeof(double) * (size_t)T->n * T->n);
        if (rc) return rc;
        rc = compute_centre(ctx, p, level, *T, s, (double*)T->rbar.p);
        if (rc) return rc;
        T->have_rbar = true;
    }
    *out = T;
    return DK_OK;
}

constexpr int kCnnBatch = 1024;   // inputs per network launch sequence

// r[count] = network(x[count][n][n]) in batches of kCnnBatch
int cnn_forward_batched(dk_context* ctx, const float* prm, int n, uint64_t count, const float* x, float* r, hipStream_t s)
{
    if (count == 0) return DK_OK;
    HIP_TRY(ctx->cnn.reserve(n, kCnnBatch));
    HIP_TRY(dk::cnn::pack(ctx->cnn, prm, s));
    for (uint64_t b = 0; b < count; b += kCnnBatch) {
        const int c = (int)std::min<uint64_t>(kCnnBatch, count - b);
        HIP_TRY(dk::cnn::forward(ctx->cnn, prm, x + b * n * n, c, r + b, s));
    }
    return DK_OK;
}

// Control-variate samples of level l >= 1: Z_i = (Y_i - r(x_i)) + mean_j r(x'_{k i + j}).
// sums_out [n_obs] receives the plain pair moments (all observables); zsum receives the
// moments of Z in the Y slots.
int run_cv_level(dk_context* ctx, const dk_problem* p, int level, uint64_t first, uint64_t count, const float* prm_host,
                 int kappa, dk_moments* sums_out, dk_moments& zsum, hipStream_t s, double* cell_updates)
{
    const int nobs = p->n_obs;
    const int nc = p->n0 << (level - 1);
    const size_t nn = (size_t)nc * nc;
    LevelTables* Tc = nullptr;
    int rc = ensure_rbar(ctx, p, level - 1, &Tc, s);
    if (rc) return rc;
    const double scale = std::sqrt(p->N) * Tc->h;
    const bool f64 = p->precision == DK_PREC_F64;
    const size_t es = f64 ? 8 : 4;
    // sub-batches bounded by the field buffers (pair fields + kappa coarse-only fields)
    const uint64_t cap = std::max<uint64_t>(256, (uint64_t)((1ull << 30) / (nn * (es + 4) * (1 + kappa))));
    rc = ctx->cv_prm.ensure(sizeof(float) * dk::cnn::NPARAM);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(ctx->cv_prm.p, prm_host, sizeof(float) * dk::cnn::NPARAM, hipMemcpyHostToDevice, s));
    const uint64_t S = std::min(cap, count);
    if ((rc = ctx->cv_fields.ensure(es * nn * S))) return rc;
    if ((rc = ctx->cv_x.ensure(4 * nn * S))) return rc;
    if ((rc = ctx->cv_r.ensure(4 * S))) return rc;
    if ((rc = ctx->cv_ps.ensure(16 * (size_t)nobs * S))) return rc;
    if ((rc = ctx->cv_fields2.ensure(es * nn * S * kappa))) return rc;
    if ((rc = ctx->cv_x2.ensure(4 * nn * S * kappa))) return rc;
    if ((rc = ctx->cv_r2.ensure(4 * S * kappa))) return rc;
    if ((rc = ctx->cv_ps2.ensure(16 * (size_t)nobs * S * kappa))) return rc;
    if ((rc = ctx->cv_z.ensure(16 * S))) return rc;
    for (int j = 0; j < nobs; ++j) std::memset(&sums_out[j], 0, sizeof(dk_moments));
    std::memset(&zsum, 0, sizeof(zsum));
    std::vector<dk_moments> part(nobs), part2(nobs);
    for (uint64_t b = 0; b < count; b += S) {
        const uint64_t c = std::min(S, count - b);
        rc = run_level(ctx, p, level, true, first + b, c, DK_TAG_MLMC, part.data(), (double*)ctx->cv_ps.p, nullptr,
                       ctx->cv_fields.p, s, cell_updates);
        if (rc < 0) return rc;
        for (int j = 0; j < nobs; ++j) {
            sums_out[j].count += part[j].count;
            for (int k = 0; k < DK_NMOM; ++k) {
                nadd(sums_out[j].sum[k], sums_out[j].comp[k], part[j].sum[k]);
                sums_out[j].comp[k] += part[j].comp[k];
            }
        }
        HIP_TRY(dk::cnn::normalize(ctx->cv_fields.p, f64, (const double*)Tc->rbar.p, (int)nn, nn * c, scale,
                                   (float*)ctx->cv_x.p, s));
        rc = cnn_forward_batched(ctx, (const float*)ctx->cv_prm.p, nc, c, (const float*)ctx->cv_x.p, (float*)ctx->cv_r.p, s);
        if (rc) return rc;
        // independent coarse-only paths k (first + b) .. k (first + b + c)
        rc = run_level(ctx, p, level - 1, false, (first + b) * kappa, c * kappa, DK_TAG_CV_COARSE, part2.data(),
                       (double*)ctx->cv_ps2.p, ctx->cv_fields2.p, nullptr, s, cell_updates);
        if (rc < 0) return rc;
        HIP_TRY(dk::cnn::normalize(ctx->cv_fields2.p, f64, (const double*)Tc->rbar.p, (int)nn, nn * c * kappa, scale,
                                   (float*)ctx->cv_x2.p, s));
        rc = cnn_forward_batched(ctx, (const float*)ctx->cv_prm.p, nc, c * kappa, (const float*)ctx->cv_x2.p,
                                 (float*)ctx->cv_r2.p, s);
        if (rc) return rc;
        HIP_TRY(dk::cnn::combine_cv((const double*)ctx->cv_ps.p, nobs, p->primary_obs, (const float*)ctx->cv_r.p,
                                    (const float*)ctx->cv_r2.p, kappa, (int)c, (double*)ctx->cv_z.p, s));
        rc = ctx->moments.ensure(sizeof(double) * DK_NMOM * 2);
        if (rc) return rc;
        HIP_TRY(dk::launch_moments((const double*)ctx->cv_z.p, c, 1, (double*)ctx->moments.p, s));
        double h[DK_NMOM * 2];
        HIP_TRY(hipMemcpyAsync(h, ctx->moments.p, sizeof(h), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        merge_moments(zsum, h, c);
    }
    if (!std::isfinite(mom_value(zsum, DK_MOM_Y)) || !std::isfinite(mom_value(zsum, DK_MOM_Y2)))
        return fail(DK_ENUMERIC, "non-finite control-variate samples on level %d", level);
    return DK_OK;
}

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

int gpu_sample(void* user, int32_t level, uint64_t first, uint64_t count, double* sums)
{
    GpuSampler& G = *(GpuSampler*)user;
    const int nobs = G.p->n_obs;
    G.tmp.assign(nobs, dk_moments{});
    const bool pair = !G.plain_mc && level >= 1;
    const bool cv = pair && G.cv_params && ((G.cv_mask >> level) & 1u);
    dk_moments z{};
    const int rc = cv ? run_cv_level(G.ctx, G.p, level, first, count, G.cv_params + (size_t)level * dk::cnn::NPARAM,
                                     G.cv_ratio, G.tmp.data(), z, G.s, &G.cell_updates)
                      : run_level(G.ctx, G.p, level, pair, first, count, G.tag, G.tmp.data(), nullptr, nullptr, nullptr,
                                  G.s, &G.cell_updates);
    if (rc < 0) return rc;
    if (cv) {
        dk_moments& d = G.zmom[level];
        d.count += z.count;
        for (int k = 0; k < DK_NMOM; ++k) {
            nadd(d.sum[k], d.comp[k], z.sum[k]);
            d.comp[k] += z.comp[k];
        }
        sums[0] = mom_value(z, DK_MOM_Y);
        sums[1] = mom_value(z, DK_MOM_Y2);
    }
    for (int j = 0; j < nobs; ++j) {
        dk_moments& d = G.mom[(size_t)level * nobs + j];
        d.count += G.tmp[j].count;
        for (int k = 0; k < DK_NMOM; ++k) {
            nadd(d.sum[k], d.comp[k], G.tmp[j].sum[k]);
            d.comp[k] += G.tmp[j].comp[k];
        }
    }
    if (!cv) {
        const dk_moments& pm = G.tmp[G.p->primary_obs];
        sums[0] = mom_value(pm, DK_MOM_Y);
        sums[1] = mom_value(pm, DK_MOM_Y2);
    }
    return DK_OK;
}


// A whole round: resident, non-control-variate levels together (run_round), the rest one by one.
int gpu_round(void* user, int L, const uint64_t* first, const uint64_t* count, double* sums)
{
    GpuSampler& G = *(GpuSampler*)user;
    const int nobs = G.p->n_obs;
    std::vector<uint64_t> cnt(count, count + L + 1);
    for (int l = 0; l <= L; ++l) {
        const int nf = level_n(G.p, l);
        const bool cv = l >= 1 && G.cv_params && ((G.cv_mask >> l) & 1u);
        const bool streamed = !fourier(G.p) && (!dk::level_supported(nf) || (G.ctx->force_stream && dk::stream_supported(nf)));
        const bool outside = fourier(G.p) || implicit(G.p) ||
                             (G.round_mode == 3 && G.p->precision == DK_PREC_F32 && !round_eligible(G.p, l, G.ctx->force_stream));
        if ((cv || streamed || outside || G.plain_mc) && count[l] > 0) {
            double s2[2] = {0, 0};
            const int rc = gpu_sample(user, l, first[l], count[l], s2);
            if (rc < 0) return rc;
            sums[2 * l] = s2[0];
            sums[2 * l + 1] = s2[1];
            cnt[l] = 0;
        }
    }
    std::vector<dk_moments> rs((size_t)(L + 1) * nobs);
    // persistent rounds need FP32 states; FP64 problems take the concurrent-stream round instead
    const bool persistent = G.round_mode == 3 && G.p->precision == DK_PREC_F32 && nobs <= dk::round_max_obs();
    const int rc = persistent ? run_round_persistent(G.ctx, G.p, L, first, cnt.data(), G.tag, rs, G.s, &G.cell_updates)
                              : run_round(G.ctx, G.p, L, first, cnt.data(), G.tag, G.round_mode == 3 ? 1 : G.round_mode, rs, G.s,
                                          &G.cell_updates);
    if (rc < 0) return rc;
    for (int l = 0; l <= L; ++l) {
        if (cnt[l] == 0) continue;
        for (int j = 0; j < nobs; ++j) {
            dk_moments& d = G.mom[(size_t)l * nobs + j];
            const dk_moments& r = rs[(size_t)l * nobs + j];
            d.count += r.count;
            for (int k = 0; k < DK_NMOM; ++k) {
                nadd(d.sum[k], d.comp[k], r.sum[k]);
                d.comp[k] += r.comp[k];
            }
        }
        const dk_moments& pm = rs[(size_t)l * nobs + G.p->primary_obs];
        sums[2 * l] = mom_value(pm, DK_MOM_Y);
        sums[2 * l + 1] = mom_value(pm, DK_MOM_Y2);
    }
    return DK_OK;
}

double level_cost(const dk_problem* p, long steps0, int level, bool pair)
{
    const double n = (double)level_n(p, level);
    return n * n * (double)level_steps(p, steps0, level) * (pair && level >= 1 ? pair_factor(p) : 1.0);
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Allocation-free batch of one resident level: every device buffer, the level tables and the
// centring run included, is carved from the caller's arena (no cache, nothing allocated, no
// events).  Same kernels and the default tile shape as run_level; the chunks are bounded by the
// arena as well as by the launch cap, so moment sums may be grouped differently (rounding-level
// differences only); per-sample values are identical.
// ------------------------------------------------------------------------------------------
namespace dk {

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }

namespace {

struct Carve {
    char* base;
    size_t cap, used = 0;
    bool ok = true;
    void* take(size_t bytes)
    {
        const size_t off = (used + 255) & ~(size_t)255;
        if (off > cap || bytes > cap - off) { ok = false; return nullptr; }
        used = off + bytes;
        return base + off;
    }
};

// I_h rho0 (state type), I_h phi_j and the per-observable {scale, centre, psi} of level l into
// the arena; the centring constants from a noise-free FP64 run in `tmp` (8 n^2 + 40 n_obs bytes).
int arena_tables(const dk_problem* p, int l, void* rho0, double* phi, double* obs, void* tmp, hipStream_t s)
{
    const int n = level_n(p, l), nobs = p->n_obs;
    const double h = p->box / n;
    const bool f64 = p->precision == DK_PREC_F64;
    HIP_TRY(dk::launch_field_eval(to_dev_on(p, p->rho0, n), p->box, n, rho0, f64, s));
    for (int j = 0; j < nobs; ++j)
        HIP_TRY(dk::launch_field_eval(to_dev_on(p, p->obs[j].phi, n), p->box, n, phi + (size_t)j * n * n, true, s));
    double centre[DK_MAX_OBS] = {0};
    bool any = false;
    for (int j = 0; j < nobs; ++j) any |= p->obs[j].centre != 0;
    double unit[3 * DK_MAX_OBS], res[2 * DK_MAX_OBS], host_obs[3 * DK_MAX_OBS];
    if (any) {
        double* r0 = (double*)tmp;
        double* obs_unit = r0 + (size_t)n * n;
        double* out = obs_unit + 3 * nobs;
        HIP_TRY(dk::launch_field_eval(to_dev_on(p, p->rho0, n), p->box, n, r0, true, s));
        for (int j = 0; j < nobs; ++j) { unit[3 * j] = 1.0; unit[3 * j + 1] = 0.0; unit[3 * j + 2] = 0.0; }
        HIP_TRY(hipMemcpyAsync(obs_unit, unit, sizeof(double) * 3 * nobs, hipMemcpyHostToDevice, s));
        dk::LevelArgs A{};
        A.nf = n; A.level_id = l; A.count = 1; A.steps = (int)level_steps(p, steps0_of(p), l);
        A.a = 0.5 * p->mu; A.h2f = h * h; A.rho0_f = r0; A.phi_f = phi; A.obs_f = obs_unit; A.n_obs = nobs; A.out = out;
        HIP_TRY(dk::launch_level(dk::LevelKind{DK_PREC_F64, false, DK_FLUX_CENTRAL, false}, A, s));
        HIP_TRY(hipMemcpyAsync(res, out, sizeof(double) * 2 * nobs, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int j = 0; j < nobs; ++j) centre[j] = res[2 * j];
    }
    for (int j = 0; j < nobs; ++j) {
        host_obs[3 * j + 0] = p->obs[j].scale_sqrtN ? std::sqrt(p->N) : 1.0;
        host_obs[3 * j + 1] = p->obs[j].centre ? centre[j] : 0.0;
        host_obs[3 * j + 2] = p->obs[j].psi == DK_PSI_SQUARE ? 1.0 : 0.0;
    }
    HIP_TRY(hipMemcpyAsync(obs, host_obs, sizeof(double) * 3 * nobs, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));   // the host sources above live on this stack frame
    return DK_OK;
}

}  // namespace

int level_pair_arena(const dk_problem* p, int level, uint64_t first, uint64_t count, uint32_t tag, dk_moments* sums_out,
                     double* per_sample_out, void* arena, size_t arena_bytes, hipStream_t s)
{
    if (!sums_out) return fail(DK_EINVAL, "sums_out is NULL");
    if (!arena) return fail(DK_EINVAL, "scratch arena is NULL");
    if (tag > 255) return fail(DK_EINVAL, "stream_tag must fit in 8 bits");
    int rc = validate(p);
    if (rc) return rc;
    if (level < 0 || level >= p->levels) return fail(DK_EINVAL, "level %d outside [0, %d)", level, p->levels);
    if (count > 0 && first + count < first) return fail(DK_EINVAL, "sample range overflows");
    if (first + count > (1ull << 48)) return fail(DK_EINVAL, "sample index beyond 2^48");
    if (fourier(p) || implicit(p))
        return fail(DK_EUNSUPPORTED, "the allocation-free entry point runs the explicit NN scheme only");
    const bool pair = level >= 1;
    const int nf = level_n(p, level), nc = nf / 2, nobs = p->n_obs;
    if (!dk::level_supported(nf))
        return fail(DK_EUNSUPPORTED, "grid %d x %d: the allocation-free entry point runs the resident grids (n <= 128)", nf, nf);
    for (int j = 0; j < nobs; ++j) std::memset(&sums_out[j], 0, sizeof(dk_moments));
    const size_t esize = p->precision == DK_PREC_F64 ? 8 : 4;
    const size_t nn = (size_t)nf * nf, ncc = (size_t)nc * nc;
    constexpr int kGroup = 8;                                  // chunks per moment read-back
    const size_t mom_stride = (size_t)nobs * DK_NMOM * 2;
    Carve C{(char*)arena, arena_bytes};
    void* rho0_f = C.take(esize * nn);
    double* phi_f = (double*)C.take(8 * nobs * nn);
    double* obs_f = (double*)C.take(8 * 3 * nobs);
    void* rho0_c = pair ? C.take(esize * ncc) : nullptr;
    double* phi_c = pair ? (double*)C.take(8 * nobs * ncc) : nullptr;
    double* obs_c = pair ? (double*)C.take(8 * 3 * nobs) : nullptr;
    void* tmp = C.take(8 * nn + 8 * 5 * (size_t)nobs);
    double* mom = (double*)C.take(8 * mom_stride * kGroup);
    if (!C.ok)
        return fail(DK_EINVAL, "level %d (%d x %d, %d observables) needs more than the %zu bytes of scratch of the "
                    "allocation-free entry point", level, nf, nf, nobs, arena_bytes);
    const double cells_per_sample = (double)nn * (double)level_steps(p, steps0_of(p), level) * (pair ? pair_factor(p) : 1.0);
    uint64_t ch = chunk_size(nobs, cells_per_sample, kMaxCellsPerLaunch);
    double* ps = per_sample_out;
    if (!ps) {
        const size_t off = (C.used + 255) & ~(size_t)255;
        const uint64_t fit = off < C.cap ? (C.cap - off) / (16 * (size_t)nobs) : 0;
        if (fit == 0)
            return fail(DK_EINVAL, "level %d (%d observables): no scratch left for per-sample values", level, nobs);
        ch = std::min<uint64_t>(ch, fit);
        ps = (double*)C.take(16 * (size_t)nobs * std::min<uint64_t>(ch, std::max<uint64_t>(count, 1)));
        if (!C.ok) return fail(DK_EINVAL, "scratch carve failed");
    }
    if ((rc = arena_tables(p, level, rho0_f, phi_f, obs_f, tmp, s))) return rc;
    if (pair && (rc = arena_tables(p, level - 1, rho0_c, phi_c, obs_c, tmp, s))) return rc;
    if (count == 0) return DK_OK;
    const double hf = p->box / nf, hc = 2.0 * hf;
    dk::LevelArgs A{};
    A.nf = nf; A.level_id = level; A.tag = tag; A.seed = p->seed;
    A.steps = (int)level_steps(p, steps0_of(p), level);
    A.a = 0.5 * p->mu;
    const double sig_f = std::sqrt(p->mu * hf * hf);
    A.kf = noise_coeff(p, hf, sig_f);
    A.kc = pair ? noise_coeff(p, hc, 0.5 * sig_f) : 0.0;
    A.h2f = hf * hf;
    A.h2c = pair ? hc * hc : 0.0;
    A.rho0_f = rho0_f; A.rho0_c = rho0_c; A.phi_f = phi_f; A.phi_c = phi_c; A.obs_f = obs_f; A.obs_c = obs_c;
    A.n_obs = nobs;
    const dk::LevelKind K{p->precision, pair, p->flux, true, 0};
    const uint64_t nchunks = (count + ch - 1) / ch;
    double host[kGroup * 2 * DK_NMOM * DK_MAX_OBS];
    for (uint64_t g0 = 0; g0 < nchunks; g0 += kGroup) {
        const uint64_t g1 = std::min<uint64_t>(nchunks, g0 + kGroup);
        for (uint64_t k = g0; k < g1; ++k) {
            const uint64_t b = k * ch, c = std::min(ch, count - b);
            A.first = first + b;
            A.count = c;
            A.out = per_sample_out ? per_sample_out + b * nobs * 2 : ps;
            HIP_TRY(dk::launch_level(K, A, s));
            HIP_TRY(dk::launch_moments(A.out, c, nobs, mom + (k - g0) * mom_stride, s));
        }
        HIP_TRY(hipMemcpyAsync(host, mom, sizeof(double) * mom_stride * (g1 - g0), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (uint64_t k = g0; k < g1; ++k) {
            const uint64_t c = std::min(ch, count - k * ch);
            for (int j = 0; j < nobs; ++j) merge_moments(sums_out[j], &host[(k - g0) * mom_stride + j * DK_NMOM * 2], c);
        }
    }
    for (int j = 0; j < nobs; ++j)
        for (int m = 0; m < DK_NMOM; ++m)
            if (!std::isfinite(mom_value(sums_out[j], m))) return fail(DK_ENUMERIC, "non-finite sample values on level %d", level);
    return DK_OK;
}

}  // namespace dk

// ============================================================================================
// C ABI
// ============================================================================================
extern "C" {

const char* dk_last_error(void) { return g_err; }

const char* dk_version(void) { return "dk_mlmc 0.1 (gfx950)"; }


int dk_cnn_init(uint64_t seed, float* params_out)
{
    if (!params_out) return fail(DK_EINVAL, "params_out is NULL");
    std::mt19937_64 gen(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    using namespace dk::cnn;
    auto he = [&](int off, int count, int fan_in) {
        const double sd = std::sqrt(2.0 / fan_in);
        for (int k = 0; k < count; ++k) params_out[off + k] = (float)(sd * nd(gen));
    };
    for (int k = 0; k < NPARAM; ++k) params_out[k] = 0.f;
    he(OFF_W1, 144, 9);
    he(OFF_W2, 2304, 144);
    he(OFF_W3, 2304, 144);
    he(OFF_U1, 1024, 16);
    he(OFF_U2, 64, 64);
    return DK_OK;
}

int dk_cnn_forward(dk_context* ctx, const float* params, int32_t n, int32_t batch, const float* x, float* r, void* stream)
{
    if (!ctx || !params || !x || !r) return fail(DK_EINVAL, "NULL argument");
    if (n < 4 || n % 4 || n > 1024 || batch < 0) return fail(DK_EINVAL, "n must be a multiple of 4 in [4, 1024]");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    int rc = ctx->cv_prm.ensure(sizeof(float) * dk::cnn::NPARAM);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(ctx->cv_prm.p, params, sizeof(float) * dk::cnn::NPARAM, hipMemcpyHostToDevice, s));
    rc = cnn_forward_batched(ctx, (const float*)ctx->cv_prm.p, n, (uint64_t)batch, x, r, s);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    return DK_OK;
}

int dk_cnn_loss_grad(dk_context* ctx, const float* params, int32_t n, int32_t batch, const float* x, const float* y,
                     float* grad_out, double* loss_out, void* stream)
{
    if (!ctx || !params || !x || !y || !grad_out) return fail(DK_EINVAL, "NULL argument");
    if (n < 4 || n % 4 || n > 1024 || batch < 1) return fail(DK_EINVAL, "n must be a multiple of 4 in [4, 1024]");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if ((rc = ctx->cv_prm.ensure(sizeof(float) * dk::cnn::NPARAM))) return rc;
    if ((rc = ctx->cv_grad.ensure(sizeof(float) * dk::cnn::NPARAM))) return rc;
    if ((rc = ctx->cv_r.ensure(sizeof(float) * batch))) return rc;
    if ((rc = ctx->cv_loss.ensure(sizeof(double)))) return rc;
    HIP_TRY(hipMemcpyAsync(ctx->cv_prm.p, params, sizeof(float) * dk::cnn::NPARAM, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(ctx->cv_loss.p, 0, sizeof(double), s));
    HIP_TRY(ctx->cnn.reserve(n, batch));
    HIP_TRY(dk::cnn::pack(ctx->cnn, (const float*)ctx->cv_prm.p, s));
    HIP_TRY(dk::cnn::forward(ctx->cnn, (const float*)ctx->cv_prm.p, x, batch, (float*)ctx->cv_r.p, s));
    HIP_TRY(dk::cnn::backward(ctx->cnn, (const float*)ctx->cv_prm.p, x, (const float*)ctx->cv_r.p, y, batch,
                              (float*)ctx->cv_grad.p, s));
    HIP_TRY(dk::cnn::accumulate_sq(ctx->cnn, batch, (double*)ctx->cv_loss.p, s));
    HIP_TRY(hipMemcpyAsync(grad_out, ctx->cv_grad.p, sizeof(float) * dk::cnn::NPARAM, hipMemcpyDeviceToHost, s));
    double l = 0;
    HIP_TRY(hipMemcpyAsync(&l, ctx->cv_loss.p, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (loss_out) *loss_out = l / batch;
    return DK_OK;
}

int dk_cv_train(dk_context* ctx, const dk_problem* problem, int32_t level, uint64_t n_train, int32_t epochs,
                int32_t batch, double lr, uint64_t n_val, float* params_inout, double* loss_hist, double* val_out,
                void* stream)
{
    if (!ctx || !params_inout) return fail(DK_EINVAL, "NULL argument");
    int rc = validate(problem);
    if (rc) return rc;
    if (level < 1 || level >= problem->levels) return fail(DK_EINVAL, "control variate needs 1 <= level < levels");
    if (epochs < 1 || batch < 1 || n_train < (uint64_t)batch) return fail(DK_EINVAL, "need epochs >= 1 and n_train >= batch >= 1");
    if (!(lr > 0)) return fail(DK_EINVAL, "lr must be > 0");
    if (fourier(problem) || implicit(problem)) return fail(DK_EUNSUPPORTED, "the control variate is built for the explicit NN scheme");
    const int nc = problem->n0 << (level - 1);
    if (nc % 4) return fail(DK_EINVAL, "coarse grid must be a multiple of 4");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int nobs = problem->n_obs;
    const size_t nn = (size_t)nc * nc;
    const bool f64 = problem->precision == DK_PREC_F64;
    const size_t es = f64 ? 8 : 4;
    LevelTables* Tc = nullptr;
    if ((rc = ensure_rbar(ctx, problem, level - 1, &Tc, s))) return rc;
    const double scale = std::sqrt(problem->N) * Tc->h;
    const uint64_t ntot = n_train + n_val;
    // training (and validation) pairs from the DK_TAG_CV_TRAIN stream
    DevBuf fields, X, Y, PS;
    if ((rc = fields.ensure(es * nn * ntot))) return rc;
    if ((rc = X.ensure(4 * nn * ntot))) return rc;
    if ((rc = Y.ensure(4 * ntot))) return rc;
    if ((rc = PS.ensure(16 * (size_t)nobs * ntot))) return rc;
    std::vector<dk_moments> mom(nobs);
    rc = run_level(ctx, problem, level, true, 0, ntot, DK_TAG_CV_TRAIN, mom.data(), (double*)PS.p, nullptr, fields.p, s,
                   nullptr);
    if (rc < 0) return rc;
    HIP_TRY(dk::cnn::normalize(fields.p, f64, (const double*)Tc->rbar.p, (int)nn, nn * ntot, scale, (float*)X.p, s));
    HIP_TRY(dk::cnn::extract_y((const double*)PS.p, nobs, problem->primary_obs, (int)ntot, (float*)Y.p, s));
    // standardise the targets (training part); the scaling is folded back into the last layer
    std::vector<float> yh(ntot);
    HIP_TRY(hipMemcpyAsync(yh.data(), Y.p, 4 * ntot, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double ym = 0, yv = 0;
    for (uint64_t i = 0; i < n_train; ++i) ym += yh[i];
    ym /= (double)n_train;
    for (uint64_t i = 0; i < n_train; ++i) yv += (yh[i] - ym) * (yh[i] - ym);
    const double ysd = std::sqrt(std::max(yv / std::max<double>(1.0, (double)n_train - 1), 1e-300));
    std::vector<float> ys(n_train);
    for (uint64_t i = 0; i < n_train; ++i) ys[i] = (float)((yh[i] - ym) / ysd);
    DevBuf YS;
    if ((rc = YS.ensure(4 * n_train))) return rc;
    HIP_TRY(hipMemcpyAsync(YS.p, ys.data(), 4 * n_train, hipMemcpyHostToDevice, s));
    using namespace dk::cnn;
    if ((rc = ctx->cv_prm.ensure(4 * NPARAM))) return rc;
    if ((rc = ctx->cv_grad.ensure(4 * NPARAM))) return rc;
    if ((rc = ctx->cv_m.ensure(4 * NPARAM))) return rc;
    if ((rc = ctx->cv_v.ensure(4 * NPARAM))) return rc;
    if ((rc = ctx->cv_r.ensure(4 * (size_t)batch))) return rc;
    if ((rc = ctx->cv_loss.ensure(sizeof(double) * epochs))) return rc;
    HIP_TRY(hipMemcpyAsync(ctx->cv_prm.p, params_inout, 4 * NPARAM, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(ctx->cv_m.p, 0, 4 * NPARAM, s));
    HIP_TRY(hipMemsetAsync(ctx->cv_v.p, 0, 4 * NPARAM, s));
    HIP_TRY(hipMemsetAsync(ctx->cv_loss.p, 0, sizeof(double) * epochs, s));
    HIP_TRY(ctx->cnn.reserve(nc, batch));
    const uint64_t steps_per_epoch = n_train / (uint64_t)batch;
    int t = 0;
    for (int e = 0; e < epochs; ++e) {
        for (uint64_t k = 0; k < steps_per_epoch; ++k) {
            const float* xb = (const float*)X.p + k * batch * nn;
            const float* yb = (const float*)YS.p + k * batch;
            HIP_TRY(pack(ctx->cnn, (const float*)ctx->cv_prm.p, s));
            HIP_TRY(forward(ctx->cnn, (const float*)ctx->cv_prm.p, xb, batch, (float*)ctx->cv_r.p, s));
            HIP_TRY(backward(ctx->cnn, (const float*)ctx->cv_prm.p, xb, (const float*)ctx->cv_r.p, yb, batch,
                             (float*)ctx->cv_grad.p, s));
            HIP_TRY(accumulate_sq(ctx->cnn, batch, (double*)ctx->cv_loss.p + e, s));
            HIP_TRY(adam_update((float*)ctx->cv_prm.p, (const float*)ctx->cv_grad.p, (float*)ctx->cv_m.p,
                                (float*)ctx->cv_v.p, (float)lr, ++t, s));
        }
    }
    std::vector<double> lh(epochs);
    HIP_TRY(hipMemcpyAsync(lh.data(), ctx->cv_loss.p, sizeof(double) * epochs, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(params_inout, ctx->cv_prm.p, 4 * NPARAM, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (loss_hist)
        for (int e = 0; e < epochs; ++e) loss_hist[e] = lh[e] / (double)(steps_per_epoch * batch);
    // fold the target scaling into the last layer: r = ysd * r_std + ym
    for (int k = 0; k < 64; ++k) params_inout[OFF_U2 + k] = (float)(ysd * params_inout[OFF_U2 + k]);
    params_inout[OFF_C2] = (float)(ysd * params_inout[OFF_C2] + ym);
    if (val_out && n_val > 0) {
        HIP_TRY(hipMemcpyAsync(ctx->cv_prm.p, params_inout, 4 * NPARAM, hipMemcpyHostToDevice, s));
        DevBuf RV;
        if ((rc = RV.ensure(4 * n_val))) return rc;
        rc = cnn_forward_batched(ctx, (const float*)ctx->cv_prm.p, nc, n_val, (const float*)X.p + n_train * nn,
                                 (float*)RV.p, s);
        if (rc) return rc;
        std::vector<float> rv(n_val);
        HIP_TRY(hipMemcpyAsync(rv.data(), RV.p, 4 * n_val, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        double my = 0, md = 0, mr = 0;
        for (uint64_t i = 0; i < n_val; ++i) { my += yh[n_train + i]; md += yh[n_train + i] - rv[i]; mr += rv[i]; }
        my /= n_val; md /= n_val; mr /= n_val;
        double vy = 0, vd = 0, vr = 0;
        for (uint64_t i = 0; i < n_val; ++i) {
            const double a = yh[n_train + i] - my, b = (yh[n_train + i] - rv[i]) - md, c = rv[i] - mr;
            vy += a * a; vd += b * b; vr += c * c;
        }
        val_out[0] = vy / (n_val - 1.0);
        val_out[1] = vd / (n_val - 1.0);
        val_out[2] = vr / (n_val - 1.0);
    }
    return DK_OK;
}

int dk_abi_sizes(int32_t* out, int32_t n)
{
    const int32_t sz[] = {(int32_t)sizeof(dk_mode), (int32_t)sizeof(dk_field), (int32_t)sizeof(dk_obs),
                          (int32_t)sizeof(dk_problem), (int32_t)sizeof(dk_moments), (int32_t)sizeof(dk_mlmc_opts),
                          (int32_t)sizeof(dk_mlmc_result), (int32_t)sizeof(dk_kernel_stats)};
    const int32_t k = (int32_t)(sizeof(sz) / sizeof(sz[0]));
    for (int32_t i = 0; i < n && i < k; ++i) out[i] = sz[i];
    return k;
}

int dk_context_create(dk_context** out, int device)
{
    if (!out) return fail(DK_EINVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(DK_EINVAL, "device %d outside [0, %d)", device, count);
    HIP_TRY(hipSetDevice(device));
    dk_context* c = new (std::nothrow) dk_context();
    if (!c) return fail(DK_ENOMEM, "context allocation failed");
    c->device = device;
    if (const char* path = std::getenv("DK_TUNE_CACHE")) {
        std::ifstream f(path);
        if (f) {
            std::stringstream ss;
            ss << f.rdbuf();
            if (load_tuning_json(c, ss.str()) != DK_OK && std::getenv("DK_LOG"))
                std::fprintf(stderr, "[dk] DK_TUNE_CACHE %s ignored: %s\n", path, dk_last_error());
        }
    }
    *out = c;
    return DK_OK;
}

int dk_context_tuning_json(dk_context* ctx, char* buf, uint64_t cap)
{
    if (!ctx) return fail(DK_EINVAL, "context is NULL");
    if (cap > 0 && !buf) return fail(DK_EINVAL, "buf is NULL");
    const std::string t = tuning_json(ctx);
    if (cap > 0) {
        const size_t n = std::min<size_t>(t.size(), (size_t)cap - 1);
        std::memcpy(buf, t.data(), n);
        buf[n] = 0;
    }
    return (int)t.size();
}

int dk_context_load_tuning_json(dk_context* ctx, const char* json)
{
    if (!ctx || !json) return fail(DK_EINVAL, "NULL argument");
    return load_tuning_json(ctx, std::string(json));
}

void dk_context_destroy(dk_context* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (int l = 0; l < DK_MAX_LEVELS; ++l) {
        if (ctx->lvl_stream[l]) (void)hipStreamDestroy(ctx->lvl_stream[l]);
        if (ctx->join_ev[l]) (void)hipEventDestroy(ctx->join_ev[l]);
    }
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->rnd_t0) (void)hipEventDestroy(ctx->rnd_t0);
    if (ctx->rnd_t1) (void)hipEventDestroy(ctx->rnd_t1);
    if (ctx->pr_exec) (void)hipGraphExecDestroy(ctx->pr_exec);
    if (ctx->pr_graph) (void)hipGraphDestroy(ctx->pr_graph);
    if (ctx->pr_t0) (void)hipEventDestroy(ctx->pr_t0);
    if (ctx->pr_t1) (void)hipEventDestroy(ctx->pr_t1);
    if (ctx->pr_host) (void)hipHostFree(ctx->pr_host);
    delete ctx;
}

int dk_context_stats(dk_context* ctx, dk_kernel_stats* out, int32_t max)
{
    if (!ctx) return fail(DK_EINVAL, "context is NULL");
    int k = 0;
    for (const auto& kv : ctx->stats) {
        if (out && k < max) {
            dk_kernel_stats& r = out[k];
            r.level = kv.first.first;
            r.coupled = kv.first.second;
            r.launches = kv.second.launches;
            r.samples = kv.second.samples;
            r.kernel_ms = kv.second.ms;
            r.cell_updates = kv.second.cells;
            r.rows = kv.second.rows;
            r.reserved = 0;
        }
        ++k;
    }
    return k;
}

int dk_context_reset(dk_context* ctx, int32_t drop_tables)
{
    if (!ctx) return fail(DK_EINVAL, "context is NULL");
    ctx->stats.clear();
    if (drop_tables) {
        ctx->problems.clear();
        ctx->tuned.clear();
        ctx->tuned_depth.clear();
    }
    return DK_OK;
}

int dk_context_set_shape(dk_context* ctx, int32_t n, int32_t variant)
{
    if (!ctx) return fail(DK_EINVAL, "context is NULL");
    if (variant >= 0 && dk::shape_rows(n, variant) == 0) return fail(DK_EINVAL, "no tile-shape variant %d for n = %d", variant, n);
    if (variant < 0) ctx->forced_shape.erase(n);
    else ctx->forced_shape[n] = variant;
    return DK_OK;
}

int dk_shape_rows(int32_t n, int32_t variant) { return dk::shape_rows(n, variant); }

int dk_shape_spw(int32_t n, int32_t variant) { return dk::shape_spw(n, variant); }

int dk_heat_steps(dk_context* ctx, int32_t n, int32_t batch, int32_t steps, double mu, float* rho, float* work,
                  double* kernel_ms, void* stream)
{
    if (!ctx || !rho || !work) return fail(DK_EINVAL, "NULL argument");
    if (n < 4 || n % 4 || batch < 1 || steps < 0) return fail(DK_EINVAL, "n must be a multiple of 4, batch >= 1");
    if (!(mu > 0) || mu > 0.5) return fail(DK_EINVAL, "mu outside (0, 1/2]");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, s));
    float* a = rho;
    float* b = work;
    for (int m = 0; m < steps; ++m) {
        HIP_TRY(dk::launch_heat_f32(a, b, n, batch, (float)(0.5 * mu), s));
        std::swap(a, b);
    }
    HIP_TRY(hipEventRecord(e1, s));
    if (a != rho) HIP_TRY(hipMemcpyAsync(rho, a, sizeof(float) * (size_t)n * n * batch, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    if (kernel_ms) *kernel_ms = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return DK_OK;
}

int dk_context_set_launch_cap(dk_context* ctx, double cells)
{
    if (!ctx) return fail(DK_EINVAL, "context is NULL");
    if (!(cells >= 0)) return fail(DK_EINVAL, "cells must be >= 0");
    ctx->max_launch_cells = cells == 0 ? kMaxCellsPerLaunch : std::max(cells, 1e6);
    return DK_OK;
}

int dk_context_set_streaming(dk_context* ctx, int32_t on)
{
    if (!ctx) return fail(DK_EINVAL, "context is NULL");
    ctx->force_stream = on != 0;
    return DK_OK;
}

int dk_context_set_stream_depth(dk_context* ctx, int32_t depth)
{
    if (!ctx) return fail(DK_EINVAL, "context is NULL");
    if (depth != 0 && !dk::stream_depth_supported(depth))
        return fail(DK_EINVAL, "streaming depth %d: use 1, 2, 4, 8 or 0 (automatic)", depth);
    ctx->stream_depth = depth;
    return DK_OK;
}

int dk_moments_mean_var(const dk_moments* m, int32_t q, double* mean, double* var)
{
    if (!m || !mean || !var) return fail(DK_EINVAL, "NULL argument");
    if (q < 0 || q > 2) return fail(DK_EINVAL, "quantity %d outside 0..2 (Y, P_fine, P_coarse)", q);
    if (m->count == 0) return fail(DK_EINVAL, "no samples");
    const int k1 = q == 0 ? DK_MOM_Y : (q == 1 ? DK_MOM_PF : DK_MOM_PC);
    const double n = (double)m->count;
    const double mu = mom_value(*m, k1) / n;
    *mean = mu;
    *var = m->count > 1 ? std::max(0.0, (mom_value(*m, k1 + 1) - n * mu * mu) / (n - 1.0)) : 0.0;
    return DK_OK;
}

int dk_mlmc_level_pair(dk_context* ctx, const dk_problem* problem, int32_t level, uint64_t first_sample,
                       uint64_t n_samples, uint32_t stream_tag, dk_moments* sums_out, double* per_sample_out, void* stream)
{
    if (!ctx) return fail(DK_EINVAL, "context is NULL");
    if (!sums_out) return fail(DK_EINVAL, "sums_out is NULL");
    if (stream_tag > 255) return fail(DK_EINVAL, "stream_tag must fit in 8 bits");
    HIP_TRY(hipSetDevice(ctx->device));
    return run_level(ctx, problem, level, level >= 1, first_sample, n_samples, stream_tag, sums_out, per_sample_out,
                     nullptr, nullptr, (hipStream_t)stream, nullptr);
}

int dk_mc_level(dk_context* ctx, const dk_problem* problem, int32_t level, uint64_t first_sample, uint64_t n_samples,
                dk_moments* sums_out, double* per_sample_out, void* stream)
{
    if (!ctx) return fail(DK_EINVAL, "context is NULL");
    if (!sums_out) return fail(DK_EINVAL, "sums_out is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    return run_level(ctx, problem, level, false, first_sample, n_samples, DK_TAG_MC, sums_out, per_sample_out, nullptr,
                     nullptr, (hipStream_t)stream, nullptr);
}

int dk_level_fields(dk_context* ctx, const dk_problem* problem, int32_t level, int32_t coupled, uint64_t first_sample,
                    uint64_t n_samples, uint32_t stream_tag, double* per_sample_out, void* rho_f_out, void* rho_c_out,
                    void* stream)
{
    if (!ctx) return fail(DK_EINVAL, "context is NULL");
    if (!rho_f_out) return fail(DK_EINVAL, "rho_f_out is NULL");
    if (coupled && !rho_c_out) return fail(DK_EINVAL, "rho_c_out is NULL");
    if (stream_tag > 255) return fail(DK_EINVAL, "stream_tag must fit in 8 bits");
    HIP_TRY(hipSetDevice(ctx->device));
    if (!problem) return fail(DK_EINVAL, "problem is NULL");
    std::vector<dk_moments> tmp(std::max(1, problem->n_obs));
    return run_level(ctx, problem, level, coupled != 0, first_sample, n_samples, stream_tag, tmp.data(), per_sample_out,
                     rho_f_out, rho_c_out, (hipStream_t)stream, nullptr);
}

int dk_meanfield(dk_context* ctx, const dk_problem* problem, int32_t level, double* centre_out, double* rho_out,
                 void* stream)
{
    if (!ctx) return fail(DK_EINVAL, "context is NULL");
    if (!centre_out) return fail(DK_EINVAL, "centre_out is NULL");
    int rc = validate(problem);
    if (rc) return rc;
    if (level < 0 || level >= problem->levels) return fail(DK_EINVAL, "level out of range");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    // level tables (phi) without requiring centring
    LevelTables* T = nullptr;
    rc = ensure_level(ctx, problem, level, &T, s);
    if (rc) return rc;
    if (!T->have_centre || rho_out) {
        rc = compute_centre(ctx, problem, level, *T, s, rho_out);
        if (rc) return rc;
    }
    for (int j = 0; j < problem->n_obs; ++j) centre_out[j] = T->centre[j];
    return DK_OK;
}

int dk_noise_dump(dk_context* ctx, uint64_t seed, uint32_t tag, int32_t level, int32_t n, uint64_t first_sample,
                  uint32_t n_samples, int32_t first_step, int32_t n_steps, float* out, void* stream)
{
    if (!ctx) return fail(DK_EINVAL, "context is NULL");
    if (!out) return fail(DK_EINVAL, "out is NULL");
    if (n < 2 || (n & 1) || n > 4096) return fail(DK_EINVAL, "n = %d must be even in [2, 4096]", n);
    if (tag > 255 || level < 0 || level > 255) return fail(DK_EINVAL, "tag and level must fit in 8 bits");
    if (first_step < 0 || n_steps < 0) return fail(DK_EINVAL, "negative step range");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(dk::launch_noise_dump(seed, tag, level, n, first_sample, n_samples, first_step, n_steps, out,
                                  (hipStream_t)stream));
    return DK_OK;
}

int dk_gauss_transform(dk_context* ctx, const uint32_t* a, const uint32_t* b, uint64_t count, float* z0, float* z1,
                       void* stream)
{
    if (!ctx) return fail(DK_EINVAL, "context is NULL");
    if (count == 0) return DK_OK;
    if (!a || !b || !z0 || !z1) return fail(DK_EINVAL, "NULL argument");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(dk::launch_gauss(a, b, count, z0, z1, (hipStream_t)stream));
    return DK_OK;
}

int dk_alg1_host(double eps, int32_t L_max, const double* cost, const dk_mlmc_opts* opts, dk_level_sampler sampler,
                 void* user, dk_mlmc_result* out)
{
    if (!cost || !sampler || !out) return fail(DK_EINVAL, "NULL argument");
    const dk_mlmc_opts o = opts ? *opts : default_opts();
    return alg1_core(eps, L_max, cost, o, sampler, user, out);
}

int dk_mlmc_round(dk_context* ctx, const dk_problem* problem, int32_t L, const uint64_t* first, const uint64_t* count,
                  uint32_t tag, int32_t round_mode, dk_moments* sums_out, void* stream)
{
    if (!ctx) return fail(DK_EINVAL, "context is NULL");
    if (!first || !count || !sums_out) return fail(DK_EINVAL, "NULL argument");
    int rc = validate(problem);
    if (rc) return rc;
    if (L < 0 || L >= problem->levels) return fail(DK_EINVAL, "L must be in [0, levels)");
    if (round_mode < 0 || round_mode > 3) return fail(DK_EINVAL, "round_mode must be 0, 1, 2 or 3");
    if (tag > 255) return fail(DK_EINVAL, "tag must be < 256");
    for (int l = 0; l <= L; ++l)
        if (count[l] > 0 && (first[l] >> 48) + ((first[l] + count[l] - 1) >> 48) != 0)
            return fail(DK_EINVAL, "sample indices must stay below 2^48");
    HIP_TRY(hipSetDevice(ctx->device));
    const int nobs = problem->n_obs;
    GpuSampler G;
    G.ctx = ctx;
    G.p = problem;
    G.s = (hipStream_t)stream;
    G.mom.assign((size_t)problem->levels * nobs, dk_moments{});
    G.zmom.assign(problem->levels, dk_moments{});
    G.tag = tag;
    G.plain_mc = false;
    G.round_mode = round_mode;
    std::vector<double> prim(2 * (L + 1), 0.0);
    if (round_mode == 0) {
        for (int l = 0; l <= L; ++l)
            if (count[l] > 0 && (rc = gpu_sample(&G, l, first[l], count[l], &prim[2 * l])) < 0) return rc;
    } else if ((rc = gpu_round(&G, L, first, count, prim.data())) < 0) {
        return rc;
    }
    for (int l = 0; l <= L; ++l)
        for (int j = 0; j < nobs; ++j) sums_out[(size_t)l * nobs + j] = G.mom[(size_t)l * nobs + j];
    return DK_OK;
}

int dk_mlmc_estimate(dk_context* ctx, const dk_problem* problem, double eps, const dk_mlmc_opts* opts,
                     dk_mlmc_result* out, dk_moments* level_moments, void* stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!ctx) return fail(DK_EINVAL, "context is NULL");
    if (!out) return fail(DK_EINVAL, "out is NULL");
    int rc = validate(problem);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    dk_mlmc_opts o = opts ? *opts : default_opts();
    if (o.m_pilot == 0) o.m_pilot = 1000;
    if (o.alpha == 0) o.alpha = 2.0;
    if (o.max_rounds == 0) o.max_rounds = 1000;
    const long s0 = steps0_of(problem);
    const int nobs = problem->n_obs;
    GpuSampler G;
    G.ctx = ctx;
    G.p = problem;
    G.s = (hipStream_t)stream;
    G.mom.assign((size_t)problem->levels * nobs, dk_moments{});
    const bool mc = o.plain_mc_level >= 0;
    if (mc && o.plain_mc_level >= problem->levels) return fail(DK_EINVAL, "plain_mc_level out of range");
    G.plain_mc = mc;
    G.tag = mc ? DK_TAG_MC : DK_TAG_MLMC;
    G.zmom.assign(problem->levels, dk_moments{});
    if (o.cv_params && !mc) {
        if (fourier(problem) || implicit(problem)) return fail(DK_EUNSUPPORTED, "the control variate is built for the explicit NN scheme");
        G.cv_params = o.cv_params;
        G.cv_mask = o.cv_level_mask & ~1u;
        G.cv_ratio = o.cv_ratio > 0 ? o.cv_ratio : 4;
        for (int l = 1; l < problem->levels; ++l)
            if ((G.cv_mask >> l) & 1u) {
                const int nc = problem->n0 << (l - 1);
                if (nc % 4) return fail(DK_EINVAL, "control variate on level %d: coarse grid must be a multiple of 4", l);
            }
    }
    if (mc && o.checkpoint_path && *o.checkpoint_path)
        return fail(DK_EINVAL, "checkpoint_path applies to MLMC runs, not plain MC");
    if (!mc) {
        std::vector<double> cost(problem->levels);
        for (int l = 0; l < problem->levels; ++l) {
            cost[l] = level_cost(problem, s0, l, true);
            if ((G.cv_mask >> l) & 1u) cost[l] += G.cv_ratio * level_cost(problem, s0, l - 1, false);
        }
        G.round_mode = o.round_mode;
        if (o.round_mode < 0 || o.round_mode > 3) return fail(DK_EINVAL, "round_mode must be 0, 1, 2 or 3");
        // checkpoints: the key covers everything that changes the samples or their grouping; the
        // sampler's per-observable moments and cell count travel with the state
        CkptHooks ck;
        {
            Fnv f;
            f.val(problem_hash(problem));
            f.val(G.cv_mask); f.val(G.cv_ratio); f.val(o.round_mode == 3);
            if (G.cv_params) f.bytes(G.cv_params, sizeof(float) * (size_t)problem->levels * dk::cnn::NPARAM);
            ck.key = f.h;
        }
        auto put = [](std::vector<double>& v, const dk_moments& m) {
            v.push_back((double)m.count);
            for (int k = 0; k < DK_NMOM; ++k) { v.push_back(m.sum[k]); v.push_back(m.comp[k]); }
        };
        ck.save = [&](std::vector<double>& v) {
            v.clear();
            v.push_back(G.cell_updates);
            for (const dk_moments& m : G.mom) put(v, m);
            for (const dk_moments& m : G.zmom) put(v, m);
        };
        ck.load = [&](const std::vector<double>& v) -> int {
            const size_t per = 1 + 2 * DK_NMOM;
            if (v.size() != 1 + per * (G.mom.size() + G.zmom.size()))
                return fail(DK_EINVAL, "checkpoint: sampler state of another shape");
            size_t i = 0;
            G.cell_updates = v[i++];
            auto get = [&](dk_moments& m) {
                m.count = (uint64_t)v[i++];
                for (int k = 0; k < DK_NMOM; ++k) { m.sum[k] = v[i++]; m.comp[k] = v[i++]; }
            };
            for (dk_moments& m : G.mom) get(m);
            for (dk_moments& m : G.zmom) get(m);
            return DK_OK;
        };
        // measured costs: kernel seconds per sample of each level since this call began
        std::map<std::pair<int, int>, KStat> base = ctx->stats;
        cost_measure measure = [&](int L, std::vector<double>& C) {
            int ref = -1;
            double ref_per_cell = 0;
            std::vector<bool> got(L + 1, false);
            for (int l = 0; l <= L; ++l) {
                if ((G.cv_mask >> l) & 1u) continue;   // control-variate levels keep the cell model
                const auto key = std::make_pair(l, l >= 1 && !G.plain_mc ? 1 : 0);
                const KStat now = ctx->stats.count(key) ? ctx->stats[key] : KStat{};
                const KStat b = base.count(key) ? base[key] : KStat{};
                const double ms = now.ms - b.ms;
                const uint64_t n = now.samples - b.samples;
                if (n > 0 && ms > 0) {
                    C[l] = ms * 1e-3 / (double)n;
                    got[l] = true;
                    ref = l;
                    ref_per_cell = C[l] / cost[l];
                }
            }
            if (ref < 0) { for (int l = 0; l <= L; ++l) C[l] = cost[l]; return; }
            for (int l = 0; l <= L; ++l)
                if (!got[l]) C[l] = cost[l] * ref_per_cell;
        };
        rc = alg1_core(eps, problem->levels - 1, cost.data(), o, gpu_sample, &G, out,
                       o.round_mode > 0 ? gpu_round : nullptr, &ck, &measure, (double)level_ratio(problem));
        if (rc < 0) return rc;
    } else {
        // plain MC on one level: pilot, then M = ceil(2 V / eps^2) so that V / M <= eps^2 / 2
        const int l = o.plain_mc_level;
        uint64_t done = 0, target = (uint64_t)o.m_pilot;
        double s1 = 0, c1 = 0, s2 = 0, c2 = 0, mean = 0, var = 0;
        int rounds = 0;
        while (done < target) {
            ++rounds;
            double sums[2];
            rc = gpu_sample(&G, l, done, target - done, sums);
            if (rc < 0) return rc;
            nadd(s1, c1, sums[0]);
            nadd(s2, c2, sums[1]);
            done = target;
            mean = (s1 + c1) / (double)done;
            var = std::max(0.0, ((s2 + c2) - (double)done * mean * mean) / ((double)done - 1.0));
            uint64_t m = (uint64_t)std::ceil(2.0 * var / (eps * eps));
            if (o.max_samples && m > o.max_samples) m = o.max_samples;
            target = std::max(done, m);
            if (rounds > o.max_rounds) return fail(DK_EINVAL, "plain MC exceeded max_rounds");
        }
        std::memset(out, 0, sizeof(*out));
        out->L = l;
        out->M[l] = done;
        out->Yhat[l] = mean;
        out->Vhat[l] = var;
        out->cost[l] = level_cost(problem, s0, l, false);
        out->estimate[0] = mean;
        out->var_est[0] = var / (double)done;
        out->rmse_est = std::sqrt(out->var_est[0]);
        out->converged = 1;
        out->rounds = rounds;
        rc = DK_OK;
    }
    // all observables from the accumulated moments
    for (int j = 0; j < nobs; ++j) {
        double est = 0.0, var = 0.0;
        for (int l = 0; l <= out->L; ++l) {
            const bool cvl = j == problem->primary_obs && ((G.cv_mask >> l) & 1u) && G.zmom[l].count > 0;
            const dk_moments& m = cvl ? G.zmom[l] : G.mom[(size_t)l * nobs + j];
            if (m.count == 0) continue;
            const double n = (double)m.count;
            const double y = mom_value(m, DK_MOM_Y) / n;
            const double v = n > 1 ? std::max(0.0, (mom_value(m, DK_MOM_Y2) - n * y * y) / (n - 1.0)) : 0.0;
            est += y;
            var += v / n;
        }
        out->estimate[j] = est;
        out->var_est[j] = var;
    }
    if (!mc) out->rmse_est = std::sqrt(out->var_est[problem->primary_obs] + out->bias_est * out->bias_est);
    out->cell_updates = G.cell_updates;
    if (level_moments) std::memcpy(level_moments, G.mom.data(), sizeof(dk_moments) * G.mom.size());
    out->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

}  // extern "C"
