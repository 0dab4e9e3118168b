// dk_api.cpp -- the C ABI: argument checks, device selection and dispatch to the host driver
// (level batches, rounds, Algorithm 1 of Sec. 7 and plain Monte Carlo, the control variate).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <random>
#include <sstream>
#include <string>
#include <vector>

#include "dk_host.h"

using namespace dkh;

// ============================================================================================
// C ABI
// ============================================================================================
extern "C" {

const char* dk_last_error(void) { return dkh::last_error(); }

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
