// dk_samplers.cpp -- the GPU samplers that Algorithm 1 drives (level by level, or a whole
// round at once) and the learned control variate.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "dk_host.h"

namespace dkh {

namespace {

constexpr int kCnnBatch = 1024;   // inputs per network launch sequence

}  // namespace

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

}  // namespace dkh
