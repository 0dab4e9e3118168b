// dk_levels.cpp -- level tables and centring constants, and the batches of one level: resident
// kernels, the streaming kernel for large grids, the Fourier coupling and the semi-implicit scheme.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "dk_host.h"

namespace dkh {

namespace {

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

}  // namespace

double noise_coeff(const dk_problem* p, double h, double sigma)
{
    // N^{-1/2} h^{-d/2} sigma / (2h) (central) or N^{-1/2} h^{-d/2} sigma / h (staggered), d = 2
    const double base = sigma / (std::sqrt(p->N) * h * h);
    return p->flux == DK_FLUX_CENTRAL ? 0.5 * base : base;
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

}  // namespace dkh
