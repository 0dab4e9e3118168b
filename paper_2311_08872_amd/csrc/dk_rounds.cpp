// dk_rounds.cpp -- whole Algorithm-1 rounds: one stream per level (optionally captured as a
// hipGraph), or all resident levels in one persistent launch.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "dk_host.h"

namespace dkh {

namespace {

struct RoundJob {
    int level = 0;
    bool pair = false;
    uint64_t first = 0, count = 0, ch = 0, nchunks = 0;
    dk::LevelArgs A{};
    dk::LevelKind K{};
    double cells_per_sample = 0;
};

}  // namespace

// ------------------------------------------------------------------------------------------
// One Algorithm-1 round of resident levels at once: every level's batches go to its own
// stream (forked from and joined to the caller's stream), so levels of very different size
// fill the GPU together; mode 2 captures the whole round into a hipGraph and launches it once.
// The per-sample values and the chunking are those of run_level, so results are identical.
// ------------------------------------------------------------------------------------------
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

}  // namespace dkh
