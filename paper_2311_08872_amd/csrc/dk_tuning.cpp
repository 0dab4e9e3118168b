// dk_tuning.cpp -- tile-shape choice for the resident kernels (forced, cached, or timed on a
// short batch) and the JSON text of the choices.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <regex>
#include <sstream>

#include "dk_host.h"

namespace dkh {

namespace {

std::string device_arch(int device)
{
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, device) != hipSuccess) return "unknown";
    std::string a = pr.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Tile-shape choices as JSON text:
//   {"format": "dk-tile-shapes-1", "arch": "gfx950",
//    "shapes": [{"n": 128, "pair": 1, "flux": 0, "rows": 8, "spw": 1}, ...]}
// ("spw", samples per block, may be left out: then the shape with that R and ~256-lane blocks)
// ------------------------------------------------------------------------------------------
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

}  // namespace dkh
