// Host-driver harness: the host sources (dk_*.cpp) built with g++ against the CPU stand-ins of fake_device.cpp,
// run under AddressSanitizer and UndefinedBehaviorSanitizer.  Test infrastructure only.
//
// Scenarios (each names itself on stdout before it starts):
//   rounds     Algorithm 1 on a five-level hierarchy of 8^2 .. 128^2 grids with every round mode
//              (0 level by level, 1 one stream per level, 2 a hipGraph per round, 3 the persistent
//              round kernel replayed from one captured graph), each from a fresh context, with
//              jobs large enough that the tile-shape tuner runs; then again with a small launch
//              cap (many chunks per level, many graph replays per round).  Modes 0-2 must agree
//              bit for bit, mode 3 to rounding, and every level mean must equal the mean of the
//              stand-in per-sample values recomputed here.
//   sequence   the same context reused for several estimates and rounds in all modes, with the
//              launch cap changed between them (buffers grow and shrink under a captured graph).
//   stream     levels on the streaming path (forced at 64^2 and 128^2, native at 256^2), each
//              temporal depth forced, then the automatic depth tuning, with several batches.
//   arena      the allocation-free level batch (dk::level_pair_arena) on a 32 MiB arena against
//              dk_mlmc_level_pair on a context: identical per-sample values, equal moment sums, on
//              two calls in a row (the second smaller), with and without a per-sample output; an
//              arena too small and a streamed grid are refused.
//   errors     argument errors return negative codes.
// At the end every stand-in device allocation, stream and event must have been released.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../../include/dk_mlmc.h"

namespace dk {
int level_pair_arena(const dk_problem* p, int level, uint64_t first, uint64_t count, uint32_t tag, dk_moments* sums_out,
                     double* per_sample_out, void* arena, size_t arena_bytes, hipStream_t s);
}

extern std::vector<std::string> g_fake_errors;
extern uint64_t g_fake_launches;
extern uint64_t g_fake_graph_launches;
extern "C" double fake_value(uint64_t seed, uint32_t tag, int level, uint64_t sample, int j, int pair, int which);
extern "C" int fake_live_device_allocations(void);
extern "C" int fake_live_streams(void);
extern "C" int fake_live_events(void);

static int g_failures = 0;

#define CHECK(cond, ...)                                                                 \
    do {                                                                                 \
        if (!(cond)) {                                                                   \
            std::printf("  FAIL %s:%d: ", __FILE__, __LINE__);                           \
            std::printf(__VA_ARGS__);                                                    \
            std::printf("\n");                                                           \
            ++g_failures;                                                                \
        }                                                                                \
    } while (0)

static bool stand_in_clean(const char* where)
{
    if (g_fake_errors.empty()) return true;
    for (const auto& e : g_fake_errors) std::printf("  FAIL %s: stand-in: %s\n", where, e.c_str());
    g_failures += (int)g_fake_errors.size();
    g_fake_errors.clear();
    return false;
}

struct Problem {
    dk_mode rho_modes[2];
    dk_mode phi_modes[2][2];
    dk_obs obs[2];
    dk_problem p;
};

// The five-level hierarchy of the config-2 workload: unit torus, 8^2 .. 128^2, tau = 0.1 h^2,
// T = 0.05, two observables (the first centred and sqrt(N)-scaled, squared).
static void make_hierarchy(Problem& P, int n0, int levels, double T)
{
    std::memset(&P, 0, sizeof(P));
    P.rho_modes[0] = {0.25, 1, 1, 0};
    P.rho_modes[1] = {0.25, 1, -1, 0};
    P.phi_modes[0][0] = {1.0, 1, 0, -1.5707963267948966};
    P.phi_modes[0][1] = {1.0, 0, 1, -1.5707963267948966};
    P.phi_modes[1][0] = {0.5, 1, 1, 0};
    P.phi_modes[1][1] = {0.5, 1, -1, 0};
    for (int j = 0; j < 2; ++j) {
        P.obs[j].phi.kind = DK_FIELD_MODES;
        P.obs[j].phi.n_modes = 2;
        P.obs[j].phi.modes = P.phi_modes[j];
    }
    P.obs[0].centre = 1;
    P.obs[0].scale_sqrtN = 1;
    P.obs[0].psi = DK_PSI_SQUARE;
    P.obs[1].psi = DK_PSI_ID;
    dk_problem& p = P.p;
    p.d = 2;
    p.n0 = n0;
    p.levels = levels;
    p.steps_policy = DK_STEPS_EXACT;
    p.box = 1.0;
    p.mu = 0.1;
    p.T = T;
    p.N = 1e4;
    p.flux = DK_FLUX_CENTRAL;
    p.precision = DK_PREC_F32;
    p.n_obs = 2;
    p.primary_obs = 0;
    p.obs = P.obs;
    p.rho0.kind = DK_FIELD_MODES;
    p.rho0.c0 = 1.0;
    p.rho0.n_modes = 2;
    p.rho0.modes = P.rho_modes;
    p.seed = 7;
    p.coupling = DK_COUPLING_NN;
    p.grid = DK_GRID_VERTEX;
}

// mean of Y over samples [0, M) of level l from the stand-in values
static double expected_mean(const dk_problem& p, uint32_t tag, int l, uint64_t M, int j)
{
    long double s = 0;
    for (uint64_t i = 0; i < M; ++i)
        s += (long double)fake_value(p.seed, tag, l, i, j, l >= 1, 0) - (long double)fake_value(p.seed, tag, l, i, j, l >= 1, 1);
    return (double)(s / (long double)M);
}

static dk_mlmc_opts opts_mode(int mode)
{
    dk_mlmc_opts o;
    std::memset(&o, 0, sizeof(o));
    o.m_pilot = 1000;
    o.L_start = 2;
    o.alpha = 2.0;
    o.max_rounds = 1000;
    o.plain_mc_level = -1;
    o.cv_ratio = 4;
    o.round_mode = mode;
    return o;
}

static bool close_rel(double a, double b, double rel) { return std::fabs(a - b) <= rel * std::max(std::fabs(a), std::fabs(b)) + 1e-300; }

static void check_against_values(const dk_problem& p, const dk_mlmc_result& r, const char* what)
{
    for (int l = 0; l <= r.L; ++l) {
        const double e = expected_mean(p, DK_TAG_MLMC, l, r.M[l], p.primary_obs);
        CHECK(close_rel(r.Yhat[l], e, 1e-12), "%s: level %d mean %.17g, stand-in values give %.17g (M = %llu)", what, l,
              r.Yhat[l], e, (unsigned long long)r.M[l]);
    }
}

static void scenario_rounds(double cap, const char* label)
{
    std::printf("[host] rounds %s\n", label);
    std::fflush(stdout);
    Problem P;
    make_hierarchy(P, 8, 5, 0.05);
    dk_mlmc_result res[4];
    for (int mode = 0; mode < 4; ++mode) {
        dk_context* ctx = nullptr;
        CHECK(dk_context_create(&ctx, 0) == DK_OK, "context: %s", dk_last_error());
        if (cap > 0) CHECK(dk_context_set_launch_cap(ctx, cap) == DK_OK, "cap: %s", dk_last_error());
        dk_mlmc_opts o = opts_mode(mode);
        std::vector<dk_moments> lm(P.p.levels * P.p.n_obs);
        const int rc = dk_mlmc_estimate(ctx, &P.p, 1e-3, &o, &res[mode], lm.data(), nullptr);
        CHECK(rc >= 0, "mode %d: dk_mlmc_estimate returned %d: %s", mode, rc, dk_last_error());
        char js[4096];
        const int nj = dk_context_tuning_json(ctx, js, sizeof(js));
        std::printf("  mode %d: rc %d, L %d, rounds %d, M = [", mode, rc, res[mode].L, res[mode].rounds);
        for (int l = 0; l <= res[mode].L; ++l) std::printf("%s%llu", l ? ", " : "", (unsigned long long)res[mode].M[l]);
        std::printf("], estimate %.15g, tuning %s\n", res[mode].estimate[0], nj > 0 ? js : "(none)");
        check_against_values(P.p, res[mode], label);
        // the level moments handed back agree with the result's means
        for (int l = 0; l <= res[mode].L; ++l) {
            const dk_moments& m = lm[l * P.p.n_obs + P.p.primary_obs];
            CHECK(m.count == res[mode].M[l], "mode %d level %d: moment count %llu, M %llu", mode, l,
                  (unsigned long long)m.count, (unsigned long long)res[mode].M[l]);
        }
        dk_context_destroy(ctx);
        stand_in_clean(label);
    }
    for (int mode = 1; mode < 3; ++mode) {
        CHECK(res[mode].L == res[0].L, "mode %d: L %d vs %d", mode, res[mode].L, res[0].L);
        CHECK(std::memcmp(res[mode].M, res[0].M, sizeof(res[0].M)) == 0, "mode %d: sample counts differ", mode);
        CHECK(std::memcmp(res[mode].Yhat, res[0].Yhat, sizeof(res[0].Yhat)) == 0, "mode %d: level means differ", mode);
        CHECK(std::memcmp(res[mode].estimate, res[0].estimate, sizeof(res[0].estimate)) == 0, "mode %d: estimates differ", mode);
    }
    CHECK(res[3].L == res[0].L, "mode 3: L %d vs %d", res[3].L, res[0].L);
    for (int l = 0; l <= res[0].L; ++l) CHECK(close_rel(res[3].Yhat[l], res[0].Yhat[l], 1e-12), "mode 3 level %d mean", l);
}

static void scenario_sequence()
{
    std::printf("[host] sequence\n");
    std::fflush(stdout);
    Problem P;
    make_hierarchy(P, 8, 5, 0.05);
    dk_context* ctx = nullptr;
    CHECK(dk_context_create(&ctx, 0) == DK_OK, "context: %s", dk_last_error());
    const double caps[] = {0, 1e8, 3e9, 0, 5e7};
    const int modes[] = {3, 1, 2, 3, 0, 2, 3, 1};
    for (int k = 0; k < 8; ++k) {
        CHECK(dk_context_set_launch_cap(ctx, caps[k % 5]) == DK_OK, "cap: %s", dk_last_error());
        P.p.seed = 100 + k;
        dk_mlmc_opts o = opts_mode(modes[k]);
        dk_mlmc_result r;
        const int rc = dk_mlmc_estimate(ctx, &P.p, k % 2 ? 3e-3 : 2e-3, &o, &r, nullptr, nullptr);
        CHECK(rc >= 0, "estimate %d (mode %d): %d %s", k, modes[k], rc, dk_last_error());
        if (rc >= 0) check_against_values(P.p, r, "sequence");
        // a round of ragged counts, with an empty level, in the same context
        const uint64_t first[5] = {13, 5, 0, 2, 1};
        const uint64_t count[5] = {1003, 517, 0, 37, 5 + (uint64_t)k};
        std::vector<dk_moments> sums(5 * P.p.n_obs);
        const int rr = dk_mlmc_round(ctx, &P.p, 4, first, count, DK_TAG_MC, modes[7 - k], sums.data(), nullptr);
        CHECK(rr >= 0, "round %d (mode %d): %d %s", k, modes[7 - k], rr, dk_last_error());
        for (int l = 0; l < 5 && rr >= 0; ++l) {
            const dk_moments& m = sums[l * P.p.n_obs + 1];
            CHECK(m.count == count[l], "round %d level %d: count %llu", k, l, (unsigned long long)m.count);
            if (!count[l]) continue;
            long double s = 0;
            for (uint64_t i = first[l]; i < first[l] + count[l]; ++i)
                s += (long double)fake_value(P.p.seed, DK_TAG_MC, l, i, 1, l >= 1, 0) -
                     (long double)fake_value(P.p.seed, DK_TAG_MC, l, i, 1, l >= 1, 1);
            CHECK(close_rel(m.sum[DK_MOM_Y] + m.comp[DK_MOM_Y], (double)s, 1e-12), "round %d level %d: sum of Y", k, l);
        }
        stand_in_clean("sequence");
    }
    dk_kernel_stats st[64];
    const int ns = dk_context_stats(ctx, st, 64);
    CHECK(ns > 0, "no kernel statistics");
    dk_context_destroy(ctx);
    stand_in_clean("sequence");
}

static void scenario_stream()
{
    std::printf("[host] stream\n");
    std::fflush(stdout);
    // 64^2, 128^2, 256^2 with 32, 128, 512 fine steps (T = 32 tau_0)
    Problem P;
    make_hierarchy(P, 64, 3, 32 * 0.1 / (64.0 * 64.0));
    struct Case { int level, depth; uint64_t first, count; bool force; };
    const Case cases[] = {
        {1, 1, 0, 37, true}, {1, 2, 5, 300, true}, {1, 4, 0, 41, true}, {1, 8, 3, 129, true},
        {2, 4, 0, 9, false}, {2, 1, 11, 7, false}, {2, 8, 0, 5, false}, {0, 2, 0, 4100, true},
    };
    for (const Case& c : cases) {
        std::printf("  level %d depth %d samples [%llu, +%llu)%s\n", c.level, c.depth, (unsigned long long)c.first,
                    (unsigned long long)c.count, c.force ? " (streaming forced)" : "");
        std::fflush(stdout);
        dk_context* ctx = nullptr;
        CHECK(dk_context_create(&ctx, 0) == DK_OK, "context: %s", dk_last_error());
        CHECK(dk_context_set_streaming(ctx, c.force ? 1 : 0) == DK_OK, "streaming: %s", dk_last_error());
        CHECK(dk_context_set_stream_depth(ctx, c.depth) == DK_OK, "depth: %s", dk_last_error());
        std::vector<dk_moments> sums(P.p.n_obs);
        const int rc = dk_mlmc_level_pair(ctx, &P.p, c.level, c.first, c.count, DK_TAG_MLMC, sums.data(), nullptr, nullptr);
        CHECK(rc == DK_OK, "level pair: %d %s", rc, dk_last_error());
        for (int j = 0; j < P.p.n_obs && rc == DK_OK; ++j) {
            long double s = 0;
            for (uint64_t i = c.first; i < c.first + c.count; ++i)
                s += (long double)fake_value(P.p.seed, DK_TAG_MLMC, c.level, i, j, c.level >= 1, 0) -
                     (long double)fake_value(P.p.seed, DK_TAG_MLMC, c.level, i, j, c.level >= 1, 1);
            CHECK(sums[j].count == c.count, "count");
            CHECK(close_rel(sums[j].sum[DK_MOM_Y] + sums[j].comp[DK_MOM_Y], (double)s, 1e-12), "level %d obs %d: sum of Y %.17g vs %.17g",
                  c.level, j, sums[j].sum[DK_MOM_Y] + sums[j].comp[DK_MOM_Y], (double)s);
        }
        dk_context_destroy(ctx);
        stand_in_clean("stream");
    }
    // automatic depth: a job above the tuning threshold (1e11 cell updates) on the 64^2 grid with
    // 4096 fine steps, two batches of the streaming buffers
    std::printf("  automatic depth, 64^2 pairs, 4096 steps\n");
    std::fflush(stdout);
    Problem Q;
    make_hierarchy(Q, 32, 2, 1024 * 0.1 / (32.0 * 32.0));
    dk_context* ctx = nullptr;
    CHECK(dk_context_create(&ctx, 0) == DK_OK, "context: %s", dk_last_error());
    CHECK(dk_context_set_streaming(ctx, 1) == DK_OK, "streaming: %s", dk_last_error());
    std::vector<dk_moments> sums(Q.p.n_obs);
    const uint64_t n = 6000;
    int rc = dk_mlmc_level_pair(ctx, &Q.p, 1, 0, n, DK_TAG_MLMC, sums.data(), nullptr, nullptr);
    CHECK(rc == DK_OK, "level pair: %d %s", rc, dk_last_error());
    long double s = 0;
    for (uint64_t i = 0; i < n; ++i)
        s += (long double)fake_value(Q.p.seed, DK_TAG_MLMC, 1, i, 0, 1, 0) - (long double)fake_value(Q.p.seed, DK_TAG_MLMC, 1, i, 0, 1, 1);
    CHECK(close_rel(sums[0].sum[DK_MOM_Y] + sums[0].comp[DK_MOM_Y], (double)s, 1e-12), "automatic depth: sum of Y");
    char js[4096];
    dk_context_tuning_json(ctx, js, sizeof(js));
    std::printf("  tuning %s\n", js);
    CHECK(std::strstr(js, "\"depth\"") != nullptr, "the automatic depth was not tuned");
    // again with the tuned depth, and a second context loading the choice from JSON
    rc = dk_mlmc_level_pair(ctx, &Q.p, 1, n, 100, DK_TAG_MLMC, sums.data(), nullptr, nullptr);
    CHECK(rc == DK_OK, "level pair after tuning: %d %s", rc, dk_last_error());
    dk_context* c2 = nullptr;
    CHECK(dk_context_create(&c2, 0) == DK_OK, "context: %s", dk_last_error());
    CHECK(dk_context_load_tuning_json(c2, js) == DK_OK, "load tuning: %s", dk_last_error());
    dk_context_destroy(c2);
    dk_context_destroy(ctx);
    stand_in_clean("stream");
}

static void scenario_arena()
{
    std::printf("[host] arena\n");
    std::fflush(stdout);
    Problem P;
    make_hierarchy(P, 8, 5, 0.05);
    const size_t arena_bytes = size_t(32) << 20;
    void* arena = nullptr;
    CHECK(hipMalloc(&arena, arena_bytes) == hipSuccess, "arena");
    dk_context* ctx = nullptr;
    CHECK(dk_context_create(&ctx, 0) == DK_OK, "context: %s", dk_last_error());
    struct Call { int level; uint64_t first, count; };
    const Call calls[] = {{4, 3, 700}, {4, 0, 41}, {0, 5, 300000}, {0, 1, 17}, {2, 0, 2000}, {1, 9, 0}};
    for (int with_ps = 0; with_ps < 2; ++with_ps)
        for (const Call& c : calls) {
            const int nobs = P.p.n_obs;
            std::vector<dk_moments> a(nobs), b(nobs);
            double *psa = nullptr, *psb = nullptr;
            const size_t psbytes = sizeof(double) * 2 * nobs * (c.count ? c.count : 1);
            if (with_ps) {
                CHECK(hipMalloc((void**)&psa, psbytes) == hipSuccess, "ps");
                CHECK(hipMalloc((void**)&psb, psbytes) == hipSuccess, "ps");
            }
            const int ra = dk::level_pair_arena(&P.p, c.level, c.first, c.count, DK_TAG_MLMC, a.data(), psa, arena, arena_bytes, nullptr);
            const int rb = dk_mlmc_level_pair(ctx, &P.p, c.level, c.first, c.count, DK_TAG_MLMC, b.data(), psb, nullptr);
            CHECK(ra == DK_OK && rb == DK_OK, "level %d: %d / %d: %s", c.level, ra, rb, dk_last_error());
            for (int j = 0; j < nobs; ++j) {
                CHECK(a[j].count == b[j].count, "level %d obs %d: count", c.level, j);
                for (int k = 0; k < DK_NMOM; ++k)
                    CHECK(close_rel(a[j].sum[k] + a[j].comp[k], b[j].sum[k] + b[j].comp[k], 1e-13),
                          "level %d obs %d moment %d: %.17g vs %.17g", c.level, j, k, a[j].sum[k] + a[j].comp[k],
                          b[j].sum[k] + b[j].comp[k]);
            }
            if (with_ps) {
                CHECK(std::memcmp(psa, psb, sizeof(double) * 2 * nobs * c.count) == 0, "level %d: per-sample values differ", c.level);
                (void)hipFree(psa);
                (void)hipFree(psb);
            }
            stand_in_clean("arena");
        }
    std::vector<dk_moments> m(P.p.n_obs);
    CHECK(dk::level_pair_arena(&P.p, 4, 0, 10, 0, m.data(), nullptr, arena, size_t(256) << 10, nullptr) == DK_EINVAL,
          "a 256 KiB arena was accepted for the 128^2 pair");
    Problem Q;
    make_hierarchy(Q, 64, 3, 32 * 0.1 / (64.0 * 64.0));
    CHECK(dk::level_pair_arena(&Q.p, 2, 0, 10, 0, m.data(), nullptr, arena, arena_bytes, nullptr) == DK_EUNSUPPORTED,
          "the streamed 256^2 level was accepted");
    dk_context_destroy(ctx);
    (void)hipFree(arena);
    stand_in_clean("arena");
}

static void scenario_errors()
{
    std::printf("[host] errors\n");
    std::fflush(stdout);
    Problem P;
    make_hierarchy(P, 8, 5, 0.05);
    dk_context* ctx = nullptr;
    CHECK(dk_context_create(&ctx, 0) == DK_OK, "context: %s", dk_last_error());
    dk_moments m[2];
    CHECK(dk_mlmc_level_pair(ctx, nullptr, 1, 0, 10, 0, m, nullptr, nullptr) < 0, "NULL problem accepted");
    CHECK(dk_mlmc_level_pair(ctx, &P.p, 5, 0, 10, 0, m, nullptr, nullptr) < 0, "level 5 of 5 accepted");
    CHECK(dk_mlmc_level_pair(ctx, &P.p, 1, ~0ull - 3, 10, 0, m, nullptr, nullptr) < 0, "overflowing range accepted");
    const uint64_t first[5] = {0, 0, 0, 0, 0}, count[5] = {1, 1, 1, 1, 1};
    std::vector<dk_moments> sums(5 * 2);
    CHECK(dk_mlmc_round(ctx, &P.p, 4, first, count, 0, 7, sums.data(), nullptr) < 0, "round mode 7 accepted");
    CHECK(dk_mlmc_round(ctx, &P.p, 5, first, count, 0, 0, sums.data(), nullptr) < 0, "L = 5 accepted");
    dk_mlmc_result r;
    dk_mlmc_opts o = opts_mode(0);
    CHECK(dk_mlmc_estimate(ctx, &P.p, -1.0, &o, &r, nullptr, nullptr) < 0, "eps < 0 accepted");
    o.m_pilot = 1;
    CHECK(dk_mlmc_estimate(ctx, &P.p, 1e-2, &o, &r, nullptr, nullptr) < 0, "m_pilot = 1 accepted");
    P.p.mu = 0.6;
    CHECK(dk_mlmc_level_pair(ctx, &P.p, 1, 0, 10, 0, m, nullptr, nullptr) < 0, "unstable mu accepted");
    dk_context_destroy(ctx);
    stand_in_clean("errors");
}

int main(int argc, char** argv)
{
    const std::string only = argc > 1 ? argv[1] : "";
    const int base_alloc = fake_live_device_allocations();
    if (only.empty() || only == "rounds") {
        scenario_rounds(0, "default launch cap");
        scenario_rounds(2e9, "launch cap 2e9");
    }
    if (only.empty() || only == "sequence") scenario_sequence();
    if (only.empty() || only == "stream") scenario_stream();
    if (only.empty() || only == "arena") scenario_arena();
    if (only.empty() || only == "errors") scenario_errors();
    CHECK(fake_live_device_allocations() == base_alloc, "%d device allocations left after every context was destroyed",
          fake_live_device_allocations() - base_alloc);
    CHECK(fake_live_streams() == 0, "%d streams left", fake_live_streams());
    CHECK(fake_live_events() == 0, "%d events left", fake_live_events());
    std::printf("[host] %llu stand-in launches, %llu graph launches, %d failure(s)\n", (unsigned long long)g_fake_launches,
                (unsigned long long)g_fake_graph_launches, g_failures);
    return g_failures ? 1 : 0;
}
