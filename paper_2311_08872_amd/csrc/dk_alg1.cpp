// dk_alg1.cpp -- Algorithm 1 of Sec. 7 (adaptive MLMC: pilot samples, optimal sample
// counts, the bias test on the finest levels) and its checkpoints.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>

#include "dk_host.h"

namespace dkh {

namespace {

double bias_remainder(const std::vector<double>& Y, int L, double alpha, double ratio)
{
    // eq. (convergence_criterion) with the refinement ratio h_{l-1}/h_l (2 in the paper)
    double r = 0.0;
    for (int j = 0; j <= std::min(2, L); ++j) r = std::max(r, std::pow(ratio, -j * alpha) * std::fabs(Y[L - j]));
    return r / (std::pow(ratio, alpha) - 1.0);
}

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

}  // namespace

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

// ------------------------------------------------------------------------------------------
// Algorithm-1 checkpoints: after every completed round the state (level, round count, samples
// done and targeted, compensated sums, and whatever the sampler adds) is written as text, doubles
// as their bit patterns, to path.tmp and renamed over path.  A run that finds the file resumes
// from it; since the sample ranges of every round follow from that state and the noise is a pure
// function of the sample index, the resumed run reproduces the uninterrupted one bit for bit.
// ------------------------------------------------------------------------------------------

int alg1_core(double eps, int L_max, const double* cost, const dk_mlmc_opts& o, dk_level_sampler sampler, void* user,
              dk_mlmc_result* out, round_sampler rsampler, const CkptHooks* ck, const cost_measure* measure,
              double ratio)
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

}  // namespace dkh
