// dk_arena.cpp -- the allocation-free batch of one resident level.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "dk_host.h"

using namespace dkh;

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
