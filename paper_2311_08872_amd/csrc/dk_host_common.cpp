// dk_host_common.cpp -- errors, compensated sums, problem hashing and validation, and the
// field tables of a level grid.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "dk_host.h"

namespace dkh {

namespace {

thread_local char g_err[512] = "";

}  // namespace

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

const char* last_error() { return g_err; }

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

}  // namespace dkh
