/*
 * dk_oracle.c -- plain FP64 CPU oracle for the MLMC Dean--Kawasaki hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no source with the HIP path.
 *
 * Everything is written out the slow, obvious way, following Cornalba & Fischer,
 * "Multilevel Monte Carlo methods for the Dean--Kawasaki equation from Fluctuating
 * Hydrodynamics" (arXiv 2311.08872):
 *
 *   - discrete model: Definition "def_discrete_DK", eq. (FullyDiscreteDK), with the explicit
 *     Euler--Maruyama weights b0 = 0, b1 = 1 (Sec. 7, "Setting and specifics");
 *   - operators: the 5-point Laplacian and the central divergence of Sec. 7; the staggered
 *     (edge-flux) divergence is an extra mode, a forward difference of edge fluxes;
 *   - noise basis e_{h,y,r} = h^{-d/2} 1_{y=z} f_r (Sec. 2) and Brownian increments of
 *     variance tau per (site, direction, step);
 *   - NN ("Right-Most") coupling, Sec. 3.2: h_{l-1} = 2 h_l, tau_{l-1} = 4 tau_l, coarse
 *     Brownian motions 2^{-d/2} times the sum over the right-most 2x2 block, and coarse
 *     increments the sum of the 4 fine increments of one coarse step;
 *   - observables P_l of eq. (eqn_MLMCLevels) with the discrete mean field of Sec. 3.
 *
 * Random numbers: Philox4x32-10 from its published definition (Salmon, Moraes, Dror,
 * Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), followed by the Box--Muller
 * transform (Box & Muller 1958) evaluated as a fixed sequence of IEEE-754 binary32
 * operations (each correctly rounded), so that any implementation that performs the same
 * sequence obtains the same bits.  This file must be compiled with -ffp-contract=off.
 *
 * The state is FP64; the FP32 normals are widened exactly to double.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11, Sec. "Philox"): the round function multiplies words 0 and 2 by  */
/* the two round constants, takes high and low halves, and XORs the high halves with     */
/* words 1 and 3 and with the round key.  The key is bumped by the Weyl constants after  */
/* every round.                                                                         */
/* ------------------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void dko_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------------------ */
/* Box--Muller on two 32-bit words, as an exact sequence of binary32 operations.          */
/*                                                                                      */
/*  radius word a: w = 2*(a >> 9) + 1,  u = w * 2^-24 in (0,1)                           */
/*     w = 2^e * m with m in [1,2) (exact), folded to m in [sqrt(1/2), sqrt(2)]          */
/*     ln u = (e - 24) ln2 + ln m,  ln m = x * g(x),  x = m - 1 (exact),                 */
/*     g(x) = ln(1 + x)/x by a degree-10 polynomial: the interpolant of g at the 11      */
/*     Chebyshev nodes of [sqrt(1/2) - 1, sqrt(2) - 1], coefficients rounded to binary32; */
/*     its error is below the rounding of the result (max relative error of ln m 1.2e-7) */
/*     R = sqrt(-2 ln u)                                                                 */
/*  angle word b: quadrant q = b >> 30, f = (2*((b >> 7) & 0x7fffff) + 1) * 2^-24        */
/*     angle inside the quadrant psi = f*pi/2, folded to g*pi/2 with g <= 1/2            */
/*     sin, cos of g*pi/2 by their Taylor series to degree 9 and 10 (Horner form in       */
/*     phi^2; the next terms are below 2e-9)                                             */
/*  z0 = R cos(2 pi (q + f)/4),  z1 = R sin(2 pi (q + f)/4)                              */
/* ------------------------------------------------------------------------------------ */
static float exp2i_f(int e)   /* 2^e for small integer e, exactly */
{
    return ldexpf(1.0f, e);
}

void dko_gauss_pair(uint32_t a, uint32_t b, float* z0, float* z1)
{
    /* radius */
    uint32_t w = 2u * (a >> 9) + 1u;          /* odd, in [1, 2^24) */
    int e = 0;
    while ((w >> (e + 1)) != 0u) ++e;          /* 2^e <= w < 2^(e+1) */
    float m = (float)w * exp2i_f(-e);          /* exact, in [1,2) */
    if (m > 1.41421356f) { m = m * 0.5f; e = e + 1; }
    int n = e - 24;

    float x = m - 1.0f;                         /* exact (Sterbenz) */
    float gx = 0x1.0d33dap-4f;                  /* g(x) = ln(1 + x)/x, degree 10 */
    gx = fmaf(gx, x, -0x1.dbfb56p-4f);
    gx = fmaf(gx, x, 0x1.e94d9cp-4f);
    gx = fmaf(gx, x, -0x1.fcc1c0p-4f);
    gx = fmaf(gx, x, 0x1.231156p-3f);
    gx = fmaf(gx, x, -0x1.5554c0p-3f);
    gx = fmaf(gx, x, 0x1.99a6e4p-3f);
    gx = fmaf(gx, x, -0x1.00002ap-2f);
    gx = fmaf(gx, x, 0x1.555540p-2f);
    gx = fmaf(gx, x, -0.5f);
    gx = fmaf(gx, x, 1.0f);
    float lnm = x * gx;                         /* ln m */
    const float LN2_HI = 0x1.62ep-1f;          /* ln 2 rounded to 12 significant bits */
    const float LN2_LO = (float)(0.69314718055994530942 - 0.693115234375);
    float fn = (float)n;
    float A = fn * LN2_HI;                      /* exact */
    float B = fmaf(fn, LN2_LO, lnm);
    float lnu = A + B;
    float r2 = -2.0f * lnu;
    float R = sqrtf(r2);

    /* angle */
    uint32_t q = b >> 30;
    uint32_t j = (b >> 7) & 0x7FFFFFu;
    float f = (float)(2u * j + 1u) * exp2i_f(-24);
    int swap = 0;
    float g = f;
    if (f > 0.5f) { g = 1.0f - f; swap = 1; }
    const float PIO2 = 0x1.921fb6p+0f;         /* pi/2 rounded to binary32 */
    float ph = g * PIO2;
    float ph2 = ph * ph;
    float sp = 1.0f / 362880.0f;
    sp = fmaf(sp, ph2, -1.0f / 5040.0f);
    sp = fmaf(sp, ph2, 1.0f / 120.0f);
    sp = fmaf(sp, ph2, -1.0f / 6.0f);
    float ph3 = ph * ph2;
    float S = fmaf(ph3, sp, ph);
    float cp = -1.0f / 3628800.0f;
    cp = fmaf(cp, ph2, 1.0f / 40320.0f);
    cp = fmaf(cp, ph2, -1.0f / 720.0f);
    cp = fmaf(cp, ph2, 1.0f / 24.0f);
    cp = fmaf(cp, ph2, -0.5f);
    float C = fmaf(ph2, cp, 1.0f);
    float cq = swap ? S : C;   /* cos and sin of the angle inside the quadrant */
    float sq = swap ? C : S;
    float c, sn;
    switch (q) {
        case 0: c = cq; sn = sq; break;
        case 1: c = -sq; sn = cq; break;
        case 2: c = -cq; sn = -sq; break;
        default: c = sq; sn = -cq; break;
    }
    *z0 = R * c;
    *z1 = R * sn;
}

/* ------------------------------------------------------------------------------------ */
/* Problem description (the oracle's own copy of the layout)                             */
/* ------------------------------------------------------------------------------------ */
typedef struct { double amp, kx, ky, phase; } dko_mode;

typedef struct {
    int32_t kind;
    int32_t n_modes;
    double c0;
    const dko_mode* modes;
    double floor_add;
    double bump_amp, bump_sigma, bump_cx, bump_cy;
    double es_a, es_b, es_s, es_x0, es_y0, es_scale;
} dko_field;

typedef struct {
    dko_field phi;
    int32_t centre;
    int32_t scale_sqrtN;
    int32_t psi;
    int32_t pad;
} dko_obs;

typedef struct {
    double box;
    int32_t n0;
    int32_t levels;
    double mu;
    double N;
    int32_t steps0;       /* number of steps on level 0 (M_l = steps0 * 4^l) */
    int32_t flux;         /* 0 central, 1 staggered */
    int32_t n_obs;
    int32_t cell_centred; /* 0: grid points x_i = i h; 1: cell centres x_i = (i + 1/2) h */
    const dko_obs* obs;
    dko_field rho0;
    uint64_t seed;
} dko_problem;

#define FIELD_MODES 0
#define FIELD_CLIPPED 1
#define FIELD_BUMP 2
#define FIELD_EXPSIN2 3

static double periodic_dist(double a, double b, double box)
{
    double d = fabs(a - b);
    d = fmod(d, box);
    if (d > 0.5 * box) d = box - d;
    return d;
}

double dko_field_at(const dko_field* f, double box, double x, double y)
{
    const double two_pi = 6.28318530717958647692;
    double v = f->c0;
    switch (f->kind) {
        case FIELD_MODES:
        case FIELD_CLIPPED:
            for (int k = 0; k < f->n_modes; ++k) {
                const dko_mode* md = &f->modes[k];
                v += md->amp * cos(two_pi * (md->kx * x + md->ky * y) / box + md->phase);
            }
            if (f->kind == FIELD_CLIPPED) v = (v > 0.0 ? v : 0.0) + f->floor_add;
            return v;
        case FIELD_BUMP: {
            double dx = periodic_dist(x, f->bump_cx, box);
            double dy = periodic_dist(y, f->bump_cy, box);
            return v + f->bump_amp * exp(-(dx * dx + dy * dy) / (2.0 * f->bump_sigma * f->bump_sigma));
        }
        case FIELD_EXPSIN2: {
            double sx = sin(x - f->es_x0), sy = sin(y - f->es_y0);
            return f->es_scale * (f->es_a + f->es_b * exp(-(sx * sx + sy * sy) / (2.0 * f->es_s)));
        }
        default:
            return NAN;
    }
}

/* I_h f on the n x n grid with points x_i = (i + offset) h, stored x fastest: out[x + n*y] */
void dko_field_grid_at(const dko_field* f, double box, int n, double offset, double* out)
{
    double h = box / n;
    for (int iy = 0; iy < n; ++iy)
        for (int ix = 0; ix < n; ++ix)
            out[ix + n * iy] = dko_field_at(f, box, (ix + offset) * h, (iy + offset) * h);
}

/* I_h f on the vertex grid x_i = i h */
void dko_field_grid(const dko_field* f, double box, int n, double* out)
{
    dko_field_grid_at(f, box, n, 0.0, out);
}

/* I_h f on the problem's grid: vertices, or the cell centres of the symmetric NN coupling
   (the remark after Sec. 3.2: the coupling unchanged on the points -pi + h/2, ..., pi - h/2) */
static void problem_field(const dko_problem* p, const dko_field* f, int n, double* out)
{
    dko_field_grid_at(f, p->box, n, p->cell_centred ? 0.5 : 0.0, out);
}

/* ------------------------------------------------------------------------------------ */
/* Noise: the standard normals z[y][x][r] of one fine step.                              */
/* One Philox call per horizontal site pair (2a, y), (2a+1, y) and step m:               */
/*   counter = (a + (n/2) y, m, sample_lo32, tag<<24 | level<<16 | sample_hi16)          */
/*   key     = (seed_lo32, seed_hi32)                                                    */
/*   words (0,1) -> site (2a, y) directions (0,1); words (2,3) -> site (2a+1, y)         */
/* ------------------------------------------------------------------------------------ */
void dko_noise_step(uint64_t seed, uint32_t tag, int level, uint64_t sample, int n, int m, double* z)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    for (int y = 0; y < n; ++y) {
        for (int a = 0; a < n / 2; ++a) {
            uint32_t ctr[4] = { (uint32_t)(a + (n / 2) * y), (uint32_t)m, (uint32_t)sample,
                                (tag << 24) | ((uint32_t)level << 16) | (uint32_t)((sample >> 32) & 0xFFFFu) };
            uint32_t o[4];
            dko_philox4x32_10(ctr, key, o);
            float z00, z01, z10, z11;
            dko_gauss_pair(o[0], o[1], &z00, &z01);
            dko_gauss_pair(o[2], o[3], &z10, &z11);
            int x0 = 2 * a, x1 = 2 * a + 1;
            z[2 * (x0 + n * y) + 0] = (double)z00;
            z[2 * (x0 + n * y) + 1] = (double)z01;
            z[2 * (x1 + n * y) + 0] = (double)z10;
            z[2 * (x1 + n * y) + 1] = (double)z11;
        }
    }
}

/* float version for bit-exact comparison of the generator */
void dko_noise_step_f32(uint64_t seed, uint32_t tag, int level, uint64_t sample, int n, int m, float* z)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    for (int y = 0; y < n; ++y) {
        for (int a = 0; a < n / 2; ++a) {
            uint32_t ctr[4] = { (uint32_t)(a + (n / 2) * y), (uint32_t)m, (uint32_t)sample,
                                (tag << 24) | ((uint32_t)level << 16) | (uint32_t)((sample >> 32) & 0xFFFFu) };
            uint32_t o[4];
            dko_philox4x32_10(ctr, key, o);
            int x0 = 2 * a, x1 = 2 * a + 1;
            dko_gauss_pair(o[0], o[1], &z[2 * (x0 + n * y) + 0], &z[2 * (x0 + n * y) + 1]);
            dko_gauss_pair(o[2], o[3], &z[2 * (x1 + n * y) + 0], &z[2 * (x1 + n * y) + 1]);
        }
    }
}

/* ------------------------------------------------------------------------------------ */
/* One explicit Euler--Maruyama step of eq. (FullyDiscreteDK) with b0 = 0, b1 = 1:        */
/*   rho' = rho + tau (1/2) Lap_h rho + N^{-1/2} div_h( b ),                             */
/*   [b]_r(y) = h^{-d/2} sqrt([rho(y)]^+) dbeta_{y,r}           (central mode)           */
/*   [b]_r(y) = h^{-d/2} sqrt([(rho(y)+rho(y+h f_r))/2]^+) dbeta_{y,r}   (staggered)     */
/*   Lap_h a(x) = (-4 a(x) + sum of the 4 neighbours)/h^2                                */
/*   central:   div_h b(x) = sum_r ([b]_r(x + h f_r) - [b]_r(x - h f_r)) / (2h)          */
/*   staggered: div_h b(x) = sum_r ([b]_r(x) - [b]_r(x - h f_r)) / h                     */
/* dbeta is stored [site][r] with site = x + n*y and already carries the factor sqrt(tau)*/
/* ------------------------------------------------------------------------------------ */
static int wrap(int i, int n) { return ((i % n) + n) % n; }

void dko_em_step(int n, double h, double tau, double N, int flux,
                 const double* rho, const double* dbeta, double* out)
{
    double* b = (double*)malloc(sizeof(double) * 2 * n * n);
    double hd2 = 1.0 / h;   /* h^{-d/2} with d = 2 */
    for (int y = 0; y < n; ++y) {
        for (int x = 0; x < n; ++x) {
            int s = x + n * y;
            if (flux == 0) {
                double r = rho[s] > 0.0 ? rho[s] : 0.0;
                b[2 * s + 0] = hd2 * sqrt(r) * dbeta[2 * s + 0];
                b[2 * s + 1] = hd2 * sqrt(r) * dbeta[2 * s + 1];
            } else {
                double rx = 0.5 * (rho[s] + rho[wrap(x + 1, n) + n * y]);
                double ry = 0.5 * (rho[s] + rho[x + n * wrap(y + 1, n)]);
                rx = rx > 0.0 ? rx : 0.0;
                ry = ry > 0.0 ? ry : 0.0;
                b[2 * s + 0] = hd2 * sqrt(rx) * dbeta[2 * s + 0];
                b[2 * s + 1] = hd2 * sqrt(ry) * dbeta[2 * s + 1];
            }
        }
    }
    double invsqrtN = 1.0 / sqrt(N);
    for (int y = 0; y < n; ++y) {
        for (int x = 0; x < n; ++x) {
            int s = x + n * y;
            int xp = wrap(x + 1, n) + n * y, xm = wrap(x - 1, n) + n * y;
            int yp = x + n * wrap(y + 1, n), ym = x + n * wrap(y - 1, n);
            double lap = (-4.0 * rho[s] + rho[xp] + rho[xm] + rho[yp] + rho[ym]) / (h * h);
            double div;
            if (flux == 0)
                div = (b[2 * xp + 0] - b[2 * xm + 0]) / (2.0 * h) + (b[2 * yp + 1] - b[2 * ym + 1]) / (2.0 * h);
            else
                div = (b[2 * s + 0] - b[2 * xm + 0]) / h + (b[2 * s + 1] - b[2 * ym + 1]) / h;
            out[s] = rho[s] + tau * 0.5 * lap + invsqrtN * div;
        }
    }
    free(b);
}

/* (f, g)_h = h^d sum_x f(x) g(x) */
static double inner_h(int n, double h, const double* f, const double* g)
{
    double acc = 0.0;
    for (int s = 0; s < n * n; ++s) acc += f[s] * g[s];
    return h * h * acc;
}

/* ------------------------------------------------------------------------------------ */
/* Level data                                                                           */
/* ------------------------------------------------------------------------------------ */
static int level_n(const dko_problem* p, int l) { return p->n0 << l; }
static double level_h(const dko_problem* p, int l) { return p->box / (double)level_n(p, l); }
static double level_tau(const dko_problem* p, int l) { double h = level_h(p, l); return p->mu * h * h; }
static long level_steps(const dko_problem* p, int l) { return (long)p->steps0 << (2 * l); }

/* Discrete mean field on level l (noise-free run of the scheme from I_h rho0), and the
 * centring constants c_j = (rho_bar^M, I_h phi_j)_h.  rho_out may be NULL. */
void dko_meanfield(const dko_problem* p, int level, double* c_out, double* rho_out)
{
    int n = level_n(p, level);
    double h = level_h(p, level), tau = level_tau(p, level);
    long M = level_steps(p, level);
    double* rho = (double*)malloc(sizeof(double) * n * n);
    double* nxt = (double*)malloc(sizeof(double) * n * n);
    double* zero = (double*)calloc(2 * n * n, sizeof(double));
    double* phi = (double*)malloc(sizeof(double) * n * n);
    problem_field(p, &p->rho0, n, rho);
    for (long m = 0; m < M; ++m) {
        dko_em_step(n, h, tau, 1.0, 0, rho, zero, nxt);   /* dbeta = 0: no noise term */
        double* t = rho; rho = nxt; nxt = t;
    }
    for (int j = 0; j < p->n_obs; ++j) {
        problem_field(p, &p->obs[j].phi, n, phi);
        c_out[j] = inner_h(n, h, rho, phi);
    }
    if (rho_out) memcpy(rho_out, rho, sizeof(double) * n * n);
    free(rho); free(nxt); free(zero); free(phi);
}

/* P_j = psi_j( s_j ((rho, I_h phi_j)_h - c_j) ) */
static void observables(const dko_problem* p, int n, double h, const double* rho,
                        const double* centre, double* P, int stride)
{
    double* phi = (double*)malloc(sizeof(double) * n * n);
    for (int j = 0; j < p->n_obs; ++j) {
        const dko_obs* o = &p->obs[j];
        problem_field(p, &o->phi, n, phi);
        double L = inner_h(n, h, rho, phi);
        double X = L - (o->centre ? centre[j] : 0.0);
        if (o->scale_sqrtN) X *= sqrt(p->N);
        P[j * stride] = (o->psi == 1) ? X * X : X;
    }
    free(phi);
}

/* ------------------------------------------------------------------------------------ */
/* One sample on one level, uncoupled (level 0 of MLMC, or plain MC).                    */
/* P_out[j] for each observable; rho_out (optional) receives the final field.            */
/* ------------------------------------------------------------------------------------ */
void dko_run_single(const dko_problem* p, int level, uint64_t sample, uint32_t tag,
                    const double* centre, double* P_out, double* rho_out)
{
    int n = level_n(p, level);
    double h = level_h(p, level), tau = level_tau(p, level);
    long M = level_steps(p, level);
    double* rho = (double*)malloc(sizeof(double) * n * n);
    double* nxt = (double*)malloc(sizeof(double) * n * n);
    double* z = (double*)malloc(sizeof(double) * 2 * n * n);
    double* db = (double*)malloc(sizeof(double) * 2 * n * n);
    problem_field(p, &p->rho0, n, rho);
    double st = sqrt(tau);
    for (long m = 0; m < M; ++m) {
        dko_noise_step(p->seed, tag, level, sample, n, (int)m, z);
        for (int k = 0; k < 2 * n * n; ++k) db[k] = st * z[k];
        dko_em_step(n, h, tau, p->N, p->flux, rho, db, nxt);
        double* t = rho; rho = nxt; nxt = t;
    }
    observables(p, n, h, rho, centre, P_out, 1);
    if (rho_out) memcpy(rho_out, rho, sizeof(double) * n * n);
    free(rho); free(nxt); free(z); free(db);
}

/* ------------------------------------------------------------------------------------ */
/* One coupled pair (fine level l >= 1, coarse level l-1), NN coupling of Sec. 3.2:       */
/*   coarse site x = (a, b) on G_{l-1} sits at fine site (2a, 2b);                       */
/*   B->(x) = { (2a + v1, 2b + v2) : v in {0,1}^2 };                                     */
/*   coarse Brownian increment over coarse step m_c, direction r:                        */
/*      dbeta_c = 2^{-d/2} sum_{j=0..3} sum_{z in B->(x)} dbeta_f^{4 m_c + j}(z, r)      */
/* P_out[2j] = P_j on the fine level, P_out[2j+1] = P_j on the coarse level.             */
/* ------------------------------------------------------------------------------------ */
void dko_run_pair(const dko_problem* p, int level, uint64_t sample, uint32_t tag,
                  const double* centre_f, const double* centre_c, double* P_out,
                  double* rho_f_out, double* rho_c_out, double* zc_out)
{
    int nf = level_n(p, level), nc = nf / 2;
    double hf = level_h(p, level), hc = level_h(p, level - 1);
    double tf = level_tau(p, level), tc = level_tau(p, level - 1);
    long Mf = level_steps(p, level);
    long Mc = Mf / 4;
    double* rf = (double*)malloc(sizeof(double) * nf * nf);
    double* rfn = (double*)malloc(sizeof(double) * nf * nf);
    double* rc = (double*)malloc(sizeof(double) * nc * nc);
    double* rcn = (double*)malloc(sizeof(double) * nc * nc);
    double* z = (double*)malloc(sizeof(double) * 2 * nf * nf);
    double* dbf = (double*)malloc(sizeof(double) * 2 * nf * nf);
    double* dbc = (double*)malloc(sizeof(double) * 2 * nc * nc);
    problem_field(p, &p->rho0, nf, rf);
    problem_field(p, &p->rho0, nc, rc);
    double stf = sqrt(tf);
    for (long mc = 0; mc < Mc; ++mc) {
        memset(dbc, 0, sizeof(double) * 2 * nc * nc);
        for (int j = 0; j < 4; ++j) {
            long m = 4 * mc + j;
            dko_noise_step(p->seed, tag, level, sample, nf, (int)m, z);
            for (int k = 0; k < 2 * nf * nf; ++k) dbf[k] = stf * z[k];
            dko_em_step(nf, hf, tf, p->N, p->flux, rf, dbf, rfn);
            double* t = rf; rf = rfn; rfn = t;
            for (int b = 0; b < nc; ++b)
                for (int a = 0; a < nc; ++a)
                    for (int v2 = 0; v2 < 2; ++v2)
                        for (int v1 = 0; v1 < 2; ++v1)
                            for (int r = 0; r < 2; ++r)
                                dbc[2 * (a + nc * b) + r] += dbf[2 * ((2 * a + v1) + nf * (2 * b + v2)) + r];
        }
        for (int k = 0; k < 2 * nc * nc; ++k) dbc[k] *= 0.5;   /* 2^{-d/2}, d = 2 */
        if (zc_out && mc == 0) {
            for (int k = 0; k < 2 * nc * nc; ++k) zc_out[k] = dbc[k] / sqrt(tc);
        }
        dko_em_step(nc, hc, tc, p->N, p->flux, rc, dbc, rcn);
        double* t = rc; rc = rcn; rcn = t;
    }
    observables(p, nf, hf, rf, centre_f, P_out, 2);
    observables(p, nc, hc, rc, centre_c, P_out + 1, 2);
    if (rho_f_out) memcpy(rho_f_out, rf, sizeof(double) * nf * nf);
    if (rho_c_out) memcpy(rho_c_out, rc, sizeof(double) * nc * nc);
    free(rf); free(rfn); free(rc); free(rcn); free(z); free(dbf); free(dbc);
}

/* Sample ranges, one after the other (threads are added by the caller).
 * Output layout: P[(i * n_obs + j) * 2 + {0: fine, 1: coarse}]; for level 0 / single-level
 * runs the coarse slot is 0. */
void dko_run_range(const dko_problem* p, int level, int coupled, uint64_t first, uint64_t count,
                   uint32_t tag, const double* centre_f, const double* centre_c, double* P)
{
    double* tmp = (double*)malloc(sizeof(double) * 2 * (p->n_obs > 0 ? p->n_obs : 1));
    for (uint64_t i = 0; i < count; ++i) {
        double* dst = P + (size_t)i * p->n_obs * 2;
        if (coupled) {
            dko_run_pair(p, level, first + i, tag, centre_f, centre_c, dst, NULL, NULL, NULL);
        } else {
            dko_run_single(p, level, first + i, tag, centre_f, tmp, NULL);
            for (int j = 0; j < p->n_obs; ++j) { dst[2 * j] = tmp[j]; dst[2 * j + 1] = 0.0; }
        }
    }
    free(tmp);
}

/* Bulk helpers for the tests. */
void dko_philox_many(int64_t count, const uint32_t* ctr, const uint32_t* key, uint32_t* out)
{
    for (int64_t i = 0; i < count; ++i) dko_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

void dko_gauss_many(int64_t count, const uint32_t* a, const uint32_t* b, float* z0, float* z1)
{
    for (int64_t i = 0; i < count; ++i) dko_gauss_pair(a[i], b[i], z0 + i, z1 + i);
}
