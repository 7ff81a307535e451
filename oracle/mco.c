/*
 * mco.c -- sequential CPU oracle of the analog Monte Carlo photon-transport
 * forward projection of arXiv 2201.13191 (section II-A).
 *
 * TEST INFRASTRUCTURE ONLY: the reference for the GPU library, never part of the
 * product path.  Written independently of the GPU library; see mco.h for the
 * scope.  Every operation that can round is spelled out in the order the
 * transport specification fixes, so that one seed has exactly one result:
 *
 *   - fp32 state (position, direction, energy, optical depth), no
 *     contraction of a*b+c into fma (build with -ffp-contract=off), IEEE
 *     division and square root, denormals kept;
 *   - every transcendental (log, sin, cos, cbrt) evaluated in fp64 and
 *     rounded once to fp32;
 *   - the Compton (Kahn) and Rayleigh samplers run in fp64 with correctly
 *     rounded + - * / only; their accept/reject decisions depend on nothing
 *     else;
 *   - cross-section tables are generated in extended precision and rounded
 *     once to fp32.
 *
 * Parity pins (tests/test_oracle_*.py) check this file against closed forms,
 * quadrature of eq. (1)/(2), Beer-Lambert transmission, solid angles and an
 * independent Philox implementation.
 */
#include "mco.h"

#include <math.h>
#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- constants
 * Classical electron radius (CODATA 2018).  Eq. (1) prints a garbled value
 * with two digits swapped; the CODATA value is used. */
#define R_E_CM 2.8179403262e-13L
/* electron rest energy, keV (eq. (1) uses 0.511 MeV) */
#define MEC2_KEV 510.99895
/* Avogadro constant, 1/mol */
#define N_AVO 6.02214076e23L
/* h*c in keV*Angstrom: lambda[A] = HC / E[keV] */
#define HC_KEV_A 12.398419843320026
/* inverse fine-structure constant (CODATA 2018) */
#define ALPHA_INV 137.035999084
/* Bohr radius, Angstrom */
#define BOHR_A 0.529177210903
/* parametric photoelectric constant per electron, cm^2 keV^3 (times Z^3) */
#define C_PE 3.2e-23L
#define TWO_PI_D 6.283185307179586
#define PI_L 3.141592653589793238462643383279502884L

#define MAX_MAT 16
#define MAX_SCATTER 1000      /* interaction safety cap per history        */
#define E_CUT_KEV 1.0f        /* lower end of the model's range            */
#define TALLY_ONE 1048576.0f  /* 2^20 least significant bits per keV       */

struct mco_ctx {
    char err[256];
    int n_mat;
    mco_material mat[MAX_MAT];
    double rayl_b[MAX_MAT];     /* (2 pi r_Z)^2 [A^2], screening of F(x,Z) */
    double pz_scale[MAX_MAT];   /* Compton-profile momentum scale / (m c)   */
    uint32_t phys;              /* MCO_PHYS_* binding effects              */
    int nx, ny, nz;
    float h;
    uint8_t *ids;
    float *rho;
    int have_phantom;
    mco_geometry g;
    int have_geom;
    int n_bins;
    float *e_bin;
    uint64_t *thr;              /* cumulative thresholds on 32-bit draws */
    float e_max;
    int have_spec;
    float *eta_user;
    int n_eta_user;
    int J;
    float *t_pe, *t_coh, *t_inc, *t_eta;
    int tables_dirty;
    int reading;                /* MCO_READING_GRID or MCO_READING_PLAIN */
    int estimator;              /* MCO_SCORE_ANALOG or MCO_SCORE_POINT   */
    int split;                  /* pseudo-particles per scattering event  */
    double rr_kev;              /* Russian-roulette threshold (0: none)   */
    mco_stats stats;
};

static int fail(mco_ctx *c, int code, const char *msg) {
    if (c) snprintf(c->err, sizeof c->err, "%s", msg);
    return code;
}

/* ------------------------------------------------------------ Philox4x32-10
 * Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
 * (SC'11): 10 rounds of two 32x32->64 multiplies, the key bumped by the
 * Weyl constants between rounds. */
void mco_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* uniform on the odd multiples of 2^-24: exact in fp32, never 0 or 1 */
static float uniform01(uint32_t x) {
    return (float)(2u * (x >> 9) + 1u) * 5.9604644775390625e-8f;
}

void mco_uniform_batch(const uint32_t *x, uint64_t n, float *out) {
    for (uint64_t i = 0; i < n; ++i) out[i] = uniform01(x[i]);
}

/* Per-photon stream: key = seed, counter = (photon id, draw index / 4, 0);
 * draw k is word k mod 4 of block k / 4. */
typedef struct {
    uint32_t key[2];
    uint64_t pid;
    uint32_t k;
    uint32_t cached_blk;
    int have_blk;
    uint32_t blk[4];
    int pseudo;           /* a pseudo-particle's stream (see rng_init_pseudo) */
    uint32_t n, tag;
} rng_t;

static void rng_init(rng_t *r, uint64_t seed, uint64_t pid) {
    r->key[0] = (uint32_t)seed;
    r->key[1] = (uint32_t)(seed >> 32);
    r->pid = pid;
    r->k = 0;
    r->have_blk = 0;
    r->pseudo = 0;
}

/* The stream of pseudo-particle i of the photon's n-th scattering when it
 * needs more than one block: counter (photon id, n, (i + 1) * 2^12 + block). */
static void rng_init_pseudo(rng_t *r, uint64_t seed, uint64_t pid, uint32_t n, uint32_t i) {
    rng_init(r, seed, pid);
    r->pseudo = 1;
    r->n = n;
    r->tag = (i + 1u) << 12;
}

static uint32_t rng_raw(rng_t *r) {
    uint32_t b = r->k >> 2;
    if (!r->have_blk || b != r->cached_blk) {
        uint32_t ctr[4] = {(uint32_t)r->pid, (uint32_t)(r->pid >> 32), b, 0u};
        if (r->pseudo) {
            ctr[2] = r->n;
            ctr[3] = r->tag | b;
        }
        mco_philox4x32_10(ctr, r->key, r->blk);
        r->cached_blk = b;
        r->have_blk = 1;
    }
    uint32_t v = r->blk[r->k & 3u];
    r->k++;
    return v;
}

static float rng_u(rng_t *r) { return uniform01(rng_raw(r)); }

/* ------------------------------------------------------------ cross sections
 * Klein-Nishina total cross section per electron: the integral of eq. (1)
 * over the sphere with S(q,Z) = 1 (textbook closed form), extended precision. */
static long double sigma_kn_l(long double e_kev) {
    long double a = e_kev / (long double)MEC2_KEV;
    long double one2a = 1.0L + 2.0L * a;
    long double lg = log1pl(2.0L * a);          /* ln(1 + 2 alpha), no rounding of 1 + 2a */
    long double t1 = (1.0L + a) / (a * a) * (2.0L * (1.0L + a) / one2a - lg / a);
    long double t2 = lg / (2.0L * a);
    long double t3 = (1.0L + 3.0L * a) / (one2a * one2a);
    return 2.0L * PI_L * R_E_CM * R_E_CM * (t1 + t2 - t3);
}

double mco_sigma_kn(double e_kev) { return (double)sigma_kn_l((long double)e_kev); }

/* Coherent integral of eq. (2) with the screened form factor
 * F(x,Z) = Z / (1 + b x^2)^2, x = sin(theta/2)/lambda, in the variable
 * v = x^2 in [0, V], V = 1/lambda^2, cos(theta) = 1 - 2 v / V:
 *   sigma_atom = 2 pi r_e^2 Z^2 * G(B),
 *   G(B) = (1/V) Int_0^V (1 + cos^2) (1 + b v)^-4 dv,   B = b V.
 * Closed form in w = 1 + b v for B >= 0.1; the alternating power series of
 * (1 + B t)^-4 below, where the closed form cancels. */
static long double coh_g(long double B) {
    if (B < 0.1L) {
        long double s = 0.0L, bn = 1.0L;
        for (int n = 0; n <= 40; ++n) {
            long double binom = (long double)(n + 1) * (n + 2) * (n + 3) / 6.0L;
            long double term = binom * bn *
                (2.0L / (n + 1) - 4.0L / (n + 2) + 4.0L / (n + 3));
            s += (n & 1) ? -term : term;
            bn *= B;
        }
        return s;
    }
    long double iw = 1.0L / (1.0L + B);
    long double iw2 = iw * iw, iw3 = iw2 * iw;
    long double j0 = (1.0L - iw3) / 3.0L;                          /* b   I0 */
    long double j1 = 1.0L / 6.0L - iw2 / 2.0L + iw3 / 3.0L;         /* b^2 I1 */
    long double j2 = 1.0L / 3.0L - iw + iw2 - iw3 / 3.0L;           /* b^3 I2 */
    return 2.0L * j0 / B - 4.0L * j1 / (B * B) + 4.0L * j2 / (B * B * B);
}

static long double rayl_b_l(long double z) {
    long double rz = 0.885L * (long double)BOHR_A / cbrtl(z);
    long double t = 2.0L * PI_L * rz;
    return t * t;
}

static void xs_l(long double z, long double zoa, long double e, long double out[3]) {
    long double ne = N_AVO * zoa;                       /* electrons per gram */
    out[0] = ne * C_PE * z * z * z / (e * e * e);
    long double t = e / (long double)HC_KEV_A;          /* 1/lambda          */
    long double B = rayl_b_l(z) * t * t;
    out[1] = ne * 2.0L * PI_L * R_E_CM * R_E_CM * z * coh_g(B);
    out[2] = ne * sigma_kn_l(e);
}

int mco_cross_sections(double z_eff, double z_over_a, double e_kev, double out[3]) {
    if (!(z_eff >= 1.0 && z_eff <= 100.0) || !(z_over_a > 0.0 && z_over_a <= 1.01) ||
        !(e_kev >= 1.0 && e_kev <= 1001.0))
        return MCO_E_INVALID_ARG;
    long double o[3];
    xs_l(z_eff, z_over_a, e_kev, o);
    for (int i = 0; i < 3; ++i) out[i] = (double)o[i];
    return MCO_OK;
}

/* ------------------------------------------------------------ context */
static const mco_material DEFAULT_MATS[5] = {
    {7.64f, 0.49919f, 0.001205f, "air"},
    {7.42f, 0.55508f, 1.0f, "water"},
    {13.0f, 0.48181f, 2.699f, "aluminium"},
    {13.8f, 0.51480f, 1.92f, "bone_ca"},
    {26.0f, 0.46557f, 7.874f, "iron"},
};

static void set_mats(mco_ctx *c, const mco_material *m, int n) {
    c->n_mat = n;
    for (int i = 0; i < n; ++i) {
        c->mat[i] = m[i];
        double rz = 0.885 * BOHR_A / cbrt((double)m[i].z_eff);
        double t = TWO_PI_D * rz;
        c->rayl_b[i] = t * t;
        /* the orbital of radius r_Z has momentum scale hbar / r_Z = (a0 / r_Z)
         * atomic units; one atomic unit of momentum is m c / ALPHA_INV */
        c->pz_scale[i] = (cbrt((double)m[i].z_eff) / 0.885) / ALPHA_INV;
    }
    c->tables_dirty = 1;
}

int mco_create(mco_ctx **out) {
    if (!out) return MCO_E_INVALID_ARG;
    mco_ctx *c = (mco_ctx *)calloc(1, sizeof *c);
    if (!c) return MCO_E_OOM;
    set_mats(c, DEFAULT_MATS, 5);
    c->split = 1;
    *out = c;
    return MCO_OK;
}

void mco_destroy(mco_ctx *c) {
    if (!c) return;
    free(c->ids); free(c->rho); free(c->e_bin); free(c->thr); free(c->eta_user);
    free(c->t_pe); free(c->t_coh); free(c->t_inc); free(c->t_eta);
    free(c);
}

const char *mco_last_error(const mco_ctx *c) { return c ? c->err : "null context"; }

int mco_set_materials(mco_ctx *c, const mco_material *m, int n) {
    if (!c) return MCO_E_INVALID_ARG;
    if (!m || n < 1 || n > MAX_MAT) return fail(c, MCO_E_INVALID_ARG, "n_mat must be 1..16");
    for (int i = 0; i < n; ++i)
        if (!(m[i].z_eff >= 1.0f && m[i].z_eff <= 100.0f) ||
            !(m[i].z_over_a > 0.0f && m[i].z_over_a <= 1.01f))
            return fail(c, MCO_E_INVALID_ARG, "material z_eff/z_over_a out of range");
    set_mats(c, m, n);
    return MCO_OK;
}

int mco_load_phantom(mco_ctx *c, const uint8_t *ids, const float *rho, int nx, int ny,
                     int nz, float h) {
    if (!c) return MCO_E_INVALID_ARG;
    if (!ids || !rho || nx < 1 || ny < 1 || nz < 1 || nx > 4096 || ny > 4096 || nz > 4096 ||
        !(h > 0.0f) || !isfinite(h))
        return fail(c, MCO_E_INVALID_ARG, "bad phantom dimensions");
    size_t nv = (size_t)nx * ny * nz;
    for (size_t i = 0; i < nv; ++i)
        if (!isfinite(rho[i]) || rho[i] < 0.0f || rho[i] > 1000.0f)
            return fail(c, MCO_E_INVALID_ARG, "density must be finite and in [0, 1000]");
    uint8_t *ni = (uint8_t *)malloc(nv);
    float *nr = (float *)malloc(nv * sizeof(float));
    if (!ni || !nr) { free(ni); free(nr); return fail(c, MCO_E_OOM, "phantom allocation"); }
    memcpy(ni, ids, nv);
    memcpy(nr, rho, nv * sizeof(float));
    free(c->ids); free(c->rho);
    c->ids = ni; c->rho = nr;
    c->nx = nx; c->ny = ny; c->nz = nz; c->h = h;
    c->have_phantom = 1;
    return MCO_OK;
}

int mco_set_geometry(mco_ctx *c, const mco_geometry *g) {
    if (!c) return MCO_E_INVALID_ARG;
    if (!g) return fail(c, MCO_E_INVALID_ARG, "null geometry");
    if (!(g->sod_mm > 0.0f) || !(g->sdd_mm > g->sod_mm) || !isfinite(g->sdd_mm))
        return fail(c, MCO_E_INVALID_ARG, "need 0 < sod < sdd");
    if (g->nu < 1 || g->nv < 1 || g->nu > 16384 || g->nv > 16384 || !(g->pu_mm > 0.0f) ||
        !(g->pv_mm > 0.0f) || !isfinite(g->pu_mm) || !isfinite(g->pv_mm))
        return fail(c, MCO_E_INVALID_ARG, "bad detector");
    if (g->snu < 1 || g->snv < 1 || g->nu % g->snu || g->nv % g->snv)
        return fail(c, MCO_E_INVALID_ARG, "scatter grid must divide the detector");
    if (!(g->step_mm > 0.0f) || !isfinite(g->step_mm))
        return fail(c, MCO_E_INVALID_ARG, "step must be > 0");
    if (g->flags & ~MCO_NO_SCATTER) return fail(c, MCO_E_INVALID_ARG, "unknown flags");
    c->g = *g;
    c->have_geom = 1;
    return MCO_OK;
}

int mco_set_spectrum(mco_ctx *c, const float *e, const float *w, int n) {
    if (!c) return MCO_E_INVALID_ARG;
    if (!e || !w || n < 1 || n > 4096) return fail(c, MCO_E_INVALID_ARG, "n_bins must be 1..4096");
    double total = 0.0;
    float emax = 0.0f;
    for (int k = 0; k < n; ++k) {
        if (!(e[k] >= 1.0f && e[k] <= 1000.0f))
            return fail(c, MCO_E_INVALID_ARG, "bin energy outside [1, 1000] keV");
        if (!(w[k] >= 0.0f) || !isfinite(w[k]))
            return fail(c, MCO_E_INVALID_ARG, "weights must be finite and >= 0");
        total += (double)w[k];
        if (e[k] > emax) emax = e[k];
    }
    if (!(total > 0.0)) return fail(c, MCO_E_INVALID_ARG, "weights sum to zero");
    float *ne = (float *)malloc(n * sizeof(float));
    uint64_t *nt = (uint64_t *)malloc(n * sizeof(uint64_t));
    if (!ne || !nt) { free(ne); free(nt); return fail(c, MCO_E_OOM, "spectrum allocation"); }
    double cum = 0.0;
    for (int k = 0; k < n; ++k) {
        ne[k] = e[k];
        cum += (double)w[k];
        nt[k] = (k == n - 1) ? (uint64_t)1 << 32
                             : (uint64_t)floor(cum / total * 4294967296.0);
    }
    free(c->e_bin); free(c->thr);
    c->e_bin = ne; c->thr = nt; c->n_bins = n; c->e_max = emax;
    c->have_spec = 1;
    c->tables_dirty = 1;
    return MCO_OK;
}

int mco_set_detector_response(mco_ctx *c, const float *eta, int n) {
    if (!c) return MCO_E_INVALID_ARG;
    if (!eta || n < 1 || n > 4096) return fail(c, MCO_E_INVALID_ARG, "eta length must be 1..4096");
    for (int i = 0; i < n; ++i)
        if (!(eta[i] >= 0.0f) || !isfinite(eta[i]))
            return fail(c, MCO_E_INVALID_ARG, "eta must be finite and >= 0");
    float *ne = (float *)malloc(n * sizeof(float));
    if (!ne) return fail(c, MCO_E_OOM, "eta allocation");
    memcpy(ne, eta, n * sizeof(float));
    free(c->eta_user);
    c->eta_user = ne;
    c->n_eta_user = n;
    c->tables_dirty = 1;
    return MCO_OK;
}

/* Tables on the grid E_j = 1 + j keV, j = 0 .. J-1, J = floor(E_max) + 2, so
 * that every energy a photon can carry has both neighbours on the grid. */
static int build_tables(mco_ctx *c) {
    if (!c->tables_dirty) return MCO_OK;
    int J = (int)floorf(c->e_max) + 2;
    size_t n = (size_t)c->n_mat * J;
    float *pe = (float *)malloc(n * sizeof(float));
    float *coh = (float *)malloc(n * sizeof(float));
    float *inc = (float *)malloc(n * sizeof(float));
    float *eta = (float *)malloc(J * sizeof(float));
    if (!pe || !coh || !inc || !eta) {
        free(pe); free(coh); free(inc); free(eta);
        return fail(c, MCO_E_OOM, "table allocation");
    }
    for (int m = 0; m < c->n_mat; ++m)
        for (int j = 0; j < J; ++j) {
            long double o[3];
            xs_l((long double)c->mat[m].z_eff, (long double)c->mat[m].z_over_a,
                 (long double)(1 + j), o);
            pe[(size_t)m * J + j] = (float)o[0];
            coh[(size_t)m * J + j] = (float)o[1];
            inc[(size_t)m * J + j] = (float)o[2];
        }
    for (int j = 0; j < J; ++j) {
        if (c->eta_user)
            eta[j] = c->eta_user[j < c->n_eta_user ? j : c->n_eta_user - 1];
        else
            eta[j] = (float)(1 + j);
    }
    free(c->t_pe); free(c->t_coh); free(c->t_inc); free(c->t_eta);
    c->t_pe = pe; c->t_coh = coh; c->t_inc = inc; c->t_eta = eta;
    c->J = J;
    c->tables_dirty = 0;
    return MCO_OK;
}

int mco_get_tables(mco_ctx *c, int *J, float *pe, float *coh, float *inc, float *eta) {
    if (!c || !J) return MCO_E_INVALID_ARG;
    if (!c->have_spec) return fail(c, MCO_E_STATE, "spectrum not set");
    int rc = build_tables(c);
    if (rc) return rc;
    *J = c->J;
    size_t n = (size_t)c->n_mat * c->J;
    if (pe) memcpy(pe, c->t_pe, n * sizeof(float));
    if (coh) memcpy(coh, c->t_coh, n * sizeof(float));
    if (inc) memcpy(inc, c->t_inc, n * sizeof(float));
    if (eta) memcpy(eta, c->t_eta, c->J * sizeof(float));
    return MCO_OK;
}

/* fp32 linear interpolation on the 1 keV grid */
static float lerp_tab(const float *t, int J, float e) {
    float em1 = e - 1.0f;
    int j = (int)em1;
    if (j < 0) j = 0;
    if (j > J - 2) j = J - 2;
    float f = em1 - (float)j;
    return t[j] + f * (t[j + 1] - t[j]);
}

/* ------------------------------------------------------------ geometry
 * Source on a circle of radius sod around the z axis at angle beta; the
 * panel is perpendicular to the central ray at distance sdd; u runs along
 * (-sin b, cos b, 0), v along z.  The phantom box is centred on the origin. */
typedef struct {
    float S[3], ax[3], eu[3], ev[3], D[3];
    float hu, hv, omc;
    float lo[3], hi[3], inv_h;
} proj_t;

static void proj_setup(const mco_ctx *c, float beta, proj_t *P) {
    float cb = (float)cos((double)beta), sb = (float)sin((double)beta);
    const mco_geometry *g = &c->g;
    P->S[0] = g->sod_mm * cb; P->S[1] = g->sod_mm * sb; P->S[2] = 0.0f;
    P->ax[0] = -cb; P->ax[1] = -sb; P->ax[2] = 0.0f;
    P->eu[0] = -sb; P->eu[1] = cb; P->eu[2] = 0.0f;
    P->ev[0] = 0.0f; P->ev[1] = 0.0f; P->ev[2] = 1.0f;
    for (int a = 0; a < 3; ++a) P->D[a] = P->S[a] + g->sdd_mm * P->ax[a];
    P->hu = 0.5f * ((float)g->nu * g->pu_mm);
    P->hv = 0.5f * ((float)g->nv * g->pv_mm);
    double sdd = g->sdd_mm, hu = P->hu, hv = P->hv;
    double ctm = sdd / sqrt(sdd * sdd + hu * hu + hv * hv);
    P->omc = (float)(1.0 - ctm);
    int n[3] = {c->nx, c->ny, c->nz};
    for (int a = 0; a < 3; ++a) {
        P->hi[a] = 0.5f * ((float)n[a] * c->h);
        P->lo[a] = -P->hi[a];
    }
    P->inv_h = 1.0f / c->h;
}

/* slab-method ray/box intersection: entry t_in >= 0 and exit t_out */
static int box_hit(const proj_t *P, const float p[3], const float d[3], float *tin,
                   float *tout) {
    float t0 = 0.0f, t1 = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0f) {
            float inv = 1.0f / d[a];
            float ta = (P->lo[a] - p[a]) * inv;
            float tb = (P->hi[a] - p[a]) * inv;
            float tn = ta < tb ? ta : tb;
            float tf = ta < tb ? tb : ta;
            if (tn > t0) t0 = tn;
            if (tf < t1) t1 = tf;
        } else if (p[a] < P->lo[a] || p[a] > P->hi[a]) {
            return 0;
        }
    }
    if (!(t0 < t1)) return 0;
    *tin = t0;
    *tout = t1;
    return 1;
}

/* pixel crossed by the straight line p + t d, or 0 */
static int panel_pixel(const mco_ctx *c, const proj_t *P, const float p[3], const float d[3],
                       int *iu, int *iv) {
    const mco_geometry *g = &c->g;
    float den = (d[0] * P->ax[0] + d[1] * P->ax[1]) + d[2] * P->ax[2];
    if (!(den > 0.0f)) return 0;
    float rel = ((p[0] - P->S[0]) * P->ax[0] + (p[1] - P->S[1]) * P->ax[1]) +
                (p[2] - P->S[2]) * P->ax[2];
    float td = (g->sdd_mm - rel) / den;
    float w[3];
    for (int a = 0; a < 3; ++a) w[a] = (p[a] + td * d[a]) - P->D[a];
    float u = (w[0] * P->eu[0] + w[1] * P->eu[1]) + w[2] * P->eu[2];
    float v = (w[0] * P->ev[0] + w[1] * P->ev[1]) + w[2] * P->ev[2];
    float fu = (u + P->hu) / g->pu_mm;
    float fv = (v + P->hv) / g->pv_mm;
    if (!(fu >= 0.0f && fu < (float)g->nu && fv >= 0.0f && fv < (float)g->nv)) return 0;
    *iu = (int)fu;
    *iv = (int)fv;
    return 1;
}

int mco_detector_pixel(mco_ctx *c, float beta, const float p[3], const float d[3], int *iu,
                       int *iv) {
    if (!c || !p || !d || !iu || !iv) return MCO_E_INVALID_ARG;
    if (!c->have_geom || !c->have_phantom) return fail(c, MCO_E_STATE, "geometry/phantom not set");
    proj_t P;
    proj_setup(c, beta, &P);
    if (!panel_pixel(c, &P, p, d, iu, iv)) { *iu = -1; *iv = -1; }
    return MCO_OK;
}

/* ------------------------------------------------------------ samplers
 * Compton polar angle by Kahn's rejection method (cited in section II-A):
 * x = E/E' in [1, 1 + 2 alpha] from two branches, accepted against the
 * Klein-Nishina shape; three draws per trial.  fp64, correctly rounded
 * operations only. */
static double kahn_x(rng_t *r, double alpha) {
    double x;
    for (;;) {
        double r1 = (double)rng_u(r);
        double r2 = (double)rng_u(r);
        double r3 = (double)rng_u(r);
        if (r1 <= (1.0 + 2.0 * alpha) / (9.0 + 2.0 * alpha)) {
            x = 1.0 + 2.0 * alpha * r2;
            if (r3 <= 4.0 * (1.0 / x - 1.0 / (x * x))) break;
        } else {
            x = (1.0 + 2.0 * alpha) / (1.0 + 2.0 * alpha * r2);
            double c = 1.0 - (x - 1.0) / alpha;
            if (r3 <= 0.5 * (c * c + 1.0 / x)) break;
        }
    }
    return x;
}

/* Rayleigh polar angle for eq. (2): v = x^2 drawn from F^2 ~ (1 + b v)^-4 on
 * [0, V] by inversion, then accepted with the Thomson factor (1 + cos^2)/2;
 * two draws per trial.  The fp32 cosine is what the decision sees. */
static float sample_rayleigh(rng_t *r, float e, double b) {
    double t = (double)e / HC_KEV_A;
    double V = t * t;
    double W = 1.0 + b * V;
    double ymin = 1.0 / (W * W * W);
    for (;;) {
        double r1 = (double)rng_u(r);
        double r2 = (double)rng_u(r);
        double y = 1.0 - r1 * (1.0 - ymin);
        double v = (1.0 / cbrt(y) - 1.0) / b;
        float cf = (float)(1.0 - 2.0 * v / V);
        double cd = (double)cf;
        if (r2 <= 0.5 * (1.0 + cd * cd)) return cf;
    }
}

/* ------------------------------------------------------------ binding effects
 * Eq. (1) carries the incoherent scattering function S(x,Z), and the Compton
 * line is broadened by the motion of the bound electrons (section II-A); the
 * paper takes both from tabulated atomic data, which this build does not
 * have.  Parametric stand-ins from one orbital model: every electron of a
 * material sits in a hydrogen-like 1s orbital whose radius is the screening
 * radius r_Z = 0.885 a0 Z^(-1/3) of the Rayleigh form factor above.  Then
 *   F(x,Z)/Z = (1 + b x^2)^-2               (the form factor already in use),
 *   S(x,Z)/Z = 1 - (F/Z)^2 = 1 - (1 + b x^2)^-4     (independent electrons),
 *   J(p_z)   = 8 / (3 pi p0) (1 + (p_z / p0)^2)^-3,   p0 = hbar / r_Z,
 * the last being the 1s Compton profile (x = sin(theta/2) / lambda of the
 * incoming photon, b = (2 pi r_Z)^2).
 *
 * S by rejection, as a null collision: the tables keep the Klein-Nishina cross
 * section; a Compton collision draws Kahn's angle and is accepted with
 * probability S/Z; a rejected one leaves the photon as it was (direction,
 * energy, primary or scattered), so the effective cross section (the KN
 * integral of S/Z) and the angular law (KN times S/Z) are both exact.
 *
 * Doppler broadening: s = |p_z| / p0 is drawn from (1 + s^2)^-3 by rejection
 * from the envelope (1 + s)^-2 (inverted exactly: s = a / (1 - a), a uniform),
 * accepted with (1 + s)^2 / (M (1 + s^2)^3), M = 1.3064 above the ratio's
 * maximum (at s = (sqrt(17) - 3) / 4); the sign of p_z comes with the same
 * draw.  The scattered energy then solves the impulse-approximation relation
 * P = p_z / (m c) = (r / tau - 1) / sqrt(1 + r^2 - 2 r mu) for r = E'/E, tau =
 * E_KN / E the Compton ratio at the sampled cosine mu: with t = P^2,
 *   r = tau ((1 - t tau mu) +- sqrt((1 - t tau mu)^2 - (1 - t tau^2)(1 - t))) / (1 - t tau^2),
 * the sign that of P.  A draw without a root in (0, 1) is drawn again; the
 * draws with p_z < 0 always have one when tau < 1, so the loop ends. */
#define DOPPLER_ENVELOPE 1.3064

/* S(x,Z)/Z at b [A^2], V = 1/lambda^2 [A^-2] and om = 1 - cos(theta) */
static double incoh_sf(double b, double V, double om) {
    const double w = 1.0 + b * (0.5 * V * om);
    const double w2 = w * w;
    return 1.0 - 1.0 / (w2 * w2);
}

/* one trial of the broadened ratio E'/E (pz = p0 / (m c)), given tau, mu and
 * the differences om = 1 - mu, omt = 1 - tau computed without cancellation;
 * 0 if rejected.  The discriminant is written as
 *   t ((1 - tau)^2 + tau (1 - mu) (2 - t tau (2 - (1 - mu)))),
 * equal to (1 - t tau mu)^2 - (1 - t tau^2)(1 - t) but free of its
 * cancellation near the forward direction, where the latter can round below
 * zero for every draw. */
static int doppler_trial(rng_t *r, double pz, double tau, double mu, double om, double omt,
                         double *ratio) {
    const double v = 2.0 * (double)rng_u(r) - 1.0;
    const double u2 = (double)rng_u(r);
    const double a = fabs(v);
    const double s = a / (1.0 - a);
    const double s2 = 1.0 + s * s;
    if (!(u2 * DOPPLER_ENVELOPE <= ((1.0 + s) * (1.0 + s)) / ((s2 * s2) * s2))) return 0;
    const double P = (v < 0.0 ? -s : s) * pz;
    const double t = P * P;
    const double c1 = 1.0 - (t * tau) * mu;
    const double c2 = 1.0 - (t * tau) * tau;
    const double disc = t * (omt * omt + tau * om * (2.0 - (t * tau) * (2.0 - om)));
    if (!(c2 > 0.0) || !(disc >= 0.0)) return 0;
    const double root = sqrt(disc);
    const double x = tau * ((P < 0.0 ? c1 - root : c1 + root) / c2);
    if (!(x > 0.0 && x < 1.0)) return 0;
    *ratio = x;
    return 1;
}

#define DOPPLER_MAX_TRIALS 256

/* E'/E at Compton ratio tau = 1 / ratio_kn and cosine 1 - om.  Without momentum
 * transfer (a point-detector direction along the photon's own) the line is
 * not shifted.  Each trial succeeds with probability above 0.2 (the draws
 * with p_z < 0 always have a root), so the cap of 256 trials, after which the
 * unbroadened ratio is returned, is reached with probability below 1e-24;
 * it bounds the loop. */
static double sample_doppler(rng_t *r, double pz, double ratio_kn, double om) {
    const double tau = 1.0 / ratio_kn;
    const double omt = (ratio_kn - 1.0) / ratio_kn;
    if (!(tau < 1.0) || !(omt > 0.0)) return 1.0;
    const double mu = 1.0 - om;
    double x;
    for (int k = 0; k < DOPPLER_MAX_TRIALS; ++k)
        if (doppler_trial(r, pz, tau, mu, om, omt, &x)) return x;
    return tau;
}

/* One Compton collision of the transport: Kahn's angle; with
 * MCO_PHYS_INCOH_SF one more draw accepts it with S/Z (0 returned: a null
 * collision); with MCO_PHYS_DOPPLER the broadened energy. */
static int compton_collision(const mco_ctx *c, rng_t *r, int m, float e, float *ct, float *e2) {
    const double alpha = (double)e / MEC2_KEV;
    const double x = kahn_x(r, alpha);
    if (c->phys & MCO_PHYS_INCOH_SF) {
        const double t = (double)e / HC_KEV_A;
        const double u = (double)rng_u(r);
        if (!(u <= incoh_sf(c->rayl_b[m], t * t, (x - 1.0) / alpha))) return 0;
    }
    *ct = (float)(1.0 - (x - 1.0) / alpha);
    if (c->phys & MCO_PHYS_DOPPLER)
        *e2 = (float)((double)e * sample_doppler(r, c->pz_scale[m], x, (x - 1.0) / alpha));
    else
        *e2 = (float)((double)e / x);
    return 1;
}

/* new direction after scattering by polar cosine ct and azimuth (cp, sp) */
static void rotate(float d[3], float ct, float cp, float sp) {
    float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
    float ux = d[0], uy = d[1], uz = d[2];
    float nx, ny, nz;
    if (fabsf(uz) < 0.99999f) {
        float t = sqrtf(1.0f - uz * uz);
        nx = st * ((ux * uz) * cp - uy * sp) / t + ux * ct;
        ny = st * ((uy * uz) * cp + ux * sp) / t + uy * ct;
        nz = uz * ct - (st * cp) * t;
    } else {
        nx = st * cp;
        ny = st * sp;
        nz = uz >= 0.0f ? ct : -ct;
    }
    float inv = 1.0f / sqrtf((nx * nx + ny * ny) + nz * nz);
    d[0] = nx * inv;
    d[1] = ny * inv;
    d[2] = nz * inv;
}

static uint32_t energy_bin(const mco_ctx *c, uint32_t x) {
    int lo = 0, hi = c->n_bins - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((uint64_t)x < c->thr[mid]) hi = mid; else lo = mid + 1;
    }
    return (uint32_t)lo;
}

static void birth(const mco_ctx *c, const proj_t *P, rng_t *r, float *e, float d[3]) {
    *e = c->e_bin[energy_bin(c, rng_raw(r))];
    float ct = 1.0f - rng_u(r) * P->omc;
    float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
    double phi = TWO_PI_D * (double)rng_u(r);
    float cp = (float)cos(phi), sp = (float)sin(phi);
    for (int a = 0; a < 3; ++a)
        d[a] = (ct * P->ax[a] + (st * cp) * P->eu[a]) + (st * sp) * P->ev[a];
}

/* ------------------------------------------------------------ transport */
typedef struct {
    uint16_t n_int;
    uint32_t steps;
    uint8_t end, first;
    float x1[3];      /* first interaction point (NaN when none)          */
    int32_t pix;      /* crossed pixel iv * nu + iu on the panel, or -1    */
    float e_end;      /* energy when the history ended                      */
} hist_t;

/* Optical-depth increments are kept on the grid of 2^-32 (and below 2^21),
 * where fp64 sums are exact: the optical depth after any run of steps does
 * not depend on how the additions are grouped. */
static double on_grid(double x) { return ldexp(rint(ldexp(x, 32)), -32); }

/* Fixed-step march from entry t_in to exit t_out (section II-C-2 fixes only
 * that the step size is a free parameter; this discretisation is the one
 * both implementations follow).  L = t_out - t_in.  Step k starts at
 * a_k = k*step (one fp32 product) and is taken while a_k < L; it is a full
 * step except the last one (the first k with (k+1)*step >= L), of length
 * l = L - a_k.  Its voxel contains the step's nominal centre (k + 1/2)*step
 * in voxel coordinates: with G = (d/h)*step and c_0 = (p_in - lo)/h + G/2,
 * c_k = c_0 + k*G for k a multiple of 4 and c_k = c_{k-1} + G otherwise
 * (fp32, each operation rounded), truncated and clamped to the object.
 * Optical depth: a full step adds on_grid(mu*step) (fp64 product of the fp32
 * values), the last one on_grid(that * min(1, l/step)); the sum is fp64 and
 * exact.  The photon interacts in the first step where it reaches tau_star,
 * at a_k + (tau_star - tau)/inc * length (fp64, rounded to fp32).  Returns 1
 * with the interaction point and voxel. */
static int march(const mco_ctx *c, const proj_t *P, const float p[3], const float d[3],
                 float tin, float tout, const float *mm, float tau_star, float pint[3],
                 size_t *vox, uint32_t *steps, double *tau_exit) {
    const float dl = c->g.step_mm;
    float pin[3], c0[3], G[3], q[3];
    for (int a = 0; a < 3; ++a) pin[a] = p[a] + d[a] * tin;
    float L = tout - tin;
    for (int a = 0; a < 3; ++a) {
        G[a] = (d[a] * P->inv_h) * dl;
        c0[a] = (pin[a] - P->lo[a]) * P->inv_h + 0.5f * G[a];
    }
    const double ts = (double)tau_star;
    double tau = 0.0;
    for (uint32_t k = 0;; ++k) {
        float a0 = (float)k * dl;
        if (!(a0 < L)) {
            if (tau_exit) *tau_exit = tau;
            return 0;
        }
        for (int a = 0; a < 3; ++a)
            q[a] = (k & 3u) == 0u ? c0[a] + (float)k * G[a] : q[a] + G[a];
        int ix = (int)q[0];
        int iy = (int)q[1];
        int iz = (int)q[2];
        ix = ix < 0 ? 0 : (ix > c->nx - 1 ? c->nx - 1 : ix);
        iy = iy < 0 ? 0 : (iy > c->ny - 1 ? c->ny - 1 : iy);
        iz = iz < 0 ? 0 : (iz > c->nz - 1 ? c->nz - 1 : iz);
        size_t v = ((size_t)iz * c->ny + iy) * c->nx + ix;
        float mu = c->rho[v] * mm[c->ids[v]];
        double inc = on_grid((double)mu * (double)dl);
        float len = dl;
        if (!((float)(k + 1u) * dl < L)) {            /* the last, clipped step */
            len = L - a0;
            double r = (double)len / (double)dl;
            if (r > 1.0) r = 1.0;
            inc = on_grid(inc * r);
        }
        (*steps)++;
        if (tau + inc >= ts) {
            float sint = a0 + (float)((ts - tau) / inc * (double)len);
            for (int a = 0; a < 3; ++a) pint[a] = pin[a] + d[a] * sint;
            *vox = v;
            return 1;
        }
        tau = tau + inc;
    }
}

/* The plain reading of the fixed-step march (section II-C-2 fixes only that
 * the step is a free parameter): from the box entry, steps of length
 * step_mm, the last one clipped at the exit; each step looks up the voxel
 * holding its true midpoint, p + d (t_in + t + len/2), and adds mu * len to
 * the optical depth; the photon interacts in the first step where the depth
 * reaches tau_star, at the distance (tau_star - tau) / mu into that step.
 * Positions, lengths and the depth are fp64 throughout; the interaction
 * point is rounded to fp32 once.  Written independently of march(): it
 * shares no step bookkeeping with it and is used only to show that the
 * rounding-exact reading above stays within the parity tolerances of this
 * one (selected by mco_set_reading). */
static int march_plain(const mco_ctx *c, const proj_t *P, const float p[3], const float d[3],
                       float tin, float tout, const float *mm, double tau_star, float pint[3],
                       size_t *vox, uint32_t *steps, double *tau_exit) {
    const double dl = (double)c->g.step_mm;
    const double t0 = (double)tin, L = (double)tout - (double)tin;
    const double h = (double)c->h;
    double tau = 0.0;
    for (uint64_t k = 0;; ++k) {
        const double t = (double)k * dl;
        if (!(t < L)) {
            if (tau_exit) *tau_exit = tau;
            return 0;
        }
        const double len = L - t < dl ? L - t : dl;
        const double s = t0 + t + 0.5 * len;
        int idx[3];
        const int n[3] = {c->nx, c->ny, c->nz};
        for (int a = 0; a < 3; ++a) {
            const double m = (double)p[a] + (double)d[a] * s;
            int i = (int)floor((m - (double)P->lo[a]) / h);
            idx[a] = i < 0 ? 0 : (i > n[a] - 1 ? n[a] - 1 : i);
        }
        const size_t v = ((size_t)idx[2] * c->ny + idx[1]) * c->nx + idx[0];
        const double mu = (double)c->rho[v] * (double)mm[c->ids[v]];
        (*steps)++;
        if (tau + mu * len >= tau_star) {
            const double si = t0 + t + (tau_star - tau) / mu;
            for (int a = 0; a < 3; ++a) pint[a] = (float)((double)p[a] + (double)d[a] * si);
            *vox = v;
            return 1;
        }
        tau += mu * len;
    }
}

static void mat_mu(const mco_ctx *c, float e, float *mm) {
    for (int m = 0; m < c->n_mat; ++m) {
        const size_t o = (size_t)m * c->J;
        float pe = lerp_tab(c->t_pe + o, c->J, e);
        float coh = lerp_tab(c->t_coh + o, c->J, e);
        float inc = lerp_tab(c->t_inc + o, c->J, e);
        mm[m] = ((pe + coh) + inc) * 0.1f;        /* cm^2/g * g/cm^3 -> 1/mm */
    }
}

static void tally(const mco_ctx *c, const proj_t *P, const float p[3], const float d[3],
                  float e, int n_int, int64_t *prim, int64_t *scat, mco_stats *st, hist_t *h) {
    int iu, iv;
    if (!panel_pixel(c, P, p, d, &iu, &iv)) { h->end = MCO_END_MISSED; return; }
    h->pix = iv * c->g.nu + iu;
    float w = lerp_tab(c->t_eta, c->J, e);
    int64_t L = (int64_t)llrintf(w * TALLY_ONE);
    const mco_geometry *g = &c->g;
    if (n_int == 0) {
        if (prim) prim[(size_t)iv * g->nu + iu] += L;
        st->primary_hits++;
        h->end = MCO_END_PRIMARY;
    } else {
        int su = iu / (g->nu / g->snu), sv = iv / (g->nv / g->snv);
        /* with the point-detector estimator the scatter image holds its scores only */
        if (scat && c->estimator == MCO_SCORE_ANALOG) scat[(size_t)sv * g->snu + su] += L;
        st->scatter_hits++;
        h->end = MCO_END_SCATTER;
    }
}

/* ------------------------------------------------------------ point detector
 * The scorer of eq. (3)-(5) with splitting and Russian roulette (section
 * II-C-1).  At every Compton or Rayleigh event the photon is split into
 * `split` pseudo-particles; each picks a random point on the panel (the
 * random pixel of the paper, with a uniform position inside it) and scores
 * the expected energy that reaches that point straight from the event:
 *
 *   x = eta(E') p(lambda) cos(gamma) A / (2 pi d^2 split) * exp(-tau),
 *
 * p(lambda) the pdf per unit scattering cosine of the event's process
 * (eq. (4) Compton, eq. (5) Rayleigh), lambda the cosine between the photon's
 * incoming direction and the direction to the point, d the distance, gamma the
 * angle of that direction to the panel normal, A the panel area (the point's
 * density is 1/A), E' the energy scattered towards the point, and tau the
 * optical depth at E' from the event to the box exit, marched with the same
 * fixed-step rule as the transport.  eq. (3) is the flux of a point detector
 * per unit area normal to the ray; cos(gamma) turns it into the flux through
 * the panel, so the expectation equals the analog scatter image's.  A
 * pseudo-particle whose unattenuated score x0 is below the threshold survives
 * with probability x0 / threshold and then scores with x0 = threshold (the
 * roulette of section II-C-1, unbiased), before its march is paid for.
 *
 * Each pseudo-particle i of the photon's n-th scattering (n counted from 0)
 * draws from its own Philox block, counter (photon id, n, i + 1) -- the
 * analog draws use counters ending in 0 -- so the photon's own history is the
 * same with and without this scorer. */

/* the integral over the scattering cosine of the bracket of eq. (1) with
 * S = 1: sigma_KN / (pi r_e^2) */
static double kn_norm(float e) {
    return (double)(sigma_kn_l((long double)e) / (PI_L * R_E_CM * R_E_CM));
}

/* pdf per unit scattering cosine `lam` of the process at energy e in
 * material m (the one its sampler draws from), and the energy scattered
 * into that direction */
static double pd_pdf(const mco_ctx *c, int proc, int m, float e, double lam, float *e_out) {
    if (proc == MCO_PROC_COMPTON) {
        const double alpha = (double)e / MEC2_KEV;
        const double ratio = 1.0 + alpha * (1.0 - lam);     /* E / E' = alpha / alpha' */
        const double r = 1.0 / ratio;
        *e_out = (float)((double)e / ratio);
        double pdf = r * r * ((r + ratio) - (1.0 - lam * lam)) / kn_norm(e);
        if (c->phys & MCO_PHYS_INCOH_SF) {
            /* a collision sends its photon into lam with KN S/Z: the law's
             * deficit is the null collisions' share, which scores nothing */
            const double t = (double)e / HC_KEV_A;
            pdf *= incoh_sf(c->rayl_b[m], t * t, 1.0 - lam);
        }
        return pdf;
    }
    /* Rayleigh: (1 + lam^2) F^2 with F = Z / (1 + b x^2)^2, x^2 = (1 - lam)/2 / wavelength^2;
     * over lam in [-1, 1] the unnormalised density integrates to 2 Z^2 G(b V) */
    const double t = (double)e / HC_KEV_A;
    const double V = t * t;
    const double w = 1.0 + c->rayl_b[m] * ((1.0 - lam) * 0.5 * V);
    *e_out = e;
    return (1.0 + lam * lam) / (((w * w) * w) * w) /
           (2.0 * (double)coh_g((long double)(c->rayl_b[m] * V)));
}

/* The mixed estimator's Rayleigh pseudo-particle: Rayleigh laws are sharply
 * forward peaked (the form factor), so a random point on the panel rarely
 * lands where the law is large and the point-detector score of eq. (5) has a
 * heavy tail.  Instead the pseudo-particle draws its direction from the
 * Rayleigh law itself (the photon's sampler, then an azimuth, from its own
 * stream) and, if that line crosses the panel, scores eta(E) / split times
 * exp(-tau) to the object's exit in the pixel it crosses: the same
 * expectation (the law's density cancels the score's p(lambda)). */
static void pd_rayleigh_along_law(const mco_ctx *c, const proj_t *P, uint64_t seed,
                                  uint64_t pid, int n, int i, const float o[3],
                                  const float d[3], float e, int m, int64_t *scat,
                                  mco_stats *st) {
    const mco_geometry *g = &c->g;
    rng_t r;
    rng_init_pseudo(&r, seed, pid, (uint32_t)n, (uint32_t)i);
    const float ct = sample_rayleigh(&r, e, c->rayl_b[m]);
    const double phi = TWO_PI_D * (double)rng_u(&r);
    float om[3] = {d[0], d[1], d[2]};
    rotate(om, ct, (float)cos(phi), (float)sin(phi));
    int iu, iv;
    if (!panel_pixel(c, P, o, om, &iu, &iv)) return;     /* misses the panel */
    double x0 = (double)lerp_tab(c->t_eta, c->J, e) / (double)c->split;
    const double u_rr = (double)rng_u(&r);
    if (c->rr_kev > 0.0 && x0 < c->rr_kev) {
        if (u_rr < x0 / c->rr_kev) {
            x0 = c->rr_kev;
        } else {
            st->pd_killed++;
            return;
        }
    }
    double tau = 0.0;
    float tin, tout;
    if (box_hit(P, o, om, &tin, &tout)) {
        float mm[MAX_MAT], pint[3];
        size_t v;
        uint32_t steps = 0;
        mat_mu(c, e, mm);
        if (c->reading == MCO_READING_PLAIN)
            (void)march_plain(c, P, o, om, tin, tout, mm, INFINITY, pint, &v, &steps, &tau);
        else
            (void)march(c, P, o, om, tin, tout, mm, INFINITY, pint, &v, &steps, &tau);
        st->pd_steps += steps;
    }
    const int64_t L = (int64_t)llrint(x0 * exp(-tau) * 1048576.0);
    scat[(size_t)(iv / (g->nv / g->snv)) * g->snu + (size_t)(iu / (g->nu / g->snu))] += L;
    st->pd_scores++;
}

static void pd_event(const mco_ctx *c, const proj_t *P, uint64_t seed, uint64_t pid,
                     int n_int, int n, const float o[3], const float d[3], float e, int m,
                     int proc, int64_t *scat, mco_stats *st) {
    if (n_int + 1 >= MAX_SCATTER) return;     /* the scattered photon is not transported */
    const mco_geometry *g = &c->g;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const double area = (double)((float)g->nu * g->pu_mm) * (double)((float)g->nv * g->pv_mm);
    for (int i = 0; i < c->split; ++i) {
        if (proc == MCO_PROC_RAYLEIGH && c->estimator == MCO_SCORE_POINT_MIXED) {
            pd_rayleigh_along_law(c, P, seed, pid, n, i, o, d, e, m, scat, st);
            continue;
        }
        const uint32_t ctr[4] = {(uint32_t)pid, (uint32_t)(pid >> 32), (uint32_t)n,
                                 (uint32_t)i + 1u};
        uint32_t w[4];
        mco_philox4x32_10(ctr, key, w);
        /* the random point on the panel, in pixel units, and its pixel */
        const float fu = uniform01(w[0]) * (float)g->nu;
        const float fv = uniform01(w[1]) * (float)g->nv;
        int iu = (int)fu, iv = (int)fv;
        if (iu > g->nu - 1) iu = g->nu - 1;
        if (iv > g->nv - 1) iv = g->nv - 1;
        const float uu = fu * g->pu_mm - P->hu, vv = fv * g->pv_mm - P->hv;
        float q[3], dq[3];
        for (int a = 0; a < 3; ++a) {
            q[a] = (P->D[a] + uu * P->eu[a]) + vv * P->ev[a];
            dq[a] = q[a] - o[a];
        }
        const double r2 = ((double)dq[0] * dq[0] + (double)dq[1] * dq[1]) + (double)dq[2] * dq[2];
        const double dist = sqrt(r2);
        double lam = (((double)d[0] * dq[0] + (double)d[1] * dq[1]) + (double)d[2] * dq[2]) / dist;
        lam = lam > 1.0 ? 1.0 : (lam < -1.0 ? -1.0 : lam);
        const double cg =
            (((double)P->ax[0] * dq[0] + (double)P->ax[1] * dq[1]) + (double)P->ax[2] * dq[2]) /
            dist;
        float e2;
        const double pdf = pd_pdf(c, proc, m, e, lam, &e2);
        if (proc == MCO_PROC_COMPTON && (c->phys & MCO_PHYS_DOPPLER)) {
            /* the broadened energy towards the point, from the pseudo-particle's
             * own stream */
            rng_t rd;
            rng_init_pseudo(&rd, seed, pid, (uint32_t)n, (uint32_t)i);
            const double alpha = (double)e / MEC2_KEV;
            const double ratio = 1.0 + alpha * (1.0 - lam);
            e2 = (float)((double)e * sample_doppler(&rd, c->pz_scale[m], ratio, 1.0 - lam));
        }
        if (e2 < E_CUT_KEV) continue;       /* such a photon would be killed */
        const double eta = (double)lerp_tab(c->t_eta, c->J, e2);
        double x0 = (((eta * pdf) * cg) * area) / ((TWO_PI_D * r2) * (double)c->split);
        if (c->rr_kev > 0.0 && x0 < c->rr_kev) {
            if ((double)uniform01(w[2]) < x0 / c->rr_kev) {
                x0 = c->rr_kev;
            } else {
                st->pd_killed++;
                continue;
            }
        }
        /* attenuation from the event to the box exit at E' */
        float om[3];
        for (int a = 0; a < 3; ++a) om[a] = (float)((double)dq[a] / dist);
        double tau = 0.0;
        float tin, tout;
        if (box_hit(P, o, om, &tin, &tout)) {
            float mm[MAX_MAT], pint[3];
            size_t v;
            uint32_t steps = 0;
            mat_mu(c, e2, mm);
            if (c->reading == MCO_READING_PLAIN)
                (void)march_plain(c, P, o, om, tin, tout, mm, INFINITY, pint, &v, &steps, &tau);
            else
                (void)march(c, P, o, om, tin, tout, mm, INFINITY, pint, &v, &steps, &tau);
            st->pd_steps += steps;
        }
        const double x = x0 * exp(-tau);
        const int64_t L = (int64_t)llrint(x * 1048576.0);
        scat[(size_t)(iv / (g->nv / g->snv)) * g->snu + (size_t)(iu / (g->nu / g->snu))] += L;
        st->pd_scores++;
    }
}

static void history(const mco_ctx *c, const proj_t *P, uint64_t seed, uint64_t pid,
                    int64_t *prim, int64_t *scat, mco_stats *st, hist_t *h) {
    rng_t r;
    rng_init(&r, seed, pid);
    h->n_int = 0; h->steps = 0; h->end = MCO_END_MISSED; h->first = MCO_FIRST_NONE;
    h->x1[0] = h->x1[1] = h->x1[2] = NAN;
    h->pix = -1;
    st->histories++;
    float e, d[3], p[3], mm[MAX_MAT];
    birth(c, P, &r, &e, d);
    for (int a = 0; a < 3; ++a) p[a] = P->S[a];
    mat_mu(c, e, mm);
    int n_int = 0;     /* scatterings                                  */
    int n_coll = 0;    /* scatterings and null collisions: PD counters */
    for (;;) {
        float tin, tout;
        if (!box_hit(P, p, d, &tin, &tout)) break;
        const double u_tau = (double)rng_u(&r);
        st->flights++;
        float pint[3];
        size_t v;
        uint32_t steps = 0;
        int hit;
        if (c->reading == MCO_READING_PLAIN)
            hit = march_plain(c, P, p, d, tin, tout, mm, -log(u_tau), pint, &v, &steps, NULL);
        else
            hit = march(c, P, p, d, tin, tout, mm, (float)(-log(u_tau)), pint, &v, &steps, NULL);
        h->steps += steps;
        st->steps += steps;
        if (!hit) break;
        for (int a = 0; a < 3; ++a) p[a] = pint[a];
        if (!n_int)
            for (int a = 0; a < 3; ++a) h->x1[a] = pint[a];
        /* interaction type at (material, E): [photo, Rayleigh, Compton] */
        const int m = c->ids[v];
        const size_t o = (size_t)m * c->J;
        float pe = lerp_tab(c->t_pe + o, c->J, e);
        float coh = lerp_tab(c->t_coh + o, c->J, e);
        float inc = lerp_tab(c->t_inc + o, c->J, e);
        float tot = (pe + coh) + inc;
        float x = rng_u(&r) * tot;
        if ((c->g.flags & MCO_NO_SCATTER) || x < pe) {
            st->photo++;
            if (!n_int) h->first = MCO_FIRST_PHOTO;
            h->end = MCO_END_PHOTO;
            h->n_int = (uint16_t)n_int;
            h->e_end = e;
            return;
        }
        float ct = 1.0f, e2 = e;
        int real = 1;
        if (x < pe + coh) {
            ct = sample_rayleigh(&r, e, c->rayl_b[m]);
            e2 = e;
            st->rayleigh++;
            if (!n_int) h->first = MCO_FIRST_RAYLEIGH;
        } else {
            real = compton_collision(c, &r, m, e, &ct, &e2);
            if (real) {
                st->compton++;
                if (!n_int) h->first = MCO_FIRST_COMPTON;
            } else {
                st->null_collisions++;
            }
        }
        double phi = TWO_PI_D * (double)rng_u(&r);
        if (c->estimator != MCO_SCORE_ANALOG && scat)
            pd_event(c, P, seed, pid, n_int, n_coll, p, d, e, m,
                     x < pe + coh ? MCO_PROC_RAYLEIGH : MCO_PROC_COMPTON, scat, st);
        n_coll++;
        if (!real) continue;     /* null collision: the same flight goes on */
        rotate(d, ct, (float)cos(phi), (float)sin(phi));
        n_int++;
        if (e2 < E_CUT_KEV) {
            st->cutoff_kills++;
            h->end = MCO_END_CUTOFF;
            h->n_int = (uint16_t)n_int;
            h->e_end = e2;
            return;
        }
        if (n_int >= MAX_SCATTER) {
            st->cap_hits++;
            h->end = MCO_END_CAP;
            h->n_int = (uint16_t)n_int;
            h->e_end = e2;
            return;
        }
        if (e2 != e) {
            e = e2;
            mat_mu(c, e, mm);
        }
    }
    h->n_int = (uint16_t)n_int;
    h->e_end = e;
    tally(c, P, p, d, e, n_int, prim, scat, st, h);
}

/* every precondition of a projection; also regenerates stale tables */
static int ready(mco_ctx *c, uint64_t n) {
    if (!c->have_phantom || !c->have_geom || !c->have_spec)
        return fail(c, MCO_E_STATE, "phantom, geometry and spectrum must be set");
    size_t nv = (size_t)c->nx * c->ny * c->nz;
    for (size_t i = 0; i < nv; ++i)
        if (c->ids[i] >= c->n_mat) return fail(c, MCO_E_INVALID_ARG, "material id >= n_mat");
    double hx = 0.5 * c->nx * c->h, hy = 0.5 * c->ny * c->h, hz = 0.5 * c->nz * c->h;
    double diag = sqrt(hx * hx + hy * hy + hz * hz);
    if (!(diag < c->g.sod_mm) || !(diag < (double)c->g.sdd_mm - c->g.sod_mm))
        return fail(c, MCO_E_INVALID_ARG, "phantom must lie strictly between source and panel");
    if (2.0 * diag / c->g.step_mm > 4194304.0)
        return fail(c, MCO_E_INVALID_ARG, "step too small for the phantom");
    int rc = build_tables(c);
    if (rc) return rc;
    float emax_eta = 0.0f;
    for (int j = 0; j < c->J; ++j)
        if (c->t_eta[j] > emax_eta) emax_eta = c->t_eta[j];
    if ((long double)n * ((long double)emax_eta * 1048576.0L + 1.0L) >= 9223372036854775807.0L)
        return fail(c, MCO_E_OVERFLOW, "tally could overflow int64");
    return MCO_OK;
}

static void stats_add(mco_stats *a, const mco_stats *b) {
    a->histories += b->histories; a->steps += b->steps; a->flights += b->flights;
    a->photo += b->photo; a->rayleigh += b->rayleigh; a->compton += b->compton;
    a->primary_hits += b->primary_hits; a->scatter_hits += b->scatter_hits;
    a->cutoff_kills += b->cutoff_kills; a->cap_hits += b->cap_hits;
    a->pd_scores += b->pd_scores; a->pd_killed += b->pd_killed; a->pd_steps += b->pd_steps;
    a->null_collisions += b->null_collisions;
}

int mco_project_range(mco_ctx *c, float beta, uint64_t first, uint64_t n, uint64_t seed,
                      int64_t *prim, int64_t *scat) {
    if (!c) return MCO_E_INVALID_ARG;
    if (!prim || !scat) return fail(c, MCO_E_INVALID_ARG, "null image");
    if (!isfinite(beta)) return fail(c, MCO_E_INVALID_ARG, "angle must be finite");
    int rc = ready(c, first + n);
    if (rc) return rc;
    proj_t P;
    proj_setup(c, beta, &P);
    hist_t h;
    for (uint64_t i = 0; i < n; ++i) history(c, &P, seed, first + i, prim, scat, &c->stats, &h);
    return MCO_OK;
}

int mco_project(mco_ctx *c, float beta, uint64_t n, uint64_t seed, int64_t *prim,
                int64_t *scat) {
    if (!c) return MCO_E_INVALID_ARG;
    if (!prim || !scat) return fail(c, MCO_E_INVALID_ARG, "null image");
    if (!c->have_geom) return fail(c, MCO_E_STATE, "geometry not set");
    memset(prim, 0, (size_t)c->g.nu * c->g.nv * sizeof(int64_t));
    memset(scat, 0, (size_t)c->g.snu * c->g.snv * sizeof(int64_t));
    return mco_project_range(c, beta, 0, n, seed, prim, scat);
}

typedef struct {
    const mco_ctx *c;
    const proj_t *P;
    uint64_t first, n, seed;
    int64_t *prim, *scat;
    mco_stats st;
} worker_t;

static void *worker(void *arg) {
    worker_t *w = (worker_t *)arg;
    hist_t h;
    for (uint64_t i = 0; i < w->n; ++i)
        history(w->c, w->P, w->seed, w->first + i, w->prim, w->scat, &w->st, &h);
    return NULL;
}

int mco_project_mt(mco_ctx *c, float beta, uint64_t n, uint64_t seed, int64_t *prim,
                   int64_t *scat, int nt) {
    if (!c) return MCO_E_INVALID_ARG;
    if (!prim || !scat || nt < 1 || nt > 1024) return fail(c, MCO_E_INVALID_ARG, "bad arguments");
    if (!c->have_geom) return fail(c, MCO_E_STATE, "geometry not set");
    int rc = ready(c, n);
    if (rc) return rc;
    proj_t P;
    proj_setup(c, beta, &P);
    size_t np = (size_t)c->g.nu * c->g.nv, ns = (size_t)c->g.snu * c->g.snv;
    worker_t *w = (worker_t *)calloc(nt, sizeof *w);
    pthread_t *th = (pthread_t *)calloc(nt, sizeof *th);
    int64_t *img = (int64_t *)calloc((size_t)nt * (np + ns), sizeof(int64_t));
    if (!w || !th || !img) { free(w); free(th); free(img); return fail(c, MCO_E_OOM, "thread images"); }
    for (int t = 0; t < nt; ++t) {
        uint64_t lo = n * (uint64_t)t / nt, hi = n * (uint64_t)(t + 1) / nt;
        w[t].c = c; w[t].P = &P; w[t].first = lo; w[t].n = hi - lo; w[t].seed = seed;
        w[t].prim = img + (size_t)t * (np + ns);
        w[t].scat = w[t].prim + np;
        pthread_create(&th[t], NULL, worker, &w[t]);
    }
    memset(prim, 0, np * sizeof(int64_t));
    memset(scat, 0, ns * sizeof(int64_t));
    for (int t = 0; t < nt; ++t) {
        pthread_join(th[t], NULL);
        for (size_t i = 0; i < np; ++i) prim[i] += w[t].prim[i];
        for (size_t i = 0; i < ns; ++i) scat[i] += w[t].scat[i];
        stats_add(&c->stats, &w[t].st);
    }
    free(w); free(th); free(img);
    return MCO_OK;
}

int mco_debug_histories(mco_ctx *c, float beta, uint64_t first, uint64_t m, uint64_t seed,
                        uint16_t *n_int, uint32_t *steps, uint8_t *end, uint8_t *first_type) {
    if (!c) return MCO_E_INVALID_ARG;
    if (!isfinite(beta)) return fail(c, MCO_E_INVALID_ARG, "angle must be finite");
    int rc = ready(c, m);
    if (rc) return rc;
    proj_t P;
    proj_setup(c, beta, &P);
    for (uint64_t i = 0; i < m; ++i) {
        hist_t h;
        history(c, &P, seed, first + i, NULL, NULL, &c->stats, &h);
        if (n_int) n_int[i] = h.n_int;
        if (steps) steps[i] = h.steps;
        if (end) end[i] = h.end;
        if (first_type) first_type[i] = h.first;
    }
    return MCO_OK;
}

int mco_set_reading(mco_ctx *c, int reading) {
    if (!c) return MCO_E_INVALID_ARG;
    if (reading != MCO_READING_GRID && reading != MCO_READING_PLAIN)
        return fail(c, MCO_E_INVALID_ARG, "unknown march reading");
    c->reading = reading;
    return MCO_OK;
}

int mco_debug_paths(mco_ctx *c, float beta, uint64_t first, uint64_t m, uint64_t seed,
                    float *x_first, int32_t *pixel, float *e_end) {
    if (!c) return MCO_E_INVALID_ARG;
    if (!isfinite(beta)) return fail(c, MCO_E_INVALID_ARG, "angle must be finite");
    int rc = ready(c, m);
    if (rc) return rc;
    proj_t P;
    proj_setup(c, beta, &P);
    for (uint64_t i = 0; i < m; ++i) {
        hist_t h;
        history(c, &P, seed, first + i, NULL, NULL, &c->stats, &h);
        if (x_first)
            for (int a = 0; a < 3; ++a) x_first[3 * i + a] = h.x1[a];
        if (pixel) pixel[i] = h.pix;
        if (e_end) e_end[i] = h.e_end;
    }
    return MCO_OK;
}

void mco_test_rotate(const float d_in[3], float cos_theta, double phi, float d_out[3]) {
    float d[3] = {d_in[0], d_in[1], d_in[2]};
    rotate(d, cos_theta, (float)cos(phi), (float)sin(phi));
    for (int a = 0; a < 3; ++a) d_out[a] = d[a];
}

int mco_test_sample(mco_ctx *c, int process, int material, float e, uint64_t n, uint64_t seed,
                    float *cos_out, float *e_out) {
    if (!c) return MCO_E_INVALID_ARG;
    if (process == MCO_PROC_SOURCE_ENERGY) {
        if (!c->have_spec || !e_out) return fail(c, MCO_E_STATE, "spectrum not set");
        for (uint64_t i = 0; i < n; ++i) {
            rng_t r;
            rng_init(&r, seed, i);
            e_out[i] = c->e_bin[energy_bin(c, rng_raw(&r))];
        }
        return MCO_OK;
    }
    if (process == MCO_PROC_SOURCE_DIR) {
        if (!c->have_geom || !c->have_phantom || !cos_out)
            return fail(c, MCO_E_STATE, "geometry/phantom not set");
        proj_t P;
        proj_setup(c, 0.0f, &P);
        for (uint64_t i = 0; i < n; ++i) {
            rng_t r;
            rng_init(&r, seed, i);
            (void)rng_raw(&r);
            cos_out[i] = 1.0f - rng_u(&r) * P.omc;
        }
        return MCO_OK;
    }
    if (process != MCO_PROC_RAYLEIGH && process != MCO_PROC_COMPTON)
        return fail(c, MCO_E_INVALID_ARG, "unknown process");
    if (material < 0 || material >= c->n_mat || !(e >= 1.0f && e <= 1000.0f) || !cos_out)
        return fail(c, MCO_E_INVALID_ARG, "bad material/energy");
    for (uint64_t i = 0; i < n; ++i) {
        rng_t r;
        rng_init(&r, seed, i);
        float ct = 2.0f, e2 = e;
        if (process == MCO_PROC_COMPTON)
            (void)compton_collision(c, &r, material, e, &ct, &e2);   /* null: ct stays 2 */
        else
            ct = sample_rayleigh(&r, e, c->rayl_b[material]);
        cos_out[i] = ct;
        if (e_out) e_out[i] = e2;
    }
    return MCO_OK;
}

int mco_get_stats(mco_ctx *c, mco_stats *out) {
    if (!c || !out) return MCO_E_INVALID_ARG;
    *out = c->stats;
    memset(&c->stats, 0, sizeof c->stats);
    return MCO_OK;
}

double mco_tally_scale(void) { return 1.0 / 1048576.0; }

int mco_set_physics(mco_ctx *c, uint32_t flags) {
    if (!c) return MCO_E_INVALID_ARG;
    if (flags & ~(MCO_PHYS_INCOH_SF | MCO_PHYS_DOPPLER))
        return fail(c, MCO_E_INVALID_ARG, "unknown physics flags");
    c->phys = flags;
    return MCO_OK;
}

int mco_set_estimator(mco_ctx *c, int mode, int split, double rr_kev) {
    if (!c) return MCO_E_INVALID_ARG;
    if (mode != MCO_SCORE_ANALOG && mode != MCO_SCORE_POINT && mode != MCO_SCORE_POINT_MIXED)
        return fail(c, MCO_E_INVALID_ARG, "unknown estimator");
    if (split < 1 || split > 1024) return fail(c, MCO_E_INVALID_ARG, "split must be 1..1024");
    if (!(rr_kev >= 0.0) || !isfinite(rr_kev))
        return fail(c, MCO_E_INVALID_ARG, "roulette threshold must be finite and >= 0");
    c->estimator = mode;
    c->split = split;
    c->rr_kev = rr_kev;
    return MCO_OK;
}

int mco_pd_pdf(mco_ctx *c, int process, int material, float e_kev, double lambda, double *pdf,
               float *e_out) {
    if (!c || !pdf) return MCO_E_INVALID_ARG;
    if (process != MCO_PROC_RAYLEIGH && process != MCO_PROC_COMPTON)
        return fail(c, MCO_E_INVALID_ARG, "process must be Rayleigh or Compton");
    if (material < 0 || material >= c->n_mat || !(e_kev >= 1.0f && e_kev <= 1000.0f) ||
        !(lambda >= -1.0 && lambda <= 1.0))
        return fail(c, MCO_E_INVALID_ARG, "bad material, energy or cosine");
    float e2;
    *pdf = pd_pdf(c, process, material, e_kev, lambda, &e2);
    if (e_out) *e_out = e2;
    return MCO_OK;
}

int mco_pd_score_event(mco_ctx *c, float beta, uint64_t seed, uint64_t pid, int n_prior,
                       const float o[3], const float d[3], float e_kev, int material,
                       int process, int64_t *scatter) {
    if (!c || !o || !d || !scatter) return MCO_E_INVALID_ARG;
    if (process != MCO_PROC_RAYLEIGH && process != MCO_PROC_COMPTON)
        return fail(c, MCO_E_INVALID_ARG, "process must be Rayleigh or Compton");
    if (material < 0 || material >= c->n_mat || !(e_kev >= 1.0f && e_kev <= 1000.0f) ||
        n_prior < 0)
        return fail(c, MCO_E_INVALID_ARG, "bad material, energy or event index");
    int rc = ready(c, 1);
    if (rc) return rc;
    proj_t P;
    proj_setup(c, beta, &P);
    pd_event(c, &P, seed, pid, n_prior, n_prior, o, d, e_kev, material, process, scatter,
             &c->stats);
    return MCO_OK;
}

/* ------------------------------------------------------------ deterministic primary
 * Eq. (7): the primary intensity as an integral over the spectrum of
 * eta(E) exp(-mu(E) L) along the ray from the source to the detector, here for
 * each pixel as the expectation of the analog primary tally per emitted
 * photon: the spectrum is the bins' draw probabilities (thresholds of the
 * sampler), the source's photons per steradian are 1 / Omega_cone (the cone
 * circumscribing the panel, with the sampler's fp32 1 - cos(theta_max)), and
 * the pixel is integrated over sub x sub sub-pixels by the midpoint rule with
 * d(Omega) = cos(gamma) dA / R^2.  Each sub-pixel ray from the source is
 * marched with the transport's fixed-step rule (nominal step centres, last
 * step clipped) and collects rho * length per material, Lambda_m (fp64), so
 * that mu(E) L = sum_m Lambda_m mu_m(E) / rho with the transport's tables.
 * Where eq. (7) writes 1/d^2, the pixel's solid angle cos(gamma) dA / R^2
 * stands (the paper leaves the pixel area and obliquity out). */
static void ray_lambda(const mco_ctx *c, const proj_t *P, const float d[3], double *lam) {
    for (int m = 0; m < c->n_mat; ++m) lam[m] = 0.0;
    float tin, tout;
    if (!box_hit(P, P->S, d, &tin, &tout)) return;
    const float dl = c->g.step_mm;
    float pin[3], c0[3], G[3], q[3];
    for (int a = 0; a < 3; ++a) pin[a] = P->S[a] + d[a] * tin;
    const float L = tout - tin;
    for (int a = 0; a < 3; ++a) {
        G[a] = (d[a] * P->inv_h) * dl;
        c0[a] = (pin[a] - P->lo[a]) * P->inv_h + 0.5f * G[a];
    }
    for (uint32_t k = 0;; ++k) {
        const float a0 = (float)k * dl;
        if (!(a0 < L)) return;
        for (int a = 0; a < 3; ++a)
            q[a] = (k & 3u) == 0u ? c0[a] + (float)k * G[a] : q[a] + G[a];
        int ix = (int)q[0], iy = (int)q[1], iz = (int)q[2];
        ix = ix < 0 ? 0 : (ix > c->nx - 1 ? c->nx - 1 : ix);
        iy = iy < 0 ? 0 : (iy > c->ny - 1 ? c->ny - 1 : iy);
        iz = iz < 0 ? 0 : (iz > c->nz - 1 ? c->nz - 1 : iz);
        const size_t v = ((size_t)iz * c->ny + iy) * c->nx + ix;
        const double len = (float)(k + 1u) * dl < L ? (double)dl : (double)(L - a0);
        lam[c->ids[v]] += (double)c->rho[v] * len;
    }
}

int mco_primary_expected(mco_ctx *c, float beta, int sub, double *out) {
    if (!c || !out) return MCO_E_INVALID_ARG;
    if (sub < 1 || sub > 64) return fail(c, MCO_E_INVALID_ARG, "sub must be 1..64");
    if (!isfinite(beta)) return fail(c, MCO_E_INVALID_ARG, "angle must be finite");
    int rc = ready(c, 1);
    if (rc) return rc;
    proj_t P;
    proj_setup(c, beta, &P);
    const mco_geometry *g = &c->g;
    /* per bin: draw probability times eta, and mu per unit density per material */
    double *wk = (double *)malloc((size_t)c->n_bins * sizeof(double));
    float *mk = (float *)malloc((size_t)c->n_bins * c->n_mat * sizeof(float));
    if (!wk || !mk) { free(wk); free(mk); return fail(c, MCO_E_OOM, "bin tables"); }
    for (int k = 0; k < c->n_bins; ++k) {
        const uint64_t lo = k ? c->thr[k - 1] : 0;
        wk[k] = (double)(c->thr[k] - lo) / 4294967296.0 *
                (double)lerp_tab(c->t_eta, c->J, c->e_bin[k]);
        mat_mu(c, c->e_bin[k], mk + (size_t)k * c->n_mat);
    }
    const double om_cone = TWO_PI_D * (double)P.omc;
    const double da = (double)g->pu_mm * (double)g->pv_mm / ((double)sub * sub);
    double lam[MAX_MAT];
    for (int iv = 0; iv < g->nv; ++iv)
        for (int iu = 0; iu < g->nu; ++iu) {
            double acc = 0.0;
            for (int b = 0; b < sub; ++b)
                for (int a = 0; a < sub; ++a) {
                    const double u = -(double)P.hu + ((double)iu + (a + 0.5) / sub) * g->pu_mm;
                    const double v = -(double)P.hv + ((double)iv + (b + 0.5) / sub) * g->pv_mm;
                    double w[3], r2 = 0.0, ax = 0.0;
                    for (int k = 0; k < 3; ++k) {
                        w[k] = ((double)P.D[k] + u * P.eu[k] + v * P.ev[k]) - (double)P.S[k];
                        r2 += w[k] * w[k];
                    }
                    const double R = sqrt(r2);
                    float d[3];
                    for (int k = 0; k < 3; ++k) {
                        d[k] = (float)(w[k] / R);
                        ax += w[k] / R * (double)P.ax[k];
                    }
                    ray_lambda(c, &P, d, lam);
                    double e_sum = 0.0;
                    for (int k = 0; k < c->n_bins; ++k) {
                        double tau = 0.0;
                        for (int m = 0; m < c->n_mat; ++m)
                            tau += lam[m] * (double)mk[(size_t)k * c->n_mat + m];
                        e_sum += wk[k] * exp(-tau);
                    }
                    acc += e_sum * (ax * da / r2);
                }
            out[(size_t)iv * g->nu + iu] = acc / om_cone;
        }
    free(wk);
    free(mk);
    return MCO_OK;
}

/* ------------------------------------------------------------ angular interpolation
 * Section II-C-3: of a scan's projections only every other one's scatter is
 * simulated; the ones between are the linear interpolation of their two
 * neighbours in angle.  sim[n_sim][n_pix] are the simulated maps at angles
 * beta_0, beta_2, ... of a full circle; full[2 n_sim][n_pix] receives them at
 * the even positions and, at odd position 2i+1, 0.5 (sim[i] + sim[i+1]) with
 * sim[n_sim] = sim[0] (the circle closes), in fp32. */
int mco_interp_angles(const float *sim, int n_sim, int64_t n_pix, float *full) {
    if (!sim || !full || n_sim < 1 || n_pix < 1) return MCO_E_INVALID_ARG;
    for (int i = 0; i < n_sim; ++i) {
        const float *a = sim + (size_t)i * n_pix;
        const float *b = sim + (size_t)((i + 1) % n_sim) * n_pix;
        float *e = full + (size_t)(2 * i) * n_pix, *o = e + n_pix;
        for (int64_t p = 0; p < n_pix; ++p) {
            e[p] = a[p];
            o[p] = 0.5f * (a[p] + b[p]);
        }
    }
    return MCO_OK;
}
