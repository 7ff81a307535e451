/*
 * mco.h -- sequential CPU oracle of the analog Monte Carlo photon-transport
 * forward projection (Alsaffar, Kiess, Sun, Simon, "Computational Scatter
 * Correction for High-Resolution Flat-Panel CT Based on a Fast Monte Carlo
 * Photon Transport Model", arXiv 2201.13191).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the reference the GPU library is
 * compared against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares
 * no code, header, table generator or constant generator with the GPU
 * library: every formula below is written out here from the paper and from
 * the published definitions it relies on.
 *
 * What it computes (paper, section II-A "The Proposed MC Photon Transport
 * Model"): photons leave a cone-beam point source with energies drawn from a
 * binned spectrum (the polychromatic source of eq. (6)/(7) as energy bins),
 * are ray-marched with a fixed, controllable step (section II-C-2
 * "Controllable Step Size of the Ray Tracing") through a voxelised
 * material/density object, and undergo photoelectric absorption, Rayleigh
 * scattering (eq. (2) with a form factor) or Compton scattering (eq. (1),
 * Klein-Nishina with S = 1, sampled by Kahn's method) between 1 keV and
 * 1 MeV.  Photons reaching the flat panel are tallied as primary (no
 * interaction, the quantity of eq. (7)) or scatter (>= 1 interaction, the
 * quantity of eq. (6)), weighted by the detector energy response eta(E).
 *
 * The default scoring is analog (each detected photon scores once in the
 * pixel it crosses); the paper's point-detector estimator of eq. (3)-(5),
 * with splitting and Russian roulette (section II-C-1), is a selectable
 * variance-reduced estimator of the same expectation (mco_set_estimator).
 *
 * Because the algorithm is stochastic, exactness is defined per seed: the
 * random draw order, the floating-point precision of every operation and the
 * fixed-point tally are fully specified, so for one seed there is exactly one
 * correct image.  Tallies are int64 fixed point (keV * 2^20), so summation
 * order never matters.
 *
 * All functions return 0 on success and a negative status on error.
 */
#ifndef MCO_H
#define MCO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MCO_OK = 0,
    MCO_E_INVALID_ARG = -1,
    MCO_E_STATE = -2,
    MCO_E_OOM = -3,
    MCO_E_OVERFLOW = -4
};

/* readings of the fixed-step march (mco_set_reading) */
enum {
    MCO_READING_GRID = 0,   /* default: nominal step centres, optical depth on the
                               2^-32 grid (the transport's specification) */
    MCO_READING_PLAIN = 1   /* true midpoints of the clipped steps, fp64 depth */
};

/* scatter estimators (mco_set_estimator) */
enum {
    MCO_SCORE_ANALOG = 0,   /* each scattered photon that crosses the panel scores
                               in the pixel it crosses */
    MCO_SCORE_POINT = 1,    /* point-detector scores of eq. (3)-(5) at every
                               scattering, with splitting and Russian roulette */
    MCO_SCORE_POINT_MIXED = 2  /* eq. (3)/(4) at Compton events; Rayleigh
                                  pseudo-particles follow the Rayleigh law and
                                  score where they cross the panel */
};

/* geometry flags */
#define MCO_NO_SCATTER 1u   /* every interaction absorbs (Beer-Lambert check) */

/* binding effects (mco_set_physics); none by default (free electrons at rest:
 * Klein-Nishina exactly) */
#define MCO_PHYS_INCOH_SF 1u  /* S(x,Z) of eq. (1) by rejection (null collisions) */
#define MCO_PHYS_DOPPLER 2u   /* Doppler broadening of the Compton energy        */

/* processes for mco_test_sample */
enum {
    MCO_PROC_SOURCE_ENERGY = 0, /* birth energy from the spectrum        */
    MCO_PROC_RAYLEIGH = 1,      /* Rayleigh polar angle                  */
    MCO_PROC_COMPTON = 2,       /* one Compton collision: polar cosine and
                                   energy, cosine 2 for a null collision   */
    MCO_PROC_SOURCE_DIR = 3     /* cosine of the birth polar angle       */
};

/* end-of-history codes written by mco_debug_histories */
enum {
    MCO_END_PRIMARY = 0,      /* reached a pixel without interacting   */
    MCO_END_SCATTER = 1,      /* reached a pixel after >= 1 scattering */
    MCO_END_MISSED = 2,       /* left without hitting the panel        */
    MCO_END_PHOTO = 3,        /* photoelectric absorption              */
    MCO_END_CUTOFF = 4,       /* energy fell below 1 keV               */
    MCO_END_CAP = 5           /* interaction safety cap reached        */
};

/* first-interaction codes written by mco_debug_histories */
enum {
    MCO_FIRST_NONE = 0,
    MCO_FIRST_PHOTO = 1,
    MCO_FIRST_RAYLEIGH = 2,
    MCO_FIRST_COMPTON = 3
};

typedef struct mco_material {
    float z_eff;       /* effective atomic number                     */
    float z_over_a;    /* electrons per nucleon, Z/A [mol/g]          */
    float rho_default; /* nominal density [g/cm^3] (informational)    */
    char name[16];
} mco_material;

typedef struct mco_geometry {
    float sod_mm;      /* source to rotation axis                     */
    float sdd_mm;      /* source to detector plane                    */
    int32_t nu, nv;    /* detector pixels along u (horizontal), v (z) */
    float pu_mm, pv_mm;
    int32_t snu, snv;  /* scatter tally grid; nu % snu == nv % snv == 0 */
    float step_mm;     /* fixed ray-march step                         */
    uint32_t flags;    /* MCO_NO_SCATTER                               */
} mco_geometry;

/* counters accumulated over every history an oracle call simulates */
typedef struct mco_stats {
    uint64_t histories;
    uint64_t steps;        /* voxel lookups of the fixed-step march   */
    uint64_t flights;      /* march segments started                  */
    uint64_t photo, rayleigh, compton;
    uint64_t primary_hits, scatter_hits;
    uint64_t cutoff_kills, cap_hits;
    uint64_t pd_scores;    /* point-detector pseudo-particles scored  */
    uint64_t pd_killed;    /* ... removed by Russian roulette         */
    uint64_t pd_steps;     /* march steps of their attenuation chords */
    uint64_t null_collisions; /* Compton collisions rejected by S/Z     */
} mco_stats;

typedef struct mco_ctx mco_ctx;

int  mco_create(mco_ctx **out);
void mco_destroy(mco_ctx *ctx);
const char *mco_last_error(const mco_ctx *ctx);

/* Material set; ids in the phantom index it.  The default set is
 * 0 air, 1 water, 2 aluminium, 3 bone-like calcium mix, 4 iron. */
int mco_set_materials(mco_ctx *ctx, const mco_material *m, int n_mat);
/* x-fastest arrays [nz][ny][nx], copied.  Voxel cube edge voxel_mm. */
int mco_load_phantom(mco_ctx *ctx, const uint8_t *ids, const float *rho_gcc,
                     int nx, int ny, int nz, float voxel_mm);
int mco_set_geometry(mco_ctx *ctx, const mco_geometry *g);
/* energy bins (keV, bin centre) and non-negative weights */
int mco_set_spectrum(mco_ctx *ctx, const float *e_kev, const float *w, int n_bins);
/* detector response on the 1 keV grid E_j = 1 + j; default eta(E) = E */
int mco_set_detector_response(mco_ctx *ctx, const float *eta, int n);

/* Photons [first, first+n) of one projection; ADDS Q43.20 tallies into
 * primary[nv*nu] and scatter[snv*snu] (does not clear them). */
int mco_project_range(mco_ctx *ctx, float angle_rad, uint64_t first, uint64_t n,
                      uint64_t seed, int64_t *primary, int64_t *scatter);
/* Clears the images, then simulates photons [0, n). */
int mco_project(mco_ctx *ctx, float angle_rad, uint64_t n, uint64_t seed,
                int64_t *primary, int64_t *scatter);
/* Same result as mco_project, photon ranges spread over n_threads POSIX
 * threads with private images summed at the end (int64: bitwise equal). */
int mco_project_mt(mco_ctx *ctx, float angle_rad, uint64_t n, uint64_t seed,
                   int64_t *primary, int64_t *scatter, int n_threads);

/* Per-history record for photons [first, first+m): scatterings, march
 * steps, end code and first-interaction code. Any pointer may be NULL. */
int mco_debug_histories(mco_ctx *ctx, float angle_rad, uint64_t first, uint64_t m,
                        uint64_t seed, uint16_t *n_int, uint32_t *steps,
                        uint8_t *end_code, uint8_t *first_type);

/* Same histories, other per-history facts for photons [first, first+m):
 * x_first[3*i..] the first interaction point (NaN if none), pixel[i] the
 * panel pixel iv*nu+iu the photon crossed (-1 if none), e_end[i] the energy
 * when the history ended.  Any pointer may be NULL. */
int mco_debug_paths(mco_ctx *ctx, float angle_rad, uint64_t first, uint64_t m, uint64_t seed,
                    float *x_first, int32_t *pixel, float *e_end);

/* Scatter estimator: MCO_SCORE_ANALOG (default), MCO_SCORE_POINT, the
 * point-detector estimator of eq. (3)-(5) (section II-A) with `split`
 * pseudo-particles per scattering event (1..1024) and Russian roulette below
 * rr_kev (keV; 0 turns it off) (section II-C-1), or MCO_SCORE_POINT_MIXED: the
 * same at Compton events, while a Rayleigh event's pseudo-particles draw their
 * directions from the Rayleigh law and score eta(E) / split exp(-tau) where
 * they cross the panel (same expectation, no heavy tail from the form
 * factor's forward peak).  With either the scatter image holds the
 * estimator's scores (same expectation as the analog image); the primary
 * image and every photon's history are unchanged. */
int mco_set_estimator(mco_ctx *ctx, int mode, int split, double rr_kev);
/* binding effects: MCO_PHYS_INCOH_SF | MCO_PHYS_DOPPLER (see mco.c) */
int mco_set_physics(mco_ctx *ctx, uint32_t flags);

/* The point-detector scorer's angular pdf per unit scattering cosine
 * (eq. (4) for MCO_PROC_COMPTON, eq. (5) for MCO_PROC_RAYLEIGH) at energy
 * e_kev in `material`, and the energy scattered into that cosine. */
int mco_pd_pdf(mco_ctx *ctx, int process, int material, float e_kev, double lambda,
               double *pdf, float *e_out);

/* Adds to scatter[snv*snu] the point-detector scores of one scattering
 * event: photon pid of `seed`, its n_prior-th collision (from 0: its
 * scatterings, plus its null collisions under MCO_PHYS_INCOH_SF), at point
 * o with incoming direction d and energy e_kev in `material`, by `process`
 * (the estimator's split and roulette settings apply). */
int mco_pd_score_event(mco_ctx *ctx, float angle_rad, uint64_t seed, uint64_t pid,
                       int n_prior, const float o[3], const float d[3], float e_kev,
                       int material, int process, int64_t *scatter);

/* Eq. (7) as the expectation of the primary image: out[nv*nu] (fp64) the
 * expected primary tally in keV per photon emitted into the cone, each pixel
 * integrated over sub x sub sub-pixel rays (1 .. 64) marched with the
 * transport's step rule. */
int mco_primary_expected(mco_ctx *ctx, float angle_rad, int sub, double *out);

/* Angular interpolation of scatter maps (section II-C-3): sim[n_sim][n_pix]
 * simulated at every other angle of a circle -> full[2 n_sim][n_pix], odd
 * entries the mean of their two neighbours (the last wraps to the first). */
int mco_interp_angles(const float *sim, int n_sim, int64_t n_pix, float *full);

/* Which reading of the fixed-step march the transport follows. */
int mco_set_reading(mco_ctx *ctx, int reading);

/* The direction update after a scattering: d_in rotated by polar cosine
 * cos_theta and azimuth phi (cos/sin taken in fp64, rounded to fp32). */
void mco_test_rotate(const float d_in[3], float cos_theta, double phi, float d_out[3]);

/* Draws n independent samples of one process (photon ids 0..n-1 of the
 * given seed).  SOURCE_ENERGY: e_out = energy.  SOURCE_DIR: cos_out =
 * cosine to the central axis.  RAYLEIGH/COMPTON at energy e_kev in material
 * `material`: cos_out = cos(theta), e_out = outgoing energy. */
int mco_test_sample(mco_ctx *ctx, int process, int material, float e_kev,
                    uint64_t n, uint64_t seed, float *cos_out, float *e_out);

/* Trace one given ray (start p, direction d) in vacuum to the panel of
 * projection angle_rad: writes the pixel (or -1,-1 on a miss). */
int mco_detector_pixel(mco_ctx *ctx, float angle_rad, const float p[3],
                       const float d[3], int *iu, int *iv);

/* Tables as used by the transport: fp32 mu/rho [cm^2/g] per material on the
 * grid E_j = 1 + j keV, j < J.  Arrays are [n_mat][J]; pass NULL to query J. */
int mco_get_tables(mco_ctx *ctx, int *J, float *pe, float *coh, float *inc,
                   float *eta);
/* Unrounded cross sections (extended precision) of one material at one
 * energy: out = {mu_pe/rho, mu_coh/rho, mu_incoh/rho} [cm^2/g]. */
int mco_cross_sections(double z_eff, double z_over_a, double e_kev, double out[3]);
/* Klein-Nishina total cross section per electron [cm^2] at energy e_kev. */
double mco_sigma_kn(double e_kev);

int mco_get_stats(mco_ctx *ctx, mco_stats *out);   /* read and reset */

/* Philox4x32-10 block and the uniform map, exported for pins. */
void mco_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void mco_uniform_batch(const uint32_t *x, uint64_t n, float *out);

double mco_tally_scale(void);  /* keV per least significant bit: 2^-20 */

#ifdef __cplusplus
}
#endif
#endif
