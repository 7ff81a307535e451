/*
 * mcx.h -- C ABI of libmcx, the MI355X (gfx950) Monte Carlo photon-transport
 * forward projector for flat-panel cone-beam CT scatter estimation
 * (Alsaffar, Kiess, Sun, Simon, arXiv 2201.13191).
 *
 * The library estimates, for one projection angle of a circular cone-beam
 * scan, the primary image Ip (photons reaching the panel without interacting,
 * the quantity of eq. (7)) and the scatter image Is (photons reaching it after
 * one or more Compton / Rayleigh events, the quantity of eq. (6)), by analog
 * Monte Carlo transport (section II-A): cone-beam point source, binned
 * polychromatic spectrum (energy bins, section II-A below eq. (7)),
 * fixed-step ray march through a voxel object (section II-C-2), photoelectric
 * absorption, Rayleigh scattering (eq. (2)), Compton scattering (eq. (1) with
 * S = 1, sampled by Kahn's method), 1 keV .. 1 MeV.
 *
 * Conventions
 *   - Every function returns an mc_status: 0 on success, < 0 on error; the
 *     context keeps a message for mc_last_error.  No C++ exception crosses
 *     the ABI.
 *   - A context is bound to one HIP device and is not thread-safe: use one
 *     context per host thread.
 *   - Host input pointers are only read during the call (data is copied).
 *     Output buffers are owned by the caller.
 *   - "_async" functions take device pointers and a hipStream_t passed as
 *     void* (NULL = the legacy default stream) and return once the work is
 *     queued; the buffers must stay valid until the stream reaches it.
 *   - Setters (materials, phantom, geometry, spectrum, response) synchronise
 *     the device before replacing device-side state.
 *   - Tallies are signed 64-bit fixed point, Q43.20: one unit is 2^-20 keV of
 *     detector response (mc_tally_scale()).  Integer addition is exact, so an
 *     image does not depend on the order photons are processed: one seed gives
 *     one bitwise result, on any launch configuration.
 *
 * Geometry (reading of section II-A; the paper gives the scanner parameters
 * but no frame): rotation axis z; at angle b the source sits at
 * sod*(cos b, sin b, 0), the panel is perpendicular to the central ray at
 * distance sdd, u runs along (-sin b, cos b, 0) and v along +z; pixel (iu, iv)
 * covers u in [-nu*pu/2 + iu*pu, +pu), v likewise; images are [nv][nu],
 * iu fastest.  The phantom is centred on the origin, x fastest ([nz][ny][nx]).
 * Outside the phantom box is vacuum.
 */
#ifndef MCX_H
#define MCX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mc_status;

#define MC_OK 0
#define MC_E_INVALID_ARG (-1) /* argument out of range / null pointer           */
#define MC_E_STATE (-2)       /* phantom, geometry or spectrum not set         */
#define MC_E_OOM (-3)         /* device or host allocation failed               */
#define MC_E_OVERFLOW (-4)    /* n_photons * max eta * 2^20 could reach 2^63     */
#define MC_E_DEVICE (-6)      /* HIP runtime error (message has its text)       */
#define MC_E_CANCELLED (-7)   /* mc_cancel was on when a blocking call ended     */

/* mc_geometry.flags */
#define MC_NO_SCATTER 1u      /* every interaction absorbs: pure attenuation    */

/* processes of mc_test_sample */
#define MC_PROC_SOURCE_ENERGY 0
#define MC_PROC_RAYLEIGH 1
#define MC_PROC_COMPTON 2
#define MC_PROC_SOURCE_DIR 3

/* end codes of mc_debug_histories */
#define MC_END_PRIMARY 0
#define MC_END_SCATTER 1
#define MC_END_MISSED 2
#define MC_END_PHOTO 3
#define MC_END_CUTOFF 4
#define MC_END_CAP 5

typedef struct mc_ctx mc_ctx;

/* Material of the voxel object: effective Z (photoelectric Z^3 scaling and the
 * Rayleigh form factor's screening radius) and electrons per nucleon Z/A. */
typedef struct mc_material {
    float z_eff;       /* 1 .. 100                                   */
    float z_over_a;    /* (0, 1.01]                                  */
    float rho_default; /* nominal density, g/cm^3 (informational)    */
    char name[16];
} mc_material;

/* Scanner geometry and transport knobs (scan parameters of section III;
 * step size of section II-C-2). */
typedef struct mc_geometry {
    float sod_mm;      /* source - rotation axis distance, > 0            */
    float sdd_mm;      /* source - panel distance, > sod                  */
    int32_t nu, nv;    /* panel pixels, 1 .. 16384                        */
    float pu_mm, pv_mm;
    int32_t snu, snv;  /* scatter grid; nu % snu == 0 and nv % snv == 0   */
    float step_mm;     /* fixed ray-march step, > 0                        */
    uint32_t flags;    /* MC_NO_SCATTER                                    */
} mc_geometry;

/* Counters accumulated by projections run while statistics are enabled. */
typedef struct mc_stats {
    uint64_t histories;
    uint64_t steps;        /* fixed steps of the march                   */
    uint64_t flights;
    uint64_t photo, rayleigh, compton;
    uint64_t primary_hits, scatter_hits;
    uint64_t cutoff_kills, cap_hits;
    uint64_t skipped_steps;  /* steps (included in `steps`) taken as runs through
                                uniform regions without a voxel lookup each     */
    uint64_t pd_scores;      /* point-detector pseudo-particles scored            */
    uint64_t pd_killed;      /* ... removed by Russian roulette                   */
    uint64_t pd_steps;       /* march steps of their chords (included in `steps`) */
    uint64_t null_collisions; /* Compton collisions rejected by S/Z (MC_PHYS_INCOH_SF) */
} mc_stats;

/* Create a context on HIP device `device`; allocates only small buffers.
 * device = -1 creates a host-only context: setters validate their arguments
 * and mc_get_tables works, anything that needs the GPU returns MC_E_STATE. */
mc_status mc_create(mc_ctx **out, int device);
void mc_destroy(mc_ctx *ctx);
/* Message of the last failing call on this context (never NULL). */
const char *mc_last_error(const mc_ctx *ctx);

/* Replace the material set (1 .. 16 entries).  The default set is
 * 0 air, 1 water, 2 aluminium, 3 bone-like calcium mix, 4 iron.
 * Cross-section tables are regenerated at the next projection. */
mc_status mc_set_materials(mc_ctx *ctx, const mc_material *m, int n_mat);

/* Voxel object (section II-A, voxelised object): ids[nz][ny][nx] material
 * index, rho_gcc[nz][ny][nx] density g/cm^3 (finite, 0 .. 1000), cube voxel
 * of edge voxel_mm.  nx*ny*nz < 2^31.  Copied to the device. */
mc_status mc_load_phantom(mc_ctx *ctx, const uint8_t *ids, const float *rho_gcc, int nx,
                          int ny, int nz, float voxel_mm);

mc_status mc_set_geometry(mc_ctx *ctx, const mc_geometry *g);

/* Polychromatic source as energy bins (the N bins of eq. (6)): bin energies
 * e_keV in [1, 1000] and weights w >= 0 with a positive sum.  A photon's
 * energy is the energy of a bin drawn with probability w_k / sum(w). */
mc_status mc_set_spectrum(mc_ctx *ctx, const float *e_keV, const float *w, int n_bins);

/* A bremsstrahlung spectrum for mc_set_spectrum (host only, no context): bins
 * [lo, lo + bin_keV) for lo = 1, 1 + bin_keV, ... < kvp, with centres
 * lo + bin_keV/2 in out_e and Kramers' weights (kvp - E)/E attenuated by al_mm
 * of aluminium in out_w (0 for a centre at or above kvp).  The aluminium
 * attenuation is a two-term fit, mu/rho = 26583/E^3 + 0.1434 cm^2/g at 2.699
 * g/cm^3: it shapes a synthetic input, it is not a cross-section table of the
 * transport (the paper's spectrum is simulated from its X-ray tube, section
 * II-D-1; this helper stands in for it with a textbook shape).
 * *n_bins receives the number of bins; with out_e and out_w both NULL only
 * that is computed, else both must hold capacity >= *n_bins floats.
 * 1 < kvp <= 1000, al_mm >= 0, bin_keV > 0. */
mc_status mc_make_kramers(double kvp, double al_mm, double bin_keV, float *out_e, float *out_w,
                          int capacity, int *n_bins);

/* Detector energy response eta(E) (eq. (3)/(7)) on the 1 keV grid
 * E_j = 1 + j keV, n >= 1 values (the last one repeats beyond n).  Default
 * eta(E) = E (energy integrating).  eta = 1 counts photons. */
mc_status mc_set_detector_response(mc_ctx *ctx, const float *eta, int n);

/* Scatter estimator (section II-A, eq. (3)-(5); section II-C-1).
 * MC_SCORE_ANALOG (default): a scattered photon that crosses the panel scores
 * eta(E) in the pixel it crosses.  MC_SCORE_POINT: the paper's point-detector
 * estimator -- at every Compton or Rayleigh event, `split` pseudo-particles
 * (1 .. 1024) each pick a uniform point on the panel (its random pixel) and
 * score eta(E') p(lambda) cos(gamma) A / (2 pi R^2 split) exp(-tau): p the
 * event's angular law per unit cosine (eq. (4) Klein-Nishina, eq. (5)
 * Rayleigh with the form factor), lambda the cosine between the photon's
 * direction and the direction to the point, R the distance, gamma that
 * direction's angle to the panel normal, A the panel area, E' the energy
 * scattered towards the point, tau the optical depth at E' from the event to
 * the object's exit, marched with the transport's step rule.  Scores below
 * rr_kev (keV; 0 turns roulette off) survive with probability score / rr_kev
 * and then score rr_kev.  The scatter image has the analog image's
 * expectation with lower variance; the primary image and every photon's
 * history are unchanged (pseudo-particles draw from their own Philox
 * counters).  Applies to mc_project, mc_project_async and
 * mc_project_range_async; mc_project_batch needs MC_SCORE_ANALOG (else
 * MC_E_STATE).  Invalid mode, split or threshold: MC_E_INVALID_ARG. */
#define MC_SCORE_ANALOG 0
#define MC_SCORE_POINT 1
/* MC_SCORE_POINT_MIXED: as MC_SCORE_POINT at Compton events; a Rayleigh
 * event's pseudo-particles draw their directions from the Rayleigh law (their
 * own Philox stream, counter (photon id, n, (i + 1) * 2^12 + block)) and score
 * eta(E) / split * exp(-tau) where that line crosses the panel.  Same
 * expectation; the form factor's forward peak gives eq. (5)'s random-point
 * scores a heavy tail that this avoids. */
#define MC_SCORE_POINT_MIXED 2
mc_status mc_set_estimator(mc_ctx *ctx, int mode, int split, double rr_kev);

/* Binding effects of eq. (1) and section II-A, off by default (free electrons
 * at rest: Klein-Nishina exactly).  The paper takes S(x,Z) and the Compton
 * profiles from tabulated atomic data; here both come from one parametric
 * orbital model: every electron of a material in a 1s-like orbital of the
 * Rayleigh form factor's screening radius r_Z = 0.885 a0 Z^(-1/3), so
 * S(x,Z)/Z = 1 - (1 + b x^2)^-4 (b, x as for the form factor) and the
 * profile J(p_z) ~ (1 + (p_z/p0)^2)^-3 with p0 = hbar / r_Z.
 * MC_PHYS_INCOH_SF: a Compton collision is accepted with probability S/Z; a
 * rejected one is a null collision that leaves the photon unchanged (the
 * tables keep the Klein-Nishina cross section, so the effective cross
 * section and the angular law are exact).  MC_PHYS_DOPPLER: the scattered
 * energy is broadened by a p_z drawn from J (impulse approximation).  The
 * point-detector scores include S/Z and broadened energies.  Applies to
 * every transport entry point including batches; unknown bits:
 * MC_E_INVALID_ARG. */
#define MC_PHYS_INCOH_SF 1u
#define MC_PHYS_DOPPLER 2u
mc_status mc_set_physics(mc_ctx *ctx, uint32_t flags);

/* Eq. (7), the primary image without Monte Carlo: d_out[nv*nu] (device fp32)
 * receives the expected primary tally per photon emitted into the cone, in
 * keV (the analog primary image of n photons has expectation n * 2^20 times
 * this in Q43.20 units).  Each pixel is integrated over sub x sub sub-pixel
 * rays from the source (1 .. 64; midpoint rule, d(Omega) = cos(gamma) dA / R^2
 * over the source cone's solid angle), each ray marched with the transport's
 * fixed-step rule; the spectrum enters as the sampler's bin probabilities
 * times eta(E), attenuation as exp(-sum_m mu_m(E) / rho * (rho * length)_m).
 * The paper's 1/d^2 is this solid angle (its pixel area and obliquity left
 * out).  Stream-ordered; one thread per pixel. */
mc_status mc_primary_expected_async(mc_ctx *ctx, float angle_rad, int sub, float *d_out,
                                    void *stream);

/* Section II-C-3's inter-projection interpolation: scatter maps simulated at
 * every other angle of a full circle, d_sim[n_sim][n_pix] (device fp32) ->
 * d_full[2 n_sim][n_pix]: entry 2i is map i, entry 2i+1 the mean of maps i
 * and i+1 (map n_sim is map 0).  Stream-ordered. */
mc_status mc_interp_angles_async(mc_ctx *ctx, const float *d_sim, int n_sim, uint64_t n_pix,
                                 float *d_full, void *stream);

/* ---- the iterative scatter correction's reconstruction side (section II-E,
 * its flowchart and eq. (8)).  Stream-ordered kernels on device buffers. */

/* a[i] = -ln(I[i] / I0[i mod n0]) (fp32; I below 1e-30 taken as 1e-30): line
 * integrals of n intensities, I0 the flat field of one projection (n0 pixels). */
mc_status mc_line_integrals_async(mc_ctx *ctx, const float *d_I, uint64_t n, const float *d_I0,
                                  uint64_t n0, float *d_a, void *stream);

/* Eq. (8): c = a - ln(Ip / (Ip + Is)), elementwise over n values. */
mc_status mc_scatter_correct_async(mc_ctx *ctx, const float *d_a, const float *d_ip,
                                   const float *d_is, uint64_t n, float *d_c, void *stream);

/* The FBP of the correction loop: Feldkamp-Davis-Kress cone-beam filtered
 * backprojection for the context's orbit and panel (mc_set_geometry), full
 * circle of n_ang equally spaced angles 2 pi i / n_ang.  d_proj[n_ang][nv][nu]
 * line integrals -> d_vol[nz][ny][nx] attenuation (per mm), cubic voxels of
 * voxel_mm centred on the axis; d_tmp holds the filtered projections (same
 * size as d_proj).  Virtual panel through the axis, cosine pre-weight, the
 * discrete Ram-Lak filter, distance-weighted bilinear backprojection.
 * MC_E_INVALID_ARG for nu > 8192, n_ang > 4096, or a volume whose corners
 * come within 1 % of the source orbit. */
mc_status mc_fdk_async(mc_ctx *ctx, const float *d_proj, int n_ang, float *d_tmp, float *d_vol,
                       int nx, int ny, int nz, float voxel_mm, void *stream);

/* Histogram for Otsu's threshold: d_hist[bins] (uint32, cleared first) counts
 * of x in [lo, hi), bin floor((x - lo) / (hi - lo) * bins). */
mc_status mc_histogram_async(mc_ctx *ctx, const float *d_x, uint64_t n, float lo, float hi,
                             int bins, uint32_t *d_hist, void *stream);

/* Volume to density: voxels with mu >= threshold (per mm) get `material` and
 * density mu / (0.1 mu_rho) (mu_rho in cm^2/g) rounded to multiples of step
 * (g/cm^3); the others material 0 at its nominal density. */
mc_status mc_to_density_async(mc_ctx *ctx, const float *d_mu, uint64_t n, float threshold,
                              float mu_rho, int material, float step, uint8_t *d_ids,
                              float *d_rho, void *stream);

/* Cancellation, for callers that must stop a long projection or batch: with
 * on = 1 every transport launch of the context that is running or queued stops
 * taking photons (each wave reads the flag, kept in mapped host memory, every
 * 64th scheduling round) and ends once the photons it holds, and the photon
 * ids its waves have reserved (at most 1024 per wave), are finished:
 * each projection's images then hold photons 0 .. m-1 for some m, bitwise what
 * a run of m photons gives, and nothing faults or hangs.  Launches made while
 * the flag is on stop within their first rounds.
 * mc_project then returns MC_E_CANCELLED (images written).  on = 0 clears the
 * flag for later launches.  The only call that may run concurrently with
 * other calls on the same context (from another host thread); an autotuner
 * run during a cancellation reports candidates as rejected.  Host-only
 * context: MC_E_STATE. */
mc_status mc_cancel(mc_ctx *ctx, int on);

/* One projection, blocking: simulates photons 0 .. n_photons-1 (emitted into
 * the cone circumscribing the panel) with Philox key `seed`, and writes the
 * Q43.20 tallies to host arrays primary[nv*nu] and scatter[snv*snu]. */
mc_status mc_project(mc_ctx *ctx, float angle_rad, uint64_t n_photons, uint64_t seed,
                     int64_t *primary, int64_t *scatter);

/* Stream-ordered: clears d_primary / d_scatter (device), then simulates
 * photons 0 .. n_photons-1 into them. */
mc_status mc_project_async(mc_ctx *ctx, float angle_rad, uint64_t n_photons, uint64_t seed,
                           int64_t *d_primary, int64_t *d_scatter, void *stream);

/* Stream-ordered: ADDS the tallies of photons first .. first+n-1 into
 * d_primary / d_scatter (no clearing).  Splitting a range into pieces gives
 * bitwise the same sum. */
mc_status mc_project_range_async(mc_ctx *ctx, float angle_rad, uint64_t first, uint64_t n,
                                 uint64_t seed, int64_t *d_primary, int64_t *d_scatter,
                                 void *stream);

/* Add another voxel object (same rules as mc_load_phantom) for batches; its
 * handle (>= 1) is written to *handle.  Handle 0 is the object of
 * mc_load_phantom. */
mc_status mc_phantom_add(mc_ctx *ctx, const uint8_t *ids, const float *rho_gcc, int nx, int ny,
                         int nz, float voxel_mm, int *handle);

/* One projection of a batch. */
typedef struct mc_job {
    int32_t phantom;           /* phantom handle                                   */
    float angle_rad;
    uint64_t n_photons;
    uint64_t seed;
    uint64_t primary_offset;   /* element offset of the job's [nv][nu] image in d_out   */
    uint64_t scatter_offset;   /* element offset of the job's [snv][snu] image in d_out */
} mc_job;

#define MC_BATCH_GRAPH 1u      /* capture clear + transport in a hipGraph and replay it */

/* Many projections (angles, phantoms of different sizes, photon counts) in
 * one persistent launch, stream-ordered: clears d_out[0 .. out_elems) (device,
 * int64), then simulates every job; each job's images are bitwise those of
 * mc_project_async with the same phantom, angle, photon count and seed.  The
 * projections of section III (many angles of one scan, independent of each
 * other) are the intended use.  With MC_BATCH_GRAPH the clear and transport
 * kernels are captured once into a graph (re-captured when buffers, job
 * count, launch shape or context state change) and replayed; the job table
 * itself is copied before each replay. */
mc_status mc_project_batch(mc_ctx *ctx, const mc_job *jobs, int n_jobs, int64_t *d_out,
                           uint64_t out_elems, uint32_t flags, void *stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): mc_project_batch
 * without MC_BATCH_GRAPH, with the same arguments and results (each job's
 * images bitwise those of mc_project_async), whose job, grid and photon-
 * counter tables live in a fixed device array of the library instead of a
 * context buffer.  It calls no hipMalloc or hipFree and no allocating
 * library routine; the caller provides d_out.  Limits: n_jobs <=
 * MC_STATIC_MAX_JOBS and at most MC_STATIC_MAX_PHANTOMS objects in the
 * context (else MC_E_INVALID_ARG).  The device tables (cross sections) must
 * already fit their buffer: after a change of spectrum, materials or response
 * that needs a larger one, run any other projection once first (else
 * MC_E_STATE).  Every call on one GPU shares that GPU's array (about 130 KiB,
 * held until the process ends): calls that overlap on one GPU, from any
 * context or stream, race and give wrong images; order them on one stream or
 * synchronise between them.  The clear of d_out and of the counters is a
 * kernel, not a memset. */
#define MC_STATIC_MAX_JOBS 1024
#define MC_STATIC_MAX_PHANTOMS 64
mc_status mc_project_batch_static(mc_ctx *ctx, const mc_job *jobs, int n_jobs, int64_t *d_out,
                                  uint64_t out_elems, void *stream);

/* March probe (a measuring instrument, not part of the method): n_rays
 * straight rays with the birth directions of photons 0 .. n_rays-1 of `seed`
 * are marched through the loaded object with the transport's fixed-step rule
 * (section II-C-2 as the transport reads it: the same step centres, clamps,
 * voxel layout and prefetch groups) and nothing else -- no optical depth,
 * interactions or tallies.  Lanes are refilled once refill_batch (1 .. 64)
 * of a wave's lanes are idle.  Adds the sum of the gathered voxel codes
 * (palette index or material id, plus the low bit of the density in the
 * generic layout) to d_sum[0] and the number of steps taken to d_sum[1]
 * (device uint64[2], not cleared).  Stream-ordered; the block size and
 * blocks per compute unit of mc_set_launch apply, and automatic blocks per
 * CU means the probe's own occupancy.  Its step rate is the ceiling of the
 * transport's march on the same object. */
mc_status mc_march_probe_async(mc_ctx *ctx, float angle_rad, uint64_t n_rays, uint64_t seed,
                               int refill_batch, uint64_t *d_sum, void *stream);

/* Tally probe (a measuring instrument, not part of the method): n_adds int64
 * atomic additions of 1 to d_image[n_pixels] (device int64, not cleared;
 * 1 <= n_pixels < 2^32).  Add i goes to pixel floor(h * n_pixels / 2^32),
 * h = H(lo32(i) ^ s ^ hi32(i) * 0x9E3779B9) with s = lo32(seed) ^ hi32(seed)
 * and H the 32-bit integer hash x ^= x >> 16; x *= 0x7feb352d; x ^= x >> 15;
 * x *= 0x846ca68b; x ^= x >> 16 (arithmetic mod 2^32), i.e. spread uniformly
 * over the image like the transport's tallies (the primary and scatter
 * images of eqs. 6-7) over a panel.  Stream-ordered; its add rate is the
 * ceiling of the transport's tally atomics on an image of that size. */
mc_status mc_atomic_probe_async(mc_ctx *ctx, uint64_t n_adds, uint64_t seed, int64_t *d_image,
                                uint64_t n_pixels, void *stream);

/* Uniform-cell map of a voxel object, as the march uses it to take runs of
 * identical voxels at once (host only, no context): codes[nz][ny][nx] are
 * per-voxel codes (the palette index of each (material, density) pair);
 * cells[ceil(nz/4)][ceil(ny/4)][ceil(nx/4)] receives, per cube of 4x4x4
 * voxels (clipped to the object), code | r << 8 where r >= 1 means that every
 * cell within Chebyshev distance r - 1 (indices clamped to the grid) holds
 * only that code (r capped at 255), and 0 for a cell holding several codes.
 * A run of fixed steps whose centres stay inside such a cube has one
 * optical-depth increment per step (section II-C-2's march is unchanged). */
mc_status mc_cell_map(const uint8_t *codes, int nx, int ny, int nz, uint16_t *cells);

/* Per-history record of photons first .. first+m-1 (blocking, host outputs,
 * any of them may be NULL): scatterings, march steps, end code (MC_END_*),
 * and the type of the first interaction (0 none, 1 photo, 2 Rayleigh,
 * 3 Compton). */
mc_status mc_debug_histories(mc_ctx *ctx, float angle_rad, uint64_t first, uint64_t m,
                             uint64_t seed, uint16_t *n_int, uint32_t *steps,
                             uint8_t *end_code, uint8_t *first_type);

/* GPU sampler hook (blocking, host outputs): n samples of one process, sample
 * i using photon id i of `seed`.  SOURCE_ENERGY: e_out = birth energy.
 * SOURCE_DIR: cos_out = cosine of the birth direction to the central ray.
 * RAYLEIGH / COMPTON at e_keV in `material`: cos_out, e_out = outgoing
 * cosine and energy; COMPTON is one collision under the context's binding
 * effects, a null collision giving cosine 2 and energy e_keV. */
mc_status mc_test_sample(mc_ctx *ctx, int process, int material, float e_keV, uint64_t n,
                         uint64_t seed, float *cos_out, float *e_out);

/* Statistics: enable (1) or disable (0) counting in later projections;
 * mc_get_stats copies and clears the counters (synchronises the device). */
mc_status mc_set_stats(mc_ctx *ctx, int enable);
mc_status mc_get_stats(mc_ctx *ctx, mc_stats *out);

/* Host-side cross-section tables exactly as the transport uses them:
 * fp32 mu/rho [cm^2/g] per material on E_j = 1 + j keV, arrays [n_mat][J]
 * for the context's whole material set, and eta[J].  *J and *n_mat are
 * always written; pass NULL arrays to query them first (each non-NULL array
 * must hold n_mat * J, eta J, floats).  Needs the spectrum. */
mc_status mc_get_tables(mc_ctx *ctx, int *J, int *n_mat, float *pe, float *coh, float *inc,
                        float *eta);

/* Device layout of the voxel object, chosen at the next mc_load_phantom.
 * AUTO: objects with <= 256 distinct (material, density) pairs are stored as
 * one-byte palette codes (per-lane attenuation table for <= 32 entries,
 * shared palette otherwise), others as material ids plus densities.  All
 * layouts are bricked (8x4x4 voxels) and give bitwise the same images. */
#define MC_LAYOUT_AUTO 0
#define MC_LAYOUT_PALETTE_LANE 1
#define MC_LAYOUT_PALETTE_SHARED 2
#define MC_LAYOUT_GENERIC 3
mc_status mc_set_layout(mc_ctx *ctx, int layout);
/* Layout in use for the loaded object (never AUTO) and its palette size
 * (0 for GENERIC). */
mc_status mc_get_layout(mc_ctx *ctx, int *layout, int *palette_size);

/* Launch shape of the transport kernel for single projections (0 =
 * automatic): threads per block (64, 128, 192 or 256), resident blocks per
 * compute unit, and the event batch: how many of a wave's 64 lanes must be
 * waiting for an interaction or a panel crossing before the wave stops
 * marching and handles them (1 .. 64; automatic: 58).  Results never depend
 * on these. */
mc_status mc_set_launch(mc_ctx *ctx, int block, int blocks_per_cu, int event_batch);
/* The same for mc_project_batch and mc_project_batch_static (automatic: 256
 * threads, blocks per CU from the occupancy, event batch 54).  The grid size
 * (blocks per CU x compute units) sets the photons each thread takes. */
mc_status mc_set_batch_launch(mc_ctx *ctx, int block, int blocks_per_cu, int event_batch);
/* Objects of the context (mc_load_phantom and mc_phantom_add), their total
 * voxel count and the largest palette (256 for objects stored with material
 * ids and densities). */
mc_status mc_get_batch_info(mc_ctx *ctx, int *n_phantoms, uint64_t *voxels, int *max_palette);

/* Dimensions of the loaded object (handle 0) and of the panel and scatter grid. */
mc_status mc_get_shape(mc_ctx *ctx, int *nx, int *ny, int *nz, int *nu, int *nv, int *snu,
                       int *snv);

/* Result of mc_autotune. */
typedef struct mc_tuning {
    int32_t block, blocks_per_cu, event_batch;
    int32_t table_layout;    /* MC_LAYOUT_PALETTE_LANE or _SHARED for palette
                                objects of <= 32 entries, else the object's own    */
    int32_t from_cache;      /* 1: taken from the cache, nothing was timed          */
    int32_t candidates;      /* launch shapes timed                                 */
    int32_t rejected;        /* shapes whose images differed bitwise (must be 0)    */
    double ms;               /* best time of one projection of n_photons            */
    double histories_per_s;
} mc_tuning;

/* Launch-shape autotuner: times block size x blocks per CU x event batch x
 * attenuation-table layout (per-lane tables of every palette entry, or the
 * shared palette with per-lane tables per material; both for palette objects
 * of <= 32 entries) on the context's current object, panel and spectrum
 * (n_photons of projection angle_rad with `seed`), checks that every
 * candidate reproduces the first one's images bitwise (rejecting any that
 * does not), applies the fastest with mc_set_launch and mc_set_layout (per-
 * lane tables as MC_LAYOUT_AUTO, the shared palette as
 * MC_LAYOUT_PALETTE_SHARED, which then also holds for later loads) and
 * appends it to the JSON-lines file cache_path (may be NULL).  If cache_path
 * already holds an entry for this device and workload class, that entry is
 * applied and nothing is timed.  Uses the GPU. */
mc_status mc_autotune(mc_ctx *ctx, float angle_rad, uint64_t n_photons, uint64_t seed,
                      const char *cache_path, mc_tuning *out);

/* The autotuner for batches (section III's many projections of one scan, and
 * objects of uneven size): times block size x blocks per CU (the grid size,
 * i.e. photons per thread) x event batch x attenuation-table layout on the
 * caller's job table with mc_project_batch (d_out: device int64[out_elems],
 * overwritten), checks that every candidate reproduces the first one's whole
 * output bitwise (rejecting any that does not), applies the fastest with
 * mc_set_batch_launch and mc_set_layout, and appends it to cache_path (may be
 * NULL) keyed by device, job count, total voxels, panel size and palette
 * class; a cached entry is applied without timing.  Uses the GPU. */
mc_status mc_autotune_batch(mc_ctx *ctx, const mc_job *jobs, int n_jobs, int64_t *d_out,
                            uint64_t out_elems, const char *cache_path, mc_tuning *out);

/* ---- post-processing of scatter images (section II-C-3 and II-C-4) ----
 * Stream-ordered kernels on device float images [ny][nx]. */

/* d_out[i] = (float)(d_in[i] * scale): Q43.20 tallies to float (scale =
 * 2^-20 gives keV; divide further by the photon count to normalise). */
mc_status mc_tally_to_float_async(mc_ctx *ctx, const int64_t *d_in, float *d_out, uint64_t n,
                                  double scale, void *stream);
/* Savitzky-Golay smoothing (the paper uses cubic order): least-squares
 * polynomial of degree `order` over `window` (odd, <= 31) samples, applied
 * along rows then columns, samples beyond an edge mirrored about the edge
 * sample.  d_tmp: caller scratch of nx*ny floats.  fp32. */
mc_status mc_savgol_async(mc_ctx *ctx, const float *d_in, float *d_out, float *d_tmp, int nx,
                          int ny, int window, int order, void *stream);
/* Cubic up-sampling by an integer factor (the paper's (576,800) -> (2304,3200)
 * cubic interpolation): Keys' kernel with a = -0.5, output pixel i at input
 * coordinate (i + 0.5)/factor - 0.5, edges clamped; d_out is
 * [ny*factor][nx*factor].  fp32. */
mc_status mc_upsample_cubic_async(mc_ctx *ctx, const float *d_in, float *d_out, int nx, int ny,
                                  int factor, void *stream);
/* Mirror image of an fp32 map [ny][nx] (device, d_out != d_in), optionally
 * accumulated: d_out[y][x] = alpha * d_in[flip_y ? ny-1-y : y][flip_x ? nx-1-x : x]
 * + beta * d_out[y][x] (d_out is not read when beta is 0).  The geometry of
 * section II-A is symmetric about both panel axes (the panel is centred on
 * the central ray), so mirrored objects give mirrored primary and scatter
 * maps: training pairs for the learned up-sampler are augmented with these
 * flips, and its predictions for the four mirror images averaged. */
mc_status mc_flip2d_async(mc_ctx *ctx, const float *d_in, float *d_out, int nx, int ny,
                          int flip_x, int flip_y, float alpha, float beta, void *stream);
/* The fp32 Savitzky-Golay weights mc_savgol_async uses (host only). */
mc_status mc_savgol_weights(int window, int order, float *weights);

/* ---- learned scatter denoiser / up-sampler: network kernels ----
 * A 2-D U-Net (bf16 weights and activations, fp32 accumulation on the
 * matrix cores) replaces the smoothing and interpolation of the paper's
 * correction loop (section II-C-3/4) and is trained by these kernels.
 * Activations are NHWC bf16 ([n][y][x][c], channels fastest) given as
 * (pointer, channel stride ld, channel offset), so concatenated skip
 * connections are channel slices of one buffer.  3x3 weights are bf16
 * [cout_alloc][9][cin] with tap = 3*(dy+1) + (dx+1); cout_alloc = 32 when
 * cout <= 32, else cout rounded up to 64; rows beyond cout are zero.
 * Requirements (checked): cin, ldx, xoff multiples of 16, 16-byte aligned
 * pointers, and the weight rows above.  All stream-ordered. */
typedef struct mc_conv3x3 {
    const uint16_t *x;      /* input activations                               */
    int32_t ldx, xoff;
    const uint16_t *w;      /* weights [cout_alloc][9][cin]                     */
    const float *bias;      /* [cout] or NULL                                   */
    uint16_t *y;            /* bf16 output (or NULL)                             */
    int32_t ldy, yoff;
    float *yf;              /* fp32 output [pixels][cout] (or NULL)              */
    const uint16_t *mask;   /* output multiplied by (mask > 0) if not NULL       */
    int32_t ldm, moff;
    int32_t n, h, w_, cin, cout;
    int32_t relu;           /* max(0, .) after the bias                          */
    int32_t accumulate;     /* add to the existing bf16 output                   */
} mc_conv3x3;

/* y = act(conv3x3(x, w) + bias), zero padding, stride 1.  With the flipped,
 * transposed weights of mc_nn_flip_weights_async and mask = the layer input,
 * it computes a convolution's input gradient through the previous ReLU. */
mc_status mc_nn_conv3x3_async(mc_ctx *ctx, const mc_conv3x3 *args, void *stream);
/* dw[co][tap][ci] (fp32) = sum over pixels of dy[p][co] * x[p + tap][ci];
 * deterministic (per-split partials summed in a fixed order).  workspace: at
 * least (splits + 1) * 9 * cout * cin floats; cin, cout multiples of 16;
 * splits 1..4096; n * h * w under 2^30 (else MC_E_INVALID_ARG). */
mc_status mc_nn_conv3x3_wgrad_async(mc_ctx *ctx, const uint16_t *x, int ldx, int xoff,
                                    const uint16_t *dy, int ldy, int yoff, int n, int h, int w,
                                    int cin, int cout, int splits, float *workspace, float *dw,
                                    void *stream);
/* db[c] = sum over npix pixels of dy[p][c] (fp32); workspace rows * c floats. */
mc_status mc_nn_bias_grad_async(mc_ctx *ctx, const uint16_t *dy, int ldy, int yoff, int npix,
                                int c, float *workspace, int rows, float *db, void *stream);
/* wt[ci][tap][co] = w[co][8 - tap][ci], zero for co >= cout or ci >= cin;
 * wt has cin_pad rows of 9 * cout_pad. */
mc_status mc_nn_flip_weights_async(mc_ctx *ctx, const uint16_t *w, uint16_t *wt, int cout, int cin,
                                   int cout_pad, int cin_pad, void *stream);
/* 2x2 average pooling of x[n][h][w] into y[n][h/2][w/2]; backward: x is the
 * pooled-size gradient, y the full-size one.  accumulate adds to y. */
mc_status mc_nn_pool2_async(mc_ctx *ctx, const uint16_t *x, int ldx, int xoff, uint16_t *y, int ldy,
                            int yoff, int n, int h, int w, int c, int backward, int accumulate,
                            void *stream);
/* nearest 2x up-sampling of x[n][h][w] into y[n][2h][2w]; backward: x is the
 * [2h][2w] gradient, y[n][h][w] the sum of each 2x2 block. */
mc_status mc_nn_upsample2_async(mc_ctx *ctx, const uint16_t *x, int ldx, int xoff, uint16_t *y,
                                int ldy, int yoff, int n, int h, int w, int c, int backward,
                                int accumulate, void *stream);
/* partial[b] = sum over block b of (out[i*ldo] - target[i])^2 (blocks of 256);
 * grad (if not NULL) channel goff of an NHWC buffer = bf16(2 (out - t) / n * gscale). */
mc_status mc_nn_mse_async(mc_ctx *ctx, const float *out, int ldo, const float *target, uint64_t n,
                          uint16_t *grad, int ldg, int goff, float gscale, float *partial,
                          void *stream);
/* Adam step t >= 1 on fp32 master weights p with gradient g * gscale; moments
 * m, v; writes the bf16 copy p_bf16 (may be NULL). */
mc_status mc_nn_adam_async(mc_ctx *ctx, float *p, const float *g, float *m, float *v,
                           uint16_t *p_bf16, uint64_t n, float lr, float beta1, float beta2,
                           float eps, int step, float gscale, void *stream);
/* g[p][goff + c] = 0 where y[p][yoff + c] <= 0 (gradient through a ReLU with
 * output y), for p < npix, c < ch. */
mc_status mc_nn_relu_mask_async(mc_ctx *ctx, uint16_t *g, int ldg, int goff, const uint16_t *y,
                                int ldy, int yoff, uint64_t npix, int ch, void *stream);
mc_status mc_nn_cast_bf16_async(mc_ctx *ctx, const float *in, uint16_t *out, uint64_t n,
                                void *stream);
/* out[p*ld + coff] = bf16(in[p] * scale) for p < npix. */
mc_status mc_nn_pack_channel_async(mc_ctx *ctx, const float *in, uint64_t npix, float scale,
                                   uint16_t *out, int ld, int coff, void *stream);

/* keV per least significant bit of a tally: 2^-20. */
double mc_tally_scale(void);

#ifdef __cplusplus
}
#endif
#endif
