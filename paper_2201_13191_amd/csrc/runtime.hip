// Host runtime of libmcx: the C ABI declared in include/mcx.h.
//
// A context owns device copies of the phantom and of the tables, a small
// control block (photon counter, statistics) and staging images for the
// blocking entry point.  Every projection is one launch of the persistent
// transport kernel on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/mcx.h"
#include "cells.hpp"
#include "kernel_params.hpp"
#include "nn_params.hpp"
#include "tables.hpp"

namespace mcx {
hipError_t launch_march_probe(const KParams &p, int layout, int grid, int block,
                              unsigned long long *sum, hipStream_t stream);
int march_probe_blocks_per_cu(int layout, int block);
hipError_t launch_atomic_probe(unsigned long long *img, uint32_t n_pix, unsigned long long n,
                               uint32_t seed, int grid, hipStream_t stream);
hipError_t launch_transport(const KParams &p, int layout, int grid, int block, bool stats,
                            bool debug, hipStream_t stream);
hipError_t launch_sample(const KParams &p, int process, int material, float e_kev, uint64_t n,
                         float *cos_out, float *e_out, hipStream_t stream);
int transport_blocks_per_cu(const KParams &p, int layout, int block, bool stats);
hipError_t launch_batch(const KParams &p, int max_lane_palette, int grid, int block, bool stats,
                        hipStream_t stream);
int batch_blocks_per_cu(const KParams &p, int max_lane_palette, int block, bool stats);
hipError_t launch_clear(unsigned long long *a, size_t na, unsigned long long *b, size_t nb,
                        hipStream_t stream);
hipError_t launch_primary(const KParams &p, int sub, const double *bin_w, const float *bin_mu,
                          int n_bins, float *out, hipStream_t stream);
hipError_t launch_interp_angles(const float *sim, int n_sim, uint64_t n_pix, float *full,
                                hipStream_t stream);
hipError_t launch_line_integrals(const float *I, uint64_t n, const float *I0, uint64_t n0,
                                 float *a, hipStream_t s);
hipError_t launch_scatter_correct(const float *a, const float *ip, const float *is, uint64_t n,
                                  float *c, hipStream_t s);
hipError_t launch_fdk(const float *proj, double R, double D, double pu, double pv, int nu, int nv,
                      int n_ang, float *q, int nx, int ny, int nz, double h, float *vol,
                      hipStream_t s);
hipError_t launch_histogram(const float *x, uint64_t n, double lo, double hi, int bins,
                            unsigned int *hist, hipStream_t s);
hipError_t launch_to_density(const float *mu, uint64_t n, double threshold, double mu_rho,
                             int material, double air_rho, double step, uint8_t *ids, float *rho,
                             hipStream_t s);
hipError_t launch_savgol(const float *in, float *out, float *tmp, int nx, int ny, int window,
                         const float *coeffs, hipStream_t s);
hipError_t launch_flip2d(const float *in, float *out, int nx, int ny, int fx, int fy, float alpha,
                         float beta, hipStream_t s);
hipError_t launch_upsample(const float *in, float *out, int nx, int ny, int f, hipStream_t s);
hipError_t launch_tally_to_float(const int64_t *in, float *out, uint64_t n, double scale,
                                 hipStream_t s);
hipError_t nn_conv3x3(const ConvArgs &a, hipStream_t s);
hipError_t nn_wgrad(const WgradArgs &a, float *tmp, float *dw, hipStream_t s);
hipError_t nn_colsum(const uint16_t *dy, int ldy, int yoff, int npix, int c, float *partial,
                     int rows, float *out, hipStream_t s);
hipError_t nn_flip(const uint16_t *w, uint16_t *wt, int cout, int cin, int cout_pad, int cin_pad,
                   hipStream_t s);
hipError_t nn_resample(int op, const uint16_t *x, int ldx, int xoff, uint16_t *y, int ldy,
                       int yoff, int n, int h, int w, int c, int backward, int accumulate,
                       hipStream_t s);
hipError_t nn_mse(const float *out, int ldo, const float *t, int64_t n, uint16_t *g, int ldg,
                  int goff, float gscale, float *partial, hipStream_t s);
hipError_t nn_adam(float *p, const float *g, float *m, float *v, uint16_t *pb, int64_t n, float lr,
                   float b1, float b2, float eps, float c1, float c2, float gscale, hipStream_t s);
hipError_t nn_cast_bf16(const float *in, uint16_t *out, int64_t n, hipStream_t s);
hipError_t nn_relu_mask(uint16_t *g, int ldg, int goff, const uint16_t *y, int ldy, int yoff,
                        int64_t npix, int c, hipStream_t s);
hipError_t nn_pack_channel(const float *in, int64_t npix, float scale, uint16_t *out, int ld,
                           int coff, hipStream_t s);
}  // namespace mcx

using namespace mcx;

namespace {
constexpr int kRing = 64;
constexpr int kCtlWords = kRing + 16;
constexpr int kMaxLanePalette = 32;   // palettes up to this size get per-lane mu tables
constexpr int kDefaultEventBatch = 44;        // single projections (swept 8..62)
#ifndef MCX_MAX_CHUNK
#define MCX_MAX_CHUNK 1024
#endif
constexpr uint64_t kMaxChunk = MCX_MAX_CHUNK;  // photon ids a wave reserves at most at once
constexpr int kDefaultBatchEventBatch = 48;   // batched launches (swept 32..60)
}  // namespace

// One voxel object on the device: bricked one-byte codes (palette index, or
// material id with a bricked density array when the object has more than 256
// distinct (id, rho) pairs).
struct Phantom {
    int nx = 0, ny = 0, nz = 0, nbx = 0, nby = 0, nbz = 0;
    int edge_pad = 0;   // copies of the face voxels past the high faces (0 or kEdgePad)
    float h = 0.0f;
    int max_id = 0;
    bool generic = false;
    int n_pal = 0;
    uint8_t *d_vox = nullptr;
    float *d_vrho = nullptr;
    unsigned char *d_pal = nullptr;     // 256 densities (f32) then 256 ids (u8)
    uint16_t *d_cells = nullptr;        // uniform-cell map (palette layouts)
    int ncx = 0, ncy = 0, ncz = 0;
    bool loaded = false;

    void release() {
        if (d_vox) (void)hipFree(d_vox);
        if (d_vrho) (void)hipFree(d_vrho);
        if (d_pal) (void)hipFree(d_pal);
        if (d_cells) (void)hipFree(d_cells);
        d_vox = nullptr;
        d_vrho = nullptr;
        d_pal = nullptr;
        d_cells = nullptr;
        loaded = false;
    }
};

struct mc_ctx {
    int device = 0;
    int n_cu = 256;
    hipStream_t stream = nullptr;        // for the blocking entry points
    char err[512] = {0};

    std::vector<mc_material> mats;
    std::vector<double> rayl_b;
    std::vector<double> pz_scale;        // Compton-profile momentum scale / (m c)
    uint32_t phys = 0;                   // MC_PHYS_* binding effects

    // voxel objects: [0] is the one of mc_load_phantom, more from mc_phantom_add
    std::vector<Phantom> phantoms = std::vector<Phantom>(1);
    int layout_req = MC_LAYOUT_AUTO;
    bool have_phantom = false;

    // batches: device job table, grid table, per-job counters, captured graph
    void *d_batch = nullptr;
    size_t d_batch_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<unsigned char> graph_key;
    // recorded after every batch launch; the next batch call waits on it before it
    // rewrites the job table and counters, whatever stream either call is on
    hipEvent_t batch_done = nullptr;
    unsigned generation = 0;             // bumped by every setter

    mc_geometry g{};
    bool have_geom = false;

    std::vector<float> e_bin;
    std::vector<uint64_t> thr;
    float e_max = 0.0f;
    bool have_spec = false;

    std::vector<float> eta_user;

    // tables (host and one device blob)
    bool tables_dirty = true;
    int J = 0;
    std::vector<float> pe, coh, inc, eta;
    void *d_tables = nullptr;
    size_t d_tables_bytes = 0;
    const float *dp_pe = nullptr, *dp_coh = nullptr, *dp_inc = nullptr, *dp_eta = nullptr;
    const float *dp_ebin = nullptr;
    const uint64_t *dp_thr = nullptr;
    const uint32_t *dp_guide = nullptr;
    const double *dp_rb = nullptr, *dp_pz = nullptr;

    // control block: [0, kRing) photon counters, one per launch in turn so
    // launches queued on different streams never share one; then statistics
    unsigned long long *d_ctl = nullptr;
    unsigned launches = 0;
    // cancellation flag in mapped host memory (mc_cancel), its device address
    int *h_cancel = nullptr;
    const int *d_cancel = nullptr;
    bool stats_on = false;

    // staging for mc_project
    int64_t *d_img = nullptr;
    size_t d_img_elems = 0;

    int block = 0, blocks_per_cu = 0, event_batch = 0;
    int batch_block = 0, batch_bpc = 0, batch_event_batch = 0;   // mc_project_batch's own

    // scatter estimator: analog, or point detector with splitting and roulette
    int estimator = MC_SCORE_ANALOG;
    int pd_split = 1;
    double pd_rr = 0.0;
    const double *dp_kn = nullptr, *dp_coh_series = nullptr;
    const double *dp_bin_w = nullptr;
    const float *dp_bin_mu = nullptr;
};

namespace {

mc_status lookup_scratch(mc_ctx *c);

mc_status fail(mc_ctx *c, mc_status code, const char *fmt, ...) {
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(c->err, sizeof c->err, fmt, ap);
        va_end(ap);
    }
    return code;
}

mc_status hip_fail(mc_ctx *c, hipError_t e, const char *what) {
    return fail(c, e == hipErrorOutOfMemory ? MC_E_OOM : MC_E_DEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

#define HIP_TRY(c, expr)                                   \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return hip_fail(c, e_, #expr); \
    } while (0)

const mc_material kDefaultMaterials[5] = {
    {7.64f, 0.49919f, 0.001205f, "air"},
    {7.42f, 0.55508f, 1.0f, "water"},
    {13.0f, 0.48181f, 2.699f, "aluminium"},
    {13.8f, 0.51480f, 1.92f, "bone_ca"},
    {26.0f, 0.46557f, 7.874f, "iron"},
};

void set_materials(mc_ctx *c, const mc_material *m, int n) {
    ++c->generation;
    c->mats.assign(m, m + n);
    c->rayl_b.resize(n);
    c->pz_scale.resize(n);
    for (int i = 0; i < n; ++i) {
        c->rayl_b[i] = rayleigh_b(m[i].z_eff);
        c->pz_scale[i] = compton_pz_scale(m[i].z_eff);
    }
    c->tables_dirty = true;
}

mc_status use_device(mc_ctx *c) {
    if (c->device < 0) return fail(c, MC_E_STATE, "host-only context (device -1) cannot run kernels");
    HIP_TRY(c, hipSetDevice(c->device));
    return MC_OK;
}

// Regenerate host tables and upload them (synchronises the device first so
// no queued kernel still reads the old blob).
mc_status refresh_tables(mc_ctx *c, bool may_alloc = true) {
    if (!c->tables_dirty) return MC_OK;
    ++c->generation;
    const int n_mat = (int)c->mats.size();
    std::vector<Material> mm(n_mat);
    for (int i = 0; i < n_mat; ++i) mm[i] = {c->mats[i].z_eff, c->mats[i].z_over_a};
    const int J = table_length(c->e_max);
    build_tables(mm.data(), n_mat, J, c->eta_user.empty() ? nullptr : c->eta_user.data(),
                 (int)c->eta_user.size(), c->pe, c->coh, c->inc, c->eta);
    c->J = J;
    // blob: rb[n_mat] f64 | pz[n_mat] f64 | kn[kKnTerms] f64 | coh series[kCohTerms] f64 |
    //       thr[n_bins] u64 | pe | coh | inc [n_mat*J] | eta[J] | e_bin[n_bins] |
    //       guide[256] u32
    const size_t nb = c->e_bin.size();
    const size_t tab = (size_t)n_mat * J;
    //       | bin_w[n_bins] f64 | bin_mu[n_bins][n_mat] f32 (the deterministic primary)
    const size_t head = (size_t)(2 * n_mat + kKnTerms + kCohTerms) * 8;
    const size_t body = nb * 8 + (3 * tab + J + nb + 256) * 4;
    const size_t bins_off = ((head + body + 7) / 8) * 8;
    const size_t bytes = bins_off + nb * 8 + nb * n_mat * 4;
    double kn[kKnTerms], cohs[kCohTerms];
    kn_norm_series(kn, kKnTerms);
    coherent_series(cohs, kCohTerms);
    // per spectrum bin: its draw probability times eta, and mu per unit density
    // per material, with the transport's fp32 interpolation
    auto lerp = [J](const float *t, float e) {
        const float x = e - 1.0f;
        int j = (int)x;
        j = j < 0 ? 0 : (j > J - 2 ? J - 2 : j);
        const float f = x - (float)j;
        return t[j] + f * (t[j + 1] - t[j]);
    };
    std::vector<double> bin_w(nb);
    std::vector<float> bin_mu(nb * n_mat);
    for (size_t k = 0; k < nb; ++k) {
        const uint64_t lo = k ? c->thr[k - 1] : 0;
        bin_w[k] = (double)(c->thr[k] - lo) / 4294967296.0 *
                   (double)lerp(c->eta.data(), c->e_bin[k]);
        for (int m = 0; m < n_mat; ++m) {
            const float *pe = c->pe.data() + (size_t)m * J, *co = c->coh.data() + (size_t)m * J,
                        *in = c->inc.data() + (size_t)m * J;
            bin_mu[k * n_mat + m] =
                ((lerp(pe, c->e_bin[k]) + lerp(co, c->e_bin[k])) + lerp(in, c->e_bin[k])) * 0.1f;
        }
    }
    uint32_t guide[256];
    for (uint32_t i = 0, k = 0; i < 256; ++i) {
        while (c->thr[k] <= ((uint64_t)i << 24)) ++k;
        guide[i] = k;
    }
    std::vector<unsigned char> blob(bytes);
    size_t off = 0;
    auto put = [&](const void *src, size_t n) {
        std::memcpy(blob.data() + off, src, n);
        off += n;
    };
    put(c->rayl_b.data(), n_mat * 8);
    put(c->pz_scale.data(), n_mat * 8);
    put(kn, sizeof kn);
    put(cohs, sizeof cohs);
    put(c->thr.data(), nb * 8);
    put(c->pe.data(), tab * 4);
    put(c->coh.data(), tab * 4);
    put(c->inc.data(), tab * 4);
    put(c->eta.data(), (size_t)J * 4);
    put(c->e_bin.data(), nb * 4);
    put(guide, sizeof guide);
    off = bins_off;
    put(bin_w.data(), nb * 8);
    put(bin_mu.data(), nb * n_mat * 4);
    if (bytes > c->d_tables_bytes && !may_alloc)
        return fail(c, MC_E_STATE,
                    "the tables need a larger device buffer: run any projection once first");
    HIP_TRY(c, hipDeviceSynchronize());
    if (bytes > c->d_tables_bytes) {
        if (c->d_tables) (void)hipFree(c->d_tables);
        c->d_tables = nullptr;
        c->d_tables_bytes = 0;
        HIP_TRY(c, hipMalloc(&c->d_tables, bytes));
        c->d_tables_bytes = bytes;
    }
    HIP_TRY(c, hipMemcpy(c->d_tables, blob.data(), bytes, hipMemcpyHostToDevice));
    unsigned char *b = (unsigned char *)c->d_tables;
    c->dp_rb = (const double *)b;
    c->dp_pz = (const double *)b + n_mat;
    c->dp_kn = (const double *)b + 2 * n_mat;
    c->dp_coh_series = (const double *)b + 2 * n_mat + kKnTerms;
    c->dp_thr = (const uint64_t *)(b + head);
    const float *f = (const float *)(b + head + nb * 8);
    c->dp_pe = f;
    c->dp_coh = f + tab;
    c->dp_inc = f + 2 * tab;
    c->dp_eta = f + 3 * tab;
    c->dp_ebin = f + 3 * tab + J;
    c->dp_guide = (const uint32_t *)(f + 3 * tab + J + nb);
    c->dp_bin_w = (const double *)(b + bins_off);
    c->dp_bin_mu = (const float *)(b + bins_off + nb * 8);
    c->tables_dirty = false;
    return MC_OK;
}

int phantom_layout(const mc_ctx *c, const Phantom &ph) {
    if (ph.generic) return kGeneric;
    if (c->layout_req == MC_LAYOUT_PALETTE_SHARED || ph.n_pal > kMaxLanePalette)
        return kPaletteShared;
    return kPaletteLane;
}

mc_status check_phantom(mc_ctx *c, const Phantom &ph) {
    if (ph.max_id >= (int)c->mats.size())
        return fail(c, MC_E_INVALID_ARG, "material id %d >= n_mat %d", ph.max_id,
                    (int)c->mats.size());
    const double hx = 0.5 * ph.nx * ph.h, hy = 0.5 * ph.ny * ph.h, hz = 0.5 * ph.nz * ph.h;
    const double diag = std::sqrt(hx * hx + hy * hy + hz * hz);
    if (!(diag < c->g.sod_mm) || !(diag < (double)c->g.sdd_mm - c->g.sod_mm))
        return fail(c, MC_E_INVALID_ARG, "phantom must lie strictly between source and panel");
    if (2.0 * diag / c->g.step_mm > 4194304.0)
        return fail(c, MC_E_INVALID_ARG, "step too small for the phantom");
    return MC_OK;
}

VoxelGrid grid_of(const mc_ctx *c, const Phantom &ph) {
    VoxelGrid G;
    std::memset(&G, 0, sizeof G);
    G.vox = ph.d_vox;
    G.vrho = ph.d_vrho;
    G.pal_rho = ph.d_pal ? (const float *)ph.d_pal : nullptr;
    G.pal_id = ph.d_pal ? ph.d_pal + 256 * 4 : nullptr;
    G.n_pal = ph.n_pal;
    G.layout = phantom_layout(c, ph);
    G.nx = ph.nx; G.ny = ph.ny; G.nz = ph.nz;
    G.nbx = ph.nbx; G.nby = ph.nby;
    G.ry = (uint32_t)ph.nbx * kBrick - 32u;
    G.rz = (uint32_t)ph.nbx * ph.nby * kBrick - 128u;
    G.unclamped = ph.edge_pad >= kEdgePad && c->g.step_mm <= ph.h;
    G.cmax[0] = (float)(ph.nx - 1);
    G.cmax[1] = (float)(ph.ny - 1);
    G.cmax[2] = (float)(ph.nz - 1);
    G.inv_h = 1.0f / ph.h;
    // runs of identical voxels through uniform cells are taken at once in
    // every layout
    G.cells = ph.d_cells;
    G.ncx = ph.ncx;
    G.ncy = ph.ncy;
    const int nd[3] = {ph.nx, ph.ny, ph.nz};
    for (int a = 0; a < 3; ++a) {
        G.hi[a] = 0.5f * ((float)nd[a] * ph.h);
        G.lo[a] = -G.hi[a];
    }
    return G;
}

// Frame of the projection at angle beta (fp32 values from fp64 sin/cos).
ProjFrame frame_of(const mc_geometry &g, float beta) {
    ProjFrame F;
    const float cb = (float)std::cos((double)beta), sb = (float)std::sin((double)beta);
    F.S[0] = g.sod_mm * cb; F.S[1] = g.sod_mm * sb; F.S[2] = 0.0f;
    F.ax[0] = -cb; F.ax[1] = -sb; F.ax[2] = 0.0f;
    F.eu[0] = -sb; F.eu[1] = cb; F.eu[2] = 0.0f;
    F.ev[0] = 0.0f; F.ev[1] = 0.0f; F.ev[2] = 1.0f;
    for (int a = 0; a < 3; ++a) F.D[a] = F.S[a] + g.sdd_mm * F.ax[a];
    F.hu = 0.5f * ((float)g.nu * g.pu_mm);
    F.hv = 0.5f * ((float)g.nv * g.pv_mm);
    const double sdd = g.sdd_mm, hu = F.hu, hv = F.hv;
    F.omc = (float)(1.0 - sdd / std::sqrt(sdd * sdd + hu * hu + hv * hv));
    return F;
}

mc_status check_overflow(mc_ctx *c, uint64_t n_max) {
    float eta_max = 0.0f;
    for (float v : c->eta) eta_max = std::max(eta_max, v);
    if ((long double)n_max * ((long double)eta_max * 1048576.0L + 1.0L) >= 9223372036854775807.0L)
        return fail(c, MC_E_OVERFLOW, "tally could overflow int64");
    return MC_OK;
}

// Tables, panel and knobs shared by single and batched launches.
void common_params(mc_ctx *c, KParams &p) {
    std::memset(&p, 0, sizeof p);
    p.pe = c->dp_pe; p.coh = c->dp_coh; p.inc = c->dp_inc; p.eta = c->dp_eta;
    p.J = c->J;
    p.n_mat = (int)c->mats.size();
    p.rayl_b = c->dp_rb;
    p.pz_scale = c->dp_pz;
    p.phys = c->phys;
    p.e_bin = c->dp_ebin;
    p.thr = c->dp_thr;
    p.guide = c->dp_guide;
    p.n_bins = (int)c->e_bin.size();
    const mc_geometry &g = c->g;
    p.sdd = g.sdd_mm; p.pu = g.pu_mm; p.pv = g.pv_mm; p.step = g.step_mm;
    p.nu = g.nu; p.nv = g.nv; p.snu = g.snu; p.snv = g.snv;
    p.bu = g.nu / g.snu; p.bv = g.nv / g.snv;
    p.flags = g.flags;
    p.event_batch = c->event_batch > 0 ? c->event_batch : kDefaultEventBatch;
    p.stats = c->d_ctl + kRing;
    p.cancel = c->d_cancel;
    p.kn_series = c->dp_kn;
    p.coh_series = c->dp_coh_series;
    p.pd_split = 0;      // single projections turn the point detector on (prepare)
    p.pd_rr = c->pd_rr;
}

// Every precondition of a projection of n photons; fills the kernel params.
mc_status prepare(mc_ctx *c, float beta, uint64_t first, uint64_t n, uint64_t seed,
                  KParams &p) {
    if (!c->have_phantom || !c->have_geom || !c->have_spec)
        return fail(c, MC_E_STATE, "phantom, geometry and spectrum must be set");
    if (!std::isfinite(beta)) return fail(c, MC_E_INVALID_ARG, "angle must be finite");
    const Phantom &ph = c->phantoms[0];
    mc_status rc = check_phantom(c, ph);
    if (rc) return rc;
    if (first + n < first) return fail(c, MC_E_INVALID_ARG, "photon range wraps");
    rc = refresh_tables(c);
    if (rc) return rc;
    rc = check_overflow(c, first + n);
    if (rc) return rc;
    common_params(c, p);
    p.G = grid_of(c, ph);
    p.F = frame_of(c->g, beta);
    p.first = first;
    p.n = n;
    p.key0 = (uint32_t)seed;
    p.key1 = (uint32_t)(seed >> 32);
    p.counter = c->d_ctl + (c->launches++ % kRing);
    if (c->estimator != MC_SCORE_ANALOG) {
        p.pd_split = c->pd_split;
        p.pd_mode = c->estimator == MC_SCORE_POINT_MIXED ? 2 : 1;
    }
    return MC_OK;
}

// photon ids a wave reserves per update of a counter that every wave of the
// launch updates: about an eighth of a wave's share of n, 64 .. kMaxChunk
uint32_t reservation_chunk(uint64_t n, int grid, int block) {
    const uint64_t waves = std::max<uint64_t>(1, (uint64_t)grid * (uint64_t)(block / 64));
    return (uint32_t)std::min<uint64_t>(kMaxChunk, std::max<uint64_t>(64, n / (8 * waves)));
}

void launch_shape(mc_ctx *c, const KParams &p, int layout, bool stats, int &grid, int &block) {
    block = c->block > 0 ? c->block : 256;
    const int bpc = c->blocks_per_cu > 0 ? c->blocks_per_cu
                                         : transport_blocks_per_cu(p, layout, block, stats);
    const uint64_t full = (uint64_t)bpc * c->n_cu;
    const uint64_t need = (p.n + block - 1) / block;
    grid = (int)std::max<uint64_t>(1, std::min(full, need));
}

mc_status run(mc_ctx *c, KParams &p, hipStream_t s, bool debug) {
    if (p.n == 0) return MC_OK;
    if (debug) p.pd_split = 0;   // per-history records are the same with either estimator
    HIP_TRY(c, hipMemsetAsync(p.counter, 0, sizeof(unsigned long long), s));
    const bool stats = c->stats_on && !debug;
    const int layout = p.G.layout;
    int grid, block;
    launch_shape(c, p, layout, stats, grid, block);
    if (!stats) p.stats = nullptr;
    p.chunk = reservation_chunk(p.n, grid, block);
    hipError_t e = launch_transport(p, layout, grid, block, stats, debug, s);
    if (e != hipSuccess) return hip_fail(c, e, "transport launch");
    return MC_OK;
}

}  // namespace

extern "C" {

mc_status mc_create(mc_ctx **out, int device) {
    if (!out) return MC_E_INVALID_ARG;
    *out = nullptr;
    if (device == -1) {
        // host-only context: argument validation and host tables, no device work
        mc_ctx *c = new (std::nothrow) mc_ctx();
        if (!c) return MC_E_OOM;
        c->device = -1;
        set_materials(c, kDefaultMaterials, 5);
        *out = c;
        return MC_OK;
    }
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || device < 0 || device >= n_dev)
        return MC_E_INVALID_ARG;
    mc_ctx *c = new (std::nothrow) mc_ctx();
    if (!c) return MC_E_OOM;
    c->device = device;
    set_materials(c, kDefaultMaterials, 5);
    mc_status rc = MC_OK;
    hipDeviceProp_t prop;
    if (hipSetDevice(device) != hipSuccess || hipGetDeviceProperties(&prop, device) != hipSuccess ||
        hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc(&c->d_ctl, kCtlWords * sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(c->d_ctl, 0, kCtlWords * sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc((void **)&c->h_cancel, sizeof(int),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
        rc = MC_E_DEVICE;
    if (!rc) {
        *c->h_cancel = 0;
        void *dp = nullptr;
        if (hipHostGetDevicePointer(&dp, c->h_cancel, 0) != hipSuccess) rc = MC_E_DEVICE;
        c->d_cancel = (const int *)dp;
    }
    if (rc) {
        mc_destroy(c);
        return rc;
    }
    c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    rc = lookup_scratch(c);
    if (rc) {
        mc_destroy(c);
        return rc;
    }
    *out = c;
    return MC_OK;
}

void mc_destroy(mc_ctx *c) {
    if (!c) return;
    if (c->device < 0) {
        delete c;
        return;
    }
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (Phantom &ph : c->phantoms) ph.release();
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->batch_done) (void)hipEventDestroy(c->batch_done);
    if (c->d_batch) (void)hipFree(c->d_batch);
    if (c->d_tables) (void)hipFree(c->d_tables);
    if (c->d_ctl) (void)hipFree(c->d_ctl);
    if (c->d_img) (void)hipFree(c->d_img);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    if (c->h_cancel) (void)hipHostFree(c->h_cancel);
    delete c;
}

const char *mc_last_error(const mc_ctx *c) { return c ? c->err : "null context"; }

mc_status mc_set_materials(mc_ctx *c, const mc_material *m, int n) {
    if (!c) return MC_E_INVALID_ARG;
    if (!m || n < 1 || n > kMaxMaterials) return fail(c, MC_E_INVALID_ARG, "n_mat must be 1..16");
    for (int i = 0; i < n; ++i)
        if (!(m[i].z_eff >= 1.0f && m[i].z_eff <= 100.0f) ||
            !(m[i].z_over_a > 0.0f && m[i].z_over_a <= 1.01f))
            return fail(c, MC_E_INVALID_ARG, "material %d: z_eff/z_over_a out of range", i);
    set_materials(c, m, n);
    return MC_OK;
}

}  // extern "C"

namespace {

// Validate a voxel object, build its bricked device representation into `out`
// (replacing what `out` held).
mc_status build_phantom(mc_ctx *c, const uint8_t *ids, const float *rho, int nx, int ny, int nz,
                        float h, Phantom &out) {
    if (!ids || !rho || nx < 1 || ny < 1 || nz < 1 || nx > 4096 || ny > 4096 || nz > 4096 ||
        !(h > 0.0f) || !std::isfinite(h))
        return fail(c, MC_E_INVALID_ARG, "bad phantom dimensions");
    // bricks covering the object and, where the 24-bit brick strides allow,
    // kEdgePad more voxels past each high face
    auto bricks = [&](int pad, int &bx, int &by, int &bz) {
        bx = (nx + pad + kBx - 1) / kBx;
        by = (ny + pad + kBy - 1) / kBy;
        bz = (nz + pad + kBz - 1) / kBz;
        return (size_t)bx * by * kBrick - kBrick < ((size_t)1 << 24) &&
               (size_t)bx * by * bz * kBrick < ((size_t)1 << 31);
    };
    int nbx, nby, nbz;
    int edge_pad = kEdgePad;
    if (!bricks(edge_pad, nbx, nby, nbz)) {
        edge_pad = 0;
        bricks(0, nbx, nby, nbz);
    }
    const size_t nv = (size_t)nx * ny * nz;
    const size_t padded = (size_t)nbx * nby * nbz * kBrick;
    if (padded >= (size_t)1 << 31) return fail(c, MC_E_INVALID_ARG, "phantom too large (2^31 voxels)");
    // the kernel multiplies brick strides in 24 bits
    if ((size_t)nbx * nby * kBrick - kBrick >= ((size_t)1 << 24))
        return fail(c, MC_E_INVALID_ARG, "phantom too large (an x-y slab of bricks above 16 MiB)");
    // validate and collect the distinct (id, density) pairs, first appearance first
    int max_id = 0;
    uint32_t pal_rho_bits[256];
    uint8_t pal_id[256];
    int n_pal = 0;
    bool palette_ok = c->layout_req != MC_LAYOUT_GENERIC;
    uint64_t table[1024] = {0};
    int16_t slot_pal[1024];
    std::memset(slot_pal, 0xff, sizeof slot_pal);
    uint64_t last_key = ~0ull;
    for (size_t i = 0; i < nv; ++i) {
        const float r = rho[i];
        if (!std::isfinite(r) || r < 0.0f || r > 1000.0f)
            return fail(c, MC_E_INVALID_ARG, "density at %zu must be finite and in [0, 1000]", i);
        max_id = std::max<int>(max_id, ids[i]);
        if (!palette_ok) continue;
        uint32_t bits;
        std::memcpy(&bits, &r, 4);
        const uint64_t key = ((uint64_t)ids[i] << 32) | bits;
        if (key == last_key) continue;
        last_key = key;
        uint32_t hsh = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 54);   // 10 bits
        for (;;) {
            if (slot_pal[hsh] < 0) {
                if (n_pal == 256) {
                    palette_ok = false;
                    break;
                }
                slot_pal[hsh] = (int16_t)n_pal;
                table[hsh] = key;
                pal_id[n_pal] = ids[i];
                pal_rho_bits[n_pal] = bits;
                ++n_pal;
                break;
            }
            if (table[hsh] == key) break;
            hsh = (hsh + 1) & 1023;
        }
    }
    if (c->layout_req != MC_LAYOUT_AUTO && c->layout_req != MC_LAYOUT_GENERIC && !palette_ok)
        return fail(c, MC_E_INVALID_ARG, "palette layout requested but the object has > 256 "
                                         "distinct (material, density) pairs");
    mc_status rc = use_device(c);
    if (rc) return rc;
    // bricked host images, and the code of each uniform cell (-1: mixed)
    std::vector<uint8_t> vox(padded, 0);
    std::vector<float> vr;
    if (!palette_ok) vr.assign(padded, 0.0f);
    const int ncx = (nx + (1 << kCellLog) - 1) >> kCellLog;
    const int ncy = (ny + (1 << kCellLog) - 1) >> kCellLog;
    const int ncz = (nz + (1 << kCellLog) - 1) >> kCellLog;
    std::vector<int16_t> cell_code((size_t)ncx * ncy * ncz, -2);   // -2: no voxel seen yet
    // generic objects: the (material, density) of each cell while it is uniform
    // (state: 0 unseen, 1 uniform, 2 mixed), coded after the pass
    std::vector<uint64_t> cell_key;
    std::vector<uint8_t> cell_state;
    if (!palette_ok) {
        cell_key.assign(cell_code.size(), 0);
        cell_state.assign(cell_code.size(), 0);
    }
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y) {
            const size_t row = ((size_t)z * ny + y) * nx;
            const size_t bzy = ((size_t)(z / kBz) * nby + (y / kBy)) * nbx;
            const int inner = ((z % kBz) * kBy + (y % kBy)) * kBx;
            uint64_t last = ~0ull;
            uint8_t last_code = 0;
            for (int x = 0; x < nx; ++x) {
                const size_t off = (bzy + x / kBx) * kBrick + inner + (x % kBx);
                if (!palette_ok) {
                    vox[off] = ids[row + x];
                    vr[off] = rho[row + x];
                    uint32_t bits;
                    std::memcpy(&bits, &rho[row + x], 4);
                    const uint64_t key = ((uint64_t)ids[row + x] << 32) | bits;
                    const size_t ci = ((size_t)(z >> kCellLog) * ncy + (y >> kCellLog)) * ncx +
                                      (x >> kCellLog);
                    if (cell_state[ci] == 0) {
                        cell_state[ci] = 1;
                        cell_key[ci] = key;
                    } else if (cell_state[ci] == 1 && cell_key[ci] != key) {
                        cell_state[ci] = 2;
                    }
                    continue;
                }
                uint32_t bits;
                std::memcpy(&bits, &rho[row + x], 4);
                const uint64_t key = ((uint64_t)ids[row + x] << 32) | bits;
                if (key != last) {
                    uint32_t hsh = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 54);
                    while (slot_pal[hsh] < 0 || table[hsh] != key) hsh = (hsh + 1) & 1023;
                    last = key;
                    last_code = (uint8_t)slot_pal[hsh];
                }
                vox[off] = last_code;
                int16_t &cc = cell_code[((size_t)(z >> kCellLog) * ncy + (y >> kCellLog)) * ncx +
                                        (x >> kCellLog)];
                if (cc == -2)
                    cc = last_code;
                else if (cc != last_code)
                    cc = -1;
            }
        }
    if (edge_pad) {
        // every bricked position past a high face takes the voxel at the
        // clamped position
        auto boff = [&](int x, int y, int z) {
            return (((size_t)(z / kBz) * nby + (y / kBy)) * nbx + x / kBx) * kBrick +
                   (size_t)(((z % kBz) * kBy + (y % kBy)) * kBx + (x % kBx));
        };
        const int X = nbx * kBx, Y = nby * kBy, Z = nbz * kBz;
        for (int z = 0; z < Z; ++z)
            for (int y = 0; y < Y; ++y)
                for (int x = (z < nz && y < ny) ? nx : 0; x < X; ++x) {
                    const size_t src = boff(std::min(x, nx - 1), std::min(y, ny - 1),
                                            std::min(z, nz - 1));
                    const size_t dst = boff(x, y, z);
                    vox[dst] = vox[src];
                    if (!palette_ok) vr[dst] = vr[src];
                }
    }
    // generic objects: the distinct values of their uniform cells, first
    // appearance first, form a palette of at most 256 entries that only runs
    // through uniform regions use (cells past the 256th value count as mixed)
    if (!palette_ok) {
        n_pal = 0;
        std::unordered_map<uint64_t, int> code_of;
        for (size_t i = 0; i < cell_code.size(); ++i) {
            if (cell_state[i] != 1) {
                cell_code[i] = -1;
                continue;
            }
            auto it = code_of.find(cell_key[i]);
            if (it == code_of.end()) {
                if (n_pal == 256) {
                    cell_code[i] = -1;
                    continue;
                }
                it = code_of.emplace(cell_key[i], n_pal).first;
                pal_id[n_pal] = (uint8_t)(cell_key[i] >> 32);
                pal_rho_bits[n_pal] = (uint32_t)cell_key[i];
                ++n_pal;
            }
            cell_code[i] = (int16_t)it->second;
        }
    }
    std::vector<uint16_t> cells;
    cell_radii(ncx, ncy, ncz, cell_code, cells);
    HIP_TRY(c, hipDeviceSynchronize());
    out.release();
    HIP_TRY(c, hipMalloc(&out.d_vox, padded));
    HIP_TRY(c, hipMemcpy(out.d_vox, vox.data(), padded, hipMemcpyHostToDevice));
    if (!palette_ok) {
        HIP_TRY(c, hipMalloc(&out.d_vrho, padded * sizeof(float)));
        HIP_TRY(c, hipMemcpy(out.d_vrho, vr.data(), padded * sizeof(float), hipMemcpyHostToDevice));
    }
    // the palette (generic objects: of their uniform cells) and the cell map
    unsigned char pal[256 * 5] = {0};
    std::memcpy(pal, pal_rho_bits, (size_t)n_pal * 4);
    std::memcpy(pal + 256 * 4, pal_id, (size_t)n_pal);
    HIP_TRY(c, hipMalloc(&out.d_pal, sizeof pal));
    HIP_TRY(c, hipMemcpy(out.d_pal, pal, sizeof pal, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMalloc(&out.d_cells, cells.size() * sizeof(uint16_t)));
    HIP_TRY(c, hipMemcpy(out.d_cells, cells.data(), cells.size() * sizeof(uint16_t),
                         hipMemcpyHostToDevice));
    out.ncx = ncx; out.ncy = ncy; out.ncz = ncz;
    out.nx = nx; out.ny = ny; out.nz = nz; out.h = h;
    out.nbx = nbx; out.nby = nby; out.nbz = nbz;
    out.edge_pad = edge_pad;
    out.max_id = max_id;
    out.generic = !palette_ok;
    out.n_pal = palette_ok ? n_pal : 0;     // generic: its cells' palette is not a voxel palette
    out.loaded = true;
    ++c->generation;
    return MC_OK;
}

// A batch's host-side preparation, shared by the allocating and the
// allocation-free entry points: validation, tables, and the device tables'
// contents (grids for every phantom, then jobs; per-job counters follow them
// on the device and are cleared by the launch's clear kernel).
struct BatchPlan {
    std::vector<unsigned char> host;   // grids | jobs
    size_t gb = 0, jbytes = 0, bytes = 0;
    int max_lane_pal = 0;
    uint64_t total = 0;
    ProjFrame F0{};
};

mc_status plan_batch(mc_ctx *c, const mc_job *jobs, int n_jobs, int64_t *d_out,
                     uint64_t out_elems, bool may_alloc, BatchPlan &b) {
    if (!jobs || n_jobs < 1 || n_jobs > 65536 || !d_out)
        return fail(c, MC_E_INVALID_ARG, "need 1..65536 jobs and an output buffer");
    if (!c->have_geom || !c->have_spec) return fail(c, MC_E_STATE, "geometry and spectrum must be set");
    if (c->estimator != MC_SCORE_ANALOG)
        return fail(c, MC_E_STATE, "batches score analog: set MC_SCORE_ANALOG first");
    mc_status rc = use_device(c);
    if (rc) return rc;
    const uint64_t np = (uint64_t)c->g.nu * c->g.nv, ns = (uint64_t)c->g.snu * c->g.snv;
    uint64_t n_max = 0;
    for (int j = 0; j < n_jobs; ++j) {
        const mc_job &jb = jobs[j];
        if (jb.phantom < 0 || jb.phantom >= (int)c->phantoms.size() || !c->phantoms[jb.phantom].loaded)
            return fail(c, MC_E_INVALID_ARG, "job %d: unknown phantom %d", j, jb.phantom);
        if (!std::isfinite(jb.angle_rad)) return fail(c, MC_E_INVALID_ARG, "job %d: bad angle", j);
        if (jb.primary_offset > out_elems || out_elems - jb.primary_offset < np ||
            jb.scatter_offset > out_elems || out_elems - jb.scatter_offset < ns)
            return fail(c, MC_E_INVALID_ARG, "job %d: images outside the output buffer", j);
        rc = check_phantom(c, c->phantoms[jb.phantom]);
        if (rc) return rc;
        n_max = std::max(n_max, jb.n_photons);
        b.total += jb.n_photons;
    }
    rc = refresh_tables(c, may_alloc);
    if (rc) return rc;
    rc = check_overflow(c, n_max);
    if (rc) return rc;
    const int n_grid = (int)c->phantoms.size();
    b.gb = ((n_grid * sizeof(VoxelGrid) + 255) / 256) * 256;
    b.jbytes = ((n_jobs * sizeof(JobDesc) + 255) / 256) * 256;
    b.bytes = b.gb + b.jbytes + (size_t)n_jobs * 8;
    b.host.assign(b.gb + b.jbytes, 0);
    VoxelGrid *hg = (VoxelGrid *)b.host.data();
    for (int i = 0; i < n_grid; ++i) {
        if (!c->phantoms[i].loaded) continue;
        hg[i] = grid_of(c, c->phantoms[i]);
        if (hg[i].layout == kPaletteLane) b.max_lane_pal = std::max(b.max_lane_pal, hg[i].n_pal);
    }
    JobDesc *hj = (JobDesc *)(b.host.data() + b.gb);
    for (int j = 0; j < n_jobs; ++j) {
        const mc_job &jb = jobs[j];
        hj[j].F = frame_of(c->g, jb.angle_rad);
        hj[j].key0 = (uint32_t)jb.seed;
        hj[j].key1 = (uint32_t)(jb.seed >> 32);
        hj[j].n = jb.n_photons;
        hj[j].prim = (unsigned long long *)(d_out + jb.primary_offset);
        hj[j].scat = (unsigned long long *)(d_out + jb.scatter_offset);
        hj[j].grid = jb.phantom;
    }
    b.F0 = hj[0].F;
    return MC_OK;
}

// Kernel parameters and launch shape of a planned batch whose device tables
// start at db.
void batch_params(mc_ctx *c, const BatchPlan &b, unsigned char *db, int n_jobs, KParams &p,
                  int &grid, int &block, bool &stats) {
    common_params(c, p);
    p.grids = (const VoxelGrid *)db;
    p.jobs = (const JobDesc *)(db + b.gb);
    p.job_counters = (unsigned long long *)(db + b.gb + b.jbytes);
    p.n_jobs = n_jobs;
    p.F = b.F0;
    p.event_batch = c->batch_event_batch > 0 ? c->batch_event_batch : kDefaultBatchEventBatch;
    stats = c->stats_on;
    if (!stats) p.stats = nullptr;
    block = c->batch_block > 0 ? c->batch_block : 256;
    const int bpc = c->batch_bpc > 0 ? c->batch_bpc
                                     : batch_blocks_per_cu(p, b.max_lane_pal, block, stats);
    grid = (int)std::max<uint64_t>(
        1, std::min<uint64_t>((uint64_t)bpc * c->n_cu, (b.total + block - 1) / block));
    p.chunk = reservation_chunk(b.total, grid, block);
}

}  // namespace

// ---- scratch of the allocation-free batch entry point -------------------------
// The device tables of mc_project_batch_static (grids, jobs, per-job photon
// counters) live in this file-scope array: one copy per GPU, held until the
// process ends.  Host code never passes the array's name to a kernel or a copy
// (on the host it is only a stand-in symbol); it uses the device address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device when a context is created on it.
namespace {
constexpr size_t kStaticGridBytes =
    ((MC_STATIC_MAX_PHANTOMS * sizeof(VoxelGrid) + 255) / 256) * 256;
constexpr size_t kStaticJobBytes = ((MC_STATIC_MAX_JOBS * sizeof(JobDesc) + 255) / 256) * 256;
constexpr size_t kStaticBytes = kStaticGridBytes + kStaticJobBytes + MC_STATIC_MAX_JOBS * 8;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {
unsigned char *g_scratch[kMaxDevices];   // device address of `scratch`, per device
std::mutex g_scratch_mu;

// once per device, with that device current
mc_status lookup_scratch(mc_ctx *c) {
    if (c->device < 0 || c->device >= kMaxDevices) return MC_OK;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[c->device]) return MC_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(c, e, "hipGetSymbolAddress(scratch)");
    g_scratch[c->device] = (unsigned char *)ptr;
    return MC_OK;
}

mc_status static_scratch(mc_ctx *c, unsigned char **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (c->device < 0 || c->device >= kMaxDevices || !g_scratch[c->device])
        return fail(c, MC_E_STATE, "no scratch address for device %d", c->device);
    *out = g_scratch[c->device];
    return MC_OK;
}
}  // namespace

extern "C" {

mc_status mc_cell_map(const uint8_t *codes, int nx, int ny, int nz, uint16_t *cells) {
    if (!codes || !cells || nx < 1 || ny < 1 || nz < 1 || nx > 4096 || ny > 4096 || nz > 4096)
        return MC_E_INVALID_ARG;
    const int ncx = (nx + (1 << kCellLog) - 1) >> kCellLog;
    const int ncy = (ny + (1 << kCellLog) - 1) >> kCellLog;
    const int ncz = (nz + (1 << kCellLog) - 1) >> kCellLog;
    std::vector<int16_t> code((size_t)ncx * ncy * ncz, -2);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const uint8_t v = codes[((size_t)z * ny + y) * nx + x];
                int16_t &cc = code[((size_t)(z >> kCellLog) * ncy + (y >> kCellLog)) * ncx +
                                   (x >> kCellLog)];
                if (cc == -2)
                    cc = v;
                else if (cc != v)
                    cc = -1;
            }
    std::vector<uint16_t> out;
    cell_radii(ncx, ncy, ncz, code, out);
    std::memcpy(cells, out.data(), out.size() * sizeof(uint16_t));
    return MC_OK;
}

mc_status mc_load_phantom(mc_ctx *c, const uint8_t *ids, const float *rho, int nx, int ny,
                          int nz, float h) {
    if (!c) return MC_E_INVALID_ARG;
    const mc_status rc = build_phantom(c, ids, rho, nx, ny, nz, h, c->phantoms[0]);
    c->have_phantom = c->phantoms[0].loaded;
    return rc;
}

mc_status mc_phantom_add(mc_ctx *c, const uint8_t *ids, const float *rho, int nx, int ny,
                         int nz, float h, int *handle) {
    if (!c) return MC_E_INVALID_ARG;
    if (!handle) return fail(c, MC_E_INVALID_ARG, "null handle");
    if (c->phantoms.size() >= 4096) return fail(c, MC_E_INVALID_ARG, "too many phantoms");
    Phantom ph;
    mc_status rc = build_phantom(c, ids, rho, nx, ny, nz, h, ph);
    if (rc) return rc;
    c->phantoms.push_back(ph);
    *handle = (int)c->phantoms.size() - 1;
    return MC_OK;
}

mc_status mc_set_layout(mc_ctx *c, int layout) {
    if (!c) return MC_E_INVALID_ARG;
    if (layout < MC_LAYOUT_AUTO || layout > MC_LAYOUT_GENERIC)
        return fail(c, MC_E_INVALID_ARG, "unknown layout %d", layout);
    c->layout_req = layout;
    return MC_OK;
}

mc_status mc_get_layout(mc_ctx *c, int *layout, int *palette_size) {
    if (!c || !layout || !palette_size) return MC_E_INVALID_ARG;
    if (!c->have_phantom) return fail(c, MC_E_STATE, "no phantom loaded");
    const Phantom &ph = c->phantoms[0];
    const int l = phantom_layout(c, ph);
    *layout = l == kGeneric ? MC_LAYOUT_GENERIC
              : l == kPaletteShared ? MC_LAYOUT_PALETTE_SHARED : MC_LAYOUT_PALETTE_LANE;
    *palette_size = ph.n_pal;
    return MC_OK;
}

mc_status mc_set_geometry(mc_ctx *c, const mc_geometry *g) {
    if (!c) return MC_E_INVALID_ARG;
    if (!g) return fail(c, MC_E_INVALID_ARG, "null geometry");
    if (!(g->sod_mm > 0.0f) || !(g->sdd_mm > g->sod_mm) || !std::isfinite(g->sdd_mm))
        return fail(c, MC_E_INVALID_ARG, "need 0 < sod < sdd");
    if (g->nu < 1 || g->nv < 1 || g->nu > 16384 || g->nv > 16384 || !(g->pu_mm > 0.0f) ||
        !(g->pv_mm > 0.0f) || !std::isfinite(g->pu_mm) || !std::isfinite(g->pv_mm))
        return fail(c, MC_E_INVALID_ARG, "bad detector");
    if (g->snu < 1 || g->snv < 1 || g->nu % g->snu || g->nv % g->snv)
        return fail(c, MC_E_INVALID_ARG, "scatter grid must divide the detector");
    if (!(g->step_mm > 0.0f) || !std::isfinite(g->step_mm))
        return fail(c, MC_E_INVALID_ARG, "step must be > 0");
    if (g->flags & ~MC_NO_SCATTER) return fail(c, MC_E_INVALID_ARG, "unknown flags");
    c->g = *g;
    c->have_geom = true;
    ++c->generation;
    return MC_OK;
}

mc_status mc_set_spectrum(mc_ctx *c, const float *e, const float *w, int n) {
    if (!c) return MC_E_INVALID_ARG;
    if (!e || !w || n < 1 || n > 4096) return fail(c, MC_E_INVALID_ARG, "n_bins must be 1..4096");
    double total = 0.0;
    float emax = 0.0f;
    for (int k = 0; k < n; ++k) {
        if (!(e[k] >= 1.0f && e[k] <= 1000.0f))
            return fail(c, MC_E_INVALID_ARG, "bin %d energy outside [1, 1000] keV", k);
        if (!(w[k] >= 0.0f) || !std::isfinite(w[k]))
            return fail(c, MC_E_INVALID_ARG, "bin %d weight must be finite and >= 0", k);
        total += (double)w[k];
        emax = std::max(emax, e[k]);
    }
    if (!(total > 0.0)) return fail(c, MC_E_INVALID_ARG, "weights sum to zero");
    c->e_bin.assign(e, e + n);
    spectrum_thresholds(w, n, c->thr);
    c->e_max = emax;
    c->have_spec = true;
    c->tables_dirty = true;
    return MC_OK;
}

mc_status mc_set_detector_response(mc_ctx *c, const float *eta, int n) {
    if (!c) return MC_E_INVALID_ARG;
    if (!eta || n < 1 || n > 4096) return fail(c, MC_E_INVALID_ARG, "eta length must be 1..4096");
    for (int i = 0; i < n; ++i)
        if (!(eta[i] >= 0.0f) || !std::isfinite(eta[i]))
            return fail(c, MC_E_INVALID_ARG, "eta[%d] must be finite and >= 0", i);
    c->eta_user.assign(eta, eta + n);
    c->tables_dirty = true;
    return MC_OK;
}

mc_status mc_project_range_async(mc_ctx *c, float beta, uint64_t first, uint64_t n,
                                 uint64_t seed, int64_t *d_prim, int64_t *d_scat, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!d_prim || !d_scat) return fail(c, MC_E_INVALID_ARG, "null image");
    mc_status rc = use_device(c);
    if (rc) return rc;
    KParams p;
    rc = prepare(c, beta, first, n, seed, p);
    if (rc) return rc;
    p.prim = (unsigned long long *)d_prim;
    p.scat = (unsigned long long *)d_scat;
    return run(c, p, (hipStream_t)stream, false);
}

mc_status mc_project_async(mc_ctx *c, float beta, uint64_t n, uint64_t seed, int64_t *d_prim,
                           int64_t *d_scat, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!d_prim || !d_scat) return fail(c, MC_E_INVALID_ARG, "null image");
    if (!c->have_geom) return fail(c, MC_E_STATE, "geometry not set");
    mc_status rc = use_device(c);
    if (rc) return rc;
    KParams p;
    rc = prepare(c, beta, 0, n, seed, p);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(c, hipMemsetAsync(d_prim, 0, (size_t)c->g.nu * c->g.nv * sizeof(int64_t), s));
    HIP_TRY(c, hipMemsetAsync(d_scat, 0, (size_t)c->g.snu * c->g.snv * sizeof(int64_t), s));
    p.prim = (unsigned long long *)d_prim;
    p.scat = (unsigned long long *)d_scat;
    return run(c, p, s, false);
}

mc_status mc_march_probe_async(mc_ctx *c, float beta, uint64_t n_rays, uint64_t seed,
                               int refill_batch, uint64_t *d_sum, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!d_sum) return fail(c, MC_E_INVALID_ARG, "null sum");
    if (refill_batch < 1 || refill_batch > 64)
        return fail(c, MC_E_INVALID_ARG, "refill_batch must be 1 .. 64");
    mc_status rc = use_device(c);
    if (rc) return rc;
    KParams p;
    rc = prepare(c, beta, 0, n_rays, seed, p);
    if (rc) return rc;
    if (n_rays == 0) return MC_OK;
    p.event_batch = refill_batch;
    p.stats = nullptr;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(c, hipMemsetAsync(p.counter, 0, sizeof(unsigned long long), s));
    // the probe's own occupancy (it uses no LDS) unless the caller fixed a shape
    const int block = c->block > 0 ? c->block : 256;
    const int bpc = c->blocks_per_cu > 0 ? c->blocks_per_cu
                                         : march_probe_blocks_per_cu(p.G.layout, block);
    const uint64_t need = (n_rays + block - 1) / block;
    const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)bpc * c->n_cu, need));
    hipError_t e = launch_march_probe(p, p.G.layout, grid, block, (unsigned long long *)d_sum, s);
    if (e != hipSuccess) return hip_fail(c, e, "march probe launch");
    return MC_OK;
}

mc_status mc_atomic_probe_async(mc_ctx *c, uint64_t n_adds, uint64_t seed, int64_t *d_image,
                                uint64_t n_pixels, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!d_image) return fail(c, MC_E_INVALID_ARG, "null image");
    if (n_pixels < 1 || n_pixels > 0xFFFFFFFFull)
        return fail(c, MC_E_INVALID_ARG, "n_pixels must be 1 .. 2^32 - 1");
    mc_status rc = use_device(c);
    if (rc) return rc;
    if (n_adds == 0) return MC_OK;
    const uint64_t need = (n_adds + 255) / 256;
    const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)8 * c->n_cu, need));
    hipError_t e = launch_atomic_probe((unsigned long long *)d_image, (uint32_t)n_pixels, n_adds,
                                       (uint32_t)seed ^ (uint32_t)(seed >> 32), grid,
                                       (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "atomic probe launch");
    return MC_OK;
}

mc_status mc_project(mc_ctx *c, float beta, uint64_t n, uint64_t seed, int64_t *prim,
                     int64_t *scat) {
    if (!c) return MC_E_INVALID_ARG;
    if (!prim || !scat) return fail(c, MC_E_INVALID_ARG, "null image");
    if (!c->have_geom) return fail(c, MC_E_STATE, "geometry not set");
    mc_status rc = use_device(c);
    if (rc) return rc;
    const size_t np = (size_t)c->g.nu * c->g.nv, ns = (size_t)c->g.snu * c->g.snv;
    if (np + ns > c->d_img_elems) {
        if (c->d_img) (void)hipFree(c->d_img);
        c->d_img = nullptr;
        c->d_img_elems = 0;
        HIP_TRY(c, hipMalloc(&c->d_img, (np + ns) * sizeof(int64_t)));
        c->d_img_elems = np + ns;
    }
    rc = mc_project_async(c, beta, n, seed, c->d_img, c->d_img + np, c->stream);
    if (rc) return rc;
    HIP_TRY(c, hipMemcpyAsync(prim, c->d_img, np * sizeof(int64_t), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(scat, c->d_img + np, ns * sizeof(int64_t), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (__atomic_load_n(c->h_cancel, __ATOMIC_SEQ_CST))
        return fail(c, MC_E_CANCELLED, "cancelled: the images hold the photons taken before it");
    return MC_OK;
}

mc_status mc_cancel(mc_ctx *c, int on) {
    if (!c) return MC_E_INVALID_ARG;
    if (!c->h_cancel) return fail(c, MC_E_STATE, "host-only context");
    __atomic_store_n(c->h_cancel, on ? 1 : 0, __ATOMIC_SEQ_CST);
    return MC_OK;
}

mc_status mc_project_batch(mc_ctx *c, const mc_job *jobs, int n_jobs, int64_t *d_out,
                           uint64_t out_elems, uint32_t flags, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (flags & ~MC_BATCH_GRAPH) return fail(c, MC_E_INVALID_ARG, "unknown batch flags");
    BatchPlan b;
    mc_status rc = plan_batch(c, jobs, n_jobs, d_out, out_elems, true, b);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (b.bytes > c->d_batch_bytes) {
        HIP_TRY(c, hipDeviceSynchronize());
        if (c->d_batch) (void)hipFree(c->d_batch);
        c->d_batch = nullptr;
        c->d_batch_bytes = 0;
        HIP_TRY(c, hipMalloc(&c->d_batch, b.bytes));
        c->d_batch_bytes = b.bytes;
        ++c->generation;
    }
    unsigned char *db = (unsigned char *)c->d_batch;
    if (!c->batch_done)
        HIP_TRY(c, hipEventCreateWithFlags(&c->batch_done, hipEventDisableTiming));
    else
        HIP_TRY(c, hipStreamWaitEvent(s, c->batch_done, 0));
    HIP_TRY(c, hipMemcpyAsync(db, b.host.data(), b.host.size(), hipMemcpyHostToDevice, s));
    KParams p;
    int grid, block;
    bool stats;
    batch_params(c, b, db, n_jobs, p, grid, block, stats);

    if (!(flags & MC_BATCH_GRAPH)) {
        hipError_t e = launch_clear((unsigned long long *)d_out, out_elems, p.job_counters,
                                    (size_t)n_jobs, s);
        if (e == hipSuccess) e = launch_batch(p, b.max_lane_pal, grid, block, stats, s);
        if (e != hipSuccess) return hip_fail(c, e, "batch launch");
        HIP_TRY(c, hipEventRecord(c->batch_done, s));
        return MC_OK;
    }
    // graph: clear kernel -> persistent transport kernel, captured once per
    // (buffers, shape, state) and replayed; the job table is uploaded above
    std::vector<unsigned char> key(sizeof(KParams) + 5 * sizeof(uint64_t));
    std::memcpy(key.data(), &p, sizeof p);
    // the captured clear kernel writes through d_out, so the buffer is part of the key
    const uint64_t extra[5] = {out_elems, (uint64_t)grid, (uint64_t)block,
                               ((uint64_t)c->generation << 8) | (uint64_t)b.max_lane_pal,
                               (uint64_t)(uintptr_t)d_out};
    std::memcpy(key.data() + sizeof p, extra, sizeof extra);
    if (!c->graph_exec || key != c->graph_key) {
        if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
        if (c->graph) (void)hipGraphDestroy(c->graph);
        c->graph_exec = nullptr;
        c->graph = nullptr;
        c->graph_key.clear();
        HIP_TRY(c, hipStreamSynchronize(s));
        HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = launch_clear((unsigned long long *)d_out, out_elems, p.job_counters,
                                    (size_t)n_jobs, c->stream);
        if (e == hipSuccess) e = launch_batch(p, b.max_lane_pal, grid, block, stats, c->stream);
        hipGraph_t gr = nullptr;
        const hipError_t e2 = hipStreamEndCapture(c->stream, &gr);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (gr) (void)hipGraphDestroy(gr);
            return hip_fail(c, e != hipSuccess ? e : e2, "batch graph capture");
        }
        c->graph = gr;
        HIP_TRY(c, hipGraphInstantiate(&c->graph_exec, gr, nullptr, nullptr, 0));
        c->graph_key = key;
    }
    HIP_TRY(c, hipGraphLaunch(c->graph_exec, s));
    HIP_TRY(c, hipEventRecord(c->batch_done, s));
    return MC_OK;
}

mc_status mc_project_batch_static(mc_ctx *c, const mc_job *jobs, int n_jobs, int64_t *d_out,
                                  uint64_t out_elems, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (n_jobs > MC_STATIC_MAX_JOBS)
        return fail(c, MC_E_INVALID_ARG, "at most %d jobs without allocation (got %d)",
                    MC_STATIC_MAX_JOBS, n_jobs);
    if ((int)c->phantoms.size() > MC_STATIC_MAX_PHANTOMS)
        return fail(c, MC_E_INVALID_ARG, "at most %d phantoms without allocation (context has %d)",
                    MC_STATIC_MAX_PHANTOMS, (int)c->phantoms.size());
    BatchPlan b;
    mc_status rc = plan_batch(c, jobs, n_jobs, d_out, out_elems, false, b);
    if (rc) return rc;
    unsigned char *db = nullptr;
    rc = static_scratch(c, &db);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(c, hipMemcpyAsync(db, b.host.data(), b.host.size(), hipMemcpyHostToDevice, s));
    KParams p;
    int grid, block;
    bool stats;
    batch_params(c, b, db, n_jobs, p, grid, block, stats);
    hipError_t e = launch_clear((unsigned long long *)d_out, out_elems, p.job_counters,
                                (size_t)n_jobs, s);
    if (e == hipSuccess) e = launch_batch(p, b.max_lane_pal, grid, block, stats, s);
    if (e != hipSuccess) return hip_fail(c, e, "static batch launch");
    return MC_OK;
}

mc_status mc_debug_histories(mc_ctx *c, float beta, uint64_t first, uint64_t m, uint64_t seed,
                             uint16_t *n_int, uint32_t *steps, uint8_t *end, uint8_t *first_t) {
    if (!c) return MC_E_INVALID_ARG;
    mc_status rc = use_device(c);
    if (rc) return rc;
    KParams p;
    rc = prepare(c, beta, first, m, seed, p);
    if (rc) return rc;
    if (m == 0) return MC_OK;
    // per-history records (8 bytes each) plus throwaway images
    const size_t np = (size_t)c->g.nu * c->g.nv, ns = (size_t)c->g.snu * c->g.snv;
    const size_t bytes = m * 8 + (np + ns) * 8;
    unsigned char *buf = nullptr;
    HIP_TRY(c, hipMalloc(&buf, bytes));
    hipStream_t s = c->stream;
    hipError_t e = hipMemsetAsync(buf, 0, bytes, s);
    if (e == hipSuccess) {
        p.prim = (unsigned long long *)buf;
        p.scat = p.prim + np;
        p.dbg_steps = (uint32_t *)(buf + (np + ns) * 8);
        p.dbg_nint = (uint16_t *)(buf + (np + ns) * 8 + m * 4);
        p.dbg_end = buf + (np + ns) * 8 + m * 6;
        p.dbg_first = buf + (np + ns) * 8 + m * 7;
        rc = run(c, p, s, true);
        if (!rc) {
            if (steps) e = hipMemcpyAsync(steps, p.dbg_steps, m * 4, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess && n_int)
                e = hipMemcpyAsync(n_int, p.dbg_nint, m * 2, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess && end)
                e = hipMemcpyAsync(end, p.dbg_end, m, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess && first_t)
                e = hipMemcpyAsync(first_t, p.dbg_first, m, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(c, e, "debug histories");
    return MC_OK;
}

mc_status mc_test_sample(mc_ctx *c, int process, int material, float e_kev, uint64_t n,
                         uint64_t seed, float *cos_out, float *e_out) {
    if (!c) return MC_E_INVALID_ARG;
    if (process < 0 || process > 3) return fail(c, MC_E_INVALID_ARG, "unknown process");
    if (n > ((uint64_t)1 << 31)) return fail(c, MC_E_INVALID_ARG, "n too large");
    mc_status rc = use_device(c);
    if (rc) return rc;
    KParams p;
    std::memset(&p, 0, sizeof p);
    const bool angular = process == MC_PROC_RAYLEIGH || process == MC_PROC_COMPTON;
    if (process == MC_PROC_SOURCE_ENERGY) {
        if (!c->have_spec || !e_out) return fail(c, MC_E_STATE, "spectrum not set");
        rc = refresh_tables(c);
        if (rc) return rc;
        p.e_bin = c->dp_ebin;
        p.thr = c->dp_thr;
        p.guide = c->dp_guide;
        p.n_bins = (int)c->e_bin.size();
    } else if (process == MC_PROC_SOURCE_DIR) {
        if (!cos_out) return fail(c, MC_E_INVALID_ARG, "null output");
        rc = prepare(c, 0.0f, 0, 0, seed, p);
        if (rc) return rc;
    } else if (material < 0 || material >= (int)c->mats.size() ||
               !(e_kev >= 1.0f && e_kev <= 1000.0f) || !cos_out) {
        return fail(c, MC_E_INVALID_ARG, "bad material/energy");
    }
    p.key0 = (uint32_t)seed;
    p.key1 = (uint32_t)(seed >> 32);
    if (n == 0) return MC_OK;
    // outputs, then the per-material Rayleigh and Compton-profile constants for
    // the samplers (with the context's binding effects)
    const size_t nm = c->mats.size();
    char *d = nullptr;
    HIP_TRY(c, hipMalloc(&d, n * 2 * sizeof(float) + 2 * nm * sizeof(double)));
    hipStream_t s = c->stream;
    double *d_rb = (double *)(d + n * 2 * sizeof(float));
    float *d_cos = (float *)d, *d_e = (float *)d + n;
    hipError_t e = hipSuccess;
    if (angular) {
        e = hipMemcpyAsync(d_rb, c->rayl_b.data(), nm * sizeof(double), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_rb + nm, c->pz_scale.data(), nm * sizeof(double),
                               hipMemcpyHostToDevice, s);
        p.rayl_b = d_rb;
        p.pz_scale = d_rb + nm;
        p.phys = c->phys;
    }
    if (e == hipSuccess) e = launch_sample(p, process, material, e_kev, n, d_cos, d_e, s);
    if (e == hipSuccess && cos_out && process != MC_PROC_SOURCE_ENERGY)
        e = hipMemcpyAsync(cos_out, d_cos, n * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && e_out && process != MC_PROC_SOURCE_DIR)
        e = hipMemcpyAsync(e_out, d_e, n * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipStreamSynchronize(s);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(c, e, "test sample");
    return MC_OK;
}

mc_status mc_set_stats(mc_ctx *c, int enable) {
    if (!c) return MC_E_INVALID_ARG;
    c->stats_on = enable != 0;
    return MC_OK;
}

mc_status mc_get_stats(mc_ctx *c, mc_stats *out) {
    if (!c || !out) return MC_E_INVALID_ARG;
    mc_status rc = use_device(c);
    if (rc) return rc;
    HIP_TRY(c, hipDeviceSynchronize());
    unsigned long long h[16];
    HIP_TRY(c, hipMemcpy(h, c->d_ctl + kRing, sizeof h, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemset(c->d_ctl + kRing, 0, sizeof h));
    out->histories = h[0]; out->steps = h[1]; out->flights = h[2];
    out->photo = h[3]; out->rayleigh = h[4]; out->compton = h[5];
    out->primary_hits = h[6]; out->scatter_hits = h[7];
    out->cutoff_kills = h[8]; out->cap_hits = h[9];
    out->skipped_steps = h[10];
    out->pd_scores = h[11];
    out->pd_killed = h[12];
    out->pd_steps = h[13];
    out->null_collisions = h[14];
    return MC_OK;
}

mc_status mc_primary_expected_async(mc_ctx *c, float beta, int sub, float *d_out, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!d_out) return fail(c, MC_E_INVALID_ARG, "null image");
    if (sub < 1 || sub > 64) return fail(c, MC_E_INVALID_ARG, "sub must be 1..64");
    mc_status rc = use_device(c);
    if (rc) return rc;
    KParams p;
    rc = prepare(c, beta, 0, 1, 0, p);
    if (rc) return rc;
    hipError_t e = launch_primary(p, sub, c->dp_bin_w, c->dp_bin_mu, (int)c->e_bin.size(), d_out,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "primary launch");
    return MC_OK;
}

mc_status mc_interp_angles_async(mc_ctx *c, const float *d_sim, int n_sim, uint64_t n_pix,
                                 float *d_full, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!d_sim || !d_full || n_sim < 1 || n_pix < 1)
        return fail(c, MC_E_INVALID_ARG, "need maps, n_sim >= 1 and n_pix >= 1");
    mc_status rc = use_device(c);
    if (rc) return rc;
    hipError_t e = launch_interp_angles(d_sim, n_sim, n_pix, d_full, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "interpolation launch");
    return MC_OK;
}

mc_status mc_line_integrals_async(mc_ctx *c, const float *d_I, uint64_t n, const float *d_I0,
                                  uint64_t n0, float *d_a, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!d_I || !d_I0 || !d_a || n0 < 1 || n < 1 || n % n0)
        return fail(c, MC_E_INVALID_ARG, "need buffers and n a multiple of n0 >= 1");
    mc_status rc = use_device(c);
    if (rc) return rc;
    hipError_t e = launch_line_integrals(d_I, n, d_I0, n0, d_a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "line integrals");
    return MC_OK;
}

mc_status mc_scatter_correct_async(mc_ctx *c, const float *d_a, const float *d_ip,
                                   const float *d_is, uint64_t n, float *d_c, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!d_a || !d_ip || !d_is || !d_c || n < 1) return fail(c, MC_E_INVALID_ARG, "bad buffers");
    mc_status rc = use_device(c);
    if (rc) return rc;
    hipError_t e = launch_scatter_correct(d_a, d_ip, d_is, n, d_c, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "scatter correction");
    return MC_OK;
}

mc_status mc_fdk_async(mc_ctx *c, const float *d_proj, int n_ang, float *d_tmp, float *d_vol,
                       int nx, int ny, int nz, float voxel_mm, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!c->have_geom) return fail(c, MC_E_STATE, "geometry not set");
    if (!d_proj || !d_tmp || !d_vol || n_ang < 1 || nx < 1 || ny < 1 || nz < 1 ||
        !(voxel_mm > 0.0f) || (int64_t)nx * ny * nz >= ((int64_t)1 << 31))
        return fail(c, MC_E_INVALID_ARG, "bad reconstruction arguments");
    // LDS: one panel row (fp64) per filter block, cos/sin of every angle per
    // backprojection block, 64 KiB each at most
    if (c->g.nu > 8192 || n_ang > 4096)
        return fail(c, MC_E_INVALID_ARG, "FDK supports nu <= 8192 and n_ang <= 4096");
    // every voxel strictly inside the source orbit (the distance weight's
    // L = R - x.s stays positive)
    const double hx = 0.5 * nx * (double)voxel_mm, hy = 0.5 * ny * (double)voxel_mm;
    if (!(sqrt(hx * hx + hy * hy) < 0.99 * (double)c->g.sod_mm))
        return fail(c, MC_E_INVALID_ARG, "volume reaches the source orbit");
    mc_status rc = use_device(c);
    if (rc) return rc;
    const mc_geometry &g = c->g;
    hipError_t e = launch_fdk(d_proj, g.sod_mm, g.sdd_mm, g.pu_mm, g.pv_mm, g.nu, g.nv, n_ang,
                              d_tmp, nx, ny, nz, voxel_mm, d_vol, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "fdk");
    return MC_OK;
}

mc_status mc_histogram_async(mc_ctx *c, const float *d_x, uint64_t n, float lo, float hi,
                             int bins, uint32_t *d_hist, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!d_x || !d_hist || bins < 1 || bins > 65536 || !(hi > lo))
        return fail(c, MC_E_INVALID_ARG, "bad histogram arguments");
    mc_status rc = use_device(c);
    if (rc) return rc;
    hipError_t e = launch_histogram(d_x, n, lo, hi, bins, d_hist, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "histogram");
    return MC_OK;
}

mc_status mc_to_density_async(mc_ctx *c, const float *d_mu, uint64_t n, float threshold,
                              float mu_rho, int material, float step, uint8_t *d_ids,
                              float *d_rho, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!d_mu || !d_ids || !d_rho || !(mu_rho > 0.0f) || !(step > 0.0f) || material < 1 ||
        material >= (int)c->mats.size())
        return fail(c, MC_E_INVALID_ARG, "bad density arguments");
    mc_status rc = use_device(c);
    if (rc) return rc;
    hipError_t e = launch_to_density(d_mu, n, threshold, mu_rho, material,
                                     (double)c->mats[0].rho_default, step, d_ids, d_rho,
                                     (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "to density");
    return MC_OK;
}

mc_status mc_set_physics(mc_ctx *c, uint32_t flags) {
    if (!c) return MC_E_INVALID_ARG;
    if (flags & ~(uint32_t)(MC_PHYS_INCOH_SF | MC_PHYS_DOPPLER))
        return fail(c, MC_E_INVALID_ARG, "unknown physics flags");
    c->phys = flags;
    ++c->generation;
    return MC_OK;
}

mc_status mc_set_estimator(mc_ctx *c, int mode, int split, double rr_kev) {
    if (!c) return MC_E_INVALID_ARG;
    if (mode != MC_SCORE_ANALOG && mode != MC_SCORE_POINT && mode != MC_SCORE_POINT_MIXED)
        return fail(c, MC_E_INVALID_ARG, "unknown estimator %d", mode);
    if (split < 1 || split > 1024) return fail(c, MC_E_INVALID_ARG, "split must be 1..1024");
    if (!(rr_kev >= 0.0) || !std::isfinite(rr_kev))
        return fail(c, MC_E_INVALID_ARG, "roulette threshold must be finite and >= 0");
    c->estimator = mode;
    c->pd_split = split;
    c->pd_rr = rr_kev;
    ++c->generation;
    return MC_OK;
}

mc_status mc_get_tables(mc_ctx *c, int *J, int *n_mat_out, float *pe, float *coh, float *inc,
                        float *eta) {
    if (!c || !J || !n_mat_out) return MC_E_INVALID_ARG;
    if (!c->have_spec) return fail(c, MC_E_STATE, "spectrum not set");
    const int n_mat = (int)c->mats.size();
    *n_mat_out = n_mat;
    std::vector<Material> mm(n_mat);
    for (int i = 0; i < n_mat; ++i) mm[i] = {c->mats[i].z_eff, c->mats[i].z_over_a};
    const int Jn = table_length(c->e_max);
    std::vector<float> a, b, cc, d;
    build_tables(mm.data(), n_mat, Jn, c->eta_user.empty() ? nullptr : c->eta_user.data(),
                 (int)c->eta_user.size(), a, b, cc, d);
    *J = Jn;
    if (pe) std::memcpy(pe, a.data(), a.size() * 4);
    if (coh) std::memcpy(coh, b.data(), b.size() * 4);
    if (inc) std::memcpy(inc, cc.data(), cc.size() * 4);
    if (eta) std::memcpy(eta, d.data(), d.size() * 4);
    return MC_OK;
}

mc_status mc_set_launch(mc_ctx *c, int block, int blocks_per_cu, int event_batch) {
    if (!c) return MC_E_INVALID_ARG;
    if (block != 0 && (block < 64 || block > 256 || block % 64))
        return fail(c, MC_E_INVALID_ARG, "block must be 64, 128, 192 or 256");
    if (blocks_per_cu < 0 || blocks_per_cu > 64 || event_batch < 0 || event_batch > 64)
        return fail(c, MC_E_INVALID_ARG, "bad launch shape");
    c->block = block;
    c->blocks_per_cu = blocks_per_cu;
    c->event_batch = event_batch;
    return MC_OK;
}

mc_status mc_set_batch_launch(mc_ctx *c, int block, int blocks_per_cu, int event_batch) {
    if (!c) return MC_E_INVALID_ARG;
    if (block != 0 && (block < 64 || block > 256 || block % 64))
        return fail(c, MC_E_INVALID_ARG, "block must be 64, 128, 192 or 256");
    if (blocks_per_cu < 0 || blocks_per_cu > 64 || event_batch < 0 || event_batch > 64)
        return fail(c, MC_E_INVALID_ARG, "bad launch shape");
    c->batch_block = block;
    c->batch_bpc = blocks_per_cu;
    c->batch_event_batch = event_batch;
    return MC_OK;
}

mc_status mc_get_batch_info(mc_ctx *c, int *n_phantoms, uint64_t *voxels, int *max_palette) {
    if (!c || !n_phantoms || !voxels || !max_palette) return MC_E_INVALID_ARG;
    *n_phantoms = 0;
    *voxels = 0;
    *max_palette = 0;
    for (const Phantom &ph : c->phantoms) {
        if (!ph.loaded) continue;
        ++*n_phantoms;
        *voxels += (uint64_t)ph.nx * ph.ny * ph.nz;
        *max_palette = std::max(*max_palette, ph.generic ? 256 : ph.n_pal);
    }
    return MC_OK;
}

mc_status mc_get_shape(mc_ctx *c, int *nx, int *ny, int *nz, int *nu, int *nv, int *snu,
                       int *snv) {
    if (!c || !nx || !ny || !nz || !nu || !nv || !snu || !snv) return MC_E_INVALID_ARG;
    if (!c->have_phantom || !c->have_geom) return fail(c, MC_E_STATE, "phantom and geometry must be set");
    const Phantom &ph = c->phantoms[0];
    *nx = ph.nx; *ny = ph.ny; *nz = ph.nz;
    *nu = c->g.nu; *nv = c->g.nv; *snu = c->g.snu; *snv = c->g.snv;
    return MC_OK;
}

mc_status mc_tally_to_float_async(mc_ctx *c, const int64_t *d_in, float *d_out, uint64_t n,
                                  double scale, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if ((!d_in || !d_out) && n) return fail(c, MC_E_INVALID_ARG, "null buffer");
    mc_status rc = use_device(c);
    if (rc) return rc;
    if (n == 0) return MC_OK;
    const hipError_t e = launch_tally_to_float(d_in, d_out, n, scale, (hipStream_t)stream);
    return e == hipSuccess ? MC_OK : hip_fail(c, e, "tally to float");
}

mc_status mc_savgol_async(mc_ctx *c, const float *d_in, float *d_out, float *d_tmp, int nx, int ny,
                          int window, int order, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!d_in || !d_out || !d_tmp || nx < 1 || ny < 1 || nx > 65536 || ny > 65535)
        return fail(c, MC_E_INVALID_ARG, "bad image");
    if (window < 1 || window > 31 || window % 2 == 0 || order < 0 || order >= window)
        return fail(c, MC_E_INVALID_ARG, "window must be odd, 1..31, and > order");
    float co[31];
    savgol_weights(window, order, co);
    mc_status rc = use_device(c);
    if (rc) return rc;
    const hipError_t e = launch_savgol(d_in, d_out, d_tmp, nx, ny, window, co, (hipStream_t)stream);
    return e == hipSuccess ? MC_OK : hip_fail(c, e, "savgol");
}

mc_status mc_upsample_cubic_async(mc_ctx *c, const float *d_in, float *d_out, int nx, int ny,
                                  int factor, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!d_in || !d_out || nx < 1 || ny < 1 || factor < 1 || factor > 16 ||
        (int64_t)nx * factor > 65536 || (int64_t)ny * factor > 65535)
        return fail(c, MC_E_INVALID_ARG, "bad image or factor");
    mc_status rc = use_device(c);
    if (rc) return rc;
    const hipError_t e = launch_upsample(d_in, d_out, nx, ny, factor, (hipStream_t)stream);
    return e == hipSuccess ? MC_OK : hip_fail(c, e, "cubic upsample");
}

mc_status mc_flip2d_async(mc_ctx *c, const float *d_in, float *d_out, int nx, int ny, int flip_x,
                          int flip_y, float alpha, float beta, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!d_in || !d_out || d_in == d_out || nx < 1 || ny < 1 || ny > 65535 || nx > (1 << 24) ||
        !std::isfinite(alpha) || !std::isfinite(beta))
        return fail(c, MC_E_INVALID_ARG, "flip: bad image (in and out must differ)");
    mc_status rc = use_device(c);
    if (rc) return rc;
    const hipError_t e =
        launch_flip2d(d_in, d_out, nx, ny, flip_x != 0, flip_y != 0, alpha, beta,
                      (hipStream_t)stream);
    return e == hipSuccess ? MC_OK : hip_fail(c, e, "flip");
}

mc_status mc_make_kramers(double kvp, double al_mm, double bin_keV, float *out_e, float *out_w,
                          int capacity, int *n_bins) {
    if (!n_bins || !(kvp > 1.0) || !(kvp <= 1000.0) || !(bin_keV > 0.0) || !(al_mm >= 0.0) ||
        !std::isfinite(al_mm) || !((kvp - 1.0) / bin_keV <= 1e6))
        return MC_E_INVALID_ARG;
    // bins [lo, lo + bin) from lo = 1 keV while lo < kVp, centres lo + bin/2
    const int n = (int)std::ceil((kvp - 1.0) / bin_keV);
    *n_bins = n;
    if (!out_e && !out_w) return MC_OK;          // size query
    if (!out_e || !out_w || capacity < n) return MC_E_INVALID_ARG;
    for (int i = 0; i < n; ++i) {
        const double e = (1.0 + (double)i * bin_keV) + 0.5 * bin_keV;
        // Kramers' (kVp - E)/E behind al_mm of aluminium (rho 2.699 g/cm^3,
        // mu/rho ~ 26583/E^3 + 0.1434 cm^2/g: a fit that only shapes an input)
        const double mu_rho = 26583.0 / (e * e * e) + 0.1434;
        const double w = (kvp - e) / e * std::exp(-mu_rho * 2.699 * (al_mm / 10.0));
        out_e[i] = (float)e;
        out_w[i] = e < kvp ? (float)w : 0.0f;
    }
    return MC_OK;
}

mc_status mc_savgol_weights(int window, int order, float *weights) {
    if (!weights || window < 1 || window > 31 || window % 2 == 0 || order < 0 || order >= window)
        return MC_E_INVALID_ARG;
    savgol_weights(window, order, weights);
    return MC_OK;
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

#define NN_RUN(c, expr, what)                                                 \
    do {                                                                      \
        mc_status rc_ = use_device(c);                                        \
        if (rc_) return rc_;                                                  \
        const hipError_t e_ = (expr);                                         \
        return e_ == hipSuccess ? MC_OK : hip_fail(c, e_, what);              \
    } while (0)

mc_status mc_nn_conv3x3_async(mc_ctx *c, const mc_conv3x3 *a, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!a || !a->x || !a->w || (!a->y && !a->yf)) return fail(c, MC_E_INVALID_ARG, "null buffer");
    if (a->n < 1 || a->h < 1 || a->w_ < 1 || a->cin < 16 || a->cin % 16 || a->cout < 1 ||
        (int64_t)a->n * a->h * a->w_ >= ((int64_t)1 << 31))
        return fail(c, MC_E_INVALID_ARG, "conv: bad shape (cin must be a multiple of 16)");
    if (a->ldx % 16 || a->xoff % 16 || a->xoff + a->cin > a->ldx || !aligned16(a->x) ||
        !aligned16(a->w))
        return fail(c, MC_E_INVALID_ARG, "conv: input slice must be 16-channel aligned");
    if (a->y && (a->yoff < 0 || a->yoff + a->cout > a->ldy))
        return fail(c, MC_E_INVALID_ARG, "conv: output slice outside its buffer");
    if (a->mask && (a->moff < 0 || a->moff + a->cout > a->ldm))
        return fail(c, MC_E_INVALID_ARG, "conv: mask slice outside its buffer");
    ConvArgs k;
    k.x = a->x; k.ldx = a->ldx; k.xoff = a->xoff; k.w = a->w; k.bias = a->bias;
    k.y = a->y; k.ldy = a->ldy; k.yoff = a->yoff; k.yf = a->yf;
    k.mask = a->mask; k.ldm = a->ldm; k.moff = a->moff;
    k.n = a->n; k.h = a->h; k.w_ = a->w_; k.cin = a->cin; k.cout = a->cout;
    k.relu = a->relu; k.accumulate = a->accumulate;
    NN_RUN(c, nn_conv3x3(k, (hipStream_t)stream), "conv3x3");
}

mc_status mc_nn_conv3x3_wgrad_async(mc_ctx *c, const uint16_t *x, int ldx, int xoff,
                                    const uint16_t *dy, int ldy, int yoff, int n, int h, int w,
                                    int cin, int cout, int splits, float *ws, float *dw,
                                    void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!x || !dy || !ws || !dw || n < 1 || h < 1 || w < 1 || cin < 16 || cin % 16 ||
        cout < 16 || cout % 16 || splits < 1 || splits > 4096 ||
        (int64_t)n * h * w >= ((int64_t)1 << 30))
        return fail(c, MC_E_INVALID_ARG,
                    "wgrad: bad arguments (cin, cout multiples of 16; under 2^30 pixels)");
    if (ldx % 16 || xoff % 16 || xoff + cin > ldx || yoff + cout > ldy || !aligned16(x))
        return fail(c, MC_E_INVALID_ARG, "wgrad: bad slices");
    WgradArgs k;
    k.x = x; k.ldx = ldx; k.xoff = xoff; k.dy = dy; k.ldy = ldy; k.yoff = yoff;
    k.n = n; k.h = h; k.w_ = w; k.cin = cin; k.cout = cout; k.splits = splits;
    k.partial = ws;
    float *tmp = ws + (size_t)splits * 9 * cout * cin;
    NN_RUN(c, nn_wgrad(k, tmp, dw, (hipStream_t)stream), "wgrad");
}

mc_status mc_nn_bias_grad_async(mc_ctx *c, const uint16_t *dy, int ldy, int yoff, int npix, int ch,
                                float *ws, int rows, float *db, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!dy || !ws || !db || npix < 1 || ch < 1 || rows < 1 || rows > 65535 || yoff + ch > ldy)
        return fail(c, MC_E_INVALID_ARG, "bias grad: bad arguments");
    NN_RUN(c, nn_colsum(dy, ldy, yoff, npix, ch, ws, rows, db, (hipStream_t)stream), "bias grad");
}

mc_status mc_nn_flip_weights_async(mc_ctx *c, const uint16_t *w, uint16_t *wt, int cout, int cin,
                                   int cout_pad, int cin_pad, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!w || !wt || cout < 1 || cin < 1 || cout_pad < cout || cin_pad < cin)
        return fail(c, MC_E_INVALID_ARG, "flip: bad arguments");
    NN_RUN(c, nn_flip(w, wt, cout, cin, cout_pad, cin_pad, (hipStream_t)stream), "flip weights");
}

static mc_status resample(mc_ctx *c, int op, const uint16_t *x, int ldx, int xoff, uint16_t *y,
                          int ldy, int yoff, int n, int h, int w, int ch, int backward,
                          int accumulate, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!x || !y || n < 1 || h < 1 || w < 1 || ch < 1 || xoff + ch > ldx || yoff + ch > ldy ||
        (op == 0 && (h % 2 || w % 2)))
        return fail(c, MC_E_INVALID_ARG, "resample: bad arguments");
    NN_RUN(c, nn_resample(op, x, ldx, xoff, y, ldy, yoff, n, h, w, ch, backward, accumulate,
                          (hipStream_t)stream),
           "resample");
}

mc_status mc_nn_pool2_async(mc_ctx *c, const uint16_t *x, int ldx, int xoff, uint16_t *y, int ldy,
                            int yoff, int n, int h, int w, int ch, int backward, int accumulate,
                            void *stream) {
    return resample(c, 0, x, ldx, xoff, y, ldy, yoff, n, h, w, ch, backward, accumulate, stream);
}

mc_status mc_nn_upsample2_async(mc_ctx *c, const uint16_t *x, int ldx, int xoff, uint16_t *y,
                                int ldy, int yoff, int n, int h, int w, int ch, int backward,
                                int accumulate, void *stream) {
    return resample(c, 1, x, ldx, xoff, y, ldy, yoff, n, h, w, ch, backward, accumulate, stream);
}

mc_status mc_nn_mse_async(mc_ctx *c, const float *out, int ldo, const float *target, uint64_t n,
                          uint16_t *grad, int ldg, int goff, float gscale, float *partial,
                          void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!out || !target || !partial || n == 0 || ldo < 1 || (grad && (goff < 0 || goff >= ldg)))
        return fail(c, MC_E_INVALID_ARG, "mse: bad arguments");
    NN_RUN(c, nn_mse(out, ldo, target, (int64_t)n, grad, ldg, goff, gscale, partial,
                     (hipStream_t)stream),
           "mse");
}

mc_status mc_nn_adam_async(mc_ctx *c, float *p, const float *g, float *m, float *v,
                           uint16_t *pb, uint64_t n, float lr, float b1, float b2, float eps,
                           int step, float gscale, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!p || !g || !m || !v || step < 1 || !(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f))
        return fail(c, MC_E_INVALID_ARG, "adam: bad arguments");
    const float c1 = (float)(1.0 - std::pow((double)b1, step));
    const float c2 = (float)(1.0 - std::pow((double)b2, step));
    NN_RUN(c, nn_adam(p, g, m, v, pb, (int64_t)n, lr, b1, b2, eps, c1, c2, gscale,
                      (hipStream_t)stream),
           "adam");
}

mc_status mc_nn_relu_mask_async(mc_ctx *c, uint16_t *g, int ldg, int goff, const uint16_t *y,
                                int ldy, int yoff, uint64_t npix, int ch, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!g || !y || ch < 1 || goff + ch > ldg || yoff + ch > ldy)
        return fail(c, MC_E_INVALID_ARG, "relu mask: bad arguments");
    NN_RUN(c, nn_relu_mask(g, ldg, goff, y, ldy, yoff, (int64_t)npix, ch, (hipStream_t)stream),
           "relu mask");
}

mc_status mc_nn_cast_bf16_async(mc_ctx *c, const float *in, uint16_t *out, uint64_t n,
                                void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!in || !out) return fail(c, MC_E_INVALID_ARG, "cast: null buffer");
    NN_RUN(c, nn_cast_bf16(in, out, (int64_t)n, (hipStream_t)stream), "cast bf16");
}

mc_status mc_nn_pack_channel_async(mc_ctx *c, const float *in, uint64_t npix, float scale,
                                   uint16_t *out, int ld, int coff, void *stream) {
    if (!c) return MC_E_INVALID_ARG;
    if (!in || !out || coff < 0 || coff >= ld) return fail(c, MC_E_INVALID_ARG, "pack: bad arguments");
    NN_RUN(c, nn_pack_channel(in, (int64_t)npix, scale, out, ld, coff, (hipStream_t)stream),
           "pack channel");
}

double mc_tally_scale(void) { return 1.0 / 1048576.0; }

}  // extern "C"
