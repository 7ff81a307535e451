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
#include <new>
#include <string>
#include <vector>

#include "../../include/mcx.h"
#include "kernel_params.hpp"
#include "tables.hpp"

namespace mcx {
hipError_t launch_transport(const KParams &p, int grid, int block, bool stats, bool debug,
                            hipStream_t stream);
hipError_t launch_sample(const KParams &p, int process, int material, float e_kev, uint64_t n,
                         float *cos_out, float *e_out, hipStream_t stream);
int transport_blocks_per_cu(int block, int n_mat, bool stats);
}  // namespace mcx

using namespace mcx;

namespace {
constexpr int kRing = 64;
constexpr int kCtlWords = kRing + 16;
}  // namespace

struct mc_ctx {
    int device = 0;
    int n_cu = 256;
    hipStream_t stream = nullptr;        // for the blocking entry points
    char err[512] = {0};

    std::vector<mc_material> mats;
    std::vector<double> rayl_b;

    // phantom
    int nx = 0, ny = 0, nz = 0;
    float h = 0.0f;
    int max_id = 0;
    uint8_t *d_ids = nullptr;
    float *d_rho = nullptr;
    bool have_phantom = false;

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
    const double *dp_rb = nullptr;

    // control block: [0, kRing) photon counters, one per launch in turn so
    // launches queued on different streams never share one; then statistics
    unsigned long long *d_ctl = nullptr;
    unsigned launches = 0;
    bool stats_on = false;

    // staging for mc_project
    int64_t *d_img = nullptr;
    size_t d_img_elems = 0;

    int block = 0, blocks_per_cu = 0, steps_per_round = 0;
};

namespace {

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
    c->mats.assign(m, m + n);
    c->rayl_b.resize(n);
    for (int i = 0; i < n; ++i) c->rayl_b[i] = rayleigh_b(m[i].z_eff);
    c->tables_dirty = true;
}

mc_status use_device(mc_ctx *c) {
    if (c->device < 0) return fail(c, MC_E_STATE, "host-only context (device -1) cannot run kernels");
    HIP_TRY(c, hipSetDevice(c->device));
    return MC_OK;
}

// Regenerate host tables and upload them (synchronises the device first so
// no queued kernel still reads the old blob).
mc_status refresh_tables(mc_ctx *c) {
    if (!c->tables_dirty) return MC_OK;
    const int n_mat = (int)c->mats.size();
    std::vector<Material> mm(n_mat);
    for (int i = 0; i < n_mat; ++i) mm[i] = {c->mats[i].z_eff, c->mats[i].z_over_a};
    const int J = table_length(c->e_max);
    build_tables(mm.data(), n_mat, J, c->eta_user.empty() ? nullptr : c->eta_user.data(),
                 (int)c->eta_user.size(), c->pe, c->coh, c->inc, c->eta);
    c->J = J;
    // blob: rb[n_mat] f64 | thr[n_bins] u64 | pe | coh | inc [n_mat*J] | eta[J] | e_bin[n_bins]
    const size_t nb = c->e_bin.size();
    const size_t tab = (size_t)n_mat * J;
    const size_t bytes = n_mat * 8 + nb * 8 + (3 * tab + J + nb) * 4;
    std::vector<unsigned char> blob(bytes);
    size_t off = 0;
    auto put = [&](const void *src, size_t n) {
        std::memcpy(blob.data() + off, src, n);
        off += n;
    };
    put(c->rayl_b.data(), n_mat * 8);
    put(c->thr.data(), nb * 8);
    put(c->pe.data(), tab * 4);
    put(c->coh.data(), tab * 4);
    put(c->inc.data(), tab * 4);
    put(c->eta.data(), (size_t)J * 4);
    put(c->e_bin.data(), nb * 4);
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
    c->dp_thr = (const uint64_t *)(b + n_mat * 8);
    const float *f = (const float *)(b + n_mat * 8 + nb * 8);
    c->dp_pe = f;
    c->dp_coh = f + tab;
    c->dp_inc = f + 2 * tab;
    c->dp_eta = f + 3 * tab;
    c->dp_ebin = f + 3 * tab + J;
    c->tables_dirty = false;
    return MC_OK;
}

// Every precondition of a projection of n photons; fills the kernel params.
mc_status prepare(mc_ctx *c, float beta, uint64_t first, uint64_t n, uint64_t seed,
                  KParams &p) {
    if (!c->have_phantom || !c->have_geom || !c->have_spec)
        return fail(c, MC_E_STATE, "phantom, geometry and spectrum must be set");
    if (!std::isfinite(beta)) return fail(c, MC_E_INVALID_ARG, "angle must be finite");
    if (c->max_id >= (int)c->mats.size())
        return fail(c, MC_E_INVALID_ARG, "material id %d >= n_mat %d", c->max_id,
                    (int)c->mats.size());
    const double hx = 0.5 * c->nx * c->h, hy = 0.5 * c->ny * c->h, hz = 0.5 * c->nz * c->h;
    const double diag = std::sqrt(hx * hx + hy * hy + hz * hz);
    if (!(diag < c->g.sod_mm) || !(diag < (double)c->g.sdd_mm - c->g.sod_mm))
        return fail(c, MC_E_INVALID_ARG, "phantom must lie strictly between source and panel");
    if (2.0 * diag / c->g.step_mm > 4194304.0)
        return fail(c, MC_E_INVALID_ARG, "step too small for the phantom");
    if (first + n < first) return fail(c, MC_E_INVALID_ARG, "photon range wraps");
    mc_status rc = refresh_tables(c);
    if (rc) return rc;
    float eta_max = 0.0f;
    for (float v : c->eta) eta_max = std::max(eta_max, v);
    if ((long double)(first + n) * ((long double)eta_max * 1048576.0L + 1.0L) >=
        9223372036854775807.0L)
        return fail(c, MC_E_OVERFLOW, "tally could overflow int64");

    std::memset(&p, 0, sizeof p);
    p.ids = c->d_ids;
    p.rho = c->d_rho;
    p.nx = c->nx; p.ny = c->ny; p.nz = c->nz;
    p.inv_h = 1.0f / c->h;
    const int nd[3] = {c->nx, c->ny, c->nz};
    for (int a = 0; a < 3; ++a) {
        p.hi[a] = 0.5f * ((float)nd[a] * c->h);
        p.lo[a] = -p.hi[a];
    }
    p.pe = c->dp_pe; p.coh = c->dp_coh; p.inc = c->dp_inc; p.eta = c->dp_eta;
    p.J = c->J;
    p.n_mat = (int)c->mats.size();
    p.rayl_b = c->dp_rb;
    p.e_bin = c->dp_ebin;
    p.thr = c->dp_thr;
    p.n_bins = (int)c->e_bin.size();
    // projection frame
    const mc_geometry &g = c->g;
    const float cb = (float)std::cos((double)beta), sb = (float)std::sin((double)beta);
    ProjFrame &F = p.F;
    F.S[0] = g.sod_mm * cb; F.S[1] = g.sod_mm * sb; F.S[2] = 0.0f;
    F.ax[0] = -cb; F.ax[1] = -sb; F.ax[2] = 0.0f;
    F.eu[0] = -sb; F.eu[1] = cb; F.eu[2] = 0.0f;
    F.ev[0] = 0.0f; F.ev[1] = 0.0f; F.ev[2] = 1.0f;
    for (int a = 0; a < 3; ++a) F.D[a] = F.S[a] + g.sdd_mm * F.ax[a];
    F.hu = 0.5f * ((float)g.nu * g.pu_mm);
    F.hv = 0.5f * ((float)g.nv * g.pv_mm);
    const double sdd = g.sdd_mm, hu = F.hu, hv = F.hv;
    F.omc = (float)(1.0 - sdd / std::sqrt(sdd * sdd + hu * hu + hv * hv));
    p.sdd = g.sdd_mm; p.pu = g.pu_mm; p.pv = g.pv_mm; p.step = g.step_mm;
    p.nu = g.nu; p.nv = g.nv; p.snu = g.snu; p.snv = g.snv;
    p.bu = g.nu / g.snu; p.bv = g.nv / g.snv;
    p.flags = g.flags;
    p.first = first;
    p.n = n;
    p.key0 = (uint32_t)seed;
    p.key1 = (uint32_t)(seed >> 32);
    p.steps_per_round = c->steps_per_round > 0 ? c->steps_per_round : 64;
    p.counter = c->d_ctl + (c->launches++ % kRing);
    p.stats = c->d_ctl + kRing;
    return MC_OK;
}

void launch_shape(mc_ctx *c, uint64_t n, bool stats, int &grid, int &block) {
    block = c->block > 0 ? c->block : 256;
    int bpc = c->blocks_per_cu > 0 ? c->blocks_per_cu
                                   : transport_blocks_per_cu(block, (int)c->mats.size(), stats);
    uint64_t full = (uint64_t)bpc * c->n_cu;
    uint64_t need = (n + block - 1) / block;
    grid = (int)std::max<uint64_t>(1, std::min(full, need));
}

mc_status run(mc_ctx *c, KParams &p, hipStream_t s, bool debug) {
    if (p.n == 0) return MC_OK;
    HIP_TRY(c, hipMemsetAsync(p.counter, 0, sizeof(unsigned long long), s));
    int grid, block;
    launch_shape(c, p.n, c->stats_on && !debug, grid, block);
    if (!c->stats_on || debug) p.stats = nullptr;
    hipError_t e = launch_transport(p, grid, block, c->stats_on && !debug, debug, s);
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
        hipMemset(c->d_ctl, 0, kCtlWords * sizeof(unsigned long long)) != hipSuccess)
        rc = MC_E_DEVICE;
    if (rc) {
        mc_destroy(c);
        return rc;
    }
    c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
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
    if (c->d_ids) (void)hipFree(c->d_ids);
    if (c->d_rho) (void)hipFree(c->d_rho);
    if (c->d_tables) (void)hipFree(c->d_tables);
    if (c->d_ctl) (void)hipFree(c->d_ctl);
    if (c->d_img) (void)hipFree(c->d_img);
    if (c->stream) (void)hipStreamDestroy(c->stream);
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

mc_status mc_load_phantom(mc_ctx *c, const uint8_t *ids, const float *rho, int nx, int ny,
                          int nz, float h) {
    if (!c) return MC_E_INVALID_ARG;
    if (!ids || !rho || nx < 1 || ny < 1 || nz < 1 || nx > 4096 || ny > 4096 || nz > 4096 ||
        !(h > 0.0f) || !std::isfinite(h))
        return fail(c, MC_E_INVALID_ARG, "bad phantom dimensions");
    const size_t nv = (size_t)nx * ny * nz;
    if (nv >= (size_t)1 << 31) return fail(c, MC_E_INVALID_ARG, "phantom must have < 2^31 voxels");
    int max_id = 0;
    for (size_t i = 0; i < nv; ++i) {
        const float r = rho[i];
        if (!std::isfinite(r) || r < 0.0f || r > 1000.0f)
            return fail(c, MC_E_INVALID_ARG, "density at %zu must be finite and in [0, 1000]", i);
        max_id = std::max<int>(max_id, ids[i]);
    }
    mc_status rc = use_device(c);
    if (rc) return rc;
    HIP_TRY(c, hipDeviceSynchronize());
    if (c->d_ids) (void)hipFree(c->d_ids);
    if (c->d_rho) (void)hipFree(c->d_rho);
    c->d_ids = nullptr;
    c->d_rho = nullptr;
    c->have_phantom = false;
    HIP_TRY(c, hipMalloc(&c->d_ids, nv));
    HIP_TRY(c, hipMalloc(&c->d_rho, nv * sizeof(float)));
    HIP_TRY(c, hipMemcpy(c->d_ids, ids, nv, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_rho, rho, nv * sizeof(float), hipMemcpyHostToDevice));
    c->nx = nx; c->ny = ny; c->nz = nz; c->h = h;
    c->max_id = max_id;
    c->have_phantom = true;
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
    // outputs, then the per-material Rayleigh constants for the samplers
    const size_t nm = c->mats.size();
    char *d = nullptr;
    HIP_TRY(c, hipMalloc(&d, n * 2 * sizeof(float) + nm * sizeof(double)));
    hipStream_t s = c->stream;
    double *d_rb = (double *)(d + n * 2 * sizeof(float));
    float *d_cos = (float *)d, *d_e = (float *)d + n;
    hipError_t e = hipSuccess;
    if (angular) {
        e = hipMemcpyAsync(d_rb, c->rayl_b.data(), nm * sizeof(double), hipMemcpyHostToDevice, s);
        p.rayl_b = d_rb;
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
    return MC_OK;
}

mc_status mc_get_tables(mc_ctx *c, int *J, float *pe, float *coh, float *inc, float *eta) {
    if (!c || !J) return MC_E_INVALID_ARG;
    if (!c->have_spec) return fail(c, MC_E_STATE, "spectrum not set");
    const int n_mat = (int)c->mats.size();
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

mc_status mc_set_launch(mc_ctx *c, int block, int blocks_per_cu, int steps_per_round) {
    if (!c) return MC_E_INVALID_ARG;
    if (block != 0 && (block < 64 || block > 256 || block % 64))
        return fail(c, MC_E_INVALID_ARG, "block must be 64, 128, 192 or 256");
    if (blocks_per_cu < 0 || blocks_per_cu > 64 || steps_per_round < 0 || steps_per_round > 4096)
        return fail(c, MC_E_INVALID_ARG, "bad launch shape");
    c->block = block;
    c->blocks_per_cu = blocks_per_cu;
    c->steps_per_round = steps_per_round;
    return MC_OK;
}

double mc_tally_scale(void) { return 1.0 / 1048576.0; }

}  // extern "C"
