// Launch-shape autotuners for the transport kernel (single projections and
// batches), written against the public C ABI only (plus HIP events for timing).
//
// Knobs: threads per block, resident blocks per compute unit, the event batch
// and, for palette objects small enough for per-lane tables, the attenuation-
// table layout (per-lane tables of every palette entry, or the shared palette
// with per-lane tables per material).  None of them changes a photon's
// history, so every candidate must
// reproduce the first candidate's images bit for bit; a candidate that does
// not is rejected (and reported), never chosen.  The winner is applied to the
// context and, when a cache path is given, appended to a JSON-lines cache
// keyed by device architecture and workload class.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mcx.h"

namespace {

struct Shape {
    int block, bpc, batch, table;
};

std::string workload_key(mc_ctx *ctx, int nx, int ny, int nz, int n_pixels) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    const size_t sp = arch.find(':');
    if (sp != std::string::npos) arch = arch.substr(0, sp);
    int layout = 0, npal = 0;
    (void)mc_get_layout(ctx, &layout, &npal);
    const double vox = (double)nx * ny * nz;
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s/vox2^%d/pix2^%d/%s/pal%d", arch.c_str(),
                  (int)std::lround(std::log2(std::max(vox, 1.0))),
                  (int)std::lround(std::log2(std::max(n_pixels, 1))),
                  layout == MC_LAYOUT_GENERIC ? "generic" : "palette",
                  npal <= 8 ? 8 : (npal <= 32 ? 32 : 256));
    return buf;
}

// the table layout of a candidate as a layout request: per-lane tables are
// what the automatic choice gives palettes of <= 32 entries; an object stored
// with material ids and densities keeps the request it has
mc_status apply_table(mc_ctx *ctx, int table) {
    if (table == MC_LAYOUT_GENERIC) return MC_OK;
    return mc_set_layout(ctx, table == MC_LAYOUT_PALETTE_LANE ? MC_LAYOUT_AUTO : table);
}

bool read_cache(const char *path, const std::string &key, Shape &s) {
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[256];
        Shape t;
        if (std::sscanf(line, "{\"key\": \"%255[^\"]\", \"block\": %d, \"blocks_per_cu\": %d, "
                              "\"event_batch\": %d, \"table_layout\": %d",
                        k, &t.block, &t.bpc, &t.batch, &t.table) == 5 &&
            key == k) {
            s = t;          // the last entry for a key wins
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

std::string arch_name() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    const size_t sp = arch.find(':');
    if (sp != std::string::npos) arch = arch.substr(0, sp);
    return arch;
}

int log2i(double v) { return (int)std::lround(std::log2(std::max(v, 1.0))); }

}  // namespace

extern "C" {

mc_status mc_autotune(mc_ctx *ctx, float angle_rad, uint64_t n_photons, uint64_t seed,
                      const char *cache_path, mc_tuning *out) {
    if (!ctx || !out || n_photons == 0) return MC_E_INVALID_ARG;
    std::memset(out, 0, sizeof *out);
    int nx = 0, ny = 0, nz = 0, nu = 0, nv = 0, snu = 0, snv = 0;
    mc_status rc = mc_get_shape(ctx, &nx, &ny, &nz, &nu, &nv, &snu, &snv);
    if (rc) return rc;
    const std::string key = workload_key(ctx, nx, ny, nz, nu * nv);
    Shape cached;
    if (read_cache(cache_path, key, cached)) {
        rc = mc_set_launch(ctx, cached.block, cached.bpc, cached.batch);
        if (rc) return rc;
        rc = apply_table(ctx, cached.table);
        if (rc) return rc;
        out->block = cached.block;
        out->blocks_per_cu = cached.bpc;
        out->event_batch = cached.batch;
        out->table_layout = cached.table;
        out->from_cache = 1;
        return MC_OK;
    }
    const size_t np = (size_t)nu * nv, ns = (size_t)snu * snv;
    int64_t *d = nullptr;
    if (hipMalloc(&d, 2 * (np + ns) * sizeof(int64_t)) != hipSuccess) return MC_E_OOM;
    hipStream_t stream = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipFree(d);
        return MC_E_DEVICE;
    }
    int64_t *ref = d, *cur = d + np + ns;
    // the table layouts open to this object: both palette forms when per-lane
    // tables fit (<= 32 entries), else the one it has
    int layout = 0, npal = 0;
    rc = mc_get_layout(ctx, &layout, &npal);
    if (rc) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipStreamDestroy(stream);
        (void)hipFree(d);
        return rc;
    }
    std::vector<int> tables{layout};
    if (layout != MC_LAYOUT_GENERIC && npal <= 32)
        tables = {MC_LAYOUT_PALETTE_LANE, MC_LAYOUT_PALETTE_SHARED};
    std::vector<Shape> cands;
    for (int table : tables)
        for (int block : {64, 128, 256})
            for (int bpc : {0, 2})
                for (int batch : {36, 40, 44, 48, 52, 58}) cands.push_back({block, bpc, batch, table});
    std::vector<int64_t> h_ref(np + ns), h_cur(np + ns);
    Shape best{0, 0, 0, layout};
    float best_ms = 1e30f;
    int rejected = 0, tried = 0;
    for (size_t i = 0; i < cands.size() && rc == MC_OK; ++i) {
        const Shape &s = cands[i];
        rc = mc_set_launch(ctx, s.block, s.bpc, s.batch);
        if (rc) break;
        rc = apply_table(ctx, s.table);
        if (rc) break;
        int64_t *img = i == 0 ? ref : cur;
        // one warm-up run (also the output checked), then the timed one
        rc = mc_project_async(ctx, angle_rad, n_photons, seed, img, img + np, stream);
        if (rc) break;
        (void)hipEventRecord(e0, stream);
        rc = mc_project_async(ctx, angle_rad, n_photons, seed, img, img + np, stream);
        if (rc) break;
        (void)hipEventRecord(e1, stream);
        if (hipEventSynchronize(e1) != hipSuccess) {
            rc = MC_E_DEVICE;
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ++tried;
        if (i == 0) {
            (void)hipMemcpy(h_ref.data(), ref, (np + ns) * sizeof(int64_t), hipMemcpyDeviceToHost);
        } else {
            (void)hipMemcpy(h_cur.data(), cur, (np + ns) * sizeof(int64_t), hipMemcpyDeviceToHost);
            if (h_cur != h_ref) {
                ++rejected;
                continue;
            }
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = s;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(stream);
    (void)hipFree(d);
    if (rc) {
        (void)apply_table(ctx, layout);
        return rc;
    }
    rc = mc_set_launch(ctx, best.block, best.bpc, best.batch);
    if (rc) return rc;
    rc = apply_table(ctx, best.table);
    if (rc) return rc;
    out->block = best.block;
    out->blocks_per_cu = best.bpc;
    out->event_batch = best.batch;
    out->table_layout = best.table;
    out->ms = best_ms;
    out->histories_per_s = best_ms > 0.0f ? (double)n_photons / (best_ms * 1e-3) : 0.0;
    out->candidates = tried;
    out->rejected = rejected;
    if (cache_path) {
        FILE *f = std::fopen(cache_path, "a");
        if (f) {
            std::fprintf(f,
                         "{\"key\": \"%s\", \"block\": %d, \"blocks_per_cu\": %d, "
                         "\"event_batch\": %d, \"table_layout\": %d, \"ms\": %.4f, "
                         "\"photons\": %llu, \"candidates\": %d, \"rejected\": %d}\n",
                         key.c_str(), best.block, best.bpc, best.batch, best.table, best_ms,
                         (unsigned long long)n_photons, tried, rejected);
            std::fclose(f);
        }
    }
    return MC_OK;
}

}  // extern "C"

extern "C" {

mc_status mc_autotune_batch(mc_ctx *ctx, const mc_job *jobs, int n_jobs, int64_t *d_out,
                            uint64_t out_elems, const char *cache_path, mc_tuning *out) {
    if (!ctx || !out || !jobs || n_jobs < 1 || !d_out || out_elems == 0) return MC_E_INVALID_ARG;
    std::memset(out, 0, sizeof *out);
    int nx = 0, ny = 0, nz = 0, nu = 0, nv = 0, snu = 0, snv = 0;
    mc_status rc = mc_get_shape(ctx, &nx, &ny, &nz, &nu, &nv, &snu, &snv);
    if (rc) return rc;
    int n_obj = 0, max_pal = 0;
    uint64_t voxels = 0;
    rc = mc_get_batch_info(ctx, &n_obj, &voxels, &max_pal);
    if (rc) return rc;
    uint64_t photons = 0;
    for (int j = 0; j < n_jobs; ++j) photons += jobs[j].n_photons;
    char kbuf[256];
    std::snprintf(kbuf, sizeof kbuf, "batch/%s/jobs2^%d/vox2^%d/pix2^%d/pal%d",
                  arch_name().c_str(), log2i(n_jobs), log2i((double)voxels), log2i((double)nu * nv),
                  max_pal <= 8 ? 8 : (max_pal <= 32 ? 32 : 256));
    const std::string key = kbuf;
    Shape cached;
    if (read_cache(cache_path, key, cached)) {
        rc = mc_set_batch_launch(ctx, cached.block, cached.bpc, cached.batch);
        if (rc) return rc;
        rc = apply_table(ctx, cached.table);
        if (rc) return rc;
        out->block = cached.block;
        out->blocks_per_cu = cached.bpc;
        out->event_batch = cached.batch;
        out->table_layout = cached.table;
        out->from_cache = 1;
        return MC_OK;
    }
    int layout = 0, npal = 0;
    rc = mc_get_layout(ctx, &layout, &npal);
    if (rc) return rc;
    // per-lane tables (for the objects of <= 32 palette entries) or the shared
    // palette for every object
    std::vector<Shape> cands;
    for (int table : {MC_LAYOUT_PALETTE_LANE, MC_LAYOUT_PALETTE_SHARED})
        for (int block : {128, 256})
            for (int bpc : {0, 1, 2})
                for (int batch : {40, 48, 54}) cands.push_back({block, bpc, batch, table});
    hipStream_t stream = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (stream) (void)hipStreamDestroy(stream);
        return MC_E_DEVICE;
    }
    std::vector<int64_t> h_ref(out_elems), h_cur(out_elems);
    Shape best{0, 0, 0, MC_LAYOUT_PALETTE_LANE};
    float best_ms = 1e30f;
    int rejected = 0, tried = 0;
    for (size_t i = 0; i < cands.size() && rc == MC_OK; ++i) {
        const Shape &s = cands[i];
        rc = mc_set_batch_launch(ctx, s.block, s.bpc, s.batch);
        if (rc) break;
        rc = apply_table(ctx, s.table);
        if (rc) break;
        // one warm-up run, then the timed one (whose output is checked)
        rc = mc_project_batch(ctx, jobs, n_jobs, d_out, out_elems, 0, stream);
        if (rc) break;
        (void)hipEventRecord(e0, stream);
        rc = mc_project_batch(ctx, jobs, n_jobs, d_out, out_elems, 0, stream);
        if (rc) break;
        (void)hipEventRecord(e1, stream);
        if (hipEventSynchronize(e1) != hipSuccess) {
            rc = MC_E_DEVICE;
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ++tried;
        std::vector<int64_t> &h = i == 0 ? h_ref : h_cur;
        if (hipMemcpy(h.data(), d_out, out_elems * sizeof(int64_t), hipMemcpyDeviceToHost) !=
            hipSuccess) {
            rc = MC_E_DEVICE;
            break;
        }
        if (i > 0 && h_cur != h_ref) {
            ++rejected;
            continue;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = s;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(stream);
    if (rc) {
        (void)mc_set_batch_launch(ctx, 0, 0, 0);
        (void)apply_table(ctx, layout);
        return rc;
    }
    rc = mc_set_batch_launch(ctx, best.block, best.bpc, best.batch);
    if (rc) return rc;
    rc = apply_table(ctx, best.table);
    if (rc) return rc;
    out->block = best.block;
    out->blocks_per_cu = best.bpc;
    out->event_batch = best.batch;
    out->table_layout = best.table;
    out->ms = best_ms;
    out->histories_per_s = best_ms > 0.0f ? (double)photons / (best_ms * 1e-3) : 0.0;
    out->candidates = tried;
    out->rejected = rejected;
    if (cache_path) {
        FILE *f = std::fopen(cache_path, "a");
        if (f) {
            std::fprintf(f,
                         "{\"key\": \"%s\", \"block\": %d, \"blocks_per_cu\": %d, "
                         "\"event_batch\": %d, \"table_layout\": %d, \"ms\": %.4f, "
                         "\"photons\": %llu, \"candidates\": %d, \"rejected\": %d}\n",
                         key.c_str(), best.block, best.bpc, best.batch, best.table, best_ms,
                         (unsigned long long)photons, tried, rejected);
            std::fclose(f);
        }
    }
    return MC_OK;
}

}  // extern "C"
