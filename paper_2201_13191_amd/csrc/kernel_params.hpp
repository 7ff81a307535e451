// Launch parameters shared by the transport kernels and the host runtime.
#pragma once

#include <cstdint>

namespace mcx {

constexpr int kMaxMaterials = 16;
constexpr int kMaxScatterings = 1000;   // safety cap on interactions per history

// Frame of one projection (fp32, computed on the host from the angle).
struct ProjFrame {
    float S[3];     // source position
    float ax[3];    // central-ray direction (unit)
    float eu[3];    // panel u axis
    float ev[3];    // panel v axis
    float D[3];     // panel centre
    float hu, hv;   // half panel extents
    float omc;      // 1 - cos(half-angle of the cone circumscribing the panel)
};

struct KParams {
    // voxel object, x fastest
    const uint8_t *ids;
    const float *rho;
    int nx, ny, nz;
    float inv_h;
    float lo[3], hi[3];
    // tables: [n_mat][J] mu/rho on E_j = 1 + j keV, eta[J]
    const float *pe, *coh, *inc, *eta;
    int J, n_mat;
    const double *rayl_b;      // [n_mat] Rayleigh screening constants
    const float *e_bin;        // [n_bins] bin energies
    const uint64_t *thr;       // [n_bins] cumulative thresholds on 32-bit draws
    int n_bins;
    // panel and march
    ProjFrame F;
    float sdd, pu, pv, step;
    int nu, nv, snu, snv, bu, bv;   // bu = nu / snu, bv = nv / snv
    uint32_t flags;
    // work
    uint64_t first, n;
    uint32_t key0, key1;
    int steps_per_round;
    unsigned long long *prim, *scat;     // int64 tallies (two's complement adds)
    unsigned long long *counter;         // next photon index (relative to first)
    unsigned long long *stats;           // mc_stats layout, or null
    // per-history records (debug kernel only)
    uint16_t *dbg_nint;
    uint32_t *dbg_steps;
    uint8_t *dbg_end, *dbg_first;
};

}  // namespace mcx
