// Launch parameters shared by the transport kernels and the host runtime.
#pragma once

#include <cstdint>

namespace mcx {

constexpr int kMaxMaterials = 16;
constexpr int kKnTerms = 30;    // Taylor terms of sigma_KN / (pi r_e^2) below E / mc^2 = 0.1
constexpr int kCohTerms = 41;   // power-series terms of the coherent shape below B = 0.1
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

// Voxel representations on the device.  Voxels are stored in bricks of
// kBx x kBy x kBz (x fastest inside a brick, bricks x fastest): a brick of
// one-byte codes is one 128-byte cache line.
constexpr int kBx = 8, kBy = 4, kBz = 4;
constexpr int kBrick = kBx * kBy * kBz;
// When it fits the 24-bit brick strides, a bricked object extends kEdgePad
// voxels past its high faces (x, y and z) with copies of the face voxels, so
// that a centre up to kEdgePad - 1 voxels past a high face, or anywhere below
// a low face (the float to unsigned conversion saturates at 0), reads the
// voxel of the clamped centre without a clamp.
#ifndef MCX_EDGE_PAD
#define MCX_EDGE_PAD 9
#endif
constexpr int kEdgePad = MCX_EDGE_PAD;
// uniform-cell map: cubes of 2^kCellLog voxels per edge (4: measured faster
// than 2, 8 or 16 on the 256^3 benchmark)
#ifndef MCX_CELL_LOG
#define MCX_CELL_LOG 2
#endif
constexpr int kCellLog = MCX_CELL_LOG;

enum Layout : int {
    kPaletteLane = 0,    // byte = palette index; per-lane mu table of every palette entry
    kPaletteShared = 1,  // byte = palette index; palette (id, rho) shared, per-lane mu per material
    kGeneric = 2         // byte = material id, separate bricked fp32 density
};

// One voxel object as the march sees it.
struct VoxelGrid {
    const uint8_t *vox;        // bricked codes (palette index or material id)
    const float *vrho;         // bricked densities (kGeneric only)
    const uint8_t *pal_id;     // [n_pal] material of each palette entry
    const float *pal_rho;      // [n_pal] density of each palette entry
    int n_pal;
    int layout;                // Layout of this object
    int nx, ny, nz;
    int nbx, nby;              // bricks along x and y
    uint32_t ry, rz;           // byte strides of one brick row (y) and one brick slab (z),
                               // less 32 and 128: the parts 8*iy and 32*iz already count
    float cmax[3];             // nx - 1, ny - 1, nz - 1 as floats (voxel-coordinate clamp)
    float inv_h;
    float lo[3], hi[3];
    // uniform-cell map (cells of 2^kCellLog voxels per edge, x fastest): palette code in the low
    // byte, in the high byte the radius r >= 1 of the cube of cells around the
    // cell (Chebyshev radius r - 1, clamped to the grid) that holds only that
    // code, 0 for a cell with several codes; null when the march does not skip
    const uint16_t *cells;
    int ncx, ncy;
    // 1 when the object has its edge copies and a step is at most one voxel:
    // a group's centres (at most 8 steps past the flight's end) then stay in
    // the extended grid and its gathers convert them without clamping
    int unclamped;
};

// One projection of a batch: its frame, Philox key, photon count, images
// and voxel object.
struct JobDesc {
    ProjFrame F;
    uint32_t key0, key1;
    uint64_t n;
    unsigned long long *prim, *scat;
    int grid;
    int pad;
};

struct KParams {
    // voxel object (single projection)
    VoxelGrid G;
    // tables: [n_mat][J] mu/rho on E_j = 1 + j keV, eta[J]
    const float *pe, *coh, *inc, *eta;
    int J, n_mat;
    const double *rayl_b;      // [n_mat] Rayleigh screening constants
    const double *pz_scale;    // [n_mat] Compton-profile momentum scale / (m c)
    uint32_t phys;             // binding effects: 1 S(x,Z) as null collisions, 2 Doppler
    const float *e_bin;        // [n_bins] bin energies
    const uint64_t *thr;       // [n_bins] cumulative thresholds on 32-bit draws
    const uint32_t *guide;     // [256] first bin whose threshold exceeds i * 2^24
    int n_bins;
    // panel and march
    ProjFrame F;
    float sdd, pu, pv, step;
    int nu, nv, snu, snv, bu, bv;   // bu = nu / snu, bv = nv / snv
    uint32_t flags;
    // work
    uint64_t first, n;
    uint32_t key0, key1;
    int event_batch;           // lanes that must wait before a wave handles events
    unsigned long long *prim, *scat;     // int64 tallies (two's complement adds)
    unsigned long long *counter;         // next photon index (relative to first)
    uint32_t chunk;            // photon ids a wave reserves per counter update (>= 1)
    unsigned long long *stats;           // mc_stats layout, or null
    const int *cancel;                   // host-memory cancellation flag (mapped), or null
    // batch: jobs run in order, each wave moving to the next job when the
    // current one has no photons left
    const JobDesc *jobs;
    const VoxelGrid *grids;
    unsigned long long *job_counters;    // [n_jobs] next photon of each job
    int n_jobs;
    // point-detector scoring (eq. (3)-(5)): pseudo-particles per scattering,
    // Russian-roulette threshold (keV, 0: off), and the series of the angular
    // laws' normalisations (Klein-Nishina kKnTerms, coherent kCohTerms)
    int pd_split;
    int pd_mode;               // 1 point detector throughout, 2 mixed (Rayleigh along its law)
    double pd_rr;
    const double *kn_series;
    const double *coh_series;
    // per-history records (debug kernel only)
    uint16_t *dbg_nint;
    uint32_t *dbg_steps;
    uint8_t *dbg_end, *dbg_first;
};

}  // namespace mcx
