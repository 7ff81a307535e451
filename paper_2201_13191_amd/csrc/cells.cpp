// Uniform-cell map of a voxel object: for each cube of 4x4x4 voxels, its
// palette code if all its voxels share one, and the Chebyshev radius (in
// cells) of the cube of cells around it that holds only that code.  The
// march uses it to take whole runs of steps through identical voxels at
// once; the map only has to be conservative, never optimistic.
#include "cells.hpp"

#include <algorithm>

namespace mcx {

void cell_radii(int ncx, int ncy, int ncz, const std::vector<int16_t> &code,
                std::vector<uint16_t> &out) {
    const size_t n = (size_t)ncx * ncy * ncz;
    std::vector<uint8_t> d(n);
    for (size_t i = 0; i < n; ++i) d[i] = code[i] < 0 ? 0 : 255;
    auto at = [&](int x, int y, int z) { return ((size_t)z * ncy + y) * ncx + x; };
    // d(c) = Chebyshev distance (capped at 255) from uniform cell c to the
    // nearest cell that is mixed or holds another code; neighbours outside the
    // grid are the clamped ones, so the grid's faces never count as different.
    // Relaxation over the 26 neighbours until nothing changes (forward and
    // backward raster passes; a few passes suffice).
    auto relax = [&](int x, int y, int z) -> bool {
        const size_t i = at(x, y, z);
        if (code[i] < 0) return false;
        int best = d[i];
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int xx = std::min(std::max(x + dx, 0), ncx - 1);
                    const int yy = std::min(std::max(y + dy, 0), ncy - 1);
                    const int zz = std::min(std::max(z + dz, 0), ncz - 1);
                    const size_t j = at(xx, yy, zz);
                    if (j == i) continue;
                    const int cand = code[j] != code[i] ? 1 : d[j] + 1;
                    best = std::min(best, cand);
                }
        if (best < d[i]) {
            d[i] = (uint8_t)best;
            return true;
        }
        return false;
    };
    for (bool changed = true; changed;) {
        changed = false;
        for (int z = 0; z < ncz; ++z)
            for (int y = 0; y < ncy; ++y)
                for (int x = 0; x < ncx; ++x) changed |= relax(x, y, z);
        for (int z = ncz - 1; z >= 0; --z)
            for (int y = ncy - 1; y >= 0; --y)
                for (int x = ncx - 1; x >= 0; --x) changed |= relax(x, y, z);
    }
    out.assign(n, 0);
    for (size_t i = 0; i < n; ++i)
        out[i] = code[i] < 0 ? 0 : (uint16_t)((uint16_t)code[i] | ((uint16_t)d[i] << 8));
}

}  // namespace mcx
