// Uniform-cell map of a voxel object (host side).
#pragma once
#include <cstdint>
#include <vector>

namespace mcx {

// code[i]: palette code of cell i (x fastest) when all its voxels share it,
// -1 otherwise.  out[i] = code | radius << 8, where radius r >= 1 means every
// cell within Chebyshev distance r - 1 (clamped to the grid) holds the same
// code, and 0 marks a mixed cell.
void cell_radii(int ncx, int ncy, int ncz, const std::vector<int16_t> &code,
                std::vector<uint16_t> &out);

}  // namespace mcx
