// Neighbour offsets for the per-site kernels (one thread per site).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lll_internal.hpp"

namespace lll {
// The six neighbours of site (x, y, z) of replica R in the order -x, +x, -y,
// +y, -z, +z: d[k] is the neighbour's index minus the site's and has[k]
// whether it exists (periodic boundaries wrap; a free boundary has no
// neighbour beyond the face, and then d[k] = 0, so that a load at the offset
// stays in bounds and the caller adds zero instead).  Per-site kernels load
// all six unconditionally, so the loads are in flight together instead of
// each one behind a branch and a wait.
__device__ __forceinline__ void nbr_offsets(const RepDev& R, int x, int y, int z, int64_t d[6],
                                            bool has[6]) {
    const int Lx = R.Lx, Ly = R.Ly, Lz = R.Lz;
    const bool pbc = R.bc == 0;
    const int64_t sy = Lx, sz = (int64_t)Lx * Ly;
    d[0] = x > 0 ? -1 : (pbc ? Lx - 1 : 0);
    d[1] = x + 1 < Lx ? 1 : (pbc ? 1 - Lx : 0);
    d[2] = y > 0 ? -sy : (pbc ? sy * (Ly - 1) : 0);
    d[3] = y + 1 < Ly ? sy : (pbc ? -sy * (Ly - 1) : 0);
    d[4] = z > 0 ? -sz : (pbc ? sz * (Lz - 1) : 0);
    d[5] = z + 1 < Lz ? sz : (pbc ? -sz * (Lz - 1) : 0);
    has[0] = pbc || x > 0;
    has[1] = pbc || x + 1 < Lx;
    has[2] = pbc || y > 0;
    has[3] = pbc || y + 1 < Ly;
    has[4] = pbc || z > 0;
    has[5] = pbc || z + 1 < Lz;
}

}  // namespace lll
