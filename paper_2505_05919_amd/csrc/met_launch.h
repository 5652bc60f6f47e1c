// Launch shape of the Metropolis colour kernels (host side).
#pragma once

#include <stdint.h>

namespace cvf {

// Target number of wavefronts of a Metropolis colour launch.
#ifndef CVF_MET_WAVES
#define CVF_MET_WAVES 4096
#endif
// Use the dword (4-column) Metropolis kernel when L % 4 == 0.
#ifndef CVF_MET_QUAD
#define CVF_MET_QUAD 1
#endif

struct MetShape {
    uint32_t quad;         // 1: lanes own 4-column quads, 0: column pairs
    uint32_t rows;         // rows per wavefront (even, 2..32)
    uint32_t row_blocks;   // grid.y: four wavefronts per workgroup stack vertically
};

// Lanes own 4-column quads (L % 4 == 0) or column pairs, 64 per wavefront;
// each wavefront walks `rows` rows of its column group.  The row count aims
// the grid at CVF_MET_WAVES wavefronts (at L = 4096: 16 rows, 1024
// workgroups, all resident at once).
inline MetShape met_shape(uint32_t L)
{
    MetShape m;
    m.quad = (L % 4 == 0) ? CVF_MET_QUAD : 0;
    const uint32_t per_lane = m.quad ? 4 : 2;
    const uint32_t groups = (L / per_lane + 63) / 64;
    const uint32_t target = CVF_MET_WAVES;
    const uint32_t waves_per_group = groups >= target ? 1 : target / groups;
    uint32_t rows = (L + waves_per_group - 1) / waves_per_group;
    rows = (rows + 1) & ~1u;
    if (rows < 2) rows = 2;
    if (rows > 32) rows = 32;
    m.rows = rows;
    m.row_blocks = ((L + rows - 1) / rows + 3) / 4;
    return m;
}

}  // namespace cvf
