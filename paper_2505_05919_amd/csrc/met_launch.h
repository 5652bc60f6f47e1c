// Launch shape of the Metropolis colour kernels (host side).
#pragma once

#include <stdint.h>

namespace cvf {

// Target number of wavefronts of a Metropolis colour launch.
#ifndef CVF_MET_WAVES
#define CVF_MET_WAVES 4096
#endif
// Use the dword (4-column) Metropolis kernel (1); 0 selects column pairs.
#ifndef CVF_MET_QUAD
#define CVF_MET_QUAD 1
#endif
// Smallest L % 4 == 2 lattice that a single-chain launch moves in quads (mode
// 2).  Measured: L = 4094 ~700 vs ~550 updates/ns with column pairs, L = 1414
// +5 %; at L = 258 the launch is latency-bound and the pairs' twice as many
// wavefronts win (19 vs 14).
#ifndef CVF_MET_RAGGED_MIN
#define CVF_MET_RAGGED_MIN 1024
#endif

struct MetShape {
    uint32_t quad;         // 1: 4-column quads (L % 4 == 0), 2: quads, L % 4 == 2, 0: column pairs
    uint32_t rows;         // rows per wavefront (even, 2..32)
    uint32_t row_blocks;   // grid.y: four wavefronts per workgroup stack vertically
};

// Lanes own 4-column quads (the last one ragged in mode 2) or column pairs
// (mode 0), 64 per wavefront; each wavefront walks `rows` rows of its column
// group.  The row count aims the grid at CVF_MET_WAVES wavefronts (at
// L = 4096: 16 rows, 1024 workgroups, all resident at once).
inline MetShape met_shape_mode(uint32_t L, uint32_t quad)
{
    MetShape m;
    m.quad = quad;
    const uint32_t per_lane = m.quad ? 4 : 2;
    const uint32_t groups = ((L + per_lane - 1) / per_lane + 63) / 64;
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

// The launch shape of a single chain.
inline MetShape met_shape(uint32_t L)
{
    const uint32_t quad = !CVF_MET_QUAD ? 0 : (L % 4 == 0) ? 1 : (L >= CVF_MET_RAGGED_MIN ? 2 : 0);
    return met_shape_mode(L, quad);
}

}  // namespace cvf
