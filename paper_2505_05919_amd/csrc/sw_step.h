// Swendsen-Wang step kernels and the lattice recount (included inside the
// kernels' namespace).  The step kernels work on kTW x kTH-cell tiles; each
// has a body shared by the single-chain kernel (grid = the chain's tiles) and
// the batched kernel (workgroup -> chain and tile through prefix sums).
#pragma once

// ---------------------------------------------------------------------------
// Recount of N_HB_raw and N_sigma for cell c (and the state counts N_q').
// ---------------------------------------------------------------------------
__device__ __forceinline__ void recount_cell(const LatticeArgs& a, uint32_t c, uint32_t x, uint32_t y, int& hb,
                                             int& co, int* cnt)
{
    const uint32_t L = a.L;
    const size_t N = a.N;
    const uint8_t* __restrict__ s = a.sigma;
    const uint32_t row = y * L;
    const uint32_t xp = (x + 1 == L) ? 0 : x + 1;
    const uint32_t rp = (y + 1 == L) ? 0 : row + L;
    const int s0 = s[c], s1 = s[N + c], s2 = s[2 * N + c], s3 = s[3 * N + c];
    hb += (s0 == s[N + xp + row]) + (s2 == s[3 * N + x + rp]);
    co += (s0 == s1) + (s0 == s2) + (s0 == s3) + (s1 == s2) + (s1 == s3) + (s2 == s3);
    if (cnt) {
#pragma unroll
        for (int k = 0; k < 6; ++k) cnt[k] += (s0 == k) + (s1 == k) + (s2 == k) + (s3 == k);
    }
}

// Row-based recount (any even L): lane i owns the cells 2i, 2i+1 of the rows
// of its wavefront; 16-bit loads of the four planes, wave-uniform row offsets.
__device__ __forceinline__ uint32_t ld16(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
}

__global__ __launch_bounds__(256) void recount_rows_kernel(LatticeArgs a, int64_t* out, int spread, int step_gate,
                                                           uint32_t rows)
{
    if (step_gate && a.st->skip) return;
    const uint32_t L = a.L, N = a.N;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t pair = blockIdx.x * 64 + lane;
    const uint32_t y0 = (blockIdx.y * 4 + wave) * rows;
    int hb = 0, co = 0;
    if (pair < (L >> 1) && y0 < L) {
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.sigma, 4 * N);
        const uint32_t x = 2 * pair, xn = (x + 2 == L) ? 0 : x + 2;
        const uint32_t y1 = min(y0 + rows, L);
        for (uint32_t y = y0; y < y1; ++y) {
            const uint32_t o = y * L, op = ((y + 1 == L) ? 0 : y + 1) * L;
            const uint32_t d0 = ld16(rs, x, o), d1 = ld16(rs, x, o + N), d2 = ld16(rs, x, o + 2 * N),
                           d3 = ld16(rs, x, o + 3 * N);
            const uint32_t u3 = ld16(rs, x, 3 * N + op);           // arm 3 of the row above
            const uint32_t n1 = ld8b(rs, xn, o + N);                // arm 1 of the cell right of the pair
            const uint32_t a0 = d0 & 255, b0 = d0 >> 8, a1 = d1 & 255, b1 = d1 >> 8;
            const uint32_t a2 = d2 & 255, b2 = d2 >> 8, a3 = d3 & 255, b3 = d3 >> 8;
            hb += (a0 == b1) + (b0 == n1) + (a2 == (u3 & 255)) + (b2 == (u3 >> 8));
            co += (a0 == a1) + (a0 == a2) + (a0 == a3) + (a1 == a2) + (a1 == a3) + (a2 == a3);
            co += (b0 == b1) + (b0 == b2) + (b0 == b3) + (b1 == b2) + (b1 == b3) + (b2 == b3);
        }
    }
    const int v[2] = {hb, co};
    block_add<2>(v, out + ((blockIdx.x + blockIdx.y * gridDim.x) & (spread - 1)), spread);
}

__global__ __launch_bounds__(kBlock) void recount_kernel(LatticeArgs a, int64_t* out, int spread, int with_counts,
                                                         int step_gate)
{
    if (step_gate && a.st->skip) return;
    const double inv_L = 1.0 / (double)a.L;
    int hb = 0, co = 0;
    int cnt[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < a.N; c += gridDim.x * kBlock) {
        uint32_t x;
        const uint32_t y = divmod(c, a.L, inv_L, x);
        recount_cell(a, c, x, y, hb, co, with_counts ? cnt : nullptr);
    }
    if (with_counts) {
        const int v[8] = {hb, co, cnt[0], cnt[1], cnt[2], cnt[3], cnt[4], cnt[5]};
        block_add<8>(v, out, 1);
    } else {
        const int v[2] = {hb, co};
        block_add<2>(v, out + (blockIdx.x & (spread - 1)), spread);
    }
}

// ---------------------------------------------------------------------------
// Swendsen-Wang (Sec. II.D).
// Bond mask per cell: bit 0 covalent +x (arm 0 of c, arm 1 of c+x), bit 1
// covalent +y (arm 2 of c, arm 3 of c+y), bits 2..7 cooperative pairs
// (0,1) (0,2) (0,3) (1,2) (1,3) (2,3).  Link l uses word l of
// Philox(c, t, 0, SWB) for l < 4 and word l-4 of Philox(c, t, 1, SWB).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool below(uint32_t w, uint64_t thr) { return (uint64_t)w < thr; }

// In-cell components of the 4 arms for each of the 64 cooperative masks:
// 2 bits per arm = smallest arm index of its component.
__device__ void build_incell_lut(uint8_t* lut)
{
    const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {1, 2, 3, 2, 3, 3};
    if (threadIdx.x < 64) {
        const int m = threadIdx.x;
        int lab[4] = {0, 1, 2, 3};
        for (int it = 0; it < 3; ++it)
            for (int l = 0; l < 6; ++l)
                if (m >> l & 1) {
                    const int mn = min(lab[pa[l]], lab[pb[l]]);
                    lab[pa[l]] = mn;
                    lab[pb[l]] = mn;
                }
        lut[m] = (uint8_t)(lab[0] | lab[1] << 2 | lab[2] << 4 | lab[3] << 6);
    }
}

struct SwBondCtx {
    uint32_t t;
    uint64_t thr_s, thr_e;
    bool cov_on;
};

__device__ __forceinline__ SwBondCtx sw_ctx(const LatticeArgs& a)
{
    const int theta = a.st->theta;
    SwBondCtx k;
    k.t = a.st->t_cur;
    k.thr_s = a.tab->sw[0];
    k.thr_e = a.tab->sw[1 + theta];
    k.cov_on = theta == 1 && a.jeff_sign != 0;
    return k;
}

// Bond activation of cell c (link mask): s0..s3 its bond indices, f0 / f2
// the facing arms of its arms 0 and 2 (arm 1 of the +x neighbour, arm 3 of
// the +y neighbour).
__device__ __forceinline__ uint32_t sw_bond_bits(const LatticeArgs& a, const SwBondCtx& k, uint32_t c, uint32_t s0,
                                                 uint32_t s1, uint32_t s2, uint32_t s3, uint32_t f0, uint32_t f2)
{
    const uint4 w0 = philox(c, k.t, 0u, kStreamSwb, a.key0, a.key1);
    const uint4 w1 = philox(c, k.t, 1u, kStreamSwb, a.key0, a.key1);
    uint32_t m = 0;
    if (k.cov_on) {
        const bool e0 = (s0 == f0) == (a.jeff_sign > 0);
        const bool e2 = (s2 == f2) == (a.jeff_sign > 0);
        m |= (e0 && below(w0.x, k.thr_e)) ? 1u : 0u;
        m |= (e2 && below(w0.y, k.thr_e)) ? 2u : 0u;
    }
    m |= (s0 == s1 && below(w0.z, k.thr_s)) ? 4u : 0u;
    m |= (s0 == s2 && below(w0.w, k.thr_s)) ? 8u : 0u;
    m |= (s0 == s3 && below(w1.x, k.thr_s)) ? 16u : 0u;
    m |= (s1 == s2 && below(w1.y, k.thr_s)) ? 32u : 0u;
    m |= (s1 == s3 && below(w1.z, k.thr_s)) ? 64u : 0u;
    m |= (s2 == s3 && below(w1.w, k.thr_s)) ? 128u : 0u;
    return m;
}

// Root of x: follow parents until a self-loop.  label[x] <= x everywhere, so
// the chain strictly decreases and ends.
__device__ __forceinline__ uint32_t find_root(const uint32_t* label, uint32_t x)
{
    uint32_t p = label[x];
    while (p != x) {
        x = p;
        p = label[x];
    }
    return x;
}

// ---------------------------------------------------------------------------
// Tiled Swendsen-Wang step.  A workgroup of kTT threads owns a tile of kTW x
// kTH cells, i.e.
// 4 kTC bond indices with local index v = arm * kTC + ly * kTW + lx, whose
// order is the order of the global flat indices arm * N + y * L + x.
//  sw_tile_kernel         bonds of the tile's cells (mask) and the in-tile
//                         unions in LDS; global labels only where the
//                         tile-crossing links can reach them: border bond
//                         indices (-> their tile root) and the roots of the
//                         components holding one (-> themselves); the old
//                         sigma facing the right and bottom edges; every
//                         bond index's tile-local root (uint16, with the
//                         border flag of its component); then the tile-
//                         crossing links, each united (global union-find)
//                         by the later of the two tiles it joins.
//  sw_flip_tile_kernel    one shift per tile-local component (its cluster
//                         minimum comes from the global labels if the
//                         component touches the border, else it is the
//                         component's own minimum), shifts sigma and
//                         recounts N_HB_raw and N_sigma of the new
//                         configuration.
//  sw_labels_kernel       the full label array, on request.
// ---------------------------------------------------------------------------
constexpr uint32_t kIdx = 4 * kTC - 1;  // local index bits of an LDS label
constexpr uint32_t kBorder = 0x8000u;  // flag on the root of a component that holds a border bond index
static_assert(4 * kTC <= kBorder, "local bond indices must stay below the border flag");
static_assert((4 * kTC & (4 * kTC - 1)) == 0, "kIdx is a bit mask");
static_assert(kTT >= kBorderIdx + kEdgeBytes, "one flip thread per border component and facing arm");
static_assert(kTW == 64, "a wavefront holds one tile row");
static_assert(4 * (kTT / 64) == kTH, "four rows per wavefront cover the tile");

struct TileGeom {
    uint32_t x0, y0, w, h, id;
};

// Tile (bx, by) of a lattice with ncx tiles per row.
__device__ __forceinline__ TileGeom tile_geom(uint32_t L, uint32_t bx, uint32_t by, uint32_t ncx)
{
    TileGeom g;
    g.x0 = bx * kTW;
    g.y0 = by * kTH;
    g.w = min(kTW, L - g.x0);
    g.h = min(kTH, L - g.y0);
    g.id = bx + by * ncx;
    return g;
}

// XCD-aware tile order.  Workgroups are dealt to the eight XCDs in turn
// (workgroup b to XCD b % 8), each with its own L2, and a tile row of one
// plane is 64 bytes, half an L2 line: with tiles in row-major order every
// line would be fetched by two XCDs.  Instead the j-th workgroup of an XCD
// takes tile kTileRun (8 (j / kTileRun) + xcd) + j % kTileRun, so each XCD
// works on runs of kTileRun consecutive tiles and shares lines with other
// XCDs only at the ends of its runs (runs of 8 measured best for 64 x 16
// tiles at L = 1414, against 2, 4, 16, 32 and 64).
constexpr uint32_t kTileXcd = 8, kTileRun = 8;

// The tile of this workgroup in a single-chain launch (grid = tiles), in the
// XCD-aware order; the last n % (8 kTileRun) tiles, which do not fill a run
// on every XCD, keep their place.
__device__ __forceinline__ TileGeom grid_tile(uint32_t L)
{
    const uint32_t ncx = gridDim.x, n = ncx * gridDim.y;
    const uint32_t b = blockIdx.x + blockIdx.y * ncx;
    uint32_t tile = b;
    if (b < n - n % (kTileXcd * kTileRun)) {
        const uint32_t xcd = b % kTileXcd, j = b / kTileXcd;
        tile = ((j / kTileRun) * kTileXcd + xcd) * kTileRun + j % kTileRun;
    }
    const uint32_t by = tile / ncx;
    return tile_geom(L, tile - by * ncx, by, ncx);
}

__device__ __forceinline__ bool tile_in(const TileGeom& g, uint32_t v)
{
    const uint32_t lc = v % kTC;
    return lc % kTW < g.w && lc / kTW < g.h;
}

__device__ __forceinline__ uint32_t tile_global(const TileGeom& g, uint32_t L, uint32_t N, uint32_t v)
{
    const uint32_t lc = v % kTC;
    return (v / kTC) * N + (g.y0 + lc / kTW) * L + g.x0 + lc % kTW;
}

// The 4 kTC / kTT = 16 bond indices of a thread: entry i lies in plane i / 4,
// tile row wave + W (i % 4) (wave-uniform; W = kTT / 64 wavefronts, so the
// four rows of a wavefront cover the kTH = 4 W rows of the tile) and tile
// column lane.
__device__ __forceinline__ uint32_t ent_row(uint32_t wave, uint32_t i) { return wave + (kTT / 64) * (i & 3); }
__device__ __forceinline__ uint32_t ent_local(uint32_t wave, uint32_t lane, uint32_t i)
{
    return (i >> 2) * kTC + ent_row(wave, i) * kTW + lane;
}

// The border bond indices of a tile -- the ends of tile-crossing covalent
// links -- numbered b < 2 kTH + 2 kTW: arm 0 in the last column and arm 1 in
// the first column (row b), arm 2 in the last row and arm 3 in the first row
// (column b); 4 kTC if b names no bond index of a ragged tile.
__device__ __forceinline__ uint32_t border_local(const TileGeom& g, uint32_t b)
{
    if (b < kTH) return b < g.h ? b * kTW + g.w - 1 : 4 * kTC;
    if (b < 2 * kTH) return b - kTH < g.h ? kTC + (b - kTH) * kTW : 4 * kTC;
    if (b < 2 * kTH + kTW) return b - 2 * kTH < g.w ? 2 * kTC + (g.h - 1) * kTW + (b - 2 * kTH) : 4 * kTC;
    return b - 2 * kTH - kTW < g.w ? 3 * kTC + (b - 2 * kTH - kTW) : 4 * kTC;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ uint32_t find_root_lds(const uint32_t* lab, uint32_t x)
{
    uint32_t p = lab[x] & kIdx;
    while (p != x) {
        x = p;
        p = lab[x] & kIdx;
    }
    return x;
}

__device__ __forceinline__ void unite_lds(uint32_t* lab, uint32_t a, uint32_t b)
{
    a = find_root_lds(lab, a);
    b = find_root_lds(lab, b);
    while (a != b) {
        if (a > b) {
            const uint32_t tmp = a;
            a = b;
            b = tmp;
        }
        const uint32_t old = atomicMin(lab + b, a);
        if (old == b) return;
        b = find_root_lds(lab, old);
        a = find_root_lds(lab, a);
    }
}

// In-tile components from the link masks mk[i] of cells lc = tid + kTT i:
// the in-cell components (LUT) and the +x links of each row (ballots), then
// the +y links inside the tile (lock-free union-find in LDS);
// finally the roots of components holding a border bond index get kBorder.
// The minimum-index root does not depend on the order of the unions, so
// every kernel that rebuilds the components from the same mask gets the
// same roots.  Expects lut ready; ends with a barrier.
__device__ void tile_components(uint32_t* lab, const uint8_t* lut, const uint32_t (&mk)[kTC / kTT], const TileGeom& g)
{
    const uint32_t lane = threadIdx.x & 63;                // = tile column: a wavefront holds a tile row
#pragma unroll
    for (uint32_t i = 0; i < kTC / kTT; ++i) {
        const uint32_t lc = threadIdx.x + kTT * i, ly = lc / kTW;
        const uint32_t m = mk[i];
        const uint32_t l4 = lut[m >> 2];
        const uint32_t r1 = (l4 >> 2) & 3;                 // arm 0 is always its own in-cell root
        // +x links inside the row: a run of cells joined arm 0 -> arm 1 of the
        // next cell, continued through every cell whose arms 0 and 1 share an
        // in-cell component, is one component whose minimum is arm 0 of the
        // run's first cell.  Found with two ballots; no atomics.
        const uint64_t lnk = __ballot((m & 1) && lane + 1 < g.w);
        const bool in = lane > 0 && ((lnk >> (lane - 1)) & 1);
        const uint64_t brk = __ballot(!(in && r1 == 0));  // bit j: a run starts at column j
        uint32_t e0 = lc;
        uint32_t b_root = 0;
        if (in) {
            const uint64_t upto = lane == 63 ? brk : (brk & ((2ull << lane) - 1));
            const uint64_t before = brk & ((1ull << lane) - 1);
            const uint32_t start = 63 - (uint32_t)__builtin_clzll(upto);
            const uint32_t start_prev = 63 - (uint32_t)__builtin_clzll(before);
            e0 = ly * kTW + start;                         // this cell's arm 0, if the run goes through
            b_root = ly * kTW + start_prev;                // the run that reaches this cell's arm 1
        }
        lab[lc] = e0;
        lab[kTC + lc] = r1 * kTC + lc;
        lab[2 * kTC + lc] = ((l4 >> 4) & 3) * kTC + lc;
        lab[3 * kTC + lc] = ((l4 >> 6) & 3) * kTC + lc;
        if (in && r1 != 0) lab[r1 * kTC + lc] = b_root;    // arm 1's own component joins the run
    }
    __syncthreads();
#pragma unroll
    for (uint32_t i = 0; i < kTC / kTT; ++i) {
        const uint32_t lc = threadIdx.x + kTT * i, ly = lc / kTW;
        if ((mk[i] & 2) && ly + 1 < g.h) unite_lds(lab, 2 * kTC + lc, 3 * kTC + lc + kTW);
    }
    __syncthreads();
    if (threadIdx.x < 2 * (kTW + kTH)) {
        const uint32_t v = border_local(g, threadIdx.x);
        if (v < 4 * kTC) atomicOr(lab + find_root_lds(lab, v), kBorder);
    }
    __syncthreads();
}

__device__ __forceinline__ void tile_masks(const LatticeArgs& a, const TileGeom& g, uint32_t (&mk)[kTC / kTT])
{
#pragma unroll
    for (uint32_t i = 0; i < kTC / kTT; ++i) {
        const uint32_t lc = threadIdx.x + kTT * i, lx = lc % kTW, ly = lc / kTW;
        mk[i] = (lx < g.w && ly < g.h) ? a.mask[(g.y0 + ly) * a.L + g.x0 + lx] : 0u;
    }
}

// Lock-free union of the clusters with roots pu and pv (minimum index wins):
// atomicMin points the larger at the smaller and returns its previous
// parent p; p == the larger means it was a root and the union is done,
// otherwise the pair (smaller, p) is united next, so no connection is lost.
// The larger element of the pair strictly decreases, so the loop ends.
__device__ __forceinline__ void unite_global(uint32_t* label, uint32_t pu, uint32_t pv)
{
    while (pu != pv) {
        if (pu > pv) {
            const uint32_t tmp = pu;
            pu = pv;
            pv = tmp;
        }
        const uint32_t old = atomicMin(label + pv, pu);
        if (old == pv) return;
        pv = old;
    }
}

// lut: 64 bytes, lab: 4 kTC words, act: kEdgeBytes bytes of LDS.
__device__ __forceinline__ void sw_tile_body(const LatticeArgs& a, const TileGeom& g, uint8_t* lut, uint32_t* lab,
                                             uint8_t* act)
{
    // Waves of a SIMD issue oldest first; a workgroup that has finished its
    // bonds yields to those still computing theirs, so all tiles reach the
    // latency-bound union phases together (priority 3, 2, 0 by phase).
    __builtin_amdgcn_s_setprio(3);
    const uint32_t L = a.L, N = a.N;
    uint8_t* edge = a.edge + (size_t)g.id * kEdgeBytes;
    // cell i of a thread: tile column lane, tile row wave + W i (wave-uniform),
    // so plane and row offsets are scalar and the loads need no vector address
    const uint32_t lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool col_in = lane < g.w;
    const uint32_t x = g.x0 + lane;
    const uint32_t vx = col_in ? x : 0u, vxp = col_in ? ((x + 1 == L) ? 0u : x + 1) : 0u;
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(a.sigma, 4 * N), rm = buf_rsrc(a.mask, N);
    if (a.st->skip) return;
    build_incell_lut(lut);
    const SwBondCtx k = sw_ctx(a);
    uint32_t mk[kTC / kTT];
#pragma unroll
    for (uint32_t i = 0; i < kTC / kTT; ++i) {
        const uint32_t ly = wave + (kTT / 64) * i;
        uint32_t m = 0;
        if (ly < g.h && col_in) {
            const uint32_t y = g.y0 + ly, row = y * L, rowp = ((y + 1 == L) ? 0u : y + 1) * L;
            const uint32_t s0 = ld8(rs, vx, row), s1 = ld8(rs, vx, N + row), s2 = ld8(rs, vx, 2 * N + row),
                           s3 = ld8(rs, vx, 3 * N + row);
            const uint32_t f0 = ld8(rs, vxp, N + row), f2 = ld8(rs, vx, 3 * N + rowp);
            m = sw_bond_bits(a, k, x + row, s0, s1, s2, s3, f0, f2);
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)m, rm, (int)vx, (int)row, 0);
            if (lane == g.w - 1) {
                edge[ly] = (uint8_t)f0;
                act[ly] = (uint8_t)(m & 1u);               // the +x link leaving the tile
            }
            if (ly == g.h - 1) {
                edge[kTH + lane] = (uint8_t)f2;
                act[kTH + lane] = (uint8_t)((m >> 1) & 1u);  // the +y link leaving the tile
            }
        }
        mk[i] = m;
    }
    __builtin_amdgcn_s_setprio(2);
    __syncthreads();
    tile_components(lab, lut, mk, g);
    __builtin_amdgcn_s_setprio(0);
    // every bond index: its tile-local root (| flag); flagged roots: a
    // global self-label; border bond indices: a global label of their root.
    // Eight bond indices at a time: their parents, then the parents' entries
    // (a root's entry is the root | flag, so nearly every index is settled by
    // these two reads); the few longer chains are followed in lockstep.
    // Rows past a ragged tile's end hold singletons and are read, not stored.
    const uint32_t voff = 2 * vx;
#pragma unroll
    for (uint32_t h = 0; h < 2; ++h) {
        uint32_t r[8], e[8];
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) r[j] = lab[(2 * h + (j >> 2)) * kTC + (j & 3) * kTT + threadIdx.x] & kIdx;
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) e[j] = lab[r[j]];
        for (;;) {
            bool more = false;
#pragma unroll
            for (uint32_t j = 0; j < 8; ++j) more = more || (e[j] & kIdx) != r[j];
            if (!more) break;
#pragma unroll
            for (uint32_t j = 0; j < 8; ++j) {
                r[j] = e[j] & kIdx;                    // unchanged where already settled
                e[j] = lab[r[j]];
            }
        }
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) {
            const uint32_t p = 2 * h + (j >> 2), ly = ent_row(wave, j & 3);
            if (ly < g.h && col_in) {
                const __amdgpu_buffer_rsrc_t rl = buf_rsrc(a.lroot + (size_t)p * N, 2 * N);
                __builtin_amdgcn_raw_buffer_store_b16((uint16_t)e[j], rl, (int)voff, (int)(2 * (g.y0 + ly) * L), 0);
                const uint32_t v = p * kTC + ly * kTW + lane;
                if (r[j] == v && (e[j] & kBorder)) {
                    // a root other tiles' unions may reach this step: written
                    // through to the device-coherent level (see below)
                    const uint32_t gv = tile_global(g, L, N, v);
                    __hip_atomic_store(a.label + gv, gv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    }
    // Tile-crossing links.  Every border bond index gets the global label of
    // its root (the flip follows these chains), and the tile publishes one
    // exchange word per border bond index: the global root of its component,
    // for the ends in the last column and row only if the link leaving there
    // is active (kNoLink otherwise).  Each tile edge has an arrival counter
    // that the two tiles beside it increment once per step (it wraps back to
    // 0); the tile that arrives second unites that edge's active links with
    // the first tile's words.  No tile ever waits for another.
    // Everything one tile reads of another's within this launch -- the
    // exchange words and the label entries the unions' atomicMin acts on --
    // is written and read only with device-scope atomic stores, loads and
    // read-modify-writes, which all act at the device-coherent level (across
    // the XCDs' separate L2 caches); no plain store touches those entries in
    // this launch.  The barrier below waits for this tile's stores to
    // complete before its counter increments are issued, and the other
    // tile's words are read only after its increment was seen.  (Device-scope
    // fences would do the same by writing back and invalidating whole L2
    // caches, which measured four times slower.)
    uint32_t* xw = a.xchg + (size_t)g.id * kBorderIdx;
    if (threadIdx.x < kBorderIdx) {
        const uint32_t b = threadIdx.x;
        const uint32_t v = border_local(g, b);
        uint32_t w = kNoLink;
        if (v < 4 * kTC) {
            const uint32_t gr = tile_global(g, L, N, find_root_lds(lab, v));
            // device-scope store: other tiles' atomicMin may act on this
            // entry (when v is its own root) before the launch ends, and a
            // plain store's dirty L2 line written back later would undo it
            __hip_atomic_store(a.label + tile_global(g, L, N, v), gr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            bool on = true;
            if (b < kTH) on = act[b] != 0;
            else if (b >= 2 * kTH && b < 2 * kTH + kTW) on = act[kTH + (b - 2 * kTH)] != 0;
            w = on ? gr : kNoLink;
        }
        __hip_atomic_store(xw + b, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_s_waitcnt(0);            // this wave's stores are complete ...
    __syncthreads();                          // ... and so are every wave's, before any increment
    const uint32_t ncx = (L + kTW - 1) / kTW, ncy = (L + kTH - 1) / kTH;
    const uint32_t bx = g.x0 / kTW, by = g.y0 / kTH;
    const uint32_t right = (bx + 1 == ncx ? 0 : bx + 1) + by * ncx, left = (bx == 0 ? ncx - 1 : bx - 1) + by * ncx;
    const uint32_t down = bx + (by + 1 == ncy ? 0 : by + 1) * ncx, up = bx + (by == 0 ? ncy - 1 : by - 1) * ncx;
    uint8_t* second = lut;                    // the in-cell table is dead: four flags
    if (threadIdx.x < 4) {
        // edges: 0 right (counter 2 id), 1 bottom (2 id + 1), 2 left (the left
        // tile's right edge), 3 top (the upper tile's bottom edge)
        const uint32_t e = threadIdx.x;
        const uint32_t c = e == 0 ? 2 * g.id : e == 1 ? 2 * g.id + 1 : e == 2 ? 2 * left : 2 * up + 1;
        second[e] = atomicInc(a.ecnt + c, 1u) == 1u ? 1 : 0;
    }
    __syncthreads();
    if (!(second[0] | second[1] | second[2] | second[3])) return;
    auto word = [](const uint32_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); };
    const uint32_t e = threadIdx.x >> 6, pos = threadIdx.x & 63;
    if (e < 4 && second[e]) {
        uint32_t pu = kNoLink, pv = kNoLink;  // pu: the word that carries the link's activity
        if (e == 0 && pos < g.h) {
            pu = word(xw + pos);
            pv = word(a.xchg + (size_t)right * kBorderIdx + kTH + pos);
        } else if (e == 2 && pos < g.h) {
            pu = word(a.xchg + (size_t)left * kBorderIdx + pos);
            pv = word(xw + kTH + pos);
        } else if (e == 1 && pos < g.w) {
            pu = word(xw + 2 * kTH + pos);
            pv = word(a.xchg + (size_t)down * kBorderIdx + 2 * kTH + kTW + pos);
        } else if (e == 3 && pos < g.w) {
            pu = word(a.xchg + (size_t)up * kBorderIdx + 2 * kTH + pos);
            pv = word(xw + 2 * kTH + kTW + pos);
        }
        if (pu != kNoLink) unite_global(a.label, pu, pv);
    }
}

__global__ __launch_bounds__(kTT) void sw_tile_kernel(LatticeArgs a)
{
    __shared__ uint8_t lut[64];
    __shared__ uint32_t lab[4 * kTC];
    __shared__ uint8_t act[kEdgeBytes];
    sw_tile_body(a, grid_tile(a.L), lut, lab, act);
}

// LDS of the flip: the compacted roots of the interior components, whose
// space then holds the new sigma of the tile; the shift of each root; the
// old (then new) sigma of the tile, kept here rather than in registers so
// that the kernel fits 8 wavefronts per SIMD; the compacted roots of the
// border components (at most one per border bond index); the new sigma
// facing the right / bottom edge; the two root counts.
struct FlipLds {
    uint16_t roots[4 * kTC];
    uint8_t sh[4 * kTC];
    uint8_t osg[4 * kTC];
    uint16_t rootb[kBorderIdx];
    uint8_t across[kEdgeBytes];
    uint32_t nroot, nrootb;
};

// Exclusive prefix sum over the wavefront of per-lane values c < 32, and
// its total: one ballot per bit.
__device__ __forceinline__ uint32_t wave_excl_scan5(uint32_t c, uint32_t& total)
{
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (uint32_t b = 0; b < 5; ++b) {
        const uint64_t m = __ballot((c >> b) & 1u);
        pre += __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u)) << b;
        tot += (uint32_t)__popcll(m) << b;
    }
    total = tot;
    return pre;
}

__device__ __forceinline__ void sw_flip_body(const LatticeArgs& a, const TileGeom& g, FlipLds& lds)
{
    uint16_t* roots = lds.roots;
    uint8_t* sh = lds.sh;
    uint8_t* across = lds.across;
    uint16_t* rootb = lds.rootb;
    uint8_t* nsg = reinterpret_cast<uint8_t*>(roots);
    if (threadIdx.x == 0) {
        lds.nroot = 0;
        lds.nrootb = 0;
    }
    const uint32_t L = a.L, N = a.N, q = a.q;
    // entry i: plane i / 4, tile row ent_row(wave, i), column lane
    const uint32_t lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool col_in = lane < g.w;
    const uint32_t voff = col_in ? g.x0 + lane : 0u;
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(a.sigma, 4 * N);
    uint32_t os[4 * kTC / kTT], lr[4 * kTC / kTT];     // old sigma, local root | kBorder
#pragma unroll
    for (uint32_t i = 0; i < 4 * kTC / kTT; ++i) {
        const uint32_t p = i >> 2, ly = ent_row(wave, i);
        os[i] = 0;
        lr[i] = ent_local(wave, lane, i);
        if (ly < g.h) {
            const uint32_t row = (g.y0 + ly) * L;
            os[i] = __builtin_amdgcn_raw_buffer_load_b8(rs, (int)voff, (int)(p * N + row), 0);
            const uint32_t l = __builtin_amdgcn_raw_buffer_load_b16(buf_rsrc(a.lroot + (size_t)p * N, 2 * N),
                                                                   (int)(2 * voff), (int)(2 * row), 0);
            if (col_in) lr[i] = l;
        }
    }
    // the loads above do not depend on the chain state; read it now
    if (a.st->skip) return;                   // step limit reached (uniform, before any barrier)
    const uint32_t t = a.st->t_cur;
    if (g.id == 0 && threadIdx.x == 0) a.st->sw_done = 1;
#pragma unroll
    for (uint32_t i = 0; i < 4 * kTC / kTT; ++i) lds.osg[ent_local(wave, lane, i)] = (uint8_t)os[i];
    // the 16-bit local roots, two per register for the rest of the kernel
    uint32_t lrp[2 * kTC / kTT];
#pragma unroll
    for (uint32_t k = 0; k < 2 * kTC / kTT; ++k) lrp[k] = lr[2 * k] | (lr[2 * k + 1] << 16);
    auto LR = [&](uint32_t i) { return (lrp[i >> 1] >> (16 * (i & 1))) & 0xFFFFu; };
    // component roots, compacted into an interior and a border list: a lane's
    // slots follow from a prefix sum of the per-lane counts over the
    // wavefront, one LDS atomic per wavefront and list places the wavefront
    // (the order of a list is immaterial: every entry sets its own root's
    // shift)
    // The lane's roots as bits of one register (bit i: entry i is an
    // interior root, bit 16 + i: a border root), so that no per-entry lane
    // masks stay live in SGPRs between the two passes.
    static_assert(4 * kTC / kTT == 16, "16 entries per thread");
    uint32_t rf = 0;
#pragma unroll
    for (uint32_t i = 0; i < 4 * kTC / kTT; ++i) {
        const bool root = col_in && ent_row(wave, i) < g.h && (LR(i) & kIdx) == ent_local(wave, lane, i);
        const uint32_t bit = ((LR(i) >> 11) & 16u) + i;   // the border flag (bit 15) selects bit 16 + i
        rf |= (root ? 1u : 0u) << bit;
    }
    const uint32_t cnt = (uint32_t)__popc(rf & 0xFFFFu), cntb = (uint32_t)__popc(rf >> 16);
    uint32_t tot, totb;
    uint32_t pos = wave_excl_scan5(cnt, tot), posb = wave_excl_scan5(cntb, totb);
    __syncthreads();                          // counts = 0
    uint32_t base = 0, baseb = 0;
    if (lane == 0) {
        base = atomicAdd(&lds.nroot, tot);
        baseb = atomicAdd(&lds.nrootb, totb);
    }
    pos += (uint32_t)__shfl((int)base, 0);
    posb += (uint32_t)__shfl((int)baseb, 0);
#pragma unroll
    for (uint32_t i = 0; i < 4 * kTC / kTT; ++i) {
        const uint32_t bi = (rf >> i) & 1u, bb = (rf >> (16 + i)) & 1u;
        if (bi) roots[pos] = (uint16_t)LR(i);
        pos += bi;
        if (bb && posb < kBorderIdx) rootb[posb] = (uint16_t)(LR(i) & kIdx);
        posb += bb;
    }
    __syncthreads();
    // One shift per component, drawn at its cluster minimum.  Border
    // components and the facing arms across the right edge (p < kTH) and
    // the bottom edge (column p - kTH) need the global root chain: one job
    // per thread, whose first link is loaded before the interior components
    // (whose minimum is their own root) are drawn, so that the load's
    // latency is hidden behind that arithmetic.
    const uint32_t nr = lds.nroot, nb = min(lds.nrootb, kBorderIdx);
    const uint8_t* edge = a.edge + (size_t)g.id * kEdgeBytes;
    uint32_t x = 0, dst = 0;
    bool live = false;
    if (threadIdx.x < nb) {
        dst = rootb[threadIdx.x];
        x = tile_global(g, L, N, dst);
        live = true;
    } else if (threadIdx.x - nb < kEdgeBytes) {
        const uint32_t p = threadIdx.x - nb;
        dst = 0x10000u | p;
        if (p < kTH) {
            live = p < g.h;
            const uint32_t xx = g.x0 + g.w - 1, yy = g.y0 + p;
            x = N + ((xx + 1 == L) ? 0 : xx + 1) + yy * L;
        } else {
            live = p - kTH < g.w;
            const uint32_t xx = g.x0 + (p - kTH), yy = g.y0 + g.h - 1;
            x = 3 * N + xx + ((yy + 1 == L) ? 0 : yy + 1) * L;
        }
    }
    uint32_t pn = live ? a.label[x] : 0u;
    for (uint32_t j = threadIdx.x; j < nr; j += kTT) {
        const uint32_t e = roots[j];
        const uint32_t w = philox(tile_global(g, L, N, e), t, 0u, kStreamSwf, a.key0, a.key1).x;
        sh[e] = (uint8_t)((w <= a.flip_lim) ? (uint32_t)((double)w * a.flip_invd) : 0u);
    }
    if (live) {
        while (pn != x) {
            x = pn;
            pn = a.label[x];
        }
        const uint32_t w = philox(x, t, 0u, kStreamSwf, a.key0, a.key1).x;
        const uint32_t sft = (w <= a.flip_lim) ? (uint32_t)((double)w * a.flip_invd) : 0u;
        if (dst < 0x10000u) {
            sh[dst] = (uint8_t)sft;
        } else {
            const uint32_t p = dst & 0xFFFFu;
            const uint32_t s = edge[p] + sft;
            across[p] = (uint8_t)(s >= q ? s - q : s);
        }
    }
    __syncthreads();
    // Empty asm, no instruction: the masked roots are recomputed here from
    // the packed registers instead of being kept live (and spilled) across
    // the draws since the compaction.
#pragma unroll
    for (uint32_t k = 0; k < 2 * kTC / kTT; ++k) __asm__("" : "+v"(lrp[k]));
#pragma unroll
    for (uint32_t i = 0; i < 4 * kTC / kTT; ++i) {
        const uint32_t ly = ent_row(wave, i);
        uint32_t s = lds.osg[ent_local(wave, lane, i)] + sh[LR(i) & kIdx];
        s = s >= q ? s - q : s;
        if (col_in && ly < g.h)
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)s, rs, (int)voff, (int)((i >> 2) * N + (g.y0 + ly) * L), 0);
        lds.osg[ent_local(wave, lane, i)] = (uint8_t)s;
    }
    __syncthreads();                          // the root list is dead: its space holds the new sigma
#pragma unroll
    for (uint32_t i = 0; i < 4 * kTC / kTT; ++i) nsg[ent_local(wave, lane, i)] = lds.osg[ent_local(wave, lane, i)];
    __syncthreads();
    // recount of the new configuration: the +x and +y HB pairs and the six
    // in-cell pairs of every cell of the tile
    int hb = 0, co = 0;
#pragma unroll
    for (uint32_t i = 0; i < kTC / kTT; ++i) {
        const uint32_t lc = threadIdx.x + kTT * i, lx = lc % kTW, ly = lc / kTW;
        if (lx < g.w && ly < g.h) {
            const uint32_t s0 = nsg[lc], s1 = nsg[kTC + lc], s2 = nsg[2 * kTC + lc], s3 = nsg[3 * kTC + lc];
            const uint32_t f0 = lx + 1 < g.w ? nsg[kTC + lc + 1] : across[ly];
            const uint32_t f2 = ly + 1 < g.h ? nsg[3 * kTC + lc + kTW] : across[kTH + lx];
            hb += (s0 == f0) + (s2 == f2);
            co += (s0 == s1) + (s0 == s2) + (s0 == s3) + (s1 == s2) + (s1 == s3) + (s2 == s3);
        }
    }
    const int v2[2] = {hb, co};
    block_add<2, kTT>(v2, a.slots + (g.id & (kSlots - 1)), kSlots);
}

__global__ __launch_bounds__(kTT) __attribute__((amdgpu_waves_per_eu(8, 8))) void sw_flip_tile_kernel(LatticeArgs a)
{
    __shared__ FlipLds lds;
    sw_flip_body(a, grid_tile(a.L), lds);
}

// label[idx] = the minimum of idx's cluster, for every bond index; written
// to out (4N uint32).  Works from the mask and the global labels left by
// either the tiled or the batched step.
__global__ __launch_bounds__(kTT) void sw_labels_kernel(LatticeArgs a, uint32_t* __restrict__ out)
{
    __shared__ uint8_t lut[64];
    __shared__ uint32_t lab[4 * kTC];
    build_incell_lut(lut);
    const uint32_t L = a.L, N = a.N;
    const TileGeom g = grid_tile(L);
    uint32_t mk[kTC / kTT];
    tile_masks(a, g, mk);
    __syncthreads();
    tile_components(lab, lut, mk, g);
#pragma unroll
    for (uint32_t i = 0; i < 4 * kTC / kTT; ++i) {
        const uint32_t v = threadIdx.x + kTT * i;
        if (!tile_in(g, v)) continue;
        const uint32_t r = find_root_lds(lab, v);
        const uint32_t gr = tile_global(g, L, N, r);
        out[tile_global(g, L, N, v)] = (lab[r] & kBorder) ? find_root(a.label, gr) : gr;
    }
}

// ---------------------------------------------------------------------------
// Batched Swendsen-Wang: the tiled step of every chain of a batch, one launch
// per stage.  Workgroup b belongs to the chain c with start[c] <= b <
// start[c+1] (prefix sums of per-chain tiles) and does
// exactly what the workgroup of that chain's own launch does.
// ---------------------------------------------------------------------------
// Tile of workgroup b of a batch whose chain's tiles are start .. end - 1:
// the XCD-aware order of grid_tile over the workgroups from the first
// multiple of 8 kTileRun at or after start, in whole groups of 8 kTileRun
// (so that b % 8 is the XCD there too); row-major order elsewhere.
__device__ __forceinline__ TileGeom batch_tile(const LatticeArgs& a, uint32_t b, uint32_t start, uint32_t end)
{
    constexpr uint32_t kGroup = kTileXcd * kTileRun;
    const uint32_t ncx = (a.L + kTW - 1) / kTW;
    const uint32_t s8 = (start + kGroup - 1) / kGroup * kGroup;
    uint32_t tile = b - start;
    if (b >= s8 && end >= s8 && b < s8 + (end - s8) / kGroup * kGroup) {
        const uint32_t r = b - s8, xcd = r % kTileXcd, j = r / kTileXcd;
        tile = s8 - start + ((j / kTileRun) * kTileXcd + xcd) * kTileRun + j % kTileRun;
    }
    const uint32_t by = tile / ncx;
    return tile_geom(a.L, tile - by * ncx, by, ncx);
}

__global__ __launch_bounds__(kTT) void sw_tile_batch_kernel(const BatchEntry* __restrict__ ent,
                                                            const uint32_t* __restrict__ tstart, uint32_t count)
{
    __shared__ uint8_t lut[64];
    __shared__ uint32_t lab[4 * kTC];
    __shared__ uint8_t act[kEdgeBytes];
    const uint32_t c = batch_chain(tstart, count, blockIdx.x);
    const LatticeArgs a = ent[c].la;
    sw_tile_body(a, batch_tile(a, blockIdx.x, tstart[c], tstart[c + 1]), lut, lab, act);
}

__global__ __launch_bounds__(kTT) __attribute__((amdgpu_waves_per_eu(8, 8))) void sw_flip_batch_kernel(
    const BatchEntry* __restrict__ ent, const uint32_t* __restrict__ tstart, uint32_t count)
{
    __shared__ FlipLds lds;
    const uint32_t c = batch_chain(tstart, count, blockIdx.x);
    const LatticeArgs a = ent[c].la;
    sw_flip_body(a, batch_tile(a, blockIdx.x, tstart[c], tstart[c + 1]), lds);
}
