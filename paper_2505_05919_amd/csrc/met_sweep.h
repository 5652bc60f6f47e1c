// Checkerboard Metropolis sweep kernels (included inside the kernels'
// namespace, after the Philox, reduction and volume-move helpers).
#pragma once

// ---------------------------------------------------------------------------
// Checkerboard Metropolis: every cell of one colour, arms 0..3 in order
// (Sec. II.C).  Cells of one colour share no interaction: arm a of c only
// couples to the other arms of c (J_sigma) and to arm a^1 of the neighbour
// in direction a (J_eff), which has the other colour.
//
// Work layout: a lane of a wavefront owns a column quad (4j..4j+3: two cells
// of the updated colour per row) or, for smaller L % 4 == 2 lattices and
// batches, a column pair (2i, 2i+1: one cell per row), and walks `rows`
// consecutive rows.  Row addresses are wave-uniform (SGPR base + lane
// column), so the loop carries no vector address arithmetic.
//
// Energy bookkeeping without compares: bond indices are held as 4*sigma and
// Z = sum_{b != a} 1 << 4 sigma_b  +  8 << 4 sigma_facing
// packs, per state v, (#other arms in v) + 8 [facing arm in v] into a 4-bit
// field, so bfe(Z, new) - bfe(Z, old) = dc + 8 dh (dc in -3..3, dh in -1..1)
// indexes an LDS table holding the acceptance threshold and a packed
// counter increment (dc + 2^10 dh + 2^20 for one accepted move).
// ---------------------------------------------------------------------------
// LE: the table holds thr - 1 (2^32 - 1 for "always"), valid when no
// threshold is 0, and a move is accepted iff word <= entry -- one compare
// instead of clamping the word below the sentinel first.
template <int Q, bool LE = false>
__device__ __forceinline__ void met_arm(uint32_t& s4, uint32_t Z, uint32_t prop, uint32_t accw,
                                        const uint2* tbl, uint32_t& wsum)
{
    constexpr uint32_t M = Q - 1;                         // proposals: the q-1 other states
    // k = floor(prop / floor(2^32/M)); kp = k + 1 = high word of (prop' M + 2^32).
    // M in {3, 5} divides 2^32 - 1 and needs prop' = prop + 1 (prop = 2^32-1 is the
    // NULL proposal); M in {1, 2, 4} divides 2^32 and has no NULL proposal.
    constexpr bool kHasNull = (M == 3 || M == 5);
    // (prop + 1) M + 2^32 = prop M + (2^32 + M): the +1 folds into the addend
    uint32_t kp = (uint32_t)(((uint64_t)prop * M + ((1ull << 32) + (kHasNull ? M : 0u))) >> 32);
    // Empty asm, no instruction: kp stays a 32-bit value, so that 4 kp + s4 is
    // one v_lshl_add_u32 instead of a 64-bit shift folded into alignbit + and.
    __asm__("" : "+v"(kp));
    const uint32_t t4 = s4 + (kp << 2);                   // 4 (sigma + 1 + k)
    const uint32_t sn4 = min(t4, t4 - 4u * Q);            // mod q, in units of 4
    const int d = (int)__builtin_amdgcn_ubfe(Z, sn4, 4) - (int)__builtin_amdgcn_ubfe(Z, s4, 4);
    const uint2 e = tbl[d + 16];
    bool acc = LE ? accw <= e.x : min(accw, 0xFFFFFFFEu) < e.x;   // thr == 2^32-1 always accepts
    if (kHasNull) acc = acc && prop != 0xFFFFFFFFu;       // the NULL proposal
    s4 = acc ? sn4 : s4;
    wsum += acc ? e.y : 0u;
}

// Raw buffer over the bond-index planes (4N bytes < 2^32): 32-bit lane
// offsets plus a wave-uniform scalar offset, so row and plane offsets stay in
// SGPRs and loads/stores need no vector address arithmetic.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t sigma_rsrc(uint8_t* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ uint32_t ld8(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_amdgcn_raw_buffer_load_b8(r, (int)voff, (int)soff, 0);
}

__device__ __forceinline__ void st8(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b8((uint8_t)v, r, (int)voff, (int)soff, 0);
}

// The eight bytes one cell's update reads: its four arms and the four
// facing arms of its neighbours (all of the other colour).
struct CellBytes {
    uint32_t s0, s1, s2, s3, f0, f1, f2, f3;
};

// Loads for the cell at column x of row y.  Row offsets go into the
// wave-uniform scalar offset when y is the same for the whole wavefront, or
// (VROW) into the per-lane offset when every lane has a row of its own.
template <bool VROW>
struct RowSplit {
    // per-lane part and scalar part of the offset of column x in the row at o
    __device__ __forceinline__ static uint32_t v(uint32_t x, uint32_t o) { return VROW ? x + o : x; }
    __device__ __forceinline__ static uint32_t s(uint32_t base, uint32_t o) { return VROW ? base : base + o; }
};

template <bool VROW = false>
__device__ __forceinline__ CellBytes met_load(const LatticeArgs& a, __amdgpu_buffer_rsrc_t rs, uint32_t y,
                                              uint32_t x, uint32_t xp, uint32_t xm)
{
    using RS = RowSplit<VROW>;
    const uint32_t L = a.L, N = a.N;
    const uint32_t yp = (y + 1 == L) ? 0 : y + 1, ym = (y == 0) ? L - 1 : y - 1;
    const uint32_t o0 = y * L, op = yp * L, om = ym * L;
    CellBytes b;
    b.s0 = ld8(rs, RS::v(x, o0), RS::s(0, o0));
    b.s1 = ld8(rs, RS::v(x, o0), RS::s(N, o0));
    b.s2 = ld8(rs, RS::v(x, o0), RS::s(2 * N, o0));
    b.s3 = ld8(rs, RS::v(x, o0), RS::s(3 * N, o0));
    b.f0 = ld8(rs, RS::v(xp, o0), RS::s(N, o0));          // arm 1 of the +x neighbour
    b.f1 = ld8(rs, RS::v(xm, o0), RS::s(0, o0));          // arm 0 of the -x neighbour
    b.f2 = ld8(rs, RS::v(x, op), RS::s(3 * N, op));       // arm 3 of the +y neighbour
    b.f3 = ld8(rs, RS::v(x, om), RS::s(2 * N, om));       // arm 2 of the -y neighbour
    return b;
}

// Update the four arms of the cell (x, y) from its loaded bytes and store them.
template <int Q, bool VROW = false, bool LE = false>
__device__ __forceinline__ void met_cell(const LatticeArgs& a, __amdgpu_buffer_rsrc_t rs, const uint2* tbl,
                                         uint32_t t, uint32_t y, uint32_t x, const CellBytes& b, uint32_t& wsum)
{
    using RS = RowSplit<VROW>;
    const uint32_t N = a.N, o0 = y * a.L;
    uint32_t s0 = b.s0 << 2, s1 = b.s1 << 2, s2 = b.s2 << 2, s3 = b.s3 << 2;
    const uint32_t f0 = b.f0 << 2, f1 = b.f1 << 2, f2 = b.f2 << 2, f3 = b.f3 << 2;
    const uint32_t c = x + o0;
    const uint4 wa = philox(c, t, 0u, kStreamMet, a.key0, a.key1);
    const uint4 wb = philox(c, t, 1u, kStreamMet, a.key0, a.key1);
    const uint32_t p23 = (1u << s2) + (1u << s3);
    met_arm<Q, LE>(s0, p23 + (1u << s1) + (8u << f0), wa.x, wa.y, tbl, wsum);
    met_arm<Q, LE>(s1, p23 + (1u << s0) + (8u << f1), wa.z, wa.w, tbl, wsum);
    const uint32_t p01 = (1u << s0) + (1u << s1);
    met_arm<Q, LE>(s2, p01 + (1u << s3) + (8u << f2), wb.x, wb.y, tbl, wsum);
    met_arm<Q, LE>(s3, p01 + (1u << s2) + (8u << f3), wb.z, wb.w, tbl, wsum);
    st8(rs, s0 >> 2, RS::v(x, o0), RS::s(0, o0));
    st8(rs, s1 >> 2, RS::v(x, o0), RS::s(N, o0));
    st8(rs, s2 >> 2, RS::v(x, o0), RS::s(2 * N, o0));
    st8(rs, s3 >> 2, RS::v(x, o0), RS::s(3 * N, o0));
}

// ---------------------------------------------------------------------------
// Quad variant: lane j owns the four columns 4j..4j+3 and moves whole dwords
// of every plane.  In a row of parity P the updated cells sit at bytes P and
// P+2 of the quad; their x neighbours are the other bytes of the same dwords
// except one, fetched with a single byte load (the column left of the quad
// for P = 0, right of it for P = 1).  The two bytes of the other colour are
// written back unchanged -- nothing writes them during this pass.  Per row
// and lane: 6 dword loads + 1 byte load + 4 dword stores for 2 cells.
// R (L % 4 == 2): plane offsets stay dword-aligned, even rows start on a
// dword and odd rows two bytes past one, so the dwords of odd rows are moved
// as two 16-bit halves.  The last quad of a row holds columns L-2, L-1 and
// two phantom bytes (the next row's first columns, or in odd rows a second
// copy of the low half): only its first cell is real, its +x neighbour for
// P = 1 is the wrapped edge byte, the phantom cell's counter increments are
// dropped, and only the low half is stored.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ld32(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
}

__device__ __forceinline__ void st32(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)voff, (int)soff, 0);
}

__device__ __forceinline__ void st16(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)v, r, (int)voff, (int)soff, 0);
}

// Dword of a row that starts two bytes past a dword boundary (MIS): two
// 16-bit halves, the high one at voff_hi (voff + 2; voff for the last quad
// of a row, whose high half is a phantom, so that no load leaves sigma).
template <bool MIS>
__device__ __forceinline__ uint32_t ld32r(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t voff_hi, uint32_t soff)
{
    if (!MIS) return ld32(r, voff, soff);
    const uint32_t lo = __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
    const uint32_t hi = __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff_hi, (int)soff, 0);
    return lo | (hi << 16);
}

// Store of a quad dword: whole, or (R) the low half only for the last quad
// of a row, and as two halves in rows that start off a dword boundary.
template <bool R, bool MIS>
__device__ __forceinline__ void st32r(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t voff, uint32_t soff,
                                      bool ragged)
{
    if (!R) {
        st32(r, v, voff, soff);
    } else if (MIS) {
        st16(r, v, voff, soff);
        if (!ragged) st16(r, v >> 16, voff + 2, soff);
    } else if (ragged) {
        st16(r, v, voff, soff);
    } else {
        st32(r, v, voff, soff);
    }
}

struct QuadBytes {
    uint32_t d0, d1, d2, d3;   // arms 0..3 of the quad, row y
    uint32_t up3, dn2;         // arm 3 of row y+1, arm 2 of row y-1
    uint32_t edge;             // P=0: arm 0 of the column left of the quad; P=1: arm 1 right of it
};

// ODD: y is odd.  With R the row of y is off a dword boundary when y is odd,
// and its neighbour rows (y +- 1, wrapping to 0 or L-1) when y is even.
// VROW: row offsets per lane (see met_load; not combined with R).
template <int P, bool R, bool ODD, bool VROW = false>
__device__ __forceinline__ QuadBytes met_load4(const LatticeArgs& a, __amdgpu_buffer_rsrc_t rs, uint32_t y,
                                               uint32_t x4, uint32_t x4h, uint32_t xl, uint32_t xr)
{
    static_assert(!(R && VROW), "ragged quads keep wave-uniform rows");
    using RS = RowSplit<VROW>;
    constexpr bool DMIS = R && ODD, NMIS = R && !ODD;
    const uint32_t L = a.L, N = a.N;
    const uint32_t yp = (y + 1 == L) ? 0 : y + 1, ym = (y == 0) ? L - 1 : y - 1;
    const uint32_t o0 = y * L, op = yp * L, om = ym * L;
    QuadBytes q;
    q.d0 = ld32r<DMIS>(rs, RS::v(x4, o0), RS::v(x4h, o0), RS::s(0, o0));
    q.d1 = ld32r<DMIS>(rs, RS::v(x4, o0), RS::v(x4h, o0), RS::s(N, o0));
    q.d2 = ld32r<DMIS>(rs, RS::v(x4, o0), RS::v(x4h, o0), RS::s(2 * N, o0));
    q.d3 = ld32r<DMIS>(rs, RS::v(x4, o0), RS::v(x4h, o0), RS::s(3 * N, o0));
    q.up3 = ld32r<NMIS>(rs, RS::v(x4, op), RS::v(x4h, op), RS::s(3 * N, op));
    q.dn2 = ld32r<NMIS>(rs, RS::v(x4, om), RS::v(x4h, om), RS::s(2 * N, om));
    q.edge = (P == 0) ? ld8(rs, RS::v(xl, o0), RS::s(0, o0)) : ld8(rs, RS::v(xr, o0), RS::s(N, o0));
    return q;
}

// 4 * (byte k of a dword pre-shifted left by 2): exact for values below 64.
template <int K>
__device__ __forceinline__ uint32_t byte4(uint32_t d4)
{
    return __builtin_amdgcn_ubfe(d4, 8 * K, 8);
}

// replace bytes B1, B2 of d by v1/4, v2/4
template <int B1, int B2>
__device__ __forceinline__ uint32_t put2(uint32_t d, uint32_t v1, uint32_t v2)
{
    constexpr uint32_t keep = ~((0xFFu << (8 * B1)) | (0xFFu << (8 * B2)));
    const uint32_t w1 = (B1 == 0) ? (v1 >> 2) : (v1 << (8 * B1 - 2));
    return (d & keep) | w1 | (v2 << (8 * B2 - 2));
}

template <int Q, int P, bool R, bool ODD, bool LE = false, bool VROW = false>
__device__ __forceinline__ void met_quad(const LatticeArgs& a, __amdgpu_buffer_rsrc_t rs, const uint2* tbl,
                                         uint32_t t, uint32_t y, uint32_t x4, const QuadBytes& q, uint32_t& wsum,
                                         bool ragged)
{
    constexpr int B1 = P, B2 = P + 2;                 // bytes of the two updated cells
    const uint32_t N = a.N, o0 = y * a.L;
    const uint32_t D0 = q.d0 << 2, D1 = q.d1 << 2, D2 = q.d2 << 2, D3 = q.d3 << 2;
    const uint32_t U3 = q.up3 << 2, M2 = q.dn2 << 2, E = q.edge << 2;
    // cell at byte B1
    uint32_t a0 = byte4<B1>(D0), a1 = byte4<B1>(D1), a2 = byte4<B1>(D2), a3 = byte4<B1>(D3);
    // cell at byte B2
    uint32_t b0 = byte4<B2>(D0), b1 = byte4<B2>(D1), b2 = byte4<B2>(D2), b3 = byte4<B2>(D3);
    {
        const uint32_t f0 = (R && P == 1 && ragged) ? E : byte4<B1 + 1>(D1);   // arm 1, column +1
        const uint32_t f1 = (P == 0) ? E : byte4<(B1 > 0 ? B1 - 1 : 0)>(D0);   // arm 0, column -1
        const uint32_t f2 = byte4<B1>(U3), f3 = byte4<B1>(M2);
        const uint32_t c = x4 + B1 + o0;
        const uint4 wa = philox(c, t, 0u, kStreamMet, a.key0, a.key1);
        const uint4 wb = philox(c, t, 1u, kStreamMet, a.key0, a.key1);
        const uint32_t p23 = (1u << a2) + (1u << a3);
        met_arm<Q, LE>(a0, p23 + (1u << a1) + (8u << f0), wa.x, wa.y, tbl, wsum);
        met_arm<Q, LE>(a1, p23 + (1u << a0) + (8u << f1), wa.z, wa.w, tbl, wsum);
        const uint32_t p01 = (1u << a0) + (1u << a1);
        met_arm<Q, LE>(a2, p01 + (1u << a3) + (8u << f2), wb.x, wb.y, tbl, wsum);
        met_arm<Q, LE>(a3, p01 + (1u << a2) + (8u << f3), wb.z, wb.w, tbl, wsum);
    }
    const uint32_t wkeep = wsum;                      // R: the last quad's second cell is a phantom
    {
        const uint32_t f0 = (P == 1) ? E : byte4<(B2 < 3 ? B2 + 1 : 3)>(D1);
        const uint32_t f1 = byte4<B2 - 1>(D0);
        const uint32_t f2 = byte4<B2>(U3), f3 = byte4<B2>(M2);
        const uint32_t c = x4 + B2 + o0;
        const uint4 wa = philox(c, t, 0u, kStreamMet, a.key0, a.key1);
        const uint4 wb = philox(c, t, 1u, kStreamMet, a.key0, a.key1);
        const uint32_t p23 = (1u << b2) + (1u << b3);
        met_arm<Q, LE>(b0, p23 + (1u << b1) + (8u << f0), wa.x, wa.y, tbl, wsum);
        met_arm<Q, LE>(b1, p23 + (1u << b0) + (8u << f1), wa.z, wa.w, tbl, wsum);
        const uint32_t p01 = (1u << b0) + (1u << b1);
        met_arm<Q, LE>(b2, p01 + (1u << b3) + (8u << f2), wb.x, wb.y, tbl, wsum);
        met_arm<Q, LE>(b3, p01 + (1u << b2) + (8u << f3), wb.z, wb.w, tbl, wsum);
    }
    if (R && ragged) wsum = wkeep;
    constexpr bool DMIS = R && ODD;
    using RS = RowSplit<VROW>;
    const uint32_t xv = RS::v(x4, o0);
    st32r<R, DMIS>(rs, put2<B1, B2>(q.d0, a0, b0), xv, RS::s(0, o0), ragged);
    st32r<R, DMIS>(rs, put2<B1, B2>(q.d1, a1, b1), xv, RS::s(N, o0), ragged);
    st32r<R, DMIS>(rs, put2<B1, B2>(q.d2, a2, b2), xv, RS::s(2 * N, o0), ragged);
    st32r<R, DMIS>(rs, put2<B1, B2>(q.d3, a3, b3), xv, RS::s(3 * N, o0), ragged);
}

// Entry i (0..63) of the two-theta table: theta = i / 32, index d + 16 with
// d = dc + 8 dh; entries that no (dc, dh) reaches hold 0.
template <bool LE>
__device__ __forceinline__ uint2 met_table_entry(const LatticeArgs& a, int i)
{
    const int th = i >> 5, dd = (i & 31) - 16;
    const int dh = (dd + 4) >> 3;
    const int dc = dd - 8 * dh;
    uint2 e = make_uint2(0u, 0u);
    if (dd >= -11 && dd <= 11 && dc >= -3 && dc <= 3) {
        const uint32_t thr = a.tab->met[th][(dh + 1) * 7 + dc + 3];
        e.x = LE ? (thr == 0xFFFFFFFFu ? thr : thr - 1u) : thr;
        e.y = (uint32_t)(dc + (dh << 10) + (1 << 20));
    }
    return e;
}

// The 32 entries of one theta's table in LDS (index d + 16); ends with a barrier.
template <bool LE = false>
__device__ __forceinline__ void met_table(const LatticeArgs& a, uint2* tbl, int theta)
{
    if (threadIdx.x < 32) tbl[threadIdx.x] = met_table_entry<LE>(a, 32 * theta + (int)threadIdx.x);
    __syncthreads();
}

__device__ __forceinline__ void met_reduce(uint32_t wsum, int64_t* slots, uint32_t slot)
{
    // unpack the per-lane sums: wsum = sum dc + 2^10 sum dh + 2^20 accepted.
    // Exact while the 10-bit fields hold the sums: a cell's four moves change
    // N_sigma of its six arm pairs by at most 6 and N_HB_raw of its four links
    // by at most 4 in all, so |sum dc| <= 6 and |sum dh| <= 4 per cell, and a
    // lane moves at most 64 cells per launch (32 rows of a column quad, or 64
    // rows of a column pair): |sum dc| <= 384, |sum dh| <= 256, accepted <= 256.
    const int ws = (int)wsum;
    const int sdc = (ws << 22) >> 22;
    const int r1v = (ws - sdc) >> 10;
    const int sdh = (r1v << 22) >> 22;
    const int nacc = (r1v - sdh) >> 10;
    const int v[3] = {sdh, sdc, nacc};
    block_add<3>(v, slots + (slot & (kSlots - 1)), kSlots);
}

// The waves of a SIMD are issued oldest first, so with equal work the oldest
// finish early and the SIMD ends the pass with few waves and poor latency
// hiding.  Lowering a wave's priority (s_setprio 3 -> 0) as it advances
// through its rows lets the laggards catch up: all waves stay resident until
// the last quarter of the pass.  it: the wave's row-pair index, n: its count.
// (Batched passes, whose workgroups belong to lattices of different sizes,
// measured faster without it: ON = false.)
template <bool ON>
struct ProgressPrio {
    uint32_t t1, t2, t3;                      // first row-pair index of levels 2, 1, 0
    __device__ __forceinline__ explicit ProgressPrio(uint32_t n)
        : t1((n + 3) / 4), t2((2 * n + 3) / 4), t3((3 * n + 3) / 4)
    {
        if (ON) __builtin_amdgcn_s_setprio(3);
    }
    __device__ __forceinline__ void step(uint32_t it) const
    {
        if (!ON) return;
        if (it == t1) __builtin_amdgcn_s_setprio(2);
        if (it == t2) __builtin_amdgcn_s_setprio(1);
        if (it == t3) __builtin_amdgcn_s_setprio(0);
    }
};

// No occupancy cap: the quad loop needs ~84 VGPRs (5 wavefronts per SIMD).
// Caps measured slower (64 VGPRs for 7 wavefronts without spills, or 8 with
// a small spill).  At L = 4096 the host picks 16 rows per wavefront: 1024
// workgroups, all resident at once.
//
// Start-up: nothing the first row's loads and the table need depends on the
// chain state, so the table entries of both theta values and the first row
// are requested before the state (skip flag, theta, step) is read, and the
// first wait covers all three at once.
template <int Q, int KAPPA, bool R, bool LE>
__global__ __launch_bounds__(256) void met_sweep4_kernel(LatticeArgs a)
{
    __shared__ uint2 tbl[64];
    const uint32_t tid = threadIdx.x;
    uint2 e = make_uint2(0u, 0u);
    if (tid < 64) e = met_table_entry<LE>(a, (int)tid);
    const uint32_t L = a.L;
    const uint32_t lane = tid & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t j = blockIdx.x * 64 + lane;
    const uint32_t y0 = (blockIdx.y * 4 + wave) * a.rows;      // even
    const bool active = j < ((L + 3) >> 2) && y0 < L;           // (L + 2) / 4 quads when R
    const uint32_t x4 = 4 * j;
    const bool ragged = R && x4 + 2 == L;
    const uint32_t x4h = ragged ? x4 : x4 + 2;                 // high halves of off-boundary rows
    const uint32_t xl = (x4 == 0) ? L - 1 : x4 - 1, xr = (x4 + 4 >= L) ? 0 : x4 + 4;
    const uint32_t y1 = min(y0 + a.rows, L);
    const __amdgpu_buffer_rsrc_t rs = sigma_rsrc(a.sigma, 4 * a.N);
    // even rows: updated cells at bytes KAPPA, KAPPA+2; odd rows: 1-KAPPA, 3-KAPPA
    constexpr int PE = KAPPA, PO = 1 - KAPPA;
    QuadBytes cur = {};
    if (active) cur = met_load4<PE, R, false>(a, rs, y0, x4, x4h, xl, xr);
    const int skip = a.st->skip, theta = a.st->theta;
    const uint32_t t = a.st->t_cur;
    if (tid < 64) tbl[tid] = e;
    __syncthreads();
    if (skip) return;                                          // step limit reached (uniform)
    const uint2* tb = tbl + (theta ? 32 : 0);
    uint32_t wsum = 0;
    if (active) {
        const ProgressPrio<true> prio((y1 - y0) >> 1);
        for (uint32_t y = y0; y < y1; y += 2) {
            prio.step((y - y0) >> 1);
            const QuadBytes odd = met_load4<PO, R, true>(a, rs, y + 1, x4, x4h, xl, xr);
            met_quad<Q, PE, R, false, LE>(a, rs, tb, t, y, x4, cur, wsum, ragged);
            const uint32_t yn = (y + 2 < y1) ? y + 2 : y;
            cur = met_load4<PE, R, false>(a, rs, yn, x4, x4h, xl, xr);
            met_quad<Q, PO, R, true, LE>(a, rs, tb, t, y + 1, x4, odd, wsum, ragged);
        }
    }
    met_reduce(wsum, a.slots, blockIdx.x + blockIdx.y * gridDim.x);
}

// Byte-lane variant (any even L): lane i owns the column pair (2i, 2i+1).
template <int Q, bool PRIO>
__device__ __forceinline__ uint32_t met_byte_block(const LatticeArgs& a, uint2* tbl, uint32_t t, int theta,
                                                   int colour, uint32_t bx, uint32_t by)
{
    const uint32_t L = a.L, half = L >> 1;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t pair = bx * 64 + lane;
    const uint32_t y0 = (by * 4 + wave) * a.rows;    // even
    const bool active = pair < half && y0 < L;
    // column of the updated cell in even rows (A) and odd rows (B), and its x neighbours
    const uint32_t xA = 2 * pair + colour, xB = 2 * pair + (1 - colour);
    const uint32_t xpA = (xA + 1 == L) ? 0 : xA + 1, xmA = (xA == 0) ? L - 1 : xA - 1;
    const uint32_t xpB = (xB + 1 == L) ? 0 : xB + 1, xmB = (xB == 0) ? L - 1 : xB - 1;
    const uint32_t y1 = min(y0 + a.rows, L);            // y1 - y0 is even
    const __amdgpu_buffer_rsrc_t rs = sigma_rsrc(a.sigma, 4 * a.N);
    // Software pipeline: the loads of the next row are issued before the
    // current row is computed.  They never alias its stores: the current
    // row writes only cells of the updated colour, the next row reads its
    // own (different) cells and facing arms of the other colour.
    CellBytes cur = {};
    if (active) cur = met_load(a, rs, y0, xA, xpA, xmA);
    met_table(a, tbl, theta);
    uint32_t wsum = 0;
    if (active) {
        const ProgressPrio<PRIO> prio((y1 - y0) >> 1);
        for (uint32_t y = y0; y < y1; y += 2) {
            prio.step((y - y0) >> 1);
            const CellBytes odd = met_load(a, rs, y + 1, xB, xpB, xmB);
            met_cell<Q>(a, rs, tbl, t, y, xA, cur, wsum);
            const uint32_t yn = (y + 2 < y1) ? y + 2 : y;     // last pair: a harmless re-read
            cur = met_load(a, rs, yn, xA, xpA, xmA);
            met_cell<Q>(a, rs, tbl, t, y + 1, xB, odd, wsum);
        }
    }
    return wsum;
}

template <int Q>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void met_sweep_kernel(LatticeArgs a, int colour)
{
    const int skip = a.st->skip, theta = a.st->theta;
    const uint32_t t = a.st->t_cur;
    if (skip) return;                                      // step limit reached
    // 32 entries: indices d + 16 for d in -15..15, so that even out-of-range
    // bond indices (a caller-supplied configuration) cannot read outside it.
    __shared__ uint2 tbl[32];
    const uint32_t wsum = met_byte_block<Q, true>(a, tbl, t, theta, colour, blockIdx.x, blockIdx.y);
    met_reduce(wsum, a.slots, blockIdx.x + blockIdx.y * gridDim.x);
}

// The chain c of workgroup b in a batched launch: start[c] <= b < start[c + 1]
// (start ascending, start[0] = 0), i.e. the number of chains whose first
// workgroup is at or before b, minus one.  Every wavefront counts them itself,
// 256 entries per round of four independent loads and ballots, instead of a
// binary search's chain of dependent loads.
__device__ __forceinline__ uint32_t batch_chain(const uint32_t* start, uint32_t count, uint32_t b)
{
    const uint32_t ln = threadIdx.x & 63;
    uint32_t nle = 0;
    for (uint32_t base = 0; base < count; base += 256) {
        uint32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t i = base + 64 * k + ln;
            v[k] = i < count ? start[i] : 0xFFFFFFFFu;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) nle += (uint32_t)__builtin_popcountll(__ballot(v[k] <= b));
    }
    return __builtin_amdgcn_readfirstlane(nle - 1);
}

// ---------------------------------------------------------------------------
// Batched colour pass: many independent chains of uneven L in one launch.
// Workgroup b belongs to the chain c with start[c] <= b < start[c+1].
// A chain's colour pass is cut into work units -- a row pair (2 rp, 2 rp + 1)
// times a column quad (L % 4 == 0) or a column pair (L % 4 == 2) -- numbered
// row pair major, and lane l of wavefront w of the chain's workgroup k moves
// the units (4 k + w) 64 K + l + 64 i, i < K.  No lane idles on a short row:
// a wavefront spans as many rows as 64 units cover (four row pairs of an
// L = 64 lattice), and only the chain's last wavefront can run out of units.
// Every unit is moved exactly as the chain's own launch moves it (same
// Philox counters, same update order inside a cell; cells of one colour do
// not interact), so each chain follows its standalone trajectory bit for bit.
// ---------------------------------------------------------------------------
// Batches are mostly small lattices: the 8-wavefront occupancy measured
// faster than the uncapped register budget.
template <int Q, int KAPPA, bool LE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void met_batch_kernel(
    const BatchEntry* __restrict__ ent, const uint32_t* __restrict__ start, uint32_t count)
{
    __shared__ uint2 tbl[32];
    const uint32_t lo = batch_chain(start, count, blockIdx.x);
    const LatticeArgs a = ent[lo].la;
    // the step state comes with the entry (written by the batched volume
    // kernel), not through a second, dependent load from la.st
    const int skip = ent[lo].skip, theta = ent[lo].theta;
    const uint32_t t = ent[lo].t_cur;
    if (skip) return;                                      // step limit reached
    const uint32_t units = ent[lo].units, upr = ent[lo].upr, K = ent[lo].iters;
    const double upr_inv = ent[lo].upr_inv;
    const uint32_t local = blockIdx.x - start[lo];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t first = (local * 4 + wave) * 64 * K + lane;
    const uint32_t L = a.L;
    const __amdgpu_buffer_rsrc_t rs = sigma_rsrc(a.sigma, 4 * a.N);
    uint32_t wsum = 0;
    if (a.quad) {
        constexpr int PE = KAPPA, PO = 1 - KAPPA;
        auto at = [&](uint32_t u, uint32_t& y, uint32_t& x4, uint32_t& xl, uint32_t& xr) {
            uint32_t qd;
            y = 2 * divmod(u, upr, upr_inv, qd);
            x4 = 4 * qd;
            xl = (x4 == 0) ? L - 1 : x4 - 1;
            xr = (x4 + 4 >= L) ? 0 : x4 + 4;
        };
        uint32_t y, x4, xl, xr;
        at(first, y, x4, xl, xr);
        QuadBytes cur = {};
        if (first < units) cur = met_load4<PE, false, false, true>(a, rs, y, x4, x4 + 2, xl, xr);
        met_table<LE>(a, tbl, theta);
        for (uint32_t i = 0; i < K; ++i) {
            const uint32_t u = first + 64 * i;
            const bool act = u < units;
            QuadBytes odd = {};
            if (act) {
                odd = met_load4<PO, false, true, true>(a, rs, y + 1, x4, x4 + 2, xl, xr);
                met_quad<Q, PE, false, false, LE, true>(a, rs, tbl, t, y, x4, cur, wsum, false);
            }
            const uint32_t un = u + 64;
            uint32_t yn, x4n, xln, xrn;
            at(un, yn, x4n, xln, xrn);
            if (i + 1 < K && un < units) cur = met_load4<PE, false, false, true>(a, rs, yn, x4n, x4n + 2, xln, xrn);
            if (act) met_quad<Q, PO, false, true, LE, true>(a, rs, tbl, t, y + 1, x4, odd, wsum, false);
            y = yn;
            x4 = x4n;
            xl = xln;
            xr = xrn;
        }
    } else {
        // column pairs: the updated cell of a pair sits at column 2 pr + KAPPA
        // in even rows and 2 pr + 1 - KAPPA in odd rows
        auto at = [&](uint32_t u, uint32_t& y, uint32_t& pr) { y = 2 * divmod(u, upr, upr_inv, pr); };
        auto nb = [&](uint32_t x, uint32_t& xp, uint32_t& xm) {
            xp = (x + 1 == L) ? 0 : x + 1;
            xm = (x == 0) ? L - 1 : x - 1;
        };
        uint32_t y, pr, xp, xm;
        at(first, y, pr);
        CellBytes cur = {};
        if (first < units) {
            nb(2 * pr + KAPPA, xp, xm);
            cur = met_load<true>(a, rs, y, 2 * pr + KAPPA, xp, xm);
        }
        met_table<LE>(a, tbl, theta);
        for (uint32_t i = 0; i < K; ++i) {
            const uint32_t u = first + 64 * i;
            const bool act = u < units;
            const uint32_t xA = 2 * pr + KAPPA, xB = 2 * pr + (1 - KAPPA);
            CellBytes odd = {};
            if (act) {
                nb(xB, xp, xm);
                odd = met_load<true>(a, rs, y + 1, xB, xp, xm);
                met_cell<Q, true, LE>(a, rs, tbl, t, y, xA, cur, wsum);
            }
            const uint32_t un = u + 64;
            uint32_t yn, prn;
            at(un, yn, prn);
            if (i + 1 < K && un < units) {
                nb(2 * prn + KAPPA, xp, xm);
                cur = met_load<true>(a, rs, yn, 2 * prn + KAPPA, xp, xm);
            }
            if (act) met_cell<Q, true, LE>(a, rs, tbl, t, y + 1, xB, odd, wsum);
            y = yn;
            pr = prn;
        }
    }
    met_reduce(wsum, a.slots, local);
}

// One wavefront per chain: fold and open the next step of every chain
// (mode kVolMet before a Metropolis sweep, kVolSw before an SW step).
__global__ __launch_bounds__(64) void volume_batch_kernel(BatchEntry* __restrict__ ent, int mode)
{
    __shared__ double term[40];
    VolArgs v = ent[blockIdx.x].va;
    v.mode = mode;
    if (mode != kVolMet) v.met_att_add = 0;
    volume_step(v, term, ent + blockIdx.x);
}

