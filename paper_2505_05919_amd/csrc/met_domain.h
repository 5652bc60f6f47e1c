// Arm-domain Metropolis pass kernels (included inside the kernels'
// namespace, after the checkerboard sweep, whose one-arm move, table and
// reduction they share).
#pragma once

// ---------------------------------------------------------------------------
// The paper's own parallel partition (Sec. II.C and its figure of layered
// domains), in 2-D: arm a of every cell forms a domain.  A bond index of arm
// a interacts with the three other arms of its cell and with arm a^1 of the
// neighbour in direction a -- none of them in the domain -- so one launch
// moves the whole domain, for any L (odd included).  A sweep is four passes,
// one per arm, in an order drawn per step.
//
// Work layout: lane i owns the column pair (2i, 2i+1) of a row -- the last
// pair of an odd row holds one cell -- and the wavefront walks `rows` rows.
// One Philox block per pair, row and pass: words 0, 1 (proposal, acceptance)
// for the even column, 2, 3 for the odd one.  Per row and lane: the four
// planes of the pair (16-bit loads when L is even), the two facing bytes, one
// store of the moved plane.
// ---------------------------------------------------------------------------

// Arm of pass `pass` at step t: Fisher-Yates on the words of
// Philox(0, t, 0, ORD), position i swapping with i + pick(w_i, 4 - i); pick
// for k = 4 and 2 is a shift, for k = 3 it is w / floor(2^32/3) with the
// NONE draw w = 2^32 - 1 keeping position 1.  The order lives in the nibbles
// of one register.
__device__ __forceinline__ uint32_t domain_arm(const LatticeArgs& a, uint32_t t, uint32_t pass)
{
    const uint4 w = philox(0u, t, 0u, kStreamOrd, a.key0, a.key1);
    uint32_t ord = 0x3210u;
    auto swap = [&ord](uint32_t i, uint32_t j) {
        const uint32_t vi = (ord >> (4 * i)) & 15u, vj = (ord >> (4 * j)) & 15u;
        ord &= ~((15u << (4 * i)) | (15u << (4 * j)));
        ord |= (vj << (4 * i)) | (vi << (4 * j));
    };
    swap(0, w.x >> 30);
    swap(1, 1 + (w.y == 0xFFFFFFFFu ? 0u : w.y / 1431655765u));
    swap(2, 2 + (w.z >> 31));
    return (ord >> (4 * pass)) & 15u;
}

// The rows of one wavefront for pass arm ARM (a template, so that the facing
// plane, the facing cell and the three other arms are fixed at compile time).
// EVEN: L even, so a pair never leaves its row and its two bytes of a plane
// are one aligned 16-bit word.
template <int Q, bool EVEN, int ARM>
__device__ __forceinline__ uint32_t dom_rows(const LatticeArgs& a, const uint2* tbl, uint32_t t, uint32_t pr,
                                             uint32_t y0, uint32_t y1)
{
    constexpr int B1 = ARM == 0 ? 1 : 0, B2 = ARM <= 1 ? 2 : 1, B3 = ARM == 3 ? 2 : 3;   // the other arms
    const uint32_t L = a.L, N = a.N, np = (L + 1) >> 1;
    const uint32_t x0 = 2 * pr, x1 = x0 + 1;
    const bool has1 = x1 < L;
    const uint32_t c1 = has1 ? x1 : x0;                    // a lone cell reads its own column twice
    // column of the facing cell: the x neighbours for arms 0, 1, else the same
    uint32_t fx0 = x0, fx1 = c1;
    if (ARM == 0) {
        fx0 = (x0 + 1 == L) ? 0 : x0 + 1;
        fx1 = (c1 + 1 == L) ? 0 : c1 + 1;
    } else if (ARM == 1) {
        fx0 = (x0 == 0) ? L - 1 : x0 - 1;
        fx1 = (c1 == 0) ? L - 1 : c1 - 1;
    }
    const __amdgpu_buffer_rsrc_t rs = sigma_rsrc(a.sigma, 4 * N);
    const uint32_t fp = (ARM ^ 1) * N, ap = ARM * N;
    uint32_t wsum = 0;
    for (uint32_t y = y0; y < y1; ++y) {
        const uint32_t o = y * L;
        const uint32_t fy = (ARM == 2) ? ((y + 1 == L) ? 0 : y + 1) : (ARM == 3) ? ((y == 0) ? L - 1 : y - 1) : y;
        uint32_t s0[4], s1[4];
#pragma unroll
        for (uint32_t b = 0; b < 4; ++b) {
            if (EVEN) {
                const uint32_t d = __builtin_amdgcn_raw_buffer_load_b16(rs, (int)x0, (int)(b * N + o), 0);
                s0[b] = (d & 255u) << 2;
                s1[b] = (d >> 8) << 2;
            } else {
                s0[b] = ld8(rs, x0, b * N + o) << 2;
                s1[b] = ld8(rs, c1, b * N + o) << 2;
            }
        }
        const uint32_t f0 = ld8(rs, fx0, fp + fy * L) << 2, f1 = ld8(rs, fx1, fp + fy * L) << 2;
        const uint4 w = philox(pr + np * y, t, ARM, kStreamDom, a.key0, a.key1);
        uint32_t a0 = s0[ARM], a1 = s1[ARM];
        met_arm<Q>(a0, (1u << s0[B1]) + (1u << s0[B2]) + (1u << s0[B3]) + (8u << f0), w.x, w.y, tbl, wsum);
        const uint32_t wkeep = wsum;                       // a lone cell's stand-in moves nothing
        met_arm<Q>(a1, (1u << s1[B1]) + (1u << s1[B2]) + (1u << s1[B3]) + (8u << f1), w.z, w.w, tbl, wsum);
        if (EVEN) {
            st16(rs, (a0 >> 2) | ((a1 >> 2) << 8), x0, ap + o);
        } else {
            if (!has1) wsum = wkeep;
            st8(rs, a0 >> 2, x0, ap + o);
            if (has1) st8(rs, a1 >> 2, x1, ap + o);
        }
    }
    return wsum;
}

// The rows of one wavefront for pass ARM when L % 4 == 0: lane j owns the
// quad of columns 4j..4j+3 (two column pairs, two Philox blocks) and moves
// whole dwords: the four planes, the facing bytes (the same dwords and one
// edge byte for arms 0 and 1, one dword of the neighbour row for arms 2 and
// 3), one dword store of the moved plane.
template <int Q, int ARM>
__device__ __forceinline__ uint32_t dom_rows_quad(const LatticeArgs& a, const uint2* tbl, uint32_t t, uint32_t j,
                                                  uint32_t y0, uint32_t y1)
{
    constexpr int B1 = ARM == 0 ? 1 : 0, B2 = ARM <= 1 ? 2 : 1, B3 = ARM == 3 ? 2 : 3;   // the other arms
    const uint32_t L = a.L, N = a.N, np = L >> 1;
    const uint32_t x4 = 4 * j;
    const uint32_t xl = (x4 == 0) ? L - 1 : x4 - 1, xr = (x4 + 4 == L) ? 0 : x4 + 4;
    const __amdgpu_buffer_rsrc_t rs = sigma_rsrc(a.sigma, 4 * N);
    const uint32_t ap = ARM * N;
    uint32_t wsum = 0;
    for (uint32_t y = y0; y < y1; ++y) {
        const uint32_t o = y * L;
        uint32_t D[4];
#pragma unroll
        for (uint32_t b = 0; b < 4; ++b) D[b] = ld32(rs, x4, b * N + o) << 2;   // bytes hold 4 sigma
        uint32_t f[4];
        if (ARM == 0) {
            f[0] = byte4<1>(D[1]);
            f[1] = byte4<2>(D[1]);
            f[2] = byte4<3>(D[1]);
            f[3] = ld8(rs, xr, N + o) << 2;
        } else if (ARM == 1) {
            f[0] = ld8(rs, xl, o) << 2;
            f[1] = byte4<0>(D[0]);
            f[2] = byte4<1>(D[0]);
            f[3] = byte4<2>(D[0]);
        } else {
            const uint32_t fy = (ARM == 2) ? ((y + 1 == L) ? 0 : y + 1) : ((y == 0) ? L - 1 : y - 1);
            const uint32_t F = ld32(rs, x4, (ARM ^ 1) * N + fy * L) << 2;
            f[0] = byte4<0>(F);
            f[1] = byte4<1>(F);
            f[2] = byte4<2>(F);
            f[3] = byte4<3>(F);
        }
        const uint4 wa = philox(2 * j + np * y, t, ARM, kStreamDom, a.key0, a.key1);
        const uint4 wb = philox(2 * j + 1 + np * y, t, ARM, kStreamDom, a.key0, a.key1);
        uint32_t s[4];
#define CVF_DOM_CELL(K, W0, W1)                                                                             \
        {                                                                                                   \
            s[K] = byte4<K>(D[ARM]);                                                                        \
            const uint32_t z = (1u << byte4<K>(D[B1])) + (1u << byte4<K>(D[B2])) + (1u << byte4<K>(D[B3])) + \
                               (8u << f[K]);                                                                \
            met_arm<Q>(s[K], z, W0, W1, tbl, wsum);                                                         \
        }
        CVF_DOM_CELL(0, wa.x, wa.y)
        CVF_DOM_CELL(1, wa.z, wa.w)
        CVF_DOM_CELL(2, wb.x, wb.y)
        CVF_DOM_CELL(3, wb.z, wb.w)
#undef CVF_DOM_CELL
        st32(rs, (s[0] >> 2) | ((s[1] >> 2) << 8) | ((s[2] >> 2) << 16) | ((s[3] >> 2) << 24), x4, ap + o);
    }
    return wsum;
}

// MODE 0: column pairs, odd L; 1: column pairs, L % 4 == 2; 2: quads, L % 4 == 0.
template <int Q, int MODE>
__global__ __launch_bounds__(256) void met_domain_kernel(LatticeArgs a, uint32_t pass, uint32_t rows)
{
    const int skip = a.st->skip, theta = a.st->theta;
    const uint32_t t = a.st->t_cur;
    if (skip) return;                                      // step limit reached
    __shared__ uint2 tbl[32];
    const uint32_t arm = __builtin_amdgcn_readfirstlane(domain_arm(a, t, pass));
    const uint32_t L = a.L;
    const uint32_t lanes = MODE == 2 ? (L >> 2) : ((L + 1) >> 1);    // quads or pairs per row
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t j = blockIdx.x * 64 + lane;
    const uint32_t y0 = (blockIdx.y * 4 + wave) * rows;
    met_table(a, tbl, theta);
    uint32_t wsum = 0;
    if (j < lanes && y0 < L) {
        const uint32_t y1 = min(y0 + rows, L);
        constexpr bool EVEN = MODE != 0;
        switch (arm) {                                     // wave-uniform
        case 0: wsum = MODE == 2 ? dom_rows_quad<Q, 0>(a, tbl, t, j, y0, y1) : dom_rows<Q, EVEN, 0>(a, tbl, t, j, y0, y1); break;
        case 1: wsum = MODE == 2 ? dom_rows_quad<Q, 1>(a, tbl, t, j, y0, y1) : dom_rows<Q, EVEN, 1>(a, tbl, t, j, y0, y1); break;
        case 2: wsum = MODE == 2 ? dom_rows_quad<Q, 2>(a, tbl, t, j, y0, y1) : dom_rows<Q, EVEN, 2>(a, tbl, t, j, y0, y1); break;
        default: wsum = MODE == 2 ? dom_rows_quad<Q, 3>(a, tbl, t, j, y0, y1) : dom_rows<Q, EVEN, 3>(a, tbl, t, j, y0, y1); break;
        }
    }
    met_reduce(wsum, a.slots, blockIdx.x + blockIdx.y * gridDim.x);
}
