// HIP kernels of libcvf for gfx950 (MI355X).
//
// The lattice kernels are integer-only: uint8 bond indices, uint32 Philox
// words and thresholds, int32 per-lane deltas reduced across the wavefront
// and the workgroup, int64 atomics into spread slots.  The single-wave
// volume kernel is the only floating-point code (FP64, no contraction).
#include "cvf_internal.h"

namespace cvf {
namespace {

constexpr int kBlock = 256;           // 4 wavefronts of 64
constexpr int kMaxBlocks = 8192;      // 256 CUs x 8 waves/SIMD x 4 SIMDs / 4 waves

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The key words are
// wave-uniform (the chain's seed), so the key schedule lives in SGPRs.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mulhilo(uint32_t m, uint32_t x, uint32_t& hi, uint32_t& lo)
{
    const uint64_t p = (uint64_t)m * (uint64_t)x;     // one v_mad_u64_u32
    hi = (uint32_t)(p >> 32);
    lo = (uint32_t)p;
}

__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo(0xD2511F53u, c0, hi0, lo0);
        mulhilo(0xCD9E8D57u, c2, hi1, lo1);
        const uint32_t n0 = hi1 ^ (c1 ^ k0);
        const uint32_t n2 = hi0 ^ (c3 ^ k1);
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return make_uint4(c0, c1, c2, c3);
}

// floor(j / d) and j mod d for j < 2^32, d < 2^15: one FP64 multiply by the
// reciprocal is at most one too small, never too large; one correction.
__device__ __forceinline__ uint32_t divmod(uint32_t j, uint32_t d, double inv, uint32_t& rem)
{
    uint32_t qt = (uint32_t)((double)j * inv);
    uint32_t r = j - qt * d;
    if (r >= d) {
        ++qt;
        r -= d;
    }
    rem = r;
    return qt;
}

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum NV int32 values over the workgroup and add them (as int64) to
// dst[i * stride] (one atomic per value per workgroup).
template <int NV>
__device__ __forceinline__ void block_add(const int (&v)[NV], int64_t* dst, int stride)
{
    __shared__ int part[NV][kBlock / 64];
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int s = wave_sum(v[i]);
        if (lane == 0) part[i][wave] = s;
    }
    __syncthreads();
    if (tid < NV) {
        int64_t s = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) s += part[tid][w];
        if (s) atomicAdd((unsigned long long*)(dst + (size_t)tid * stride), (unsigned long long)s);
    }
}

inline unsigned grid_for(uint64_t work)
{
    uint64_t b = (work + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > kMaxBlocks) b = kMaxBlocks;
    return (unsigned)b;
}

// ---------------------------------------------------------------------------
// Lennard-Jones lattice energy per molecule (Sec. II.A): hard core r0,
// cutoff 6 r0, square lattice of spacing sqrt(v) r0.  Same operation order as
// the definition: ascending shells m = |n|^2, s = (v m)^-3, 2 sum r2 (s^2-s).
// ---------------------------------------------------------------------------
__device__ double lj_energy(double v, const double* r2)
{
    double s = 0.0;
    for (int m = 1; v * (double)m <= 36.0; ++m) {
        const double d2 = v * (double)m;
        const double s6 = 1.0 / (d2 * d2 * d2);
        s = s + r2[m] * (s6 * s6 - s6);
    }
    return 2.0 * s;
}

// ---------------------------------------------------------------------------
// State initialisation.
// ---------------------------------------------------------------------------
__global__ void state_init_kernel(DevState* st, int64_t* slots, const DevTables* tab, double v_init)
{
    const int i = threadIdx.x;
    for (int k = i; k < 3 * kSlots; k += blockDim.x) slots[k] = 0;
    if (i == 0) {
        st->t_next = 0;
        st->n_hb_raw = 0;
        st->n_coop = 0;
        st->met_att = st->met_acc = st->vol_att = st->vol_acc = 0;
        st->v = v_init;
        st->u = lj_energy(v_init, tab->r2);
        st->t_cur = 0;
        st->theta = v_init < 2.0 ? 1 : 0;
        st->sw_done = 0;
        st->pad_ = 0;
    }
}

// sigma[a][c] = floor(w_a q / 2^32), (w0..w3) = Philox(c, 0, 0, INIT).
__global__ __launch_bounds__(kBlock) void sigma_init_kernel(LatticeArgs a)
{
    for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < a.N; c += gridDim.x * kBlock) {
        const uint4 w = philox(c, 0u, 0u, kStreamInit, a.key0, a.key1);
        a.sigma[c] = (uint8_t)(((uint64_t)w.x * a.q) >> 32);
        a.sigma[(size_t)a.N + c] = (uint8_t)(((uint64_t)w.y * a.q) >> 32);
        a.sigma[2 * (size_t)a.N + c] = (uint8_t)(((uint64_t)w.z * a.q) >> 32);
        a.sigma[3 * (size_t)a.N + c] = (uint8_t)(((uint64_t)w.w * a.q) >> 32);
    }
}

// ---------------------------------------------------------------------------
// Volume move + counter fold: one wavefront.  Folds the per-workgroup slots
// of the previous sigma update into the totals, opens step t, and performs
// the Metropolis move of v_iso (Sec. II.B step 1) with the full dH of
// Eq. (1) and (3):  N (u(v') - u(v)) + P N (v' - v)
//                   + (theta(v') - theta(v)) (P v_HB - J) N_HB_raw.
// u(v) of the current volume is cached; the shell terms of u(v') are
// evaluated one per lane and summed by lane 0 in ascending shell order, the
// same order as the sequential definition.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void volume_kernel(VolArgs a)
{
    __shared__ double term[40];
    const int lane = threadIdx.x;
    int64_t hb = 0, co = 0, ac = 0;
    for (int i = lane; i < kSlots; i += 64) {
        hb += a.slots[i];
        co += a.slots[kSlots + i];
        ac += a.slots[2 * kSlots + i];
        a.slots[i] = 0;
        a.slots[kSlots + i] = 0;
        a.slots[2 * kSlots + i] = 0;
    }
    hb = wave_sum64(hb);
    co = wave_sum64(co);
    ac = wave_sum64(ac);
    DevState* st = a.st;
    if (a.mode == kVolFold) {
        if (lane == 0) {
            st->n_hb_raw += hb;
            st->n_coop += co;
            st->met_acc += ac;
        }
        return;
    }
    const uint32_t t = (uint32_t)st->t_next;
    const uint4 w = philox(0u, t, 0u, kStreamVol, a.key0, a.key1);
    const double u = (double)((int64_t)2 * (int64_t)w.x + 1 - 4294967296LL) * (1.0 / 4294967296.0);
    const double v0 = st->v;
    const double v1 = v0 + a.dv_max * u;
    const bool inside = a.do_volume && v1 >= 1.0;
    if (inside && lane >= 1 && lane <= 36) {
        const double d2 = v1 * (double)lane;
        const double s6 = 1.0 / (d2 * d2 * d2);
        term[lane] = a.tab->r2[lane] * (s6 * s6 - s6);
    }
    __syncthreads();
    if (lane != 0) return;
    st->n_hb_raw += hb;
    st->n_coop += co;
    st->met_acc += ac;
    st->t_cur = t;
    st->t_next += 1;
    st->met_att += a.met_att_add;
    if (a.do_volume) {
        st->vol_att += 1;
        if (inside) {
            double sum = 0.0;
            for (int m = 1; v1 * (double)m <= 36.0; ++m) sum = sum + term[m];
            const double u1 = 2.0 * sum;
            const int th0 = st->theta;
            const int th1 = v1 < 2.0 ? 1 : 0;
            const double dH = (a.Nd * (u1 - st->u))
                            + ((a.P * a.Nd) * (v1 - v0))
                            + (((double)(th1 - th0) * (a.P * a.vHB - a.J)) * (double)st->n_hb_raw);
            bool acc = dH <= 0.0;
            if (!acc) acc = ((double)w.y + 0.5) * (1.0 / 4294967296.0) < exp(-a.beta * dH);
            if (acc) {
                st->v = v1;
                st->u = u1;
                st->theta = th1;
                st->vol_acc += 1;
            }
        }
    }
    if (a.mode == kVolSw) {         // the SW step ends with a full recount
        st->n_hb_raw = 0;
        st->n_coop = 0;
    }
}

// ---------------------------------------------------------------------------
// Checkerboard Metropolis: every cell of one colour, arms 0..3 in order
// (Sec. II.C).  Cells of one colour share no interaction: arm a of c only
// couples to the other arms of c (J_sigma) and to arm a^1 of the neighbour
// in direction a (J_eff), which has the other colour.
//
// Work layout: lane i of a wavefront owns the column pair (2i, 2i+1) and
// walks `rows` consecutive rows; in every row exactly one of its two cells
// has the colour being updated.  Row addresses are wave-uniform (SGPR base +
// lane column), so the loop carries no vector address arithmetic.
//
// Energy bookkeeping without compares: bond indices are held as 4*sigma and
// Z = sum_{b != a} 1 << 4 sigma_b  +  8 << 4 sigma_facing
// packs, per state v, (#other arms in v) + 8 [facing arm in v] into a 4-bit
// field, so bfe(Z, new) - bfe(Z, old) = dc + 8 dh (dc in -3..3, dh in -1..1)
// indexes an LDS table holding the acceptance threshold and a packed
// counter increment (dc + 2^10 dh + 2^20 for one accepted move).
// ---------------------------------------------------------------------------
template <int Q>
__device__ __forceinline__ void met_arm(uint32_t& s4, uint32_t Z, uint32_t prop, uint32_t accw,
                                        const uint2* tbl, uint32_t& wsum)
{
    constexpr uint32_t M = Q - 1;                         // proposals: the q-1 other states
    // k = floor(prop / floor(2^32/M)); kp = k + 1 = high word of (prop' M + 2^32).
    // M in {3, 5} divides 2^32 - 1 and needs prop' = prop + 1 (prop = 2^32-1 is the
    // NULL proposal); M in {1, 2, 4} divides 2^32 and has no NULL proposal.
    constexpr bool kHasNull = (M == 3 || M == 5);
    const uint32_t pp = kHasNull ? prop + 1u : prop;
    const uint32_t kp = (uint32_t)(((uint64_t)pp * M + (1ull << 32)) >> 32);
    const uint32_t t4 = s4 + (kp << 2);                   // 4 (sigma + 1 + k)
    const uint32_t sn4 = min(t4, t4 - 4u * Q);            // mod q, in units of 4
    const int d = (int)__builtin_amdgcn_ubfe(Z, sn4, 4) - (int)__builtin_amdgcn_ubfe(Z, s4, 4);
    const uint2 e = tbl[d + 16];
    bool acc = min(accw, 0xFFFFFFFEu) < e.x;              // thr == 2^32-1 always accepts
    if (kHasNull) acc = acc && pp != 0u;
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

// Loads for the cell at column x of row y (wave-uniform y: every row/plane
// offset is a scalar register).
__device__ __forceinline__ CellBytes met_load(const LatticeArgs& a, __amdgpu_buffer_rsrc_t rs, uint32_t y,
                                              uint32_t x, uint32_t xp, uint32_t xm)
{
    const uint32_t L = a.L, N = a.N;
    const uint32_t yp = (y + 1 == L) ? 0 : y + 1, ym = (y == 0) ? L - 1 : y - 1;
    const uint32_t o0 = y * L;
    CellBytes b;
    b.s0 = ld8(rs, x, o0);
    b.s1 = ld8(rs, x, o0 + N);
    b.s2 = ld8(rs, x, o0 + 2 * N);
    b.s3 = ld8(rs, x, o0 + 3 * N);
    b.f0 = ld8(rs, xp, o0 + N);                 // arm 1 of the +x neighbour
    b.f1 = ld8(rs, xm, o0);                     // arm 0 of the -x neighbour
    b.f2 = ld8(rs, x, 3 * N + yp * L);          // arm 3 of the +y neighbour
    b.f3 = ld8(rs, x, 2 * N + ym * L);          // arm 2 of the -y neighbour
    return b;
}

// Update the four arms of the cell (x, y) from its loaded bytes and store them.
template <int Q>
__device__ __forceinline__ void met_cell(const LatticeArgs& a, __amdgpu_buffer_rsrc_t rs, const uint2* tbl,
                                         uint32_t t, uint32_t y, uint32_t x, const CellBytes& b, uint32_t& wsum)
{
    const uint32_t N = a.N, o0 = y * a.L;
    uint32_t s0 = b.s0 << 2, s1 = b.s1 << 2, s2 = b.s2 << 2, s3 = b.s3 << 2;
    const uint32_t f0 = b.f0 << 2, f1 = b.f1 << 2, f2 = b.f2 << 2, f3 = b.f3 << 2;
    const uint32_t c = x + o0;
    const uint4 wa = philox(c, t, 0u, kStreamMet, a.key0, a.key1);
    const uint4 wb = philox(c, t, 1u, kStreamMet, a.key0, a.key1);
    const uint32_t p23 = (1u << s2) + (1u << s3);
    met_arm<Q>(s0, p23 + (1u << s1) + (8u << f0), wa.x, wa.y, tbl, wsum);
    met_arm<Q>(s1, p23 + (1u << s0) + (8u << f1), wa.z, wa.w, tbl, wsum);
    const uint32_t p01 = (1u << s0) + (1u << s1);
    met_arm<Q>(s2, p01 + (1u << s3) + (8u << f2), wb.x, wb.y, tbl, wsum);
    met_arm<Q>(s3, p01 + (1u << s2) + (8u << f3), wb.z, wb.w, tbl, wsum);
    st8(rs, s0 >> 2, x, o0);
    st8(rs, s1 >> 2, x, o0 + N);
    st8(rs, s2 >> 2, x, o0 + 2 * N);
    st8(rs, s3 >> 2, x, o0 + 3 * N);
}

// ---------------------------------------------------------------------------
// Quad variant (L % 4 == 0): lane j owns the four columns 4j..4j+3 and moves
// whole dwords of every plane.  In a row of parity P the updated cells sit at
// bytes P and P+2 of the quad; their x neighbours are the other bytes of the
// same dwords except one, fetched with a single byte load (the column left of
// the quad for P = 0, right of it for P = 1).  The two bytes of the other
// colour are written back unchanged -- nothing writes them during this pass.
// Per row and lane: 6 dword loads + 1 byte load + 4 dword stores for 2 cells.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ld32(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
}

__device__ __forceinline__ void st32(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)voff, (int)soff, 0);
}

struct QuadBytes {
    uint32_t d0, d1, d2, d3;   // arms 0..3 of the quad, row y
    uint32_t up3, dn2;         // arm 3 of row y+1, arm 2 of row y-1
    uint32_t edge;             // P=0: arm 0 of the column left of the quad; P=1: arm 1 right of it
};

template <int P>
__device__ __forceinline__ QuadBytes met_load4(const LatticeArgs& a, __amdgpu_buffer_rsrc_t rs, uint32_t y,
                                               uint32_t x4, uint32_t xl, uint32_t xr)
{
    const uint32_t L = a.L, N = a.N;
    const uint32_t yp = (y + 1 == L) ? 0 : y + 1, ym = (y == 0) ? L - 1 : y - 1;
    const uint32_t o0 = y * L;
    QuadBytes q;
    q.d0 = ld32(rs, x4, o0);
    q.d1 = ld32(rs, x4, o0 + N);
    q.d2 = ld32(rs, x4, o0 + 2 * N);
    q.d3 = ld32(rs, x4, o0 + 3 * N);
    q.up3 = ld32(rs, x4, 3 * N + yp * L);
    q.dn2 = ld32(rs, x4, 2 * N + ym * L);
    q.edge = (P == 0) ? ld8(rs, xl, o0) : ld8(rs, xr, o0 + N);
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

template <int Q, int P>
__device__ __forceinline__ void met_quad(const LatticeArgs& a, __amdgpu_buffer_rsrc_t rs, const uint2* tbl,
                                         uint32_t t, uint32_t y, uint32_t x4, const QuadBytes& q, uint32_t& wsum)
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
        const uint32_t f0 = byte4<B1 + 1>(D1);                          // arm 1, column +1
        const uint32_t f1 = (P == 0) ? E : byte4<(B1 > 0 ? B1 - 1 : 0)>(D0);   // arm 0, column -1
        const uint32_t f2 = byte4<B1>(U3), f3 = byte4<B1>(M2);
        const uint32_t c = x4 + B1 + o0;
        const uint4 wa = philox(c, t, 0u, kStreamMet, a.key0, a.key1);
        const uint4 wb = philox(c, t, 1u, kStreamMet, a.key0, a.key1);
        const uint32_t p23 = (1u << a2) + (1u << a3);
        met_arm<Q>(a0, p23 + (1u << a1) + (8u << f0), wa.x, wa.y, tbl, wsum);
        met_arm<Q>(a1, p23 + (1u << a0) + (8u << f1), wa.z, wa.w, tbl, wsum);
        const uint32_t p01 = (1u << a0) + (1u << a1);
        met_arm<Q>(a2, p01 + (1u << a3) + (8u << f2), wb.x, wb.y, tbl, wsum);
        met_arm<Q>(a3, p01 + (1u << a2) + (8u << f3), wb.z, wb.w, tbl, wsum);
    }
    {
        const uint32_t f0 = (P == 1) ? E : byte4<(B2 < 3 ? B2 + 1 : 3)>(D1);
        const uint32_t f1 = byte4<B2 - 1>(D0);
        const uint32_t f2 = byte4<B2>(U3), f3 = byte4<B2>(M2);
        const uint32_t c = x4 + B2 + o0;
        const uint4 wa = philox(c, t, 0u, kStreamMet, a.key0, a.key1);
        const uint4 wb = philox(c, t, 1u, kStreamMet, a.key0, a.key1);
        const uint32_t p23 = (1u << b2) + (1u << b3);
        met_arm<Q>(b0, p23 + (1u << b1) + (8u << f0), wa.x, wa.y, tbl, wsum);
        met_arm<Q>(b1, p23 + (1u << b0) + (8u << f1), wa.z, wa.w, tbl, wsum);
        const uint32_t p01 = (1u << b0) + (1u << b1);
        met_arm<Q>(b2, p01 + (1u << b3) + (8u << f2), wb.x, wb.y, tbl, wsum);
        met_arm<Q>(b3, p01 + (1u << b2) + (8u << f3), wb.z, wb.w, tbl, wsum);
    }
    st32(rs, put2<B1, B2>(q.d0, a0, b0), x4, o0);
    st32(rs, put2<B1, B2>(q.d1, a1, b1), x4, o0 + N);
    st32(rs, put2<B1, B2>(q.d2, a2, b2), x4, o0 + 2 * N);
    st32(rs, put2<B1, B2>(q.d3, a3, b3), x4, o0 + 3 * N);
}

__device__ __forceinline__ void met_table(const LatticeArgs& a, uint2* tbl)
{
    const int theta = a.st->theta;
    const int tid = threadIdx.x;
    if (tid < 32) {
        const int dd = tid - 16;                          // dc + 8 dh
        const int dh = (dd + 4) >> 3;
        const int dc = dd - 8 * dh;
        uint2 e = make_uint2(0u, 0u);
        if (dd >= -11 && dd <= 11 && dc >= -3 && dc <= 3) {
            e.x = a.tab->met[theta][(dh + 1) * 7 + dc + 3];
            e.y = (uint32_t)(dc + (dh << 10) + (1 << 20));
        }
        tbl[tid] = e;
    }
    __syncthreads();
}

__device__ __forceinline__ void met_reduce(uint32_t wsum, int64_t* slots)
{
    // unpack the per-lane sums: wsum = sum dc + 2^10 sum dh + 2^20 accepted
    const int ws = (int)wsum;
    const int sdc = (ws << 22) >> 22;
    const int r1v = (ws - sdc) >> 10;
    const int sdh = (r1v << 22) >> 22;
    const int nacc = (r1v - sdh) >> 10;
    const int v[3] = {sdh, sdc, nacc};
    block_add<3>(v, slots + ((blockIdx.x + blockIdx.y * gridDim.x) & (kSlots - 1)), kSlots);
}

// 8 wavefronts per SIMD (<= 64 VGPRs): the latency of the row loads and of the
// LDS table lookups is hidden by the other waves.
template <int Q, int KAPPA>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void met_sweep4_kernel(LatticeArgs a)
{
    __shared__ uint2 tbl[32];
    met_table(a, tbl);
    const uint32_t t = a.st->t_cur;
    const uint32_t L = a.L;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t j = blockIdx.x * 64 + lane;
    const uint32_t y0 = (blockIdx.y * 4 + wave) * a.rows;    // even
    uint32_t wsum = 0;
    if (j < (L >> 2) && y0 < L) {
        const uint32_t x4 = 4 * j;
        const uint32_t xl = (x4 == 0) ? L - 1 : x4 - 1, xr = (x4 + 4 == L) ? 0 : x4 + 4;
        const uint32_t y1 = min(y0 + a.rows, L);
        const __amdgpu_buffer_rsrc_t rs = sigma_rsrc(a.sigma, 4 * a.N);
        // even rows: updated cells at bytes KAPPA, KAPPA+2; odd rows: 1-KAPPA, 3-KAPPA
        constexpr int PE = KAPPA, PO = 1 - KAPPA;
        QuadBytes cur = met_load4<PE>(a, rs, y0, x4, xl, xr);
        for (uint32_t y = y0; y < y1; y += 2) {
            const QuadBytes odd = met_load4<PO>(a, rs, y + 1, x4, xl, xr);
            met_quad<Q, PE>(a, rs, tbl, t, y, x4, cur, wsum);
            const uint32_t yn = (y + 2 < y1) ? y + 2 : y;
            cur = met_load4<PE>(a, rs, yn, x4, xl, xr);
            met_quad<Q, PO>(a, rs, tbl, t, y + 1, x4, odd, wsum);
        }
    }
    met_reduce(wsum, a.slots);
}

template <int Q>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void met_sweep_kernel(LatticeArgs a, int colour)
{
    // 32 entries: indices d + 16 for d in -15..15, so that even out-of-range
    // bond indices (a caller-supplied configuration) cannot read outside it.
    __shared__ uint2 tbl[32];
    met_table(a, tbl);
    const uint32_t t = a.st->t_cur;
    const uint32_t L = a.L, half = L >> 1;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t pair = blockIdx.x * 64 + lane;
    const uint32_t y0 = (blockIdx.y * 4 + wave) * a.rows;    // even
    uint32_t wsum = 0;
    if (pair < half && y0 < L) {
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
        CellBytes cur = met_load(a, rs, y0, xA, xpA, xmA);
        for (uint32_t y = y0; y < y1; y += 2) {
            const CellBytes odd = met_load(a, rs, y + 1, xB, xpB, xmB);
            met_cell<Q>(a, rs, tbl, t, y, xA, cur, wsum);
            const uint32_t yn = (y + 2 < y1) ? y + 2 : y;     // last pair: a harmless re-read
            cur = met_load(a, rs, yn, xA, xpA, xmA);
            met_cell<Q>(a, rs, tbl, t, y + 1, xB, odd, wsum);
        }
    }
    met_reduce(wsum, a.slots);
}

// ---------------------------------------------------------------------------
// Full recount of N_HB_raw, N_sigma (and optionally N_q').
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void recount_kernel(LatticeArgs a, int64_t* out, int spread, int with_counts)
{
    const uint32_t L = a.L;
    const size_t N = a.N;
    const double inv_L = 1.0 / (double)L;
    const uint8_t* __restrict__ s = a.sigma;
    int hb = 0, co = 0;
    int cnt[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < a.N; c += gridDim.x * kBlock) {
        uint32_t x;
        const uint32_t y = divmod(c, L, inv_L, x);
        const uint32_t row = y * L;
        const uint32_t xp = (x + 1 == L) ? 0 : x + 1;
        const uint32_t rp = (y + 1 == L) ? 0 : row + L;
        const int s0 = s[c], s1 = s[N + c], s2 = s[2 * N + c], s3 = s[3 * N + c];
        hb += (s0 == s[N + xp + row]) + (s2 == s[3 * N + x + rp]);
        co += (s0 == s1) + (s0 == s2) + (s0 == s3) + (s1 == s2) + (s1 == s3) + (s2 == s3);
        if (with_counts) {
#pragma unroll
            for (int k = 0; k < 6; ++k) cnt[k] += (s0 == k) + (s1 == k) + (s2 == k) + (s3 == k);
        }
    }
    if (with_counts) {
        const int v[8] = {hb, co, cnt[0], cnt[1], cnt[2], cnt[3], cnt[4], cnt[5]};
        block_add<8>(v, out, 1);
    } else {
        const int v[2] = {hb, co};
        block_add<2>(v, out + (blockIdx.x & (spread - 1)), spread);
    }
}

__global__ void obs_zero_kernel(DevObs* o)
{
    if (threadIdx.x < 8) o->acc[threadIdx.x] = 0;
}

// Observables from the recount and the chain scalars (Eq. (1), (3)).
__global__ void obs_final_kernel(DevObs* o, const DevState* st, const DevTables* tab, double Nd, double J,
                                 double Jsigma, double P, double vHB)
{
    if (threadIdx.x != 0) return;
    cvf_obs& r = o->out;
    r.step = st->t_next;
    r.n_hb_raw = o->acc[0];
    r.n_hb = st->theta ? o->acc[0] : 0;
    r.n_coop = o->acc[1];
    int64_t mx = 0;
    for (int k = 0; k < 6; ++k) {
        r.count[k] = o->acc[2 + k];
        mx = r.count[k] > mx ? r.count[k] : mx;
    }
    r.met_attempted = st->met_att;
    r.met_accepted = st->met_acc;
    r.vol_attempted = st->vol_att;
    r.vol_accepted = st->vol_acc;
    r.v = st->v;
    r.V = (Nd * st->v) + (vHB * (double)r.n_hb);
    r.H = (((Nd * lj_energy(st->v, tab->r2)) - (J * (double)r.n_hb)) - (Jsigma * (double)r.n_coop)) + (P * r.V);
    r.M = (double)mx / (4.0 * Nd);
    r.consistent = (st->n_hb_raw == o->acc[0] && st->n_coop == o->acc[1]) ? 1 : 0;
    r.reserved = 0;
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

__global__ __launch_bounds__(kBlock) void sw_bonds_kernel(LatticeArgs a)
{
    __shared__ uint8_t lut[64];
    build_incell_lut(lut);
    __syncthreads();
    const uint32_t t = a.st->t_cur;
    const int theta = a.st->theta;
    const uint64_t thr_s = a.tab->sw[0];
    const uint64_t thr_e = a.tab->sw[1 + theta];
    const bool cov_on = theta == 1 && a.jeff_sign != 0;
    const uint32_t L = a.L;
    const size_t N = a.N;
    const double inv_L = 1.0 / (double)L;
    const uint8_t* __restrict__ s = a.sigma;
    for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < a.N; c += gridDim.x * kBlock) {
        uint32_t x;
        const uint32_t y = divmod(c, L, inv_L, x);
        const uint32_t row = y * L;
        const uint32_t xp = (x + 1 == L) ? 0 : x + 1;
        const uint32_t rp = (y + 1 == L) ? 0 : row + L;
        const int s0 = s[c], s1 = s[N + c], s2 = s[2 * N + c], s3 = s[3 * N + c];
        const int f0 = s[N + xp + row];
        const int f2 = s[3 * N + x + rp];
        const uint4 w0 = philox(c, t, 0u, kStreamSwb, a.key0, a.key1);
        const uint4 w1 = philox(c, t, 1u, kStreamSwb, a.key0, a.key1);
        uint32_t m = 0;
        if (cov_on) {
            const bool e0 = (s0 == f0) == (a.jeff_sign > 0);
            const bool e2 = (s2 == f2) == (a.jeff_sign > 0);
            m |= (e0 && below(w0.x, thr_e)) ? 1u : 0u;
            m |= (e2 && below(w0.y, thr_e)) ? 2u : 0u;
        }
        m |= (s0 == s1 && below(w0.z, thr_s)) ? 4u : 0u;
        m |= (s0 == s2 && below(w0.w, thr_s)) ? 8u : 0u;
        m |= (s0 == s3 && below(w1.x, thr_s)) ? 16u : 0u;
        m |= (s1 == s2 && below(w1.y, thr_s)) ? 32u : 0u;
        m |= (s1 == s3 && below(w1.z, thr_s)) ? 64u : 0u;
        m |= (s2 == s3 && below(w1.w, thr_s)) ? 128u : 0u;
        a.mask[c] = (uint8_t)m;
        const uint32_t l4 = lut[m >> 2];
        a.label[c] = (l4 & 3) * (uint32_t)N + c;
        a.label[N + c] = ((l4 >> 2) & 3) * (uint32_t)N + c;
        a.label[2 * N + c] = ((l4 >> 4) & 3) * (uint32_t)N + c;
        a.label[3 * N + c] = ((l4 >> 6) & 3) * (uint32_t)N + c;
    }
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

// Lock-free union by minimum index (atomicMin on the larger root).  A failed
// attempt means the larger root got a parent meanwhile; that parent is then
// united with the smaller root, so no connection is lost.  The largest of
// the two roots strictly decreases each round.
__device__ void unite(uint32_t* label, uint32_t a, uint32_t b)
{
    a = find_root(label, a);
    b = find_root(label, b);
    while (a != b) {
        if (a > b) {
            const uint32_t tmp = a;
            a = b;
            b = tmp;
        }
        const uint32_t old = atomicMin(label + b, a);
        if (old == b) return;
        b = find_root(label, old);
        a = find_root(label, a);
    }
}

__global__ __launch_bounds__(kBlock) void sw_union_kernel(LatticeArgs a)
{
    const uint32_t L = a.L, N = a.N;
    const double inv_L = 1.0 / (double)L;
    for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < N; c += gridDim.x * kBlock) {
        const uint32_t m = a.mask[c];
        if (!(m & 3)) continue;
        uint32_t x;
        const uint32_t y = divmod(c, L, inv_L, x);
        const uint32_t row = y * L;
        if (m & 1) unite(a.label, c, N + ((x + 1 == L) ? 0 : x + 1) + row);
        if (m & 2) unite(a.label, 2 * N + c, 3 * N + x + ((y + 1 == L) ? 0 : row + L));
    }
}

// Flatten every label to its root (the cluster minimum) and shift sigma by
// the cluster's r = pick(w0 of Philox(root, t, 0, SWF), q), NULL -> 0.
__global__ __launch_bounds__(kBlock) void sw_flip_kernel(LatticeArgs a)
{
    const uint32_t t = a.st->t_cur;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.st->sw_done = 1;
    const uint32_t N = a.N;
    const int q = (int)a.q;
    for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < N; c += gridDim.x * kBlock) {
#pragma unroll
        for (int arm = 0; arm < 4; ++arm) {
            const uint32_t idx = arm * N + c;
            const uint32_t r = find_root(a.label, idx);
            a.label[idx] = r;
            const uint32_t w = philox(r, t, 0u, kStreamSwf, a.key0, a.key1).x;
            const int k = (w <= a.flip_lim) ? (int)((double)w * a.flip_invd) : 0;
            int sv = a.sigma[idx] + k;
            sv = sv >= q ? sv - q : sv;
            a.sigma[idx] = (uint8_t)sv;
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
hipError_t launch_state_init(DevState* st, int64_t* slots, const DevTables* tab, double v_init, hipStream_t s)
{
    state_init_kernel<<<1, 64, 0, s>>>(st, slots, tab, v_init);
    return hipGetLastError();
}

hipError_t launch_sigma_init(const LatticeArgs& a, hipStream_t s)
{
    sigma_init_kernel<<<grid_for(a.N), kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_volume(const VolArgs& a, hipStream_t s)
{
    volume_kernel<<<1, 64, 0, s>>>(a);
    return hipGetLastError();
}

template <int Q>
void launch_quad(const LatticeArgs& a, int colour, dim3 grid, hipStream_t s)
{
    if (colour == 0) met_sweep4_kernel<Q, 0><<<grid, 256, 0, s>>>(a);
    else met_sweep4_kernel<Q, 1><<<grid, 256, 0, s>>>(a);
}

hipError_t launch_met_colour(const LatticeArgs& a, int colour, hipStream_t s)
{
    if (a.quad) {
        const dim3 grid((a.L / 4 + 63) / 64, a.row_blocks);
        switch (a.q) {
        case 2: launch_quad<2>(a, colour, grid, s); break;
        case 3: launch_quad<3>(a, colour, grid, s); break;
        case 4: launch_quad<4>(a, colour, grid, s); break;
        case 5: launch_quad<5>(a, colour, grid, s); break;
        default: launch_quad<6>(a, colour, grid, s); break;
        }
        return hipGetLastError();
    }
    const dim3 grid((a.L / 2 + 63) / 64, a.row_blocks), block(256);
    switch (a.q) {
    case 2: met_sweep_kernel<2><<<grid, block, 0, s>>>(a, colour); break;
    case 3: met_sweep_kernel<3><<<grid, block, 0, s>>>(a, colour); break;
    case 4: met_sweep_kernel<4><<<grid, block, 0, s>>>(a, colour); break;
    case 5: met_sweep_kernel<5><<<grid, block, 0, s>>>(a, colour); break;
    default: met_sweep_kernel<6><<<grid, block, 0, s>>>(a, colour); break;
    }
    return hipGetLastError();
}

hipError_t launch_recount(const LatticeArgs& a, int64_t* out, int spread, int with_counts, hipStream_t s)
{
    recount_kernel<<<grid_for(a.N), kBlock, 0, s>>>(a, out, spread, with_counts);
    return hipGetLastError();
}

hipError_t launch_obs_zero(DevObs* o, hipStream_t s)
{
    obs_zero_kernel<<<1, 64, 0, s>>>(o);
    return hipGetLastError();
}

hipError_t launch_obs_final(DevObs* o, const DevState* st, const DevTables* tab, double Nd, double J,
                            double Jsigma, double P, double vHB, hipStream_t s)
{
    obs_final_kernel<<<1, 64, 0, s>>>(o, st, tab, Nd, J, Jsigma, P, vHB);
    return hipGetLastError();
}

hipError_t launch_sw_bonds(const LatticeArgs& a, hipStream_t s)
{
    sw_bonds_kernel<<<grid_for(a.N), kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_sw_union(const LatticeArgs& a, hipStream_t s)
{
    sw_union_kernel<<<grid_for(a.N), kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_sw_flip(const LatticeArgs& a, hipStream_t s)
{
    sw_flip_kernel<<<grid_for(a.N), kBlock, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace cvf
