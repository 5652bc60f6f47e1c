// CVF water model on the periodic simple-cubic lattice with the eta bond
// constraint (Sec. II.A-C, App. A): device kernels and the cvf3_* C ABI.
//
// One MC step on the caller's stream (Sec. II.B):
//   vol3_kernel   one workgroup: folds the previous step's per-workgroup
//                 counter slots, performs the FP64 volume move, draws the
//                 order of the six arm passes
//   eta3_kernel   one thread per checkerboard cube: Metropolis move of the
//                 cube's eta configuration (one of the nine perfect matchings
//                 of the cube graph marks the eta = 0 edges)
//   pass3_kernel  x6, one per arm in the drawn order: every cell's bond index
//                 of that arm moves once (the arm-domain partition of
//                 Sec. II.C); a lane moves two x-adjacent cells, which share
//                 one Philox block
// A Swendsen-Wang step (Sec. II.D) replaces the passes by sw3_bonds_kernel
// (link masks, cooperative links closed in registers), sw3_tile_union_kernel
// (in-tile covalent links, LDS union-find), sw3_union_kernel (tile-crossing
// links, global union-find), sw3_flip_kernel (cluster shifts) and a recount.
// Layout: sigma[a*N + c], eta[d*N + c] (edge from c to its +d neighbour),
// c = x + L*(y + L*z); arms 0:+x 1:-x 2:+y 3:-y 4:+z 5:-z.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "cvf.h"
#include "cvf3.h"
#include "dispatch.h"

namespace {

#include "philox.h"

constexpr uint32_t kInit = 0, kVol = 1, kSwb = 3, kSwf = 4, kOrd = 5, kDom = 6, kEta = 7;
constexpr int kSlots = 256;              // counter slots, spread to avoid one hot atomic
constexpr int kAcc = 4;                  // d N_HB_raw, d N_sigma, sigma accepted, eta accepted
constexpr int kRc = 10;                  // recount: N_HB_raw, N_sigma, N_q' (6), eta = 0 edges, spare
constexpr int kBlock = 256;
constexpr uint32_t kQuadsPerLane = 4;    // quad pass: quads per lane (grid-stride)

struct Dev3State {
    double  v, u;
    int64_t t_next, t_cur;
    int64_t n_hb_raw, n_coop;
    int64_t met_att, met_acc, eta_att, eta_acc, vol_att, vol_acc;
    int32_t theta, pad0;
    int32_t order[6];
    int32_t pad[2];
};

struct Tab3 {
    uint32_t met[2][3][11];   // sigma move: [theta*eta][dh+1][dc+5]
    uint32_t eta[9];          // eta move in the liquid: [dn+4]
    uint32_t match[9];        // perfect matchings of the cube graph (12-bit edge masks, eta = 0)
    uint64_t sw_sigma, sw_eff; // SW bond thresholds floor(p 2^32): cooperative, covalent (liquid)
    int32_t  jeff_sign;        // sign of J_eff
    double   r3[40];          // r3(m), m = 0..36
};

struct Lat3 {
    uint8_t*   sigma;
    uint8_t*   eta;
    Dev3State* st;
    int64_t*   slots;         // [kAcc][kSlots]
    int64_t*   rc;            // [kRc][kSlots]
    const Tab3* tab;          // device copy
    uint32_t*  mask;          // [N] SW link masks (NULL without SW)
    uint32_t*  par;           // [6N] SW union-find parents, then labels
    uint32_t L, N, h, q;
    uint32_t key0, key1;
    uint32_t pass;
    uint32_t quad;            // 1: L % 4 == 0, four cells per lane; 0: cell pairs
    double   invL, invH, invQ4, Nd, beta, J, P, vHB, dv_max;
    int32_t  do_volume;
};

__device__ __forceinline__ uint32_t udiv(uint32_t n, uint32_t d, double inv)
{
    uint32_t q = (uint32_t)((double)n * inv);
    const int64_t r = (int64_t)n - (int64_t)q * d;
    if (r < 0) --q;
    else if (r >= (int64_t)d) ++q;
    return q;
}

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sums K per-thread values over the workgroup and adds them to slot
// (blockIdx % kSlots) of each of K counters (stride kSlots).
template <int K>
__device__ void block_slots(int (&v)[K], int64_t* dst)
{
    __shared__ int part[K][kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int s = wave_sum(v[k]);
        if (lane == 0) part[k][w] = s;
    }
    __syncthreads();
    if (threadIdx.x < K) {
        int64_t s = 0;
        for (int i = 0; i < kBlock / 64; ++i) s += part[threadIdx.x][i];
        if (s) atomicAdd((unsigned long long*)(dst + (size_t)threadIdx.x * kSlots + blockIdx.x % kSlots),
                         (unsigned long long)s);
    }
}

// U_LJ per molecule on the cubic lattice (Sec. II.A): shells m = |n|^2 in
// ascending order, (distance/r0)^6 = v^2 m^3, cutoff 6^6.
__device__ __host__ double lj3(double v, const double* r3)
{
    double s = 0.0;
    for (int m = 1; m <= 36; ++m) {
        const double d6 = (v * v) * (double)(m * m * m);
        if (!(d6 <= 46656.0)) break;
        const double s6 = 1.0 / d6;
        s = s + r3[m] * (s6 * s6 - s6);
    }
    return 2.0 * s;
}

// Uniform draw of {0..k-1} from one word by the exact-block rule (NONE = -1
// when the word falls in the incomplete top block).
__device__ __forceinline__ int pick_div(uint32_t w, uint32_t k)
{
    const uint32_t d = (uint32_t)(4294967296ull / k);
    if ((uint64_t)w >= (uint64_t)k * d) return -1;
    return (int)(w / d);
}

// The exact-block draw of {0..q-2} from one word, in closed form: with
// d = floor(2^32/(q-1)), (q-1) d = 2^32 when q-1 is a power of two (never
// NONE, k = floor(w (q-1) / 2^32)) and 2^32 - 1 when q-1 is 3 or 5 (NONE only
// for w = 2^32 - 1, k = floor((w+1)(q-1) / 2^32)).  Returns false for NONE.
__device__ __forceinline__ bool pick_other(uint32_t w, uint32_t qm1, bool odd, uint32_t& k)
{
    if (odd && w == 0xFFFFFFFFu) return false;
    k = __umulhi(odd ? w + 1 : w, qm1);
    return true;
}

// Corner vtx (bit 0: +x, 1: +y, 2: +z) of cube k: parity k / h^3 sets the
// lowest corner (2i+par, 2j+par, 2l+par).
struct Cube {
    uint32_t x0, y0, z0;
};

__device__ __forceinline__ Cube cube_of(const Lat3& a, uint32_t k)
{
    const uint32_t h3 = a.h * a.h * a.h;
    const uint32_t par = k >= h3 ? 1u : 0u;
    const uint32_t r = k - par * h3;
    const uint32_t jl = udiv(r, a.h, a.invH);
    const uint32_t i = r - jl * a.h;
    const uint32_t l = udiv(jl, a.h, a.invH);
    const uint32_t j = jl - l * a.h;
    return {2 * i + par, 2 * j + par, 2 * l + par};
}

__device__ __forceinline__ uint32_t cell_at(const Lat3& a, const Cube& q, uint32_t vtx)
{
    uint32_t x = q.x0 + (vtx & 1), y = q.y0 + ((vtx >> 1) & 1), z = q.z0 + ((vtx >> 2) & 1);
    x = x == a.L ? 0 : x;
    y = y == a.L ? 0 : y;
    z = z == a.L ? 0 : z;
    return x + a.L * (y + a.L * z);
}

// Ends of cube edge e: axis d = e / 4, r = e % 4 places it along the two
// other axes (lower axis in bit 0).
__device__ __forceinline__ void edge_vtx(int e, uint32_t& lo, uint32_t& hi)
{
    const int d = e >> 2, r = e & 3;
    uint32_t v;
    if (d == 0) v = ((r & 1) << 1) | ((r >> 1) << 2);
    else if (d == 1) v = (r & 1) | ((r >> 1) << 2);
    else v = (r & 1) | ((r >> 1) << 1);
    lo = v;
    hi = v | (1u << d);
}

// ---------------------------------------------------------------------------
// Initial state: sigma of cell c from words 0..3 of Philox(c, 0, 0, INIT) and
// words 0, 1 of Philox(c, 0, 1, INIT); eta of cube k from configuration
// pick(word 0 of Philox(k, 0, 2, INIT), 9), NONE -> 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void init3_sigma_kernel(Lat3 a)
{
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= a.N) return;
    const uint4 w0 = philox(c, 0u, 0u, kInit, a.key0, a.key1);
    const uint4 w1 = philox(c, 0u, 1u, kInit, a.key0, a.key1);
    const uint32_t w[6] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y};
#pragma unroll
    for (int b = 0; b < 6; ++b) a.sigma[(size_t)b * a.N + c] = (uint8_t)(((uint64_t)w[b] * a.q) >> 32);
}

__global__ __launch_bounds__(kBlock) void init3_eta_kernel(Lat3 a)
{
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= a.N / 4) return;
    const uint4 w = philox(k, 0u, 2u, kInit, a.key0, a.key1);
    int m = pick_div(w.x, 9);
    if (m < 0) m = 0;
    const uint32_t mask = a.tab->match[m];
    const Cube q = cube_of(a, k);
#pragma unroll
    for (int e = 0; e < 12; ++e) {
        uint32_t lo, hi;
        edge_vtx(e, lo, hi);
        a.eta[(size_t)(e >> 2) * a.N + cell_at(a, q, lo)] = (uint8_t)(((mask >> e) & 1) ^ 1);
    }
}

__global__ void state3_init_kernel(Lat3 a, double v_init)
{
    for (int i = threadIdx.x; i < kAcc * kSlots; i += blockDim.x) a.slots[i] = 0;
    if (threadIdx.x == 0) {
        Dev3State* s = a.st;
        memset(s, 0, sizeof(*s));
        s->v = v_init;
        s->u = lj3(v_init, a.tab->r3);
        s->theta = v_init < 2.0 ? 1 : 0;
        for (int i = 0; i < 6; ++i) s->order[i] = i;
    }
}

constexpr int kVolMet = 0, kVolFold = 1, kVolSw = 2;

// ---------------------------------------------------------------------------
// Counter fold + volume move (Sec. II.B step 1) + pass order of the step.
// dH = N (u(v') - u(v)) + P N (v' - v) + (theta' - theta)(P v_HB - J) N_HB_raw
// with words 0, 1 of Philox(0, t, 0, VOL); order: Fisher-Yates over 0..5
// with words 0..3 of Philox(0, t, 0, ORD) and word 0 of Philox(0, t, 1, ORD).
// mode 0: full step opening; mode 1: fold only.
// ---------------------------------------------------------------------------
// One wavefront: lanes fold the counter slots (kSlots / 64 each), lanes 0-2
// draw the VOL block and the two ORD blocks at once, lanes 1..36 evaluate one
// U_LJ shell term each; lane 0 then sums the terms in ascending shell order
// up to the first shell beyond the cutoff (the order of lj3) and takes the
// decisions.  Every global load (slots, chain state, shell counts) is issued
// before the first store, and the four slot sums share one butterfly.
__global__ __launch_bounds__(64) void vol3_kernel(Lat3 a, int mode)
{
    __shared__ double term[40];
    __shared__ uint32_t words[3][4];
    const int lane = threadIdx.x;
    Dev3State* s = a.st;
    int64_t sl[kAcc][kSlots / 64];
#pragma unroll
    for (int k = 0; k < kAcc; ++k)
#pragma unroll
        for (int j = 0; j < kSlots / 64; ++j) sl[k][j] = a.slots[k * kSlots + j * 64 + lane];
    const uint32_t t = (uint32_t)s->t_next;
    const int64_t t_next = s->t_next;
    const double v0 = s->v, u0 = s->u;
    const int th0 = s->theta;
    const int64_t hb0 = s->n_hb_raw, co0 = s->n_coop, ma0 = s->met_acc, ea0 = s->eta_acc;
    const int64_t matt0 = s->met_att, eatt0 = s->eta_att, vatt0 = s->vol_att, vacc0 = s->vol_acc;
    const double r3 = (lane >= 1 && lane <= 36) ? a.tab->r3[lane] : 0.0;
    int64_t r[kAcc];
#pragma unroll
    for (int k = 0; k < kAcc; ++k) {
        r[k] = 0;
#pragma unroll
        for (int j = 0; j < kSlots / 64; ++j) {
            r[k] += sl[k][j];
            a.slots[k * kSlots + j * 64 + lane] = 0;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        int64_t x[kAcc];
#pragma unroll
        for (int k = 0; k < kAcc; ++k) x[k] = __shfl_xor(r[k], o, 64);
#pragma unroll
        for (int k = 0; k < kAcc; ++k) r[k] += x[k];
    }
    if (mode != kVolFold && lane < 3) {
        const uint4 w = philox(0u, t, lane == 2 ? 1u : 0u, lane == 0 ? kVol : kOrd, a.key0, a.key1);
        words[lane][0] = w.x;
        words[lane][1] = w.y;
        words[lane][2] = w.z;
        words[lane][3] = w.w;
    }
    __syncthreads();
    double v1 = 0.0;
    bool inside = false;
    if (mode != kVolFold && a.do_volume) {
        const double u = (double)((int64_t)2 * (int64_t)words[0][0] + 1 - 4294967296LL) * (1.0 / 4294967296.0);
        v1 = v0 + a.dv_max * u;
        inside = v1 >= 1.0;
        if (inside && lane >= 1 && lane <= 36) {
            const double d6 = (v1 * v1) * (double)(lane * lane * lane);
            const double s6 = 1.0 / d6;
            term[lane] = d6 <= 46656.0 ? r3 * (s6 * s6 - s6) : 0.0;
        }
    }
    __syncthreads();
    if (lane != 0) return;
    const int64_t n_hb = hb0 + r[0];
    s->n_hb_raw = n_hb;
    s->n_coop = co0 + r[1];
    s->met_acc = ma0 + r[2];
    s->eta_acc = ea0 + r[3];
    if (mode == kVolFold) return;
    if (a.do_volume) {
        s->vol_att = vatt0 + 1;
        if (inside) {
            // all 36 terms read first, then added in ascending m while within
            // the cutoff: the condition is monotone in m, so the terms added
            // and their order are those of the loop that stops at the first
            // shell beyond it
            double tm[36];
#pragma unroll
            for (int m = 1; m <= 36; ++m) tm[m - 1] = term[m];
            double sum = 0.0;
#pragma unroll
            for (int m = 1; m <= 36; ++m) {
                const double d6 = (v1 * v1) * (double)(m * m * m);
                if (d6 <= 46656.0) sum = sum + tm[m - 1];
            }
            const double u1 = 2.0 * sum;
            const int th1 = v1 < 2.0 ? 1 : 0;
            const double dH = (a.Nd * (u1 - u0)) + ((a.P * a.Nd) * (v1 - v0))
                            + (((double)(th1 - th0) * (a.P * a.vHB - a.J)) * (double)n_hb);
            bool acc = dH <= 0.0;
            if (!acc) acc = ((double)words[0][1] + 0.5) * (1.0 / 4294967296.0) < exp(-a.beta * dH);
            if (acc) {
                s->v = v1;
                s->u = u1;
                s->theta = th1;
                s->vol_acc = vacc0 + 1;
            }
        }
    }
    const uint32_t ow[5] = {words[1][0], words[1][1], words[1][2], words[1][3], words[2][0]};
    int ord[6] = {0, 1, 2, 3, 4, 5};
    for (int i = 0; i < 5; ++i) {
        int k = pick_div(ow[i], (uint32_t)(6 - i));
        if (k < 0) k = 0;
        const int tmp = ord[i];
        ord[i] = ord[i + k];
        ord[i + k] = tmp;
    }
    for (int i = 0; i < 6; ++i) s->order[i] = ord[i];
    s->t_cur = t;
    s->t_next = t_next + 1;
    if (mode == kVolMet) s->met_att = matt0 + 6 * (int64_t)a.N;
    s->eta_att = eatt0 + a.N / 4;
}

// ---------------------------------------------------------------------------
// eta update (Sec. II.B step 2, App. A): one thread per cube.  Proposal
// pick(w0, 9) of Philox(k, t, 0, ETA) (NONE: no move); dn = change of
// N_HB_raw inside the cube; accepted through the eta table and w1 in the
// liquid, always in the gas.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void eta3_kernel(Lat3 a)
{
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    int cnt[2] = {0, 0};
    if (k < a.N / 4) {
        const uint32_t t = (uint32_t)a.st->t_cur;
        const int theta = a.st->theta;
        const uint4 w = philox(k, t, 0u, kEta, a.key0, a.key1);
        const int m = pick_div(w.x, 9);
        if (m >= 0) {
            const uint32_t mask = a.tab->match[m];
            const Cube q = cube_of(a, k);
            uint32_t cell[8];
#pragma unroll
            for (int v = 0; v < 8; ++v) cell[v] = cell_at(a, q, v);
            int dn = 0;
            uint32_t old = 0;
#pragma unroll
            for (int e = 0; e < 12; ++e) {
                uint32_t lo, hi;
                edge_vtx(e, lo, hi);
                const int d = e >> 2;
                const int eq = a.sigma[(size_t)(2 * d) * a.N + cell[lo]] == a.sigma[(size_t)(2 * d + 1) * a.N + cell[hi]];
                const int eo = a.eta[(size_t)d * a.N + cell[lo]];
                old |= (uint32_t)eo << e;
                const int en = (int)(((mask >> e) & 1) ^ 1);
                dn += (en - eo) * eq;
            }
            bool acc = true;
            if (theta) {
                const uint32_t thr = a.tab->eta[dn + 4];
                acc = thr == 0xFFFFFFFFu || w.y < thr;
            }
            if (acc) {
                cnt[0] = dn;
                cnt[1] = 1;
                const uint32_t neu = (~mask) & 0xFFFu;
                if (neu != old) {
#pragma unroll
                    for (int e = 0; e < 12; ++e) {
                        uint32_t lo, hi;
                        edge_vtx(e, lo, hi);
                        if (((neu ^ old) >> e) & 1)
                            a.eta[(size_t)(e >> 2) * a.N + cell[lo]] = (uint8_t)((neu >> e) & 1);
                    }
                }
            }
        }
    }
    int v4[2] = {cnt[0], cnt[1]};
    // slots: 0 = d N_HB_raw, 3 = eta accepted
    __shared__ int part[2][kBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int j = 0; j < 2; ++j) {
        const int s = wave_sum(v4[j]);
        if (lane == 0) part[j][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        int64_t s = 0;
        for (int i = 0; i < kBlock / 64; ++i) s += part[threadIdx.x][i];
        const int slot = threadIdx.x == 0 ? 0 : 3;
        if (s) atomicAdd((unsigned long long*)(a.slots + (size_t)slot * kSlots + blockIdx.x % kSlots),
                         (unsigned long long)s);
    }
}

// Two cubes per lane (L % 4 == 0): cubes 2i', 2i'+1 of one parity and one
// (j, l) span x = 4i' + par .. 4i' + par + 3.  Every plane row the pair
// touches is one aligned 32-bit word for the even parity; for the odd parity
// the word is shifted down one byte and takes the first byte of the next
// word (wrapping at the row end), so that byte i of a row word is always
// x = 4i' + par + i: 24 row words for 24 edges.  Each cube's move is the one
// of eta3_kernel.
__device__ __forceinline__ uint32_t row4(const uint8_t* plane, uint32_t rowbase, uint32_t xa, uint32_t xb, bool odd)
{
    const uint32_t w = *(const uint32_t*)(plane + rowbase + xa);
    if (!odd) return w;
    return __builtin_amdgcn_alignbyte((uint32_t)plane[rowbase + xb], w, 1);
}

__device__ __forceinline__ uint32_t byte_at(uint32_t w, uint32_t i) { return (w >> (8 * i)) & 0xFFu; }

__global__ __launch_bounds__(kBlock) void eta3_pair_kernel(Lat3 a)
{
    const uint32_t g = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t npar = a.N / 16;
    int cnt[2] = {0, 0};
    if (g < 2 * npar) {
        const uint32_t L = a.L, N = a.N, h = a.h;
        const uint32_t par = g >= npar ? 1u : 0u;
        const bool odd = par != 0;
        const uint32_t r = g - par * npar;
        const uint32_t q4 = L / 4;
        const uint32_t jl = udiv(r, q4, a.invQ4);
        const uint32_t ip = r - jl * q4;
        const uint32_t l = udiv(jl, h, a.invH);
        const uint32_t j = jl - l * h;
        const uint32_t yv[2] = {2 * j + par, 2 * j + par + 1 == L ? 0u : 2 * j + par + 1};
        const uint32_t zv[2] = {2 * l + par, 2 * l + par + 1 == L ? 0u : 2 * l + par + 1};
        const uint32_t xa = 4 * ip, xb = xa + 4 == L ? 0u : xa + 4;
        uint32_t rb[2][2];                                 // [dy][dz] row bases
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dz = 0; dz < 2; ++dz) rb[dy][dz] = L * (yv[dy] + L * zv[dz]);
        const uint8_t* S = a.sigma;
        const uint8_t* E = a.eta;
        uint32_t e0[2][2], s0[2][2], s1[2][2], e1[2], s2[2], s3[2], e2[2], s4[2], s5[2];
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dz = 0; dz < 2; ++dz) {
                e0[dy][dz] = row4(E, rb[dy][dz], xa, xb, odd);
                s0[dy][dz] = row4(S, rb[dy][dz], xa, xb, odd);
                s1[dy][dz] = row4(S + (size_t)N, rb[dy][dz], xa, xb, odd);
            }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            e1[k] = row4(E + (size_t)N, rb[0][k], xa, xb, odd);          // y-edges: row (y0, z_k)
            s2[k] = row4(S + 2 * (size_t)N, rb[0][k], xa, xb, odd);
            s3[k] = row4(S + 3 * (size_t)N, rb[1][k], xa, xb, odd);      // upper ends: row (y1, z_k)
            e2[k] = row4(E + 2 * (size_t)N, rb[k][0], xa, xb, odd);      // z-edges: row (y_k, z0)
            s4[k] = row4(S + 4 * (size_t)N, rb[k][0], xa, xb, odd);
            s5[k] = row4(S + 5 * (size_t)N, rb[k][1], xa, xb, odd);      // upper ends: row (y_k, z1)
        }
        const uint32_t t = (uint32_t)a.st->t_cur;
        const int theta = a.st->theta;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const uint32_t k = par * (h * h * h) + 2 * ip + (uint32_t)c + h * jl;
            const uint4 w = philox(k, t, 0u, kEta, a.key0, a.key1);
            const int m = pick_div(w.x, 9);
            if (m < 0) continue;
            const uint32_t mask = a.tab->match[m];
            const uint32_t b0 = 2 * c;                     // byte of the cube's lowest x in the row words
            uint32_t old = 0, eqm = 0;
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int lo = rr & 1, hi = rr >> 1;
                // x-edge (dy, dz) = (lo, hi)
                old |= byte_at(e0[lo][hi], b0) << rr;
                eqm |= (uint32_t)(byte_at(s0[lo][hi], b0) == byte_at(s1[lo][hi], b0 + 1)) << rr;
                // y-edge (dx, dz) = (lo, hi)
                old |= byte_at(e1[hi], b0 + lo) << (4 + rr);
                eqm |= (uint32_t)(byte_at(s2[hi], b0 + lo) == byte_at(s3[hi], b0 + lo)) << (4 + rr);
                // z-edge (dx, dy) = (lo, hi)
                old |= byte_at(e2[hi], b0 + lo) << (8 + rr);
                eqm |= (uint32_t)(byte_at(s4[hi], b0 + lo) == byte_at(s5[hi], b0 + lo)) << (8 + rr);
            }
            const uint32_t neu = (~mask) & 0xFFFu;
            const int dn = __popc(neu & eqm) - __popc(old & eqm);
            bool acc = true;
            if (theta) {
                const uint32_t thr = a.tab->eta[dn + 4];
                acc = thr == 0xFFFFFFFFu || w.y < thr;
            }
            if (!acc) continue;
            cnt[0] += dn;
            cnt[1] += 1;
            const uint32_t chg = neu ^ old;
            if (!chg) continue;
#pragma unroll
            for (int e = 0; e < 12; ++e) {
                if (!((chg >> e) & 1)) continue;
                const int d = e >> 2, lo = e & 1, hi = (e >> 1) & 1;
                uint32_t rbase, bx;
                if (d == 0) { rbase = rb[lo][hi]; bx = b0; }
                else if (d == 1) { rbase = rb[0][hi]; bx = b0 + lo; }
                else { rbase = rb[hi][0]; bx = b0 + lo; }
                const uint32_t x = par + bx == 4 ? xb : xa + par + bx;
                a.eta[(size_t)d * N + rbase + x] = (uint8_t)((neu >> e) & 1);
            }
        }
    }
    __shared__ int part[2][kBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int sm = wave_sum(cnt[q]);
        if (lane == 0) part[q][wv] = sm;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        int64_t sm = 0;
        for (int i = 0; i < kBlock / 64; ++i) sm += part[threadIdx.x][i];
        const int slot = threadIdx.x == 0 ? 0 : 3;
        if (sm) atomicAdd((unsigned long long*)(a.slots + (size_t)slot * kSlots + blockIdx.x % kSlots),
                          (unsigned long long)sm);
    }
}

// ---------------------------------------------------------------------------
// Arm-domain pass (Sec. II.C): arm A of every cell.  Lane = cell pair
// (2p, 2p+1) of one x-row, Philox(p, t, A, DOM) words 0, 1 for the even cell
// and 2, 3 for the odd one.  Own bond indices and the aligned facing/eta
// pairs are 16-bit loads; the x arms' facing and eta pairs straddle the pair
// and wrap at the row end, so they are byte loads.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void move_one(const uint32_t* met, int q, int theta, uint32_t own[6],
                                         int A, uint32_t facing, uint32_t eta, uint32_t prop, uint32_t accw,
                                         int& dhb, int& dco, int& nacc)
{
    const uint32_t qm1 = (uint32_t)q - 1;
    uint32_t k;
    if (!pick_other(prop, qm1, (qm1 & 1) && qm1 > 1, k)) return;      // NONE
    const uint32_t old = own[A];
    uint32_t neu = old + 1 + (uint32_t)k;
    neu = neu >= (uint32_t)q ? neu - (uint32_t)q : neu;
    const int dh = (int)(neu == facing) - (int)(old == facing);
    int dc = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b)
        if (b != A) dc += (int)(neu == own[b]) - (int)(old == own[b]);
    const int th = (theta && eta) ? 1 : 0;
    const uint32_t thr = met[th * 33 + (dh + 1) * 11 + dc + 5];
    if (thr == 0xFFFFFFFFu || accw < thr) {
        own[A] = neu;
        dhb += (int)eta * dh;
        dco += dc;
        nacc += 1;
    }
}

template <int A>
__device__ __forceinline__ void pass_pair(const Lat3& a, const uint32_t* met, uint32_t p,
                                          uint32_t t, int theta, int (&cnt)[3])
{
    const uint32_t L = a.L, N = a.N;
    const uint32_t c0 = 2 * p;
    uint32_t own0[6], own1[6];
#pragma unroll
    for (int b = 0; b < 6; ++b) {
        const uint32_t v = *(const uint16_t*)(a.sigma + (size_t)b * N + c0);
        own0[b] = v & 0xFFu;
        own1[b] = v >> 8;
    }
    uint32_t f0, f1, e0, e1, o = 0;
    if (A == 0 || A == 1) {
        const uint32_t yz = udiv(c0, L, a.invL);
        const uint32_t x0 = c0 - yz * L;
        if (A == 0) {                                     // facing: arm 1 of x0+1, x0+2
            const uint32_t r2 = x0 + 2 == L ? c0 + 2 - L : c0 + 2;
            f0 = a.sigma[(size_t)N + c0 + 1];
            f1 = a.sigma[(size_t)N + r2];
            const uint32_t ee = *(const uint16_t*)(a.eta + c0);
            e0 = ee & 0xFFu;
            e1 = ee >> 8;
        } else {                                          // facing: arm 0 of x0-1, x0
            const uint32_t l1 = x0 == 0 ? c0 + L - 1 : c0 - 1;
            f0 = a.sigma[l1];
            f1 = a.sigma[c0];
            e0 = a.eta[l1];
            e1 = a.eta[c0];
        }
    } else {
        const uint32_t L2 = L * L;
        if (A == 2 || A == 3) {
            const uint32_t yz = udiv(c0, L, a.invL);
            const uint32_t z = udiv(yz, L, a.invL);
            const uint32_t y = yz - z * L;
            if (A == 2) o = y == L - 1 ? c0 + L - L2 : c0 + L;
            else o = y == 0 ? c0 + L2 - L : c0 - L;
        } else if (A == 4) {
            o = c0 + L2 >= N ? c0 + L2 - N : c0 + L2;
        } else {
            o = c0 >= L2 ? c0 - L2 : c0 + N - L2;
        }
        const uint32_t ff = *(const uint16_t*)(a.sigma + (size_t)(A ^ 1) * N + o);
        f0 = ff & 0xFFu;
        f1 = ff >> 8;
        const uint32_t ee = *(const uint16_t*)(a.eta + (size_t)(A >> 1) * N + ((A & 1) ? o : c0));
        e0 = ee & 0xFFu;
        e1 = ee >> 8;
    }
    const uint4 w = philox(p, t, (uint32_t)A, kDom, a.key0, a.key1);
    const uint32_t old0 = own0[A], old1 = own1[A];
    move_one(met, (int)a.q, theta, own0, A, f0, e0, w.x, w.y, cnt[0], cnt[1], cnt[2]);
    move_one(met, (int)a.q, theta, own1, A, f1, e1, w.z, w.w, cnt[0], cnt[1], cnt[2]);
    if (own0[A] != old0 || own1[A] != old1)
        *(uint16_t*)(a.sigma + (size_t)A * N + c0) = (uint16_t)(own0[A] | (own1[A] << 8));
}

// 0x01 in every byte of x that is zero, 0x00 elsewhere (no carry crosses a byte).
__device__ __forceinline__ uint32_t zero_bytes(uint32_t x)
{
    return (~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x | 0x7F7F7F7Fu)) >> 7;
}

// Sum of the four bytes of x (each small enough that no partial sum reaches 256).
__device__ __forceinline__ uint32_t byte_sum(uint32_t x) { return (x * 0x01010101u) >> 24; }

// Four cells per lane (L % 4 == 0): cells 4u..4u+3 of one x-row use the
// Philox blocks of pairs 2u and 2u+1; own, facing and eta words are 32-bit
// loads, the x arms' facing and eta words borrow one byte from the next or
// previous word (wrapping at the row end).  The four moves are decided
// together on packed bytes: the same proposals, table index and acceptance
// as move_one, cell by cell.
// Raw buffer over one plane (N bytes < 2^31): 32-bit lane offsets, base in SGPRs.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(uint8_t* base, uint32_t n)
{
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)n, 0x00020000);
}

__device__ __forceinline__ uint32_t bld32(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
}

__device__ __forceinline__ uint32_t bld8(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_amdgcn_raw_buffer_load_b8(r, (int)off, 0, 0);
}

template <int A>
__device__ __forceinline__ void pass_quad(const Lat3& a, const uint32_t* met, uint32_t u, uint32_t t, int theta,
                                          int (&cnt)[3])
{
    const uint32_t L = a.L, N = a.N;
    const uint32_t c0 = 4 * u;
    uint32_t ow[6];
#pragma unroll
    for (int b = 0; b < 6; ++b) ow[b] = bld32(plane_rsrc(a.sigma + (size_t)b * N, N), c0);
    uint32_t fw, ew;
    if (A == 0 || A == 1) {
        const uint32_t yz = udiv(c0, L, a.invL);
        const uint32_t x0 = c0 - yz * L;
        const __amdgpu_buffer_rsrc_t e0 = plane_rsrc(a.eta, N);
        if (A == 0) {                                     // arm 1 of x0+1 .. x0+4
            const uint32_t nx = x0 + 4 == L ? c0 + 4 - L : c0 + 4;
            const __amdgpu_buffer_rsrc_t s1 = plane_rsrc(a.sigma + (size_t)N, N);
            fw = __builtin_amdgcn_alignbyte(bld8(s1, nx), ow[1], 1);
            ew = bld32(e0, c0);
        } else {                                          // arm 0 of x0-1 .. x0+2
            const uint32_t px = x0 == 0 ? c0 + L - 1 : c0 - 1;
            const __amdgpu_buffer_rsrc_t s0 = plane_rsrc(a.sigma, N);
            fw = (ow[0] << 8) | bld8(s0, px);
            ew = (bld32(e0, c0) << 8) | bld8(e0, px);
        }
    } else {
        const uint32_t L2 = L * L;
        uint32_t o;
        if (A == 2 || A == 3) {
            const uint32_t yz = udiv(c0, L, a.invL);
            const uint32_t z = udiv(yz, L, a.invL);
            const uint32_t y = yz - z * L;
            if (A == 2) o = y == L - 1 ? c0 + L - L2 : c0 + L;
            else o = y == 0 ? c0 + L2 - L : c0 - L;
        } else if (A == 4) {
            o = c0 + L2 >= N ? c0 + L2 - N : c0 + L2;
        } else {
            o = c0 >= L2 ? c0 - L2 : c0 + N - L2;
        }
        fw = bld32(plane_rsrc(a.sigma + (size_t)(A ^ 1) * N, N), o);
        ew = bld32(plane_rsrc(a.eta + (size_t)(A >> 1) * N, N), (A & 1) ? o : c0);
    }
    const uint4 w0 = philox(2 * u, t, (uint32_t)A, kDom, a.key0, a.key1);
    const uint4 w1 = philox(2 * u + 1, t, (uint32_t)A, kDom, a.key0, a.key1);
    const uint32_t prop[4] = {w0.x, w0.z, w1.x, w1.z}, accw[4] = {w0.y, w0.w, w1.y, w1.w};
    // proposals of the four cells, one byte each (a NONE draw keeps the old state)
    const uint32_t q = a.q, qm1 = q - 1, oldw = ow[A];
    const bool odd = (qm1 & 1) && qm1 > 1;
    uint32_t nw = 0, valid = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t old = (oldw >> (8 * j)) & 0xFFu;
        uint32_t k = 0;
        const bool ok = pick_other(prop[j], qm1, odd, k);
        uint32_t neu = old + 1 + k;
        neu = neu >= q ? neu - q : neu;
        neu = ok ? neu : old;
        valid |= ok ? (0xFFu << (8 * j)) : 0u;
        nw |= neu << (8 * j);
    }
    // equal-byte counts for all four cells at once: cn / co = other arms equal
    // to the new / old state, hn / ho = facing arm equal to the new / old state
    uint32_t cn = 0, co = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
        if (b == A) continue;
        cn += zero_bytes(nw ^ ow[b]);
        co += zero_bytes(oldw ^ ow[b]);
    }
    const uint32_t hn = zero_bytes(nw ^ fw), ho = zero_bytes(oldw ^ fw);
    const uint32_t thw = theta ? (ew & 0x01010101u) : 0u;
    // table index th*33 + (dh+1)*11 + dc+5 per byte; every byte of the first
    // term is >= 16 >= every byte of the second, so no borrow crosses bytes
    const uint32_t idxw = (11u * hn + cn + 0x10101010u + 33u * thw) - (11u * ho + co);
    uint32_t accm = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t thr = met[(idxw >> (8 * j)) & 0xFFu];
        const bool acc = thr == 0xFFFFFFFFu || accw[j] < thr;
        accm |= acc ? (0xFFu << (8 * j)) : 0u;
    }
    accm &= valid;
    const uint32_t out = (nw & accm) | (oldw & ~accm);
    const uint32_t em = accm & (ew * 0xFFu);            // accepted cells whose edge has eta = 1
    cnt[0] += (int)byte_sum(hn & em) - (int)byte_sum(ho & em);
    cnt[1] += (int)byte_sum(cn & accm) - (int)byte_sum(co & accm);
    cnt[2] += __popc(accm) >> 3;
    if (out != oldw) __builtin_amdgcn_raw_buffer_store_b32(out, plane_rsrc(a.sigma + (size_t)A * N, N), (int)c0, 0, 0);
}

__global__ __launch_bounds__(kBlock) void pass3_kernel(Lat3 a)
{
    __shared__ uint32_t met[66];
    if (threadIdx.x < 66) met[threadIdx.x] = (&a.tab->met[0][0][0])[threadIdx.x];
    const int arm = a.st->order[a.pass];
    const uint32_t t = (uint32_t)a.st->t_cur;
    const int theta = a.st->theta;
    __syncthreads();
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    int cnt[3] = {0, 0, 0};
    if (a.quad) {
        // grid-stride over the quads: kQuadsPerLane per lane spreads the
        // lane's fixed work (table load, counter reduction) over more moves
        const uint32_t nq = a.N / 4, stride = gridDim.x * kBlock;
#define CVF3_QUADS(ARM) for (uint32_t u = p; u < nq; u += stride) pass_quad<ARM>(a, met, u, t, theta, cnt)
        switch (arm) {
        case 0: CVF3_QUADS(0); break;
        case 1: CVF3_QUADS(1); break;
        case 2: CVF3_QUADS(2); break;
        case 3: CVF3_QUADS(3); break;
        case 4: CVF3_QUADS(4); break;
        default: CVF3_QUADS(5); break;
        }
#undef CVF3_QUADS
    } else if (p < a.N / 2) {
        switch (arm) {
        case 0: pass_pair<0>(a, met, p, t, theta, cnt); break;
        case 1: pass_pair<1>(a, met, p, t, theta, cnt); break;
        case 2: pass_pair<2>(a, met, p, t, theta, cnt); break;
        case 3: pass_pair<3>(a, met, p, t, theta, cnt); break;
        case 4: pass_pair<4>(a, met, p, t, theta, cnt); break;
        default: pass_pair<5>(a, met, p, t, theta, cnt); break;
        }
    }
    // The three counters of a lane (d N_HB_raw in [-16, 16], d N_sigma in
    // [-80, 80], accepted in [0, 16] for four quads) biased and packed into
    // one word and summed over 16 lanes (sums at most 512, 2560 and 256:
    // fields of 10, 12 and 9 bits), then unpacked and summed over the four
    // 16-lane rows.
    static_assert(kQuadsPerLane <= 4, "field widths below hold for up to four quads per lane");
    uint32_t v = (uint32_t)(cnt[1] + 80) | ((uint32_t)(cnt[0] + 16) << 12) | ((uint32_t)cnt[2] << 22);
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) v += (uint32_t)__shfl_xor((int)v, o, 64);
    int r3[3] = {(int)((v >> 12) & 0x3FFu) - 16 * 16, (int)(v & 0xFFFu) - 16 * 80, (int)(v >> 22)};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r3[k] += __shfl_xor(r3[k], 16, 64);
        r3[k] += __shfl_xor(r3[k], 32, 64);
    }
    __shared__ int part[3][kBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        part[0][wv] = r3[0];
        part[1][wv] = r3[1];
        part[2][wv] = r3[2];
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        int64_t sm = 0;
        for (int i = 0; i < kBlock / 64; ++i) sm += part[threadIdx.x][i];
        if (sm) atomicAdd((unsigned long long*)(a.slots + (size_t)threadIdx.x * kSlots + blockIdx.x % kSlots),
                          (unsigned long long)sm);
    }
}

// ---------------------------------------------------------------------------
// Swendsen-Wang on the cubic lattice (Sec. II.D).  Links of cell c, bit l of
// its mask: l = 0..2 the covalent link of its +d edge (arm 2d of c with arm
// 2d+1 of the +d neighbour; liquid and eta = 1 only; equal arms for
// J_eff > 0, unequal for J_eff < 0), l = 3..17 the 15 cooperative pairs
// (a, b), a < b, lexicographic (equal arms).  Link l uses word l mod 4 of
// Philox(c, t, l / 4, SWB); bond iff word < 64-bit threshold.
// Clusters by a lock-free union-find over the 6N bond indices: a link hooks
// the larger of its two roots under the smaller (CAS on a root's own entry),
// finds halve paths with plain stores of ancestors into non-roots only, so
// parents only decrease and every component ends with its smallest index as
// root -- the label the method's fixed point gives.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void sw3_bonds_kernel(Lat3 a)
{
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= a.N) return;
    const uint32_t L = a.L, N = a.N, L2 = L * L;
    const uint32_t t = (uint32_t)a.st->t_cur;
    const int theta = a.st->theta;
    uint32_t s[6];
#pragma unroll
    for (int b = 0; b < 6; ++b) s[b] = a.sigma[(size_t)b * N + c];
    const uint32_t yz = udiv(c, L, a.invL);
    const uint32_t x = c - yz * L;
    const uint32_t z = udiv(yz, L, a.invL);
    const uint32_t y = yz - z * L;
    const uint32_t nbr[3] = {x == L - 1 ? c + 1 - L : c + 1, y == L - 1 ? c + L - L2 : c + L,
                             c + L2 >= N ? c + L2 - N : c + L2};
    uint32_t w[20];
#pragma unroll
    for (int b = 0; b < 5; ++b) {
        const uint4 r = philox(c, t, (uint32_t)b, kSwb, a.key0, a.key1);
        w[4 * b] = r.x;
        w[4 * b + 1] = r.y;
        w[4 * b + 2] = r.z;
        w[4 * b + 3] = r.w;
    }
    const uint64_t ts = a.tab->sw_sigma, te = theta ? a.tab->sw_eff : 0;
    const int sgn = a.tab->jeff_sign;
    uint32_t m = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const bool eq = s[2 * d] == a.sigma[(size_t)(2 * d + 1) * N + nbr[d]];
        const bool allowed = theta && a.eta[(size_t)d * N + c] != 0;
        const bool want = sgn > 0 ? eq : (sgn < 0 ? !eq : false);
        if (allowed && want && (uint64_t)w[d] < te) m |= 1u << d;
    }
    int l = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i + 1; j < 6; ++j, ++l)
            if (s[i] == s[j] && (uint64_t)w[3 + l] < ts) m |= 1u << (3 + l);
    a.mask[c] = m;
    // The cooperative links join arms of this cell only: their components
    // (transitive closure of the six arms' adjacency, Warshall's order) are
    // resolved here, each arm's parent set to the smallest arm of its
    // component -- the smallest flat index, since arm a of c is a N + c.
    uint32_t comp[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) comp[i] = 1u << i;
    l = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i + 1; j < 6; ++j, ++l)
            if ((m >> (3 + l)) & 1u) {
                comp[i] |= 1u << j;
                comp[j] |= 1u << i;
            }
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int i = 0; i < 6; ++i)
            if ((comp[i] >> k) & 1u) comp[i] |= comp[k];
#pragma unroll
    for (int b = 0; b < 6; ++b) a.par[(size_t)b * N + c] = (uint32_t)(__builtin_ctz(comp[b])) * N + c;
}

__device__ __forceinline__ uint32_t uf_find(uint32_t* par, uint32_t x)
{
    uint32_t p = par[x];
    while (p != x) {
        const uint32_t g = par[p];
        if (g != p) par[x] = g;                            // halve: an ancestor into a non-root
        x = p;
        p = g;
    }
    return x;
}

__device__ __forceinline__ void uf_unite(uint32_t* par, uint32_t u, uint32_t v)
{
    while (true) {
        u = uf_find(par, u);
        v = uf_find(par, v);
        if (u == v) return;
        if (u < v) {
            const uint32_t tmp = u;
            u = v;
            v = tmp;
        }
        const uint32_t old = atomicCAS(par + u, u, v);    // hook the larger root
        if (old == u) return;
        u = old;
    }
}

// Tile phase (L % 8 == 0): one workgroup per TX x TY x TZ cells.  Its 6 T
// bond indices get local indices a T + lx + TX (ly + TY lz), which order
// them as their flat indices a N + c do, so the same rule (hook the larger
// root under the smaller, CAS in LDS) leaves every in-tile component rooted
// at its smallest flat index.  Covalent links inside the tile are united
// here; each bond index's global parent becomes its in-tile root, and only
// links that cross a tile face remain for sw3_union_kernel.
__device__ __forceinline__ uint32_t lds_find(uint32_t* lp, uint32_t x)
{
    uint32_t p = lp[x];
    while (p != x) {
        const uint32_t g = lp[p];
        if (g != p) lp[x] = g;
        x = p;
        p = g;
    }
    return x;
}

__device__ __forceinline__ void lds_unite(uint32_t* lp, uint32_t u, uint32_t v)
{
    while (true) {
        u = lds_find(lp, u);
        v = lds_find(lp, v);
        if (u == v) return;
        if (u < v) {
            const uint32_t tmp = u;
            u = v;
            v = tmp;
        }
        const uint32_t old = atomicCAS(lp + u, u, v);
        if (old == u) return;
        u = old;
    }
}

template <int TX, int TY, int TZ>
__global__ __launch_bounds__(TX * TY * TZ) void sw3_tile_union_kernel(Lat3 a)
{
    constexpr uint32_t T = TX * TY * TZ;
    __shared__ uint32_t lp[6 * T];
    const uint32_t L = a.L, N = a.N;
    const uint32_t tx = L / TX, ty = L / TY;
    // Workgroups are dealt to the eight XCDs in turn, and a tile's row of a
    // plane is TX bytes, a fraction of an L2 line: the j-th workgroup of an
    // XCD takes tile 8 (8 (j / 8) + xcd) + j % 8, so each XCD works on runs of
    // 8 tiles along x that share their lines (the last n % 64 tiles keep
    // their place).
    const uint32_t nt = gridDim.x;
    uint32_t b = blockIdx.x;
    if (b < nt - nt % 64) {
        const uint32_t xcd = b % 8, j = b / 8;
        b = ((j / 8) * 8 + xcd) * 8 + j % 8;
    }
    const uint32_t bx = b % tx, by = (b / tx) % ty, bz = b / (tx * ty);
    const uint32_t t = threadIdx.x, lx = t % TX, ly = (t / TX) % TY, lz = t / (TX * TY);
    const uint32_t c = (TX * bx + lx) + L * ((TY * by + ly) + L * (TZ * bz + lz));
    // in-cell roots from the bonds kernel: parent of arm k is arm r of the same cell
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const uint32_t r = a.par[(size_t)k * N + c] / N;
        lp[k * T + t] = r * T + t;
    }
    __syncthreads();
    const uint32_t m = a.mask[c] & 7u;
    if ((m & 1u) && lx < TX - 1) lds_unite(lp, 0 * T + t, 1 * T + t + 1);
    if ((m & 2u) && ly < TY - 1) lds_unite(lp, 2 * T + t, 3 * T + t + TX);
    if ((m & 4u) && lz < TZ - 1) lds_unite(lp, 4 * T + t, 5 * T + t + TX * TY);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        uint32_t x = k * T + t, q = lp[x];
        while (q != x) {                                   // read-only: lp is not written any more
            x = q;
            q = lp[x];
        }
        const uint32_t rt = x % T, ra = x / T;
        const uint32_t rc = (TX * bx + rt % TX) + L * ((TY * by + (rt / TX) % TY) + L * (TZ * bz + rt / (TX * TY)));
        a.par[(size_t)k * N + c] = ra * N + rc;
    }
}

__global__ __launch_bounds__(kBlock) void sw3_union_kernel(Lat3 a, uint32_t tx_, uint32_t ty_, uint32_t tz_)
{
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= a.N) return;
    uint32_t m = a.mask[c] & 7u;                        // covalent links; cooperative ones are resolved
    if (!m) return;
    const uint32_t L = a.L, N = a.N, L2 = L * L;
    {
        const uint32_t yz = udiv(c, L, a.invL);
        const uint32_t x = c - yz * L;
        const uint32_t z = udiv(yz, L, a.invL);
        const uint32_t y = yz - z * L;
        const uint32_t nbr[3] = {x == L - 1 ? c + 1 - L : c + 1, y == L - 1 ? c + L - L2 : c + L,
                                 c + L2 >= N ? c + L2 - N : c + L2};
        if (tx_) {                                        // in-tile links were united by the tile phase
            if (x % tx_ != tx_ - 1) m &= ~1u;
            if (y % ty_ != ty_ - 1) m &= ~2u;
            if (z % tz_ != tz_ - 1) m &= ~4u;
        }
        // A link whose two ends have the same parents as the active link of
        // the same direction one cell lower along another axis (no wrap) is
        // already implied: each parent is an ancestor of its end, ancestors
        // stay ancestors, so equal parents mean the same two components, and
        // the lower link is united or itself implied by a link lower still.
        // On a percolating cluster most face links repeat a neighbour's pair.
        const uint32_t crd[3] = {x, y, z}, stride[3] = {1u, L, L2};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (!((m >> d) & 1u)) continue;
            const uint32_t u = (2 * d) * N + c, v = (2 * d + 1) * N + nbr[d];
            const uint32_t pu = a.par[u], pv = a.par[v];
            bool implied = false;
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                if (e == d || crd[e] == 0) continue;
                const uint32_t cl = c - stride[e];
                if (!((a.mask[cl] >> d) & 1u)) continue;
                if (a.par[(2 * d) * N + cl] == pu && a.par[(2 * d + 1) * N + nbr[d] - stride[e]] == pv) implied = true;
            }
            if (!implied) uf_unite(a.par, u, v);
        }
    }
}

// Every bond index gets its root (the smallest index of its cluster), and
// shifts by pick(word 0 of Philox(root, t, 0, SWF), q), NONE -> 0.
// Workgroup 0 also clears the recount accumulators for the recount that
// follows (nothing in this launch reads them).
__global__ __launch_bounds__(kBlock) void sw3_flip_kernel(Lat3 a)
{
    if (blockIdx.x == 0)
        for (uint32_t j = threadIdx.x; j < (uint32_t)(kRc * kSlots); j += kBlock) a.rc[j] = 0;
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= 6 * a.N) return;
    const uint32_t r = uf_find(a.par, i);
    const uint32_t t = (uint32_t)a.st->t_cur;
    const uint4 w = philox(r, t, 0u, kSwf, a.key0, a.key1);
    int k = pick_div(w.x, a.q);
    if (k < 0) k = 0;
    uint32_t v = a.sigma[i] + (uint32_t)k;
    v = v >= a.q ? v - a.q : v;
    a.sigma[i] = (uint8_t)v;
}

// Flattening in place: each lane stores only its own entry, and finds here
// never write (a halving store by another lane could otherwise overwrite an
// entry already flattened with an ancestor short of the root); concurrent
// readers see either the old parent or the root, both on the path.
__global__ __launch_bounds__(kBlock) void sw3_labels_kernel(Lat3 a)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= 6 * a.N) return;
    uint32_t x = i, p = a.par[x];
    while (p != x) {
        x = p;
        p = a.par[x];
    }
    a.par[i] = x;
}

// After the flip: the counters become the recount's (slots of the eta move's
// N_HB_raw change are discarded; accepted-eta counts stay).
__global__ void sw3_finish_kernel(Lat3 a)
{
    __shared__ int64_t part[2][kBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t v[2] = {a.rc[threadIdx.x], a.rc[kSlots + threadIdx.x]};
    a.slots[threadIdx.x] = 0;
    a.slots[kSlots + threadIdx.x] = 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        int64_t sm = v[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sm += __shfl_xor(sm, o, 64);
        if (lane == 0) part[k][wv] = sm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t h = 0, c = 0;
        for (int i = 0; i < kBlock / 64; ++i) {
            h += part[0][i];
            c += part[1][i];
        }
        a.st->n_hb_raw = h;
        a.st->n_coop = c;
    }
}

// ---------------------------------------------------------------------------
// Full recount of the configuration (observables): N_HB_raw (eta = 1 edges
// with equal facing sigma), N_sigma (15 pairs per cell), N_q', eta = 0 edges.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void recount3_kernel(Lat3 a)
{
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    int v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (c < a.N) {
        const uint32_t L = a.L, N = a.N, L2 = L * L;
        const uint32_t yz = udiv(c, L, a.invL);
        const uint32_t x = c - yz * L;
        const uint32_t z = udiv(yz, L, a.invL);
        const uint32_t y = yz - z * L;
        uint32_t s[6];
#pragma unroll
        for (int b = 0; b < 6; ++b) s[b] = a.sigma[(size_t)b * N + c];
        const uint32_t nbr[3] = {x == L - 1 ? c + 1 - L : c + 1, y == L - 1 ? c + L - L2 : c + L,
                                 c + L2 >= N ? c + L2 - N : c + L2};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const uint32_t e = a.eta[(size_t)d * N + c];
            v[0] += (e != 0 && s[2 * d] == a.sigma[(size_t)(2 * d + 1) * N + nbr[d]]) ? 1 : 0;
            v[8] += e == 0 ? 1 : 0;
        }
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i + 1; j < 6; ++j) v[1] += s[i] == s[j] ? 1 : 0;
#pragma unroll
        for (int b = 0; b < 6; ++b)
#pragma unroll
            for (int k = 0; k < 6; ++k) v[2 + k] += s[b] == (uint32_t)k ? 1 : 0;
    }
    block_slots<9>(v, a.rc);
}

// N_q' of the current sigma added to out[0..5]: the 6N bytes read as 32-bit
// words; the bytes of w equal to k are the zero bytes of w ^ k 0x01010101,
// counted exactly (no carry crosses a byte) with one popcount.
__global__ __launch_bounds__(kBlock) void counts3_kernel(const uint32_t* __restrict__ words, uint32_t nwords,
                                                         int64_t* out)
{
    int c[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < nwords; i += gridDim.x * kBlock) {
        const uint32_t w = words[i];
#pragma unroll
        for (uint32_t k = 0; k < 6; ++k) c[k] += __popc(zero_bytes(w ^ (k * 0x01010101u)));
    }
    __shared__ int part[6][kBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int sm = wave_sum(c[k]);
        if (lane == 0) part[k][wv] = sm;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        int64_t sm = 0;
        for (int i = 0; i < kBlock / 64; ++i) sm += part[threadIdx.x][i];
        if (sm) atomicAdd((unsigned long long*)(out + threadIdx.x), (unsigned long long)sm);
    }
}

__global__ void zero_kernel(int64_t* p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

inline unsigned blocks_for(uint64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

// ===========================================================================
// Host side: the cvf3_* C ABI.
// ===========================================================================
struct cvf3_state {
    cvf_params p;
    Lat3       la;
    Tab3       htab;
    Tab3*      dtab;
    uint8_t*   sigma;
    uint8_t*   eta;
    bool       timing;
    bool       sw;
    bool       sw_done;
    std::vector<hipEvent_t> ev[CVF3_K_COUNT];
    int64_t    launches[CVF3_K_COUNT];
    double     total_ms[CVF3_K_COUNT];
};

namespace {

size_t al256(size_t n) { return (n + 255) & ~(size_t)255; }

size_t ws3_bytes(const cvf_params* p, int algo_mask)
{
    size_t b = al256(sizeof(Dev3State)) + al256(sizeof(int64_t) * kAcc * kSlots) +
               al256(sizeof(int64_t) * kRc * kSlots) + al256(sizeof(Tab3));
    if (algo_mask & CVF_ALGO_SW) {
        const size_t N = (size_t)p->L * p->L * p->L;
        b += al256(N * sizeof(uint32_t)) + al256(6 * N * sizeof(uint32_t));
    }
    return b;
}

// r3(m): integer points on the sphere i^2 + j^2 + k^2 = m, counted as
// octant points with signs (each nonzero coordinate doubles the count).
double sphere_points(int m)
{
    int n = 0;
    for (int i = 0; i * i <= m; ++i)
        for (int j = 0; i * i + j * j <= m; ++j)
            for (int k = 0; i * i + j * j + k * k <= m; ++k)
                if (i * i + j * j + k * k == m) n += (i ? 2 : 1) * (j ? 2 : 1) * (k ? 2 : 1);
    return (double)n;
}

uint32_t thr_of(double beta, double dH)
{
    if (!(dH > 0.0)) return 0xFFFFFFFFu;
    const double acc = exp(-beta * dH);
    if (acc >= 1.0) return 0xFFFFFFFFu;
    const double f = floor(acc * 4294967296.0);
    return f > 4294967294.0 ? 0xFFFFFFFEu : (uint32_t)f;
}

// Perfect matchings of the cube graph, built from its structure: the three
// one-axis matchings (four parallel edges), and for each axis d the two
// faces perpendicular to d each taking one of their two non-d matchings
// where the two faces differ (2 x 3 = 6), sorted by edge mask.
void cube_matchings(uint32_t out[9])
{
    // edge index of the edge along axis d whose other coordinates are (o1, o2)
    auto edge = [](int d, int o_lo, int o_hi) { return 4 * d + o_lo + 2 * o_hi; };
    std::vector<uint32_t> ms;
    for (int d = 0; d < 3; ++d) ms.push_back(0xFu << (4 * d));
    for (int d = 0; d < 3; ++d) {
        const int a1 = d == 0 ? 1 : 0, a2 = d == 2 ? 1 : 2;   // the two other axes, a1 < a2
        // face at coordinate s along d: a 4-cycle, matched along a1 or a2
        for (int f0 = 0; f0 < 2; ++f0) {
            const int f1 = 1 - f0;
            uint32_t m = 0;
            for (int s = 0; s < 2; ++s) {
                const int along = (s == 0 ? f0 : f1) ? a2 : a1;   // axis of this face's two edges
                // the edge along `along` has its d coordinate = s and the remaining axis r in {0,1}
                const int r = 3 - d - along;
                for (int rv = 0; rv < 2; ++rv) {
                    int coord[3] = {0, 0, 0};
                    coord[d] = s;
                    coord[r] = rv;
                    int o[2], n = 0;
                    for (int ax = 0; ax < 3; ++ax)
                        if (ax != along) o[n++] = coord[ax];
                    m |= 1u << edge(along, o[0], o[1]);
                }
            }
            ms.push_back(m);
        }
    }
    for (size_t i = 0; i < ms.size(); ++i)
        for (size_t j = i + 1; j < ms.size(); ++j)
            if (ms[j] < ms[i]) std::swap(ms[i], ms[j]);
    for (int i = 0; i < 9; ++i) out[i] = ms[i];
}

void build_tab3(const cvf_params* p, Tab3* t)
{
    memset(t, 0, sizeof(*t));
    const double Jeff = p->J - p->P * p->vHB;
    for (int th = 0; th < 2; ++th)
        for (int dh = -1; dh <= 1; ++dh)
            for (int dc = -5; dc <= 5; ++dc)
                t->met[th][dh + 1][dc + 5] = thr_of(p->beta, -((double)th * Jeff * (double)dh) - p->Jsigma * (double)dc);
    for (int dn = -4; dn <= 4; ++dn) t->eta[dn + 4] = thr_of(p->beta, -(Jeff * (double)dn));
    cube_matchings(t->match);
    const double xs = p->beta * p->Jsigma, xe = p->beta * fabs(Jeff);
    t->sw_sigma = xs > 0.0 ? (uint64_t)floor(-expm1(-xs) * 4294967296.0) : 0;
    t->sw_eff = xe > 0.0 ? (uint64_t)floor(-expm1(-xe) * 4294967296.0) : 0;
    t->jeff_sign = Jeff > 0.0 ? 1 : (Jeff < 0.0 ? -1 : 0);
    for (int m = 0; m < 40; ++m) t->r3[m] = m <= 36 ? sphere_points(m) : 0.0;
}

int hs(hipError_t e) { return e == hipSuccess ? CVF_OK : CVF_EHIP; }

int validate3(const cvf_params* p)
{
    if (!p) return CVF_EINVAL;
    if (p->L < 2 || p->L > CVF3_MAX_L || (p->L & 1)) return CVF_EINVAL;
    if (p->q < 2 || p->q > 6) return CVF_EINVAL;
    if (!(p->beta >= 0.0) || !std::isfinite(p->beta)) return CVF_EINVAL;
    if (!std::isfinite(p->J) || !std::isfinite(p->Jsigma) || !std::isfinite(p->P) || !std::isfinite(p->vHB))
        return CVF_EINVAL;
    if (!(p->v_init >= 1.0) || !std::isfinite(p->v_init)) return CVF_EINVAL;
    if (!(p->dv_max >= 0.0) || !std::isfinite(p->dv_max)) return CVF_EINVAL;
    if (p->flags & ~(uint32_t)(CVF_NO_VOLUME_MOVE | CVF_KEEP_SIGMA)) return CVF_EINVAL;
    if (p->reserved != 0) return CVF_EINVAL;
    return CVF_OK;
}

using cvf::DispatchEvents;
using cvf::go;

// With timing on: start/stop events that the next launch of this kind
// records on its own dispatch.
DispatchEvents t_events(cvf3_state* st, int kind)
{
    DispatchEvents ev;
    if (!st->timing) return ev;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return ev;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return ev;
    }
    st->ev[kind].push_back(e0);
    st->ev[kind].push_back(e1);
    ev.start = e0;
    ev.stop = e1;
    return ev;
}

// Events on the stream around several launches (their interval includes
// the gaps between them).
void t_begin(cvf3_state* st, int kind, hipStream_t s)
{
    if (!st->timing) return;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return;
    }
    (void)hipEventRecord(e0, s);
    st->ev[kind].push_back(e0);
    st->ev[kind].push_back(e1);
}

void t_end(cvf3_state* st, int kind, hipStream_t s)
{
    if (!st->timing || st->ev[kind].empty()) return;
    (void)hipEventRecord(st->ev[kind].back(), s);
}

int drain3(cvf3_state* st)
{
    int rc = CVF_OK;
    for (int k = 0; k < CVF3_K_COUNT; ++k) {
        std::vector<hipEvent_t>& v = st->ev[k];
        for (size_t i = 0; i + 1 < v.size(); i += 2) {
            float ms = 0.f;
            if (hipEventSynchronize(v[i + 1]) != hipSuccess || hipEventElapsedTime(&ms, v[i], v[i + 1]) != hipSuccess)
                rc = CVF_EHIP;
            st->launches[k] += 1;
            st->total_ms[k] += ms;
        }
        for (hipEvent_t e : v) (void)hipEventDestroy(e);
        v.clear();
    }
    return rc;
}

}  // namespace

extern "C" {

int validate_algo3(const cvf_params* p, int algo_mask)
{
    if (algo_mask & ~(CVF_ALGO_METROPOLIS | CVF_ALGO_SW)) return CVF_EINVAL;
    if ((algo_mask & CVF_ALGO_SW) && 6ull * (uint64_t)p->L * p->L * p->L >= (1ull << 32)) return CVF_EINVAL;
    return CVF_OK;
}

int cvf3_workspace_bytes(const cvf_params* p, int algo_mask, size_t* bytes)
{
    if (!bytes) return CVF_EINVAL;
    int rc = validate3(p);
    if (rc == CVF_OK) rc = validate_algo3(p, algo_mask);
    if (rc != CVF_OK) return rc;
    *bytes = ws3_bytes(p, algo_mask);
    return CVF_OK;
}

int cvf3_tables(const cvf_params* p, uint32_t met[2][3][11], uint32_t eta[9], uint32_t match[9])
{
    if (!met || !eta || !match) return CVF_EINVAL;
    const int rc = validate3(p);
    if (rc != CVF_OK) return rc;
    Tab3 t;
    build_tab3(p, &t);
    memcpy(met, t.met, sizeof(t.met));
    memcpy(eta, t.eta, sizeof(t.eta));
    memcpy(match, t.match, sizeof(t.match));
    return CVF_OK;
}

int cvf3_init(const cvf_params* p, int algo_mask, uint8_t* d_sigma, uint8_t* d_eta, void* d_work, size_t work_bytes,
              void* stream, cvf3_state** out)
{
    if (!out) return CVF_EINVAL;
    *out = nullptr;
    int rc = validate3(p);
    if (rc == CVF_OK) rc = validate_algo3(p, algo_mask);
    if (rc != CVF_OK) return rc;
    if (!d_sigma || !d_eta || !d_work) return CVF_EINVAL;
    if (((uintptr_t)d_sigma & 3) || ((uintptr_t)d_eta & 3) || ((uintptr_t)d_work & 255)) return CVF_EINVAL;
    if (work_bytes < ws3_bytes(p, algo_mask)) return CVF_ENOMEM;
    cvf3_state* st = new (std::nothrow) cvf3_state();
    if (!st) return CVF_ENOMEM;
    st->p = *p;
    st->sigma = d_sigma;
    st->eta = d_eta;
    build_tab3(p, &st->htab);
    uint8_t* w = (uint8_t*)d_work;
    Lat3& a = st->la;
    a.sigma = d_sigma;
    a.eta = d_eta;
    a.st = (Dev3State*)w;
    w += al256(sizeof(Dev3State));
    a.slots = (int64_t*)w;
    w += al256(sizeof(int64_t) * kAcc * kSlots);
    a.rc = (int64_t*)w;
    w += al256(sizeof(int64_t) * kRc * kSlots);
    st->dtab = (Tab3*)w;
    a.tab = st->dtab;
    w += al256(sizeof(Tab3));
    st->sw = (algo_mask & CVF_ALGO_SW) != 0;
    a.mask = nullptr;
    a.par = nullptr;
    if (st->sw) {
        const size_t N = (size_t)p->L * p->L * p->L;
        a.mask = (uint32_t*)w;
        w += al256(N * sizeof(uint32_t));
        a.par = (uint32_t*)w;
    }
    a.L = (uint32_t)p->L;
    a.N = a.L * a.L * a.L;
    a.h = a.L / 2;
    a.q = (uint32_t)p->q;
    a.key0 = (uint32_t)p->seed;
    a.key1 = (uint32_t)(p->seed >> 32);
    a.invL = 1.0 / (double)a.L;
    a.invH = 1.0 / (double)a.h;
    a.invQ4 = 1.0 / (double)(a.L / 4 ? a.L / 4 : 1);
    a.Nd = (double)a.N;
    a.beta = p->beta;
    a.J = p->J;
    a.P = p->P;
    a.vHB = p->vHB;
    a.dv_max = p->dv_max;
    a.do_volume = (p->flags & CVF_NO_VOLUME_MOVE) ? 0 : 1;
    a.quad = (a.L % 4 == 0) ? 1u : 0u;
    hipStream_t s = (hipStream_t)stream;
    rc = hs(hipMemcpyAsync(st->dtab, &st->htab, sizeof(Tab3), hipMemcpyHostToDevice, s));
    if (rc == CVF_OK) {
        state3_init_kernel<<<1, kBlock, 0, s>>>(a, p->v_init);
        rc = hs(hipGetLastError());
    }
    if (rc == CVF_OK && !(p->flags & CVF_KEEP_SIGMA)) {
        init3_sigma_kernel<<<blocks_for(a.N), kBlock, 0, s>>>(a);
        init3_eta_kernel<<<blocks_for(a.N / 4), kBlock, 0, s>>>(a);
        rc = hs(hipGetLastError());
    }
    if (rc == CVF_OK) {                              // initial counters from a recount
        zero_kernel<<<1, kBlock, 0, s>>>(a.rc, kRc * kSlots);
        recount3_kernel<<<blocks_for(a.N), kBlock, 0, s>>>(a);
        rc = hs(hipGetLastError());
    }
    std::vector<int64_t> h((size_t)kRc * kSlots);
    if (rc == CVF_OK) rc = hs(hipMemcpyAsync(h.data(), a.rc, h.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (rc == CVF_OK) rc = hs(hipStreamSynchronize(s));
    if (rc == CVF_OK) {
        Dev3State ds;
        rc = hs(hipMemcpy(&ds, a.st, sizeof(ds), hipMemcpyDeviceToHost));
        if (rc == CVF_OK) {
            ds.n_hb_raw = ds.n_coop = 0;
            for (int i = 0; i < kSlots; ++i) {
                ds.n_hb_raw += h[0 * kSlots + i];
                ds.n_coop += h[1 * kSlots + i];
            }
            rc = hs(hipMemcpy(a.st, &ds, sizeof(ds), hipMemcpyHostToDevice));
        }
    }
    if (rc != CVF_OK) {
        delete st;
        return rc;
    }
    *out = st;
    return CVF_OK;
}

namespace {

// The eta move of one step: two checkerboard cubes per lane when L % 4 == 0.
hipError_t eta_step(cvf3_state* st, const Lat3& a, hipStream_t s)
{
    const DispatchEvents ev = t_events(st, CVF3_K_ETA);
    if (a.quad) return go(eta3_pair_kernel, dim3(blocks_for(a.N / 8)), dim3(kBlock), s, ev, a);
    return go(eta3_kernel, dim3(blocks_for(a.N / 4)), dim3(kBlock), s, ev, a);
}

}  // namespace

int cvf3_steps(cvf3_state* st, int64_t nsteps, void* stream)
{
    if (!st || nsteps < 0) return CVF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Lat3 a = st->la;
    for (int64_t i = 0; i < nsteps; ++i) {
        if (go(vol3_kernel, dim3(1), dim3(64), s, t_events(st, CVF3_K_VOLUME), a, kVolMet) != hipSuccess)
            return CVF_EHIP;
        if (eta_step(st, a, s) != hipSuccess) return CVF_EHIP;
        const unsigned grid = blocks_for(a.quad ? (a.N / 4 + kQuadsPerLane - 1) / kQuadsPerLane : a.N / 2);
        for (uint32_t pass = 0; pass < 6; ++pass) {
            a.pass = pass;
            if (go(pass3_kernel, dim3(grid), dim3(kBlock), s, t_events(st, CVF3_K_PASS), a) != hipSuccess)
                return CVF_EHIP;
        }
    }
    return CVF_OK;
}

int cvf3_sw_steps(cvf3_state* st, int64_t nsteps, void* stream)
{
    if (!st || nsteps < 0) return CVF_EINVAL;
    if (!st->sw) return CVF_ESTATE;
    hipStream_t s = (hipStream_t)stream;
    const Lat3& a = st->la;
    for (int64_t i = 0; i < nsteps; ++i) {
        if (go(vol3_kernel, dim3(1), dim3(64), s, t_events(st, CVF3_K_VOLUME), a, kVolSw) != hipSuccess)
            return CVF_EHIP;
        if (eta_step(st, a, s) != hipSuccess) return CVF_EHIP;
        if (go(sw3_bonds_kernel, dim3(blocks_for(a.N)), dim3(kBlock), s, t_events(st, CVF3_K_SW_BONDS), a) !=
            hipSuccess)
            return CVF_EHIP;
        t_begin(st, CVF3_K_SW_UNION, s);
        // tile phase: 16 x 8 x 8 cells (a sixteenth of the x links and an
        // eighth of the y and z links cross a face) or 8 x 8 x 4
        if (a.L % 16 == 0) {
            sw3_tile_union_kernel<16, 8, 8><<<a.N / 1024, 1024, 0, s>>>(a);
            sw3_union_kernel<<<blocks_for(a.N), kBlock, 0, s>>>(a, 16, 8, 8);
        } else if (a.L % 8 == 0) {
            sw3_tile_union_kernel<8, 8, 4><<<a.N / 256, 256, 0, s>>>(a);
            sw3_union_kernel<<<blocks_for(a.N), kBlock, 0, s>>>(a, 8, 8, 4);
        } else {
            sw3_union_kernel<<<blocks_for(a.N), kBlock, 0, s>>>(a, 0, 0, 0);
        }
        t_end(st, CVF3_K_SW_UNION, s);
        t_begin(st, CVF3_K_SW_FLIP, s);
        sw3_flip_kernel<<<blocks_for(6ull * a.N), kBlock, 0, s>>>(a);    // also clears the recount's accumulators
        recount3_kernel<<<blocks_for(a.N), kBlock, 0, s>>>(a);
        sw3_finish_kernel<<<1, kBlock, 0, s>>>(a);
        t_end(st, CVF3_K_SW_FLIP, s);
        const int rc = hs(hipGetLastError());
        if (rc != CVF_OK) return rc;
        st->sw_done = true;
    }
    return CVF_OK;
}

int cvf3_labels(cvf3_state* st, uint32_t* d_out, void* stream)
{
    if (!st || !d_out) return CVF_EINVAL;
    if (!st->sw || !st->sw_done) return CVF_ESTATE;
    hipStream_t s = (hipStream_t)stream;
    const Lat3& a = st->la;
    sw3_labels_kernel<<<blocks_for(6ull * a.N), kBlock, 0, s>>>(a);
    int rc = hs(hipGetLastError());
    if (rc == CVF_OK)
        rc = hs(hipMemcpyAsync(d_out, a.par, 6ull * a.N * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    return rc;
}

int cvf3_state_counts(cvf3_state* st, int64_t* d_counts, void* stream)
{
    if (!st || !d_counts || ((uintptr_t)d_counts & 7)) return CVF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const uint32_t nwords = (uint32_t)(6ull * st->la.N / 4);
    uint64_t blocks = (nwords + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    counts3_kernel<<<(unsigned)blocks, kBlock, 0, s>>>((const uint32_t*)st->sigma, nwords, d_counts);
    return hs(hipGetLastError());
}

int cvf3_observables(cvf3_state* st, cvf3_obs* out, void* stream)
{
    if (!st || !out) return CVF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const Lat3& a = st->la;
    vol3_kernel<<<1, 64, 0, s>>>(a, kVolFold);
    zero_kernel<<<1, kBlock, 0, s>>>(a.rc, kRc * kSlots);
    recount3_kernel<<<blocks_for(a.N), kBlock, 0, s>>>(a);
    int rc = hs(hipGetLastError());
    std::vector<int64_t> h((size_t)kRc * kSlots);
    Dev3State ds;
    if (rc == CVF_OK) rc = hs(hipMemcpyAsync(h.data(), a.rc, h.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (rc == CVF_OK) rc = hs(hipMemcpyAsync(&ds, a.st, sizeof(ds), hipMemcpyDeviceToHost, s));
    if (rc == CVF_OK) rc = hs(hipStreamSynchronize(s));
    if (rc != CVF_OK) return rc;
    int64_t tot[kRc] = {0};
    for (int k = 0; k < kRc; ++k)
        for (int i = 0; i < kSlots; ++i) tot[k] += h[(size_t)k * kSlots + i];
    memset(out, 0, sizeof(*out));
    const double Nd = a.Nd;
    out->step = ds.t_next;
    out->n_hb_raw = tot[0];
    out->n_hb = ds.theta ? tot[0] : 0;
    out->n_coop = tot[1];
    int64_t mx = 0;
    for (int k = 0; k < 6; ++k) {
        out->count[k] = tot[2 + k];
        mx = tot[2 + k] > mx ? tot[2 + k] : mx;
    }
    out->n_eta0 = tot[8];
    out->met_attempted = ds.met_att;
    out->met_accepted = ds.met_acc;
    out->eta_attempted = ds.eta_att;
    out->eta_accepted = ds.eta_acc;
    out->vol_attempted = ds.vol_att;
    out->vol_accepted = ds.vol_acc;
    out->v = ds.v;
    out->V = (Nd * ds.v) + (st->p.vHB * (double)out->n_hb);
    out->H = (((Nd * lj3(ds.v, st->htab.r3)) - (st->p.J * (double)out->n_hb)) - (st->p.Jsigma * (double)out->n_coop)) +
             (st->p.P * out->V);
    out->M = (double)mx / (6.0 * Nd);
    out->consistent = (ds.n_hb_raw == tot[0] && ds.n_coop == tot[1]) ? 1 : 0;
    return CVF_OK;
}

int cvf3_timing_enable(cvf3_state* st, int enable)
{
    if (!st) return CVF_EINVAL;
    const int rc = drain3(st);
    for (int k = 0; k < CVF3_K_COUNT; ++k) {
        st->launches[k] = 0;
        st->total_ms[k] = 0.0;
    }
    st->timing = enable != 0;
    return rc;
}

int cvf3_kernel_times(cvf3_state* st, int kind, int64_t* launches, double* mean_ms)
{
    if (!st || kind < 0 || kind >= CVF3_K_COUNT || !launches || !mean_ms) return CVF_EINVAL;
    const int rc = drain3(st);
    *launches = st->launches[kind];
    *mean_ms = st->launches[kind] ? st->total_ms[kind] / (double)st->launches[kind] : 0.0;
    return rc;
}

int cvf3_destroy(cvf3_state* st)
{
    if (!st) return CVF_EINVAL;
    drain3(st);
    delete st;
    return CVF_OK;
}

}  // extern "C"
