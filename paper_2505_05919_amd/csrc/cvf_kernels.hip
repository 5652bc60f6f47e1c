// HIP kernels of libcvf for gfx950 (MI355X).
//
// The lattice kernels are integer-only: uint8 bond indices, uint32 Philox
// words and thresholds, int32 per-lane deltas reduced across the wavefront
// and the workgroup, int64 atomics into spread slots.  The single-wave
// volume kernel is the only floating-point code (FP64, no contraction).
#include "cvf_internal.h"

#include <atomic>

namespace cvf {

// Fixed device workspace of the allocation-free entry point
// (cvf_sw_steps_noalloc): every GPU the library runs on holds one copy,
// from module load until the process ends.  Host code never passes this
// name to a kernel or a copy (on the host it is only a stand-in for the
// symbol); it uses the device address from noalloc_scratch().
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kBlock = 256;           // 4 wavefronts of 64
constexpr int kMaxBlocks = 8192;      // 256 CUs x 8 waves/SIMD x 4 SIMDs / 4 waves

#include "philox.h"

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
template <int NV, int BLOCK = kBlock>
__device__ __forceinline__ void block_add(const int (&v)[NV], int64_t* dst, int stride)
{
    __shared__ int part[NV][BLOCK / 64];
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
        for (int w = 0; w < BLOCK / 64; ++w) s += part[tid][w];
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
        st->skip = 0;
        st->stop_at = INT64_MAX;
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
// Executed by one full wavefront (lanes 0..63); `term` is 40 doubles of LDS.
// Every global load is issued before the first store, so the whole move
// costs one memory round trip.  `out` (batches): the batch entry that also
// receives the opened step (skip, theta, step index).
__device__ void volume_step(const VolArgs& a, double* term, BatchEntry* out = nullptr)
{
    const int lane = threadIdx.x & 63;
    DevState* st = a.st;
    int64_t sl[3][kSlots / 64];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int k = 0; k < kSlots / 64; ++k) sl[j][k] = a.slots[j * kSlots + k * 64 + lane];
    const int64_t t_next = st->t_next, stop_at = st->stop_at;
    const int64_t hb0 = st->n_hb_raw, co0 = st->n_coop, macc0 = st->met_acc, matt0 = st->met_att;
    const int64_t vatt0 = st->vol_att, vacc0 = st->vol_acc;
    const double v0 = st->v, u0 = st->u;
    const int th0 = st->theta;
    const double r2 = lane < 40 ? a.tab->r2[lane] : 0.0;
    int64_t hb = 0, co = 0, ac = 0;
#pragma unroll
    for (int k = 0; k < kSlots / 64; ++k) {
        hb += sl[0][k];
        co += sl[1][k];
        ac += sl[2][k];
    }
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int k = 0; k < kSlots / 64; ++k) a.slots[j * kSlots + k * 64 + lane] = 0;
    // the three sums in one butterfly: each step's six 32-bit exchanges are
    // issued together and waited for once
    int64_t r[3] = {hb, co, ac};
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        int64_t x[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) x[j] = __shfl_xor(r[j], o, 64);
#pragma unroll
        for (int j = 0; j < 3; ++j) r[j] += x[j];
    }
    const int64_t n_hb = hb0 + r[0];
    const int64_t n_co = co0 + r[1];
    const int64_t m_acc = macc0 + r[2];
    if (a.mode == kVolFold || t_next >= stop_at) {   // fold only; at the step limit the step kernels skip
        if (lane == 0) {
            st->n_hb_raw = n_hb;
            st->n_coop = n_co;
            st->met_acc = m_acc;
            if (a.mode != kVolFold) st->skip = 1;
            if (out) out->skip = 1;
        }
        return;
    }
    const uint32_t t = (uint32_t)t_next;
    const uint4 w = philox(0u, t, 0u, kStreamVol, a.key0, a.key1);
    const double u = (double)((int64_t)2 * (int64_t)w.x + 1 - 4294967296LL) * (1.0 / 4294967296.0);
    const double v1 = v0 + a.dv_max * u;
    const bool inside = a.do_volume && v1 >= 1.0;
    if (inside && lane >= 1 && lane <= 36) {
        const double d2 = v1 * (double)lane;
        const double s6 = 1.0 / (d2 * d2 * d2);
        term[lane] = r2 * (s6 * s6 - s6);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (lane != 0) return;
    double v = v0, uu = u0;
    int th = th0;
    int64_t vatt = vatt0, vacc = vacc0;
    if (a.do_volume) {
        vatt += 1;
        if (inside) {
            // all 36 shell terms read first, then added in ascending m while
            // v' m <= 36 (v' >= 1, so the condition fails past m = 36; it is
            // monotone in m, so the terms added and their order are those of
            // the loop that stops at the first failing m)
            double tm[36];
#pragma unroll
            for (int m = 1; m <= 36; ++m) tm[m - 1] = term[m];
            double sum = 0.0;
#pragma unroll
            for (int m = 1; m <= 36; ++m)
                if (v1 * (double)m <= 36.0) sum = sum + tm[m - 1];
            const double u1 = 2.0 * sum;
            const int th1 = v1 < 2.0 ? 1 : 0;
            const double dH = (a.Nd * (u1 - u0))
                            + ((a.P * a.Nd) * (v1 - v0))
                            + (((double)(th1 - th0) * (a.P * a.vHB - a.J)) * (double)n_hb);
            bool acc = dH <= 0.0;
            if (!acc) acc = ((double)w.y + 0.5) * (1.0 / 4294967296.0) < exp(-a.beta * dH);
            if (acc) {
                v = v1;
                uu = u1;
                th = th1;
                vacc += 1;
            }
        }
    }
    st->skip = 0;
    st->t_cur = t;
    if (out) {
        out->skip = 0;
        out->theta = th;
        out->t_cur = t;
    }
    st->t_next = t_next + 1;
    st->met_att = matt0 + a.met_att_add;
    st->met_acc = m_acc;
    st->vol_att = vatt;
    st->vol_acc = vacc;
    st->v = v;
    st->u = uu;
    st->theta = th;
    const bool sw = a.mode == kVolSw;            // the SW step ends with a full recount
    st->n_hb_raw = sw ? 0 : n_hb;
    st->n_coop = sw ? 0 : n_co;
}

__global__ __launch_bounds__(64) void volume_kernel(VolArgs a)
{
    __shared__ double term[40];
    volume_step(a, term);
}

#include "met_sweep.h"
#include "met_domain.h"

// Raw buffer helpers for the recount (the sweep kernels have their own).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(uint8_t* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ uint32_t ld8b(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_amdgcn_raw_buffer_load_b8(r, (int)voff, (int)soff, 0);
}

#include "sw_step.h"

// N_q' of the current sigma (q' < 6), added to out[0..5].  The planes are
// read as 32-bit words; the bytes of w equal to k are the zero bytes of
// x = w ^ k 0x01010101, flagged in bit 7 of every byte of
// ~(((x & 0x7F7F7F7F) + 0x7F7F7F7F) | x | 0x7F7F7F7F) (no carry crosses a
// byte), and counted with one popcount.
__global__ __launch_bounds__(kBlock) void state_counts_kernel(const uint32_t* __restrict__ words, uint32_t nwords,
                                                              int64_t* out)
{
    int c[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < nwords; i += gridDim.x * kBlock) {
        const uint32_t w = words[i];
#pragma unroll
        for (uint32_t k = 0; k < 6; ++k) {
            const uint32_t x = w ^ (k * 0x01010101u);
            c[k] += __popc(~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x | 0x7F7F7F7Fu));
        }
    }
    block_add<6>(c, out, 1);
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

hipError_t launch_volume(const VolArgs& a, hipStream_t s, DispatchEvents ev)
{
    return go(volume_kernel, dim3(1), dim3(64), s, ev, a);
}

template <int Q, bool R, bool LE>
hipError_t launch_quad_r(const LatticeArgs& a, int colour, dim3 grid, hipStream_t s, const DispatchEvents& ev)
{
    if (colour == 0) return go(met_sweep4_kernel<Q, 0, R, LE>, grid, dim3(256), s, ev, a);
    return go(met_sweep4_kernel<Q, 1, R, LE>, grid, dim3(256), s, ev, a);
}

template <int Q>
hipError_t launch_quad(const LatticeArgs& a, int colour, dim3 grid, hipStream_t s, const DispatchEvents& ev)
{
    if (a.quad == 2) {
        if (a.met_le) return launch_quad_r<Q, true, true>(a, colour, grid, s, ev);
        return launch_quad_r<Q, true, false>(a, colour, grid, s, ev);
    }
    if (a.met_le) return launch_quad_r<Q, false, true>(a, colour, grid, s, ev);
    return launch_quad_r<Q, false, false>(a, colour, grid, s, ev);
}

hipError_t launch_met_colour(const LatticeArgs& a, int colour, hipStream_t s, DispatchEvents ev)
{
    if (a.quad) {
        const dim3 grid(((a.L + 3) / 4 + 63) / 64, a.row_blocks);
        switch (a.q) {
        case 2: return launch_quad<2>(a, colour, grid, s, ev);
        case 3: return launch_quad<3>(a, colour, grid, s, ev);
        case 4: return launch_quad<4>(a, colour, grid, s, ev);
        case 5: return launch_quad<5>(a, colour, grid, s, ev);
        default: return launch_quad<6>(a, colour, grid, s, ev);
        }
    }
    const dim3 grid((a.L / 2 + 63) / 64, a.row_blocks), block(256);
    switch (a.q) {
    case 2: return go(met_sweep_kernel<2>, grid, block, s, ev, a, colour);
    case 3: return go(met_sweep_kernel<3>, grid, block, s, ev, a, colour);
    case 4: return go(met_sweep_kernel<4>, grid, block, s, ev, a, colour);
    case 5: return go(met_sweep_kernel<5>, grid, block, s, ev, a, colour);
    default: return go(met_sweep_kernel<6>, grid, block, s, ev, a, colour);
    }
}

__global__ void set_stop_kernel(DevState* st, int64_t stop_at)
{
    if (threadIdx.x == 0) st->stop_at = stop_at;
}

__global__ void tables_init_kernel(DevTables* dst, DevTables src)
{
    const uint32_t* in = (const uint32_t*)&src;
    uint32_t* out = (uint32_t*)dst;
    for (uint32_t i = threadIdx.x; i < sizeof(DevTables) / 4; i += blockDim.x) out[i] = in[i];
}

hipError_t launch_tables_init(DevTables* dst, const DevTables& src, hipStream_t s)
{
    tables_init_kernel<<<1, 64, 0, s>>>(dst, src);
    return hipGetLastError();
}

// Per-device address of `scratch`, taken once per device with that device
// current (each GPU holds its own copy at its own address).
hipError_t noalloc_scratch(void** ptr)
{
    constexpr int kMaxDevices = 64;
    static std::atomic<void*> addr[kMaxDevices];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    void* p = addr[dev].load(std::memory_order_acquire);
    if (!p) {
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || ((uintptr_t)p & 255) != 0) return hipErrorInvalidSymbol;
        addr[dev].store(p, std::memory_order_release);
    }
    *ptr = p;
    return hipSuccess;
}

hipError_t launch_set_stop(DevState* st, int64_t stop_at, hipStream_t s)
{
    set_stop_kernel<<<1, 64, 0, s>>>(st, stop_at);
    return hipGetLastError();
}

template <int Q>
hipError_t launch_domain_q(const LatticeArgs& a, uint32_t pass, dim3 grid, uint32_t rows, hipStream_t s,
                           const DispatchEvents& ev)
{
    if (a.L % 4 == 0) return go(met_domain_kernel<Q, 2>, grid, dim3(256), s, ev, a, pass, rows);
    if (a.L % 2 == 0) return go(met_domain_kernel<Q, 1>, grid, dim3(256), s, ev, a, pass, rows);
    return go(met_domain_kernel<Q, 0>, grid, dim3(256), s, ev, a, pass, rows);
}

hipError_t launch_met_domain(const LatticeArgs& a, uint32_t pass, hipStream_t s, DispatchEvents ev)
{
    // lanes own column quads (L % 4 == 0) or pairs, (L + 1) / 2 per row; rows
    // per wavefront for ~8192 wavefronts (measured at L = 4096 with pairs:
    // 515 vs 458 updates/ns for 4096)
    const uint32_t lanes = (a.L % 4 == 0) ? a.L / 4 : (a.L + 1) / 2;
    const uint32_t groups = (lanes + 63) / 64;
    const uint32_t wpg = groups >= 8192 ? 1 : 8192 / groups;
    const uint32_t rows = min(32u, (a.L + wpg - 1) / wpg);
    const dim3 grid(groups, ((a.L + rows - 1) / rows + 3) / 4);
    switch (a.q) {
    case 2: return launch_domain_q<2>(a, pass, grid, rows, s, ev);
    case 3: return launch_domain_q<3>(a, pass, grid, rows, s, ev);
    case 4: return launch_domain_q<4>(a, pass, grid, rows, s, ev);
    case 5: return launch_domain_q<5>(a, pass, grid, rows, s, ev);
    default: return launch_domain_q<6>(a, pass, grid, rows, s, ev);
    }
}

hipError_t launch_recount(const LatticeArgs& a, int64_t* out, int spread, int with_counts, int step_gate,
                          hipStream_t s)
{
    if (!with_counts && a.L % 2 == 0) {               // column pairs: even L
        // rows per wavefront for ~8192 wavefronts
        const uint32_t groups = (a.L / 2 + 63) / 64;
        const uint32_t wpg = groups >= 8192 ? 1 : 8192 / groups;
        const uint32_t rows = (a.L + wpg - 1) / wpg;
        const uint32_t segs = (a.L + rows - 1) / rows;
        const dim3 grid(groups, (segs + 3) / 4);
        recount_rows_kernel<<<grid, 256, 0, s>>>(a, out, spread, step_gate, rows);
        return hipGetLastError();
    }
    recount_kernel<<<grid_for(a.N), kBlock, 0, s>>>(a, out, spread, with_counts, step_gate);
    return hipGetLastError();
}

hipError_t launch_state_counts(const LatticeArgs& a, int64_t* out, hipStream_t s)
{
    const uint32_t nwords = a.N;                          // 4N bytes
    state_counts_kernel<<<grid_for(nwords), kBlock, 0, s>>>(reinterpret_cast<const uint32_t*>(a.sigma), nwords, out);
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

hipError_t launch_sw_tiles(const LatticeArgs& a, hipStream_t s, DispatchEvents ev)
{
    const dim3 grid((a.L + kTW - 1) / kTW, (a.L + kTH - 1) / kTH);
    return go(sw_tile_kernel, grid, dim3(kTT), s, ev, a);
}

__global__ void sw_counters_init_kernel(uint32_t* ecnt, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) ecnt[i] = 0;
}

hipError_t launch_sw_counters_init(const LatticeArgs& a, hipStream_t s)
{
    const uint32_t n = 2 * ((a.L + kTW - 1) / kTW) * ((a.L + kTH - 1) / kTH);
    sw_counters_init_kernel<<<grid_for(n), kBlock, 0, s>>>(a.ecnt, n);
    return hipGetLastError();
}

template <int Q>
void launch_batch_q(const BatchEntry* ent, const uint32_t* start, uint32_t count, uint32_t total, int colour,
                    int le, hipStream_t s)
{
    if (le) {
        if (colour == 0) met_batch_kernel<Q, 0, true><<<total, 256, 0, s>>>(ent, start, count);
        else met_batch_kernel<Q, 1, true><<<total, 256, 0, s>>>(ent, start, count);
    } else {
        if (colour == 0) met_batch_kernel<Q, 0, false><<<total, 256, 0, s>>>(ent, start, count);
        else met_batch_kernel<Q, 1, false><<<total, 256, 0, s>>>(ent, start, count);
    }
}

hipError_t launch_met_batch(const BatchEntry* ent, const uint32_t* start, uint32_t count, uint32_t total_blocks,
                            int q, int colour, int le, hipStream_t s)
{
    switch (q) {
    case 2: launch_batch_q<2>(ent, start, count, total_blocks, colour, le, s); break;
    case 3: launch_batch_q<3>(ent, start, count, total_blocks, colour, le, s); break;
    case 4: launch_batch_q<4>(ent, start, count, total_blocks, colour, le, s); break;
    case 5: launch_batch_q<5>(ent, start, count, total_blocks, colour, le, s); break;
    default: launch_batch_q<6>(ent, start, count, total_blocks, colour, le, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_volume_batch(BatchEntry* ent, uint32_t count, int mode, hipStream_t s)
{
    volume_batch_kernel<<<count, 64, 0, s>>>(ent, mode);
    return hipGetLastError();
}

hipError_t launch_sw_batch(const BatchEntry* ent, const uint32_t* start, uint32_t count, uint32_t total_blocks,
                           int stage, hipStream_t s)
{
    if (total_blocks == 0) return hipSuccess;
    if (stage == 0) sw_tile_batch_kernel<<<total_blocks, kTT, 0, s>>>(ent, start, count);
    else sw_flip_batch_kernel<<<total_blocks, kTT, 0, s>>>(ent, start, count);
    return hipGetLastError();
}

hipError_t launch_sw_flip_tiles(const LatticeArgs& a, hipStream_t s, DispatchEvents ev)
{
    const dim3 grid((a.L + kTW - 1) / kTW, (a.L + kTH - 1) / kTH);
    return go(sw_flip_tile_kernel, grid, dim3(kTT), s, ev, a);
}

hipError_t launch_sw_labels(const LatticeArgs& a, uint32_t* out, hipStream_t s)
{
    const dim3 grid((a.L + kTW - 1) / kTW, (a.L + kTH - 1) / kTH);
    sw_labels_kernel<<<grid, kTT, 0, s>>>(a, out);
    return hipGetLastError();
}

}  // namespace cvf
