// Host side of libcvf: parameter validation, host-computed tables, workspace
// carving, step sequencing on the caller's stream, kernel timing.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "cvf_internal.h"
#include "met_launch.h"

using namespace cvf;


struct cvf_state {
    cvf_params p;
    uint8_t* sigma;
    char* work;
    size_t work_bytes;
    bool has_sw;
    uint32_t N;
    DevState* dst;
    int64_t* slots;
    DevTables* dtab;
    DevObs* dobs;
    uint32_t* label;
    uint8_t* mask;
    uint8_t* edge;
    uint16_t* lroot;
    uint32_t* xchg;
    uint32_t* ecnt;
    DevTables htab;          // host copy (source of the init copy, test hook)
    LatticeArgs la;
    VolArgs va;
    bool timing;
    std::vector<hipEvent_t> ev[CVF_K_COUNT];   // start/stop pairs pending
    double ms[CVF_K_COUNT];
    int64_t launches[CVF_K_COUNT];
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Rows per lane of a batched Metropolis pass before the autotuner runs.
constexpr uint32_t kBatchDefaultRows = 4;

int validate(const cvf_params* p)
{
    if (!p) return CVF_EINVAL;
    if (p->L < 2 || p->L > 32766) return CVF_EINVAL;
    if (p->q < 2 || p->q > 6) return CVF_EINVAL;
    if (!(p->beta >= 0.0) || !isfinite(p->beta)) return CVF_EINVAL;
    if (!isfinite(p->J) || !isfinite(p->Jsigma) || !isfinite(p->P) || !isfinite(p->vHB)) return CVF_EINVAL;
    if (!(p->v_init >= 1.0) || !isfinite(p->v_init)) return CVF_EINVAL;
    if (!(p->dv_max >= 0.0) || !isfinite(p->dv_max)) return CVF_EINVAL;
    if (p->flags & ~(CVF_NO_VOLUME_MOVE | CVF_KEEP_SIGMA)) return CVF_EINVAL;
    if (p->reserved != 0) return CVF_EINVAL;
    return CVF_OK;
}

// SW workspace (labels, bond mask, tile edge bytes, tile-local roots).
size_t sw_tiles(uint64_t L) { return sw_tiles_of(L); }
size_t sw_bytes(uint64_t L) { return sw_bytes_of(L); }

// Number of integer points on the circle i^2 + j^2 = m, counted over the
// first quadrant (i > 0, j >= 0) and multiplied by the 4 rotations.
double lattice_points(int m)
{
    if (m == 0) return 1.0;
    int n = 0;
    for (int i = 1; i * i <= m; ++i)
        for (int j = 0; i * i + j * j <= m; ++j)
            if (i * i + j * j == m) ++n;
    return 4.0 * n;
}

// Acceptance tables, Sec. II.C / II.D with Eq. (3): dH = -theta J_eff dh -
// J_sigma dc for one bond-index change; bond probability 1 - exp(-beta|J|).
void build_tables(const cvf_params* p, DevTables* t)
{
    memset(t, 0, sizeof(*t));
    const double Jeff = p->J - p->P * p->vHB;
    for (int th = 0; th < 2; ++th)
        for (int dh = -1; dh <= 1; ++dh)
            for (int dc = -3; dc <= 3; ++dc) {
                const double dH = -((double)th * Jeff * (double)dh) - p->Jsigma * (double)dc;
                uint32_t thr = 0xFFFFFFFFu;
                if (dH > 0.0) {
                    const double acc = exp(-p->beta * dH);
                    if (acc < 1.0) {
                        const double f = floor(acc * 4294967296.0);
                        thr = f > 4294967294.0 ? 0xFFFFFFFEu : (uint32_t)f;
                    }
                }
                t->met[th][(dh + 1) * 7 + dc + 3] = thr;
            }
    const double xs = p->beta * p->Jsigma;
    t->sw[0] = xs > 0.0 ? (uint64_t)floor(-expm1(-xs) * 4294967296.0) : 0;
    t->sw[1] = 0;
    const double xe = p->beta * fabs(Jeff);
    t->sw[2] = xe > 0.0 ? (uint64_t)floor(-expm1(-xe) * 4294967296.0) : 0;
    for (int m = 0; m < 40; ++m) t->r2[m] = m <= 36 ? lattice_points(m) : 0.0;
}

int hip_status(hipError_t e) { return e == hipSuccess ? CVF_OK : CVF_EHIP; }

// With timing on: a start/stop event pair for the next launch of this kind,
// which its dispatch records (the kernel's execution time alone).
DispatchEvents timing_events(cvf_state* st, int kind)
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

int drain_timing(cvf_state* st)
{
    int rc = CVF_OK;
    for (int k = 0; k < CVF_K_COUNT; ++k) {
        std::vector<hipEvent_t>& v = st->ev[k];
        for (size_t i = 0; i + 1 < v.size(); i += 2) {
            float ms = 0.f;
            if (hipEventSynchronize(v[i + 1]) != hipSuccess || hipEventElapsedTime(&ms, v[i], v[i + 1]) != hipSuccess)
                rc = CVF_EHIP;
            st->ms[k] += ms;
            st->launches[k] += 1;
        }
        for (hipEvent_t e : v) (void)hipEventDestroy(e);
        v.clear();
    }
    return rc;
}

// A launch whose launcher takes the kind's dispatch events as last argument.
#define TIMED(kind, launcher, ...)                                                    \
    do {                                                                              \
        if ((launcher)(__VA_ARGS__, timing_events(st, kind)) != hipSuccess) return CVF_EHIP; \
    } while (0)

}  // namespace

extern "C" {

int cvf_params_from_si(double T_kelvin, double P_MPa, cvf_params* out)
{
    if (!out || !(T_kelvin > 0.0) || !isfinite(T_kelvin) || !isfinite(P_MPa)) return CVF_EINVAL;
    const double N_A = 6.02214076e23;   // 1/mol (SI 2019, exact)
    const double k_B = 1.380649e-23;    // J/K (SI 2019, exact)
    const double eps = 5.5e3;           // J/mol, Table I
    const double r0 = 2.9e-10;          // m, Table I
    const double R = N_A * k_B;
    memset(out, 0, sizeof(*out));
    out->L = 64;
    out->q = 6;
    out->beta = eps / (R * T_kelvin);
    out->J = 4.0 * 0.5;                 // J / (4 eps) = 0.5
    out->Jsigma = 4.0 * 0.08;           // J_sigma / (4 eps) = 0.08
    out->P = ((P_MPa * 1.0e6) * (r0 * r0 * r0)) * N_A / eps;
    out->vHB = 0.6;                     // v_HB = 0.6 v0
    out->v_init = 1.25;
    out->dv_max = 0.01 * 1.25;
    out->seed = 1;
    out->flags = 0;
    return CVF_OK;
}

int cvf_workspace_bytes(const cvf_params* p, int algo_mask, size_t* bytes)
{
    if (!bytes || (algo_mask & ~(CVF_ALGO_METROPOLIS | CVF_ALGO_SW))) return CVF_EINVAL;
    int rc = validate(p);
    if (rc) return rc;
    size_t b = kBaseBytes;
    if (algo_mask & CVF_ALGO_SW) b += sw_bytes((uint64_t)p->L);
    *bytes = b;
    return CVF_OK;
}

}  // extern "C"

namespace {

// Host fields of a chain over sigma and the workspace at `work` (no device
// call, no allocation).
void chain_setup(const cvf_params* p, uint8_t* d_sigma, char* work, size_t work_bytes, cvf_state* st)
{
    st->p = *p;
    st->sigma = d_sigma;
    st->work = work;
    st->work_bytes = work_bytes;
    st->N = (uint32_t)p->L * (uint32_t)p->L;
    st->has_sw = work_bytes >= kBaseBytes + sw_bytes((uint64_t)p->L);
    st->dst = (DevState*)(st->work + kOffState);
    st->slots = (int64_t*)(st->work + kOffSlots);
    st->dtab = (DevTables*)(st->work + kOffTables);
    st->dobs = (DevObs*)(st->work + kOffObs);
    st->label = st->has_sw ? (uint32_t*)(st->work + kBaseBytes) : nullptr;
    st->mask = st->has_sw ? (uint8_t*)(st->work + kBaseBytes + align256(4ull * st->N * sizeof(uint32_t))) : nullptr;
    st->edge = st->has_sw ? st->mask + align256(st->N) : nullptr;
    st->lroot = st->has_sw ? (uint16_t*)(st->edge + align256(sw_tiles((uint64_t)p->L) * kEdgeBytes)) : nullptr;
    st->xchg = st->has_sw ? (uint32_t*)((char*)st->lroot + align256(4ull * st->N * sizeof(uint16_t))) : nullptr;
    st->ecnt = st->has_sw ? st->xchg + align256(sw_tiles((uint64_t)p->L) * kBorderIdx * sizeof(uint32_t)) / 4 : nullptr;
    build_tables(p, &st->htab);

    const double Jeff = p->J - p->P * p->vHB;
    const uint32_t qm1 = (uint32_t)p->q - 1;
    const uint64_t dm = (1ull << 32) / qm1, dq = (1ull << 32) / (uint32_t)p->q;
    LatticeArgs& a = st->la;
    a.sigma = d_sigma;
    a.st = st->dst;
    a.slots = st->slots;
    a.tab = st->dtab;
    a.label = st->label;
    a.mask = st->mask;
    a.edge = st->edge;
    a.lroot = st->lroot;
    a.xchg = st->xchg;
    a.ecnt = st->ecnt;
    a.L = (uint32_t)p->L;
    a.N = st->N;
    a.key0 = (uint32_t)p->seed;
    a.key1 = (uint32_t)(p->seed >> 32);
    a.q = (uint32_t)p->q;
    a.met_lim = (uint32_t)(qm1 * dm - 1);
    a.flip_lim = (uint32_t)((uint64_t)p->q * dq - 1);
    a.jeff_sign = Jeff > 0.0 ? 1 : (Jeff < 0.0 ? -1 : 0);
    a.met_invd = 1.0 / (double)dm;
    a.flip_invd = 1.0 / (double)dq;
    {
        const MetShape m = met_shape(a.L);
        a.quad = m.quad;
        a.rows = m.rows;
        a.row_blocks = m.row_blocks;
    }
    a.met_le = 1;                        // every threshold >= 1: acceptance is word <= thr - 1
    for (int th = 0; th < 2; ++th)
        for (int i = 0; i < 21; ++i)
            if (st->htab.met[th][i] == 0) a.met_le = 0;

    VolArgs& v = st->va;
    v.st = st->dst;
    v.slots = st->slots;
    v.tab = st->dtab;
    v.Nd = (double)st->N;
    v.beta = p->beta;
    v.J = p->J;
    v.P = p->P;
    v.vHB = p->vHB;
    v.dv_max = p->dv_max;
    v.key0 = a.key0;
    v.key1 = a.key1;
    v.met_att_add = 0;
    v.mode = kVolMet;
    v.do_volume = (p->flags & CVF_NO_VOLUME_MOVE) ? 0 : 1;
}

// Device side of a new chain: tables (copied from the host state, or written
// by a kernel when the caller may not copy), scalars and counter slots, the
// initial sigma, the full count.
hipError_t chain_start(cvf_state* st, bool tables_by_kernel, hipStream_t s)
{
    hipError_t e = tables_by_kernel ? launch_tables_init(st->dtab, st->htab, s)
                                    : hipMemcpyAsync(st->dtab, &st->htab, sizeof(DevTables), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_state_init(st->dst, st->slots, st->dtab, st->p.v_init, s);
    if (e == hipSuccess && !(st->p.flags & CVF_KEEP_SIGMA)) e = launch_sigma_init(st->la, s);
    if (e == hipSuccess && st->has_sw) e = launch_sw_counters_init(st->la, s);
    if (e == hipSuccess) e = launch_recount(st->la, st->slots, kSlots, 0, 0, s);
    return e;
}

}  // namespace

extern "C" {

int cvf_init(const cvf_params* p, uint8_t* d_sigma, void* d_work, size_t work_bytes, void* stream,
             cvf_state** out)
{
    if (!out || !d_sigma || !d_work) return CVF_EINVAL;
    int rc = validate(p);
    if (rc) return rc;
    if (((uintptr_t)d_work & 255) != 0 || ((uintptr_t)d_sigma & 3) != 0) return CVF_EINVAL;
    if (work_bytes < kBaseBytes) return CVF_ENOMEM;
    cvf_state* st = new (std::nothrow) cvf_state();
    if (!st) return CVF_EINVAL;
    chain_setup(p, d_sigma, (char*)d_work, work_bytes, st);
    if (chain_start(st, true, (hipStream_t)stream) != hipSuccess) {
        delete st;
        return CVF_EHIP;
    }
    *out = st;
    return CVF_OK;
}

int cvf_metropolis_sweeps(cvf_state* st, int64_t nsweeps, void* stream)
{
    if (!st || nsweeps < 0 || (st->p.L & 1)) return CVF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    VolArgs v = st->va;
    v.mode = kVolMet;
    v.met_att_add = 4 * (int64_t)st->N;
    for (int64_t i = 0; i < nsweeps; ++i) {
        TIMED(CVF_K_VOLUME, launch_volume, v, s);
        TIMED(CVF_K_MET_SWEEP, launch_met_colour, st->la, 0, s);
        TIMED(CVF_K_MET_SWEEP, launch_met_colour, st->la, 1, s);
    }
    return CVF_OK;
}

int cvf_metropolis_domain_sweeps(cvf_state* st, int64_t nsweeps, void* stream)
{
    if (!st || nsweeps < 0) return CVF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    VolArgs v = st->va;
    v.mode = kVolMet;
    v.met_att_add = 4 * (int64_t)st->N;
    for (int64_t i = 0; i < nsweeps; ++i) {
        TIMED(CVF_K_VOLUME, launch_volume, v, s);
        for (uint32_t pass = 0; pass < 4; ++pass) TIMED(CVF_K_MET_DOMAIN, launch_met_domain, st->la, pass, s);
    }
    return CVF_OK;
}

int cvf_sw_steps(cvf_state* st, int64_t nsteps, void* stream)
{
    if (!st || nsteps < 0 || (st->p.L & 1)) return CVF_EINVAL;
    if (!st->has_sw) return CVF_ENOMEM;
    if (!(st->p.Jsigma >= 0.0)) return CVF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    VolArgs v = st->va;
    v.mode = kVolSw;
    for (int64_t i = 0; i < nsteps; ++i) {
        TIMED(CVF_K_VOLUME, launch_volume, v, s);
        TIMED(CVF_K_SW_BONDS, launch_sw_tiles, st->la, s);
        TIMED(CVF_K_SW_FLIP, launch_sw_flip_tiles, st->la, s);
    }
    return CVF_OK;
}

int cvf_observables(cvf_state* st, cvf_obs* out, void* stream);

int cvf_sw_steps_noalloc(const cvf_params* p, uint8_t* d_sigma, int64_t nsteps, cvf_obs* out, void* stream)
{
    // every check that can fail comes before the first device call
    if (!d_sigma || !out || nsteps < 0) return CVF_EINVAL;
    int rc = validate(p);
    if (rc) return rc;
    if ((p->L & 1) || !(p->Jsigma >= 0.0) || ((uintptr_t)d_sigma & 3) != 0) return CVF_EINVAL;
    if ((uint32_t)p->L > kNoAllocMaxL) return CVF_ENOMEM;
    static_assert(kNoAllocBytes >= kBaseBytes + sw_bytes_of(kNoAllocMaxL), "scratch too small");
    void* scr = nullptr;
    if (noalloc_scratch(&scr) != hipSuccess) return CVF_EHIP;
    cvf_state st = cvf_state();          // host state on the stack; timing off, so nothing is allocated
    chain_setup(p, d_sigma, (char*)scr, kNoAllocBytes, &st);
    hipStream_t s = (hipStream_t)stream;
    if (chain_start(&st, true, s) != hipSuccess) return CVF_EHIP;
    rc = cvf_sw_steps(&st, nsteps, stream);
    if (rc) return rc;
    return cvf_observables(&st, out, stream);
}

namespace {

// The recount and the observables record in the workspace (DevObs::out).
hipError_t observables_launch(cvf_state* st, hipStream_t s)
{
    VolArgs v = st->va;
    v.mode = kVolFold;
    hipError_t e = launch_volume(v, s);
    if (e == hipSuccess) e = launch_obs_zero(st->dobs, s);
    if (e == hipSuccess) e = launch_recount(st->la, st->dobs->acc, 1, 1, 0, s);
    if (e == hipSuccess)
        e = launch_obs_final(st->dobs, st->dst, st->dtab, (double)st->N, st->p.J, st->p.Jsigma, st->p.P,
                             st->p.vHB, s);
    return e;
}

}  // namespace

int cvf_observables_async(cvf_state* st, cvf_obs* out, void* stream)
{
    if (!st || !out || ((uintptr_t)out & 7) != 0) return CVF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = observables_launch(st, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, &st->dobs->out, sizeof(cvf_obs), hipMemcpyDefault, s);
    return hip_status(e);
}

int cvf_observables(cvf_state* st, cvf_obs* out, void* stream)
{
    if (!st || !out) return CVF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = observables_launch(st, s);
    cvf_obs tmp;
    if (e == hipSuccess) e = hipMemcpyAsync(&tmp, &st->dobs->out, sizeof(cvf_obs), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return CVF_EHIP;
    *out = tmp;
    return CVF_OK;
}

int cvf_state_counts(cvf_state* st, int64_t* d_counts, void* stream)
{
    if (!st || !d_counts || ((uintptr_t)d_counts & 7) != 0) return CVF_EINVAL;
    return hip_status(launch_state_counts(st->la, d_counts, (hipStream_t)stream));
}

int cvf_labels(cvf_state* st, uint32_t* d_out, void* stream)
{
    if (!st || !d_out) return CVF_EINVAL;
    if (!st->has_sw) return CVF_ESTATE;
    hipStream_t s = (hipStream_t)stream;
    int32_t done = 0;
    hipError_t e = hipMemcpyAsync(&done, &st->dst->sw_done, sizeof(done), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return CVF_EHIP;
    if (!done) return CVF_ESTATE;
    return hip_status(launch_sw_labels(st->la, d_out, s));
}

int cvf_set_stop(cvf_state* st, int64_t stop_at, void* stream)
{
    if (!st || stop_at < 0) return CVF_EINVAL;
    return hip_status(launch_set_stop(st->dst, stop_at, (hipStream_t)stream));
}

int cvf_tables(const cvf_state* st, uint32_t met[2][3][7], uint64_t sw[3])
{
    if (!st || !met || !sw) return CVF_EINVAL;
    for (int th = 0; th < 2; ++th)
        for (int i = 0; i < 21; ++i) met[th][i / 7][i % 7] = st->htab.met[th][i];
    for (int i = 0; i < 3; ++i) sw[i] = st->htab.sw[i];
    return CVF_OK;
}

int cvf_timing_enable(cvf_state* st, int enable)
{
    if (!st) return CVF_EINVAL;
    int rc = drain_timing(st);
    for (int k = 0; k < CVF_K_COUNT; ++k) {
        st->ms[k] = 0.0;
        st->launches[k] = 0;
    }
    st->timing = enable != 0;
    return rc;
}

int cvf_kernel_times(cvf_state* st, int kind, int64_t* launches, double* mean_ms)
{
    if (!st || kind < 0 || kind >= CVF_K_COUNT || !launches || !mean_ms) return CVF_EINVAL;
    int rc = drain_timing(st);
    *launches = st->launches[kind];
    *mean_ms = st->launches[kind] ? st->ms[kind] / (double)st->launches[kind] : 0.0;
    return rc;
}

int cvf_destroy(cvf_state* st)
{
    if (!st) return CVF_EINVAL;
    drain_timing(st);
    delete st;
    return CVF_OK;
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
struct cvf_batch {
    std::vector<cvf_state*> chains;
    std::vector<BatchEntry> host;     // descriptor source (kept alive for async copies)
    std::vector<uint32_t> start;      // prefix sums of Metropolis workgroups, count + 1
    std::vector<uint32_t> tstart;     // prefix sums of SW tiles, count + 1
    BatchEntry* d_ent;
    uint32_t* d_start;
    uint32_t* d_tstart;
    uint32_t total_blocks;
    uint32_t sw_tiles;
    bool has_sw;
    int q;
    int le;                           // every chain's table allows the one-compare acceptance
    int32_t rows;                     // 0 = per-chain default
    hipStream_t capture;              // private stream for graph capture (created at the first capture)
    hipGraphExec_t exec;
    int32_t exec_block;               // sweeps held by exec (0 = none)
};

namespace {

// Descriptor: the entries, then two prefix-sum arrays (Metropolis
// workgroups, SW tiles).
size_t batch_layout(int32_t count, size_t* off_start, size_t* off_tstart)
{
    const size_t ent = align256((size_t)count * sizeof(BatchEntry));
    const size_t st = align256(((size_t)count + 1) * sizeof(uint32_t));
    *off_start = ent;
    *off_tstart = ent + st;
    return ent + 2 * st;
}


void drop_graph(cvf_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    b->exec_block = 0;
}

int batch_upload(cvf_batch* b, hipStream_t s, uint8_t* staging)
{
    const uint32_t count = (uint32_t)b->chains.size();
    b->host.resize(count);
    b->start.assign(count + 1, 0);
    b->tstart.assign(count + 1, 0);
    uint32_t total = 0, ttotal = 0;
    for (uint32_t c = 0; c < count; ++c) {
        const cvf_state* st = b->chains[c];
        BatchEntry& e = b->host[c];
        memset(&e, 0, sizeof(e));
        e.la = st->la;
        // batched passes: quads for L % 4 == 0, column pairs for L % 4 == 2
        // (no ragged quads: their body raises the register need of the
        // batched kernel past its 8-wavefront budget)
        e.la.quad = (e.la.L % 4 == 0) ? 1u : 0u;
        e.va = st->va;
        e.va.mode = kVolMet;
        e.va.met_att_add = 4 * (int64_t)st->N;
        const uint32_t Lc = e.la.L;
        e.upr = e.la.quad ? Lc / 4 : Lc / 2;
        e.upr_inv = 1.0 / (double)e.upr;
        e.units = e.upr * (Lc / 2);
        // the tuned parameter: a quad lane moves `rows` rows (rows / 2 units of
        // two rows, 8 rows updates); a column-pair lane makes as many updates
        // with twice the units, so that every full workgroup has the same work
        const uint32_t rows = b->rows > 0 ? (uint32_t)b->rows : kBatchDefaultRows;
        e.iters = e.la.quad ? (rows / 2 < 1 ? 1 : rows / 2) : rows;
        e.blocks = (uint32_t)(((uint64_t)e.units + 256ull * e.iters - 1) / (256ull * e.iters));
        b->start[c] = total;
        total += e.blocks;
        const uint32_t L = (uint32_t)st->p.L;
        const uint32_t ncx = (L + kTW - 1) / kTW, ncy = (L + kTH - 1) / kTH;
        b->tstart[c] = ttotal;
        ttotal += ncx * ncy;
    }
    b->start[count] = total;
    b->tstart[count] = ttotal;
    b->total_blocks = total;
    b->sw_tiles = ttotal;
    if (staging) {
        // the descriptor image, laid out as on the device, in the caller's
        // pinned staging: one copy, nothing to wait for
        const size_t off_start = (size_t)((char*)b->d_start - (char*)b->d_ent);
        const size_t off_tstart = (size_t)((char*)b->d_tstart - (char*)b->d_ent);
        memcpy(staging, b->host.data(), count * sizeof(BatchEntry));
        memcpy(staging + off_start, b->start.data(), (count + 1) * sizeof(uint32_t));
        memcpy(staging + off_tstart, b->tstart.data(), (count + 1) * sizeof(uint32_t));
        return hip_status(hipMemcpyAsync(b->d_ent, staging, off_tstart + (count + 1) * sizeof(uint32_t),
                                         hipMemcpyHostToDevice, s));
    }
    hipError_t e = hipMemcpyAsync(b->d_ent, b->host.data(), count * sizeof(BatchEntry), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_start, b->start.data(), (count + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_tstart, b->tstart.data(), (count + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, s);
    // the host vectors must stay unchanged until the copies are done
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return hip_status(e);
}

hipError_t batch_sweep(cvf_batch* b, hipStream_t s)
{
    const uint32_t count = (uint32_t)b->chains.size();
    hipError_t e = launch_volume_batch(b->d_ent, count, kVolMet, s);
    if (e == hipSuccess) e = launch_met_batch(b->d_ent, b->d_start, count, b->total_blocks, b->q, 0, b->le, s);
    if (e == hipSuccess) e = launch_met_batch(b->d_ent, b->d_start, count, b->total_blocks, b->q, 1, b->le, s);
    return e;
}

int batch_capture(cvf_batch* b, int32_t block)
{
    drop_graph(b);
    if (!b->capture && hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess) return CVF_EHIP;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
    for (int32_t i = 0; e == hipSuccess && i < block; ++i) e = batch_sweep(b, b->capture);
    hipError_t e2 = hipStreamEndCapture(b->capture, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->exec = nullptr;
        return CVF_EHIP;
    }
    b->exec_block = block;
    return CVF_OK;
}

}  // namespace

int cvf_batch_desc_bytes(int32_t count, size_t* bytes)
{
    if (!bytes || count <= 0) return CVF_EINVAL;
    size_t off, off2;
    *bytes = batch_layout(count, &off, &off2);
    return CVF_OK;
}

namespace {

// Both creation calls: h_staging NULL uploads from the batch's host vectors
// and waits; otherwise the table is written into the caller's pinned
// staging (staging_bytes >= desc_bytes) and copied without waiting.
int batch_create(cvf_state* const* chains, int32_t count, void* d_desc, size_t desc_bytes, void* h_staging,
                 size_t staging_bytes, void* stream, cvf_batch** out)
{
    (void)staging_bytes;
    if (!chains || count <= 0 || !d_desc || !out) return CVF_EINVAL;
    if (((uintptr_t)d_desc & 255) != 0) return CVF_EINVAL;
    size_t off_start, off_tstart;
    if (desc_bytes < batch_layout(count, &off_start, &off_tstart)) return CVF_ENOMEM;
    for (int32_t c = 0; c < count; ++c)
        if (!chains[c] || chains[c]->p.q != chains[0]->p.q || (chains[c]->p.L & 1)) return CVF_EINVAL;
    cvf_batch* b = new (std::nothrow) cvf_batch();
    if (!b) return CVF_EINVAL;
    b->chains.assign(chains, chains + count);
    b->d_ent = (BatchEntry*)d_desc;
    b->d_start = (uint32_t*)((char*)d_desc + off_start);
    b->d_tstart = (uint32_t*)((char*)d_desc + off_tstart);
    b->q = chains[0]->p.q;
    b->le = 1;
    for (int32_t c = 0; c < count; ++c)
        if (!chains[c]->la.met_le) b->le = 0;
    b->has_sw = true;
    for (int32_t c = 0; c < count; ++c) b->has_sw = b->has_sw && chains[c]->has_sw && chains[c]->p.Jsigma >= 0.0;
    b->rows = 0;
    b->exec = nullptr;
    b->exec_block = 0;
    b->capture = nullptr;
    int rc = batch_upload(b, (hipStream_t)stream, (uint8_t*)h_staging);
    if (rc) {
        delete b;
        return rc;
    }
    *out = b;
    return CVF_OK;
}

}  // namespace

int cvf_batch_create(cvf_state* const* chains, int32_t count, void* d_desc, size_t desc_bytes, void* stream,
                     cvf_batch** out)
{
    return batch_create(chains, count, d_desc, desc_bytes, nullptr, 0, stream, out);
}

int cvf_batch_create_async(cvf_state* const* chains, int32_t count, void* d_desc, size_t desc_bytes,
                           void* h_staging, size_t staging_bytes, void* stream, cvf_batch** out)
{
    if (!h_staging || staging_bytes < desc_bytes) return CVF_EINVAL;
    return batch_create(chains, count, d_desc, desc_bytes, h_staging, staging_bytes, stream, out);
}

int cvf_batch_set_rows(cvf_batch* b, int32_t rows, void* stream)
{
    if (!b || rows < 0 || rows > 32 || (rows & 1)) return CVF_EINVAL;
    drop_graph(b);
    b->rows = rows;
    return batch_upload(b, (hipStream_t)stream, nullptr);
}

int cvf_batch_metropolis_sweeps(cvf_batch* b, int64_t nsweeps, int32_t graph_block, void* stream)
{
    if (!b || nsweeps < 0 || graph_block < 0) return CVF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int64_t done = 0;
    if (graph_block > 0 && nsweeps >= graph_block) {
        if (b->exec_block != graph_block) {
            int rc = batch_capture(b, graph_block);
            if (rc) return rc;
        }
        for (; done + graph_block <= nsweeps; done += graph_block)
            if (hipGraphLaunch(b->exec, s) != hipSuccess) return CVF_EHIP;
    }
    for (; done < nsweeps; ++done)
        if (batch_sweep(b, s) != hipSuccess) return CVF_EHIP;
    return CVF_OK;
}

int cvf_batch_sw_steps(cvf_batch* b, int64_t nsteps, void* stream)
{
    if (!b || nsteps < 0) return CVF_EINVAL;
    if (!b->has_sw) return CVF_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    const uint32_t count = (uint32_t)b->chains.size();
    for (int64_t i = 0; i < nsteps; ++i) {
        hipError_t e = launch_volume_batch(b->d_ent, count, kVolSw, s);
        if (e == hipSuccess) e = launch_sw_batch(b->d_ent, b->d_tstart, count, b->sw_tiles, 0, s);
        if (e == hipSuccess) e = launch_sw_batch(b->d_ent, b->d_tstart, count, b->sw_tiles, 2, s);
        if (e != hipSuccess) return CVF_EHIP;
    }
    return CVF_OK;
}

int cvf_batch_autotune(cvf_batch* b, int32_t sweeps, void* stream, int32_t* rows_out)
{
    if (!b || sweeps <= 0 || !rows_out) return CVF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int32_t cand[5] = {2, 4, 8, 16, 32};
    float best = 0.f;
    int32_t best_rows = 0;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return CVF_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return CVF_EHIP;
    }
    // one untimed block first (clocks and caches settle), then two timed
    // rounds over the candidates; each keeps its faster time
    int rc = cvf_batch_set_rows(b, cand[0], stream);
    for (int32_t k = 0; k < sweeps && rc == CVF_OK; ++k)
        if (batch_sweep(b, s) != hipSuccess) rc = CVF_EHIP;
    float t_min[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    for (int round = 0; round < 2 && rc == CVF_OK; ++round) {
        for (int i = 0; i < 5 && rc == CVF_OK; ++i) {
            rc = cvf_batch_set_rows(b, cand[i], stream);
            if (rc) break;
            if (hipEventRecord(e0, s) != hipSuccess) { rc = CVF_EHIP; break; }
            for (int32_t k = 0; k < sweeps && rc == CVF_OK; ++k)
                if (batch_sweep(b, s) != hipSuccess) rc = CVF_EHIP;
            float ms = 0.f;
            if (rc == CVF_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = CVF_EHIP;
            if (rc == CVF_OK && (round == 0 || ms < t_min[i])) t_min[i] = ms;
        }
    }
    for (int i = 0; i < 5 && rc == CVF_OK; ++i) {
        if (best_rows == 0 || t_min[i] < best) {
            best = t_min[i];
            best_rows = cand[i];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    rc = cvf_batch_set_rows(b, best_rows, stream);
    if (rc == CVF_OK) *rows_out = best_rows;
    return rc;
}

int cvf_batch_destroy(cvf_batch* b)
{
    if (!b) return CVF_EINVAL;
    drop_graph(b);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    delete b;
    return CVF_OK;
}

const char* cvf_strerror(int code)
{
    switch (code) {
    case CVF_OK: return "ok";
    case CVF_EINVAL: return "invalid argument";
    case CVF_ENOMEM: return "workspace too small";
    case CVF_EHIP: return "HIP runtime error";
    case CVF_ESTATE: return "invalid state for this call";
    default: return "unknown error";
    }
}

}  // extern "C"
