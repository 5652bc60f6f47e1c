// Internal definitions shared by the host API and the HIP kernels of libcvf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cvf.h"
#include "dispatch.h"

namespace cvf {

// Philox stream ids (fourth counter word): one per kind of random decision.
constexpr uint32_t kStreamInit = 0;   // initial configuration
constexpr uint32_t kStreamVol = 1;    // volume move
constexpr uint32_t kStreamMet = 2;    // Metropolis proposal + acceptance
constexpr uint32_t kStreamSwb = 3;    // Swendsen-Wang bond activation
constexpr uint32_t kStreamSwf = 4;    // Swendsen-Wang cluster shift
constexpr uint32_t kStreamOrd = 5;    // arm-domain sweep: pass order
constexpr uint32_t kStreamDom = 6;    // arm-domain sweep: proposal + acceptance

// Per-workgroup partial sums are spread over this many int64 slots so that
// same-address atomics do not serialise; the volume kernel folds them.
constexpr int kSlots = 256;

// Swendsen-Wang tiles: kTW x kTH cells per workgroup (the last tile of a row
// or column is ragged).  Per tile the bond kernel keeps, for the step's
// fused recount, the old sigma of the facing arm across the right edge (kTH
// bytes, one per row) and across the bottom edge (kTW bytes, one per column).
#ifndef CVF_SW_TILE_H
#define CVF_SW_TILE_H 16
#endif
constexpr uint32_t kTW = 64, kTH = CVF_SW_TILE_H, kTC = kTW * kTH;
constexpr uint32_t kTT = kTC / 4;        // threads of a tile workgroup: 4 cells, 16 bond indices each
constexpr uint32_t kEdgeBytes = kTW + kTH;

// Mutable per-chain scalars, at offset 0 of the workspace.
struct DevState {
    int64_t t_next;          // index of the next MC step
    int64_t n_hb_raw;        // incremental totals (after folding the slots)
    int64_t n_coop;
    int64_t met_att, met_acc, vol_att, vol_acc;
    double v;                // v_iso / v0
    double u;                // u_LJ(v), cached: the volume move needs u(v) and u(v')
    uint32_t t_cur;          // step being executed (Philox counter word 1)
    int32_t theta;           // 1 liquid (v < 2), 0 gas
    int32_t sw_done;         // a Swendsen-Wang step has produced labels
    int32_t skip;            // 1: the step limit is reached, step kernels do nothing
    int64_t stop_at;         // no step with index >= stop_at is performed
};

// Host-computed constants copied to the workspace at init.
struct DevTables {
    uint32_t met[2][21];     // Metropolis thresholds [theta][(dh+1)*7 + dc+3]
    uint32_t pad_[2];
    uint64_t sw[3];          // SW thresholds: cooperative, covalent theta=0, theta=1
    double r2[40];           // lattice-point counts r2(m), m = 0..36
};

// Observable accumulators + the final record copied to the host.
struct DevObs {
    int64_t acc[8];          // recount: n_hb_raw, n_coop, count[0..5]
    cvf_obs out;
};

// Workspace layout (byte offsets, all 256-aligned).
constexpr size_t kOffState = 0;
constexpr size_t kOffSlots = 256;
constexpr size_t kOffTables = kOffSlots + 3 * kSlots * sizeof(int64_t);   // 6400
constexpr size_t kOffObs = kOffTables + 768;                                // 7168
constexpr size_t kBaseBytes = kOffObs + 512;                                // 7680

// Border bond indices of a tile (the ends of its tile-crossing links):
// arm 0 of the last column and arm 1 of the first (one per row), arm 2 of
// the last row and arm 3 of the first (one per column).
constexpr uint32_t kBorderIdx = 2 * (kTW + kTH);

// Swendsen-Wang part of a workspace, each piece 256-aligned: labels (4N
// uint32), bond mask (N bytes), per-tile edge bytes, tile-local roots (4N
// uint16), per-tile exchange words (kBorderIdx uint32: the global root of
// each border bond index, or kNoLink), per-tile edge counters (2 uint32).
constexpr size_t align256c(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t sw_tiles_of(uint64_t L) { return ((L + kTW - 1) / kTW) * ((L + kTH - 1) / kTH); }
constexpr size_t sw_bytes_of(uint64_t L)
{
    return align256c(4 * L * L * sizeof(uint32_t)) + align256c(L * L) + align256c(sw_tiles_of(L) * kEdgeBytes) +
           align256c(4 * L * L * sizeof(uint16_t)) + align256c(sw_tiles_of(L) * kBorderIdx * sizeof(uint32_t)) +
           align256c(sw_tiles_of(L) * 2 * sizeof(uint32_t));
}
// An exchange word that names no link (flat indices are at most 4N - 1 <= 2^32 - 2).
constexpr uint32_t kNoLink = 0xFFFFFFFFu;

// The allocation-free entry point keeps a whole Swendsen-Wang workspace for
// lattices up to kNoAllocMaxL in one fixed device array.
constexpr uint32_t kNoAllocMaxL = 512;
constexpr size_t kNoAllocBytes = kBaseBytes + sw_bytes_of(kNoAllocMaxL);

static_assert(sizeof(DevState) <= 256, "DevState");
static_assert(sizeof(DevTables) <= 768, "DevTables");
static_assert(sizeof(DevObs) <= 512, "DevObs");

// Arguments common to the lattice kernels (passed by value).
struct LatticeArgs {
    uint8_t* sigma;
    DevState* st;
    int64_t* slots;
    const DevTables* tab;
    uint32_t* label;         // Swendsen-Wang only
    uint8_t* mask;           // Swendsen-Wang only
    uint8_t* edge;           // Swendsen-Wang only: kEdgeBytes per tile
    uint16_t* lroot;         // Swendsen-Wang only: tile-local root of every bond index (| border flag)
    uint32_t* xchg;          // Swendsen-Wang only: kBorderIdx exchange words per tile
    uint32_t* ecnt;          // Swendsen-Wang only: arrival counters of each tile's right and bottom edge
    uint32_t L, N;           // side, L*L
    uint32_t key0, key1;     // Philox key (seed)
    uint32_t q;
    uint32_t met_lim;        // largest proposal word that is not NULL (q-1 states)
    uint32_t flip_lim;       // same for the q-state cluster shift
    int32_t jeff_sign;       // sign of J_eff = J - P v_HB
    double met_invd;         // 1 / floor(2^32/(q-1))
    double flip_invd;        // 1 / floor(2^32/q)
    uint32_t rows;           // Metropolis: rows per wavefront (even, <= 32)
    uint32_t row_blocks;     // Metropolis: grid.y
    uint32_t quad;           // Metropolis: 1 / 2 = dword (4-column) lanes, L % 4 == 0 / 2; 0 = column pairs
    uint32_t met_le;         // 1: no Metropolis threshold is 0, so acceptance is one compare (word <= thr - 1)
};

struct VolArgs {
    DevState* st;
    int64_t* slots;
    const DevTables* tab;
    double Nd, beta, J, P, vHB, dv_max;
    uint32_t key0, key1;
    int64_t met_att_add;     // Metropolis proposals per sweep (4N) or 0
    int32_t mode;            // 0: Metropolis step, 1: SW step, 2: fold only
    int32_t do_volume;
};

enum VolMode { kVolMet = 0, kVolSw = 1, kVolFold = 2 };

// One chain of a batch: its launch arguments and the work units of a
// batched Metropolis colour pass (row pair x column quad, or x column pair
// for L % 4 == 2), `iters` units per lane, `blocks` workgroups.
struct BatchEntry {
    LatticeArgs la;
    VolArgs va;
    uint32_t units;          // units per colour pass: (L / 2) * upr
    uint32_t upr;            // units per row pair: L / 4 quads, or L / 2 column pairs
    double upr_inv;          // 1 / upr
    uint32_t iters;          // units per lane
    uint32_t blocks;         // workgroups of this chain: ceil(units / (256 iters))
    // The chain's step as the batched volume kernel opened it (device-written
    // before every sweep's colour passes, which read it with the entry instead
    // of following la.st)
    int32_t skip;
    int32_t theta;
    uint32_t t_cur;
    uint32_t pad;
};

// Launchers (cvf_kernels.hip).  Each returns the launch status.
hipError_t launch_state_init(DevState* st, int64_t* slots, const DevTables* tab, double v_init, hipStream_t s);
hipError_t launch_set_stop(DevState* st, int64_t stop_at, hipStream_t s);
// The tables written by a kernel (argument by value) instead of a copy.
hipError_t launch_tables_init(DevTables* dst, const DevTables& src, hipStream_t s);
// Device address of the library's fixed scratch array on the current device
// (kNoAllocBytes bytes, 256-aligned), looked up once per device.
hipError_t noalloc_scratch(void** ptr);
hipError_t launch_sigma_init(const LatticeArgs& a, hipStream_t s);
hipError_t launch_volume(const VolArgs& a, hipStream_t s, DispatchEvents ev = {});
hipError_t launch_met_colour(const LatticeArgs& a, int colour, hipStream_t s, DispatchEvents ev = {});
// Arm-domain sweep: pass 0..3 of the step's drawn arm order (any L >= 2).
hipError_t launch_met_domain(const LatticeArgs& a, uint32_t pass, hipStream_t s, DispatchEvents ev = {});
// step_gate: the recount closes an SW step and is skipped with it.
hipError_t launch_recount(const LatticeArgs& a, int64_t* out, int spread, int with_counts, int step_gate,
                          hipStream_t s);
hipError_t launch_obs_zero(DevObs* o, hipStream_t s);
// N_q' of the current sigma added to out[0..5] (sigma 4-byte aligned).
hipError_t launch_state_counts(const LatticeArgs& a, int64_t* out, hipStream_t s);
hipError_t launch_obs_final(DevObs* o, const DevState* st, const DevTables* tab, double Nd, double J,
                            double Jsigma, double P, double vHB, hipStream_t s);
// Tiled SW step: bonds + in-tile unions + the tile-crossing links (each
// united by the later of its two tiles), then the cluster shift fused with
// the recount.  Labels are written out on request.
hipError_t launch_sw_tiles(const LatticeArgs& a, hipStream_t s, DispatchEvents ev = {});
// Zero the edge arrival counters (once, when the chain is created).
hipError_t launch_sw_counters_init(const LatticeArgs& a, hipStream_t s);
hipError_t launch_sw_flip_tiles(const LatticeArgs& a, hipStream_t s, DispatchEvents ev = {});
hipError_t launch_sw_labels(const LatticeArgs& a, uint32_t* out, hipStream_t s);
// Batched Metropolis: `ent` / `start` are device arrays (count entries,
// count+1 prefix sums of workgroups); all chains share q; le: every chain's
// table allows the one-compare acceptance.
hipError_t launch_met_batch(const BatchEntry* ent, const uint32_t* start, uint32_t count, uint32_t total_blocks,
                            int q, int colour, int le, hipStream_t s);
hipError_t launch_volume_batch(BatchEntry* ent, uint32_t count, int mode, hipStream_t s);
// Batched Swendsen-Wang stage: 0 tiles (bonds, in-tile unions and the
// tile-crossing links), 2 shift + recount; start: count+1 prefix sums of the
// per-chain tiles.
hipError_t launch_sw_batch(const BatchEntry* ent, const uint32_t* start, uint32_t count, uint32_t total_blocks,
                           int stage, hipStream_t s);

}  // namespace cvf
