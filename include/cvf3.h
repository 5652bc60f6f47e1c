/*
 * cvf3.h -- C ABI of the CVF water model on the periodic simple-cubic lattice
 * with the eta bond constraint (Coronas, Vilanova, Franzese, arXiv
 * 2505.05919: model Sec. II.A and Eq. (1)-(3), MC step Sec. II.B,
 * arm-domain Metropolis Sec. II.C, eta partition App. A).
 *
 * State on the device, owned by the caller:
 *   sigma  6N bytes, sigma[a*N + c] in {0..q-1}; arm a = 0:+x 1:-x 2:+y 3:-y
 *          4:+z 5:-z; cell c = x + L*(y + L*z), N = L^3 (the plane-major
 *          layout of Sec. II.C)
 *   eta    3N bytes, eta[d*N + c] in {0, 1} for the edge from c to its +d
 *          neighbour (d = 0:x 1:y 2:z); every edge is stored once
 *   work   cvf3_workspace_bytes() bytes: chain scalars, counter slots,
 *          tables
 * Both lattice buffers must be 4-byte aligned and the workspace 256-byte
 * aligned; all three must stay valid until cvf3_destroy.  Every call that
 * takes a stream enqueues its kernels there (NULL = the default stream).
 *
 * One MC step (cvf3_steps), in the paper's order:
 *   1. volume move of v_iso with sigma, eta fixed (Metropolis, FP64);
 *   2. eta move: the lattice's unit cubes with all-even or all-odd lowest
 *      corner ("checkerboard cubes") partition the edges; each cube proposes
 *      one of the nine perfect matchings of the cube graph as its eta = 0
 *      edges (so every molecule keeps four eta = 1 edges) and accepts it by
 *      Metropolis on dH = -J_eff dN_HB in the liquid (always in the gas);
 *   3. six arm-domain passes of sigma, one per arm in an order drawn for the
 *      step; a move changes one bond index to one of the q - 1 other states
 *      with dH = -theta eta J_eff dh - J_sigma dc (dc over the five other
 *      arms of the cell).
 * Random numbers: Philox4x32-10 keyed by the seed, one counter per draw, so
 * a chain's trajectory depends only on (params, seed) and the sequence of
 * calls, not on the launch; the step enters the counter as 32 bits, so a
 * chain runs at most 2^32 steps before its draws repeat.
 *
 * Conventions (as in cvf.h): every function returns CVF_OK or a negative
 * CVF_E* code, validation happens before any device call and leaves the
 * state unchanged; the library allocates no device memory; cvf3_init,
 * cvf3_observables and cvf3_kernel_times synchronise the stream, the other
 * calls are asynchronous on it; a cvf3_state is not thread-safe, distinct
 * states are independent and may run concurrently on different streams.
 */
#ifndef CVF3_H
#define CVF3_H

#include <stddef.h>
#include <stdint.h>

#include "cvf.h"

#ifdef __cplusplus
extern "C" {
#endif

#define CVF3_MAX_L 1290    /* N = L^3 < 2^31 */

typedef struct cvf3_obs {
    int64_t step;           /* MC steps done                                      */
    int64_t n_hb_raw;       /* edges with eta = 1 and equal facing sigma          */
    int64_t n_hb;           /* N_HB = theta * n_hb_raw                            */
    int64_t n_coop;         /* N_sigma: equal pairs among each cell's 15 arm pairs */
    int64_t count[6];       /* N_q', q' = 0..5                                    */
    int64_t n_eta0;         /* edges with eta = 0 (N in a valid state)            */
    int64_t met_attempted, met_accepted;
    int64_t eta_attempted, eta_accepted;
    int64_t vol_attempted, vol_accepted;
    double  v;              /* v_iso / v0                                         */
    double  V;              /* Eq. (1), units of v0                               */
    double  H;              /* Eq. (3), units of eps                              */
    double  M;              /* max_q' N_q' / (6N)                                 */
    int32_t consistent;     /* 1 if the incremental counters equal the recount    */
    int32_t reserved;
} cvf3_obs;

typedef struct cvf3_state cvf3_state;

/* Workspace size for params p (L even, 2..CVF3_MAX_L; q 2..6; the rest as
 * for cvf_init) and the algorithms the chain will run (algo_mask:
 * CVF_ALGO_METROPOLIS | CVF_ALGO_SW).  Metropolis needs a few KB; SW adds
 * 4N bytes of link masks and 24N bytes of labels and needs 6N < 2^32
 * (L <= 894).  CVF_EINVAL on invalid parameters, mask or a NULL bytes. */
int cvf3_workspace_bytes(const cvf_params *p, int algo_mask, size_t *bytes);

/* Host-only: the tables the kernels use -- met[th][dh+1][dc+5] (sigma move,
 * 32-bit acceptance thresholds, 2^32-1 = always), eta[dn+4] (eta move in the
 * liquid) and the nine perfect matchings of the cube graph as 12-bit edge
 * masks in ascending order (edge e: axis e/4, the other two coordinates in
 * bits 0 and 1 of e%4, lower axis first).  CVF_EINVAL on invalid p or NULL. */
int cvf3_tables(const cvf_params *p, uint32_t met[2][3][11], uint32_t eta[9], uint32_t match[9]);

/* Creates a chain: sets v_iso = v_init, draws sigma and eta from the seed
 * (or keeps the caller's when p->flags has CVF_KEEP_SIGMA; eta must then be
 * a valid state: every cube's eta = 0 edges a perfect matching), and counts
 * N_HB_raw and N_sigma.  Synchronises the stream.  Errors: CVF_EINVAL
 * (parameters, NULL or misaligned pointers), CVF_ENOMEM (work_bytes too
 * small or host allocation), CVF_EHIP. */
int cvf3_init(const cvf_params *p, int algo_mask, uint8_t *d_sigma, uint8_t *d_eta, void *d_work,
              size_t work_bytes, void *stream, cvf3_state **out);

/* nsteps MC steps (volume, eta, six sigma passes each).  CVF_EINVAL for a
 * NULL state or nsteps < 0, CVF_EHIP if a launch fails. */
int cvf3_steps(cvf3_state *st, int64_t nsteps, void *stream);

/* nsteps Swendsen-Wang steps (Sec. II.B order: volume move, eta move, then
 * one SW update of sigma, Sec. II.D): links per cell -- the 15 cooperative
 * pairs (equal arms, p = 1 - exp(-beta J_sigma)) and the three covalent
 * links of its +x, +y, +z edges (liquid and eta = 1 only; equal facing arms
 * for J_eff > 0, unequal for J_eff < 0, p = 1 - exp(-beta |J_eff|)) --
 * clusters of the 6N bond indices labelled by their smallest flat index,
 * one uniform shift per cluster from Philox(label, t, 0, SWF).  CVF_ESTATE
 * if the chain was created without CVF_ALGO_SW. */
int cvf3_sw_steps(cvf3_state *st, int64_t nsteps, void *stream);

/* Cluster labels of the last SW step (6N uint32, the smallest flat index of
 * each bond index's cluster) into d_out.  CVF_ESTATE before the first SW
 * step or without CVF_ALGO_SW. */
int cvf3_labels(cvf3_state *st, uint32_t *d_out, void *stream);

/* Adds N_q' (q' = 0..5) of the current sigma into d_counts[0..5] (device,
 * int64, 8-byte aligned; the caller zeroes it), without synchronising: one
 * call per step records the order parameter M(t) = max_q' N_q' / (6N) of
 * Sec. III.A on the device.  CVF_EINVAL for NULL or misaligned pointers. */
int cvf3_state_counts(cvf3_state *st, int64_t *d_counts, void *stream);

/* Observables of the current state from a full recount, with the chain's
 * counters; `consistent` compares the incrementally kept N_HB_raw, N_sigma
 * with the recount.  Synchronises the stream. */
int cvf3_observables(cvf3_state *st, cvf3_obs *out, void *stream);

/* Per-kernel HIP-event timing (off by default): enabling or disabling
 * clears the totals; times are collected when read.  Each launch records
 * its start/stop events on its own dispatch (the kernel's execution alone);
 * CVF3_K_SW_UNION and CVF3_K_SW_FLIP span their two and four launches with
 * events on the stream. */
#define CVF3_K_VOLUME 0     /* counter fold + volume move + pass order */
#define CVF3_K_ETA    1     /* eta move over the checkerboard cubes    */
#define CVF3_K_PASS   2     /* one arm-domain sigma pass               */
#define CVF3_K_SW_BONDS 3   /* SW link masks                           */
#define CVF3_K_SW_UNION 4   /* SW union-find over the links            */
#define CVF3_K_SW_FLIP  5   /* SW cluster shift + recount              */
#define CVF3_K_COUNT  6
int cvf3_timing_enable(cvf3_state *st, int enable);
int cvf3_kernel_times(cvf3_state *st, int kind, int64_t *launches, double *mean_ms);

/* Frees the host-side state (not the caller's buffers). */
int cvf3_destroy(cvf3_state *st);

#ifdef __cplusplus
}
#endif
#endif
