/*
 * cvf.h -- C ABI of libcvf: Monte Carlo hot path of the CVF water model on
 * AMD Instinct MI355X (gfx950).
 *
 * Model: Coronas, Vilanova, Franzese, "Efficient parallel algorithms for
 * free-energy calculation of millions of water molecules in the fluid
 * phases".  This library implements the model on a periodic L x L square
 * lattice (the monolayer form of the model: 4 nearest neighbours, 4 bond
 * indices per molecule, eta == 1):
 *
 *   state      {v_iso, sigma}            Sec. II.B (configuration)
 *   enthalpy   H = U_LJ - J N_HB - J_sigma N_sigma + P V,
 *              V = V_iso + v_HB N_HB     Eq. (1), Eq. (3), Table I
 *   MC step    volume move, then the sigma update: a checkerboard or an
 *              arm-domain Metropolis sweep, or a Swendsen-Wang step
 *                                        Sec. II.B-II.D
 *
 * Layout (part of the ABI).  sigma is caller-owned device memory of 4*L*L
 * bytes, plane-major as in Sec. II.C: sigma[a*N + c], N = L*L, cell
 * c = x + L*y, arm a = 0:+x, 1:-x, 2:+y, 3:-y.  Arm a of cell c faces arm
 * a^1 of the neighbour in direction a (periodic).  Values are 0..q-1.
 *
 * Randomness.  Philox4x32-10 keyed by the 64-bit seed, counter
 * (index, step, sub, stream): a run is a pure function of (params, seed)
 * and of the sequence of calls, independent of launch shape and of other
 * jobs on the device.
 *
 * Conventions.
 *  - Every function returns CVF_OK (0) or a negative CVF_E* code; nothing
 *    aborts or throws across the ABI.  Validation failures leave the state
 *    unchanged.  After CVF_EHIP the device state is undefined.
 *  - Ownership: the caller allocates and frees all device memory (sigma and
 *    the workspace); both must stay valid until cvf_destroy.  The library
 *    allocates no device memory.  Host state is owned by the library and
 *    freed by cvf_destroy.
 *  - stream: a hipStream_t passed as void* (NULL = the null stream).  All
 *    calls are asynchronous on that stream except cvf_observables,
 *    cvf_labels, cvf_kernel_times, cvf_batch_create, cvf_batch_set_rows and
 *    cvf_batch_autotune, which synchronise it.  cvf_init writes its tables
 *    with a kernel (no host copy), so it never waits for earlier work on
 *    its stream.
 *  - Threading: a cvf_state is not thread-safe; distinct states are
 *    independent and may run concurrently on different streams.
 */
#ifndef CVF_H
#define CVF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define CVF_OK       0
#define CVF_EINVAL  (-1)   /* invalid argument or parameter            */
#define CVF_ENOMEM  (-2)   /* workspace smaller than required          */
#define CVF_EHIP    (-3)   /* a HIP runtime call or launch failed      */
#define CVF_ESTATE  (-4)   /* call not valid in the current state      */

/* algorithm masks (cvf_workspace_bytes) */
#define CVF_ALGO_METROPOLIS 1
#define CVF_ALGO_SW         2

/* cvf_params.flags */
#define CVF_NO_VOLUME_MOVE  1u  /* skip the volume move of every step        */
#define CVF_KEEP_SIGMA      2u  /* cvf_init keeps the caller's sigma          */

/* Reduced units: energies in eps = 5.5 kJ/mol, volumes in v0 = r0^3
 * (Table I).  beta = eps/(k_B T N_A); P is P r0^3 N_A / eps. */
typedef struct cvf_params {
    int32_t  L;        /* lattice side, 2 <= L <= 32766; odd L only for
                          the arm-domain sweep (see below)                */
    int32_t  q;        /* states per bond index, 2..6 (paper: q = 6)     */
    double   beta;     /* inverse reduced temperature, >= 0, finite      */
    double   J;        /* covalent HB energy (Table I: 2.0)              */
    double   Jsigma;   /* cooperative energy (Table I: 0.32), >= 0       */
    double   P;        /* reduced pressure                               */
    double   vHB;      /* volume per HB (Table I: 0.6)                   */
    double   v_init;   /* initial v_iso/v0 per molecule, >= 1            */
    double   dv_max;   /* half-width of the volume proposal, >= 0        */
    uint64_t seed;     /* Philox key                                     */
    uint32_t flags;    /* CVF_NO_VOLUME_MOVE | CVF_KEEP_SIGMA            */
    uint32_t reserved; /* must be 0                                      */
} cvf_params;

/* Observables (Eq. (1), Eq. (3), Eq. (4)'s order parameter). */
typedef struct cvf_obs {
    int64_t step;           /* MC steps done                                   */
    int64_t n_hb_raw;       /* facing pairs with equal sigma                    */
    int64_t n_hb;           /* N_HB = theta * n_hb_raw (theta = [v < 2])        */
    int64_t n_coop;         /* N_sigma: equal same-cell arm pairs               */
    int64_t count[6];       /* N_q': sigma values in state q' (0 past q-1)      */
    int64_t met_attempted;  /* Metropolis proposals                             */
    int64_t met_accepted;
    int64_t vol_attempted;  /* volume moves                                     */
    int64_t vol_accepted;
    double  v;              /* v_iso / v0                                       */
    double  V;              /* N v + v_HB N_HB, units of v0                     */
    double  H;              /* N u_LJ(v) - J N_HB - J_sigma N_sigma + P V       */
    double  M;              /* max_q' N_q' / (4N)                               */
    int32_t consistent;     /* 1 if the incremental counters equal a recount    */
    int32_t reserved;
} cvf_obs;

typedef struct cvf_state cvf_state;

/* Table I parameters at temperature T (K) and pressure P (MPa) in reduced
 * units (SI-2019 N_A, k_B); L = 64, q = 6, v_init = 1.25, dv_max = 0.0125,
 * seed = 1, flags = 0.  Host only.  CVF_EINVAL if out is NULL or T <= 0. */
int cvf_params_from_si(double T_kelvin, double P_MPa, cvf_params *out);

/* Device workspace needed for the algorithms in algo_mask.  Metropolis
 * (Sec. II.C) needs a few KB: the chain's scalars, counter slots and the
 * acceptance table.  Swendsen-Wang (Sec. II.D) adds the state of its
 * labelling -- the paper's bond array and label array of every bond index
 * -- as 25 bytes per cell (uint32 labels and uint16 tile-local roots of the
 * 4N bond indices, one bond mask byte per cell) and 728 bytes per 64 x
 * 16-cell tile (edge bytes, the words two tiles exchange for the links
 * between them, arrival counters).  Host only.  CVF_EINVAL for a NULL
 * argument, invalid parameters or an empty algo_mask. */
int cvf_workspace_bytes(const cvf_params *p, int algo_mask, size_t *bytes);

/* Create a chain.  d_sigma: 4*L*L bytes of device memory (4-byte aligned:
 * the sweeps move dwords), layout above;
 * filled from Philox stream INIT (sigma[a][c] = floor(w_a q / 2^32) of the
 * block at counter (c, 0, 0, INIT)) unless CVF_KEEP_SIGMA.  d_work /
 * work_bytes: caller-owned device workspace (256-byte aligned), at least
 * cvf_workspace_bytes(p, CVF_ALGO_METROPOLIS); Swendsen-Wang steps need the
 * larger size.  v = v_init, step = 0, counters from a full count.  *out
 * receives the new state.  Asynchronous on stream. */
int cvf_init(const cvf_params *p, uint8_t *d_sigma, void *d_work, size_t work_bytes,
             void *stream, cvf_state **out);

/* nsweeps MC steps, each a volume move (Sec. II.B step 1) followed by one
 * checkerboard Metropolis sweep over every bond index (Sec. II.C): colour 0
 * cells ((x+y) even) then colour 1, arms 0..3 in order inside a cell, each
 * proposing a uniformly chosen different state and accepting it with
 * min(1, exp(-beta dH)) through a 2^32-scaled table.  Asynchronous.
 * nsweeps >= 0; CVF_EINVAL for odd L (the checkerboard needs even L). */
int cvf_metropolis_sweeps(cvf_state *st, int64_t nsweeps, void *stream);

/* nsweeps MC steps, each a volume move followed by one arm-domain Metropolis
 * sweep: the paper's own layered partition (Sec. II.C and its figure of the
 * domains), in 2-D.  Arm a of every cell is a domain whose bond indices
 * interact only with other domains, so a pass moves all of them at once;
 * a sweep is four passes, one per arm, in an order drawn per step (a
 * uniform permutation, Fisher-Yates on Philox(0, t, 0, ORD)).  The move of
 * arm a of cell (x, y) takes proposal and acceptance words 0, 1 (even x) or
 * 2, 3 (odd x) of Philox(floor(x/2) + ceil(L/2) y, t, a, DOM), and accepts
 * through the same table as cvf_metropolis_sweeps.  A different trajectory
 * from the checkerboard sweep with the same stationary distribution; any L,
 * odd included.  Asynchronous.  nsweeps >= 0. */
int cvf_metropolis_domain_sweeps(cvf_state *st, int64_t nsweeps, void *stream);

/* nsteps MC steps, each a volume move followed by one Swendsen-Wang step
 * (Sec. II.D): bond activation, connected-component labelling to the
 * minimum flat index of every cluster (the result Table II converges to),
 * and a cluster-wide shift sigma <- (sigma + r) mod q with r drawn per
 * cluster.  Needs the Swendsen-Wang workspace (CVF_ENOMEM otherwise),
 * J_sigma >= 0 and even L (CVF_EINVAL otherwise).  Asynchronous. */
int cvf_sw_steps(cvf_state *st, int64_t nsteps, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): a fresh
 * chain (as cvf_init with these parameters over d_sigma), nsteps
 * Swendsen-Wang MC steps (as cvf_sw_steps), and its observables in *out (as
 * cvf_observables) -- the same results as that sequence, bit for bit.  No
 * caller workspace: the chain's scalars, counter slots, tables, labels, bond
 * masks and tile roots live in a fixed device array inside the library
 * (about 6.4 MiB on every GPU it runs on, held until the process ends), so
 * L <= 512; CVF_ENOMEM for a larger L.  The call allocates nothing (no
 * hipMalloc/hipFree, no host allocation).  d_sigma: 4*L*L bytes of device
 * memory, 4-byte aligned, filled from Philox stream INIT unless
 * CVF_KEEP_SIGMA.  CVF_EINVAL for invalid parameters, odd L, J_sigma < 0,
 * nsteps < 0 or a NULL pointer (all checked before any device call).  Every
 * call on one GPU uses that GPU's one array, which keeps the last call's
 * contents (each call re-initialises what it reads): calls that overlap on
 * one device, on any streams or threads, race and must not be issued.
 * Synchronises stream. */
int cvf_sw_steps_noalloc(const cvf_params *p, uint8_t *d_sigma, int64_t nsteps, cvf_obs *out, void *stream);

/* Recount the lattice, evaluate Eq. (1) and (3), and copy everything to
 * *out.  Synchronises stream. */
int cvf_observables(cvf_state *st, cvf_obs *out, void *stream);

/* The same record (Eq. (1), (3), the counts of Sec. III.A) without
 * synchronising: it is written to out -- device memory, or pinned host
 * memory such as hipHostMalloc gives, 8-byte aligned -- when the stream
 * reaches this call's work, so that a caller (a server retiring finished
 * jobs while later ones run) never waits for earlier work on the stream.
 * CVF_EINVAL for a NULL state or a NULL or misaligned out. */
int cvf_observables_async(cvf_state *st, cvf_obs *out, void *stream);

/* Add the state counts N_q' of the current configuration (the number of
 * bond indices in state q', q' = 0..5, from which Sec. III.A builds the
 * order parameter M = max N_q' over the number of bond indices, 4N in 2-D,
 * and its autocorrelation C_M) to the six int64 at d_counts (device
 * memory, 8-byte aligned, zeroed by the caller beforehand: the kernel
 * accumulates).  No host synchronisation, so a caller can record one row
 * per step of a long run and read the series once.  Asynchronous. */
int cvf_state_counts(cvf_state *st, int64_t *d_counts, void *stream);

/* Write the cluster labels of the last Swendsen-Wang step (Sec. II.D: the
 * label array of every bond index, converged to the smallest flat index of
 * its cluster, the fixed point of the worked example in Table II; 4*L*L
 * uint32, label[idx] = smallest flat index in idx's cluster) to device memory
 * d_out, which must not overlap the chain's workspace or sigma.
 * CVF_ESTATE if no Swendsen-Wang step has run.  Waits for the stream's
 * earlier work (to read that flag), then enqueues the write. */
int cvf_labels(cvf_state *st, uint32_t *d_out, void *stream);

/* Step limit: steps with index >= stop_at (counted from 0 at cvf_init) are
 * not performed -- later calls, single or batched, leave the chain as it is
 * (sigma, v, counters).  Default: no limit.  Lets a batch run fixed-length
 * quanta while every chain stops exactly at its own step count.  stop_at >= 0.
 * Asynchronous. */
int cvf_set_stop(cvf_state *st, int64_t stop_at, void *stream);

/* Test hook: the host-computed acceptance tables of this chain.  They
 * encode the Metropolis acceptance min(1, exp(-beta dH)) of Sec. II.C with
 * dH from Eq. (3) (dH = -theta J_eff dN_HB - J_sigma dN_sigma, J_eff =
 * J - P v_HB), and the Swendsen-Wang bond probabilities 1 - exp(-beta J_sigma)
 * and 1 - exp(-beta |J_eff|) of Sec. II.D, scaled by 2^32.
 * met[theta][dh+1][dc+3]: accept iff thr == 0xFFFFFFFF or word < thr.
 * sw[0] cooperative bond threshold, sw[1], sw[2] covalent thresholds for
 * theta = 0, 1 (bond iff word < thr, 64-bit compare).  Host only;
 * CVF_EINVAL for a NULL argument. */
int cvf_tables(const cvf_state *st, uint32_t met[2][3][7], uint64_t sw[3]);

/* Kernel timing.  While enabled, every launch of the kernels of one kind
 * carries a start/stop pair of HIP events that its own dispatch records
 * (hipExtLaunchKernel), so each interval is that kernel's execution alone.
 * cvf_kernel_times synchronises those events and returns, for kind k, the
 * number of launches and their mean duration in ms since timing was
 * enabled. */
#define CVF_K_VOLUME    0   /* volume move / counter fold          */
#define CVF_K_MET_SWEEP 1   /* one checkerboard colour sweep       */
#define CVF_K_SW_BONDS  2   /* bond activation + in-tile labels
                               + the tile-crossing unions          */
#define CVF_K_SW_UNION  3   /* not launched: the tile-crossing
                               unions run in the CVF_K_SW_BONDS
                               launch (value kept for the ABI)     */
#define CVF_K_SW_FLIP   4   /* cluster shift + recount             */
#define CVF_K_RECOUNT   5   /* lattice recount (separate launches) */
#define CVF_K_MET_DOMAIN 6  /* one arm-domain pass                 */
#define CVF_K_COUNT     7
int cvf_timing_enable(cvf_state *st, int enable);
int cvf_kernel_times(cvf_state *st, int kind, int64_t *launches, double *mean_ms);

/* Release the host state (device memory stays with the caller). */
int cvf_destroy(cvf_state *st);

/* ---------------------------------------------------------------------------
 * Batched execution: many independent chains advanced together, one launch
 * per colour phase for all of them (plus one volume launch with a wavefront
 * per chain).  Every chain computes exactly what cvf_metropolis_sweeps
 * computes for it alone (same Philox keying, same update order), so results
 * are identical alone and in the batch.
 * ------------------------------------------------------------------------- */
typedef struct cvf_batch cvf_batch;

/* Device bytes for the descriptor table of `count` chains. */
int cvf_batch_desc_bytes(int32_t count, size_t *bytes);

/* Group `count` existing chains (created by cvf_init, all with the same q
 * and even L -- CVF_EINVAL otherwise; each keeps its own sigma and
 * workspace).  d_desc: caller-owned device memory of
 * cvf_batch_desc_bytes(count) bytes, 256-byte aligned.  The chains must
 * outlive the batch; the batch holds no device memory of its own besides a
 * private capture stream for graphs.  Uploads the descriptor table on stream
 * and waits for the copy. */
int cvf_batch_create(cvf_state *const *chains, int32_t count, void *d_desc, size_t desc_bytes,
                     void *stream, cvf_batch **out);

/* As cvf_batch_create, without waiting for the upload: the descriptor table
 * is written into h_staging -- caller-owned pinned host memory (such as
 * hipHostMalloc gives) of staging_bytes >= desc_bytes -- and copied on
 * stream; h_staging must stay unchanged until the stream has passed this
 * call.  For callers that rebuild batches while earlier work runs on the
 * stream.  CVF_EINVAL also for a NULL or small staging buffer. */
int cvf_batch_create_async(cvf_state *const *chains, int32_t count, void *d_desc, size_t desc_bytes,
                           void *h_staging, size_t staging_bytes, void *stream, cvf_batch **out);

/* Launch shape of the batched Metropolis pass: a chain's colour pass is cut
 * into work units of two rows times a column quad (L % 4 == 0) or a column
 * pair (L % 4 == 2), numbered row-pair major; a quad lane moves `rows` / 2
 * consecutive-by-64 units, i.e. `rows` rows (even, 2..32), and a column-pair
 * lane `rows` units, the same 8 `rows` updates; 0 restores the default (4).
 * Invalidates captured graphs.  Re-uploads the descriptor table on stream
 * and waits for the copy. */
int cvf_batch_set_rows(cvf_batch *b, int32_t rows, void *stream);

/* nsweeps Metropolis MC steps of every chain.  graph_block > 0: the sweeps
 * run as replays of one hipGraph holding graph_block sweeps (captured once,
 * on first use), the remainder as plain launches; 0: plain launches.
 * Asynchronous. */
int cvf_batch_metropolis_sweeps(cvf_batch *b, int64_t nsweeps, int32_t graph_block, void *stream);

/* nsteps Swendsen-Wang MC steps of every chain (each chain as in
 * cvf_sw_steps), one launch per stage for all chains.  CVF_ENOMEM unless
 * every chain has the Swendsen-Wang workspace.  Asynchronous. */
int cvf_batch_sw_steps(cvf_batch *b, int64_t nsteps, void *stream);

/* Autotuner: after one untimed block of `sweeps` sweeps, times `sweeps`
 * sweeps for each candidate rows value (2, 4, 8, 16, 32) with HIP events,
 * in two rounds, and keeps the candidate with the fastest of its two times;
 * *rows_out receives it.  The sweeps are real: every chain advances by
 * 11 * sweeps steps.  Synchronises stream. */
int cvf_batch_autotune(cvf_batch *b, int32_t sweeps, void *stream, int32_t *rows_out);

/* Release the batch's host state, its captured graph and capture stream;
 * the chains and d_desc stay with the caller. */
int cvf_batch_destroy(cvf_batch *b);

/* Static description of an error code. */
const char *cvf_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* CVF_H */
