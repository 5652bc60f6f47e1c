#!/usr/bin/env python3
"""Benchmark of the CVF Monte Carlo hot path on one MI355X.

Headline (the paper-scale Metropolis job): bond-variable updates per ns of
checkerboard Metropolis sweeps (each with its volume move) on an L = 4096
lattice (16.8 M molecules, 67.1 M uint8 bond indices) at 300 K and
P in {0.1, 25, 50} MPa, one chain per pressure, lattices resident in HBM.
Also reported: Swendsen-Wang steps/s on L = 1414 (~2 M molecules) at the
same state points, the roofline of the dominant kernel, and the CPU oracle
timed on a bounded sample of the same workload.

One JSON line on stdout; progress on stderr.
"""
from __future__ import annotations

import argparse
import hashlib

import numpy as np
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# full-rate 32-bit VALU issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (lane-ops/s)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic integer ops per bond update: half a Philox4x32-10 block (10 rounds x
# (2 single-instruction 32x32->64 products + 2 three-input XORs) / 2 = 20) + the
# decision (14)
ALU_OPS_PER_UPDATE = 34
COUNTERS_FILE = os.path.join(ROOT, "profiles", "met_colour_L4096_counters.json")
KERNEL_SRCS = [os.path.join(ROOT, "paper_2505_05919_amd", "csrc", f) for f in ("philox.h", "met_sweep.h", "met_launch.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the sources the Metropolis colour kernel is built from."""
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_counters(launch_ms_unused=None):
    """HBM bytes per colour launch from committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs, scaled by the same counters' reading of a plain copy of
    known size; None when absent or taken on another kernel version."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    with open(COUNTERS_FILE) as f:
        c = json.load(f)
    if c.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    fetch = c["fetch_kib_per_dispatch"] * 1024.0 * c["fetch_scale"]
    write = c["write_kib_per_dispatch"] * 1024.0 * c["write_scale"]
    return fetch + write


def make_chain(cvf, L, T, P, seed, algo_mask):
    p = cvf.cvf_params_from_si(T, P, L=L, seed=seed)
    return cvf.Chain(p, algo_mask)


def timed(torch, fn, K):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        fn(i)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def instrumented(cvf, chains, fn, K, kinds):
    for ch in chains:
        cvf.cvf_timing_enable(ch.h, True)
    for i in range(K):
        fn(i)
    out = {}
    for k in kinds:
        n_tot, ms_tot = 0, 0.0
        for ch in chains:
            n, ms = cvf.cvf_kernel_times(ch.h, k)
            n_tot += n
            ms_tot += n * ms
        out[k] = (n_tot, ms_tot / n_tot if n_tot else 0.0)
    for ch in chains:
        cvf.cvf_timing_enable(ch.h, False)
    return out


def bench_autocorr(torch, cvf, L=256, points=((270.0, 7), (300.0, 9))):
    """Sec. III.A / III.C at the C2 SW lattice size: tau of the order
    parameter and the cost of one independent configuration for checkerboard
    Metropolis and SW (autocorr.measure: warm-up, M(t) recorded on the device
    after every step, C_M, tau = the 1/e lag, steps timed without
    recording)."""
    from paper_2505_05919_amd import autocorr
    warm = {"met": 20000, "sw": 2000}
    n_rec = {"met": 50000, "sw": 5000}
    out = {"L": L, "P_MPa": 0.1, "max_lag": 2000, "points": []}
    for T, seed in points:
        pt = {"T_K": T}
        for algo in ("met", "sw"):
            r = autocorr.measure(cvf, torch, L, T, 0.1, seed, algo, warm[algo], n_rec[algo])
            assert r.pop("consistent")
            pt[algo] = r
        cm, cs = pt["met"]["cost_per_independent_us"], pt["sw"]["cost_per_independent_us"]
        pt["cheaper"] = None if cs is None else ("sw" if cm is None or cs < cm else "met")
        out["points"].append(pt)
    return out


ALU_OPS_3D = 39      # half a Philox block (20) + decision over five other arms (18) + eta gate (1)
BYTES_3D = 9         # six own bond indices + facing one + the edge's eta read, one written


def bench_cvf3(torch, W, K, L=260, with_autocorr=True):
    """The paper's own model and size: cubic lattice with eta, N = 260^3, one
    step = volume move + eta moves + six arm-domain passes (Sec. II.B-C)."""
    from paper_2505_05919_amd import cvf, cvf3
    p = cvf.cvf_params_from_si(300.0, 0.1, L=L, seed=2026)
    ch = cvf3.Chain3(p)
    N = L ** 3
    ch.steps(W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch.steps(K)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    cvf3.cvf3_timing_enable(ch.h, True)
    ch.steps(K)
    kt = {k: cvf3.cvf3_kernel_times(ch.h, k) for k in (cvf3.CVF3_K_VOLUME, cvf3.CVF3_K_ETA, cvf3.CVF3_K_PASS)}
    cvf3.cvf3_timing_enable(ch.h, False)
    o = ch.obs()
    assert o["consistent"] == 1 and o["n_eta0"] == N
    ch.close()
    pass_s = kt[cvf3.CVF3_K_PASS][1] * 1e-3
    gbs = N * BYTES_3D / pass_s / 1e9
    tops = N * ALU_OPS_3D / pass_s / 1e12
    return {"L": L, "N": N, "steps": K, "ms_per_step": round(t / K * 1e3, 4),
            "updates_per_ns": round(6 * N * K / t / 1e9, 2),
            "kernel_mean_us": {"volume": round(kt[cvf3.CVF3_K_VOLUME][1] * 1e3, 2),
                               "eta": round(kt[cvf3.CVF3_K_ETA][1] * 1e3, 2),
                               "pass": round(kt[cvf3.CVF3_K_PASS][1] * 1e3, 2)},
            "pass_roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(gbs / HBM_PEAK_GBS, 4), "alg_bytes_per_update": BYTES_3D,
                              "alu": {"achieved": round(tops, 2), "peak": round(VALU_PEAK_TOPS, 2),
                                      "frac": round(tops / VALU_PEAK_TOPS, 4), "ops_per_update": ALU_OPS_3D}},
            "paper_rtx3060_ms_per_step": 280.0,
            "sw": bench_cvf3_sw(torch, W, max(K // 2, 10)),
            "autocorr": bench_cvf3_autocorr(torch) if with_autocorr else None}


def bench_cvf3_autocorr(torch, L=32):
    """Sec. III.A / III.C in the paper's own model and size (N = 32^3 =
    32 768): tau of the order parameter and the cost of an independent
    configuration for the arm-domain Metropolis and for Swendsen-Wang at the
    three state points of its Metropolis/SW comparison."""
    from paper_2505_05919_amd import autocorr, cvf, cvf3
    pts = []
    for T, P in ((205.0, -300.0), (205.0, 0.1), (195.0, 160.0)):
        met = autocorr.measure3(cvf, cvf3, torch, L, T, P, 31, "met", warm=5000, n_rec=20000)
        sw = autocorr.measure3(cvf, cvf3, torch, L, T, P, 31, "sw", warm=1000, n_rec=4000)
        cheaper = None
        if met["cost_per_independent_us"] and sw["cost_per_independent_us"]:
            cheaper = "sw" if sw["cost_per_independent_us"] < met["cost_per_independent_us"] else "met"
        elif sw["cost_per_independent_us"]:
            cheaper = "sw"
        pts.append({"T_K": T, "P_MPa": P, "met": met, "sw": sw, "cheaper": cheaper})
    return {"L": L, "N": L ** 3, "max_lag": 2000, "points": pts}


def bench_cvf3_sw(torch, W, K, L=128):
    """Swendsen-Wang on the cubic lattice with eta at the paper's SW size,
    N = 128^3 = 2 097 152 (volume move + eta moves + SW update per step)."""
    from paper_2505_05919_amd import cvf, cvf3
    p = cvf.cvf_params_from_si(210.0, 0.1, L=L, seed=2048)
    ch = cvf3.Chain3(p, algo_mask=cvf.CVF_ALGO_SW)
    ch.sw(W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch.sw(K)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    cvf3.cvf3_timing_enable(ch.h, True)
    ch.sw(K)
    kinds = {"volume": cvf3.CVF3_K_VOLUME, "eta": cvf3.CVF3_K_ETA, "bonds": cvf3.CVF3_K_SW_BONDS,
             "union": cvf3.CVF3_K_SW_UNION, "flip_recount": cvf3.CVF3_K_SW_FLIP}
    kt = {nm: round(cvf3.cvf3_kernel_times(ch.h, k)[1] * 1e3, 2) for nm, k in kinds.items()}
    cvf3.cvf3_timing_enable(ch.h, False)
    o = ch.obs()
    assert o["consistent"] == 1 and o["n_eta0"] == L ** 3
    ch.close()
    return {"L": L, "N": L ** 3, "T_K": 210.0, "steps": K, "steps_per_s": round(K / t, 1),
            "ms_per_step": round(t / K * 1e3, 4), "kernel_mean_us": kt,
            "paper_rtx3060_steps_per_s_fit_bound": 13.1}


def cpu_baseline(budget_s: float):
    """The oracle as it stands (single thread), Metropolis on the headline
    lattice, sweeps until the budget is used."""
    import oracle
    oracle.build(force=False)
    op = oracle.params_from_si(300.0, 0.1, L=4096, seed=12)
    ch = oracle.Chain(op)
    n, t = 0, 0.0
    while t < budget_s and n < 16:
        t0 = time.perf_counter()
        ch.metropolis(1)
        t += time.perf_counter() - t0
        n += 1
    N = 4096 * 4096
    return {"value": 4 * N * n / (t * 1e9), "unit": "bond-variable updates/ns", "cores": 1, "kind": "oracle",
            "sample": f"oracle Metropolis L=4096 T=300K P=0.1MPa seed 12, {n} sweeps after init "
                      f"({4 * N * n} updates, {t:.1f} s, one thread)"}


def bench_batched(torch, cvf, sweeps, alone_sweeps):
    """256 independent replicas of uneven L (log-uniform 64..512) on a 16x16
    (T, P) grid: one batched launch per colour phase, 100-sweep blocks replayed
    from a hipGraph, launch shape from the autotuner -- against the same jobs
    run one at a time with plain launches; per-replica sigma digests must be
    identical at equal sweep counts."""
    import hashlib
    from paper_2505_05919_amd.workloads import c4_jobs
    jobs = c4_jobs()

    def chains():
        return [make_chain(cvf, j.L, j.T, j.P, j.seed, cvf.CVF_ALGO_METROPOLIS) for j in jobs]

    def digests(chs):
        return [hashlib.sha256(c.sigma.cpu().numpy().tobytes()).hexdigest() for c in chs]

    upd_per_sweep = sum(4 * j.L * j.L for j in jobs)
    tune = chains()
    b = cvf.Batch(tune)
    rows = b.autotune(3)
    b.close()
    for c in tune:
        c.close()
    chs = chains()
    b = cvf.Batch(chs)
    b.set_rows(rows)
    block = 100 if sweeps % 100 == 0 else 0
    b.metropolis(block if block else 1, graph_block=block)      # capture + warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.metropolis(sweeps, graph_block=block)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    b.close()
    # identity check at alone_sweeps: fresh batch vs fresh single chains
    chk = chains()
    bb = cvf.Batch(chk)
    bb.set_rows(rows)
    bb.metropolis(alone_sweeps, graph_block=0)
    d_batch = digests(chk)
    bb.close()
    for c in chk:
        c.close()
    alone = chains()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in alone:
        c.metropolis(alone_sweeps)
    torch.cuda.synchronize()
    t_alone = time.perf_counter() - t0
    d_alone = digests(alone)
    for c in alone + chs:
        c.close()
    v_batch = upd_per_sweep * sweeps / t_batch / 1e9
    v_alone = upd_per_sweep * alone_sweeps / t_alone / 1e9
    return {"replicas": len(jobs), "sweeps": sweeps, "graph_block": block, "rows": rows,
            "updates_per_ns": round(v_batch, 1), "ms": round(t_batch * 1e3, 2),
            "one_at_a_time_updates_per_ns": round(v_alone, 2), "speedup": round(v_batch / v_alone, 1),
            "identical_digests": d_batch == d_alone, "digests_compared_at_sweeps": alone_sweeps}


def bench_served(torch, n_jobs):
    """The served stream: Poisson arrivals at 200 jobs/s, L log-uniform 32..2048,
    T ~ U(270, 330) K, P ~ U(0, 50) MPa, nsteps ~ U[100, 10^4], 80 % Metropolis /
    20 % SW, admitted by HBM footprint, lattices resident; p50/p99 latency next
    to throughput, against a one-job-at-a-time FCFS server with plain launches
    on the same trace (service times measured job by job).  Quanta advance the
    jobs with the least remaining work first (until they hold 2^24 cells); the
    same trace under processor sharing (every resident job in every quantum)
    is reported beside it."""
    from paper_2505_05919_amd import serve
    from paper_2505_05919_amd.workloads import c5_stream
    jobs = c5_stream(n_jobs=n_jobs)
    ps = serve.Server(memory_budget=32 << 30, max_slots=512, quantum=100, keep_digest=True, schedule="all")
    s_ps = serve.summarize(ps.run(jobs, realtime=True))
    srv = serve.Server(memory_budget=32 << 30, max_slots=512, quantum=100, keep_digest=True, schedule="srpt",
                       fill_cells=1 << 24)
    recs = srv.run(jobs, realtime=True)
    s = serve.summarize(recs)
    ps_digest = {r.job.seed: r.digest for r in ps.records}
    by_seed = {r.job.seed: r for r in recs}
    service, same = [], True
    for j in jobs:
        o, dg, dt = serve.run_alone(j)
        service.append(dt)
        r = by_seed[j.seed]
        same = same and r.digest == dg and r.obs == o and ps_digest[j.seed] == dg
    lat = serve.fcfs_latencies(jobs, service)
    span_alone = max(max(j.arrival for j in jobs), 0.0)
    done = 0.0
    for j, t in zip(jobs, service):
        done = max(done, j.arrival) + t
    upd = sum(4 * j.L ** 2 * j.nsteps for j in jobs if j.algo == "met")
    offered = upd / max(j.arrival for j in jobs) / 1e9
    return {"jobs": n_jobs, "rate_per_s": 200.0, "quantum": srv.quantum,
            "schedule": "least remaining work first, >= 2^24 cells per quantum",
            "processor_sharing": {"p50_ms": round(s_ps["p50_s"] * 1e3, 1), "p99_ms": round(s_ps["p99_s"] * 1e3, 1),
                                  "makespan_s": round(s_ps["makespan_s"], 3)},
            "p50_ms": round(s["p50_s"] * 1e3, 1), "p99_ms": round(s["p99_s"] * 1e3, 1),
            "queue_p50_ms": round(s["queue_p50_s"] * 1e3, 1), "queue_p99_ms": round(s["queue_p99_s"] * 1e3, 1),
            "makespan_s": round(s["makespan_s"], 3), "met_updates_per_ns": round(s["met_updates_per_ns"], 1),
            "offered_met_updates_per_ns": round(offered, 1),
            "peak_resident_jobs": srv.peak_resident_jobs, "peak_resident_MB": round(srv.peak_resident_bytes / 2**20, 1),
            "quanta": srv.quanta, "loop_phase_s": {k: round(v, 3) for k, v in srv.phase_s.items()},
            "one_at_a_time": {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 1),
                              "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 1),
                              "makespan_s": round(done - min(j.arrival for j in jobs), 3),
                              "met_updates_per_ns": round(upd / (done - min(j.arrival for j in jobs)) / 1e9, 1)},
            "identical_to_alone": same}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--warmup", type=int, default=100,
                    help="untimed steps per chain first: the GPU needs some tens of ms of load to reach its steady clock")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain device copy of 1 GiB (counter calibration)")
    ap.add_argument("--skip-sw", action="store_true")
    ap.add_argument("--skip-domain", action="store_true")
    ap.add_argument("--skip-autocorr", action="store_true")
    ap.add_argument("--skip-batch", action="store_true")
    ap.add_argument("--skip-cvf3", action="store_true")
    ap.add_argument("--skip-concurrent", action="store_true",
                    help="skip the three-stream Metropolis leg (profiled runs: it overlaps launches)")
    ap.add_argument("--cvf3-steps", type=int, default=200)
    ap.add_argument("--batch-sweeps", type=int, default=1000)
    ap.add_argument("--serve-jobs", type=int, default=120,
                    help="jobs of the served Poisson stream (0 = skip)")
    ap.add_argument("--alone-sweeps", type=int, default=100,
                    help="sweeps per replica for the one-at-a-time comparison (digests compared at this count)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}): "
              "this build has no multi-GPU path; the workloads are single-lattice or independent jobs.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2505_05919_amd import cvf
    from paper_2505_05919_amd.workloads import c3_jobs
    cvf.lib()
    torch.cuda.set_device(0)
    K, W = args.steps, args.warmup

    jobs = c3_jobs()
    met_jobs = [j for j in jobs if j.algo == "met"]
    sw_jobs = [j for j in jobs if j.algo == "sw"]

    # ---------------- Metropolis L = 4096 (headline) ----------------
    log(f"metropolis: {len(met_jobs)} chains L={met_jobs[0].L}, warmup {W}, steps {K}")
    mch = [make_chain(cvf, j.L, j.T, j.P, j.seed, cvf.CVF_ALGO_METROPOLIS) for j in met_jobs]
    N = met_jobs[0].L ** 2

    def met_step(i):
        mch[i % len(mch)].metropolis(1)

    for i in range(W * len(mch)):
        met_step(i)
    t_met = timed(torch, met_step, K)
    ms_per_step = t_met / K * 1e3
    value = 4 * N * K / (t_met * 1e9)
    log(f"metropolis: {ms_per_step:.4f} ms/sweep, {value:.1f} updates/ns")
    ktimes = instrumented(cvf, mch, met_step, K, [cvf.CVF_K_MET_SWEEP, cvf.CVF_K_VOLUME])
    n_launch, mean_ms = ktimes[cvf.CVF_K_MET_SWEEP]
    upd_per_launch = 2 * N                      # one colour: N/2 cells x 4 arms
    alg_bytes = 2 * upd_per_launch               # each uint8 read once + written once
    alg_ops = ALU_OPS_PER_UPDATE * upd_per_launch
    secs = mean_ms * 1e-3
    achieved_tops = alg_ops / secs / 1e12
    achieved_gbs = alg_bytes / secs / 1e9
    traffic = traffic_from_counters()
    roofline = {
        "kernel": "met_sweep4_kernel (one checkerboard colour, L=4096)",
        "bound": "alu", "achieved": round(achieved_tops, 2), "peak": round(VALU_PEAK_TOPS, 2),
        "unit": "Tops/s (32-bit integer VALU lane-ops)",
        "frac": round(achieved_tops / VALU_PEAK_TOPS, 4),
        "traffic": traffic,
        "alu_ops_per_update": ALU_OPS_PER_UPDATE,
        "hbm": {"achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                "traffic_gbs": round(traffic / secs / 1e9, 1) if traffic else None},
        "launches_timed": n_launch, "mean_launch_ms": round(mean_ms, 5),
        "algorithmic_bytes_per_launch": alg_bytes, "algorithmic_ops_per_launch": alg_ops,
        "updates_per_launch": upd_per_launch,
        "timing": "HIP events around every launch, separate instrumented pass of the same K steps",
        "volume_kernel_mean_ms": round(ktimes[cvf.CVF_K_VOLUME][1], 5),
    }
    # The three chains are independent jobs: on three streams of default
    # priority one chain's volume kernel and launch gaps overlap another's
    # sweep.  Reported beside the single-stream value (which the per-launch
    # roofline and the profiles describe), not as it.
    concurrent = None
    if not args.skip_concurrent:
        torch.cuda.synchronize()
        streams = [torch.cuda.Stream() for _ in mch]
        for ch, st in zip(mch, streams):
            ch.stream = st

        def met_step_streams(i):
            mch[i % len(mch)].metropolis(1)

        for i in range(W * len(mch)):
            met_step_streams(i)
        t_ms = timed(torch, met_step_streams, K)
        concurrent = {"streams": len(mch), "updates_per_ns": round(4 * N * K / (t_ms * 1e9), 2),
                      "ms_per_step": round(t_ms / K * 1e3, 5)}
        log(f"metropolis on {len(mch)} streams: {concurrent}")
        for ch in mch:
            ch.stream = None
    for ch in mch:
        o = ch.obs()
        assert o["consistent"] == 1, "incremental counters disagree with the recount"
    for ch in mch:
        ch.close()
    del mch

    # ---------------- Swendsen-Wang L = 1414 ----------------
    sw = None
    if not args.skip_sw:
        log(f"sw: {len(sw_jobs)} chains L={sw_jobs[0].L}, warmup {W}, steps {K}")
        sch = [make_chain(cvf, j.L, j.T, j.P, j.seed, cvf.CVF_ALGO_SW | cvf.CVF_ALGO_METROPOLIS) for j in sw_jobs]

        def sw_step(i):
            sch[i % len(sch)].sw(1)

        for i in range(W * len(sch)):
            sw_step(i)
        t_sw = timed(torch, sw_step, K)
        kinds = [cvf.CVF_K_VOLUME, cvf.CVF_K_SW_BONDS, cvf.CVF_K_SW_UNION, cvf.CVF_K_SW_FLIP, cvf.CVF_K_RECOUNT]
        names = ["volume", "bonds", "union", "flip", "recount"]
        kt = instrumented(cvf, sch, sw_step, K, kinds)
        sw = {"L": sw_jobs[0].L, "steps_per_s": round(K / t_sw, 1), "ms_per_step": round(t_sw / K * 1e3, 4),
              "kernel_mean_us": {nm: round(kt[k][1] * 1e3, 2) for k, nm in zip(kinds, names)}}
        log(f"sw: {sw}")
        for ch in sch:
            assert ch.obs()["consistent"] == 1
            ch.close()
        del sch

    # ---------------- arm-domain Metropolis L = 4096 ----------------
    dom = None
    if not args.skip_domain:
        log(f"arm-domain: {len(met_jobs)} chains L={met_jobs[0].L}, warmup {W}, steps {K}")
        dch = [make_chain(cvf, j.L, j.T, j.P, j.seed, cvf.CVF_ALGO_METROPOLIS) for j in met_jobs]

        def dom_step(i):
            dch[i % len(dch)].metropolis_domain(1)

        for i in range(W * len(dch)):
            dom_step(i)
        t_dom = timed(torch, dom_step, K)
        kt = instrumented(cvf, dch, dom_step, K, [cvf.CVF_K_MET_DOMAIN])
        n_pass, pass_ms = kt[cvf.CVF_K_MET_DOMAIN]
        # one pass moves one arm of every cell: N updates, 6 algorithmic bytes
        # each (the cell's four bond indices and the facing one read, one written)
        pass_s = pass_ms * 1e-3
        dom_tops = N * ALU_OPS_PER_UPDATE / pass_s / 1e12
        dom_gbs = N * 6 / pass_s / 1e9
        dom = {"L": met_jobs[0].L, "updates_per_ns": round(4 * N * K / t_dom / 1e9, 2),
               "ms_per_sweep": round(t_dom / K * 1e3, 4), "passes_timed": n_pass,
               "pass_mean_us": round(pass_ms * 1e3, 2),
               "alu": {"achieved": round(dom_tops, 2), "peak": round(VALU_PEAK_TOPS, 2),
                       "frac": round(dom_tops / VALU_PEAK_TOPS, 4)},
               "hbm": {"achieved": round(dom_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(dom_gbs / HBM_PEAK_GBS, 4), "alg_bytes_per_update": 6}}
        log(f"arm-domain: {dom}")
        for ch in dch:
            assert ch.obs()["consistent"] == 1
            ch.close()
        del dch

    # ---------------- cubic lattice with eta, N = 260^3 ----------------
    c3 = None
    if not args.skip_cvf3:
        log(f"cubic lattice with eta: L=260, warmup {min(W, 20)}, steps {args.cvf3_steps}")
        c3 = bench_cvf3(torch, min(W, 20), args.cvf3_steps, with_autocorr=not args.skip_autocorr)
        log(f"cvf3: {c3}")

    # ---------------- autocorrelation and cost per independent configuration ----------------
    auto = None
    if not args.skip_autocorr:
        auto = bench_autocorr(torch, cvf)
        log(f"autocorr: {auto}")

    batched = None
    if not args.skip_batch:
        batched = bench_batched(torch, cvf, args.batch_sweeps, args.alone_sweeps)
        log(f"batched: {batched}")

    served = None
    if args.serve_jobs > 0:
        served = bench_served(torch, args.serve_jobs)
        log(f"served: {served}")

    if args.copy_calib:
        # plain device copy of exactly 1 GiB: FETCH_SIZE / WRITE_SIZE calibration
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 1 GiB device copies")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(args.cpu_budget)
        log(f"cpu baseline: {cpu}")

    line = {
        "metric": "bond-variable updates/ns (L=4096 Metropolis); SW steps/s at 2M; p50/p99 job latency",
        "value": round(value, 2), "unit": "bond-variable updates/ns",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "paper-scale single jobs: Metropolis L=4096 (16.8M molecules, 67.1M uint8 "
                               "bond indices), T=300K, P in {0.1,25,50} MPa, one chain per P, a step = one "
                               "sweep + one volume move of one chain (round robin); SW L=1414 likewise",
                   "L": 4096, "T_K": 300.0, "P_MPa": [0.1, 25.0, 50.0], "q": 6, "seeds": [12, 13, 14]},
        "met_concurrent_streams": concurrent,
        "sw": sw,
        "met_domain": dom,
        "cvf3": c3,
        "autocorr": auto,
        "batched": batched,
        "served": served,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
