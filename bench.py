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
# Swendsen-Wang: algorithmic bytes per cell and step (sigma read + written,
# a 32-bit label per bond index written + read)
SW_ALG_BYTES_PER_CELL = 40
SW_COUNTERS_FILE = os.path.join(ROOT, "profiles", "sw_step_L1414_counters.json")
SW_SRCS = [os.path.join(ROOT, "paper_2505_05919_amd", "csrc", f) for f in ("philox.h", "sw_step.h", "cvf_internal.h")]
COUNTERS_FILE = os.path.join(ROOT, "profiles", "met_colour_L4096_counters.json")
KERNEL_SRCS = [os.path.join(ROOT, "paper_2505_05919_amd", "csrc", f)
               for f in ("philox.h", "met_sweep.h", "met_launch.h", "cvf_internal.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the sources the Metropolis colour kernel is built from."""
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def met_counters():
    """HBM bytes per colour launch from committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs, scaled by the same counters' reading of a plain copy of
    known size, plus the SQ counters' VALU figures; None when absent or taken
    on another version of the kernel's sources."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    with open(COUNTERS_FILE) as f:
        c = json.load(f)
    if c.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    fetch = c["fetch_kib_per_dispatch"] * 1024.0 * c["fetch_scale"]
    write = c["write_kib_per_dispatch"] * 1024.0 * c["write_scale"]
    return {"traffic_bytes": fetch + write, "valu_instr_per_update": c.get("valu_instr_per_update"),
            "valu_busy": c.get("valu_busy")}


def sw_counters():
    """Per-kernel HBM bytes and VALU busy of the Swendsen-Wang step from
    committed rocprofv3 counter runs; None when absent or stale."""
    if not os.path.exists(SW_COUNTERS_FILE):
        return None
    with open(SW_COUNTERS_FILE) as f:
        c = json.load(f)
    h = hashlib.sha256()
    for p in SW_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    if c.get("kernel_source_sha256_16") != h.hexdigest()[:16]:
        return None
    return c.get("kernels")


def warm_until(torch, chains, method, min_s: float) -> int:
    """Advance every chain by 8 steps at a time until min_s seconds of wall
    time (synchronised) have passed; returns the steps taken in all."""
    n = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < min_s:
        run_blocks(chains, method, 8 * len(chains))
        n += 8 * len(chains)
        torch.cuda.synchronize()
    return n


def make_chain(cvf, L, T, P, seed, algo_mask):
    p = cvf.cvf_params_from_si(T, P, L=L, seed=seed)
    return cvf.Chain(p, algo_mask)


def run_blocks(chains, method, K):
    """K steps of a workload of several chains: chain c advances by its share
    of K (K // n, the first K % n chains one more) in one call."""
    n = len(chains)
    for c, ch in enumerate(chains):
        k = K // n + (1 if c < K % n else 0)
        if k:
            getattr(ch, method)(k)


def timed(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def instrumented(cvf, chains, fn, kinds):
    for ch in chains:
        cvf.cvf_timing_enable(ch.h, True)
    fn()
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


def host_facts() -> dict:
    """Core count and CPU model of the host the oracle is timed on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": usable, "os_cpu_count": os.cpu_count(), "cpu_model": model}


def _oracle_sweeps(args):
    """One oracle process: Metropolis sweeps of one chain until the budget is
    used (host-aggregate leg)."""
    L, T, P, seed, budget = args
    import oracle
    op = oracle.params_from_si(T, P, L=L, seed=seed)
    ch = oracle.Chain(op)
    n, t = 0, 0.0
    while t < budget:
        t0 = time.perf_counter()
        ch.metropolis(1)
        t += time.perf_counter() - t0
        n += 1
    return 4 * L * L * n, t, n


def cpu_baseline(budget_s: float, aggregate_budget_s: float):
    """The oracle as it stands, single thread, Metropolis on the headline
    lattice, sweeps until the budget is used; then the host aggregate: the
    temperature scan's five L = 1024 Metropolis jobs at once, one oracle
    process per job."""
    import multiprocessing as mp

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
    facts = host_facts()
    out = {"value": 4 * N * n / (t * 1e9), "unit": "bond-variable updates/ns", "cores": 1, "kind": "oracle",
           "sample": f"oracle Metropolis L=4096 T=300K P=0.1MPa seed 12, {n} sweeps after init "
                     f"({4 * N * n} updates, {t:.1f} s, one thread)",
           "host": facts}
    if aggregate_budget_s > 0:
        from paper_2505_05919_amd.workloads import c2_jobs
        jobs = [j for j in c2_jobs() if j.algo == "met"]
        ctx = mp.get_context("spawn")
        t0 = time.perf_counter()
        with ctx.Pool(len(jobs)) as pool:
            res = pool.map(_oracle_sweeps, [(j.L, j.T, j.P, j.seed, aggregate_budget_s) for j in jobs])
        wall = time.perf_counter() - t0
        upd = sum(r[0] for r in res)
        busy = max(r[1] for r in res)
        out["host_aggregate"] = {
            "value": round(upd / busy / 1e9, 4), "unit": "bond-variable updates/ns", "cores": len(jobs),
            "kind": "oracle", "per_process_updates_per_ns": [round(r[0] / r[1] / 1e9, 4) for r in res],
            "sample": f"the L=1024 Metropolis temperature scan (T = 270..330 K, 0.1 MPa, seeds 2-6), one oracle "
                      f"process per job, {[r[2] for r in res]} sweeps each in ~{aggregate_budget_s:.0f} s "
                      f"({wall:.1f} s wall incl. start-up) on a host with {facts['nproc']} usable cores"}
    return out


def bench_batched(torch, cvf, sweeps, with_alone=True):
    """256 independent replicas of uneven L (log-uniform 64..512) on a 16x16
    (T, P) grid: one batched launch per colour phase, 100-sweep blocks replayed
    from a hipGraph, launch shape from the autotuner.  The first block (graph
    capture and first replay) is untimed, the remaining sweeps - 100 timed.
    Then the same jobs one at a time with plain launches, `sweeps` each; per-
    replica sigma digests and counters after `sweeps` sweeps must be identical
    in both runs and equal to the stored oracle results (all 256 replicas at
    1000 sweeps, tests/golden/c4_replicas.json)."""
    import hashlib
    from paper_2505_05919_amd.workloads import c4_jobs
    jobs = c4_jobs()
    block = 100
    assert sweeps % block == 0 and sweeps >= 2 * block

    def chains():
        return [make_chain(cvf, j.L, j.T, j.P, j.seed, cvf.CVF_ALGO_METROPOLIS) for j in jobs]

    def results(chs):
        out = []
        for c in chs:
            o = c.obs()
            out.append((hashlib.sha256(c.sigma.cpu().numpy().tobytes()).hexdigest(), o["n_hb_raw"], o["n_coop"],
                        tuple(o["count"]), o["met_accepted"], o["vol_accepted"], o["v"], o["step"]))
        return out

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
    b.metropolis(block, graph_block=block)          # capture + first replay, untimed
    timed_sweeps = sweeps - block
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.metropolis(timed_sweeps, graph_block=block)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    b.close()
    r_batch = results(chs)
    for c in chs:
        c.close()
    v_batch = upd_per_sweep * timed_sweeps / t_batch / 1e9
    out = {"replicas": len(jobs), "sweeps": sweeps, "timed_sweeps": timed_sweeps, "graph_block": block,
           "rows": rows, "updates_per_ns": round(v_batch, 1), "ms": round(t_batch * 1e3, 2),
           # whole sweeps (volume and both colour launches), 2 algorithmic bytes and
           # the 34-op floor per update, as the single-chain roofline
           "roofline": {"bound": "hbm", "achieved": round(2 * v_batch, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(2 * v_batch / HBM_PEAK_GBS, 4), "alg_bytes_per_update": 2,
                        "alu_frac": round(v_batch * 1e9 * ALU_OPS_PER_UPDATE / 1e12 / VALU_PEAK_TOPS, 4),
                        "basis": "wall time of the timed sweeps"}}
    gold_path = os.path.join(ROOT, "tests", "golden", "c4_replicas.json")
    if os.path.exists(gold_path) and sweeps == 1000:
        with open(gold_path) as f:
            gold = json.load(f)["replicas"]
        bad = []
        for k, r in enumerate(r_batch):
            g = gold[f"r{k:03d}"]["checkpoints"][-1]
            want = (g["sha256"], g["n_hb_raw"], g["n_coop"], tuple(g["count"]), g["met_accepted"],
                    g["vol_accepted"])
            if r[:6] != want or abs(r[6] - g["v"]) > 1e-12 * abs(g["v"]) or r[7] != g["step"]:
                bad.append(k)
        out["oracle"] = {"replicas_compared": len(r_batch), "mismatches": bad[:20], "identical": not bad}
        assert not bad, f"batched replicas differ from the stored oracle results: {bad[:10]}"
    if with_alone:
        alone = chains()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in alone:
            c.metropolis(sweeps)
        torch.cuda.synchronize()
        t_alone = time.perf_counter() - t0
        r_alone = results(alone)
        for c in alone:
            c.close()
        v_alone = upd_per_sweep * sweeps / t_alone / 1e9
        same = r_alone == r_batch
        assert same, "batched replicas differ from the same jobs run one at a time"
        out.update({"one_at_a_time_updates_per_ns": round(v_alone, 2), "speedup": round(v_batch / v_alone, 1),
                    "identical_to_alone": same, "compared_at_sweeps": sweeps})
    return out


def bench_sizes(torch, cvf):
    """One chain per lattice size (300 K, 0.1 MPa), single stream: time per
    Metropolis sweep (L 256..16384) and per SW step (L 256..4096), each after
    0.3 s of warm-up load, so that where a step is launch latency and where it
    is throughput shows."""
    def per_step(fn, n):
        fn(10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 0.3:
            fn(10)
            torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(n)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    out = {"met": {}, "sw": {}}
    for L in (256, 512, 1024, 2048, 4096, 8192, 16384):
        ch = make_chain(cvf, L, 300.0, 0.1, 12, cvf.CVF_ALGO_METROPOLIS)
        dt = per_step(lambda k: ch.metropolis(k), min(2000, max(20, int(2e9 / (4 * L * L)))))
        out["met"][str(L)] = {"us_per_sweep": round(dt * 1e6, 2), "updates_per_ns": round(4 * L * L / dt / 1e9, 1)}
        assert ch.obs()["consistent"] == 1
        ch.close()
    for L in (256, 512, 1024, 1414, 2048, 4096):
        ch = make_chain(cvf, L, 300.0, 0.1, 15, cvf.CVF_ALGO_METROPOLIS | cvf.CVF_ALGO_SW)
        dt = per_step(lambda k: ch.sw(k), min(2000, max(20, int(2e8 / (L * L)))))
        out["sw"][str(L)] = {"us_per_step": round(dt * 1e6, 2), "steps_per_s": round(1.0 / dt, 1),
                             "cell_steps_per_ns": round(L * L / dt / 1e9, 2)}
        assert ch.obs()["consistent"] == 1
        ch.close()
    return out


def bench_served(torch, n_jobs, compare_jobs):
    """The served stream: Poisson arrivals at 200 jobs/s, L log-uniform 32..2048,
    T ~ U(270, 330) K, P ~ U(0, 50) MPa, nsteps ~ U[100, 10^4], 80 % Metropolis /
    20 % SW, admitted by HBM footprint, lattices resident.  Quanta advance the
    resident jobs with the least remaining work first (until they hold 2^24
    cells).  Reported: p50/p99 latency (arrival to completion) split into
    queueing and service, offered and achieved load; the final sigma digest
    and integer counters of every job in the stored CPU-oracle subset (every
    job with L <= 256 plus 16 drawn at random) must equal the stored ones.
    Then the first `compare_jobs` jobs of the same stream, as a trace of their
    own: served (least remaining work first, and processor sharing) against a
    one-job-at-a-time FCFS server with plain launches (service times measured
    job by job), every result identical alone and in the mix."""
    from paper_2505_05919_amd import serve
    from paper_2505_05919_amd.workloads import c5_oracle_subset, c5_stream
    jobs = c5_stream(n_jobs=n_jobs)
    # sigma digests only for the jobs checked against the oracle (hashing
    # every served lattice would keep the GPU idle while the host hashes)
    check = c5_oracle_subset(jobs) if n_jobs == 2000 else []
    srv = serve.Server(memory_budget=32 << 30, max_slots=1024, quantum=100, keep_digest=True, schedule="srpt",
                       fill_cells=1 << 24, digest_seeds=frozenset(jobs[n].seed for n in check))
    recs = srv.run(jobs, realtime=True)
    s = serve.summarize(recs)
    by_seed = {r.job.seed: r for r in recs}
    # the stored oracle results (tests/golden/c5_subset.json, written from the oracle alone)
    gold_path = os.path.join(ROOT, "tests", "golden", "c5_subset.json")
    oracle_check = None
    if os.path.exists(gold_path) and n_jobs == 2000:
        with open(gold_path) as f:
            gold = json.load(f)["jobs"]
        want = c5_oracle_subset(jobs)
        bad = []
        for n in want:
            g = gold[f"j{n:04d}"]["checkpoints"][-1]
            r = by_seed[jobs[n].seed]
            ok = (r.digest == g["sha256"] and all(r.obs[k] == g[k] for k in
                                                  ("n_hb_raw", "n_coop", "count", "met_accepted", "vol_accepted"))
                  and abs(r.obs["v"] - g["v"]) <= 1e-12 * abs(g["v"]) and r.obs["step"] == g["step"])
            if not ok:
                bad.append(n)
        oracle_check = {"jobs_compared": len(want), "mismatches": bad[:20], "identical": not bad,
                        "subset": "every job with L <= 256 plus 16 of the others drawn by default_rng(5005)"}
        assert not bad, f"served jobs differ from the stored oracle results: {bad[:10]}"
    met_upd = sum(4 * j.L ** 2 * j.nsteps for j in jobs if j.algo == "met")
    sw_cells = sum(j.L ** 2 * j.nsteps for j in jobs if j.algo == "sw")
    span_arr = max(j.arrival for j in jobs)
    out = {"jobs": n_jobs, "rate_per_s": 200.0, "quantum": srv.quantum, "max_resident_jobs": srv.max_slots,
           "schedule": "least remaining work first, >= 2^24 cells per quantum",
           "p50_ms": round(s["p50_s"] * 1e3, 1), "p99_ms": round(s["p99_s"] * 1e3, 1),
           "queue_p50_ms": round(s["queue_p50_s"] * 1e3, 1), "queue_p99_ms": round(s["queue_p99_s"] * 1e3, 1),
           "service_p50_ms": round(float(np.percentile([r.completed - r.admitted for r in recs], 50)) * 1e3, 1),
           "service_p99_ms": round(float(np.percentile([r.completed - r.admitted for r in recs], 99)) * 1e3, 1),
           "makespan_s": round(s["makespan_s"], 3),
           "achieved": {"met_updates_per_ns": round(s["met_updates_per_ns"], 1),
                        "sw_cell_steps_per_ns": round(s["sw_cell_steps_per_ns"], 2)},
           "offered": {"met_updates_per_ns": round(met_upd / span_arr / 1e9, 1),
                       "sw_cell_steps_per_ns": round(sw_cells / span_arr / 1e9, 2),
                       "arrival_span_s": round(span_arr, 3)},
           "peak_resident_jobs": srv.peak_resident_jobs, "peak_resident_MB": round(srv.peak_resident_bytes / 2**20, 1),
           "quanta": srv.quanta, "loop_phase_s": {k: round(v, 3) for k, v in srv.phase_s.items()},
           "oracle_subset": oracle_check}
    if compare_jobs > 0:
        out["vs_one_at_a_time"] = bench_served_compare(torch, compare_jobs)
    return out


def bench_served_compare(torch, n_jobs):
    """The first n_jobs jobs of the served stream (their own arrival times):
    served with both schedules against one-at-a-time FCFS plain launches."""
    from paper_2505_05919_amd import serve
    from paper_2505_05919_amd.workloads import c5_stream
    jobs = c5_stream(n_jobs=n_jobs)
    ps = serve.Server(memory_budget=32 << 30, max_slots=1024, quantum=100, keep_digest=True, schedule="all")
    s_ps = serve.summarize(ps.run(jobs, realtime=True))
    srv = serve.Server(memory_budget=32 << 30, max_slots=1024, quantum=100, keep_digest=True, schedule="srpt",
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
    assert same, "a served job differs from the same job run alone"
    lat = serve.fcfs_latencies(jobs, service)
    done = 0.0
    for j, t in zip(jobs, service):
        done = max(done, j.arrival) + t
    t_first = min(j.arrival for j in jobs)
    upd = sum(4 * j.L ** 2 * j.nsteps for j in jobs if j.algo == "met")
    return {"jobs": n_jobs, "trace": f"the first {n_jobs} jobs of the same stream",
            "served": {"p50_ms": round(s["p50_s"] * 1e3, 1), "p99_ms": round(s["p99_s"] * 1e3, 1),
                       "makespan_s": round(s["makespan_s"], 3),
                       "met_updates_per_ns": round(s["met_updates_per_ns"], 1)},
            "processor_sharing": {"p50_ms": round(s_ps["p50_s"] * 1e3, 1), "p99_ms": round(s_ps["p99_s"] * 1e3, 1),
                                  "makespan_s": round(s_ps["makespan_s"], 3)},
            "one_at_a_time": {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 1),
                              "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 1),
                              "makespan_s": round(done - t_first, 3),
                              "met_updates_per_ns": round(upd / (done - t_first) / 1e9, 1)},
            "identical_to_alone": same}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--warmup", type=int, default=100,
                    help="untimed steps per chain first: the GPU needs some tens of ms of load to reach its steady clock")
    ap.add_argument("--min-warmup-s", type=float, default=0.5,
                    help="after the W warm-up steps, keep running untimed steps until this much wall time "
                         "of GPU load has passed (clock ramp)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--cpu-aggregate-budget", type=float, default=8.0,
                    help="seconds per oracle process of the host-aggregate leg (0 = skip)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain device copy of 1 GiB (counter calibration)")
    ap.add_argument("--skip-sw", action="store_true")
    ap.add_argument("--sw-min-steps", type=int, default=300,
                    help="Swendsen-Wang steps timed (at least --steps)")
    ap.add_argument("--skip-domain", action="store_true")
    ap.add_argument("--skip-autocorr", action="store_true")
    ap.add_argument("--skip-batch", action="store_true")
    ap.add_argument("--skip-cvf3", action="store_true")
    ap.add_argument("--sizes", action="store_true",
                    help="also time one chain per lattice size (Metropolis L 256..16384, SW L 256..4096)")
    ap.add_argument("--skip-concurrent", action="store_true",
                    help="skip the three-stream Metropolis leg (profiled runs: it overlaps launches)")
    ap.add_argument("--cvf3-steps", type=int, default=200)
    ap.add_argument("--batch-sweeps", type=int, default=1000)
    ap.add_argument("--skip-batch-alone", action="store_true",
                    help="batched leg without the one-at-a-time comparison (profiled runs)")
    ap.add_argument("--serve-jobs", type=int, default=2000,
                    help="jobs of the served Poisson stream (0 = skip)")
    ap.add_argument("--serve-compare-jobs", type=int, default=200,
                    help="leading jobs of the stream also served against one-at-a-time launches (0 = skip)")
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

    # A step is one sweep (with its volume move) of one chain; the K timed
    # steps are each chain's share of K in one call per chain.
    run_blocks(mch, "metropolis", W * len(mch))
    # The GPU reaches its steady clock only after some tens of ms of load: a
    # short warm-up (a few sweeps) would put the clock ramp inside the timed
    # region.  Keep sweeping, untimed, until min_warmup_s of load has passed.
    warm_extra = warm_until(torch, mch, "metropolis", args.min_warmup_s)
    t_met = timed(torch, lambda: run_blocks(mch, "metropolis", K))
    ms_per_step = t_met / K * 1e3
    value = 4 * N * K / (t_met * 1e9)
    log(f"metropolis: {ms_per_step:.4f} ms/sweep, {value:.1f} updates/ns (+{warm_extra} clock warm-up sweeps)")
    ktimes = instrumented(cvf, mch, lambda: run_blocks(mch, "metropolis", K), [cvf.CVF_K_MET_SWEEP, cvf.CVF_K_VOLUME])
    n_launch, mean_ms = ktimes[cvf.CVF_K_MET_SWEEP]
    upd_per_launch = 2 * N                      # one colour: N/2 cells x 4 arms
    alg_bytes = 2 * upd_per_launch               # each uint8 read once + written once
    alg_ops = ALU_OPS_PER_UPDATE * upd_per_launch
    secs = mean_ms * 1e-3
    achieved_tops = alg_ops / secs / 1e12
    achieved_gbs = alg_bytes / secs / 1e9
    counters = met_counters()
    traffic = counters["traffic_bytes"] if counters else None
    roofline = {
        "kernel": "met_sweep4_kernel (one checkerboard colour, L=4096)",
        "bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "alg_bytes_per_update": 2,
        "limiter": "VALU issue, not HBM: see alu (the fraction of the 8 TB/s roofline is what the path reaches; "
                   "the integer work per update caps it well below 1)",
        "alu": {"achieved": round(achieved_tops, 2), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "T lane-ops/s (full-rate 32-bit VALU issue)",
                "frac": round(achieved_tops / VALU_PEAK_TOPS, 4), "ops_per_update_floor": ALU_OPS_PER_UPDATE,
                "valu_instr_per_update": counters.get("valu_instr_per_update") if counters else None,
                "valu_busy": counters.get("valu_busy") if counters else None,
                "counters_from": "profiles/met_colour_L4096_counters.json" if counters else None},
        "traffic_gbs": round(traffic / secs / 1e9, 1) if traffic else None,
        "launches_timed": n_launch, "mean_launch_ms": round(mean_ms, 5),
        "algorithmic_bytes_per_launch": alg_bytes, "updates_per_launch": upd_per_launch,
        "timing": "HIP start/stop events recorded by every launch's own dispatch (hipExtLaunchKernel), in a separate instrumented pass of the same K steps",
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

        run_blocks(mch, "metropolis", W * len(mch))
        t_ms = timed(torch, lambda: run_blocks(mch, "metropolis", K))
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
        KS = max(K, args.sw_min_steps)
        log(f"sw: {len(sw_jobs)} chains L={sw_jobs[0].L}, warmup {W}, steps {KS}")
        sch = [make_chain(cvf, j.L, j.T, j.P, j.seed, cvf.CVF_ALGO_SW | cvf.CVF_ALGO_METROPOLIS) for j in sw_jobs]

        run_blocks(sch, "sw", W * len(sch))
        warm_until(torch, sch, "sw", 0.2)
        t_sw = timed(torch, lambda: run_blocks(sch, "sw", KS))
        kinds = [cvf.CVF_K_VOLUME, cvf.CVF_K_SW_BONDS, cvf.CVF_K_SW_UNION, cvf.CVF_K_SW_FLIP, cvf.CVF_K_RECOUNT]
        names = ["volume", "bonds", "union", "flip", "recount"]
        kt = instrumented(cvf, sch, lambda: run_blocks(sch, "sw", KS), kinds)
        Ls = sw_jobs[0].L
        step_s = t_sw / KS
        gbs = SW_ALG_BYTES_PER_CELL * Ls * Ls / step_s / 1e9
        swc = sw_counters()
        sw = {"L": Ls, "steps": KS, "steps_per_s": round(KS / t_sw, 1), "ms_per_step": round(step_s * 1e3, 4),
              "kernel_mean_us": {nm: round(kt[k][1] * 1e3, 2) for k, nm in zip(kinds, names) if kt[k][0]},
              "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(gbs / HBM_PEAK_GBS, 4), "alg_bytes_per_cell": SW_ALG_BYTES_PER_CELL,
                           "basis": "whole step (every launch), wall time per step; algorithmic bytes per cell: "
                                    "sigma read and written (8) and a 32-bit label of each of the 4 bond indices "
                                    "written and read (32)",
                           "kernels": swc}}
        # the three SW jobs on three streams (as for Metropolis above): the
        # latency-bound tile launches, volume kernels and launch gaps of one
        # chain overlap another's; aggregate steps/s of the three jobs
        if not args.skip_concurrent:
            torch.cuda.synchronize()
            streams = [torch.cuda.Stream() for _ in sch]
            for ch, st in zip(sch, streams):
                ch.stream = st
            run_blocks(sch, "sw", W * len(sch))
            t_c = timed(torch, lambda: run_blocks(sch, "sw", KS))
            sw["concurrent_streams"] = {"streams": len(sch), "steps_per_s": round(KS / t_c, 1),
                                        "ms_per_step": round(t_c / KS * 1e3, 5)}
            for ch in sch:
                ch.stream = None
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

        run_blocks(dch, "metropolis_domain", W * len(dch))
        t_dom = timed(torch, lambda: run_blocks(dch, "metropolis_domain", K))
        kt = instrumented(cvf, dch, lambda: run_blocks(dch, "metropolis_domain", K), [cvf.CVF_K_MET_DOMAIN])
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
        batched = bench_batched(torch, cvf, args.batch_sweeps, with_alone=not args.skip_batch_alone)
        log(f"batched: {batched}")

    sizes = None
    if args.sizes:
        sizes = bench_sizes(torch, cvf)
        log(f"sizes: {sizes}")

    served = None
    if args.serve_jobs > 0:
        served = bench_served(torch, args.serve_jobs, args.serve_compare_jobs)
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
        cpu = cpu_baseline(args.cpu_budget, args.cpu_aggregate_budget)
        log(f"cpu baseline: {cpu}")

    line = {
        "metric": "bond-variable updates/ns (L=4096 Metropolis); SW steps/s at 2M; p50/p99 job latency",
        "value": round(value, 2), "unit": "bond-variable updates/ns",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "paper-scale single jobs: Metropolis L=4096 (16.8M molecules, 67.1M uint8 "
                               "bond indices), T=300K, P in {0.1,25,50} MPa, one chain per P, a step = one "
                               "sweep + one volume move of one chain; the K timed steps are each chain's "
                               "share of K, one call per chain; SW L=1414 likewise",
                   "L": 4096, "T_K": 300.0, "P_MPa": [0.1, 25.0, 50.0], "q": 6, "seeds": [12, 13, 14]},
        "met_concurrent_streams": concurrent,
        "sw": sw,
        "met_domain": dom,
        "cvf3": c3,
        "autocorr": auto,
        "batched": batched,
        "served": served,
        "sizes": sizes,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
