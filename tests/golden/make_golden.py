"""Writes the stored CPU-oracle results under tests/golden/:

* trajectories.json -- sigma SHA-256, integer counters and v at checkpoints up
  to each configuration's full length: the temperature scan (L = 1024,
  10^4 Metropolis sweeps; L = 256, 10^3 Swendsen-Wang steps; five
  temperatures each) and the pressure scan on the paper-scale lattices
  (L = 4096 Metropolis and L = 1414 Swendsen-Wang, 10^3 steps, three
  pressures);
* c4_replicas.json -- the same at 100 and 1000 sweeps for every one of the 256
  batched replicas;
* c5_subset.json -- the final state of the served jobs that workloads.py's
  c5_oracle_subset names (every job with L <= 256 plus 16 drawn at random).

Every value comes from the oracle alone.  The job descriptions come from
paper_2505_05919_amd/workloads.py, loaded as a plain module (it draws job
parameters only; nothing of the library is imported).  Run from the
repository root:

    python tests/golden/make_golden.py --jobs 6 --parts /some/dir

Each finished task is written to its own file under --parts first, so an
interrupted run resumes where it stopped; the three JSON files are written
once every task of their kind is there.  The whole set is about 13 core-hours
of oracle time.
"""
import argparse
import hashlib
import importlib.util
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)


def _workloads():
    path = os.path.join(ROOT, "paper_2505_05919_amd", "workloads.py")
    spec = importlib.util.spec_from_file_location("cvf_workloads_plain", path)
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod          # dataclasses look the module up by name
    spec.loader.exec_module(mod)
    return mod


TEMPS = [270.0, 285.0, 300.0, 315.0, 330.0]
PRESS = [0.1, 25.0, 50.0]
# (name, algo, L, T [K], P [MPa], seed, checkpoints)
TRAJ = ([(f"c2a_L1024_T{int(T)}", "met", 1024, T, 0.1, 2 + k, [10, 100, 1000, 10000])
         for k, T in enumerate(TEMPS)]
        + [(f"c2b_L256_T{int(T)}", "sw", 256, T, 0.1, 7 + k, [20, 100, 200, 1000])
           for k, T in enumerate(TEMPS)]
        + [(f"c3a_L4096_P{P}", "met", 4096, 300.0, P, 12 + k, [2, 10, 100, 1000])
           for k, P in enumerate(PRESS)]
        + [(f"c3b_L1414_P{P}", "sw", 1414, 300.0, P, 15 + k, [2, 10, 100, 1000])
           for k, P in enumerate(PRESS)])

INT_KEYS = ("n_hb_raw", "n_coop", "count", "met_accepted", "vol_accepted")


def tasks():
    wl = _workloads()
    out = [("traj", name, algo, L, T, P, seed, cps) for name, algo, L, T, P, seed, cps in TRAJ]
    for k, j in enumerate(wl.c4_jobs()):
        out.append(("c4", f"r{k:03d}", j.algo, j.L, j.T, j.P, j.seed, [100, j.nsteps]))
    stream = wl.c5_stream()
    for n in wl.c5_oracle_subset(stream):
        j = stream[n]
        out.append(("c5", f"j{n:04d}", j.algo, j.L, j.T, j.P, j.seed, [j.nsteps]))
    return out


def cost(task):
    """Rough single-core seconds, used only to start the longest tasks first."""
    _, _, algo, L, _, _, _, cps = task
    per = 4 * 39e-9 if algo == "met" else 315e-9
    return per * L * L * cps[-1]


def run(task):
    import oracle
    kind, name, algo, L, T, P, seed, cps = task
    op = oracle.params_from_si(T, P, L=L, seed=seed)
    ch = oracle.Chain(op)
    out, done = [], 0
    t0 = time.time()
    for cp in cps:
        (ch.metropolis if algo == "met" else ch.sw)(cp - done)
        done = cp
        o = ch.obs()
        out.append({"step": cp, "sha256": hashlib.sha256(ch.sigma().tobytes()).hexdigest(),
                    **{k: o[k] for k in INT_KEYS}, "v": o["v"]})
    return kind, name, {"algo": algo, "L": L, "T": T, "P": P, "seed": seed, "checkpoints": out,
                        "oracle_s": round(time.time() - t0, 1)}


def _part(parts, task):
    return os.path.join(parts, f"{task[0]}_{task[1]}.json")


def _run_to_part(args):
    parts, task = args
    kind, name, res = run(task)
    tmp = _part(parts, task) + ".tmp"
    with open(tmp, "w") as f:
        json.dump(res, f)
    os.replace(tmp, _part(parts, task))
    return kind, name, res["oracle_s"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=6)
    ap.add_argument("--parts", required=True, help="directory for per-task results (resumable)")
    ap.add_argument("--kinds", default="traj,c4,c5")
    a = ap.parse_args()
    import oracle
    oracle.build(force=False)
    os.makedirs(a.parts, exist_ok=True)
    kinds = a.kinds.split(",")
    todo = [t for t in tasks() if t[0] in kinds]
    pending = sorted((t for t in todo if not os.path.exists(_part(a.parts, t))), key=cost, reverse=True)
    print(f"{len(todo)} tasks, {len(pending)} to run, ~{sum(map(cost, pending)) / 3600:.1f} core-hours",
          flush=True)
    if pending:
        with Pool(a.jobs) as pool:
            for i, (kind, name, s) in enumerate(pool.imap_unordered(
                    _run_to_part, [(a.parts, t) for t in pending], chunksize=1)):
                print(f"[{i + 1}/{len(pending)}] {kind} {name} {s} s", flush=True)
    files = {"traj": ("trajectories.json", "cases"), "c4": ("c4_replicas.json", "replicas"),
             "c5": ("c5_subset.json", "jobs")}
    for kind in kinds:
        group = [t for t in todo if t[0] == kind]
        res = {}
        for t in group:
            with open(_part(a.parts, t)) as f:
                r = json.load(f)
            r.pop("oracle_s", None)
            res[t[1]] = r
        fname, key = files[kind]
        with open(os.path.join(HERE, fname), "w") as f:
            json.dump({"generator": "tests/golden/make_golden.py (oracle only)", key: res}, f, indent=None,
                      separators=(",", ":"))
            f.write("\n")
        print("wrote", fname, len(res), flush=True)


if __name__ == "__main__":
    main()
