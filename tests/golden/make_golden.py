"""Writes tests/golden/trajectories.json: oracle trajectories (sigma SHA-256
digests, integer counters and v at checkpoints) for full-size workloads whose
oracle runs take minutes.  Calls only the oracle; run from the repository
root:  python tests/golden/make_golden.py  (uses one process per case)."""
import hashlib
import json
import os
import sys
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

# (name, algo, L, T [K], P [MPa], seed, checkpoints)
CASES = [(f"c2a_L1024_T{int(T)}", "met", 1024, T, 0.1, 2 + k, [10, 50, 100])
         for k, T in enumerate([270.0, 285.0, 300.0, 315.0, 330.0])] + \
        [(f"c3a_L4096_P{P}", "met", 4096, 300.0, P, 12 + k, [2, 5, 10])
         for k, P in enumerate([0.1, 25.0, 50.0])] + \
        [(f"c3b_L1414_P{P}", "sw", 1414, 300.0, P, 15 + k, [2, 5, 10])
         for k, P in enumerate([0.1, 25.0, 50.0])] + \
        [(f"c2b_L256_T{int(T)}", "sw", 256, T, 0.1, 7 + k, [20, 100, 200])
         for k, T in enumerate([270.0, 300.0, 330.0])]


def run(case):
    import oracle
    name, algo, L, T, P, seed, cps = case
    op = oracle.params_from_si(T, P, L=L, seed=seed)
    ch = oracle.Chain(op)
    out, done = [], 0
    for cp in cps:
        (ch.metropolis if algo == "met" else ch.sw)(cp - done)
        done = cp
        o = ch.obs()
        out.append({"step": cp, "sha256": hashlib.sha256(ch.sigma().tobytes()).hexdigest(),
                    **{k: o[k] for k in ("n_hb_raw", "n_coop", "count", "met_accepted", "vol_accepted")},
                    "v": o["v"]})
    return name, {"algo": algo, "L": L, "T": T, "P": P, "seed": seed, "checkpoints": out}


if __name__ == "__main__":
    import oracle
    oracle.build(force=False)
    with Pool(min(8, len(CASES))) as pool:
        res = dict(pool.map(run, CASES))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "trajectories.json")
    with open(path, "w") as f:
        json.dump({"generator": "tests/golden/make_golden.py (oracle only)", "cases": res}, f, indent=1)
    print("wrote", path, len(res), "cases")
