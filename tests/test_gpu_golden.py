"""Full-size GPU parity against stored oracle trajectories.

tests/golden/trajectories.json holds, for the temperature scan (L = 1024,
five temperatures), the pressure scan on the headline lattice (L = 4096
Metropolis, L = 1414 Swendsen-Wang, three pressures) and a small SW scan,
the SHA-256 of sigma, every integer counter and v at checkpoints, written by
tests/golden/make_golden.py from the oracle alone.  The library replays each
trajectory in the launch configuration the benchmark times: single chains
with default launches, and the Metropolis cases again as one batch with the
autotuned row count and hipGraph-replayed sweep blocks.
"""
import hashlib
import json
import os
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "trajectories.json")) as f:
    GOLD = json.load(f)["cases"]
INT_KEYS = ("n_hb_raw", "n_coop", "count", "met_accepted", "vol_accepted")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cvf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_05919_amd import cvf as mod
    mod.lib()
    return mod


def make(cvf, case):
    p = cvf.cvf_params_from_si(case["T"], case["P"], L=case["L"], seed=case["seed"])
    mask = cvf.CVF_ALGO_METROPOLIS | (cvf.CVF_ALGO_SW if case["algo"] == "sw" else 0)
    return cvf.Chain(p, mask)


def check(ch, cp, ctx):
    o = ch.obs()
    for k in INT_KEYS:
        assert o[k] == cp[k], (ctx, k, o[k], cp[k])
    assert o["consistent"] == 1, ctx
    assert o["v"] == pytest.approx(cp["v"], rel=1e-12), (ctx, o["v"], cp["v"])
    assert hashlib.sha256(ch.sigma.cpu().numpy().tobytes()).hexdigest() == cp["sha256"], ctx


@pytest.mark.parametrize("name", sorted(GOLD))
def test_golden_single(cvf, name):
    case = GOLD[name]
    say(f"case golden {name} algo={case['algo']} L={case['L']} seed={case['seed']}")
    ch = make(cvf, case)
    done = 0
    for cp in case["checkpoints"]:
        n = cp["step"] - done
        (ch.metropolis if case["algo"] == "met" else ch.sw)(n)
        done = cp["step"]
        check(ch, cp, f"{name} step {done}")
    ch.close()


@pytest.mark.parametrize("scan", ["c2a", "c3a"])
def test_golden_batched(cvf, scan):
    """A scan's Metropolis chains as one batch: autotuned rows, graph blocks."""
    names = sorted(n for n in GOLD if n.startswith(scan) and GOLD[n]["algo"] == "met")
    say(f"case golden batch {scan}: {names}")
    tune = [make(cvf, GOLD[n]) for n in names]       # the autotuner advances its chains
    tb = cvf.Batch(tune)
    rows = tb.autotune(2)
    tb.close()
    for ch in tune:
        ch.close()
    chains = [make(cvf, GOLD[n]) for n in names]
    b = cvf.Batch(chains)
    b.set_rows(rows)
    done = 0
    cps = GOLD[names[0]]["checkpoints"]
    for i, cp in enumerate(cps):
        n = cp["step"] - done
        blk = 5 if n % 5 == 0 else 0
        b.metropolis(n, graph_block=blk)
        done = cp["step"]
        for nm, ch in zip(names, chains):
            assert GOLD[nm]["checkpoints"][i]["step"] == done
            check(ch, GOLD[nm]["checkpoints"][i], f"batch {nm} step {done} rows {rows}")
    b.close()
    for ch in chains:
        ch.close()
