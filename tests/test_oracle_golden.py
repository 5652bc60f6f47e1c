"""The stored oracle trajectories still match the oracle (the smallest
cases, re-run here), so a change to the oracle's arithmetic cannot leave
tests/golden/trajectories.json silently stale."""
import hashlib
import json
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("name", ["c2b_L256_T270", "c2a_L1024_T300"])
def test_golden_first_checkpoint(oracle_mod, name):
    with open(os.path.join(HERE, "golden", "trajectories.json")) as f:
        case = json.load(f)["cases"][name]
    cp = case["checkpoints"][0]
    ch = oracle_mod.Chain(oracle_mod.params_from_si(case["T"], case["P"], L=case["L"], seed=case["seed"]))
    (ch.metropolis if case["algo"] == "met" else ch.sw)(cp["step"])
    o = ch.obs()
    for k in ("n_hb_raw", "n_coop", "count", "met_accepted", "vol_accepted"):
        assert o[k] == cp[k], (name, k)
    assert o["v"] == cp["v"]
    assert hashlib.sha256(ch.sigma().tobytes()).hexdigest() == cp["sha256"]
