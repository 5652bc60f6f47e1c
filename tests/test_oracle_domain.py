"""Pins of the oracle's arm-domain Metropolis sweep (the paper's layered
partition, Sec. II.C): the pass order is a uniform random permutation of the
four arms; the chain samples the model's Boltzmann distribution -- exact
enumeration on L = 2, closed forms in the limits J_sigma = 0, J_eff = 0 and
beta = 0 on odd lattices, agreement with the checkerboard sweep at the
paper's parameters; its incremental counters equal the recount; and the
sweep is the composition of its one-arm moves in the drawn pass order.
"""
import itertools
import math

import numpy as np
import pytest

from tests.test_oracle_chain import PAIRS, base_params, batch_z, enumerate_L2, run_series


def test_pass_order_is_a_uniform_permutation(oracle_mod):
    p = oracle_mod.params_from_si(300.0, 0.1, L=4, seed=77)
    perms = list(itertools.permutations(range(4)))
    counts = dict.fromkeys(perms, 0)
    n = 24000
    for t in range(n):
        o = tuple(oracle_mod.domain_order(p, t))
        assert sorted(o) == [0, 1, 2, 3], o
        counts[o] += 1
    exp = n / 24
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    assert chi2 < 60.0                            # 23 d.o.f., p ~ 4e-5
    # the order depends on the seed
    q = oracle_mod.params_from_si(300.0, 0.1, L=4, seed=78)
    assert [oracle_mod.domain_order(q, t) for t in range(16)] != [oracle_mod.domain_order(p, t) for t in range(16)]


@pytest.mark.parametrize("q,beta,J,Js", [(2, 1.0, 1.0, 0.5), (2, 0.7, -0.8, 0.9), (3, 0.8, 1.0, 0.6)])
def test_bruteforce_L2(oracle_mod, q, beta, J, Js):
    p = base_params(oracle_mod, q=q, beta=beta, J=J, Jsigma=Js, seed=21 + q)
    hb_ex, co_ex, hb2_ex, co2_ex = enumerate_L2(q, beta * J, beta * Js)
    s, _ = run_series(oracle_mod, p, 60000, "dom")
    for key, ex in (("n_hb_raw", hb_ex), ("n_coop", co_ex)):
        z = batch_z(s[key], ex)
        assert abs(z) < 4.5, (key, z, s[key].mean(), ex)
    assert abs(batch_z(s["n_hb_raw"] ** 2, hb2_ex)) < 4.5
    assert abs(batch_z(s["n_coop"] ** 2, co2_ex)) < 4.5


@pytest.mark.parametrize("L", [3, 5])
def test_closed_form_jsigma_zero_odd(oracle_mod, L):
    q, beta, J = 6, 1.3, 1.0
    N = L * L
    p = base_params(oracle_mod, L=L, q=q, beta=beta, J=J, Jsigma=0.0, seed=3 + L)
    s, _ = run_series(oracle_mod, p, 20000, "dom")
    e = math.exp(beta * J)
    assert abs(batch_z(s["n_hb_raw"][500:], 2 * N * e / (e + q - 1))) < 4.5
    assert abs(batch_z(s["n_coop"][500:], 6 * N / q)) < 4.5


@pytest.mark.parametrize("L", [3, 5])
def test_closed_form_jeff_zero_odd(oracle_mod, L):
    q, beta, Js = 4, 1.0, 0.9
    N = L * L
    Z = m = 0.0
    for st in itertools.product(range(q), repeat=4):
        n = sum(st[a] == st[b] for a, b in PAIRS)
        w = math.exp(beta * Js * n)
        Z += w
        m += w * n
    p = base_params(oracle_mod, L=L, q=q, beta=beta, J=0.0, Jsigma=Js, seed=5 + L)
    s, _ = run_series(oracle_mod, p, 20000, "dom")
    assert abs(batch_z(s["n_coop"][500:], N * m / Z)) < 4.5
    assert abs(batch_z(s["n_hb_raw"][500:], 2 * N / q)) < 4.5


def test_beta_zero_uniform_odd(oracle_mod):
    L, q = 7, 6
    N = L * L
    p = base_params(oracle_mod, L=L, q=q, beta=0.0, J=2.0, Jsigma=0.32, seed=9)
    s, ch = run_series(oracle_mod, p, 3000, "dom")
    o = ch.obs()
    assert o["met_accepted"] == o["met_attempted"] == 4 * N * 3000
    assert abs(batch_z(s["n_hb_raw"], 2 * N / q)) < 4.5
    assert abs(batch_z(s["n_coop"], 6 * N / q)) < 4.5


def test_agrees_with_checkerboard(oracle_mod):
    """At the paper's parameters (T = 300 K, P = 0.1 MPa) both update orders
    sample the same fixed-volume distribution."""
    res = {}
    for algo in ("met", "dom"):
        p = oracle_mod.params_from_si(300.0, 0.1, L=16, seed=51, flags=oracle_mod.NO_VOLUME_MOVE)
        s, _ = run_series(oracle_mod, p, 4000, algo)
        res[algo] = {k: v[400:] for k, v in s.items()}
    for k in ("n_hb_raw", "n_coop"):
        za = np.asarray(res["met"][k]).reshape(40, -1).mean(axis=1)
        zb = np.asarray(res["dom"][k]).reshape(40, -1).mean(axis=1)
        err = math.sqrt(za.var(ddof=1) / 40 + zb.var(ddof=1) / 40)
        assert abs(za.mean() - zb.mean()) < 4.5 * err, (k, za.mean(), zb.mean(), err)


@pytest.mark.parametrize("L", [12, 7])
def test_counters_and_invariants(oracle_mod, L):
    p = oracle_mod.params_from_si(300.0, 0.1, L=L, seed=41)
    ch = oracle_mod.Chain(p)
    N = L * L
    for _ in range(20):
        ch.metropolis_domain(3)
        o = ch.obs()
        t, hb, co = ch.incremental()
        assert (hb, co) == (o["n_hb_raw"], o["n_coop"])
        assert sum(o["count"]) == 4 * N
        assert o["met_attempted"] == 4 * N * t
        assert o["step"] == t


def nbr(L, x, y, a):
    return [((x + 1) % L, y), ((x - 1) % L, y), (x, (y + 1) % L), (x, (y - 1) % L)][a]


@pytest.mark.parametrize("L", [3, 4])
def test_sweep_is_its_passes(oracle_mod, L):
    """One sweep equals the four passes, in the drawn order, each moving arm a
    of every cell against the other arms of the cell and arm a^1 of the
    neighbour in direction a (taken before the pass: nothing in the pass
    writes plane a^1)."""
    N = L * L
    p = oracle_mod.params_from_si(285.0, 25.0, L=L, seed=61, flags=oracle_mod.NO_VOLUME_MOVE)
    met, _ = oracle_mod.tables(p)
    ch = oracle_mod.Chain(p)
    for t in range(4):
        sg = ch.sigma().reshape(4, N).astype(np.int64)
        tab = met[1 if ch.obs()["v"] < 2.0 else 0]
        for a in oracle_mod.domain_order(p, t):
            new = sg.copy()
            for y in range(L):
                for x in range(L):
                    c = x + L * y
                    fx, fy = nbr(L, x, y, a)
                    s4, _, _, _ = oracle_mod.dom_arm(p, tab, c, t, a, sg[:, c], int(sg[a ^ 1, fx + L * fy]))
                    assert all(s4[b] == sg[b, c] for b in range(4) if b != a)
                    new[a, c] = s4[a]
            sg = new
        ch.metropolis_domain(1)
        assert np.array_equal(ch.sigma().reshape(4, N), sg), t
