"""Statistical and structural pins for the oracle's Markov chain.

The Metropolis sweep, the Swendsen-Wang step and the volume move are checked
against what the model's definition (Sec. II.A, Eq. (1)-(3)) fixes exactly:
closed forms in the limits J_sigma = 0, J_eff = 0 and beta = 0, brute-force
enumeration of all states of an L = 2 lattice, a 1-D quadrature of the volume
marginal, invariants of the counters, and agreement of the two algorithms.
A dropped term, a wrong sign or a mis-indexed neighbour in the oracle moves
one of these averages by many standard errors.
"""
import functools
import itertools
import math

import numpy as np
import pytest
from scipy import integrate

# independent description of the 2-D lattice: arm 0:+x 1:-x 2:+y 3:-y
PAIRS = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def bond_lists(L):
    N = L * L
    cov, coop = [], []
    for y in range(L):
        for x in range(L):
            c = x + L * y
            cov.append((0 * N + c, 1 * N + (x + 1) % L + L * y))
            cov.append((2 * N + c, 3 * N + x + L * ((y + 1) % L)))
            for a, b in PAIRS:
                coop.append((a * N + c, b * N + c))
    return np.array(cov), np.array(coop)


@functools.lru_cache(maxsize=None)
def density_of_states_L2(q):
    """g[hb, co] = number of the q^16 configurations of an L = 2 lattice with
    N_HB_raw = hb and N_coop = co (exhaustive enumeration, split into two
    halves of 8 bond indices so that numpy vectorises over one half)."""
    cov, coop = bond_lists(2)
    pairs = np.concatenate([cov, coop])
    is_cov = np.arange(len(pairs)) < len(cov)
    half = q ** 8
    dig = (np.arange(half)[:, None] // (q ** np.arange(8))[None, :]) % q     # [half, 8]
    low_hb = np.zeros(half, np.int64)
    low_co = np.zeros(half, np.int64)
    mixed = []
    high_only = []
    for (i, j), cv in zip(pairs, is_cov):
        i, j = min(i, j), max(i, j)
        if j < 8:
            e = (dig[:, i] == dig[:, j]).astype(np.int64)
            if cv:
                low_hb += e
            else:
                low_co += e
        elif i >= 8:
            high_only.append((i - 8, j - 8, cv))
        else:
            mixed.append((i, j - 8, cv))
    onehot = [[(dig[:, i] == v).astype(np.int64) for v in range(q)] for i in range(8)]
    g = np.zeros((2 * 4 + 1, 6 * 4 + 1), dtype=np.int64)
    for h in range(half):
        hd = dig[h]
        hb = low_hb.copy()
        co = low_co.copy()
        for i, j, cv in high_only:
            if hd[i] == hd[j]:
                if cv:
                    hb += 1
                else:
                    co += 1
        for i, j, cv in mixed:
            if cv:
                hb += onehot[i][hd[j]]
            else:
                co += onehot[i][hd[j]]
        g += np.bincount(hb * g.shape[1] + co, minlength=g.size).reshape(g.shape)
    assert g.sum() == q ** 16
    return g


def enumerate_L2(q, beta_jeff, beta_js):
    """Exact moments of (N_HB_raw, N_coop) on L = 2 (16 bond indices) with
    weight exp(beta_jeff * N_HB_raw + beta_js * N_coop)."""
    g = density_of_states_L2(q).astype(np.float64)
    hb = np.arange(g.shape[0])[:, None].astype(np.float64)
    co = np.arange(g.shape[1])[None, :].astype(np.float64)
    w = g * np.exp(beta_jeff * hb + beta_js * co)
    Z = w.sum()
    return (w * hb).sum() / Z, (w * co).sum() / Z, (w * hb * hb).sum() / Z, (w * co * co).sum() / Z


def batch_z(samples, exact, nbatch=50):
    x = np.asarray(samples, dtype=np.float64)
    x = x[: len(x) // nbatch * nbatch].reshape(nbatch, -1).mean(axis=1)
    err = x.std(ddof=1) / math.sqrt(nbatch)
    return (x.mean() - exact) / max(err, 1e-12)


def run_series(oracle_mod, p, n, algo="met", keys=("n_hb_raw", "n_coop")):
    ch = oracle_mod.Chain(p)
    out = {k: np.empty(n) for k in keys}
    step = {"met": ch.metropolis, "sw": ch.sw, "dom": ch.metropolis_domain}[algo]
    for i in range(n):
        step(1)
        o = ch.obs()
        for k in keys:
            out[k][i] = o[k]
    return out, ch


def base_params(oracle_mod, **kw):
    d = dict(L=2, q=2, beta=1.0, J=1.0, Jsigma=0.5, P=0.0, vHB=0.6, v_init=1.25, dv_max=0.0,
             seed=7, flags=oracle_mod.NO_VOLUME_MOVE)
    d.update(kw)
    return oracle_mod.make_params(**d)


@pytest.mark.parametrize("algo", ["met", "sw"])
@pytest.mark.parametrize("q,beta,J,Js", [(2, 1.0, 1.0, 0.5), (2, 0.7, -0.8, 0.9), (3, 0.8, 1.0, 0.6)])
def test_bruteforce_L2(oracle_mod, algo, q, beta, J, Js):
    if algo == "sw" and J < 0:
        pytest.skip("SW with J_eff < 0 bonds unequal pairs; its stationarity is not claimed")
    p = base_params(oracle_mod, q=q, beta=beta, J=J, Jsigma=Js, seed=11 + q)
    hb_ex, co_ex, hb2_ex, co2_ex = enumerate_L2(q, beta * J, beta * Js)
    n = 60000 if algo == "met" else 30000
    s, _ = run_series(oracle_mod, p, n, algo)
    for key, ex in (("n_hb_raw", hb_ex), ("n_coop", co_ex)):
        z = batch_z(s[key], ex)
        assert abs(z) < 4.5, (key, z, s[key].mean(), ex)
    z2 = batch_z(s["n_hb_raw"] ** 2, hb2_ex)
    assert abs(z2) < 4.5


def test_closed_form_jsigma_zero(oracle_mod):
    """J_sigma = 0: facing pairs are independent two-state systems;
    <N_HB_raw> = 2N e^{bJ}/(e^{bJ}+q-1), arms of one cell independent so
    <N_coop> = 6N/q."""
    L, q, beta, J = 8, 6, 1.3, 1.0
    N = L * L
    for algo in ("met", "sw"):
        p = base_params(oracle_mod, L=L, q=q, beta=beta, J=J, Jsigma=0.0, seed=3)
        s, _ = run_series(oracle_mod, p, 6000, algo)
        e = math.exp(beta * J)
        assert abs(batch_z(s["n_hb_raw"][500:], 2 * N * e / (e + q - 1))) < 4.5
        assert abs(batch_z(s["n_coop"][500:], 6 * N / q)) < 4.5


def test_closed_form_jeff_zero(oracle_mod):
    """J = P = 0: each cell is an independent 4-state Potts clique (K4);
    <N_coop> = N <n>_K4 by enumerating q^4 states, <N_HB_raw> = 2N/q."""
    L, q, beta, Js = 8, 4, 1.0, 0.9
    N = L * L
    Z = m = 0.0
    for st in itertools.product(range(q), repeat=4):
        n = sum(st[a] == st[b] for a, b in PAIRS)
        w = math.exp(beta * Js * n)
        Z += w
        m += w * n
    for algo in ("met", "sw"):
        p = base_params(oracle_mod, L=L, q=q, beta=beta, J=0.0, Jsigma=Js, seed=5)
        s, _ = run_series(oracle_mod, p, 6000, algo)
        assert abs(batch_z(s["n_coop"][500:], N * m / Z)) < 4.5
        assert abs(batch_z(s["n_hb_raw"][500:], 2 * N / q)) < 4.5


def test_beta_zero_uniform(oracle_mod):
    L, q = 8, 6
    N = L * L
    p = base_params(oracle_mod, L=L, q=q, beta=0.0, J=2.0, Jsigma=0.32, seed=9)
    s, ch = run_series(oracle_mod, p, 3000, "met")
    o = ch.obs()
    # every proposal is accepted unless it is a NULL draw (probability 2^-32)
    assert o["met_accepted"] == o["met_attempted"] == 4 * N * 3000
    assert abs(batch_z(s["n_hb_raw"], 2 * N / q)) < 4.5
    assert abs(batch_z(s["n_coop"], 6 * N / q)) < 4.5


def test_metropolis_sw_agree(oracle_mod):
    """At the paper's parameters (T = 300 K, P = 0.1 MPa, Table I) both
    algorithms sample the same fixed-volume distribution."""
    res = {}
    for algo in ("met", "sw"):
        p = oracle_mod.params_from_si(300.0, 0.1, L=16, seed=21, flags=oracle_mod.NO_VOLUME_MOVE)
        s, _ = run_series(oracle_mod, p, 4000, algo)
        res[algo] = {k: v[400:] for k, v in s.items()}
    for k in ("n_hb_raw", "n_coop"):
        a, b = res["met"][k], res["sw"][k]
        za = np.asarray(a).reshape(40, -1).mean(axis=1)
        zb = np.asarray(b).reshape(40, -1).mean(axis=1)
        err = math.sqrt(za.var(ddof=1) / 40 + zb.var(ddof=1) / 40)
        assert abs(za.mean() - zb.mean()) < 4.5 * err, (k, za.mean(), zb.mean(), err)


def direct_u(v):
    e = 0.0
    for i in range(-7, 8):
        for j in range(-7, 8):
            if (i or j) and v * (i * i + j * j) <= 36.0:
                d2 = v * (i * i + j * j)
                e += 2.0 * (d2 ** -6 - d2 ** -3)
    return e


def test_volume_marginal_quadrature(oracle_mod):
    """Volume move + Metropolis on L = 2, q = 2: the stationary marginal of v
    is exp(-beta N (u(v) + P v)) Z_sigma(theta(v)), with
    Z_sigma(theta) = sum exp(beta theta J_eff N_HB_raw + beta J_sigma N_coop)."""
    L, q, beta, J, Js, P, vHB = 2, 2, 1.0, 1.0, 0.5, 1.0, 0.6
    N = L * L
    Jeff = J - P * vHB
    cov, coop = bond_lists(L)
    dig = (np.arange(1 << 16)[:, None] >> np.arange(16)[None, :]) & 1
    hb = (dig[:, cov[:, 0]] == dig[:, cov[:, 1]]).sum(axis=1)
    co = (dig[:, coop[:, 0]] == dig[:, coop[:, 1]]).sum(axis=1)
    Zs = {th: float(np.exp(beta * th * Jeff * hb + beta * Js * co).sum()) for th in (0, 1)}
    hbm = {th: float((hb * np.exp(beta * th * Jeff * hb + beta * Js * co)).sum()) / Zs[th] for th in (0, 1)}
    pts = sorted({1.0, 2.0, 36.0, 60.0} | {36.0 / m for m in range(1, 37) if 36.0 / m > 1.0})

    def f(v, moment):
        th = 1 if v < 2.0 else 0
        w = math.exp(-beta * N * (direct_u(v) + P * v)) * Zs[th]
        return w * (v if moment == "v" else hbm[th] if moment == "hb" else 1.0)
    Z = m_v = m_h = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        Z += integrate.quad(f, a, b, args=("1",), epsabs=0, epsrel=1e-10)[0]
        m_v += integrate.quad(f, a, b, args=("v",), epsabs=0, epsrel=1e-10)[0]
        m_h += integrate.quad(f, a, b, args=("hb",), epsabs=0, epsrel=1e-10)[0]
    v_ex, hb_ex = m_v / Z, m_h / Z
    p = oracle_mod.make_params(L=L, q=q, beta=beta, J=J, Jsigma=Js, P=P, vHB=vHB, v_init=1.25,
                               dv_max=0.15, seed=31, flags=0)
    s, ch = run_series(oracle_mod, p, 120000, "met", keys=("v", "n_hb_raw"))
    assert abs(batch_z(s["v"][2000:], v_ex)) < 4.5, (s["v"].mean(), v_ex)
    assert abs(batch_z(s["n_hb_raw"][2000:], hb_ex)) < 4.5
    o = ch.obs()
    assert 0 < o["vol_accepted"] < o["vol_attempted"] == 120000


def test_counters_and_invariants(oracle_mod):
    for algo in ("met", "sw"):
        p = oracle_mod.params_from_si(300.0, 0.1, L=12, seed=41)
        ch = oracle_mod.Chain(p)
        for _ in range(20):
            (ch.metropolis if algo == "met" else ch.sw)(3)
            o = ch.obs()
            t, hb, co = ch.incremental()
            assert (hb, co) == (o["n_hb_raw"], o["n_coop"])
            N = 144
            assert 0 <= o["n_hb_raw"] <= 2 * N and 0 <= o["n_coop"] <= 6 * N
            assert sum(o["count"]) == 4 * N
            assert o["V"] == pytest.approx(N * o["v"] + 0.6 * o["n_hb"], rel=1e-15)
            assert o["n_hb"] == (o["n_hb_raw"] if o["v"] < 2.0 else 0)
            assert o["step"] == t
        sg = ch.sigma()
        assert sg.max() < 6


def test_gas_phase_has_no_hydrogen_bonds(oracle_mod):
    """theta = 0 (v >= 2): facing pairs carry no energy, so N_HB_raw relaxes
    to the non-interacting 2N/q and N_HB = 0; SW places no covalent bond."""
    L, q = 8, 6
    N = L * L
    for algo in ("met", "sw"):
        p = oracle_mod.params_from_si(300.0, 0.1, L=L, v_init=2.5, seed=43, flags=oracle_mod.NO_VOLUME_MOVE)
        s, ch = run_series(oracle_mod, p, 3000, algo)
        assert abs(batch_z(s["n_hb_raw"][300:], 2 * N / q)) < 4.5
        assert ch.obs()["n_hb"] == 0
        if algo == "sw":
            assert not np.any(ch.mask() & 3)


def test_sw_labels_are_components_of_mask(oracle_mod):
    p = oracle_mod.params_from_si(300.0, 0.1, L=10, seed=45)
    ch = oracle_mod.Chain(p)
    ch.sw(3)
    from tests.test_oracle_ccl import reference_labels
    assert np.array_equal(ch.labels(), reference_labels(10, ch.mask()))


def test_init_is_uniform(oracle_mod):
    p = oracle_mod.params_from_si(300.0, 0.1, L=128, seed=1)
    sg = oracle_mod.Chain(p).sigma()
    counts = np.bincount(sg, minlength=6)
    exp = sg.size / 6
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 25.0                            # 5 d.o.f., p ~ 1e-4
