"""Pins of the oracle's observables: the enthalpy H (Eq. (3)), the volume V
(Eq. (1)) and the order parameter M (Sec. III.A), in the square-lattice model
and in the cubic model with eta.

None of these restates the oracle's own expression.  H and V are checked
through thermodynamic identities of the ensemble the chain samples:
<H> = -d ln Z / d beta and <V> = -(1/beta) d ln Z / dP, with Z built from an
exhaustive enumeration of the L = 2 lattice (square model), a quadrature over
the volume, or the closed forms of the J_sigma = 0 and J_eff = 0 limits
(cubic model), and differentiated numerically.  A term of H that the chain's
weight does not contain (P V dropped, N_HB_raw used in the gas, a wrong sign)
moves the chain's mean away from the derivative by many standard errors.
M is recomputed from the configuration with numpy (bincount over all bond
indices), and a few configurations worked by hand fix every counter.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from tests.test_oracle_chain import batch_z, density_of_states_L2, direct_u

pytestmark = pytest.mark.filterwarnings("ignore")


def _logsumexp(x):
    m = np.max(x)
    return float(m + np.log(np.exp(x - m).sum()))


def _series(ch, step, n, keys):
    out = {k: np.empty(n) for k in keys}
    for i in range(n):
        step(1)
        o = ch.obs()
        for k in keys:
            out[k][i] = o[k]
    return out


# --------------------------------------------------------------------------
# Square lattice: M from the configuration, hand-worked configurations
# --------------------------------------------------------------------------
@pytest.mark.parametrize("algo,L,q", [("met", 6, 6), ("sw", 6, 6), ("dom", 5, 6), ("met", 8, 3)])
def test_counts_and_M_from_the_configuration(oracle_mod, algo, L, q):
    """N_q' is the number of bond indices in state q' and M = max N_q' over
    the number of bond indices (Sec. III.A; four per molecule here)."""
    p = oracle_mod.params_from_si(300.0, 0.1, L=L, q=q, seed=61)
    ch = oracle_mod.Chain(p)
    step = {"met": ch.metropolis, "sw": ch.sw, "dom": ch.metropolis_domain}[algo]
    for _ in range(12):
        step(2)
        s = ch.sigma()
        o = ch.obs()
        cnt = np.bincount(s, minlength=6)
        assert list(cnt) == o["count"]
        assert o["M"] == cnt.max() / s.size


def _l2_config(kind):
    """sigma[a][c] (4 x 4 bond indices of an L = 2 lattice) and its counts,
    worked out by hand.  On L = 2 the +x neighbour of x is x ^ 1 and the +y
    neighbour of y is y ^ 1; cell c = x + 2 y."""
    if kind == "arm":          # sigma = a: four distinct states per cell
        # no two arms of a cell agree (N_coop = 0); arm 0 (state 0) faces an
        # arm 1 (state 1), arm 2 (2) faces an arm 3 (3): N_HB_raw = 0
        s = np.repeat(np.arange(4), 4)
        return s, dict(hb=0, coop=0, count=[4, 4, 4, 4, 0, 0])
    if kind == "axis":         # sigma = a >> 1: arms 0, 1 in state 0, arms 2, 3 in 1
        # pairs (0,1) and (2,3) agree in each cell: N_coop = 2 * 4 = 8;
        # every facing pair joins two arms of one axis: N_HB_raw = 2N = 8
        s = np.repeat(np.array([0, 0, 1, 1]), 4)
        return s, dict(hb=8, coop=8, count=[8, 8, 0, 0, 0, 0])
    if kind == "cell":         # sigma = cell index: all four arms of a cell equal
        # N_coop = 6 per cell = 24; a facing pair joins two different cells,
        # always unequal: N_HB_raw = 0; each state held by 4 bond indices
        s = np.tile(np.arange(4), 4)
        return s, dict(hb=0, coop=24, count=[4, 4, 4, 4, 0, 0])
    if kind == "one":          # a single bond index changed from all-zero:
        # sigma[0][0] = 1 breaks its facing pair (arm 1 of cell 1) and its
        # three pairs in cell 0: N_HB_raw = 8 - 1, N_coop = 24 - 3
        s = np.zeros(16, dtype=np.int64)
        s[0] = 1
        return s, dict(hb=7, coop=21, count=[15, 1, 0, 0, 0, 0])
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["arm", "axis", "cell", "one"])
@pytest.mark.parametrize("v", [1.25, 2.5])
def test_hand_worked_configurations(oracle_mod, kind, v):
    s, ex = _l2_config(kind)
    J, Js, P, vHB = 2.0, 0.32, 0.7, 0.6
    p = oracle_mod.make_params(L=2, q=6, beta=1.0, J=J, Jsigma=Js, P=P, vHB=vHB, v_init=v, dv_max=0.0,
                               seed=1, flags=oracle_mod.NO_VOLUME_MOVE)
    ch = oracle_mod.Chain(p)
    ch.set_sigma(s.astype(np.uint8))
    o = ch.obs()
    liquid = v < 2.0
    assert (o["n_hb_raw"], o["n_coop"], o["count"]) == (ex["hb"], ex["coop"], ex["count"])
    assert o["n_hb"] == (ex["hb"] if liquid else 0)
    n_hb = ex["hb"] if liquid else 0
    # Eq. (2): every molecule's volume is v_iso plus v_HB per half bond, so the
    # sum over the four cells is 4 v + v_HB N_HB
    cell_hb = np.zeros(4)
    for a in range(4):
        for c in range(4):
            x, y = c % 2, c // 2
            nb = (x ^ 1) + 2 * y if a < 2 else x + 2 * (y ^ 1)
            if s[a * 4 + c] == s[(a ^ 1) * 4 + nb]:
                cell_hb[c] += 1
    V_cells = sum(v + vHB * (cell_hb[c] if liquid else 0) / 2 for c in range(4))
    assert o["V"] == pytest.approx(V_cells, rel=1e-14)
    U = 4 * direct_u(v)
    assert o["H"] == pytest.approx(U - J * n_hb - Js * ex["coop"] + P * V_cells, rel=1e-12, abs=1e-12)
    assert o["M"] == max(ex["count"]) / 16


# --------------------------------------------------------------------------
# Square lattice, fixed volume: <H> and <V> against derivatives of the
# exactly enumerated ln Z of L = 2
# --------------------------------------------------------------------------
def _lnZ_L2(q, beta, J, Js, P, vHB, v):
    """ln of the L = 2 partition function at fixed v_iso (no volume move):
    the configuration weight exp(-beta H) with H of Eq. (3), over the density
    of states g[N_HB_raw, N_coop] from exhaustive enumeration."""
    N = 4
    g = density_of_states_L2(q)
    hb = np.arange(g.shape[0])[:, None].astype(np.float64)
    co = np.arange(g.shape[1])[None, :].astype(np.float64)
    th = 1.0 if v < 2.0 else 0.0
    e = N * direct_u(v) - J * th * hb - Js * co + P * (N * v + vHB * th * hb)
    keep = g > 0
    return _logsumexp((np.log(g[keep].astype(np.float64)) - beta * np.broadcast_to(e, g.shape)[keep]))


@pytest.mark.parametrize("v", [1.25, 2.5])
def test_fixed_volume_H_and_V_are_derivatives_of_lnZ(oracle_mod, v):
    q, beta, J, Js, P, vHB = 2, 1.0, 1.0, 0.5, 1.0, 0.6
    p = oracle_mod.make_params(L=2, q=q, beta=beta, J=J, Jsigma=Js, P=P, vHB=vHB, v_init=v, dv_max=0.0,
                               seed=71, flags=oracle_mod.NO_VOLUME_MOVE)
    ch = oracle_mod.Chain(p)
    s = _series(ch, ch.metropolis, 60000, ("H", "V"))
    h = 1e-5
    H_ex = -(_lnZ_L2(q, beta + h, J, Js, P, vHB, v) - _lnZ_L2(q, beta - h, J, Js, P, vHB, v)) / (2 * h)
    V_ex = -(_lnZ_L2(q, beta, J, Js, P + h, vHB, v) - _lnZ_L2(q, beta, J, Js, P - h, vHB, v)) / (2 * h) / beta
    assert abs(batch_z(s["H"][1000:], H_ex)) < 4.5, (s["H"].mean(), H_ex)
    if v < 2.0:
        assert abs(batch_z(s["V"][1000:], V_ex)) < 4.5, (s["V"].mean(), V_ex)
    else:
        # gas: no bond contributes to V, which is then N v in every configuration
        assert V_ex == pytest.approx(4 * v, rel=1e-8)
        assert np.all(s["V"] == 4 * v)


# --------------------------------------------------------------------------
# Square lattice with the volume move: <H>, <V> and <v> against derivatives
# of ln Z from a quadrature over v
# --------------------------------------------------------------------------
def _lnZ_npt_L2(q, beta, J, Js, P, vHB):
    N = 4
    g = density_of_states_L2(q).astype(np.float64)
    hb = np.arange(g.shape[0])[:, None].astype(np.float64)
    co = np.arange(g.shape[1])[None, :].astype(np.float64)
    Zs = {th: float((g * np.exp(beta * th * (J - P * vHB) * hb + beta * Js * co)).sum()) for th in (0, 1)}
    pts = sorted({1.0, 2.0, 36.0, 80.0} | {36.0 / m for m in range(1, 37) if 36.0 / m > 1.0})

    def f(v):
        th = 1 if v < 2.0 else 0
        return math.exp(-beta * N * (direct_u(v) + P * v)) * Zs[th]
    Z = sum(integrate.quad(f, a, b, epsabs=0, epsrel=1e-13, limit=200)[0] for a, b in zip(pts[:-1], pts[1:]))
    return math.log(Z)


def test_npt_H_and_V_are_derivatives_of_lnZ(oracle_mod):
    q, beta, J, Js, P, vHB = 2, 1.0, 1.0, 0.5, 1.0, 0.6
    p = oracle_mod.make_params(L=2, q=q, beta=beta, J=J, Jsigma=Js, P=P, vHB=vHB, v_init=1.25,
                               dv_max=0.15, seed=73, flags=0)
    ch = oracle_mod.Chain(p)
    s = _series(ch, ch.metropolis, 120000, ("H", "V"))
    h = 1e-4
    H_ex = -(_lnZ_npt_L2(q, beta + h, J, Js, P, vHB) - _lnZ_npt_L2(q, beta - h, J, Js, P, vHB)) / (2 * h)
    V_ex = -(_lnZ_npt_L2(q, beta, J, Js, P + h, vHB) - _lnZ_npt_L2(q, beta, J, Js, P - h, vHB)) / (2 * h) / beta
    assert abs(batch_z(s["H"][2000:], H_ex)) < 4.5, (s["H"].mean(), H_ex)
    assert abs(batch_z(s["V"][2000:], V_ex)) < 4.5, (s["V"].mean(), V_ex)


# --------------------------------------------------------------------------
# Cubic lattice with eta
# --------------------------------------------------------------------------
def _p3(oracle_mod, **kw):
    base = dict(L=4, q=6, beta=1.0, J=2.0, Jsigma=0.32, P=0.0, vHB=0.6, v_init=1.25, dv_max=0.0,
                seed=11, flags=oracle_mod.NO_VOLUME_MOVE)
    base.update(kw)
    return oracle_mod.make_params(**base)


def _direct_u3(v):
    a = v ** (1.0 / 3.0)
    n = int(6.0 / a) + 1
    tot = 0.0
    r = np.arange(-n, n + 1)
    i, j, k = np.meshgrid(r, r, r, indexing="ij")
    m = (i * i + j * j + k * k).ravel()
    m = m[m > 0]
    d = a * np.sqrt(m.astype(np.float64))
    d = d[d <= 6.0 * (1 + 1e-12)]
    tot = float((0.5 * 4.0 * (d ** -12 - d ** -6)).sum())
    return tot


def test_cubic_counts_and_M_from_the_configuration(oracle_mod):
    from oracle import cvf3
    for sw in (False, True):
        ch = cvf3.Chain3(oracle_mod.params_from_si(260.0, 0.1, L=4, seed=62))
        for _ in range(6):
            (ch.sw if sw else ch.steps)(2)
            s = ch.sigma()
            o = ch.obs()
            cnt = np.bincount(s, minlength=6)
            assert list(cnt) == o["count"]
            assert o["M"] == cnt.max() / s.size


def _lnZ3_jsigma0(N, q, beta, J, P, vHB, v):
    """J_sigma = 0: every molecule has four eta = 1 edges (App. A), so 2N of
    the 3N edges carry a covalent term and each of them joins two bond
    indices found in no other edge: the sigma sum factorises into 2N facing
    pairs, q (e^{beta theta J_eff} + q - 1) each, times q^{2N} for the bond
    indices on eta = 0 edges, times the (constant) number of eta states."""
    th = 1.0 if v < 2.0 else 0.0
    x = beta * th * (J - P * vHB)
    return -beta * N * (_direct_u3(v) + P * v) + 2 * N * math.log(q * (math.exp(x) + q - 1))


@pytest.mark.parametrize("v", [1.25, 2.5])
def test_cubic_H_and_V_at_jsigma_zero(oracle_mod, v):
    from oracle import cvf3
    L, q, beta, J, P, vHB = 4, 6, 0.6, 2.0, 0.8, 0.6
    N = L ** 3
    p = _p3(oracle_mod, L=L, q=q, beta=beta, J=J, Jsigma=0.0, P=P, vHB=vHB, v_init=v, seed=81)
    ch = cvf3.Chain3(p)
    ch.steps(200)
    s = _series(ch, ch.steps, 3000, ("H", "V"))
    h = 1e-5
    H_ex = -(_lnZ3_jsigma0(N, q, beta + h, J, P, vHB, v) - _lnZ3_jsigma0(N, q, beta - h, J, P, vHB, v)) / (2 * h)
    V_ex = -(_lnZ3_jsigma0(N, q, beta, J, P + h, vHB, v)
             - _lnZ3_jsigma0(N, q, beta, J, P - h, vHB, v)) / (2 * h) / beta
    if v < 2.0:
        assert abs(batch_z(s["H"], H_ex, 20)) < 4.5, (s["H"].mean(), H_ex)
        assert abs(batch_z(s["V"], V_ex, 20)) < 4.5, (s["V"].mean(), V_ex)
    else:
        # gas with J_sigma = 0: H = N (u + P v) and V = N v for every configuration
        assert np.allclose(s["H"], H_ex, rtol=1e-9, atol=1e-9), (s["H"][:3], H_ex)
        assert np.allclose(s["V"], V_ex, rtol=1e-9, atol=1e-9)


def test_cubic_H_at_zero_effective_coupling(oracle_mod):
    """J = P v_HB (J_eff = 0): cells are independent six-arm cliques with
    weight exp(beta J_sigma N_sigma(cell)); ln Z = -beta N (u + P v) +
    N ln sum_cell + const.  The derivative is taken with J_eff held at 0."""
    import itertools
    from oracle import cvf3
    L, q, beta, Js, P, vHB = 4, 6, 1.0, 0.5, 1.0, 0.6
    J = P * vHB
    N = L ** 3
    v = 1.25
    st = np.array(list(itertools.product(range(q), repeat=6)))
    npairs = sum((st[:, a] == st[:, b]).astype(np.float64) for a in range(6) for b in range(a + 1, 6))

    def lnZ(b):
        return -b * N * (_direct_u3(v) + P * v) + N * _logsumexp(b * Js * npairs)
    p = _p3(oracle_mod, L=L, q=q, beta=beta, J=J, Jsigma=Js, P=P, vHB=vHB, v_init=v, seed=82)
    ch = cvf3.Chain3(p)
    ch.steps(200)
    s = _series(ch, ch.steps, 3000, ("H",))
    h = 1e-5
    H_ex = -(lnZ(beta + h) - lnZ(beta - h)) / (2 * h)
    assert abs(batch_z(s["H"], H_ex, 20)) < 4.5, (s["H"].mean(), H_ex)
