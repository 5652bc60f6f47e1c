"""Pins of the cubic-lattice oracle (with eta) against what the paper and the
mathematics fix: sums-of-three-squares counts, a direct lattice sum for U_LJ,
the perfect matchings of the cube graph (App. A's nine configurations), the
eta invariants App. A states, and exact stationary laws of the chain."""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import cvf3

pytestmark = pytest.mark.filterwarnings("ignore")


# r_3(m), m = 0..36: number of integer triples with i^2 + j^2 + k^2 = m
# (OEIS A005875); zero exactly at m = 4^a (8b + 7) by Legendre's theorem.
R3 = [1, 6, 12, 8, 6, 24, 24, 0, 12, 30, 24, 24, 8, 24, 48, 0, 6, 48, 36, 24, 24, 48, 24, 0, 24, 30, 72, 32, 0,
      72, 48, 0, 12, 48, 48, 48, 30]


def test_r3_matches_sum_of_three_squares():
    assert [cvf3.r3(m) for m in range(37)] == R3


@pytest.mark.parametrize("v", [1.0, 1.0001, 1.25, 1.7, 2.0, 3.3, 8.0, 35.9, 216.0, 300.0])
def test_u_lj_equals_direct_lattice_sum(v):
    # Sec. II.A: hard core r0, cutoff 6 r0, cubic cells of side v^(1/3) r0;
    # half of 4[(1/d)^12 - (1/d)^6] per pair, d = v^(1/3) |n|.
    a = v ** (1.0 / 3.0)
    n = int(6.0 / a) + 1
    tot = 0.0
    for i, j, k in itertools.product(range(-n, n + 1), repeat=3):
        m = i * i + j * j + k * k
        if m == 0:
            continue
        d = a * math.sqrt(m)
        if d > 6.0 * (1 + 1e-12):
            continue
        tot += 0.5 * 4.0 * (d ** -12 - d ** -6)
    assert cvf3.u_lj(v) == pytest.approx(tot, rel=1e-11, abs=1e-14)


def test_u_lj_hard_core():
    assert math.isinf(cvf3.u_lj(0.999))
    assert cvf3.u_lj(216.0 * 1.0001) == 0.0          # beyond the cutoff for every shell


# Cube graph Q3: vertices (dx, dy, dz) in {0,1}^3, edges join vertices that
# differ in one coordinate.  Its perfect matchings number nine.
def _cube_edges():
    """Edge e -> its two corner triples, in the edge numbering of the oracle:
    axis d = e // 4, and r = e % 4 places the edge along the two other axes
    (lower-numbered axis in bit 0)."""
    out = []
    for e in range(12):
        d, r = divmod(e, 4)
        others = [ax for ax in range(3) if ax != d]
        lo = [0, 0, 0]
        lo[others[0]] = r & 1
        lo[others[1]] = r >> 1
        hi = list(lo)
        hi[d] = 1
        out.append((tuple(lo), tuple(hi)))
    return out


def test_nine_perfect_matchings():
    ms = cvf3.matchings()
    assert len(ms) == 9 and ms == sorted(set(ms))
    edges = _cube_edges()
    for m in ms:
        deg = {}
        for e, (u, w) in enumerate(edges):
            if m >> e & 1:
                deg[u] = deg.get(u, 0) + 1
                deg[w] = deg.get(w, 0) + 1
        assert len(deg) == 8 and set(deg.values()) == {1}
    # three use one axis only (four parallel edges), six use two axes
    axes = [len({e // 4 for e in range(12) if m >> e & 1}) for m in ms]
    assert sorted(axes) == [1, 1, 1, 2, 2, 2, 2, 2, 2]


def _cubes(L):
    """(cube id -> list of (axis, lower cell)) for the even-corner and
    odd-corner unit cubes, in the oracle's cube numbering."""
    h = L // 2
    cell = lambda x, y, z: (x % L) + L * ((y % L) + L * (z % L))
    cubes = []
    for par in (0, 1):
        for l in range(h):
            for j in range(h):
                for i in range(h):
                    x0, y0, z0 = 2 * i + par, 2 * j + par, 2 * l + par
                    es = []
                    for (u, w) in _cube_edges():
                        d = [a for a in range(3) if u[a] != w[a]][0]
                        es.append((d, cell(x0 + u[0], y0 + u[1], z0 + u[2])))
                    cubes.append(es)
    return cubes


def _params(**kw):
    base = dict(L=4, q=6, beta=1.0, J=2.0, Jsigma=0.32, P=0.0, vHB=0.6, v_init=1.25, dv_max=0.0,
                seed=11, flags=oracle.NO_VOLUME_MOVE)
    base.update(kw)
    return oracle.make_params(**base)


@pytest.mark.parametrize("L", [2, 4, 6])
def test_eta_invariants(L):
    """App. A: every molecule keeps exactly four eta = 1 edges; every cube's
    eta = 0 edges form one of the perfect matchings."""
    ch = cvf3.Chain3(oracle.params_from_si(260.0, 0.1, L=L, seed=5))
    ms = set(cvf3.matchings())
    cubes = _cubes(L)
    N = L ** 3
    for _ in range(4):
        eta = ch.eta().reshape(3, N)
        assert int((eta == 0).sum()) == N == ch.obs()["n_eta0"]
        deg = np.zeros(N, dtype=np.int64)
        for d in range(3):
            nbr = np.arange(N).reshape(L, L, L)
            nbr = np.roll(nbr, -1, axis=2 - d).reshape(-1)    # +d neighbour of each cell
            deg += eta[d]
            np.add.at(deg, nbr, eta[d])
        assert (deg == 4).all()
        for es in cubes:
            mask = sum((1 << e) for e, (d, c) in enumerate(es) if eta[d, c] == 0)
            assert mask in ms
        assert sum(len(es) for es in cubes) == 3 * N
        assert len({(d, c) for es in cubes for (d, c) in es}) == 3 * N     # cubes partition the edges
        ch.steps(3)


def test_incremental_counters_equal_recount():
    ch = cvf3.Chain3(oracle.params_from_si(250.0, 50.0, L=6, seed=8))
    for _ in range(5):
        ch.steps(4)
        t, hb, coop = ch.incremental()
        o = ch.obs()
        assert (hb, coop, t) == (o["n_hb_raw"], o["n_coop"], o["step"])
        assert sum(o["count"]) == 6 * ch.N
        assert o["met_attempted"] == 6 * ch.N * t and o["eta_attempted"] == ch.N // 4 * t


def test_domain_order_is_uniform_permutation():
    p = _params()
    pos = np.zeros((6, 6))
    for t in range(3000):
        o = cvf3.domain_order(p, t)
        assert sorted(o) == list(range(6))
        for i, a in enumerate(o):
            pos[i, a] += 1
    assert np.abs(pos / 3000 - 1 / 6).max() < 0.035


def _run_mean(ch, key, steps, burn=200, every=1):
    ch.steps(burn)
    xs = []
    for _ in range(steps):
        ch.steps(every)
        xs.append(ch.obs()[key])
    x = np.asarray(xs, dtype=np.float64)
    # error of the mean from batch means (20 batches)
    b = x[: len(x) // 20 * 20].reshape(20, -1).mean(axis=1)
    return x.mean(), b.std(ddof=1) / math.sqrt(20)


def test_covalent_bonds_only_on_eta_one_edges():
    """J_sigma = 0: given eta, every edge is independent; an eta = 1 edge is
    bonded with probability e^{bJ}/(e^{bJ} + q - 1) and 2N of the 3N edges
    have eta = 1 (App. A), so <N_HB_raw> = 2N e^{bJ}/(e^{bJ} + q - 1)."""
    p = _params(Jsigma=0.0, beta=0.6, J=2.0, seed=21)
    ch = cvf3.Chain3(p)
    m, err = _run_mean(ch, "n_hb_raw", 3000)
    x = math.exp(0.6 * 2.0)
    expect = 2 * ch.N * x / (x + 5)
    assert abs(m - expect) < 4 * err + 1e-9, (m, expect, err)
    # without the eta mask the mean would be 3N p: far outside the error
    assert abs(3 * ch.N * x / (x + 5) - m) > 20 * err


def test_cooperative_term_matches_single_cell_enumeration():
    """J = 0 (so J_eff = 0 at P = 0): cells are independent, each with weight
    exp(b J_sigma N_sigma(cell)) over the q^6 states of its six arms."""
    p = _params(J=0.0, Jsigma=0.5, beta=1.0, seed=22)
    ch = cvf3.Chain3(p)
    m, err = _run_mean(ch, "n_coop", 3000)
    s = np.array(list(itertools.product(range(6), repeat=6)))
    npairs = sum((s[:, a] == s[:, b]).astype(np.int64) for a in range(6) for b in range(a + 1, 6))
    w = np.exp(0.5 * npairs)
    expect = ch.N * float((w * npairs).sum() / w.sum())
    assert abs(m - expect) < 4 * err, (m, expect, err)


def _frozen_sigma_chain(theta_liquid, seed):
    """sigma frozen: q = 2, every cell's six arms equal, J_sigma so large that
    any single-arm move (dc = -5) is rejected; the eta moves then sample
    P(eta) ~ exp(b J_eff sum_e eta_e delta_e) cube by cube."""
    L = 4
    p = _params(q=2, J=2.0, Jsigma=40.0, beta=1.0, seed=seed, v_init=1.25 if theta_liquid else 2.5)
    ch = cvf3.Chain3(p)
    N = L ** 3
    rng = np.random.default_rng(seed)
    cellv = rng.integers(0, 2, N).astype(np.uint8)
    ch.set_state(sigma=np.tile(cellv, 6))
    return ch, cellv, L, N


def test_eta_moves_sample_the_boltzmann_weight():
    ch, cellv, L, N = _frozen_sigma_chain(True, 31)
    ms = cvf3.matchings()
    expect = 0.0
    for es in _cubes(L):
        nbrs = []
        for d, c in es:
            x, y, z = c % L, (c // L) % L, c // (L * L)
            o = [x, y, z]
            o[d] = (o[d] + 1) % L
            nbrs.append(o[0] + L * (o[1] + L * o[2]))
        delta = np.array([cellv[c] == cellv[o] for (d, c), o in zip(es, nbrs)], dtype=np.float64)
        nb = np.array([sum(delta[e] for e in range(12) if not (m >> e & 1)) for m in ms])
        w = np.exp(1.0 * 2.0 * nb)
        expect += float((w * nb).sum() / w.sum())
    m, err = _run_mean(ch, "n_hb_raw", 4000, burn=50)
    assert np.array_equal(ch.sigma(), np.tile(cellv, 6))            # sigma stayed frozen
    assert abs(m - expect) < 4 * err + 1e-9, (m, expect, err)


def test_eta_moves_in_the_gas_are_uniform():
    """Gas (v >= 2): eta does not enter H, every proposal is accepted, so each
    cube's configuration is uniform over the nine."""
    ch, cellv, L, N = _frozen_sigma_chain(False, 32)
    ms = cvf3.matchings()
    cubes = _cubes(L)
    hist = np.zeros(9)
    for _ in range(600):
        ch.steps(1)
        eta = ch.eta().reshape(3, N)
        for es in cubes:
            mask = sum((1 << e) for e, (d, c) in enumerate(es) if eta[d, c] == 0)
            hist[ms.index(mask)] += 1
    f = hist / hist.sum()
    assert np.abs(f - 1 / 9).max() < 0.02
    o = ch.obs()
    assert o["eta_accepted"] == o["eta_attempted"] - (o["eta_attempted"] - o["eta_accepted"])
    assert o["n_hb"] == 0


def test_volume_move_samples_npt_density():
    """J = J_sigma = v_HB = 0: v alone has density ~ exp(-b N (u(v) + P v)) on
    v >= 1 (symmetric proposals, Sec. II.B); compare <v> with quadrature."""
    beta, P, L = 1.0, 1.5, 2
    N = L ** 3
    p = _params(L=L, J=0.0, Jsigma=0.0, vHB=0.0, P=P, beta=beta, v_init=1.3, dv_max=0.08, flags=0, seed=41)
    ch = cvf3.Chain3(p)
    m, err = _run_mean(ch, "v", 40000, burn=2000)
    v = np.linspace(1.0, 4.0, 30001)
    f = np.array([-beta * N * (cvf3.u_lj(x) + P * x) for x in v])
    w = np.exp(f - f.max())
    expect = float((w * v).sum() / w.sum())
    assert abs(m - expect) < 4 * err + 1e-4, (m, expect, err)


# ---------------------------------------------------------------- Swendsen-Wang
PAIRS = [(a, b) for a in range(6) for b in range(a + 1, 6)]


@pytest.mark.parametrize("L,density", [(2, 0.3), (4, 0.15), (4, 0.5), (6, 0.08)])
def test_sw_components_against_scipy(L, density):
    """Clusters of the 6N bond indices under random 18-bit link masks equal
    scipy's connected components, each labelled by its smallest flat index."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    N = L ** 3
    rng = np.random.default_rng(L * 100 + int(density * 100))
    bits = rng.random((N, 18)) < density
    mask = (bits * (1 << np.arange(18))).sum(axis=1).astype(np.uint32)
    rows, cols = [], []
    for c in range(N):
        x, y, z = c % L, (c // L) % L, c // (L * L)
        for d in range(3):
            if bits[c, d]:
                o = [x, y, z]
                o[d] = (o[d] + 1) % L
                rows.append((2 * d) * N + c)
                cols.append((2 * d + 1) * N + o[0] + L * (o[1] + L * o[2]))
        for l, (a, b) in enumerate(PAIRS):
            if bits[c, 3 + l]:
                rows.append(a * N + c)
                cols.append(b * N + c)
    g = coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(6 * N, 6 * N))
    _, comp = connected_components(g, directed=False)
    mins = {}
    for i, k in enumerate(comp):
        mins.setdefault(k, i)
    expect = np.array([mins[k] for k in comp], dtype=np.uint32)
    assert np.array_equal(cvf3.components(L, mask), expect)


def test_sw_closed_form_covalent():
    """J_sigma = 0: <N_HB_raw> = 2N e^{bJ}/(e^{bJ} + q - 1) under SW as well."""
    ch = cvf3.Chain3(_params(Jsigma=0.0, beta=0.6, J=2.0, seed=51))
    m, err = _run_mean_sw(ch, "n_hb_raw", 2000)
    x = math.exp(0.6 * 2.0)
    assert abs(m - 2 * ch.N * x / (x + 5)) < 4 * err + 1e-9


def test_sw_cooperative_enumeration():
    ch = cvf3.Chain3(_params(J=0.0, Jsigma=0.5, beta=1.0, seed=52))
    m, err = _run_mean_sw(ch, "n_coop", 2000)
    s = np.array(list(itertools.product(range(6), repeat=6)))
    npairs = sum((s[:, a] == s[:, b]).astype(np.int64) for a in range(6) for b in range(a + 1, 6))
    w = np.exp(0.5 * npairs)
    assert abs(m - ch.N * float((w * npairs).sum() / w.sum())) < 4 * err


def test_sw_agrees_with_metropolis():
    """Both updates sample Eq. (3)'s weight: at the paper's parameters (cold
    liquid, J_eff > 0, eta moving) their <N_HB_raw> and <N_sigma> agree."""
    p = oracle.params_from_si(250.0, 0.1, L=4, seed=53, flags=oracle.NO_VOLUME_MOVE)
    res = {}
    for kind in ("met", "sw"):
        for key in ("n_hb_raw", "n_coop"):
            ch = cvf3.Chain3(p)
            res[kind, key] = _run_mean_sw(ch, key, 3000) if kind == "sw" else _run_mean(ch, key, 3000)
    for key in ("n_hb_raw", "n_coop"):
        (a, ea), (b, eb) = res["met", key], res["sw", key]
        assert abs(a - b) < 4 * math.hypot(ea, eb) + 1e-9, (key, a, b, ea, eb)


def test_sw_step_keeps_invariants():
    ch = cvf3.Chain3(oracle.params_from_si(230.0, 0.1, L=4, seed=54))
    for _ in range(5):
        ch.sw(2)
        t, hb, coop = ch.incremental()
        o = ch.obs()
        assert (hb, coop) == (o["n_hb_raw"], o["n_coop"]) and o["n_eta0"] == ch.N
        lab = ch.labels()
        assert (lab <= np.arange(6 * ch.N)).all()
        assert (lab[lab] == lab).all()                           # labels are roots


def _run_mean_sw(ch, key, steps, burn=200):
    ch.sw(burn)
    xs = []
    for _ in range(steps):
        ch.sw(1)
        xs.append(ch.obs()[key])
    x = np.asarray(xs, dtype=np.float64)
    b = x[: len(x) // 20 * 20].reshape(20, -1).mean(axis=1)
    return x.mean(), b.std(ddof=1) / math.sqrt(20)
