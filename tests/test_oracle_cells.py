"""The oracle's one-cell functions compose to its full sweeps: a Metropolis
sweep rebuilt cell by cell (colour 0, then colour 1 against the updated
neighbours) and a Swendsen-Wang step rebuilt from per-cell bond masks and
per-cluster shifts equal the oracle's own sweep and step.  (The full sweeps
are pinned elsewhere; this pins the cell API that the maximum-size GPU
tests use on sampled cells.)"""
import numpy as np
import pytest


def nbr(L, x, y, a):
    return [((x + 1) % L, y), ((x - 1) % L, y), (x, (y + 1) % L), (x, (y - 1) % L)][a]


@pytest.mark.parametrize("L,P", [(6, 0.1), (10, 50.0)])
def test_metropolis_sweep_from_cells(oracle_mod, L, P):
    p = oracle_mod.params_from_si(285.0, P, L=L, seed=7, flags=oracle_mod.NO_VOLUME_MOVE)
    ch = oracle_mod.Chain(p)
    N = L * L
    s = ch.sigma().reshape(4, L, L).copy()            # [arm][y][x]
    met, _ = oracle_mod.tables(p)
    tab = met[1 if p.v_init < 2.0 else 0]
    for colour in (0, 1):
        new = s.copy()
        for y in range(L):
            for x in range(L):
                if (x + y) % 2 != colour:
                    continue
                f4 = []
                for a in range(4):
                    nx, ny = nbr(L, x, y, a)
                    f4.append(s[a ^ 1, ny, nx])
                s4, _, _, _ = oracle_mod.met_cell(p, tab, x + L * y, 0, s[:, y, x], f4)
                new[:, y, x] = s4
        s = new
    ch.metropolis(1)
    assert np.array_equal(ch.sigma(), s.reshape(4 * N))


def test_sw_step_from_cells(oracle_mod):
    L = 8
    p = oracle_mod.params_from_si(300.0, 0.1, L=L, seed=11, flags=oracle_mod.NO_VOLUME_MOVE)
    ch = oracle_mod.Chain(p)
    N = L * L
    s0 = ch.sigma().copy()
    _, sw = oracle_mod.tables(p)
    ch.sw(1)
    mask = ch.mask()
    for c in range(N):
        x, y = c % L, c // L
        f0 = s0[1 * N + (x + 1) % L + L * y]
        f2 = s0[3 * N + x + L * ((y + 1) % L)]
        assert oracle_mod.sw_cell_mask(p, sw, 1, c, 0, s0[[c, N + c, 2 * N + c, 3 * N + c]], f0, f2) == mask[c]
    lab = ch.labels()
    want = np.array([(int(s0[i]) + oracle_mod.sw_shift(p, int(lab[i]), 0)) % p.q for i in range(4 * N)], np.uint8)
    assert np.array_equal(ch.sigma(), want)
