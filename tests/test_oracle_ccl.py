"""Pins for the oracle's cluster labelling (Sec. II.D, step 3; Table II).

Labels must be the minimum flat index of each connected component of the
sigma graph.  Checked against scipy's connected_components on an edge list the
test builds itself from the bond-mask definition, against a 2-D transcription
of the worked example of Table II, and against the structural properties any
min-root labelling has.
"""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

PAIRS = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def reference_labels(L, mask):
    N = L * L
    rows, cols = [], []
    for c in range(N):
        x, y = c % L, c // L
        m = int(mask[c])
        if m & 1:
            rows.append(0 * N + c); cols.append(1 * N + (x + 1) % L + L * y)
        if m & 2:
            rows.append(2 * N + c); cols.append(3 * N + x + L * ((y + 1) % L))
        for l, (a, b) in enumerate(PAIRS):
            if m >> (2 + l) & 1:
                rows.append(a * N + c); cols.append(b * N + c)
    V = 4 * N
    g = coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(V, V))
    ncomp, comp = connected_components(g, directed=False)
    mins = np.full(ncomp, V, dtype=np.int64)
    np.minimum.at(mins, comp, np.arange(V))
    return mins[comp].astype(np.uint32)


@pytest.mark.parametrize("L,density,seed", [(2, 0.5, 0), (4, 0.3, 1), (6, 0.7, 2), (16, 0.2, 3),
                                            (16, 0.6, 4), (32, 0.9, 5), (64, 0.45, 6)])
def test_components_match_scipy(oracle_mod, L, density, seed):
    rng = np.random.default_rng(seed)
    bits = rng.random((L * L, 8)) < density
    mask = (bits * (1 << np.arange(8))).sum(axis=1).astype(np.uint8)
    got = oracle_mod.components(L, mask)
    assert np.array_equal(got, reference_labels(L, mask))


def test_components_properties(oracle_mod):
    L = 32
    rng = np.random.default_rng(11)
    mask = rng.integers(0, 256, L * L).astype(np.uint8)
    lab = oracle_mod.components(L, mask).astype(np.int64)
    idx = np.arange(4 * L * L)
    assert np.all(lab <= idx)
    assert np.array_equal(lab[lab], lab)


def test_table2_topology_in_2d(oracle_mod):
    """Table II's cluster, 3-D N = 64 -> 2-D L = 4 (N = 16), z -> y:
    sigma {64, 0, 65, 257, 337, 17, 82} become {16, 0, 17, 33, 53, 5, 22};
    covalent (0,65) (257,337) (17,82) -> (0,17) (33,53) (5,22);
    cooperative pairs in cells 0, 1, 17 -> cells 0, 1, 5.  The converged
    label of the whole cluster is its minimum index, 0."""
    L, N = 4, 16
    mask = np.zeros(N, dtype=np.uint8)
    mask[0] |= 1                        # arm 0 of cell 0 -- arm 1 of cell 1   (0, 17)
    mask[0] |= 1 << (2 + 0)             # cell 0 pair (0,1)                    (0, 16)
    mask[1] |= 2                        # arm 2 of cell 1 -- arm 3 of cell 5   (33, 53)
    mask[1] |= 1 << (2 + 3)             # cell 1 pair (1,2)                    (17, 33)
    mask[5] |= 1                        # arm 0 of cell 5 -- arm 1 of cell 6   (5, 22)
    mask[5] |= 1 << (2 + 2)             # cell 5 pair (0,3)                    (5, 53)
    lab = oracle_mod.components(L, mask)
    cluster = [16, 0, 17, 33, 53, 5, 22]
    assert all(lab[i] == 0 for i in cluster)
    others = [i for i in range(4 * N) if i not in cluster]
    assert all(lab[i] == i for i in others)


def test_empty_and_full_masks(oracle_mod):
    L = 8
    N = L * L
    lab = oracle_mod.components(L, np.zeros(N, dtype=np.uint8))
    assert np.array_equal(lab, np.arange(4 * N, dtype=np.uint32))
    lab = oracle_mod.components(L, np.full(N, 255, dtype=np.uint8))
    assert np.all(lab == 0)
