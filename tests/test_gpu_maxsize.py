"""The largest lattices the library accepts (L up to 32766, 4 L^2 close to
2^32 bond indices), checked on sampled cells against the oracle's one-cell
functions -- a full oracle run at this size would take hours.

Metropolis (no volume move, so a sweep needs no global count): a colour-0
cell moves against its initial neighbours, a colour-1 cell against its
neighbours after their colour-0 moves; both are rebuilt cell by cell from
the oracle's initial configuration and compared bit for bit.  L = 32764
runs the dword-quad kernel, L = 32766 the quad kernel with a two-column last
quad (L % 4 == 2) and, through a batch of one, the column-pair kernel.

Swendsen-Wang: properties that hold at any size, on sampled bond indices:
every label is a root (label[label[i]] == label[i]) not above its index; the
two ends of every link the oracle's bond mask activates carry the same label;
the new bond index equals the old one shifted by the oracle's shift of the
cluster's label; and the incremental counters equal the full recount.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

T_K, P_MPA, SEED = 300.0, 25.0, 20260


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def cvf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_05919_amd import cvf as mod
    mod.lib()
    return mod


def samples(L, n, seed):
    rng = np.random.default_rng(seed)
    pts = [(0, 0), (L - 1, 0), (0, L - 1), (L - 1, L - 1), (1, 0), (0, 1), (L // 2, L - 1), (L - 1, L // 2)]
    pts += [(int(x), int(y)) for x, y in rng.integers(0, L, size=(n, 2))]
    return pts


def nbr(L, x, y, a):
    return [((x + 1) % L, y), ((x - 1) % L, y), (x, (y + 1) % L), (x, (y - 1) % L)][a]


@pytest.mark.parametrize("L,batched", [(32764, False), (32766, False), (32766, True)])
def test_metropolis_max_size_sampled(cvf, oracle_mod, L, batched):
    import torch
    say(f"case metropolis max size L={L} batched={batched}")
    p = cvf.cvf_params_from_si(T_K, P_MPA, L=L, seed=SEED, flags=cvf.CVF_NO_VOLUME_MOVE)
    op = oracle_mod.params_from_si(T_K, P_MPA, L=L, seed=SEED, flags=oracle_mod.NO_VOLUME_MOVE)
    met, _ = oracle_mod.tables(op)
    tab = met[1 if op.v_init < 2.0 else 0]
    N = L * L
    ch = cvf.Chain(p, cvf.CVF_ALGO_METROPOLIS)
    if batched:
        b = cvf.Batch([ch])
        b.metropolis(1)
        b.close()
    else:
        ch.metropolis(1)
    o = ch.obs()
    assert o["consistent"] == 1 and o["met_attempted"] == 4 * N

    def init(x, y):
        return oracle_mod.init_cell(op, x + L * y)

    def colour0(x, y):
        f4 = [init(*nbr(L, x, y, a))[a ^ 1] for a in range(4)]
        return oracle_mod.met_cell(op, tab, x + L * y, 0, init(x, y), f4)[0]

    pts = samples(L, 400, L)
    want = []
    for x, y in pts:
        if (x + y) % 2 == 0:
            want.append(colour0(x, y))
        else:
            f4 = [colour0(*nbr(L, x, y, a))[a ^ 1] for a in range(4)]
            want.append(oracle_mod.met_cell(op, tab, x + L * y, 0, init(x, y), f4)[0])
    idx = torch.tensor([a * N + x + L * y for x, y in pts for a in range(4)], dtype=torch.int64, device="cuda")
    got = ch.sigma[idx].cpu().numpy().reshape(-1, 4)
    assert np.array_equal(got, np.array(want)), [(pts[i], got[i], want[i]) for i in range(len(pts))
                                                 if not np.array_equal(got[i], want[i])][:5]
    ch.close()
    del ch
    torch.cuda.empty_cache()


def test_sw_max_size_properties(cvf, oracle_mod):
    import torch
    L = 32766
    say(f"case sw max size L={L}")
    p = cvf.cvf_params_from_si(T_K, P_MPA, L=L, seed=SEED, flags=cvf.CVF_NO_VOLUME_MOVE)
    op = oracle_mod.params_from_si(T_K, P_MPA, L=L, seed=SEED, flags=oracle_mod.NO_VOLUME_MOVE)
    _, sw = oracle_mod.tables(op)
    theta = 1 if op.v_init < 2.0 else 0
    N = L * L
    ch = cvf.Chain(p, cvf.CVF_ALGO_METROPOLIS | cvf.CVF_ALGO_SW)
    ch.sw(1)
    o = ch.obs()
    assert o["consistent"] == 1
    lab = ch.labels()

    def init(x, y):
        return oracle_mod.init_cell(op, x + L * y)

    pts = samples(L, 300, L + 1)
    idx, pairs = [], []
    for x, y in pts:
        c = x + L * y
        s4 = init(x, y)
        xp, yp = (x + 1) % L, (y + 1) % L
        m = oracle_mod.sw_cell_mask(op, sw, theta, c, 0, s4, init(xp, y)[1], init(x, yp)[3])
        idx += [a * N + c for a in range(4)]
        if m & 1:
            pairs.append((c, N + xp + L * y))
        if m & 2:
            pairs.append((2 * N + c, 3 * N + x + L * yp))
        for l, (a, b) in enumerate([(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]):
            if m >> (2 + l) & 1:
                pairs.append((a * N + c, b * N + c))
    it = torch.tensor(idx, dtype=torch.int64, device="cuda")
    li = lab[it].to(torch.int64) & 0xFFFFFFFF
    l = li.cpu().numpy()
    assert (l <= np.array(idx)).all()
    ll = (lab[li].to(torch.int64) & 0xFFFFFFFF).cpu().numpy()
    assert np.array_equal(ll, l), "labels must be roots"
    if pairs:
        pa = torch.tensor([u for u, _ in pairs], dtype=torch.int64, device="cuda")
        pb = torch.tensor([v for _, v in pairs], dtype=torch.int64, device="cuda")
        assert torch.equal(lab[pa], lab[pb]), "both ends of an active link share the label"
    s_new = ch.sigma[it].cpu().numpy()
    s_old = np.concatenate([init(x, y) for x, y in pts]).reshape(-1, 4)
    want = [(int(s_old[k // 4][k % 4]) + oracle_mod.sw_shift(op, int(l[k]), 0)) % op.q for k in range(len(idx))]
    assert np.array_equal(s_new, np.array(want, dtype=np.uint8))
    del lab
    ch.close()
    del ch
    torch.cuda.empty_cache()
