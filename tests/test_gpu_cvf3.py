"""GPU parity of the cubic-lattice model with eta (volume move, eta moves over
the checkerboard cubes, six arm-domain sigma passes per step) against the
oracle, through the C ABI: sigma, eta and every counter bit for bit after
each block of steps -- tiny lattices (L = 2 wraps every neighbour), several
workgroups with ragged tails, liquid, gas and J_eff < 0 state points,
reduced q, a kept caller state, and the paper's N = 260^3 lattice."""
import numpy as np
import pytest

from tests.test_gpu_parity import gpu_params, say

pytestmark = pytest.mark.gpu

INT_KEYS = ("step", "n_hb_raw", "n_hb", "n_coop", "count", "n_eta0", "met_attempted", "met_accepted",
            "eta_attempted", "eta_accepted", "vol_attempted", "vol_accepted")


@pytest.fixture(scope="module")
def c3():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_05919_amd import cvf, cvf3
    cvf.lib()
    cvf3.lib()
    return cvf3


def compare(ch, oc, ctx):
    assert np.array_equal(ch.sigma.cpu().numpy(), oc.sigma()), ctx + " sigma"
    assert np.array_equal(ch.eta.cpu().numpy(), oc.eta()), ctx + " eta"
    og, oo = ch.obs(), oc.obs()
    for k in INT_KEYS:
        assert og[k] == oo[k], (ctx, k, og[k], oo[k])
    assert og["consistent"] == 1, ctx
    assert og["v"] == oo["v"], (ctx, og["v"], oo["v"])
    for k in ("V", "H", "M"):
        assert og[k] == pytest.approx(oo[k], rel=1e-13, abs=1e-12), (ctx, k)
    return og


def run3(c3, oracle_mod, op, plan, keep=None):
    from oracle import cvf3 as o3
    from paper_2505_05919_amd import cvf
    ctx = f"L={op.L} q={op.q} seed={op.seed} beta={op.beta:.6g} P={op.P:.6g} v0={op.v_init} flags={op.flags}"
    say("case " + ctx)
    oc = o3.Chain3(op)
    if keep is not None:
        import torch
        sig, eta = keep
        oc.set_state(sigma=sig, eta=eta)
        p = gpu_params(cvf, op)
        p.flags |= cvf.CVF_KEEP_SIGMA
        ch = c3.Chain3(p, sigma=torch.from_numpy(sig.copy()).cuda(), eta=torch.from_numpy(eta.copy()).cuda())
    else:
        ch = c3.Chain3(gpu_params(cvf, op))
    compare(ch, oc, ctx + " init")
    done = 0
    for n in plan:
        ch.steps(n)
        oc.steps(n)
        done += n
        og = compare(ch, oc, f"{ctx} after {done}")
    ch.close()
    return og


@pytest.mark.parametrize("L,plan", [(2, [1, 20]), (4, [1, 10]), (6, [3, 6]), (8, [5]), (10, [4]), (16, [3]),
                                    (18, [2]), (36, [2]), (64, [1])])
def test_cvf3_parity(c3, oracle_mod, L, plan):
    op = oracle_mod.params_from_si(300.0, 0.1, L=L, seed=700 + L)
    run3(c3, oracle_mod, op, plan)


@pytest.mark.parametrize("T,P,v0", [(250.0, 100.0, 1.25), (210.0, 0.1, 1.1), (330.0, 0.1, 2.5), (300.0, 1500.0, 1.2),
                                    (400.0, -200.0, 1.9)])
def test_cvf3_state_points(c3, oracle_mod, T, P, v0):
    """Liquid, cold liquid, gas (eta moves always accepted), J_eff < 0
    (P v_HB > J), and a volume that crosses v = 2 during the run."""
    op = oracle_mod.params_from_si(T, P, L=12, seed=int(T) + 3, v_init=v0, dv_max=0.3 if v0 == 1.9 else 0.0125)
    og = run3(c3, oracle_mod, op, [2, 6])
    assert og["n_eta0"] == 12 ** 3


@pytest.mark.parametrize("L", [14, 16])
@pytest.mark.parametrize("q", [2, 3, 4, 5])
def test_cvf3_reduced_q(c3, oracle_mod, q, L):
    """q - 1 = 1, 2, 4 (power-of-two draws, never NONE) and 3 (NONE at the
    top word), on the pair path (L = 14) and the quad path (L = 16)."""
    op = oracle_mod.params_from_si(260.0, 25.0, L=L, q=q, seed=800 + q)
    run3(c3, oracle_mod, op, [4])


def test_cvf3_no_volume_move_and_kept_state(c3, oracle_mod):
    """CVF_KEEP_SIGMA: the chain starts from the caller's sigma and eta (here
    a state the oracle reached after some steps with another seed)."""
    from oracle import cvf3 as o3
    src = o3.Chain3(oracle_mod.params_from_si(280.0, 0.1, L=10, seed=5)).steps(7)
    keep = (src.sigma(), src.eta())
    op = oracle_mod.params_from_si(280.0, 0.1, L=10, seed=6, flags=oracle_mod.NO_VOLUME_MOVE)
    og = run3(c3, oracle_mod, op, [3, 3], keep=keep)
    assert og["vol_attempted"] == 0


def test_cvf3_paper_size(c3, oracle_mod):
    """N = 260^3 = 17 576 000 (the paper's largest Metropolis lattice): init
    and one full step bit for bit."""
    op = oracle_mod.params_from_si(300.0, 0.1, L=260, seed=2026)
    run3(c3, oracle_mod, op, [1])


@pytest.mark.parametrize("L", [1288, 1290])
def test_cvf3_max_size(c3, oracle_mod, L):
    """The largest lattices (N = L^3 < 2^31; 1288 runs the quad pass and the
    two-cube eta kernel, 1290 the pair pass and the one-cube kernel): the
    initial bond indices of sampled cells equal the oracle's definition
    (Philox(c, 0, sub, INIT) words), and after one step the incremental
    counters equal the recount, every sampled molecule has four eta = 1
    edges and all N/4 cubes and 6N bond indices were attempted."""
    import torch
    from paper_2505_05919_amd import cvf
    op = oracle_mod.params_from_si(300.0, 0.1, L=L, seed=4242)
    say(f"case max size L={L}")
    ch = c3.Chain3(gpu_params(cvf, op))
    N = L ** 3
    rng = np.random.default_rng(L)
    cells = np.concatenate([rng.integers(0, N, 300), [0, 1, L - 1, L, N - L * L, N - 2, N - 1]]).astype(np.int64)
    idx = torch.from_numpy(np.concatenate([cells + b * N for b in range(6)])).cuda()
    got = ch.sigma[idx].cpu().numpy().reshape(6, -1)
    for k, c in enumerate(cells):
        w0 = oracle_mod.philox([int(c), 0, 0, 0], op.seed)
        w1 = oracle_mod.philox([int(c), 0, 1, 0], op.seed)
        want = [(int(w) * op.q) >> 32 for w in (w0[0], w0[1], w0[2], w0[3], w1[0], w1[1])]
        assert list(got[:, k]) == want, (L, int(c))
    ch.steps(1)
    o = ch.obs()
    assert o["consistent"] == 1 and o["n_eta0"] == N and sum(o["count"]) == 6 * N
    assert o["met_attempted"] == 6 * N and o["eta_attempted"] == N // 4 and o["step"] == 1
    x, y, z = cells % L, (cells // L) % L, cells // (L * L)
    lower = [((x - 1) % L) + L * (y + L * z), x + L * (((y - 1) % L) + L * z), x + L * (y + L * ((z - 1) % L))]
    eidx = np.concatenate([cells + d * N for d in range(3)] + [lower[d] + d * N for d in range(3)])
    e = ch.eta[torch.from_numpy(eidx.astype(np.int64)).cuda()].cpu().numpy().reshape(6, -1)
    assert (e.sum(axis=0) == 4).all()
    ch.close()
    del ch
    torch.cuda.empty_cache()


# ---------------------------------------------------------------- Swendsen-Wang
def run3_mixed(c3, oracle_mod, op, plan):
    """plan: ("met" | "sw", n) items applied to both; sigma, eta, counters and
    (after SW) the cluster labels compared after each item."""
    from oracle import cvf3 as o3
    from paper_2505_05919_amd import cvf
    ctx = f"L={op.L} q={op.q} seed={op.seed} beta={op.beta:.6g} P={op.P:.6g} v0={op.v_init} plan={plan}"
    say("case " + ctx)
    ch = c3.Chain3(gpu_params(cvf, op), algo_mask=cvf.CVF_ALGO_METROPOLIS | cvf.CVF_ALGO_SW)
    oc = o3.Chain3(op)
    compare(ch, oc, ctx + " init")
    for kind, n in plan:
        if kind == "sw":
            ch.sw(n)
            oc.sw(n)
        else:
            ch.steps(n)
            oc.steps(n)
        og = compare(ch, oc, f"{ctx} after {kind} {n}")
        if kind == "sw":
            assert np.array_equal(ch.labels().cpu().numpy().view(np.uint32), oc.labels()), ctx + " labels"
    ch.close()
    return og


@pytest.mark.parametrize("L,n", [(2, 10), (4, 6), (6, 4), (8, 3), (16, 2), (18, 2), (24, 2), (32, 2), (36, 1)])
def test_cvf3_sw_parity(c3, oracle_mod, L, n):
    op = oracle_mod.params_from_si(230.0, 0.1, L=L, seed=900 + L)
    run3_mixed(c3, oracle_mod, op, [("sw", 1), ("sw", n)])


@pytest.mark.parametrize("T,P,v0", [(195.0, 0.1, 1.1), (330.0, 0.1, 2.5), (300.0, 1500.0, 1.2), (400.0, -200.0, 1.9)])
def test_cvf3_sw_state_points(c3, oracle_mod, T, P, v0):
    """Near-percolating cold liquid, gas (no covalent links), J_eff < 0
    (unequal facing arms bond) and a volume crossing v = 2."""
    op = oracle_mod.params_from_si(T, P, L=10, seed=int(T) + 7, v_init=v0, dv_max=0.3 if v0 == 1.9 else 0.0125)
    run3_mixed(c3, oracle_mod, op, [("sw", 2), ("sw", 4)])


@pytest.mark.parametrize("L", [16, 24])
def test_cvf3_sw_tiled_cold(c3, oracle_mod, L):
    """A cold liquid on tiled lattices (16 x 8 x 8 tiles at L = 16, 8 x 8 x 4
    at L = 24): clusters span many tiles, so most face links join roots that
    a neighbouring link of the same face has already joined."""
    op = oracle_mod.params_from_si(195.0, 0.1, L=L, seed=960 + L, v_init=1.1)
    run3_mixed(c3, oracle_mod, op, [("sw", 1), ("sw", 3), ("met", 1), ("sw", 1)])


@pytest.mark.parametrize("q", [2, 3, 5])
def test_cvf3_sw_reduced_q_mixed(c3, oracle_mod, q):
    op = oracle_mod.params_from_si(240.0, 25.0, L=12, q=q, seed=950 + q)
    run3_mixed(c3, oracle_mod, op, [("sw", 2), ("met", 2), ("sw", 2)])


def test_cvf3_sw_paper_size(c3, oracle_mod):
    """N = 128^3 = 2 097 152, the paper's largest SW lattice: two steps bit
    for bit, labels included."""
    op = oracle_mod.params_from_si(210.0, 0.1, L=128, seed=2048)
    run3_mixed(c3, oracle_mod, op, [("sw", 2)])


def test_cvf3_sw_state_errors(c3, oracle_mod):
    from paper_2505_05919_amd import cvf
    op = oracle_mod.params_from_si(300.0, 0.1, L=4, seed=1)
    ch = c3.Chain3(gpu_params(cvf, op))                      # Metropolis only
    with pytest.raises(cvf.CvfError) as e:
        ch.sw(1)
    assert e.value.code == cvf.CVF_ESTATE
    ch.close()
    ch = c3.Chain3(gpu_params(cvf, op), algo_mask=cvf.CVF_ALGO_SW)
    with pytest.raises(cvf.CvfError) as e:
        ch.labels()                                          # before the first SW step
    assert e.value.code == cvf.CVF_ESTATE
    ch.close()


@pytest.mark.parametrize("algo", ["met", "sw"])
def test_cvf3_state_counts_series(c3, oracle_mod, algo):
    """The per-step N_q' series recorded on the device (the order parameter
    of Sec. III.A) equals the oracle's counts after every step."""
    from oracle import cvf3 as o3
    from paper_2505_05919_amd import autocorr, cvf
    op = oracle_mod.params_from_si(220.0, 0.1, L=6, seed=77)
    ch = c3.Chain3(gpu_params(cvf, op), algo_mask=cvf.CVF_ALGO_METROPOLIS | cvf.CVF_ALGO_SW)
    oc = o3.Chain3(op)
    got = autocorr.record_counts3(c3, ch, ch.steps if algo == "met" else ch.sw, 40)
    want = []
    for _ in range(40):
        (oc.steps if algo == "met" else oc.sw)(1)
        want.append(oc.obs()["count"])
    assert np.array_equal(got, np.asarray(want, dtype=np.int64))
    ch.close()
