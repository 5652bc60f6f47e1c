"""GPU parity of the arm-domain Metropolis sweep (the paper's layered
partition, Sec. II.C) against the oracle, through the C ABI: bond indices and
every counter bit for bit after each block of sweeps, on even and odd
lattices (one-cell last pairs, the 16-bit pair path for L % 4 == 2, the
quad path for L % 4 == 0, several workgroup tiles and ragged tails), mixed with checkerboard sweeps and Swendsen-Wang
steps on even L; odd L rejected by the checkerboard, SW and batch entry
points; and the largest odd and even lattices on sampled cells.
"""
import numpy as np
import pytest

from tests.test_gpu_parity import gpu_params, run_pair, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cvf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_05919_amd import cvf as mod
    mod.lib()
    return mod


@pytest.mark.parametrize("L,n", [(2, 40), (3, 40), (4, 30), (5, 30), (7, 20), (33, 10), (64, 10), (65, 10),
                                 (130, 5), (257, 3), (1025, 1)])
def test_domain_parity(cvf, oracle_mod, L, n):
    op = oracle_mod.params_from_si(300.0, 0.1, L=L, seed=500 + L)
    run_pair(cvf, oracle_mod, op, [("dom", 1), ("dom", n)], algo_mask=cvf.CVF_ALGO_METROPOLIS)


@pytest.mark.parametrize("q", [2, 3, 4, 5])
def test_domain_reduced_q(cvf, oracle_mod, q):
    op = oracle_mod.params_from_si(285.0, 25.0, L=35, q=q, seed=600 + q)
    run_pair(cvf, oracle_mod, op, [("dom", 8)], algo_mask=cvf.CVF_ALGO_METROPOLIS)


def test_domain_mixed_with_checkerboard_and_sw(cvf, oracle_mod):
    op = oracle_mod.params_from_si(315.0, 50.0, L=48, seed=611)
    run_pair(cvf, oracle_mod, op, [("dom", 3), ("met", 2), ("sw", 2), ("dom", 4), ("sw", 1), ("dom", 1)])


def test_domain_gas_phase_and_negative_jeff(cvf, oracle_mod):
    op = oracle_mod.params_from_si(300.0, 0.1, L=41, v_init=2.3, dv_max=0.4, seed=612)
    run_pair(cvf, oracle_mod, op, [("dom", 10)], algo_mask=cvf.CVF_ALGO_METROPOLIS)
    op = oracle_mod.params_from_si(300.0, 3000.0, L=31, seed=613)
    run_pair(cvf, oracle_mod, op, [("dom", 10)], algo_mask=cvf.CVF_ALGO_METROPOLIS)


def test_odd_L_rejected_by_checkerboard_sw_and_batch(cvf, oracle_mod):
    op = oracle_mod.params_from_si(300.0, 0.1, L=9, seed=614)
    ch = cvf.Chain(gpu_params(cvf, op))
    for call in (lambda: ch.metropolis(1), lambda: ch.sw(1), lambda: cvf.Batch([ch])):
        with pytest.raises(cvf.CvfError, match=str(cvf.CVF_EINVAL)):
            call()
    ch.metropolis_domain(2)                       # the chain is untouched by the refusals
    oc = oracle_mod.Chain(op).metropolis_domain(2)
    assert np.array_equal(ch.sigma.cpu().numpy(), oc.sigma())
    ch.close()


def nbr(L, x, y, a):
    return [((x + 1) % L, y), ((x - 1) % L, y), (x, (y + 1) % L), (x, (y - 1) % L)][a]


@pytest.mark.parametrize("L", [32764, 32765, 32766])
def test_domain_max_size_sampled(cvf, oracle_mod, L):
    """One sweep at the largest sizes, without the volume move: a sampled
    cell after pass k is rebuilt from its own state and its facing
    neighbour's after pass k-1 (memoised), back to the initial
    configuration, with the oracle's one-arm moves."""
    import torch
    say(f"case domain max size L={L}")
    op = oracle_mod.params_from_si(300.0, 25.0, L=L, seed=20261, flags=oracle_mod.NO_VOLUME_MOVE)
    met, _ = oracle_mod.tables(op)
    tab = met[1 if op.v_init < 2.0 else 0]
    N = L * L
    ch = cvf.Chain(gpu_params(cvf, op), cvf.CVF_ALGO_METROPOLIS)
    ch.metropolis_domain(1)
    o = ch.obs()
    assert o["consistent"] == 1 and o["met_attempted"] == 4 * N
    order = oracle_mod.domain_order(op, 0)
    memo = {}

    def state(x, y, k):
        key = (x, y, k)
        if key not in memo:
            if k == 0:
                memo[key] = oracle_mod.init_cell(op, x + L * y)
            else:
                a = order[k - 1]
                s = state(x, y, k - 1)
                fx, fy = nbr(L, x, y, a)
                f = int(state(fx, fy, k - 1)[a ^ 1])
                memo[key] = oracle_mod.dom_arm(op, tab, x + L * y, 0, a, s, f)[0]
        return memo[key]

    rng = np.random.default_rng(L)
    pts = [(0, 0), (L - 1, 0), (0, L - 1), (L - 1, L - 1), (L - 2, 3), (1, L - 1)]
    pts += [(int(x), int(y)) for x, y in rng.integers(0, L, size=(300, 2))]
    want = np.array([state(x, y, 4) for x, y in pts])
    idx = torch.tensor([a * N + x + L * y for x, y in pts for a in range(4)], dtype=torch.int64, device="cuda")
    got = ch.sigma[idx].cpu().numpy().reshape(-1, 4)
    assert np.array_equal(got, want), [(pts[i], got[i], want[i]) for i in range(len(pts))
                                       if not np.array_equal(got[i], want[i])][:5]
    ch.close()
    del ch
    torch.cuda.empty_cache()


def test_domain_step_limit_and_zero_sweeps(cvf, oracle_mod):
    """cvf_set_stop stops the arm-domain sweep exactly at its step; zero
    sweeps change nothing."""
    op = oracle_mod.params_from_si(300.0, 25.0, L=21, seed=620)
    ch = cvf.Chain(gpu_params(cvf, op), cvf.CVF_ALGO_METROPOLIS)
    ch.metropolis_domain(0)
    assert ch.obs()["step"] == 0
    ch.set_stop(5)
    ch.metropolis_domain(9)                       # 4 of them are skipped
    oc = oracle_mod.Chain(op).metropolis_domain(5)
    og, oo = ch.obs(), oc.obs()
    assert og["step"] == 5 and og["met_attempted"] == oo["met_attempted"] == 4 * 21 * 21 * 5
    assert np.array_equal(ch.sigma.cpu().numpy(), oc.sigma())
    for k in ("n_hb_raw", "n_coop", "count", "met_accepted", "vol_accepted"):
        assert og[k] == oo[k], k
    ch.close()
