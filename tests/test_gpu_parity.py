"""GPU parity: libcvf (HIP, gfx950) against the CPU oracle, through the C ABI.

Bond indices, cluster labels and every integer counter must agree bit for
bit; the FP64 volume v to 1e-12 relative (it is bit-exact unless an
exp() rounding difference flips a volume decision, probability ~1e-16 per
move).  Sizes span several workgroup tiles, ragged tails (L not a multiple
of the 256-lane block, odd half-rows) and the degenerate L = 2 lattice.
"""
import hashlib
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

V_RTOL = 1e-12
INT_KEYS = ("step", "n_hb_raw", "n_hb", "n_coop", "count", "met_attempted", "met_accepted",
            "vol_attempted", "vol_accepted")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cvf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_05919_amd import cvf as mod
    mod.lib()
    return mod


def gpu_params(cvf, op):
    """The oracle's parameter record, field by field, as a library record."""
    p = cvf.cvf_params()
    for k, v in op.as_dict().items():
        setattr(p, k, v)
    return p


def check_obs(og, oo, ctx):
    for k in INT_KEYS:
        assert og[k] == oo[k], (ctx, k, og[k], oo[k])
    assert og["consistent"] == 1, ctx
    for k in ("v", "V", "H", "M"):
        assert og[k] == pytest.approx(oo[k], rel=V_RTOL, abs=1e-300), (ctx, k, og[k], oo[k])


def run_pair(cvf, oracle_mod, op, plan, labels=False, algo_mask=3):
    """plan: list of ("met"|"dom"|"sw", n) applied to both; compares after each item."""
    ctx = f"L={op.L} q={op.q} seed={op.seed} beta={op.beta:.6g} P={op.P:.6g} flags={op.flags} plan={plan}"
    say("case " + ctx)
    ch = cvf.Chain(gpu_params(cvf, op), algo_mask)
    oc = oracle_mod.Chain(op)
    assert np.array_equal(ch.sigma.cpu().numpy(), oc.sigma()), ctx + " init"
    for algo, n in plan:
        if algo == "met":
            ch.metropolis(n)
            oc.metropolis(n)
        elif algo == "dom":
            ch.metropolis_domain(n)
            oc.metropolis_domain(n)
        else:
            ch.sw(n)
            oc.sw(n)
        og, oo = ch.obs(), oc.obs()
        check_obs(og, oo, ctx)
        assert np.array_equal(ch.sigma.cpu().numpy(), oc.sigma()), ctx + f" sigma after {algo} {n}"
        if labels and algo == "sw":
            assert np.array_equal(ch.labels().cpu().numpy().view(np.uint32), oc.labels()), ctx + " labels"
    ch.close()
    return oc


@pytest.mark.parametrize("L", [2, 4, 6, 64, 66, 130, 1000, 1026])
def test_init_parity(cvf, oracle_mod, L):
    op = oracle_mod.params_from_si(300.0, 0.1, L=L, seed=1 + L)
    say(f"case init L={L}")
    ch = cvf.Chain(gpu_params(cvf, op), cvf.CVF_ALGO_METROPOLIS)
    oc = oracle_mod.Chain(op)
    assert np.array_equal(ch.sigma.cpu().numpy(), oc.sigma())
    check_obs(ch.obs(), oc.obs(), f"init L={L}")
    ch.close()


@pytest.mark.parametrize("T,P", [(270.0, 0.1), (300.0, 25.0), (330.0, 50.0), (300.0, 3000.0)])
def test_tables_parity(cvf, oracle_mod, T, P):
    op = oracle_mod.params_from_si(T, P, L=4)
    ch = cvf.Chain(gpu_params(cvf, op), cvf.CVF_ALGO_METROPOLIS)
    met_g, sw_g = ch.tables()
    met_o, sw_o = oracle_mod.tables(op)
    assert np.array_equal(met_g, met_o)
    assert np.array_equal(sw_g, sw_o)
    ch.close()


@pytest.mark.parametrize("L,n", [(2, 50), (4, 40), (6, 30), (64, 20), (66, 20), (130, 10), (256, 5), (1026, 2), (2046, 1)])
def test_metropolis_parity(cvf, oracle_mod, L, n):
    op = oracle_mod.params_from_si(300.0, 0.1, L=L, seed=100 + L)
    run_pair(cvf, oracle_mod, op, [("met", 1), ("met", n)])


@pytest.mark.parametrize("L,n", [(2, 50), (4, 40), (6, 20), (64, 10), (66, 10), (130, 5), (256, 3)])
def test_sw_parity(cvf, oracle_mod, L, n):
    op = oracle_mod.params_from_si(300.0, 0.1, L=L, seed=200 + L)
    run_pair(cvf, oracle_mod, op, [("sw", 1), ("sw", n)], labels=True)


@pytest.mark.parametrize("q", [2, 3, 4, 5])
def test_reduced_q_parity(cvf, oracle_mod, q):
    op = oracle_mod.params_from_si(285.0, 25.0, L=34, q=q, seed=300 + q)
    run_pair(cvf, oracle_mod, op, [("met", 7), ("sw", 4), ("met", 3)], labels=True)


def test_negative_jeff_parity(cvf, oracle_mod):
    # J_eff = J - P v_HB < 0 above ~1248 MPa: SW bonds unequal facing pairs
    op = oracle_mod.params_from_si(300.0, 3000.0, L=32, seed=401)
    assert op.J - op.P * op.vHB < 0
    run_pair(cvf, oracle_mod, op, [("met", 5), ("sw", 5)], labels=True)


def test_gas_phase_parity(cvf, oracle_mod):
    op = oracle_mod.params_from_si(300.0, 0.1, L=40, v_init=2.3, dv_max=0.4, seed=402)
    run_pair(cvf, oracle_mod, op, [("met", 10), ("sw", 10)], labels=True)


def test_volume_crossing_theta(cvf, oracle_mod):
    # large volume steps at high T and low P: v wanders across v = 2 (theta flips)
    op = oracle_mod.make_params(L=4, q=6, beta=0.3, J=2.0, Jsigma=0.32, P=0.01, vHB=0.6, v_init=1.9,
                                dv_max=0.5, seed=403, flags=0)
    oc = run_pair(cvf, oracle_mod, op, [("met", 200), ("sw", 200), ("met", 100)], labels=True)
    assert oc.obs()["vol_accepted"] > 50


def test_no_volume_move_and_beta_zero(cvf, oracle_mod):
    op = oracle_mod.params_from_si(300.0, 0.1, L=20, seed=404, flags=oracle_mod.NO_VOLUME_MOVE)
    run_pair(cvf, oracle_mod, op, [("met", 5), ("sw", 5)], labels=True)
    op = oracle_mod.params_from_si(300.0, 0.1, L=20, seed=405)
    op.beta = 0.0
    run_pair(cvf, oracle_mod, op, [("met", 5), ("sw", 5)], labels=True)


def test_mixed_algorithms(cvf, oracle_mod):
    op = oracle_mod.params_from_si(315.0, 50.0, L=48, seed=406)
    run_pair(cvf, oracle_mod, op, [("met", 3), ("sw", 2), ("met", 1), ("sw", 1), ("met", 4)], labels=True)


def test_c1_full_trajectory(cvf, oracle_mod):
    """Plain Metropolis, L = 64, T = 300 K, P = 0.1 MPa, seed 1, 1000 sweeps,
    one volume move per sweep: per-step counters and v for the first 100
    steps, sigma digests every 100 steps."""
    op = oracle_mod.params_from_si(300.0, 0.1, L=64, seed=1)
    say("case C1 L=64 1000 sweeps")
    ch = cvf.Chain(gpu_params(cvf, op), cvf.CVF_ALGO_METROPOLIS)
    oc = oracle_mod.Chain(op)
    for step in range(1, 1001):
        ch.metropolis(1)
        oc.metropolis(1)
        if step <= 100 or step % 100 == 0:
            check_obs(ch.obs(), oc.obs(), f"C1 step {step}")
        if step % 100 == 0:
            dg = hashlib.sha256(ch.sigma.cpu().numpy().tobytes()).hexdigest()
            do = hashlib.sha256(oc.sigma().tobytes()).hexdigest()
            assert dg == do, step
    ch.close()


@pytest.mark.parametrize("T", [270.0, 285.0, 300.0, 315.0, 330.0])
def test_c2_state_points(cvf, oracle_mod, T):
    """L = 1024 Metropolis and L = 256 Swendsen-Wang across 270-330 K at
    0.1 MPa (a few steps each; the oracle bounds the length)."""
    k = int((T - 270.0) / 15.0)
    op = oracle_mod.params_from_si(T, 0.1, L=1024, seed=2 + k)
    run_pair(cvf, oracle_mod, op, [("met", 3)])
    op = oracle_mod.params_from_si(T, 0.1, L=256, seed=7 + k)
    run_pair(cvf, oracle_mod, op, [("sw", 4)], labels=True)


def test_c3_full_size_metropolis(cvf, oracle_mod):
    """L = 4096 (16.8 M molecules, 67 M bond indices), T = 300 K, P = 0.1 MPa:
    two full sweeps in the launch configuration the benchmark times."""
    op = oracle_mod.params_from_si(300.0, 0.1, L=4096, seed=12)
    run_pair(cvf, oracle_mod, op, [("met", 2)])


def test_c3_full_size_sw(cvf, oracle_mod):
    """L = 1414 (~2 M molecules), T = 300 K, P = 50 MPa: two Swendsen-Wang
    steps, labels included."""
    op = oracle_mod.params_from_si(300.0, 50.0, L=1414, seed=17)
    run_pair(cvf, oracle_mod, op, [("sw", 2)], labels=True)


@pytest.mark.parametrize("L,P", [(1602, 25.0), (2048, 0.1)])
def test_sw_parity_more_tiles_than_one_round(cvf, oracle_mod, L, P):
    """More 64 x 16 tiles than the GPU holds at once (2626 and 4096 tiles
    against 2048 resident workgroups), so that the tile-crossing unions pair
    tiles of different dispatch rounds; 1602 leaves a ragged last tile column
    and row."""
    op = oracle_mod.params_from_si(300.0, P, L=L, seed=31)
    run_pair(cvf, oracle_mod, op, [("sw", 2), ("met", 1), ("sw", 1)], labels=True)


def test_determinism(cvf, oracle_mod):
    op = oracle_mod.params_from_si(300.0, 0.1, L=512, seed=77)
    res = []
    for _ in range(2):
        ch = cvf.Chain(gpu_params(cvf, op))
        ch.metropolis(5).sw(5).metropolis(5)
        res.append((ch.sigma.cpu().numpy().copy(), ch.labels().cpu().numpy().copy(), ch.obs()))
        ch.close()
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])
    assert res[0][2] == res[1][2]


def test_error_paths(cvf, oracle_mod):
    import torch
    op = oracle_mod.params_from_si(300.0, 0.1, L=16, seed=5)
    ch = cvf.Chain(gpu_params(cvf, op), cvf.CVF_ALGO_METROPOLIS)     # no SW workspace
    with pytest.raises(cvf.CvfError) as e:
        ch.sw(1)
    assert e.value.code == cvf.CVF_ENOMEM
    with pytest.raises(cvf.CvfError) as e:
        ch.labels()
    assert e.value.code == cvf.CVF_ESTATE
    ch.close()
    ch = cvf.Chain(gpu_params(cvf, op))
    with pytest.raises(cvf.CvfError) as e:
        ch.labels()                     # no SW step yet
    assert e.value.code == cvf.CVF_ESTATE
    with pytest.raises(cvf.CvfError):
        cvf.cvf_metropolis_sweeps(ch.h, -1)
    ch.metropolis(0).sw(0)
    assert ch.obs()["step"] == 0
    ch.close()
    torch.cuda.synchronize()


def test_keep_sigma_resume(cvf, oracle_mod):
    """CVF_KEEP_SIGMA: a chain started from a given configuration counts it
    exactly (the counters of the oracle after set_sigma)."""
    import torch
    op = oracle_mod.params_from_si(300.0, 0.1, L=50, seed=9)
    src = oracle_mod.Chain(op).metropolis(7).sigma()
    p = gpu_params(cvf, op)
    p.flags = cvf.CVF_KEEP_SIGMA
    sig = torch.from_numpy(src.copy()).cuda()
    ch = cvf.Chain(p, sigma=sig)
    assert np.array_equal(ch.sigma.cpu().numpy(), src)
    oc = oracle_mod.Chain(op)
    oc.set_sigma(src)
    og, oo = ch.obs(), oc.obs()
    for k in ("n_hb_raw", "n_coop", "count"):
        assert og[k] == oo[k]
    ch.close()
