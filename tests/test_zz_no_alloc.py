"""The allocation-free Swendsen-Wang entry point (cvf_sw_steps_noalloc)
against the existing path (cvf_init + cvf_sw_steps + cvf_observables) on the
same parameters: sigma bit for bit and every observable, on two calls in a
row -- the second on a smaller lattice, so the fixed scratch array still holds
the first call's larger contents -- and the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cvf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_05919_amd import cvf as mod
    mod.lib()
    return mod


def _reference(cvf, p, nsteps):
    ch = cvf.Chain(p, cvf.CVF_ALGO_METROPOLIS | cvf.CVF_ALGO_SW)
    ch.sw(nsteps)
    o = ch.obs()
    s = ch.sigma.cpu().numpy().copy()
    ch.close()
    return s, o


@pytest.mark.parametrize("sizes", [((512, 300.0, 0.1, 91, 6), (128, 280.0, 25.0, 92, 9))])
def test_noalloc_matches_existing_path(cvf, sizes):
    import torch
    for L, T, P, seed, n in sizes:
        print(f"case noalloc L={L} T={T} P={P} seed={seed} steps={n}", flush=True)
        p = cvf.cvf_params_from_si(T, P, L=L, seed=seed)
        sig = torch.empty(4 * L * L, dtype=torch.uint8, device="cuda")
        o = cvf.cvf_sw_steps_noalloc(p, sig, n)
        s_ref, o_ref = _reference(cvf, p, n)
        assert np.array_equal(sig.cpu().numpy(), s_ref), (L, seed)
        for k in ("step", "n_hb_raw", "n_hb", "n_coop", "count", "met_attempted", "met_accepted",
                  "vol_attempted", "vol_accepted", "consistent"):
            assert o[k] == o_ref[k], (L, k, o[k], o_ref[k])
        for k in ("v", "V", "H", "M"):
            assert o[k] == o_ref[k], (L, k, o[k], o_ref[k])
        assert o["consistent"] == 1 and o["step"] == n


def test_noalloc_keep_sigma_and_limits(cvf):
    import torch
    L = 64
    p = cvf.cvf_params_from_si(300.0, 0.1, L=L, seed=93)
    ch = cvf.Chain(p, cvf.CVF_ALGO_METROPOLIS | cvf.CVF_ALGO_SW)
    ch.metropolis(3)
    start = ch.sigma.clone()          # a configuration the caller keeps
    ch.close()
    pk = cvf.cvf_params_from_si(300.0, 0.1, L=L, seed=93, flags=cvf.CVF_KEEP_SIGMA)
    ref = cvf.Chain(pk, cvf.CVF_ALGO_METROPOLIS | cvf.CVF_ALGO_SW, sigma=start.clone())
    ref.sw(4)
    s2, o2 = ref.sigma.cpu().numpy().copy(), ref.obs()
    ref.close()
    sig = start.clone()
    o = cvf.cvf_sw_steps_noalloc(pk, sig, 4)
    assert np.array_equal(sig.cpu().numpy(), s2)
    assert o["n_hb_raw"] == o2["n_hb_raw"] and o["n_coop"] == o2["n_coop"] and o["v"] == o2["v"]
    big = cvf.cvf_params_from_si(300.0, 0.1, L=514, seed=1)
    with pytest.raises(cvf.CvfError) as e:
        cvf.cvf_sw_steps_noalloc(big, torch.empty(4 * 514 * 514, dtype=torch.uint8, device="cuda"), 1)
    assert e.value.code == cvf.CVF_ENOMEM
    odd = cvf.cvf_params_from_si(300.0, 0.1, L=63, seed=1)
    with pytest.raises(cvf.CvfError) as e:
        cvf.cvf_sw_steps_noalloc(odd, torch.empty(4 * 63 * 63, dtype=torch.uint8, device="cuda"), 1)
    assert e.value.code == cvf.CVF_EINVAL
