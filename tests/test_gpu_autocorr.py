"""GPU parity of the recorded order-parameter series (Sec. III.A): the state
counts cvf_state_counts records after every step equal the oracle's counts
after the same step, bit for bit, for checkerboard Metropolis, Swendsen-Wang
and the arm-domain sweep (odd L included); hence M(t), C_M and tau computed
from either series are identical.  The counter also agrees with
cvf_observables and accumulates into its destination."""
import numpy as np
import pytest

from paper_2505_05919_amd import autocorr
from tests.test_gpu_parity import gpu_params, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cvf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_05919_amd import cvf as mod
    mod.lib()
    return mod


@pytest.mark.parametrize("algo,L", [("met", 64), ("sw", 64), ("dom", 64), ("dom", 33), ("met", 130)])
def test_counts_series_parity(cvf, oracle_mod, algo, L):
    say(f"case counts series {algo} L={L}")
    n = 40
    op = oracle_mod.params_from_si(270.0, 0.1, L=L, seed=700 + L)
    ch = cvf.Chain(gpu_params(cvf, op))
    oc = oracle_mod.Chain(op)
    step = {"met": ch.metropolis, "sw": ch.sw, "dom": ch.metropolis_domain}[algo]
    ostep = {"met": oc.metropolis, "sw": oc.sw, "dom": oc.metropolis_domain}[algo]
    got = autocorr.record_counts(cvf, ch, step, n)
    want = []
    for _ in range(n):
        ostep(1)
        want.append(oc.obs()["count"])
    want = np.array(want, dtype=np.int64)
    assert np.array_equal(got, want)
    M_g = autocorr.order_parameter(got, 4 * L * L)
    M_o = autocorr.order_parameter(want, 4 * L * L)
    assert np.array_equal(autocorr.c_m(M_g, 10), autocorr.c_m(M_o, 10))
    ch.close()


def test_counts_match_observables_and_accumulate(cvf, oracle_mod):
    import torch
    op = oracle_mod.params_from_si(300.0, 25.0, L=90, seed=710)
    ch = cvf.Chain(gpu_params(cvf, op))
    ch.metropolis(3)
    buf = torch.zeros(6, dtype=torch.int64, device="cuda")
    cvf.cvf_state_counts(ch.h, buf.data_ptr())
    first = buf.cpu().numpy().copy()
    assert list(first) == list(ch.obs()["count"])
    assert first.sum() == 4 * 90 * 90
    cvf.cvf_state_counts(ch.h, buf.data_ptr())
    assert np.array_equal(buf.cpu().numpy(), 2 * first)
    with pytest.raises(cvf.CvfError):
        cvf.cvf_state_counts(ch.h, buf.data_ptr() + 4)       # not 8-byte aligned
    ch.close()
