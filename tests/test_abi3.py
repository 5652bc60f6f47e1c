"""Host-side checks of the cubic-lattice entry points (no GPU): every function
include/cvf3.h declares is exported, parameters are validated, and the tables
the kernels use equal the oracle's (thresholds from the same rule, the nine
perfect matchings built from the cube's structure vs enumerated)."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def c3():
    from paper_2505_05919_amd import cvf as base
    if not os.path.exists(base.LIB_PATH):
        from paper_2505_05919_amd import _build
        _build.build()
    from paper_2505_05919_amd import cvf3
    cvf3.lib()
    return cvf3


def test_exports_every_declared_symbol(c3):
    text = open(os.path.join(ROOT, "include", "cvf3.h")).read()
    names = sorted(set(re.findall(r"^int\s*(cvf3_\w+)\s*\(", text, flags=re.M)))
    assert "cvf3_sw_steps" in names and "cvf3_labels" in names
    L = c3.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(c3.EXPORTS) == names


def _p(c3, **kw):
    from paper_2505_05919_amd import cvf
    p = cvf.cvf_params_from_si(300.0, 0.1, L=8)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("T,P,q", [(300.0, 0.1, 6), (250.0, 200.0, 6), (330.0, -150.0, 4), (200.0, 1000.0, 3),
                                   (280.0, 5000.0, 2)])
def test_tables_equal_oracle(c3, oracle_mod, T, P, q):
    from oracle import cvf3 as o3
    p = _p(c3, q=q)
    from paper_2505_05919_amd import cvf
    pp = cvf.cvf_params_from_si(T, P, L=8, q=q)
    op = oracle_mod.params_from_si(T, P, L=8, q=q)
    met, eta, match = c3.cvf3_tables(pp)
    omet, oeta = o3.tables(op)
    assert np.array_equal(met, omet)
    assert np.array_equal(eta, oeta)
    assert [int(m) for m in match] == o3.matchings()
    del p


@pytest.mark.parametrize("field,value", [("L", 7), ("L", 0), ("L", 1292), ("q", 7), ("q", 1), ("v_init", 0.5),
                                         ("dv_max", -1.0), ("reserved", 1), ("flags", 8)])
def test_invalid_params_rejected(c3, field, value):
    from paper_2505_05919_amd import cvf
    p = _p(c3, **{field: value})
    with pytest.raises(cvf.CvfError) as e:
        c3.cvf3_workspace_bytes(p)
    assert e.value.code == cvf.CVF_EINVAL


def test_workspace_bytes_small_and_independent_of_L(c3):
    a = c3.cvf3_workspace_bytes(_p(c3, L=2))
    b = c3.cvf3_workspace_bytes(_p(c3, L=1290))
    assert a == b and a < 64 * 1024


def test_sw_workspace_and_limit(c3):
    from paper_2505_05919_amd import cvf
    base = c3.cvf3_workspace_bytes(_p(c3, L=128))
    sw = c3.cvf3_workspace_bytes(_p(c3, L=128), cvf.CVF_ALGO_SW | cvf.CVF_ALGO_METROPOLIS)
    assert sw >= base + 28 * 128 ** 3
    c3.cvf3_workspace_bytes(_p(c3, L=894), cvf.CVF_ALGO_SW)            # 6N < 2^32
    for bad in ((_p(c3, L=896), cvf.CVF_ALGO_SW), (_p(c3, L=8), 4)):
        with pytest.raises(cvf.CvfError) as e:
            c3.cvf3_workspace_bytes(*bad)
        assert e.value.code == cvf.CVF_EINVAL


def test_null_pointers_rejected(c3):
    import ctypes
    from paper_2505_05919_amd import cvf
    p = _p(c3)
    h = ctypes.c_void_p()
    L = c3.lib()
    assert L.cvf3_init(ctypes.byref(p), 1, None, None, None, 0, None, ctypes.byref(h)) == cvf.CVF_EINVAL
    assert L.cvf3_steps(None, 1, None) == cvf.CVF_EINVAL
    assert L.cvf3_sw_steps(None, 1, None) == cvf.CVF_EINVAL
    assert L.cvf3_labels(None, None, None) == cvf.CVF_EINVAL
    assert L.cvf3_state_counts(None, None, None) == cvf.CVF_EINVAL
    assert L.cvf3_observables(None, None, None) == cvf.CVF_EINVAL
    assert L.cvf3_destroy(None) == cvf.CVF_EINVAL
    assert L.cvf3_workspace_bytes(ctypes.byref(p), 1, None) == cvf.CVF_EINVAL


def test_init_rejects_misaligned_and_short_arguments(c3):
    """cvf3_init validates before any device call: misaligned lattice or
    workspace pointers and a short workspace come back as errors."""
    import ctypes
    from paper_2505_05919_amd import cvf
    p = _p(c3, L=8)
    need = c3.cvf3_workspace_bytes(p)
    L = c3.lib()
    h = ctypes.c_void_p()
    ok, odd = ctypes.c_void_p(1 << 20), ctypes.c_void_p((1 << 20) + 2)
    assert L.cvf3_init(ctypes.byref(p), 1, odd, ok, ok, need, None, ctypes.byref(h)) == cvf.CVF_EINVAL
    assert L.cvf3_init(ctypes.byref(p), 1, ok, odd, ok, need, None, ctypes.byref(h)) == cvf.CVF_EINVAL
    assert L.cvf3_init(ctypes.byref(p), 1, ok, ok, ctypes.c_void_p((1 << 20) + 64), need, None,
                       ctypes.byref(h)) == cvf.CVF_EINVAL
    assert L.cvf3_init(ctypes.byref(p), 1, ok, ok, ok, need - 1, None, ctypes.byref(h)) == cvf.CVF_ENOMEM
    assert L.cvf3_init(ctypes.byref(p), 8, ok, ok, ok, need, None, ctypes.byref(h)) == cvf.CVF_EINVAL
    assert not h.value
