"""Host-side checks of libcvf (no GPU): the shared library loads, exports every
function include/cvf.h declares, and its host-only entry points (parameter
conversion, workspace sizing, validation) behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def cvf():
    from paper_2505_05919_amd import cvf as mod
    if not os.path.exists(mod.LIB_PATH):
        from paper_2505_05919_amd import _build
        _build.build()
    mod.lib()
    return mod


def declared_functions():
    text = open(os.path.join(ROOT, "include", "cvf.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(cvf_\w+)\s*\(", text, flags=re.M)))


def test_exports_every_declared_symbol(cvf):
    names = declared_functions()
    assert len(names) >= 12
    L = cvf.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(cvf.EXPORTS) == names


def test_params_from_si_bit_identical_to_oracle(cvf, oracle_mod):
    for T in (270.0, 285.0, 300.0, 315.0, 330.0, 195.0):
        for P in (0.0, 0.1, 25.0, 50.0, 1234.5):
            a = cvf.cvf_params_from_si(T, P).as_dict()
            b = oracle_mod.params_from_si(T, P).as_dict()
            for k, v in b.items():
                assert a[k] == v, (T, P, k)


def test_workspace_bytes(cvf):
    p = cvf.cvf_params_from_si(300.0, 0.1, L=1414)
    met = cvf.cvf_workspace_bytes(p, cvf.CVF_ALGO_METROPOLIS)
    both = cvf.cvf_workspace_bytes(p, cvf.CVF_ALGO_METROPOLIS | cvf.CVF_ALGO_SW)
    N = 1414 * 1414
    tiles = ((1414 + 63) // 64) * ((1414 + 15) // 16)
    assert met < 8192
    # labels 16 B + tile-local roots 8 B + bond mask 1 B per cell; per 64x16
    # tile 80 edge bytes, 160 exchange words and 2 edge counters (728 B)
    assert both - met >= 25 * N + 728 * tiles
    assert both - met < 25 * N + 728 * tiles + 6 * 256


@pytest.mark.parametrize("field,value", [("L", 1), ("L", 0), ("L", 32768), ("q", 1), ("q", 7),
                                         ("beta", -1.0), ("beta", float("inf")), ("v_init", 0.5),
                                         ("dv_max", -0.1), ("flags", 8), ("reserved", 1)])
def test_invalid_params_rejected(cvf, field, value):
    p = cvf.cvf_params_from_si(300.0, 0.1)
    setattr(p, field, value)
    n = ctypes.c_size_t()
    assert cvf.lib().cvf_workspace_bytes(ctypes.byref(p), 1, ctypes.byref(n)) == cvf.CVF_EINVAL
    # validation happens before any device call: fake pointers are never touched
    h = ctypes.c_void_p()
    rc = cvf.lib().cvf_init(ctypes.byref(p), ctypes.c_void_p(4096), ctypes.c_void_p(4096), 1 << 20, None,
                            ctypes.byref(h))
    assert rc == cvf.CVF_EINVAL


def test_odd_L_is_a_valid_parameter(cvf):
    # odd L runs the arm-domain sweep only; the checkerboard sweep, SW steps
    # and batches reject it when called
    p = cvf.cvf_params_from_si(300.0, 0.1, L=1413)
    assert cvf.cvf_workspace_bytes(p, cvf.CVF_ALGO_METROPOLIS) < 8192


def test_init_rejects_small_or_misaligned_workspace(cvf):
    p = cvf.cvf_params_from_si(300.0, 0.1)
    h = ctypes.c_void_p()
    L = cvf.lib()
    assert L.cvf_init(ctypes.byref(p), ctypes.c_void_p(4096), ctypes.c_void_p(4096 + 8), 1 << 20, None,
                      ctypes.byref(h)) == cvf.CVF_EINVAL
    assert L.cvf_init(ctypes.byref(p), ctypes.c_void_p(4096), ctypes.c_void_p(4096), 64, None,
                      ctypes.byref(h)) == cvf.CVF_ENOMEM
    assert L.cvf_init(ctypes.byref(p), None, ctypes.c_void_p(4096), 1 << 20, None,
                      ctypes.byref(h)) == cvf.CVF_EINVAL
    # sigma must be 4-byte aligned (the sweeps move dwords)
    assert L.cvf_init(ctypes.byref(p), ctypes.c_void_p(4096 + 2), ctypes.c_void_p(4096), 1 << 20, None,
                      ctypes.byref(h)) == cvf.CVF_EINVAL


def test_null_state_and_strerror(cvf):
    L = cvf.lib()
    assert L.cvf_metropolis_sweeps(None, 1, None) == cvf.CVF_EINVAL
    assert L.cvf_sw_steps(None, 1, None) == cvf.CVF_EINVAL
    assert L.cvf_destroy(None) == cvf.CVF_EINVAL
    assert L.cvf_metropolis_domain_sweeps(None, 1, None) == cvf.CVF_EINVAL
    assert L.cvf_state_counts(None, ctypes.c_void_p(4096), None) == cvf.CVF_EINVAL
    assert L.cvf_params_from_si(0.0, 0.1, None) == cvf.CVF_EINVAL
    for code in (0, -1, -2, -3, -4, -99):
        assert isinstance(cvf.cvf_strerror(code), str)


def test_struct_layouts_match_header(cvf):
    # cvf_params: 2 int32 + 7 double + uint64 + 2 uint32 = 80 bytes; cvf_obs: 14 int64 + 4 double + 2 int32
    assert ctypes.sizeof(cvf.cvf_params) == 80
    assert ctypes.sizeof(cvf.cvf_obs) == 14 * 8 + 4 * 8 + 8


def test_noalloc_entry_rejects_before_any_device_call(cvf):
    """cvf_sw_steps_noalloc checks its arguments and the size limit of its
    fixed scratch array (L <= 512) before touching the device, so the
    errors come back on a host without a GPU too."""
    import ctypes
    lib = cvf.lib()
    fake = ctypes.c_void_p(1 << 20)                  # aligned, never dereferenced
    o = cvf.cvf_obs()
    big = cvf.cvf_params_from_si(300.0, 0.1, L=514)
    assert lib.cvf_sw_steps_noalloc(ctypes.byref(big), fake, 1, ctypes.byref(o), None) == cvf.CVF_ENOMEM
    odd = cvf.cvf_params_from_si(300.0, 0.1, L=63)
    assert lib.cvf_sw_steps_noalloc(ctypes.byref(odd), fake, 1, ctypes.byref(o), None) == cvf.CVF_EINVAL
    ok = cvf.cvf_params_from_si(300.0, 0.1, L=64)
    assert lib.cvf_sw_steps_noalloc(ctypes.byref(ok), None, 1, ctypes.byref(o), None) == cvf.CVF_EINVAL
    assert lib.cvf_sw_steps_noalloc(ctypes.byref(ok), fake, -1, ctypes.byref(o), None) == cvf.CVF_EINVAL
    assert lib.cvf_sw_steps_noalloc(ctypes.byref(ok), fake, 1, None, None) == cvf.CVF_EINVAL
    neg = cvf.cvf_params_from_si(300.0, 0.1, L=64, Jsigma=-0.1)
    assert lib.cvf_sw_steps_noalloc(ctypes.byref(neg), fake, 1, ctypes.byref(o), None) == cvf.CVF_EINVAL
