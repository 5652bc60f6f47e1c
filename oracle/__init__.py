"""CPU oracle for the CVF water model Monte Carlo (2-D square-lattice reading).

TEST INFRASTRUCTURE ONLY.  A plain single-threaded C implementation
(``cvf_oracle.c``) written from the paper, wrapped with ctypes.  Only the
test-suite, the smoke check and the CPU-baseline leg of ``bench.py`` may import
this package; the HIP library never does, and shares no code with it.

Notation follows the paper: sigma[a][c] are the bond indices of Sec. II.A,
arm a = 0:+x, 1:-x, 2:+y, 3:-y, cell c = x + L*y, flat index a*N + c
(Sec. II.C's plane-major layout).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cvf_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "cvf3_oracle.c")]
_LIB = os.path.join(_HERE, "libcvf_oracle.so")

INIT, VOL, MET, SWB, SWF = 0, 1, 2, 3, 4
NO_VOLUME_MOVE = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction)."""
    newest = max(os.path.getmtime(f) for f in _SRCS + [os.path.join(_HERE, "cvf_oracle.h"),
                                                       os.path.join(_HERE, "cvf3_oracle.h")])
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", *_SRCS, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("q", ctypes.c_int32), ("beta", ctypes.c_double),
                ("J", ctypes.c_double), ("Jsigma", ctypes.c_double), ("P", ctypes.c_double),
                ("vHB", ctypes.c_double), ("v_init", ctypes.c_double), ("dv_max", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32), ("pad_", ctypes.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


class Obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("n_hb_raw", ctypes.c_int64), ("n_hb", ctypes.c_int64),
                ("n_coop", ctypes.c_int64), ("count", ctypes.c_int64 * 6),
                ("met_attempted", ctypes.c_int64), ("met_accepted", ctypes.c_int64),
                ("vol_attempted", ctypes.c_int64), ("vol_accepted", ctypes.c_int64),
                ("v", ctypes.c_double), ("V", ctypes.c_double), ("H", ctypes.c_double),
                ("M", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["count"] = list(self.count)
        return d


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P, u32p, u8p, u64p = ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_uint32), \
            ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_uint64)
        L.ocvf_philox4x32_10.argtypes = [u32p, ctypes.c_uint64, u32p]
        L.ocvf_pick.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.ocvf_pick.restype = ctypes.c_int32
        L.ocvf_r2.argtypes = [ctypes.c_int32]
        L.ocvf_r2.restype = ctypes.c_int32
        L.ocvf_u_lj.argtypes = [ctypes.c_double]
        L.ocvf_u_lj.restype = ctypes.c_double
        L.ocvf_params_from_si.argtypes = [ctypes.c_double, ctypes.c_double, P]
        L.ocvf_tables.argtypes = [P, u32p, u64p]
        L.ocvf_components.argtypes = [ctypes.c_int32, u8p, u32p]
        L.ocvf_init_cell.argtypes = [P, ctypes.c_int64, u8p]
        L.ocvf_met_cell.argtypes = [P, u32p, ctypes.c_int64, ctypes.c_uint32, u8p, u8p,
                                    ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_int64)]
        L.ocvf_sw_cell_mask.argtypes = [P, u64p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, u8p,
                                        ctypes.c_uint8, ctypes.c_uint8]
        L.ocvf_sw_cell_mask.restype = ctypes.c_uint8
        L.ocvf_sw_shift.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32]
        L.ocvf_sw_shift.restype = ctypes.c_int32
        L.ocvf_domain_order.argtypes = [P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_int32)]
        L.ocvf_dom_arm.argtypes = [P, u32p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32, u8p, ctypes.c_uint8,
                                   ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_int64)]
        L.ocvf_create.argtypes = [P]
        L.ocvf_create.restype = ctypes.c_void_p
        L.ocvf_destroy.argtypes = [ctypes.c_void_p]
        L.ocvf_metropolis_sweeps.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.ocvf_metropolis_domain_sweeps.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.ocvf_sw_steps.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.ocvf_observables.argtypes = [ctypes.c_void_p, ctypes.POINTER(Obs)]
        L.ocvf_get_sigma.argtypes = [ctypes.c_void_p, u8p]
        L.ocvf_set_sigma.argtypes = [ctypes.c_void_p, u8p]
        L.ocvf_get_labels.argtypes = [ctypes.c_void_p, u32p]
        L.ocvf_get_mask.argtypes = [ctypes.c_void_p, u8p]
        L.ocvf_incremental.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int64)]
        L.ocvf_incremental.restype = ctypes.c_int64
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def philox(ctr, seed: int) -> np.ndarray:
    """Philox4x32-10 of one 128-bit counter (4 uint32) under a 64-bit key."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib().ocvf_philox4x32_10(_ptr(c, ctypes.c_uint32), ctypes.c_uint64(seed), _ptr(out, ctypes.c_uint32))
    return out


def pick(w: int, k: int) -> int:
    return lib().ocvf_pick(w, k)


def r2(m: int) -> int:
    return lib().ocvf_r2(m)


def u_lj(v: float) -> float:
    return lib().ocvf_u_lj(v)


def params_from_si(T_kelvin: float, P_MPa: float, **over) -> Params:
    p = Params()
    lib().ocvf_params_from_si(T_kelvin, P_MPa, ctypes.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def make_params(**kw) -> Params:
    p = Params()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def tables(p: Params):
    met = np.zeros((2, 3, 7), dtype=np.uint32)
    sw = np.zeros(3, dtype=np.uint64)
    lib().ocvf_tables(ctypes.byref(p), _ptr(met, ctypes.c_uint32), _ptr(sw, ctypes.c_uint64))
    return met, sw


def init_cell(p: Params, c: int) -> np.ndarray:
    """Initial bond indices of cell c (uint8[4])."""
    out = np.zeros(4, dtype=np.uint8)
    lib().ocvf_init_cell(ctypes.byref(p), c, _ptr(out, ctypes.c_uint8))
    return out


def met_cell(p: Params, tab: np.ndarray, c: int, t: int, s4, f4):
    """Metropolis update of the four arms of cell c at step t (tab: uint32[3][7]
    of the current theta).  Returns (new s4, d_hb, d_coop, accepted)."""
    s = np.ascontiguousarray(np.asarray(s4, dtype=np.uint8)).copy()
    f = np.ascontiguousarray(np.asarray(f4, dtype=np.uint8))
    tb = np.ascontiguousarray(np.asarray(tab, dtype=np.uint32))
    dh, dc, na = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    lib().ocvf_met_cell(ctypes.byref(p), _ptr(tb, ctypes.c_uint32), c, t, _ptr(s, ctypes.c_uint8),
                        _ptr(f, ctypes.c_uint8), ctypes.byref(dh), ctypes.byref(dc), ctypes.byref(na))
    return s, dh.value, dc.value, na.value


def sw_cell_mask(p: Params, sw: np.ndarray, theta: int, c: int, t: int, s4, f0: int, f2: int) -> int:
    """Bond mask of cell c at step t."""
    s = np.ascontiguousarray(np.asarray(s4, dtype=np.uint8))
    w = np.ascontiguousarray(np.asarray(sw, dtype=np.uint64))
    return int(lib().ocvf_sw_cell_mask(ctypes.byref(p), _ptr(w, ctypes.c_uint64), theta, c, t,
                                       _ptr(s, ctypes.c_uint8), f0, f2))


def sw_shift(p: Params, root: int, t: int) -> int:
    """Shift of the cluster with minimum index root at step t."""
    return int(lib().ocvf_sw_shift(ctypes.byref(p), root, t))


def domain_order(p: Params, t: int) -> list:
    """Arms of the four passes of the arm-domain sweep at step t."""
    out = (ctypes.c_int32 * 4)()
    lib().ocvf_domain_order(ctypes.byref(p), t, out)
    return list(out)


def dom_arm(p: Params, tab: np.ndarray, c: int, t: int, a: int, s4, facing: int):
    """Arm-domain move of arm a of cell c at step t.  Returns (new s4, d_hb,
    d_coop, accepted)."""
    s = np.ascontiguousarray(np.asarray(s4, dtype=np.uint8)).copy()
    tb = np.ascontiguousarray(np.asarray(tab, dtype=np.uint32))
    dh, dc, na = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    lib().ocvf_dom_arm(ctypes.byref(p), _ptr(tb, ctypes.c_uint32), c, t, a, _ptr(s, ctypes.c_uint8), facing,
                       ctypes.byref(dh), ctypes.byref(dc), ctypes.byref(na))
    return s, dh.value, dc.value, na.value


def components(L: int, mask: np.ndarray) -> np.ndarray:
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    assert m.size == L * L
    lab = np.zeros(4 * L * L, dtype=np.uint32)
    lib().ocvf_components(L, _ptr(m, ctypes.c_uint8), _ptr(lab, ctypes.c_uint32))
    return lab


class Chain:
    """One Markov chain of the oracle: init, volume moves, Metropolis sweeps and
    Swendsen-Wang steps, exactly as defined in the paper's Sec. II.B-D."""

    def __init__(self, p: Params):
        self.p = Params.from_buffer_copy(p)
        self.N = p.L * p.L
        self._s = lib().ocvf_create(ctypes.byref(self.p))

    def __del__(self):
        if getattr(self, "_s", None):
            lib().ocvf_destroy(self._s)
            self._s = None

    def metropolis(self, n: int):
        lib().ocvf_metropolis_sweeps(self._s, n)
        return self

    def sw(self, n: int):
        lib().ocvf_sw_steps(self._s, n)
        return self

    def metropolis_domain(self, n: int):
        lib().ocvf_metropolis_domain_sweeps(self._s, n)
        return self

    def obs(self) -> dict:
        o = Obs()
        lib().ocvf_observables(self._s, ctypes.byref(o))
        return o.as_dict()

    def sigma(self) -> np.ndarray:
        out = np.zeros(4 * self.N, dtype=np.uint8)
        lib().ocvf_get_sigma(self._s, _ptr(out, ctypes.c_uint8))
        return out

    def set_sigma(self, s: np.ndarray):
        a = np.ascontiguousarray(s, dtype=np.uint8)
        assert a.size == 4 * self.N
        lib().ocvf_set_sigma(self._s, _ptr(a, ctypes.c_uint8))

    def labels(self) -> np.ndarray:
        out = np.zeros(4 * self.N, dtype=np.uint32)
        lib().ocvf_get_labels(self._s, _ptr(out, ctypes.c_uint32))
        return out

    def mask(self) -> np.ndarray:
        out = np.zeros(self.N, dtype=np.uint8)
        lib().ocvf_get_mask(self._s, _ptr(out, ctypes.c_uint8))
        return out

    def incremental(self):
        hb, coop = ctypes.c_int64(), ctypes.c_int64()
        t = lib().ocvf_incremental(self._s, ctypes.byref(hb), ctypes.byref(coop))
        return int(t), int(hb.value), int(coop.value)
