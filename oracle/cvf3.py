"""CPU oracle of the CVF model on the cubic lattice with the eta constraint.

TEST INFRASTRUCTURE ONLY (like the rest of this package).  ctypes wrapper of
``cvf3_oracle.c``: sigma[a][c] with arm a = 0:+x 1:-x 2:+y 3:-y 4:+z 5:-z,
cell c = x + L*(y + L*z); eta[d][c] for the edge from c to its +d neighbour.
One step = volume move, eta update over the checkerboard cubes (App. A),
arm-domain Metropolis sweep of sigma (Sec. II.C).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import Params, _ptr, lib as _lib2d

ETA = 7


class Obs3(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("n_hb_raw", ctypes.c_int64), ("n_hb", ctypes.c_int64),
                ("n_coop", ctypes.c_int64), ("count", ctypes.c_int64 * 6), ("n_eta0", ctypes.c_int64),
                ("met_attempted", ctypes.c_int64), ("met_accepted", ctypes.c_int64),
                ("eta_attempted", ctypes.c_int64), ("eta_accepted", ctypes.c_int64),
                ("vol_attempted", ctypes.c_int64), ("vol_accepted", ctypes.c_int64),
                ("v", ctypes.c_double), ("V", ctypes.c_double), ("H", ctypes.c_double),
                ("M", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["count"] = list(self.count)
        return d


_done = False


def lib():
    global _done
    L = _lib2d()
    if not _done:
        P, u8p, u16p, u32p = (ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_uint8),
                              ctypes.POINTER(ctypes.c_uint16), ctypes.POINTER(ctypes.c_uint32))
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.ocvf_r3.argtypes = [ctypes.c_int32]
        L.ocvf_r3.restype = ctypes.c_int32
        L.ocvf3_u_lj.argtypes = [ctypes.c_double]
        L.ocvf3_u_lj.restype = ctypes.c_double
        L.ocvf3_matchings.argtypes = [u16p]
        L.ocvf3_matchings.restype = ctypes.c_int32
        L.ocvf3_tables.argtypes = [P, u32p, u32p]
        L.ocvf3_domain_order.argtypes = [P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_int32)]
        L.ocvf3_create.argtypes = [P]
        L.ocvf3_create.restype = ctypes.c_void_p
        L.ocvf3_destroy.argtypes = [ctypes.c_void_p]
        L.ocvf3_steps.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.ocvf3_observables.argtypes = [ctypes.c_void_p, ctypes.POINTER(Obs3)]
        L.ocvf3_get_sigma.argtypes = [ctypes.c_void_p, u8p]
        L.ocvf3_get_eta.argtypes = [ctypes.c_void_p, u8p]
        L.ocvf3_set_state.argtypes = [ctypes.c_void_p, u8p, u8p]
        L.ocvf3_sw_steps.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.ocvf3_components.argtypes = [ctypes.c_int32, u32p, u32p]
        L.ocvf3_get_labels.argtypes = [ctypes.c_void_p, u32p]
        L.ocvf3_get_mask.argtypes = [ctypes.c_void_p, u32p]
        L.ocvf3_incremental.argtypes = [ctypes.c_void_p, i64p, i64p]
        L.ocvf3_incremental.restype = ctypes.c_int64
        _done = True
    return L


def r3(m: int) -> int:
    return lib().ocvf_r3(m)


def u_lj(v: float) -> float:
    return lib().ocvf3_u_lj(v)


def matchings() -> list:
    out = np.zeros(16, dtype=np.uint16)
    n = lib().ocvf3_matchings(_ptr(out, ctypes.c_uint16))
    return [int(x) for x in out[:n]]


def components(L: int, mask: np.ndarray) -> np.ndarray:
    m = np.ascontiguousarray(mask, dtype=np.uint32)
    assert m.size == L ** 3
    lab = np.zeros(6 * L ** 3, dtype=np.uint32)
    lib().ocvf3_components(L, _ptr(m, ctypes.c_uint32), _ptr(lab, ctypes.c_uint32))
    return lab


def tables(p: Params):
    met = np.zeros((2, 3, 11), dtype=np.uint32)
    eta = np.zeros(9, dtype=np.uint32)
    lib().ocvf3_tables(ctypes.byref(p), _ptr(met, ctypes.c_uint32), _ptr(eta, ctypes.c_uint32))
    return met, eta


def domain_order(p: Params, t: int) -> list:
    out = (ctypes.c_int32 * 6)()
    lib().ocvf3_domain_order(ctypes.byref(p), t, out)
    return list(out)


class Chain3:
    """One Markov chain of the cubic-lattice model with eta (oracle)."""

    def __init__(self, p: Params):
        assert p.L >= 2 and p.L % 2 == 0
        self.p = Params.from_buffer_copy(p)
        self.N = p.L ** 3
        self._s = lib().ocvf3_create(ctypes.byref(self.p))

    def __del__(self):
        if getattr(self, "_s", None):
            lib().ocvf3_destroy(self._s)
            self._s = None

    def steps(self, n: int):
        lib().ocvf3_steps(self._s, n)
        return self

    def sw(self, n: int):
        lib().ocvf3_sw_steps(self._s, n)
        return self

    def labels(self) -> np.ndarray:
        out = np.zeros(6 * self.N, dtype=np.uint32)
        lib().ocvf3_get_labels(self._s, _ptr(out, ctypes.c_uint32))
        return out

    def mask(self) -> np.ndarray:
        out = np.zeros(self.N, dtype=np.uint32)
        lib().ocvf3_get_mask(self._s, _ptr(out, ctypes.c_uint32))
        return out

    def obs(self) -> dict:
        o = Obs3()
        lib().ocvf3_observables(self._s, ctypes.byref(o))
        return o.as_dict()

    def sigma(self) -> np.ndarray:
        out = np.zeros(6 * self.N, dtype=np.uint8)
        lib().ocvf3_get_sigma(self._s, _ptr(out, ctypes.c_uint8))
        return out

    def eta(self) -> np.ndarray:
        out = np.zeros(3 * self.N, dtype=np.uint8)
        lib().ocvf3_get_eta(self._s, _ptr(out, ctypes.c_uint8))
        return out

    def set_state(self, sigma=None, eta=None):
        s = None if sigma is None else np.ascontiguousarray(sigma, dtype=np.uint8)
        e = None if eta is None else np.ascontiguousarray(eta, dtype=np.uint8)
        assert s is None or s.size == 6 * self.N
        assert e is None or e.size == 3 * self.N
        lib().ocvf3_set_state(self._s, None if s is None else _ptr(s, ctypes.c_uint8),
                              None if e is None else _ptr(e, ctypes.c_uint8))

    def incremental(self):
        hb, coop = ctypes.c_int64(), ctypes.c_int64()
        t = lib().ocvf3_incremental(self._s, ctypes.byref(hb), ctypes.byref(coop))
        return int(t), int(hb.value), int(coop.value)
