"""ctypes binding of the cubic-lattice model with eta (include/cvf3.h):
argument marshalling only, names of the C entry points.

Device buffers are torch tensors on the GPU; streams default to torch's
current stream.  There is no fallback when libcvf.so is missing.
"""
from __future__ import annotations

import ctypes

import numpy as np

from .cvf import CVF_ALGO_METROPOLIS, CVF_ALGO_SW, CvfError, _check, _devptr, _stream, cvf_params, lib as _lib

CVF3_MAX_L = 1290
(CVF3_K_VOLUME, CVF3_K_ETA, CVF3_K_PASS, CVF3_K_SW_BONDS, CVF3_K_SW_UNION, CVF3_K_SW_FLIP,
 CVF3_K_COUNT) = range(7)

EXPORTS = ["cvf3_workspace_bytes", "cvf3_tables", "cvf3_init", "cvf3_steps", "cvf3_sw_steps", "cvf3_labels",
           "cvf3_state_counts", "cvf3_observables", "cvf3_timing_enable", "cvf3_kernel_times", "cvf3_destroy"]


class cvf3_obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("n_hb_raw", ctypes.c_int64), ("n_hb", ctypes.c_int64),
                ("n_coop", ctypes.c_int64), ("count", ctypes.c_int64 * 6), ("n_eta0", ctypes.c_int64),
                ("met_attempted", ctypes.c_int64), ("met_accepted", ctypes.c_int64),
                ("eta_attempted", ctypes.c_int64), ("eta_accepted", ctypes.c_int64),
                ("vol_attempted", ctypes.c_int64), ("vol_accepted", ctypes.c_int64),
                ("v", ctypes.c_double), ("V", ctypes.c_double), ("H", ctypes.c_double),
                ("M", ctypes.c_double), ("consistent", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}
        d["count"] = list(self.count)
        return d


_done = False


def lib():
    global _done
    L = _lib()
    if not _done:
        vp, P = ctypes.c_void_p, ctypes.POINTER(cvf_params)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.cvf3_workspace_bytes.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
        L.cvf3_tables.argtypes = [P, u32p, u32p, u32p]
        L.cvf3_init.argtypes = [P, ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.cvf3_steps.argtypes = [vp, ctypes.c_int64, vp]
        L.cvf3_sw_steps.argtypes = [vp, ctypes.c_int64, vp]
        L.cvf3_labels.argtypes = [vp, vp, vp]
        L.cvf3_state_counts.argtypes = [vp, vp, vp]
        L.cvf3_observables.argtypes = [vp, ctypes.POINTER(cvf3_obs), vp]
        L.cvf3_timing_enable.argtypes = [vp, ctypes.c_int]
        L.cvf3_kernel_times.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_double)]
        L.cvf3_destroy.argtypes = [vp]
        for name in EXPORTS:
            getattr(L, name).restype = ctypes.c_int
        _done = True
    return L


def cvf3_workspace_bytes(p: cvf_params, algo_mask: int = CVF_ALGO_METROPOLIS) -> int:
    n = ctypes.c_size_t()
    _check("cvf3_workspace_bytes", lib().cvf3_workspace_bytes(ctypes.byref(p), algo_mask, ctypes.byref(n)))
    return n.value


def cvf3_tables(p: cvf_params):
    """(met uint32[2][3][11], eta uint32[9], matchings uint32[9]) as the kernels use them."""
    met = np.zeros((2, 3, 11), dtype=np.uint32)
    eta = np.zeros(9, dtype=np.uint32)
    match = np.zeros(9, dtype=np.uint32)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    _check("cvf3_tables", lib().cvf3_tables(ctypes.byref(p), met.ctypes.data_as(u32p), eta.ctypes.data_as(u32p),
                                            match.ctypes.data_as(u32p)))
    return met, eta, match


def cvf3_init(p: cvf_params, sigma, eta, work, stream=None, algo_mask: int = CVF_ALGO_METROPOLIS):
    N = p.L ** 3
    sp, _ = _devptr(sigma, "torch.uint8", 6 * N)
    ep, _ = _devptr(eta, "torch.uint8", 3 * N)
    wp, wn = _devptr(work, "torch.uint8", 1)
    h = ctypes.c_void_p()
    _check("cvf3_init", lib().cvf3_init(ctypes.byref(p), algo_mask, sp, ep, wp, wn, _stream(stream), ctypes.byref(h)))
    return h


def cvf3_steps(h, nsteps: int, stream=None):
    _check("cvf3_steps", lib().cvf3_steps(h, nsteps, _stream(stream)))


def cvf3_sw_steps(h, nsteps: int, stream=None):
    _check("cvf3_sw_steps", lib().cvf3_sw_steps(h, nsteps, _stream(stream)))


def cvf3_labels(h, out, stream=None):
    """Labels of the last SW step into `out` (a GPU int32 tensor of 6N; the
    values are uint32 cluster minima, read them with .view(torch.uint32)
    or numpy .view(np.uint32))."""
    op, _ = _devptr(out, "torch.int32", out.numel() * 4)
    _check("cvf3_labels", lib().cvf3_labels(h, op, _stream(stream)))
    return out


def cvf3_state_counts(h, d_counts: int, stream=None):
    """Add N_q' of the current sigma into the 6 int64 at device address d_counts."""
    _check("cvf3_state_counts", lib().cvf3_state_counts(h, ctypes.c_void_p(d_counts), _stream(stream)))


def cvf3_observables(h, stream=None) -> dict:
    o = cvf3_obs()
    _check("cvf3_observables", lib().cvf3_observables(h, ctypes.byref(o), _stream(stream)))
    return o.as_dict()


def cvf3_timing_enable(h, enable: bool):
    _check("cvf3_timing_enable", lib().cvf3_timing_enable(h, 1 if enable else 0))


def cvf3_kernel_times(h, kind: int):
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _check("cvf3_kernel_times", lib().cvf3_kernel_times(h, kind, ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def cvf3_destroy(h):
    _check("cvf3_destroy", lib().cvf3_destroy(h))


class Chain3:
    """Owner of one cubic-lattice chain's device buffers (sigma 6N, eta 3N,
    workspace) and its library handle."""

    def __init__(self, p: cvf_params, stream=None, sigma=None, eta=None, algo_mask: int = CVF_ALGO_METROPOLIS):
        import torch
        self.p = cvf_params.from_buffer_copy(p)
        self.N = p.L ** 3
        self.sigma = sigma if sigma is not None else torch.empty(6 * self.N, dtype=torch.uint8, device="cuda")
        self.eta = eta if eta is not None else torch.empty(3 * self.N, dtype=torch.uint8, device="cuda")
        self.work = torch.empty(cvf3_workspace_bytes(self.p, algo_mask), dtype=torch.uint8, device="cuda")
        self.stream = stream
        if stream is not None:
            # the kernels use these buffers on that stream: their blocks are
            # not handed out again before the stream has passed them
            ts = stream if isinstance(stream, torch.cuda.Stream) else torch.cuda.ExternalStream(int(stream))
            for t in (self.sigma, self.eta, self.work):
                t.record_stream(ts)
        self.h = cvf3_init(self.p, self.sigma, self.eta, self.work, stream, algo_mask)

    def steps(self, n):
        cvf3_steps(self.h, n, self.stream)
        return self

    def sw(self, n):
        cvf3_sw_steps(self.h, n, self.stream)
        return self

    def labels(self):
        import torch
        out = torch.empty(6 * self.N, dtype=torch.int32, device=self.sigma.device)
        return cvf3_labels(self.h, out, self.stream)

    def obs(self):
        return cvf3_observables(self.h, self.stream)

    def close(self):
        if getattr(self, "h", None) is not None:
            cvf3_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["CvfError", "Chain3", "cvf3_obs"] + EXPORTS
