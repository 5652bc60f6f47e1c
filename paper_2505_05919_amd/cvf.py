"""ctypes binding of libcvf (include/cvf.h): argument marshalling only.

Every function has the name of its C entry point and forwards to it; errors
come back as ``CvfError``.  Device buffers are torch tensors on the GPU
(their ``data_ptr()`` is passed), streams default to torch's current stream.
The library must be built (``__graft_entry__.build()``); there is no
fallback of any kind when it is missing.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcvf.so")

CVF_OK, CVF_EINVAL, CVF_ENOMEM, CVF_EHIP, CVF_ESTATE = 0, -1, -2, -3, -4
CVF_ALGO_METROPOLIS, CVF_ALGO_SW = 1, 2
CVF_NO_VOLUME_MOVE, CVF_KEEP_SIGMA = 1, 2
(CVF_K_VOLUME, CVF_K_MET_SWEEP, CVF_K_SW_BONDS, CVF_K_SW_UNION, CVF_K_SW_FLIP,
 CVF_K_RECOUNT, CVF_K_MET_DOMAIN, CVF_K_COUNT) = range(8)

EXPORTS = ["cvf_params_from_si", "cvf_workspace_bytes", "cvf_init", "cvf_metropolis_sweeps",
           "cvf_metropolis_domain_sweeps", "cvf_state_counts",
           "cvf_sw_steps", "cvf_observables", "cvf_labels", "cvf_tables", "cvf_timing_enable",
           "cvf_kernel_times", "cvf_destroy", "cvf_strerror", "cvf_set_stop", "cvf_batch_desc_bytes", "cvf_batch_create",
           "cvf_batch_set_rows", "cvf_batch_metropolis_sweeps", "cvf_batch_sw_steps", "cvf_batch_autotune",
           "cvf_batch_destroy", "cvf_sw_steps_noalloc", "cvf_observables_async", "cvf_batch_create_async"]


class CvfError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed: {code} ({cvf_strerror(code)})")
        self.code = code


class cvf_params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("q", ctypes.c_int32), ("beta", ctypes.c_double),
                ("J", ctypes.c_double), ("Jsigma", ctypes.c_double), ("P", ctypes.c_double),
                ("vHB", ctypes.c_double), ("v_init", ctypes.c_double), ("dv_max", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class cvf_obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("n_hb_raw", ctypes.c_int64), ("n_hb", ctypes.c_int64),
                ("n_coop", ctypes.c_int64), ("count", ctypes.c_int64 * 6),
                ("met_attempted", ctypes.c_int64), ("met_accepted", ctypes.c_int64),
                ("vol_attempted", ctypes.c_int64), ("vol_accepted", ctypes.c_int64),
                ("v", ctypes.c_double), ("V", ctypes.c_double), ("H", ctypes.c_double),
                ("M", ctypes.c_double), ("consistent", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}
        d["count"] = list(self.count)
        return d


_lib = None


def lib():
    """Load libcvf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, P = ctypes.c_void_p, ctypes.POINTER(cvf_params)
        L.cvf_params_from_si.argtypes = [ctypes.c_double, ctypes.c_double, P]
        L.cvf_workspace_bytes.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
        L.cvf_init.argtypes = [P, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.cvf_metropolis_sweeps.argtypes = [vp, ctypes.c_int64, vp]
        L.cvf_metropolis_domain_sweeps.argtypes = [vp, ctypes.c_int64, vp]
        L.cvf_state_counts.argtypes = [vp, vp, vp]
        L.cvf_sw_steps.argtypes = [vp, ctypes.c_int64, vp]
        L.cvf_observables.argtypes = [vp, ctypes.POINTER(cvf_obs), vp]
        L.cvf_observables_async.argtypes = [vp, vp, vp]
        L.cvf_labels.argtypes = [vp, vp, vp]
        L.cvf_set_stop.argtypes = [vp, ctypes.c_int64, vp]
        L.cvf_tables.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)]
        L.cvf_timing_enable.argtypes = [vp, ctypes.c_int]
        L.cvf_kernel_times.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_double)]
        L.cvf_destroy.argtypes = [vp]
        L.cvf_batch_desc_bytes.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
        L.cvf_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, vp, ctypes.c_size_t, vp,
                                       ctypes.POINTER(vp)]
        L.cvf_batch_create_async.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, vp, ctypes.c_size_t, vp,
                                             ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.cvf_batch_set_rows.argtypes = [vp, ctypes.c_int32, vp]
        L.cvf_batch_metropolis_sweeps.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, vp]
        L.cvf_batch_sw_steps.argtypes = [vp, ctypes.c_int64, vp]
        L.cvf_batch_autotune.argtypes = [vp, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_int32)]
        L.cvf_batch_destroy.argtypes = [vp]
        L.cvf_sw_steps_noalloc.argtypes = [P, vp, ctypes.c_int64, ctypes.POINTER(cvf_obs), vp]
        L.cvf_strerror.argtypes = [ctypes.c_int]
        L.cvf_strerror.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name != "cvf_strerror":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(fn, code):
    if code != CVF_OK:
        raise CvfError(fn, code)


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _devptr(t, dtype_name, min_bytes):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("device buffers must be contiguous GPU tensors")
    if str(t.dtype) != dtype_name:
        raise ValueError(f"expected {dtype_name}, got {t.dtype}")
    nbytes = t.numel() * t.element_size()
    if nbytes < min_bytes:
        raise ValueError(f"buffer of {nbytes} bytes, need {min_bytes}")
    return ctypes.c_void_p(t.data_ptr()), nbytes


def cvf_strerror(code: int) -> str:
    return lib().cvf_strerror(code).decode()


def cvf_params_from_si(T_kelvin: float, P_MPa: float, **override) -> cvf_params:
    p = cvf_params()
    _check("cvf_params_from_si", lib().cvf_params_from_si(T_kelvin, P_MPa, ctypes.byref(p)))
    for k, v in override.items():
        setattr(p, k, v)
    return p


def cvf_workspace_bytes(p: cvf_params, algo_mask: int) -> int:
    n = ctypes.c_size_t()
    _check("cvf_workspace_bytes", lib().cvf_workspace_bytes(ctypes.byref(p), algo_mask, ctypes.byref(n)))
    return n.value


def cvf_init(p: cvf_params, sigma, work, stream=None) -> ctypes.c_void_p:
    N = p.L * p.L
    sp, _ = _devptr(sigma, "torch.uint8", 4 * N)
    wp, wbytes = _devptr(work, "torch.uint8", 1)
    h = ctypes.c_void_p()
    _check("cvf_init", lib().cvf_init(ctypes.byref(p), sp, wp, wbytes, _stream(stream), ctypes.byref(h)))
    return h


def cvf_metropolis_sweeps(st, nsweeps: int, stream=None):
    _check("cvf_metropolis_sweeps", lib().cvf_metropolis_sweeps(st, nsweeps, _stream(stream)))


def cvf_metropolis_domain_sweeps(st, nsweeps: int, stream=None):
    _check("cvf_metropolis_domain_sweeps", lib().cvf_metropolis_domain_sweeps(st, nsweeps, _stream(stream)))


def cvf_state_counts(st, d_counts, stream=None):
    """Add the six state counts N_q' of the current sigma to the int64[6]
    at device address d_counts (an int, e.g. a tensor's data_ptr())."""
    _check("cvf_state_counts", lib().cvf_state_counts(st, ctypes.c_void_p(d_counts), _stream(stream)))


def cvf_sw_steps(st, nsteps: int, stream=None):
    _check("cvf_sw_steps", lib().cvf_sw_steps(st, nsteps, _stream(stream)))


def cvf_sw_steps_noalloc(p: cvf_params, sigma, nsteps: int, stream=None) -> dict:
    """A fresh chain over sigma (uint8 GPU tensor of 4 L^2 bytes), nsteps
    Swendsen-Wang steps and its observables, with the library's fixed
    scratch array as workspace (L <= 512); synchronises the stream."""
    sp, _ = _devptr(sigma, "torch.uint8", 4 * p.L * p.L)
    o = cvf_obs()
    _check("cvf_sw_steps_noalloc",
           lib().cvf_sw_steps_noalloc(ctypes.byref(p), sp, nsteps, ctypes.byref(o), _stream(stream)))
    return o.as_dict()


def cvf_observables(st, stream=None) -> dict:
    o = cvf_obs()
    _check("cvf_observables", lib().cvf_observables(st, ctypes.byref(o), _stream(stream)))
    return o.as_dict()


def cvf_observables_async(st, out_ptr: int, stream=None):
    """Enqueue the observables record into out_ptr (device or pinned host
    memory, 8-byte aligned; read it as cvf_obs.from_address once the stream
    has passed this call)."""
    _check("cvf_observables_async", lib().cvf_observables_async(st, ctypes.c_void_p(out_ptr), _stream(stream)))


def cvf_labels(st, out, stream=None):
    op, _ = _devptr(out, "torch.int32", 4)
    _check("cvf_labels", lib().cvf_labels(st, op, _stream(stream)))
    return out


def cvf_set_stop(st, stop_at: int, stream=None):
    _check("cvf_set_stop", lib().cvf_set_stop(st, stop_at, _stream(stream)))


def cvf_tables(st):
    import numpy as np
    met = np.zeros((2, 3, 7), dtype=np.uint32)
    sw = np.zeros(3, dtype=np.uint64)
    _check("cvf_tables", lib().cvf_tables(st, met.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                          sw.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    return met, sw


def cvf_timing_enable(st, enable: bool):
    _check("cvf_timing_enable", lib().cvf_timing_enable(st, 1 if enable else 0))


def cvf_kernel_times(st, kind: int):
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _check("cvf_kernel_times", lib().cvf_kernel_times(st, kind, ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def cvf_destroy(st):
    _check("cvf_destroy", lib().cvf_destroy(st))


def cvf_batch_desc_bytes(count: int) -> int:
    n = ctypes.c_size_t()
    _check("cvf_batch_desc_bytes", lib().cvf_batch_desc_bytes(count, ctypes.byref(n)))
    return n.value


def cvf_batch_create(handles, desc, stream=None) -> ctypes.c_void_p:
    arr = (ctypes.c_void_p * len(handles))(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    dp, nbytes = _devptr(desc, "torch.uint8", 1)
    b = ctypes.c_void_p()
    _check("cvf_batch_create", lib().cvf_batch_create(arr, len(handles), dp, nbytes, _stream(stream), ctypes.byref(b)))
    return b


def cvf_batch_create_async(handles, desc, staging, stream=None) -> ctypes.c_void_p:
    """cvf_batch_create without waiting: staging is a pinned host uint8 tensor
    of at least desc.numel() bytes, kept unchanged until the stream has passed
    the upload."""
    arr = (ctypes.c_void_p * len(handles))(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    dp, nbytes = _devptr(desc, "torch.uint8", 1)
    if not staging.is_pinned() or staging.numel() < nbytes:
        raise CvfError("cvf_batch_create_async", CVF_EINVAL)
    b = ctypes.c_void_p()
    _check("cvf_batch_create_async", lib().cvf_batch_create_async(arr, len(handles), dp, nbytes,
                                                                  ctypes.c_void_p(staging.data_ptr()),
                                                                  staging.numel(), _stream(stream),
                                                                  ctypes.byref(b)))
    return b


def cvf_batch_set_rows(b, rows: int, stream=None):
    _check("cvf_batch_set_rows", lib().cvf_batch_set_rows(b, rows, _stream(stream)))


def cvf_batch_metropolis_sweeps(b, nsweeps: int, graph_block: int = 0, stream=None):
    _check("cvf_batch_metropolis_sweeps", lib().cvf_batch_metropolis_sweeps(b, nsweeps, graph_block, _stream(stream)))


def cvf_batch_sw_steps(b, nsteps: int, stream=None):
    _check("cvf_batch_sw_steps", lib().cvf_batch_sw_steps(b, nsteps, _stream(stream)))


def cvf_batch_autotune(b, sweeps: int, stream=None) -> int:
    r = ctypes.c_int32()
    _check("cvf_batch_autotune", lib().cvf_batch_autotune(b, sweeps, _stream(stream), ctypes.byref(r)))
    return r.value


def cvf_batch_destroy(b):
    _check("cvf_batch_destroy", lib().cvf_batch_destroy(b))


class Batch:
    """Owner of a batch's descriptor buffer; the chains stay owned by their
    Chain objects (which must outlive the batch)."""

    def __init__(self, chains, stream=None, nowait=False):
        """nowait: upload the descriptor table from a pinned staging buffer
        (kept with the batch) without waiting for earlier work on stream."""
        import torch
        self.chains = list(chains)
        nbytes = cvf_batch_desc_bytes(len(self.chains))
        self.desc = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.stream = stream
        self.uploaded = None
        ts = (torch.cuda.current_stream() if stream is None else
              stream if isinstance(stream, torch.cuda.Stream) else torch.cuda.ExternalStream(int(stream)))
        # the kernels read desc on that stream: its block is not handed out
        # again before the stream has passed them
        self.desc.record_stream(ts)
        if nowait:
            self.staging = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
            self.h = cvf_batch_create_async([c.h for c in self.chains], self.desc, self.staging, stream)
            # the pinned staging buffer is read by a copy on the stream that
            # the host allocator does not know of: close() waits for it
            self.uploaded = torch.cuda.Event()
            self.uploaded.record(ts)
        else:
            self.h = cvf_batch_create([c.h for c in self.chains], self.desc, stream)

    def metropolis(self, n, graph_block=0):
        cvf_batch_metropolis_sweeps(self.h, n, graph_block, self.stream)
        return self

    def sw(self, n):
        cvf_batch_sw_steps(self.h, n, self.stream)
        return self

    def set_rows(self, rows):
        cvf_batch_set_rows(self.h, rows, self.stream)

    def autotune(self, sweeps=3):
        return cvf_batch_autotune(self.h, sweeps, self.stream)

    def close(self):
        """Destroys the handle; with nowait, first waits until the descriptor
        upload has read the staging buffer (long done in normal use)."""
        if getattr(self, "uploaded", None) is not None:
            self.uploaded.synchronize()
            self.uploaded = None
        if getattr(self, "h", None) is not None:
            cvf_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Chain:
    """Convenience owner of one chain's device buffers (sigma, workspace) and
    its library handle; every method forwards to the C entry point."""

    def __init__(self, p: cvf_params, algo_mask: int = CVF_ALGO_METROPOLIS | CVF_ALGO_SW,
                 stream=None, sigma=None):
        import torch
        self.p = cvf_params.from_buffer_copy(p)
        self.N = p.L * p.L
        self.sigma = sigma if sigma is not None else torch.empty(4 * self.N, dtype=torch.uint8, device="cuda")
        self.work = torch.empty(cvf_workspace_bytes(self.p, algo_mask), dtype=torch.uint8, device="cuda")
        self.stream = stream
        if stream is not None:
            # the kernels use both buffers on that stream: their blocks are
            # not handed out again before the stream has passed them
            ts = stream if isinstance(stream, torch.cuda.Stream) else torch.cuda.ExternalStream(int(stream))
            self.sigma.record_stream(ts)
            self.work.record_stream(ts)
        self.h = cvf_init(self.p, self.sigma, self.work, stream)

    def metropolis(self, n):
        cvf_metropolis_sweeps(self.h, n, self.stream)
        return self

    def metropolis_domain(self, n):
        cvf_metropolis_domain_sweeps(self.h, n, self.stream)
        return self

    def sw(self, n):
        cvf_sw_steps(self.h, n, self.stream)
        return self

    def obs(self):
        return cvf_observables(self.h, self.stream)

    def labels(self):
        import torch
        out = torch.empty(4 * self.N, dtype=torch.int32, device=self.sigma.device)
        return cvf_labels(self.h, out, self.stream)

    def tables(self):
        return cvf_tables(self.h)

    def set_stop(self, stop_at):
        cvf_set_stop(self.h, stop_at, self.stream)
        return self

    def close(self):
        if getattr(self, "h", None) is not None:
            cvf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
