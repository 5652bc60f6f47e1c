"""MI355X-native Monte Carlo hot path of the CVF water model.

The compute path is libcvf.so (hand-written HIP kernels for gfx950 behind a
C ABI, declared in include/cvf.h); ``paper_2505_05919_amd.cvf`` is its thin
ctypes binding with the same function names.  PyTorch only provides device
memory and streams.
"""
from . import cvf  # noqa: F401

__all__ = ["cvf"]
