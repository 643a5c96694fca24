"""MI355X-native engine for the local problems of the Multiscale Hybrid-Mixed
(MHM) method: assembly, Cholesky factorisation, multi-right-hand-side solves,
FP64 refinement and the skeleton contribution, as hand-written gfx950 HIP
kernels behind the C ABI of ``include/mhm.h``.

``abi`` is the ctypes binding, ``batch`` the host-side layout of a ragged
batch, ``engine`` small drivers over the three calls and the fused call.
Nothing here computes on the CPU.
"""
from . import abi  # noqa: F401
