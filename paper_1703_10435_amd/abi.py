"""ctypes binding of ``libmhm.so`` (declared in ``include/mhm.h``).

Argument marshalling only: every step of the local-problem path runs in the
library's HIP kernels.  Importing this module does not touch the GPU; the
first call that needs the library loads it and raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmhm.so")

MHM_OK, MHM_E_ARG, MHM_E_NOMEM, MHM_E_DEVICE, MHM_E_UNSUPPORTED = 0, 1, 2, 3, 4
MHM_FP64, MHM_FP32_IR = 0, 1
MHM_S_LIMIT, MHM_L_LIMIT, MHM_P_LIMIT = 64, 4, 16

INFO_OK, INFO_IR_FALLBACK, INFO_BAD_DESC, INFO_TOO_LARGE = 0, -1, -2, -3

EXPORTS = (
    "mhm_create", "mhm_destroy", "mhm_set_stream", "mhm_last_error", "mhm_sync", "mhm_workspace_bytes",
    "mhm_local_assemble", "mhm_local_factor_solve", "mhm_skeleton_contrib", "mhm_local_batch_run",
    "mhm_autotune", "mhm_tune_report", "mhm_graph_create", "mhm_graph_launch", "mhm_graph_destroy",
    "mhm_factor_bytes", "mhm_local_batch_run_cached", "mhm_skeleton_scatter", "mhm_reconstruct",
    "mhm_local_source_step", "mhm_skeleton_solve", "mhm_set_option", "mhm_local_batch_run_noalloc",
    "mhm_class_times", "mhm_source_hash",
)

# Context options (mhm_set_option)
(MHM_OPT_REFINE64, MHM_OPT_NO_RR, MHM_OPT_NO_LL, MHM_OPT_LL_OCC2, MHM_OPT_LL_NW16, MHM_OPT_LL_PW, MHM_OPT_RR_OCC,
 MHM_OPT_CLASS_TIMING, MHM_OPT_CONCURRENT_CLASSES) = range(9)
OPTION_NAMES = {"refine64": MHM_OPT_REFINE64, "no_rr": MHM_OPT_NO_RR, "no_ll": MHM_OPT_NO_LL,
                "ll_occ2": MHM_OPT_LL_OCC2, "ll_nw16": MHM_OPT_LL_NW16, "ll_pw": MHM_OPT_LL_PW,
                "rr_occ": MHM_OPT_RR_OCC, "class_timing": MHM_OPT_CLASS_TIMING,
                "concurrent_classes": MHM_OPT_CONCURRENT_CLASSES}


class mhm_batch(ctypes.Structure):
    _fields_ = [
        ("n_elem", ctypes.c_int32), ("s_max", ctypes.c_int32), ("l_max", ctypes.c_int32),
        ("s_min", ctypes.c_int32),
        ("s", ctypes.c_void_p), ("l", ctypes.c_void_p), ("vert", ctypes.c_void_p),
        ("sigma", ctypes.c_void_p), ("flip", ctypes.c_void_p), ("kappa", ctypes.c_void_p),
        ("f", ctypes.c_void_p), ("tri_off", ctypes.c_void_p), ("mat_off", ctypes.c_void_p),
        ("rhs_off", ctypes.c_void_p), ("node_off", ctypes.c_void_p),
        ("tri_total", ctypes.c_int64), ("mat_total", ctypes.c_int64), ("rhs_total", ctypes.c_int64),
        ("node_total", ctypes.c_int64),
        ("m", ctypes.c_void_p), ("p_max", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class MhmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mhm status {status}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (once).  Raises FileNotFoundError when it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is not built; run `python -m paper_1703_10435_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64p = ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p
    bp = ctypes.POINTER(mhm_batch)
    sig = {
        "mhm_create": (i32, [ctypes.POINTER(vp), i32, vp]),
        "mhm_destroy": (i32, [vp]),
        "mhm_set_stream": (i32, [vp, vp]),
        "mhm_set_option": (i32, [vp, i32, i32]),
        "mhm_class_times": (i32, [vp, vp, vp, i32]),
        "mhm_last_error": (ctypes.c_char_p, [vp]),
        "mhm_source_hash": (ctypes.c_char_p, []),
        "mhm_sync": (i32, [vp]),
        "mhm_workspace_bytes": (ctypes.c_size_t, [vp, bp, i32]),
        "mhm_local_assemble": (i32, [vp, bp, vp, vp, vp, vp, i64p]),
        "mhm_local_factor_solve": (i32, [vp, bp, i32, vp, vp, vp, vp, vp, i32]),
        "mhm_skeleton_contrib": (i32, [vp, bp, vp, vp, vp, vp, vp, vp]),
        "mhm_local_batch_run": (i32, [vp, bp, i32, vp, vp, vp, vp, vp, vp, vp, i32]),
        "mhm_local_batch_run_noalloc": (i32, [vp, bp, i32, vp, vp, vp, vp, vp, vp, vp, i32]),
        "mhm_autotune": (i32, [vp, bp, i32, vp, vp, vp, vp, vp, vp, vp, i32]),
        "mhm_tune_report": (ctypes.c_size_t, [vp, ctypes.c_char_p, ctypes.c_size_t]),
        "mhm_graph_create": (i32, [vp, bp, i32, vp, vp, vp, vp, vp, vp, vp, i32, ctypes.POINTER(vp)]),
        "mhm_graph_launch": (i32, [vp]),
        "mhm_graph_destroy": (i32, [vp]),
        "mhm_factor_bytes": (ctypes.c_size_t, [i32, i32]),
        "mhm_local_batch_run_cached": (i32, [vp, bp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32]),
        "mhm_skeleton_scatter": (i32, [vp, bp] + [vp] * 8 + [i32] + [vp] * 4),
        "mhm_reconstruct": (i32, [vp, bp, vp, vp, vp, vp, i32, vp, vp]),
        "mhm_local_source_step": (i32, [vp, bp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32]),
        "mhm_skeleton_solve": (i32, [vp, i32, i32, i32, vp, vp, vp, vp, vp, ctypes.c_double, i32,
                                     ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def factor_bytes(s: int, prec: int) -> int:
    """Device bytes of one element's stored factor (mhm_factor_bytes)."""
    return int(load().mhm_factor_bytes(s, prec))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    """An ``mhm_ctx`` bound to a device and a torch HIP stream."""

    def __init__(self, device: int = 0, stream=None, **options):
        """``options``: context options by name (``refine64``, ``no_rr``,
        ``no_ll``, ``ll_occ2``, ``ll_nw16``, ``ll_pw``, ``rr_occ``; see
        mhm_set_option)."""
        import torch
        lib = load()
        self.lib = lib
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        st = lib.mhm_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if st != MHM_OK:
            raise MhmError(st, "mhm_create: " + lib.mhm_last_error(None).decode())
        self.h = h
        for name, value in options.items():
            self.set_option(name, value)

    def set_option(self, option, value: int):
        """mhm_set_option; ``option`` is an MHM_OPT_* value or its name."""
        opt = OPTION_NAMES[option] if isinstance(option, str) else int(option)
        self._check(self.lib.mhm_set_option(self.h, opt, int(value)))

    def set_stream(self, stream):
        self.stream = stream
        self._check(self.lib.mhm_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)))

    def _check(self, st):
        if st != MHM_OK:
            raise MhmError(st, self.lib.mhm_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.mhm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------- the C ABI calls
    def sync(self):
        self._check(self.lib.mhm_sync(self.h))

    def workspace_bytes(self, batch, prec: int) -> int:
        return int(self.lib.mhm_workspace_bytes(self.h, ctypes.byref(batch.desc), prec))

    def local_assemble(self, batch, Ahat, Btil, c, area, info):
        self._check(self.lib.mhm_local_assemble(self.h, ctypes.byref(batch.desc), _ptr(Ahat), _ptr(Btil),
                                                _ptr(c), _ptr(area), _ptr(info)))

    def local_factor_solve(self, batch, prec, Ahat_io, Btil, X, info, ir_iters=None, max_iters: int = 10):
        self._check(self.lib.mhm_local_factor_solve(self.h, ctypes.byref(batch.desc), prec, _ptr(Ahat_io),
                                                    _ptr(Btil), _ptr(X), _ptr(info), _ptr(ir_iters), max_iters))

    def skeleton_contrib(self, batch, X, M, E, B, F, info=None):
        self._check(self.lib.mhm_skeleton_contrib(self.h, ctypes.byref(batch.desc), _ptr(X), _ptr(M), _ptr(E),
                                                  _ptr(B), _ptr(F), _ptr(info)))

    def local_batch_run(self, batch, prec, X, M, E, B, F, info, ir_iters=None, max_iters: int = 10):
        self._check(self.lib.mhm_local_batch_run(self.h, ctypes.byref(batch.desc), prec, _ptr(X), _ptr(M),
                                                 _ptr(E), _ptr(B), _ptr(F), _ptr(info), _ptr(ir_iters),
                                                 max_iters))

    def local_batch_run_noalloc(self, batch, prec, X, M, E, B, F, info, ir_iters=None, max_iters: int = 10):
        self._check(self.lib.mhm_local_batch_run_noalloc(self.h, ctypes.byref(batch.desc), prec, _ptr(X), _ptr(M),
                                                         _ptr(E), _ptr(B), _ptr(F), _ptr(info), _ptr(ir_iters),
                                                         max_iters))

    def autotune(self, batch, prec, X, M, E, B, F, info, ir_iters=None, max_iters: int = 10):
        self._check(self.lib.mhm_autotune(self.h, ctypes.byref(batch.desc), prec, _ptr(X), _ptr(M), _ptr(E),
                                          _ptr(B), _ptr(F), _ptr(info), _ptr(ir_iters), max_iters))

    def local_batch_run_cached(self, batch, prec, factors, factor_off, factor_state, X, M, E, B, F, info,
                              ir_iters=None, max_iters: int = 10):
        self._check(self.lib.mhm_local_batch_run_cached(
            self.h, ctypes.byref(batch.desc), prec, _ptr(factors), _ptr(factor_off), _ptr(factor_state), _ptr(X),
            _ptr(M), _ptr(E), _ptr(B), _ptr(F), _ptr(info), _ptr(ir_iters), max_iters))

    def local_source_step(self, batch, prec, factors, factor_off, factor_state, X, M, E, B, F, info,
                          ir_iters=None, max_iters: int = 10):
        self._check(self.lib.mhm_local_source_step(
            self.h, ctypes.byref(batch.desc), prec, _ptr(factors), _ptr(factor_off), _ptr(factor_state), _ptr(X),
            _ptr(M), _ptr(E), _ptr(B), _ptr(F), _ptr(info), _ptr(ir_iters), max_iters))

    def skeleton_solve(self, n_rows, n_lambda, row_ptr, col_idx, vals, rhs, sol, tol=1e-12, max_iters=20000,
                       lambda_block=1):
        """MINRES on the CSR skeleton system; returns (iterations, relative residual)."""
        it = ctypes.c_int32(0)
        rr = ctypes.c_double(0.0)
        self._check(self.lib.mhm_skeleton_solve(self.h, int(n_rows), int(n_lambda), int(lambda_block),
                                                _ptr(row_ptr), _ptr(col_idx),
                                                _ptr(vals), _ptr(rhs), _ptr(sol), float(tol), int(max_iters),
                                                ctypes.byref(it), ctypes.byref(rr)))
        return int(it.value), float(rr.value)

    def skeleton_scatter(self, batch, M, E, B, F, gdof, erow, row_ptr, col_idx, n_rows, vals, rhs, info=None,
                         missing=None):
        self._check(self.lib.mhm_skeleton_scatter(self.h, ctypes.byref(batch.desc), _ptr(M), _ptr(E), _ptr(B), _ptr(F),
                                                  _ptr(gdof), _ptr(erow), _ptr(row_ptr), _ptr(col_idx), int(n_rows),
                                                  _ptr(vals), _ptr(rhs), _ptr(info), _ptr(missing)))

    def reconstruct(self, batch, X, gdof, erow, sol, n_rows, u, info=None):
        self._check(self.lib.mhm_reconstruct(self.h, ctypes.byref(batch.desc), _ptr(X), _ptr(gdof), _ptr(erow),
                                             _ptr(sol), int(n_rows), _ptr(u), _ptr(info)))

    def class_times(self):
        """[(s_cap, ms)] of the last call timed with the class_timing option,
        largest class first; None when nothing was timed."""
        cap = (ctypes.c_int32 * 8)()
        ms = (ctypes.c_float * 8)()
        k = int(self.lib.mhm_class_times(self.h, cap, ms, 8))
        return None if k < 0 else [(int(cap[i]), float(ms[i])) for i in range(k)]

    def tune_report(self) -> str:
        n = int(self.lib.mhm_tune_report(self.h, None, 0))
        buf = ctypes.create_string_buffer(max(n, 1))
        self.lib.mhm_tune_report(self.h, buf, n)
        return buf.value.decode()

    def graph_create(self, batch, prec, X, M, E, B, F, info, ir_iters=None, max_iters: int = 10) -> "Graph":
        g = ctypes.c_void_p()
        self._check(self.lib.mhm_graph_create(self.h, ctypes.byref(batch.desc), prec, _ptr(X), _ptr(M), _ptr(E),
                                              _ptr(B), _ptr(F), _ptr(info), _ptr(ir_iters), max_iters,
                                              ctypes.byref(g)))
        return Graph(self, g)


class Graph:
    """An ``mhm_graph``: one captured mhm_local_batch_run, replayed by launch()."""

    def __init__(self, ctx: Context, h):
        self.ctx = ctx
        self.h = h

    def launch(self):
        self.ctx._check(self.ctx.lib.mhm_graph_launch(self.h))

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.mhm_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
