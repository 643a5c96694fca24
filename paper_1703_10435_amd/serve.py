"""ctypes binding of the serving runtime (``mhm_server_*`` in include/mhm.h)
and an open-loop driver: requests are submitted at their scheduled arrival
times whatever the state of the device, results are collected as they
finish, and latency is measured from the scheduled arrival to the results
being on the host.

Argument marshalling and timing only; batching, admission, the factor cache
and all arithmetic are in libmhm.so.
"""
from __future__ import annotations

import ctypes
import hashlib
import time

import numpy as np

from . import abi


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("prec", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("max_batch", ctypes.c_int32),
        ("in_flight", ctypes.c_int32), ("s_max", ctypes.c_int32), ("l_max", ctypes.c_int32),
        ("reuse", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("hbm_budget", ctypes.c_uint64), ("factor_cache_max", ctypes.c_uint64),
    ]


class Request(ctypes.Structure):
    _fields_ = [
        ("key_hi", ctypes.c_uint64), ("key_lo", ctypes.c_uint64), ("s", ctypes.c_int32), ("l", ctypes.c_int32),
        ("vert", ctypes.c_double * 6), ("sigma", ctypes.c_int8 * 3), ("flip", ctypes.c_int8 * 3),
        ("pad", ctypes.c_int8 * 2), ("kappa", ctypes.c_void_p), ("f", ctypes.c_void_p),
        ("t_arrival", ctypes.c_double),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("ticket", ctypes.c_uint64), ("info", ctypes.c_int32), ("ir_iters", ctypes.c_int32),
        ("cache_hit", ctypes.c_int32), ("s", ctypes.c_int32), ("l", ctypes.c_int32), ("n", ctypes.c_int32),
        ("r", ctypes.c_int32), ("pad", ctypes.c_int32), ("t_arrival", ctypes.c_double), ("t_done", ctypes.c_double),
        ("X", ctypes.POINTER(ctypes.c_double)), ("M", ctypes.POINTER(ctypes.c_double)),
        ("E", ctypes.POINTER(ctypes.c_double)), ("B", ctypes.POINTER(ctypes.c_double)), ("F", ctypes.c_double),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "submitted", "completed", "launches", "cache_hits", "ir_fallbacks", "errors", "queued", "max_batch_seen",
        "cache_entries", "cache_bytes", "cache_evictions", "arena_bytes", "fixed_bytes")]


SERVER_EXPORTS = ("mhm_server_now", "mhm_server_create", "mhm_server_submit", "mhm_server_poll",
                  "mhm_server_stats_get", "mhm_server_last_error", "mhm_server_destroy")


def _lib():
    lib = abi.load()
    if not getattr(lib, "_server_sig", False):
        vp = ctypes.c_void_p
        sig = {
            "mhm_server_now": (ctypes.c_double, []),
            "mhm_server_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]),
            "mhm_server_submit": (ctypes.c_int, [vp, ctypes.POINTER(Request), ctypes.c_int,
                                                 ctypes.POINTER(ctypes.c_uint64)]),
            "mhm_server_poll": (ctypes.c_int, [vp, ctypes.POINTER(Result), ctypes.c_int]),
            "mhm_server_stats_get": (ctypes.c_int, [vp, ctypes.POINTER(ServerStats)]),
            "mhm_server_last_error": (ctypes.c_char_p, [vp]),
            "mhm_server_destroy": (ctypes.c_int, [vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        lib._server_sig = True
    return lib


def content_key(vert, s: int, kappa) -> tuple:
    """128-bit content key of (geometry, s, kappa), as two uint64."""
    h = hashlib.blake2b(digest_size=16)
    h.update(np.ascontiguousarray(vert, dtype=np.float64).tobytes())
    h.update(np.int32(s).tobytes())
    h.update(np.ascontiguousarray(kappa, dtype=np.float64).tobytes())
    d = h.digest()
    hi, lo = int.from_bytes(d[:8], "little"), int.from_bytes(d[8:], "little")
    return (hi or 1), lo


class Server:
    def __init__(self, device: int = 0, prec: int = abi.MHM_FP32_IR, max_iters: int = 10, max_batch: int = 1024,
                 in_flight: int = 4, s_max: int = 48, l_max: int = 3, reuse: bool = True,
                 hbm_budget: int = 64 << 30, factor_cache_max: int = 0):
        self.lib = _lib()
        cfg = ServerConfig(prec, max_iters, max_batch, in_flight, s_max, l_max, int(reuse), 0, hbm_budget,
                           factor_cache_max)
        h = ctypes.c_void_p()
        st = self.lib.mhm_server_create(device, ctypes.byref(cfg), ctypes.byref(h))
        if st != abi.MHM_OK:
            raise abi.MhmError(st, "mhm_server_create")
        self.h = h
        self._keep = []   # host arrays referenced by submitted requests until submit returns

    def now(self) -> float:
        return float(self.lib.mhm_server_now())

    def submit(self, reqs: list) -> list:
        """reqs: dicts with s, l, vert[6], sigma[3], flip[3], kappa, f (float64
        arrays of s*s), optional key (hi, lo) and t_arrival."""
        n = len(reqs)
        if n == 0:
            return []
        arr = (Request * n)()
        keep = []
        for k, q in enumerate(reqs):
            kap = np.ascontiguousarray(q["kappa"], dtype=np.float64)
            ff = np.ascontiguousarray(q["f"], dtype=np.float64)
            keep += [kap, ff]
            r = arr[k]
            r.key_hi, r.key_lo = q.get("key", (0, 0))
            r.s, r.l = int(q["s"]), int(q["l"])
            r.vert[:] = [float(v) for v in q["vert"]]
            r.sigma[:] = [int(v) for v in q["sigma"]]
            r.flip[:] = [int(v) for v in q["flip"]]
            r.kappa = kap.ctypes.data
            r.f = ff.ctypes.data
            r.t_arrival = float(q.get("t_arrival", self.now()))
        tickets = (ctypes.c_uint64 * n)()
        st = self.lib.mhm_server_submit(self.h, arr, n, tickets)
        if st != abi.MHM_OK:
            raise abi.MhmError(st, self.lib.mhm_server_last_error(self.h).decode())
        return list(tickets)

    def poll(self, max_n: int = 4096, copy_arrays: bool = True, copy_tickets=None) -> list:
        """Finished results; their arrays (X, M, E, B) are copied when
        copy_arrays is set or the ticket is in copy_tickets (the library's
        buffers are reused by the next poll)."""
        out = (Result * max_n)()
        k = self.lib.mhm_server_poll(self.h, out, max_n)
        res = []
        for i in range(k):
            r = out[i]
            d = dict(ticket=int(r.ticket), info=int(r.info), ir_iters=int(r.ir_iters), cache_hit=bool(r.cache_hit),
                     s=int(r.s), l=int(r.l), n=int(r.n), r=int(r.r), t_arrival=float(r.t_arrival),
                     t_done=float(r.t_done), F=float(r.F))
            if copy_arrays or (copy_tickets is not None and int(r.ticket) in copy_tickets):
                ni = r.r - 1
                d["X"] = np.ctypeslib.as_array(r.X, shape=(r.n * r.r,)).reshape(r.r, r.n).T.copy()
                d["M"] = np.ctypeslib.as_array(r.M, shape=(ni * ni,)).reshape(ni, ni).T.copy()
                d["E"] = np.ctypeslib.as_array(r.E, shape=(ni,)).copy()
                d["B"] = np.ctypeslib.as_array(r.B, shape=(ni,)).copy()
            res.append(d)
        return res

    def stats(self) -> dict:
        s = ServerStats()
        self.lib.mhm_server_stats_get(self.h, ctypes.byref(s))
        return {k: int(getattr(s, k)) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.mhm_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_open_loop(server: Server, reqs: list, arrivals, copy_arrays: bool = False, timeout_s: float = 120.0,
                  progress=None, keep=None) -> dict:
    """Submit reqs[k] at server clock t0 + arrivals[k] (open loop), collect
    every result; returns per-request latency and throughput.  Result arrays
    are kept for every request (copy_arrays) or for the indices in keep."""
    keep = set() if keep is None else set(int(k) for k in keep)
    keep_tickets = set()
    arrivals = np.asarray(arrivals, dtype=np.float64)
    n = len(reqs)
    t0 = server.now() + 0.01
    for k, q in enumerate(reqs):
        q["t_arrival"] = t0 + float(arrivals[k])
    results = {}
    i = 0
    tick_of = {}
    last_report = time.time()
    while len(results) < n:
        now = server.now()
        j = int(np.searchsorted(arrivals, now - t0, side="right"))
        if j > i:
            tk = server.submit(reqs[i:j])
            for a, t in enumerate(tk):
                tick_of[t] = i + a
                if i + a in keep:
                    keep_tickets.add(int(t))
            i = j
        got = server.poll(copy_arrays=copy_arrays, copy_tickets=keep_tickets)
        for r in got:
            results[tick_of[r["ticket"]]] = r
        if not got and j == i:
            time.sleep(5e-5)
        if now - t0 > timeout_s + (arrivals[-1] if n else 0):
            raise TimeoutError(f"served {len(results)} of {n} requests")
        if progress and time.time() - last_report > 5.0:
            progress(len(results), n)
            last_report = time.time()
    t_end = max(r["t_done"] for r in results.values())
    lat = np.array([results[k]["t_done"] - results[k]["t_arrival"] for k in range(n)])
    return dict(results=[results[k] for k in range(n)], latency=lat, wall=t_end - t0,
                throughput=n / max(t_end - t0, 1e-9))
