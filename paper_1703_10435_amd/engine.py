"""Convenience drivers over the C ABI: run a batch through the three-call path
(assemble -> factor/solve -> contribution) or the fused call, on one stream.

Only marshalling and buffer management here; all arithmetic is in libmhm.so.
"""
from __future__ import annotations

from . import abi
from .batch import DeviceBatch


def run_three_call(ctx: abi.Context, db: DeviceBatch, prec: int = abi.MHM_FP64, out: dict | None = None,
                   max_iters: int = 10) -> dict:
    """solveLocalProblem + the element share of reduceLocalProblems as three
    library calls: mhm_local_assemble, mhm_local_factor_solve,
    mhm_skeleton_contrib."""
    if out is None:
        out = db.alloc_outputs(three_call=True)
    ctx.local_assemble(db, out["Ahat"], out["Btil"], out["c"], out["area"], out["info"])
    ctx.local_factor_solve(db, prec, out["Ahat"], out["Btil"], out["X"], out["info"], out["ir_iters"], max_iters)
    ctx.skeleton_contrib(db, out["X"], out["M"], out["E"], out["B"], out["F"], out["info"])
    return out


def run_fused(ctx: abi.Context, db: DeviceBatch, prec: int = abi.MHM_FP64, out: dict | None = None,
              max_iters: int = 10) -> dict:
    """The same work as one mhm_local_batch_run call."""
    if out is None:
        out = db.alloc_outputs(three_call=False)
    ctx.local_batch_run(db, prec, out["X"], out["M"], out["E"], out["B"], out["F"], out["info"],
                        out["ir_iters"], max_iters)
    return out


def autotune(ctx: abi.Context, db: DeviceBatch, prec: int = abi.MHM_FP64, out: dict | None = None,
             max_iters: int = 10) -> dict:
    """Choose the kernel family / panel width per size class by timing
    (mhm_autotune); the outputs are those of one fused run."""
    if out is None:
        out = db.alloc_outputs(three_call=False)
    ctx.autotune(db, prec, out["X"], out["M"], out["E"], out["B"], out["F"], out["info"], out["ir_iters"],
                 max_iters)
    return out


def capture_fused(ctx: abi.Context, db: DeviceBatch, prec: int = abi.MHM_FP64, out: dict | None = None,
                  max_iters: int = 10):
    """A HIP graph of one fused run (binning, per-class launches, fallback
    passes); ``graph.launch()`` replays it on the context's stream."""
    if out is None:
        out = db.alloc_outputs(three_call=False)
    g = ctx.graph_create(db, prec, out["X"], out["M"], out["E"], out["B"], out["F"], out["info"], out["ir_iters"],
                         max_iters)
    return g, out


def run_three_call_bucketed(ctx: abi.Context, sub_batches: list, prec: int = abi.MHM_FP64, outs: list | None = None,
                            max_iters: int = 10) -> list:
    """The plain unfused form over a ragged batch: the three calls launched
    once per size bucket (each bucket a DeviceBatch of its own)."""
    if outs is None:
        outs = [db.alloc_outputs(three_call=True) for db in sub_batches]
    for db, out in zip(sub_batches, outs):
        run_three_call(ctx, db, prec, out, max_iters)
    return outs


def solve_batch(batch: dict, prec: int = abi.MHM_FP64, mode: str = "fused", ctx: abi.Context | None = None,
                max_iters: int = 10):
    """Upload a host batch, run it, return per-element results (numpy)."""
    ctx = ctx or abi.Context()
    db = DeviceBatch(batch)
    run = run_fused if mode == "fused" else run_three_call
    out = run(ctx, db, prec, max_iters=max_iters)
    ctx.sync()
    return db.unpack(out), out, db


class FactorStore:
    """Device store of one factor per element (mhm_local_batch_run_cached):
    offsets 256-byte aligned, state 0 until a call has factored the element."""

    def __init__(self, db: DeviceBatch, prec: int, device="cuda"):
        import numpy as np
        import torch
        sizes = np.array([abi.factor_bytes(int(s), prec) for s in db.s], dtype=np.int64)
        sizes = (sizes + 255) // 256 * 256
        off = np.zeros(len(sizes) + 1, dtype=np.int64)
        np.cumsum(sizes, out=off[1:])
        self.prec = prec
        self.nbytes = int(off[-1])
        self.store = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=device)
        self.off = torch.as_tensor(off[:-1], dtype=torch.int64, device=device)
        self.state = torch.zeros(max(len(sizes), 1), dtype=torch.int8, device=device)

    def mark_valid(self, info):
        """Elements whose call reported info == 0 keep their factor."""
        import torch
        n = info.numel()
        self.state[:n] = torch.where(info == 0, 1, 0).to(torch.int8)


def with_source(db: DeviceBatch, f) -> DeviceBatch:
    """A view of the batch with the per-sub-triangle source f replaced (a
    new load for the same elements, e.g. the next time step)."""
    import copy
    import ctypes
    v = copy.copy(db)
    v.desc = abi.mhm_batch.from_buffer_copy(db.desc)
    v.desc.f = ctypes.c_void_p(f.data_ptr()).value
    v._f_ref = f
    return v


def run_cached(ctx: abi.Context, db: DeviceBatch, fs: FactorStore, out: dict | None = None,
               max_iters: int = 10, update_state: bool = True) -> dict:
    """mhm_local_batch_run_cached: factor the elements whose state is 0,
    reuse the stored factor of the others; afterwards (update_state) every
    element with info == 0 is marked as holding its factor."""
    if out is None:
        out = db.alloc_outputs(three_call=False)
    ctx.local_batch_run_cached(db, fs.prec, fs.store, fs.off, fs.state, out["X"], out["M"], out["E"], out["B"],
                               out["F"], out["info"], out["ir_iters"], max_iters)
    if update_state:
        fs.mark_valid(out["info"][:db.n_elem])
    return out


def source_step(ctx: abi.Context, db: DeviceBatch, fs: FactorStore, out: dict, max_iters: int = 10) -> dict:
    """mhm_local_source_step: a time step with a new source on the stored
    factors; rewrites the source column of X, E and F in ``out`` (the
    outputs of the call that stored the factors)."""
    ctx.local_source_step(db, fs.prec, fs.store, fs.off, fs.state, out["X"], out["M"], out["E"], out["B"],
                          out["F"], out["info"], out["ir_iters"], max_iters)
    return out
