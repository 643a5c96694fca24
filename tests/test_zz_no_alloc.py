"""mhm_local_batch_run_noalloc against mhm_local_batch_run, through the C ABI:
two calls in a row on the library's scratch array (the second with a smaller
batch, which must not see the first call's leftovers), in both precisions,
on a ragged batch whose largest class needs workspace slots.  The two entry
points run the same kernels, so the results must agree to the FP64 bar of
the parity tests (1e-10 relative per element), and in fact bit for bit
wherever the launch does not depend on the grid size."""
from __future__ import annotations

import numpy as np
import pytest

from tests.parity_util import ensure_built, rel_errors, say

pytestmark = pytest.mark.gpu

BAR = 1e-10


def _batches():
    from tests.test_parity_gpu import _random_batch
    from mhm_inputs import configs
    big = _random_batch(71, [4, 8, 16, 24, 33, 48, 48, 32, 12, 40, 20, 48], [1, 2, 3, 0, 2, 3, 1, 2, 3, 1, 0, 2],
                        "noalloc-1")
    c3 = configs.sub_batch(configs.make("C3"), [3452, 1280, 5])        # channel elements (refinement pass)
    from tests.test_channel_gpu import _concat
    first = _concat([big, c3])
    second = _random_batch(72, [8, 48, 16, 33], [2, 1, 3, 2], "noalloc-2")
    return first, second


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_the_allocating_entry_point(prec):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ensure_built()
    from paper_1703_10435_amd import abi
    from paper_1703_10435_amd.batch import DeviceBatch
    ctx = abi.Context(0)
    try:
        for k, b in enumerate(_batches()):
            db = DeviceBatch(b)
            ref = db.alloc_outputs()
            out = db.alloc_outputs()
            for t in out.values():
                t.fill_(-7)    # poison: every output must be written
            say(f"[gpu] noalloc call {k} prec={prec} n_elem={b['n_elem']}")
            ctx.local_batch_run(db, prec, ref["X"], ref["M"], ref["E"], ref["B"], ref["F"], ref["info"],
                                ref["ir_iters"], 10)
            ctx.local_batch_run_noalloc(db, prec, out["X"], out["M"], out["E"], out["B"], out["F"], out["info"],
                                        out["ir_iters"], 10)
            ctx.sync()
            r_ref, r_out = db.unpack(ref), db.unpack(out)
            worst = 0.0
            for e in range(b["n_elem"]):
                assert r_out[e]["info"] == r_ref[e]["info"], (k, e, r_out[e]["info"], r_ref[e]["info"])
                assert r_out[e]["ir_iters"] == r_ref[e]["ir_iters"], (k, e)
                ex, eb = rel_errors(r_out[e], r_ref[e])
                worst = max(worst, ex, eb)
                assert ex <= BAR and eb <= BAR, (k, e, ex, eb)
            say(f"  call {k}: worst rel diff {worst:.2e}")
    finally:
        ctx.close()


def test_noalloc_rejects_a_batch_beyond_the_scratch_array():
    """A ragged batch of 14 million elements (all s = 1 but one s = 17, so
    two size classes): its class lists need 4 (5 E + 5) = 280 MB, beyond the
    256 MiB array, and the call must fail on the host before enqueuing
    anything.  The arrays are real and valid, so even a missing check could
    only run the batch, never read out of bounds."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ensure_built()
    from paper_1703_10435_amd import abi
    E = 14_000_000
    dev = "cuda"
    i32, i64, f64 = torch.int32, torch.int64, torch.float64
    s = torch.ones(E, dtype=i32, device=dev)
    s[E // 2] = 17
    l = torch.zeros(E, dtype=i32, device=dev)
    n = (s + 1) * (s + 2) // 2
    r = torch.full((E,), 4, dtype=i32, device=dev)   # l = 0: N_I = 3, r = 4

    def prefix(x):
        o = torch.zeros(E + 1, dtype=i64, device=dev)
        o[1:] = torch.cumsum(x.to(i64), 0)
        return o
    tri_off, rhs_off, node_off, mat_off = prefix(s * s), prefix(n * r), prefix(n), prefix(n * n)
    T = int(tri_off[-1])
    t = dict(s=s, l=l, vert=torch.tensor([0.0, 0.0, 1.0, 0.0, 0.0, 1.0], dtype=f64, device=dev).repeat(E),
             sigma=torch.ones(3 * E, dtype=torch.int8, device=dev), flip=torch.zeros(3 * E, dtype=torch.int8, device=dev),
             kappa=torch.ones(T, dtype=f64, device=dev), f=torch.ones(T, dtype=f64, device=dev), tri_off=tri_off,
             rhs_off=rhs_off, node_off=node_off, mat_off=mat_off)
    d = abi.mhm_batch()
    d.n_elem, d.s_max, d.s_min, d.l_max, d.p_max = E, 17, 1, 0, 1
    for k, v in t.items():
        setattr(d, k, v.data_ptr())
    d.tri_total, d.rhs_total, d.node_total, d.mat_total = T, int(rhs_off[-1]), int(node_off[-1]), int(mat_off[-1])

    class _B:
        desc = d
    X = torch.zeros(int(rhs_off[-1]), dtype=f64, device=dev)
    M = torch.zeros(9 * E, dtype=f64, device=dev)
    Ev = torch.zeros(3 * E, dtype=f64, device=dev)
    Bv = torch.zeros(3 * E, dtype=f64, device=dev)
    F = torch.zeros(E, dtype=f64, device=dev)
    info = torch.full((E,), 5, dtype=i32, device=dev)
    ctx = abi.Context(0)
    try:
        say("[gpu] noalloc rejection of a 14M-element batch")
        with pytest.raises(abi.MhmError) as ei:
            ctx.local_batch_run_noalloc(_B, 0, X, M, Ev, Bv, F, info, None, 10)
        assert ei.value.status == abi.MHM_E_ARG and "too large" in str(ei.value)
        ctx.sync()
        assert bool((info == 5).all())   # nothing ran
    finally:
        ctx.close()
