"""GPU parity with more than 16 right-hand sides per factor (Section 2's
richer multiplier spaces: m segments of degree l, N_I = 3 m (l + 1) up to 48,
so r = N_I + 1 up to 49).  The left-looking kernel takes the right-hand sides
in chunks of 16 columns over one factor; every chunk, both precisions, the
three-call and fused forms, stored factors, the time-step call and the
skeleton steps are compared with the FP64 oracle.  The kernels that hold a
single chunk report such elements as too large."""
from __future__ import annotations

import numpy as np
import pytest

from mhm_inputs import configs
from mhm_inputs.fields import manufactured_source
from mhm_inputs.mesh import coarse_mesh
from oracle import local, skeleton as oskel
from tests.parity_util import rel_errors, say
from tests.test_parity_gpu import TOL, _check
from tests.test_segments_gpu import _batch, _ctx

pytestmark = pytest.mark.gpu

# (s, l, m): r = 3 m (l + 1) + 1 from 25 to 49 (two to four chunks, ragged
# last chunks), one element per size class up to s = 48, with one-chunk
# elements mixed in
WIDE = [(2, 4, 2), (4, 3, 4), (6, 1, 6), (8, 1, 8), (12, 2, 4), (16, 3, 4), (16, 4, 1), (24, 0, 8),
        (32, 1, 8), (36, 2, 4), (48, 3, 4), (10, 1, 1), (40, 4, 2), (20, 0, 5)]


@pytest.fixture(scope="module")
def ctx():
    c = _ctx()
    yield c
    c.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_wide_rhs_every_size_class(ctx, prec):
    from paper_1703_10435_amd import engine
    b = _batch(71, WIDE, "wide")
    for mode in ("fused", "three_call"):
        say(f"[gpu] wide rhs prec={prec} mode={mode}")
        res, out, db = engine.solve_batch(b, prec=prec, mode=mode, ctx=ctx)
        assert db.NImax == 48
        _check(res, b, range(b["n_elem"]), prec, f"wide prec={prec} {mode}")


@pytest.mark.parametrize("prec", [0, 1])
def test_wide_rhs_on_stored_factors(ctx, prec):
    """Factor once, then a reuse step and a source-only step on the stored
    factors, every chunk against the oracle for that step's data."""
    import torch
    from paper_1703_10435_amd import engine
    from paper_1703_10435_amd.batch import DeviceBatch
    b = _batch(72, [(8, 1, 8), (16, 3, 4), (24, 1, 6), (48, 1, 8), (6, 2, 1)], "wide-steps")
    db = DeviceBatch(b)
    fs = engine.FactorStore(db, prec)
    say(f"[gpu] wide rhs factor step prec={prec}")
    out = engine.run_cached(ctx, db, fs)
    ctx.sync()
    _check(db.unpack(out), b, range(b["n_elem"]), prec, f"wide factor step prec={prec}")
    held = fs.state[:b["n_elem"]].cpu().numpy() == 1
    assert held.sum() >= b["n_elem"] - 1, held
    rng = np.random.default_rng(73)
    f = rng.standard_normal(b["f"].shape)
    dstep = engine.with_source(db, torch.as_tensor(f, device="cuda"))
    say(f"[gpu] wide rhs reuse step prec={prec}")
    out = engine.run_cached(ctx, dstep, fs)
    ctx.sync()
    _check(dstep.unpack(out), dict(b, f=f), range(b["n_elem"]), prec, f"wide reuse prec={prec}")
    f2 = rng.standard_normal(b["f"].shape)
    dstep2 = engine.with_source(db, torch.as_tensor(f2, device="cuda"))
    say(f"[gpu] wide rhs source step prec={prec}")
    engine.source_step(ctx, dstep2, fs, out)
    ctx.sync()
    _check(dstep2.unpack(out), dict(b, f=f2), np.flatnonzero(held), prec, f"wide source step prec={prec}")


@pytest.mark.parametrize("opts", [{"no_ll": 1}])
def test_wide_rhs_without_the_left_looking_kernel_reports(opts):
    """Only the left-looking kernel takes more than one chunk: with it
    switched off, wide elements report info -3 and the others are solved."""
    from paper_1703_10435_amd import engine
    c = _ctx(opts)
    try:
        cases = [(8, 1, 8), (8, 1, 1), (16, 0, 8), (16, 2, 1)]
        b = _batch(74, cases, "wide-no-ll")
        for prec in (0, 1):
            say(f"[gpu] wide rhs opts={opts} prec={prec}")
            res, out, db = engine.solve_batch(b, prec=prec, mode="fused", ctx=c)
            info = [res[e]["info"] for e in range(b["n_elem"])]
            assert info[0] == -3 and info[2] == -3, info
            _check(res, b, [1, 3], prec, f"wide no-ll prec={prec}")
    finally:
        c.close()


def test_wide_rhs_beyond_the_left_looking_range_reports(ctx):
    """s = 56 with 25 right-hand sides: no kernel takes it (info -3); the
    small element of the same batch is solved."""
    from paper_1703_10435_amd import engine
    b = _batch(75, [(56, 0, 8), (8, 1, 4)], "wide-too-large")
    say("[gpu] wide rhs beyond s = 48")
    res, out, db = engine.solve_batch(b, prec=0, mode="fused", ctx=ctx)
    assert res[0]["info"] == -3, res[0]["info"]
    _check(res, b, [1], 0, "wide beyond range")


def test_wide_rhs_scatter_and_reconstruct(ctx):
    import torch
    from paper_1703_10435_amd import engine
    from paper_1703_10435_amd.skeleton import SkeletonSystem
    N, s, l, m = 3, 8, 3, 4
    mesh = coarse_mesh(N)
    E = mesh["elems"].shape[0]
    b = configs.build_batch(mesh, np.arange(E), np.full(E, s), np.full(E, l),
                            lambda p: np.exp(np.sin(7.0 * p[..., 0]) * np.cos(5.0 * p[..., 1])), manufactured_source,
                            m_arr=np.full(E, m))
    say(f"[gpu] wide rhs skeleton N={N} s={s} l={l} m={m}")
    res, out, db = engine.solve_batch(b, prec=1, mode="fused", ctx=ctx)
    assert db.NImax == 48
    sk = SkeletonSystem(mesh, l, p_max=db.p_max, m=m)
    vals, rhs, missing = sk.scatter(ctx, db, out)
    ora = local.solve_batch(b)
    Ko, ro = oskel.assemble_global(mesh, ora, np.arange(E), l, m)
    ctx.sync()
    assert int(missing.item()) == 0
    K = np.zeros_like(Ko)
    v = vals.cpu().numpy()
    for i in range(sk.n_rows):
        K[i, sk.col_idx_h[sk.row_ptr_h[i]:sk.row_ptr_h[i + 1]]] = v[sk.row_ptr_h[i]:sk.row_ptr_h[i + 1]]
    scale = max(np.abs(Ko).max(), np.abs(ro).max())
    assert np.abs(K - Ko).max() <= 2 * TOL[1] * scale
    assert np.abs(rhs.cpu().numpy() - ro).max() <= 2 * TOL[1] * scale
    lam, u0, _, _ = oskel.reduce_and_solve(mesh, ora, np.arange(E), l, m)
    u = sk.reconstruct(ctx, db, out, torch.as_tensor(np.concatenate([lam, u0]), device="cuda"))
    ctx.sync()
    u = u.cpu().numpy()
    want = oskel.reconstruct(mesh, ora, np.arange(E), l, lam, u0, m)
    wsum = max(np.abs(r["X"]).max() * (1.0 + np.abs(lam[oskel.global_dofs(mesh, e, l, m)]).sum())
               for e, r in enumerate(ora))
    for e in range(E):
        assert np.abs(u[db.node_off[e]:db.node_off[e + 1]] - want[e]).max() <= TOL[1] * wsum + 1e-14, e
