"""GPU parity of the segmented multiplier space (Section 2: m segments per
face, a polynomial of degree l on each): every kernel family, both
precisions, the three-call and fused forms, mixed m in one batch, the
time-step call, and the skeleton scatter and reconstruction, each against
the FP64 oracle."""
from __future__ import annotations


import numpy as np
import pytest

from mhm_inputs import configs
from mhm_inputs.fields import manufactured_solution, manufactured_source
from mhm_inputs.mesh import coarse_mesh
from oracle import local, skeleton as oskel
from tests.parity_util import ensure_built, rel_errors, say
from tests.test_parity_gpu import TOL, _check, _random_batch

pytestmark = pytest.mark.gpu

# (s, l, m): m divides s, m (l + 1) <= 5; every size class and kernel family
CASES = [(2, 0, 2), (4, 1, 2), (6, 0, 3), (8, 0, 4), (10, 4, 1), (12, 1, 2), (15, 0, 5), (16, 1, 2),
         (20, 0, 4), (24, 1, 2), (30, 0, 5), (33, 0, 3), (36, 1, 2), (48, 0, 4), (48, 1, 2)]


def _batch(seed, cases, name):
    b = _random_batch(seed, [c[0] for c in cases], [c[1] for c in cases], name)
    b["m"] = np.asarray([c[2] for c in cases], dtype=np.int32)
    return b


def _ctx(opts=None):
    """A context with launch options (mhm_set_option) by name."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ensure_built()
    from paper_1703_10435_amd import abi
    return abi.Context(0, **(opts or {}))


@pytest.fixture(scope="module")
def ctx():
    c = _ctx()
    yield c
    c.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_segmented_faces_every_size_class(ctx, prec):
    from paper_1703_10435_amd import engine
    b = _batch(61, CASES, "segments")
    for mode in ("fused", "three_call"):
        say(f"[gpu] segments prec={prec} mode={mode}")
        res, out, db = engine.solve_batch(b, prec=prec, mode=mode, ctx=ctx)
        _check(res, b, range(b["n_elem"]), prec, f"segments prec={prec} {mode}")


@pytest.mark.parametrize("opts", [{"no_rr": 1}, {"no_ll": 1}])
def test_segmented_faces_other_families(opts):
    from paper_1703_10435_amd import engine
    c = _ctx(opts)
    try:
        b = _batch(62, [(4, 1, 2), (16, 0, 4), (24, 1, 2), (40, 0, 5)], "segments-families")
        for prec in (0, 1):
            say(f"[gpu] segments opts={opts} prec={prec}")
            res, out, db = engine.solve_batch(b, prec=prec, mode="fused", ctx=c)
            _check(res, b, range(b["n_elem"]), prec, f"segments {opts} prec={prec}")
    finally:
        c.close()


def test_segmented_and_whole_faces_in_one_batch(ctx):
    """m = 1 and m > 1 elements mixed; padded blocks 3 p_max wide."""
    from paper_1703_10435_amd import engine
    cases = [(8, 4, 1), (8, 1, 2), (16, 2, 1), (16, 0, 4), (12, 0, 3), (6, 1, 1)]
    b = _batch(63, cases, "segments-mixed")
    say("[gpu] segments mixed")
    res, out, db = engine.solve_batch(b, prec=0, mode="fused", ctx=ctx)
    assert db.NImax == 15
    _check(res, b, range(b["n_elem"]), 0, "segments mixed")


@pytest.mark.parametrize("prec", [0, 1])
def test_segmented_source_steps(ctx, prec):
    import torch
    from paper_1703_10435_amd import engine
    from paper_1703_10435_amd.batch import DeviceBatch
    b = _batch(64, [(4, 1, 2), (16, 1, 2), (24, 0, 4), (48, 0, 5 if 48 % 5 == 0 else 4)], "segments-steps")
    db = DeviceBatch(b)
    fs = engine.FactorStore(db, prec)
    out = engine.run_cached(ctx, db, fs)
    ctx.sync()
    held = fs.state[:b["n_elem"]].cpu().numpy() == 1
    f = np.random.default_rng(65).standard_normal(b["f"].shape)
    dstep = engine.with_source(db, torch.as_tensor(f, device="cuda"))
    say(f"[gpu] segments source step prec={prec}")
    engine.source_step(ctx, dstep, fs, out)
    ctx.sync()
    res = dstep.unpack(out)
    _check(res, dict(b, f=f), np.flatnonzero(held), prec, f"segments source step prec={prec}")


@pytest.mark.parametrize("N,s,l,m", [(4, 8, 1, 2), (3, 6, 0, 3)])
def test_segmented_scatter_and_reconstruct(ctx, N, s, l, m):
    import torch
    from paper_1703_10435_amd import engine
    from paper_1703_10435_amd.skeleton import SkeletonSystem
    mesh = coarse_mesh(N)
    E = mesh["elems"].shape[0]
    b = configs.build_batch(mesh, np.arange(E), np.full(E, s), np.full(E, l),
                            lambda p: np.exp(np.sin(7.0 * p[..., 0]) * np.cos(5.0 * p[..., 1])), manufactured_source,
                            m_arr=np.full(E, m))
    say(f"[gpu] segments skeleton N={N} s={s} l={l} m={m}")
    res, out, db = engine.solve_batch(b, prec=0, mode="fused", ctx=ctx)
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
    assert np.abs(K - Ko).max() <= 2 * TOL[0] * scale
    assert np.abs(rhs.cpu().numpy() - ro).max() <= 2 * TOL[0] * scale
    lam, u0, _, _ = oskel.reduce_and_solve(mesh, ora, np.arange(E), l, m)
    u = sk.reconstruct(ctx, db, out, torch.as_tensor(np.concatenate([lam, u0]), device="cuda"))
    ctx.sync()
    u = u.cpu().numpy()
    want = oskel.reconstruct(mesh, ora, np.arange(E), l, lam, u0, m)
    wsum = max(np.abs(r["X"]).max() * (1.0 + np.abs(lam[oskel.global_dofs(mesh, e, l, m)]).sum())
               for e, r in enumerate(ora))
    for e in range(E):
        assert np.abs(u[db.node_off[e]:db.node_off[e + 1]] - want[e]).max() <= TOL[0] * wsum + 1e-14, e


def test_segmented_chain_converges_at_second_order(ctx):
    """m = 2, l = 0 through the device path (local solves, scatter, host
    solve, reconstruction): second-order L2 convergence."""
    import torch
    from paper_1703_10435_amd import engine
    from paper_1703_10435_amd.skeleton import SkeletonSystem
    errs = []
    for N in (2, 4, 8):
        mesh = coarse_mesh(N)
        E = mesh["elems"].shape[0]
        b = configs.build_batch(mesh, np.arange(E), np.full(E, 4), np.full(E, 0), lambda p: np.ones(p.shape[:-1]),
                                manufactured_source, m_arr=np.full(E, 2))
        say(f"[gpu] segments chain N={N}")
        res, out, db = engine.solve_batch(b, prec=0, mode="fused", ctx=ctx)
        sk = SkeletonSystem(mesh, 0, p_max=db.p_max, m=2)
        vals, rhs, missing = sk.scatter(ctx, db, out)
        ctx.sync()
        K = np.zeros((sk.n_rows, sk.n_rows))
        v = vals.cpu().numpy()
        for i in range(sk.n_rows):
            K[i, sk.col_idx_h[sk.row_ptr_h[i]:sk.row_ptr_h[i + 1]]] = v[sk.row_ptr_h[i]:sk.row_ptr_h[i + 1]]
        sol = np.linalg.lstsq(K, rhs.cpu().numpy(), rcond=1e-12)[0]
        u = sk.reconstruct(ctx, db, out, torch.as_tensor(sol, device="cuda"))
        ctx.sync()
        u = u.cpu().numpy()
        errs.append(oskel.l2_error(b, [u[db.node_off[e]:db.node_off[e + 1]] for e in range(E)],
                                   manufactured_solution))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    say(f"  errors {errs} rates {rates}")
    assert np.all((rates > 1.8) & (rates < 2.3)), (errs, rates)
