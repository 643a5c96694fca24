"""GPU tests of the two steps either side of the local solves: the scatter of
the element blocks into the skeleton system eq. (6) and the reconstruction
of u_{H,h}, eq. (4).  Each is compared with the FP64 oracle on the same
seeded mesh; the whole chain (local solves, scatter, a host solve of the
assembled system, reconstruction) is checked against the manufactured
solution's second-order convergence."""
from __future__ import annotations

import numpy as np
import pytest

from mhm_inputs import configs
from mhm_inputs.fields import manufactured_solution, manufactured_source
from mhm_inputs.mesh import coarse_mesh
from oracle import local, skeleton as oskel
from tests.parity_util import ensure_built, say
from tests.test_parity_gpu import TOL

pytestmark = pytest.mark.gpu


def _ones(p):
    return np.ones(p.shape[:-1])


def _rough_k(p):
    return np.exp(np.sin(7.0 * p[..., 0]) * np.cos(5.0 * p[..., 1]))


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ensure_built()
    from paper_1703_10435_amd import abi
    c = abi.Context(0)
    yield c
    c.close()


def _gpu_local(ctx, mesh, s, l, kfun, prec):
    from paper_1703_10435_amd import engine
    E = mesh["elems"].shape[0]
    b = configs.build_batch(mesh, np.arange(E), np.full(E, s), np.full(E, l), kfun, manufactured_source)
    res, out, db = engine.solve_batch(b, prec=prec, mode="fused", ctx=ctx)
    return b, res, out, db


def _dense(rp, ci, vals, n):
    K = np.zeros((n, n))
    for i in range(n):
        K[i, ci[rp[i]:rp[i + 1]]] = vals[rp[i]:rp[i + 1]]
    return K


def _host_solve(K, rhs):
    """Test-side solve of the assembled system (rank deficient when l >= s)."""
    if np.linalg.cond(K) < 1e12:
        return np.linalg.solve(K, rhs)
    return np.linalg.lstsq(K, rhs, rcond=1e-12)[0]


@pytest.mark.parametrize("N,s,l,prec", [(4, 8, 1, 0), (4, 6, 2, 1), (3, 5, 4, 0), (2, 3, 0, 0)])
def test_scatter_matches_oracle_assembly(ctx, N, s, l, prec):
    from paper_1703_10435_amd.skeleton import SkeletonSystem
    mesh = coarse_mesh(N)
    say(f"[gpu] scatter N={N} s={s} l={l} prec={prec}")
    b, res, out, db = _gpu_local(ctx, mesh, s, l, _rough_k, prec)
    sk = SkeletonSystem(mesh, l, p_max=db.p_max)
    vals, rhs, missing = sk.scatter(ctx, db, out)
    ctx.sync()
    assert int(missing.item()) == 0
    K = _dense(sk.row_ptr_h, sk.col_idx_h, vals.cpu().numpy(), sk.n_rows)
    ora = local.solve_batch(b)
    Ko, ro = oskel.assemble_global(mesh, ora, np.arange(b["n_elem"]), l)
    # every entry is a sum of at most two element values, each within TOL of
    # the oracle relative to its element's block
    scale = max(np.abs(Ko).max(), np.abs(ro).max())
    tol = 2 * TOL[prec] * scale
    assert np.abs(K - Ko).max() <= tol, np.abs(K - Ko).max() / scale
    assert np.abs(rhs.cpu().numpy() - ro).max() <= tol
    # every nonzero of the oracle's system lies in the pattern
    mask = np.zeros_like(Ko, dtype=bool)
    for i in range(sk.n_rows):
        mask[i, sk.col_idx_h[sk.row_ptr_h[i]:sk.row_ptr_h[i + 1]]] = True
    assert not np.any(Ko[~mask])


def test_scatter_skips_failed_elements_and_reports_missing(ctx):
    import torch
    from paper_1703_10435_amd.skeleton import SkeletonSystem
    mesh = coarse_mesh(2)
    l = 1
    b, res, out, db = _gpu_local(ctx, mesh, 4, l, _ones, 0)
    sk = SkeletonSystem(mesh, l, p_max=db.p_max)
    bad = 3
    info = out["info"].clone()
    info[bad] = 7                                     # as a failed factorisation would report
    o2 = dict(out, info=info)
    say("[gpu] scatter with a failed element")
    vals, rhs, missing = sk.scatter(ctx, db, o2)
    ctx.sync()
    assert int(missing.item()) == 0
    keep = [e for e in range(b["n_elem"]) if e != bad]
    Ko, ro = oskel.assemble_global(mesh, [res[e] for e in keep], keep, l)
    K = _dense(sk.row_ptr_h, sk.col_idx_h, vals.cpu().numpy(), sk.n_rows)
    assert np.abs(K - Ko).max() <= 1e-14 * np.abs(Ko).max()
    assert np.abs(rhs.cpu().numpy() - ro).max() <= 1e-14 * np.abs(ro).max()
    # drop the first entry of element 0's u_0 row (a B coupling entry, which
    # only element 0 adds to): exactly one addition has no place
    rp, ci = sk.row_ptr_h.copy(), sk.col_idx_h.copy()
    row = int(sk.erow_h[0])
    drop = rp[row]
    ci2 = np.delete(ci, drop)
    rp2 = rp.copy()
    rp2[row + 1:] -= 1
    sk.row_ptr = torch.as_tensor(rp2, dtype=torch.int32, device="cuda")
    sk.col_idx = torch.as_tensor(ci2, dtype=torch.int32, device="cuda")
    sk.nnz = int(rp2[-1])
    say("[gpu] scatter with an entry missing from the pattern")
    vals, rhs, missing = sk.scatter(ctx, db, out)
    ctx.sync()
    assert int(missing.item()) == 1


@pytest.mark.parametrize("N,s,l,prec", [(4, 8, 1, 0), (4, 6, 2, 1), (3, 5, 4, 0)])
def test_reconstruct_matches_oracle(ctx, N, s, l, prec):
    import torch
    from paper_1703_10435_amd.skeleton import SkeletonSystem
    mesh = coarse_mesh(N)
    say(f"[gpu] reconstruct N={N} s={s} l={l} prec={prec}")
    b, res, out, db = _gpu_local(ctx, mesh, s, l, _rough_k, prec)
    ora = local.solve_batch(b)
    lam, u0, _, _ = oskel.reduce_and_solve(mesh, ora, np.arange(b["n_elem"]), l)
    sol = np.concatenate([lam, u0])
    sk = SkeletonSystem(mesh, l, p_max=db.p_max)
    u = sk.reconstruct(ctx, db, out, torch.as_tensor(sol, device="cuda"))
    ctx.sync()
    u = u.cpu().numpy()
    want = oskel.reconstruct(mesh, ora, np.arange(b["n_elem"]), l, lam, u0)
    scale = max(np.abs(w).max() for w in want)
    # |X err| <= TOL |X|, times the multipliers' weight in the sum
    wsum = max(np.abs(r["X"]).max() * (1.0 + np.abs(lam[oskel.global_dofs(mesh, e, l)]).sum())
               for e, r in enumerate(ora))
    for e in range(b["n_elem"]):
        got = u[db.node_off[e]:db.node_off[e + 1]]
        assert np.abs(got - want[e]).max() <= TOL[prec] * wsum + 1e-14 * scale, e


def test_reconstruct_skips_failed_elements(ctx):
    import torch
    from paper_1703_10435_amd.skeleton import SkeletonSystem
    mesh = coarse_mesh(2)
    b, res, out, db = _gpu_local(ctx, mesh, 4, 1, _ones, 0)
    sk = SkeletonSystem(mesh, 1, p_max=db.p_max)
    info = out["info"].clone()
    info[2] = 5
    sol = torch.ones(sk.n_rows, dtype=torch.float64, device="cuda")
    u = torch.full((db.node_total,), -7.0, dtype=torch.float64, device="cuda")
    say("[gpu] reconstruct with a failed element")
    sk.reconstruct(ctx, db, dict(out, info=info), sol, u)
    ctx.sync()
    u = u.cpu().numpy()
    assert np.all(u[db.node_off[2]:db.node_off[3]] == -7.0)
    assert np.all(u[db.node_off[3]:db.node_off[4]] != -7.0)


@pytest.mark.parametrize("prec", [0, 1])
def test_chain_converges_at_second_order(ctx, prec):
    """Local solves, scatter, host solve of eq. (6), reconstruction: the L2
    error against the manufactured solution falls at rate 2 (K = 1, l = 1)."""
    import torch
    from paper_1703_10435_amd.skeleton import SkeletonSystem
    errs = []
    for N in (2, 4, 8):
        mesh = coarse_mesh(N)
        say(f"[gpu] chain N={N} prec={prec}")
        b, res, out, db = _gpu_local(ctx, mesh, 4, 1, _ones, prec)
        sk = SkeletonSystem(mesh, 1, p_max=db.p_max)
        vals, rhs, missing = sk.scatter(ctx, db, out)
        ctx.sync()
        assert int(missing.item()) == 0
        K = _dense(sk.row_ptr_h, sk.col_idx_h, vals.cpu().numpy(), sk.n_rows)
        sol = _host_solve(K, rhs.cpu().numpy())
        u = sk.reconstruct(ctx, db, out, torch.as_tensor(sol, device="cuda"))
        ctx.sync()
        u = u.cpu().numpy()
        nodal = [u[db.node_off[e]:db.node_off[e + 1]] for e in range(b["n_elem"])]
        errs.append(oskel.l2_error(b, nodal, manufactured_solution))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    say(f"  errors {errs} rates {rates}")
    assert np.all((rates > 1.8) & (rates < 2.3)), (errs, rates)


def test_empty_batch_is_a_no_op(ctx):
    import torch
    from paper_1703_10435_amd.batch import DeviceBatch
    from tests.test_parity_gpu import _random_batch
    db = DeviceBatch(_random_batch(15, [], [], "empty"))
    z = torch.zeros(1, dtype=torch.float64, device="cuda")
    zi = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.skeleton_scatter(db, z, z, z, z, zi, zi, zi, zi, 1, z, z, zi, zi)
    ctx.reconstruct(db, z, zi, zi, z, 1, z, zi)
    ctx.sync()


# ------------------------------------------------------------ skeleton solve
def _gpu_system(ctx, N, s, l, m, kfun, prec=0):
    from paper_1703_10435_amd import engine
    from paper_1703_10435_amd.skeleton import SkeletonSystem
    mesh = coarse_mesh(N)
    E = mesh["elems"].shape[0]
    b = configs.build_batch(mesh, np.arange(E), np.full(E, s), np.full(E, l), kfun, manufactured_source,
                            m_arr=np.full(E, m))
    res, out, db = engine.solve_batch(b, prec=prec, mode="fused", ctx=ctx)
    sk = SkeletonSystem(mesh, l, p_max=db.p_max, m=m)
    vals, rhs, missing = sk.scatter(ctx, db, out)
    return mesh, b, out, db, sk, vals, rhs


@pytest.mark.parametrize("lambda_block", [None, 1])
@pytest.mark.parametrize("N,s,l,m", [(4, 8, 1, 1), (4, 6, 2, 1), (3, 6, 0, 3), (4, 8, 1, 2), (8, 4, 1, 1)])
def test_skeleton_solve_matches_oracle(ctx, N, s, l, m, lambda_block):
    """MINRES on the device-assembled system against the oracle's dense
    solve of its own assembly: u_0 and lambda within 10 cond(K) times the
    assembly and solve tolerances, the true residual below 1e-10; with the
    face-block preconditioner (default) and the diagonal one (1)."""
    mesh, b, out, db, sk, vals, rhs = _gpu_system(ctx, N, s, l, m, _rough_k)
    say(f"[gpu] skeleton solve N={N} s={s} l={l} m={m} rows={sk.n_rows} lambda_block={lambda_block}")
    sol, it, rr = sk.solve(ctx, vals, rhs, tol=1e-13, lambda_block=lambda_block)
    ctx.sync()
    say(f"  {it} MINRES steps, relative residual {rr:.2e}")
    assert rr < 1e-10
    ora = local.solve_batch(b)
    lam, u0, K, rhs_o = oskel.reduce_and_solve(mesh, ora, np.arange(b["n_elem"]), l, m)
    kappa = np.linalg.cond(K)
    x = sol.cpu().numpy()
    want = np.concatenate([lam, u0])
    bound = 10.0 * kappa * (2 * TOL[0] + 1e-13)
    err = np.abs(x - want).max() / np.abs(want).max()
    say(f"  cond {kappa:.2e}, max rel err {err:.2e} (bound {bound:.2e})")
    assert err <= bound


@pytest.mark.parametrize("N,s,l,m", [(16, 4, 1, 1), (8, 8, 2, 1), (6, 6, 0, 3)])
def test_face_block_preconditioner_takes_fewer_steps(ctx, N, s, l, m):
    """Face blocks of -M and the Jacobi sweeps on B D^-1 B^T: the same
    solution as the diagonal preconditioner in far fewer MINRES steps."""
    mesh, b, out, db, sk, vals, rhs = _gpu_system(ctx, N, s, l, m, _rough_k)
    assert sk.face_dofs == m * (l + 1) > 1
    say(f"[gpu] skeleton preconditioners N={N} s={s} l={l} m={m}")
    sol_d, it_d, rr_d = sk.solve(ctx, vals, rhs, tol=1e-12, lambda_block=1)
    sol_b, it_b, rr_b = sk.solve(ctx, vals, rhs, tol=1e-12)
    ctx.sync()
    say(f"  diagonal: {it_d} steps, residual {rr_d:.2e}; face blocks: {it_b} steps, residual {rr_b:.2e}")
    assert rr_d < 1e-9 and rr_b < 1e-9
    assert it_b < it_d
    u_d = sk.reconstruct(ctx, db, out, sol_d).cpu().numpy()
    u_b = sk.reconstruct(ctx, db, out, sol_b).cpu().numpy()
    assert np.abs(u_b - u_d).max() <= 1e-7 * np.abs(u_d).max()


@pytest.mark.parametrize("N", [48, 68])
def test_schur_preconditioner_on_large_meshes(ctx, N):
    """More elements than the Chebyshev steps hold in registers: 4,608
    elements re-read their rows of S each step, 9,248 take the diagonal of
    S.  The solve reaches a small true residual (computed on the device from
    the CSR system) and u is finite."""
    mesh, b, out, db, sk, vals, rhs = _gpu_system(ctx, N, 2, 1, 1, _ones)
    say(f"[gpu] skeleton preconditioner paths N={N} elements={b['n_elem']} rows={sk.n_rows}")
    sol, it, rr = sk.solve(ctx, vals, rhs, tol=1e-11)
    u = sk.reconstruct(ctx, db, out, sol).cpu().numpy()
    ctx.sync()
    say(f"  {it} steps, residual {rr:.2e}")
    assert rr < 1e-8
    assert np.all(np.isfinite(u))


def test_skeleton_solve_singular_multiplier_block(ctx):
    """l = s: the multiplier block is rank deficient; u (through the
    reconstruction) is still unique and matches the oracle."""
    N, s, l = 2, 2, 2
    mesh, b, out, db, sk, vals, rhs = _gpu_system(ctx, N, s, l, 1, _rough_k)
    say("[gpu] skeleton solve, singular multiplier block")
    sol, it, rr = sk.solve(ctx, vals, rhs, tol=1e-13)
    u = sk.reconstruct(ctx, db, out, sol)
    ctx.sync()
    assert rr < 1e-9, rr
    ora = local.solve_batch(b)
    lam, u0, K, _ = oskel.reduce_and_solve(mesh, ora, np.arange(b["n_elem"]), l)
    want = oskel.reconstruct(mesh, ora, np.arange(b["n_elem"]), l, lam, u0)
    u = u.cpu().numpy()
    scale = max(np.abs(w).max() for w in want)
    for e in range(b["n_elem"]):
        assert np.abs(u[db.node_off[e]:db.node_off[e + 1]] - want[e]).max() <= 1e-8 * scale, e


@pytest.mark.parametrize("prec", [0, 1])
def test_device_chain_converges_at_second_order(ctx, prec):
    """Every step on the device: local solves, scatter, MINRES, reconstruction."""
    errs, its = [], []
    for N in (2, 4, 8, 16):
        mesh, b, out, db, sk, vals, rhs = _gpu_system(ctx, N, 4, 1, 1, _ones, prec)
        say(f"[gpu] device chain N={N} prec={prec}")
        sol, it, rr = sk.solve(ctx, vals, rhs, tol=1e-12)
        u = sk.reconstruct(ctx, db, out, sol)
        ctx.sync()
        assert rr < 1e-9
        its.append(it)
        u = u.cpu().numpy()
        errs.append(oskel.l2_error(b, [u[db.node_off[e]:db.node_off[e + 1]] for e in range(b["n_elem"])],
                                   manufactured_solution))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    say(f"  errors {errs} rates {rates} MINRES steps {its}")
    assert np.all((rates > 1.8) & (rates < 2.3)), (errs, rates)


def test_skeleton_solve_edge_cases(ctx):
    import torch
    from paper_1703_10435_amd import abi
    mesh, b, out, db, sk, vals, rhs = _gpu_system(ctx, 2, 3, 1, 1, _ones)
    say("[gpu] skeleton solve edge cases")
    sol, it, rr = sk.solve(ctx, vals, torch.zeros_like(rhs))
    ctx.sync()
    assert it == 0 and rr == 0.0 and not torch.any(sol != 0).item()
    bad = sk.col_idx.clone()
    bad[5] = sk.n_rows + 3
    sol = torch.empty(sk.n_rows, dtype=torch.float64, device="cuda")
    with pytest.raises(abi.MhmError, match="out of range"):
        ctx.skeleton_solve(sk.n_rows, sk.n_lambda, sk.row_ptr, bad, vals, rhs, sol)
    for pb in (0, 9, 5):   # outside [1, 8]; not a divisor of n_lambda (2 per face here, 16 faces)
        with pytest.raises(abi.MhmError, match="lambda_block"):
            ctx.skeleton_solve(sk.n_rows, sk.n_lambda, sk.row_ptr, sk.col_idx, vals, rhs, sol, lambda_block=pb)
    it, rr = ctx.skeleton_solve(0, 0, None, None, None, None, None)
    assert it == 0
