"""GPU tests of factor reuse over time steps (Section 3: with coefficients
that do not change in time the local matrix is assembled and factored once,
in the first step, and later steps only build and solve their load vectors).
Every step is compared with the FP64 oracle for that step's source and face
degree."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import local
from tests.parity_util import ensure_built, rel_errors, say
from tests.test_parity_gpu import TOL, _random_batch

pytestmark = pytest.mark.gpu


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


def _check_all(res, b, prec, label, elems=None):
    worst = 0.0
    for e in (range(b["n_elem"]) if elems is None else elems):
        ora = local.solve_element(b, e)
        assert res[e]["info"] in (0, -1), (label, e, res[e]["info"])
        ex, eb = rel_errors(res[e], ora)
        assert ex <= TOL[prec] and eb <= TOL[prec], (label, e, ex, eb)
        worst = max(worst, ex, eb)
    return worst


@pytest.mark.parametrize("prec", [0, 1])
def test_time_steps_reuse_the_first_factor(ctx, prec):
    import torch
    from paper_1703_10435_amd import engine
    from paper_1703_10435_amd.batch import DeviceBatch
    s_list, l_list = [5, 16, 24, 33, 48, 9], [2, 1, 3, 0, 2, 4]
    b = _random_batch(31, s_list, l_list, "steps")
    db = DeviceBatch(b)
    fs = engine.FactorStore(db, prec)
    rng = np.random.default_rng(32)
    say(f"[gpu] reuse step 0 prec={prec}")
    out = engine.run_cached(ctx, db, fs)
    ctx.sync()
    assert int(fs.state[:b["n_elem"]].sum().item()) >= 1
    _check_all(db.unpack(out), b, prec, "step 0")
    for step in (1, 2, 3):
        f = rng.standard_normal(b["f"].shape)
        bs = dict(b, f=f)
        if step == 2:                      # another face degree on the same factors
            bs["l"] = np.asarray([4, 0, 1, 2, 3, 1], dtype=np.int32)
            dstep = DeviceBatch(bs)
        else:
            dstep = engine.with_source(db, torch.as_tensor(f, device="cuda"))
        say(f"[gpu] reuse step {step} prec={prec}")
        out = engine.run_cached(ctx, dstep, fs)
        ctx.sync()
        w = _check_all(dstep.unpack(out), bs, prec, f"step {step}")
        say(f"  step {step}: worst rel err {w:.2e}")


def test_reused_factor_matches_fresh_factor(ctx):
    """A reuse step gives the results of factoring afresh (FP64, within the
    rounding of the two solves)."""
    import torch
    from paper_1703_10435_amd import engine
    from paper_1703_10435_amd.batch import DeviceBatch
    b = _random_batch(33, [12, 20, 40], [1, 2, 3], "fresh")
    db = DeviceBatch(b)
    fs = engine.FactorStore(db, 0)
    engine.run_cached(ctx, db, fs)
    f = np.random.default_rng(34).standard_normal(b["f"].shape)
    dstep = engine.with_source(db, torch.as_tensor(f, device="cuda"))
    say("[gpu] reuse vs fresh")
    reuse = dstep.unpack(engine.run_cached(ctx, dstep, fs))
    fresh_fs = engine.FactorStore(db, 0)
    fresh = dstep.unpack(engine.run_cached(ctx, dstep, fresh_fs))
    ctx.sync()
    for e in range(b["n_elem"]):
        ex, eb = rel_errors(reuse[e], fresh[e])
        assert ex <= 1e-13 and eb <= 1e-13, (e, ex, eb)


@pytest.mark.parametrize("prec", [0, 1])
def test_source_only_steps_match_oracle(ctx, prec):
    """Time steps that only change f: the source column of X, E and F are
    recomputed on the stored factors, the multiplier columns, M and B stay
    those of the first step, and the whole result equals the oracle's for
    the new source."""
    import torch
    from paper_1703_10435_amd import engine
    from paper_1703_10435_amd.batch import DeviceBatch
    s_list, l_list = [1, 5, 16, 17, 24, 33, 48, 9, 3], [2, 1, 3, 0, 2, 4, 1, 0, 2]
    b = _random_batch(35, s_list, l_list, "source-steps")
    db = DeviceBatch(b)
    fs = engine.FactorStore(db, prec)
    out = engine.run_cached(ctx, db, fs)
    ctx.sync()
    held = fs.state[:b["n_elem"]].cpu().numpy() == 1      # factors kept by the first step
    assert held.sum() >= b["n_elem"] - 1, held
    first = {k: out[k].cpu().numpy().copy() for k in ("X", "M", "B")}
    NI = db.NImax
    rng = np.random.default_rng(36)
    for step in (1, 2):
        f = rng.standard_normal(b["f"].shape)
        bs = dict(b, f=f)
        dstep = engine.with_source(db, torch.as_tensor(f, device="cuda"))
        say(f"[gpu] source-only step {step} prec={prec}")
        engine.source_step(ctx, dstep, fs, out)
        ctx.sync()
        info = out["info"].cpu().numpy()[:b["n_elem"]]
        assert np.all(info[~held] == -4) and np.all((info[held] == 0) | (info[held] == -1)), info
        res = dstep.unpack(out)
        w = _check_all(res, bs, prec, f"source step {step}", np.flatnonzero(held))
        say(f"  step {step}: worst rel err {w:.2e}, info {info.tolist()}, "
            f"iters {out['ir_iters'].cpu().numpy()[:b['n_elem']].tolist()}")
        X, M, B = (out[k].cpu().numpy() for k in ("X", "M", "B"))
        for e in np.flatnonzero(info == 0):     # untouched: multiplier columns, M, B
            o0, n, r = int(db.rhs_off[e]), int(db.n[e]), int(db.r[e])
            np.testing.assert_array_equal(X[o0:o0 + (r - 1) * n], first["X"][o0:o0 + (r - 1) * n])
            np.testing.assert_array_equal(M[e * NI * NI:(e + 1) * NI * NI], first["M"][e * NI * NI:(e + 1) * NI * NI])
            np.testing.assert_array_equal(B[e * NI:(e + 1) * NI], first["B"][e * NI:(e + 1) * NI])


def test_source_step_without_factor_reports_and_skips(ctx):
    import torch
    from paper_1703_10435_amd import engine
    from paper_1703_10435_amd.batch import DeviceBatch
    b = _random_batch(37, [6, 10, 14], [1, 2, 1], "no-factor")
    db = DeviceBatch(b)
    fs = engine.FactorStore(db, 0)
    out = engine.run_cached(ctx, db, fs)
    fs.state[1] = 0                                      # element 1: no valid factor
    ctx.sync()
    before = out["E"].clone()
    f = np.random.default_rng(38).standard_normal(b["f"].shape)
    dstep = engine.with_source(db, torch.as_tensor(f, device="cuda"))
    say("[gpu] source step with a missing factor")
    engine.source_step(ctx, dstep, fs, out)
    ctx.sync()
    info = out["info"].cpu().numpy()[:3]
    assert info.tolist() == [0, -4, 0], info
    NI = db.NImax
    np.testing.assert_array_equal(out["E"][NI:2 * NI].cpu().numpy(), before[NI:2 * NI].cpu().numpy())
    bs = dict(b, f=f)
    res = dstep.unpack(out)
    for e in (0, 2):
        ex, eb = rel_errors(res[e], local.solve_element(bs, e))
        assert ex <= TOL[0] and eb <= TOL[0], (e, ex, eb)


@pytest.mark.parametrize("prec", [0, 1])
def test_stored_factors_beyond_the_left_looking_range_are_refused(ctx, prec):
    """Factors are stored only by the left-looking kernel (s <= 48): a batch
    with a larger element is refused with MHM_E_UNSUPPORTED before anything
    is launched, both for the factoring call and for a source step, and the
    context stays usable."""
    from paper_1703_10435_amd import abi, engine
    from paper_1703_10435_amd.batch import DeviceBatch
    b = _random_batch(39, [16, 52], [1, 1], "cached-too-large")
    db = DeviceBatch(b)
    fs = engine.FactorStore(db, prec)
    say(f"[gpu] stored factors with s = 52 prec={prec} (refused on the host)")
    with pytest.raises(abi.MhmError) as ei:
        engine.run_cached(ctx, db, fs)
    assert ei.value.status == abi.MHM_E_UNSUPPORTED
    out = db.alloc_outputs(three_call=False)
    with pytest.raises(abi.MhmError) as ei:
        engine.source_step(ctx, db, fs, out)
    assert ei.value.status == abi.MHM_E_UNSUPPORTED
    ok = _random_batch(40, [16, 24], [1, 2], "cached-after-refusal")
    dok = DeviceBatch(ok)
    fok = engine.FactorStore(dok, prec)
    res = dok.unpack(engine.run_cached(ctx, dok, fok))
    ctx.sync()
    _check_all(res, ok, prec, "after refusal")
