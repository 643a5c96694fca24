"""GPU tests of the batching layer: ragged batches binned into size classes,
every kernel family, HIP-graph replays and the autotuner, each checked
against the FP64 oracle (or bit for bit against the eager run of the same
launch configuration)."""
from __future__ import annotations

import json

import numpy as np
import pytest

from mhm_inputs import configs
from mhm_inputs.configs import sub_batch
from oracle import local
from tests.parity_util import ensure_built, rel_errors, say
from tests.test_parity_gpu import TOL, _check, _random_batch

pytestmark = pytest.mark.gpu

# one or two elements in every size class (s <= 16, 17-25, 26-33, 34-48, 49-64)
S_ALL = [2, 16, 17, 25, 26, 33, 34, 48, 8, 20, 52]
L_ALL = [1, 3, 0, 2, 4, 1, 3, 2, 0, 4, 1]


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


def _fused(ctx, db, prec, out=None):
    from paper_1703_10435_amd import engine
    return engine.run_fused(ctx, db, prec, out)


def _snapshot(out, E):
    return {k: out[k].detach().cpu().numpy().copy() for k in ("X", "M", "E", "B", "F", "info")}


@pytest.mark.parametrize("prec", [0, 1])
def test_every_size_class_in_one_batch(ctx, prec):
    from paper_1703_10435_amd import engine
    b = _random_batch(21, S_ALL, L_ALL, "all-classes")
    for mode in ("fused", "three_call"):
        say(f"[gpu] all-classes prec={prec} mode={mode}")
        res, out, db = engine.solve_batch(b, prec=prec, mode=mode, ctx=ctx)
        _check(res, b, range(b["n_elem"]), prec, f"all-classes prec={prec} {mode}")


@pytest.mark.parametrize("opts", [{"no_rr": 1}, {"no_ll": 1}, {"no_rr": 1, "no_ll": 1},
                                 {"no_rr": 1, "ll_occ2": 1}, {"ll_nw16": 1}, {"ll_pw": 1},
                                 {"ll_pw": 4}])
def test_kernel_families_agree_with_oracle(opts):
    """The families the defaults do not pick (LDS tiles for small FP64
    elements, the right-looking workspace kernel for large ones, the
    left-looking kernel built for two workgroups per CU, with 16 waves, with
    one-tile panels in FP64 and two-tile panels in FP32 at s = 48, or with
    four-tile FP64 panels taken in five row passes)."""
    from paper_1703_10435_amd import engine
    c = _ctx(opts)
    try:
        b = _random_batch(22, [5, 12, 16, 20, 30, 40, 48], [2, 1, 3, 0, 2, 3, 1], "families")
        for prec in (0, 1):
            say(f"[gpu] families opts={opts} prec={prec}")
            res, out, db = engine.solve_batch(b, prec=prec, mode="fused", ctx=c)
            _check(res, b, range(b["n_elem"]), prec, f"families {opts} prec={prec}")
    finally:
        c.close()


@pytest.mark.parametrize("occ", ["2", "3"])
@pytest.mark.parametrize("mode", ["fused", "three"])
def test_register_tile_kernel_both_occupancies(occ, mode):
    """The FP64 register-tile kernel built for two (the default) and for
    three resident workgroups per CU (a tuner candidate), fused and as the
    three calls."""
    from paper_1703_10435_amd import engine
    c = _ctx({"rr_occ": int(occ)})
    try:
        b = _random_batch(26, [2, 5, 9, 12, 16, 16, 7], [0, 1, 2, 3, 2, 3, 1], "occupancy")
        say(f"[gpu] register tiles occ={occ} mode={mode}")
        res, out, db = engine.solve_batch(b, prec=0, mode=mode, ctx=c)
        _check(res, b, range(b["n_elem"]), 0, f"register tiles occ={occ} {mode}")
    finally:
        c.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replays_match_eager(ctx, prec):
    import torch
    from paper_1703_10435_amd import engine
    from paper_1703_10435_amd.batch import DeviceBatch
    b = _random_batch(23, S_ALL[:8], L_ALL[:8], "graph")
    db = DeviceBatch(b)
    say(f"[gpu] graph eager prec={prec}")
    ref_out = _fused(ctx, db, prec)
    ctx.sync()
    ref = _snapshot(ref_out, b["n_elem"])
    g, out = engine.capture_fused(ctx, db, prec)
    try:
        for rep in range(3):
            for k in ("X", "M", "E", "B", "F"):
                out[k].fill_(float("nan"))
            out["info"].fill_(99)
            # unrelated eager work and a synchronisation between replays
            junk = torch.randn(1 << 16, device="cuda", dtype=torch.float64)
            _ = (junk * junk).sum().item()
            say(f"[gpu] graph replay {rep} prec={prec}")
            g.launch()
            ctx.sync()
            got = _snapshot(out, b["n_elem"])
            for k in ref:
                np.testing.assert_array_equal(got[k], ref[k], err_msg=f"replay {rep} {k}")
    finally:
        g.close()
    res = db.unpack(out)
    _check(res, b, range(b["n_elem"]), prec, f"graph prec={prec}")


def test_graph_of_uniform_batch(ctx):
    """One size class: the graph holds a single launch (no binning)."""
    from paper_1703_10435_amd import engine
    from paper_1703_10435_amd.batch import DeviceBatch
    b = configs.make("C2", n_elem=64)
    db = DeviceBatch(b)
    say("[gpu] graph uniform C2[:64]")
    g, out = engine.capture_fused(ctx, db, 0)
    try:
        g.launch()
        g.launch()
        ctx.sync()
    finally:
        g.close()
    res = db.unpack(out)
    _check(res, b, [0, 31, 63], 0, "graph uniform")


def test_autotune_report_and_results(ctx):
    from paper_1703_10435_amd import engine
    from paper_1703_10435_amd.batch import DeviceBatch
    b = _random_batch(24, S_ALL[:8] * 2, L_ALL[:8] * 2, "tune")
    db = DeviceBatch(b)
    for prec in (0, 1):
        say(f"[gpu] autotune prec={prec}")
        out = engine.autotune(ctx, db, prec)
        ctx.sync()
        rep = json.loads(ctx.tune_report())
        assert rep, "autotuning timed no candidate"
        for r in rep:
            assert r["ms"] > 0 and r["elements"] > 0 and r["kernel"] in (
                "register-tiles", "lds-tiles", "left-looking", "workspace"), r
        _check(db.unpack(out), b, range(b["n_elem"]), prec, f"autotune prec={prec}")
        # later runs use the tuned choices
        out2 = _fused(ctx, db, prec)
        ctx.sync()
        _check(db.unpack(out2), b, range(b["n_elem"]), prec, f"tuned run prec={prec}")


def test_c4_graph_sampled(ctx):
    """The uneven 8192-element batch (s in {8,16,32,48}, l in {1,2,3}) in one
    graph launch, FP32 + refinement and FP64, sampled per size class."""
    from paper_1703_10435_amd import engine
    from paper_1703_10435_amd.batch import DeviceBatch
    b = configs.make("C4")
    db = DeviceBatch(b)
    rng = np.random.default_rng(7)
    idx = []
    for s in configs.C4_SIZES:
        ids = np.flatnonzero(b["s"] == s)
        idx += list(rng.choice(ids, size=3, replace=False))
    for prec in (1, 0):
        say(f"[gpu] C4 graph prec={prec}")
        g, out = engine.capture_fused(ctx, db, prec)
        try:
            g.launch()
            ctx.sync()
        finally:
            g.close()
        info = out["info"].cpu().numpy()[:b["n_elem"]]
        assert np.all((info == 0) | (info == -1)), np.unique(info)
        res = db.unpack(out)
        _check(res, b, idx, prec, f"C4 graph prec={prec}")


def test_bucketed_alone_vs_mixed_bitwise(ctx):
    """An element's results do not depend on the other elements of its batch
    as long as its size class launch is the same."""
    b = _random_batch(25, S_ALL, L_ALL, "mix")
    from paper_1703_10435_amd import engine
    full, _, _ = engine.solve_batch(b, prec=0, mode="fused", ctx=ctx)
    for e in (1, 3, 7):
        # a batch of the element plus one element of the smallest class keeps
        # the element in its own class launch
        sb = sub_batch(b, [0, e])
        alone, _, _ = engine.solve_batch(sb, prec=0, mode="fused", ctx=ctx)
        np.testing.assert_array_equal(alone[1]["X"], full[e]["X"])
        np.testing.assert_array_equal(alone[1]["M"], full[e]["M"])


@pytest.mark.parametrize("prec", [0, 1])
def test_concurrent_classes_match_serial_bitwise(ctx, prec):
    """The size classes on forked streams (MHM_OPT_CONCURRENT_CLASSES) give
    the same bits as the default, one class after another."""
    from paper_1703_10435_amd import engine
    b = _random_batch(27, S_ALL, L_ALL, "concurrent")
    say(f"[gpu] concurrent classes prec={prec}")
    # fresh contexts: the module's context carries an earlier test's tuning
    c0, c = _ctx(), _ctx({"concurrent_classes": 1})
    try:
        serial, _, _ = engine.solve_batch(b, prec=prec, mode="fused", ctx=c0)
        conc, _, _ = engine.solve_batch(b, prec=prec, mode="fused", ctx=c)
    finally:
        c.close()
        c0.close()
    for e in range(b["n_elem"]):
        for k in ("X", "M", "E", "B"):
            np.testing.assert_array_equal(conc[e][k], serial[e][k])
        assert conc[e]["info"] == serial[e]["info"]
