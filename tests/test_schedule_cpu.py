"""The left-looking kernel's schedule, checked on the host (model in
ll_schedule_model.py): for the instances the library launches, every
wave's workspace, LDS, X and (non-fused) Ahat accesses stay inside their
buffers, no two waves touch the same entries between two barriers with one
of them writing, every wave passes the same barriers, and the non-fused form
never reads an operator entry after the factor was written over it.  The
model's own tests plant mistakes (a dropped barrier, a short LDS allocation,
a misplaced published tile) and check that each is found."""
from __future__ import annotations

import pytest

from tests.ll_schedule_model import Instance, Launch, check, launch_rows, simulate

# (fp32, panel width, s of the launch class, l_max, elements' s, refining instance)
CASES = [
    (False, 4, 48, 3, [48, 34], False),   # C4's s = 48 class (FP64 default)
    (False, 2, 48, 3, [48], True),        # the FP64 refinement pass at s = 48
    (False, 4, 33, 3, [32, 26], False),   # s <= 33 class (FP64 default: four-tile panels, ten-row instance)
    (False, 2, 33, 3, [32, 26], False),   # the same class with two-tile panels (the tuner's other choice)
    (False, 2, 33, 3, [32], True),
    (False, 2, 16, 2, [10, 12, 16], True),   # the refinement pass over small deferred elements
    (True, 4, 48, 3, [48, 40], False),    # FP32 + refinement
    (True, 4, 33, 3, [32], False),
    (True, 2, 25, 2, [20, 25], False),
]


def _run(fp32, pw, s_cap, l_max, s, ref, **kw):
    nt = ((s_cap + 1) * (s_cap + 2) // 2 + 15) // 16
    inst = Instance(fp32=fp32, pw=pw, rpw=launch_rows(fp32, pw, nt, ref), ref=ref, fused=not kw.get("three_call", False))
    logs, meta = simulate(inst, Launch.for_class(s_cap, l_max), s, l_max, ref64=ref, **kw)
    return check(logs, meta)


@pytest.mark.parametrize("fp32,pw,s_cap,l_max,sizes,ref", CASES)
def test_left_looking_schedule_has_no_race(fp32, pw, s_cap, l_max, sizes, ref):
    for s in sizes:
        probs = _run(fp32, pw, s_cap, l_max, s, ref)
        assert not probs, (s, probs[:5])


@pytest.mark.parametrize("fp32,pw", [(False, 2), (False, 4), (True, 2), (True, 4)])
def test_three_call_form_reads_the_operator_before_writing_the_factor(fp32, pw):
    """Non-fused: the operator tiles come from Ahat and the factor goes back
    into the same array after the factorisation; also with the factor
    written from inside the factorisation (the earlier schedule), where the
    model finds no read-after-overwrite either."""
    for lo_inside in (False, True):
        probs = _run(fp32, pw, 48, 2, 40, False, three_call=True, lo_inside=lo_inside)
        assert not probs, (lo_inside, probs[:5])


def test_model_finds_a_dropped_barrier():
    probs = _run(False, 2, 33, 3, 32, False, drop=("panel solve",))
    assert any("publish" in p and "in-panel pub" in p for p in probs), probs[:3]
    probs = _run(False, 2, 33, 3, 32, False, drop=("backward step",))
    assert any("backward" in p for p in probs), probs[:3]
    probs = _run(False, 2, 33, 3, 32, True, drop=("accumulate 0 a", "accumulate 0 b"))
    assert any("residual" in p and "accumulate" in p for p in probs), probs[:3]


def test_model_finds_a_short_lds_allocation():
    probs = _run(False, 4, 48, 3, 48, False, lds_short=1)
    assert any("outside" in p and "lds" in p for p in probs), probs[:3]


def test_model_finds_a_misplaced_published_tile():
    probs = _run(False, 2, 33, 3, 32, False, publish_shift=1)
    assert probs, "a shifted publish slot went unnoticed"


def test_model_finds_a_barrier_only_some_waves_pass():
    """A row pass skipped by some waves only (here: a pass cut at the wrong
    row) leaves the waves with different barrier sequences."""
    from tests import ll_schedule_model as m
    inst = Instance(fp32=False, pw=4, rpw=10)
    logs, meta = m.simulate(inst, Launch.for_class(48, 3), 48, 3)
    logs[3].barriers.pop(10)
    assert any("barrier sequence" in p for p in check(logs, meta))


# ---------------------------------------------------------------- k_local
@pytest.mark.parametrize("s,l,fp32,fused,three_call", [
    (4, 1, True, True, False), (16, 2, True, True, False), (16, 2, False, True, False),
    (12, 2, False, False, True), (16, 2, True, False, True), (25, 3, True, True, False)])
def test_local_kernel_schedule_has_no_race(s, l, fp32, fused, three_call):
    """The right-looking tile kernel (LDS or workspace tiles): fill, panel,
    trailing update with the look-ahead diagonal factorisation, sweeps,
    refinement; the three-call form reads all of Ahat before writing L."""
    from tests.local_schedule_model import simulate as lsim
    logs, meta = lsim(s, l, fp32, fused, three_call=three_call)
    assert not check(logs, meta)


def test_local_model_finds_planted_mistakes():
    from tests.local_schedule_model import simulate as lsim
    logs, meta = lsim(16, 2, True, True, trail_skip_first=False)   # waves 1-3 also take tile (k+1, k+1)
    assert any("look-ahead" in p or "diagonal factor" in p for p in check(logs, meta))
    logs, meta = lsim(16, 2, True, True, drop=("panel",))
    assert any("panel" in p and "trailing" in p for p in check(logs, meta))
    logs, meta = lsim(16, 2, True, True, drop=("fill a",))
    assert any("stencil add" in p for p in check(logs, meta))
