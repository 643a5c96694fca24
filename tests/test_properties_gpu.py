"""Whole-batch properties of the results at the benchmark sizes, on every
element (the oracle checks a sample; these hold for any size):

* B_a = (sigma_e psi_a, 1)_{F_e}: sigma_e |F_e| / m for the degree-0 DoF of
  each face segment and 0 for q >= 1 (Legendre orthogonality; eq. (6));
* F = (f, 1)_K, the centroid rule over the sub-triangles;
* the solutions have zero mean, c^T X = 0 (the constraint of the local
  Neumann problems, eqs. (8)-(9));
* M = -R^T X_I is symmetric and negative definite (l + 1 <= s).

The helpers are pinned to the oracle on the CPU (``not gpu`` tests below),
then applied to every element of C4 (fused, both precisions, the headline
workload), C3 (the three calls, both precisions) and C3 with four segments
per face (both forms and precisions)."""
from __future__ import annotations

import numpy as np
import pytest

from tests.parity_util import ensure_built, say

TOL = {0: 1e-10, 1: 1e-8}


def _face_lengths(vert):
    """|F_e| for face e opposite vertex e (v1-v2, v2-v0, v0-v1)."""
    p = vert.reshape(3, 2)
    return np.array([np.linalg.norm(p[2] - p[1]), np.linalg.norm(p[0] - p[2]), np.linalg.norm(p[1] - p[0])])


def _area(vert):
    p = vert.reshape(3, 2)
    return 0.5 * abs((p[1, 0] - p[0, 0]) * (p[2, 1] - p[0, 1]) - (p[2, 0] - p[0, 0]) * (p[1, 1] - p[0, 1]))


def expected_B(batch, e):
    s, l = int(batch["s"][e]), int(batch["l"][e])
    m = int(batch["m"][e]) if batch.get("m") is not None else 1
    L = _face_lengths(batch["vert"][e])
    P = m * (l + 1)
    B = np.zeros(3 * P)
    for f in range(3):
        for seg in range(m):
            B[f * P + seg * (l + 1)] = float(batch["sigma"][e][f]) * L[f] / m
    return B


def expected_F(batch, e):
    s = int(batch["s"][e])
    t0, t1 = batch["tri_off"][e], batch["tri_off"][e + 1]
    return _area(batch["vert"][e]) / (s * s) * float(np.sum(batch["f"][t0:t1]))


_COUNTS = {}


def _node_counts(s):
    if s not in _COUNTS:
        w = []
        for j in range(s + 1):
            for i in range(s + 1 - j):
                corner = (i, j) in ((0, 0), (s, 0), (0, s))
                edge = j == 0 or i == 0 or i + j == s
                w.append(1 if corner else 3 if edge else 6)
        _COUNTS[s] = np.asarray(w, dtype=np.float64)
    return _COUNTS[s]


def mass_weights(batch, e):
    """c_j = |K| / (3 s^2) times the number of sub-triangles at node j (1 at
    a corner, 3 on an edge, 6 inside), in lattice order (row j, then i)."""
    s = int(batch["s"][e])
    return _area(batch["vert"][e]) / (3.0 * s * s) * _node_counts(s)


def check_properties(res, batch, prec, label):
    tol = TOL[prec]
    worst = dict(B=0.0, F=0.0, mean=0.0, sym=0.0, eig=-np.inf)
    Ms = {}
    for e, r in enumerate(res):
        assert r["info"] in (0, -1), (label, e, r["info"])
        Bx = expected_B(batch, e)
        dB = np.max(np.abs(r["B"] - Bx)) / np.max(np.abs(Bx))
        dF = abs(r["F"] - expected_F(batch, e)) / max(abs(expected_F(batch, e)), 1e-300)
        c = mass_weights(batch, e)
        X = r["X"]
        # relative to the element's whole block (a column can vanish: with a
        # constant f the projected source column is zero)
        dm = np.max(np.abs(c @ X)) / max(float(np.max(np.abs(c) @ np.abs(X))), 1e-300)
        M = r["M"]
        ds = np.max(np.abs(M - M.T)) / np.max(np.abs(M))
        assert dB <= 1e-12 and dF <= 1e-12 and dm <= 1e-11 and ds <= tol, (label, e, dB, dF, dm, ds)
        worst.update(B=max(worst["B"], dB), F=max(worst["F"], dF), mean=max(worst["mean"], dm),
                     sym=max(worst["sym"], ds))
        Ms.setdefault(M.shape[0], []).append(0.5 * (M + M.T))
    for ni, lst in Ms.items():
        lam = np.linalg.eigvalsh(np.stack(lst))
        rel = lam[:, -1] / np.abs(lam[:, 0])   # largest eigenvalue over the largest magnitude
        worst["eig"] = max(worst["eig"], float(rel.max()))
        assert np.all(lam[:, -1] < 0.0), (label, ni, float(lam[:, -1].max()))
    say(f"  {label}: {len(res)} elements; B {worst['B']:.1e}, F {worst['F']:.1e}, c^T X {worst['mean']:.1e}, "
        f"M asym {worst['sym']:.1e}, max eig / |min eig| {worst['eig']:.2e}")


# ------------------------------------------------ pins of the helpers (CPU)
@pytest.mark.parametrize("cfg,elems", [("C1", [0, 7, 31]), ("C4", [0, 1, 2, 3])])
def test_property_helpers_match_the_oracle(cfg, elems):
    from mhm_inputs import configs
    from oracle import local
    b = configs.make(cfg)
    if cfg == "C4":   # the smallest elements of C4 (s = 8, 16) keep the oracle quick
        small = np.flatnonzero(b["s"] <= 16)[: len(elems)]
        b = configs.sub_batch(b, small)
    for e in range(len(elems)) if cfg == "C4" else elems:
        ora = local.solve_element(b, e)
        np.testing.assert_allclose(expected_B(b, e), ora["B"], rtol=0, atol=1e-13 * np.max(np.abs(ora["B"])))
        assert abs(expected_F(b, e) - ora["F"]) <= 1e-13 * max(abs(ora["F"]), 1.0)
        c = mass_weights(b, e)
        np.testing.assert_allclose(c, ora["c"], rtol=1e-13, atol=0)
        assert abs(c.sum() - ora["area"]) <= 1e-14 * ora["area"]
        X = ora["X"]
        assert np.max(np.abs(c @ X)) <= 1e-12 * np.max(np.abs(c) @ np.abs(X))
        M = ora["M"]
        assert np.max(np.abs(M - M.T)) <= 1e-12 * np.max(np.abs(M))
        assert np.linalg.eigvalsh(0.5 * (M + M.T))[-1] < 0.0


def test_property_check_catches_a_planted_mistake():
    """A wrong sign of one face's B, a shifted X column and an asymmetric M
    each fail the check (mistakes planted in oracle results on the CPU)."""
    from mhm_inputs import configs
    from oracle import local
    b = configs.make("C1")
    good = [dict(X=o["X"], M=o["M"], B=o["B"], F=o["F"], info=0) for o in local.solve_batch(b, [0, 1])]
    check_properties(good, configs.sub_batch(b, np.arange(2)), 0, "oracle")
    sb = configs.sub_batch(b, np.arange(2))
    for plant in ("B", "X", "M"):
        bad = [dict(r) for r in good]
        if plant == "B":
            bad[1]["B"] = bad[1]["B"].copy()
            bad[1]["B"][0] = -bad[1]["B"][0]
        elif plant == "X":
            bad[1]["X"] = bad[1]["X"] + 1e-3 * np.max(np.abs(bad[1]["X"]))
        else:
            bad[1]["M"] = bad[1]["M"].copy()
            bad[1]["M"][0, 1] *= 1.0 + 1e-6
        with pytest.raises(AssertionError):
            check_properties(bad, sb, 0, f"planted {plant}")


# ------------------------------------------------------ every element (GPU)
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


@pytest.mark.gpu
@pytest.mark.parametrize("cfg,mode", [("C4", "fused"), ("C3", "three_call"), ("W", "fused"), ("W", "three_call")])
@pytest.mark.parametrize("prec", [0, 1])
def test_every_element_of_the_benchmark_batches(ctx, cfg, mode, prec):
    """W: C3's mesh and fields with m = 4 segments per face (N_I = 48, 49
    right-hand sides in four 16-column chunks)."""
    from mhm_inputs import configs
    from paper_1703_10435_amd import engine
    if cfg == "W":
        b = configs.make("C3")
        b["m"] = np.full(b["n_elem"], 4, dtype=np.int32)
    else:
        b = configs.make(cfg)
    say(f"[gpu] {cfg} all {b['n_elem']} elements prec={prec} mode={mode}")
    res, out, db = engine.solve_batch(b, prec=prec, mode=mode, ctx=ctx)
    check_properties(res, b, prec, f"{cfg} prec={prec} {mode}")
