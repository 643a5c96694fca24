"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these compares the oracle with itself: each one checks a closed form,
an invariant, an exact worked example, a reduction to a textbook method, or a
convergence rate.  They run on the CPU only.
"""
from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np
import pytest

from mhm_inputs import configs
from mhm_inputs.fields import manufactured_solution, manufactured_source
from mhm_inputs.mesh import coarse_mesh, element_vertices
from oracle import local, skeleton
from tests import galerkin_ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _ones(p):
    return np.ones(p.shape[:-1])


def _smooth_k(p):
    return 1.0 + 0.5 * np.sin(3.0 * p[..., 0] + 1.0) * np.cos(2.0 * p[..., 1])


def _rand_element(rng, s, l):
    """A random counter-clockwise triangle with log-normal K and random f."""
    while True:
        v = rng.uniform(-1, 1, size=6)
        cross = (v[2] - v[0]) * (v[5] - v[1]) - (v[4] - v[0]) * (v[3] - v[1])
        if abs(cross) > 0.2:
            break
    if cross < 0:
        v = np.array([v[0], v[1], v[4], v[5], v[2], v[3]])
    sigma = rng.choice([-1, 1], size=3).astype(np.int8)
    flip = rng.integers(0, 2, size=3).astype(np.int8)
    kappa = np.exp(rng.standard_normal(s * s))
    f = rng.standard_normal(s * s)
    return v, s, l, sigma, flip, kappa, f


# --------------------------------------------------------------- exact s = 1
def test_s1_exact_rational_worked_example():
    """Oracle == exact rational derivation for one sub-triangle (s = 1, l = 2)."""
    with open(os.path.join(GOLDEN, "s1_triangle_345.json")) as fh:
        g = json.load(fh)
    vert = np.array(g["vert"], dtype=np.float64).ravel()
    r = local.local_problem(vert, 1, g["l"], np.array(g["sigma"], np.int8), np.array(g["flip"], np.int8),
                            np.array([float(Fraction(g["kappa"]))]), np.array([float(Fraction(g["f"]))]))
    for key in ("A", "c", "R", "b", "X", "M", "E", "B"):
        want = np.array([[float(Fraction(x)) for x in row] if isinstance(row, list) else float(Fraction(row))
                         for row in g["values"][key]])
        np.testing.assert_allclose(r[key], want, rtol=1e-13, atol=1e-13, err_msg=key)
    assert r["F"] == pytest.approx(float(Fraction(g["values"]["F"])), rel=1e-14)


def test_golden_fixture_is_reproducible(tmp_path):
    from tests.golden import make_s1_triangle_345 as mk
    out = mk.main(str(tmp_path / "g.json"))
    with open(os.path.join(GOLDEN, "s1_triangle_345.json")) as fh:
        assert json.load(fh)["values"] == out["values"]


# --------------------------------------------------------------------- A, c
@pytest.mark.parametrize("s", [1, 3, 8])
def test_stiffness_symmetric_zero_row_sum(s):
    rng = np.random.default_rng(s)
    v, s, l, sg, fl, kap, f = _rand_element(rng, s, 1)
    A = local.stiffness(v, s, kap)
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    assert np.abs(A.sum(axis=1)).max() <= 1e-13 * np.abs(A).max()
    # positive semi-definite with the constants as its only null vector
    w = np.linalg.eigvalsh(A)
    assert abs(w[0]) < 1e-12 * w[-1] and w[1] > 1e-8 * w[-1]


def test_stiffness_is_five_point_stencil_for_unit_k():
    """K = 1 on a right-isoceles parent: the P1 matrix is the 5-point stencil.
    Couplings along the two axis directions are -1 inside the element and -1/2
    along its boundary (one sub-triangle instead of two), couplings across the
    hypotenuse direction vanish, interior diagonals are 4 and boundary
    diagonals are 0.5, 1 or 2."""
    s = 6
    mesh = coarse_mesh(1)
    for vert in element_vertices(mesh):
        nodes, _ = local.submesh(vert, s)
        A = local.stiffness(vert, s, np.ones(s * s))
        h = 1.0 / s
        on_face = [set(local.face_nodes(e, s)) for e in range(3)]
        boundary = set().union(*on_face)
        for p in range(nodes.shape[0]):
            for q in range(nodes.shape[0]):
                if p == q:
                    continue
                dist = np.hypot(*(nodes[q] - nodes[p]))
                if abs(dist - h) < 1e-12:
                    shared = any(p in fs and q in fs for fs in on_face)
                    assert A[p, q] == pytest.approx(-0.5 if shared else -1.0, abs=1e-13)
                else:
                    assert abs(A[p, q]) < 1e-13
            if p in boundary:
                assert round(A[p, p], 12) in (0.5, 1.0, 2.0)
            else:
                assert A[p, p] == pytest.approx(4.0, abs=1e-13)


@pytest.mark.parametrize("s", [1, 2, 5, 16])
def test_mean_vector_closed_form(s):
    rng = np.random.default_rng(10 + s)
    v = _rand_element(rng, s, 0)[0]
    c = local.mean_vector(v, s)
    area = 0.5 * abs((v[2] - v[0]) * (v[5] - v[1]) - (v[4] - v[0]) * (v[3] - v[1]))
    assert c.sum() == pytest.approx(area, rel=1e-14)
    unit = area / (3.0 * s * s)
    counts = set(np.round(c / unit).astype(int).tolist())
    assert counts <= {1, 3, 6}
    assert np.allclose(c / unit, np.round(c / unit), atol=1e-12)


# ----------------------------------------------------------------- face loads
@pytest.mark.parametrize("s,l", [(1, 0), (4, 1), (7, 3)])
def test_face_load_sum_rule_and_q0_values(s, l):
    rng = np.random.default_rng(20 + s)
    v, s, l, sg, fl, kap, f = _rand_element(rng, s, l)
    R = local.face_loads(v, s, l, sg, fl)
    for e in range(3):
        L = local.face_length(v, e)
        for q in range(l + 1):
            col = R[:, e * (l + 1) + q]
            want = -sg[e] * L if q == 0 else 0.0
            assert col.sum() == pytest.approx(want, abs=1e-13)
        col0 = R[:, e * (l + 1)]
        nodes = local.face_nodes(e, s)
        assert col0[nodes[0]] == pytest.approx(-sg[e] * L / (2 * s))
        assert col0[nodes[-1]] == pytest.approx(-sg[e] * L / (2 * s))
        for k in nodes[1:-1]:
            assert col0[k] == pytest.approx(-sg[e] * L / s)
        others = np.setdiff1d(np.arange(R.shape[0]), nodes)
        assert np.all(R[others, e * (l + 1):(e + 1) * (l + 1)] == 0.0)


@pytest.mark.parametrize("s,l", [(3, 2), (6, 3)])
def test_face_loads_against_gauss_quadrature_moments(s, l):
    """sum_j R[j,(e,q)] g(x_j) = -sigma int_F P_q g ds for every linear g
    (nodal interpolation is exact for linear g); the right side is computed
    with a 10-point Gauss rule in the global face orientation."""
    rng = np.random.default_rng(30 + s)
    v, s, l, sg, fl, kap, f = _rand_element(rng, s, l)
    R = local.face_loads(v, s, l, sg, fl)
    nodes, _ = local.submesh(v, s)
    gx, gw = np.polynomial.legendre.leggauss(10)
    for a_vec in ([1.0, 0.0], [0.0, 1.0], [0.3, -0.7]):
        g = nodes @ np.array(a_vec) + 0.25
        for e in range(3):
            p_start = v[2 * ((e + 1) % 3): 2 * ((e + 1) % 3) + 2]
            p_end = v[2 * ((e + 2) % 3): 2 * ((e + 2) % 3) + 2]
            L = np.hypot(*(p_end - p_start))
            lo, hi = (p_end, p_start) if fl[e] else (p_start, p_end)   # t = -1 at 'lo'
            pts = lo[None, :] + 0.5 * (gx[:, None] + 1.0) * (hi - lo)[None, :]
            gval = pts @ np.array(a_vec) + 0.25
            for q in range(l + 1):
                Pq = np.polynomial.legendre.legval(gx, [0] * q + [1])
                want = -sg[e] * 0.5 * L * np.sum(gw * Pq * gval)
                got = R[:, e * (l + 1) + q] @ g
                assert got == pytest.approx(want, abs=1e-13)


@pytest.mark.parametrize("s,l,m", [(4, 0, 2), (6, 1, 2), (8, 0, 4), (6, 1, 3), (5, 0, 5)])
def test_segmented_face_loads_against_gauss_quadrature(s, l, m):
    """m segments per face: sum_j R[j,a] g(x_j) = -sigma int_{segment} P_q(t) g ds
    for every linear g, t running over [-1, 1] on the segment in the global
    face orientation; 10-point Gauss rule per segment, points placed from
    the coordinates (this pins segment placement, order, orientation and
    sign independently of the oracle's polynomial algebra)."""
    rng = np.random.default_rng(40 + s + m)
    v, s, l, sg, fl, kap, f = _rand_element(rng, s, l)
    R = local.face_loads(v, s, l, sg, fl, m)
    Bv = local.face_moments(v, l, sg, fl, m)
    assert R.shape[1] == 3 * m * (l + 1)
    nodes, _ = local.submesh(v, s)
    gx, gw = np.polynomial.legendre.leggauss(10)
    for a_vec in ([1.0, 0.0], [0.0, 1.0], [0.3, -0.7]):
        g = nodes @ np.array(a_vec) + 0.25
        for e in range(3):
            p_start = v[2 * ((e + 1) % 3): 2 * ((e + 1) % 3) + 2]
            p_end = v[2 * ((e + 2) % 3): 2 * ((e + 2) % 3) + 2]
            L = np.hypot(*(p_end - p_start))
            lo, hi = (p_end, p_start) if fl[e] else (p_start, p_end)   # global orientation
            for seg in range(m):
                a0 = lo + (hi - lo) * seg / m
                a1 = lo + (hi - lo) * (seg + 1) / m
                pts = a0[None, :] + 0.5 * (gx[:, None] + 1.0) * (a1 - a0)[None, :]
                gval = pts @ np.array(a_vec) + 0.25
                for q in range(l + 1):
                    Pq = np.polynomial.legendre.legval(gx, [0] * q + [1])
                    a = (e * m + seg) * (l + 1) + q
                    want = -sg[e] * 0.5 * (L / m) * np.sum(gw * Pq * gval)
                    assert R[:, a] @ g == pytest.approx(want, abs=1e-13)
                    wantB = sg[e] * 0.5 * (L / m) * np.sum(gw * Pq)
                    assert Bv[a] == pytest.approx(wantB, abs=1e-13)


def _exact_segment_integrals(s, l, m, flip):
    """Exact rational values of int_{sub-edge k} P_q(t) phi ds / (ds/dtau)
    for both end nodes of every sub-edge, written directly in the face
    parameter tau in [0, 1] (power basis in tau, the form that loses
    digits in floating point for the far segments of a fine face), with
    P_q from the three-term recurrence in exact arithmetic.
    Returns {(k_node, seg, q): value} for one face of orientation `flip`."""
    from fractions import Fraction as Fr

    def mul(a, b):
        out = [Fr(0)] * (len(a) + len(b) - 1)
        for i, x in enumerate(a):
            for j, y in enumerate(b):
                out[i + j] += x * y
        return out

    def add(a, b):
        n = max(len(a), len(b))
        return [(a[i] if i < len(a) else 0) + (b[i] if i < len(b) else 0) for i in range(n)]

    def integ(a, lo, hi):
        return sum(c * (hi ** (j + 1) - lo ** (j + 1)) / (j + 1) for j, c in enumerate(a))

    per = s // m
    out = {}
    for seg in range(m):
        # t(tau) = 2 (m g - seg) - 1 with g = tau or 1 - tau
        t_lin = [Fr(2 * m - 2 * seg - 1), Fr(-2 * m)] if flip else [Fr(-2 * seg - 1), Fr(2 * m)]
        P = [[Fr(1)], t_lin]
        for k in range(1, l):
            P.append([c / (k + 1) for c in add([Fr(2 * k + 1) * x for x in mul(t_lin, P[k])],
                                                [Fr(-k) * x for x in P[k - 1]])])
        for k in range(s):
            if (s - 1 - k if flip else k) // per != seg:
                continue
            t0, t1 = Fr(k, s), Fr(k + 1, s)
            left = [t1 * s, Fr(-s)]       # hat of node k on [t0, t1]
            right = [-t0 * s, Fr(s)]      # hat of node k + 1
            for q in range(l + 1):
                for node, hat in ((k, left), (k + 1, right)):
                    out[(node, seg, q)] = out.get((node, seg, q), Fr(0)) + integ(mul(P[q], hat), t0, t1)
    return out


@pytest.mark.parametrize("s,l,m", [(48, 4, 4), (48, 3, 8), (36, 4, 6), (64, 2, 16)])
def test_segmented_face_loads_match_exact_rational_integrals(s, l, m):
    """Fine faces with many segments and high degree: every entry of R and
    B against the exact rational integrals (times -sigma |F_e| and sigma
    |F_e|), to a few units of the last place of the column scale.  An
    evaluation that cancels (a power basis in the face parameter on the far
    segments) is off by orders of magnitude more here."""
    from fractions import Fraction as Fr
    rng = np.random.default_rng(70 + s + m)
    v, s, l, sg, fl, kap, f = _rand_element(rng, s, l)
    fl = np.array([0, 1, 0], dtype=np.int8)      # both orientations
    R = local.face_loads(v, s, l, sg, fl, m)
    Bv = local.face_moments(v, l, sg, fl, m)
    for e in range(3):
        L = local.face_length(v, e)
        nodes = local.face_nodes(e, s)
        ex = _exact_segment_integrals(s, l, m, int(fl[e]))
        want = np.zeros((R.shape[0], m * (l + 1)))
        for (k, seg, q), val in ex.items():
            want[nodes[k], seg * (l + 1) + q] = -float(sg[e]) * L * float(val)
        got = R[:, e * m * (l + 1):(e + 1) * m * (l + 1)]
        scale = np.abs(want).max(axis=0)
        assert np.all(np.abs(got - want) <= 4e-16 * 8 * scale), np.abs(got - want).max(axis=0) / scale
        for seg in range(m):
            for q in range(l + 1):
                exact_b = Fr(1, m) if q == 0 else Fr(0)      # int over the segment of P_q d tau
                assert Bv[(e * m + seg) * (l + 1) + q] == pytest.approx(float(sg[e]) * L * float(exact_b),
                                                                        abs=4e-16 * L)


@pytest.mark.parametrize("s,l,m", [(4, 1, 2), (6, 0, 3), (8, 1, 2)])
def test_whole_face_space_is_inside_the_segmented_one(s, l, m):
    """Lambda^{1,l} lies inside Lambda^{m,l}: P_q on the whole face is a
    polynomial of degree q on each segment, so R^(1) = R^(m) T with T given
    by Legendre re-expansion (computed here from the polynomials alone, not
    by fitting), and then X^(1)_I = X^(m)_I T and M^(1) = T^T M^(m) T."""
    from numpy.polynomial import legendre as L_
    rng = np.random.default_rng(50 + s)
    v, s, l, sg, fl, kap, f = _rand_element(rng, s, l)
    r1 = local.local_problem(v, s, l, sg, fl, kap, f, 1)
    rm = local.local_problem(v, s, l, sg, fl, kap, f, m)
    N1, Nm = 3 * (l + 1), 3 * m * (l + 1)
    T = np.zeros((Nm, N1))
    for e in range(3):
        for q in range(l + 1):
            for seg in range(m):
                # P_q(T) with T = (2 seg + 1 + t) / m - 1 on segment seg, in Legendre P_k(t)
                poly = L_.leg2poly([0] * q + [1])                  # power coefficients in T
                comp = np.polynomial.Polynomial(poly)(np.polynomial.Polynomial([(2 * seg + 1) / m - 1.0, 1.0 / m]))
                coef = L_.poly2leg(comp.coef)
                for k, ck in enumerate(coef):
                    if abs(ck) > 0:
                        T[(e * m + seg) * (l + 1) + k, e * (l + 1) + q] = ck
    np.testing.assert_allclose(r1["R"], rm["R"] @ T, atol=1e-14, rtol=0)
    scale = np.abs(r1["X"]).max()
    np.testing.assert_allclose(r1["X"][:, :N1], rm["X"][:, :Nm] @ T, atol=1e-12 * scale, rtol=0)
    np.testing.assert_allclose(r1["X"][:, N1], rm["X"][:, Nm], atol=1e-12 * scale, rtol=0)
    np.testing.assert_allclose(r1["M"], T.T @ rm["M"] @ T, atol=1e-12 * np.abs(r1["M"]).max(), rtol=0)
    np.testing.assert_allclose(r1["B"], T.T @ rm["B"], atol=1e-14, rtol=0)
    np.testing.assert_allclose(r1["E"], T.T @ rm["E"], atol=1e-12 * max(np.abs(r1["E"]).max(), 1e-300), rtol=0)


def test_sigma_flip_match_geometric_definition():
    """The generator's sign n.n^K_F and orientation flags, re-derived from the
    coordinates: +1 where the element's outward normal agrees with the face's
    global normal (taken outward on the boundary, else pointing out of the
    lower-indexed neighbour)."""
    mesh = coarse_mesh(3)
    V = mesh["verts"]
    for g, (a, b) in enumerate(mesh["faces"]):
        owners = [t for t in mesh["face_elems"][g] if t >= 0]
        t_ref = min(owners)
        e_ref = list(mesh["elem_face"][t_ref]).index(g)
        for t in owners:
            e = list(mesh["elem_face"][t]).index(g)
            tri = V[mesh["elems"][t]]
            d = tri[(e + 2) % 3] - tri[(e + 1) % 3]
            n_out = np.array([d[1], -d[0]])
            tri_r = V[mesh["elems"][t_ref]]
            dr = tri_r[(e_ref + 2) % 3] - tri_r[(e_ref + 1) % 3]
            n_glob = np.array([dr[1], -dr[0]])
            assert mesh["sigma"][t, e] == (1 if n_out @ n_glob > 0 else -1)
            ia, ib = mesh["elems"][t][(e + 1) % 3], mesh["elems"][t][(e + 2) % 3]
            assert mesh["flip"][t, e] == (1 if ia > ib else 0)
        if len(owners) == 1:
            mid = 0.5 * (V[a] + V[b])
            assert np.isclose(mid, 0).any() or np.isclose(mid, 1).any()


# ----------------------------------------------------------- local solutions
def test_linear_reproduction_constant_k():
    """For constant K0 and a vector a, sum_e -sigma_e K0 (a.n_e) eta^(e,0) is
    the zero-mean linear function a.(x - centroid), exactly, at the nodes."""
    rng = np.random.default_rng(7)
    for s in (2, 5, 9):
        v, s, l, sg, fl, _, f = _rand_element(rng, s, 1)
        K0 = 3.7
        r = local.local_problem(v, s, l, sg, fl, np.full(s * s, K0), f)
        nodes, _ = local.submesh(v, s)
        cen = v.reshape(3, 2).mean(axis=0)
        for a_vec in (np.array([1.0, 0.0]), np.array([0.2, -1.3])):
            u = np.zeros(nodes.shape[0])
            for e in range(3):
                p0 = v[2 * ((e + 1) % 3): 2 * ((e + 1) % 3) + 2]
                p1 = v[2 * ((e + 2) % 3): 2 * ((e + 2) % 3) + 2]
                d = p1 - p0
                n_out = np.array([d[1], -d[0]]) / np.hypot(*d)
                u += -sg[e] * K0 * (a_vec @ n_out) * r["X"][:, e * (l + 1)]
            np.testing.assert_allclose(u, (nodes - cen) @ a_vec, atol=1e-13)


def test_constant_source_gives_zero_eta_f():
    rng = np.random.default_rng(8)
    v, s, l, sg, fl, kap, _ = _rand_element(rng, 6, 2)
    r = local.local_problem(v, s, l, sg, fl, kap, np.full(s * s, 2.5))
    assert np.abs(r["X"][:, -1]).max() < 1e-14
    assert np.abs(r["E"]).max() < 1e-14
    assert r["F"] == pytest.approx(2.5 * r["area"], rel=1e-14)


def test_solutions_zero_mean_and_galerkin_equations():
    rng = np.random.default_rng(9)
    v, s, l, sg, fl, kap, f = _rand_element(rng, 5, 3)
    r = local.local_problem(v, s, l, sg, fl, kap, f)
    X = r["X"]
    assert np.abs(r["c"] @ X).max() < 1e-15
    Bfull = np.column_stack([r["R"], r["b"]])
    # A X = B - c mu with mu = (1^T B)/|K|: the equations hold for all zero-mean w
    mu = Bfull.sum(axis=0) / r["area"]
    np.testing.assert_allclose(r["A"] @ X, Bfull - np.outer(r["c"], mu), atol=1e-13)


@pytest.mark.parametrize("s,l", [(3, 0), (6, 1), (8, 3)])
def test_m_symmetric_negative_definite(s, l):
    rng = np.random.default_rng(40 + s)
    v, s, l, sg, fl, kap, f = _rand_element(rng, s, l)
    r = local.local_problem(v, s, l, sg, fl, kap, f)
    M = r["M"]
    assert np.abs(M - M.T).max() < 1e-13 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).max() < 0


def test_rank_one_augmented_matrix_gives_same_solution_for_any_gamma():
    """The SPD system (A + gamma c c^T) X = B - c (1^T B)/|K| has the zero-mean
    solution for every gamma > 0; it matches the bordered (KKT) solve."""
    rng = np.random.default_rng(11)
    v, s, l, sg, fl, kap, f = _rand_element(rng, 7, 2)
    r = local.local_problem(v, s, l, sg, fl, kap, f)
    A, c = r["A"], r["c"]
    B = np.column_stack([r["R"], r["b"]])
    Bt = B - np.outer(c, B.sum(axis=0)) / r["area"]
    g0 = np.trace(A) / (A.shape[0] * (c @ c))
    scale = np.abs(r["X"]).max()
    for gamma in (g0, 100.0 * g0, 0.01 * g0):
        L = np.linalg.cholesky(A + gamma * np.outer(c, c))
        X = np.linalg.solve(L.T, np.linalg.solve(L, Bt))
        assert np.abs(X - r["X"]).max() < 1e-12 * scale


def _exact_bordered_solve(A, c, B):
    """The bordered system [[A, c], [c^T, 0]] [X; mu] = [B; 0] solved in
    exact rational arithmetic (Gaussian elimination on Fractions of the FP64
    entries), rounded to FP64."""
    n, r = B.shape
    N = n + 1
    M = [[Fraction(float(A[i, j])) for j in range(n)] + [Fraction(float(c[i]))] for i in range(n)]
    M.append([Fraction(float(x)) for x in c] + [Fraction(0)])
    R = [[Fraction(float(B[i, k])) for k in range(r)] for i in range(n)] + [[Fraction(0)] * r]
    for k in range(N):
        piv = next(i for i in range(k, N) if M[i][k] != 0)
        M[k], M[piv] = M[piv], M[k]
        R[k], R[piv] = R[piv], R[k]
        for i in range(k + 1, N):
            if M[i][k] == 0:
                continue
            f = M[i][k] / M[k][k]
            for j in range(k, N):
                M[i][j] -= f * M[k][j]
            for j in range(r):
                R[i][j] -= f * R[k][j]
    X = [[Fraction(0)] * r for _ in range(N)]
    for i in reversed(range(N)):
        for j in range(r):
            X[i][j] = (R[i][j] - sum(M[i][k] * X[k][j] for k in range(i + 1, N))) / M[i][i]
    return np.array([[float(X[i][j]) for j in range(r)] for i in range(n)])


@pytest.mark.parametrize("s,contrast", [(6, 1.0e8), (8, 1.0e10), (8, 1.0e4)])
def test_refined_solve_is_the_exact_solution_of_high_contrast_elements(s, contrast):
    """A channel of sub-triangles with kappa = contrast across the element
    (two row strips), kappa = 1 elsewhere: the condition number of the
    bordered system reaches 1e9-1e12, where a plain FP64 LU solve is off by
    1e-10-1e-7.  The oracle's refined solve equals the exact rational
    solution of the same FP64 system to rounding."""
    h = 0.25
    vert = np.array([0.0, 0.0, h, 0.0, h, h])
    kap = np.ones(s * s)
    for j in (s // 2, s // 2 + 1):
        for i in range(s - j):
            kap[j * (2 * s - j) + 2 * i] = contrast
            if i < s - j - 1:
                kap[j * (2 * s - j) + 2 * i + 1] = contrast
    sig = np.array([1, -1, 1], dtype=np.int8)
    fl = np.array([0, 1, 0], dtype=np.int8)
    rng = np.random.default_rng(int(s))
    f = rng.uniform(0.5, 1.5, s * s)
    A = local.stiffness(vert, s, kap)
    c = local.mean_vector(vert, s)
    B = np.column_stack([local.face_loads(vert, s, 1, sig, fl), local.source_load(vert, s, f)])
    Xe = _exact_bordered_solve(A, c, B)
    scale = np.abs(Xe).max()
    X, _ = local.solve_zero_mean(A, c, B)
    assert np.abs(X - Xe).max() <= 2e-16 * scale
    X0, _ = local.solve_zero_mean(A, c, B, refine=False)
    if contrast >= 1e8:   # the plain solve really is inaccurate here
        assert np.abs(X0 - Xe).max() > 1e-12 * scale


@pytest.mark.parametrize("s", [1, 2, 5, 16])
def test_subtriangle_order_matches_the_coefficient_sampling_points(s):
    """kappa and f are sampled at mhm_inputs' sub-triangle centroids; the
    oracle's sub-triangle t must be the one whose centroid is sample t."""
    from mhm_inputs.mesh import subtri_centroids
    vert = np.array([0.1, 0.2, 0.9, 0.3, 0.4, 1.1])
    nodes, tris = local.submesh(vert, s)
    cent = nodes[tris].mean(axis=1)
    np.testing.assert_allclose(cent, subtri_centroids(vert, s), rtol=0, atol=1e-14)


# ------------------------------------------------------------ skeleton level
def _solve_global(N, s, l, kfun, ffun):
    mesh = coarse_mesh(N)
    E = mesh["elems"].shape[0]
    b = configs.build_batch(mesh, np.arange(E), np.full(E, s), np.full(E, l), kfun, ffun)
    res = local.solve_batch(b)
    lam, u0, K, rhs = skeleton.reduce_and_solve(mesh, res, np.arange(E), l)
    return mesh, b, res, lam, u0, K


def test_skeleton_symmetric_and_constant_null_space():
    mesh, b, res, lam, u0, K = _solve_global(2, 4, 1, _smooth_k, manufactured_source)
    assert np.abs(K - K.T).max() < 1e-14 * np.abs(K).max()
    nl = mesh["faces"].shape[0] * 2
    z = np.zeros(K.shape[0])
    z[nl:] = 1.0                                  # lambda = 0, u0 = 1
    Kz = K @ z
    for g in range(mesh["faces"].shape[0]):
        for q in range(2):
            row = Kz[g * 2 + q]
            if mesh["face_boundary"][g] and q == 0:
                assert row == pytest.approx(mesh["face_len"][g], rel=1e-13)
            else:
                assert abs(row) < 1e-14
    assert np.abs(Kz[nl:]).max() < 1e-14


@pytest.mark.parametrize("N,s", [(2, 2), (2, 3), (3, 4)])
def test_l_equals_s_reduces_to_conforming_galerkin(N, s):
    """With m = 1 and l = s the MHM solution equals textbook P1 Galerkin on the
    composite fine mesh (homogeneous Dirichlet), node by node."""
    mesh, b, res, lam, u0, K = _solve_global(N, s, s, _smooth_k, manufactured_source)
    uh = skeleton.reconstruct(mesh, res, np.arange(b["n_elem"]), s, lam, u0)
    nodes_l, tris_l, kap_l, f_l = [], [], [], []
    for e in range(b["n_elem"]):
        nodes, tris = local.submesh(b["vert"][e], s)
        o0, o1 = b["tri_off"][e], b["tri_off"][e + 1]
        nodes_l.append(nodes)
        tris_l.append(tris)
        kap_l.append(b["kappa"][o0:o1])
        f_l.append(b["f"][o0:o1])
    ref = galerkin_ref.fine_mesh_solve(nodes_l, tris_l, kap_l, f_l, N * s)
    scale = max(abs(x) for x in ref.values())
    for e in range(b["n_elem"]):
        for p, val in zip(nodes_l[e], uh[e]):
            k = (int(round(p[0] * N * s)), int(round(p[1] * N * s)))
            assert abs(val - ref[k]) < 1e-11 * scale


@pytest.mark.parametrize("N,s,m", [(2, 2, 2), (2, 4, 4), (3, 3, 3)])
def test_m_equals_s_linear_reduces_to_conforming_galerkin(N, s, m):
    """m = s segments of degree 1 (one linear function pair per sub-edge)
    force continuity across every face, so MHM equals textbook P1 Galerkin
    on the composite fine mesh node by node, as for l = s with m = 1."""
    mesh = coarse_mesh(N)
    E = mesh["elems"].shape[0]
    b = configs.build_batch(mesh, np.arange(E), np.full(E, s), np.full(E, 1), _smooth_k, manufactured_source)
    b["m"] = np.full(E, m, dtype=np.int32)
    res = local.solve_batch(b)
    lam, u0, K, rhs = skeleton.reduce_and_solve(mesh, res, np.arange(E), 1, m)
    uh = skeleton.reconstruct(mesh, res, np.arange(E), 1, lam, u0, m)
    nodes_l, tris_l, kap_l, f_l = [], [], [], []
    for e in range(E):
        nodes, tris = local.submesh(b["vert"][e], s)
        o0, o1 = b["tri_off"][e], b["tri_off"][e + 1]
        nodes_l.append(nodes)
        tris_l.append(tris)
        kap_l.append(b["kappa"][o0:o1])
        f_l.append(b["f"][o0:o1])
    ref = galerkin_ref.fine_mesh_solve(nodes_l, tris_l, kap_l, f_l, N * s)
    scale = max(abs(x) for x in ref.values())
    for e in range(E):
        for p, val in zip(nodes_l[e], uh[e]):
            k = (int(round(p[0] * N * s)), int(round(p[1] * N * s)))
            assert abs(val - ref[k]) < 1e-11 * scale


def test_segmented_multipliers_converge_at_second_order():
    """m = 2, l = 0 (piecewise constant multipliers on two segments): L2
    error falls at rate 2 under coarse-mesh refinement."""
    errs = []
    for N in (2, 4, 8):
        mesh = coarse_mesh(N)
        E = mesh["elems"].shape[0]
        b = configs.build_batch(mesh, np.arange(E), np.full(E, 4), np.full(E, 0), _ones, manufactured_source)
        b["m"] = np.full(E, 2, dtype=np.int32)
        res = local.solve_batch(b)
        lam, u0, K, rhs = skeleton.reduce_and_solve(mesh, res, np.arange(E), 0, 2)
        uh = skeleton.reconstruct(mesh, res, np.arange(E), 0, lam, u0, 2)
        errs.append(skeleton.l2_error(b, uh, manufactured_solution))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((rates > 1.8) & (rates < 2.3)), (errs, rates)


def test_manufactured_solution_converges_at_second_order():
    errs = []
    for N in (2, 4, 8):
        mesh, b, res, lam, u0, K = _solve_global(N, 4, 1, _ones, manufactured_source)
        uh = skeleton.reconstruct(mesh, res, np.arange(b["n_elem"]), 1, lam, u0)
        errs.append(skeleton.l2_error(b, uh, manufactured_solution))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((rates > 1.8) & (rates < 2.3)), (errs, rates)


def test_config_shapes():
    b = configs.make("C1")
    assert b["n_elem"] == 32 and set(b["s"]) == {4} and set(b["l"]) == {1}
    assert b["tri_off"][-1] == 32 * 16
    b2 = configs.make("C2", n_elem=8)
    assert b2["kappa"].shape == (8 * 256,) and np.all(b2["kappa"] > 0)
