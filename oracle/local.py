"""FP64 CPU oracle for the MHM local problems.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It shares no code
with the HIP path; the only common input is the seeded generator in
``mhm_inputs`` (mesh, lattice conventions, fields).

What it computes (Sections 2-3 and 4.2 of the paper, specialised to 2D Darcy
with P1 elements on a uniformly refined triangle, m = 1):

* the local space V_h(K) of continuous P1 functions on the sub-mesh, with the
  zero-mean constraint of V_0^perp(K) (Section 2, space list and local space);
* the source subproblem, eq. (2) / eq. (8): a(eta^f, w) = (f, w);
* the multiplier subproblems, eq. (3) / eq. (9):
  a(eta^i, w) = -(sigma_e psi_i, w)_{dK} for the face polynomials psi_i;
* the coefficient vectors c_j, d_{i,j} of eq. (5), returned as the columns of
  X (one column per face DoF, then the source column);
* the element's blocks of the skeleton system, eq. (6):
  M[j,i] = (sigma psi_j, eta^i)_{dK}, E_j = -(sigma psi_j, eta^f)_{dK},
  B_j = (sigma psi_j, 1)_{dK}, F = (1, f)_K.

How: the stiffness matrix A is assembled sub-triangle by sub-triangle from the
textbook P1 formula (barycentric gradients through the inverse Jacobian), the
face loads are integrated exactly with numpy's polynomial algebra, and each
zero-mean Neumann problem is solved as the bordered system
``[[A, c], [c^T, 0]] [X; mu] = [B; 0]`` with LAPACK LU (LU as in the paper's
implementation, Section 4.1.1), refined with extended-precision residuals so
that the result is the system's exact solution rounded to FP64.  The oracle never
forms the rank-one-augmented matrix that the GPU path factors.

Readings of the paper (where it is silent) follow the project's design notes:
2D, P1, uniform refinement, m = 1, unnormalised Legendre face basis on the
globally oriented face, sign +1 for the lower-indexed neighbour and on the
boundary, K and f piecewise constant on the sub-triangles.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import Polynomial
from numpy.polynomial import legendre as npleg


# ----------------------------------------------------------------- sub-mesh
def node_index(i: int, j: int, s: int) -> int:
    return j * (s + 1) - (j * (j - 1)) // 2 + i


def submesh(vert6: np.ndarray, s: int):
    """Nodes (n, 2) and sub-triangles (s*s, 3) of the uniform refinement.

    Sub-triangles are listed in row strips: the up triangle (i, j) with nodes
    (i,j),(i+1,j),(i,j+1), then the down triangle (i, j) with nodes
    (i+1,j+1),(i,j+1),(i+1,j).  Both are counter-clockwise."""
    v0, v1, v2 = vert6[0:2], vert6[2:4], vert6[4:6]
    n = (s + 1) * (s + 2) // 2
    nodes = np.empty((n, 2))
    for j in range(s + 1):
        for i in range(s + 1 - j):
            nodes[node_index(i, j, s)] = v0 + (i / s) * (v1 - v0) + (j / s) * (v2 - v0)
    tris = []
    for j in range(s):
        for i in range(s - j):
            tris.append((node_index(i, j, s), node_index(i + 1, j, s), node_index(i, j + 1, s)))
            if i < s - j - 1:
                tris.append((node_index(i + 1, j + 1, s), node_index(i, j + 1, s),
                             node_index(i + 1, j, s)))
    return nodes, np.array(tris, dtype=np.int64)


def _p1_gradients(nodes, tris):
    """Barycentric gradients (T, 3, 2) and areas (T,) of each sub-triangle."""
    p = nodes[tris]                                  # (T, 3, 2)
    J = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]], axis=2)   # columns
    det = J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]
    Jinv = np.linalg.inv(J)                          # rows: grad lambda_1, grad lambda_2
    g1 = Jinv[:, 0, :]
    g2 = Jinv[:, 1, :]
    g0 = -g1 - g2
    return np.stack([g0, g1, g2], axis=1), 0.5 * det


# ------------------------------------------------------------ assembly, a(.,.)
def stiffness(vert6, s, kappa):
    """A[p, q] = sum over sub-triangles of K_tau * |tau| * grad phi_p . grad phi_q
    (the Darcy form (kappa grad u, grad w) of eqs. (8)-(9), K piecewise constant)."""
    nodes, tris = submesh(vert6, s)
    g, area = _p1_gradients(nodes, tris)
    loc = np.einsum("tad,tbd->tab", g, g) * (np.asarray(kappa) * area)[:, None, None]
    n = nodes.shape[0]
    A = np.zeros((n, n))
    rows = np.repeat(tris, 3, axis=1)
    cols = np.tile(tris, (1, 3))
    np.add.at(A, (rows.ravel(), cols.ravel()), loc.reshape(-1))
    return A


def mean_vector(vert6, s):
    """c_j = integral of phi_j over K (each sub-triangle adds |tau|/3)."""
    nodes, tris = submesh(vert6, s)
    _, area = _p1_gradients(nodes, tris)
    c = np.zeros(nodes.shape[0])
    for a in range(3):
        np.add.at(c, tris[:, a], area / 3.0)
    return c


def source_load(vert6, s, f):
    """b_j = (f, phi_j)_K with f constant on each sub-triangle: f_tau |tau| / 3."""
    nodes, tris = submesh(vert6, s)
    _, area = _p1_gradients(nodes, tris)
    b = np.zeros(nodes.shape[0])
    for a in range(3):
        np.add.at(b, tris[:, a], np.asarray(f) * area / 3.0)
    return b


def face_nodes(e: int, s: int):
    """Node indices along face e from its local start v[e+1] to its end v[e+2]."""
    if e == 0:
        return [node_index(s - k, k, s) for k in range(s + 1)]
    if e == 1:
        return [node_index(0, s - k, s) for k in range(s + 1)]
    return [node_index(k, 0, s) for k in range(s + 1)]


def face_length(vert6, e):
    a = vert6[2 * ((e + 1) % 3): 2 * ((e + 1) % 3) + 2]
    b = vert6[2 * ((e + 2) % 3): 2 * ((e + 2) % 3) + 2]
    return float(np.hypot(*(b - a)))


def _t_at(k: int, s: int, flip: int, m: int, seg: int) -> float:
    """The segment variable t in [-1, 1] of segment `seg` (global
    orientation) at the face node at local position k of s: with the global
    parameter g = k/s (or 1 - k/s when the local direction runs high -> low),
    t = 2 (m g - seg) - 1, formed from integers and rounded once."""
    kk = s - k if flip else k
    return 2.0 * (m * kk - seg * s) / s - 1.0


def _segment_of(k: int, s: int, flip: int, m: int) -> int:
    """Global segment holding local sub-edge k (between face nodes k and k+1)."""
    return (s - 1 - k if flip else k) // (s // m)


def face_dof(e: int, seg: int, q: int, l: int, m: int = 1) -> int:
    """Local index of face DoF (segment seg in the global orientation,
    degree q) of local face e: e m(l+1) + seg (l+1) + q."""
    return (e * m + seg) * (l + 1) + q


def face_loads(vert6, s, l, sigma, flip, m: int = 1):
    """R[:, face_dof(e, seg, q)] = -sigma_e * integral over F_e of psi phi_j ds
    (eq. (9) right-hand side) for the discontinuous face space of Section 2
    with m segments per face (m must divide s, so that every sub-edge lies
    in one segment), integrated exactly on each of the s sub-edges.  On a
    sub-edge the integrand is written in the sub-edge variable u in [0, 1]
    (hats 1 - u and u, P_q(t) with t linear in u), so every polynomial that
    is integrated has coefficients of order one."""
    if s % m:
        raise ValueError("m must divide s")
    n = (s + 1) * (s + 2) // 2
    NI = 3 * m * (l + 1)
    R = np.zeros((n, NI))
    u = Polynomial([0.0, 1.0])
    for e in range(3):
        L = face_length(vert6, e)
        nodes = face_nodes(e, s)
        fl = int(flip[e])
        for k in range(s):
            seg = _segment_of(k, s, fl, m)
            ta, tb = _t_at(k, s, fl, m, seg), _t_at(k + 1, s, fl, m, seg)
            t_of_u = Polynomial([ta, tb - ta])
            for q in range(l + 1):
                P = Polynomial(npleg.leg2poly([0] * q + [1]))(t_of_u)
                for node, hat in ((nodes[k], 1.0 - u), (nodes[k + 1], u)):
                    anti = (P * hat).integ()
                    # d(arc length) = (L / s) du
                    R[node, face_dof(e, seg, q, l, m)] += -float(sigma[e]) * (L / s) * (anti(1.0) - anti(0.0))
    return R


def face_moments(vert6, l, sigma, flip, m: int = 1):
    """B_j = (sigma psi_j, 1)_{dK}: integral of the signed face polynomial
    over its segment (length |F_e| / m; ds = |F_e| / (2 m) dt)."""
    NI = 3 * m * (l + 1)
    Bv = np.zeros(NI)
    for e in range(3):
        L = face_length(vert6, e)
        for seg in range(m):
            for q in range(l + 1):
                anti = Polynomial(npleg.leg2poly([0] * q + [1])).integ()
                Bv[face_dof(e, seg, q, l, m)] = float(sigma[e]) * L / (2.0 * m) * (anti(1.0) - anti(-1.0))
    return Bv


# ------------------------------------------------------------------- solve
# Error-free transformations of IEEE double arithmetic (numpy rounds every
# operation to nearest and never fuses a multiply-add): Dekker's splitting
# and product, Knuth's two-sum.  They let the residual of the refinement
# below be computed exactly and rounded once.
_SPLITTER = 134217729.0   # 2^27 + 1


def _split(a):
    t = _SPLITTER * a
    hi = t - (t - a)
    return hi, a - hi


def _two_prod(a, b):
    """p + e == a * b exactly (Dekker)."""
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def _two_sum(a, b):
    """s + e == a + b exactly (Knuth)."""
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def _bordered_residual(A, c, B, x, mu):
    """Residual of the bordered system, [B - A x - c mu; -c^T x], every
    product formed exactly and the sums carried as double-double (head and
    tail), rounded to FP64 once at the end."""
    n, r = x.shape
    hi = B.copy()
    lo = np.zeros_like(B)

    def sub(rows, p, e):
        h, t = _two_sum(hi[rows], -p)
        hi[rows] = h
        lo[rows] = lo[rows] + (t - e)

    # A x over the nonzeros of A, one nonzero per row at a time
    rows, cols = np.nonzero(A)
    vals = A[rows, cols]
    # rows come sorted (np.nonzero is row-major): rank of each nonzero in its row
    rank = np.arange(rows.size) - np.searchsorted(rows, rows, side="left")
    for k in range(int(rank.max()) + 1 if rows.size else 0):
        sel = rank == k
        p, e = _two_prod(vals[sel][:, None], x[cols[sel]])
        sub(rows[sel], p, e)
    p, e = _two_prod(c[:, None], np.broadcast_to(mu, (n, r)))
    sub(np.arange(n), p, e)
    last = np.empty(r)
    for j in range(r):
        p, e = _two_prod(c, x[:, j])
        last[j] = -math.fsum(np.concatenate([p, e]))   # correctly rounded
    return hi + lo, last


def solve_zero_mean(A, c, B, refine: bool = True):
    """Zero-mean Galerkin solution of A X = B - c mu (the Neumann problems on
    V_h(K) inside V_0^perp), by LU of the bordered system.

    The result is the exact solution of this linear system (the discrete
    definition), to FP64 rounding.  An FP64 LU solve alone is only accurate
    to about cond(A) times the unit roundoff: with a coefficient contrast of
    1e4 inside an element (cond near 1e7) that is 1e-10, the size of the
    parity tolerance.  So the LU solution is refined (the LU factors reused)
    with exactly computed residuals until the correction is below the FP64
    rounding of the solution (at most eight steps); `refine=False` gives the
    plain LU solve."""
    import scipy.linalg
    n = A.shape[0]
    K = np.zeros((n + 1, n + 1))
    K[:n, :n] = A
    K[:n, n] = c
    K[n, :n] = c
    rhs = np.zeros((n + 1, B.shape[1]))
    rhs[:n] = B
    lu = scipy.linalg.lu_factor(K)
    sol = scipy.linalg.lu_solve(lu, rhs)
    x, mu = sol[:n].copy(), sol[n].copy()
    if not refine:
        return x, mu
    for _ in range(8):
        r, r_last = _bordered_residual(A, c, B, x, mu)
        corr = scipy.linalg.lu_solve(lu, np.vstack([r, r_last[None, :]]))
        x = x + corr[:n]
        mu = mu + corr[n]
        if np.max(np.abs(corr[:n])) <= 2.0 ** -54 * np.max(np.abs(x)):
            break
    return x, mu


def local_problem(vert6, s, l, sigma, flip, kappa, f, m: int = 1):
    """solveLocalProblem for one element plus its share of the skeleton
    system (face space: m segments per face, degree l on each).  Returns a
    dict with A, c, R, b, X (n x (N_I+1), source last), M, E, B, F and the
    element area."""
    vert6 = np.asarray(vert6, dtype=np.float64)
    A = stiffness(vert6, s, kappa)
    c = mean_vector(vert6, s)
    R = face_loads(vert6, s, l, sigma, flip, m)
    b = source_load(vert6, s, f)
    X, mu = solve_zero_mean(A, c, np.column_stack([R, b]))
    NI = R.shape[1]
    M = -R.T @ X[:, :NI]
    E = R.T @ X[:, NI]
    Bv = face_moments(vert6, l, sigma, flip, m)
    F = float(np.sum(np.asarray(f) * _p1_gradients(*submesh(vert6, s))[1]))
    area = 0.5 * abs((vert6[2] - vert6[0]) * (vert6[5] - vert6[1]) - (vert6[4] - vert6[0]) * (vert6[3] - vert6[1]))
    return dict(A=A, c=c, R=R, b=b, X=X, mu=mu, M=M, E=E, B=Bv, F=F, area=area)


def element_inputs(batch: dict, e: int):
    o0, o1 = batch["tri_off"][e], batch["tri_off"][e + 1]
    m = int(batch["m"][e]) if batch.get("m") is not None else 1
    return (batch["vert"][e], int(batch["s"][e]), int(batch["l"][e]), batch["sigma"][e],
            batch["flip"][e], batch["kappa"][o0:o1], batch["f"][o0:o1], m)


def solve_element(batch: dict, e: int) -> dict:
    return local_problem(*element_inputs(batch, e))


def solve_batch(batch: dict, elems=None) -> list:
    idx = range(batch["n_elem"]) if elems is None else elems
    return [solve_element(batch, int(e)) for e in idx]
