"""Write ``s1_triangle_345.json``: an exact worked example of one local problem.

The paper prints no numbers for a single local problem, so this fixture is a
hand derivation in exact rational arithmetic (Python ``fractions``) of the
smallest case, s = 1 (one sub-triangle, three P1 nodes), for the Darcy local
problems of eqs. (8)-(9) with the face space of Section 2 (m = 1, l = 2).
It uses closed forms only:

* P1 stiffness of a triangle: K (D_a . D_b) / (4 |K|), D_a the edge vector
  opposite vertex a (the gradient of a barycentric coordinate is the rotated
  opposite edge over 2 |K|);
* integral of phi_j over the triangle: |K| / 3;
* face integrals of P_q against the two end hats for s = 1, from the
  orthogonality of Legendre polynomials: 1/2 for q = 0, -+1/6 for q = 1
  (sign by direction), 0 for q >= 2;
* the zero-mean Neumann solution from the bordered system, eliminated
  exactly.

Triangle (0,0), (4,0), (0,3) (edges 5, 3, 4, area 6), K = 2, f = 3,
sigma = (+1, -1, +1), flip = (0, 1, 0).
"""
from __future__ import annotations

import json
import os
from fractions import Fraction as Fr

VERT = [(0, 0), (4, 0), (0, 3)]
KAPPA = Fr(2)
F_SRC = Fr(3)
L_DEG = 2
SIGMA = (1, -1, 1)
FLIP = (0, 1, 0)
FACE_LEN = (Fr(5), Fr(3), Fr(4))     # |v2 - v1|, |v0 - v2|, |v1 - v0|


def _solve_exact(Mat, rhs):
    """Gauss-Jordan elimination with exact fractions (row pivoting on nonzero)."""
    n = len(Mat)
    A = [row[:] + r[:] for row, r in zip(Mat, rhs)]
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        p = A[col][col]
        A[col] = [v / p for v in A[col]]
        for r in range(n):
            if r != col and A[r][col] != 0:
                m = A[r][col]
                A[r] = [a - m * b for a, b in zip(A[r], A[col])]
    return [row[n:] for row in A]


def derive():
    area = Fr(6)
    v = [tuple(map(Fr, p)) for p in VERT]
    D = [(v[2][0] - v[1][0], v[2][1] - v[1][1]),
         (v[0][0] - v[2][0], v[0][1] - v[2][1]),
         (v[1][0] - v[0][0], v[1][1] - v[0][1])]
    A = [[KAPPA * (D[a][0] * D[b][0] + D[a][1] * D[b][1]) / (4 * area) for b in range(3)] for a in range(3)]
    c = [area / 3] * 3
    NI = 3 * (L_DEG + 1)
    # face e runs from local vertex e+1 to e+2; s = 1 lattice node ids:
    # v0 -> 0, v1 -> 1, v2 -> 2
    R = [[Fr(0)] * NI for _ in range(3)]
    for e in range(3):
        start, end = (e + 1) % 3, (e + 2) % 3
        for q in range(L_DEG + 1):
            if q == 0:
                i_start, i_end = Fr(1, 2), Fr(1, 2)
            elif q == 1:
                i_start, i_end = Fr(-1, 6), Fr(1, 6)
                if FLIP[e]:
                    i_start, i_end = -i_start, -i_end
            else:
                i_start, i_end = Fr(0), Fr(0)
            a = e * (L_DEG + 1) + q
            R[start][a] += -SIGMA[e] * FACE_LEN[e] * i_start
            R[end][a] += -SIGMA[e] * FACE_LEN[e] * i_end
    b = [F_SRC * area / 3] * 3
    Bcols = [R[j] + [b[j]] for j in range(3)]
    K = [A[j] + [c[j]] for j in range(3)] + [c + [Fr(0)]]
    rhs = Bcols + [[Fr(0)] * (NI + 1)]
    sol = _solve_exact(K, rhs)
    X = sol[:3]
    M = [[-sum(R[j][a] * X[j][i] for j in range(3)) for i in range(NI)] for a in range(NI)]
    E = [sum(R[j][a] * X[j][NI] for j in range(3)) for a in range(NI)]
    Bv = [SIGMA[e] * FACE_LEN[e] * (1 if q == 0 else 0) for e in range(3) for q in range(L_DEG + 1)]
    F = F_SRC * area
    return dict(A=A, c=c, R=R, b=b, X=X, M=M, E=E, B=Bv, F=F)


def _to_str(x):
    if isinstance(x, list):
        return [_to_str(y) for y in x]
    return str(Fr(x))


def main(path=None):
    path = path or os.path.join(os.path.dirname(os.path.abspath(__file__)), "s1_triangle_345.json")
    out = dict(
        source="exact derivation, eqs. (5), (6), (8), (9); see make_s1_triangle_345.py",
        vert=[list(p) for p in VERT], s=1, l=L_DEG, kappa=str(KAPPA), f=str(F_SRC),
        sigma=list(SIGMA), flip=list(FLIP),
        values={k: _to_str(v) for k, v in derive().items()},
    )
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


if __name__ == "__main__":
    main()
