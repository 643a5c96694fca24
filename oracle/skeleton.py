"""FP64 CPU oracle for the skeleton (global) system and the reconstruction.

TEST INFRASTRUCTURE ONLY (see ``oracle/local.py``).

* ``reduce_and_solve`` assembles eq. (6) from the per-element blocks, rows
  ordered as face DoF ``g*(l+1)+q`` then element t, and solves it (the
  reduceLocalProblems primitive of Algorithm 1).  When the multiplier block is
  rank deficient (l >= s) it uses a least-squares solve; u stays unique.
* ``reconstruct`` evaluates u_{H,h} = u_0 + sum_i k_i eta^i + eta^f at the
  sub-mesh nodes of every element (eq. (4), computeSolution).
* ``l2_error`` integrates (u_{H,h} - u)^2 with a collapsed Gauss-Legendre
  rule on every sub-triangle.
"""
from __future__ import annotations

import numpy as np

from .local import _p1_gradients, submesh


def global_dofs(mesh: dict, t: int, l: int, m: int = 1):
    """Global multiplier index of each local face DoF a = (e m + seg)(l+1) + q
    of element t: face g's DoF (seg, q) is (g m + seg)(l+1) + q (segments in
    the face's global orientation, as in the local numbering)."""
    return np.array([(mesh["elem_face"][t, e] * m + seg) * (l + 1) + q
                     for e in range(3) for seg in range(m) for q in range(l + 1)])


def assemble_global(mesh: dict, results: list, elem_ids, l: int, m: int = 1):
    ne = mesh["faces"].shape[0]
    nt = mesh["elems"].shape[0]
    nl = ne * m * (l + 1)
    K = np.zeros((nl + nt, nl + nt))
    rhs = np.zeros(nl + nt)
    for t, r in zip(elem_ids, results):
        g = global_dofs(mesh, int(t), l, m)
        K[np.ix_(g, g)] += r["M"]
        K[nl + t, g] += r["B"]
        K[g, nl + t] += r["B"]
        rhs[g] += r["E"]
        rhs[nl + t] += r["F"]
    return K, rhs


def reduce_and_solve(mesh: dict, results: list, elem_ids, l: int, m: int = 1):
    K, rhs = assemble_global(mesh, results, elem_ids, l, m)
    nl = mesh["faces"].shape[0] * m * (l + 1)
    try:
        cond = np.linalg.cond(K)
    except np.linalg.LinAlgError:
        cond = np.inf
    if np.isfinite(cond) and cond < 1e12:
        sol = np.linalg.solve(K, rhs)
    else:
        sol = np.linalg.lstsq(K, rhs, rcond=1e-12)[0]
    return sol[:nl], sol[nl:], K, rhs


def reconstruct(mesh: dict, results: list, elem_ids, l: int, lam, u0, m: int = 1):
    """Nodal values of u_{H,h} on each element's sub-mesh (list of arrays)."""
    out = []
    NI = 3 * m * (l + 1)
    for t, r in zip(elem_ids, results):
        g = global_dofs(mesh, int(t), l, m)
        X = r["X"]
        out.append(u0[t] + X[:, :NI] @ lam[g] + X[:, NI])
    return out


def _collapsed_gauss(order: int = 6):
    x, w = np.polynomial.legendre.leggauss(order)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    xi, eta = np.meshgrid(x, x, indexing="ij")
    wi, we = np.meshgrid(w, w, indexing="ij")
    # square -> reference triangle (lambda_1, lambda_2) = (xi, eta (1 - xi))
    l1 = xi.ravel()
    l2 = (eta * (1.0 - xi)).ravel()
    wt = (wi * we * (1.0 - xi)).ravel()      # weights sum to 1/2
    return l1, l2, wt


def l2_error(batch: dict, nodal: list, exact) -> float:
    l1, l2, wt = _collapsed_gauss()
    total = 0.0
    for e, uh in enumerate(nodal):
        s = int(batch["s"][e])
        nodes, tris = submesh(batch["vert"][e], s)
        _, area = _p1_gradients(nodes, tris)
        p = nodes[tris]                          # (T, 3, 2)
        pts = (p[:, None, 0] * (1 - l1 - l2)[None, :, None] + p[:, None, 1] * l1[None, :, None]
               + p[:, None, 2] * l2[None, :, None])
        u = uh[tris]                              # (T, 3)
        uq = u[:, :1] * (1 - l1 - l2)[None, :] + u[:, 1:2] * l1[None, :] + u[:, 2:3] * l2[None, :]
        d = uq - exact(pts)
        total += float(np.sum((d * d) @ wt * 2.0 * area))
    return float(np.sqrt(total))
