"""Textbook conforming P1 Galerkin on the composite fine mesh (test helper).

Used to pin the oracle: with m = 1 and face degree l = s the MHM solution
u_{H,h} of eq. (4) coincides with the conforming P1 Galerkin solution of the
same discrete data (the multipliers then enforce full continuity of the P1
traces).  The element matrices here come from the cotangent formula, a route
independent of the oracle's Jacobian-based assembly.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _cot(a, b, c):
    """cotangent of the angle at vertex a of triangle (a, b, c)."""
    u = b - a
    v = c - a
    return float(np.dot(u, v) / abs(u[0] * v[1] - u[1] * v[0]))


def fine_mesh_solve(elem_nodes, elem_tris, kappa_list, f_list, scale: int):
    """Solve -div(K grad u) = f, u = 0 on the boundary of (0,1)^2.

    ``elem_nodes[e]`` (n_e, 2) and ``elem_tris[e]`` (T_e, 3) list each coarse
    element's sub-mesh; nodes are merged on the lattice of spacing 1/scale.
    Returns a dict mapping integer lattice keys to nodal values.
    """
    key_of = {}
    keys = []

    def key(p):
        k = (int(round(p[0] * scale)), int(round(p[1] * scale)))
        if k not in key_of:
            key_of[k] = len(keys)
            keys.append(k)
        return key_of[k]

    rows, cols, vals = [], [], []
    n_glob_rhs = {}
    for nodes, tris, kap, ff in zip(elem_nodes, elem_tris, kappa_list, f_list):
        gid = [key(p) for p in nodes]
        for t, (a, b, c) in enumerate(tris):
            pa, pb, pc = nodes[a], nodes[b], nodes[c]
            area = 0.5 * abs((pb[0] - pa[0]) * (pc[1] - pa[1]) - (pc[0] - pa[0]) * (pb[1] - pa[1]))
            cots = {(b, c): _cot(pa, pb, pc), (c, a): _cot(pb, pc, pa), (a, b): _cot(pc, pa, pb)}
            for (i, j), ct in cots.items():
                w = 0.5 * kap[t] * ct
                gi, gj = gid[i], gid[j]
                rows += [gi, gj, gi, gj]
                cols += [gj, gi, gi, gj]
                vals += [-w, -w, w, w]
            for v in (a, b, c):
                n_glob_rhs[gid[v]] = n_glob_rhs.get(gid[v], 0.0) + ff[t] * area / 3.0
    n = len(keys)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    rhs = np.zeros(n)
    for g, v in n_glob_rhs.items():
        rhs[g] = v
    boundary = np.array([k[0] in (0, scale) or k[1] in (0, scale) for k in keys])
    interior = np.nonzero(~boundary)[0]
    u = np.zeros(n)
    u[interior] = spla.spsolve(A[interior][:, interior].tocsc(), rhs[interior])
    return {k: u[key_of[k]] for k in keys}
