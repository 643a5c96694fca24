"""Skeleton numbering and sparsity pattern for the global system, eq. (6),
and thin wrappers of ``mhm_skeleton_scatter`` / ``mhm_reconstruct``.

Unknowns are ordered as in the paper's reduced system: the multiplier DoFs
first, face g's q-th coefficient at g*(l+1)+q, then one u_0 per element.
The element's local face DoF a = e*(l+1)+q (local face e, Section 2) maps to
the global face ``elem_face[t, e]``.  The CSR pattern is the union over
elements of the dense (N_I + 1)^2 blocks they touch, columns sorted in every
row, which is what the scatter kernel searches.

Host index bookkeeping only; the additions and the reconstruction run in
libmhm.so.
"""
from __future__ import annotations

import numpy as np


def numbering(elem_face: np.ndarray, n_faces: int, l: int, elem_ids=None, p_max: int | None = None, m: int = 1):
    """gdof [n_elem, 3 p_max] (entries past N_I = 3 m (l+1) are -1), erow
    [n_elem] and the number of rows, for the elements ``elem_ids`` (default
    all) of a mesh with a uniform face space (m segments of degree l per
    face).  Face g's DoF (seg, q) is row (g m + seg)(l + 1) + q; the
    element's local DoF (e m + seg)(l + 1) + q refers to the same function
    (segments in the face's global orientation)."""
    elem_face = np.asarray(elem_face, dtype=np.int64)
    nt = elem_face.shape[0]
    ids = np.arange(nt) if elem_ids is None else np.asarray(elem_ids, dtype=np.int64)
    P = m * (l + 1)
    p_max = P if p_max is None else p_max
    if p_max < P:
        raise ValueError("p_max < m (l + 1)")
    NI, NImax = 3 * P, 3 * p_max
    nl = n_faces * P
    gdof = np.full((len(ids), NImax), -1, dtype=np.int64)
    k = np.arange(P)
    gdof[:, :NI] = (elem_face[ids][:, :, None] * P + k[None, None, :]).reshape(len(ids), NI)
    erow = nl + ids
    return gdof.astype(np.int32), erow.astype(np.int32), nl + nt


def csr_pattern(gdof: np.ndarray, erow: np.ndarray, n_rows: int, ni=None):
    """row_ptr [n_rows+1], col_idx (int32, sorted within each row) of the
    union of the element blocks over (gdof[e, :ni[e]], erow[e])."""
    gdof = np.asarray(gdof, dtype=np.int64)
    erow = np.asarray(erow, dtype=np.int64)
    n_elem, NImax = gdof.shape
    ni = np.full(n_elem, NImax) if ni is None else np.asarray(ni)
    rows, cols = [], []
    for e in range(n_elem):
        idx = np.concatenate([gdof[e, :ni[e]], erow[e:e + 1]])
        rows.append(np.repeat(idx, len(idx)))
        cols.append(np.tile(idx, len(idx)))
    if n_elem:
        key = np.unique(np.concatenate(rows) * n_rows + np.concatenate(cols))
    else:
        key = np.zeros(0, dtype=np.int64)
    r, c = key // n_rows, key % n_rows
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    if row_ptr[-1] >= 2 ** 31:
        raise ValueError("pattern exceeds int32 indexing")
    return row_ptr.astype(np.int32), c.astype(np.int32)


class SkeletonSystem:
    """Device copies of the numbering and pattern of one mesh, and the two
    calls around the local solves: scatter the element blocks into the CSR
    system, reconstruct u from a skeleton solution."""

    def __init__(self, mesh: dict, l: int, elem_ids=None, p_max: int | None = None, device="cuda", m: int = 1):
        import torch
        self.gdof_h, self.erow_h, self.n_rows = numbering(mesh["elem_face"], mesh["faces"].shape[0], l, elem_ids,
                                                          p_max, m)
        ni = np.full(len(self.erow_h), 3 * m * (l + 1))
        self.row_ptr_h, self.col_idx_h = csr_pattern(self.gdof_h, self.erow_h, self.n_rows, ni)
        i32 = dict(dtype=torch.int32, device=device)
        self.gdof = torch.as_tensor(self.gdof_h.ravel(), **i32)
        self.erow = torch.as_tensor(self.erow_h, **i32)
        self.row_ptr = torch.as_tensor(self.row_ptr_h, **i32)
        self.col_idx = torch.as_tensor(self.col_idx_h, **i32)
        self.nnz = int(self.row_ptr_h[-1])
        self.n_lambda = self.n_rows - mesh["elems"].shape[0]   # multiplier rows come first
        # DoFs of one face: consecutive multiplier rows, the solve's preconditioner blocks
        # (faces with more than 8 fall back to the diagonal preconditioner)
        self.face_dofs = m * (l + 1) if m * (l + 1) <= 8 else 1
        self.device = device

    def scatter(self, ctx, db, out, vals=None, rhs=None, clear: bool = True):
        """Add every element's (M, B, E, F) into vals / rhs (allocated and
        zeroed here unless given); returns (vals, rhs, missing)."""
        import torch
        f64 = dict(dtype=torch.float64, device=self.device)
        if vals is None:
            vals = torch.zeros(max(self.nnz, 1), **f64)
        elif clear:
            vals.zero_()
        if rhs is None:
            rhs = torch.zeros(self.n_rows, **f64)
        elif clear:
            rhs.zero_()
        missing = torch.zeros(1, dtype=torch.int32, device=self.device)
        if self.gdof.numel() != db.n_elem * db.NImax or self.erow.numel() != db.n_elem:
            raise ValueError("numbering does not match the batch (elements or l_max)")
        ctx.skeleton_scatter(db, out["M"], out["E"], out["B"], out["F"], self.gdof, self.erow, self.row_ptr,
                             self.col_idx, self.n_rows, vals, rhs, out["info"], missing)
        return vals, rhs, missing

    def reconstruct(self, ctx, db, out, sol, u=None):
        """Nodal values of u_{H,h} on every element's sub-mesh, in the batch's
        node layout."""
        import torch
        if u is None:
            u = torch.zeros(max(db.node_total, 1), dtype=torch.float64, device=self.device)
        if self.gdof.numel() != db.n_elem * db.NImax or self.erow.numel() != db.n_elem:
            raise ValueError("numbering does not match the batch (elements or l_max)")
        if sol.numel() < self.n_rows:
            raise ValueError("sol shorter than the skeleton system")
        ctx.reconstruct(db, out["X"], self.gdof, self.erow, sol, self.n_rows, u, out["info"])
        return u

    def solve(self, ctx, vals, rhs, sol=None, tol: float = 1e-12, max_iters: int = 20000, lambda_block=None):
        """mhm_skeleton_solve on the scattered system; returns (sol, iterations,
        relative residual).  lambda_block: the preconditioner's face blocks,
        by default one face's m (l + 1) DoFs (1: the diagonal preconditioner)."""
        import torch
        if sol is None:
            sol = torch.empty(self.n_rows, dtype=torch.float64, device=self.device)
        pb = self.face_dofs if lambda_block is None else int(lambda_block)
        it, rr = ctx.skeleton_solve(self.n_rows, self.n_lambda, self.row_ptr, self.col_idx, vals, rhs, sol, tol,
                                    max_iters, pb)
        return sol, it, rr
