"""Host-side batch layout: offsets, validation and upload of a ragged batch.

A batch (see ``mhm_inputs.configs``) lists per element s, l, optionally m
(segments per face, default 1), the vertices, face signs and orientation
flags, and kappa, f per sub-triangle.  Here the
prefix offsets of every per-element block are computed, the descriptor is
checked on the host (sizes, ranges, finite values) and the arrays are copied
to device memory owned by torch tensors.
"""
from __future__ import annotations

import numpy as np

from . import abi


def n_nodes(s):
    s = np.asarray(s, dtype=np.int64)
    return (s + 1) * (s + 2) // 2


def n_rhs(l, m=1):
    return 3 * np.asarray(m, dtype=np.int64) * (np.asarray(l, dtype=np.int64) + 1) + 1


def segments(b: dict) -> np.ndarray:
    """Per-element m (segments per face) of a batch dict, 1 when absent."""
    m = b.get("m")
    return np.ones(int(b["n_elem"]), dtype=np.int32) if m is None else np.asarray(m, dtype=np.int32)


def _prefix(x):
    out = np.zeros(len(x) + 1, dtype=np.int64)
    np.cumsum(x, out=out[1:])
    return out


def layout(s, l, m=1) -> dict:
    """Offsets of the per-element blocks (Ahat n^2, Btilde/X n*r, c n, kappa s^2)."""
    n = n_nodes(s)
    r = n_rhs(l, m)
    s64 = np.asarray(s, dtype=np.int64)
    return dict(n=n, r=r, tri_off=_prefix(s64 * s64), mat_off=_prefix(n * n), rhs_off=_prefix(n * r),
                node_off=_prefix(n))


def validate(b: dict) -> None:
    """Reject malformed batches before anything is launched."""
    E = int(b["n_elem"])
    s = np.asarray(b["s"])
    l = np.asarray(b["l"])
    if s.shape != (E,) or l.shape != (E,):
        raise ValueError("s and l must have one entry per element")
    if E and (s.min() < 1 or s.max() > abi.MHM_S_LIMIT):
        raise ValueError(f"s must lie in [1, {abi.MHM_S_LIMIT}]")
    if E and (l.min() < 0 or l.max() > abi.MHM_L_LIMIT):
        raise ValueError(f"l must lie in [0, {abi.MHM_L_LIMIT}]")
    m = segments(b)
    if m.shape != (E,):
        raise ValueError("m must have one entry per element")
    if E and (m.min() < 1 or np.any(s % m != 0)):
        raise ValueError("m must be >= 1 and divide s")
    if E and np.max(m * (l + 1)) > abi.MHM_P_LIMIT:
        raise ValueError(f"m (l + 1) must be at most {abi.MHM_P_LIMIT}")
    if np.asarray(b["vert"]).shape != (E, 6):
        raise ValueError("vert must be (n_elem, 6)")
    for k in ("sigma", "flip"):
        if np.asarray(b[k]).shape != (E, 3):
            raise ValueError(f"{k} must be (n_elem, 3)")
    if E and not np.all(np.abs(np.asarray(b["sigma"])) == 1):
        raise ValueError("sigma must be +1 or -1")
    if E and not np.all((np.asarray(b["flip"]) == 0) | (np.asarray(b["flip"]) == 1)):
        raise ValueError("flip must be 0 or 1")
    T = int(np.sum(s.astype(np.int64) ** 2))
    for k in ("kappa", "f"):
        a = np.asarray(b[k])
        if a.shape != (T,):
            raise ValueError(f"{k} must hold sum(s^2) = {T} values")
        if not np.all(np.isfinite(a)):
            raise ValueError(f"{k} contains non-finite values")
    if not np.all(np.isfinite(b["vert"])):
        raise ValueError("vert contains non-finite values")
    if E:
        v = np.asarray(b["vert"], dtype=np.float64)
        cross = (v[:, 2] - v[:, 0]) * (v[:, 5] - v[:, 1]) - (v[:, 4] - v[:, 0]) * (v[:, 3] - v[:, 1])
        if np.any(cross <= 0):
            raise ValueError("every element must be counter-clockwise with positive area")


class DeviceBatch:
    """A batch resident in device memory plus its ``mhm_batch`` descriptor."""

    def __init__(self, b: dict, device="cuda", check: bool = True):
        import torch
        if check:
            validate(b)
        E = int(b["n_elem"])
        s = np.asarray(b["s"], dtype=np.int32)
        l = np.asarray(b["l"], dtype=np.int32)
        m = segments(b)
        lay = layout(s, l, m)
        self.n_elem = E
        self.s = s
        self.l = l
        self.m = m
        self.n = lay["n"]
        self.r = lay["r"]
        self.s_max = int(s.max()) if E else 1
        self.s_min = int(s.min()) if E else 1
        self.l_max = int(l.max()) if E else 0
        self.p_max = int(np.max(m * (l + 1))) if E else 1
        self.NImax = 3 * self.p_max
        self.has_m = b.get("m") is not None
        self.mat_off = lay["mat_off"]
        self.rhs_off = lay["rhs_off"]
        self.node_off = lay["node_off"]

        def up(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)

        self.t = dict(
            s=up(s, np.int32), l=up(l, np.int32), vert=up(b["vert"], np.float64),
            sigma=up(b["sigma"], np.int8), flip=up(b["flip"], np.int8),
            kappa=up(b["kappa"], np.float64), f=up(b["f"], np.float64),
            tri_off=up(lay["tri_off"], np.int64), mat_off=up(lay["mat_off"], np.int64),
            rhs_off=up(lay["rhs_off"], np.int64), node_off=up(lay["node_off"], np.int64),
        )
        d = abi.mhm_batch()
        d.n_elem = E
        d.s_max = self.s_max
        d.s_min = self.s_min
        d.l_max = self.l_max
        for k, v in self.t.items():
            setattr(d, k, v.data_ptr() if v.numel() else None)
        d.tri_total = int(lay["tri_off"][-1])
        d.mat_total = int(lay["mat_off"][-1])
        d.rhs_total = int(lay["rhs_off"][-1])
        d.node_total = int(lay["node_off"][-1])
        if self.has_m:
            self.t["m"] = up(m, np.int32)
            d.m = self.t["m"].data_ptr() if E else None
        d.p_max = self.p_max
        self.desc = d
        self.mat_total = d.mat_total
        self.rhs_total = d.rhs_total
        self.node_total = d.node_total

    # --------------------------------------------------------------- outputs
    def alloc_outputs(self, three_call: bool = False, device="cuda") -> dict:
        import torch
        E, NI = self.n_elem, self.NImax
        f64 = dict(dtype=torch.float64, device=device)
        out = dict(
            X=torch.empty(max(self.rhs_total, 1), **f64),
            M=torch.empty(max(E * NI * NI, 1), **f64),
            E=torch.empty(max(E * NI, 1), **f64),
            B=torch.empty(max(E * NI, 1), **f64),
            F=torch.empty(max(E, 1), **f64),
            info=torch.empty(max(E, 1), dtype=torch.int32, device=device),
            ir_iters=torch.empty(max(E, 1), dtype=torch.int32, device=device),
        )
        if three_call:
            out.update(
                Ahat=torch.empty(max(self.mat_total, 1), **f64),
                Btil=torch.empty(max(self.rhs_total, 1), **f64),
                c=torch.empty(max(self.node_total, 1), **f64),
                area=torch.empty(max(E, 1), **f64),
            )
        return out

    def unpack(self, out: dict) -> list:
        """Per-element numpy views of X and the contribution blocks."""
        X = out["X"].cpu().numpy()
        M = out["M"].cpu().numpy()
        Ev = out["E"].cpu().numpy()
        Bv = out["B"].cpu().numpy()
        F = out["F"].cpu().numpy()
        info = out["info"].cpu().numpy()
        it = out["ir_iters"].cpu().numpy()
        NI = self.NImax
        res = []
        for e in range(self.n_elem):
            n, r = int(self.n[e]), int(self.r[e])
            ni = r - 1
            x = X[self.rhs_off[e]:self.rhs_off[e + 1]].reshape(r, n).T
            m = M[e * NI * NI:(e + 1) * NI * NI].reshape(NI, NI).T[:ni, :ni]
            res.append(dict(X=x, M=m, E=Ev[e * NI:e * NI + ni], B=Bv[e * NI:e * NI + ni], F=float(F[e]),
                            info=int(info[e]), ir_iters=int(it[e])))
        return res
