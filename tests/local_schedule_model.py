"""Host model of the schedule of ``k_local`` (paper_1703_10435_amd/csrc/
mhm_kernels.hip): the right-looking tile kernel with its tiles in LDS or in
a workspace slot, used for the small FP32 elements and as the workspace
fallback.  Same method as ll_schedule_model.py: every wave is walked through
the kernel's loops as the source issues them - the fill of the tiles (the
operator, its stencil additions, the right-hand-side row), the factorisation
steps k = -1 .. nt - 1 (panel, trailing update with the look-ahead
factorisation of tile (k+1, k+1) by wave 0), the forward and backward
sweeps, the X output and the refinement passes - and each wave's accesses
of the tiles, of X and of the non-fused Ahat are tagged by the barriers
passed.  check() of ll_schedule_model reports out-of-bounds accesses,
unordered overlaps, differing barrier sequences and operator entries read
after the factor was written over them.

Tiles are tracked by entry (16 rows of stride 17) in the fill, whose threads
write single entries, and as whole tiles elsewhere.
"""
from __future__ import annotations

from tests.ll_schedule_model import TILE, TST, WaveLog, _node_ij, n_of

NTH = 256
NWAVES = NTH // 64


def _trail_ij(t, k, nt):
    m = nt - 1 - k
    jj, rem = 0, t
    while rem >= m - jj + 1:
        rem -= m - jj + 1
        jj += 1
    j = k + 1 + jj
    return j + rem, j


def simulate(s: int, l: int, fp32: bool, fused: bool = True, refine: bool = None, ir_steps: int = 2,
             three_call: bool = False, drop: tuple = (), trail_skip_first: bool = True):
    """All waves' logs for one element; `drop` leaves out barriers (the
    model's own tests), trail_skip_first=False lets waves 1-3 also take
    trailing tile 0, the one wave 0 factors (a planted race)."""
    n = n_of(s)
    nt = (n + 15) // 16
    NI = 3 * (l + 1)
    r = NI + 1
    refine = fp32 if refine is None else refine
    ntiles = nt * (nt + 1) // 2 + nt

    def off(I, J):
        assert 0 <= J <= I <= nt and (I < nt or J < nt), (I, J)
        return ((I * (I + 1)) // 2 + J) * TILE

    logs = []
    for wave in range(NWAVES):
        g = WaveLog(wave, drop=tuple(drop))
        threads = range(64 * wave, 64 * wave + 64)

        def trd(I, J, where):
            o = off(I, J)
            g.rd("ws", o, o + TILE, where)

        def twr(I, J, where):
            o = off(I, J)
            g.wr("ws", o, o + TILE, where)

        def ent(kind, I, J, row, col, where):
            o = off(I, J) + row * TST + col
            (g.wr if kind == "w" else g.rd)("ws", o, o + 1, where)

        g.bar("element start")
        g.bar("element loaded")
        g.bar("set-up tables")
        g.bar("block_sum3 a")
        g.bar("block_sum3 b")
        g.bar("set-up end")
        if not fp32:
            g.bar("refine64 a")
            g.bar("refine64 b")
        # ------------------------------------------------ fill
        if fused:
            for tid in threads:
                rr, cl = tid >> 4, tid & 15
                for I in range(nt):
                    for J in range(I + 1):
                        ent("w", I, J, rr, cl, "fill g c c")
            g.bar("fill a")
            for q in range(n):
                if (q % NTH) // 64 != wave:
                    continue
                i, j = _node_ij(q, s)
                ps = [q]
                if i + j <= s - 1:
                    ps += [q + 1, q + (s + 1 - j)]
                if i >= 1:
                    ps.append(q + (s - j))
                for p in ps:
                    ent("r", p >> 4, q >> 4, p & 15, q & 15, "stencil add")
                    ent("w", p >> 4, q >> 4, p & 15, q & 15, "stencil add")
            for tid in threads:
                a, cl = tid >> 4, tid & 15
                for J in range(nt):
                    ent("w", nt, J, a, cl, "fill rhs")
        else:
            for tid in threads:
                rr, cl = tid & 15, tid >> 4
                for I in range(nt):
                    for J in range(I + 1):
                        p, q = 16 * I + rr, 16 * J + cl
                        if p < n and q < n:
                            g.rd("Ahat", q * n + p, q * n + p + 1, "fill from Ahat")
                        ent("w", I, J, rr, cl, "fill from Ahat")
            for tid in threads:
                a, cl = tid >> 4, tid & 15
                for J in range(nt):
                    ent("w", nt, J, a, cl, "fill rhs")
        g.bar("fill end")

        def lo_tile(I, J, where):
            for rr in range(16):
                for cl in range(16):
                    p, q = 16 * I + rr, 16 * J + cl
                    if p < n and q < n and p >= q:
                        g.wr("Ahat", q * n + p, q * n + p + 1, where)

        # ------------------------------------------------ factorisation
        for k in range(-1, nt):
            if k >= 0:
                for i in range(k + 1 + wave, nt + 1, 2 * NWAVES):
                    i2 = i + NWAVES
                    two = i2 <= nt
                    trd(k, k, "panel W")
                    trd(i, k, "panel A1")
                    trd(i2 if two else i, k, "panel A2")
                    twr(i, k, "panel L1")
                    if three_call and i < nt:
                        lo_tile(i, k, "panel L into Lo")
                    if two:
                        twr(i2, k, "panel L2")
                        if three_call and i2 < nt:
                            lo_tile(i2, k, "panel L into Lo")
                g.bar(f"panel {k}")
            m = nt - 1 - k
            if wave == 0:
                if m > 0:
                    if k >= 0:
                        trd(k + 1, k + 1, "look-ahead update")
                        trd(k + 1, k, "look-ahead update")
                        twr(k + 1, k + 1, "look-ahead update")
                    trd(k + 1, k + 1, "diagonal factor")
                    twr(k + 1, k + 1, "diagonal factor")
                    if three_call:
                        lo_tile(k + 1, k + 1, "diagonal L into Lo")
            elif k >= 0 and m > 0:
                ntr = m * (m + 3) // 2
                nw = NWAVES - 1
                t0 = wave if trail_skip_first else wave - 1
                for t in range(t0, ntr, 2 * nw):
                    t2 = t + nw
                    two = t2 < ntr
                    i1, j1 = _trail_ij(t, k, nt)
                    i2, j2 = _trail_ij(t2, k, nt) if two else (i1, j1)
                    for (I, J) in ((i1, j1), (i2, j2)):
                        trd(I, J, "trailing C")
                        trd(I, k, "trailing L")
                        trd(J, k, "trailing L")
                    twr(i1, j1, "trailing C")
                    if two:
                        twr(i2, j2, "trailing C")
            g.bar(f"trailing {k}")

        def backward(tag):
            for j in range(nt - 1, -1, -1):
                if wave == (j & (NWAVES - 1)):
                    trd(nt, j, tag)
                    trd(j, j, tag)
                    twr(nt, j, tag)
                g.bar(f"{tag} solve {j}")
                for i in range(wave, j, NWAVES):
                    trd(nt, i, tag)
                    trd(nt, j, tag)
                    trd(j, i, tag)
                    twr(nt, i, tag)
                g.bar(f"{tag} update {j}")

        def forward(tag):
            for j in range(nt):
                if wave == (j & (NWAVES - 1)):
                    trd(nt, j, tag)
                    trd(j, j, tag)
                    twr(nt, j, tag)
                g.bar(f"{tag} solve {j}")
                for i in range(j + 1 + wave, nt, NWAVES):
                    trd(nt, i, tag)
                    trd(nt, j, tag)
                    trd(i, j, tag)
                    twr(nt, i, tag)
                g.bar(f"{tag} update {j}")

        backward("backward")

        def rhs_entry(kind, p, a, where):
            ent(kind, nt, p >> 4, a, p & 15, where)

        if refine:
            gpc = NTH // 256

            def accumulate(init, where):
                for tid in threads:
                    grp, cl = tid >> 4, tid & 15
                    a, kk = grp & 15, grp >> 4
                    if a >= r:
                        continue
                    for p in range(16 * kk + cl, n, 16 * gpc):
                        rhs_entry("r", p, a, where)
                        if not init:
                            g.rd("X", a * n + p, a * n + p + 1, where)
                        g.wr("X", a * n + p, a * n + p + 1, where)
                g.bar(f"{where} a")
                g.bar(f"{where} b")

            def residual(where):
                for p in range(16 * nt):
                    if (p % NTH) // 64 == wave:
                        for a in range(0 if p >= n else r, 16):
                            rhs_entry("w", p, a, where + " padding")
                for p in range(n):
                    if (p % NTH) // 64 != wave:
                        continue
                    i, j = _node_ij(p, s)
                    nb = [p]
                    if i + j <= s - 1:
                        nb += [p + 1, p + (s + 1 - j)]
                    if i >= 1:
                        nb += [p - 1, p + (s - j)]
                    if j >= 1:
                        nb += [p - (s + 2 - j), p - (s + 1 - j)]
                    for a in range(r):
                        for q in nb:
                            g.rd("X", a * n + q, a * n + q + 1, where)
                        rhs_entry("w", p, a, where)
                g.bar(f"{where} max a")
                g.bar(f"{where} max b")

            def colmax(where):
                for tid in threads:
                    grp, cl = tid >> 4, tid & 15
                    a, kk = grp & 15, grp >> 4
                    if a < r:
                        for p in range(16 * kk + cl, n, 16 * gpc):
                            rhs_entry("r", p, a, where)
                g.bar(f"{where} a")
                g.bar(f"{where} b")

            accumulate(True, "accumulate 0")
            for it in range(ir_steps + 1):
                if not fp32 and it >= 1:
                    g.bar("converged")
                    break
                residual(f"residual {it}")
                if fp32:
                    if it == 0:
                        colmax("bmax")
                    colmax(f"rmax {it}")
                    g.bar(f"decide {it}")
                    if it == ir_steps:
                        break
                forward(f"forward {it}")
                backward(f"backward {it}")
                accumulate(False, f"accumulate {it + 1}")
            for idx in range(n * r):
                if (idx % NTH) // 64 == wave:
                    g.rd("X", idx, idx + 1, "projection")
                    g.wr("X", idx, idx + 1, "projection")
            g.bar("projection")
        else:
            for tid in threads:
                ca, cl16 = tid >> 4, tid & 15
                if ca < r:
                    for p in range(cl16, n, 16):
                        rhs_entry("r", p, ca, "column sums")
            g.bar("cx")
            for idx in range(n * r):
                if (idx % NTH) // 64 == wave:
                    a, p = divmod(idx, n)
                    rhs_entry("r", p, a, "X out")
                    g.wr("X", idx, idx + 1, "X out")
            g.bar("X out")
        if fused:
            P = NI // 3
            from tests.ll_schedule_model import _face_node
            for idx in range(NI * r):
                if (idx % NTH) // 64 == wave:
                    a, b = idx % NI, idx // NI
                    for kk in range(s + 1):
                        q = _face_node(a // P, kk, s)
                        g.rd("X", b * n + q, b * n + q + 1, "contribution")
        logs.append(g)
    lds = dict(stage=1 << 62, size=1 << 62)   # no LDS regions of their own in this model
    return logs, dict(n=n, nt=nt, r=r, NI=NI, lds=lds, ws_elems=ntiles * TILE, x_elems=n * r, a_elems=n * n)
