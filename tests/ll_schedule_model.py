"""Host model of the left-looking kernel's schedule (``k_local_ll`` in
paper_1703_10435_amd/csrc/mhm_local_ll.h), for the race and bounds checks of
test_schedule_cpu.py.

For one element and one kernel instance the model walks every wave through
the kernel's loops as the source issues them - the panel loop with its row
passes, the earlier-column updates, the diagonal tile, the panel solve and
the in-panel update, the triangular sweeps, the output of X and the
refinement passes - and records each wave's reads and writes of

  * the workgroup's workspace slot (factor tiles and the right-hand-side
    tile row, in elements of the factor type),
  * the dynamic LDS regions (c, bf, ft, the two staging tiles, the panel's
    diagonal inverses, the published panel tiles, each wave's scratch tile),
  * the element's X block (column-major n x r),

tagged with the number of barriers the wave has passed.  Accesses with the
same tag run concurrently.  check() then reports every access outside its
buffer, every pair of waves that touch the same entries between two
barriers with at least one write, and any difference in the barrier
sequence of the waves (a barrier some wave would skip).

Thread-level loops are modelled by the threads' index sets (a wave is
threads 64 w .. 64 w + 63); tile operations by whole tiles (16 rows of
stride 17).  The model mirrors the kernel's index arithmetic; it is a check
of the schedule as written, not of the compiled code.
"""
from __future__ import annotations

from dataclasses import dataclass, field

TST = 17
TILE = 16 * TST
R_CHUNK = 16


def n_of(s: int) -> int:
    return (s + 1) * (s + 2) // 2


def rows_per_wave(nt: int, nw: int) -> int:
    rows = nt + 1
    for rpw in (2, 3, 5):
        if rows <= rpw * nw:
            return rpw
    if rows <= 10 * nw and nw == 8:
        return 10
    return -1


def launch_rows(fp32: bool, pw: int, nt: int, ref: bool = False, mc: bool = False) -> int:
    """Rows per wave of the instance the library launches (one workgroup per
    CU, 8 waves): FP64 four-tile panels for five rows per wave run on the
    ten-row instance."""
    rpw = rows_per_wave(nt, 8)
    if not fp32 and not ref and not mc and pw == 4 and rpw == 5:
        return 10
    return rpw


@dataclass
class Instance:
    """Template parameters of one k_local_ll instance (one-chunk forms)."""
    fp32: bool
    pw: int
    rpw: int
    nw: int = 8
    occ: int = 1
    ref: bool = False
    fused: bool = True

    @property
    def tsize(self) -> int:
        return 4 if self.fp32 else 8

    @property
    def rs(self) -> int:
        """Row passes per block column (the kernel's RS)."""
        acc = self.pw * 4 * (self.tsize // 4)
        if self.occ != 1:
            return 1
        if self.nw == 8 and self.rpw == 10:
            return 1 if 10 * acc <= 80 else 2 if 5 * acc <= 80 else 5
        if self.nw == 16 and self.rpw == 5:
            return 1 if 5 * acc <= 40 else 5
        return 1

    @property
    def nb(self) -> int:
        """Operand buffers of the earlier-column loop (the kernel's NB)."""
        rh = self.rpw // self.rs
        w = self.tsize // 4
        accr, stg = rh * self.pw * 4 * w, (rh + self.pw) * 4 * w
        bud = 88 if (self.nw == 16 or self.occ == 2) else 150
        return 3 if accr + 3 * stg <= bud else 2 if accr + 2 * stg <= bud else 1

    @property
    def sweep_nb(self) -> int:
        if self.occ == 2 or self.nw == 16:
            return 1
        if self.fp32:
            return 3 if self.rpw <= 5 else 2
        return 2 if self.rpw <= 5 else 1


@dataclass
class Launch:
    """Launch-wide capacities (the plan's n_cap, f_cap, tile_cap)."""
    n_cap: int
    f_cap: int
    tile_cap: int

    @staticmethod
    def for_class(s_cap: int, l_max: int) -> "Launch":
        n_cap = n_of(s_cap)
        nt = (n_cap + 15) // 16
        return Launch(n_cap, 3 * (l_max + 1) * (s_cap + 1), nt * (nt + 1) // 2 + nt + nt)


@dataclass
class Access:
    epoch: int
    wave: int
    write: bool
    space: str
    lo: int
    hi: int          # exclusive
    where: str


@dataclass
class WaveLog:
    wave: int
    epoch: int = 0
    barriers: list = field(default_factory=list)
    acc: list = field(default_factory=list)

    drop: tuple = ()

    def bar(self, site: str):
        if any(site.startswith(d) for d in self.drop):
            return
        self.barriers.append(site)
        self.epoch += 1

    def rd(self, space, lo, hi, where):
        self.acc.append(Access(self.epoch, self.wave, False, space, lo, hi, where))

    def wr(self, space, lo, hi, where):
        self.acc.append(Access(self.epoch, self.wave, True, space, lo, hi, where))


def lds_layout(inst: Instance, lau: Launch) -> dict:
    """Byte ranges of the kernel's dynamic LDS regions (as the kernel carves
    dyn[]) and the size the launch allocates (local_ll_lds_bytes)."""
    d = 8
    c0 = 0
    bf0 = c0 + d * lau.n_cap
    ft0 = bf0 + d * lau.n_cap
    st0 = ft0 + d * lau.f_cap
    tb = TILE * inst.tsize
    wt0 = st0 + 2 * tb
    pub0 = wt0 + inst.pw * tb
    scr0 = pub0 + inst.pw * inst.pw * tb
    size = d * (2 * lau.n_cap + lau.f_cap) + (2 + inst.pw + inst.pw * inst.pw + inst.nw) * tb
    return dict(c=c0, bf=bf0, ft=ft0, stage=st0, Wt=wt0, pub=pub0, scr=scr0, size=size, tile=tb)


def simulate(inst: Instance, lau: Launch, s: int, l: int, ref64: bool = False, ir_steps: int = 2,
             three_call: bool = False, lo_inside: bool = False, drop: tuple = (), lds_short: int = 0,
             publish_shift: int = 0):
    """All waves' logs for one element (s, l) of one launch.

    three_call: the non-fused form (operator tiles read from Ahat, the
    factor written back into the same array, Lo = Ahat).  lo_inside: the
    factor written from inside the factorisation (diagonal tile and panel
    solve) instead of one pass after it, as an earlier version of the kernel
    did.  The last three arguments plant mistakes for the model's own tests:
    barriers whose site starts with a prefix in `drop` are left out, the LDS
    allocation is `lds_short` tiles short, and the panel solve publishes its
    tile `publish_shift` slots off."""
    n = n_of(s)
    nt = (n + 15) // 16
    NI = 3 * (l + 1)
    r = NI + 1
    NW, PW, RPW = inst.nw, inst.pw, inst.rpw
    RS = inst.rs
    RH = RPW // RS
    NTH = 64 * NW
    L = lds_layout(inst, lau)
    tb = L["tile"]
    L["size"] -= lds_short * tb
    fp32 = inst.fp32
    refine = fp32 or ref64

    def tl(I, J):
        """Workspace offset (elements) of tile (I, J): the factor's lower
        triangle, then the right-hand-side row."""
        if I == nt:
            return (nt * (nt + 1)) // 2 * TILE + J * TILE
        assert 0 <= J <= I < nt, (I, J, nt)
        return ((I * (I + 1)) // 2 + J) * TILE

    def ldiag(J):
        return (nt * (nt + 1)) // 2 * TILE + (1 * nt + J) * TILE

    held = lambda i: i <= nt
    rhs = lambda i: i == nt

    logs = []
    for wave in range(NW):
        g = WaveLog(wave, drop=tuple(drop))
        threads = range(64 * wave, 64 * wave + 64)

        def ahat_tile_rd(I, J, where):
            """init_tile of the non-fused form: A[q n + p] for the tile's
            entries (p, q) inside the element (the upper part of a diagonal
            tile included)."""
            for rr in range(16):
                p = 16 * I + rr
                for cl in range(16):
                    q = 16 * J + cl
                    if p < n and q < n:
                        g.rd("Ahat", q * n + p, q * n + p + 1, where)

        def lo_tile_wr(I, J, where):
            """The factor's entries (p >= q) of tile (I, J) into Lo = Ahat."""
            for rr in range(16):
                p = 16 * I + rr
                for cl in range(16):
                    q = 16 * J + cl
                    if p < n and q < n and p >= q:
                        g.wr("Ahat", q * n + p, q * n + p + 1, where)

        def tile_rd(I, J, where):
            o = tl(I, J)
            g.rd("ws", o, o + TILE, where)

        def tile_wr(I, J, where):
            o = tl(I, J)
            g.wr("ws", o, o + TILE, where)

        def lds(kind, base, k, where):
            lo = L[base] + k * tb
            (g.wr if kind == "w" else g.rd)("lds", lo, lo + tb, where)

        def lds_d(kind, base, idx, where):   # one double of c, bf or ft
            lo = L[base] + 8 * idx
            (g.wr if kind == "w" else g.rd)("lds", lo, lo + 8, where)

        scr_k = L["scr"] - L["pub"] - PW * PW * tb + wave * tb   # scratch tile of this wave
        # ------------------------------------------------ element start
        g.bar("element start")
        g.bar("element loaded")
        # ------------------------------------------------ set-up
        if inst.fused:
            for idx in range(NI * (s + 1)):
                if (idx % NTH) // 64 == wave:
                    lds_d("w", "ft", idx, "face table")
        g.bar("face table")
        for p in range(n):
            if (p % NTH) // 64 == wave:
                lds_d("w", "c", p, "c")
                if inst.fused:
                    lds_d("w", "bf", p, "bf")
        g.bar("block_sum3 a")
        g.bar("block_sum3 b")
        if inst.fused and wave == 0:
            for a in range(min(NI, 64)):
                for k in range(s + 1):
                    lds_d("r", "ft", a * (s + 1) + k, "face colsums")
        g.bar("set-up end")
        if not fp32 or inst.fused:   # FP64: the refinement criterion; fused FP32: the deferral test
            g.bar("refine64 a")
            g.bar("refine64 b")
        # ------------------------------------------------ factorisation
        for j0 in range(0, nt, PW):
            pw = min(PW, nt - j0)
            for h in range(RS):
                if h > 0 and j0 + NW * RH * h >= nt + 1:
                    break
                row_of = lambda ri: j0 + wave + NW * (h * RH + ri)
                # (b) earlier columns: no barriers
                if j0 > 0 and held(row_of(0)):
                    r0 = row_of(0)
                    for m in range(j0):
                        for ri in range(RH):
                            i = row_of(ri)
                            if held(i):
                                tile_rd(i, m, "update A")
                            elif inst.nb == 1:
                                tile_rd(r0, m, "update A (clamped)")
                        for jj in range(PW):
                            if jj < pw:
                                tile_rd(j0 + jj, m, "update B")
                            elif inst.nb == 1:
                                tile_rd(j0, m, "update B (clamped)")
                # operator: reads of c, bf, ft (or of Ahat in the non-fused form)
                for ri in range(RH):
                    i = row_of(ri)
                    if held(i) and three_call and not rhs(i):
                        for jj in range(pw):
                            if i >= j0 + jj:
                                ahat_tile_rd(i, j0 + jj, "operator Ahat")
                    if held(i):
                        g.rd("lds", L["c"], L["c"] + 8 * n, "operator c")
                        if inst.fused:
                            g.rd("lds", L["bf"], L["bf"] + 8 * n, "operator bf")
                            g.rd("lds", L["ft"], L["ft"] + 8 * NI * (s + 1), "operator ft")
                # (c) the panel
                for jj in range(pw):
                    col = j0 + jj
                    if h == 0:
                        if wave == jj:
                            lds("w", "Wt", jj, "diag store")
                            lds("r", "Wt", jj, "potrf")
                            lds("w", "Wt", jj, "potrf")
                            if three_call and lo_inside:
                                lo_tile_wr(col, col, "L_jj into Lo")
                            elif three_call:
                                o = ldiag(col)
                                g.wr("ws", o, o + TILE, "L_jj output")
                            lds("r", "Wt", jj, "diag copy")
                            tile_wr(col, col, "diag copy")
                        g.bar(f"diag {col}")
                    for ri in range(RH):
                        i = row_of(ri)
                        if i > col and held(i):
                            g.wr("lds", L["scr"] + wave * tb, L["scr"] + (wave + 1) * tb, "panel solve scr")
                            g.rd("lds", L["scr"] + wave * tb, L["scr"] + (wave + 1) * tb, "panel solve scr")
                            lds("r", "Wt", jj, "panel solve W")
                            tile_wr(i, col, "panel solve")
                            if three_call and lo_inside and i < nt:
                                lo_tile_wr(i, col, "L_i,col into Lo")
                            if i < j0 + pw:
                                lds("w", "pub", jj * PW + i - j0 + publish_shift, "publish")
                    if h == 0:
                        g.bar(f"panel solve {col}")
                    if jj + 1 < pw:
                        for ri in range(RH):
                            i = row_of(ri)
                            if i > col and held(i):
                                g.wr("lds", L["scr"] + wave * tb, L["scr"] + (wave + 1) * tb, "in-panel scr")
                                g.rd("lds", L["scr"] + wave * tb, L["scr"] + (wave + 1) * tb, "in-panel scr")
                                for j2 in range(jj + 1, PW):
                                    if j2 < pw and (rhs(i) or i >= j0 + j2):
                                        lds("r", "pub", jj * PW + j2, "in-panel pub")
                g.bar(f"pass end {j0}/{h}")
        # ------------------------------------------------ factor output
        if three_call and not lo_inside:
            for t in range(wave, nt * (nt + 1) // 2, NW):
                I = 0
                while (I + 1) * (I + 2) // 2 <= t:
                    I += 1
                J = t - I * (I + 1) // 2
                if I == J:
                    o = ldiag(J)
                    g.rd("ws", o, o + TILE, "factor output diag")
                else:
                    tile_rd(I, J, "factor output")
                lo_tile_wr(I, J, "factor output into Lo")

        # ------------------------------------------------ sweeps
        def sweep(back: bool, tag: str):
            NB = inst.sweep_nb
            colj = (lambda st: nt - 1 - st) if back else (lambda st: st)
            upd = (lambda i, j: i < j) if back else (lambda i, j: j < i < nt)
            own = [wave + NW * ri for ri in range(RPW) if wave + NW * ri < nt]
            for i in own:
                tile_rd(nt, i, f"{tag} z load")

            def fetch(st):
                if st >= nt:
                    return
                j = colj(st)
                for i in own:
                    if upd(i, j):
                        tile_rd(j, i, f"{tag} L") if back else tile_rd(i, j, f"{tag} L")
                if st + 1 < nt and wave == colj(st + 1) % NW:
                    tile_rd(colj(st + 1), colj(st + 1), f"{tag} W")

            j = colj(0)
            if wave == j % NW:
                tile_rd(j, j, f"{tag} W0")
            for q in range(NB):
                fetch(q)
            if j in own:
                g.wr("lds", L["scr"] + wave * tb, L["scr"] + (wave + 1) * tb, f"{tag} solve scr")
                g.rd("lds", L["scr"] + wave * tb, L["scr"] + (wave + 1) * tb, f"{tag} solve scr")
                lds("w", "stage", 0, f"{tag} publish")
            g.bar(f"{tag} start")
            for st in range(nt):
                j = colj(st)
                jn = colj(st + 1) if st + 1 < nt else -1
                lds("r", "stage", st & 1, f"{tag} read x")
                for i in own:
                    if upd(i, j) and i == jn:
                        g.wr("lds", L["scr"] + wave * tb, L["scr"] + (wave + 1) * tb, f"{tag} solve scr")
                        g.rd("lds", L["scr"] + wave * tb, L["scr"] + (wave + 1) * tb, f"{tag} solve scr")
                        lds("w", "stage", (st + 1) & 1, f"{tag} publish")
                g.bar(f"{tag} step {st}")
                fetch(st + NB)
            for i in own:
                tile_wr(nt, i, f"{tag} z store")
            g.bar(f"{tag} end")

        sweep(True, "backward")

        # ------------------------------------------------ X and refinement
        def x_write_all(where):     # idx = tid .. n r step NTH: X[a n + p]
            for idx in range(n * r):
                if (idx % NTH) // 64 == wave:
                    g.wr("X", idx, idx + 1, where)

        def rhs_read_all(where):
            for J in range(nt):
                tile_rd(nt, J, where)

        ca_groups = [tid >> 4 for tid in threads]
        if not refine:
            if any(ca < r for ca in ca_groups):
                rhs_read_all("column sums")
            g.bar("cx")
            for idx in range(n * r):
                if (idx % NTH) // 64 == wave:
                    a, p = divmod(idx, n)
                    g.wr("X", idx, idx + 1, "X out")
                    o = tl(nt, p >> 4) + a * TST + (p & 15)
                    g.rd("ws", o, o + 1, "X out")
            g.bar("X out")
            if inst.fused:
                _contribution(g, wave, NTH, n, r, NI, s)
            logs.append(g)
            continue

        gpc = NTH // 256

        def accumulate(init, where):
            for tid in threads:
                grp, cl = tid >> 4, tid & 15
                a, k = grp & 15, grp >> 4
                if a >= r:
                    continue
                step = 16 * gpc
                for p in range(16 * k + cl, n, step):
                    o = tl(nt, p >> 4) + a * TST + (p & 15)
                    g.rd("ws", o, o + 1, where)
                    if not init:
                        g.rd("X", a * n + p, a * n + p + 1, where)
                    g.wr("X", a * n + p, a * n + p + 1, where)
            g.bar(f"{where} a")
            g.bar(f"{where} b")

        def residual(where):
            for p in range(16 * nt):
                if (p % NTH) // 64 == wave:
                    for a in range(0 if p >= n else r, 16):
                        o = tl(nt, p >> 4) + a * TST + (p & 15)
                        g.wr("ws", o, o + 1, where + " padding")
            for p in range(n):
                if (p % NTH) // 64 == wave:
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
                        o = tl(nt, p >> 4) + a * TST + (p & 15)
                        g.wr("ws", o, o + 1, where)
            g.bar(f"{where} max a")
            g.bar(f"{where} max b")

        def colmax(where):
            for tid in threads:
                grp, cl = tid >> 4, tid & 15
                a, k = grp & 15, grp >> 4
                if a < r:
                    for p in range(16 * k + cl, n, 16 * gpc):
                        o = tl(nt, p >> 4) + a * TST + (p & 15)
                        g.rd("ws", o, o + 1, where)
            g.bar(f"{where} a")
            g.bar(f"{where} b")

        accumulate(True, "accumulate 0")
        for it in range(ir_steps + 1):
            if not fp32 and it >= 1:
                break
            residual(f"residual {it}")
            if fp32:
                if it == 0:
                    colmax("bmax")
                colmax(f"rmax {it}")
                g.bar(f"decide {it}")
                if it == ir_steps:
                    break
            sweep(False, f"forward {it}")
            sweep(True, f"backward {it}")
            accumulate(False, f"accumulate {it + 1}")
        for idx in range(n * r):
            if (idx % NTH) // 64 == wave:
                g.rd("X", idx, idx + 1, "projection")
                g.wr("X", idx, idx + 1, "projection")
        g.bar("projection")
        if inst.fused:
            _contribution(g, wave, NTH, n, r, NI, s)
        logs.append(g)
    return logs, dict(n=n, nt=nt, r=r, NI=NI, lds=L, ws_elems=lau.tile_cap * TILE, x_elems=n * r, a_elems=n * n)


def _node_ij(p: int, s: int):
    j = 0
    while (j + 1) * (2 * s + 3 - (j + 1)) // 2 <= p:
        j += 1
    return p - j * (2 * s + 3 - j) // 2, j


def _face_node(e: int, k: int, s: int) -> int:
    row = lambda j: j * (2 * s + 3 - j) // 2
    if e == 0:
        return row(k) + (s - k)
    if e == 1:
        return row(s - k)
    return k


def _contribution(g: WaveLog, wave: int, nth: int, n: int, r: int, NI: int, s: int):
    """contrib_element: thread idx < NI r reads its face's X column entries."""
    P = NI // 3
    for idx in range(NI * r):
        if (idx % nth) // 64 == wave:
            a, b = idx % NI, idx // NI
            for k in range(s + 1):
                q = _face_node(a // P, k, s)
                g.rd("X", b * n + q, b * n + q + 1, "contribution")


def check(logs, meta) -> list:
    """Problems found: barrier sequences that differ between waves,
    accesses outside their buffer, and unordered conflicting accesses."""
    probs = []
    seq0 = logs[0].barriers
    for g in logs[1:]:
        if g.barriers != seq0:
            k = next((i for i, (a, b) in enumerate(zip(seq0, g.barriers)) if a != b), min(len(seq0), len(g.barriers)))
            probs.append(f"barrier sequence of wave {g.wave} differs from wave 0 at barrier {k}: "
                         f"{g.barriers[k:k + 1]} vs {seq0[k:k + 1]}")
    limits = {"ws": meta["ws_elems"], "lds": meta["lds"]["size"], "X": meta["x_elems"], "Ahat": meta["a_elems"]}
    # LDS tiles (staging, diagonal inverses, published panel tiles, scratch)
    # are only read after some wave wrote them: before, in an earlier barrier
    # interval, or the same wave earlier in its program
    tiles0 = meta["lds"]["stage"]
    first_lds = {}
    for g in logs:
        for k, a in enumerate(g.acc):
            if a.space == "lds" and a.write and a.lo >= tiles0:
                first_lds.setdefault(a.lo, []).append((a.epoch, g.wave, k))
    for g in logs:
        for k, a in enumerate(g.acc):
            if a.space == "lds" and not a.write and a.lo >= tiles0:
                ws = first_lds.get(a.lo, [])
                if not any(ep < a.epoch or (w == g.wave and pos < k) for ep, w, pos in ws):
                    probs.append(f"wave {g.wave} reads LDS tile at byte {a.lo} ({a.where}) before any wave "
                                 f"has written it (barrier interval {a.epoch})")
                    if len(probs) > 50:
                        return probs
    # the operator must come from the assembled Ahat: no read of an entry
    # after the factor has been written over it (any wave, any interval; a
    # wave's own accesses are in program order, other waves' in barrier order)
    first_write = {}
    for g in logs:
        for k, a in enumerate(g.acc):
            if a.space == "Ahat" and a.write and a.lo not in first_write:
                first_write[a.lo] = (a.epoch, k, g.wave)
            elif a.space == "Ahat" and a.write:
                first_write[a.lo] = min(first_write[a.lo], (a.epoch, k, g.wave))
    if first_write:
        for g in logs:
            for k, a in enumerate(g.acc):
                if a.space == "Ahat" and not a.write and a.lo in first_write:
                    ep, pos, w = first_write[a.lo]
                    if ep < a.epoch or (ep == a.epoch and (w != g.wave or pos < k)):
                        probs.append(f"wave {g.wave} reads Ahat[{a.lo}] ({a.where}) after the factor was written "
                                     f"over it in barrier interval {ep}")
                        if len(probs) > 50:
                            return probs
    by_epoch = {}
    for g in logs:
        for a in g.acc:
            if a.lo < 0 or a.hi > limits[a.space]:
                probs.append(f"wave {a.wave} {'writes' if a.write else 'reads'} {a.space}[{a.lo}:{a.hi}] "
                             f"outside [0:{limits[a.space]}] ({a.where})")
            by_epoch.setdefault((a.epoch, a.space), []).append(a)
    for (ep, space), lst in by_epoch.items():
        writes = [a for a in lst if a.write]
        if not writes:
            continue
        # sweep over sorted intervals: a write overlapping any access of another wave
        ev = sorted(lst, key=lambda a: a.lo)
        active = []
        for a in ev:
            active = [b for b in active if b.hi > a.lo]
            for b in active:
                if b.wave != a.wave and (a.write or b.write):
                    probs.append(f"barrier interval {ep}, {space}[{max(a.lo, b.lo)}:{min(a.hi, b.hi)}]: wave "
                                 f"{b.wave} {'writes' if b.write else 'reads'} ({b.where}) and wave {a.wave} "
                                 f"{'writes' if a.write else 'reads'} ({a.where})")
                    if len(probs) > 50:
                        return probs
            active.append(a)
    return probs
