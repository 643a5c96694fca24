"""Host model of the dynamic LDS layouts of the two stand-alone HBM-bound
kernels (paper_1703_10435_amd/csrc/mhm_kernels.hip), the same arithmetic as
their launchers, checked over every batch shape the library accepts
(s_max 1..64, p_max 1..16): the regions the kernels index stay inside what
the launch allocates, and the allocation fits the CU's 160 KB next to the
kernels' static arrays.

k_contrib: per wave, the face-load table R (NImax (s_max + 1) doubles, the
element's NI (s + 1) entries used), the staged face rows (ccmax columns of
3 (s_max + 1) doubles) and the 3 (s_max + 1) face-node offsets (ints); nw
waves per workgroup.
k_assemble: kappa (s_max^2), c and bf (n_max each), the face table
(NImax (s_max + 1)), the stencil table (7 tn doubles) and the lattice rows
(tn ints), tn = n_max where that fits, else 256 (elements of more nodes take
their stencils on the fly)."""
from __future__ import annotations

import pytest

LDS = 160 * 1024
STATIC_MAX = 4096          # bytes kept for the kernels' static arrays
ASM_TAB = 256


def n_of(s):
    return (s + 1) * (s + 2) // 2


def contrib_layout(s_max, p_max):
    nimax = 3 * p_max
    fcap = nimax * (s_max + 1)
    nf = 3 * (s_max + 1)
    ncap = (nf + 1) // 2
    cc = 16
    while cc > 4 and (fcap + cc * nf + ncap) * 8 > 10240:
        cc //= 2
    cap = fcap + cc * nf + ncap
    nw = max(1, min(4, 65536 // (8 * cap)))
    return dict(fcap=fcap, nf=nf, ncap=ncap, cc=cc, cap=cap, nw=nw, bytes=8 * cap * nw)


def assemble_layout(s_max, p_max):
    nmax = n_of(s_max)
    fcap = 3 * p_max * (s_max + 1)

    def lds_of(tn):
        return 8 * (s_max * s_max + 2 * nmax + fcap + 7 * tn) + 4 * tn
    full = lds_of(nmax) + STATIC_MAX <= LDS
    tn = nmax if (full or nmax < ASM_TAB) else ASM_TAB
    return dict(full=full, tn=tn, bytes=lds_of(tn), nmax=nmax)


SHAPES = [(s, p) for s in range(1, 65) for p in range(1, 17)]


@pytest.mark.parametrize("s_max,p_max", [(s, p) for s, p in SHAPES if p in (1, 4, 16) or s in (1, 16, 32, 48, 54, 55, 64)])
def test_contrib_layout_holds_every_element(s_max, p_max):
    L = contrib_layout(s_max, p_max)
    assert L["nw"] >= 1 and L["bytes"] + STATIC_MAX <= LDS
    for s in range(1, s_max + 1):
        for P in range(1, p_max + 1):
            NI, sp1 = 3 * P, s + 1
            r = NI + 1
            # R table: ft[a sp1 + k], a < NI, k <= s
            assert (NI - 1) * sp1 + s < L["fcap"]
            # staged rows: xs[c nf_e + j], c < min(r, cc), j < 3 sp1, nf_e = 3 sp1
            cc = min(r, L["cc"])
            assert (cc - 1) * 3 * sp1 + 3 * sp1 - 1 < L["cc"] * L["nf"]
            # face-node offsets: 3 sp1 ints after ft and xs
            assert 3 * sp1 <= 2 * L["ncap"]
    assert L["fcap"] + L["cc"] * L["nf"] + L["ncap"] == L["cap"]


def test_contrib_chunks_at_the_benchmark_shapes():
    assert contrib_layout(32, 4)["cc"] == 8          # C3: eight columns per chunk, 9.9 KB per wave
    assert contrib_layout(16, 3)["cc"] == 16         # C2
    assert contrib_layout(32, 16)["cc"] == 4         # m = 4 (r = 49): never fewer than four
    assert contrib_layout(64, 16)["nw"] == 2


@pytest.mark.parametrize("s_max,p_max", SHAPES)
def test_assemble_layout_fits(s_max, p_max):
    L = assemble_layout(s_max, p_max)
    assert L["bytes"] + STATIC_MAX <= LDS, (s_max, p_max, L)
    # elements that use the table have at most tn nodes
    for s in range(1, s_max + 1):
        n = n_of(s)
        tab = L["full"] or n <= ASM_TAB
        if tab:
            assert n <= L["tn"]


def test_assemble_full_table_up_to_s53():
    assert assemble_layout(53, 16)["full"] and not assemble_layout(54, 16)["full"]
    assert assemble_layout(48, 4)["full"] and not assemble_layout(64, 5)["full"]
