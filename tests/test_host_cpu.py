"""CPU-only checks of the boundary: the built library exports every symbol the
header declares, the host-side layout and validation, loud failure when the
library is missing."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

from mhm_inputs import configs
from paper_1703_10435_amd import abi
from paper_1703_10435_amd import batch as hb
from tests.parity_util import ROOT, ensure_built


def _declared():
    with open(os.path.join(ROOT, "include", "mhm.h")) as fh:
        txt = fh.read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)          # drop comments
    return sorted(set(re.findall(r"\b(mhm_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_1703_10435_amd import serve
    path = ensure_built()
    lib = ctypes.CDLL(path)
    names = _declared()
    assert set(names) == set(abi.EXPORTS) | set(serve.SERVER_EXPORTS)
    for name in names:
        assert hasattr(lib, name), name


def test_missing_library_fails_loudly(tmp_path):
    saved = abi._lib
    abi._lib = None
    try:
        with pytest.raises(FileNotFoundError):
            abi.load(str(tmp_path / "nope.so"))
    finally:
        abi._lib = saved


def test_structs_match_header_layout(tmp_path):
    """sizeof and every field offset of the ctypes mirrors against the C
    compiler's view of include/mhm.h."""
    import shutil
    import subprocess
    from paper_1703_10435_amd import serve
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"mhm_batch": abi.mhm_batch, "mhm_server_config": serve.ServerConfig, "mhm_request": serve.Request,
               "mhm_result": serve.Result, "mhm_server_stats": serve.ServerStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mhm.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in mirrors.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_layout_offsets():
    lay = hb.layout(np.array([4, 1, 16]), np.array([1, 0, 2]))
    assert list(lay["n"]) == [15, 3, 153]
    assert list(lay["r"]) == [7, 4, 10]
    assert list(lay["mat_off"]) == [0, 225, 234, 234 + 153 * 153]
    assert list(lay["rhs_off"]) == [0, 105, 117, 117 + 1530]
    assert list(lay["tri_off"]) == [0, 16, 17, 273]


@pytest.mark.parametrize("mutate,msg", [
    (lambda b: b["kappa"].__setitem__(3, np.nan), "non-finite"),
    (lambda b: b["s"].__setitem__(0, 0), "s must"),
    (lambda b: b["l"].__setitem__(0, 9), "l must"),
    (lambda b: b["sigma"].__setitem__((0, 0), 2), "sigma"),
    (lambda b: b["vert"].__setitem__(0, b["vert"][0][[0, 1, 4, 5, 2, 3]]), "counter-clockwise"),
    (lambda b: b.__setitem__("m", np.full(b["n_elem"], 3, dtype=np.int32)), "divide s"),
    (lambda b: (b.__setitem__("m", np.full(b["n_elem"], 4, dtype=np.int32)), b["l"].fill(4)), "at most"),
])
def test_validate_rejects_malformed_batches(mutate, msg):
    b = configs.make("C1")
    for k in ("kappa", "s", "l", "sigma", "vert"):
        b[k] = np.array(b[k], copy=True)
    mutate(b)
    with pytest.raises(ValueError, match=msg):
        hb.validate(b)


def test_validate_accepts_configs():
    hb.validate(configs.make("C1"))
    hb.validate(configs.make("C2", n_elem=4))


@pytest.mark.parametrize("N,l,l_max,m", [(2, 1, 1, 1), (3, 0, 2, 1), (4, 2, 4, 1), (2, 1, 1, 2), (3, 0, 4, 3)])
def test_skeleton_numbering_and_pattern(N, l, l_max, m):
    """The host numbering gives the oracle's global DoFs, and the CSR pattern
    is exactly the set of positions that a dense assembly of nonzero element
    blocks touches, with sorted columns."""
    from mhm_inputs.mesh import coarse_mesh
    from oracle import skeleton as oskel
    from paper_1703_10435_amd import skeleton as sk
    mesh = coarse_mesh(N)
    nt = mesh["elems"].shape[0]
    p_max = max(l_max + 1, m * (l + 1))
    gdof, erow, n_rows = sk.numbering(mesh["elem_face"], mesh["faces"].shape[0], l, p_max=p_max, m=m)
    NI = 3 * m * (l + 1)
    assert gdof.shape == (nt, 3 * p_max) and np.all(gdof[:, NI:] == -1)
    for t in range(nt):
        np.testing.assert_array_equal(gdof[t, :NI], oskel.global_dofs(mesh, t, l, m))
    rng = np.random.default_rng(N)
    res = [dict(M=rng.uniform(1, 2, (NI, NI)), B=rng.uniform(1, 2, NI), E=rng.uniform(1, 2, NI), F=1.0)
           for _ in range(nt)]
    K, _ = oskel.assemble_global(mesh, res, np.arange(nt), l, m)
    assert K.shape == (n_rows, n_rows)
    rp, ci = sk.csr_pattern(gdof, erow, n_rows, np.full(nt, NI))
    mask = np.zeros((n_rows, n_rows), dtype=bool)
    for i in range(n_rows):
        cols = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cols) > 0)
        mask[i, cols] = True
    # the block pattern holds the u_0 diagonal, which eq. (6) leaves zero
    diag = np.zeros_like(mask)
    diag[erow, erow] = True
    np.testing.assert_array_equal(mask & ~diag, K != 0)
    assert rp.dtype == np.int32 and ci.dtype == np.int32


def test_library_carries_the_hash_of_its_sources(tmp_path):
    """The built library is stamped with the SHA-256 of the sources it was
    built from; a library with another stamp (or none) counts as stale and
    ensure() would rebuild it."""
    from paper_1703_10435_amd import build
    path = ensure_built()
    h = build.source_hash()
    assert len(h) == 64 and build.stamp_of(path) == h and build.is_current(path)
    assert abi.load().mhm_source_hash().decode() == h
    stale = tmp_path / "stale.so"
    stale.write_bytes(b"\0" * 64 + build.STAMP_TAG + b"0" * 64 + b"\0")
    assert build.stamp_of(str(stale)) == "0" * 64 and not build.is_current(str(stale))
    (tmp_path / "none.so").write_bytes(b"\0" * 128)
    assert build.stamp_of(str(tmp_path / "none.so")) is None
    assert not build.is_current(str(tmp_path / "missing.so"))
