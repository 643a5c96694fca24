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
    path = ensure_built()
    lib = ctypes.CDLL(path)
    names = _declared()
    assert set(names) == set(abi.EXPORTS)
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


def test_descriptor_struct_matches_header_layout():
    # 4 int32, 11 pointers, 4 int64 on LP64
    assert ctypes.sizeof(abi.mhm_batch) == 16 + 11 * 8 + 4 * 8


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
