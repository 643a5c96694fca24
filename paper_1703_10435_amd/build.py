"""Build ``libmhm.so`` (the C-ABI library) in-tree with hipcc for gfx950.

Usage: ``python -m paper_1703_10435_amd.build``.  ``build()`` compiles every
time it is called.  The library carries the SHA-256 of the sources and flags
it was built from (``mhm_source_hash()``, and the same text in the file), so
``ensure()`` rebuilds a library whose sources have changed since: a stale
library is never reused silently.
"""
from __future__ import annotations

import glob
import hashlib
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmhm.so")
SOURCES = ["mhm_kernels.hip", "mhm_local_rr.hip", "mhm_local_ll.hip", "mhm_local_ll_f32.hip", "mhm_local_ll_f64.hip",
           "mhm_local_ll_f64r.hip",
           "mhm_source_step.hip", "mhm_skeleton_solve.hip", "mhm_api.hip", "mhm_server.hip"]
ARCH = "gfx950"
INCLUDE = os.path.join(os.path.dirname(HERE), "include", "mhm.h")
STAMP_TAG = b"MHM_SOURCE_SHA256="   # followed by 64 hex digits in the built library


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_flags() -> list:
    return [
        f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
        # packed FP32 arithmetic stays off (plain scalar FP32 code only)
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function",
    ]


def stamped_files() -> list:
    """Every file the library is built from: the HIP sources and headers and
    the public header."""
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.h"))) + [INCLUDE]


def source_hash() -> str:
    """SHA-256 over the file names and contents of stamped_files() and the
    compile flags."""
    h = hashlib.sha256()
    for path in stamped_files():
        h.update(os.path.basename(path).encode() + b"\0")
        with open(path, "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(compile_flags()).encode())
    return h.hexdigest()


def stamp_of(path: str = LIB):
    """The source hash a built library carries (None: no library, or none)."""
    if not os.path.exists(path):
        return None
    with open(path, "rb") as fh:
        data = fh.read()
    k = data.find(STAMP_TAG)
    if k < 0:
        return None
    return data[k + len(STAMP_TAG):k + len(STAMP_TAG) + 64].decode("ascii", "replace")


def is_current(path: str = LIB) -> bool:
    return stamp_of(path) == source_hash()


def ensure(verbose: bool = False) -> str:
    """The library, rebuilt first if it is missing or its sources changed."""
    if not is_current(LIB):
        build(verbose)
    return LIB


def build(verbose: bool = False) -> str:
    cc = hipcc()
    objs = [os.path.join(CSRC, src.replace(".hip", ".o")) for src in SOURCES]
    stamp = f'-DMHM_SOURCE_HASH="{source_hash()}"'

    def compile_one(i):
        cmd = [cc, *compile_flags(), stamp, "-c", os.path.join(CSRC, SOURCES[i]), "-o", objs[i]]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    # one translation unit per worker; .result() re-raises a failed compile
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as pool:
        for f in [pool.submit(compile_one, i) for i in range(len(SOURCES))]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
