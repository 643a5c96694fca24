"""Build ``libmhm.so`` (the C-ABI library) in-tree with hipcc for gfx950.

Usage: ``python -m paper_1703_10435_amd.build``.  Compiles every time it is
called (a stale library is never reused silently).
"""
from __future__ import annotations

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


def build(verbose: bool = False) -> str:
    cc = hipcc()
    objs = [os.path.join(CSRC, src.replace(".hip", ".o")) for src in SOURCES]

    def compile_one(i):
        cmd = [cc, *compile_flags(), "-c", os.path.join(CSRC, SOURCES[i]), "-o", objs[i]]
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
