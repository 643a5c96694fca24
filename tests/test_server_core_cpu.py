"""The serving runtime's host state (factor arena, admission, completion and
failed-launch bookkeeping) built on its own with g++ under AddressSanitizer
and UndefinedBehaviorSanitizer, and run on the CPU."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

from tests.parity_util import ROOT


def test_server_core_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "server_core_test")
    src = os.path.join(ROOT, "tests", "server_core_test.cpp")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-Wall", "-Werror", src, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok", r.stdout + r.stderr
