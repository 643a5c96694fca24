"""Shared helpers of the GPU parity tests (no GPU work here)."""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def ensure_built():
    """The library, rebuilt when it is missing or was built from other sources
    (its stamped source hash differs from the tree's)."""
    from paper_1703_10435_amd import abi, build
    build.ensure()
    return abi.LIB_PATH


def block_of(res: dict) -> np.ndarray:
    """The element's contribution block [[M, B^T], [B, 0] | [E; F]]."""
    M = np.asarray(res["M"])
    ni = M.shape[0]
    blk = np.zeros((ni + 1, ni + 2))
    blk[:ni, :ni] = M
    blk[:ni, ni] = res["B"]
    blk[ni, :ni] = res["B"]
    blk[:ni, ni + 1] = res["E"]
    blk[ni, ni + 1] = res["F"]
    return blk


def rel_errors(gpu: dict, ora: dict):
    """Max-norm relative errors of X (whole n x r block) and of the
    contribution block, per element."""
    ex = np.max(np.abs(gpu["X"] - ora["X"])) / max(np.max(np.abs(ora["X"])), 1e-300)
    bg, bo = block_of(gpu), block_of(ora)
    eb = np.max(np.abs(bg - bo)) / max(np.max(np.abs(bo)), 1e-300)
    return float(ex), float(eb)


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()
