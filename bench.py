"""Throughput of the MHM local-problem path on one MI355X.

A step is one pass of the whole path (assemble, factor, solve, contribution)
over one batch of synthetic local problems, through the fused library call.
The headline workload is the plain-FP64 batch: 32x32x2 = 2048 coarse
triangles, s = 16 (153 P1 nodes), l = 2 (9 face right-hand sides + source),
K = exp(2 g) with g a seeded Gaussian field (correlation length 0.05),
f = 2 pi^2 sin(pi x) sin(pi y).

Prints one JSON line (rank 0).  Timing uses HIP events on the stream the
kernels run on, with all inputs resident in device memory.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 matrix
PEAK_FP32_TFLOPS = 157.3    # MI355X dense FP32 matrix
PEAK_HBM_GBS = 8000.0

WORKLOAD = ("C2: plain FP64 batched, 32x32x2=2048 coarse triangles, s=16 (153 P1 nodes), l=2 (9 face RHS + 1 "
            "source), K=exp(2g) seeded Gaussian field (ell=0.05, seed 2000), f=2pi^2 sin(pi x) sin(pi y)")


def _flops_per_element(n, r):
    """Algorithmic flops of the dense method: Cholesky n^3/3 + forward and
    backward solves 2 n^2 r (the SURVEY's per-element count)."""
    n = np.asarray(n, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    return n ** 3 / 3.0 + 2.0 * n * n * r


def _source_hash():
    """sha256 over the library sources (the same recipe as profiles/*_counters.md)."""
    import glob
    import hashlib
    files = sorted(glob.glob(os.path.join(ROOT, "paper_1703_10435_amd", "csrc", "*.hip"))
                   + glob.glob(os.path.join(ROOT, "paper_1703_10435_amd", "csrc", "*.h"))
                   + [os.path.join(ROOT, "include", "mhm.h")])
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(profile="k_local_rr_C2_fp64_counters.md"):
    """HBM bytes per launch from the committed counter summary (FETCH_SIZE x 2
    + WRITE_SIZE, calibrated on a plain copy), or None when the kernel sources
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "source_sha256"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != _source_hash() or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


# ----------------------------------------------------------- CPU baseline leg
def _oracle_one(args):
    batch_path, e = args
    from oracle import local
    b = _POOL_BATCH
    t = time.perf_counter()
    r = local.solve_element(b, e)
    return e, time.perf_counter() - t, r["X"], r["M"], r["E"], r["B"], r["F"]


_POOL_BATCH = None


def _pool_init(batch):
    global _POOL_BATCH
    _POOL_BATCH = batch
    os.environ["OMP_NUM_THREADS"] = "1"


def cpu_baseline(batch, sample_idx, cores):
    """Time the FP64 oracle (one element per task, one thread per process) on
    a bounded sample of the workload; return rate and its results."""
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores, initializer=_pool_init, initargs=(batch,)) as pool:
        out = pool.map(_oracle_one, [(None, int(e)) for e in sample_idx], chunksize=4)
    wall = time.perf_counter() - t0
    cpu = sum(o[1] for o in out)
    return dict(rate=len(sample_idx) / wall, wall=wall, cpu_seconds=cpu,
                results={o[0]: dict(X=o[2], M=o[3], E=o[4], B=o[5], F=o[6]) for o in out})


# -------------------------------------------------------------------- timing
def time_launches(torch, fn, steps, warmup):
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    per = np.array([a.elapsed_time(b) for a, b in evs])
    return t0.elapsed_time(t1), per


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle sample size (0: auto)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--extra", action="store_true", help="also time the three-call and FP32+IR forms")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a 256 MiB device-to-device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; --gpus must be 1 (the local problems shard "
                                   "by element across GPUs, see DESIGN.md)"}))
        sys.exit(2)

    import torch
    from mhm_inputs import configs
    from paper_1703_10435_amd import abi, engine
    from paper_1703_10435_amd.batch import DeviceBatch

    if not os.path.exists(abi.LIB_PATH):
        from paper_1703_10435_amd import build as _b
        _b.build()
    if args.copy_calib:
        src = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    batch = configs.make("C2")
    db = DeviceBatch(batch)
    out = db.alloc_outputs(three_call=True)
    ctx = abi.Context(0)
    E = batch["n_elem"]

    def step():
        engine.run_fused(ctx, db, abi.MHM_FP64, out)

    total_ms, per = time_launches(torch, step, args.steps, args.warmup)
    ms_per_step = total_ms / args.steps
    info = out["info"].cpu().numpy()[:E]
    res = db.unpack(out)

    flops = float(np.sum(_flops_per_element(db.n, db.r)))
    kern_ms = float(np.mean(per))
    achieved = flops / (kern_ms * 1e-3) / 1e12
    line = {
        "metric": "local problems solved/sec at stated rel. error vs FP64 oracle",
        "value": E / (ms_per_step * 1e-3),
        "unit": "local problems/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOAD, "n_elem": E, "s": 16, "n": 153, "l": 2, "r": 10, "path": "fused mhm_local_batch_run"},
        "info_nonzero": int(np.sum(info != 0)),
        "kernel_ms": {"mean": kern_ms, "p50": float(np.median(per)), "p99": float(np.percentile(per, 99))},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": measured_traffic(),
                     "kernel": "k_local_rr<fused> (FP64, register-resident tiles)", "flops_per_launch": flops,
                     "flops_per_element": "n^3/3 + 2 n^2 r (Cholesky + forward/backward solves)"},
    }

    if args.extra:
        three = lambda: engine.run_three_call(ctx, db, abi.MHM_FP64, out)  # noqa: E731
        t3, p3 = time_launches(torch, three, args.steps, args.warmup)
        fp32 = lambda: engine.run_fused(ctx, db, abi.MHM_FP32_IR, out)  # noqa: E731
        t4, p4 = time_launches(torch, fp32, args.steps, args.warmup)
        its = out["ir_iters"].cpu().numpy()[:E]
        line["extra"] = {
            "three_call_fp64_ms": t3 / args.steps,
            "fused_fp32_ir_ms": t4 / args.steps,
            "fp32_ir_steps_mean": float(its.mean()),
            "fp32_ir_fallbacks": int(np.sum(out["info"].cpu().numpy()[:E] == -1)),
        }
        # leave the FP64 results in `out` for the error check below
        step()
        torch.cuda.synchronize()
        res = db.unpack(out)

    if not args.no_cpu:
        cores = len(os.sched_getaffinity(0))
        cores = min(cores, 16)
        n_s = args.cpu_sample or max(64, min(E, int(25.0 / 0.04)))
        rng = np.random.default_rng(1)
        idx = np.sort(rng.choice(E, size=min(n_s, E), replace=False))
        cb = cpu_baseline(batch, idx, cores)
        errs = []
        for e, o in cb["results"].items():
            g = res[e]
            ex = np.max(np.abs(g["X"] - o["X"])) / np.max(np.abs(o["X"]))
            errs.append(ex)
        line["cpu_baseline"] = {"value": cb["rate"], "unit": "local problems/s", "cores": cores, "kind": "oracle",
                                "sample": f"{len(idx)} of the {E} elements (seeded), one element per task, "
                                          f"{cb['cpu_seconds']:.1f} CPU-s in {cb['wall']:.1f} s wall"}
        line["max_rel_err"] = float(np.max(errs))
        line["rel_err_p99"] = float(np.percentile(errs, 99))
        line["error_check"] = "pass" if line["max_rel_err"] <= 1e-10 and line["info_nonzero"] == 0 else "FAIL"
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
