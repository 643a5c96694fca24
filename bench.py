"""Throughput of the MHM local-problem path on one MI355X.

A step is one pass of the whole path (assemble, factor, solve, contribution)
over one batch of synthetic local problems, through the fused library call.
The headline workload is the largest single-GPU configuration: the uneven
batch of 64x64x2 = 8192 coarse triangles with s in {8, 16, 32, 48} (by
quartile of each element's local variance of log K, 2048 each), l ~ U{1,2,3},
K = exp(3 g) with g a seeded Gaussian field (correlation length 0.05) and
f = 2 pi^2 sin(pi x) sin(pi y), in plain FP64 (Cholesky on the FP64 matrix
cores; the refinement step where an element needs it).

Prints one JSON line.  Timing uses HIP events on the stream the kernels run
on, with all inputs resident in device memory.
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
# parity bars (max-norm relative error per element against the FP64 oracle)
BAR = {"fp64": 1e-10, "fp32_ir": 1e-8}

WORKLOAD = ("C4: uneven batch, 64x64x2=8192 coarse triangles, s in {8,16,32,48} (45/153/561/1225 P1 nodes, by "
            "quartile of the local log-K variance, 2048 each), l~U{1,2,3} (seed 4001), K=exp(3g) seeded Gaussian "
            "field (ell=0.05, seed 4000), f=2pi^2 sin(pi x) sin(pi y); plain FP64")
# the sources the headline's dominant kernel (k_local_ll, FP64) is built from
LL_SOURCES = ("mhm_device.h", "mhm_common.h", "mhm_kernels.h", "mhm_local_ll.h", "mhm_local_ll_f64.hip")


def _flops_per_element(n, r):
    """Algorithmic flops of the dense method: Cholesky n^3/3 + forward and
    backward solves 2 n^2 r per element."""
    n = np.asarray(n, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    return n ** 3 / 3.0 + 2.0 * n * n * r


def _source_hash(sources=LL_SOURCES):
    """sha256 over the sources a kernel is built from (the same recipe as
    profiles/*_counters.md)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1703_10435_amd", "csrc")
    files = [os.path.join(csrc, f) for f in sources]
    files.append(os.path.join(ROOT, "include", "mhm.h"))
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(profile="k_local_ll_C4_s48_fp64_counters.md", sources=LL_SOURCES):
    """HBM bytes per launch from the committed counter summary (FETCH_SIZE
    and WRITE_SIZE, each scaled by the factor a plain copy calibrates), or
    None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "source_sha256"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != _source_hash(sources) or "traffic_bytes_per_launch" not in vals:
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
    # the BLAS pools were sized when the parent imported numpy: one thread
    # per worker process from here on
    from threadpoolctl import threadpool_limits
    globals()["_LIMITS"] = threadpool_limits(1)


def oracle_solve(batch, e):
    """The FP64 oracle's results for one element (error checks)."""
    from oracle import local
    return local.solve_element(batch, e)


def cpu_baseline(batch, sample_idx, cores):
    """Time the FP64 oracle (one element per task, one thread per process) on
    a bounded sample of the workload; return rate and its results.  The
    tasks go largest element first, one at a time, so that the pool drains
    evenly."""
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    order = sorted((int(e) for e in sample_idx), key=lambda e: -int(batch["s"][e]))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores, initializer=_pool_init, initargs=(batch,)) as pool:
        out = pool.map(_oracle_one, [(None, e) for e in order], chunksize=1)
    wall = time.perf_counter() - t0
    cpu = sum(o[1] for o in out)
    return dict(rate=len(order) / wall, wall=wall, cpu_seconds=cpu, single_core_rate=len(order) / max(cpu, 1e-9),
                results={o[0]: dict(X=o[2], M=o[3], E=o[4], B=o[5], F=o[6]) for o in out})


def stratified(batch, per_class, seed):
    """A seeded sample of per_class elements of each distinct s."""
    rng = np.random.default_rng(seed)
    return np.sort(np.concatenate([rng.choice(np.flatnonzero(batch["s"] == s), size=min(per_class, int(np.sum(batch["s"] == s))),
                                              replace=False) for s in np.unique(batch["s"])]))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            return next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "unknown CPU")
    except OSError:
        return "unknown CPU"


# ----------------------------------------------------------- further legs
def _ms(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _rel_err(gpu, ora):
    """Max-norm relative error of X (whole n x r block) and of the
    contribution block (M, B, E, F), the larger of the two."""
    ex = np.max(np.abs(gpu["X"] - ora["X"])) / max(np.max(np.abs(ora["X"])), 1e-300)
    blk = lambda r: np.concatenate([np.ravel(r["M"]), np.ravel(r["B"]), np.ravel(r["E"]), [r["F"]]])  # noqa: E731
    eb = np.max(np.abs(blk(gpu) - blk(ora))) / max(np.max(np.abs(blk(ora))), 1e-300)
    return float(max(ex, eb))


CLASS_HI = (16, 25, 33, 48, 64)   # upper s of the library's size classes


def class_members(s_arr, s_cap, single):
    """Elements of the size class whose launch had upper bound s_cap (all of
    them when the batch is one class)."""
    if single:
        return np.ones(len(s_arr), dtype=bool)
    k = next(i for i, hi in enumerate(CLASS_HI) if s_cap <= hi)
    lo = CLASS_HI[k - 1] if k > 0 else 0
    return (s_arr > lo) & (s_arr <= s_cap)


def class_timing(torch, ctx, db, prec, out, reps):
    """Mean duration of each size class's main kernel in the fused run
    (HIP events the library records on the class's stream) and the dominant
    class's algorithmic flop rate against the MFMA peak of its precision."""
    from paper_1703_10435_amd import abi, engine
    ctx.set_option("class_timing", 1)
    acc = {}
    for k in range(reps + 1):
        engine.run_fused(ctx, db, prec, out)
        t = ctx.class_times()
        if k > 0:
            for cap, ms in t:
                acc.setdefault(cap, []).append(ms)
    ctx.set_option("class_timing", 0)
    single = len(acc) == 1
    per = {cap: float(np.mean(v)) for cap, v in acc.items()}
    dom = max(per, key=per.get)
    mask = class_members(db.s, dom, single)
    flops = float(np.sum(_flops_per_element(db.n[mask], db.r[mask])))
    peak = PEAK_FP32_TFLOPS if prec == abi.MHM_FP32_IR else PEAK_FP64_TFLOPS
    tf = flops / (per[dom] * 1e-3) / 1e12
    return {"class_kernel_ms": {str(c): v for c, v in per.items()}, "dominant_s_max": int(dom),
            "dominant_elements": int(mask.sum()), "dominant_kernel_ms": per[dom], "dominant_flops": flops,
            "dominant_tflops": tf, "dominant_frac_mfma_peak": tf / peak, "peak_tflops": peak}


def _assemble_bytes(db):
    """Algorithmic bytes of steps a2-a3 alone: kappa and f in; Ahat, Btilde,
    c and the area out."""
    n_, r_, s_ = db.n.astype(np.float64), db.r.astype(np.float64), db.s.astype(np.float64)
    return float(np.sum(16 * s_ ** 2 + 8 * n_ ** 2 + 8 * n_ * r_ + 8 * n_ + 8))


def _contrib_bytes(db):
    """Algorithmic bytes of step a6 alone: the face rows of X (3 s nodes, r
    columns) and f in; M, E, B, F out."""
    r_, s_ = db.r.astype(np.float64), db.s.astype(np.float64)
    ni = float(db.NImax)
    return float(np.sum(8 * 3 * s_ * r_ + 8 * s_ ** 2 + 8 * (ni * ni + 2 * ni + 1)))


def _batched_leg(torch, ctx, name, checks, sample_idx, reps=3):
    """FP32+IR and FP64 batched forms (autotuned, one HIP-graph launch each),
    the plain FP64 form (the three calls per size bucket, unfused, no graph),
    and each form's dominant kernel against the MFMA roofline."""
    from mhm_inputs import configs
    from paper_1703_10435_amd import abi, engine
    from paper_1703_10435_amd.batch import DeviceBatch
    b = configs.make(name)
    db = DeviceBatch(b)
    E = b["n_elem"]
    leg = {"n_elem": E, "s": sorted(int(x) for x in np.unique(b["s"]))}
    for prec, tag in ((abi.MHM_FP32_IR, "fp32_ir"), (abi.MHM_FP64, "fp64")):
        o = db.alloc_outputs(three_call=False)
        engine.autotune(ctx, db, prec, o)
        leg[f"{tag}_tuning"] = ctx.tune_report()
        g, go = engine.capture_fused(ctx, db, prec)
        ms = _ms(torch, g.launch, reps)
        g.close()
        info = go["info"].cpu().numpy()[:E]
        its = go["ir_iters"].cpu().numpy()[:E]
        leg[f"{tag}_graph_ms"] = ms
        leg[f"{tag}_graph_problems_per_s"] = E / (ms * 1e-3)
        tf = float(np.sum(_flops_per_element(db.n, db.r))) / (ms * 1e-3) / 1e12
        peak = PEAK_FP32_TFLOPS if prec == abi.MHM_FP32_IR else PEAK_FP64_TFLOPS
        leg[f"{tag}_graph_algorithmic_tflops"] = tf
        leg[f"{tag}_graph_frac_mfma_peak"] = tf / peak
        leg[f"{tag}_fallbacks"] = int(np.sum(info == -1))
        leg[f"{tag}_bad"] = int(np.sum((info != 0) & (info != -1)))
        leg[f"{tag}_refinement_steps_histogram"] = np.bincount(its).tolist()
        res = db.unpack(go)
        checks += [(name, f"{tag}_max_rel_err_sampled", b, int(e), BAR[tag], res[int(e)]) for e in sample_idx]
        leg[f"{tag}_fused_dominant_kernel"] = class_timing(torch, ctx, db, prec, o, reps)
    subs = [DeviceBatch(configs.sub_batch(b, np.flatnonzero(b["s"] == s))) for s in np.unique(b["s"])]
    outs = [d.alloc_outputs(three_call=True) for d in subs]
    ms3 = _ms(torch, lambda: engine.run_three_call_bucketed(ctx, subs, abi.MHM_FP64, outs), reps)
    leg["fp64_three_call_per_bucket_ms"] = ms3
    leg["fp64_three_call_problems_per_s"] = E / (ms3 * 1e-3)
    # steps a2-a3 (k_assemble) and a6 (k_contrib) alone on the three-call
    # buffers, bucket by bucket (assembly last: it rewrites Ahat)
    ms_c, by_c, ms_a, by_a = 0.0, 0.0, 0.0, 0.0
    for d, o in zip(subs, outs):
        ms_c += _ms(torch, lambda: ctx.skeleton_contrib(d, o["X"], o["M"], o["E"], o["B"], o["F"], o["info"]), reps)
        by_c += _contrib_bytes(d)
        ms_a += _ms(torch, lambda: ctx.local_assemble(d, o["Ahat"], o["Btil"], o["c"], o["area"], o["info"]), reps)
        by_a += _assemble_bytes(d)
    leg.update({"contrib_ms": ms_c, "contrib_GBps": by_c / (ms_c * 1e-3) / 1e9,
                "contrib_frac_hbm": by_c / (ms_c * 1e-3) / 8e12,
                "assemble_ms": ms_a, "assemble_GBps": by_a / (ms_a * 1e-3) / 1e9,
                "assemble_frac_hbm": by_a / (ms_a * 1e-3) / 8e12})
    leg["fp32_ir_graph_vs_plain_fp64_three_call"] = ms3 / leg["fp32_ir_graph_ms"]
    leg["fp32_ir_graph_vs_fp64_graph"] = leg["fp64_graph_ms"] / leg["fp32_ir_graph_ms"]
    leg["sample"] = f"{len(sample_idx)} elements against the FP64 oracle"
    del outs, subs, db
    torch.cuda.empty_cache()
    return leg


def _wide_leg(torch, ctx, checks, m=4, reps=3):
    """The C3 workload (s = 32, l = 3) with a richer multiplier space: m
    segments of degree l per face, N_I = 3 m (l + 1) face right-hand sides
    per factor (49 in all for m = 4, in four 16-column chunks) instead of
    C3's 13.  The factorisation is the same; the solves grow with r."""
    from mhm_inputs import configs
    from paper_1703_10435_amd import abi, engine
    from paper_1703_10435_amd.batch import DeviceBatch
    b = configs.make("C3")
    E = b["n_elem"]
    b["m"] = np.full(E, m, dtype=np.int32)
    db = DeviceBatch(b)
    s = int(b["s"][0])
    n, r = (s + 1) * (s + 2) // 2, int(db.r[0])
    idx = np.random.default_rng(10).choice(E, size=3, replace=False)
    leg = {"n_elem": E, "s": s, "l": int(b["l"][0]), "m": m, "n": n, "r": r}
    for prec, tag in ((abi.MHM_FP32_IR, "fp32_ir"), (abi.MHM_FP64, "fp64")):
        o = db.alloc_outputs(three_call=False)
        engine.autotune(ctx, db, prec, o)
        g, go = engine.capture_fused(ctx, db, prec)
        ms = _ms(torch, g.launch, reps)
        g.close()
        info = go["info"].cpu().numpy()[:E]
        leg[f"{tag}_graph_ms"] = ms
        leg[f"{tag}_graph_problems_per_s"] = E / (ms * 1e-3)
        leg[f"{tag}_rhs_columns_per_s"] = E * r / (ms * 1e-3)
        leg[f"{tag}_algorithmic_tflops"] = E * float(_flops_per_element(n, r)) / (ms * 1e-3) / 1e12
        leg[f"{tag}_fallbacks"] = int(np.sum(info == -1))
        leg[f"{tag}_bad"] = int(np.sum((info != 0) & (info != -1)))
        res = db.unpack(go)
        checks += [("W", f"{tag}_max_rel_err_sampled", b, int(e), BAR[tag], res[int(e)]) for e in idx]
        leg[f"{tag}_tuning"] = ctx.tune_report()
    leg["flops_per_element"] = "n^3/3 + 2 n^2 r"
    leg["sample"] = f"{len(idx)} elements against the FP64 oracle"
    del db
    torch.cuda.empty_cache()
    return leg


def _serve_leg(seconds, warmup, checks, rate=20000.0):
    """C5: an open-loop Poisson stream through the serving runtime, `warmup`
    seconds of arrivals and then `seconds` measured (latency and throughput
    over the requests that arrive after the warm-up)."""
    from mhm_inputs import configs
    from paper_1703_10435_amd import abi
    from paper_1703_10435_amd.serve import Server, content_key, run_open_loop
    n = int(rate * (seconds + warmup))
    st = configs.served_requests(n, rate=rate)
    keys = st["keys"]
    kk = [content_key(keys["vert"][e], int(keys["s"][e]), keys["kappa"][keys["tri_off"][e]:keys["tri_off"][e + 1]])
          for e in range(keys["n_elem"])]
    reqs = []
    for k in range(n):
        e = int(st["key_idx"][k])
        o0, o1 = keys["tri_off"][e], keys["tri_off"][e + 1]
        reqs.append(dict(s=int(keys["s"][e]), l=int(st["l"][k]), vert=keys["vert"][e], sigma=keys["sigma"][e],
                         flip=keys["flip"][e], kappa=keys["kappa"][o0:o1], f=keys["f"][o0:o1], key=kk[e]))
    window = np.flatnonzero(st["t"] >= warmup)
    sample = np.random.default_rng(11).choice(window, size=8, replace=False)
    srv = Server(prec=abi.MHM_FP32_IR, max_batch=1024, in_flight=4, s_max=48, l_max=3, reuse=True,
                 hbm_budget=64 << 30)
    try:
        out = run_open_loop(srv, reqs, st["t"], keep=sample, progress=lambda d, t: print(
            f"# C5 stream: {d} of {t} requests served", file=sys.stderr, flush=True))
        s = srv.stats()
    finally:
        srv.close()
    res = out["results"]
    lat = out["latency"][window]
    t_first = min(res[k]["t_arrival"] for k in window)
    t_last = max(res[k]["t_done"] for k in window)
    hits = sum(1 for k in window if res[k]["cache_hit"])
    fb = sum(1 for k in window if res[k]["info"] == -1)
    bad = sum(1 for k in window if res[k]["info"] not in (0, -1))
    for k in sample:
        checks.append(("C5", "max_rel_err_sampled", configs.request_batch(st, int(k)), 0, BAR["fp32_ir"], res[int(k)]))
    return {"requests_measured": int(window.size), "warmup_requests": int(n - window.size),
            "arrival_rate_per_s": rate, "seconds_measured": seconds, "seconds_warmup": warmup,
            "throughput_per_s": window.size / max(t_last - t_first, 1e-9),
            "p50_ms": float(np.median(lat) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "max_ms": float(np.max(lat) * 1e3), "cache_hit_rate": hits / window.size, "ir_fallbacks": fb,
            "bad_info": bad, "launches": s["launches"], "hbm_budget_gb": 64,
            "factor_arena_gb": s["arena_bytes"] / 2 ** 30, "cache_evictions": s["cache_evictions"],
            "errors": s["errors"], "sample": "8 measured requests against the FP64 oracle",
            "latency": "scheduled arrival to contribution on the host"}


def _transient_leg(torch, ctx, batch, db, steps, checks, n_loads=4):
    """Factor once, then time steps that reuse the stored factors with a new
    source each step (only the load vectors are built and solved)."""
    from paper_1703_10435_amd import abi, engine
    E = batch["n_elem"]
    rng = np.random.default_rng(5)
    loads = [batch["f"] * (1.0 + 0.25 * k) + 0.1 * rng.standard_normal(batch["f"].shape) for k in range(n_loads)]
    views = [engine.with_source(db, torch.as_tensor(f, device="cuda")) for f in loads]
    leg = {"n_elem": E, "loads": f"{n_loads} seeded sources used in turn"}
    for prec, tag in ((abi.MHM_FP64, "fp64"), (abi.MHM_FP32_IR, "fp32_ir")):
        fs = engine.FactorStore(db, prec)
        o = db.alloc_outputs(three_call=False)

        def first():
            fs.state.zero_()
            engine.run_cached(ctx, views[0], fs, o, update_state=False)
        leg[f"{tag}_factor_step_ms"] = _ms(torch, first, 3)
        engine.run_cached(ctx, views[0], fs, o)          # stores the factors, marks them valid
        torch.cuda.synchronize()
        leg[f"{tag}_factors_held"] = int(fs.state[:E].sum().item())
        k = [0]

        def later():
            k[0] = (k[0] + 1) % n_loads
            engine.run_cached(ctx, views[k[0]], fs, o, update_state=False)
        ms = _ms(torch, later, steps)
        leg[f"{tag}_reuse_step_ms"] = ms
        leg[f"{tag}_reuse_solves_per_s"] = E / (ms * 1e-3)
        leg[f"{tag}_factor_store_mb"] = fs.nbytes / 2 ** 20

        # source-only steps (coefficients constant in time): the source
        # column of X, E and F on the stored factors
        def src():
            k[0] = (k[0] + 1) % n_loads
            engine.source_step(ctx, views[k[0]], fs, o)
        ms_s = _ms(torch, src, steps)
        last = k[0]
        leg[f"{tag}_source_step_ms"] = ms_s
        leg[f"{tag}_source_steps_per_s"] = 1e3 / ms_s
        leg[f"{tag}_source_solves_per_s"] = E / (ms_s * 1e-3)
        leg[f"{tag}_source_step_vs_factoring"] = leg[f"{tag}_factor_step_ms"] / ms_s
        # algorithmic bytes: the factor once, f (and kappa for the FP64
        # residual of the refinement), the source column of X, E and F
        nbytes = (fs.nbytes + batch["f"].size * 8 * (2 if prec == abi.MHM_FP32_IR else 1)
                  + int(np.sum(db.n)) * 8 + E * (db.NImax + 1) * 8)
        leg[f"{tag}_source_step_GBps"] = nbytes / (ms_s * 1e-3) / 1e9
        leg[f"{tag}_source_step_frac_hbm"] = leg[f"{tag}_source_step_GBps"] / PEAK_HBM_GBS
        info = o["info"].cpu().numpy()[:E]
        leg[f"{tag}_bad"] = int(np.sum((info != 0) & (info != -1)))
        leg[f"{tag}_source_fallbacks"] = int(np.sum(info == -1))
        if prec == abi.MHM_FP32_IR:
            leg["fp32_ir_source_steps_mean"] = float(o["ir_iters"].cpu().numpy()[:E][info == 0].mean())
        res = db.unpack(o)
        bl = dict(batch, f=loads[last])
        for e in np.random.default_rng(13).choice(E, size=4, replace=False):
            checks.append(("T", f"{tag}_max_rel_err_sampled", bl, int(e), BAR[tag], res[int(e)]))
        leg[f"{tag}_speedup_vs_factoring"] = leg[f"{tag}_factor_step_ms"] / ms
        del fs, o
    leg["sample"] = "4 elements per precision against the FP64 oracle, for the last source-only step's source"
    leg["bytes"] = "source step: factor store once + f (+ kappa for FP32 refinement) + X source column + E, F"
    return leg


def _skeleton_leg(torch, ctx, batch, db, out, steps):
    """Scatter of the C2 blocks into the CSR skeleton system (eq. (6)) and the
    reconstruction of u (eq. (4)); HBM-bound, priced by algorithmic bytes."""
    import scipy.sparse as sp
    from paper_1703_10435_amd.skeleton import SkeletonSystem
    E = batch["n_elem"]
    l = int(batch["l"][0])
    sk = SkeletonSystem(batch["mesh"], l, p_max=db.p_max)
    NI, NImax = 3 * (l + 1), db.NImax
    vals = torch.zeros(sk.nnz, dtype=torch.float64, device="cuda")
    rhs = torch.zeros(sk.n_rows, dtype=torch.float64, device="cuda")
    missing = torch.zeros(1, dtype=torch.int32, device="cuda")

    def scatter():   # the library call alone (buffers allocated beforehand)
        ctx.skeleton_scatter(db, out["M"], out["E"], out["B"], out["F"], sk.gdof, sk.erow, sk.row_ptr,
                             sk.col_idx, sk.n_rows, vals, rhs, out["info"], missing)
    ms_s = _ms(torch, scatter, steps)
    vals.zero_()
    rhs.zero_()
    missing.zero_()
    scatter()
    sol = torch.as_tensor(np.random.default_rng(3).standard_normal(sk.n_rows), device="cuda")
    u = torch.zeros(db.node_total, dtype=torch.float64, device="cuda")
    ms_r = _ms(torch, lambda: ctx.reconstruct(db, out["X"], sk.gdof, sk.erow, sol, sk.n_rows, u, out["info"]),
               steps)
    torch.cuda.synchronize()
    b_scatter = (E * (NImax * NImax + 3 * NImax + 1) * 8 + E * (NImax + 2) * 4
                 + sk.nnz * (16 + 4) + (sk.n_rows + 1) * 4 + sk.n_rows * 16)
    b_recon = db.rhs_total * 8 + E * (NImax + 2) * 4 + sk.n_rows * 8 + db.node_total * 8
    # consistency of both with the same blocks, on the host
    res = db.unpack(out)
    x = np.random.default_rng(4).standard_normal(sk.n_rows)
    y = np.zeros(sk.n_rows)
    for e in range(E):
        g, t = sk.gdof_h[e, :NI], sk.erow_h[e]
        y[g] += res[e]["M"] @ x[g] + res[e]["B"] * x[t]
        y[t] += res[e]["B"] @ x[g]
    K = sp.csr_matrix((vals.cpu().numpy(), sk.col_idx_h, sk.row_ptr_h), shape=(sk.n_rows, sk.n_rows))
    err_s = float(np.abs(K @ x - y).max() / np.abs(y).max())
    uh = u.cpu().numpy()
    sh = sol.cpu().numpy()
    err_r = 0.0
    for e in range(0, E, 97):
        want = sh[sk.erow_h[e]] + res[e]["X"][:, :NI] @ sh[sk.gdof_h[e, :NI]] + res[e]["X"][:, NI]
        got = uh[db.node_off[e]:db.node_off[e + 1]]
        err_r = max(err_r, float(np.abs(got - want).max() / np.abs(want).max()))
    # the skeleton solve (MINRES on the device; it synchronises, so it is
    # timed by the host clock around the call)
    import time
    import scipy.sparse.linalg as spla
    xs = torch.empty(sk.n_rows, dtype=torch.float64, device="cuda")
    sk.solve(ctx, vals, rhs, xs, tol=1e-10)             # warm-up
    t0 = time.perf_counter()
    _, it_s, rr_s = sk.solve(ctx, vals, rhs, xs, tol=1e-10)
    ms_solve = (time.perf_counter() - t0) * 1e3
    xd = spla.spsolve(K.tocsc(), rhs.cpu().numpy())     # host sparse direct solve of the same system
    nl = sk.n_lambda
    err_solve = float(np.abs(xs.cpu().numpy()[nl:] - xd[nl:]).max() / np.abs(xd[nl:]).max())
    gbs = lambda b, ms: b / (ms * 1e-3) / 1e9  # noqa: E731
    return {"n_rows": sk.n_rows, "nnz": sk.nnz,
            "solve_ms": ms_solve, "solve_minres_steps": it_s, "solve_relres": rr_s,
            "solve_ms_per_step": ms_solve / max(it_s, 1),
            "solve_u0_rel_diff_vs_host_direct": err_solve,
            "scatter_ms": ms_s, "scatter_GBps": gbs(b_scatter, ms_s),
            "scatter_frac_hbm": gbs(b_scatter, ms_s) / PEAK_HBM_GBS, "scatter_bytes": b_scatter,
            "reconstruct_ms": ms_r, "reconstruct_GBps": gbs(b_recon, ms_r),
            "reconstruct_frac_hbm": gbs(b_recon, ms_r) / PEAK_HBM_GBS, "reconstruct_bytes": b_recon,
            "missing": int(missing.item()), "scatter_rel_err_vs_host_sum": err_s,
            "reconstruct_rel_err_vs_host": err_r,
            "bytes": "scatter: blocks, indices, CSR values and rhs read+written once, pattern read once; "
                     "reconstruct: X, indices, solution read once, u written once"}


def _c2_leg(torch, ctx, args, checks):
    """C2 (the plain FP64 batch of 2048 s = 16 elements): the fused FP64 run
    (register-resident tiles), the three calls, FP32 + refinement, the
    HBM-bound assembly and contribution kernels alone, and a host-to-host
    time.  Returns the leg and the C2 batch, its device copy and outputs
    (for the time-step and skeleton legs)."""
    from mhm_inputs import configs
    from paper_1703_10435_amd import abi, engine
    from paper_1703_10435_amd.batch import DeviceBatch
    batch = configs.make("C2")
    db = DeviceBatch(batch)
    E = db.n_elem
    out = db.alloc_outputs(three_call=True)
    ms = _ms(torch, lambda: engine.run_fused(ctx, db, abi.MHM_FP64, out), args.steps)
    leg = {"fp64_fused_ms": ms, "fp64_fused_problems_per_s": E / (ms * 1e-3)}
    leg["fp64_fused_dominant_kernel"] = class_timing(torch, ctx, db, abi.MHM_FP64, out, args.steps)
    res = db.unpack(out)
    for e in stratified(batch, 6, 21):
        checks.append(("C2", "fp64_max_rel_err_sampled", batch, int(e), BAR["fp64"], res[int(e)]))
    o3 = db.alloc_outputs(three_call=True)
    ms3 = _ms(torch, lambda: engine.run_three_call(ctx, db, abi.MHM_FP64, o3), args.steps)
    fp32 = db.alloc_outputs(three_call=False)
    ms32 = _ms(torch, lambda: engine.run_fused(ctx, db, abi.MHM_FP32_IR, fp32), args.steps)
    info = fp32["info"].cpu().numpy()[:E]
    leg.update({"fp64_three_call_ms": ms3, "fp32_ir_fused_ms": ms32,
                "fp32_ir_steps_mean": float(fp32["ir_iters"].cpu().numpy()[:E].mean()),
                "fp32_ir_fallbacks": int(np.sum(info == -1))})
    # the HBM-bound steps of the three-call form on their own
    ms_a = _ms(torch, lambda: ctx.local_assemble(db, o3["Ahat"], o3["Btil"], o3["c"], o3["area"], o3["info"]),
               args.steps)
    engine.run_three_call(ctx, db, abi.MHM_FP64, o3)
    ms_c = _ms(torch, lambda: ctx.skeleton_contrib(db, o3["X"], o3["M"], o3["E"], o3["B"], o3["F"], o3["info"]),
               args.steps)
    by_a = _assemble_bytes(db)
    by_c = _contrib_bytes(db)
    leg.update({"assemble_ms": ms_a, "assemble_GBps": by_a / (ms_a * 1e-3) / 1e9,
                "assemble_frac_hbm": by_a / (ms_a * 1e-3) / 8e12,
                "contrib_ms": ms_c, "contrib_GBps": by_c / (ms_c * 1e-3) / 1e9,
                "contrib_frac_hbm": by_c / (ms_c * 1e-3) / 8e12,
                "bytes": "assemble: 16 s^2 + 8 n^2 + 8 n r + 8 n + 8 per element; contrib: "
                         "8 (3 s r + s^2 + NImax^2 + 2 NImax + 1) per element"})
    del o3

    # host to host: the host batch validated, offset and uploaded, the fused
    # FP64 run, and X, M, E, B, F, info copied back (never `value`)
    def h2h():
        dbh = DeviceBatch(batch)
        oh = dbh.alloc_outputs(three_call=False)
        engine.run_fused(ctx, dbh, abi.MHM_FP64, oh)
        return [oh[k].cpu() for k in ("X", "M", "E", "B", "F", "info")]
    h2h()
    torch.cuda.synchronize()
    reps = max(3, min(args.steps, 10))
    t0 = time.perf_counter()
    for _ in range(reps):
        h2h()
    ms_h = (time.perf_counter() - t0) * 1e3 / reps
    leg.update({"host_to_host_ms": ms_h, "host_to_host_problems_per_s": E / (ms_h * 1e-3),
                "host_to_host": "host batch validated and uploaded, fused FP64 run, "
                                "X, M, E, B, F, info downloaded; wall clock"})
    engine.run_fused(ctx, db, abi.MHM_FP64, out)   # leave the FP64 results for the skeleton leg
    return leg, batch, db, out


def extra_legs(torch, ctx, args, checks):
    ex = {}
    legs = [x.strip().upper() for x in args.legs.split(",") if x.strip()]
    c2 = None
    if any(k in legs for k in ("C2", "T", "SKEL")):
        ex["C2"], *c2 = _c2_leg(torch, ctx, args, checks)
    if "C3" in legs:
        from mhm_inputs import configs
        b3 = configs.make("C3")
        to = b3["tri_off"]
        kmax = np.array([b3["kappa"][to[e]:to[e + 1]].max() for e in range(b3["n_elem"])])
        chan, back = np.flatnonzero(kmax > 1.0), np.flatnonzero(kmax == 1.0)
        rng = np.random.default_rng(3)
        sample = np.concatenate([[3452], rng.choice(chan, 7, replace=False), rng.choice(back, 2, replace=False)])
        ex["C3"] = _batched_leg(torch, ctx, "C3", checks, sample)
        ex["C3"]["sample"] += " (element 3452 and 7 more crossed by a K = 1e4 channel, 2 without)"
    if "C4" in legs:
        from mhm_inputs import configs
        ex["C4"] = _batched_leg(torch, ctx, "C4", checks, stratified(configs.make("C4"), 2, 9))
    if "C5" in legs:
        ex["C5"] = _serve_leg(args.serve_seconds, args.serve_warmup, checks)
    if "T" in legs:
        batch, db, out = c2
        ex["T"] = _transient_leg(torch, ctx, batch, db, args.steps, checks)
    if "SKEL" in legs:
        batch, db, out = c2
        ex["SKEL"] = _skeleton_leg(torch, ctx, batch, db, out, args.steps)
    if "W" in legs:
        ex["W"] = _wide_leg(torch, ctx, checks)
    return ex


# -------------------------------------------------------------------- timing
def time_launches(torch, fn, steps, warmup, after=None):
    """W untimed steps, then K steps, each bracketed by events on the current
    stream; `after` (if given) runs after each timed step (it may
    synchronise: the per-step events time the device work only)."""
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
        if after:
            after()
    t1.record(stream)
    torch.cuda.synchronize()
    per = np.array([a.elapsed_time(b) for a, b in evs])
    return t0.elapsed_time(t1), per


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-per-class", type=int, default=24,
                    help="oracle sample of the headline workload: elements per s (C4 has four values of s)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="the headline only (no further legs)")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="measured length of the C5 open-loop stream")
    ap.add_argument("--serve-warmup", type=float, default=1.0, help="warm-up arrivals before the measured C5 window")
    ap.add_argument("--legs", default="C2,C3,C4,C5,T,SKEL,W",
                    help="which extra legs to run (comma list): C2, C3, C4 (FP32+IR and FP64 graphs, plain FP64 "
                         "three calls), C5 (serving), T (time steps reusing factors), SKEL (skeleton scatter, "
                         "reconstruction, solve), W (C3 with m = 4 segments per face, 49 right-hand sides)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a 256 MiB device-to-device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 (the local problems are "
                                   "independent and would shard by element across GPUs)"}))
        sys.exit(2)

    import torch
    from mhm_inputs import configs
    from paper_1703_10435_amd import abi, engine
    from paper_1703_10435_amd.batch import DeviceBatch

    from paper_1703_10435_amd import build as _b
    _b.ensure()   # rebuilt only if missing or built from other sources
    if args.copy_calib:
        src = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    batch = configs.make("C4")
    db = DeviceBatch(batch)
    out = db.alloc_outputs(three_call=False)
    ctx = abi.Context(0, class_timing=1)
    E = batch["n_elem"]

    def step():
        engine.run_fused(ctx, db, abi.MHM_FP64, out)

    per_class = {}

    def after():
        for cap, ms in ctx.class_times():
            per_class.setdefault(cap, []).append(ms)

    total_ms, per = time_launches(torch, step, args.steps, args.warmup, after)
    ms_per_step = total_ms / args.steps
    info = out["info"].cpu().numpy()[:E]
    its = out["ir_iters"].cpu().numpy()[:E]
    res = db.unpack(out)
    ctx.set_option("class_timing", 0)

    # dominant kernel: the size class whose main launch takes longest (s = 48
    # on the left-looking FP64 kernel), its algorithmic flops per launch over
    # its mean event-timed duration
    cls_ms = {cap: float(np.mean(v)) for cap, v in per_class.items()}
    dom = max(cls_ms, key=cls_ms.get)
    mask = class_members(db.s, dom, len(cls_ms) == 1)
    flops = float(np.sum(_flops_per_element(db.n[mask], db.r[mask])))
    achieved = flops / (cls_ms[dom] * 1e-3) / 1e12
    line = {
        "metric": "local problems solved/sec at stated rel. error vs FP64 oracle",
        "value": E / (ms_per_step * 1e-3),
        "unit": "local problems/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOAD, "n_elem": E, "s": sorted(int(x) for x in np.unique(batch["s"])),
                   "l": [1, 2, 3], "precision": "plain FP64", "path": "fused mhm_local_batch_run (one launch per "
                   "size class, the classes one after another on one stream)"},
        "info_nonzero": int(np.sum(info != 0)),
        "refinement_steps_histogram": np.bincount(its).tolist(),
        "step_ms": {"mean": float(np.mean(per)), "p50": float(np.median(per)), "p99": float(np.percentile(per, 99))},
        "class_kernel_ms": {str(c): v for c, v in sorted(cls_ms.items())},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": measured_traffic(),
                     "kernel": f"k_local_ll<double> (FP64 left-looking), the s <= {dom} class "
                               f"({int(mask.sum())} elements, {cls_ms[dom]:.3f} ms per launch)",
                     "flops_per_launch": flops,
                     "flops_per_element": "n^3/3 + 2 n^2 r (Cholesky + forward/backward solves)"},
    }

    checks = []   # (leg, field, batch, element, bar, GPU result): compared with the oracle below
    if not args.no_extra:
        line["extra"] = extra_legs(torch, ctx, args, checks)

    if not args.no_cpu:
        # one worker process per core of the machine's CPU share for one GPU (16;
        # the affinity mask may show the whole host)
        affinity = len(os.sched_getaffinity(0))
        cores = min(affinity, 16)
        model = cpu_model()
        idx = stratified(batch, args.cpu_per_class, 1)
        cb = cpu_baseline(batch, idx, cores)
        errs = [_rel_err(res[e], o) for e, o in cb["results"].items()]
        others = {}
        for name, per_cls in (("C1", 32), ("C2", 48), ("C3", 24)):
            b = configs.make(name)
            sub = stratified(b, per_cls, 2) if name != "C3" else np.concatenate(
                [np.random.default_rng(2).choice(b["n_elem"], per_cls, replace=False)])
            cbo = cpu_baseline(b, sub, cores)
            others[name] = {"value": cbo["rate"], "single_core": cbo["single_core_rate"],
                            "sample": f"{len(sub)} of {b['n_elem']} elements (seeded)"}
        line["cpu_baseline"] = {
            "value": cb["rate"], "unit": "local problems/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(idx)} of the {E} C4 elements ({args.cpu_per_class} per s, seeded; the batch has 2048 "
                      f"of each s, so the sample's rate is the batch's), one element per task on {cores} worker "
                      f"processes (the GPU box's CPU share for one GPU; affinity mask {affinity} CPUs), "
                      f"{cb['cpu_seconds']:.1f} CPU-s in {cb['wall']:.1f} s wall; {model}",
            "single_core": cb["single_core_rate"], "other_configs": others}
        line["max_rel_err"] = float(np.max(errs))
        line["rel_err_p99"] = float(np.percentile(errs, 99))
        line["error_check"] = ("pass" if line["max_rel_err"] <= BAR["fp64"] and line["info_nonzero"] == 0
                               else "FAIL")
        line["error_check_sample"] = f"the {len(idx)} oracle-timed elements, stratified by s, at 1e-10"
        verdict = {}
        for leg, field, b, e, bar, g in checks:
            err = _rel_err(g, oracle_solve(b, e))
            d = line["extra"][leg]
            d[field] = max(d.get(field) or 0.0, err)
            verdict[leg] = verdict.get(leg, True) and err <= bar
        for leg, ok in verdict.items():
            line["extra"][leg]["error_check"] = "pass" if ok else "FAIL"
            line["extra"][leg]["tolerance"] = "1e-10 (FP64 forms) / 1e-8 (FP32 + refinement) per element"
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
