"""GPU tests of the serving runtime: open-loop request streams of uneven
single-element local problems, continuous batching, factor reuse and
admission under a small HBM budget, each result checked against the FP64
oracle, and a request giving the same result alone and in the mix."""
from __future__ import annotations

import numpy as np
import pytest

from mhm_inputs import configs
from oracle import local
from tests.parity_util import ensure_built, rel_errors, say
from tests.test_parity_gpu import TOL

pytestmark = pytest.mark.gpu


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ensure_built()


@pytest.fixture(scope="module")
def stream():
    return configs.served_requests(64, rate=4000.0, reuse_p=0.5)


def _requests(st, idx):
    from paper_1703_10435_amd.serve import content_key
    keys = st["keys"]
    out = []
    for k in idx:
        e = int(st["key_idx"][k])
        o0, o1 = keys["tri_off"][e], keys["tri_off"][e + 1]
        kap = keys["kappa"][o0:o1]
        out.append(dict(s=int(keys["s"][e]), l=int(st["l"][k]), vert=keys["vert"][e], sigma=keys["sigma"][e],
                        flip=keys["flip"][e], kappa=kap, f=keys["f"][o0:o1],
                        key=content_key(keys["vert"][e], int(keys["s"][e]), kap)))
    return out


def _check_result(res, st, k, prec, label):
    b = configs.request_batch(st, k)
    ora = local.solve_element(b, 0)
    assert res["info"] in (0, -1), (label, k, res["info"])
    ex, eb = rel_errors(res, ora)
    assert ex <= TOL[prec] and eb <= TOL[prec], (label, k, ex, eb)
    return ex, eb


@pytest.mark.parametrize("prec", [1, 0])
def test_served_stream_matches_oracle(stream, prec):
    from paper_1703_10435_amd.serve import Server, run_open_loop
    _need_gpu()
    n = 48
    srv = Server(prec=prec, max_batch=16, in_flight=3, s_max=48, l_max=3, reuse=True, hbm_budget=16 << 30)
    try:
        say(f"[gpu] served stream n={n} prec={prec}")
        out = run_open_loop(srv, _requests(stream, range(n)), stream["t"][:n], copy_arrays=True)
        stats = srv.stats()
    finally:
        srv.close()
    say(f"  stats {stats}")
    assert stats["completed"] == n and stats["errors"] == 0
    assert stats["cache_hits"] > 0, "the stream repeats keys; some factors must be reused"
    assert stats["launches"] < n, "requests should share launches"
    worst = 0.0
    for k, r in enumerate(out["results"]):
        worst = max(worst, max(_check_result(r, stream, k, prec, f"served prec={prec}")))
    say(f"  served prec={prec}: worst rel err {worst:.2e}, p50 {np.median(out['latency'])*1e3:.2f} ms")


@pytest.mark.parametrize("reuse", [False, True])
def test_result_alone_and_in_the_mix(stream, reuse):
    """One request served alone, then again inside a burst of uneven
    requests: bit for bit the same without factor reuse (same kernels, same
    arithmetic), within the tolerance with its factor taken from the cache."""
    from paper_1703_10435_amd.serve import Server, run_open_loop
    _need_gpu()
    prec = 1
    target = 7
    srv = Server(prec=prec, max_batch=32, in_flight=2, s_max=48, l_max=3, reuse=reuse, hbm_budget=16 << 30)
    try:
        say(f"[gpu] alone reuse={reuse}")
        alone = run_open_loop(srv, _requests(stream, [target]), [0.0], copy_arrays=True)["results"][0]
        mix_idx = list(range(20, 40))
        mix_idx.insert(9, target)
        say(f"[gpu] in the mix reuse={reuse}")
        mixed = run_open_loop(srv, _requests(stream, mix_idx), np.zeros(len(mix_idx)), copy_arrays=True)
        m = mixed["results"][9]
        stats = srv.stats()
    finally:
        srv.close()
    assert stats["max_batch_seen"] > 1, "the burst should have been batched"
    if reuse:
        assert m["cache_hit"]
        ex, eb = rel_errors(m, alone)
        assert ex <= TOL[prec] and eb <= TOL[prec], (ex, eb)
    else:
        np.testing.assert_array_equal(m["X"], alone["X"])
        np.testing.assert_array_equal(m["M"], alone["M"])
        np.testing.assert_array_equal(m["E"], alone["E"])
    _check_result(alone, stream, target, prec, "alone")
    _check_result(m, stream, target, prec, "mix")


def test_admission_under_a_small_factor_budget(stream):
    """Room for a handful of factors only: requests wait for memory, factors
    are evicted and re-made, every result stays correct."""
    from paper_1703_10435_amd import abi
    from paper_1703_10435_amd.serve import Server, run_open_loop
    _need_gpu()
    prec = 1
    cap = 3 * abi.factor_bytes(48, prec)
    n = 40
    srv = Server(prec=prec, max_batch=8, in_flight=2, s_max=48, l_max=3, reuse=True, hbm_budget=16 << 30,
                 factor_cache_max=cap)
    try:
        say(f"[gpu] small budget cap={cap}")
        out = run_open_loop(srv, _requests(stream, range(n)), np.zeros(n), copy_arrays=True)
        stats = srv.stats()
    finally:
        srv.close()
    say(f"  stats {stats}")
    assert stats["completed"] == n and stats["errors"] == 0
    assert stats["arena_bytes"] == cap
    assert stats["cache_evictions"] > 0
    for k in range(0, n, 4):
        _check_result(out["results"][k], stream, k, prec, "small budget")
