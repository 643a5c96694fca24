"""Seeded synthetic workloads: ragged batches of MHM local problems.

A batch is a plain dict of numpy arrays (one row per coarse element, the
p_t = (K_t, {F_t}) of Algorithm 1):

``s``, ``l`` int32 (E,)       subdivisions and face-polynomial degree
``vert`` float64 (E, 6)       x0 y0 x1 y1 x2 y2, counter-clockwise
``sigma``, ``flip`` int8 (E,3) face sign and orientation flags
``kappa``, ``f`` float64 (sum s^2,)  per sub-triangle, concatenated
``tri_off`` int64 (E+1,)      prefix sums of s^2
``elem_id`` int64 (E,)        global coarse element id in ``mesh``
``mesh``                      the coarse mesh dict (for the skeleton solve)

Workloads (the MHM Darcy local problems of Section 4.2, eqs. (8)-(9)):

* C1: 4x4x2 = 32 elements, s = 4, l = 1, K = 1, f = 1.
* C2: 32x32x2 = 2048 elements, s = 16, l = 2, K = exp(2 g) with g a unit
  Gaussian field of correlation length 0.05 (seed 2000),
  f = 2 pi^2 sin(pi x) sin(pi y).
* C3: 64x64x2 = 8192 elements, s = 32, l = 3, K = 1 with 10 channels of
  width 0.01 and K = 1e4 (seed 3000), f = 1.
* C4: 64x64x2 = 8192 elements, s in {8,16,32,48} by quartile of each
  element's variance of log K (sampled at its 64 s=8 centroids),
  l ~ U{1,2,3} (seed 4001), K = exp(3 g) (seed 4000), f manufactured.
* C5: a stream of single-element requests (see ``request_stream``).
"""
from __future__ import annotations

import numpy as np

from .fields import ChannelField, GaussianField, manufactured_source
from .mesh import coarse_mesh, element_vertices, subtri_lattice_centroids


def _centroids_grouped(vert: np.ndarray, s_arr: np.ndarray):
    """Yield (element indices, centroids (E_s, s*s, 2)) per distinct s."""
    for s in np.unique(s_arr):
        idx = np.nonzero(s_arr == s)[0]
        ab = subtri_lattice_centroids(int(s)) / float(s)
        v0 = vert[idx, 0:2][:, None, :]
        v1 = vert[idx, 2:4][:, None, :]
        v2 = vert[idx, 4:6][:, None, :]
        pts = v0 + ab[None, :, :1] * (v1 - v0) + ab[None, :, 1:] * (v2 - v0)
        yield idx, pts


def build_batch(mesh: dict, elem_ids, s_arr, l_arr, kappa_fn, f_fn, name: str = "", m_arr=None) -> dict:
    elem_ids = np.asarray(elem_ids, dtype=np.int64)
    E = elem_ids.size
    s_arr = np.asarray(s_arr, dtype=np.int32).reshape(E)
    l_arr = np.asarray(l_arr, dtype=np.int32).reshape(E)
    vert_all = element_vertices(mesh)
    vert = vert_all[elem_ids] if E else np.zeros((0, 6))
    tri_off = np.zeros(E + 1, dtype=np.int64)
    np.cumsum(s_arr.astype(np.int64) ** 2, out=tri_off[1:])
    kappa = np.empty(int(tri_off[-1]), dtype=np.float64)
    f = np.empty(int(tri_off[-1]), dtype=np.float64)
    for idx, pts in _centroids_grouped(vert, s_arr):
        kv = np.broadcast_to(kappa_fn(pts), pts.shape[:2])
        fv = np.broadcast_to(f_fn(pts), pts.shape[:2])
        T = pts.shape[1]
        for row, e in enumerate(idx):
            o = tri_off[e]
            kappa[o:o + T] = kv[row]
            f[o:o + T] = fv[row]
    return dict(
        name=name,
        n_elem=E,
        s=s_arr,
        l=l_arr,
        vert=np.ascontiguousarray(vert, dtype=np.float64),
        sigma=np.ascontiguousarray(mesh["sigma"][elem_ids], dtype=np.int8),
        flip=np.ascontiguousarray(mesh["flip"][elem_ids], dtype=np.int8),
        kappa=kappa,
        f=f,
        tri_off=tri_off,
        elem_id=elem_ids,
        mesh=mesh,
        m=None if m_arr is None else np.asarray(m_arr, dtype=np.int32).reshape(E),
    )


def _one(pts):
    return np.ones(pts.shape[:-1])


def config_c1() -> dict:
    mesh = coarse_mesh(4)
    E = mesh["elems"].shape[0]
    return build_batch(mesh, np.arange(E), np.full(E, 4), np.full(E, 1), _one, _one, "C1")


def config_c2(n_elem: int | None = None) -> dict:
    mesh = coarse_mesh(32)
    g = GaussianField(seed=2000, ell=0.05)
    E = mesh["elems"].shape[0] if n_elem is None else n_elem
    return build_batch(mesh, np.arange(E), np.full(E, 16), np.full(E, 2),
                       lambda p: np.exp(2.0 * g(p)), manufactured_source, "C2")


def config_c3(n_elem: int | None = None) -> dict:
    mesh = coarse_mesh(64)
    ch = ChannelField(seed=3000)
    E = mesh["elems"].shape[0] if n_elem is None else n_elem
    return build_batch(mesh, np.arange(E), np.full(E, 32), np.full(E, 3), ch, _one, "C3")


C4_SIZES = (8, 16, 32, 48)


def config_c4(n_elem: int | None = None) -> dict:
    mesh = coarse_mesh(64)
    g = GaussianField(seed=4000, ell=0.05)
    E_all = mesh["elems"].shape[0]
    vert = element_vertices(mesh)
    # per-element variance of log K over its 64 s=8 centroids
    _, pts8 = next(_centroids_grouped(vert, np.full(E_all, 8)))
    var = np.var(3.0 * g(pts8), axis=1)
    q = np.quantile(var, [0.25, 0.5, 0.75])
    s_all = np.asarray(C4_SIZES)[np.searchsorted(q, var, side="right")]
    l_all = np.random.default_rng(4001).integers(1, 4, size=E_all)
    E = E_all if n_elem is None else n_elem
    ids = np.arange(E)
    return build_batch(mesh, ids, s_all[ids], l_all[ids],
                       lambda p: np.exp(3.0 * g(p)), manufactured_source, "C4")


def sub_batch(batch: dict, idx) -> dict:
    """Elements ``idx`` of a batch, as a batch of their own."""
    idx = np.asarray(idx, dtype=np.int64)
    s = batch["s"][idx]
    tri_off = np.zeros(idx.size + 1, dtype=np.int64)
    np.cumsum(s.astype(np.int64) ** 2, out=tri_off[1:])
    kap = np.empty(int(tri_off[-1]))
    ff = np.empty(int(tri_off[-1]))
    src = batch["tri_off"]
    for k, e in enumerate(idx):
        kap[tri_off[k]:tri_off[k + 1]] = batch["kappa"][src[e]:src[e + 1]]
        ff[tri_off[k]:tri_off[k + 1]] = batch["f"][src[e]:src[e + 1]]
    return dict(name=batch["name"], n_elem=int(idx.size), s=s.copy(), l=batch["l"][idx].copy(),
                vert=batch["vert"][idx].copy(), sigma=batch["sigma"][idx].copy(),
                flip=batch["flip"][idx].copy(), kappa=kap, f=ff, tri_off=tri_off,
                elem_id=batch["elem_id"][idx].copy(), mesh=batch["mesh"],
                m=None if batch.get("m") is None else np.asarray(batch["m"])[idx].copy())


def make(name: str, n_elem: int | None = None) -> dict:
    name = name.upper()
    if name == "C1":
        b = config_c1()
        return b if n_elem is None else sub_batch(b, np.arange(n_elem))
    return {"C2": config_c2, "C3": config_c3, "C4": config_c4}[name](n_elem)


# ---------------------------------------------------------------- C5 stream
C5_SIZES = (16, 24, 32, 48)


def request_stream(n_req: int, rate: float = 20000.0, reuse_p: float = 0.5):
    """Open-loop Poisson arrivals of single-element local problems.

    Returns a list of dicts ``{t_arrival, key, elem, s, l}`` and the field
    sampler; a request with probability ``reuse_p`` repeats the (element, s)
    key of an earlier request (its K is then identical) with a fresh l.
    """
    mesh = coarse_mesh(64)
    E_all = mesh["elems"].shape[0]
    r_sl = np.random.default_rng(5001)
    r_arr = np.random.default_rng(5002)
    r_re = np.random.default_rng(5003)
    t = np.cumsum(r_arr.exponential(1.0 / rate, size=n_req))
    out = []
    keys = []
    for k in range(n_req):
        l = int(r_sl.integers(1, 4))
        if keys and r_re.random() < reuse_p:
            elem, s = keys[int(r_re.integers(0, len(keys)))]
        else:
            elem = int(r_sl.integers(0, E_all))
            s = int(C5_SIZES[int(r_sl.integers(0, 4))])
            keys.append((elem, s))
        out.append(dict(t_arrival=float(t[k]), elem=elem, s=s, l=l))
    return mesh, out


def c5_field():
    return GaussianField(seed=5000, ell=0.05)


def served_requests(n_req: int, rate: float = 20000.0, reuse_p: float = 0.5) -> dict:
    """The C5 stream with its element data: ``keys`` is a batch holding each
    distinct (element, s) once (K = exp(2 g), g the seeded unit Gaussian
    field of correlation length 0.05; f manufactured), and per request
    ``key_idx``, ``l`` and the arrival time ``t`` (seconds from 0)."""
    mesh, reqs = request_stream(n_req, rate, reuse_p)
    uniq = {}
    key_idx = np.empty(n_req, dtype=np.int64)
    for k, q in enumerate(reqs):
        key_idx[k] = uniq.setdefault((q["elem"], q["s"]), len(uniq))
    pairs = sorted(uniq.items(), key=lambda kv: kv[1])
    elems = np.array([p[0][0] for p in pairs], dtype=np.int64)
    s_arr = np.array([p[0][1] for p in pairs], dtype=np.int32)
    g = c5_field()
    keys = build_batch(mesh, elems, s_arr, np.full(elems.size, 3), lambda p: np.exp(2.0 * g(p)),
                       manufactured_source, "C5-keys")
    return dict(keys=keys, key_idx=key_idx, l=np.array([q["l"] for q in reqs], dtype=np.int32),
                t=np.array([q["t_arrival"] for q in reqs]))


def request_batch(stream: dict, k: int) -> dict:
    """Request k of a served stream as a one-element batch (for the oracle)."""
    b = sub_batch(stream["keys"], [int(stream["key_idx"][k])])
    b["l"] = np.array([stream["l"][k]], dtype=np.int32)
    return b
