"""Coarse mesh, face table and lattice conventions (the splitProblem step, Algorithm 1, Section 3).

This module builds inputs only.  It contains none of the local-problem
arithmetic (no stiffness, no load vectors, no solves); both the HIP path and
the oracle read what it produces.

Conventions
-----------
* Coarse mesh of the unit square (Section 2, "mesh" T_H): an N x N grid of
  squares, vertex id ``j*(N+1)+i`` at ``(i/N, j/N)``.  Square (i, j) is split
  into ``T0 = (SW, SE, NE)`` and ``T1 = (SW, NE, NW)``, both counter-clockwise,
  with element ids ``2*(j*N+i) + 0/1``.
* Face ``e`` of an element is the edge opposite its vertex ``e``; it runs in
  the element's local direction ``v[e+1] -> v[e+2]`` (indices mod 3).
* Global faces are the unique vertex pairs, numbered in lexicographic order of
  ``(min id, max id)``.
* Sign of a face seen from an element (the factor n . n^K_F, Section 2):
  +1 for a boundary face (the face normal points outward on the boundary) and
  for the lower-indexed of the two neighbours, -1 for the other neighbour.
* ``flip[t, e] = 1`` when the element's local direction along face e runs
  from the higher to the lower global vertex id.  Face polynomials use the
  global orientation t = -1 at the lower vertex id, so both neighbours see the
  same polynomial.
* Sub-mesh of an element (uniform refinement with s subdivisions): lattice
  node (i, j), i, j >= 0, i + j <= s, sits at ``v0 + (i/s)(v1-v0) + (j/s)(v2-v0)``
  with index ``j*(s+1) - j*(j-1)/2 + i``.  Sub-triangles come in row strips
  j = 0..s-1: the up triangle (i, j) with nodes (i,j),(i+1,j),(i,j+1) has index
  ``j*(2s-j) + 2i``; the down triangle (i, j) with nodes
  (i+1,j+1),(i,j+1),(i+1,j) has index ``j*(2s-j) + 2i + 1``.
"""
from __future__ import annotations

import numpy as np


def coarse_mesh(N: int) -> dict:
    """Return the coarse triangulation of (0,1)^2 with 2*N*N elements.

    Keys: ``verts`` (V,2) float64, ``elems`` (Nt,3) int64 vertex ids (CCW),
    ``faces`` (Ne,2) int64 sorted vertex ids, ``elem_face`` (Nt,3),
    ``sigma`` (Nt,3) int8, ``flip`` (Nt,3) int8, ``face_boundary`` (Ne,) bool,
    ``face_len`` (Ne,) float64, ``face_elems`` (Ne,2) int64 (-1 if none).
    """
    if N < 1:
        raise ValueError("N must be >= 1")
    ii, jj = np.meshgrid(np.arange(N + 1), np.arange(N + 1), indexing="xy")
    verts = np.stack([ii.ravel() / N, jj.ravel() / N], axis=1).astype(np.float64)

    def vid(i, j):
        return j * (N + 1) + i

    elems = np.empty((2 * N * N, 3), dtype=np.int64)
    for j in range(N):
        for i in range(N):
            sw, se, ne, nw = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            t = 2 * (j * N + i)
            elems[t] = (sw, se, ne)
            elems[t + 1] = (sw, ne, nw)

    nt = elems.shape[0]
    pairs = {}
    for t in range(nt):
        for e in range(3):
            a, b = elems[t, (e + 1) % 3], elems[t, (e + 2) % 3]
            key = (min(a, b), max(a, b))
            pairs.setdefault(key, []).append((t, e))
    keys = sorted(pairs)
    face_index = {k: n for n, k in enumerate(keys)}
    faces = np.array(keys, dtype=np.int64)
    ne = len(keys)
    elem_face = np.empty((nt, 3), dtype=np.int64)
    sigma = np.empty((nt, 3), dtype=np.int8)
    flip = np.empty((nt, 3), dtype=np.int8)
    face_elems = -np.ones((ne, 2), dtype=np.int64)
    face_boundary = np.zeros(ne, dtype=bool)
    for k, owners in pairs.items():
        g = face_index[k]
        owners = sorted(owners)
        if len(owners) == 1:
            face_boundary[g] = True
        for slot, (t, e) in enumerate(owners):
            face_elems[g, slot] = t
            elem_face[t, e] = g
            sigma[t, e] = 1 if slot == 0 else -1
            a, b = elems[t, (e + 1) % 3], elems[t, (e + 2) % 3]
            flip[t, e] = 1 if a > b else 0
    face_len = np.linalg.norm(verts[faces[:, 1]] - verts[faces[:, 0]], axis=1)
    return dict(N=N, verts=verts, elems=elems, faces=faces, elem_face=elem_face,
                sigma=sigma, flip=flip, face_boundary=face_boundary,
                face_len=face_len, face_elems=face_elems)


def element_vertices(mesh: dict) -> np.ndarray:
    """(Nt, 6) float64: x0 y0 x1 y1 x2 y2 per element."""
    return mesh["verts"][mesh["elems"]].reshape(-1, 6).copy()


def n_nodes(s: int) -> int:
    return (s + 1) * (s + 2) // 2


def subtri_lattice_centroids(s: int) -> np.ndarray:
    """(s*s, 2) lattice coordinates (a, b) of sub-triangle centroids, in the
    row-strip order described in the module docstring; the physical point is
    ``v0 + (a/s)(v1-v0) + (b/s)(v2-v0)``."""
    out = np.empty((s * s, 2), dtype=np.float64)
    for j in range(s):
        base = j * (2 * s - j)
        for i in range(s - j):
            out[base + 2 * i] = (i + 1.0 / 3.0, j + 1.0 / 3.0)
            if i < s - j - 1:
                out[base + 2 * i + 1] = (i + 2.0 / 3.0, j + 2.0 / 3.0)
    return out


def subtri_centroids(vert6: np.ndarray, s: int) -> np.ndarray:
    """Physical centroids (s*s, 2) of the sub-triangles of one element."""
    v0 = vert6[0:2]
    v1 = vert6[2:4]
    v2 = vert6[4:6]
    ab = subtri_lattice_centroids(s) / s
    return v0[None, :] + ab[:, :1] * (v1 - v0)[None, :] + ab[:, 1:] * (v2 - v0)[None, :]
