"""Seeded synthetic coefficient and source fields.

The paper's model problem is itself synthetic (a manufactured Darcy problem on
the unit cube, Section 5); these fields stand in for the heterogeneous
coefficients the MHM method targets (Section 1, "highly heterogeneous
problems").  Nothing here is part of the local-problem arithmetic.

Seeds follow ``1000*config + purpose`` (purpose 0: field, 1: s/l draws,
2: arrivals, 3: reuse) with numpy's PCG64 ``default_rng``.
"""
from __future__ import annotations

import numpy as np


class GaussianField:
    """Stationary Gaussian random field on (0,1)^2 with unit variance and
    squared-exponential covariance ``exp(-|r|^2 / (2 ell^2))``.

    Spectral synthesis on a periodic ``M x M`` grid over [0, period)^2 (the
    period 2 keeps the unit square away from the wrap-around), sampled with
    bilinear interpolation.
    """

    def __init__(self, seed: int, ell: float = 0.05, M: int = 2048, period: float = 2.0):
        rng = np.random.default_rng(seed)
        k1 = 2.0 * np.pi * np.fft.fftfreq(M, d=period / M)
        kx, ky = np.meshgrid(k1, k1, indexing="ij")
        # continuous 2D spectral density of the covariance, times the lattice
        # cell of the dual grid (2 pi / period)^2 / (2 pi)^2
        dens = 2.0 * np.pi * ell * ell * np.exp(-0.5 * ell * ell * (kx * kx + ky * ky))
        amp = np.sqrt(dens / (period * period))
        xi = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
        z = np.fft.ifft2(amp * xi) * (M * M)
        self.grid = np.ascontiguousarray(z.real)
        self.M = M
        self.h = period / M

    def __call__(self, pts: np.ndarray) -> np.ndarray:
        x = pts[..., 0] / self.h
        y = pts[..., 1] / self.h
        i0 = np.floor(x).astype(np.int64)
        j0 = np.floor(y).astype(np.int64)
        fx = x - i0
        fy = y - j0
        M = self.M
        i0 %= M
        j0 %= M
        i1 = (i0 + 1) % M
        j1 = (j0 + 1) % M
        g = self.grid
        return ((1 - fx) * (1 - fy) * g[i0, j0] + fx * (1 - fy) * g[i1, j0]
                + (1 - fx) * fy * g[i0, j1] + fx * fy * g[i1, j1])


class ChannelField:
    """Background 1 with ``n`` horizontal channels ``|y - y_k| < width/2`` of
    value ``k_hi``; channel centres ``y_k ~ U(0, 1)``."""

    def __init__(self, seed: int, n: int = 10, width: float = 0.01, k_hi: float = 1.0e4):
        rng = np.random.default_rng(seed)
        self.yk = np.sort(rng.uniform(0.0, 1.0, size=n))
        self.half = 0.5 * width
        self.k_hi = k_hi

    def __call__(self, pts: np.ndarray) -> np.ndarray:
        y = pts[..., 1]
        inside = np.zeros(y.shape, dtype=bool)
        for yk in self.yk:
            inside |= np.abs(y - yk) < self.half
        return np.where(inside, self.k_hi, 1.0)


def manufactured_source(pts: np.ndarray) -> np.ndarray:
    """f = 2 pi^2 sin(pi x) sin(pi y), the source of u = sin(pi x) sin(pi y)
    for -div(grad u) = f (the 2D analogue of the paper's Section 5 problem)."""
    x = pts[..., 0]
    y = pts[..., 1]
    return 2.0 * np.pi * np.pi * np.sin(np.pi * x) * np.sin(np.pi * y)


def manufactured_solution(pts: np.ndarray) -> np.ndarray:
    return np.sin(np.pi * pts[..., 0]) * np.sin(np.pi * pts[..., 1])
