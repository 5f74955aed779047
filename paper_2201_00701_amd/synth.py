"""Seeded synthetic inputs (points, landmarks, 2-D landmark grids).

This module only draws random numbers and shapes arrays; it holds none of the
projection's arithmetic.  Both the GPU tests and the CPU oracle consume the
float32 arrays produced here.  Everything is drawn in float64 from
``numpy.random.Generator(PCG64(seed))`` and cast to float32 once.

The workloads stand in for the paper's cytometry data (a 39-dimensional,
841,644-cell bone-marrow sample and "more than 50 features, millions of
cells"), which is not available here: cytometry-shaped Gaussian mixtures with
a uniform background, landmarks sampled from the data, and a regular 2-D
landmark grid (a SOM-style topology).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

CHUNK = 1 << 20


def _streams(seed: int, n: int = 4):
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(n)]


def mixture(n: int, d: int, n_clusters: int, seed: int, *, sd_range=(0.3, 2.0),
            isotropic: bool = False, background: float = 0.05, bg_box: float = 8.0,
            mean_box: float = 5.0, lognormal_weights: bool = False,
            out: np.ndarray | None = None) -> np.ndarray:
    """Gaussian mixture with an optional uniform background, float32 n x d.

    Cluster means ~ U[-mean_box, mean_box]^d; per-cluster standard deviations
    ~ U[sd_range] (one per cluster if ``isotropic``, else one per dimension);
    cluster weights equal, or proportional to exp(N(0,1)) if
    ``lognormal_weights``.  A fraction ``background`` of the rows (drawn per
    row) is uniform on [-bg_box, bg_box]^d.  Rows are produced in fixed chunks
    of 2^20 so the result does not depend on available memory.
    """
    rp, rx = _streams(seed, 2)
    means = rp.uniform(-mean_box, mean_box, (n_clusters, d))
    if isotropic:
        sds = np.repeat(rp.uniform(sd_range[0], sd_range[1], (n_clusters, 1)), d, axis=1)
    else:
        sds = rp.uniform(sd_range[0], sd_range[1], (n_clusters, d))
    w = np.exp(rp.normal(0.0, 1.0, n_clusters)) if lognormal_weights else np.ones(n_clusters)
    p = np.concatenate([(1.0 - background) * w / w.sum(), [background]])
    p /= p.sum()
    X = np.empty((n, d), np.float32) if out is None else out
    for s in range(0, n, CHUNK):
        m = min(CHUNK, n - s)
        lab = rx.choice(n_clusters + 1, size=m, p=p)
        z = rx.standard_normal((m, d))
        bg = lab == n_clusters
        cl = np.where(bg, 0, lab)
        rows = means[cl] + sds[cl] * z
        nb = int(bg.sum())
        if nb:
            rows[bg] = rx.uniform(-bg_box, bg_box, (nb, d))
        X[s:s + m] = rows.astype(np.float32)
    return X


def landmarks_from_data(X: np.ndarray, g: int, seed: int, noise: float = 0.1) -> np.ndarray:
    """g distinct random rows of X plus N(0, noise^2) per coordinate, float32 g x d."""
    rc, rn = _streams(seed + 7919, 2)
    idx = np.sort(rc.choice(X.shape[0], size=g, replace=False))
    L = X[idx].astype(np.float64) + rn.normal(0.0, noise, (g, X.shape[1]))
    return L.astype(np.float32)


def grid2d(g: int, cols: int | None = None, spacing: float = 1.0) -> np.ndarray:
    """Row-major 2-D grid positions l_j = (j mod cols, j div cols) * spacing."""
    if cols is None:
        cols = int(math.ceil(math.sqrt(g)))
    j = np.arange(g)
    return (np.stack([j % cols, j // cols], axis=1) * spacing).astype(np.float32)


def uniform_points(n: int, d: int, seed: int) -> np.ndarray:
    """All coordinates from one U[0,1) distribution (the paper's benchmark data shape)."""
    (r,) = _streams(seed, 1)
    X = np.empty((n, d), np.float32)
    for s in range(0, n, CHUNK):
        m = min(CHUNK, n - s)
        X[s:s + m] = r.random((m, d)).astype(np.float32)
    return X


@dataclass
class Workload:
    name: str
    X: np.ndarray
    L: np.ndarray
    l: np.ndarray
    k: int
    modes: tuple
    params: dict = field(default_factory=dict)

    @property
    def span(self) -> float:
        """max(range_x(l), range_y(l)), the scale of the coordinate tolerance."""
        return float(max(np.ptp(self.l[:, 0]), np.ptp(self.l[:, 1])))


# name -> (N, D, clusters, g, grid cols, k, seed, kwargs for mixture, modes)
CONFIGS = {
    "c1_plain_fp32": (10_000, 8, 10, 64, 8, 8, 1,
                      dict(sd_range=(0.5, 1.5), isotropic=True, background=0.0), ("fp32",)),
    "c2_fp32_1m": (1_000_000, 32, 30, 400, 20, 16, 2, dict(), ("fp32", "bf16")),
    "c3_bf16_1m": (1_000_000, 48, 30, 1024, 32, 20, 3, dict(), ("bf16", "fp32")),
    "c4_large_10m": (10_000_000, 64, 50, 1024, 32, 16, 4,
                     dict(lognormal_weights=True), ("bf16", "fp32")),
}


def make(name: str, n: int | None = None) -> Workload:
    """Build a named workload.  ``n`` overrides the point count (a prefix of the
    same stream is NOT guaranteed; use ``subsample`` for that)."""
    N, D, ncl, g, cols, k, seed, kw, modes = CONFIGS[name]
    if n is not None:
        N = n
    X = mixture(N, D, ncl, seed, **kw)
    L = landmarks_from_data(X, g, seed)
    l = grid2d(g, cols)
    return Workload(name, X, L, l, k, modes)


def subsample(n_total: int, n: int, seed: int) -> np.ndarray:
    """Sorted seeded sample of n row indices out of n_total."""
    (r,) = _streams(seed + 104729, 1)
    return np.sort(r.choice(n_total, size=n, replace=False))


def paper_shaped(d: int, seed: int = 11, n: int = 1 << 20, g: int = 256, k: int = 16) -> Workload:
    """n = 2^20 uniform points, g = 256 landmarks (16 x 16 grid), k = 16."""
    X = uniform_points(n, d, seed)
    L = landmarks_from_data(X, g, seed, noise=0.0)
    return Workload("paper_uniform_d%d" % d, X, L, grid2d(g, 16), k, ("fp32",))
