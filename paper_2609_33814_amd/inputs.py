"""Seeded synthetic OT problems of the shapes the paper measures on.

This module only draws inputs; it holds none of the solver's arithmetic and
imports neither the native library nor the oracle, so both sides (the HIP
path and the FP64 oracle) can take their problems from it.

Two families, standing in for data that is not shipped with the paper:

* grid histograms (the DOTmark setting of the experiment appendix, "Data and
  ground cost"): pixels of an s x s grid with integer coordinates
  z in {0..s-1}^2, squared Euclidean cost normalised by 2 (s-1)^2 so that
  C lies in [0, 1] with max 1.  The histogram is a seeded mixture of 3-6
  isotropic Gaussians plus a 1e-6 floor, renormalised (the paper floors
  empty pixels at 1e-15; strictly positive marginals are required by the
  problem statement, Eq. 1).
* colour point clouds (the colour-transfer appendix, "Pixel-level OT
  formulation"): N RGB points in [0,1]^3 drawn from a seeded 8-component
  Gaussian mixture and clipped, uniform weights 1/N, cost normalised by the
  largest pairwise squared distance so that C lies in [0, 1].
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Problem:
    """One OT instance: C_ij = cost_scale * ||x_i - y_j||^2, marginals r, c."""

    x: np.ndarray          # (m, d) float32 source points
    y: np.ndarray          # (n, d) float32 target points
    r: np.ndarray          # (m,) float64, positive, sums to 1
    c: np.ndarray          # (n,) float64, positive, sums to 1
    cost_scale: float      # s in C_ij = s * ||x_i - y_j||^2
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.x.shape[0])

    @property
    def n(self) -> int:
        return int(self.y.shape[0])

    @property
    def dim(self) -> int:
        return int(self.x.shape[1])


def grid_points(side: int) -> np.ndarray:
    """Integer pixel coordinates of a side x side grid, row-major, float32."""
    ii, jj = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    return np.stack([ii.ravel(), jj.ravel()], axis=1).astype(np.float32)


def grid_mixture(side: int, seed: int, floor: float = 1e-6) -> np.ndarray:
    """Seeded Gaussian-mixture histogram on a side x side grid (float64, sums to 1).

    Recipe: K ~ U{3..6} components; means ~ U[0.15, 0.85]^2, sigmas ~
    U[0.05, 0.20], weights ~ U[0.5, 1.5], all in unit coordinates
    u = z / (side - 1); h = sum_k w_k exp(-|u - mu_k|^2 / (2 sigma_k^2));
    normalise, add the floor, renormalise.  Pixel order is row-major.
    """
    rng = np.random.default_rng(seed)
    k = int(rng.integers(3, 7))
    means = rng.uniform(0.15, 0.85, size=(k, 2))
    sig = rng.uniform(0.05, 0.20, size=k)
    w = rng.uniform(0.5, 1.5, size=k)
    u = grid_points(side).astype(np.float64) / max(side - 1, 1)
    h = np.zeros(side * side)
    for q in range(k):
        d2 = ((u - means[q]) ** 2).sum(axis=1)
        h += w[q] * np.exp(-d2 / (2.0 * sig[q] ** 2))
    h /= h.sum()
    h += floor
    h /= h.sum()
    return h


def grid_problem(side: int, seed_r: int, seed_c: int) -> Problem:
    """Grid-histogram OT problem with the max-1 normalised squared cost."""
    z = grid_points(side)
    scale = 1.0 / (2.0 * (side - 1) ** 2) if side > 1 else 1.0
    return Problem(x=z, y=z.copy(), r=grid_mixture(side, seed_r),
                   c=grid_mixture(side, seed_c), cost_scale=scale,
                   name=f"grid{side}x{side}")


def colour_mixture(npts: int, seed: int, comps: int = 8) -> np.ndarray:
    """Seeded RGB point cloud in [0,1]^3 (float32): 8-component Gaussian mixture, clipped."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(0.1, 0.9, size=(comps, 3))
    sig = rng.uniform(0.03, 0.12, size=comps)
    w = rng.dirichlet(np.ones(comps))
    lab = rng.choice(comps, size=npts, p=w)
    pts = means[lab] + sig[lab, None] * rng.standard_normal((npts, 3))
    return np.clip(pts, 0.0, 1.0).astype(np.float32)


def _hull_vertices(p: np.ndarray) -> np.ndarray:
    if p.shape[0] <= 64:
        return p
    try:
        from scipy.spatial import ConvexHull
        return p[ConvexHull(p).vertices]
    except Exception:  # degenerate (flat) clouds: fall back to all points
        return p


def max_sq_distance(x: np.ndarray, y: np.ndarray) -> float:
    """max_{p,q} ||x_p - y_q||^2 in float64.

    The squared distance is convex in each argument, so the maximum over the
    two clouds is attained at a pair of convex-hull vertices; only those pairs
    are enumerated.
    """
    hx = _hull_vertices(x.astype(np.float64))
    hy = _hull_vertices(y.astype(np.float64))
    best = 0.0
    for s in range(0, hx.shape[0], 256):
        blk = hx[s:s + 256]
        d2 = ((blk[:, None, :] - hy[None, :, :]) ** 2).sum(axis=2)
        best = max(best, float(d2.max()))
    return best


def colour_problem(npts_x: int, npts_y: int, seed_x: int, seed_y: int) -> Problem:
    """Colour-transfer stand-in: uniform weights, cost scaled to max 1."""
    x = colour_mixture(npts_x, seed_x)
    y = colour_mixture(npts_y, seed_y)
    dmax = max_sq_distance(x, y)
    return Problem(x=x, y=y, r=np.full(npts_x, 1.0 / npts_x),
                   c=np.full(npts_y, 1.0 / npts_y), cost_scale=1.0 / dmax,
                   name=f"colour{npts_x}x{npts_y}")


def random_problem(m: int, n: int, dim: int, seed: int, integer: bool = False,
                   span: float = 1.0) -> Problem:
    """Small random instance for tests: Dirichlet-ish marginals, points in a box."""
    rng = np.random.default_rng(seed)
    if integer:
        x = rng.integers(0, int(span) + 1, size=(m, dim)).astype(np.float32)
        y = rng.integers(0, int(span) + 1, size=(n, dim)).astype(np.float32)
    else:
        x = (span * rng.random((m, dim))).astype(np.float32)
        y = (span * rng.random((n, dim))).astype(np.float32)
    r = rng.uniform(0.2, 1.0, m)
    c = rng.uniform(0.2, 1.0, n)
    r /= r.sum()
    c /= c.sum()
    dmax = max_sq_distance(x, y)
    return Problem(x=x, y=y, r=r, c=c, cost_scale=1.0 / dmax if dmax > 0 else 1.0,
                   name=f"rand{m}x{n}d{dim}")


# Workload recipes (seeds fixed per workload).
def c1_problem() -> Problem:
    """Two 32x32 grid histograms (n = m = 1024)."""
    return grid_problem(32, 11, 12)


def c2_problem() -> Problem:
    """Two 128x128 grid histograms (n = m = 16384)."""
    return grid_problem(128, 21, 22)


def c3_problem() -> Problem:
    """Colour transfer: 1024x1024 = 1,048,576 RGB points per side (seeds 31, 32)."""
    return colour_problem(1 << 20, 1 << 20, 31, 32)


def c3b_problem() -> Problem:
    """Colour transfer at 4238x2365 = 10,022,870 RGB points per side (seeds 33, 34)."""
    return colour_problem(10022870, 10022870, 33, 34)


def batch_sides(count: int = 64, seed: int = 41) -> list[int]:
    """Grid sides for the uneven batch: drawn from {32, 64, 128, 256}."""
    idx = np.random.default_rng(seed).integers(0, 4, count)
    return [[32, 64, 128, 256][int(i)] for i in idx]


def batch_problem(p: int, side: int) -> Problem:
    return grid_problem(side, 4100 + 2 * p, 4101 + 2 * p)
