"""Seeded synthetic inputs shaped like the SNG-DBSCAN workloads.

This module only draws point sets and carries their hyperparameters. It holds
none of the method's arithmetic (no sampling of pairs, no distances, no graph
work), so both the oracle-based tests and the HIP path can take their inputs
from here without sharing any of the computation under test.

Every generator draws its points from ``numpy.random.default_rng(data_seed)``
(PCG64), concatenates the parts, applies one random permutation and returns a
C-contiguous float32 array ``X[n, d]``. ``seed`` is the pair-sampler seed that
the method itself consumes.

The paper evaluates on public UCI/OpenML datasets (Section 5, Figs. 2-7); those
are not available here, so these generators stand in for them with the same
kind of structure: dense well-separated blobs plus uniform clutter
(Assumption 1 of Section 4.1 is the regime the method is designed for).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Workload:
    """One clustering instance: points plus the method's hyperparameters."""

    name: str
    X: np.ndarray                   # float32 [n, d], C-contiguous
    s: float                        # sampling rate
    eps: float                      # neighbourhood radius
    min_pts: int                    # core threshold on the sampled degree
    seed: int                       # pair-sampler seed
    X_lp: Optional[np.ndarray] = None   # uint16 bit patterns of a 16-bit copy
    lp_kind: Optional[str] = None       # "bf16" or "fp16"
    lp_scale: float = 1.0               # X ~= lp_scale * X_lp
    eps_grid: Optional[np.ndarray] = None     # sweep: float64 [K]
    min_pts_grid: Optional[np.ndarray] = None  # sweep: int32 [P]
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def d(self) -> int:
        return int(self.X.shape[1])


def _finish(parts, rng) -> np.ndarray:
    X = np.concatenate(parts, axis=0)
    X = X[rng.permutation(X.shape[0])]
    return np.ascontiguousarray(X.astype(np.float32))


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even) and
    return the 16-bit patterns. NaNs are kept quiet NaNs."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounded = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    nan = np.isnan(x)
    out = rounded.astype(np.uint16)
    out[nan] = 0x7FC0
    return out


def bf16_to_f32(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << 16).view(np.float32)


def fp16_bits(x: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float32).astype(np.float16).view(np.uint16)


# ---------------------------------------------------------------------------
# The five workload shapes
# ---------------------------------------------------------------------------

def blobs_2d(data_seed: int = 1001) -> Workload:
    """n=10,000, d=2: five isotropic Gaussian blobs (sigma 0.05, centres uniform
    in the unit square, 1,900 points each) plus 500 uniform points; s=0.01,
    eps=0.05, MinPts=3."""
    rng = np.random.default_rng(data_seed)
    centres = rng.uniform(0.0, 1.0, size=(5, 2))
    parts = [rng.normal(c, 0.05, size=(1900, 2)) for c in centres]
    parts.append(rng.uniform(0.0, 1.0, size=(500, 2)))
    return Workload("blobs2d_n10k", _finish(parts, rng), s=0.01, eps=0.05,
                    min_pts=3, seed=1, meta={"data_seed": data_seed})


def mixture_16d(sigma: float = 1.0, data_seed: int = 1002,
                n_total: int = 1_000_000) -> Workload:
    """n=1,000,000, d=16: 50-component Gaussian mixture (centres N(0, 25 I),
    per-coordinate standard deviation ``sigma``) plus 2% points uniform over the
    bounding box of the mixture; s=0.001, eps=2.0, MinPts=5.

    ``sigma=1`` is the unit-variance literal shape. ``sigma=0.25`` is a denser
    variant in which the sampled graph has real clusters at the same eps.
    ``n_total`` scales the instance down for tests (same recipe)."""
    rng = np.random.default_rng(data_seed)
    k, d = 50, 16
    n_noise = n_total // 50
    per = (n_total - n_noise) // k
    n_noise = n_total - per * k
    centres = rng.normal(0.0, 5.0, size=(k, d))
    parts = [rng.normal(c, sigma, size=(per, d)) for c in centres]
    mix = np.concatenate(parts, axis=0)
    lo, hi = mix.min(axis=0), mix.max(axis=0)
    parts.append(rng.uniform(lo, hi, size=(n_noise, d)))
    name = "gmm16d_n%d%s" % (n_total, "" if sigma == 1.0 else "_sigma%g" % sigma)
    return Workload(name, _finish(parts, rng), s=0.001, eps=2.0, min_pts=5, seed=2,
                    meta={"data_seed": data_seed, "sigma": sigma})


# eps for the 784-d workload: the 1st percentile of the sampled distances
# (seed 3, all non-self slots), placed at the midpoint of the gap between that
# order statistic and the next larger distinct value (so no sampled pair sits
# exactly on the threshold). Derived from the oracle by
# tests/golden/derive_mnistlike_eps.py and re-checked by a test.
MNISTLIKE_EPS = 3.97555975992872


def mnistlike_784d(data_seed: int = 1003, n_per: int = 7000) -> Workload:
    """n=70,000, d=784: 8-bit quantised images in [0,1] built from 10 sparse
    random prototypes (30% non-zero, values U(0,1)) plus per-pixel Gaussian
    noise sigma 0.15, clipped; stored as float32 and as a bfloat16 copy.
    s=0.01, MinPts=10, eps at the 1st percentile of sampled distances."""
    rng = np.random.default_rng(data_seed)
    d, k = 784, 10
    nnz = int(0.3 * d)
    protos = np.zeros((k, d))
    for p in range(k):
        pos = rng.choice(d, size=nnz, replace=False)
        protos[p, pos] = rng.uniform(0.0, 1.0, size=nnz)
    parts = [np.clip(protos[p] + rng.normal(0.0, 0.15, size=(n_per, d)), 0.0, 1.0)
             for p in range(k)]
    X = np.concatenate(parts, axis=0)
    X = X[rng.permutation(X.shape[0])]
    q = np.rint(255.0 * X).astype(np.uint8)
    X32 = np.ascontiguousarray((q.astype(np.float64) / 255.0).astype(np.float32))
    eps = MNISTLIKE_EPS if (MNISTLIKE_EPS is not None and n_per == 7000
                            and data_seed == 1003) else float("nan")
    return Workload("mnistlike784d_n%d" % (k * n_per), X32, s=0.01, eps=eps,
                    min_pts=10, seed=3, X_lp=bf16_bits(X32), lp_kind="bf16",
                    lp_scale=1.0, meta={"data_seed": data_seed, "q": q})


def sweep_32d(data_seed: int = 1004, n_per: int = 5000, k: int = 100) -> Workload:
    """n=500,000, d=32: 100-component Gaussian mixture with anisotropic
    covariances Q diag(lambda) Q^T (lambda uniform in [0.1, 2], Q Haar),
    centres N(0, 25 I); s=0.002; eps grid 4*3^(k/31), k=0..31; MinPts
    {2, 4, 8, 16}."""
    rng = np.random.default_rng(data_seed)
    d = 32
    centres = rng.normal(0.0, 5.0, size=(k, d))
    parts = []
    for c in centres:
        lam = rng.uniform(0.1, 2.0, size=d)
        g = rng.normal(size=(d, d))
        Q, R = np.linalg.qr(g)
        Q = Q * np.sign(np.diag(R))[None, :]
        z = rng.normal(size=(n_per, d))
        parts.append(c + (z * np.sqrt(lam)) @ Q.T)
    X = _finish(parts, rng)
    grid = 4.0 * 3.0 ** (np.arange(32) / 31.0)
    return Workload("aniso32d_n%d" % X.shape[0], X, s=0.002, eps=float(grid[0]), min_pts=2,
                    seed=4, eps_grid=grid, min_pts_grid=np.array([2, 4, 8, 16], np.int32),
                    meta={"data_seed": data_seed})


def small_blobs_3d(n: int, data_seed: int, seed: int) -> Workload:
    """One instance of the uneven batch: five isotropic 3-d Gaussian blobs
    (sigma 0.05, centres uniform in the unit cube) holding 95% of the points
    in equal shares, plus 5% uniform points; s=0.01, eps=0.1, MinPts=4."""
    rng = np.random.default_rng(data_seed)
    n_noise = int(round(0.05 * n))
    n_blob = n - n_noise
    centres = rng.uniform(0.0, 1.0, size=(5, 3))
    counts = [n_blob // 5 + (1 if b < n_blob % 5 else 0) for b in range(5)]
    parts = [rng.normal(c, 0.05, size=(cnt, 3)) for c, cnt in zip(centres, counts)]
    parts.append(rng.uniform(0.0, 1.0, size=(n_noise, 3)))
    return Workload("blobs3d_n%d" % n, _finish(parts, rng), s=0.01, eps=0.1,
                    min_pts=4, seed=seed, meta={"data_seed": data_seed})


def uneven_batch(count: int = 64, size_seed: int = 1051,
                 n_lo: float = 1e3, n_hi: float = 2e5) -> List[Workload]:
    """``count`` independent instances with n log-uniform in [n_lo, n_hi]."""
    rng = np.random.default_rng(size_seed)
    ns = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=count)))
    return [small_blobs_3d(int(ns[k]), 1100 + k, 500 + k) for k in range(count)]


def lidar_3d(data_seed: int = 1005, n_total: int = 5_000_000) -> Workload:
    """LiDAR-like scene, n=5,000,000, d=3: a ground plane (70%, z ~ N(0, 0.02)
    over 200 m x 200 m), 300 objects sampled on ellipsoid surfaces (29%,
    semi-axes 0.25-2.5 m, random yaw, resting on the ground) and 1% uniform
    clutter up to 10 m; s=0.0005, eps=0.3, MinPts=4."""
    rng = np.random.default_rng(data_seed)
    n_ground = int(round(0.70 * n_total))
    n_clutter = int(round(0.01 * n_total))
    n_obj = n_total - n_ground - n_clutter
    ground = np.column_stack([rng.uniform(0, 200, n_ground), rng.uniform(0, 200, n_ground),
                              rng.normal(0.0, 0.02, n_ground)])
    axes = rng.uniform(0.25, 2.5, size=(300, 3))
    area = axes[:, 0] * axes[:, 1] + axes[:, 1] * axes[:, 2] + axes[:, 2] * axes[:, 0]
    cnt = np.floor(n_obj * area / area.sum()).astype(np.int64)
    cnt[: n_obj - cnt.sum()] += 1
    parts = [ground]
    for o in range(300):
        u = rng.normal(size=(cnt[o], 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        p = u * axes[o]
        yaw = rng.uniform(0, 2 * math.pi)
        c, s_ = math.cos(yaw), math.sin(yaw)
        rot = np.array([[c, -s_, 0.0], [s_, c, 0.0], [0.0, 0.0, 1.0]])
        centre = np.array([rng.uniform(0, 200), rng.uniform(0, 200), axes[o, 2]])
        parts.append(p @ rot.T + centre)
    parts.append(np.column_stack([rng.uniform(0, 200, n_clutter), rng.uniform(0, 200, n_clutter),
                                  rng.uniform(0, 10, n_clutter)]))
    return Workload("lidar3d_n%d" % n_total, _finish(parts, rng), s=0.0005, eps=0.3,
                    min_pts=4, seed=5, meta={"data_seed": data_seed})


def balls_3d(n: int, data_seed: int = 1061) -> tuple[Workload, np.ndarray]:
    """Three uniform balls in R^3 (the paper's simulated recovery study,
    Section 3, Fig. 1): equal weights, radius 1, centres on an equilateral
    triangle of side 4; ceil(20 ln n) samples per point (s = that / n),
    eps = 0.3, MinPts = 3, sampler seed 6. Returns the workload and the
    true ball of every point (after the shuffle)."""
    rng = np.random.default_rng(data_seed)
    centres = np.array([[0.0, 0.0, 0.0], [4.0, 0.0, 0.0], [2.0, 2.0 * math.sqrt(3.0), 0.0]])
    ball = rng.integers(0, 3, n)
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    r = rng.random(n) ** (1.0 / 3.0)
    X = centres[ball] + u * r[:, None]
    perm = rng.permutation(n)
    m = int(math.ceil(20.0 * math.log(n))) if n > 1 else 1
    W = Workload("balls3d_n%d" % n, np.ascontiguousarray(X[perm].astype(np.float32)),
                 s=m / n, eps=0.3, min_pts=3, seed=6, meta={"data_seed": data_seed, "m": m})
    return W, ball[perm]


def random_instance(rng: np.random.Generator, n: int, d: int, kind: str = "blobs",
                    spread: float = 0.05) -> np.ndarray:
    """Small random point sets for property and parity tests.

    kind: "blobs" (a few Gaussian blobs plus uniform clutter), "grid" (small
    integers, so every squared distance is exact in any precision and order),
    "uniform", or "dupes" (many exact duplicate points)."""
    if n == 0:
        return np.zeros((0, d), np.float32)
    if kind == "grid":
        return rng.integers(-6, 7, size=(n, d)).astype(np.float32)
    if kind == "uniform":
        return rng.uniform(0, 1, size=(n, d)).astype(np.float32)
    if kind == "dupes":
        base = rng.uniform(0, 1, size=(max(1, n // 8), d))
        return base[rng.integers(0, base.shape[0], size=n)].astype(np.float32)
    k = int(rng.integers(1, 6))
    centres = rng.uniform(0, 1, size=(k, d))
    lab = rng.integers(0, k + 1, size=n)
    X = rng.uniform(0, 1, size=(n, d))
    blob = lab < k
    X[blob] = centres[lab[blob]] + rng.normal(0, spread, size=(int(blob.sum()), d))
    return X.astype(np.float32)
