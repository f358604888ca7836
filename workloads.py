"""Seeded synthetic inputs for the 2D vortex-particle FMM.

This module only draws particle positions and circulations; it holds none of
the method's arithmetic (no kernel, no expansion, no tree).  Both the CPU
oracle tests and the GPU path consume the arrays it returns, so neither side
needs its own random-number generator.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) and draws in
the order x, then y, then gamma.  The five named workloads follow the paper's
vortex-method client (Section 3, eqs. 4-9) and its test case (Section 7.1:
Lamb-Oseen vortex on a lattice, uniform core size sigma):

  C1  4,096 particles uniform in the unit square, gamma ~ U(-1,1),
      sigma = 0.005, depth 4, p = 12, FP64.
  C2  1,048,576 particles on a jittered 1024x1024 cell-centred lattice sampling
      a Lamb-Oseen vortex (core 0.1, total circulation 1, gamma = vorticity x
      cell area), sigma = 0.002, depth 8, p = 17, FP64.
  C3  4,194,304 particles from a 16-component Gaussian mixture (stds
      U(0.01, 0.1), rejection to the unit square), gamma ~ N(0,1),
      sigma = 0.001, depth 9, p = 17, mixed precision.
  C4  512 independent instances, N_i log-uniform in [2048, 65536], uniform in
      the unit square, gamma ~ U(-1,1), sigma = 0.005, p = 12, depth chosen so
      leaves hold ~64 particles, batched.
  C5  67,108,864 particles uniform in the unit square, gamma ~ U(-1,1),
      sigma = 2e-4, depth 11, p = 20, mixed precision.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    x: np.ndarray
    y: np.ndarray
    gamma: np.ndarray
    sigma: float
    depth: int
    p: int
    precision: str = "fp64"          # "fp64" or "mixed"
    fp32_fine_levels: int = 0        # mixed: number of finest levels whose M2L runs in FP32
    x0: float = 0.0
    y0: float = 0.0
    width: float = 1.0
    # batched workloads only: CSR offsets into x/y/gamma and per-instance depth
    offsets: np.ndarray | None = None
    depths: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def uniform_square(n: int, seed: int) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """n points uniform in [0,1)^2 with gamma ~ U(-1,1)."""
    rng = np.random.default_rng(seed)
    x = rng.random(n)
    y = rng.random(n)
    g = rng.uniform(-1.0, 1.0, n)
    return x, y, g


def uniform_cube(n: int, seed: int) -> tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """n points uniform in [0,1)^3 with charges q ~ U(-1,1) (the 3D form)."""
    rng = np.random.default_rng(seed)
    x = rng.random(n)
    y = rng.random(n)
    z = rng.random(n)
    q = rng.uniform(-1.0, 1.0, n)
    return x, y, z, q


def lamb_oseen_lattice(m: int, core: float, total_circulation: float = 1.0,
                       jitter: float = 0.0, seed: int = 0,
                       lo: float = 0.0, hi: float = 1.0,
                       centre: tuple[float, float] = (0.5, 0.5)):
    """Cell-centred m x m lattice on [lo, hi)^2 sampling a Lamb-Oseen vortex.

    Vorticity omega(r) = G0/(pi c^2) exp(-r^2/c^2) with c^2 = 4 nu t
    (Section 7.1, eq. 16); each particle carries gamma = omega(x_j) * h^2
    (vorticity times cell area).  ``jitter`` is the half-width, in units of
    the spacing h, of a uniform per-axis displacement.
    """
    h = (hi - lo) / m
    i = np.arange(m, dtype=np.float64)
    cx = lo + (i + 0.5) * h
    X, Y = np.meshgrid(cx, cx, indexing="xy")
    x = X.ravel().copy()
    y = Y.ravel().copy()
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        x += rng.uniform(-jitter * h, jitter * h, x.shape[0])
        y += rng.uniform(-jitter * h, jitter * h, y.shape[0])
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2
    g = h * h * total_circulation / (math.pi * core * core) * np.exp(-r2 / (core * core))
    return x, y, g, h


def gaussian_mixture(n: int, components: int, seed: int):
    """n points from an equal-weight isotropic Gaussian mixture in [0,1)^2.

    Means ~ U[0,1)^2, stds ~ U(0.01, 0.1); samples outside the unit square are
    rejected and redrawn from the same component; gamma ~ N(0,1).  The points
    are shuffled so the input order carries no clustering.
    """
    rng = np.random.default_rng(seed)
    means = rng.random((components, 2))
    stds = rng.uniform(0.01, 0.1, components)
    per = n // components
    xs, ys = [], []
    for c in range(components):
        cnt = per if c < components - 1 else n - per * (components - 1)
        got_x, got_y, have = [], [], 0
        while have < cnt:
            need = cnt - have
            draw = rng.standard_normal((max(need, 1024), 2)) * stds[c] + means[c]
            ok = (draw[:, 0] >= 0.0) & (draw[:, 0] < 1.0) & (draw[:, 1] >= 0.0) & (draw[:, 1] < 1.0)
            draw = draw[ok][:need]
            got_x.append(draw[:, 0])
            got_y.append(draw[:, 1])
            have += draw.shape[0]
        xs.append(np.concatenate(got_x))
        ys.append(np.concatenate(got_y))
    x = np.concatenate(xs)
    y = np.concatenate(ys)
    order = rng.permutation(n)
    x = x[order].copy()
    y = y[order].copy()
    g = rng.standard_normal(n)
    return x, y, g, means, stds


def batched_depth(n_i: int) -> int:
    """Depth giving ~64 particles per leaf: max(2, round_half_up(log4(n/64)))."""
    return max(2, int(math.floor(math.log(n_i / 64.0, 4.0) + 0.5)))


def make(name: str) -> Workload:
    """Build one of the named workloads C1..C5."""
    name = name.upper()
    if name == "C1":
        x, y, g = uniform_square(4096, 1)
        return Workload("C1", x, y, g, sigma=0.005, depth=4, p=12)
    if name == "C2":
        m = 1024
        x, y, g, h = lamb_oseen_lattice(m, core=0.1, jitter=0.25, seed=2)
        return Workload("C2", x, y, g, sigma=0.002, depth=8, p=17,
                        meta={"lattice_h": h, "core": 0.1, "gamma0": 1.0})
    if name == "C3":
        x, y, g, means, stds = gaussian_mixture(4_194_304, 16, 3)
        return Workload("C3", x, y, g, sigma=0.001, depth=9, p=17,
                        precision="mixed", fp32_fine_levels=2,
                        meta={"means": means, "stds": stds})
    if name == "C4":
        rng = np.random.default_rng(4)
        k = 512
        ns = np.rint(np.exp(rng.uniform(math.log(2048.0), math.log(65536.0), k))).astype(np.int64)
        xs, ys, gs = [], [], []
        for n_i in ns:
            xs.append(rng.random(int(n_i)))
            ys.append(rng.random(int(n_i)))
            gs.append(rng.uniform(-1.0, 1.0, int(n_i)))
        offsets = np.zeros(k + 1, dtype=np.int64)
        offsets[1:] = np.cumsum(ns)
        depths = np.array([batched_depth(int(n_i)) for n_i in ns], dtype=np.int32)
        return Workload("C4", np.concatenate(xs), np.concatenate(ys), np.concatenate(gs),
                        sigma=0.005, depth=int(depths.max()), p=12, precision="mixed",
                        fp32_fine_levels=2, offsets=offsets, depths=depths)
    if name == "C5":
        x, y, g = uniform_square(1 << 26, 5)
        return Workload("C5", x, y, g, sigma=2e-4, depth=11, p=20,
                        precision="mixed", fp32_fine_levels=2)
    raise KeyError(name)


def probe_lattice(m: int, lo: float = 0.0, hi: float = 1.0) -> tuple[np.ndarray, np.ndarray]:
    """m x m vertex lattice lo + (i, j) (hi - lo) / m, i, j = 0 .. m-1, row by
    row: evaluation points for the velocity field (with m a multiple of the
    leaf count per side, every leaf edge carries points)."""
    h = (hi - lo) / m
    c = lo + np.arange(m, dtype=np.float64) * h
    X, Y = np.meshgrid(c, c, indexing="xy")
    return X.ravel().copy(), Y.ravel().copy()


def sample_targets(n: int, m: int, seed: int) -> np.ndarray:
    """Seeded target subset (sorted int64 indices) for sampled error checks."""
    if m >= n:
        return np.arange(n, dtype=np.int64)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, m, replace=False)).astype(np.int64)
