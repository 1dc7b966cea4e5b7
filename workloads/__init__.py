"""Seeded synthetic lattice instances: the one input generator shared by the
tests, the benchmark and the oracle.

This module holds none of the solver's arithmetic. It only draws random
numbers and does the lattice bookkeeping (which bars exist, which nodes are
clamped), so that the CPU oracle and the GPU library see identical inputs.

Workload (paper, section 3.1): a 2-D triangle-lattice truss of elastic rods
with a load random in magnitude and direction on every node.  Concretely:

* node (i, j), 0 <= i < nx, 0 <= j < ny, sits at (i + j/2, j*sqrt(3)/2);
* every node stores its three "forward" bars
    d = 0 : (i, j) -- (i+1, j)
    d = 1 : (i, j) -- (i, j+1)
    d = 2 : (i, j) -- (i-1, j+1)
  in ``ea[d, j, i]`` (float32, EA of the rod, rod length L = 1); bars that
  would leave the lattice have ea = 0;
* the nodes with i = 0 are clamped (``fixed[j, i] = 1``) with a prescribed
  displacement of zero;
* loads ``f[j, i, c]`` are iid N(0, 1) per DOF, drawn for every DOF so that
  the random stream does not depend on the clamp mask, then zeroed on the
  clamped DOFs.

Draw order for one instance from ``numpy.random.default_rng(seed)``: the
lognormal EA planes first (only when ``ea="lognormal"``), then the loads.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Instance",
    "make_instance",
    "absent_bar_mask",
    "batch_shapes",
    "served_sides",
    "poisson_arrivals",
]


@dataclasses.dataclass
class Instance:
    nx: int
    ny: int
    ea: np.ndarray        # float32 [3, ny, nx]
    fixed: np.ndarray     # uint8   [ny, nx]
    u_fixed: np.ndarray   # float64 [ny, nx, 2]
    f: np.ndarray         # float64 [ny, nx, 2]
    seed: int = 0

    @property
    def dof(self) -> int:
        """DOF count as the workloads count it: 2 per node, clamped included."""
        return 2 * self.nx * self.ny


def absent_bar_mask(nx: int, ny: int) -> np.ndarray:
    """Boolean [3, ny, nx]: True where the forward bar would leave the lattice."""
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    m = np.zeros((3, ny, nx), dtype=bool)
    m[0] = np.broadcast_to(i == nx - 1, (ny, nx))
    m[1] = np.broadcast_to(j == ny - 1, (ny, nx))
    m[2] = (i == 0) | (j == ny - 1)
    return m


def make_instance(nx: int, ny: int, seed: int = 0, ea: str = "unit",
                  sigma: float = 0.5, clamp: str = "left") -> Instance:
    """One seeded lattice instance.

    ea    : "unit" (EA = 1 everywhere) or "lognormal" (EA ~ lognormal(0, sigma)
            per bar, rounded to float32).
    clamp : "left" (nodes with i = 0 clamped) or "none" (no supports; the
            stiffness is then singular, which only the oracle's checks use).
    """
    if nx < 1 or ny < 1:
        raise ValueError("lattice needs at least one node per side")
    rng = np.random.default_rng(seed)
    if ea == "lognormal":
        e = rng.lognormal(0.0, sigma, (3, ny, nx)).astype(np.float32)
    elif ea == "unit":
        e = np.ones((3, ny, nx), dtype=np.float32)
    else:
        raise ValueError(f"unknown ea kind {ea!r}")
    e[absent_bar_mask(nx, ny)] = 0.0
    f = rng.standard_normal((ny, nx, 2))
    fixed = np.zeros((ny, nx), dtype=np.uint8)
    if clamp == "left":
        fixed[:, 0] = 1
    elif clamp != "none":
        raise ValueError(f"unknown clamp kind {clamp!r}")
    f[fixed.astype(bool)] = 0.0
    u_fixed = np.zeros((ny, nx, 2))
    return Instance(nx, ny, e, fixed, u_fixed, f, seed)


def batch_shapes(count: int = 256, seed: int = 1000, lo: int = 32, hi: int = 512):
    """Shapes of the batched workload: side nx ~ U{lo..hi}, aspect r ~ U[0.5, 2],
    ny = round(r * nx), with r redrawn until lo <= ny <= hi.  Lattice b of the
    batch is then drawn with seed 2000 + b."""
    rng = np.random.default_rng(seed)
    shapes = []
    for _ in range(count):
        nx = int(rng.integers(lo, hi + 1))
        while True:
            r = rng.uniform(0.5, 2.0)
            ny = int(round(r * nx))
            if lo <= ny <= hi:
                break
        shapes.append((nx, ny))
    return shapes


def served_sides(count: int, seed: int = 3000, lo: int = 64, hi: int = 2048):
    """Square lattice sides of the served workload, log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return [int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
            for _ in range(count)]


def poisson_arrivals(count: int, rate_per_s: float, seed: int = 3000) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson stream."""
    rng = np.random.default_rng(seed + 1)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, count))
