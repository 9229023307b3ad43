"""Seeded synthetic inputs: point clouds, right-hand sides and batch parameters.

This module holds random-number generation only, none of the method's
arithmetic; both the HIP library's tests and the oracle's tests draw their
inputs from it.  The paper measures on boundary-element matrices on a
triangulated unit sphere; point clouds on the unit sphere (and, for the volume
case, in the unit cube) stand in for them.

Generator: numpy ``default_rng(seed)`` (PCG64).  Sphere points are normalised
standard-normal 3-vectors; cube points are uniform in [0, 1)^3.  Right-hand
sides are i.i.d. N(0, 1).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


def sphere_points(n: int, seed: int) -> np.ndarray:
    g = np.random.default_rng(seed)
    v = g.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def cube_points(n: int, seed: int) -> np.ndarray:
    g = np.random.default_rng(seed)
    return g.random((n, 3))


def line_points(n: int, seed: int) -> np.ndarray:
    """Points on a segment of the x axis (an almost one-dimensional cloud)."""
    g = np.random.default_rng(seed)
    P = np.zeros((n, 3))
    P[:, 0] = g.random(n)
    return P


def rhs(n: int, m: int, seed: int) -> np.ndarray:
    g = np.random.default_rng(seed)
    return g.standard_normal((n, m))


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    geometry: str  # "sphere" or "cube"
    n: int
    ell: float
    shift: float
    leaf: int
    eta: float
    p: int
    m: int
    index: int  # seeds: points 1000 + index, right-hand sides 2000 + index

    @property
    def k(self) -> int:
        return self.p ** 3

    def points(self) -> np.ndarray:
        f = sphere_points if self.geometry == "sphere" else cube_points
        return f(self.n, 1000 + self.index)

    def rhs(self, m: int | None = None) -> np.ndarray:
        return rhs(self.n, self.m if m is None else m, 2000 + self.index)

    def params(self) -> dict:
        return dict(ell=self.ell, shift=self.shift, eta=self.eta, leaf=self.leaf, p=self.p)


# Five workloads: small plain FP64, the FP64 throughput case, the precision
# case (volume), the differentiation case; the batch is generated separately.
SMALL = Workload("sphere-n4096-k27-m4", "sphere", 4096, 0.5, 1.0, 32, 1.0, 3, 4, 0)
FP64 = Workload("sphere-n65536-k64-m32", "sphere", 65536, 0.5, 1.0, 64, 1.0, 4, 32, 1)
PRECISION = Workload("cube-n262144-k64-m64", "cube", 262144, 0.25, 0.5, 64, 1.0, 4, 64, 2)
GRADIENT = Workload("sphere-n131072-k64-m16", "sphere", 131072, 0.5, 1.0, 64, 1.0, 4, 16, 4)
WORKLOADS = {w.name: w for w in (SMALL, FP64, PRECISION, GRADIENT)}


@dataclasses.dataclass(frozen=True)
class BatchSystem:
    n: int
    ell: float
    shift: float
    p: int
    leaf: int
    m: int
    point_seed: int
    rhs_seed: int

    @property
    def k(self) -> int:
        return self.p ** 3

    def points(self) -> np.ndarray:
        return sphere_points(self.n, self.point_seed)

    def rhs(self) -> np.ndarray:
        return rhs(self.n, self.m, self.rhs_seed)


def batch_systems(count: int = 64, seed: int = 3004, n_lo: int = 2048, n_hi: int = 32768) -> list[BatchSystem]:
    """Independent systems: n log-uniform in [n_lo, n_hi], ell ~ U[0.2, 1.0],
    shift 1, order 3 (k = 27, leaf 32) or 4 (k = 64, leaf 64) with probability
    1/2 each, m uniform in {1..32}; system i's points from seed 4000 + i."""
    g = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        ell = float(g.uniform(0.2, 1.0))
        p = 3 if g.random() < 0.5 else 4
        m = int(g.integers(1, 33))
        out.append(BatchSystem(n, ell, 1.0, p, 32 if p == 3 else 64, m, 4000 + i, 5000 + i))
    return out
