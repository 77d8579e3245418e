"""Seeded synthetic problem statements for the refined-wall solve.

This module is the one place where random inputs are drawn.  It hands out
*problem statements* only -- curve parameters, which reference panels to
refine and by how many dyadic levels, and exterior Stokeslet positions and
strengths -- and never discretizes, assembles or solves anything.  Both the
FP64 oracle (``oracle/``) and the GPU library receive the same statement and
each discretizes it independently.

Workload family (stand-ins for the paper's channel / Fallopian / lattice
walls, which are not available; see the paper's numerical section):

* wall: smooth star curve r(theta) = 1 + a cos(m theta), a = 0.3, m = 5,
  ``n_panels`` 16-point Gauss-Legendre panels uniform in theta;
* refinement: panels near a seeded point are split into 2**L equal-theta
  children (the paper refines 1 -> 4, 8 -> 64 and 6 -> 24 panels);
* right-hand side: velocity of exterior Stokeslets at radius 2.5 with
  N(0, I2) strengths (the paper generates boundary data from a known
  exterior-Stokeslet flow).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

STAR_A = 0.3
STAR_M = 5
STOKESLET_RADIUS = 2.5


@dataclasses.dataclass(frozen=True)
class Curve:
    """Star curve gamma(theta) = (1 + a cos(m theta)) (cos theta, sin theta)."""

    a: float = STAR_A
    m: int = STAR_M

    def point(self, theta):
        """Curve point at parameter ``theta`` (used only to place seeds)."""
        th = np.asarray(theta, dtype=np.float64)
        r = 1.0 + self.a * np.cos(self.m * th)
        return np.stack([r * np.cos(th), r * np.sin(th)], axis=-1)

    def outward_normal(self, theta):
        """Unit outward normal at ``theta`` (used only to place seeds)."""
        th = np.asarray(theta, dtype=np.float64)
        r = 1.0 + self.a * np.cos(self.m * th)
        dr = -self.a * self.m * np.sin(self.m * th)
        dx = dr * np.cos(th) - r * np.sin(th)
        dy = dr * np.sin(th) + r * np.cos(th)
        s = np.hypot(dx, dy)
        return np.stack([dy / s, -dx / s], axis=-1)


@dataclasses.dataclass(frozen=True)
class Refinement:
    """Which reference panels are split and into 2**level children each."""

    panel_ids: tuple
    levels: tuple

    @property
    def n_sel(self) -> int:
        return len(self.panel_ids)


@dataclasses.dataclass(frozen=True)
class Stokeslets:
    """Exterior point forces: positions (m, 2) and strengths (m, 2), mu = 1."""

    z: np.ndarray
    f: np.ndarray


@dataclasses.dataclass(frozen=True)
class Problem:
    curve: Curve
    n_panels: int
    order: int
    leaf_nodes: int
    refinement: Refinement
    rhs: List[Stokeslets]  # one Stokeslet set per right-hand side
    seed: int
    name: str = ""

    @property
    def n_nodes_ref(self) -> int:
        return self.n_panels * self.order


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def nearest_panels(curve: Curve, n_panels: int, p0: np.ndarray, n_sel: int) -> List[int]:
    """Indices of the ``n_sel`` reference panels closest to point ``p0``.

    Distance of a panel = min distance from p0 to the curve sampled at the
    panel's two end parameters and its mid parameter; ties go to the lower
    index.  Returned in increasing panel order.
    """
    h = 2.0 * math.pi / n_panels
    th = np.arange(n_panels) * h
    samples = np.stack([th, th + 0.5 * h, th + h], axis=1)
    pts = curve.point(samples)  # (P, 3, 2)
    d = np.min(np.linalg.norm(pts - p0[None, None, :], axis=-1), axis=1)
    order = np.lexsort((np.arange(n_panels), d))
    return sorted(int(i) for i in order[:n_sel])


def contiguous_panels(n_panels: int, theta0: float, n_sel: int) -> List[int]:
    """``n_sel`` consecutive panels (cyclic) centred on the panel holding theta0.

    For even ``n_sel`` the extra panel goes on the +theta side.
    """
    h = 2.0 * math.pi / n_panels
    c = int(math.floor((theta0 % (2.0 * math.pi)) / h)) % n_panels
    lo = c - (n_sel - 1) // 2
    return sorted({(lo + i) % n_panels for i in range(n_sel)})


def stokeslets(rng: np.random.Generator, count: int, radius: float = STOKESLET_RADIUS) -> Stokeslets:
    phi = rng.uniform(0.0, 2.0 * math.pi, size=count)
    z = np.stack([radius * np.cos(phi), radius * np.sin(phi)], axis=1)
    f = rng.standard_normal(size=(count, 2))
    return Stokeslets(z=z, f=f)


def seeded_point(curve: Curve, rng: np.random.Generator, dist: float):
    """Seed point p0 = gamma(theta0) + dist * n(theta0), theta0 ~ U[0, 2pi)."""
    theta0 = float(rng.uniform(0.0, 2.0 * math.pi))
    p0 = curve.point(theta0) + dist * curve.outward_normal(theta0)
    return theta0, p0


def near_point_problem(name: str, n_panels: int, n_sel: int, level: int, dist: float,
                       n_stokeslets: int, nrhs: int, seed: int,
                       order: int = 16, leaf_nodes: int = 64) -> Problem:
    """Refine the ``n_sel`` panels nearest a seeded point at ``dist`` outside."""
    curve = Curve()
    rng = _rng(seed)
    _, p0 = seeded_point(curve, rng, dist)
    ids = nearest_panels(curve, n_panels, p0, n_sel) if n_sel > 0 else []
    ref = Refinement(tuple(ids), tuple([level] * len(ids)))
    rhs = [stokeslets(rng, n_stokeslets) for _ in range(nrhs)]
    return Problem(curve, n_panels, order, leaf_nodes, ref, rhs, seed, name)


def config1(seed: int = 0, nrhs: int = 1) -> Problem:
    """64 panels (1024 nodes); 4 panels nearest a point at 0.02 split 3 levels;
    8 Stokeslets."""
    return near_point_problem("star64_refine4x3", 64, 4, 3, 0.02, 8, nrhs, seed)


def config2(seed: int = 0, nrhs: int = 1) -> Problem:
    """1024 panels (16384 nodes); 16 panels nearest a point at 1e-3 split
    4 levels; 16 Stokeslets."""
    return near_point_problem("star1024_refine16x4", 1024, 16, 4, 1e-3, 16, nrhs, seed)


def config4(seed: int = 0, nrhs: int = 32) -> Problem:
    """4096 panels (65536 nodes); 32 panels split 4 levels; 32 right-hand sides."""
    return near_point_problem("star4096_refine32x4", 4096, 32, 4, 1e-3, 16, nrhs, seed)


def batched_instances(n_inst: int = 64, seed: int = 0, n_panels: int = 1024,
                      nrhs: int = 8) -> List[Problem]:
    """Uneven refinement instances on one wall: n_sel ~ U{2..32},
    level ~ U{2..5}, contiguous panels around a seeded arc position."""
    curve = Curve()
    rng = _rng(seed)
    out = []
    for i in range(n_inst):
        n_sel = int(rng.integers(2, 33))
        level = int(rng.integers(2, 6))
        theta0 = float(rng.uniform(0.0, 2.0 * math.pi))
        ids = contiguous_panels(n_panels, theta0, n_sel)
        ref = Refinement(tuple(ids), tuple([level] * len(ids)))
        rhs = [stokeslets(rng, 16) for _ in range(nrhs)]
        out.append(Problem(curve, n_panels, 16, 64, ref, rhs, seed, f"inst{i}"))
    return out


def small_problem(n_panels: int = 16, ids: Sequence[int] = (3,), levels: Sequence[int] = (2,),
                  n_stokeslets: int = 4, nrhs: int = 1, seed: int = 0, curve: Curve = None,
                  order: int = 16, leaf_nodes: int = 64) -> Problem:
    """Tiny explicit problem for pins and edge cases."""
    curve = curve or Curve()
    rng = _rng(seed)
    ref = Refinement(tuple(int(i) for i in ids), tuple(int(l) for l in levels))
    rhs = [stokeslets(rng, n_stokeslets) for _ in range(nrhs)]
    return Problem(curve, n_panels, order, leaf_nodes, ref, rhs, seed, "small")


# four instances of the 64-instance batched family (seed 0) whose dense
# oracle fits (at most 48200 unknowns), chosen by
# numpy.random.default_rng(2024) among the 56 that do
BATCH_GOLDEN_INSTANCES = (6, 14, 42, 63)


def golden_cases() -> dict:
    """Full-size refinements whose dense-oracle solutions are stored under
    tests/golden (1024-panel wall, 16384 reference nodes):

    * ``config2_seed0``, ``config2_seed7``: the headline family (16 panels
      nearest a point at 1e-3, 4 levels);
    * ``wrap_16x4``: 16 consecutive panels across theta = 0 (1021..1023,
      0..12), 4 levels, Stokeslets of seed 3;
    * ``near4x6``: the 4 panels nearest a seeded point at 1e-3, 6 levels
      (64 children each);
    * ``pattern32x4``: the refinement pattern of the 65536-node workload
      (32 panels nearest a point at 1e-3, 4 levels) on this wall, where the
      dense oracle still fits (48128 unknowns);
    * ``batch0_inst<i>``: instances of the 64-instance batched family (their
      first right-hand side)."""
    wrap_ids = [1021, 1022, 1023] + list(range(13))
    return {
        "config2_seed0": config2(seed=0),
        "config2_seed7": config2(seed=7),
        "wrap_16x4": small_problem(n_panels=1024, ids=wrap_ids, levels=[4] * 16,
                                   n_stokeslets=16, seed=3),
        "near4x6": near_point_problem("star1024_refine4x6", 1024, 4, 6, 1e-3, 16, 1, seed=5),
        "pattern32x4": near_point_problem("star1024_refine32x4", 1024, 32, 4, 1e-3, 16, 1, seed=0),
        **{f"batch0_inst{i}": batched_instances(n_inst=64, seed=0, n_panels=1024, nrhs=8)[i]
           for i in BATCH_GOLDEN_INSTANCES},
    }


@dataclasses.dataclass(frozen=True)
class Request:
    """One served solve: arrival time (s), a refinement, nrhs Stokeslet sets."""

    t_arrival: float
    problem: Problem


def serving_requests(n: int, rate: float, seed: int = 0, n_panels: int = 4096, max_sel: int = 64,
                     max_level: int = 5, max_rhs: int = 16) -> List[Request]:
    """Poisson arrivals at ``rate`` requests/s; each request refines a
    contiguous block of n_sel ~ U{1..max_sel} panels around a seeded arc
    position by level ~ U{1..max_level} and asks for nrhs ~ U{1..max_rhs}
    right-hand sides of 16 exterior Stokeslets each."""
    curve = Curve()
    rng = _rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate))
        n_sel = int(rng.integers(1, max_sel + 1))
        level = int(rng.integers(1, max_level + 1))
        theta0 = float(rng.uniform(0.0, 2.0 * math.pi))
        ids = contiguous_panels(n_panels, theta0, n_sel)
        nrhs = int(rng.integers(1, max_rhs + 1))
        rhs = [stokeslets(rng, 16) for _ in range(nrhs)]
        out.append(Request(t, Problem(curve, n_panels, 16, 64, Refinement(tuple(ids), tuple([level] * len(ids))),
                                      rhs, seed, f"req{i}")))
    return out
