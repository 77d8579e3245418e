"""Oracle geometry: star curve, Gauss-Legendre panels, local refinement.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows Sec. 2.1 (Nystrom discretization of the boundary) and Sec. 3.1
(locally refined discretization: kept points I_k, cut points I_c, added points
I_p; I_o = I_k + I_c, I_n = I_k + I_p) and the numerical section's statement
that boundaries use 16-point composite Gauss panels uniform in the curve
parameter.

Readings where the paper is silent:
* the curve is counter-clockwise; t = gamma'/|gamma'|; the outward normal is
  n = (t_y, -t_x); curvature kappa = (x'y'' - y'x'')/|gamma'|^3;
* a refined panel splits into 2**L equal-parameter children, L = 0 leaving it
  as it is;
* unknowns are node-major, (u_x, u_y) interleaved, panels in parameter order.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


def gauss_legendre(q: int):
    """q-point Gauss-Legendre nodes and weights on [-1, 1] (NumPy's rule)."""
    s, w = np.polynomial.legendre.leggauss(q)
    return s.astype(np.float64), w.astype(np.float64)


def star_derivatives(theta, a: float, m: int):
    """gamma, gamma', gamma'' of r(theta) (cos theta, sin theta),
    r = 1 + a cos(m theta).  Each returned array has shape (..., 2)."""
    th = np.asarray(theta, dtype=np.float64)
    c, s = np.cos(th), np.sin(th)
    r = 1.0 + a * np.cos(m * th)
    r1 = -a * m * np.sin(m * th)
    r2 = -a * m * m * np.cos(m * th)
    g0 = np.stack([r * c, r * s], axis=-1)
    g1 = np.stack([r1 * c - r * s, r1 * s + r * c], axis=-1)
    g2 = np.stack([r2 * c - 2.0 * r1 * s - r * c, r2 * s + 2.0 * r1 * c - r * s], axis=-1)
    return g0, g1, g2


@dataclasses.dataclass
class Discretization:
    """Nodes, outward unit normals, unit tangents, curvature and quadrature
    weights (w = w_GL * (dtheta / 2) * |gamma'|) of a panel discretization."""

    x: np.ndarray        # (N, 2)
    normal: np.ndarray   # (N, 2)
    tangent: np.ndarray  # (N, 2)
    kappa: np.ndarray    # (N,)
    w: np.ndarray        # (N,)
    panels: np.ndarray   # (P, 2) parameter intervals

    @property
    def n(self) -> int:
        return self.x.shape[0]


def discretize(panels: np.ndarray, a: float, m: int, q: int = 16) -> Discretization:
    """Place a q-point Gauss-Legendre rule on every parameter panel."""
    panels = np.asarray(panels, dtype=np.float64).reshape(-1, 2)
    s, wq = gauss_legendre(q)
    half = 0.5 * (panels[:, 1] - panels[:, 0])
    mid = 0.5 * (panels[:, 1] + panels[:, 0])
    theta = (mid[:, None] + half[:, None] * s[None, :]).reshape(-1)
    wth = (half[:, None] * wq[None, :]).reshape(-1)
    g0, g1, g2 = star_derivatives(theta, a, m)
    speed = np.hypot(g1[:, 0], g1[:, 1])
    t = g1 / speed[:, None]
    nrm = np.stack([t[:, 1], -t[:, 0]], axis=1)
    kappa = (g1[:, 0] * g2[:, 1] - g1[:, 1] * g2[:, 0]) / speed ** 3
    return Discretization(g0, nrm, t, kappa, wth * speed, panels)


def reference_panels(n_panels: int) -> np.ndarray:
    """n_panels parameter intervals uniform on [0, 2 pi)."""
    h = 2.0 * math.pi / n_panels
    lo = np.arange(n_panels, dtype=np.float64) * h
    return np.stack([lo, lo + h], axis=1)


@dataclasses.dataclass
class RefinedSets:
    """Reference and refined discretizations plus the index sets of Sec. 3.1.

    ``ref`` holds I_o in reference order, ``new`` holds I_n in refined panel
    order.  ``k_in_ref``/``c_in_ref`` index nodes of ``ref``;
    ``k_in_new``/``p_in_new`` index nodes of ``new`` (both in parameter
    order).  Kept nodes appear in the same relative order in both.
    """

    ref: Discretization
    new: Discretization
    k_in_ref: np.ndarray
    c_in_ref: np.ndarray
    k_in_new: np.ndarray
    p_in_new: np.ndarray


def refine(n_panels: int, panel_ids, levels, a: float, m: int, q: int = 16) -> RefinedSets:
    """Replace each selected reference panel by 2**level equal-parameter
    children and return both discretizations with the index sets."""
    ref_p = reference_panels(n_panels)
    lev = {int(i): int(l) for i, l in zip(panel_ids, levels)}
    new_p, is_new = [], []
    for i in range(n_panels):
        a0, b0 = ref_p[i]
        if i in lev:
            nch = 2 ** lev[i]
            h = (b0 - a0) / nch
            for j in range(nch):
                new_p.append((a0 + j * h, a0 + (j + 1) * h))
                is_new.append(True)
        else:
            new_p.append((a0, b0))
            is_new.append(False)
    new_p = np.array(new_p, dtype=np.float64).reshape(-1, 2)
    ref = discretize(ref_p, a, m, q)
    new = discretize(new_p, a, m, q)
    cut = np.zeros(n_panels, dtype=bool)
    cut[list(lev.keys())] = True
    ref_node_cut = np.repeat(cut, q)
    new_node_added = np.repeat(np.array(is_new, dtype=bool), q)
    return RefinedSets(ref, new,
                       np.flatnonzero(~ref_node_cut), np.flatnonzero(ref_node_cut),
                       np.flatnonzero(~new_node_added), np.flatnonzero(new_node_added))


def dofs(node_idx: np.ndarray) -> np.ndarray:
    """Unknown indices (interleaved x, y) of the given nodes."""
    node_idx = np.asarray(node_idx, dtype=np.int64)
    return np.stack([2 * node_idx, 2 * node_idx + 1], axis=1).reshape(-1)
