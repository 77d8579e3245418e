"""Pins of the oracle's discretization against closed forms (CPU only).

Each check uses a formula independent of the one in ``oracle/geometry.py``:
the polar-curve arc-length and curvature formulas, the unit circle, exact
polynomial integration, and the Sec. 3.1 index-set bookkeeping.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle import geometry as G


def test_gauss_legendre_exact_to_degree_31():
    s, w = G.gauss_legendre(16)
    for k in range(32):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * s ** k) - exact) < 1e-14
    # degree 32 is not integrated exactly (the rule really has 16 points)
    assert abs(np.sum(w * s ** 32) - 2.0 / 33) > 1e-11


def test_gauss_legendre_small_rules_closed_form():
    s, w = G.gauss_legendre(2)
    assert np.allclose(np.sort(s), [-1 / math.sqrt(3), 1 / math.sqrt(3)], atol=1e-15)
    assert np.allclose(w, [1.0, 1.0], atol=1e-15)
    s, w = G.gauss_legendre(3)
    o = np.argsort(s)
    assert np.allclose(s[o], [-math.sqrt(0.6), 0.0, math.sqrt(0.6)], atol=1e-15)
    assert np.allclose(w[o], [5 / 9, 8 / 9, 5 / 9], atol=1e-15)


def test_circle_geometry():
    d = G.discretize(G.reference_panels(12), a=0.0, m=5)
    r = np.linalg.norm(d.x, axis=1)
    assert np.allclose(r, 1.0, atol=1e-15)
    assert np.allclose(d.normal, d.x, atol=1e-14)          # outward
    assert np.allclose(d.tangent, np.stack([-d.x[:, 1], d.x[:, 0]], 1), atol=1e-14)
    assert np.allclose(d.kappa, 1.0, atol=1e-13)
    assert abs(d.w.sum() - 2 * math.pi) < 1e-13


def _polar(theta, a, m):
    r = 1 + a * np.cos(m * theta)
    r1 = -a * m * np.sin(m * theta)
    r2 = -a * m * m * np.cos(m * theta)
    return r, r1, r2


def test_star_weights_sum_to_perimeter_and_curvature_polar_formula():
    a, m = 0.3, 5
    d = G.discretize(G.reference_panels(64), a, m)
    per, _ = integrate.quad(lambda t: math.hypot(*_polar(t, a, m)[:2]), 0, 2 * math.pi,
                            limit=400, epsabs=1e-14, epsrel=1e-14)
    assert abs(d.w.sum() - per) < 1e-12 * per
    theta = np.arctan2(d.x[:, 1], d.x[:, 0])
    r, r1, r2 = _polar(theta, a, m)
    kap = (r * r + 2 * r1 * r1 - r * r2) / (r * r + r1 * r1) ** 1.5
    assert np.allclose(d.kappa, kap, rtol=1e-12, atol=1e-12)
    assert np.allclose(np.linalg.norm(d.x, axis=1), r, atol=1e-14)


def test_star_normals_outward_and_orthogonal_to_chord():
    d = G.discretize(G.reference_panels(32), 0.3, 5)
    assert np.all(np.sum(d.normal * d.x, axis=1) > 0)       # star-shaped about 0
    assert np.allclose(np.linalg.norm(d.normal, axis=1), 1.0, atol=1e-15)
    # central-difference tangent along the curve is perpendicular to n
    h = 1e-6
    th = np.linspace(0.1, 6.0, 7)
    p_plus = W.Curve().point(th + h)
    p_minus = W.Curve().point(th - h)
    t_fd = (p_plus - p_minus)
    t_fd /= np.linalg.norm(t_fd, axis=1, keepdims=True)
    g0, g1, _ = G.star_derivatives(th, 0.3, 5)
    n = np.stack([g1[:, 1], -g1[:, 0]], 1) / np.linalg.norm(g1, axis=1, keepdims=True)
    assert np.max(np.abs(np.sum(t_fd * n, axis=1))) < 1e-8


def test_refinement_index_sets_config1():
    p = W.config1()
    s = G.refine(p.n_panels, p.refinement.panel_ids, p.refinement.levels, 0.3, 5)
    assert (s.k_in_ref.size, s.c_in_ref.size, s.p_in_new.size) == (960, 64, 512)
    assert s.new.n == 1472
    # kept nodes are the same points with the same weights, same order
    assert np.array_equal(s.ref.x[s.k_in_ref], s.new.x[s.k_in_new])
    assert np.array_equal(s.ref.w[s.k_in_ref], s.new.w[s.k_in_new])
    # added nodes discretize the same arc as the cut nodes
    assert abs(s.ref.w[s.c_in_ref].sum() - s.new.w[s.p_in_new].sum()) < 1e-13
    # and are strictly inside the cut panels' parameter range
    th = np.mod(np.arctan2(s.new.x[s.p_in_new, 1], s.new.x[s.p_in_new, 0]), 2 * math.pi)
    ids = np.array(p.refinement.panel_ids)
    h = 2 * math.pi / p.n_panels
    assert th.min() > ids.min() * h and th.max() < (ids.max() + 1) * h


def test_refinement_level_zero_is_identity():
    s = G.refine(16, [2, 9], [0, 0], 0.3, 5)
    assert np.array_equal(s.ref.x, s.new.x)
    assert np.array_equal(s.c_in_ref, s.p_in_new)


def test_workload_panel_selection_contiguous_and_nearest():
    p = W.config2()
    ids = np.array(p.refinement.panel_ids)
    assert ids.size == 16
    gaps = np.diff(ids) % p.n_panels
    assert np.all((gaps == 1)) or sorted(set(gaps)) == [1, p.n_panels - 15]
    assert W.contiguous_panels(10, 0.05, 4) in ([9, 0, 1, 2], [0, 1, 2, 9])
