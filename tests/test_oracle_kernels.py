"""Pins of the oracle's Nystrom operator and right-hand side (CPU only).

Pins: the double-layer Gauss identity (-1/2 I on the curve, -I inside, 0
outside), the circle closed form of D, the rank-1 nullspace of -1/2 I + D
that N removes (remark after eq. interior_BIE_discretized), zero flux of
Stokeslet data (consistency condition of Sec. 2.1), incompressibility of the
Stokeslet field, and the paper's own accuracy measure: the interior velocity
of the solved density reproduces the exterior-Stokeslet flow.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import geometry as G, kernels as K, solve as S


@pytest.fixture(scope="module")
def star64():
    return G.discretize(G.reference_panels(64), 0.3, 5)


def test_gauss_identity_on_curve_inside_outside(star64):
    d = star64
    Dm = K.dlp_only_matrix(d) + 0.5 * np.eye(2 * d.n)
    rowsum = Dm.reshape(d.n, 2, d.n, 2).sum(axis=2)
    assert np.max(np.abs(rowsum + 0.5 * np.eye(2))) < 1e-11
    inside = np.array([[0.0, 0.0], [0.5, 0.2], [-0.6, -0.3]])
    outside = np.array([[2.0, 0.0], [0.0, -1.7], [1.2, 1.2]])
    for pts, val in ((inside, -1.0), (outside, 0.0)):
        s = K.dlp_block(pts, d.x, d.normal, d.w).reshape(len(pts), 2, d.n, 2).sum(axis=2)
        assert np.max(np.abs(s - val * np.eye(2))) < 1e-12


def test_circle_closed_form():
    R = 1.0
    d = G.discretize(G.reference_panels(6), 0.0, 5)
    Dm = K.dlp_only_matrix(d) + 0.5 * np.eye(2 * d.n)
    blocks = Dm.reshape(d.n, 2, d.n, 2).transpose(0, 2, 1, 3)
    for i in (0, 7, 40):
        for j in (0, 3, 41, 90):
            if i == j:
                t = np.array([-d.x[i, 1], d.x[i, 0]])
                ref = -(1 / (2 * math.pi * R)) * np.outer(t, t)
            else:
                rhat = (d.x[i] - d.x[j]) / np.linalg.norm(d.x[i] - d.x[j])
                ref = -(1 / (2 * math.pi * R)) * np.outer(rhat, rhat)
            assert np.allclose(blocks[i, j], ref * d.w[j], atol=1e-15, rtol=1e-13)


def test_nullspace_removed_by_N(star64):
    d = star64
    s0 = np.linalg.svd(K.dlp_only_matrix(d), compute_uv=False)
    assert s0[-1] / s0[0] < 1e-13          # rank-1 deficient without N
    assert s0[-2] / s0[0] > 1e-3
    s1 = np.linalg.svd(K.nystrom_matrix(d), compute_uv=False)
    assert s1[-1] / s1[0] > 1e-3           # well conditioned with N
    # the N term is exactly w_j n_i n_j^T
    Nm = K.nystrom_matrix(d) - K.dlp_only_matrix(d)
    assert np.allclose(Nm[2 * 5:2 * 5 + 2, 2 * 9:2 * 9 + 2],
                       d.w[9] * np.outer(d.normal[5], d.normal[9]), atol=1e-16)


def test_stokeslet_data_zero_flux_and_divergence_free(star64):
    rng = np.random.default_rng(3)
    st = W.stokeslets(rng, 8)
    g = K.rhs_vector(star64, st.z, st.f).reshape(-1, 2)
    assert abs(np.sum(g * star64.normal * star64.w[:, None])) < 1e-13
    x = np.array([[0.3, -0.2], [0.1, 0.4]])
    h = 1e-5
    div = (K.stokeslet_velocity(x + [h, 0], st.z, st.f)[:, 0] - K.stokeslet_velocity(x - [h, 0], st.z, st.f)[:, 0]
           + K.stokeslet_velocity(x + [0, h], st.z, st.f)[:, 1] - K.stokeslet_velocity(x - [0, h], st.z, st.f)[:, 1]) / (2 * h)
    assert np.max(np.abs(div)) < 1e-8


@pytest.mark.parametrize("refined", [False, True])
def test_interior_velocity_reproduces_exterior_stokeslets(refined):
    p = W.config1(seed=4)
    s = G.refine(p.n_panels, p.refinement.panel_ids, p.refinement.levels, 0.3, 5)
    d = s.new if refined else s.ref
    st = p.rhs[0]
    g = K.rhs_vector(d, st.z, st.f)
    tau = S.solve_refined(K.nystrom_matrix(d), g)
    # the solution carries no flux (N tau = 0), so u = D tau solves the BVP
    assert abs(np.sum(tau.reshape(-1, 2) * d.normal * d.w[:, None])) < 1e-12
    tg = np.array([[0.0, 0.0], [0.3, 0.1], [-0.2, -0.35], [0.1, 0.38]])
    u = K.interior_velocity(tg, d, tau)
    ue = K.stokeslet_velocity(tg, st.z, st.f)
    assert np.max(np.abs(u - ue)) < 1e-12 * np.max(np.abs(ue))


def test_spectral_convergence_with_panels():
    rng = np.random.default_rng(7)
    st = W.stokeslets(rng, 4, radius=1.6)
    tg = np.array([[0.2, 0.1], [-0.4, 0.2]])
    errs = []
    for P in (8, 16, 32):
        d = G.discretize(G.reference_panels(P), 0.3, 5)
        tau = S.solve_refined(K.nystrom_matrix(d), K.rhs_vector(d, st.z, st.f))
        errs.append(np.max(np.abs(K.interior_velocity(tg, d, tau) - K.stokeslet_velocity(tg, st.z, st.f))))
    assert errs[1] < 0.1 * errs[0] and errs[2] < max(0.1 * errs[1], 1e-13)


def test_nystrom_rows_match_full_matrix(star64):
    A = K.nystrom_matrix(star64)
    rows = np.array([0, 17, 500, 1023])
    sub = K.nystrom_rows(star64, rows)
    idx = np.stack([2 * rows, 2 * rows + 1], 1).reshape(-1)
    assert np.array_equal(sub, A[idx])


def test_residual_rows_closed_forms():
    """residual_rows(rows, tau, g) = g - A tau on the given rows, pinned by
    closed forms of the operator (not by re-forming the same rows):
    * rigid motions v (a constant vector, the rotation (-y, x)): the
      double-layer kernel is the Stokeslet's stress, which a rigid motion
      does not feel, so D v = -1/2 v on the curve; N v = n int v.n ds = 0
      (zero flux); hence A v = -v and the residual is g + v;
    * on a circle of radius R the normal field spans the nullspace of
      -1/2 I + D and N n = n int |n|^2 ds = 2 pi R n, so the residual is
      g - 2 pi R n.
    The rows are unsorted and span several 512-row chunks; g is random, so a
    wrong gather of g, a dropped term, a sign error or a transposed operand
    fails."""
    d = G.discretize(G.reference_panels(96), 0.3, 5)
    rng = np.random.default_rng(5)
    rows = rng.permutation(d.n)[:1100]
    g = rng.standard_normal(2 * d.n)
    gr = g.reshape(-1, 2)[rows]
    c = np.array([0.7, -1.3])
    r_c = K.residual_rows(d, rows, np.tile(c, d.n), g).reshape(-1, 2)
    assert np.max(np.abs(r_c - (gr + c))) < 1e-11
    rot = np.stack([-d.x[:, 1], d.x[:, 0]], axis=1)
    r_rot = K.residual_rows(d, rows, rot.reshape(-1), g).reshape(-1, 2)
    assert np.max(np.abs(r_rot - (gr + rot[rows]))) < 1e-11
    R = 1.0
    dc = G.discretize(G.reference_panels(12), 0.0, 5)
    gc = rng.standard_normal(2 * dc.n)
    rc_rows = rng.permutation(dc.n)[:150]
    r_n = K.residual_rows(dc, rc_rows, dc.normal.reshape(-1), gc).reshape(-1, 2)
    assert np.max(np.abs(r_n - (gc.reshape(-1, 2)[rc_rows] - 2 * math.pi * R * dc.normal[rc_rows]))) < 1e-12
    # and the residual of the dense solution vanishes on the same rows
    tau = S.solve_refined(K.nystrom_matrix(d), g)
    assert np.max(np.abs(K.residual_rows(d, rows, tau, g))) < 1e-12 * np.max(np.abs(g))
