"""Pins of the oracle's linear algebra: dense solve, ELS, Woodbury, ID, lemma.

* dense LU solve == brute-force inverse on a tiny wall;
* the ELS (Sec. 3.2) restricted to (tau_k, tau_p) == A_nn^{-1} g_n, and
  A_ext = A~ + Q with A_kk identical from either discretization;
* the Woodbury formula (eq. wood) with untruncated factors == the dense solve
  of A~ + L R; with factors truncated at eps the error is O(eps * kappa);
* the ID (Definition 3.1): P(J, :) = I, error <= c eps ||W||, exact on
  exactly low-rank input, rank close to the SVD eps-rank;
* Lemma thm:woodbury's bound holds; SVD recompression does not worsen the
  Woodbury operator (the trend of the paper's conditioning table).
"""
import numpy as np
import pytest

import workloads as W
from oracle import geometry as G, kernels as K, solve as S


@pytest.fixture(scope="module")
def small_els():
    p = W.small_problem(n_panels=12, ids=(3, 4), levels=(2, 1), seed=2)
    sets = G.refine(p.n_panels, p.refinement.panel_ids, p.refinement.levels, 0.3, 5)
    E = S.els(sets)
    g = K.rhs_vector(sets.new, p.rhs[0].z, p.rhs[0].f)
    kn, pn = G.dofs(sets.k_in_new), G.dofs(sets.p_in_new)
    return sets, E, g, kn, pn


def test_dense_solve_matches_bruteforce_inverse():
    d = G.discretize(G.reference_panels(8), 0.3, 5)
    A = K.nystrom_matrix(d)
    g = np.random.default_rng(0).standard_normal(2 * d.n)
    x = S.solve_refined(A, g)
    assert np.linalg.norm(A @ x - g) / (np.linalg.norm(A, 2) * np.linalg.norm(x)) < 1e-15
    assert np.allclose(x, np.linalg.inv(A) @ g, rtol=1e-12, atol=1e-13)


def test_els_equivalent_to_refined_system(small_els):
    sets, E, g, kn, pn = small_els
    assert np.array_equal(E.A_kk_from_ref, E.A_kk_from_new)
    assert np.array_equal(E.A_ext, E.A_tilde + E.Q)
    tau = S.solve_refined(K.nystrom_matrix(sets.new), g)
    te = np.linalg.solve(E.A_ext, E.g_ext(g[kn], g[pn]))
    assert np.allclose(te[:E.nk], tau[kn], atol=1e-12)
    assert np.allclose(te[E.nk + E.nc:], tau[pn], atol=1e-12)
    # Q has exactly the three non-zero blocks of the ELS
    assert not np.any(E.Q[E.nk:E.nk + E.nc])
    assert not np.any(E.Q[:E.nk, :E.nk]) and not np.any(E.Q[E.nk + E.nc:, E.nk:])


def test_woodbury_exact_with_untruncated_factors(small_els):
    sets, E, g, kn, pn = small_els
    F = S.block_svd_factors(E, eps=0.0)
    assert np.allclose(F.L @ F.R, E.Q, atol=1e-13)
    ge = E.g_ext(g[kn], g[pn])
    tw = S.woodbury_solve(lambda b: np.linalg.solve(E.A_tilde, b), F.L, F.R, ge)
    td = np.linalg.solve(E.A_tilde + F.L @ F.R, ge)
    assert np.linalg.norm(tw - td) / np.linalg.norm(td) < 1e-11


@pytest.mark.parametrize("factor", ["block_svd", "optimal_svd", "block_id", "two_step"])
def test_woodbury_truncated_error_is_eps_kappa(small_els, factor):
    sets, E, g, kn, pn = small_els
    eps = 1e-10
    F = getattr(S, factor + "_factors")(E, eps)
    ge = E.g_ext(g[kn], g[pn])
    tw = S.woodbury_solve(lambda b: np.linalg.solve(E.A_tilde, b), F.L, F.R, ge)
    te = np.linalg.solve(E.A_ext, ge)
    kappa = np.linalg.cond(E.A_ext)
    assert np.linalg.norm(tw - te) / np.linalg.norm(te) < 100 * eps * kappa
    assert np.linalg.norm(F.L @ F.R - E.Q) < 100 * eps * np.linalg.norm(E.Q) * max(1, F.k)


def test_row_id_definition():
    rng = np.random.default_rng(5)
    # exactly rank-7 matrix: ID is exact and finds rank 7
    M = rng.standard_normal((60, 7)) @ rng.standard_normal((7, 40))
    rid = S.row_id(M, 1e-12)
    assert rid.k == 7
    assert np.array_equal(rid.P[rid.J], np.eye(7))
    assert np.linalg.norm(M - rid.P @ M[rid.J]) < 1e-12 * np.linalg.norm(M)
    # numerically low-rank kernel block: error <= c eps ||W|| and rank near SVD rank
    d = G.discretize(G.reference_panels(32), 0.3, 5)
    A = K.nystrom_matrix(d)
    B = A[:64, 256:]
    for eps in (1e-6, 1e-10):
        rid = S.row_id(B, eps)
        err = np.linalg.norm(B - rid.P @ B[rid.J], 2)
        assert err <= 50 * eps * np.linalg.norm(B, 2)
        sv = np.linalg.svd(B, compute_uv=False)
        ksvd = int(np.sum(sv > eps * sv[0]))
        assert ksvd <= rid.k <= int(1.5 * ksvd) + 3
        assert np.max(np.abs(rid.P)) < 10.0


def test_lemma_bound_and_recompression_trend(small_els):
    sets, E, g, kn, pn = small_els
    eps = 1e-10
    Fb = S.block_svd_factors(E, eps)
    Fo = S.optimal_svd_factors(E, eps)
    for F in (Fb, Fo):
        kW = np.linalg.cond(S.woodbury_operator(E.A_tilde, F.L, F.R))
        assert kW <= S.lemma_bound(E.A_tilde, F.L, F.R) * (1 + 1e-8)
    assert Fo.k <= Fb.k
    kb = np.linalg.cond(S.woodbury_operator(E.A_tilde, Fb.L, Fb.R))
    ko = np.linalg.cond(S.woodbury_operator(E.A_tilde, Fo.L, Fo.R))
    assert ko <= 1.05 * kb


def test_two_step_recompression_reduces_rank(small_els):
    sets, E, g, kn, pn = small_els
    F1 = S.block_id_factors(E, 1e-10)
    F2 = S.two_step_factors(E, 1e-10)
    assert F2.k <= F1.k
    # the final factors keep the uniform ID format: L has an identity block
    rid_rows = np.flatnonzero(np.all(np.isin(F2.L, [0.0, 1.0]), axis=1) & (np.abs(F2.L).sum(1) == 1))
    assert rid_rows.size >= F2.k


def test_no_refinement_means_empty_update():
    p = W.small_problem(n_panels=8, ids=(), levels=())
    sets = G.refine(8, [], [], 0.3, 5)
    E = S.els(sets)
    assert E.nc == 0 and E.np_ == 0 and not np.any(E.Q)
    assert S.block_id_factors(E, 1e-10).k == 0
