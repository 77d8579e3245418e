"""Oracle linear algebra: dense refined solve, ELS, Woodbury, ID, SVD factors.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``solve_refined``: tau_n = A_nn^{-1} g_n by dense LU (LAPACK through
  scipy) plus one step of iterative refinement on the same factors.  This is the plain definition the fast method reaches
  to within its compression tolerance (Sec. 3.2: the ELS is equivalent to the
  refined system).
* ``els``: the extended linear system of Sec. 3.2 (eq.
  extendedlLinearSystem), its splitting A_ext = A~ + Q, and the right-hand
  side g_ext = (g_k; 0; g_p), all in the block order [k; c; p].
* ``woodbury_solve``: eq. (wood) with dense factors L, R.
* ``row_id``: the interpolative decomposition of Definition 3.1 (rows),
  computed from a column-pivoted QR (a library primitive).
* ``block_id_factors`` / ``two_step_factors``: the block ID factorization of
  Q (eqs. block_lr and QeqLR, with the uniform row-ID format of the remark in
  Sec. 3.3) followed by the random-sampling row-ID recompression of L_1
  described in Sec. 3.4.
* ``block_svd_factors`` / ``optimal_svd_factors``: eq. (uniform_concat) and
  its SVD recompression (Sec. 3.4), used as small-size references.
* ``lemma_bound``: the right side of Lemma thm:woodbury.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from .geometry import RefinedSets, dofs
from .kernels import nystrom_matrix


def solve_refined(A_nn: np.ndarray, g_n: np.ndarray, refine_steps: int = 1) -> np.ndarray:
    """tau_n = A_nn^{-1} g_n: LU with partial pivoting (LAPACK getrf/getrs
    through scipy), then ``refine_steps`` steps of iterative refinement with
    the same factors (tau += LU^{-1} (g - A tau), residual in FP64).

    The refinement only brings the computed tau to the definition: at
    n ~ 4e4 unknowns the plain LU solve leaves a backward error of about
    1e-12 (a few n eps), which kappa ~ 4e2 could turn into an error near the
    1e-10 parity bar; one step takes it to a few eps."""
    lu = sla.lu_factor(A_nn, check_finite=False)
    tau = sla.lu_solve(lu, g_n, check_finite=False)
    for _ in range(refine_steps):
        tau = tau + sla.lu_solve(lu, g_n - A_nn @ tau, check_finite=False)
    return tau


@dataclasses.dataclass
class ELS:
    """Blocks of the extended linear system in the order [k; c; p] (dofs)."""

    A_ext: np.ndarray
    A_tilde: np.ndarray
    Q: np.ndarray
    nk: int   # number of k unknowns (2 N_k)
    nc: int
    np_: int
    A_kk_from_ref: np.ndarray
    A_kk_from_new: np.ndarray

    def g_ext(self, g_k: np.ndarray, g_p: np.ndarray) -> np.ndarray:
        shape = (self.nc,) + g_k.shape[1:]
        return np.concatenate([g_k, np.zeros(shape), g_p], axis=0)


def els(sets: RefinedSets, A_oo: np.ndarray = None, A_nn: np.ndarray = None) -> ELS:
    """Assemble the ELS from the reference and refined Nystrom matrices."""
    if A_oo is None:
        A_oo = nystrom_matrix(sets.ref)
    if A_nn is None:
        A_nn = nystrom_matrix(sets.new)
    k_o, c_o = dofs(sets.k_in_ref), dofs(sets.c_in_ref)
    k_n, p_n = dofs(sets.k_in_new), dofs(sets.p_in_new)
    nk, nc, npp = k_o.size, c_o.size, p_n.size
    A_kk = A_oo[np.ix_(k_o, k_o)]
    A_kc = A_oo[np.ix_(k_o, c_o)]
    A_ck = A_oo[np.ix_(c_o, k_o)]
    A_cc = A_oo[np.ix_(c_o, c_o)]
    A_kp = A_nn[np.ix_(k_n, p_n)]
    A_pk = A_nn[np.ix_(p_n, k_n)]
    A_pp = A_nn[np.ix_(p_n, p_n)]
    Z = np.zeros
    A_ext = np.block([[A_kk, Z((nk, nc)), A_kp],
                      [A_ck, A_cc, Z((nc, npp))],
                      [A_pk, Z((npp, nc)), A_pp]])
    A_tilde = np.block([[A_kk, A_kc, Z((nk, npp))],
                        [A_ck, A_cc, Z((nc, npp))],
                        [Z((npp, nk)), Z((npp, nc)), A_pp]])
    Q = np.block([[Z((nk, nk)), -A_kc, A_kp],
                  [Z((nc, nk)), Z((nc, nc)), Z((nc, npp))],
                  [A_pk, Z((npp, nc)), Z((npp, npp))]])
    return ELS(A_ext, A_tilde, Q, nk, nc, npp, A_kk, A_nn[np.ix_(k_n, k_n)])


def woodbury_solve(A_tilde_inv, L: np.ndarray, R: np.ndarray, g_ext: np.ndarray) -> np.ndarray:
    """tau_ext = A~^{-1} g - A~^{-1} L (I + R A~^{-1} L)^{-1} R A~^{-1} g.

    ``A_tilde_inv`` is a callable applying A~^{-1} to a block of columns."""
    y = A_tilde_inv(g_ext)
    X = A_tilde_inv(L)
    W = np.eye(L.shape[1]) + R @ X
    return y - X @ np.linalg.solve(W, R @ y)


def woodbury_operator(A_tilde: np.ndarray, L: np.ndarray, R: np.ndarray) -> np.ndarray:
    """W = I + R A~^{-1} L (the Woodbury operator of Sec. 3.4)."""
    return np.eye(L.shape[1]) + R @ np.linalg.solve(A_tilde, L)


@dataclasses.dataclass
class RowID:
    """W ~= P W(J, :), P(J, :) = I (Definition 3.1)."""

    P: np.ndarray
    J: np.ndarray

    @property
    def k(self) -> int:
        return self.J.size


def row_id(W: np.ndarray, eps: float, k: int = None) -> RowID:
    """Row interpolative decomposition of W at relative tolerance ``eps``.

    Pivoted QR of W^T orders the rows; the rank k is the number of diagonal
    entries of R above eps*|R_11| (unless ``k`` is given); the interpolation
    block is T = R11^{-1} R12 so that W(rest, :) ~= T^T W(J, :)."""
    m = W.shape[0]
    if m == 0 or not np.any(W):
        return RowID(np.zeros((m, 0)), np.zeros(0, dtype=np.int64))
    Qf, Rf, piv = sla.qr(W.T, mode="economic", pivoting=True)
    d = np.abs(np.diag(Rf))
    if k is None:
        k = int(np.sum(d > eps * d[0]))
    k = max(0, min(k, d.size))
    J = piv[:k]
    T = sla.solve_triangular(Rf[:k, :k], Rf[:k, k:])
    P = np.zeros((m, k))
    P[J, :] = np.eye(k)
    P[piv[k:], :] = T.T
    return RowID(P, J)


@dataclasses.dataclass
class Factors:
    """Q ~= L R with L of size (2 N_ext, k) and R of size (k, 2 N_ext)."""

    L: np.ndarray
    R: np.ndarray

    @property
    def k(self) -> int:
        return self.L.shape[1]


def _embed(rows_total, r0, blockL):
    out = np.zeros((rows_total, blockL.shape[1]))
    out[r0:r0 + blockL.shape[0]] = blockL
    return out


def block_id_factors(E: ELS, eps: float) -> Factors:
    """First step of Sec. 3.3/3.4: row IDs of A_pk, A_kc, A_kp separately,
    L_1 = interpolation matrices, R_1 = skeleton rows (eq. QeqLR, uniform
    row-ID format of the remark closing Sec. 3.3)."""
    nk, nc, npp = E.nk, E.nc, E.np_
    n = nk + nc + npp
    A_kc = -E.Q[:nk, nk:nk + nc]
    A_kp = E.Q[:nk, nk + nc:]
    A_pk = E.Q[nk + nc:, :nk]
    Ls, Rs = [], []
    # A_pk block: rows p, columns k
    idp = row_id(A_pk, eps)
    Ls.append(_embed(n, nk + nc, idp.P))
    R = np.zeros((idp.k, n)); R[:, :nk] = A_pk[idp.J]; Rs.append(R)
    # -A_kc block: rows k, columns c
    idc = row_id(A_kc, eps)
    Ls.append(_embed(n, 0, -idc.P))
    R = np.zeros((idc.k, n)); R[:, nk:nk + nc] = A_kc[idc.J]; Rs.append(R)
    # A_kp block: rows k, columns p
    idk = row_id(A_kp, eps)
    Ls.append(_embed(n, 0, idk.P))
    R = np.zeros((idk.k, n)); R[:, nk + nc:] = A_kp[idk.J]; Rs.append(R)
    return Factors(np.concatenate(Ls, axis=1), np.concatenate(Rs, axis=0))


def two_step_factors(E: ELS, eps: float, oversample: int = 10, seed: int = 0) -> Factors:
    """Sec. 3.4's two-step construction: block ID factors (L_1, R_1), then a
    random-sampling row ID of L_1, L_1 ~= P L_1(J, :), giving L = P and
    R = L_1(J, :) R_1.  The sketch is L_1 times a Gaussian matrix."""
    F1 = block_id_factors(E, eps)
    k1 = F1.k
    if k1 == 0:
        return F1
    rng = np.random.Generator(np.random.PCG64(seed))
    Om = rng.standard_normal((k1, min(k1, k1 + oversample)))
    Y = F1.L @ Om
    rid = row_id(Y, eps)
    return Factors(rid.P, F1.L[rid.J] @ F1.R)


def _tsvd(M: np.ndarray, eps: float):
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    if s.size == 0 or s[0] == 0.0:
        return U[:, :0], s[:0], Vt[:0]
    k = int(np.sum(s > eps * s[0]))
    return U[:, :k], s[:k], Vt[:k]


def block_svd_factors(E: ELS, eps: float) -> Factors:
    """eq. (uniform_concat): truncated SVDs of A_pk, A_kc, A_kp with
    L_block = [0, -U_kc, U_kp; 0 0 0; U_pk 0 0] and
    R_block = blkdiag(S V^T) placed on the matching column blocks."""
    nk, nc, npp = E.nk, E.nc, E.np_
    n = nk + nc + npp
    A_kc = -E.Q[:nk, nk:nk + nc]
    A_kp = E.Q[:nk, nk + nc:]
    A_pk = E.Q[nk + nc:, :nk]
    Ls, Rs = [], []
    U, s, Vt = _tsvd(A_pk, eps)
    Ls.append(_embed(n, nk + nc, U)); R = np.zeros((s.size, n)); R[:, :nk] = s[:, None] * Vt; Rs.append(R)
    U, s, Vt = _tsvd(A_kc, eps)
    Ls.append(_embed(n, 0, -U)); R = np.zeros((s.size, n)); R[:, nk:nk + nc] = s[:, None] * Vt; Rs.append(R)
    U, s, Vt = _tsvd(A_kp, eps)
    Ls.append(_embed(n, 0, U)); R = np.zeros((s.size, n)); R[:, nk + nc:] = s[:, None] * Vt; Rs.append(R)
    return Factors(np.concatenate(Ls, axis=1), np.concatenate(Rs, axis=0))


def optimal_svd_factors(E: ELS, eps: float) -> Factors:
    """SVD recompression of L_block (Sec. 3.4): L = U_block,
    R = S_block V_block^T R_block."""
    Fb = block_svd_factors(E, eps)
    U, s, Vt = _tsvd(Fb.L, eps)
    return Factors(U, (s[:, None] * Vt) @ Fb.R)


def pinv_cond(M: np.ndarray, rows: bool) -> float:
    """kappa-hat of the lemma: ||M^+|| ||M|| with the one-sided pseudo-inverse
    (columns independent for L, rows independent for R)."""
    if rows:
        Mp = M.T @ np.linalg.inv(M @ M.T)
    else:
        Mp = np.linalg.inv(M.T @ M) @ M.T
    return np.linalg.norm(Mp, 2) * np.linalg.norm(M, 2)


def lemma_bound(A_tilde: np.ndarray, L: np.ndarray, R: np.ndarray) -> float:
    """min(kappa(L)^2, kappa(R)^2) kappa(A~ + L R) kappa(A~)."""
    a2 = min(pinv_cond(L, rows=False) ** 2, pinv_cond(R, rows=True) ** 2)
    return a2 * np.linalg.cond(A_tilde + L @ R) * np.linalg.cond(A_tilde)
