"""Oracle kernels: Stokeslet, Stokes double layer, dense Nystrom assembly.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 2 of the paper:
* Stokeslet (eq. stokeslet): S_ij(x, y) = (1/(4 pi mu)) (delta_ij log(1/r)
  + r_i r_j / r^2), r = x - y; viscosity mu = 1 (the paper leaves it free;
  it only scales data and solution together);
* double layer: D_ij(x, y) = (1/pi) (r_i r_j / r^2) (r . n_y / r^2);
* nullspace correction (eq. null): (N tau)(x) = n_x int tau . n_y ds_y;
* interior system (eq. interior_BIE_discretized2): (-1/2 I + D + N) tau = g.

Nystrom entries (2x2 block for target node i, source node j):
    A[i, j] = -1/2 delta_ij I + w_j (D(x_i, y_j) + n_i n_j^T)
with the diagonal of D replaced by its on-curve limit
    D(x_i, x_i) = -(kappa_i / (2 pi)) t_i t_i^T
(the paper does not state it; it follows from expanding the curve to second
order about x_i).  The double layer is smooth on a smooth curve, so the plain
Gauss rule needs no singular correction.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import Discretization


def stokeslet_velocity(x: np.ndarray, z: np.ndarray, f: np.ndarray) -> np.ndarray:
    """u(x) = sum_m S(x, z_m) f_m at targets x (M, 2); returns (M, 2)."""
    x = np.asarray(x, np.float64)
    u = np.zeros_like(x)
    for zm, fm in zip(np.asarray(z, np.float64), np.asarray(f, np.float64)):
        r = x - zm[None, :]
        r2 = np.sum(r * r, axis=1)
        rf = r @ fm
        u += (1.0 / (4.0 * math.pi)) * (-0.5 * np.log(r2)[:, None] * fm[None, :]
                                         + (rf / r2)[:, None] * r)
    return u


def rhs_vector(disc: Discretization, z, f) -> np.ndarray:
    """Boundary data g at the nodes, interleaved (2N,)."""
    return stokeslet_velocity(disc.x, z, f).reshape(-1)


def dlp_block(xt: np.ndarray, ys: np.ndarray, ny: np.ndarray, wy: np.ndarray) -> np.ndarray:
    """Dense (2M, 2N) matrix of w_j D(x_i, y_j) for well-separated x != y."""
    r = xt[:, None, :] - ys[None, :, :]                     # (M, N, 2)
    r2 = np.sum(r * r, axis=2)
    rn = np.sum(r * ny[None, :, :], axis=2)
    c = (rn / (math.pi * r2 * r2)) * wy[None, :]
    blk = c[:, :, None, None] * r[:, :, :, None] * r[:, :, None, :]  # (M, N, 2, 2)
    return blk.transpose(0, 2, 1, 3).reshape(2 * xt.shape[0], 2 * ys.shape[0])


def nystrom_rows(disc: Discretization, rows: np.ndarray) -> np.ndarray:
    """Rows of A = -1/2 I + D + N for target nodes ``rows`` (all columns).

    Returns (2 len(rows), 2N)."""
    rows = np.asarray(rows, dtype=np.int64)
    M, N = rows.size, disc.n
    xt = disc.x[rows]
    r = xt[:, None, :] - disc.x[None, :, :]
    r2 = np.sum(r * r, axis=2)
    self_mask = (rows[:, None] == np.arange(N)[None, :])
    r2 = np.where(self_mask, 1.0, r2)
    rn = np.sum(r * disc.normal[None, :, :], axis=2)
    c = (rn / (math.pi * r2 * r2)) * disc.w[None, :]
    blk = c[:, :, None, None] * r[:, :, :, None] * r[:, :, None, :]
    # on-curve limit of D on the diagonal
    ii = np.flatnonzero(self_mask.any(axis=1))
    jj = rows[ii]
    t = disc.tangent[jj]
    blk[ii, jj] = (-(disc.kappa[jj] / (2.0 * math.pi)) * disc.w[jj])[:, None, None] * \
        (t[:, :, None] * t[:, None, :])
    # nullspace term  w_j n_i n_j^T
    blk += disc.w[None, :, None, None] * disc.normal[rows][:, None, :, None] * \
        disc.normal[None, :, None, :]
    blk[ii, jj] += -0.5 * np.eye(2)[None, :, :]
    return blk.transpose(0, 2, 1, 3).reshape(2 * M, 2 * N)


def nystrom_matrix(disc: Discretization, chunk: int = 2048) -> np.ndarray:
    """Dense 2N x 2N Nystrom matrix of -1/2 I + D + N, assembled in row chunks."""
    N = disc.n
    A = np.empty((2 * N, 2 * N), dtype=np.float64)
    for s in range(0, N, chunk):
        e = min(N, s + chunk)
        A[2 * s:2 * e] = nystrom_rows(disc, np.arange(s, e))
    return A


def dlp_only_matrix(disc: Discretization) -> np.ndarray:
    """Dense -1/2 I + D without the nullspace term (for the nullspace pin)."""
    A = nystrom_matrix(disc)
    nv = disc.normal.reshape(-1)
    wv = np.repeat(disc.w, 2)
    return A - np.outer(nv, nv * wv)


def interior_velocity(targets: np.ndarray, disc: Discretization, tau: np.ndarray) -> np.ndarray:
    """u(x) = sum_j w_j D(x, y_j) tau_j at off-curve targets; returns (M, 2)."""
    K = dlp_block(np.asarray(targets, np.float64), disc.x, disc.normal, disc.w)
    return (K @ np.asarray(tau, np.float64).reshape(-1)).reshape(-1, 2)


def residual_rows(disc: Discretization, rows: np.ndarray, tau: np.ndarray, g: np.ndarray) -> np.ndarray:
    """g - A tau restricted to target nodes ``rows`` (matrix-free in the sense
    that only those rows of A are ever formed)."""
    rows = np.asarray(rows, dtype=np.int64)
    out = np.empty(2 * rows.size)
    for s in range(0, rows.size, 512):
        blk = rows[s:s + 512]
        out[2 * s:2 * s + 2 * blk.size] = g.reshape(-1)[np.stack([2 * blk, 2 * blk + 1], 1).reshape(-1)] \
            - nystrom_rows(disc, blk) @ tau.reshape(-1)
    return out
