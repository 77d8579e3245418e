"""The far-field expansions behind the Q sketches (Sec. 3.3, Fig. 3).

The sketch of Q's far part is the product A(far, sources) Omega evaluated
through expansions about the centre c of a circle of radius rho around the
refined arc, instead of entry by entry.  This checks that reading of the
double-layer block on the CPU, in FP64, against the oracle's direct entries:

  D mu = (w / 4 pi) [nu mu / r + 2 Re(conj(nu) mu) / conj(r)
                     + r conj(nu) conj(mu) / conj(r)^2],   r = z - tau,
  N mu = n(z) w Re(conj(nu) mu),

with the geometric series of 1 / (zeta - t) and 1 / conj(zeta - t)^2 in
t / zeta (multipole: far targets, arc sources) or zeta / t (local: arc
targets, far sources), zeta = (z - c) / rho, t = (tau - c) / rho.  Forty
terms at the ratio 0.4 (targets or sources beyond 2.5 rho) must reproduce the
direct sums to 1e-13 relative; a dropped or mis-signed term fails at 1e-2.
"""
import numpy as np

import workloads as W
from oracle import geometry as G, kernels as K

P_TERMS = 40
RATIO = 2.5


def _cplx(v):
    return v[:, 0] + 1j * v[:, 1]


def _direct(xt, nt, ys, ny, wy, mu):
    """sum_j (D + N)(x_i, y_j) mu_j from the oracle's dense double-layer block."""
    blk = K.dlp_block(xt, ys, ny, wy)                       # (2M, 2N)
    u = (blk @ mu.reshape(-1)).reshape(-1, 2)
    flux = np.sum(wy * np.sum(ny * mu, axis=1))
    return _cplx(u) + _cplx(nt) * flux


def _coeffs(c, rho, ys, ny, wy, mu, local):
    t = (_cplx(ys) - c) / rho
    nu = _cplx(ny)
    m = _cplx(mu)
    re = np.real(np.conj(nu) * m)
    p = np.arange(P_TERMS)[:, None]
    if local:
        tp, tb = t[None, :] ** -(p + 1), np.conj(t)[None, :] ** -(p + 1)
        tb2 = np.conj(t)[None, :] ** -(p + 2)
        A = (wy * nu * m * tp).sum(1)
        B = (2 * wy * re * tb).sum(1)
        C = ((p + 1) * wy * np.conj(nu) * np.conj(m) * tb2).sum(1)
        D = ((p + 1) * wy * np.conj(nu) * np.conj(m) * t * tb2).sum(1)
    else:
        tp, tb = t[None, :] ** p, np.conj(t)[None, :] ** p
        A = (wy * nu * m * tp).sum(1)
        B = (2 * wy * re * tb).sum(1)
        C = ((p + 1) * wy * np.conj(nu) * np.conj(m) * tb).sum(1)
        D = ((p + 1) * wy * np.conj(nu) * np.conj(m) * t * tb).sum(1)
    S = np.sum(wy * re)
    return A, B, C, D, S


def _evaluate(c, rho, coef, xt, nt, local):
    A, B, C, D, S = coef
    z = (_cplx(xt) - c) / rho
    u = np.zeros(len(z), complex)
    for p in range(P_TERMS):
        if local:
            zp, zb = z ** p, np.conj(z) ** p
            u += -A[p] * zp - B[p] * zb + (z * C[p] - D[p]) * zb
        else:
            zp, zb = z ** -(p + 1), np.conj(z) ** -(p + 1)
            u += A[p] * zp + B[p] * zb + (z * C[p] - D[p]) * zb / np.conj(z)
    return u / (4 * np.pi * rho) + _cplx(nt) * S


def _split():
    p = W.config1(seed=0)
    sets = G.refine(p.n_panels, p.refinement.panel_ids, p.refinement.levels, p.curve.a, p.curve.m)
    ref, new = sets.ref, sets.new
    arc = np.vstack([ref.x[sets.c_in_ref], new.x[sets.p_in_new]])
    lo, hi = arc.min(0), arc.max(0)
    c2 = 0.5 * (lo + hi)
    rho = np.max(np.hypot(*(arc - c2).T))
    k = sets.k_in_ref
    far = k[np.hypot(*(ref.x[k] - c2).T) >= RATIO * rho]
    return sets, c2[0] + 1j * c2[1], rho, far


def test_multipole_far_rows_match_direct_sum():
    sets, c, rho, far = _split()
    ref, new = sets.ref, sets.new
    assert len(far) > len(sets.k_in_ref) // 2
    ys = np.vstack([ref.x[sets.c_in_ref], new.x[sets.p_in_new]])
    ny = np.vstack([ref.normal[sets.c_in_ref], new.normal[sets.p_in_new]])
    # the cut columns enter Q with a minus sign (-A_kc)
    wy = np.concatenate([-ref.w[sets.c_in_ref], new.w[sets.p_in_new]])
    rng = np.random.default_rng(7)
    for _ in range(3):
        mu = rng.choice([-1.0, 1.0], size=(len(ys), 2))
        u = _direct(ref.x[far], ref.normal[far], ys, ny, wy, mu)
        ue = _evaluate(c, rho, _coeffs(c, rho, ys, ny, wy, mu, local=False), ref.x[far], ref.normal[far], local=False)
        assert np.max(np.abs(ue - u)) <= 1e-13 * np.max(np.abs(u))


def test_local_expansion_at_arc_targets_matches_direct_sum():
    sets, c, rho, far = _split()
    ref, new = sets.ref, sets.new
    xt, nt = new.x[sets.p_in_new], new.normal[sets.p_in_new]
    rng = np.random.default_rng(8)
    mu = rng.choice([-1.0, 1.0], size=(len(far), 2))
    u = _direct(xt, nt, ref.x[far], ref.normal[far], ref.w[far], mu)
    ue = _evaluate(c, rho, _coeffs(c, rho, ref.x[far], ref.normal[far], ref.w[far], mu, local=True), xt, nt, local=True)
    assert np.max(np.abs(ue - u)) <= 1e-13 * np.max(np.abs(u))


def test_a_dropped_term_is_detected():
    """Planted mistake: without the conj(r)^-2 family the sums disagree."""
    sets, c, rho, far = _split()
    ref, new = sets.ref, sets.new
    ys, ny = new.x[sets.p_in_new], new.normal[sets.p_in_new]
    wy = new.w[sets.p_in_new]
    mu = np.random.default_rng(9).choice([-1.0, 1.0], size=(len(ys), 2))
    u = _direct(ref.x[far], ref.normal[far], ys, ny, wy, mu)
    A, B, C, D, S = _coeffs(c, rho, ys, ny, wy, mu, local=False)
    bad = _evaluate(c, rho, (A, B, 0 * C, 0 * D, S), ref.x[far], ref.normal[far], local=False)
    assert np.max(np.abs(bad - u)) > 1e-2 * np.max(np.abs(u))
