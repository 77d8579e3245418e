"""FP64 evaluation floor of parity on deeply refined panels (CPU only).

Two correct FP64 discretizations of the same refined wall (for instance the
oracle's and the library's, each with its own Gauss-Legendre roots and
trigonometric evaluations) place the nodes a few ulps apart.  On a child
panel of level L the nearest nodes are about 2^-L times closer, and the
double-layer entry between them carries r . n_y ~ kappa |r|^2 / 2, so a
position change delta normal to the curve changes that entry by about
delta / (kappa |r|^2): the solution moves by an amount that grows roughly
2-3x per level.  This test measures that floor on the oracle alone (nodes
jittered by 2e-15 along the normal, a bound on the observed node
differences) and checks that it grows with the level and stays below the
1e-10 FP64 bar (2-norm) through level 6.  At level 8 of a 64-panel wall
(the child size of a 4-level refinement of a 1024-panel wall) the same
jitter moves tau by about 1.5e-10; the observed node differences between
two discretizations are smaller than the jitter, and their effect (about
5e-12 in the 2-norm, 3e-11 in the max norm at that child size) is what the
full-size tolerances allow for.
"""
import dataclasses

import numpy as np

import workloads as W
from oracle import geometry as G, kernels as K, solve as S


def _floor(level: int, rng) -> tuple:
    ids, lev = [20, 21], [level, level]
    sets = G.refine(64, ids, lev, 0.3, 5)
    d = sets.new
    st = W.stokeslets(np.random.default_rng(1), 8)
    t0 = S.solve_refined(K.nystrom_matrix(d), K.rhs_vector(d, st.z, st.f))
    dj = dataclasses.replace(d, x=d.x + 2e-15 * rng.choice([-1.0, 1.0], d.n)[:, None] * d.normal)
    t1 = S.solve_refined(K.nystrom_matrix(dj), K.rhs_vector(dj, st.z, st.f))
    return (float(np.linalg.norm(t1 - t0) / np.linalg.norm(t0)),
            float(np.max(np.abs(t1 - t0)) / np.max(np.abs(t0))))


def test_fp64_floor_grows_with_level():
    rng = np.random.default_rng(7)
    e3, m3 = _floor(3, rng)
    e6, m6 = _floor(6, rng)
    assert e3 < 1e-11 and m3 < 5e-11
    assert e6 > 4 * e3                 # the floor grows with the level
    assert e6 < 1e-10                  # and stays below the FP64 bar through level 6
