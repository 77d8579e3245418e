"""Refinement reuse across time steps (Sec. 5.3) through the C ABI: a
particle moving along the wall asks for its nearest panels to be refined
at every step; the cache serves consecutive steps with one refinement of a
widened region.
* every served refinement covers the request (each requested panel refined
  at least as deep);
* a served (reused) refinement solves to the FP64 oracle's solution of its
  own discretization within the FP64 bar, and equals a fresh rw_refine of
  the same region;
* most steps are served from the cache."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import geometry as G, kernels as K, solve as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2108_07205_amd as rw  # noqa: E402


def _say(msg):
    print(f"[gpu-refcache] {msg}", flush=True)


def test_moving_particle_reuses_refinements():
    ctx = rw.Context(0)
    wall = rw.Wall(ctx, 64)
    cache = rw.RefCache(wall, capacity=3, margin=2)
    curve = W.Curve()
    st = W.stokeslets(np.random.default_rng(8), 8)
    theta0, h = 1.1, 2 * math.pi / 64
    hits = 0
    for t in range(12):
        th = theta0 + 0.4 * h * t
        p0 = curve.point(th) + 0.02 * curve.outward_normal(th)
        ids = W.nearest_panels(curve, 64, p0, 2)
        lev = [3, 3]
        ref, hit = cache.get(ids, lev)
        hits += int(hit)
        cids, clev = cache.panels(ref)
        cov = dict(zip(cids.tolist(), clev.tolist()))
        assert all(cov.get(i, -1) >= l for i, l in zip(ids, lev))
        g = ref.stokeslet_rhs(st.z, st.f)
        tau = ref.solve(g).cpu().numpy()
        if t in (0, 3, 7, 11):
            sets = G.refine(64, cids, clev, 0.3, 5)
            gor = K.rhs_vector(sets.new, st.z, st.f)
            tor = S.solve_refined(K.nystrom_matrix(sets.new), gor)
            e = float(np.linalg.norm(tau - tor) / np.linalg.norm(tor))
            fresh = wall.refine(cids, clev)
            tf = fresh.solve(fresh.stokeslet_rhs(st.z, st.f)).cpu().numpy()
            d = float(np.linalg.norm(tau - tf) / np.linalg.norm(tf))
            fresh.close()
            _say(f"step {t}: request {ids} -> region {cids.tolist()} (hit {hit}); vs oracle {e:.1e}, "
                 f"vs fresh refine {d:.1e}")
            assert e <= 1e-10 and d <= 1e-13
    stats = cache.stats()
    _say(f"12 steps: {stats}")
    assert stats["hits"] == hits and hits >= 6
    cache.close()
    wall.close()
    ctx.close()
