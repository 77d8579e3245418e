"""Serving through the C ABI (rw_server_*): requests of uneven refinement
size and right-hand-side count, run by several slots whose device work
overlaps, against one resident wall.
* each result in the mix equals the same request solved alone (one slot,
  nothing else running) to 1e-12, and the small wall's results equal the
  FP64 oracle's dense solutions to the FP64 bar;
* admission by memory: a request that could never fit the budget is
  refused at submission; with a budget that fits one request at a time all
  requests still complete."""
import numpy as np
import pytest

import workloads as W
from oracle import geometry as G, kernels as K, solve as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2108_07205_amd as rw  # noqa: E402


def _say(msg):
    print(f"[gpu-serving] {msg}", flush=True)


def _stk(p):
    return [(s.z, s.f) for s in p.rhs]


def _run(wall, reqs, slots, budget=0):
    sv = rw.Server(wall, slots=slots, hbm_budget_bytes=budget)
    ids = [sv.submit(r.problem.refinement.panel_ids, r.problem.refinement.levels, _stk(r.problem)) for r in reqs]
    out = [sv.wait(i) for i in ids]
    sv.close()
    return out


def test_mix_equals_alone_and_oracle():
    ctx = rw.Context(0)
    wall = rw.Wall(ctx, 64)
    reqs = W.serving_requests(8, rate=2000.0, seed=3, n_panels=64, max_sel=6, max_level=4, max_rhs=3)
    mix = _run(wall, reqs, slots=4)
    slots_used = {inf["slot"] for _, inf in mix}
    _say(f"64-panel mix: slots used {sorted(slots_used)}, "
         f"nodes {[inf['n_nodes'] for _, inf in mix]}, resid max {max(inf['resid'] for _, inf in mix):.1e}")
    for r, (tau, inf) in zip(reqs, mix):
        alone, ainf = _run(wall, [r], slots=1)[0]
        d = np.max(np.linalg.norm(tau - alone, axis=1) / np.linalg.norm(alone, axis=1))
        p = r.problem
        sets = G.refine(p.n_panels, p.refinement.panel_ids, p.refinement.levels, p.curve.a, p.curve.m)
        A = K.nystrom_matrix(sets.new)
        g = np.stack([K.rhs_vector(sets.new, s.z, s.f) for s in p.rhs], axis=1)
        tor = S.solve_refined(A, g).T
        e = np.max(np.linalg.norm(tau - tor, axis=1) / np.linalg.norm(tor, axis=1))
        assert inf["status"] == rw.RW_OK and d <= 1e-12 and e <= 1e-10, (d, e)
    assert len(slots_used) > 1
    wall.close()
    ctx.close()


def test_mix_equals_alone_full_size_and_admission():
    ctx = rw.Context(0)
    wall = rw.Wall(ctx, 1024)
    reqs = W.serving_requests(6, rate=2000.0, seed=5, n_panels=1024, max_sel=32, max_level=5, max_rhs=4)
    mix = _run(wall, reqs, slots=3)
    alone = [_run(wall, [r], slots=1)[0] for r in reqs]
    worst = max(float(np.max(np.linalg.norm(a[0] - m[0], axis=1) / np.linalg.norm(a[0], axis=1)))
                for a, m in zip(alone, mix))
    _say(f"1024-panel mix of {len(reqs)}: nodes {[m[1]['n_nodes'] for m in mix]}, alone vs mix {worst:.1e}")
    assert all(m[1]["status"] == rw.RW_OK for m in mix) and worst <= 1e-12
    # a budget too small for any request: refused at submission
    sv = rw.Server(wall, slots=2, hbm_budget_bytes=1 << 20)
    with pytest.raises(rw.RwError) as ei:
        p = reqs[0].problem
        sv.submit(p.refinement.panel_ids, p.refinement.levels, _stk(p))
    assert ei.value.code == rw.RW_ENOMEM
    sv.close()
    # a budget that fits one request at a time (about 0.6 GB here): all complete
    seq = _run(wall, reqs[:3], slots=3, budget=700 << 20)
    assert all(s[1]["status"] == rw.RW_OK for s in seq)
    wall.close()
    ctx.close()


@pytest.mark.parametrize("app_dense_max_nodes", [1024, 0])
def test_one_stream_ctx_matches_default(app_dense_max_nodes):
    """A ctx with one_stream = 1 (what each slot of a multi-slot server
    uses: A_pp^{-1} built before the compression of Q, on the same stream,
    no helper thread) gives the same refinement and solution as the default
    ctx, for the dense and the GPU-built HBS A_pp^{-1}."""
    res = []
    for one in (0, 1):
        ctx = rw.Context(0)
        ctx.set_options(app_dense_max_nodes=app_dense_max_nodes, one_stream=one)
        wall = rw.Wall(ctx, 64)
        p = W.config1(seed=4)
        ref = wall.refine(p.refinement.panel_ids, p.refinement.levels)
        g = torch.stack([ref.stokeslet_rhs(s.z, s.f) for s in p.rhs]).contiguous()
        tau = torch.empty_like(g)
        info = {}
        rw.rw_solve(ctx.h, ref.h, g, tau, ref.n_unknowns, info=info)
        inf = ref.info()
        res.append((tau.cpu().numpy(), inf["k"], inf["app_entries"], info["ir_iters"]))
        ref.close()
        wall.close()
        ctx.close()
    d = np.max(np.linalg.norm(res[0][0] - res[1][0], axis=1) / np.linalg.norm(res[0][0], axis=1))
    _say(f"one_stream vs default (dense max {app_dense_max_nodes}): k {res[0][1]}/{res[1][1]}, "
         f"app entries {res[0][2]}/{res[1][2]}, diff {d:.1e}")
    assert res[0][1:] == res[1][1:]
    assert d <= 1e-13


def test_multi_rhs_solve_right_after_refine():
    """A solve of several right-hand sides enqueued right behind its
    refinement (whose last part still runs on the side stream) equals the
    same solve repeated once everything has finished, bit for bit, on the
    GPU-built A_pp inverse (16384-node wall, 16 panels x 4 levels), and
    meets the FP64 residual bar: the solve's A_pp^{-1} applies must not share
    a workspace with the refinement's X_p = A_pp^{-1} L_p."""
    ctx = rw.Context(0)
    wall = rw.Wall(ctx, 1024)
    for seed in (0, 3):
        p = W.config2(seed=seed)
        rng = np.random.default_rng(seed)
        sts = [W.stokeslets(rng, 16) for _ in range(8)]
        ref = wall.refine(p.refinement.panel_ids, p.refinement.levels)
        g = torch.stack([ref.stokeslet_rhs(s.z, s.f) for s in sts]).contiguous()
        info1, info2 = {}, {}
        t1 = ref.solve(g, info=info1)
        torch.cuda.synchronize()
        t2 = ref.solve(g, info=info2)
        _say(f"multi-RHS right after refine (seed {seed}): resid {info1['resid']:.1e} / {info2['resid']:.1e}, "
             f"equal {bool(torch.equal(t1, t2))}")
        assert info1["resid"] <= 1e-13 and torch.equal(t1, t2)
        ref.close()
    wall.close()
    ctx.close()
