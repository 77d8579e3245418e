"""The residual r = g - A_nn tau with far node clusters through multipole
expansions (RW_RESID_EXPAND) against the one that sums every pair
(RW_RESID_PAIRS) and against the FP64 oracle's dense product.

Both GPU forms evaluate the same Nystrom operator (Sec. 2) on the same
nodes: they differ by the cut of the expansions (below 1e-17 of a cluster's
contribution) and by rounding in a different order, so they agree to a few
ulps of the largest partial sums: bound 1e-14 of max_i sum_j |A_ij tau_j|
(estimated by max |A tau| times 10).  Against the oracle the bound of the
pairwise tests holds (independent discretizations, smooth densities).
"""
import numpy as np
import pytest

import workloads as W
from oracle import geometry as G, kernels as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2108_07205_amd as rw  # noqa: E402


def _say(msg):
    print(f"[gpu-resid] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = rw.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def wall64(ctx):
    return rw.Wall(ctx, 64)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _resid(ctx, ref, g, t, mode):
    ctx.set_options(resid_mode=mode)
    try:
        return ref.residual(_dev(g), _dev(t)).cpu().numpy()
    finally:
        ctx.set_options(resid_mode=rw.RW_RESID_AUTO)


@pytest.mark.parametrize("ids,levels,nrhs", [((3,), (1,), 1), ((3, 20, 40, 50), (6, 6, 6, 6), 1),
                                             ((10, 11, 12), (3, 3, 3), 3), ((63, 0), (4, 4), 2)])
def test_expansions_match_pairs_and_oracle(ctx, wall64, ids, levels, nrhs):
    """Node counts 1040, 5056, 1360 and 1504 (ragged last cluster and last
    wave), one to three right-hand sides, a refinement across theta = 0."""
    p = W.small_problem(n_panels=64, ids=ids, levels=levels, n_stokeslets=4, nrhs=nrhs)
    sets = G.refine(p.n_panels, p.refinement.panel_ids, p.refinement.levels, p.curve.a, p.curve.m)
    ref = wall64.refine(p.refinement.panel_ids, p.refinement.levels)
    n = ref.n_nodes
    assert n == sets.new.x.shape[0]
    A = K.nystrom_matrix(sets.new)
    gs = np.stack([K.rhs_vector(sets.new, s.z, s.f) for s in p.rhs])
    x = sets.new.x
    ts = np.stack([np.stack([np.sin(2 * x[:, 0] + 0.3 * c), np.cos(3 * x[:, 1] - 0.7 * c)], 1).reshape(-1)
                   for c in range(nrhs)])
    rng = np.random.default_rng(n)
    rand = rng.standard_normal(ts.shape)
    for name, t in (("smooth", ts), ("random", rand)):
        g, tt = (gs[0], t[0]) if nrhs == 1 else (gs, t)
        r_e = _resid(ctx, ref, g, tt, rw.RW_RESID_EXPAND).reshape(nrhs, -1)
        r_p = _resid(ctx, ref, g, tt, rw.RW_RESID_PAIRS).reshape(nrhs, -1)
        for c in range(nrhs):
            at = A @ t[c]
            d = np.max(np.abs(r_e[c] - r_p[c]))
            _say(f"n={n} {name} rhs {c}: |expand - pairs| {d:.2e} (max |A tau| {np.max(np.abs(at)):.2e})")
            assert d <= 1e-13 * np.max(np.abs(at))
            if name == "smooth":
                r_or = gs[c] - at
                assert np.max(np.abs(r_e[c] - r_or)) < 1e-11 * np.max(np.abs(r_or))
    ref.close()


def test_expansions_full_size(ctx):
    """1024 panels, 16 panels x 4 levels (20224 nodes, 79 clusters): the two
    forms on a random density with 1, 4, 5, 4, 1 and 40 right-hand sides
    (40 columns: one item per target group, near and far clusters in the
    same wave), and the refined solve with each (same tau, same
    corrections).  The column counts go up and down on one handle, whose
    residual workspace is sized by the largest count so far: it must hold
    every smaller count too (the one-column pairwise form takes the most
    splits)."""
    p = W.config2(seed=3)
    wall = rw.Wall(ctx, 1024)
    ref = wall.refine(p.refinement.panel_ids, p.refinement.levels)
    n = ref.n_nodes
    assert n == 20224
    rng = np.random.default_rng(5)
    for nrhs in (1, 4, 5, 4, 1, 40):
        t = rng.standard_normal((nrhs, 2 * n))
        g = rng.standard_normal((nrhs, 2 * n))
        gg, tt = (g[0], t[0]) if nrhs == 1 else (g, t)
        r_e = _resid(ctx, ref, gg, tt, rw.RW_RESID_EXPAND).reshape(nrhs, -1)
        r_p = _resid(ctx, ref, gg, tt, rw.RW_RESID_PAIRS).reshape(nrhs, -1)
        worst = 0.0
        for c in range(nrhs):
            at = np.max(np.abs(g[c] - r_p[c]))
            d = np.max(np.abs(r_e[c] - r_p[c]))
            worst = max(worst, d / at)
            assert d <= 1e-13 * at
        _say(f"full size, {nrhs} rhs: largest |expand - pairs| / max |A tau| {worst:.2e}")
    s0 = p.rhs[0]
    g = ref.stokeslet_rhs(s0.z, s0.f)
    out = {}
    for mode in (rw.RW_RESID_EXPAND, rw.RW_RESID_PAIRS):
        ctx.set_options(resid_mode=mode)
        tau = ref.solve(g).cpu().numpy()
        inf = ref.info()
        out[mode] = (tau, inf["ir_iters"], inf["resid"])
    ctx.set_options(resid_mode=rw.RW_RESID_AUTO)
    (te, ie, re), (tp, ip, rp) = out[rw.RW_RESID_EXPAND], out[rw.RW_RESID_PAIRS]
    rel = np.linalg.norm(te - tp) / np.linalg.norm(tp)
    _say(f"full-size solve: ir {ie}/{ip}, resid {re:.2e}/{rp:.2e}, |tau_e - tau_p| / |tau_p| {rel:.2e}")
    assert ie == ip and re <= 1e-13 and rp <= 1e-13
    assert rel <= 1e-13
    ref.close()
    wall.close()


def test_expansions_two_levels(ctx):
    """4096 panels, 32 panels x 4 levels (73216 nodes, 286 clusters of 256
    nodes under 36 of 2048): second-level clusters far from a target group
    are taken by one expansion each, near ones by their first-level clusters;
    against the pairwise form on random densities (1 and 3 right-hand sides)
    and in the refined solve."""
    p = W.config4(seed=1, nrhs=1)
    wall = rw.Wall(ctx, 4096)
    ref = wall.refine(p.refinement.panel_ids, p.refinement.levels)
    n = ref.n_nodes
    assert n == 73216
    rng = np.random.default_rng(9)
    for nrhs in (1, 3):
        t = rng.standard_normal((nrhs, 2 * n))
        g = rng.standard_normal((nrhs, 2 * n))
        gg, tt = (g[0], t[0]) if nrhs == 1 else (g, t)
        r_e = _resid(ctx, ref, gg, tt, rw.RW_RESID_EXPAND).reshape(nrhs, -1)
        r_p = _resid(ctx, ref, gg, tt, rw.RW_RESID_PAIRS).reshape(nrhs, -1)
        worst = 0.0
        for c in range(nrhs):
            at = np.max(np.abs(g[c] - r_p[c]))
            d = np.max(np.abs(r_e[c] - r_p[c]))
            worst = max(worst, d / at)
            assert d <= 1e-13 * at
        _say(f"73216 nodes, {nrhs} rhs: largest |expand - pairs| / max |A tau| {worst:.2e}")
    g = ref.stokeslet_rhs(p.rhs[0].z, p.rhs[0].f)
    out = {}
    for mode in (rw.RW_RESID_EXPAND, rw.RW_RESID_PAIRS):
        ctx.set_options(resid_mode=mode)
        tau = ref.solve(g).cpu().numpy()
        inf = ref.info()
        out[mode] = (tau, inf["ir_iters"], inf["resid"])
    ctx.set_options(resid_mode=rw.RW_RESID_AUTO)
    (te, ie, re), (tp, ip, rp) = out[rw.RW_RESID_EXPAND], out[rw.RW_RESID_PAIRS]
    rel = np.linalg.norm(te - tp) / np.linalg.norm(tp)
    _say(f"73216-node solve: ir {ie}/{ip}, resid {re:.2e}/{rp:.2e}, |tau_e - tau_p| / |tau_p| {rel:.2e}")
    assert ie == ip and re <= 1e-13 and rp <= 1e-13 and rel <= 1e-13
    ref.close()
    wall.close()


def test_resid_mode_checked(ctx):
    with pytest.raises(rw.RwError):
        ctx.set_options(resid_mode=3)
    with pytest.raises(rw.RwError):
        ctx.set_options(resid_mode=-1)
    assert ctx.options()["resid_mode"] == rw.RW_RESID_AUTO
