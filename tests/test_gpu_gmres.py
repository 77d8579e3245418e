"""Preconditioned GMRES on the exact refined operator (Sec. 4: the solver of
the extended system as the preconditioner; here applied on the right),
through the C ABI, against the FP64 oracle:
* GMRES reaches the oracle's solution to the FP64 bar (config 1, and the
  full-size golden case) in a few iterations;
* with a deliberately coarse compression of Q (q_tol = 0.3: k = 2)
  Richardson refinement stops contracting while GMRES still converges
  (measured: Richardson stalls at a residual of 5e-3 after 30 corrections,
  GMRES reaches 1e-13 in 13 iterations);
* plain GMRES (no preconditioner) needs many times more iterations than the
  preconditioned one (the paper's comparison of iteration counts)."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import geometry as G, kernels as K, solve as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2108_07205_amd as rw  # noqa: E402


def _say(msg):
    print(f"[gpu-gmres] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = rw.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def wall64(ctx):
    w = rw.Wall(ctx, 64)
    yield w
    w.close()


def _oracle(p):
    sets = G.refine(p.n_panels, p.refinement.panel_ids, p.refinement.levels, p.curve.a, p.curve.m)
    st = p.rhs[0]
    g = K.rhs_vector(sets.new, st.z, st.f)
    return g, S.solve_refined(K.nystrom_matrix(sets.new), g)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _solve(ctx, ref, g, **opts):
    old = ctx.options()
    ctx.set_options(**opts)
    try:
        tau = torch.empty(ref.n_unknowns, dtype=torch.float64, device="cuda")
        info = {}
        rc = rw.rw_solve(ctx.h, ref.h, _dev(g), tau, ref.n_unknowns, check=False, info=info)
    finally:
        ctx.set_options(**{k: old[k] for k in opts})
    return rc, tau.cpu().numpy(), info


@pytest.mark.parametrize("seed", [0, 1])
def test_gmres_matches_oracle(ctx, wall64, seed):
    p = W.config1(seed=seed)
    g, tau_or = _oracle(p)
    ref = wall64.refine(p.refinement.panel_ids, p.refinement.levels)
    rc, tau, info = _solve(ctx, ref, g, solver=rw.RW_SOLVE_GMRES)
    e = _rel(tau, tau_or)
    _say(f"config1 seed {seed}: rc={rc} its={info['ir_iters']} resid={info['resid']:.1e} "
         f"first={info['resid_direct']:.1e} err={e:.2e}")
    assert rc == rw.RW_OK and e <= 1e-10 and info["ir_iters"] <= 4
    ref.close()


def test_gmres_golden_full_size(ctx):
    path = os.path.join(os.path.dirname(__file__), "golden", "config2_seed0_tau.npy")
    tau_or = np.load(path, allow_pickle=False)
    p = W.golden_cases()["config2_seed0"]
    wall = rw.Wall(ctx, 1024)
    ref = wall.refine(p.refinement.panel_ids, p.refinement.levels)
    g = ref.stokeslet_rhs(p.rhs[0].z, p.rhs[0].f).cpu().numpy()
    rc, tau, info = _solve(ctx, ref, g, solver=rw.RW_SOLVE_GMRES)
    e = _rel(tau, tau_or)
    _say(f"config2 golden: rc={rc} its={info['ir_iters']} resid={info['resid']:.1e} err={e:.2e}")
    assert rc == rw.RW_OK and e <= 1e-10
    ref.close()
    wall.close()


def test_gmres_converges_where_richardson_stalls(ctx, wall64):
    p = W.config1(seed=0)
    g, tau_or = _oracle(p)
    ref = wall64.refine(p.refinement.panel_ids, p.refinement.levels, q_tol=0.3)
    rc_ir, tau_ir, inf_ir = _solve(ctx, ref, g, solver=rw.RW_SOLVE_IR, ir_maxit=20)
    rc_gm, tau_gm, inf_gm = _solve(ctx, ref, g, solver=rw.RW_SOLVE_GMRES, ir_maxit=40)
    e_gm = _rel(tau_gm, tau_or)
    _say(f"q_tol 0.3 (k={ref.info()['k']}): Richardson rc={rc_ir} corrections={inf_ir['ir_iters']} "
         f"resid={inf_ir['resid']:.1e}; GMRES rc={rc_gm} its={inf_gm['ir_iters']} resid={inf_gm['resid']:.1e} "
         f"err={e_gm:.2e}")
    assert rc_gm == rw.RW_OK and e_gm <= 1e-10 and inf_gm["ir_iters"] <= 20
    assert rc_ir == rw.RW_ENOCONV and inf_ir["resid"] > 1e-6
    ref.close()


@pytest.mark.parametrize("resid_mode", [rw.RW_RESID_AUTO, rw.RW_RESID_EXPAND])
def test_plain_gmres_needs_many_more_iterations(ctx, wall64, resid_mode):
    """Also with the products A z formed with far node clusters by expansion
    (RW_RESID_EXPAND; config 1 is below the size where RW_RESID_AUTO takes
    them): the long unpreconditioned Krylov run still reaches the oracle."""
    p = W.config1(seed=0)
    g, tau_or = _oracle(p)
    ref = wall64.refine(p.refinement.panel_ids, p.refinement.levels)
    rc_p, tau_p, inf_p = _solve(ctx, ref, g, solver=rw.RW_SOLVE_GMRES, resid_mode=resid_mode)
    rc_n, tau_n, inf_n = _solve(ctx, ref, g, solver=rw.RW_SOLVE_GMRES, gmres_precond=0, gmres_restart=200,
                                ir_maxit=1000, resid_mode=resid_mode)
    _say(f"residual mode {resid_mode}: iterations to 1e-13: preconditioned {inf_p['ir_iters']}, plain "
         f"{inf_n['ir_iters']} (rc {rc_p}, {rc_n}); errors {_rel(tau_p, tau_or):.1e}, {_rel(tau_n, tau_or):.1e}")
    assert rc_p == rw.RW_OK and rc_n == rw.RW_OK
    assert _rel(tau_n, tau_or) <= 1e-10
    assert inf_n["ir_iters"] >= 5 * inf_p["ir_iters"]
    ref.close()
