"""Mixed precision through the C ABI: the reference inverse's generators in
FP64, FP32 and BF16 (BF16: FP32 accumulation on the BF16 matrix cores from
16 right-hand sides, FP64 sums with one), against the FP64 oracle:
* the applies against the dense inverse, bounded by the storage rounding
  (FP32 2^-24, BF16 2^-9, times kappa ~ 3e2);
* refined solves whose FP64 refinement (Richardson or preconditioned
  GMRES, the exact FP64 residual in both) brings every precision to the
  oracle's solution within the FP64 bar; the iteration counts show what the
  narrow generators cost."""
import numpy as np
import pytest

import workloads as W
from oracle import geometry as G, kernels as K, solve as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2108_07205_amd as rw  # noqa: E402

BOUND = {rw.RW_F64: 2e-9, rw.RW_F32: 1e-4, rw.RW_BF16: 0.5}


def _say(msg):
    print(f"[gpu-mixed] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = rw.Context(0)
    yield c
    c.close()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("nrhs", [1, 5, 20, 70])
def test_bf16_apply(ctx, nrhs):
    wall = rw.Wall(ctx, 64, precision=rw.RW_BF16)
    d = G.discretize(G.reference_panels(64), 0.3, 5)
    A = K.nystrom_matrix(d)
    B = np.random.default_rng(40 + nrhs).standard_normal((nrhs, 2 * d.n))
    X = wall.hbs_apply(_dev(B)).cpu().numpy()
    Xo = np.linalg.solve(A, B.T).T
    worst = max(float(np.linalg.norm(X[c] - Xo[c]) / np.linalg.norm(Xo[c])) for c in range(nrhs))
    _say(f"bf16 generators, {nrhs} RHS: worst rel err {worst:.2e} (crossover {wall.stats()['mfma_from_f32']})")
    assert worst < BOUND[rw.RW_BF16]
    wall.close()


@pytest.mark.parametrize("prec", [rw.RW_F64, rw.RW_F32, rw.RW_BF16])
@pytest.mark.parametrize("nrhs", [20, 70])
def test_matrix_core_apply_each_precision(ctx, prec, nrhs):
    """The matrix-core path forced from 16 right-hand sides (mfma_from) for
    each generator precision, against the dense inverse."""
    wall = rw.Wall(ctx, 64, precision=prec)
    d = G.discretize(G.reference_panels(64), 0.3, 5)
    A = K.nystrom_matrix(d)
    B = np.random.default_rng(60 + nrhs).standard_normal((nrhs, 2 * d.n))
    ctx.set_options(mfma_from=16)
    try:
        X = wall.hbs_apply(_dev(B)).cpu().numpy()
    finally:
        ctx.set_options(mfma_from=0)
    Xo = np.linalg.solve(A, B.T).T
    worst = max(float(np.linalg.norm(X[c] - Xo[c]) / np.linalg.norm(Xo[c])) for c in range(nrhs))
    _say(f"matrix cores, precision {prec}, {nrhs} RHS: worst rel err {worst:.2e}")
    assert worst < BOUND[prec]
    wall.close()


@pytest.mark.parametrize("prec", [rw.RW_F64, rw.RW_F32, rw.RW_BF16])
def test_refined_solve_each_precision(ctx, prec):
    p = W.config1(seed=0)
    sets = G.refine(p.n_panels, p.refinement.panel_ids, p.refinement.levels, p.curve.a, p.curve.m)
    g = K.rhs_vector(sets.new, p.rhs[0].z, p.rhs[0].f)
    tau_or = S.solve_refined(K.nystrom_matrix(sets.new), g)
    wall = rw.Wall(ctx, 64, precision=prec)
    ref = wall.refine(p.refinement.panel_ids, p.refinement.levels)
    res = {}
    for solver, maxit in ((rw.RW_SOLVE_IR, 30), (rw.RW_SOLVE_GMRES, 60)):
        ctx.set_options(solver=solver, ir_maxit=maxit)
        try:
            tau = torch.empty(ref.n_unknowns, dtype=torch.float64, device="cuda")
            info = {}
            rc = rw.rw_solve(ctx.h, ref.h, _dev(g), tau, ref.n_unknowns, check=False, info=info)
        finally:
            ctx.set_options(solver=rw.RW_SOLVE_IR, ir_maxit=6)
        e = float(np.linalg.norm(tau.cpu().numpy() - tau_or) / np.linalg.norm(tau_or))
        res[solver] = (rc, info["ir_iters"], info["resid_direct"], e)
    _say(f"precision {prec}: Richardson rc={res[0][0]} its={res[0][1]} direct={res[0][2]:.1e} err={res[0][3]:.1e}; "
         f"GMRES rc={res[1][0]} its={res[1][1]} err={res[1][3]:.1e}")
    assert res[rw.RW_SOLVE_GMRES][0] == rw.RW_OK and res[rw.RW_SOLVE_GMRES][3] <= 1e-10
    if prec != rw.RW_BF16:
        assert res[rw.RW_SOLVE_IR][0] == rw.RW_OK and res[rw.RW_SOLVE_IR][3] <= 1e-10
    ref.close()
    wall.close()
