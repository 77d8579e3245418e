"""The batched workload at full size through the C ABI: 64 uneven
refinement instances of the 16384-node wall (2..32 contiguous panels, 2..5
levels, 8 Stokeslet right-hand sides each) solved by one rw_solve_batch call.
* the batch equals one rw_solve per instance to 1e-12;
* four seeded instances (those whose dense oracle fits) equal the oracle's
  whole solution (tests/golden, first right-hand side) to 1e-10 (2-norm)."""
import os

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2108_07205_amd as rw  # noqa: E402


def _say(msg):
    print(f"[gpu-batch64] {msg}", flush=True)


def test_batch_of_64_instances():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ctx = rw.Context(0)
    wall = rw.Wall(ctx, 1024)
    probs = W.batched_instances(n_inst=64, seed=0, n_panels=1024, nrhs=8)
    refs, gs = [], []
    for p in probs:
        ref = wall.refine(p.refinement.panel_ids, p.refinement.levels)
        refs.append(ref)
        gs.append(torch.stack([ref.stokeslet_rhs(q.z, q.f) for q in p.rhs]).contiguous())
    taus, infos = wall.solve_batch(refs, gs)
    seq = [ref.solve(g) for ref, g in zip(refs, gs)]
    diff = max(float(((a - b).norm(dim=1) / b.norm(dim=1)).max()) for a, b in zip(taus, seq))
    n_p = [r.info()["n_p"] for r in refs]
    _say(f"64 instances, {sum(g.shape[0] for g in gs)} RHS, N_p {min(n_p)}..{max(n_p)}: batch vs single {diff:.1e}, "
         f"max resid {max(i['resid'] for i in infos):.1e}, corrections {max(i['ir_iters'] for i in infos)}")
    assert diff <= 1e-12
    here = os.path.join(os.path.dirname(__file__), "golden")
    for i in W.BATCH_GOLDEN_INSTANCES:
        path = os.path.join(here, f"batch0_inst{i}_tau.npy")
        if not os.path.exists(path):
            _say(f"  instance {i}: golden solution not generated")
            continue
        t_or = np.load(path, allow_pickle=False)
        t = taus[i][0].cpu().numpy()
        e = float(np.linalg.norm(t - t_or) / np.linalg.norm(t_or))
        _say(f"  instance {i} ({len(probs[i].refinement.panel_ids)} panels x {probs[i].refinement.levels[0]} levels) "
             f"vs oracle: {e:.2e}")
        assert e <= 1e-10
    for r in refs:
        r.close()
    wall.close()
    ctx.close()
