"""rw_hbs_apply_noalloc (one-RHS reference-inverse apply whose partial
vectors live in a static device array) against rw_hbs_apply, through the C
ABI: two calls in a row, the second on a smaller wall, each equal to the
allocating entry point's result (same kernels, same order), and the small
one also against the FP64 oracle's dense inverse."""
import numpy as np
import pytest

from oracle import geometry as G, kernels as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2108_07205_amd as rw  # noqa: E402


def test_noalloc_apply_matches_allocating_apply():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ctx = rw.Context(0)
    rng = np.random.default_rng(21)
    for n_panels in (1024, 64):
        print(f"[no-alloc] wall {n_panels} panels", flush=True)
        wall = rw.Wall(ctx, n_panels)
        n = 2 * wall.n_nodes
        b = torch.as_tensor(rng.standard_normal(n), dtype=torch.float64, device="cuda")
        x_ref = torch.empty_like(b)
        rw.rw_hbs_apply(ctx.h, wall.h, b, x_ref, n)
        x = torch.full_like(b, float("nan"))
        rw.rw_hbs_apply_noalloc(ctx.h, wall.h, b, x, n)
        torch.cuda.synchronize()
        xr, xa = x_ref.cpu().numpy(), x.cpu().numpy()
        assert np.all(np.isfinite(xa))
        assert np.array_equal(xa, xr)
        if n_panels == 64:
            d = G.discretize(G.reference_panels(64), 0.3, 5)
            xo = np.linalg.solve(K.nystrom_matrix(d), b.cpu().numpy())
            assert np.linalg.norm(xa - xo) / np.linalg.norm(xo) < 2e-9
        wall.close()
    ctx.close()
