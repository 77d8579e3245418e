"""Write tests/golden/*.txt from the FP64 oracle only (dense assembly + LU).

config2_seed0_tau_sample.txt: the 1024-panel wall with 16 panels refined 4
levels (40448 unknowns), Stokeslet data of seed 0; the oracle's tau_n is
stored at 4096 seeded sample indices plus its 2-norm and max-norm, so the GPU
test can check the full-size solve without the 13 GB dense solve.

Run:  python tests/golden/make_golden.py   (about 5 minutes, ~30 GB RAM)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import geometry as G, kernels as K, solve as S  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def config2_sample(seed: int = 0, nsample: int = 4096):
    p = W.config2(seed=seed)
    sets = G.refine(p.n_panels, p.refinement.panel_ids, p.refinement.levels, p.curve.a, p.curve.m)
    st = p.rhs[0]
    g = K.rhs_vector(sets.new, st.z, st.f)
    t0 = time.time()
    A = K.nystrom_matrix(sets.new)
    t1 = time.time()
    tau = S.solve_refined(A, g)
    t2 = time.time()
    del A
    rng = np.random.default_rng(12345)
    idx = np.unique(np.concatenate([rng.choice(tau.size, nsample - 512, replace=False),
                                    np.sort(rng.choice(2 * sets.p_in_new, 256, replace=False)),
                                    np.sort(rng.choice(2 * sets.p_in_new + 1, 256, replace=False))]))
    out = os.path.join(HERE, f"config2_seed{seed}_tau_sample.txt")
    with open(out, "w") as fh:
        fh.write(f"# oracle tau_n for workloads.config2(seed={seed}): dense FP64 assembly + LU\n")
        fh.write(f"# n_unknowns {tau.size} norm2 {np.linalg.norm(tau):.17e} normmax {np.max(np.abs(tau)):.17e}\n")
        fh.write(f"# assembly {t1 - t0:.1f} s, LU solve {t2 - t1:.1f} s\n")
        for i in idx:
            fh.write(f"{int(i)} {tau[i]:.17e}\n")
    print(f"wrote {out}: {idx.size} samples, assembly {t1 - t0:.1f} s, solve {t2 - t1:.1f} s")


if __name__ == "__main__":
    config2_sample(0)
