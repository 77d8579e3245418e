"""Write the full-size golden solutions under tests/golden from the FP64
oracle only (dense assembly + LU of the refined Nystrom system).

For every case of ``workloads.golden_cases()`` (1024-panel wall, 16384
reference nodes; 16 panels x 4 levels at two seeds, 16 panels x 4 levels
across theta = 0, 4 panels x 6 levels) the oracle's full tau_n (Stokeslet
data of the case's first right-hand side) is stored as ``<case>_tau.npy``
(float64, 2 N_n values, node-major interleaved) and its provenance
(refinement, sizes, norms, assembly and LU times, BLAS threads) in
``golden_meta.json``.  Nothing here calls the HIP library.

Run:  python tests/golden/make_golden.py [case ...]
(about 5 minutes and 30 GB of RAM per case on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import geometry as G, kernels as K, solve as S  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
META = os.path.join(HERE, "golden_meta.json")


def _threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        return -1


def solve_case(name: str, p: W.Problem) -> dict:
    sets = G.refine(p.n_panels, p.refinement.panel_ids, p.refinement.levels, p.curve.a, p.curve.m)
    st = p.rhs[0]
    g = K.rhs_vector(sets.new, st.z, st.f)
    t0 = time.time()
    A = K.nystrom_matrix(sets.new)
    t1 = time.time()
    tau = S.solve_refined(A, g)
    t2 = time.time()
    # backward error of the LU solve, from the same matrix
    res = float(np.linalg.norm(g - A @ tau) / np.linalg.norm(g))
    del A
    np.save(os.path.join(HERE, f"{name}_tau.npy"), tau)
    return {"n_panels": p.n_panels, "panel_ids": list(p.refinement.panel_ids),
            "levels": list(p.refinement.levels), "seed": p.seed,
            "n_nodes": int(sets.new.n), "n_p": int(sets.p_in_new.size),
            "norm2": float(np.linalg.norm(tau)), "normmax": float(np.max(np.abs(tau))),
            "lu_backward_error": res, "assembly_s": round(t1 - t0, 1), "lu_s": round(t2 - t1, 1),
            "blas_threads": _threads(), "host_cpus": os.cpu_count()}


def main(names):
    cases = W.golden_cases()
    meta = json.load(open(META)) if os.path.exists(META) else {}
    for name in names or list(cases):
        m = solve_case(name, cases[name])
        meta[name] = m
        with open(META, "w") as fh:
            json.dump(meta, fh, indent=1, sort_keys=True)
        print(f"{name}: {m['n_nodes']} nodes, assembly {m['assembly_s']} s, LU {m['lu_s']} s, "
              f"backward error {m['lu_backward_error']:.2e}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
