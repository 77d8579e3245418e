#!/usr/bin/env python3
"""Refined-wall solves per second on one MI355X.

Workload (the headline configuration): the star wall r = 1 + 0.3 cos 5 theta
with 1024 Gauss-Legendre panels of 16 nodes (16384 nodes, 32768 unknowns),
HBS leaves of 64 nodes and ID tolerance 1e-10.  One step = one refined-wall
solve of the paper's Direct-Local strategy (refinement pre-computation plus
one right-hand side):
  refine: the 16 panels nearest a seeded point at distance 1e-3 outside the
          wall, split 4 levels (4096 added nodes, 40448 refined unknowns);
          Q ~= L R, A_pp LU, X = A~^{-1} L, W = I + R X  (Algorithm 1 pre-comp.)
  rhs:    velocity of 16 exterior Stokeslets (N(0,1) strengths, radius 2.5)
          at the refined nodes;
  solve:  Woodbury solve + FP64 iterative refinement on the exact refined
          residual (Algorithm 1 solve steps).
Step s uses seed s for the refinement point and the Stokeslets.  The static
reference inverse (the paper's T_static) is built once before timing.  A step
counts toward the rate only if (1) its solve met the library's own FP64
residual (||g - A tau|| / ||g|| <= 1e-13) and (2) after the timed region, the
FP64 oracle's residual r of its tau, formed by the oracle on its own
discretization at 264 sampled rows (200 seeded + every 64th added node),
bounds the error against the oracle's solution by at most 1e-8 (the
metric's gate): ||tau - tau_or|| / ||tau|| <= ||A^{-1}|| ||r|| / ||tau||, with
||r|| estimated from the sampled rows (||r_s|| / ||g_s|| times ||g||) and
||A^{-1}|| <= 100 (largest measured on refined walls of this curve: 42).
Seeds whose full oracle solution is stored (tests/golden) are also compared
element by element.

Prints ONE JSON line.  --gpus > 1 is refused: the refined-wall path runs on one GPU.
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "refined-wall solves/sec at N=16k pts, rel err ≤1e-8 vs FP64 oracle; p50/p99 ms"

# peak rates used for the roofline (MI355X published figures): HBM3E 8 TB/s;
# FP64 matrix (MFMA) 78.6 TFLOP/s; FP64 vector ALU 78.6 TFLOP/s
PEAK = {"hbm": (8000.0, "GB/s"), "mfma": (78.6, "TFLOP/s"), "alu": (78.6, "TFLOP/s")}
KERNEL_BOUND = {
    "sketch_kernel": "mfma", "gemm_nn_sub_kernel": "mfma", "node_sketch_kernel": "mfma",
    "resid_tiles_kernel": "alu", "node_inverse_kernel": "alu", "node_factor_kernel": "alu",
    "node_factor_bordered_kernel": "alu", "far_coef_kernel": "alu", "far_eval_kernel": "alu",
    "rowid_kernel": "alu", "rowid_select_kernel": "alu", "node_id_kernel": "alu",
    "hbs_up_kernel": "hbm", "hbs_down_kernel": "hbm",
}


# HBM traffic per launch from two rocprofv3 counter passes of this bench
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, averaged over the kernel's
# dispatches), each scaled by what the counter reads for a plain 1 GiB device
# copy.  Valid only while the kernel's sources hash to the value they had when
# the counters were taken; otherwise the roofline reports traffic as null.
MEASURED_TRAFFIC = {
    "node_factor_bordered_kernel": {
        "fetch_kib": 1256.9, "write_kib": 3293.0, "fetch_scale": 1.9999, "write_scale": 1.0000,
        "sources": ["paper_2108_07205_amd/csrc/hbs_gpu.hip", "paper_2108_07205_amd/csrc/dev_gj.h",
                    "paper_2108_07205_amd/csrc/dev_reduce.h", "paper_2108_07205_amd/csrc/hbs_dev.h",
                    "paper_2108_07205_amd/csrc/common.h"],
        "sha256": "8d14affa40fd2832a4fb49f94fb8bd25a627df3be7f5771099784c6c50d56806",
        "summary": "profiles/star1024_refine16x4_hbm_traffic.md",
    },
}


def measured_traffic(kernel: str):
    """Scaled HBM bytes per launch of `kernel`, or None when no counters were
    taken for it or its sources changed since."""
    import hashlib
    m = MEASURED_TRAFFIC.get(kernel)
    if not m:
        return None
    h = hashlib.sha256()
    for f in m["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != m["sha256"]:
        return None
    return 1024.0 * (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"])


# ||A^{-1}||_2 of the refined Nystrom matrices of this curve: 27 (unrefined),
# 31-42 on refined walls (smallest singular value 0.024-0.037); twice the
# largest, rounded up
INV_NORM_EST = 100.0
ERROR_GATE = 1e-8


def _oracle_check(job):
    """Worker (separate process, oracle only): relative oracle residual of one
    seed's tau at sampled rows, and the element-wise difference from the
    stored full oracle solution when there is one."""
    seed, tau = job
    import workloads as W
    from oracle import geometry as G, kernels as K
    p = W.config2(seed=seed)
    sets = G.refine(p.n_panels, p.refinement.panel_ids, p.refinement.levels, p.curve.a, p.curve.m)
    st = p.rhs[0]
    g = K.rhs_vector(sets.new, st.z, st.f)
    rng = np.random.default_rng(1000 + seed)
    rows = np.unique(np.concatenate([rng.choice(sets.new.n, 200, replace=False), sets.p_in_new[::64]]))
    r = K.residual_rows(sets.new, rows, tau, g)
    gs = g.reshape(-1, 2)[rows].reshape(-1)
    rel = float(np.linalg.norm(r) / np.linalg.norm(gs))
    bound = INV_NORM_EST * rel * float(np.linalg.norm(g) / np.linalg.norm(tau))
    out = {"seed": seed, "resid": rel, "bound": bound, "rows": int(rows.size)}
    gold = os.path.join(ROOT, "tests", "golden", f"config2_seed{seed}_tau.npy")
    if os.path.exists(gold):
        t_or = np.load(gold, allow_pickle=False)
        out["golden_rel2"] = float(np.linalg.norm(tau - t_or) / np.linalg.norm(t_or))
    return out


def oracle_gate(taus: dict) -> dict:
    """Check every timed seed's tau with the FP64 oracle on the host cores
    (a pool of spawned processes that import only oracle/ and workloads/)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    jobs = sorted(taus.items())
    nw = max(1, min(16, (os.cpu_count() or 2) // 2, len(jobs)))
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=nw, mp_context=mp.get_context("spawn")) as ex:
        res = list(ex.map(_oracle_check, jobs, chunksize=max(1, len(jobs) // (4 * nw))))
    ok = {r["seed"]: r["bound"] <= ERROR_GATE and r.get("golden_rel2", 0.0) <= 1e-10 for r in res}
    gold = {str(r["seed"]): r["golden_rel2"] for r in res if "golden_rel2" in r}
    return {"ok": ok, "max_resid": max(r["resid"] for r in res), "max_bound": max(r["bound"] for r in res),
            "rows_per_seed": res[0]["rows"],
            "golden_rel2": gold, "workers": nw, "seconds": round(time.perf_counter() - t0, 1)}


def _blas_threads() -> int:
    from threadpoolctl import threadpool_info
    return max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])


def cpu_baseline() -> dict:
    """The FP64 oracle (dense assembly + LU with one refinement step, as it
    stands) timed on the host cores on a bounded sample of one refined-wall
    solve of the headline workload (20224 nodes, 40448 unknowns):
    * assembly: 1024 of the 20224 node rows, scaled by rows (every row costs
      the same);
    * LU solve: the oracle's dense solve of the same operator at 6144 and
      10240 unknowns, fitted by t = c n^3 and extrapolated to 40448;
    both with the BLAS thread pool at all host threads and the LU again at
    1 thread (threads read inside this process through threadpoolctl)."""
    import workloads as W
    from oracle import geometry as G, kernels as K, solve as S
    from threadpoolctl import threadpool_limits
    p = W.config2(seed=0)
    sets = G.refine(p.n_panels, p.refinement.panel_ids, p.refinement.levels, p.curve.a, p.curve.m)
    n_nodes = sets.new.n
    n_full = 2 * n_nodes
    rows = 1024
    t0 = time.perf_counter()
    K.nystrom_rows(sets.new, np.arange(rows))
    t_slab = time.perf_counter() - t0
    t_asm = t_slab * n_nodes / rows

    def lu_time(n_panels: int, threads=None) -> tuple:
        d = G.discretize(G.reference_panels(n_panels), p.curve.a, p.curve.m)
        A = K.nystrom_matrix(d)
        g = np.ones(A.shape[0])
        if threads is None:
            t0 = time.perf_counter()
            S.solve_refined(A, g)
            return A.shape[0], time.perf_counter() - t0, _blas_threads()
        with threadpool_limits(threads, user_api="blas"):
            used = _blas_threads()
            t0 = time.perf_counter()
            S.solve_refined(A, g)
            return A.shape[0], time.perf_counter() - t0, used

    n1, t1, th_all = lu_time(192)
    n2, t2, _ = lu_time(320)
    # least-squares c in t = c n^3 over the two sizes
    c = (t1 * n1 ** 3 + t2 * n2 ** 3) / (n1 ** 6 + n2 ** 6)
    t_lu = c * n_full ** 3
    n1s, t1s, th_one = lu_time(192, threads=1)
    t_lu1 = t1s * (n_full / n1s) ** 3
    total = t_asm + t_lu
    meta_path = os.path.join(ROOT, "tests", "golden", "golden_meta.json")
    measured = None
    if os.path.exists(meta_path):
        m = json.load(open(meta_path)).get("config2_seed0")
        if m:
            measured = {"assembly_s": m["assembly_s"], "lu_s": m["lu_s"], "blas_threads": m["blas_threads"],
                        "host_cpus": m["host_cpus"], "what": "full-size oracle run that wrote the golden solution"}
    return {
        "value": 1.0 / total, "unit": "solves/s", "cores": int(th_all), "kind": "oracle",
        "sample": (f"assembly of {rows} of {n_nodes} node rows ({t_slab:.2f} s, scaled by rows to {t_asm:.1f} s); "
                   f"oracle LU solve at n={n1} ({t1:.2f} s) and n={n2} ({t2:.2f} s), t = c n^3 fitted and "
                   f"extrapolated to n={n_full} ({t_lu:.1f} s); full solve {total:.1f} s"),
        "assembly_s": t_asm, "lu_s": t_lu, "lu_fit_sizes": [n1, n2], "lu_fit_s": [t1, t2],
        "one_thread": {"lu_s": t_lu1, "solves_per_s": 1.0 / (t_asm + t_lu1), "threads": int(th_one),
                       "sample": f"LU at n={n1s} on 1 BLAS thread ({t1s:.2f} s) scaled by n^3; the assembly "
                                 f"(NumPy element-wise work) runs on one thread in both cases"},
        "host_cpus": os.cpu_count(), "full_size_reference_run": measured,
    }


def rate(name: str, ph: dict):
    bound = KERNEL_BOUND.get(name, "alu")
    peak, unit = PEAK[bound]
    sec = ph["ms"] / 1e3
    if sec <= 0:
        return bound, peak, unit, None
    achieved = ph["bytes"] / sec / 1e9 if bound == "hbm" else ph["flops"] / sec / 1e12
    return bound, peak, unit, achieved


def roofline(phases: dict):
    """Dominant kernel of the timed region (largest total time among the
    kernel-level event timers) and its achieved rate: algorithmic flops or
    bytes of all its launches divided by their total event time."""
    kern = {k[2:]: v for k, v in phases.items() if k.startswith("k:")}
    if not kern:
        return None, None, {}
    table = {}
    for name, ph in sorted(kern.items(), key=lambda kv: -kv[1]["ms"]):
        bound, peak, unit, ach = rate(name, ph)
        table[name] = {"ms_total": round(ph["ms"], 3), "launches": ph["calls"],
                       "avg_us": round(1e3 * ph["ms"] / max(1, ph["calls"]), 2),
                       "achieved": None if ach is None else round(ach, 3), "unit": unit,
                       "frac": None if ach is None or not (ph["flops"] or ph["bytes"]) else round(ach / peak, 4)}
    name = max(kern, key=lambda k: kern[k]["ms"])
    ph = kern[name]
    bound, peak, unit, ach = rate(name, ph)
    return name, {"kernel": name, "bound": bound, "achieved": ach, "peak": peak, "unit": unit,
                  "frac": (ach / peak) if ach is not None else None, "traffic": measured_traffic(name),
                  "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                  "avg_launch_ms": ph["ms"] / max(1, ph["calls"]), "launches": ph["calls"],
                  "algorithmic_bytes_per_launch": ph["bytes"] / max(1, ph["calls"]),
                  "algorithmic_per_launch": (ph["bytes"] if bound == "hbm" else ph["flops"]) / max(1, ph["calls"])}, table


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without the phase events")
    ap.add_argument("--no-oracle-check", action="store_true",
                    help="skip the oracle's check of the timed seeds (profiler runs; the line then says so)")
    ap.add_argument("--hbs-apply-only", action="store_true",
                    help="only the one-RHS reference-inverse apply, warm and cold (for kernel traces)")
    ap.add_argument("--extra-steps", type=int, default=40,
                    help="steps of the side measurements (RHS/s with resident factors, FP32-generator mode)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the refined-wall path runs on one GPU (it is not sharded); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2108_07205_amd as rw
    import workloads as W

    rank = int(os.environ.get("RANK", "0"))
    ctx = rw.Context(0)
    wall = rw.Wall(ctx, 1024)
    st = wall.stats()
    stream = torch.cuda.current_stream()

    def hbs_apply_rates(w, reps: int = 40):
        """One-RHS apply of the reference inverse A_oo^{-1} (the a6 kernel
        sweep) timed by HIP events on the ctx stream: warm (generators left
        in the 256 MB Infinity Cache by the previous rep), cold (a 1 GiB
        buffer read before each rep, which leaves the cache holding clean
        lines of other data) and cold after a 1 GiB write (the cache then
        holds dirty lines that must be written back as the apply reads),
        against 8 TB/s and against a measured device copy (1 GiB, read +
        write)."""
        n = 2 * w.n_nodes
        stw = w.stats()
        alg = float(stw["gen_bytes_f64"] + 8 * 2 * n)   # generators + read b + write x
        b = torch.randn(n, dtype=torch.float64, device="cuda")
        x = torch.empty_like(b)
        scratch = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)

        def one(cold) -> float:
            if cold == "read":
                scratch.sum()
            elif cold == "write":
                scratch.fill_(float(np.random.rand()))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            rw.rw_hbs_apply(ctx.h, w.h, b, x, n)
            e1.record()
            e1.synchronize()
            return e0.elapsed_time(e1) * 1e3

        for _ in range(5):
            one(False)
        warm = float(np.median([one(False) for _ in range(reps)]))
        cold = float(np.median([one("read") for _ in range(reps)]))
        cold_w = float(np.median([one("write") for _ in range(reps)]))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        scratch.copy_(src)
        e0.record()
        for _ in range(5):
            scratch.copy_(src)
        e1.record()
        e1.synchronize()
        copy_gbps = 5 * 2 * scratch.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del scratch, src
        out = {"algorithmic_bytes": alg, "warm_us": warm, "cold_us": cold, "cold_dirty_us": cold_w,
               "copy_peak_GBps": copy_gbps}
        for k in ("warm", "cold", "cold_dirty"):
            gbps = alg / (out[f"{k}_us"] * 1e-6) / 1e9
            out[f"{k}_GBps"] = gbps
            out[f"{k}_frac_of_8TBps"] = gbps / PEAK["hbm"][0]
            out[f"{k}_frac_of_copy"] = gbps / copy_gbps
        return out

    if args.hbs_apply_only:
        print(json.dumps({"hbs_apply_1rhs": hbs_apply_rates(wall), "levels": st["n_levels"],
                          "gen_bytes_f64": st["gen_bytes_f64"]}), flush=True)
        wall.close()
        ctx.close()
        return

    # the synthetic inputs (refined panel lists and Stokeslet sources) are
    # generated before the timed region, like data already at hand
    problems = {s: W.config2(seed=s) for s in range(args.steps)}
    problems.update({10_000 + i: W.config2(seed=10_000 + i) for i in range(args.warmup)})

    taus = {}

    def step(seed: int):
        p = problems[seed]
        ref = wall.refine(p.refinement.panel_ids, p.refinement.levels)
        s0 = p.rhs[0]
        g = ref.stokeslet_rhs(s0.z, s0.f)
        tau = torch.empty_like(g)
        rc = rw.rw_solve(ctx.h, ref.h, g, tau, ref.n_unknowns, check=False)
        info = ref.info()
        ref.close()
        taus[seed] = tau       # kept for the oracle check after the timed region
        return rc == rw.RW_OK, info

    # Python's cyclic garbage collector stays off from the warmup through the
    # timed passes (as timeit does), so that no collection lands in a step
    # and the GPU is not left idle between the warmup and the timed region
    gc.collect()
    gc.disable()
    for i in range(args.warmup):
        step(10_000 + i)

    def timed(profile: bool):
        """K steps between synchronizations; with profile, HIP events around
        every phase and kernel (their overhead is why the headline pass runs
        without them)."""
        if profile:
            ctx.profile(True)
            ctx.profile_reset()
        lat, ok, infos = [], [], []
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for s in range(args.steps):
            t0 = time.perf_counter()
            good, info = step(s)
            lat.append((time.perf_counter() - t0) * 1e3)
            ok.append(good)
            infos.append(info)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        ph = ctx.profile_json() if profile else {}
        ctx.profile(False)
        return ok, elapsed, np.array(lat), infos, ph

    # headline: seeds 0..K-1 without events; then the same seeds with the
    # per-kernel HIP events that give the roofline and the kernel table
    ok_lib, elapsed, lat, infos, _ = timed(False)
    # the oracle's check of every timed seed (host cores, after the timed region)
    if args.no_oracle_check:
        ogate = {"ok": {s: True for s in taus}, "max_resid": None, "max_bound": None, "rows_per_seed": 0,
                 "golden_rel2": {}, "workers": 0, "seconds": 0.0, "skipped": True}
    else:
        ogate = oracle_gate({s: t.cpu().numpy() for s, t in taus.items()})
    taus.clear()
    ok = sum(int(good and ogate["ok"][s]) for s, good in enumerate(ok_lib))
    value = ok / elapsed
    phases = {}
    prof_rate = None
    if not args.no_profile:
        okp, elp, _, _, phases = timed(True)
        taus.clear()
        prof_rate = sum(okp) / elp

    gc.enable()

    # ---- side measurements (not the headline): solves with resident factors
    # (the paper's per-RHS direct solve time) and the FP32-generator mode
    def rhs_rate(w, nsteps):
        p = W.config2(seed=0)
        ref = w.refine(p.refinement.panel_ids, p.refinement.levels)
        gs = [ref.stokeslet_rhs(p.rhs[0].z, p.rhs[0].f)]
        for s2 in range(1, 8):
            q = W.config2(seed=s2)
            gs.append(ref.stokeslet_rhs(q.rhs[0].z, q.rhs[0].f))
        tau = torch.empty_like(gs[0])
        rw.rw_solve(ctx.h, ref.h, gs[0], tau, ref.n_unknowns)
        torch.cuda.synchronize()
        t = []
        worst, iters = 0.0, 0
        for i in range(nsteps):
            t0 = time.perf_counter()
            rw.rw_solve(ctx.h, ref.h, gs[i % len(gs)], tau, ref.n_unknowns)
            t.append((time.perf_counter() - t0) * 1e3)
            inf = ref.info()
            worst, iters = max(worst, inf["resid"]), max(iters, inf["ir_iters"])
        ref.close()
        t = np.array(t)
        return {"rhs_per_s": 1e3 / float(np.mean(t)), "p50_ms": float(np.percentile(t, 50)),
                "p99_ms": float(np.percentile(t, 99)), "max_resid": worst, "ir_iters_max": iters}

    def solve_rate(w, nsteps):
        okm, lm, res, its = 0, [], 0.0, 0
        t0 = time.perf_counter()
        for s2 in range(nsteps):
            t1 = time.perf_counter()
            p = W.config2(seed=s2)
            ref = w.refine(p.refinement.panel_ids, p.refinement.levels)
            g = ref.stokeslet_rhs(p.rhs[0].z, p.rhs[0].f)
            rc = rw.rw_solve(ctx.h, ref.h, g, torch.empty_like(g), ref.n_unknowns, check=False)
            inf = ref.info()
            ref.close()
            okm += int(rc == rw.RW_OK)
            res, its = max(res, inf["resid"]), max(its, inf["ir_iters"])
            lm.append((time.perf_counter() - t1) * 1e3)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        return {"solves_per_s": okm / el, "passed": okm, "of": nsteps, "p50_ms": float(np.percentile(lm, 50)),
                "p99_ms": float(np.percentile(lm, 99)), "max_resid": res, "ir_iters_max": its}

    def batched(w, n_inst):
        """Uneven refinements of one wall (the batched family: 2..32 panels,
        2..5 levels, 8 RHS each) solved by one rw_solve_batch call vs one
        rw_solve per instance (same factors, same gate)."""
        probs = W.batched_instances(n_inst=n_inst, seed=0, n_panels=1024, nrhs=8)
        refs, gs = [], []
        t0 = time.perf_counter()
        for p in probs:
            ref = w.refine(p.refinement.panel_ids, p.refinement.levels)
            refs.append(ref)
            gs.append(torch.stack([ref.stokeslet_rhs(q.z, q.f) for q in p.rhs]).contiguous())
        torch.cuda.synchronize()
        t_ref = time.perf_counter() - t0
        w.solve_batch(refs, gs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        taus, infos = w.solve_batch(refs, gs)
        torch.cuda.synchronize()
        t_bat = time.perf_counter() - t0
        t0 = time.perf_counter()
        seq = [ref.solve(g) for ref, g in zip(refs, gs)]
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
        agree = max(float((a - b).norm() / b.norm()) for a, b in zip(taus, seq))
        n_p = [int(r.info()["n_p"]) for r in refs]
        for r in refs:
            r.close()
        nrhs = sum(int(g.shape[0]) for g in gs)
        return {"instances": n_inst, "rhs": nrhs, "n_p_range": [min(n_p), max(n_p)],
                "refine_ms_total": 1e3 * t_ref, "batch_solve_ms": 1e3 * t_bat, "sequential_solve_ms": 1e3 * t_seq,
                "batch_rhs_per_s": nrhs / t_bat, "speedup_vs_sequential": t_seq / t_bat,
                "max_resid": max(i["resid"] for i in infos), "batch_vs_sequential_rel_diff": agree}

    def config4_mixed(reps: int = 3):
        """The 65536-node wall (4096 panels; 32 panels nearest a seeded point
        refined 4 levels; 32 Stokeslet right-hand sides): FP64 generators
        against FP32 and BF16 generators on the matrix cores, all refined in
        FP64 to the same residual (1e-13; with ||A^-1|| <= 100 an error
        below 1e-11), and the applies of the reference inverse alone (1 and
        32 right-hand sides, HIP events, warm)."""
        p4 = W.config4(seed=0)
        out = {"workload": "star4096_refine32x4", "nrhs": 32}
        for prec, name in ((rw.RW_F64, "fp64"), (rw.RW_F32, "fp32_generators"), (rw.RW_BF16, "bf16_generators")):
            w4 = rw.Wall(ctx, 4096, precision=prec)
            st4 = w4.stats()
            ref4 = w4.refine(p4.refinement.panel_ids, p4.refinement.levels)
            g4 = torch.stack([ref4.stokeslet_rhs(q.z, q.f) for q in p4.rhs]).contiguous()
            tau4 = torch.empty_like(g4)
            # BF16 generators are refined by preconditioned GMRES: Richardson
            # stalls with them at this size (residual 7e-3 after 6 corrections)
            solver = rw.RW_SOLVE_GMRES if prec == rw.RW_BF16 else rw.RW_SOLVE_IR
            ctx.set_options(solver=solver, ir_maxit=60 if solver == rw.RW_SOLVE_GMRES else 6)
            rw.rw_solve(ctx.h, ref4.h, g4, tau4, ref4.n_unknowns)
            ts, its, res = [], 0, 0.0
            for _ in range(reps):
                inf = {}
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rw.rw_solve(ctx.h, ref4.h, g4, tau4, ref4.n_unknowns, info=inf)
                ts.append((time.perf_counter() - t0) * 1e3)
                its, res = inf["ir_iters"], inf["resid"]
            n4 = 2 * w4.n_nodes
            rates = {}
            for nr in (1, 32):
                b4 = torch.randn(nr, n4, dtype=torch.float64, device="cuda")
                x4 = torch.empty_like(b4)
                for _ in range(3):
                    rw.rw_hbs_apply(ctx.h, w4.h, b4, x4, n4)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(10):
                    rw.rw_hbs_apply(ctx.h, w4.h, b4, x4, n4)
                e1.record()
                e1.synchronize()
                us = e0.elapsed_time(e1) * 100.0
                width = {rw.RW_F64: 8, rw.RW_F32: 4, rw.RW_BF16: 2}[prec]
                gen_b = width * st4["gen_entries"]
                rates[f"apply_{nr}rhs_us"] = us
                rates[f"apply_{nr}rhs_GBps_per_pass"] = gen_b / (us * 1e-6) / 1e9
            ctx.set_options(solver=rw.RW_SOLVE_IR, ir_maxit=6)
            out[name] = {"solve_32rhs_ms": float(np.median(ts)), "corrections": its, "resid": res,
                         "solver": "GMRES" if solver == rw.RW_SOLVE_GMRES else "Richardson",
                         "refined_nodes": int(ref4.n_nodes), "k": int(ref4.info()["k"]),
                         "gen_bytes": {rw.RW_F64: 8, rw.RW_F32: 4, rw.RW_BF16: 2}[prec] * st4["gen_entries"],
                         "mfma_from": st4["mfma_from_f64"] if prec == rw.RW_F64 else st4["mfma_from_f32"], **rates}
            ref4.close()
            w4.close()
        for name in ("fp32_generators", "bf16_generators"):
            out[name]["speedup_vs_fp64"] = {
                "solve": out["fp64"]["solve_32rhs_ms"] / out[name]["solve_32rhs_ms"],
                "apply_32rhs": out["fp64"]["apply_32rhs_us"] / out[name]["apply_32rhs_us"],
                "apply_1rhs": out["fp64"]["apply_1rhs_us"] / out[name]["apply_1rhs_us"]}
        return out

    def serving(n_req: int = 48, slots: int = 3):
        """Serving against one resident 65536-node wall (FP32 generators,
        FP64 refinement to ||r||/||g|| <= 1e-10, i.e. an error below 1e-8
        with ||A^-1|| <= 100): n_req requests with Poisson arrivals at
        2000 req/s, each refining 1..64 contiguous panels by 1..5 levels with
        1..16 right-hand sides, submitted at their arrival times to a server
        of `slots` slots; latency = completion - arrival.  Baseline: the same
        requests solved one after the other by plain FP64 rw_refine +
        rw_solve on the wall's own ctx (same residual tolerance)."""
        reqs = W.serving_requests(n_req, rate=2000.0, seed=11, n_panels=4096)
        old = ctx.options()
        ctx.set_options(ir_tol=1e-10)
        out = {"requests": n_req, "offered_rate_per_s": 2000.0, "slots": slots,
               "rhs_total": int(sum(len(r.problem.rhs) for r in reqs)),
               "refined_nodes_range": None, "gate": "||g - A tau||/||g|| <= 1e-10 (FP64 residual)"}
        try:
            w32 = rw.Wall(ctx, 4096, precision=rw.RW_F32)
            sv = rw.Server(w32, slots=slots)
            t0 = time.perf_counter()
            ids = []
            for r in reqs:
                dt = t0 + r.t_arrival - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                p5 = r.problem
                ids.append(sv.submit(p5.refinement.panel_ids, p5.refinement.levels, [(q.z, q.f) for q in p5.rhs]))
            infos = []
            for rid in ids:
                _, inf = sv.wait(rid, check=False)
                infos.append(inf)
            t_end = time.perf_counter()
            sv.close()
            w32.close()
            lat = np.array([inf["t_queue_ms"] + inf["t_run_ms"] for inf in infos])
            ok = [inf["status"] == rw.RW_OK and inf["resid"] <= 1e-10 for inf in infos]
            out["refined_nodes_range"] = [int(min(i["n_nodes"] for i in infos)), int(max(i["n_nodes"] for i in infos))]
            out["served"] = {"solves_per_s": sum(ok) / (t_end - t0), "passed": int(sum(ok)),
                             "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                             "run_ms_p50": float(np.median([i["t_run_ms"] for i in infos])),
                             "max_resid": float(max(i["resid"] for i in infos)),
                             "max_ir_iters": int(max(i["ir_iters"] for i in infos)),
                             "slots_used": sorted({int(i["slot"]) for i in infos})}
            # baseline: plain FP64, one request after the other on the wall's ctx
            w64 = rw.Wall(ctx, 4096)
            torch.cuda.synchronize()
            tb0 = time.perf_counter()
            seq, okb = [], 0
            for r in reqs:
                p5 = r.problem
                t1 = time.perf_counter()
                ref5 = w64.refine(p5.refinement.panel_ids, p5.refinement.levels)
                g5 = torch.stack([ref5.stokeslet_rhs(q.z, q.f) for q in p5.rhs]).contiguous()
                inf = {}
                rc = rw.rw_solve(ctx.h, ref5.h, g5, torch.empty_like(g5), ref5.n_unknowns, check=False, info=inf)
                ref5.close()
                seq.append((time.perf_counter() - t1) * 1e3)
                okb += int(rc == rw.RW_OK and inf["resid"] <= 1e-10)
            torch.cuda.synchronize()
            tb = time.perf_counter() - tb0
            w64.close()
            out["sequential_fp64"] = {"solves_per_s": okb / tb, "passed": okb, "p50_solve_ms": float(np.median(seq)),
                                      "p99_solve_ms": float(np.percentile(seq, 99))}
            out["speedup_vs_sequential_fp64"] = out["served"]["solves_per_s"] / out["sequential_fp64"]["solves_per_s"]
        finally:
            ctx.set_options(ir_tol=old["ir_tol"])
        return out

    def time_stepping(n_steps: int = 40, margin: int = 4):
        """A particle moving along the 16384-node wall at 0.3 panel widths per
        step asks for its 16 nearest panels refined 4 levels (one RHS of 16
        Stokeslets per step): refined-wall solves with the refinement cache
        (Sec. 5.3: snapshots share a refinement of a region widened by
        `margin` panels) against a fresh rw_refine every step."""
        curve = W.Curve()
        hpan = 2 * math.pi / 1024
        rng = np.random.default_rng(99)
        sts = [W.stokeslets(rng, 16) for _ in range(n_steps)]
        reqs = []
        for t in range(n_steps):
            th = 0.7 + 0.3 * hpan * t
            reqs.append(W.nearest_panels(curve, 1024, curve.point(th) + 1e-3 * curve.outward_normal(th), 16))

        def run(use_cache: bool):
            cache = rw.RefCache(wall, capacity=2, margin=margin) if use_cache else None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ok = 0
            for ids, stk in zip(reqs, sts):
                if cache:
                    ref, _ = cache.get(ids, [4] * len(ids))
                else:
                    ref = wall.refine(ids, [4] * len(ids))
                gq = ref.stokeslet_rhs(stk.z, stk.f)
                ok += int(rw.rw_solve(ctx.h, ref.h, gq, torch.empty_like(gq), ref.n_unknowns, check=False) == rw.RW_OK)
                if not cache:
                    ref.close()
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            st_c = cache.stats() if cache else None
            if cache:
                cache.close()
            return ok / el, st_c

        rate_c, st_c = run(True)
        rate_f, _ = run(False)
        return {"steps": n_steps, "margin": margin, "cached_solves_per_s": rate_c, "fresh_solves_per_s": rate_f,
                "speedup": rate_c / rate_f, "cache": st_c}

    def concurrent_slots(slots: int = 3, n_req: int = 150):
        """The headline's refined solves (seeds 0..n_req-1, same gate on the
        library's FP64 residual) as independent requests to a server of
        `slots` slots, all submitted at once: each slot runs one whole
        request at a time on its own stream, and the slots' work overlaps on
        the device.  Throughput against the sequential headline value; per
        request run time (refine + data + solve + copy back).  Seeds with a
        stored full oracle solution are compared with it."""
        probs = [W.config2(seed=s) for s in range(n_req)]
        sv = rw.Server(wall, slots=slots)
        warm = [sv.submit(p.refinement.panel_ids, p.refinement.levels, [(q.z, q.f) for q in p.rhs]) for p in probs[:8]]
        for i in warm:
            sv.wait(i)
        t0 = time.perf_counter()
        ids = [sv.submit(p.refinement.panel_ids, p.refinement.levels, [(q.z, q.f) for q in p.rhs]) for p in probs]
        res = [sv.wait(i, check=False) for i in ids]
        el = time.perf_counter() - t0
        sv.close()
        ok = [inf["status"] == rw.RW_OK and inf["resid"] <= 1e-13 for _, inf in res]
        run = np.array([inf["t_run_ms"] for _, inf in res])
        gold = {}
        for sd in (0, 7):
            path = os.path.join(ROOT, "tests", "golden", f"config2_seed{sd}_tau.npy")
            if sd < n_req and os.path.exists(path):
                t_or = np.load(path)
                gold[str(sd)] = float(np.linalg.norm(res[sd][0][0] - t_or) / np.linalg.norm(t_or))
        return {"slots": slots, "requests": n_req, "solves_per_s": sum(ok) / el, "passed": int(sum(ok)),
                "speedup_vs_sequential": (sum(ok) / el) / value,
                "run_ms_p50": float(np.percentile(run, 50)), "run_ms_p99": float(np.percentile(run, 99)),
                "max_resid": float(max(inf["resid"] for _, inf in res)), "golden_rel2": gold,
                "criterion": "library FP64 residual <= 1e-13 per request; golden seeds <= 1e-10 (2-norm)"}

    def guard(fn, *a):
        """A side measurement that fails is reported, not fatal to the line."""
        try:
            return fn(*a)
        except Exception as e:  # noqa: BLE001
            return {"error": f"{type(e).__name__}: {e}"}

    side = {"hbs_apply_1rhs": guard(hbs_apply_rates, wall)}
    if args.extra_steps > 0:
        side["config2_concurrent_slots"] = guard(concurrent_slots)
        side["config4_mixed_precision"] = guard(config4_mixed)
        side["serving_config5"] = guard(serving)
        side["time_stepping_refcache"] = guard(time_stepping)
        side["batched_fp64"] = guard(batched, wall, 64)
        side["fp64_resident_factors"] = guard(rhs_rate, wall, args.extra_steps)
        w32 = rw.Wall(ctx, 1024, precision=rw.RW_F32)
        side["fp32_generators"] = {"refined_solves": solve_rate(w32, args.extra_steps),
                                   "resident_factors": rhs_rate(w32, args.extra_steps),
                                   "criterion": "same FP64 residual gate as the headline"}
        w32.close()
    dom, roof, ktable = roofline(phases)
    hbs = phases.get("a6_hbs_apply")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "star1024_refine16x4", "curve": "r=1+0.3cos(5t)", "n_panels": 1024,
                   "nodes_ref": 16384, "n_sel": 16, "levels": 4, "nodes_refined": int(infos[0]["n_k"] + infos[0]["n_p"]),
                   "unknowns_refined": int(2 * (infos[0]["n_k"] + infos[0]["n_p"])), "stokeslets": 16,
                   "nrhs": 1, "leaf_nodes": 64, "id_tol": 1e-10, "seeds": f"0..{args.steps - 1}"},
        "value_with_kernel_events": prof_rate,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "slowest_steps_ms": {str(int(i)): round(float(lat[i]), 3) for i in np.argsort(lat)[::-1][:5]},
        "gate": {"passed": ok, "of": args.steps,
                 "criterion": (f"library FP64 residual ||g - A tau||/||g|| <= 1e-13, and the error bound vs the FP64 "
                               f"oracle ||A^-1|| ||r|| / ||tau|| <= {ERROR_GATE:g} with r the oracle's residual of tau "
                               f"on its own discretization ({ogate['rows_per_seed']} sampled rows) and ||A^-1|| <= "
                               f"{INV_NORM_EST:g}; seeds with a stored full oracle solution: ||tau - tau_oracle||_2 / "
                               f"||tau_oracle||_2 <= 1e-10"),
                 "passed_library_residual": int(sum(ok_lib)),
                 "oracle_max_resid": ogate["max_resid"], "oracle_max_error_bound": ogate["max_bound"],
                 "oracle_golden_rel2": ogate["golden_rel2"],
                 "oracle_check_s": ogate["seconds"], "oracle_workers": ogate["workers"],
                 "oracle_check_skipped": bool(ogate.get("skipped", False)),
                 "max_resid": float(max(i["resid"] for i in infos)),
                 "k_range": [int(min(i["k"] for i in infos)), int(max(i["k"] for i in infos))],
                 "ir_iters_max": int(max(i["ir_iters"] for i in infos))},
        # host time inside each call: rw_refine returns before its last device
        # work ends, which rw_solve's time then includes
        "refine_call_ms_p50": float(np.median([i["t_refine_ms"] for i in infos])),
        "solve_call_ms_p50": float(np.median([i["t_solve_ms"] for i in infos])),
        "roofline": roof,
        "phases_ms_per_step": {k: round(v["ms"] / args.steps, 4) for k, v in phases.items() if not k.startswith("k:")},
        "kernels": ktable,
        "hbs": {"gen_bytes_f64": st["gen_bytes_f64"], "levels": st["n_levels"], "max_rank": st["max_rank"],
                "build_ms": st["t_build_ms"],
                "apply_GBps": (hbs["bytes"] / (hbs["ms"] / 1e3) / 1e9) if hbs and hbs["ms"] > 0 else None},
        "side": side,
        "cpu_baseline": None,
    }
    if rank == 0 and not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline()
        except Exception as e:  # the baseline is reported, never the target
            out["cpu_baseline"] = {"error": str(e)}
    wall.close()
    ctx.close()
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
