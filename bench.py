#!/usr/bin/env python3
"""Benchmark of the stochastic-Galerkin slab hot path on one MI355X.

Metric (one JSON line on stdout):
  * value = SG operator apply throughput in GDoF/s (N_DoF per apply / apply time) on the 3D
    workload "Q2 on 32^3 cells, dG(1), M = 4, p_xi = 3" (19,223,750 DoFs), with % of HBM peak;
  * solve = FGMRES-GMG slab solve time to a true relative residual of 1e-8, FP64 and mixed.
A step is one FP64 slab solve (FGMRES + V-cycles + Vanka + applies: the whole path); the apply
rate is timed separately over rotating input/output pairs so the 256 MB Infinity Cache cannot hold
them.  All inputs are synthetic and seeded.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 (vector and matrix)


def apply_model(w):
    """Algorithmic bytes and flops of one operator apply (definitions in the design doc).

    bytes: read x, write y (8 B per DoF each) and read the coefficient at the quadrature points.
    flops: sum-factorised evaluation as implemented (FMA = 2 flops): per cell and component
           4 d (k+1)^(d+1) FMAs for interpolation, derivatives and their transposes, N_t + 1 per
           point for the mass term, and 3 flops per coupling entry per point and direction.
    """
    d, k, nt = w.dim, w.fe_degree, w.n_time
    n1 = k + 1
    npnt = n1 ** d
    cells = w.n_cells_1d ** d
    nxi = w.n_chaos
    # affine coefficient: G_0 = I (N_xi entries); G_{e_m} pairs alpha with alpha + e_m, which exists for
    # every alpha of total degree <= p_xi - 1, in both orders
    M, p = w.n_vars, w.chaos_degree
    nnz = nxi + (2 * M * math.comb(M + p - 1, p - 1) if p >= 1 else 0)
    n_mu = M + 1
    n_dof = w.n_dofs(0)
    bytes_ = 8 * 2 * n_dof + 8 * n_mu * cells * npnt
    per_cell_comp = 2 * 4 * d * n1 ** (d + 1) + npnt * (2 * nt + 1)
    coupling = 3 * d * npnt * nnz * nt          # summed over all components of a cell
    flops = cells * (nxi * nt * per_cell_comp + coupling)
    return n_dof, bytes_, flops


def cpu_baseline(w, seconds_target=15.0):
    """The oracle's route-2 apply (scipy sparse x dense blocks), single thread, on a reduced mesh of
    the same discretisation; assembly is not timed (as on the GPU)."""
    from threadpoolctl import threadpool_limits
    import sg_inputs
    from oracle.slab import from_workload
    n_small = 12 if w.dim == 3 else 64
    ws = w.with_(n_cells_1d=n_small, n_levels=1)
    with threadpool_limits(limits=1):
        P = from_workload(ws)
        x = sg_inputs.uniform_vector(P.n, sg_inputs.SEED_APPLY_INPUT)
        P.apply_route2(x)
        t0 = time.perf_counter()
        reps = 0
        while True:
            P.apply_route2(x)
            reps += 1
            if time.perf_counter() - t0 > seconds_target or reps >= 50:
                break
        dt = (time.perf_counter() - t0) / reps
    return {"value": P.n / dt / 1e9, "unit": "GDoF/s", "cores": 1, "kind": "oracle",
            "sample": f"route-2 Kronecker apply (scipy CSR x dense), same k/r/M/p_xi on {n_small}^{w.dim} cells "
                      f"({P.n} DoFs), {reps} applies, assembly excluded, 1 thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed FP64 slab solves")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--only-apply", action="store_true", help="skip the solves (for profiling the apply)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device copy 5 times (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is described in DESIGN.md, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    import sg_inputs
    from paper_2605_21046_amd import sgheat

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        a = torch.rand(64 * 1024 * 1024, dtype=torch.float64, device=dev)
        c = torch.empty_like(a)
        for _ in range(5):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": a.numel() * 8, "copy_calibration_bytes_written": c.numel() * 8}))
        return
    w = sg_inputs.WORKLOADS[args.workload]
    stream = torch.cuda.current_stream()
    t_setup = time.perf_counter()
    G = sgheat.problem_from_workload(w, sgheat.SG_FP64)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    n = G.n(0)
    print(f"[bench] {args.workload}: {n} DoFs, setup {setup_s:.2f} s", file=sys.stderr, flush=True)

    # ---- operator apply over rotating (x, y) pairs --------------------------------------------------
    n_dof, abytes, aflops = apply_model(w)
    pairs = max(1, math.ceil(1.2e9 / (16 * n)))
    xs = [torch.from_numpy(sg_inputs.uniform_vector(n, sg_inputs.SEED_APPLY_INPUT + 100 * i)).to(dev)
          for i in range(pairs)]
    ys = [torch.empty_like(xs[0]) for _ in range(pairs)]
    for i in range(5):
        G.apply(xs[i % pairs], ys[i % pairs])
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for i in range(args.apply_reps):
        G.apply(xs[i % pairs], ys[i % pairs])
    ev1.record(stream)
    torch.cuda.synchronize()
    t_apply = ev0.elapsed_time(ev1) / 1e3 / args.apply_reps
    gdofs = n_dof / t_apply / 1e9
    achieved_gbs = abytes / t_apply / 1e9
    achieved_tf = aflops / t_apply / 1e12
    print(f"[bench] apply {t_apply * 1e6:.1f} us  {gdofs:.1f} GDoF/s  {achieved_gbs:.0f} GB/s  "
          f"{achieved_tf:.1f} TFLOP/s", file=sys.stderr, flush=True)
    del xs, ys

    out = {"metric": "SG operator apply GDoF/s + % HBM peak; FGMRES-GMG slab solve time, FP64 vs mixed",
           "value": round(gdofs, 3), "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded PCG64 U[-1,1] input; analytic sine-mode coefficient)",
           "config": {"workload": f"{args.workload}: {w.dim}D Q{w.fe_degree} on {w.n_cells_1d}^{w.dim} cells, "
                                  f"dG({w.time_degree}), M={w.n_vars}, p_xi={w.chaos_degree} ({w.n_chaos} modes), "
                                  f"{n_dof} DoFs, {w.n_levels}-level GMG", "n_dofs": n_dof},
           "apply_us": round(t_apply * 1e6, 2),
           "roofline": {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                        "kernel": "sg_operator_apply (2^d colour launches of k_apply)",
                        "algorithmic_bytes_per_apply": abytes},
           "roofline_fp64": {"bound": "alu", "achieved": round(achieved_tf, 2), "peak": FP64_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(achieved_tf / FP64_PEAK_TFLOPS, 4),
                             "algorithmic_flops_per_apply": aflops},
           "setup_s": round(setup_s, 2)}

    # ---- slab solves -------------------------------------------------------------------------------
    if not args.only_apply:
        xstar = sg_inputs.uniform_vector(n, sg_inputs.SEED_SOLVE_TARGET)
        xg = torch.from_numpy(xstar).to(dev)
        # right-hand side b = AA x* for a seeded x*; the identity rows carry x* on Dirichlet DoFs
        b = G.apply(xg)
        torch.cuda.synchronize()
        x = torch.zeros_like(b)

        def run_solves(P, count):
            times, infos = [], []
            for _ in range(count):
                x.zero_()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                _, info = P.solve(b, x, rtol=1e-8, max_iter=500)
                e1.record(stream)
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
                infos.append(info)
            return times, infos

        run_solves(G, args.warmup)
        t64, i64 = run_solves(G, args.steps)
        x64 = x.clone()
        res = {"fp64_ms": round(float(np.mean(t64)), 2), "fp64_iterations": i64[-1]["iterations"],
               "fp64_rel_residual_true": i64[-1]["rel_residual_true"],
               "fp64_t_apply_ms": round(i64[-1]["t_apply_ms"], 2), "fp64_t_prec_ms": round(i64[-1]["t_prec_ms"], 2),
               "fp64_applies": i64[-1]["applies"], "work_proxy": i64[-1]["work_proxy"]}
        out["ms_per_step"] = res["fp64_ms"]
        print(f"[bench] fp64 solve {res['fp64_ms']} ms, {res['fp64_iterations']} it", file=sys.stderr, flush=True)
        if not args.no_mixed:
            G32 = sgheat.problem_from_workload(w, sgheat.SG_MIXED)
            run_solves(G32, args.warmup)
            t32, i32 = run_solves(G32, args.steps)
            err = float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
            res.update({"mixed_ms": round(float(np.mean(t32)), 2), "mixed_iterations": i32[-1]["iterations"],
                        "mixed_rel_residual_true": i32[-1]["rel_residual_true"],
                        "mixed_vs_fp64_solution_rel_diff": err,
                        "mixed_speedup": round(float(np.mean(t64)) / float(np.mean(t32)), 3)})
            print(f"[bench] mixed solve {res['mixed_ms']} ms, {res['mixed_iterations']} it", file=sys.stderr,
                  flush=True)
            G32.close()
        out["solve"] = res
    else:
        out["ms_per_step"] = round(t_apply * 1e3, 4)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
        print(f"[bench] cpu baseline {out['cpu_baseline']['value']:.4f} GDoF/s", file=sys.stderr, flush=True)
    G.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
