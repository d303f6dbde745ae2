#!/usr/bin/env python3
"""Benchmark of the stochastic-Galerkin slab hot path on one MI355X.

One JSON line on stdout:
  * value = SG operator apply throughput in GDoF/s (N_DoF / median apply time) on the 3D workload
    "Q2 on 32^3 cells, dG(1), M = 4, p_xi = 3" (19,223,750 DoFs), timed over rotating input/output
    pairs so the 256 MB Infinity Cache cannot hold them;
  * roofline = the apply against the 8 TB/s HBM peak: algorithmic bytes (read x, write y, read the
    coefficient at the quadrature points) over the apply time, with the HBM bytes rocprofv3's
    FETCH_SIZE / WRITE_SIZE counters measured for the same kernels (`traffic`);
    roofline_fp64 = the same apply against the FP64 peak with the flop count of the sum-factorised
    method (even-odd 1D contractions), not the count of the code as written;
  * solve = FGMRES-GMG slab solve time to a true relative residual of 1e-8, FP64 and mixed; a step is
    one FP64 slab solve (FGMRES + V-cycles + Vanka + applies: the whole path);
  * c3 = the same apply and solve figures for "Q3 on 24^3 cells, dG(2), M = 3, p_xi = 4"
    (40,846,785 DoFs), where the mixed-precision solve is to beat the FP64 one;
  * cpu_baseline = the FP64 CPU oracle's apply on the full 3D Q2 workload, one thread and all of
    this process's cores.
All inputs are synthetic and seeded.
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

_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2605_21046_amd", "csrc")
# sources of the two kernels of one operator apply (k_apply, then k_node_gather)
APPLY_SOURCES = ["device_common.hpp", "kernels.hpp", "apply_impl.hpp", "apply_3d_f64.hip", "apply_2d_f64.hip",
                 "kernels_apply.hip", "kernels_misc.hip"]

# HBM bytes per operator apply from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (k_apply + k_node_gather),
# each scaled by what the same counter reads for a plain device copy of known size.  Keyed by workload,
# by the hash of the kernel sources the counters were taken on and by the apply's cells per workgroup:
# after any change to those the entry no longer matches and the traffic is reported as null until it
# is measured again.
MEASURED_TRAFFIC = {
    # profiles/sg_apply_c2_c3_hbm_traffic.md
    ("c2", "29658c635a08167e", 3): {"fetch_bytes": 645793914, "write_bytes": 547435020},
    ("c3", "29658c635a08167e", 2): {"fetch_bytes": 1241649678, "write_bytes": 1001379419},
}


def apply_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in APPLY_SOURCES:
        with open(os.path.join(_CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def apply_model(w):
    """Algorithmic bytes and flops of one operator apply.

    bytes: what the method must move: read x, write y (8 B per DoF each) and read the coefficient at
           the quadrature points (the geometry of a uniform Cartesian mesh is implicit).
    flops: the sum-factorised method with even-odd decomposition of the 1D contractions (FMA = 2 flops):
           per cell and component 4 d (k+1)^(d+1) for interpolating values and gradients to the
           quadrature points and integrating back, and per cell and point the quadrature-point work
           2 d N_t (N_xi + nnz_G) (chaos coupling of the gradient: G_0 = I plus the off-diagonal
           entries of the G_{e_m}) + 2 N_t^2 N_xi (time coupling of the mass term) + 2 d N_t N_xi
           (coefficient scaling).  flops_plain is the same without the even-odd halving.
    """
    d, k, nt = w.dim, w.fe_degree, w.n_time
    n1 = k + 1
    npnt = n1 ** d
    cells = w.n_cells_1d ** d
    nxi = w.n_chaos
    # affine coefficient: G_{e_m} pairs alpha with alpha + e_m, which exists for every alpha of total
    # degree <= p_xi - 1, in both orders
    M, p = w.n_vars, w.chaos_degree
    nnz_off = 2 * M * math.comb(M + p - 1, p - 1) if p >= 1 else 0
    n_mu = M + 1
    n_dof = w.n_dofs(0)
    bytes_ = 8 * 2 * n_dof + 8 * n_mu * cells * npnt
    sweeps = 4 * d * n1 ** (d + 1)
    point = npnt * (2 * d * nt * (nxi + nnz_off) + 2 * nt * nt * nxi + 2 * d * nt * nxi)
    flops = cells * (nxi * nt * sweeps + point)
    flops_plain = cells * (nxi * nt * 2 * sweeps + point)
    return n_dof, bytes_, flops, flops_plain


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_threads() -> int:
    """Cores this process may use: its CPU affinity, at most 16 (a one-GPU host share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _time_oracle_apply(P, x, seconds_target, max_reps=50, min_reps=1):
    P.apply_route2(x)
    t0 = time.perf_counter()
    reps = 0
    while True:
        P.apply_route2(x)
        reps += 1
        if reps >= max_reps or (reps >= min_reps and time.perf_counter() - t0 > seconds_target):
            break
    return (time.perf_counter() - t0) / reps, reps


def _oracle_apply_threaded(P, x, nthreads):
    """The oracle's route-2 apply split over row blocks of the node dimension, one block per thread:
    Y[rows] = (M_x[rows] X)(I (x) A_t)^T + sum_mu (K_mu[rows] X)(G_mu (x) B_t)^T.  Each row is computed
    by the same sequence of operations as in the single-threaded route 2, so the result is the same;
    returns a closure that performs one apply (the row slices are cut once, outside the timing)."""
    from concurrent.futures import ThreadPoolExecutor
    bm = P.full_boundary_mask()
    edges = np.linspace(0, P.n_x, nthreads + 1).astype(int)
    blocks = [(r0, r1, P.Mx[r0:r1], [K[r0:r1] for K in P.K]) for r0, r1 in zip(edges[:-1], edges[1:])]
    TA = np.kron(np.eye(P.n_xi), P.At)
    TG = [np.kron(G, P.Bt) for G in P.G]
    Y = np.empty((P.n_x, P.n_xi * P.n_t))
    pool = ThreadPoolExecutor(nthreads)

    def one():
        xin = np.where(bm, 0.0, x)
        X = xin.reshape(P.n_xi * P.n_t, P.n_x).T

        def work(blk):
            r0, r1, M, Ks = blk
            acc = (M @ X) @ TA.T
            for K, T in zip(Ks, TG):
                acc = acc + (K @ X) @ T.T
            Y[r0:r1] = acc

        list(pool.map(work, blocks))
        y = Y.T.reshape(-1).copy()
        y[bm] = x[bm]
        return y

    return one, pool


def cpu_baseline(w, seconds_target=6.0, extra=()):
    """The oracle's route-2 apply (scipy sparse x dense blocks) at full size on the GPU host's cores:
    one thread, and all the cores this process may use (row blocks of the node dimension in a thread
    pool); assembly is not timed (as on the GPU).  Also the oracle on the small 2D workload c1: its
    apply and a direct sparse solve of the slab system.  `extra`: more workloads timed the same way."""
    from threadpoolctl import threadpool_limits
    import scipy.sparse.linalg as spla
    import sg_inputs
    from oracle.slab import from_workload
    nthr = _host_threads()
    out = {"unit": "GDoF/s", "kind": "oracle", "host_threads": nthr, "cpu_model": _cpu_model(),
           "os_cpu_count": os.cpu_count()}
    for k, wk in enumerate((w,) + tuple(extra)):
        with threadpool_limits(limits=1):
            P = from_workload(wk)
            x = sg_inputs.uniform_vector(P.n, sg_inputs.SEED_APPLY_INPUT)
            dt1, reps1 = _time_oracle_apply(P, x, seconds_target, max_reps=5)
            one, pool = _oracle_apply_threaded(P, x, nthr)
            one()
            t0 = time.perf_counter()
            repsn = 0
            while repsn < 3 or (time.perf_counter() - t0 < seconds_target and repsn < 20):
                one()
                repsn += 1
            dtn = (time.perf_counter() - t0) / repsn
            pool.shutdown()
        entry = {"workload": wk.name, "n_dofs": P.n, "gdofs_1thread": round(P.n / dt1 / 1e9, 5), "reps_1thread": reps1,
                 "gdofs_all_threads": round(P.n / dtn / 1e9, 5), "reps_all_threads": repsn}
        if k == 0:
            out.update({"value": entry["gdofs_all_threads"], "cores": nthr,
                        "sample": f"route-2 Kronecker apply (scipy CSR x dense) of the full {wk.name} workload "
                                  f"({P.n} DoFs), {repsn} applies on {nthr} threads (row blocks) and {reps1} on one, "
                                  f"assembly excluded"})
            out[wk.name] = entry
        else:
            out[wk.name] = entry
        del P, x
    with threadpool_limits(limits=1):
        c1 = sg_inputs.WORKLOADS["c1"]
        P1 = from_workload(c1)
        x1 = sg_inputs.uniform_vector(P1.n, sg_inputs.SEED_APPLY_INPUT)
        dt1, _ = _time_oracle_apply(P1, x1, 1.0, 200)
        A1 = P1.assemble_full().tocsc()
        b1 = A1 @ sg_inputs.interior_target(c1)
        t0 = time.perf_counter()
        spla.spsolve(A1, b1)
        t_sp = time.perf_counter() - t0
    out["c1_apply_gdofs_1thread"] = round(P1.n / dt1 / 1e9, 5)
    out["c1_spsolve_s"] = round(t_sp, 4)
    return out


def adjoint_timing(torch, name="c5", reps=2):
    """Gradient of J = E[Q] + Var[Q] with respect to the 3 amplitudes and the 4096 cell values of a_0
    (forward sweep with slab-end checkpoints + adjoint sweep); wall time per gradient, set-up of the two
    handles included."""
    import sg_inputs
    from paper_2605_21046_amd.adjoint import SlabSequence
    aw = sg_inputs.ADJOINT_WORKLOADS[name]
    seq = SlabSequence(aw, rtol=1e-10)
    th, a0 = aw.theta0(), aw.a0_cells0()
    seq.gradient(th, a0)
    times, fwd = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J, _ = seq.forward(th, a0)[0], None
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dth, da0 = seq.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times.append(t2 - t0)
        fwd.append(t1 - t0)
    stats = {k: int(sum(v)) for k, v in seq.stats.items()}
    seq.close()
    w = aw.base
    return {"workload": f"{name}: {w.dim}D Q{w.fe_degree} on {w.n_cells_1d}^{w.dim} cells, dG({w.time_degree}), "
                        f"M={w.n_vars}, p_xi={w.chaos_degree} ({w.n_chaos} modes), {aw.n_slabs} slabs of tau={w.tau}",
            "gradient_ms": round(1e3 * float(np.mean(times)), 1), "forward_ms": round(1e3 * float(np.mean(fwd)), 1),
            "J": J, "n_params": len(th) + len(a0), "fgmres_iterations": stats}


CYCLE_VARIANTS = (("kernels", False, False), ("graph", False, True), ("segment", True, False),
                  ("segment_graph", True, True))


def _cycle_variants(torch, handles, run, reps):
    """Wall time of `run` (min over reps, after one untimed run) with the V-cycle launched kernel by
    kernel, replayed from a HIP graph, with its coarse levels as one persistent launch, and both."""
    out = {}
    for label, segment, graph in CYCLE_VARIANTS:
        for P in handles:
            P.set_vcycle_segment(segment)
            P.set_vcycle_graph(graph)
        run()
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        out[label] = round(1e3 * float(np.min(times)), 1)
    for P in handles:
        P.set_vcycle_segment(False)
        P.set_vcycle_graph(False)
    return out


def sample_batch_timing(torch, name="c4", reps=2):
    """All slabs of the Monte-Carlo batch (256 pathwise problems in one handle): wall time of the whole
    time march (right-hand sides, slab solves to 1e-8, transfers) and of the sample statistics, FP64 and
    mixed precision; set-up excluded.  FP64 also with the V-cycle variants (graph replay, persistent
    coarse segment, both; march only)."""
    import sg_inputs
    from paper_2605_21046_amd import sgheat
    from paper_2605_21046_amd.montecarlo import SampleBatch
    sw = sg_inputs.SAMPLE_WORKLOADS[name]
    w = sw.base
    out = {"workload": f"{name}: {sw.n_samples} samples xi ~ N(0, I_{w.n_vars}) (seed {sw.seed}), {w.dim}D "
                       f"Q{w.fe_degree} on {w.n_cells_1d}^{w.dim} cells, dG({w.time_degree}), {sw.n_slabs} slabs of "
                       f"tau={w.tau}, {w.n_levels}-level GMG, slab solves to rtol 1e-8"}
    for label, prec in (("fp64", sgheat.SG_FP64), ("mixed", sgheat.SG_MIXED)):
        B = SampleBatch(sw, rtol=1e-8, precision=prec)
        n_dofs = B.P.n(0)
        B.run()
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u = B.run()
            mean, var = B.statistics(u)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        its = [i["iterations"] for i in B.info]
        t = float(np.min(times))
        out[f"{label}_ms"] = round(1e3 * t, 1)
        out[f"{label}_ms_per_slab"] = round(1e3 * t / sw.n_slabs, 2)
        out[f"{label}_iterations_per_slab"] = [min(its), max(its)]
        out[f"{label}_sample_slabs_per_s"] = round(sw.n_samples * sw.n_slabs / t, 1)
        out["dofs_per_slab"] = n_dofs
        if label == "fp64":
            out["fp64_cycle_variants_ms"] = _cycle_variants(torch, [B.P], B.run, reps)
        B.close()
    return out


def member_batch_timing(torch, name="c4", reps=2):
    """All slabs of the 64 SG problems of degree 1..4 (packed into member-batch handles): wall time of
    the whole time march (slab solves to 1e-8, transfers) and of the chaos moments, FP64 and mixed;
    set-up excluded.  FP64 also with the V-cycle variants (graph replay, persistent coarse segment,
    both; march only)."""
    import sg_inputs
    from paper_2605_21046_amd import sgheat
    from paper_2605_21046_amd.sgbatch import MemberBatch
    mw = sg_inputs.MEMBER_WORKLOADS[name]
    w = mw.base
    out = {"workload": f"{name}: {len(mw.degrees)} SG problems of total degree "
                       f"{'/'.join(str(p) for p in sorted(set(mw.degrees)))} (M={w.n_vars}), {w.dim}D Q{w.fe_degree} "
                       f"on {w.n_cells_1d}^{w.dim} cells, dG({w.time_degree}), {mw.n_slabs} slabs of tau={w.tau}, "
                       f"{w.n_levels}-level GMG, slab solves to rtol 1e-8"}
    for label, prec in (("fp64", sgheat.SG_FP64), ("mixed", sgheat.SG_MIXED)):
        B = MemberBatch(mw, rtol=1e-8, precision=prec)
        B.run()
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            us = B.run()
            B.moments(us)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        its = [i["iterations"] for i in B.info]
        t = float(np.min(times))
        out["handles"] = len(B.handles)
        out["modes_per_handle"] = [B.handles[k].shape[0] for k in range(len(B.handles))]
        out["dofs_per_slab"] = int(sum(P.n(0) for P in B.handles))
        out[f"{label}_ms"] = round(1e3 * t, 1)
        out[f"{label}_iterations_per_slab"] = [min(its), max(its)]
        out[f"{label}_problem_slabs_per_s"] = round(len(mw.degrees) * mw.n_slabs / t, 1)
        if label == "fp64":
            out["fp64_cycle_variants_ms"] = _cycle_variants(torch, B.handles, B.run, reps)
        B.close()
    return out


def finite_chaos_table(torch, p_max, n_cells=128, n_slabs=64, n_levels=5, march_slabs=None):
    """The finite-chaos benchmark at the paper's discretisation (2D Q3 on n_cells^2 cells of (-1,1)^2,
    dG(3), n_slabs slabs): error quantities and wall time per stochastic degree p = 0..p_max."""
    import sg_inputs
    from paper_2605_21046_amd.finitechaos import FiniteChaosRun
    rows = []
    for p in range(p_max + 1):
        fw = sg_inputs.finite_chaos_workload(n_cells, 3, 3, n_slabs, p, n_levels)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        R = FiniteChaosRun(fw, rtol=1e-10)
        errs, _ = R.run(march_slabs)
        torch.cuda.synchronize()
        its = [i["iterations"] for i in R.info]
        rows.append({"p_xi": p, "N_xi": R.P.shape[0], "dofs_per_slab": R.P.n(0), **{k: float(f"{v:.6e}") for k, v in errs.items()},
                     "wall_s": round(time.perf_counter() - t0, 2), "iterations_per_slab": [min(its), max(its)]})
        R.close()
        print(f"[bench] finite chaos p={p}: {rows[-1]}", file=sys.stderr, flush=True)
    done = n_slabs if march_slabs is None else march_slabs
    return {"workload": f"finite-chaos benchmark: 2D Q3 on {n_cells}^2 cells of (-1,1)^2, dG(3), tau = 1/{n_slabs}, "
                        f"{done} of {n_slabs} slabs marched, M=4, q=6, eta=0.35, slab solves to rtol 1e-10", "rows": rows}


def mc_root_n(torch, name="c7", diag_blocks=1):
    """Monte-Carlo error split of the finite-chaos benchmark over cumulative sample windows (the first
    k handles of 128 samples), with the observed rates r = log(E_N0 / E_N) / log(N / N0) against the
    first window."""
    import sg_inputs
    from paper_2605_21046_amd.mcerrors import MCErrorStudy
    ew = sg_inputs.MC_ERROR_WORKLOADS[name]
    w = ew.base
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = MCErrorStudy(ew, rtol=1e-10, diag_blocks=diag_blocks)
    rows = S.run(windows=True, progress=lambda n: print(f"[bench] Monte-Carlo windows: slab {n} done", file=sys.stderr,
                                                      flush=True))
    torch.cuda.synchronize()
    its = [i["iterations"] for i in S.info]
    G = np.concatenate(S.G)
    C2 = S.C2
    S.close()
    # ||phi|| over the space-time domain, from the first window (mc_mean = |g_bar - 1| ||phi||)
    phi = rows[0]["mc_mean"] / abs(float(np.mean(G[: rows[0]["N"]])) - 1.0)
    groups = []
    size = rows[0]["N"]
    while size <= len(G):
        k = len(G) // size
        gb = G[: k * size].reshape(k, size).mean(axis=1)
        # pure sampling error of the mean: RMS over k disjoint groups of `size` samples, and the
        # Hilbert-space root-N lemma's value ||phi|| sqrt(Var[G_q] / N) with Var[G_q] = C2
        groups.append({"N": size, "groups": k, "rms_mc_mean": float(f"{phi * math.sqrt(np.mean((gb - 1.0) ** 2)):.5e}"),
                       "lemma_rms_mc_mean": float(f"{phi * math.sqrt(C2 / size):.5e}")})
        size *= 2
    r0 = rows[0]
    for r in rows[1:]:
        for key in ["tot_mean", "mc_mean", "tot_var", "mc_var"]:
            r[f"rate_{key}"] = round(math.log(r0[key] / r[key]) / math.log(r["N"] / r0["N"]), 4)
    for r in rows:
        for key in ["tot_mean", "disc_mean", "mc_mean", "tot_var", "disc_var", "mc_var"]:
            r[key] = float(f"{r[key]:.5e}")
    return {"workload": f"{name}: finite-chaos benchmark pathwise, 2D Q{w.fe_degree} on {w.n_cells_1d}^2 cells of (-1,1)^2, "
                        f"dG({w.time_degree}), {ew.n_slabs} slabs (h = tau), {ew.n_samples} samples (seed {ew.seed}) in "
                        f"handles of {ew.batch}, slab solves to rtol 1e-10",
            "preconditioner": "per-sample diagonal blocks" if diag_blocks else "mean block",
            "wall_s": round(time.perf_counter() - t0, 1), "iterations_per_slab": [min(its), max(its)], "windows": rows,
            "disjoint_groups": groups}


def copy_bandwidth(torch, dev, reps=20):
    """Achievable HBM bandwidth of a plain device copy over two disjoint 1 GiB buffer pairs."""
    n = 1 << 27
    src = [torch.ones(n, dtype=torch.float64, device=dev) for _ in range(2)]
    dst = [torch.empty_like(s) for s in src]
    for i in range(4):
        dst[i % 2].copy_(src[i % 2])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(reps):
        dst[i % 2].copy_(src[i % 2])
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    return 2 * 8 * n / t / 1e9


def run_workload(torch, dev, stream, sgheat, sg_inputs, w, args, src_hash):
    """One workload: set-up, apply tiles, the operator apply over rotating (x, y) pairs (median of
    HIP-event-timed applies on the library's stream) with its HBM and FP64 rooflines, then the FP64 and
    mixed-precision slab solves to a true relative residual of 1e-8."""
    name = w.name
    t_setup = time.perf_counter()
    G = sgheat.problem_from_workload(w, sgheat.SG_FP64)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    tiles = G.autotune(reps=10) if not args.no_autotune else None
    cpb = tiles["fp64_full"] if tiles else int(os.environ.get("SGHEAT_APPLY_CPB", "0")) or None
    n = G.n(0)
    print(f"[bench] {name}: {n} DoFs, setup {setup_s:.2f} s", file=sys.stderr, flush=True)

    n_dof, abytes, aflops, aflops_plain = apply_model(w)
    pairs = max(1, math.ceil(1.2e9 / (16 * n)))
    xs = [torch.from_numpy(sg_inputs.uniform_vector(n, sg_inputs.SEED_APPLY_INPUT + 100 * i)).to(dev)
          for i in range(pairs)]
    ys = [torch.empty_like(xs[0]) for _ in range(pairs)]
    for i in range(5):
        G.apply(xs[i % pairs], ys[i % pairs])
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.apply_reps + 1)]
    evs[0].record(stream)
    for i in range(args.apply_reps):
        G.apply(xs[i % pairs], ys[i % pairs])
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    per_apply = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.apply_reps)]) / 1e3
    t_apply = float(np.median(per_apply))
    gdofs = n_dof / t_apply / 1e9
    achieved_gbs = abytes / t_apply / 1e9
    achieved_tf = aflops / t_apply / 1e12
    print(f"[bench] {name} apply {t_apply * 1e6:.1f} us  {gdofs:.1f} GDoF/s  {achieved_gbs:.0f} GB/s  "
          f"{achieved_tf:.1f} TFLOP/s (method flops)", file=sys.stderr, flush=True)
    del xs, ys
    meas = MEASURED_TRAFFIC.get((name, src_hash, cpb))
    traffic = meas["fetch_bytes"] + meas["write_bytes"] if meas else None
    leg = {"config": {"workload": f"{name}: {w.dim}D Q{w.fe_degree} on {w.n_cells_1d}^{w.dim} cells, dG({w.time_degree}), "
                                  f"M={w.n_vars}, p_xi={w.chaos_degree} ({w.n_chaos} modes), {n_dof} DoFs, "
                                  f"{w.n_levels}-level GMG", "n_dofs": n_dof},
           "apply_us": round(t_apply * 1e6, 2), "gdofs": round(gdofs, 3),
           "roofline": {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                        "kernel": "operator apply: k_apply then k_node_gather, one stream, median of "
                                  f"{args.apply_reps} HIP-event-timed applies",
                        "algorithmic_bytes_per_apply": abytes, "source_hash": src_hash, "cells_per_workgroup": cpb,
                        "traffic_over_algorithmic": round(traffic / abytes, 3) if traffic else None},
           "roofline_fp64": {"bound": "alu", "achieved": round(achieved_tf, 2), "peak": FP64_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(achieved_tf / FP64_PEAK_TFLOPS, 4),
                             "algorithmic_flops_per_apply": aflops, "flops_per_dof": round(aflops / n_dof, 1),
                             "flops_without_even_odd": aflops_plain},
           "apply_tiles": tiles, "setup_s": round(setup_s, 2)}

    if not args.only_apply:
        # right-hand side b = AA x* for a seeded x* that vanishes on the Dirichlet boundary (so b does too)
        xg = torch.from_numpy(sg_inputs.interior_target(w)).to(dev)
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
               "fp64_applies": i64[-1]["applies"], "fp64_vcycles": i64[-1]["vcycles"],
               "fp64_err_vs_xstar": float(torch.linalg.norm(x - xg) / torch.linalg.norm(xg)),
               "work_proxy": i64[-1]["work_proxy"]}
        print(f"[bench] {name} fp64 solve {res['fp64_ms']} ms, {res['fp64_iterations']} it", file=sys.stderr,
              flush=True)
        if not args.no_mixed:
            G32 = sgheat.problem_from_workload(w, sgheat.SG_MIXED)
            if not args.no_autotune:
                res["mixed_tiles"] = G32.autotune(reps=10)
            run_solves(G32, args.warmup)
            t32, i32 = run_solves(G32, args.steps)
            err = float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
            res.update({"mixed_ms": round(float(np.mean(t32)), 2), "mixed_iterations": i32[-1]["iterations"],
                        "mixed_rel_residual_true": i32[-1]["rel_residual_true"],
                        "mixed_t_apply_ms": round(i32[-1]["t_apply_ms"], 2),
                        "mixed_t_prec_ms": round(i32[-1]["t_prec_ms"], 2),
                        "mixed_err_vs_xstar": float(torch.linalg.norm(x - xg) / torch.linalg.norm(xg)),
                        "mixed_vs_fp64_solution_rel_diff": err,
                        "mixed_speedup": round(float(np.mean(t64)) / float(np.mean(t32)), 3)})
            print(f"[bench] {name} mixed solve {res['mixed_ms']} ms, {res['mixed_iterations']} it", file=sys.stderr,
                  flush=True)
            G32.close()
        leg["solve"] = res
        del b, x, xg, x64
    G.close()
    torch.cuda.empty_cache()
    return leg


def vanka_sweeps(torch, dev, sgheat, sg_inputs, names, reps):
    """Finest-level Vanka sweeps (residual, patch corrections, update gather) of each workload in FP64 and
    with SG_MIXED (FP32 sweeps), with the fast-diagonalisation corrections (SGHEAT_VANKA_FDM=1: the
    register form where the patch fits it), their LDS form (=lds) and the dense position-class
    inverses (=0); 20 untimed sweeps first."""
    for name in names:
        w = sg_inputs.WORKLOADS[name]
        for prec, label in ((sgheat.SG_FP64, "fp64"), (sgheat.SG_MIXED, "mixed")):
            G = sgheat.problem_from_workload(w, prec)
            n = G.n(0)
            b = torch.from_numpy(sg_inputs.uniform_vector(n, 5)).to(dev)
            x = torch.zeros(n, dtype=torch.float64, device=dev)
            for fdm in ("1", "lds", "0"):
                os.environ["SGHEAT_VANKA_FDM"] = fdm
                G.vanka_smooth(0, b, x, sweeps=20)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                G.vanka_smooth(0, b, x, sweeps=reps)
                e1.record()
                torch.cuda.synchronize()
                kind = {"1": "fast diagonalisation", "lds": "fast diagonalisation, LDS form",
                        "0": "dense inverses"}[fdm]
                print(f"[bench] {name} {label} Vanka sweep ({kind}): {e0.elapsed_time(e1) / reps * 1e3:.1f} us",
                      file=sys.stderr, flush=True)
            os.environ.pop("SGHEAT_VANKA_FDM", None)
            del G
            torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed FP64 slab solves")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-gradient timing (16^3 cells, 10 slabs)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the occupancy-based apply tiles")
    ap.add_argument("--no-batch", action="store_true", help="skip the Monte-Carlo batch timing (256 samples, 20 slabs)")
    ap.add_argument("--only-apply", action="store_true", help="skip the solves (for profiling the apply)")
    ap.add_argument("--no-c3", action="store_true", help="skip the 3D Q3 24^3 dG(2) leg (apply and solves)")
    ap.add_argument("--cpu-c3", action="store_true",
                    help="also time the CPU oracle's apply on the full 3D Q3 workload (about 2 minutes of assembly)")
    ap.add_argument("--finite-chaos", type=int, default=-1, metavar="P",
                    help="also run the finite-chaos benchmark for p_xi = 0..P at the paper's discretisation")
    ap.add_argument("--mc-rootn", action="store_true",
                    help="also run the Monte-Carlo error split over cumulative windows of 128..2048 samples")
    ap.add_argument("--mc-mean-block", action="store_true",
                    help="precondition every sample of the --mc-rootn leg with the mean block instead of its own")
    ap.add_argument("--fc-slabs", type=int, default=None, metavar="N",
                    help="march only the first N of the 64 slabs of the finite-chaos benchmark (for profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device copy 5 times (reference for the HBM byte counters)")
    ap.add_argument("--vanka-sweeps", default=None, metavar="W[,W]",
                    help="only time finest-level Vanka sweeps of these workloads (FP64 and mixed), with the "
                         "fast-diagonalisation patch corrections and with the dense position-class inverses")
    ap.add_argument("--vanka-reps", type=int, default=5, help="timed sweeps per --vanka-sweeps case")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(it has no multi-GPU path)", file=sys.stderr)
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
    if args.vanka_sweeps:
        vanka_sweeps(torch, dev, sgheat, sg_inputs, args.vanka_sweeps.split(","), args.vanka_reps)
        return
    w = sg_inputs.WORKLOADS[args.workload]
    stream = torch.cuda.current_stream()
    src_hash = apply_source_hash()
    leg = run_workload(torch, dev, stream, sgheat, sg_inputs, w, args, src_hash)
    copy_gbs = copy_bandwidth(torch, dev)
    print(f"[bench] device copy {copy_gbs:.0f} GB/s; apply sources {src_hash}", file=sys.stderr, flush=True)
    out = {"metric": "SG operator apply GDoF/s + % HBM peak; FGMRES-GMG slab solve time, FP64 vs mixed",
           "value": leg["gdofs"], "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded PCG64 U[-1,1] input; analytic sine-mode coefficient)",
           "config": leg["config"], "apply_us": leg["apply_us"], "roofline": leg["roofline"],
           "roofline_fp64": leg["roofline_fp64"], "copy_gbs": round(copy_gbs, 1), "apply_tiles": leg["apply_tiles"],
           "setup_s": leg["setup_s"]}
    if "solve" in leg:
        out["solve"] = leg["solve"]
        out["ms_per_step"] = leg["solve"]["fp64_ms"]
    else:
        out["ms_per_step"] = round(leg["apply_us"] / 1e3, 4)
    if not args.no_c3 and args.workload == "c2":
        out["c3"] = run_workload(torch, dev, stream, sgheat, sg_inputs, sg_inputs.WORKLOADS["c3"], args, src_hash)

    if not args.no_adjoint and not args.only_apply:
        out["adjoint"] = adjoint_timing(torch)
        print(f"[bench] adjoint gradient {out['adjoint']['gradient_ms']} ms", file=sys.stderr, flush=True)

    if not args.no_batch and not args.only_apply:
        out["sample_batch"] = sample_batch_timing(torch)
        print(f"[bench] sample batch {out['sample_batch']['fp64_ms']} ms fp64, {out['sample_batch']['mixed_ms']} ms mixed",
              file=sys.stderr, flush=True)
        out["member_batch"] = member_batch_timing(torch)
        print(f"[bench] member batch {out['member_batch']['fp64_ms']} ms fp64, {out['member_batch']['mixed_ms']} ms mixed",
              file=sys.stderr, flush=True)

    if args.finite_chaos >= 0:
        out["finite_chaos"] = finite_chaos_table(torch, args.finite_chaos, march_slabs=args.fc_slabs)

    if args.mc_rootn:
        out["mc_root_n"] = mc_root_n(torch, diag_blocks=0 if args.mc_mean_block else 1)
        print(f"[bench] Monte-Carlo root-N windows: {out['mc_root_n']['windows']}", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        extra = (sg_inputs.WORKLOADS["c3"],) if args.cpu_c3 else ()
        out["cpu_baseline"] = cpu_baseline(w, extra=extra)
        print(f"[bench] cpu baseline {out['cpu_baseline']['value']:.4f} GDoF/s", file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
