#!/usr/bin/env python3
"""Throughput of the first-stage PDD nodal solve on one MI355X.

Workload: (1/2) Lap u + b.grad u + c u = f on [0, 4]^2 with b = (0.5 x, -0.3 y),
c = -(1 + x^2 + y^2), u = sin(pi x) cos(pi y) + x^2 y; 1,792 interface nodes
of an 8 x 8 partition; h = 1e-4; bridge exit test; FP32 path arithmetic with
FP64 integrals and sums. One benchmark step is one solve call over every
node with the next block of `--paths-per-step` paths (path_offset = step *
paths): 62,500 paths per node per step, 16 steps make 10^6 per node.

Prints one JSON line: path-steps/s over the timed steps (inputs resident on
the device, timed with HIP events on the solve's stream), the roofline of the
path kernel (VALU-issue bound; the per-step work is STEP_OPS weighted by
CLASS_SLOTS below), node-solves/s at a fixed RMS error for the correction estimator in
FP32 and the plain estimator in FP64, the correction iterates, a batched
solve, the serving loop (200 requests/s and a sweep of lower rates), the
FP64 variant of the workload, and the CPU oracle timed on a bounded sample of
the same workload (one core, and every core of the host share).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

H = 1e-4
SEED = 0

# Algorithmic VALU work of one 2D path step of this workload (plain
# estimator, bridge exit, one trig term and the polynomial y - 0.3 x^2 y -
# x^4 y - x^2 y^3 in f), counted from the operations the step must perform
# (not from the compiled code), by instruction class.
STEP_OPS = {
    # class: count per path-step
    "single": 10 + 2 + 1 + 1 + 3 + 3,  # Philox 32x32->64 products (10 per half block), 2 word->float
                                       # conversions, FP64 Z update (convert + add), box distance (3 min),
                                       # exit / bridge / step-cap compares
    "xor3": 10,                        # Philox three-way XORs (10 per half block)
    "fma": 2 + 4 + 3 + 1 + 6 + 1 + 4,  # uniform scaling, b = b0 + B x, c = c_a + c_b |x|^2, f polynomial,
                                       # f trig term (arguments, combination), Y, X
    "simple": 3 + 5 + 5 + 2 + 4 + 2,   # Box-Muller scale and products, f polynomial, trig products,
                                       # h Y and h Y f, four face distances, bridge bound
    "trans": 8,                        # Box-Muller log2, sqrt, sin, cos; sin, cos of the two trig arguments
}
# Issue cost of each class in dual-issue slots (one slot = one lane-operation
# at 128 lane-operations per compute-unit clock), from the sustained issue rate
# of each class alone measured on gfx950 (profiles/valu_issue_rates_gfx950.md,
# `bench.py --issue-rates`): 128 / lane-operations per CU clock.
CLASS_SLOTS = {
    "single": 128 / 62.6,  # v_mad_u64_u32, v_cvt_f32_u32, v_add_f64, v_max_i32: no dual issue
    "xor3": 128 / 68.9,    # v_bitop3_b32: pairs with FP32 FMAs, not with itself
    "fma": 128 / 69.3,     # v_fma_f32 / v_fmac_f32: pairs with v_bitop3_b32, not with itself
    "simple": 128 / 117.2,  # v_mul_f32, v_add_u32, v_xor_b32, v_mov_b32: dual issue
    "trans": 128 / 31.5,   # v_exp/log/sin/sqrt_f32: half the single-issue rate
}
OPS_PER_STEP = sum(STEP_OPS[k] * CLASS_SLOTS[k] for k in STEP_OPS)
# FP32 FLOPs of the same step (FMA = 2; simple arithmetic 1; transcendentals,
# integer work and compares not counted)
FLOPS_PER_STEP = 2 * STEP_OPS["fma"] + STEP_OPS["simple"] + 3
# Peak VALU issue of the chip: 256 CUs x 4 SIMDs x 16 lanes x 2 instructions
# per cycle (each SIMD issues up to two VALU instructions per cycle; the
# SQ_ACTIVE_INST_VALU2 counter counts such cycles) x 2.4 GHz = 78.6 T
# lane-operations/s, the 157.3 TFLOP/s FP32 vector figure / 2. Measured: a
# v_mul_f32 stream sustains 117.2 of the 128 lane-operations per CU clock.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
FP32_PEAK_TFLOPS = 157.3


def kernel_source_hash() -> str:
    """sha256 over the path kernel's sources and build flags: HBM counters
    taken for another version of the kernel are not reported."""
    import hashlib
    from paper_1512_02818_amd import build as B
    h = hashlib.sha256()
    for name in ("path_kernel.hip", "pdd_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1512_02818_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    h.update(" ".join(B.FLAGS[:-1]).encode())  # the include path differs between machines
    return h.hexdigest()


def stored_traffic(path: str, precision: str, paths_per_step: int):
    """HBM bytes per launch from the profiler counters stored at `path`, or
    None unless they were taken for this precision, launch size and the
    current kernel sources."""
    try:
        with open(path) as f:
            tj = json.load(f)
    except (OSError, ValueError):
        return None
    if (tj.get("precision") == precision and tj.get("paths_per_step") == paths_per_step
            and tj.get("source_sha256") == kernel_source_hash()):
        return tj.get("bytes_per_launch")
    return None


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--paths-per-step", type=int, default=62500)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--cpu-paths", type=int, default=10,
                    help="oracle sample: paths 0..n-1 of every node (0 = skip)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before warmup, one plain device copy of this many MiB (scales the "
                         "HBM byte counters of a profiler run)")
    ap.add_argument("--rms-tol", type=float, default=1e-3,
                    help="RMS error target of the node-solve comparison (0 = skip it)")
    ap.add_argument("--rms-replicas-plain", type=int, default=50,
                    help="copies of the 18 unit-square nodes (distinct streams), plain FP64")
    ap.add_argument("--rms-replicas-cv", type=int, default=2000,
                    help="copies of the 18 unit-square nodes (distinct streams), CV + FP32")
    ap.add_argument("--rms-replicas-ito", type=int, default=500,
                    help="copies of the 18 unit-square nodes (distinct streams), Ito CV + FP32")
    ap.add_argument("--serve-duration", type=float, default=2.0,
                    help="seconds of Poisson arrivals at 200 requests/s for the serving loop, then twice "
                         "as long at 10 requests/s (0 = skip)")
    ap.add_argument("--serve-drain", type=float, default=10.0,
                    help="seconds to wait for completions after the last arrival")
    ap.add_argument("--serve-sweep", type=int, default=1,
                    help="1: also serve the same request mix at 0.5, 1, 2, 5 and 20 requests/s (0 = skip)")
    ap.add_argument("--iterpdd", default="0.01,0.0025",
                    help="nodal tolerances a0 of the outer-iteration runs on the unit square ('' = skip)")
    ap.add_argument("--fp64-paths", type=int, default=4096,
                    help="paths per node of the FP64 variant of the throughput workload, with the FP32 "
                         "paths of the same pairs beside it (0 = skip)")
    ap.add_argument("--tuning", default="cache",
                    help="launch shape block,blocks_per_cu,grab[,refill,bridge] of the path kernel, "
                         "'cache' (the autotuner's cached shape for this GPU, else the default) or 'default'")
    ap.add_argument("--cv-iterates", type=int, default=1,
                    help="1: report the correction iterates 10^3 -> 10^5 (0 = skip)")
    ap.add_argument("--fit-cloud", type=int, default=100,
                    help="time steps of the nodal-constant fit's cloud in [1e-3, 1e-2] (0 = skip)")
    ap.add_argument("--paper-example", type=int, default=1,
                    help="1: solve the paper's example PDE on the stand-in box (0 = skip)")
    ap.add_argument("--batch-scale", type=float, default=1.0,
                    help="path-count scale of the 64-problem batched solve (0 = skip)")
    ap.add_argument("--profile-correction", type=int, default=0,
                    help="only run the correction solve (unit square, 257^2 FP32 grids, h=1e-3) with "
                         "this many paths per node three times and print its timing (for profilers)")
    ap.add_argument("--profile-estimator", choices=["correction", "ito"], default="correction",
                    help="with --profile-correction: the correction estimator, or phi + xi with the Ito "
                         "control variate from 257^2 FP32 gradient grids of the same u_prev")
    ap.add_argument("--profile-paper", type=int, default=0,
                    help="only run the paper's example PDE (513^2 FP32 tabulated grids, h=1e-3) with this "
                         "many paths per node three times and print its timing (for profilers)")
    ap.add_argument("--profile-plain64", type=int, default=0,
                    help="only run the plain FP64 solve of the node-solve measurement (unit square, h=1e-4, "
                         "--profile-replicas copies of the 18 nodes with distinct streams, this many paths per "
                         "node) three times and print its timing (for profilers)")
    ap.add_argument("--profile-stage2", type=int, default=0,
                    help="run only the second stage on the unit square's strips on this n^2 grid, for profiling")
    ap.add_argument("--profile-batch", type=float, default=0.0,
                    help="only run the 64-problem batched solve at this path-count scale and print its timing "
                         "(for profilers)")
    ap.add_argument("--profile-replicas", type=int, default=1,
                    help="with --profile-correction: that many 18-node solves (distinct streams) in one batch")
    ap.add_argument("--issue-rates", action="store_true",
                    help="only measure the VALU issue rate of each instruction class the path kernel "
                         "uses (libpdd_probe.so) and print them as one JSON line")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="HBM bytes per launch measured with rocprofv3 counters")
    return ap.parse_args()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def host_cores() -> int:
    """Cores this process may use, at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_paths(args):
    """Oracle walk of an explicit list of (node, path) pairs (a worker of the
    aggregate CPU baseline); returns the path-steps walked."""
    ni, pj = args
    import numpy as np

    from oracle import oracle as O
    from paper_1512_02818_amd import workloads as W
    rec = O.run_paths(W.big_square_problem(seed=SEED), W.big_square_nodes(), ni, pj, h=H)
    return int(np.sum(rec["steps"]))


def cpu_baseline(pd, nodes, n_paths):
    """The oracle on a bounded sample of the workload: paths 0..n_paths-1 of
    every node on one core, and paths n_paths..5 n_paths-1 on every core of
    the host share at once (one process per core, disjoint (node, path)
    pairs)."""
    import multiprocessing as mp

    import numpy as np

    from oracle import oracle as O
    t0 = time.perf_counter()
    _, rec = O.solve_nodes(pd, nodes, record=True, h=H, n_paths=n_paths)
    dt = time.perf_counter() - t0
    steps = int(rec["steps"].sum())
    procs = host_cores()
    ni = np.repeat(np.arange(len(nodes), dtype=np.uint32), 4 * n_paths)
    pj = np.tile(np.arange(n_paths, 5 * n_paths, dtype=np.uint64), len(nodes))
    order = np.random.default_rng(0).permutation(len(ni))  # spread long and short nodes over the workers
    jobs = [(ni[c], pj[c]) for c in np.array_split(order, 4 * procs)]
    t1 = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        agg_steps = sum(pool.map(_oracle_paths, jobs))
    agg_dt = time.perf_counter() - t1
    return {"value": steps / dt, "unit": "path-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(nodes)} nodes x paths 0..{n_paths - 1} of the same workload, "
                      f"FP64, single thread: {steps} path-steps in {dt:.1f} s",
            "cpu_model": cpu_model(),
            "aggregate": {"value": agg_steps / agg_dt, "unit": "path-steps/s", "cores": procs,
                          "sample": f"{len(nodes)} nodes x paths {n_paths}..{5 * n_paths - 1}, "
                                    f"{procs} oracle processes on disjoint (node, path) pairs: "
                                    f"{agg_steps} path-steps in {agg_dt:.1f} s"}}


DT_LADDER = (1e-3, 5e-4, 2.5e-4, 1e-4)
N_PILOT = 1000


def node_solves_at_rms(ctx, tol, replicas_plain, replicas_cv, replicas_ito):
    """Interface-node solves per second at an RMS error `tol` against the
    manufactured solution, for the plain FP64 estimator, for the FP32
    correction estimator with u_prev = U + p on a 257^2 grid (32 Fourier modes
    of amplitude 1e-2) as control variate, and for the FP32 plain estimator
    with the pathwise Ito control variate built from the gradient of the same
    U + p on 257^2 grids, on the 18 unit-square nodes replicated with distinct
    RNG streams. The error budget is split evenly:
    RMS bias <= tol/sqrt(2) picks dt from a ladder (largest first; bias
    measured against U with many paths, untimed), SE <= tol/sqrt(2) per node
    sets the paths through a 1,000-path pilot and the planner (timed, with the
    pilot, after an untimed warm-up solve of the same batch at a 10x looser
    target)."""
    import numpy as np
    import torch

    from paper_1512_02818_amd import pdd
    from paper_1512_02818_amd import workloads as W

    pd = W.unit_square_problem(seed=SEED)
    nodes = W.unit_square_nodes()
    exact = W.manufactured_u(pd, nodes)
    t0 = time.perf_counter()
    prob = pdd.Problem(ctx, pd)
    gu, gr, _ = W.correction_grids(pd, n=257, seed=1, dtype=np.float32)
    tu = torch.as_tensor(gu["data"]).cuda().contiguous()
    tr = torch.as_tensor(gr["data"]).cuda().contiguous()
    gg = W.gradient_grids(pd, n=257, seed=1, dtype=np.float32)
    gt = [torch.as_tensor(g["data"]).cuda().contiguous() for g in gg]
    gu64, gr64, _ = W.correction_grids(pd, n=257, seed=1, dtype=np.float64)
    tu64 = torch.as_tensor(gu64["data"]).cuda().contiguous()
    tr64 = torch.as_tensor(gr64["data"]).cuda().contiguous()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    budget = tol / np.sqrt(2.0)
    nstat = pdd.STATS_DTYPE.itemsize

    precision = {"plain": "fp64", "plain32": "fp32", "cv": "fp32", "cv64": "fp64", "ito": "fp32"}

    def items_for(kind, dt, replicas, stream0, out):
        its = []
        for r in range(replicas):
            it = {"problem": prob, "nodes": nodes,
                  "out": out[r * len(nodes) * nstat:(r + 1) * len(nodes) * nstat],
                  "opts": dict(dt=dt, precision=precision[kind], stream_id=stream0 + r)}
            if kind == "cv":
                it.update(u_prev=gu, u_prev_t=tu, resid=gr, resid_t=tr)
            elif kind == "cv64":
                it.update(u_prev=gu64, u_prev_t=tu64, resid=gr64, resid_t=tr64)
            elif kind == "ito":
                it.update(grad=gg, grad_t=gt)
            its.append(it)
        return its

    res = {}
    # plain FP32 and correction FP64 take the step of their other-precision
    # twin (the time-step bias is the scheme's; FP32 and FP64 paths of the
    # [0,4]^2 workload differ by 2e-5 RMS per node), and separate the
    # node-solve ratio of the correction estimator into its factors
    twin = {"plain32": "plain", "cv64": "cv"}
    for kind, reps in (("plain", replicas_plain), ("plain32", replicas_plain), ("cv", replicas_cv),
                       ("cv64", max(1, replicas_cv // 4)), ("ito", replicas_ito)):
        # dt: the largest rung whose measured RMS bias fits half the budget
        # (the bias estimate removes the sampling variance of the means)
        ladder = []
        chosen = res[twin[kind]]["dt"] if kind in twin else DT_LADDER[-1]
        cal_reps, cal_paths = (8, 1_000_000) if kind == "plain" else (8, 200_000)
        cal_out = pdd.alloc_stats(cal_reps * len(nodes))
        for dt in (DT_LADDER if kind not in twin else []):
            its = items_for(kind, dt, cal_reps, 1 << 20, cal_out)
            for it in its:
                it["opts"]["n_paths"] = cal_paths
                it["opts"]["plain_alongside"] = kind == "cv"  # variance reduction, reported (Ito: always)
            pdd.solve_batch(ctx, its)
            st = pdd.stats_to_numpy(cal_out).reshape(cal_reps, len(nodes))
            m = st["mean"].mean(axis=0)
            se2 = (st["var"] / (cal_reps * cal_paths)).mean(axis=0)
            bias = float(np.sqrt(max(0.0, np.mean((m - exact) ** 2 - se2))))
            noise = float(np.sqrt(np.mean(se2)))
            ladder.append({"dt": dt, "rms_bias": bias, "rms_se_of_estimate": noise,
                           "mean_vr": float(np.mean(st["vr"])) if kind != "plain" else None,
                           "mean_abs_rho": float(np.mean(np.abs(st["rho"]))) if kind != "plain" else None})
            if bias + noise <= budget:
                chosen = dt
                break
        out = pdd.alloc_stats(reps * len(nodes))
        batch = pdd.Batch(items_for(kind, chosen, reps, 16, out))
        # untimed warm-up at a 10x looser target: the context's buffers reach
        # the sizes of this batch before the timed solve
        pdd.solve_to_tolerance(ctx, batch, 10 * budget, N_PILOT, 1 << 31)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pdd.solve_to_tolerance(ctx, batch, budget, N_PILOT, 1 << 31)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = pdd.stats_to_numpy(out).reshape(reps, len(nodes))
        err = st["mean"] - exact[None, :]
        if kind == "cv":
            # the same batch with a 128-path pilot: the balanced plan of eq.
            # F:N_y_h needs only ~100 paths per node here (V[e] ~ 5e-5), so the
            # 1,000-path pilot alone overshoots the accuracy (untimed warm-up first)
            pdd.solve_to_tolerance(ctx, batch, 10 * budget, 128, 1 << 31)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            pdd.solve_to_tolerance(ctx, batch, budget, 128, 1 << 31)
            torch.cuda.synchronize()
            wall_small = time.perf_counter() - t1
            ss = pdd.stats_to_numpy(out).reshape(reps, len(nodes))
            small = {"pilot_paths": 128, "wall_s": wall_small, "node_solves_per_s": reps * len(nodes) / wall_small,
                     "rms_error": float(np.sqrt(np.mean((ss["mean"] - exact[None, :]) ** 2))),
                     "mean_paths_per_node": float(ss["n"].mean()), "max_paths_per_node": int(ss["n"].max())}
        res[kind] = {"node_solves": int(reps * len(nodes)), "wall_s": wall,
                     "node_solves_per_s": reps * len(nodes) / wall,
                     "rms_error": float(np.sqrt(np.mean(err ** 2))),
                     "dt": chosen, "mean_paths_per_node": float(st["n"].mean()),
                     "path_steps": int(st["steps_sum"].sum()),
                     "precision": precision[kind],
                     "dt_ladder": ladder if kind not in twin else f"the step of {twin[kind]}"}
        if kind == "cv":
            res[kind]["small_pilot"] = small
            print(f"cv with a 128-path pilot: {small['node_solves_per_s']:.3e} node-solves/s, RMS err "
                  f"{small['rms_error']:.2e}, mean N {small['mean_paths_per_node']:.0f}", file=sys.stderr, flush=True)
        print(f"{kind}: dt={chosen} {reps * len(nodes)} node-solves in {wall:.3f} s, "
              f"RMS err {res[kind]['rms_error']:.2e}, mean N {st['n'].mean():.0f}",
              file=sys.stderr, flush=True)
    prob.close()
    return {"tol": tol, "setup_s": setup_s, "pilot_paths": N_PILOT,
            "workload": "unit square, 18 interface nodes per replica, manufactured u; "
                        "CV: u_prev = u + 32-mode Fourier perturbation (amplitude 1e-2) on 257^2, FP32 grids; "
                        "Ito CV: the gradient of the same u_prev on 257^2 FP32 grids",
            "plain_fp64": res["plain"], "plain_fp32": res["plain32"], "cv_fp32": res["cv"], "cv_fp64": res["cv64"],
            "ito_cv_fp32": res["ito"],
            "ratio_cv_fp32_over_plain_fp64": res["cv"]["node_solves_per_s"] / res["plain"]["node_solves_per_s"],
            "ratio_ito_cv_fp32_over_plain_fp64": res["ito"]["node_solves_per_s"] / res["plain"]["node_solves_per_s"],
            # the correction estimator's ratio in factors: the precision of
            # the paths (plain FP32 / plain FP64, same dt), the estimator and
            # its larger step at FP64 (correction FP64 / plain FP64), and
            # the precision again under the correction estimator
            "ratio_factors": {
                "plain_fp32_over_plain_fp64": res["plain32"]["node_solves_per_s"] / res["plain"]["node_solves_per_s"],
                "cv_fp64_over_plain_fp64": res["cv64"]["node_solves_per_s"] / res["plain"]["node_solves_per_s"],
                "cv_fp32_over_cv_fp64": res["cv"]["node_solves_per_s"] / res["cv64"]["node_solves_per_s"]}}


def cv_iteration(ctx):
    """The correction estimator on the unit-square problem with u_prev = U + p
    on a 257^2 FP32 grid and its residual: iterates of 10^3, 10^4 and 10^5
    paths per node (RNG stream = iterate, u_prev fixed), FP32, with the plain
    score alongside for the variance reduction V[phi]/V[e] and rho; beside it
    the paper's Ito control variate from the gradient of the same u_prev on
    257^2 FP32 grids, on the same paths."""
    import numpy as np
    import torch

    from paper_1512_02818_amd import pdd
    from paper_1512_02818_amd import workloads as W
    pd = W.unit_square_problem(seed=SEED)
    nodes = W.unit_square_nodes()
    exact = W.manufactured_u(pd, nodes)
    prob = pdd.Problem(ctx, pd)
    gu, gr, _ = W.correction_grids(pd, n=257, seed=1, dtype=np.float32)
    tu = torch.as_tensor(gu["data"]).cuda().contiguous()
    tr = torch.as_tensor(gr["data"]).cuda().contiguous()
    gg = W.gradient_grids(pd, n=257, seed=1, dtype=np.float32)
    gt = [torch.as_tensor(g["data"]).cuda().contiguous() for g in gg]
    out = []
    for it, n in enumerate((1_000, 10_000, 100_000)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = pdd.stats_to_numpy(pdd.solve_correction(prob, gu, tu, gr, tr, nodes, dt=1e-3, n_paths=n,
                                                     stream_id=it, precision="fp32", plain_alongside=True))
        wall = time.perf_counter() - t0
        out.append({"iterate": it, "paths_per_node": n, "mean_vr": float(np.mean(st["vr"])),
                    "min_vr": float(np.min(st["vr"])), "mean_abs_rho": float(np.mean(np.abs(st["rho"]))),
                    "rms_error": float(np.sqrt(np.mean((st["mean"] - exact) ** 2))),
                    "rms_error_plain": float(np.sqrt(np.mean((st["mean_plain"] - exact) ** 2))),
                    "mean_stderr": float(np.mean(st["stderr"])), "wall_s": wall})
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        si = pdd.stats_to_numpy(pdd.solve_ito(prob, gg, gt, nodes, dt=1e-3, n_paths=n, stream_id=it,
                                              precision="fp32"))
        out[-1]["ito"] = {"mean_vr": float(np.mean(si["vr"])), "min_vr": float(np.min(si["vr"])),
                          "mean_abs_rho": float(np.mean(np.abs(si["rho"]))),
                          "rms_error": float(np.sqrt(np.mean((si["mean"] - exact) ** 2))),
                          "mean_stderr": float(np.mean(si["stderr"])), "wall_s": time.perf_counter() - t0}
    prob.close()
    return {"workload": "unit square, 18 nodes, dt=1e-3, u_prev = u + 32-mode Fourier perturbation "
                        "(amplitude 1e-2) on 257^2 with its residual, FP32; 'ito': phi + xi with xi "
                        "from the gradient of the same u_prev on 257^2 FP32 grids", "iterates": out}


def fit_cloud(ctx, m_hat, n_hat=1000, tol=1e-3):
    """The fast fit of nodal constants (Alg. A:Fitting) on the 18 unit-square
    nodes: a cloud of m_hat equispaced steps in [1e-3, 1e-2], n_hat paths per
    node and step, FP32, one batched launch, then the per-node fits. Reports
    the wall time (launch + fits), the fitted limits against the exact u, and
    the step a planner would take from the fitted bias: the largest h with
    RMS(beta) h <= tol / sqrt(2)."""
    import numpy as np
    import torch

    from paper_1512_02818_amd import pdd
    from paper_1512_02818_amd import workloads as W
    pd = W.unit_square_problem(seed=SEED)
    nodes = W.unit_square_nodes()
    exact = W.manufactured_u(pd, nodes)
    prob = pdd.Problem(ctx, pd)
    h = np.linspace(1e-3, 1e-2, m_hat)
    item = {"problem": prob, "nodes": nodes, "opts": dict(precision="fp32", stream_id=1000)}
    pdd.fit_constants(ctx, item, h[:3], 64)  # warm-up: code and buffers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c = pdd.fit_constants(ctx, item, h, n_hat)
    wall = time.perf_counter() - t0
    prob.close()
    z = (c["E_phi"] - exact) / c["se_E_phi"]
    beta_rms = float(np.sqrt(np.mean(c["beta"] ** 2)))
    return {"workload": f"unit square, 18 nodes, {m_hat} steps in [1e-3, 1e-2], {n_hat} paths per node and "
                        "step, FP32, bridge exit, delta = 1",
            "wall_s": wall, "paths": int(m_hat * n_hat * len(nodes)),
            "rms_abs_error_E_phi": float(np.sqrt(np.mean((c["E_phi"] - exact) ** 2))),
            "median_abs_z_E_phi": float(np.median(np.abs(z))), "mean_se_E_phi": float(np.mean(c["se_E_phi"])),
            "beta_rms": beta_rms, "beta_range": [float(c["beta"].min()), float(c["beta"].max())],
            "V_phi_mean": float(np.mean(c["V_phi"])), "alpha_mean": float(np.mean(c["alpha"])),
            "E_tau_mean": float(np.mean(c["E_tau"])),
            "dt_from_beta": tol / np.sqrt(2.0) / beta_rms}


def paper_example(ctx):
    """The paper's own example (Sec. 6, eq. F:PDE_ejemplo: trig-rational b and
    c, sigma = sqrt(2)) with b, c, f and g tabulated on 513^2 FP32 grids over
    the stand-in box [0, 2]^2, at 18 nodes laid out like the unit square's:
    10^6 paths per node at h = 1e-3 (plain, FP32), and the Ito control variate
    with the exact gradient (257^2 grids) at h = 2.5e-4 with 10^5 paths."""
    import numpy as np
    import torch

    from paper_1512_02818_amd import pdd
    from paper_1512_02818_amd import workloads as W
    pd = W.paper_example_problem(n=513, dtype=np.float32)
    nodes = W.paper_example_nodes()
    exact = W.paper_example_u(nodes)
    prob = pdd.Problem(ctx, pd)
    pdd.solve_nodes(prob, nodes, dt=1e-3, n_paths=1000, precision="fp32")  # warm-up
    torch.cuda.synchronize()
    # three solves of disjoint paths (path offsets 0, 10^6, 2 x 10^6): the rate
    # is their total; the accuracy figures are those of the first
    kern, steps, wall, st = [], 0, 0.0, None
    for q in range(3):
        pdd.kernel_times(ctx)
        t0 = time.perf_counter()
        sq = pdd.stats_to_numpy(pdd.solve_nodes(prob, nodes, dt=1e-3, n_paths=1_000_000, precision="fp32",
                                                stream_id=1, path_offset=q * 1_000_000, time_kernel=True))
        wall += time.perf_counter() - t0
        kern += pdd.kernel_times(ctx)
        steps += int(sq["steps_sum"].sum())
        st = sq if st is None else st
    gg = W.paper_example_gradient_grids(n=257, dtype=np.float32)
    gt = [torch.as_tensor(g["data"]).cuda().contiguous() for g in gg]
    si = pdd.stats_to_numpy(pdd.solve_ito(prob, gg, gt, nodes, dt=2.5e-4, n_paths=100_000, precision="fp32",
                                          stream_id=2))
    prob.close()
    return {"workload": "paper's example PDE (trig-rational b, c; sigma = sqrt(2)) on [0,2]^2, b, c, f, g on "
                        "513^2 FP32 grids, 18 nodes, 10^6 paths per node, h = 1e-3, FP32, bridge exit; three "
                        "solves of disjoint paths timed, accuracy from the first",
            "wall_s": wall, "path_kernel_ms": [float(k) for k in kern], "path_steps": steps,
            "path_steps_per_s": steps / (sum(kern) / 1e3), "mean_steps_per_path": float(st["mean_steps"].mean()),
            "rms_error": float(np.sqrt(np.mean((st["mean"] - exact) ** 2))),
            "mean_stderr": float(np.mean(st["stderr"])), "mean_var_phi": float(np.mean(st["var"])),
            "ito_exact_gradient": {"dt": 2.5e-4, "paths_per_node": 100_000,
                                   "rms_error": float(np.sqrt(np.mean((si["mean"] - exact) ** 2))),
                                   "mean_stderr": float(np.mean(si["stderr"])), "mean_vr": float(np.mean(si["vr"]))}}


def batch_solve(ctx, scale):
    """64 random 2D/3D box problems (uneven node counts, paths per node and
    exit times; dt 1e-3 or 1e-4) in one pdd_solve_batch, FP32."""
    import numpy as np
    import torch

    from paper_1512_02818_amd import pdd
    from paper_1512_02818_amd import workloads as W
    wl = W.batch_workload(seed=4, n_problems=64, scale=scale)
    probs = [pdd.Problem(ctx, w["problem"]) for w in wl]
    items = [{"problem": p, "nodes": w["nodes"], "opts": dict(dt=w["dt"], n_paths=w["n_paths"], precision="fp32",
                                                               stream_id=q, time_kernel=True)}
             for q, (p, w) in enumerate(zip(probs, wl))]
    batch = pdd.Batch(items)
    pdd.kernel_times(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pdd.solve_batch(ctx, batch)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = pdd.kernel_times(ctx)
    st = [pdd.stats_to_numpy(o) for o in batch.outs]
    steps = int(sum(int(s["steps_sum"].sum()) for s in st))
    paths = int(sum(int(s["n"].sum()) for s in st))
    exact_err = []
    for w, s in zip(wl, st):
        exact_err.append(np.abs(s["mean"] - W.manufactured_u(w["problem"], w["nodes"])) / s["stderr"])
    z = np.concatenate(exact_err)
    for p in probs:
        p.close()
    return {"workload": f"64 random 2D/3D boxes (seed 4), log-uniform 10-5,000 nodes and 10^3-10^6 paths per "
                        f"node x {scale}, dt in {{1e-3, 1e-4}}, FP32, one pdd_solve_batch",
            "scale": scale, "problems": len(wl), "dims": [int(w["problem"]["dim"]) for w in wl],
            "nodes": int(sum(len(w["nodes"]) for w in wl)), "paths": paths, "path_steps": steps,
            "wall_s": wall, "path_steps_per_s": steps / wall,
            "path_kernel_ms": [float(k) for k in kern],
            "median_abs_z_vs_exact": float(np.median(z))}


def fp64_variant(ctx, prob, nodes, paths):
    """The throughput workload with FP64 path arithmetic, and the FP32 paths
    of the same (node, path) pairs beside it: FP64 path-steps/s, and per node
    the bias of the FP32 mean against the FP64 mean of the same paths in units
    of the FP64 standard error (the FP32 path arithmetic of this library
    against FP64 path arithmetic)."""
    import numpy as np
    import torch

    from paper_1512_02818_amd import pdd
    off = 1 << 30  # a path range no other measurement uses
    res = {}
    for prec in ("fp64", "fp32"):
        pdd.solve_nodes(prob, nodes[:64], dt=H, n_paths=64, path_offset=off, precision=prec)  # warm-up
        torch.cuda.synchronize()
        pdd.kernel_times(ctx)
        st = pdd.stats_to_numpy(pdd.solve_nodes(prob, nodes, dt=H, n_paths=paths, path_offset=off,
                                                precision=prec, time_kernel=True))
        ms = pdd.kernel_times(ctx)
        res[prec] = (st, float(sum(ms)))
    s64, ms64 = res["fp64"]
    s32, ms32 = res["fp32"]
    bias = s32["mean"] - s64["mean"]
    z = np.abs(bias) / s64["stderr"]
    steps64 = int(s64["steps_sum"].sum())
    return {"workload": f"[0,4]^2, 1,792 nodes x {paths} paths (path offset 2^30), h=1e-4, bridge exit",
            "fp64_path_steps_per_s": steps64 / (ms64 / 1e3), "fp64_kernel_ms": ms64,
            "fp32_path_steps_per_s_same_paths": int(s32["steps_sum"].sum()) / (ms32 / 1e3),
            "fp32_over_fp64": (int(s32["steps_sum"].sum()) / ms32) / (steps64 / ms64),
            "per_node_bias_fp32_vs_fp64": {
                "max_abs": float(np.max(np.abs(bias))), "median_abs": float(np.median(np.abs(bias))),
                "rms": float(np.sqrt(np.mean(bias ** 2))),
                "max_abs_over_se": float(np.max(z)), "median_abs_over_se": float(np.median(z)),
                "median_se": float(np.median(s64["stderr"])),
                "nodes_within_3se_plus_1e-5": int(np.sum(np.abs(bias) <= 3 * s64["stderr"] + 1e-5)),
                "nodes": int(len(nodes))}}


def iterpdd_runs(ctx, tols):
    """The outer iteration (Alg. A:IterPDD) on the unit square's four strips
    (u~ on a 129^2 grid): per nodal tolerance a0, the schedule, the cost and
    RMS error of every level, and PlainPDD(a0) beside it."""
    from paper_1512_02818_amd import iterpdd
    from paper_1512_02818_amd import workloads as W
    pd = W.unit_square_problem(seed=SEED)
    out = []
    for a0 in tols:
        rep = iterpdd.run(ctx, pd, W.unit_square_nodes(), W.unit_square_partition(129), a0=a0,
                          exact=lambda p: W.manufactured_u(pd, p),
                          log=lambda m: print(m, file=sys.stderr, flush=True))
        rep.pop("constants")
        out.append(rep)
        print(f"IterPDD(a0={a0}): {rep['iterpdd_path_steps']:.3e} path-steps vs PlainPDD "
              f"{rep['plainpdd']['path_steps']:.3e} (x{rep['speedup_path_steps']:.1f}); final RMS error "
              f"{rep['levels'][-1]['rms_error_nodes']:.2e}", file=sys.stderr, flush=True)
    return {"workload": "unit square, 18 nodes on the interfaces x = 1/4, 1/2, 3/4, u~ on 129^2 (multiquadric "
                        "shape 3, FD subdomain solves), q = 2, bridge exit (delta = 1), FP32 paths, Ito control "
                        "variate from grad(u~) of the previous level", "runs": out}


SWEEP_RATES = (0.5, 1.0, 2.0, 5.0, 20.0)


def knee_rate(rates, busy_limit=None):
    """The highest rate up to which every rate of a sweep (dicts with
    rate_per_s, offered, completed, cancelled and, with busy_limit, busy_frac)
    completed all its requests (and kept the device busy less than busy_limit
    of the time); None if the lowest rate already fails."""
    knee = None
    for r in sorted(rates, key=lambda r: r["rate_per_s"]):
        if r["cancelled"] or r["completed"] != r["offered"]:
            break
        if busy_limit is not None and r["busy_frac"] >= busy_limit:
            break
        knee = r["rate_per_s"]
    return knee


LIGHT_RATES = (10.0, 25.0, 50.0, 100.0)


def serving_sweep_light(ctx, duration=4.0, drain_s=20.0):
    """The serving loop on a lighter mix whose requests one GPU can keep up
    with (up to 400 nodes, RMS tolerance 1e-2 or 3e-3, 30 % with a u_prev
    grid), at Poisson rates of 10 to 100 requests/s for `duration` seconds
    each: completions, latency, the lag (last arrival to last completion) and
    the fraction of the run with an epoch in flight. The knee is the highest
    rate up to which every rate completed all its requests with the device
    busy less than 95 % of the time (above it the backlog grows: the device
    never idles and the lag rises)."""
    from paper_1512_02818_amd import serving
    from paper_1512_02818_amd import workloads as W
    out = []
    for q, rate in enumerate(LIGHT_RATES):
        problems, reqs = W.serving_stream(seed=60 + q, rate=rate, duration=duration, node_range=(1, 400),
                                          tols=(1e-2, 3e-3))
        rep, _ = serving.run_stream(ctx, problems, reqs, drain_s=drain_s,
                                    server_opts=dict(epoch_paths=1 << 24, chunk_paths=1 << 22))
        out.append({"rate_per_s": rate, "offered": len(reqs), "completed": rep["completed"],
                    "cancelled": rep["cancelled"], "lag_s": rep["drain_s"], "p50_ms": rep["p50_ms"],
                    "p99_ms": rep["p99_ms"], "p99_censored": rep["p99_censored"],
                    "node_solves_per_s": rep["node_solves_per_s"], "busy_s": rep["busy_s"],
                    "wall_s": rep["wall_s"], "busy_frac": rep["busy_s"] / max(rep["wall_s"], 1e-9)})
        print(f"light serving at {rate:g} requests/s: {rep['completed']} of {len(reqs)} completed, lag "
              f"{rep['drain_s']:.2f} s, p50 {rep['p50_ms']:.0f} ms, p99 {rep['p99_ms']:.0f} ms",
              file=sys.stderr, flush=True)
    knee = knee_rate(out, busy_limit=0.95)
    return {"workload": f"Poisson arrivals for {duration:g} s per rate, 1-400 nodes (log-uniform) on 16 random "
                        "2D/3D box problems, RMS tolerance in {1e-2, 3e-3}, 30% with a u_prev grid, FP32, "
                        f"drain up to {drain_s:g} s", "rates": out, "knee_rate_per_s": knee}


def serving_pipeline(ctx, depths=(1, 2, 3)):
    """The serving loop with 1, 2 and 3 epochs in flight on one burst of
    requests (all arriving within 0.1 s; up to 400 nodes, RMS tolerance 1e-2
    or 3e-3, 30% with a u_prev grid): time to complete all of them, the time
    with an epoch in flight, throughput and latency. Results are bitwise the
    same at every depth (checked here on every request)."""
    from paper_1512_02818_amd import serving
    from paper_1512_02818_amd import workloads as W
    problems, reqs = W.serving_stream(seed=41, rate=1000.0, duration=0.1, node_range=(1, 400),
                                      tols=(1e-2, 3e-3))
    fx = serving.Fixtures(ctx, problems, reqs)
    out, ref = [], None
    for depth in depths:
        rep, done = serving.run_stream(ctx, problems, reqs, drain_s=120.0, fixtures=fx,
                                       server_opts=dict(epoch_paths=1 << 24, chunk_paths=1 << 22,
                                                        pipeline=depth))
        same = None
        if ref is None:
            ref = done
        else:
            same = sorted(done) == sorted(ref) and all(done[k]["stats"].tobytes() == ref[k]["stats"].tobytes()
                                                       for k in ref)
        out.append({"pipeline": depth, "completed": rep["completed"], "offered": len(reqs),
                    "wall_s": rep["wall_s"], "busy_s": rep["busy_s"], "epochs": rep["epochs"], "paths_run": rep["paths_run"],
                    "path_steps": rep["path_steps"], "path_steps_per_s": rep["path_steps"] / max(rep["wall_s"], 1e-9),
                    "node_solves_per_s": rep["node_solves_per_s"], "p50_ms": rep["p50_ms"],
                    "p99_ms": rep["p99_ms"], "bitwise_equal_to_depth_1": same})
        print(f"serving burst, {depth} epoch(s) in flight: {rep['completed']} of {len(reqs)} in "
              f"{rep['wall_s']:.2f} s, {out[-1]['path_steps_per_s']:.3e} path-steps/s", file=sys.stderr, flush=True)
    fx.close()
    return {"workload": f"burst of {len(reqs)} requests within 0.1 s, 1-400 nodes (log-uniform) on 16 random "
                        "2D/3D box problems, RMS tolerance in {1e-2, 3e-3}, 30% with a u_prev grid, FP32",
            "depths": out}


def serving_sweep(ctx, drain_s):
    """The serving loop at offered loads below the 200 requests/s of the main
    serving run (same request mix, seeded Poisson arrivals, about 12 requests
    per rate, at least 2 s and at most 12 s of arrivals): completed, cancelled
    and latency percentiles per rate; the knee is the highest rate up to which
    every rate of the sweep completed all its requests within the drain."""
    from paper_1512_02818_amd import serving
    from paper_1512_02818_amd import workloads as W
    out = []
    for q, rate in enumerate(SWEEP_RATES):
        dur = min(12.0, max(2.0, 12.0 / rate))
        problems, reqs = W.serving_stream(seed=20 + q, rate=rate, duration=dur)
        if not reqs:
            continue
        rep, _ = serving.run_stream(ctx, problems, reqs, drain_s=drain_s,
                                    server_opts=dict(epoch_paths=1 << 24, chunk_paths=1 << 22))
        out.append({"rate_per_s": rate, "arrival_window_s": dur, "offered": len(reqs),
                    "completed": rep["completed"], "cancelled": rep["cancelled"],
                    "p50_ms": rep["p50_ms"], "p99_ms": rep["p99_ms"], "p50_censored": rep["p50_censored"],
                    "p99_censored": rep["p99_censored"], "p99_done_ms": rep["p99_done_ms"],
                    "node_solves_per_s": rep["node_solves_per_s"], "drain_s": rep["drain_s"]})
        print(f"serving at {rate:g} requests/s: {rep['completed']} of {len(reqs)} completed, "
              f"p50 {rep['p50_ms']:.0f} ms, p99 {'>= ' if rep['p99_censored'] else ''}{rep['p99_ms']:.0f} ms",
              file=sys.stderr, flush=True)
    return {"workload": "the request mix of 'serving' at lower Poisson rates (seeds 20..), drain "
                        f"{drain_s:g} s", "rates": out, "knee_rate_per_s": knee_rate(out)}


def calibration_copy(mib):
    """One plain device copy of `mib` MiB: its HBM byte counters give the
    scale of a profiler's FETCH_SIZE / WRITE_SIZE readings."""
    import torch
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def profile_correction(paths, calibrate_mib=0, replicas=1, estimator="correction"):
    """The correction estimator alone, for kernel-trace and counter runs: 18
    unit-square nodes, u_prev = U + p and its residual on 257^2 FP32 grids
    (about 0.26 MB each, so the grid gathers are served by L2), h = 1e-3.
    replicas > 1: that many solves of the 18 nodes with distinct RNG streams
    in one pdd_solve_batch, as in the node-solve measurement. estimator
    "ito": the Ito control variate instead, from the gradient of the same
    u_prev on two 257^2 FP32 grids."""
    import numpy as np
    import torch

    from paper_1512_02818_amd import pdd, tuning
    from paper_1512_02818_amd import workloads as W
    ctx = pdd.Context(0)
    tuning.load(ctx)  # the launch shapes of the node-solve measurement
    pd = W.unit_square_problem(seed=SEED)
    nodes = W.unit_square_nodes()
    prob = pdd.Problem(ctx, pd)
    gu, gr, _ = W.correction_grids(pd, n=257, seed=1, dtype=np.float32)
    tu = torch.as_tensor(gu["data"]).cuda().contiguous()
    tr = torch.as_tensor(gr["data"]).cuda().contiguous()
    grids = {"u_prev": gu, "u_prev_t": tu, "resid": gr, "resid_t": tr}
    if estimator == "ito":
        gg = W.gradient_grids(pd, n=257, seed=1, dtype=np.float32)
        grids = {"grad": gg, "grad_t": [torch.as_tensor(g["data"]).cuda().contiguous() for g in gg]}
    out = pdd.alloc_stats(replicas * len(nodes))
    nstat = pdd.STATS_DTYPE.itemsize
    if calibrate_mib > 0:
        calibration_copy(calibrate_mib)
    steps = 0
    for r in range(3):
        if replicas == 1:
            pdd.solve_batch(ctx, [dict({"problem": prob, "nodes": nodes, "out": out,
                                        "opts": dict(dt=1e-3, n_paths=paths, path_offset=r * paths,
                                                     precision="fp32", time_kernel=True)}, **grids)])
        else:
            pdd.solve_batch(ctx, [dict({"problem": prob, "nodes": nodes,
                                        "out": out[q * len(nodes) * nstat:(q + 1) * len(nodes) * nstat],
                                        "opts": dict(dt=1e-3, n_paths=paths, path_offset=r * paths,
                                                     precision="fp32", stream_id=16 + q, time_kernel=q == 0)},
                                       **grids)
                                  for q in range(replicas)])
        steps += int(pdd.stats_to_numpy(out)["steps_sum"].sum())
    ms = pdd.kernel_times(ctx)
    print(json.dumps({"correction_profile": {"estimator": estimator, "paths_per_node": paths,
                                             "nodes": len(nodes), "replicas": replicas,
                                             "path_steps": steps, "kernel_ms": ms,
                                             "path_steps_per_s": steps / (sum(ms) / 1e3)}}), flush=True)
    prob.close()
    ctx.close()


def profile_paper(paths, calibrate_mib=0):
    """The paper's example PDE alone (every coefficient and g tabulated on
    513^2 FP32 grids over [0, 2]^2, 18 nodes, h = 1e-3, FP32), three solves
    with distinct path ranges, for kernel-trace and counter runs."""
    import numpy as np

    from paper_1512_02818_amd import pdd
    from paper_1512_02818_amd import workloads as W
    ctx = pdd.Context(0)
    prob = pdd.Problem(ctx, W.paper_example_problem(n=513, dtype=np.float32))
    nodes = W.paper_example_nodes()
    if calibrate_mib > 0:
        calibration_copy(calibrate_mib)
    steps = 0
    for r in range(3):
        st = pdd.stats_to_numpy(pdd.solve_nodes(prob, nodes, dt=1e-3, n_paths=paths, path_offset=r * paths,
                                                precision="fp32", time_kernel=True))
        steps += int(st["steps_sum"].sum())
    ms = pdd.kernel_times(ctx)
    print(json.dumps({"paper_profile": {"paths_per_node": paths, "nodes": len(nodes), "path_steps": steps,
                                        "kernel_ms": ms, "path_steps_per_s": steps / (sum(ms) / 1e3)}}), flush=True)
    prob.close()
    ctx.close()


def issue_rates(blocks_per_cu=8, target_ms=40.0):
    """Sustained issue rate of each VALU instruction class of the path kernel
    on its own (libpdd_probe.so: 8 independent chains per lane, 8 waves per
    SIMD), in lane-operations per second and per compute-unit clock at the
    clock the chip ran at (shader-clock counter over the constant wall clock,
    read by the probe around its loop)."""
    import ctypes as C

    import torch
    from paper_1512_02818_amd import build as B
    if not os.path.exists(B.PROBE_LIB):
        raise RuntimeError(f"{B.PROBE_LIB} is missing: run `python -m paper_1512_02818_amd.build`")
    torch.cuda.init()
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    L = C.CDLL(B.PROBE_LIB)
    L.probe_kind_name.restype = C.c_char_p
    L.probe_issue_rate.argtypes = [C.c_int, C.c_int, C.c_uint32] + [C.POINTER(C.c_double)] * 4
    rows = []
    for kind in range(L.probe_kinds()):
        ms, ops, cyc, wall = C.c_double(), C.c_double(), C.c_double(), C.c_double()
        iters = 64
        for _ in range(2):  # size the loop to about target_ms
            rc = L.probe_issue_rate(kind, blocks_per_cu, iters, C.byref(ms), C.byref(ops), C.byref(cyc),
                                    C.byref(wall))
            if rc != 0:
                raise RuntimeError(f"probe {kind} failed with HIP error {rc}")
            iters = max(64, int(iters * target_ms / max(ms.value, 1e-3)))
        ghz = cyc.value / wall.value
        rate = ops.value / (ms.value / 1e3)
        rows.append({"instruction": L.probe_kind_name(kind).decode(), "ms": ms.value, "lane_ops": ops.value,
                     "lane_ops_per_s": rate, "clock_ghz": ghz,
                     "lane_ops_per_cu_clock": rate / (n_cu * ghz * 1e9)})
        print(f"{rows[-1]['instruction']:>14}: {rate / 1e12:7.2f} T lane-ops/s, "
              f"{rows[-1]['lane_ops_per_cu_clock']:6.1f} per CU-clock at {ghz:.3f} GHz", file=sys.stderr, flush=True)
    print(json.dumps({"issue_rates": rows, "n_cu": n_cu, "blocks_per_cu": blocks_per_cu,
                      "waves_per_simd": blocks_per_cu * 4 // 4}), flush=True)


def profile_plain64(paths, replicas, calibrate_mib=0):
    """The plain FP64 solve of the node-solve measurement alone (unit square,
    h = 1e-4, `replicas` copies of the 18 nodes with distinct RNG streams in
    one batch), three times, for kernel-trace and counter runs."""
    from paper_1512_02818_amd import pdd, tuning
    from paper_1512_02818_amd import workloads as W
    ctx = pdd.Context(0)
    tuning.load(ctx)
    prob = pdd.Problem(ctx, W.unit_square_problem(seed=SEED))
    nodes = W.unit_square_nodes()
    nstat = pdd.STATS_DTYPE.itemsize
    out = pdd.alloc_stats(replicas * len(nodes))
    if calibrate_mib > 0:
        calibration_copy(calibrate_mib)
    steps = 0
    for r in range(3):
        pdd.solve_batch(ctx, [{"problem": prob, "nodes": nodes,
                               "out": out[q * len(nodes) * nstat:(q + 1) * len(nodes) * nstat],
                               "opts": dict(dt=1e-4, n_paths=paths, path_offset=r * paths, precision="fp64",
                                            stream_id=16 + q, time_kernel=q == 0)} for q in range(replicas)])
        steps += int(pdd.stats_to_numpy(out)["steps_sum"].sum())
    ms = pdd.kernel_times(ctx)
    print(json.dumps({"plain64_profile": {"paths_per_node": paths, "nodes": len(nodes), "replicas": replicas,
                                          "path_steps": steps, "kernel_ms": ms,
                                          "path_steps_per_s": steps / (sum(ms) / 1e3)}}), flush=True)
    prob.close()
    ctx.close()


def profile_stage2(n):
    """The second stage alone, for kernel-trace runs: the unit square's four
    strips on an n^2 grid, four problems with the same operator (so the LU
    factors are kept across them while each needs its own response columns),
    two calls each with the exact nodal values; wall time of every call."""
    import time

    import torch

    from paper_1512_02818_amd import pdd
    from paper_1512_02818_amd import workloads as W
    ctx = pdd.Context(0)
    pd = W.unit_square_problem(seed=SEED)
    part = W.unit_square_partition(n)
    nodes = W.unit_square_nodes()
    vals = W.manufactured_u(pd, nodes)
    ms = []
    for k in range(4):
        prob = pdd.Problem(ctx, pd)
        for _ in range(2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            pdd.stage2(prob, part["n"], part["cuts"], nodes, vals, part["rbf_eps"])
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t) * 1e3)
        prob.close()
    print(json.dumps({"stage2_profile": {"grid": n, "call_ms": ms}}), flush=True)
    ctx.close()


def profile_batch(scale):
    """The 64-problem batched solve alone at path-count scale `scale`, for
    kernel-trace and counter runs."""
    from paper_1512_02818_amd import pdd
    ctx = pdd.Context(0)
    b = batch_solve(ctx, scale)
    b.pop("dims")
    print(json.dumps({"batch_profile": b}), flush=True)
    ctx.close()


def main():
    args = parse()
    if args.issue_rates:
        issue_rates()
        return
    if args.profile_plain64 > 0:
        profile_plain64(args.profile_plain64, args.profile_replicas, args.calibrate_copy_mib)
        return
    if args.profile_stage2 > 0:
        profile_stage2(args.profile_stage2)
        return
    if args.profile_batch > 0:
        profile_batch(args.profile_batch)
        return
    if args.profile_paper > 0:
        profile_paper(args.profile_paper, args.calibrate_copy_mib)
        return
    if args.profile_correction > 0:
        profile_correction(args.profile_correction, args.calibrate_copy_mib, args.profile_replicas,
                           args.profile_estimator)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(a multi-GPU run would split each node's paths across GPUs and merge the "
              "per-node sums)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1512_02818_amd import pdd
    from paper_1512_02818_amd import workloads as W

    pd = W.big_square_problem(seed=SEED)
    nodes = W.big_square_nodes()
    P = args.paths_per_step
    cpu = None
    if args.cpu_paths > 0:
        # before anything touches the GPU: the aggregate's worker processes are forked
        print("timing the CPU oracle sample ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(pd, nodes, args.cpu_paths)
        print(f"oracle: {cpu['value']:.3e} path-steps/s on one core, {cpu['aggregate']['value']:.3e} on "
              f"{cpu['aggregate']['cores']} cores ({cpu['cpu_model']})", file=sys.stderr, flush=True)
    ctx = pdd.Context(0)
    from paper_1512_02818_amd import tuning
    shape = None
    if args.tuning == "cache":
        tuning.load(ctx)
    elif args.tuning != "default":
        shape = tuning.to_fields(args.tuning.split(","))
    prob = pdd.Problem(ctx, pd)
    outs = [pdd.alloc_stats(len(nodes)) for _ in range(args.warmup + args.steps)]

    if args.calibrate_copy_mib > 0:
        calibration_copy(args.calibrate_copy_mib)

    def step(s):
        pdd.solve_nodes(prob, nodes, out=outs[s], dt=H, n_paths=P, path_offset=s * P,
                        precision=args.precision, time_kernel=True,
                        tuning=shape)

    for s in range(args.warmup):
        step(s)
    torch.cuda.synchronize()
    pdd.kernel_times(ctx)  # drop warmup timings
    print(f"warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for s in range(args.warmup, args.warmup + args.steps):
        step(s)
    end.record()
    torch.cuda.synchronize()
    elapsed_ms = start.elapsed_time(end)
    kern_ms = pdd.kernel_times(ctx)

    timed = [pdd.stats_to_numpy(outs[s]) for s in range(args.warmup, args.warmup + args.steps)]
    steps_per_launch = [int(t["steps_sum"].sum()) for t in timed]
    total_steps = sum(steps_per_launch)
    value = total_steps / (elapsed_ms / 1e3)
    avg_kern_s = float(np.mean(kern_ms)) / 1e3
    achieved = OPS_PER_STEP * float(np.mean(steps_per_launch)) / avg_kern_s / 1e12
    fp32_tflops = FLOPS_PER_STEP * float(np.mean(steps_per_launch)) / avg_kern_s / 1e12
    traffic = stored_traffic(args.traffic_json, args.precision, P)
    exact = W.manufactured_u(pd, nodes)
    z = np.abs(timed[-1]["mean"] - exact) / timed[-1]["stderr"]
    print(f"timed {args.steps} steps: {elapsed_ms:.1f} ms, path kernel {np.mean(kern_ms):.1f} ms/launch, "
          f"{total_steps:.3e} path-steps, node z-scores median {np.median(z):.2f}",
          file=sys.stderr, flush=True)

    result = {
        "metric": "path-steps/s",
        "value": value,
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "[0,4]^2 first-stage nodal solve: 1,792 interface nodes, "
                               f"{P} paths per node per step (step s walks paths s*{P} .. "
                               f"(s+1)*{P}-1 of every node, warmup steps first), h=1e-4, bridge exit, "
                               f"{args.precision} paths, fp64 sums",
                   "nodes": int(len(nodes)), "paths_per_step": P, "dt": H, "tuning": args.tuning,
                   "mean_steps_per_path": total_steps / (args.steps * len(nodes) * P)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "T VALU issue slots/s (lane-operations at the dual-issue rate)",
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic,
                     "slots_per_step": OPS_PER_STEP, "ops_per_step": STEP_OPS,
                     "kernel_ms_per_launch": float(np.mean(kern_ms)),
                     "fp32_tflops": fp32_tflops, "fp32_peak_tflops": FP32_PEAK_TFLOPS,
                     "fp32_flop_frac": fp32_tflops / FP32_PEAK_TFLOPS,
                     "fp32_flop_frac_target_met": fp32_tflops / FP32_PEAK_TFLOPS >= 0.5},
    }
    if args.fp64_paths > 0:
        print("FP64 variant of the throughput workload ...", file=sys.stderr, flush=True)
        result["fp64_variant"] = fp64_variant(ctx, prob, nodes, args.fp64_paths)
        fv = result["fp64_variant"]
        print(f"fp64: {fv['fp64_path_steps_per_s']:.3e} path-steps/s; fp32 vs fp64 per node: max |bias|/SE "
              f"{fv['per_node_bias_fp32_vs_fp64']['max_abs_over_se']:.3f}", file=sys.stderr, flush=True)
    if args.rms_tol > 0:
        print("node solves at fixed RMS error ...", file=sys.stderr, flush=True)
        result["node_solves_at_rms"] = node_solves_at_rms(ctx, args.rms_tol, args.rms_replicas_plain,
                                                          args.rms_replicas_cv, args.rms_replicas_ito)
    if args.cv_iterates:
        print("correction iterates ...", file=sys.stderr, flush=True)
        result["cv_iteration"] = cv_iteration(ctx)
    if args.fit_cloud > 0:
        print("nodal-constant fit ...", file=sys.stderr, flush=True)
        result["fit_constants"] = fit_cloud(ctx, args.fit_cloud)
        f = result["fit_constants"]
        print(f"fit: {f['paths']} paths in {f['wall_s']:.3f} s, beta RMS {f['beta_rms']:.3f}, "
              f"dt from beta {f['dt_from_beta']:.2e}", file=sys.stderr, flush=True)
    if args.iterpdd:
        print("outer iteration (IterPDD) ...", file=sys.stderr, flush=True)
        result["iterpdd"] = iterpdd_runs(ctx, [float(v) for v in args.iterpdd.split(",")])
    if args.paper_example:
        print("the paper's example PDE ...", file=sys.stderr, flush=True)
        result["paper_example"] = paper_example(ctx)
        pe = result["paper_example"]
        print(f"paper example: {pe['path_steps_per_s']:.3e} path-steps/s, RMS err {pe['rms_error']:.2e} "
              f"(SE {pe['mean_stderr']:.1e})", file=sys.stderr, flush=True)
    if args.batch_scale > 0:
        print("batched solve ...", file=sys.stderr, flush=True)
        result["batch"] = batch_solve(ctx, args.batch_scale)
        print(f"batch: {result['batch']['path_steps']:.3e} path-steps in {result['batch']['wall_s']:.2f} s",
              file=sys.stderr, flush=True)
    if args.serve_duration > 0:
        print("serving loop ...", file=sys.stderr, flush=True)
        from paper_1512_02818_amd import serving
        problems, reqs = W.serving_stream(seed=5, rate=200.0, duration=args.serve_duration)
        rep, _ = serving.run_stream(ctx, problems, reqs, drain_s=args.serve_drain,
                                    server_opts=dict(epoch_paths=1 << 24, chunk_paths=1 << 22))
        rep["workload"] = ("Poisson 200 requests/s of 1-2,000 nodes (log-uniform) on 16 random 2D/3D "
                           "box problems, RMS tolerance in {1e-2, 3e-3, 1e-3}, 30% with a u_prev grid "
                           "(129^2-513^2 or 65^3), FP32, 64 GiB budget; requests still running after "
                           "the drain are cancelled and reported")
        result["serving"] = rep
        print(f"serving at 200 requests/s: {rep['completed']} of {rep['offered_requests']} completed, "
              f"p50 {rep['p50_ms']:.0f} ms, p99 {'>= ' if rep['p99_censored'] else ''}{rep['p99_ms']:.0f} ms",
              file=sys.stderr, flush=True)
        if args.serve_sweep:
            result["serving_sweep"] = serving_sweep(ctx, args.serve_drain)
            result["serving_sweep_light"] = serving_sweep_light(ctx)
            result["serving_pipeline"] = serving_pipeline(ctx)
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)
    prob.close()
    ctx.close()


if __name__ == "__main__":
    main()
