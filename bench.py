#!/usr/bin/env python3
"""Throughput of the first-stage PDD nodal solve on one MI355X.

Workload: (1/2) Lap u + b.grad u + c u = f on [0, 4]^2 with b = (0.5 x, -0.3 y),
c = -(1 + x^2 + y^2), u = sin(pi x) cos(pi y) + x^2 y; 1,792 interface nodes
of an 8 x 8 partition; h = 1e-4; bridge exit test; FP32 path arithmetic with
FP64 integrals and sums; 10^6 paths per node in total. One benchmark step is
one solve call over every node with the next block of `--paths-per-step` paths
(path_offset = step * paths), so 16 steps of 62,500 paths are the whole job.

Prints one JSON line: path-steps/s over the timed steps (inputs resident on
the device, timed with HIP events on the solve's stream), the roofline of the
path kernel (VALU-issue bound; the per-step operation count is STEP_COST
below), node-solves/s at a fixed RMS error for the correction estimator in
FP32 and the plain estimator in FP64, the correction iterates, a batched
solve, two serving runs (overload and a sustainable load), and the CPU
oracle timed on a bounded sample of the same workload.
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

# Algorithmic VALU cost of one 2D path step of this workload, in full-rate
# FP32 lane slots; transcendentals (log2, sqrt, sin, cos, exp2) and 32x32-bit
# multiplies issue at a quarter of the FP32 rate and count 4, an FP64 add 2.
# Derived from the operations the step must perform, not from the compiled
# code.
STEP_COST = {
    "philox_half_block": (10 * 2 * 4 + 10 * 2) // 2,  # 10 rounds x (2 wide mul + 2 xor3); 2 steps/block
    "uniforms": 2 * 2,                                # convert + fma per word
    "box_muller": 4 * 4 + 5,                          # log2, sqrt, sin, cos; scale, 2 mul
    "drift_killing": 4 + 3,                           # b = b0 + B x; c = c_a + c_b |x|^2
    "poly_source": 20,                                # degree-5 Horner form of the polynomial part of f
    "trig_source": 2 + 4 * 4 + 8,                     # 2 arguments, sin/cos x 2, combination
    "euler_step": 9 + 2,                              # hY, Z (FP64 add), Y, X
    "exit_test": 12,                                  # distance to the box, exit, bridge bound
}
OPS_PER_STEP = sum(STEP_COST.values())
# FP32 FLOPs of the same step (FMA = 2; transcendentals not counted)
FLOPS_PER_STEP = 4 + 3 + 8 + 5 + 40 + 16 + 12 + 7
# 256 CUs x 128 FP32 lanes x 2.4 GHz: the 157.3 TFLOP/s FP32 vector peak / 2
VALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
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
    ap.add_argument("--tuning", default="cache",
                    help="launch shape block,blocks_per_cu,grab of the path kernel, 'cache' (the "
                         "autotuner's cached shape for this GPU, else the default) or 'default'")
    ap.add_argument("--cv-iterates", type=int, default=1,
                    help="1: report the correction iterates 10^3 -> 10^5 (0 = skip)")
    ap.add_argument("--fit-cloud", type=int, default=100,
                    help="time steps of the nodal-constant fit's cloud in [1e-3, 1e-2] (0 = skip)")
    ap.add_argument("--paper-example", type=int, default=1,
                    help="1: solve the paper's example PDE on the stand-in box (0 = skip)")
    ap.add_argument("--batch-scale", type=float, default=0.1,
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
    ap.add_argument("--profile-replicas", type=int, default=1,
                    help="with --profile-correction: that many 18-node solves (distinct streams) in one batch")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="HBM bytes per launch measured with rocprofv3 counters")
    return ap.parse_args()


def cpu_baseline(pd, nodes, n_paths):
    from oracle import oracle as O
    t0 = time.perf_counter()
    _, rec = O.solve_nodes(pd, nodes, record=True, h=H, n_paths=n_paths)
    dt = time.perf_counter() - t0
    steps = int(rec["steps"].sum())
    return {"value": steps / dt, "unit": "path-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(nodes)} nodes x paths 0..{n_paths - 1} of the same workload, "
                      f"FP64, single thread: {steps} path-steps in {dt:.1f} s",
            "host": platform.processor() or platform.machine()}


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
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    budget = tol / np.sqrt(2.0)
    nstat = pdd.STATS_DTYPE.itemsize

    def items_for(kind, dt, replicas, stream0, out):
        its = []
        for r in range(replicas):
            it = {"problem": prob, "nodes": nodes,
                  "out": out[r * len(nodes) * nstat:(r + 1) * len(nodes) * nstat],
                  "opts": dict(dt=dt, precision="fp64" if kind == "plain" else "fp32",
                               stream_id=stream0 + r)}
            if kind == "cv":
                it.update(u_prev=gu, u_prev_t=tu, resid=gr, resid_t=tr)
            elif kind == "ito":
                it.update(grad=gg, grad_t=gt)
            its.append(it)
        return its

    res = {}
    for kind, reps in (("plain", replicas_plain), ("cv", replicas_cv), ("ito", replicas_ito)):
        # dt: the largest rung whose measured RMS bias fits half the budget
        # (the bias estimate removes the sampling variance of the means)
        ladder = []
        chosen = DT_LADDER[-1]
        cal_reps, cal_paths = (8, 1_000_000) if kind == "plain" else (8, 200_000)
        cal_out = pdd.alloc_stats(cal_reps * len(nodes))
        for dt in DT_LADDER:
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
                     "precision": "fp64" if kind == "plain" else "fp32",
                     "dt_ladder": ladder}
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
            "plain_fp64": res["plain"], "cv_fp32": res["cv"], "ito_cv_fp32": res["ito"],
            "ratio_cv_fp32_over_plain_fp64": res["cv"]["node_solves_per_s"] / res["plain"]["node_solves_per_s"],
            "ratio_ito_cv_fp32_over_plain_fp64": res["ito"]["node_solves_per_s"] / res["plain"]["node_solves_per_s"]}


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
    pdd.kernel_times(ctx)
    t0 = time.perf_counter()
    st = pdd.stats_to_numpy(pdd.solve_nodes(prob, nodes, dt=1e-3, n_paths=1_000_000, precision="fp32",
                                            stream_id=1, time_kernel=True))
    wall = time.perf_counter() - t0
    kern = pdd.kernel_times(ctx)
    steps = int(st["steps_sum"].sum())
    gg = W.paper_example_gradient_grids(n=257, dtype=np.float32)
    gt = [torch.as_tensor(g["data"]).cuda().contiguous() for g in gg]
    si = pdd.stats_to_numpy(pdd.solve_ito(prob, gg, gt, nodes, dt=2.5e-4, n_paths=100_000, precision="fp32",
                                          stream_id=2))
    prob.close()
    return {"workload": "paper's example PDE (trig-rational b, c; sigma = sqrt(2)) on [0,2]^2, b, c, f, g on "
                        "513^2 FP32 grids, 18 nodes, 10^6 paths per node, h = 1e-3, FP32, bridge exit",
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


def main():
    args = parse()
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
    ctx = pdd.Context(0)
    from paper_1512_02818_amd import tuning
    shape = None
    if args.tuning == "cache":
        tuning.load(ctx)
    elif args.tuning != "default":
        shape = tuple(int(v) for v in args.tuning.split(","))
    prob = pdd.Problem(ctx, pd)
    outs = [pdd.alloc_stats(len(nodes)) for _ in range(args.warmup + args.steps)]

    if args.calibrate_copy_mib > 0:
        calibration_copy(args.calibrate_copy_mib)

    def step(s):
        pdd.solve_nodes(prob, nodes, out=outs[s], dt=H, n_paths=P, path_offset=s * P,
                        precision=args.precision, time_kernel=True,
                        tuning=None if shape is None else shape + (0,))

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
                               f"{P} paths per node per step (10^6 per node over "
                               f"{1_000_000 // P} steps), h=1e-4, bridge exit, "
                               f"{args.precision} paths, fp64 sums",
                   "nodes": int(len(nodes)), "paths_per_step": P, "dt": H, "tuning": args.tuning,
                   "mean_steps_per_path": total_steps / (args.steps * len(nodes) * P)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "Top/s (FP32 VALU lane slots)",
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic,
                     "ops_per_step": OPS_PER_STEP,
                     "kernel_ms_per_launch": float(np.mean(kern_ms)),
                     "fp32_tflops": FLOPS_PER_STEP * float(np.mean(steps_per_launch)) / avg_kern_s / 1e12,
                     "fp32_peak_tflops": FP32_PEAK_TFLOPS},
    }
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
                                    server_opts=dict(epoch_paths=1 << 24, chunk_paths=1 << 20))
        rep["workload"] = ("Poisson 200 requests/s of 1-2,000 nodes (log-uniform) on 16 random 2D/3D "
                           "box problems, RMS tolerance in {1e-2, 3e-3, 1e-3}, 30% with a u_prev grid "
                           "(129^2-513^2 or 65^3), FP32, 64 GiB budget; requests still running after "
                           "the drain are cancelled and reported")
        result["serving"] = rep
        # the same kind of stream at a load one GPU sustains: latency without a backlog
        problems, reqs = W.serving_stream(seed=6, rate=10.0, duration=2 * args.serve_duration)
        rep, _ = serving.run_stream(ctx, problems, reqs, drain_s=args.serve_drain,
                                    server_opts=dict(epoch_paths=1 << 24, chunk_paths=1 << 20))
        rep["workload"] = ("the same request mix as 'serving' (seed 6), Poisson 10 requests/s for "
                           f"{2 * args.serve_duration:g} s")
        result["serving_light"] = rep
        print(f"serving at 10 requests/s: {rep['completed']} of {rep['offered_requests']} completed, "
              f"p50 {rep['p50_ms']:.0f} ms, p99 {rep['p99_ms']:.0f} ms", file=sys.stderr, flush=True)
    if args.cpu_paths > 0:
        print("timing the CPU oracle sample ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(pd, nodes, args.cpu_paths)
    print(json.dumps(result), flush=True)
    prob.close()
    ctx.close()


if __name__ == "__main__":
    main()
