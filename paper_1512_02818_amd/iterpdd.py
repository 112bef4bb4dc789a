"""The multigrid-like outer iteration of PDD (Alg. A:IterPDD) on a 2D box
cut by axis-parallel interfaces, driven through the library: the fast fit of
the nodal constants (Alg. A:Fitting, pdd_fit_constants), the auxiliary variate
psi-bar from the error-propagation function w-bar (eq. F:w_bar, pdd_stage2 on
the homogeneous problem, and the Ito solve with grad(w-bar)), the cost ratio
kappa, the schedule a_J > ... > a_1 > a_0 (Alg. A:Scheduling, pdd_schedule),
then the levels: nodal solves to the balanced accuracy of each level (eq.
F:N_y_h: h_i = (a / (2 |beta_i|))^(1/delta) per node, N_i planned from a pilot
so that q SE_i = a / 2), the first one plain and every later one with the
pathwise control variate from the previous level's u~ (its gradient grids),
each followed by the second stage (pdd_stage2) that gives the level's u~.
Every path, interpolation and subdomain solve runs in the HIP library; this
module only sequences the calls and keeps the books.

Readings (where the algorithm's text is terse): level j (J >= j >= 1) runs
its nodal solves at accuracy a_{j-1} with the control variate built from
u~_j, and u~_J comes from plain solves at a_J, so that the last level reaches
a_0 (IterPDD(a_{j-1}, a_j) nests as in Sec. 1); grad(u~) is the
second-order difference gradient of the assembled grid (central differences
mix the two sides' slopes on an interface line itself), stored as the lookup
table of Sec. 6; V[psi-bar] and rho[phi, psi-bar] come from one Ito solve at
the smallest step of the fitting cloud rather than from a fit over the cloud.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import pdd


def _sync():
    import torch
    torch.cuda.synchronize()


def homogeneous(pd: dict) -> dict:
    """The same operator with f = 0 and g = 0 (no manufactured terms, no
    tabulated source or boundary data): the problem of w-bar (eq. F:w_bar)."""
    out = dict(pd, trig=[], mono=[], fx=[], gx=[])
    if pd.get("tab"):
        tab = dict(pd["tab"])
        tab.pop("f", None)
        tab.pop("g", None)
        out["tab"] = tab
    return out


def grid_dict(pd: dict, n):
    return {"dim": 2, "n": [int(n[0]), int(n[1])], "lo": list(pd["lo"][:2]), "hi": list(pd["hi"][:2])}


def fit(ctx, prob, nodes, m_hat=100, n_hat=1000, h_range=(1e-3, 1e-2), delta=1.0, stream0=1 << 24):
    """Alg. A:Fitting's cloud of m_hat steps in h_range, n_hat paths per node
    and step, FP32: the fitted E[phi], beta, V[phi], alpha, E[tau] per node."""
    h = np.linspace(h_range[0], h_range[1], m_hat)
    item = {"problem": prob, "nodes": nodes, "opts": dict(precision="fp32", stream_id=stream0)}
    return pdd.fit_constants(ctx, item, h, n_hat, delta=delta)


def psi_bar(ctx, pd, prob, nodes, part, beta, h, n_paths, stream_id=(1 << 24) + 4096):
    """V[psi-bar] and rho[phi, psi-bar] per node: w-bar solves the
    homogeneous BVP with interface data R[sign(beta_i)] (eq. F:w_bar), and the
    Ito solve with grad(w-bar) gives xi = -int Y sigma grad(w-bar).dW, whose
    variance is V[psi-bar] and whose correlation with phi is -rho[phi, psi-bar]
    (eq. F:Bar_psi; only squares enter the schedule)."""
    p0 = pdd.Problem(ctx, homogeneous(pd))
    w = pdd.stage2(p0, part["n"], part["cuts"], nodes, np.sign(beta), part["rbf_eps"])
    p0.close()
    g = grid_dict(pd, part["n"])
    gd, gt = pdd.grid_gradient(ctx, g, w)
    gt = [t.float().contiguous() for t in gt]
    st = pdd.stats_to_numpy(pdd.solve_ito(prob, gd, gt, nodes, dt=h, n_paths=n_paths, precision="fp32",
                                          stream_id=stream_id))
    v_xi = st["var"] - st["var_plain"] - 2.0 * st["cov"]
    return np.maximum(v_xi, 0.0), -st["rho"], w


def measure_kappa(ctx, prob, nodes, pd, part, h, n_paths, stream_id=(1 << 24) + 8192):
    """Cost of a path step with the Ito control variate over one without
    (kappa of eq. F:VR_Pointwise_cost): two solves of the same paths, their
    path-kernel times per path-step (HIP events)."""
    n = part["n"]
    g = grid_dict(pd, n)
    import torch
    zero = torch.zeros((n[1], n[0]), dtype=torch.float64, device="cuda")
    gd, gt = pdd.grid_gradient(ctx, g, zero)
    gt = [t.float().contiguous() for t in gt]
    rates = []
    for ito in (False, True):
        for rep in range(2):  # the first of each is a warm-up
            pdd.kernel_times(ctx)
            if ito:
                st = pdd.solve_ito(prob, gd, gt, nodes, dt=h, n_paths=n_paths, precision="fp32", stream_id=stream_id,
                                   time_kernel=True)
            else:
                st = pdd.solve_nodes(prob, nodes, dt=h, n_paths=n_paths, precision="fp32", stream_id=stream_id,
                                     time_kernel=True)
            steps = int(pdd.stats_to_numpy(st)["steps_sum"].sum())
            ms = sum(pdd.kernel_times(ctx))
        rates.append(ms / steps)
    return rates[1] / rates[0]


def level_solve(ctx, prob, nodes, a, beta, q, delta, grads=None, n_pilot=128, n_max=1 << 30, stream0=0,
                h_bounds=(1e-5, 1e-2)):
    """Nodal solves to the balanced accuracy a (eq. F:N_y_h): per node its
    own step h_i = (a / (2 |beta_i|))^(1/delta) (within h_bounds) and paths
    until q SE_i = a / 2 (pilot, then plan); with `grads` (gradient grids and
    tensors) the Ito control variate. One pdd_solve_to_tolerance over the
    nodes as separate items. Returns (stats per node, h per node)."""
    h = np.clip((a / (2.0 * np.abs(beta))) ** (1.0 / delta), *h_bounds)
    # one statistics buffer for all the nodes (one copy back, not one per node)
    out = pdd.alloc_stats(len(nodes))
    sz = pdd.STATS_DTYPE.itemsize
    items = []
    for i, x in enumerate(nodes):
        it = {"problem": prob, "nodes": x[None, :], "out": out[i * sz:(i + 1) * sz],
              "opts": dict(dt=float(h[i]), precision="fp32", stream_id=stream0 + i)}
        if grads is not None:
            it["grad"], it["grad_t"] = grads
        items.append(it)
    pdd.solve_to_tolerance(ctx, items, a / (2.0 * q), n_pilot, n_max)
    return pdd.stats_to_numpy(out), h


def run(ctx, pd, nodes, part, a0, q=2.0, delta=1.0, a_max=1.0, exact=None, schedule=None, fit_cloud=(100, 1000),
        psi_paths=20000, log=None):
    """Alg. A:IterPDD to the nodal tolerance a0. `exact`: a callable giving
    the exact u at points (for the error columns only). `schedule`: levels
    a_0 < ... < a_J to use instead of pdd_schedule's. Returns a report dict:
    constants, schedule, per-level records (accuracy, mean step, mean paths,
    path-steps, wall time, RMS errors of the nodal values and of u~, mean VR)
    and the totals."""
    import torch
    t_all = time.perf_counter()
    prob = pdd.Problem(ctx, pd)
    nodes = np.asarray(nodes, dtype=np.float64).reshape(-1, 2)
    t0 = time.perf_counter()
    c = fit(ctx, prob, nodes, m_hat=fit_cloud[0], n_hat=fit_cloud[1], delta=delta)
    beta, V, alpha, E_tau = c["beta"], c["V_phi"], c["alpha"], c["E_tau"]
    V = np.maximum(V, 1e-12)
    h_psi = 1e-3
    V_psi, rho_psi, _ = psi_bar(ctx, pd, prob, nodes, part, beta, h_psi, psi_paths)
    kappa = measure_kappa(ctx, prob, nodes, pd, part, h_psi, 20000)
    K = 4.0 * q * q * np.maximum(E_tau, 1e-6) * (2.0 * np.abs(beta)) ** (1.0 / delta)
    if schedule is None:
        levels, pred = pdd.schedule(K, V, alpha, beta, V_psi, np.clip(rho_psi, -1, 1), a0, kappa, delta, a_max)
    else:
        levels, pred = list(schedule), []
    _sync()
    setup_s = time.perf_counter() - t0
    if log:
        log(f"iterpdd: kappa {kappa:.2f}, schedule {['%.4g' % a for a in levels]}")
    g = grid_dict(pd, part["n"])
    ax = [np.linspace(pd["lo"][d], pd["hi"][d], part["n"][d]) for d in range(2)]
    X, Y = np.meshgrid(ax[0], ax[1])
    U = exact(np.stack([X.ravel(), Y.ravel()], axis=1)).reshape(part["n"][1], part["n"][0]) if exact else None
    u_nodes = exact(nodes) if exact else None
    records = []
    grads = None
    J = len(levels) - 1
    for lev in range(J, -1, -1):  # the first solve at a_J is plain; each later one uses the previous u~
        a = levels[lev]
        _sync()
        t1 = time.perf_counter()
        st, h = level_solve(ctx, prob, nodes, a, beta, q, delta, grads=grads, stream0=(J - lev) * 4096)
        vals = st["mean"]
        u = pdd.stage2(prob, part["n"], part["cuts"], nodes, vals, part["rbf_eps"])
        gd, gt = pdd.grid_gradient(ctx, g, u)
        _sync()
        wall = time.perf_counter() - t1
        grads = (gd, [t.float().contiguous() for t in gt])
        rec = {"accuracy": a, "control_variate": lev < J, "mean_dt": float(np.mean(h)),
               "mean_paths": float(np.mean(st["n"])), "path_steps": int(st["steps_sum"].sum()), "wall_s": wall,
               "max_q_se_over_half_a": float(np.max(q * st["stderr"] / (a / 2)))}
        if lev < J:
            rec["mean_vr"] = float(np.mean(st["vr"]))
            rec["mean_abs_rho"] = float(np.mean(np.abs(st["rho"])))
        if exact:
            rec["rms_error_nodes"] = float(np.sqrt(np.mean((vals - u_nodes) ** 2)))
            rec["max_error_nodes"] = float(np.max(np.abs(vals - u_nodes)))
            rec["rms_error_u_tilde"] = float(np.sqrt(np.mean((u.cpu().numpy() - U) ** 2)))
        records.append(rec)
        if log:
            log(f"  level a={a:.4g}: {rec['path_steps']:.3e} path-steps, {wall * 1e3:.1f} ms"
                + (f", RMS err {rec['rms_error_nodes']:.2e}" if exact else ""))
    # the comparison: PlainPDD(a0), the same balanced rule without control variate
    _sync()
    t2 = time.perf_counter()
    st0, _ = level_solve(ctx, prob, nodes, a0, beta, q, delta, grads=None, stream0=1 << 20)
    _sync()
    plain = {"accuracy": a0, "path_steps": int(st0["steps_sum"].sum()), "wall_s": time.perf_counter() - t2,
             "mean_paths": float(np.mean(st0["n"]))}
    if exact:
        plain["rms_error_nodes"] = float(np.sqrt(np.mean((st0["mean"] - u_nodes) ** 2)))
    prob.close()
    iter_steps = sum(r["path_steps"] for r in records)
    iter_wall = sum(r["wall_s"] for r in records)
    return {"a0": a0, "q": q, "delta": delta, "kappa": kappa, "schedule": levels, "predicted_speedups": pred,
            "constants": {"beta": beta.tolist(), "V_phi": V.tolist(), "alpha": alpha.tolist(), "E_tau": E_tau.tolist(),
                          "V_psi": V_psi.tolist(), "rho_phi_psi": rho_psi.tolist(), "K": K.tolist()},
            "setup_s": setup_s, "levels": records, "iterpdd_path_steps": iter_steps, "iterpdd_wall_s": iter_wall,
            "plainpdd": plain, "speedup_path_steps": plain["path_steps"] / max(iter_steps, 1),
            "speedup_wall": plain["wall_s"] / max(iter_wall, 1e-12), "total_s": time.perf_counter() - t_all}
