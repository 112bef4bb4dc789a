"""Pins of the oracle's correction estimator and node statistics (CPU only).

* Exact control variate (Lemma 1 and eq. F:Combining_method): when u_prev is
  the solution and the grid reproduces it exactly (a bilinear u, so that
  Lap u = 0 and bilinear interpolation is exact), the correction score
  e = (g - u_prev)(X_tau) Y - int r Y vanishes on every path: zero variance,
  and the estimate equals u(x0) whatever the paths did.
* Perturbed u_prev (32 Fourier modes, amplitude 1e-2, on a 257^2 grid): the
  estimate stays within 3 SE + O(dx^2) of u, the variance drops (VR > 1,
  eq. F:Variance_Reduction) and VR matches 1/(1 - rho^2) (eq. F:Rho) to
  first order.
* Node sums and statistics against math.fsum of the per-path records.
* Resume: paths [0, a) + [a, N) are the same paths as [0, N).
"""
import math

import numpy as np

from paper_1512_02818_amd import workloads as W


def test_exact_control_variate_zero_variance(orc):
    pd = W.bilinear_problem(seed=12)
    grid_u = W.sampled_grid(pd, lambda p: W.manufactured_u(pd, p), n=33)
    grid_r = W.sampled_grid(pd, lambda p: np.zeros(len(p)), n=33)
    nodes = W.unit_square_nodes()[::3]
    st = orc.solve_nodes(pd, nodes, h=1e-3, n_paths=3000, u_prev=grid_u, resid=grid_r)
    exact = W.manufactured_u(pd, nodes)
    assert np.all(st["var"] < 1e-24)
    assert np.allclose(st["mean"], exact, rtol=0, atol=1e-13)
    # the plain estimator of the same paths is noisy and agrees statistically
    assert np.all(st["var_plain"] > 1e-2)
    assert np.all(np.abs(st["mean_plain"] - exact) <= 3 * np.sqrt(st["var_plain"] / 3000) + 2e-3)
    assert np.all(np.abs(st["rho"] + 1.0) < 1e-6)


def test_perturbed_control_variate(orc):
    pd = W.unit_square_problem(seed=13)
    gu, gr, _ = W.correction_grids(pd, n=257, seed=1, dtype=np.float32)
    nodes = W.unit_square_nodes()
    n = 4000
    st = orc.solve_nodes(pd, nodes, h=1e-3, n_paths=n, u_prev=gu, resid=gr)
    exact = W.manufactured_u(pd, nodes)
    # bias allowance: O(dx^2) interpolation error of u_prev and r plus the O(h) scheme bias
    assert np.all(np.abs(st["mean"] - exact) <= 3 * st["stderr"] + 1e-3)
    assert np.all(st["vr"] > 20.0)
    assert np.all(st["rho"] < -0.97)
    vr_rho = 1.0 / (1.0 - st["rho"] ** 2)
    assert np.allclose(st["vr"], vr_rho, rtol=0.35)


def test_sums_against_fsum(orc):
    pd = W.unit_square_problem(seed=14)
    gu, gr, _ = W.correction_grids(pd, n=129, seed=2, dtype=np.float64)
    nodes = W.unit_square_nodes()[:4]
    n = 2500
    st, rec = orc.solve_nodes(pd, nodes, record=True, h=1e-3, n_paths=n, u_prev=gu, resid=gr)
    for i in range(len(nodes)):
        r = rec[i * n:(i + 1) * n]
        phi, e = r["phi"], r["e"]
        mean_phi = math.fsum(phi) / n
        var_phi = math.fsum((phi - mean_phi) ** 2) / (n - 1)
        mean_e = math.fsum(e) / n
        var_e = math.fsum((e - mean_e) ** 2) / (n - 1)
        cov_pe = math.fsum((phi - mean_phi) * (e - mean_e)) / (n - 1)
        u0 = orc.interp(gu, nodes[i:i + 1])[0]
        assert math.isclose(st["mean_plain"][i], mean_phi, rel_tol=1e-14, abs_tol=1e-15)
        assert math.isclose(st["var_plain"][i], var_phi, rel_tol=1e-11)
        assert math.isclose(st["mean"][i], u0 + mean_e, rel_tol=1e-14, abs_tol=1e-15)
        assert math.isclose(st["var"][i], var_e, rel_tol=1e-8)
        cov_xi = cov_pe - var_phi
        v_xi = var_e + var_phi - 2 * cov_pe
        assert math.isclose(st["cov"][i], cov_xi, rel_tol=1e-8)
        assert math.isclose(st["rho"][i], cov_xi / math.sqrt(var_phi * v_xi), rel_tol=1e-6)
        assert st["steps_sum"][i] == int(r["steps"].sum())
        assert math.isclose(st["stderr"][i], math.sqrt(var_e / n), rel_tol=1e-8)
        # the compensated pairs sum to the exact sums
        assert math.isclose(st["sums"][i][0] + st["sums"][i][1], math.fsum(phi), rel_tol=1e-15)
        assert math.isclose(st["sums"][i][2] + st["sums"][i][3], math.fsum(phi * phi),
                            rel_tol=1e-15)


def test_split_resume_is_the_same_paths(orc):
    pd = W.unit_square_problem(seed=15)
    nodes = W.unit_square_nodes()[5:8]
    n, a = 900, 377
    _, full = orc.solve_nodes(pd, nodes, record=True, h=1e-3, n_paths=n)
    _, r1 = orc.solve_nodes(pd, nodes, record=True, h=1e-3, n_paths=a)
    _, r2 = orc.solve_nodes(pd, nodes, record=True, h=1e-3, n_paths=n - a, path_offset=a)
    for i in range(len(nodes)):
        joined = np.concatenate([r1[i * a:(i + 1) * a], r2[i * (n - a):(i + 1) * (n - a)]])
        assert joined.tobytes() == full[i * n:(i + 1) * n].tobytes()  # bitwise, NaN e included
    # run_paths draws exactly the same path as solve_nodes for a (node, path) pair
    sel = orc.run_paths(pd, nodes, [1, 2, 0], [5, 899, 400], h=1e-3)
    assert sel[0:1].tobytes() == full[1 * n + 5:1 * n + 6].tobytes()
    assert sel[1:2].tobytes() == full[2 * n + 899:2 * n + 900].tobytes()
    assert sel[2:3].tobytes() == full[400:401].tobytes()


def test_cap_and_empty(orc):
    pd = W.unit_square_problem(seed=16)
    nodes = W.unit_square_nodes()[:2]
    st, rec = orc.solve_nodes(pd, nodes, record=True, h=1e-3, n_paths=200, max_steps=20)
    assert np.all(rec["steps"] <= 20)
    assert st["n_capped"].sum() == int(np.sum(rec["capped"]))
    assert st["n_capped"].sum() > 0
    capped = rec[rec["capped"] == 1]
    assert np.all(capped["steps"] == 20)
    empty = orc.solve_nodes(pd, nodes, h=1e-3, n_paths=0)
    assert np.all(empty["n"] == 0) and np.all(np.isnan(empty["mean"]))
