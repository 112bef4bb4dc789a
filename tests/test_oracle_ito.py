"""Pins of the oracle's Ito control variate (Sec. 2.3, eq. F:xiControlVariate).

xi = -int Y sigma grad(u~) . dW is accumulated along the Euler-Maruyama path
with the left-point rule, xi_{k+1} = xi_k - Y_k sigma grad(u~)(X_k) . sqrt(h)
N_k, and the estimator is phi + xi. What fixes it, independently of the code:

* E[xi] = 0 exactly for the discrete scheme: each increment is an adapted
  integrand times a centred increment, summed up to a stopping time. Checked
  over every Rademacher sign sequence of a short walk (exact enumeration).
* Closed form for a linear solution with b = c = f = 0: sum sqrt(h) sigma N_k
  = X_K - x0, so phi + xi = U(x0) + grad U . (Pi(X_K) - X_K) on every path,
  with X_K rebuilt from the path's normals.
* Exact control variate (u~ = u): V[phi + xi] vanishes as h -> 0 (paper, the
  remark after eq. F:xiControlVariate), here linearly in h.
* Ito's formula links xi to the correction estimator: with the same u~,
  phi + xi - (u~(x0) + e) -> 0 path by path as h -> 0 (at rate sqrt(h)).
* Node statistics against the records.
"""
import itertools
import math

import numpy as np
import pytest

from paper_1512_02818_amd import workloads as W


def _enum_problem():
    pd = {"dim": 2, "domain": "box", "lo": [0.1, 0.0], "hi": [0.35, 0.3], "sigma": 0.9,
          "b0": [0.2, -0.1], "B": [[0.5, 0.3], [-0.2, -0.3]], "c_a": -1.0, "c_b": -2.0,
          "trig": [{"amp": 0.5, "k": [2.0, 3.0], "phase": [0.3, -0.2]}],
          "mono": [{"coef": 1.0, "e": [2, 1]}, {"coef": -0.4, "e": [0, 3]}], "seed": 77}
    return pd, (0.2, 0.16)


@pytest.mark.parametrize("mode", ["naive", "shift"])
def test_xi_has_mean_zero_over_every_rademacher_path(orc, mode):
    pd, x0 = _enum_problem()
    grad = W.gradient_grids(pd, n=65, amp=0.0, dtype=np.float64)
    h, K = 4e-3, 6
    xis, psis, phis = [], [], []
    # every sequence of K steps x 2 signs is equally likely (4^-K); a path that
    # stops early ignores the rest of its sequence
    for seq in itertools.product((-1.0, 1.0), repeat=2 * K):
        r = orc.run_path_noise(pd, x0, np.array(seq), np.ones(K), h=h, exit=mode, max_steps=K,
                               grad=grad)
        xis.append(r["e"] - r["phi"])
        psis.append(r["e"])
        phis.append(r["phi"])
    xis = np.array(xis)
    assert np.std(xis) > 1e-2  # not degenerate
    assert abs(math.fsum(xis) / len(xis)) < 1e-14
    # and it is a control variate: phi + xi varies far less than phi
    assert np.var(psis) < 0.05 * np.var(phis)


@pytest.mark.parametrize("dim,mode", [(2, "shift"), (2, "naive"), (2, "bridge"), (3, "shift")])
def test_linear_solution_closed_form(orc, dim, mode):
    sigma = 1.3
    coef = [1.0, 0.5] if dim == 2 else [1.0, 0.0, -0.7]
    mono = [{"coef": c, "e": [int(q == d) for q in range(dim)]} for d, c in enumerate(coef) if c]
    pd = {"dim": dim, "domain": "box", "lo": [0.0] * dim, "hi": [1.0] * dim, "sigma": sigma,
          "b0": [0.0] * dim, "B": np.zeros((dim, dim)).tolist(), "c_a": 0.0, "c_b": 0.0,
          "mono": mono, "seed": 5}
    grad = W.gradient_grids(pd, n=5, amp=0.0, dtype=np.float64)
    for d in range(dim):
        assert np.all(grad[d]["data"] == coef[d])
    h, n = 1e-3, 60
    nodes = np.array([[0.3, 0.6, 0.5][:dim], [0.8, 0.2, 0.4][:dim]])
    _, rec = orc.solve_nodes(pd, nodes, record=True, h=h, n_paths=n, exit=mode, grad=grad)
    g = np.array(coef)
    for q, r in enumerate(rec):
        i, j = divmod(q, n)
        # the last point of the walk before its exit projection, from its normals
        XK = nodes[i] + sigma * math.sqrt(h) * sum(orc.step_normals(pd, i, j, k) for k in range(int(r["steps"])))
        want = nodes[i] @ g + g @ (np.array(r["x_exit"][:dim]) - XK)
        assert abs(r["e"] - want) <= 1e-12, (q, r["e"], want)
    assert np.all(rec["capped"] == 0)
    # phi alone moves by O(1), phi + xi only by the exit projection
    assert np.std(rec["phi"]) > 0.1
    assert np.abs(rec["e"] - np.repeat(nodes @ g, n)).max() < 7 * sigma * math.sqrt(h)


def test_exact_gradient_variance_vanishes_with_h(orc):
    pd = W.unit_square_problem(seed=13)
    nodes = W.unit_square_nodes()[::4]
    exact = W.manufactured_u(pd, nodes)
    grad = W.gradient_grids(pd, n=257, amp=0.0, dtype=np.float64)
    vr = {}
    for h, bias in ((1e-3, 3e-3), (2.5e-4, 1e-3)):
        st = orc.solve_nodes(pd, nodes, h=h, n_paths=2000, grad=grad)
        assert np.all(np.abs(st["mean"] - exact) <= 3 * st["stderr"] + bias)
        assert np.all(st["rho"] < -0.99)
        vr[h] = st["vr"]
    assert np.all(vr[1e-3] > 30.0)
    ratio = vr[2.5e-4] / vr[1e-3]  # V[phi + xi] ~ h
    assert np.all((ratio > 2.5) & (ratio < 6.5)), ratio


def test_agrees_with_correction_estimator_as_h_shrinks(orc):
    pd = W.unit_square_problem(seed=13)
    nodes = W.unit_square_nodes()[::4]
    gu, gr, _ = W.correction_grids(pd, n=257, seed=1, dtype=np.float64)
    grad = W.gradient_grids(pd, n=257, seed=1, dtype=np.float64)
    n = 800
    up0 = np.repeat(orc.interp(gu, nodes), n)
    rms = []
    for h in (4e-3, 1e-3, 2.5e-4):
        _, ri = orc.solve_nodes(pd, nodes, record=True, h=h, n_paths=n, grad=grad)
        _, rc = orc.solve_nodes(pd, nodes, record=True, h=h, n_paths=n, u_prev=gu, resid=gr)
        assert np.array_equal(ri["phi"], rc["phi"]) and np.array_equal(ri["steps"], rc["steps"])
        rms.append(np.sqrt(np.mean((ri["e"] - (up0 + rc["e"])) ** 2)))
        xi_rms = np.sqrt(np.mean((ri["e"] - ri["phi"]) ** 2))
    for a, b in zip(rms, rms[1:]):
        assert 1.5 < a / b < 2.7, rms  # sqrt(4) = 2
    assert rms[-1] < 0.1 * xi_rms


def test_statistics_against_records(orc):
    pd = W.unit_square_problem(seed=14)
    grad = W.gradient_grids(pd, n=129, seed=2, dtype=np.float64)
    nodes = W.unit_square_nodes()[:3]
    n = 1500
    st, rec = orc.solve_nodes(pd, nodes, record=True, h=1e-3, n_paths=n, grad=grad)
    for i in range(len(nodes)):
        r = rec[i * n:(i + 1) * n]
        psi, phi = r["e"], r["phi"]
        assert math.isclose(st["mean"][i], math.fsum(psi) / n, rel_tol=1e-13)
        assert math.isclose(st["mean_plain"][i], math.fsum(phi) / n, rel_tol=1e-13)
        assert math.isclose(st["var"][i], np.var(psi, ddof=1), rel_tol=1e-9)
        xi = psi - phi
        assert math.isclose(st["cov"][i], np.cov(phi, xi)[0, 1], rel_tol=1e-8)
        assert math.isclose(st["rho"][i], np.corrcoef(phi, xi)[0, 1], rel_tol=1e-8)
        assert math.isclose(st["vr"][i], np.var(phi, ddof=1) / np.var(psi, ddof=1), rel_tol=1e-9)


def test_bad_gradient_options_are_rejected(orc):
    pd = W.unit_square_problem(seed=1)
    grad = W.gradient_grids(pd, n=9, amp=0.0, dtype=np.float64)
    gu, gr, _ = W.correction_grids(pd, n=9, seed=1, dtype=np.float64)
    with pytest.raises(ValueError):
        orc.run_path(pd, (0.5, 0.5), 0, 0, h=1e-3, grad=grad[:1])  # one component in 2D
    with pytest.raises(ValueError):
        orc.make_opts(1e-3, u_prev=gu, resid=gr, grad=grad)
