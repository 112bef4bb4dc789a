"""Pins of the oracle's second stage (interfacial interpolation, subdomain
solves, u~ assembly) and of its scheduling algorithm (Alg. A:Scheduling),
against what the mathematics fixes: interpolation conditions, linearity (Def.
D:Linear_interpolator) and the two-point closed form of the multiquadric
interpolant; exactness of the second-order finite-difference solve for
quadratic solutions and its second-order convergence; the closed-form
minimiser of the scheduling objective for a single uncorrelated node."""
import math

import numpy as np
import pytest

from oracle import stage2 as S2


def test_rbf_interpolates_the_data_and_is_linear():
    rng = np.random.default_rng(1)
    # nodes about 1/7 apart, as on the interfaces (flat multiquadrics on
    # clustered nodes are ill-conditioned)
    t = np.linspace(0, 1, 8) + rng.uniform(-0.02, 0.02, 8)
    z1, z2 = rng.normal(size=8), rng.normal(size=8)
    for eps in (2.0, 3.0, 7.0):
        assert np.allclose(S2.rbf_interpolate(t, z1, eps, t), z1, rtol=0, atol=1e-9)
        te = np.linspace(0, 1, 41)
        lhs = S2.rbf_interpolate(t, 2.5 * z1 - 0.7 * z2, eps, te)
        rhs = 2.5 * S2.rbf_interpolate(t, z1, eps, te) - 0.7 * S2.rbf_interpolate(t, z2, eps, te)
        assert np.allclose(lhs, rhs, atol=1e-9)


def test_rbf_two_point_closed_form():
    # s(t) = l1 q(t - t1) + l2 q(t - t2), q(r) = sqrt(1 + (eps r)^2); with
    # Q = q(t2 - t1): l1 = (z1 - Q z2) / (1 - Q^2), l2 = (z2 - Q z1) / (1 - Q^2)
    t1, t2, z1, z2, eps = 0.2, 0.9, 1.3, -0.4, 2.0
    Q = math.sqrt(1 + (eps * (t2 - t1)) ** 2)
    l1, l2 = (z1 - Q * z2) / (1 - Q * Q), (z2 - Q * z1) / (1 - Q * Q)
    te = np.array([0.0, 0.35, 0.5, 1.0])
    want = l1 * np.sqrt(1 + (eps * (te - t1)) ** 2) + l2 * np.sqrt(1 + (eps * (te - t2)) ** 2)
    assert np.allclose(S2.rbf_interpolate([t1, t2], [z1, z2], eps, te), want, atol=1e-13)


def test_rbf_converges_on_smooth_data():
    f = lambda t: np.sin(2 * t) + t * t  # noqa: E731
    te = np.linspace(0, 1, 201)
    errs = []
    for m in (5, 9, 17):
        t = np.linspace(0, 1, m)
        errs.append(np.max(np.abs(S2.rbf_interpolate(t, f(t), 3.0, te) - f(te))))
    assert errs[0] > 5 * errs[1] > 0 and errs[1] > 5 * errs[2]


def quad_problem(seed=0):
    """A quadratic manufactured u with affine drift and |x|^2 killing: the
    second-order differences are exact for it."""
    rng = np.random.default_rng(seed)
    co = rng.uniform(-1, 1, 6)
    return {"dim": 2, "domain": "box", "lo": [0.0, 0.0], "hi": [1.0, 1.5], "sigma": 1.3,
            "b0": [0.2, -0.4], "B": [[0.5, 0.3], [-0.2, 0.1]], "c_a": -1.0, "c_b": -0.7,
            "trig": [], "mono": [{"coef": float(co[0]), "e": [2, 0]}, {"coef": float(co[1]), "e": [1, 1]},
                                 {"coef": float(co[2]), "e": [0, 2]}, {"coef": float(co[3]), "e": [1, 0]},
                                 {"coef": float(co[4]), "e": [0, 1]}, {"coef": float(co[5]), "e": [0, 0]}],
            "fx": [], "gx": [], "seed": 0}


def exact_on_grid(pd, n):
    from paper_1512_02818_amd import workloads as W
    ax = S2.grid_axes(n, pd["lo"], pd["hi"])
    X, Y = np.meshgrid(ax[0], ax[1])
    return W.manufactured_u(pd, np.stack([X.ravel(), Y.ravel()], axis=1)).reshape(n[1], n[0])


def test_subdomain_solve_is_exact_for_quadratics(orc):
    pd = quad_problem()
    n = (21, 31)
    U = exact_on_grid(pd, n)
    for box in ((0, 20, 0, 30), (5, 12, 3, 30), (0, 7, 10, 19)):
        u = np.full_like(U, np.nan)
        i0, i1, j0, j1 = box
        u[j0:j1 + 1, i0:i1 + 1] = U[j0:j1 + 1, i0:i1 + 1]
        u[j0 + 1:j1, i0 + 1:i1] = np.nan
        v = S2.subdomain_solve(pd, n, box, u)
        assert np.max(np.abs(v[j0:j1 + 1, i0:i1 + 1] - U[j0:j1 + 1, i0:i1 + 1])) < 1e-10, box


def test_subdomain_solve_converges_at_second_order(orc):
    from paper_1512_02818_amd import workloads as W
    pd = W.unit_square_problem(seed=0)
    errs = []
    for m in (17, 33, 65):
        n = (m, m)
        U = exact_on_grid(pd, n)
        box = (0, (m - 1) // 2, 0, m - 1)  # the left half, exact values on its boundary
        u = U.copy()
        u[1:-1, 1:(m - 1) // 2] = np.nan
        v = S2.subdomain_solve(pd, n, box, u)
        errs.append(np.max(np.abs(v - U)))
    assert 3.3 < errs[0] / errs[1] < 4.7 and 3.3 < errs[1] / errs[2] < 4.7, errs


def test_stage2_from_exact_nodal_values(orc):
    """u~ from the exact u at the unit-square nodes: the interface lines carry
    the interpolation error of 6 nodes + 2 ends per line, the subdomains add
    their O(dx^2) error; u~ equals g on the boundary."""
    from paper_1512_02818_amd import workloads as W
    pd = W.unit_square_problem(seed=0)
    nodes = W.unit_square_nodes()
    vals = W.manufactured_u(pd, nodes)
    n = (129, 129)
    u = S2.stage2(pd, n, [[0.25, 0.5, 0.75], []], nodes, vals, 3.0)
    U = exact_on_grid(pd, n)
    assert not np.isnan(u).any()
    assert np.max(np.abs(u[0, :] - U[0, :])) < 1e-12 and np.max(np.abs(u[:, -1] - U[:, -1])) < 1e-12
    err = np.abs(u - U)
    assert np.max(err) < 2e-2 and np.sqrt(np.mean(err ** 2)) < 5e-3, (np.max(err), np.sqrt(np.mean(err ** 2)))
    # at the nodes themselves u~ is the nodal value (interpolation condition)
    for x, z in zip(nodes, vals):
        i, j = int(round(x[0] * 128)), x[1] * 128
        jj = int(np.floor(j))
        if abs(j - jj) < 1e-9:
            assert abs(u[jj, i] - z) < 1e-9


def test_scheduling_single_node_closed_form():
    """One node with rho[phi, psi] = 0 and alpha = 0: the objective is
    K V (kappa Vpsi a^2 / (4 V) + (a_j / a)^p), p = 2 + 1/delta, minimal at
    a* = (2 p V a_j^p / (kappa Vpsi))^(1 / (p + 2))."""
    K, V, Vpsi, kappa, delta, a0 = [2.0], [0.4], [30.0], 1.8, 1.0, 0.01
    p = 2 + 1 / delta
    a_star = (2 * p * V[0] * a0 ** p / (kappa * Vpsi[0])) ** (1 / (p + 2))
    seq = S2.schedule(a0, K, V, Vpsi, [0.0], [0.0], [1.0], kappa, delta, a_max=2.0, s_min=1.5, max_levels=1)
    assert len(seq) == 2 and abs(seq[1] / a_star - 1) < 2e-3, (seq, a_star)
    obj = S2.schedule_cost(a_star, a0, K, V, Vpsi, [0.0], [0.0], [1.0], kappa, delta)
    want = K[0] * V[0] * (kappa * Vpsi[0] * a_star ** 2 / (4 * V[0]) + (a0 / a_star) ** p)
    assert abs(obj - want) < 1e-12 * want


def test_scheduling_stops_on_small_speedup():
    # a node whose control variate barely helps: no level is worth it
    seq = S2.schedule(0.01, [1.0], [0.5], [5e4], [0.0], [0.0], [1.0], 1.8, 1.0, a_max=1.0)
    assert seq == [0.01]
    # a strongly helping one: several nested levels, each coarser
    seq = S2.schedule(0.0025, [1.0, 2.0], [0.5, 0.3], [2.0, 3.0], [0.3, 0.1], [0.1, 0.2], [1.0, -2.0], 1.8, 1.0,
                      a_max=1.0)
    assert len(seq) >= 3 and all(b > a for a, b in zip(seq, seq[1:]))
