"""Pins of the oracle's grid gradient (second-order differences).

* Exact, at every point including the edges, for quadratic polynomials
  (the central and three-point one-sided differences are exact to degree 2).
* Second-order convergence on a smooth non-polynomial function.
* Equal to numpy.gradient with edge_order=2 (the same formulas for a uniform
  grid) in 2D and 3D.
"""
import numpy as np
import pytest

from oracle import grid as G
from paper_1512_02818_amd import workloads as W


def _grid(fn, n, lo, hi):
    D = len(n)
    pts = W.grid_points(n, lo, hi)
    return {"dim": D, "n": list(n), "lo": list(lo), "hi": list(hi), "data": fn(pts).reshape(n[::-1])}, pts


def test_exact_for_quadratics():
    q = lambda p: 0.3 + 1.5 * p[:, 0] - 2.0 * p[:, 1] + 0.7 * p[:, 0] ** 2 - 1.1 * p[:, 0] * p[:, 1] + 0.4 * p[:, 1] ** 2  # noqa: E731
    g, pts = _grid(q, (9, 13), (0.2, -1.0), (1.4, 0.5))
    gx, gy = G.gradient(g)
    ex = 1.5 + 1.4 * pts[:, 0] - 1.1 * pts[:, 1]
    ey = -2.0 - 1.1 * pts[:, 0] + 0.8 * pts[:, 1]
    assert np.allclose(gx["data"].ravel(), ex, rtol=0, atol=1e-12)
    assert np.allclose(gy["data"].ravel(), ey, rtol=0, atol=1e-12)


def test_second_order_convergence():
    f = lambda p: np.sin(2 * p[:, 0]) * np.cos(3 * p[:, 1])  # noqa: E731
    errs = []
    for n in (33, 65, 129):
        g, pts = _grid(f, (n, n), (0.0, 0.0), (1.0, 1.0))
        gx, _ = G.gradient(g)
        ex = 2 * np.cos(2 * pts[:, 0]) * np.cos(3 * pts[:, 1])
        errs.append(np.max(np.abs(gx["data"].ravel() - ex)))
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.5, errs


@pytest.mark.parametrize("n", [(7, 5), (6, 9, 4)])
def test_matches_numpy_gradient(n):
    rng = np.random.default_rng(1)
    D = len(n)
    lo, hi = [0.1, -0.3, 2.0][:D], [0.9, 0.6, 2.5][:D]
    data = rng.normal(size=n[::-1])
    g = {"dim": D, "n": list(n), "lo": lo, "hi": hi, "data": data}
    ours = G.gradient(g)
    spacing = [(hi[d] - lo[d]) / (n[d] - 1) for d in range(D)]
    ref = np.gradient(data, *spacing[::-1], edge_order=2)  # arrays per array axis (z, y, x)
    for d in range(D):
        assert np.allclose(ours[d]["data"], ref[D - 1 - d], rtol=1e-13, atol=1e-13)


def test_residual_exact_for_quadratic_u():
    """For a quadratic u~ the differences are exact, so r = f - (L + c) u~ in
    closed form (b, c, f of the unit-square problem, sigma = 1)."""
    from oracle import oracle as O
    pd = W.unit_square_problem(seed=0)
    q = lambda p: 0.3 + 1.5 * p[:, 0] - 2.0 * p[:, 1] + 0.7 * p[:, 0] ** 2 - 1.1 * p[:, 0] * p[:, 1] + 0.4 * p[:, 1] ** 2  # noqa: E731
    g, pts = _grid(q, (9, 7), (0.0, 0.0), (1.0, 1.0))
    r = G.residual(pd, g).ravel()
    ux = 1.5 + 1.4 * pts[:, 0] - 1.1 * pts[:, 1]
    uy = -2.0 - 1.1 * pts[:, 0] + 0.8 * pts[:, 1]
    lap = 1.4 + 0.8
    b = np.stack([0.5 * pts[:, 0], -0.3 * pts[:, 1]], axis=1)  # the problem's drift
    c = -(1.0 + pts[:, 0] ** 2 + pts[:, 1] ** 2)
    want = O.source(pd, pts) - (0.5 * lap + b[:, 0] * ux + b[:, 1] * uy + c * q(pts))
    assert np.allclose(r, want, rtol=0, atol=1e-11)


def test_residual_of_the_solution_vanishes_at_second_order():
    """u~ = U (the exact solution): r -> 0 like dx^2; and for u~ = U + p the
    difference residual approaches the exact one -(L + c) p."""
    pd = W.unit_square_problem(seed=0)
    errs0, errs1 = [], []
    for n in (33, 65, 129):
        g, _ = _grid(lambda p: W.manufactured_u(pd, p), (n, n), (0.0, 0.0), (1.0, 1.0))
        errs0.append(np.max(np.abs(G.residual(pd, g))))
    for a, b in zip(errs0, errs0[1:]):
        assert 3.3 < a / b < 4.7, errs0
    # p has modes up to k = 16: finer grids, and at least second order
    for n in (129, 257, 513):
        gu, gr, _ = W.correction_grids(pd, n=n, seed=1, dtype=np.float64)
        errs1.append(np.max(np.abs(G.residual(pd, gu) - gr["data"])))
    for a, b in zip(errs1, errs1[1:]):
        assert a / b > 3.3, errs1
    assert errs1[-1] < 1e-3 * np.max(np.abs(gr["data"]))
