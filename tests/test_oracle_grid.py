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
