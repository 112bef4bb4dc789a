"""Pins of the oracle on the paper's own example (Sec. 6, eq. F:PDE_ejemplo)
with every coefficient, the source and the boundary data tabulated, on the
stand-in box [0, 2]^2 (the paper's domain figure is missing).

* A tabulated g that reproduces an analytic g exactly (bilinear data) gives
  the same scores path by path.
* The generator's source f = Lap u + b.grad u + c u (sigma = sqrt(2)) against
  central finite differences of the exact u.
* The manufactured solution u = 2 cos(2 (y - 2) x) + sin(3 (x - 2) y) + 3.1
  is recovered: plain estimator, and the Ito control variate with u~ = u
  (its far smaller variance makes the check sharp), within 3 SE plus the
  scheme's O(h) bias.
"""
import numpy as np

from paper_1512_02818_amd import workloads as W


def test_tabulated_g_equals_analytic_g(orc):
    pd = W.bilinear_problem(seed=12)
    g = W.sampled_grid(pd, lambda p: W.manufactured_u(pd, p), n=17)
    tab = dict(pd, tab={"g": g})
    nodes = W.unit_square_nodes()[::4]
    _, r0 = orc.solve_nodes(pd, nodes, record=True, h=1e-3, n_paths=300)
    _, r1 = orc.solve_nodes(tab, nodes, record=True, h=1e-3, n_paths=300)
    assert np.array_equal(r0["steps"], r1["steps"])
    assert np.max(np.abs(r0["phi"] - r1["phi"])) < 1e-13
    # a different g grid changes the scores (the grid is really read)
    g2 = dict(g, data=g["data"] + 1.0)
    _, r2 = orc.solve_nodes(dict(pd, tab={"g": g2}), nodes, record=True, h=1e-3, n_paths=300)
    assert np.min(np.abs(r2["phi"] - r0["phi"])) > 0.1


def test_paper_example_source_matches_finite_differences():
    rng = np.random.default_rng(0)
    pts = rng.uniform(0.05, 1.95, size=(200, 2))
    b, c, f, u = W.paper_example_fields(pts)
    e = 1e-4
    U = W.paper_example_u
    ex, ey = np.array([e, 0.0]), np.array([0.0, e])
    ux = (U(pts + ex) - U(pts - ex)) / (2 * e)
    uy = (U(pts + ey) - U(pts - ey)) / (2 * e)
    lap = (U(pts + ex) + U(pts - ex) + U(pts + ey) + U(pts - ey) - 4 * U(pts)) / (e * e)
    fd = lap + b[:, 0] * ux + b[:, 1] * uy + c * U(pts)
    assert np.allclose(u, U(pts), rtol=0, atol=1e-14)
    assert np.max(np.abs(fd - f)) < 1e-4 * np.max(np.abs(f)), np.max(np.abs(fd - f))
    # the paper's coefficients: c < 0 and b along [1, 1]
    assert np.all(c < 0) and np.array_equal(b[:, 0], b[:, 1])


def test_paper_example_manufactured_solution(orc):
    pd = W.paper_example_problem(n=513)
    nodes = W.paper_example_nodes()[::3]
    exact = W.paper_example_u(nodes)
    st = orc.solve_nodes(pd, nodes, h=1e-3, n_paths=2000)
    assert np.all(np.abs(st["mean"] - exact) <= 3.5 * st["stderr"] + 0.03), (st["mean"] - exact, st["stderr"])
    gg = W.paper_example_gradient_grids(n=513)
    st = orc.solve_nodes(pd, nodes, h=2.5e-4, n_paths=3000, grad=gg)
    assert np.all(st["vr"] > 100)
    assert np.all(np.abs(st["mean"] - exact) <= 3 * st["stderr"] + 0.01), (st["mean"] - exact, st["stderr"])
