"""Pins of the oracle's tabulated coefficients (CPU only).

The coefficients b, c and f of eq. F:EllipticBVP are general functions of x
(Sec. 2.1); a tabulated problem gives some of them on grids, read through
the bilinear / trilinear interpolation already pinned for grids.

* The input module's derivatives of U against central finite differences.
* Interpolation reproduces affine functions exactly, so a problem whose
  affine drift is tabulated walks the same paths as the analytic problem
  (same exit steps, scores equal to rounding), in 2D and 3D; likewise a
  tabulated constant killing rate.
* With non-affine tabulated b and c and the matching tabulated f, U is still
  the exact solution up to the interpolation error: node means within
  3 SE + the bias allowance of the closed-form pins.
* Malformed grids are rejected.
"""
import numpy as np
import pytest

from paper_1512_02818_amd import workloads as W

H = 1e-3


def test_manufactured_derivs_against_finite_differences():
    rng = np.random.default_rng(8)
    for dim in (2, 3):
        pd = W.random_problem(rng, dim=dim)
        pts = rng.uniform(0.2, 0.8, size=(20, dim)) * (np.asarray(pd["hi"][:dim]) - np.asarray(pd["lo"][:dim])) \
            + np.asarray(pd["lo"][:dim])
        u, grad, lap = W.manufactured_derivs(pd, pts)
        assert np.allclose(u, W.manufactured_u(pd, pts), rtol=0, atol=1e-13)
        eps = 1e-4
        lap_fd = np.zeros(len(pts))
        for d in range(dim):
            e = np.zeros(dim)
            e[d] = eps
            up, um = W.manufactured_u(pd, pts + e), W.manufactured_u(pd, pts - e)
            assert np.allclose(grad[:, d], (up - um) / (2 * eps), rtol=1e-6, atol=1e-6)
            lap_fd += (up - 2 * u + um) / eps ** 2
        assert np.allclose(lap, lap_fd, rtol=1e-4, atol=1e-3)


def _same_walks(orc, pd, tab_pd, nodes, n):
    st, rec = orc.solve_nodes(pd, nodes, record=True, h=H, n_paths=n)
    st2, rec2 = orc.solve_nodes(tab_pd, nodes, record=True, h=H, n_paths=n)
    same = rec["steps"] == rec2["steps"]
    assert same.mean() > 0.999, same.mean()
    assert np.all(np.abs(rec["phi"][same] - rec2["phi"][same]) <= 1e-10 * np.maximum(1.0, np.abs(rec["phi"][same])))
    assert np.allclose(st2["mean"], st["mean"], rtol=0, atol=1e-6)


@pytest.mark.parametrize("dim", [2, 3])
def test_tabulated_affine_drift_walks_the_same_paths(orc, dim):
    if dim == 2:
        pd = W.unit_square_problem(seed=3)
        nodes = W.unit_square_nodes()[::3]
    else:
        rng = np.random.default_rng(4)
        pd = W.random_problem(rng, dim=3)
        lo, hi = np.asarray(pd["lo"][:3]), np.asarray(pd["hi"][:3])
        nodes = lo + (hi - lo) * np.array([[0.5, 0.5, 0.5], [0.2, 0.7, 0.4]])
    # coarse grid (9 points per axis): exact for the affine drift
    tab = W.tabulated_problem(pd, n=9, fields=("b",), amp=0.0)
    _same_walks(orc, pd, tab, nodes, 400)


def test_tabulated_constant_killing_walks_the_same_paths(orc):
    pd = dict(W.unit_square_problem(seed=5), c_b=0.0, c_a=-1.5)
    tab = W.tabulated_problem(pd, n=5, fields=("c",), amp=0.0)
    _same_walks(orc, pd, tab, W.unit_square_nodes()[::4], 400)


def test_tabulated_nonaffine_coefficients_keep_the_exact_solution(orc):
    pd = W.unit_square_problem(seed=0)
    tab = W.tabulated_problem(pd, n=257, fields=("b", "c", "f"), amp=0.6, seed=2)
    nodes = W.unit_square_nodes()
    st = orc.solve_nodes(tab, nodes, h=H, n_paths=8000)
    exact = W.manufactured_u(pd, nodes)
    assert np.all(np.abs(st["mean"] - exact) <= 3 * st["stderr"] + 2e-3), (st["mean"] - exact, st["stderr"])
    # the perturbed coefficients do change the walk: the analytic source with
    # the tabulated b and c does not give U (mean squared z-score far above 1)
    wrong = dict(tab, tab={"b": tab["tab"]["b"], "c": tab["tab"]["c"]})
    st_w = orc.solve_nodes(wrong, nodes, h=H, n_paths=24000)
    z2 = np.mean(((st["mean"] - exact) / st["stderr"]) ** 2)
    z2_w = np.mean(((st_w["mean"] - exact) / st_w["stderr"]) ** 2)
    assert z2 < 3 and z2_w > 8, (z2, z2_w)


def test_tabulated_grid_errors(orc):
    pd = W.unit_square_problem(seed=0)
    tab = W.tabulated_problem(pd, n=9, fields=("c",), amp=0.0)
    bad = dict(tab, tab={"c": dict(tab["tab"]["c"], dim=3, n=[9, 9, 9])})
    with pytest.raises(ValueError):
        orc.solve_nodes(bad, W.unit_square_nodes()[:2], h=H, n_paths=10)
    bad = dict(tab, tab={"b": [None, None, tab["tab"]["c"]]})
    with pytest.raises(ValueError):
        orc.solve_nodes(bad, W.unit_square_nodes()[:2], h=H, n_paths=10)
