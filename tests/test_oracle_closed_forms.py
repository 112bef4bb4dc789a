"""Pins of the oracle's integrator and exit tests against closed forms (CPU).

Each check is |mean - exact| <= 3 SE + ALLOW, the error bound of eq.
F:Bound_of_error with q = 3 and a bias allowance ALLOW for the O(h) bias of
the bridge and shifted-boundary tests at h = 1e-3 (calibrated once: observed
bias magnitudes stay below 1e-3 on every case here, while the naive test's
sqrt(h) bias is ~2e-2).

* manufactured solution on the unit square (drift, killing, trig + monomial
  U, box bridge exit) - exact values of U at the 18 interface nodes;
* exit time of a ball, E[tau] = (R^2 - |x - c|^2) / (D sigma^2), 2D and 3D,
  sigma = 1 and 0.8; the mean exit step times h must match it too (eq. F:nu);
* killing in a ball with constant c: modified Bessel I0 (2D) and the
  sinh form (3D);
* harmonic boundary data with b = c = f = 0: u = g;
* exit time of a rectangle: the Fourier series of the torsion function.
"""
import numpy as np
import pytest
from scipy.special import i0

from paper_1512_02818_amd import workloads as W

ALLOW = 1e-3
H = 1e-3


def _check(st, exact, allow=ALLOW):
    err = np.abs(st["mean"] - exact)
    bound = 3 * st["stderr"] + allow
    assert np.all(err <= bound), (st["mean"], exact, st["stderr"])


@pytest.mark.parametrize("exit_mode", ["bridge", "shift"])
def test_unit_square_manufactured(orc, exit_mode):
    pd = W.unit_square_problem(seed=0)
    nodes = W.unit_square_nodes()
    st = orc.solve_nodes(pd, nodes, h=H, n_paths=12000, exit=exit_mode)
    _check(st, W.manufactured_u(pd, nodes), allow=2e-3)
    assert np.all(st["n_capped"] == 0)


def test_unit_square_naive_shows_sqrt_h_bias(orc):
    """The naive test's bias (delta = 1/2) is visible at these sizes."""
    pd = W.unit_square_problem(seed=0)
    nodes = W.unit_square_nodes()
    st = orc.solve_nodes(pd, nodes, h=H, n_paths=12000, exit="naive")
    z = (st["mean"] - W.manufactured_u(pd, nodes)) / st["stderr"]
    assert np.max(np.abs(z)) > 3.0


@pytest.mark.parametrize("sigma", [1.0, 0.8])
def test_ball_exit_time_2d(orc, sigma):
    pd = W.ball_exit_time_problem(dim=2, sigma=sigma, seed=3)
    pts = np.array([[0.0, 0.0], [0.5, 0.2], [-0.3, 0.7]])
    exact = (1.0 - np.sum(pts ** 2, axis=1)) / (2 * sigma ** 2)
    st = orc.solve_nodes(pd, pts, h=H, n_paths=12000)
    _check(st, exact, allow=1.5e-3)
    # nu = E[tau] / h: the mean exit step is the same estimator of E[tau]
    tau = st["mean_steps"] * H
    assert np.all(np.abs(tau - exact) <= 3 * st["stderr"] + 1.5e-3)


def test_ball_exit_time_3d_off_center(orc):
    cen = [0.1, 0.2, -0.1]
    pd = W.ball_exit_time_problem(dim=3, center=cen, seed=4)
    pts = np.array([cen, [0.5, 0.2, 0.1]])
    exact = (1.0 - np.sum((pts - np.array(cen)) ** 2, axis=1)) / 3.0
    for mode in ("bridge", "shift"):
        st = orc.solve_nodes(pd, pts, h=H, n_paths=12000, exit=mode)
        _check(st, exact)


def test_ball_killing_bessel_2d(orc):
    c = -2.0
    kappa = np.sqrt(2 * abs(c))
    pd = W.ball_killing_problem(dim=2, c=c, seed=5)
    pts = np.array([[0.0, 0.0], [0.6, 0.0], [0.3, -0.5]])
    r = np.sqrt(np.sum(pts ** 2, axis=1))
    st = orc.solve_nodes(pd, pts, h=H, n_paths=12000)
    _check(st, i0(kappa * r) / i0(kappa))


def test_ball_killing_3d(orc):
    c = -2.0
    k = np.sqrt(2 * abs(c))
    pd = W.ball_killing_problem(dim=3, c=c, seed=6)
    pts = np.array([[0.0, 0.0, 0.0], [0.6, 0.0, 0.2]])
    r = np.sqrt(np.sum(pts ** 2, axis=1))
    radial = np.where(r > 0, np.sinh(k * r) / (k * np.maximum(r, 1e-300)), 1.0)
    st = orc.solve_nodes(pd, pts, h=H, n_paths=12000)
    _check(st, radial / (np.sinh(k) / k))


@pytest.mark.parametrize("kind,domain", [("saddle", "box"), ("xy", "box"), ("saddle", "ball")])
def test_harmonic_data(orc, kind, domain):
    pd = W.harmonic_problem(kind, domain=domain, seed=8)
    pts = np.array([[0.5, 0.5], [0.2, 0.7], [0.9, 0.15]]) if domain == "box" else \
        np.array([[0.0, 0.0], [0.4, -0.3], [-0.6, 0.5]])
    st = orc.solve_nodes(pd, pts, h=H, n_paths=12000)
    _check(st, W.manufactured_u(pd, pts))


def _torsion(x, y, a, b, M=401):
    """E[tau] in [0,a]x[0,b] for (1/2) Lap: sum over odd m, n of
    32 sin(m pi x/a) sin(n pi y/b) / (pi^4 m n (m^2/a^2 + n^2/b^2))."""
    m = np.arange(1, M, 2)[:, None]
    n = np.arange(1, M, 2)[None, :]
    return float(np.sum(32 * np.sin(m * np.pi * x / a) * np.sin(n * np.pi * y / b)
                        / (np.pi ** 4 * m * n * (m ** 2 / a ** 2 + n ** 2 / b ** 2))))


def test_rectangle_exit_time(orc):
    pd = W.box_exit_time_problem(hi=(1.0, 2.0), seed=9)
    pts = np.array([[0.5, 1.0], [0.2, 0.3], [0.8, 1.7]])
    exact = np.array([_torsion(x, y, 1.0, 2.0) for x, y in pts])
    for mode in ("bridge", "shift"):
        st = orc.solve_nodes(pd, pts, h=H, n_paths=12000, exit=mode)
        _check(st, exact)
