"""Plain references of the gradient of a gridded function (the grad(u~) grids
that the pathwise control variate of eq. F:xiControlVariate needs when only
values of u~ on a grid are known, as inside the outer iteration), and of the
residual r = f - (L + c) u~ that the correction estimator needs then.

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this module; it shares no code with
the GPU library.

Second-order finite differences on a uniform grid (spacing dx_d = (hi_d -
lo_d) / (n_d - 1)): the central difference (u[i+1] - u[i-1]) / (2 dx) at
interior points and the three-point one-sided differences
(-3 u[0] + 4 u[1] - u[2]) / (2 dx) and (3 u[n-1] - 4 u[n-2] + u[n-3]) / (2 dx)
at the two ends of each axis (n_d >= 3). Second derivatives: the central
(u[i+1] - 2 u[i] + u[i-1]) / dx^2 inside and the four-point one-sided
(2 u[0] - 5 u[1] + 4 u[2] - u[3]) / dx^2 (mirrored at the far end; n_d >= 4),
also second order. Arrays are indexed [z][y][x] (x fastest), like the grids.
"""
from __future__ import annotations

import numpy as np


def _axis_derivative(u, axis, dx):
    u = np.moveaxis(u, axis, -1)
    out = np.empty_like(u)
    out[..., 1:-1] = (u[..., 2:] - u[..., :-2]) / (2.0 * dx)
    out[..., 0] = (-3.0 * u[..., 0] + 4.0 * u[..., 1] - u[..., 2]) / (2.0 * dx)
    out[..., -1] = (3.0 * u[..., -1] - 4.0 * u[..., -2] + u[..., -3]) / (2.0 * dx)
    return np.moveaxis(out, -1, axis)


def gradient(grid: dict) -> list:
    """The dim gradient grids (dicts like the input, float64) of a grid dict."""
    D = int(grid["dim"])
    n = [int(v) for v in grid["n"][:D]]
    if min(n) < 3:
        raise ValueError("second-order differences need n >= 3 per axis")
    u = np.asarray(grid["data"], dtype=np.float64).reshape(n[::-1])
    out = []
    for d in range(D):
        dx = (float(grid["hi"][d]) - float(grid["lo"][d])) / (n[d] - 1)
        # array axis of coordinate d: x is the last axis
        g = _axis_derivative(u, D - 1 - d, dx)
        out.append({"dim": D, "n": list(grid["n"]), "lo": list(grid["lo"]), "hi": list(grid["hi"]), "data": g})
    return out


def _axis_second_derivative(u, axis, dx):
    u = np.moveaxis(u, axis, -1)
    out = np.empty_like(u)
    out[..., 1:-1] = (u[..., 2:] - 2.0 * u[..., 1:-1] + u[..., :-2]) / (dx * dx)
    out[..., 0] = (2.0 * u[..., 0] - 5.0 * u[..., 1] + 4.0 * u[..., 2] - u[..., 3]) / (dx * dx)
    out[..., -1] = (2.0 * u[..., -1] - 5.0 * u[..., -2] + 4.0 * u[..., -3] - u[..., -4]) / (dx * dx)
    return np.moveaxis(out, -1, axis)


def residual(problem: dict, grid: dict) -> np.ndarray:
    """r = f - ((1/2) sigma^2 Lap u + b.grad u + c u) at the grid's points
    (eq. F:EllipticBVP written for u~), with b, c, f those of the problem
    (the oracle's own evaluation) and the derivatives of u~ by the second-order
    differences above. Returns an array shaped like the grid's data."""
    from oracle import oracle as O
    D = int(grid["dim"])
    n = [int(v) for v in grid["n"][:D]]
    if min(n) < 4:
        raise ValueError("second derivatives at the edges need n >= 4 per axis")
    u = np.asarray(grid["data"], dtype=np.float64).reshape(n[::-1])
    axes = [np.linspace(float(grid["lo"][d]), float(grid["hi"][d]), n[d]) for d in range(D)]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")
    pts = np.stack([m.ravel() for m in mesh[::-1]], axis=1)
    b = O.drift(problem, pts)
    c = O.kill(problem, pts).reshape(u.shape)
    f = O.source(problem, pts).reshape(u.shape)
    lap = np.zeros_like(u)
    adv = np.zeros_like(u)
    for d in range(D):
        dx = (float(grid["hi"][d]) - float(grid["lo"][d])) / (n[d] - 1)
        lap += _axis_second_derivative(u, D - 1 - d, dx)
        adv += b[:, d].reshape(u.shape) * _axis_derivative(u, D - 1 - d, dx)
    s2 = float(problem.get("sigma", 1.0)) ** 2
    return f - (0.5 * s2 * lap + adv + c * u)
