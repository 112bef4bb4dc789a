"""Plain reference of the gradient of a gridded function (the grad(u~) grids
that the pathwise control variate of eq. F:xiControlVariate needs when only
values of u~ on a grid are known, as inside the outer iteration).

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this module; it shares no code with
the GPU library.

Second-order finite differences on a uniform grid (spacing dx_d = (hi_d -
lo_d) / (n_d - 1)): the central difference (u[i+1] - u[i-1]) / (2 dx) at
interior points and the three-point one-sided differences
(-3 u[0] + 4 u[1] - u[2]) / (2 dx) and (3 u[n-1] - 4 u[n-2] + u[n-3]) / (2 dx)
at the two ends of each axis (n_d >= 3). Arrays are indexed [z][y][x]
(x fastest), like the grids.
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
