"""Plain reference of the second stage of probabilistic domain decomposition
on a box cut by axis-parallel interfaces (2D): the interfacial interpolation
of the nodal values and the subdomain solves that give the global
approximation u~ = (+)_k v_k (Sec. 1; Alg. A:IterPDD, the subdomain-BVP step:
L v_k + c v_k = f in Omega_k, v_k = g on the physical boundary, v_k = R[nodal
values] on the interfaces), and the scheduling of the outer iteration
(Alg. A:Scheduling).

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this module; it shares no code with
the GPU library.

Interpolator R (Def. D:Linear_interpolator; multiquadric radial basis
functions, as in the paper's experiment, Sec. 6): along an interface line the
data are the nodal values of the nodes on that line and the boundary data g
at the line's two ends on the physical boundary; with t the coordinate along
the line, s(t) = sum_m lambda_m sqrt(1 + (eps (t - t_m))^2), the lambda from
the linear system s(t_m) = z_m. A grid point where two interface lines cross
takes the mean of the two lines' values.

Subdomain solver (the paper uses FEM and only asks that its error be
negligible): the global grid of n_0 x n_1 points over the box carries u~;
every subdomain is the grid box between consecutive interfaces, and its
interior values solve the second-order finite-difference form of
(1/2) sigma^2 Lap v + b.grad v + c v = f, namely at point (i, j)
  (1/2) sigma^2 [(v[i+1,j] - 2 v[i,j] + v[i-1,j]) / dx0^2 + (v[i,j+1] - 2 v[i,j] + v[i,j-1]) / dx1^2]
  + b0 (v[i+1,j] - v[i-1,j]) / (2 dx0) + b1 (v[i,j+1] - v[i,j-1]) / (2 dx1) + c v[i,j] = f(x_i, y_j),
with b, c, f from the oracle's own coefficient functions and the values on
the subdomain's boundary taken from the grid; solved directly (sparse LU).
Arrays are indexed [y][x] (x fastest), like the grids.
"""
from __future__ import annotations

import math

import numpy as np


# --------------------------------------------------------------------------- interpolation
def rbf_coefficients(t_nodes, values, eps):
    """Multiquadric weights lambda with s(t_m) = values_m."""
    t = np.asarray(t_nodes, dtype=np.float64)
    z = np.asarray(values, dtype=np.float64)
    phi = np.sqrt(1.0 + (eps * (t[:, None] - t[None, :])) ** 2)
    return np.linalg.solve(phi, z)


def rbf_eval(t_nodes, lam, eps, t):
    t_nodes = np.asarray(t_nodes, dtype=np.float64)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    return np.sqrt(1.0 + (eps * (t[:, None] - t_nodes[None, :])) ** 2) @ lam


def rbf_interpolate(t_nodes, values, eps, t):
    """R[values | t_nodes](t) for the multiquadric interpolant."""
    return rbf_eval(t_nodes, rbf_coefficients(t_nodes, values, eps), eps, t)


# --------------------------------------------------------------------------- geometry
def grid_axes(n, lo, hi):
    return [lo[d] + (hi[d] - lo[d]) * np.arange(n[d]) / (n[d] - 1) for d in range(2)]


def cut_index(c, lo, hi, n):
    """Grid index of an interface coordinate, which must sit on a grid line."""
    t = (c - lo) * (n - 1) / (hi - lo)
    i = int(round(t))
    if abs(t - i) > 1e-9 or not (0 < i < n - 1):
        raise ValueError(f"interface {c} is not on an interior grid line")
    return i


def fill_boundary_and_interfaces(problem, n, cuts, nodes, values, eps, tol=1e-12):
    """Grid array [n1][n0] with g on the physical boundary, the interpolated
    nodal values on the interface lines (NaN elsewhere). cuts = [xs, ys]: the
    interface coordinates on each axis."""
    from oracle import oracle as O
    lo, hi = problem["lo"], problem["hi"]
    ax = grid_axes(n, lo, hi)
    u = np.full((n[1], n[0]), np.nan)
    nodes = np.asarray(nodes, dtype=np.float64).reshape(-1, 2)
    values = np.asarray(values, dtype=np.float64)

    def bnd(pts):
        return O.boundary(problem, pts)
    # physical boundary
    for j in (0, n[1] - 1):
        u[j, :] = bnd(np.stack([ax[0], np.full(n[0], ax[1][j])], axis=1))
    for i in (0, n[0] - 1):
        u[:, i] = bnd(np.stack([np.full(n[1], ax[0][i]), ax[1]], axis=1))
    # interface lines: the line x_d = c, parametrised by the other coordinate
    line_vals = {}
    for d in range(2):
        e = 1 - d
        for c in cuts[d]:
            on = np.abs(nodes[:, d] - c) <= tol * max(1.0, abs(c))
            t_nodes = np.concatenate([[lo[e]], nodes[on, e], [hi[e]]])
            ends = np.zeros((2, 2))
            ends[:, d] = c
            ends[:, e] = [lo[e], hi[e]]
            z = np.concatenate([[bnd(ends[:1])[0]], values[on], [bnd(ends[1:])[0]]])
            line_vals[(d, c)] = rbf_interpolate(t_nodes, z, eps, ax[e])
    acc = np.zeros_like(u)
    cnt = np.zeros_like(u)
    for (d, c), v in line_vals.items():
        k = cut_index(c, lo[d], hi[d], n[d])
        if d == 0:
            acc[1:-1, k] += v[1:-1]
            cnt[1:-1, k] += 1
        else:
            acc[k, 1:-1] += v[1:-1]
            cnt[k, 1:-1] += 1
    inner = cnt > 0
    u[inner] = acc[inner] / cnt[inner]
    return u


# --------------------------------------------------------------------------- subdomain solves
def subdomain_solve(problem, n, box, u):
    """Interior values of the grid box box = (i0, i1, j0, j1) (inclusive
    boundary indices) solving the finite-difference BVP above with the values
    of u on the box's boundary; returns a copy of u with them filled in."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    from oracle import oracle as O
    lo, hi = problem["lo"], problem["hi"]
    ax = grid_axes(n, lo, hi)
    dx = [(hi[d] - lo[d]) / (n[d] - 1) for d in range(2)]
    s2 = float(problem.get("sigma", 1.0)) ** 2
    i0, i1, j0, j1 = box
    mx, my = i1 - i0 - 1, j1 - j0 - 1
    if mx < 1 or my < 1:
        return u.copy()
    ii, jj = np.meshgrid(np.arange(i0 + 1, i1), np.arange(j0 + 1, j1))  # [my][mx]
    pts = np.stack([ax[0][ii.ravel()], ax[1][jj.ravel()]], axis=1)
    b = O.drift(problem, pts)
    c = O.kill(problem, pts)
    f = O.source(problem, pts)
    cx = 0.5 * s2 / dx[0] ** 2
    cy = 0.5 * s2 / dx[1] ** 2
    aW = cx - b[:, 0] / (2 * dx[0])
    aE = cx + b[:, 0] / (2 * dx[0])
    aS = cy - b[:, 1] / (2 * dx[1])
    aN = cy + b[:, 1] / (2 * dx[1])
    aC = -2 * cx - 2 * cy + c
    N = mx * my
    idx = np.arange(N).reshape(my, mx)
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [aC]
    rhs = f.copy()
    gi, gj = ii.ravel(), jj.ravel()
    for a, di, dj in ((aW, -1, 0), (aE, 1, 0), (aS, 0, -1), (aN, 0, 1)):
        ni, nj = gi + di, gj + dj
        inside = (ni > i0) & (ni < i1) & (nj > j0) & (nj < j1)
        rows.append(idx.ravel()[inside])
        cols.append(((nj[inside] - j0 - 1) * mx + (ni[inside] - i0 - 1)))
        vals.append(a[inside])
        rhs[~inside] -= a[~inside] * u[nj[~inside], ni[~inside]]
    A = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    v = spla.spsolve(A, rhs)
    out = u.copy()
    out[j0 + 1:j1, i0 + 1:i1] = v.reshape(my, mx)
    return out


def stage2(problem, n, cuts, nodes, values, eps):
    """u~ on the n[0] x n[1] grid over the box: boundary and interface values
    (fill_boundary_and_interfaces), then every subdomain between consecutive
    interfaces solved (subdomain_solve). Returns the [n1][n0] array."""
    lo, hi = problem["lo"], problem["hi"]
    u = fill_boundary_and_interfaces(problem, n, cuts, nodes, values, eps)
    ix = [0] + sorted(cut_index(c, lo[0], hi[0], n[0]) for c in cuts[0]) + [n[0] - 1]
    iy = [0] + sorted(cut_index(c, lo[1], hi[1], n[1]) for c in cuts[1]) + [n[1] - 1]
    for a in range(len(ix) - 1):
        for b in range(len(iy) - 1):
            u = subdomain_solve(problem, n, (ix[a], ix[a + 1], iy[b], iy[b + 1]), u)
    return u


# --------------------------------------------------------------------------- scheduling
def schedule_cost(a, a_j, K, V, Vpsi, rho_psi, alpha, beta, kappa, delta):
    """The objective of Alg. A:Scheduling at a > a_j: sum over nodes of
    K_i V_i [kappa (1 - r_i^2(a) + |alpha_i r_i(a) / beta_i| a_j) + (a_j / a)^(2 + 1/delta)],
    r_i^2(a) = 1 - V_i[psi] a^2 (1 - rho_i^2[phi, psi]) / (4 V_i[phi]) (eq.
    F:Sensitivity_formula); r_i^2 is kept in [0, 1]."""
    a = float(a)
    r2 = 1.0 - np.asarray(Vpsi) * a * a * (1.0 - np.asarray(rho_psi) ** 2) / (4.0 * np.asarray(V))
    r2 = np.clip(r2, 0.0, 1.0)
    r = np.sqrt(r2)
    term = kappa * (1.0 - r2 + np.abs(np.asarray(alpha) * r / np.asarray(beta)) * a_j) + (a_j / a) ** (2.0 + 1.0 / delta)
    return float(np.sum(np.asarray(K) * np.asarray(V) * term))


def plain_cost(a, K, V, delta):
    """Cost of PlainPDD(a) (eq. F:PlainPDD_cost without the subdomain part):
    sum K_i V_i / a^(2 + 1/delta)."""
    return float(np.sum(np.asarray(K) * np.asarray(V))) / a ** (2.0 + 1.0 / delta)


def schedule(a0, K, V, Vpsi, rho_psi, alpha, beta, kappa, delta, a_max, s_min=1.5, n_grid=4000, max_levels=8):
    """Alg. A:Scheduling by brute force: each a_{j+1} minimises the objective
    over a log-spaced grid of n_grid values in (a_j, a_max]; the loop stops
    once the predicted speedup cost(PlainPDD(a_j)) / cost(IterPDD(a_j,
    a_{j+1})) falls below s_min (the paper's criterion, Sec. 6), that level
    not taken. Returns [a_0, a_1, ..., a_J]."""
    seq = [float(a0)]
    while len(seq) <= max_levels:
        a_j = seq[-1]
        if a_j >= a_max:
            break
        grid = np.exp(np.linspace(math.log(a_j), math.log(a_max), n_grid + 1)[1:])
        costs = np.array([schedule_cost(a, a_j, K, V, Vpsi, rho_psi, alpha, beta, kappa, delta) for a in grid])
        k = int(np.argmin(costs))
        speedup = plain_cost(a_j, K, V, delta) / (costs[k] / a_j ** (2.0 + 1.0 / delta))
        if speedup < s_min:
            break
        seq.append(float(grid[k]))
    return seq
