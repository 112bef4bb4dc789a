"""Seeded synthetic inputs: problem descriptions, interface nodes and grids.

Both the GPU library's binding and the CPU oracle's wrapper take these plain
dicts and arrays and convert them into their own structures. Nothing here runs
the Monte Carlo method; the module only states problems (coefficients, the
manufactured solution U from which f and g follow, the domain) and where the
interfacial nodes sit.

Problem dict fields::

    dim            2 or 3
    domain         "box" (lo, hi) or "ball" (center, radius)
    sigma          isotropic diffusion, a_ij = sigma^2 delta_ij
    b0, B          drift b(x) = b0 + B x
    c_a, c_b       killing rate c(x) = c_a + c_b |x|^2
    trig           [{amp, k[dim], phase[dim]}]  amp * prod sin(k_d x_d + phase_d)
    mono           [{coef, e[dim]}]             coef * prod x_d^e_d
    fx, gx         monomials added to f and to g
    seed           64-bit key of the path generator

For (1/2) sigma^2 Lap u + b.grad u + c u = f (the paper's eq. F:EllipticBVP
with A = sigma^2 I), the source is f = (1/2) sigma^2 Lap U + b.grad U + c U +
sum(fx) and the Dirichlet data is g = U + sum(gx); when fx = gx = 0 the exact
solution is U.
"""
from __future__ import annotations

import math

import numpy as np

PI = math.pi


# --------------------------------------------------------------------------- problems
def operator_problem(lo, hi, seed=0):
    """The unit-square workload operator on the box [lo, hi]^2:
    b = (0.5 x, -0.3 y), c = -(1 + x^2 + y^2), sigma = 1 (generator 1/2 Lap),
    manufactured solution u = sin(pi x) cos(pi y) + x^2 y."""
    return {
        "dim": 2, "domain": "box", "lo": [float(lo)] * 2, "hi": [float(hi)] * 2,
        "sigma": 1.0, "b0": [0.0, 0.0], "B": [[0.5, 0.0], [0.0, -0.3]],
        "c_a": -1.0, "c_b": -1.0,
        "trig": [{"amp": 1.0, "k": [PI, PI], "phase": [0.0, PI / 2]}],
        "mono": [{"coef": 1.0, "e": [2, 1]}],
        "fx": [], "gx": [], "seed": int(seed),
    }


def unit_square_problem(seed=0):
    """Plain first-stage workload: unit square, 18 interface nodes."""
    return operator_problem(0.0, 1.0, seed)


def unit_square_nodes():
    """4 subdomains cut by the interfaces x = 1/4, 1/2, 3/4, six equispaced
    nodes each at y = j/7, j = 1..6 (end points on the boundary excluded),
    interface-major. 18 x 2 array."""
    pts = [(xi, j / 7.0) for xi in (0.25, 0.5, 0.75) for j in range(1, 7)]
    return np.array(pts, dtype=np.float64)


def big_square_problem(seed=0):
    """Throughput workload: the same operator on [0, 4]^2."""
    return operator_problem(0.0, 4.0, seed)


def big_square_nodes(side=4.0, cells=8, per_segment=16):
    """[0, side]^2 cut into cells x cells subdomains. Every interior grid line
    is split into `cells` segments by the crossing lines; each segment carries
    `per_segment` equispaced nodes at offsets (len * j / (per_segment + 1)),
    j = 1..per_segment (crossing points excluded). Vertical segments first
    (line by line, bottom to top), then horizontal ones. For the defaults,
    7 * 8 * 2 = 112 segments, 1,792 nodes."""
    step = side / cells
    pts = []
    for a in range(1, cells):
        x = a * step
        for s in range(cells):
            for j in range(1, per_segment + 1):
                pts.append((x, s * step + step * j / (per_segment + 1)))
    for a in range(1, cells):
        y = a * step
        for s in range(cells):
            for j in range(1, per_segment + 1):
                pts.append((s * step + step * j / (per_segment + 1), y))
    return np.array(pts, dtype=np.float64)


def ball_exit_time_problem(dim=2, radius=1.0, center=None, sigma=1.0, seed=0):
    """E[tau] from x for (1/2) sigma^2 Lap: u = (R^2 - |x - c|^2) / (dim sigma^2),
    b = c = 0, so f = -1, g = 0 on the sphere. Centered at the origin unless
    center is given (then U is written about the origin through monomials)."""
    cen = [0.0] * dim if center is None else [float(v) for v in center]
    s2 = sigma * sigma
    mono = [{"coef": (radius * radius - sum(v * v for v in cen)) / (dim * s2), "e": [0] * dim}]
    for d in range(dim):
        e2 = [0] * dim
        e2[d] = 2
        mono.append({"coef": -1.0 / (dim * s2), "e": e2})
        if cen[d] != 0.0:
            e1 = [0] * dim
            e1[d] = 1
            mono.append({"coef": 2.0 * cen[d] / (dim * s2), "e": e1})
    return {"dim": dim, "domain": "ball", "center": cen, "radius": float(radius),
            "sigma": float(sigma), "b0": [0.0] * dim, "B": [[0.0] * dim for _ in range(dim)],
            "c_a": 0.0, "c_b": 0.0, "trig": [], "mono": mono, "fx": [], "gx": [],
            "seed": int(seed)}


def ball_killing_problem(dim=2, radius=1.0, c=-1.0, sigma=1.0, seed=0):
    """u(x) = E[exp(c tau)] in a ball: f = 0, g = 1, constant c < 0. With
    kappa = sqrt(2|c|)/sigma: 2D u = I0(kappa r)/I0(kappa R); 3D
    u = [sinh(kappa r)/(kappa r)] / [sinh(kappa R)/(kappa R)]."""
    return {"dim": dim, "domain": "ball", "center": [0.0] * dim, "radius": float(radius),
            "sigma": float(sigma), "b0": [0.0] * dim, "B": [[0.0] * dim for _ in range(dim)],
            "c_a": float(c), "c_b": 0.0, "trig": [], "mono": [], "fx": [],
            "gx": [{"coef": 1.0, "e": [0] * dim}], "seed": int(seed)}


def box_exit_time_problem(lo=(0.0, 0.0), hi=(1.0, 1.0), sigma=1.0, seed=0):
    """E[tau] in a box: U = 0, f = -1 (fx), g = 0, b = c = 0."""
    dim = len(lo)
    return {"dim": dim, "domain": "box", "lo": [float(v) for v in lo],
            "hi": [float(v) for v in hi], "sigma": float(sigma), "b0": [0.0] * dim,
            "B": [[0.0] * dim for _ in range(dim)], "c_a": 0.0, "c_b": 0.0,
            "trig": [], "mono": [], "fx": [{"coef": -1.0, "e": [0] * dim}], "gx": [],
            "seed": int(seed)}


def harmonic_problem(kind="saddle", domain="box", seed=0):
    """b = c = f = 0 and harmonic g, so u = g: 'saddle' x^2 - y^2, 'xy' x y,
    'linear' x."""
    mono = {"saddle": [{"coef": 1.0, "e": [2, 0]}, {"coef": -1.0, "e": [0, 2]}],
            "xy": [{"coef": 1.0, "e": [1, 1]}],
            "linear": [{"coef": 1.0, "e": [1, 0]}]}[kind]
    pd = {"dim": 2, "domain": domain, "sigma": 1.0, "b0": [0.0, 0.0],
          "B": [[0.0, 0.0], [0.0, 0.0]], "c_a": 0.0, "c_b": 0.0, "trig": [], "mono": mono,
          "fx": [], "gx": [], "seed": int(seed)}
    if domain == "box":
        pd.update(lo=[0.0, 0.0], hi=[1.0, 1.0])
    else:
        pd.update(center=[0.0, 0.0], radius=1.0)
    return pd


def bilinear_problem(coef=(0.3, 1.0, -0.5, 2.0), lo=0.0, hi=1.0, seed=0):
    """u = a + b x + c y + d x y with the unit-square drift and killing.
    Lap u = 0, so f = b.grad u + c u. A grid reproduces u exactly under
    bilinear interpolation, which makes u a zero-variance control variate."""
    a, bx, cy, dxy = coef
    pd = operator_problem(lo, hi, seed)
    pd["trig"] = []
    pd["mono"] = [{"coef": a, "e": [0, 0]}, {"coef": bx, "e": [1, 0]},
                  {"coef": cy, "e": [0, 1]}, {"coef": dxy, "e": [1, 1]}]
    return pd


# --------------------------------------------------------------------------- exact values
def manufactured_u(pd: dict, pts) -> np.ndarray:
    """U at the points (the exact solution when fx = gx = 0)."""
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    dim = pd["dim"]
    out = np.zeros(len(pts))
    for t in pd.get("trig", []):
        v = np.full(len(pts), float(t["amp"]))
        for d in range(dim):
            v = v * np.sin(t["k"][d] * pts[:, d] + t["phase"][d])
        out += v
    for m in pd.get("mono", []):
        v = np.full(len(pts), float(m["coef"]))
        for d in range(dim):
            v = v * pts[:, d] ** int(m["e"][d])
        out += v
    return out


def manufactured_derivs(pd: dict, pts):
    """U, grad U (n x dim) and Lap U at the points, term by term from the
    trig and monomial terms of U."""
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    dim = pd["dim"]
    u = np.zeros(len(pts))
    grad = np.zeros((len(pts), dim))
    lap = np.zeros(len(pts))
    for t in pd.get("trig", []):
        s = np.stack([np.sin(t["k"][d] * pts[:, d] + t["phase"][d]) for d in range(dim)], axis=1)
        c = np.stack([np.cos(t["k"][d] * pts[:, d] + t["phase"][d]) for d in range(dim)], axis=1)
        v = float(t["amp"]) * np.prod(s, axis=1)
        u += v
        lap -= sum(t["k"][d] ** 2 for d in range(dim)) * v
        for d in range(dim):
            grad[:, d] += float(t["amp"]) * t["k"][d] * c[:, d] * np.prod(np.delete(s, d, axis=1), axis=1)
    for m in pd.get("mono", []):
        e = [int(m["e"][d]) for d in range(dim)]
        pw = lambda d, k: pts[:, d] ** k if k >= 0 else np.zeros(len(pts))  # noqa: E731
        u += float(m["coef"]) * np.prod([pw(d, e[d]) for d in range(dim)], axis=0)
        for d in range(dim):
            rest = np.prod([pw(q, e[q]) for q in range(dim) if q != d], axis=0)
            grad[:, d] += float(m["coef"]) * e[d] * pw(d, e[d] - 1) * rest
            lap += float(m["coef"]) * e[d] * (e[d] - 1) * pw(d, e[d] - 2) * rest
    return u, grad, lap


def bounding_box(pd: dict):
    """lo, hi of the domain's bounding box."""
    D = pd["dim"]
    if pd.get("domain", "box") == "box":
        return [float(v) for v in pd["lo"][:D]], [float(v) for v in pd["hi"][:D]]
    c, r = pd["center"], float(pd["radius"])
    return [float(c[d]) - r for d in range(D)], [float(c[d]) + r for d in range(D)]


def tabulated_problem(pd: dict, n=65, fields=("b", "c", "f"), seed=0, amp=0.3, dtype=np.float64):
    """pd with tabulated coefficients ("tab") on n^dim grids over the domain's
    bounding box. Tabulated b and c are the analytic ones plus smooth
    non-affine terms (amp = 0: exactly the analytic ones):
      b_d += amp sin(2 pi k_d.x + ph_d),  c -= amp (1 + cos(2 pi k_c.x + ph_c)) / 2,
    with random integer wave vectors k in 1..2; a tabulated f is
    (1/2) sigma^2 Lap U + b.grad U + c U + sum(fx) for the b and c the walk
    uses, so U stays the exact solution up to the interpolation error (with f
    analytic, only amp = 0 keeps that)."""
    D = pd["dim"]
    lo, hi = bounding_box(pd)
    shape = (int(n),) * D
    pts = grid_points(shape, lo, hi)
    rng = np.random.default_rng(seed)
    b = np.asarray(pd.get("b0", [0.0] * 3), dtype=np.float64)[None, :D] + pts @ np.asarray(
        pd.get("B", np.zeros((3, 3))), dtype=np.float64)[:D, :D].T
    c = pd.get("c_a", 0.0) + pd.get("c_b", 0.0) * np.sum(pts ** 2, axis=1)
    if "b" in fields:
        for d in range(D):
            k = rng.integers(1, 3, size=D)
            b[:, d] += amp * np.sin(2 * PI * pts @ k + rng.uniform(0, 2 * PI))
    if "c" in fields:
        k = rng.integers(1, 3, size=D)
        c = c - amp * 0.5 * (1.0 + np.cos(2 * PI * pts @ k + rng.uniform(0, 2 * PI)))
    mk = lambda v: {"dim": D, "n": list(shape), "lo": list(lo), "hi": list(hi),  # noqa: E731
                    "data": np.asarray(v).astype(dtype).reshape(shape[::-1])}
    tab = {}
    if "b" in fields:
        tab["b"] = [mk(b[:, d]) for d in range(D)]
    if "c" in fields:
        tab["c"] = mk(c)
    if "f" in fields:
        u, grad, lap = manufactured_derivs(pd, pts)
        f = 0.5 * pd["sigma"] ** 2 * lap + np.sum(b * grad, axis=1) + c * u
        for m in pd.get("fx", []):
            f += m["coef"] * np.prod([pts[:, d] ** m["e"][d] for d in range(D)], axis=0)
        tab["f"] = mk(f)
    out = dict(pd)
    out["tab"] = tab
    return out


PAPER_SIDE = 2.0  # stand-in box [0, 2]^2 for the paper's example (its figure is missing)


def paper_example_u(pts) -> np.ndarray:
    """The exact solution of the paper's example (Sec. 6, eq. F:PDE_ejemplo):
    2 cos(2 (y - 2) x) + sin(3 (x - 2) y) + 3.1."""
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    x, y = pts[:, 0], pts[:, 1]
    return 2.0 * np.cos(2.0 * (y - 2.0) * x) + np.sin(3.0 * (x - 2.0) * y) + 3.1


def paper_example_fields(pts):
    """b (n x 2), c, f and u of the paper's example at the points. With
    sigma = sqrt(2) (so (1/2) sigma^2 Lap = Lap), b = cos(x + y) [1, 1] /
    (1.1 + sin(x + y)), c = -(x^2 + y^2) / (1.1 + sin(x + y)); the source in
    this library's convention (1/2 sigma^2 Lap u + b.grad u + c u = f) is
    f = Lap u + b.grad u + c u with u's derivatives written out (the paper's
    f is the negative of this)."""
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    x, y = pts[:, 0], pts[:, 1]
    den = 1.1 + np.sin(x + y)
    b = np.stack([np.cos(x + y) / den] * 2, axis=1)
    c = -(x * x + y * y) / den
    A, B = 2.0 * (y - 2.0) * x, 3.0 * (x - 2.0) * y
    Ax, Ay, Bx, By = 2.0 * (y - 2.0), 2.0 * x, 3.0 * y, 3.0 * (x - 2.0)
    u = 2.0 * np.cos(A) + np.sin(B) + 3.1
    ux = -2.0 * np.sin(A) * Ax + np.cos(B) * Bx
    uy = -2.0 * np.sin(A) * Ay + np.cos(B) * By
    lap = -2.0 * np.cos(A) * (Ax * Ax + Ay * Ay) - np.sin(B) * (Bx * Bx + By * By)
    f = lap + b[:, 0] * ux + b[:, 1] * uy + c * u
    return b, c, f, u


def paper_example_problem(n=257, dtype=np.float64, seed=0):
    """The paper's example PDE on the stand-in box [0, 2]^2: every
    coefficient, the source and the boundary data tabulated on n x n grids
    (the descriptor's analytic parts are zero)."""
    lo, hi = [0.0, 0.0], [PAPER_SIDE, PAPER_SIDE]
    pts = grid_points((n, n), lo, hi)
    b, c, f, u = paper_example_fields(pts)
    mk = lambda v: {"dim": 2, "n": [n, n], "lo": list(lo), "hi": list(hi),  # noqa: E731
                    "data": np.asarray(v).astype(dtype).reshape(n, n)}
    return {"dim": 2, "domain": "box", "lo": lo, "hi": hi, "sigma": float(np.sqrt(2.0)),
            "b0": [0.0, 0.0], "B": [[0.0, 0.0], [0.0, 0.0]], "c_a": 0.0, "c_b": 0.0, "seed": int(seed),
            "tab": {"b": [mk(b[:, 0]), mk(b[:, 1])], "c": mk(c), "f": mk(f), "g": mk(u)}}


def paper_example_gradient_grids(n=257, dtype=np.float64):
    """grad u of the paper's example on n x n grids over [0, 2]^2 (the
    gradient grids of an Ito control variate with u~ = u)."""
    lo, hi = [0.0, 0.0], [PAPER_SIDE, PAPER_SIDE]
    pts = grid_points((n, n), lo, hi)
    x, y = pts[:, 0], pts[:, 1]
    A, B = 2.0 * (y - 2.0) * x, 3.0 * (x - 2.0) * y
    ux = -2.0 * np.sin(A) * 2.0 * (y - 2.0) + np.cos(B) * 3.0 * y
    uy = -2.0 * np.sin(A) * 2.0 * x + np.cos(B) * 3.0 * (x - 2.0)
    return [{"dim": 2, "n": [n, n], "lo": lo, "hi": hi, "data": v.astype(dtype).reshape(n, n)} for v in (ux, uy)]


def paper_example_nodes():
    """18 nodes laid out like the unit-square ones, scaled to [0, 2]^2: three
    vertical interfaces x = 0.5, 1, 1.5, six nodes each at y = 2 j / 7."""
    return unit_square_nodes() * PAPER_SIDE


# --------------------------------------------------------------------------- partitions
def unit_square_partition(n=257):
    """The unit square's 4 strips: interfaces x = 1/4, 1/2, 3/4 on an n x n
    grid (n - 1 divisible by 4), multiquadric shape parameter 3 (about 0.4 /
    node spacing 1/7)."""
    return {"n": (n, n), "cuts": [[0.25, 0.5, 0.75], []], "rbf_eps": 3.0}


def big_square_partition(n=257, side=4.0, cells=8, per_segment=16):
    """The [0, side]^2 box cut into cells x cells subdomains: interfaces at
    the multiples of side / cells on both axes, on an n x n grid; the shape
    parameter is the inverse node spacing along a line (side / cells /
    (per_segment + 1))."""
    step = side / cells
    cuts = [a * step for a in range(1, cells)]
    return {"n": (n, n), "cuts": [cuts, cuts], "rbf_eps": (per_segment + 1) / step}


# --------------------------------------------------------------------------- grids
def grid_points(n, lo, hi):
    """Coordinates of an n[0] x n[1] (x n[2]) uniform grid, x fastest, shape
    (prod(n), len(n))."""
    axes = [np.linspace(lo[d], hi[d], n[d]) for d in range(len(n))]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")  # slowest axis first
    return np.stack([m.ravel() for m in mesh[::-1]], axis=1)


def fourier_perturbation(seed=1, n_modes=32, amp=1e-2, kmax=16, dim=2):
    """p(x) = sum_m A_m prod_d sin(pi k_{m,d} xhat_d), xhat = (x - lo)/(hi - lo):
    k_{m,d} uniform on 1..kmax, random sign, A_m = amp * sign * dim / |k_m|^2
    (so the lowest mode has amplitude amp and the modes decay as k^-2).
    p vanishes on the boundary of the box."""
    rng = np.random.default_rng(seed)
    ks = rng.integers(1, kmax + 1, size=(n_modes, dim))
    sg = rng.choice([-1.0, 1.0], size=n_modes)
    A = amp * sg * dim / np.sum(ks.astype(np.float64) ** 2, axis=1)
    return {"k": ks, "A": A}


def _pert_eval(pert, pts, lo, hi):
    """p, grad p and Lap p at the points (box [lo, hi]^dim)."""
    dim = pts.shape[1]
    L = np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64)
    xh = (pts - np.asarray(lo)) / L
    val = np.zeros(len(pts))
    grad = np.zeros_like(pts)
    lap = np.zeros(len(pts))
    for m in range(len(pert["A"])):
        w = PI * pert["k"][m] / L           # angular wavenumber per coordinate
        s = np.sin(PI * pert["k"][m] * xh)
        c = np.cos(PI * pert["k"][m] * xh)
        term = pert["A"][m] * np.prod(s, axis=1)
        val += term
        lap += -np.sum(w ** 2) * term
        for d in range(dim):
            others = np.prod(np.delete(s, d, axis=1), axis=1)
            grad[:, d] += pert["A"][m] * w[d] * c[:, d] * others
    return val, grad, lap


def _pert_grid(pert, shape, lo, hi):
    """p, grad p and Lap p on the uniform grid of `shape` (x fastest), flat
    like grid_points; the modes are products of 1D sines, so each factor is
    evaluated per axis and the products are formed by einsum."""
    D = len(shape)
    L = np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64)
    k = np.asarray(pert["k"], dtype=np.float64)  # (modes, D)
    A = np.asarray(pert["A"], dtype=np.float64)
    xs = [np.linspace(0.0, 1.0, shape[d]) for d in range(D)]
    S = [np.sin(PI * k[:, d][:, None] * xs[d][None, :]) for d in range(D)]   # (modes, n_d)
    Cd = [PI * k[:, d][:, None] / L[d] * np.cos(PI * k[:, d][:, None] * xs[d][None, :]) for d in range(D)]
    w2 = np.sum((PI * k / L[None, :]) ** 2, axis=1)
    axes = "xyz"[:D]
    spec = ",".join("m" + a for a in axes)
    out = "".join(reversed(axes))  # slowest axis first
    val = np.einsum("m," + spec + "->" + out, A, *S).ravel()
    lap = np.einsum("m," + spec + "->" + out, -A * w2, *S).ravel()
    grad = np.stack([np.einsum("m," + spec + "->" + out, A, *[Cd[e] if e == d else S[e] for e in range(D)]).ravel()
                     for d in range(D)], axis=1)
    return val, grad, lap


def correction_grids(pd: dict, n=257, seed=1, dtype=np.float32, n_modes=32, amp=1e-2):
    """u_prev = U + p on an n x n grid over the box (n: points per axis, or one
    count per axis), and the residual r = f - (L + c) u_prev =
    -(1/2 sigma^2 Lap p + b.grad p + c p), both evaluated exactly at the grid
    points in float64 and stored in `dtype`. Returns (u_prev_grid,
    resid_grid, perturbation)."""
    lo, hi = pd["lo"], pd["hi"]
    D = pd["dim"]
    shape = tuple(int(v) for v in np.broadcast_to(np.asarray(n), (D,)))
    pts = grid_points(shape, lo, hi)
    pert = fourier_perturbation(seed, n_modes=n_modes, amp=amp, dim=D)
    p, gp, lp = _pert_grid(pert, shape, lo, hi)
    b = np.asarray(pd["b0"])[None, :] + pts @ np.asarray(pd["B"]).T
    c = pd["c_a"] + pd["c_b"] * np.sum(pts ** 2, axis=1)
    s2 = pd["sigma"] ** 2
    resid = -(0.5 * s2 * lp + np.sum(b * gp, axis=1) + c * p)
    u_prev = manufactured_u(pd, pts) + p
    mk = lambda v: {"dim": D, "n": list(shape), "lo": list(lo), "hi": list(hi),  # noqa: E731
                    "data": v.astype(dtype).reshape(shape[::-1])}
    return mk(u_prev), mk(resid), pert


def gradient_grids(pd: dict, n=257, seed=1, dtype=np.float32, n_modes=32, amp=1e-2):
    """The components of grad(U + p) on an n^dim grid over the domain's
    bounding box (n: points per axis, or one count per axis), evaluated
    exactly at the grid points in float64 and stored in `dtype`: a list of dim
    grids. p is the perturbation of correction_grids with the same seed,
    n_modes and amp (amp = 0: grad U, the exact gradient when fx = gx = 0), so
    both estimators can use the same u~."""
    lo, hi = bounding_box(pd)
    D = pd["dim"]
    shape = tuple(int(v) for v in np.broadcast_to(np.asarray(n), (D,)))
    pts = grid_points(shape, lo, hi)
    _, grad, _ = manufactured_derivs(pd, pts)
    if amp:
        pert = fourier_perturbation(seed, n_modes=n_modes, amp=amp, dim=D)
        grad = grad + _pert_grid(pert, shape, lo, hi)[1]
    return [{"dim": D, "n": list(shape), "lo": list(lo), "hi": list(hi),
             "data": grad[:, d].astype(dtype).reshape(shape[::-1])} for d in range(D)]


def sampled_grid(pd: dict, fn, n=257, dtype=np.float64):
    """fn sampled on an n x n grid over the box of pd."""
    lo, hi = pd["lo"], pd["hi"]
    pts = grid_points((n, n), lo, hi)
    return {"dim": 2, "n": [n, n], "lo": list(lo), "hi": list(hi),
            "data": np.asarray(fn(pts), dtype=dtype).reshape(n, n)}


# --------------------------------------------------------------------------- batches
def random_problem(rng, dim=None):
    """One random problem of the batched workload: the box [0, L]^D with
    L ~ U[0.5, 4]; drift b_d = beta_d x_d, beta ~ U[-1, 1]; killing
    c = c0 (1 + |x|^2), c0 ~ U[-3, -0.1]; manufactured U = sum of 8 separable
    terms A prod_d sin(k_d x_d + phase_d), A ~ U[-1, 1], k ~ (pi/L) U[0.5, 3],
    phase ~ U[0, 2 pi); sigma = 1."""
    D = int(dim if dim is not None else rng.choice([2, 3]))
    L = float(rng.uniform(0.5, 4.0))
    beta = rng.uniform(-1.0, 1.0, size=D)
    c0 = float(rng.uniform(-3.0, -0.1))
    trig = []
    for _ in range(8):
        trig.append({"amp": float(rng.uniform(-1, 1)),
                     "k": [float(v) for v in (PI / L) * rng.uniform(0.5, 3.0, size=D)],
                     "phase": [float(v) for v in rng.uniform(0, 2 * PI, size=D)]})
    return {"dim": D, "domain": "box", "lo": [0.0] * D, "hi": [L] * D, "sigma": 1.0,
            "b0": [0.0] * D, "B": [[float(beta[i]) if i == j else 0.0 for j in range(D)] for i in range(D)],
            "c_a": c0, "c_b": c0, "trig": trig, "mono": [], "fx": [], "gx": [],
            "seed": int(rng.integers(0, 2**63))}


def face_nodes(rng, pd, n):
    """n nodes uniform on the internal faces of an m^D partition of the box,
    m = max(2, round(L / 0.5)): pick one of the D (m - 1) interior hyperplanes
    x_d = L a / m, then a uniform point of the box on it (strictly inside)."""
    D = pd["dim"]
    L = pd["hi"][0] - pd["lo"][0]
    m = max(2, int(round(L / 0.5)))
    pts = rng.uniform(0.0, 1.0, size=(n, D))
    # keep strictly inside: the open unit interval, mapped to the box
    pts = np.clip(pts, 1e-9, 1 - 1e-9) * L + pd["lo"][0]
    d = rng.integers(0, D, size=n)
    a = rng.integers(1, m, size=n)
    pts[np.arange(n), d] = pd["lo"][0] + L * a / m
    return pts


def batch_workload(seed=4, n_problems=64, node_range=(10, 5000), path_range=(1e3, 1e6),
                   dts=(1e-3, 1e-4), scale=1.0):
    """The batched uneven workload: n_problems random problems (random_problem)
    with log-uniform node counts and paths per node, h drawn from dts.
    `scale` multiplies the path counts (for smaller test versions).
    Returns a list of dicts {problem, nodes, n_paths, dt}."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_problems):
        pd = random_problem(rng)
        n = int(round(np.exp(rng.uniform(np.log(node_range[0]), np.log(node_range[1])))))
        npath = int(round(np.exp(rng.uniform(np.log(path_range[0]), np.log(path_range[1]))) * scale))
        out.append({"problem": pd, "nodes": face_nodes(rng, pd, n), "n_paths": max(npath, 1),
                    "dt": float(rng.choice(dts))})
    return out


# --------------------------------------------------------------------------- serving
# time step by tolerance for plain requests (the bias of the bridge scheme is
# first order; these keep it below tol / sqrt(2) on the unit-square problem)
PLAIN_DT = {1e-2: 1e-3, 3e-3: 5e-4, 1e-3: 2.5e-4}
CV_DT = 1e-3


def serving_stream(seed=5, rate=200.0, duration=5.0, n_problems=16, node_range=(1, 2000),
                   tols=(1e-2, 3e-3, 1e-3), cv_frac=0.3, grid_sizes_2d=(129, 257, 513), grid_3d=65):
    """Seeded Poisson stream of node-solve requests: problems from the batched
    generator (random_problem), node counts log-uniform in node_range on the
    internal faces, tolerance uniform on `tols` (RMS target; per-node SE =
    tol / sqrt(2)), a fraction cv_frac carrying a u_prev grid (2D: n uniform
    on grid_sizes_2d, 3D: grid_3d^3) built like correction_grids.
    Returns (problems, requests); a request is a dict with arrival time `t`,
    problem index, nodes, tol, target_se, dt, cv, grid_n and stream_id."""
    rng = np.random.default_rng(seed)
    problems = [random_problem(rng) for _ in range(n_problems)]
    reqs = []
    t = 0.0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > duration:
            break
        q = int(rng.integers(n_problems))
        pd = problems[q]
        n = int(round(np.exp(rng.uniform(np.log(node_range[0]), np.log(node_range[1])))))
        nodes = face_nodes(rng, pd, max(n, 1))
        tol = float(tols[int(rng.integers(len(tols)))])
        cv = bool(rng.random() < cv_frac)
        gn = (int(grid_sizes_2d[int(rng.integers(len(grid_sizes_2d)))]) if pd["dim"] == 2 else grid_3d) \
            if cv else None
        reqs.append({"t": t, "problem": q, "nodes": nodes, "tol": tol,
                     "target_se": tol / np.sqrt(2.0), "dt": CV_DT if cv else PLAIN_DT[tol],
                     "cv": cv, "grid_n": gn, "stream_id": len(reqs)})
    return problems, reqs
