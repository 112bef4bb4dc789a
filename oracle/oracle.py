"""ctypes wrapper of the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this module. It does not import the GPU
package; problems arrive as plain dicts (see the package's ``workloads``
module for their fields) and are converted here into the oracle's own struct.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB lets a mutation check point the wrapper at a deliberately broken build.
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

EXIT_MODES = {"bridge": 0, "shift": 1, "naive": 2}
LAWS = {"gauss": 0, "rademacher": 1}
MAX_TRIG, MAX_MONO = 16, 8


class _Trig(C.Structure):
    _fields_ = [("amp", C.c_double), ("k", C.c_double * 3), ("phase", C.c_double * 3)]


class _Mono(C.Structure):
    _fields_ = [("coef", C.c_double), ("e", C.c_int32 * 3)]


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("data", C.POINTER(C.c_double))]


class Problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("domain", C.c_int32),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("center", C.c_double * 3), ("radius", C.c_double),
        ("sigma", C.c_double),
        ("b0", C.c_double * 3), ("B", (C.c_double * 3) * 3),
        ("c_a", C.c_double), ("c_b", C.c_double),
        ("n_trig", C.c_int32), ("n_mono", C.c_int32), ("n_fx", C.c_int32), ("n_gx", C.c_int32),
        ("trig", _Trig * MAX_TRIG), ("mono", _Mono * MAX_MONO),
        ("fx", _Mono * MAX_MONO), ("gx", _Mono * MAX_MONO),
        ("seed", C.c_uint64),
        ("tab_b", C.POINTER(Grid) * 3), ("tab_c", C.POINTER(Grid)), ("tab_f", C.POINTER(Grid)),
        ("tab_g", C.POINTER(Grid)),
    ]


class Opts(C.Structure):
    _fields_ = [("h", C.c_double), ("n_paths", C.c_uint64), ("path_offset", C.c_uint64),
                ("stream", C.c_uint32), ("exit_mode", C.c_int32), ("law", C.c_int32),
                ("max_steps", C.c_uint64),
                ("u_prev", C.POINTER(Grid)), ("resid", C.POINTER(Grid)),
                ("grad", C.POINTER(Grid) * 3)]


class PathRec(C.Structure):
    _fields_ = [("phi", C.c_double), ("e", C.c_double), ("steps", C.c_uint64),
                ("capped", C.c_int32), ("pad", C.c_int32), ("x_exit", C.c_double * 3)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_capped", C.c_int64), ("steps_sum", C.c_int64),
                ("mean", C.c_double), ("var", C.c_double), ("stderr", C.c_double),
                ("mean_steps", C.c_double),
                ("mean_plain", C.c_double), ("var_plain", C.c_double), ("cov", C.c_double),
                ("rho", C.c_double), ("vr", C.c_double), ("vr_opt", C.c_double),
                ("sums", C.c_double * 10)]


PATH_DTYPE = np.dtype([("phi", "<f8"), ("e", "<f8"), ("steps", "<u8"), ("capped", "<i4"),
                       ("pad", "<i4"), ("x_exit", "<f8", (3,))])
assert PATH_DTYPE.itemsize == C.sizeof(PathRec)
STATS_DTYPE = np.dtype([("n", "<i8"), ("n_capped", "<i8"), ("steps_sum", "<i8"),
                        ("mean", "<f8"), ("var", "<f8"), ("stderr", "<f8"), ("mean_steps", "<f8"),
                        ("mean_plain", "<f8"), ("var_plain", "<f8"), ("cov", "<f8"),
                        ("rho", "<f8"), ("vr", "<f8"), ("vr_opt", "<f8"), ("sums", "<f8", (10,))])
assert STATS_DTYPE.itemsize == C.sizeof(Stats)

_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so with the plain C compiler (seconds)."""
    if os.environ.get("ORACLE_LIB"):
        return _LIB_PATH
    if force or not os.path.exists(_LIB_PATH):
        subprocess.run(["make", "-s", "-B" if force else "-s", "-C", _HERE], check=True)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB_PATH)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.orc_step_normals.argtypes = [C.POINTER(Problem), C.POINTER(Opts), C.c_uint32,
                                       C.c_uint64, C.c_uint64, C.POINTER(C.c_double)]
        L.orc_bridge_uniform.argtypes = [C.POINTER(Problem), C.POINTER(Opts), C.c_uint32,
                                         C.c_uint64, C.c_uint64]
        L.orc_bridge_uniform.restype = C.c_double
        for name in ("orc_U", "orc_source", "orc_boundary", "orc_kill"):
            getattr(L, name).argtypes = [C.POINTER(Problem), C.POINTER(C.c_double)]
            getattr(L, name).restype = C.c_double
        L.orc_drift.argtypes = [C.POINTER(Problem), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_interp.argtypes = [C.POINTER(Grid), C.POINTER(C.c_double)]
        L.orc_interp.restype = C.c_double
        L.orc_run_path.argtypes = [C.POINTER(Problem), C.POINTER(Opts), C.POINTER(C.c_double),
                                   C.c_uint32, C.c_uint64, C.POINTER(PathRec)]
        L.orc_run_path_noise.argtypes = [C.POINTER(Problem), C.POINTER(Opts),
                                         C.POINTER(C.c_double), C.POINTER(C.c_double),
                                         C.POINTER(C.c_double), C.c_uint64, C.POINTER(PathRec)]
        L.orc_solve_nodes.argtypes = [C.POINTER(Problem), C.POINTER(Opts), C.POINTER(C.c_double),
                                      C.c_int64, C.c_void_p, C.c_void_p]
        L.orc_run_paths.argtypes = [C.POINTER(Problem), C.POINTER(Opts), C.POINTER(C.c_double),
                                    C.POINTER(C.c_uint32), C.POINTER(C.c_uint64), C.c_int64,
                                    C.c_void_p]
        for name in ("orc_run_path", "orc_run_path_noise", "orc_solve_nodes", "orc_run_paths"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


# --------------------------------------------------------------------------- conversion
def make_problem(pd: dict) -> Problem:
    p = Problem()
    p.dim = int(pd["dim"])
    p.domain = {"box": 0, "ball": 1}[pd.get("domain", "box")]
    for d in range(3):
        p.lo[d] = float(pd.get("lo", [0.0] * 3)[d]) if d < len(pd.get("lo", [])) else 0.0
        p.hi[d] = float(pd.get("hi", [0.0] * 3)[d]) if d < len(pd.get("hi", [])) else 0.0
        cen = pd.get("center", [])
        p.center[d] = float(cen[d]) if d < len(cen) else 0.0
        b0 = pd.get("b0", [])
        p.b0[d] = float(b0[d]) if d < len(b0) else 0.0
    p.radius = float(pd.get("radius", 0.0))
    p.sigma = float(pd.get("sigma", 1.0))
    B = pd.get("B", [])
    for i in range(len(B)):
        for j in range(len(B[i])):
            p.B[i][j] = float(B[i][j])
    p.c_a = float(pd.get("c_a", 0.0))
    p.c_b = float(pd.get("c_b", 0.0))
    trig = pd.get("trig", [])
    if len(trig) > MAX_TRIG:
        raise ValueError("too many trig terms")
    p.n_trig = len(trig)
    for m, t in enumerate(trig):
        p.trig[m].amp = float(t["amp"])
        for d in range(len(t["k"])):
            p.trig[m].k[d] = float(t["k"][d])
            p.trig[m].phase[d] = float(t["phase"][d])
    for field, nfield in (("mono", "n_mono"), ("fx", "n_fx"), ("gx", "n_gx")):
        terms = pd.get(field, [])
        if len(terms) > MAX_MONO:
            raise ValueError(f"too many {field} terms")
        setattr(p, nfield, len(terms))
        arr = getattr(p, field)
        for m, t in enumerate(terms):
            arr[m].coef = float(t["coef"])
            for d in range(len(t["e"])):
                arr[m].e[d] = int(t["e"][d])
    p.seed = int(pd.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF
    # tabulated coefficients: {"b": [grid or None per axis], "c": grid, "f": grid, "g": grid}
    tab = pd.get("tab") or {}
    keep = []
    for d, gd in enumerate(tab.get("b") or []):
        if gd is not None:
            keep.append(_GridHolder(gd))
            p.tab_b[d] = C.pointer(keep[-1].grid)
    for field in ("c", "f", "g"):
        if tab.get(field) is not None:
            keep.append(_GridHolder(tab[field]))
            setattr(p, "tab_" + field, C.pointer(keep[-1].grid))
    p._keep = keep  # noqa: SLF001 - lifetime of the grid copies
    return p


class _GridHolder:
    """Keeps the float64 copy of a grid alive while the oracle reads it."""

    def __init__(self, gd: dict):
        self.data = np.ascontiguousarray(np.asarray(gd["data"], dtype=np.float64).ravel())
        g = Grid()
        g.dim = int(gd["dim"])
        for d in range(3):
            g.n[d] = int(gd["n"][d]) if d < len(gd["n"]) else 1
            g.lo[d] = float(gd["lo"][d]) if d < len(gd["lo"]) else 0.0
            g.hi[d] = float(gd["hi"][d]) if d < len(gd["hi"]) else 0.0
        g.data = self.data.ctypes.data_as(C.POINTER(C.c_double))
        self.grid = g


def make_opts(h, n_paths=1, path_offset=0, stream=0, exit="bridge", law="gauss",
              max_steps=1 << 26, u_prev=None, resid=None, grad=None):
    """Options; u_prev + resid select the correction estimator, grad (a list of
    dim grids, the components of grad(u~)) the Ito control variate."""
    o = Opts()
    o.h = float(h)
    o.n_paths = int(n_paths)
    o.path_offset = int(path_offset)
    o.stream = int(stream)
    o.exit_mode = EXIT_MODES[exit]
    o.law = LAWS[law]
    o.max_steps = int(max_steps)
    keep = []
    if (u_prev is None) != (resid is None):
        raise ValueError("u_prev and resid come together")
    if u_prev is not None:
        gu, gr = _GridHolder(u_prev), _GridHolder(resid)
        keep = [gu, gr]
        o.u_prev = C.pointer(gu.grid)
        o.resid = C.pointer(gr.grid)
    if grad is not None:
        if u_prev is not None:
            raise ValueError("grad excludes u_prev / resid")
        for d, g in enumerate(grad):
            keep.append(_GridHolder(g))
            o.grad[d] = C.pointer(keep[-1].grid)
    o._keep = keep  # noqa: SLF001 - lifetime of the grid copies
    return o


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# --------------------------------------------------------------------------- API
def philox(ctr, key):
    L = lib()
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    out = (C.c_uint32 * 4)()
    L.orc_philox4x32_10(c, k, out)
    return [int(v) for v in out]


def step_normals(problem: dict, node, path, step, stream=0, law="gauss"):
    p = make_problem(problem)
    o = make_opts(1.0, stream=stream, law=law)
    out = (C.c_double * 3)()
    lib().orc_step_normals(C.byref(p), C.byref(o), node, path, step, out)
    return np.array(out[: p.dim])


def bridge_uniform(problem: dict, node, path, step, stream=0):
    p = make_problem(problem)
    o = make_opts(1.0, stream=stream)
    return lib().orc_bridge_uniform(C.byref(p), C.byref(o), node, path, step)


def _point_fn(name, problem, pts):
    p = make_problem(problem)
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    out = np.empty(len(pts))
    fn = getattr(lib(), name)
    for q, x in enumerate(pts):
        xx = np.zeros(3)
        xx[: len(x)] = x
        out[q] = fn(C.byref(p), _dptr(xx))
    return out


def U(problem, pts):
    return _point_fn("orc_U", problem, pts)


def source(problem, pts):
    return _point_fn("orc_source", problem, pts)


def boundary(problem, pts):
    return _point_fn("orc_boundary", problem, pts)


def kill(problem, pts):
    return _point_fn("orc_kill", problem, pts)


def drift(problem, pts):
    """b at the points, n x dim."""
    p = make_problem(problem)
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    out = np.zeros((len(pts), p.dim))
    b = (C.c_double * 3)()
    for q, x in enumerate(pts):
        xx = np.zeros(3)
        xx[: len(x)] = x
        lib().orc_drift(C.byref(p), _dptr(xx), b)
        out[q] = b[: p.dim]
    return out


def interp(grid: dict, pts):
    gh = _GridHolder(grid)
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    out = np.empty(len(pts))
    for q, x in enumerate(pts):
        xx = np.zeros(3)
        xx[: len(x)] = x
        out[q] = lib().orc_interp(C.byref(gh.grid), _dptr(xx))
    return out


def run_path(problem, x0, node, path, **opt):
    p = make_problem(problem)
    o = make_opts(**opt)
    xx = np.zeros(3)
    xx[: len(x0)] = x0
    r = PathRec()
    rc = lib().orc_run_path(C.byref(p), C.byref(o), _dptr(xx), node, path, C.byref(r))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return {"phi": r.phi, "e": r.e, "steps": r.steps, "capped": r.capped,
            "x_exit": list(r.x_exit)[: p.dim]}


def run_path_noise(problem, x0, normals, unif, **opt):
    p = make_problem(problem)
    o = make_opts(**opt)
    normals = np.ascontiguousarray(normals, dtype=np.float64)
    unif = np.ascontiguousarray(unif, dtype=np.float64)
    xx = np.zeros(3)
    xx[: len(x0)] = x0
    r = PathRec()
    rc = lib().orc_run_path_noise(C.byref(p), C.byref(o), _dptr(xx), _dptr(normals),
                                  _dptr(unif), len(unif), C.byref(r))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return {"phi": r.phi, "e": r.e, "steps": r.steps, "capped": r.capped,
            "x_exit": list(r.x_exit)[: p.dim]}


def solve_nodes(problem, nodes, record=False, **opt):
    """Node statistics (structured array, STATS_DTYPE) and optionally the
    per-path records (PATH_DTYPE, node-major)."""
    p = make_problem(problem)
    o = make_opts(**opt)
    nodes = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64).reshape(-1, p.dim))
    n = len(nodes)
    stats = np.zeros(n, dtype=STATS_DTYPE)
    rec = np.zeros(n * o.n_paths, dtype=PATH_DTYPE) if record else None
    rc = lib().orc_solve_nodes(C.byref(p), C.byref(o), _dptr(nodes), n,
                               stats.ctypes.data, rec.ctypes.data if record else None)
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return (stats, rec) if record else stats


def run_paths(problem, nodes, node_idx, path_idx, **opt):
    """Per-path records for an explicit list of (node, path) pairs."""
    p = make_problem(problem)
    o = make_opts(**opt)
    nodes = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64).reshape(-1, p.dim))
    ni = np.ascontiguousarray(node_idx, dtype=np.uint32)
    pi = np.ascontiguousarray(path_idx, dtype=np.uint64)
    rec = np.zeros(len(ni), dtype=PATH_DTYPE)
    rc = lib().orc_run_paths(C.byref(p), C.byref(o), _dptr(nodes),
                             ni.ctypes.data_as(C.POINTER(C.c_uint32)),
                             pi.ctypes.data_as(C.POINTER(C.c_uint64)), len(ni), rec.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return rec
