"""Python binding of the C ABI in include/pdd.h (argument marshalling only).

Every step of the solve runs in the HIP library ``libpdd.so``; PyTorch
provides device memory (result and record tensors) and the HIP stream. If the
library is missing, the first call that needs it raises: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdd.so")

PDD_OK = 0
DOMAINS = {"box": 0, "ball": 1}
EXITS = {"bridge": 0, "shift": 1, "naive": 2}
LAWS = {"gauss": 0, "rademacher": 1}
PRECISIONS = {"fp32": 0, "fp64": 1}
PLAIN_ALONGSIDE = 1
TIME_KERNEL = 2
ACCUMULATE = 4
MAX_TRIG, MAX_MONO = 16, 8
NOALLOC_MAX_NODES = 32768  # PDD_NOALLOC_MAX_NODES


class TrigTerm(C.Structure):
    _fields_ = [("amp", C.c_double), ("k", C.c_double * 3), ("phase", C.c_double * 3)]


class MonoTerm(C.Structure):
    _fields_ = [("coef", C.c_double), ("e", C.c_int32 * 3)]


class ProblemDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("domain", C.c_int32),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("center", C.c_double * 3), ("radius", C.c_double),
        ("sigma", C.c_double),
        ("b0", C.c_double * 3), ("B", (C.c_double * 3) * 3),
        ("c_a", C.c_double), ("c_b", C.c_double),
        ("n_trig", C.c_int32), ("n_mono", C.c_int32), ("n_fx", C.c_int32), ("n_gx", C.c_int32),
        ("trig", TrigTerm * MAX_TRIG), ("mono", MonoTerm * MAX_MONO),
        ("fx", MonoTerm * MAX_MONO), ("gx", MonoTerm * MAX_MONO),
        ("seed", C.c_uint64),
    ]


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("dtype", C.c_int32), ("n", C.c_int32 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("data", C.c_void_p)]


class CoefGrids(C.Structure):
    _fields_ = [("b", C.POINTER(Grid) * 3), ("c", C.POINTER(Grid)), ("f", C.POINTER(Grid)),
                ("g", C.POINTER(Grid))]


class Tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("blocks_per_cu", C.c_int32), ("grab", C.c_int32),
                ("max_launch_paths", C.c_int32), ("refill", C.c_int32), ("bridge", C.c_int32)]


def as_tuning(tuning) -> Tuning:
    """A Tuning from a Tuning or from its fields in order (block, blocks_per_cu,
    grab[, max_launch_paths[, refill[, bridge]]]); fields not given are 0 (the default)."""
    if isinstance(tuning, Tuning):
        return tuning
    v = [int(x) for x in tuning]
    if not 3 <= len(v) <= 6:
        raise ValueError(f"a tuning has 3 to 6 fields, got {len(v)}")
    return Tuning(*(v + [0] * (6 - len(v))))


class SolveOpts(C.Structure):
    _fields_ = [("dt", C.c_double), ("n_paths", C.c_uint64),
                ("n_paths_per_node", C.POINTER(C.c_uint64)), ("path_offset", C.c_uint64),
                ("stream_id", C.c_uint32), ("precision", C.c_int32), ("exit_mode", C.c_int32),
                ("law", C.c_int32), ("max_steps", C.c_uint64), ("flags", C.c_uint32),
                ("reserved", C.c_int32),
                ("rec_phi", C.c_void_p), ("rec_e", C.c_void_p), ("rec_steps", C.c_void_p),
                ("tuning", C.POINTER(Tuning))]


class NodeStats(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_capped", C.c_int64), ("steps_sum", C.c_int64),
                ("mean", C.c_double), ("var", C.c_double), ("stderr_", C.c_double),
                ("mean_steps", C.c_double), ("mean_plain", C.c_double), ("var_plain", C.c_double),
                ("cov", C.c_double), ("rho", C.c_double), ("vr", C.c_double),
                ("vr_opt", C.c_double), ("sums", C.c_double * 10)]


class WorkItem(C.Structure):
    _fields_ = [("problem", C.c_void_p), ("nodes", C.POINTER(C.c_double)),
                ("n_nodes", C.c_int64), ("opts", C.POINTER(SolveOpts)),
                ("u_prev", C.POINTER(Grid)), ("resid", C.POINTER(Grid)), ("out", C.c_void_p),
                ("grad", C.POINTER(Grid))]


STATS_DTYPE = np.dtype([("n", "<i8"), ("n_capped", "<i8"), ("steps_sum", "<i8"),
                        ("mean", "<f8"), ("var", "<f8"), ("stderr", "<f8"), ("mean_steps", "<f8"),
                        ("mean_plain", "<f8"), ("var_plain", "<f8"), ("cov", "<f8"),
                        ("rho", "<f8"), ("vr", "<f8"), ("vr_opt", "<f8"), ("sums", "<f8", (10,))])
assert STATS_DTYPE.itemsize == C.sizeof(NodeStats)

class NodeConstants(C.Structure):
    _fields_ = [("E_phi", C.c_double), ("beta", C.c_double), ("se_E_phi", C.c_double),
                ("se_beta", C.c_double), ("V_phi", C.c_double), ("alpha", C.c_double),
                ("se_V_phi", C.c_double), ("se_alpha", C.c_double), ("E_tau", C.c_double),
                ("beta_tau", C.c_double), ("se_E_tau", C.c_double), ("iterations", C.c_int32),
                ("pad", C.c_int32)]


CONSTANTS_DTYPE = np.dtype([(n, "<f8") for n in ("E_phi", "beta", "se_E_phi", "se_beta", "V_phi", "alpha",
                                                   "se_V_phi", "se_alpha", "E_tau", "beta_tau", "se_E_tau")]
                           + [("iterations", "<i4"), ("pad", "<i4")])
assert CONSTANTS_DTYPE.itemsize == C.sizeof(NodeConstants)
GLM_FAMILIES = {"normal": 0, "gamma": 1}


class Partition(C.Structure):
    _fields_ = [("n", C.c_int32 * 2), ("n_cuts", C.c_int32 * 2), ("cuts", C.POINTER(C.c_double) * 2),
                ("rbf_eps", C.c_double)]


class SchedNode(C.Structure):
    _fields_ = [(f, C.c_double) for f in ("K", "V", "alpha", "beta", "V_psi", "rho_psi")]


class TuningKey(C.Structure):
    _fields_ = [("precision", C.c_int32), ("dim", C.c_int32), ("correction", C.c_int32),
                ("generic", C.c_int32)]


class ServerOpts(C.Structure):
    _fields_ = [("memory_budget", C.c_uint64), ("max_inflight", C.c_int32), ("max_queued", C.c_int32),
                ("n_pilot", C.c_uint64), ("n_max", C.c_uint64), ("chunk_paths", C.c_uint64),
                ("epoch_paths", C.c_uint64), ("pipeline", C.c_int32), ("reserved", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("problem", C.c_void_p), ("nodes", C.POINTER(C.c_double)), ("n_nodes", C.c_int64),
                ("dt", C.c_double), ("target_se", C.c_double), ("precision", C.c_int32),
                ("exit_mode", C.c_int32), ("stream_id", C.c_uint32), ("reserved", C.c_int32),
                ("u_prev", C.POINTER(Grid)), ("resid", C.POINTER(Grid)), ("out", C.c_void_p),
                ("user_tag", C.c_uint64), ("grad", C.POINTER(Grid))]


class Completion(C.Structure):
    _fields_ = [("id", C.c_uint64), ("user_tag", C.c_uint64), ("status", C.c_int32),
                ("reserved", C.c_int32), ("queued_ms", C.c_double), ("latency_ms", C.c_double),
                ("paths", C.c_uint64), ("path_steps", C.c_uint64), ("n_nodes", C.c_int64)]


class ServerReport(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("submitted", "shed", "admitted", "completed", "failed",
                                           "queued", "inflight", "epochs", "nodes_completed",
                                           "path_steps", "mem_in_use", "mem_peak", "mem_fixed")] + \
               [(n, C.c_double) for n in ("p50_ms", "p99_ms", "mean_ms", "wall_s", "node_solves_per_s",
                                          "epoch_s")] + \
               [("cancelled", C.c_uint64), ("censored", C.c_uint64), ("p50_censored", C.c_int32),
                ("p99_censored", C.c_int32), ("p50_done_ms", C.c_double), ("p99_done_ms", C.c_double),
                ("busy_s", C.c_double), ("paths_run", C.c_uint64)]


# Every entry point of include/pdd.h with its ctypes signature.
SIGNATURES = {
    "pdd_init": (C.c_int32, [C.POINTER(C.c_void_p), C.c_int]),
    "pdd_shutdown": (None, [C.c_void_p]),
    "pdd_create_problem": (C.c_int32, [C.c_void_p, C.POINTER(ProblemDesc), C.POINTER(C.c_void_p)]),
    "pdd_destroy_problem": (None, [C.c_void_p]),
    "pdd_create_problem_tabulated": (C.c_int32, [C.c_void_p, C.POINTER(ProblemDesc), C.POINTER(CoefGrids),
                                                 C.POINTER(C.c_void_p)]),
    "pdd_solve_nodes": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.c_int64,
                                    C.POINTER(SolveOpts), C.c_void_p, C.c_void_p]),
    "pdd_solve_nodes_noalloc": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.c_int64,
                                            C.POINTER(SolveOpts), C.c_void_p, C.c_void_p]),
    "pdd_schedule": (C.c_int32, [C.POINTER(SchedNode), C.c_int64, C.c_double, C.c_double, C.c_double, C.c_double,
                                 C.c_double, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.POINTER(C.c_int32)]),
    "pdd_stage2": (C.c_int32, [C.c_void_p, C.POINTER(Partition), C.POINTER(C.c_double), C.POINTER(C.c_double),
                               C.c_int64, C.c_void_p, C.c_void_p]),
    "pdd_solve_correction": (C.c_int32, [C.c_void_p, C.POINTER(Grid), C.POINTER(Grid),
                                         C.POINTER(C.c_double), C.c_int64, C.POINTER(SolveOpts),
                                         C.c_void_p, C.c_void_p]),
    "pdd_solve_ito": (C.c_int32, [C.c_void_p, C.POINTER(Grid), C.POINTER(C.c_double), C.c_int64,
                                  C.POINTER(SolveOpts), C.c_void_p, C.c_void_p]),
    "pdd_solve_batch": (C.c_int32, [C.c_void_p, C.POINTER(WorkItem), C.c_int32, C.c_void_p]),
    "pdd_autotune": (C.c_int32, [C.c_void_p, C.POINTER(WorkItem), C.POINTER(Tuning)]),
    "pdd_set_tuning": (C.c_int32, [C.c_void_p, C.POINTER(TuningKey), C.POINTER(Tuning)]),
    "pdd_kernel_times": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.c_int32,
                                     C.POINTER(C.c_int32)]),
    "pdd_plan_paths": (C.c_int32, [C.c_void_p, C.c_int64, C.c_double, C.c_uint64,
                                   C.POINTER(C.c_uint64)]),
    "pdd_solve_to_tolerance": (C.c_int32, [C.c_void_p, C.POINTER(WorkItem), C.c_int32,
                                           C.POINTER(C.c_double), C.c_uint64, C.c_uint64,
                                           C.c_void_p]),
    "pdd_server_create": (C.c_int32, [C.c_void_p, C.POINTER(ServerOpts), C.POINTER(C.c_void_p)]),
    "pdd_server_submit": (C.c_int32, [C.c_void_p, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    "pdd_server_poll": (C.c_int32, [C.c_void_p, C.POINTER(Completion), C.c_int32,
                                    C.POINTER(C.c_int32), C.c_int32]),
    "pdd_server_report_get": (C.c_int32, [C.c_void_p, C.POINTER(ServerReport)]),
    "pdd_server_destroy": (None, [C.c_void_p]),
    "pdd_glm_fit": (C.c_int32, [C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32, C.c_int32,
                                C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "pdd_fit_constants": (C.c_int32, [C.c_void_p, C.POINTER(WorkItem), C.POINTER(C.c_double), C.c_int32,
                                      C.c_uint64, C.c_double, C.c_void_p, C.c_void_p]),
    "pdd_grid_gradient": (C.c_int32, [C.c_void_p, C.POINTER(Grid), C.POINTER(C.c_void_p), C.c_void_p]),
    "pdd_grid_residual": (C.c_int32, [C.c_void_p, C.POINTER(Grid), C.c_void_p, C.c_void_p]),
    "pdd_last_error": (C.c_char_p, []),
}

_lib = None


class PDDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pdd status {status}: {msg}")
        self.status = status


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1512_02818_amd.build` (no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != PDD_OK:
        raise PDDError(status, lib().pdd_last_error().decode())


# --------------------------------------------------------------------------- marshalling
def problem_desc(pd: dict) -> ProblemDesc:
    """Fills the C descriptor from a problem dict (see workloads)."""
    d = ProblemDesc()
    d.dim = int(pd["dim"])
    d.domain = DOMAINS[pd.get("domain", "box")]
    for key in ("lo", "hi", "center", "b0"):
        vals = pd.get(key, [])
        arr = getattr(d, key)
        for i, v in enumerate(vals):
            arr[i] = float(v)
    d.radius = float(pd.get("radius", 0.0))
    d.sigma = float(pd.get("sigma", 1.0))
    for i, row in enumerate(pd.get("B", [])):
        for j, v in enumerate(row):
            d.B[i][j] = float(v)
    d.c_a = float(pd.get("c_a", 0.0))
    d.c_b = float(pd.get("c_b", 0.0))
    trig = pd.get("trig", [])
    if len(trig) > MAX_TRIG:
        raise ValueError("too many trig terms")
    d.n_trig = len(trig)
    for m, t in enumerate(trig):
        d.trig[m].amp = float(t["amp"])
        for i, v in enumerate(t["k"]):
            d.trig[m].k[i] = float(v)
        for i, v in enumerate(t["phase"]):
            d.trig[m].phase[i] = float(v)
    for field in ("mono", "fx", "gx"):
        terms = pd.get(field, [])
        if len(terms) > MAX_MONO:
            raise ValueError(f"too many {field} terms")
        setattr(d, "n_" + field, len(terms))
        arr = getattr(d, field)
        for m, t in enumerate(terms):
            arr[m].coef = float(t["coef"])
            for i, v in enumerate(t["e"]):
                arr[m].e[i] = int(v)
    d.seed = int(pd.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF
    return d


def grid_struct(gd: dict, tensor) -> Grid:
    """C grid over a device tensor holding the values (x fastest)."""
    import torch
    g = Grid()
    g.dim = int(gd["dim"])
    if tensor.dtype == torch.float32:
        g.dtype = 0
    elif tensor.dtype == torch.float64:
        g.dtype = 1
    else:
        raise TypeError("grid values must be float32 or float64")
    if not tensor.is_cuda or not tensor.is_contiguous():
        raise ValueError("grid values must be a contiguous device tensor")
    for i in range(g.dim):
        g.n[i] = int(gd["n"][i])
        g.lo[i] = float(gd["lo"][i])
        g.hi[i] = float(gd["hi"][i])
    g.data = tensor.data_ptr()
    return g


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Context:
    """A library context on one HIP device (owns the solve scratch)."""

    def __init__(self, device: int = 0):
        import torch
        torch.cuda.init()
        self.device = device
        h = C.c_void_p()
        _check(lib().pdd_init(C.byref(h), int(device)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().pdd_shutdown(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Problem:
    """A problem uploaded to a context (pdd_create_problem). A "tab" entry of
    the problem dict ({"b": [grid or None per axis], "c": grid, "f": grid, "g": grid},
    grids as for correction solves) gives tabulated coefficients
    (pdd_create_problem_tabulated); their values are copied to the device for
    the call and kept by the library."""

    def __init__(self, ctx: Context, pd: dict):
        import torch
        self.ctx = ctx
        self.pd = pd
        self.dim = int(pd["dim"])
        self.desc = problem_desc(pd)
        h = C.c_void_p()
        tab = pd.get("tab")
        if tab:
            cg = CoefGrids()
            keep = []

            def dev(gd):
                t = torch.as_tensor(np.ascontiguousarray(gd["data"])).cuda().contiguous()
                g = grid_struct(gd, t)
                keep.append((t, g))
                return C.pointer(g)
            for d, gd in enumerate(tab.get("b") or []):
                if gd is not None:
                    cg.b[d] = dev(gd)
            for field in ("c", "f", "g"):
                if tab.get(field) is not None:
                    setattr(cg, field, dev(tab[field]))
            _check(lib().pdd_create_problem_tabulated(ctx.handle, C.byref(self.desc), C.byref(cg),
                                                      C.byref(h)))
        else:
            _check(lib().pdd_create_problem(ctx.handle, C.byref(self.desc), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().pdd_destroy_problem(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


def make_opts(dt, n_paths=0, n_paths_per_node=None, path_offset=0, stream_id=0,
              precision="fp32", exit="bridge", law="gauss", max_steps=0, plain_alongside=False,
              records=None, tuning=None, time_kernel=False, accumulate=False):
    o = SolveOpts()
    o.dt = float(dt)
    o.n_paths = int(n_paths)
    keep = []
    if n_paths_per_node is not None:
        counts = np.ascontiguousarray(n_paths_per_node, dtype=np.uint64)
        keep.append(counts)
        o.n_paths_per_node = counts.ctypes.data_as(C.POINTER(C.c_uint64))
    o.path_offset = int(path_offset)
    o.stream_id = int(stream_id)
    o.precision = PRECISIONS[precision]
    o.exit_mode = EXITS[exit]
    o.law = LAWS[law]
    o.max_steps = int(max_steps)
    o.flags = ((PLAIN_ALONGSIDE if plain_alongside else 0) | (TIME_KERNEL if time_kernel else 0)
               | (ACCUMULATE if accumulate else 0))
    if records is not None:
        o.rec_phi = records["phi"].data_ptr() if records.get("phi") is not None else None
        o.rec_e = records["e"].data_ptr() if records.get("e") is not None else None
        o.rec_steps = records["steps"].data_ptr()
    if tuning is not None:
        t = as_tuning(tuning)
        keep.append(t)
        o.tuning = C.pointer(t)
    o._keep = keep  # noqa: SLF001 - lifetime of the arrays the struct points to
    return o


def alloc_stats(n_nodes, device="cuda"):
    import torch
    return torch.empty(n_nodes * STATS_DTYPE.itemsize, dtype=torch.uint8, device=device)


def stats_to_numpy(t) -> np.ndarray:
    """Copies a stats tensor to the host as a structured array (synchronises)."""
    return t.cpu().numpy().view(STATS_DTYPE)


def alloc_records(total, correction=False, plain=True, device="cuda"):
    import torch
    rec = {"steps": torch.empty(total, dtype=torch.int32, device=device)}
    rec["phi"] = torch.empty(total, dtype=torch.float64, device=device) if plain else None
    rec["e"] = torch.empty(total, dtype=torch.float64, device=device) if correction else None
    return rec


def solve_nodes(problem: Problem, nodes, out=None, stream=None, **opt):
    """pdd_solve_nodes: returns the device stats tensor (asynchronous)."""
    nodes = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64).reshape(-1, problem.dim))
    n = len(nodes)
    if out is None:
        out = alloc_stats(n)
    o = make_opts(**opt)
    _check(lib().pdd_solve_nodes(problem.handle, nodes.ctypes.data_as(C.POINTER(C.c_double)), n,
                                 C.byref(o), C.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def solve_nodes_noalloc(problem: Problem, nodes, out, stream=None, **opt):
    """pdd_solve_nodes_noalloc: the plain solve without allocation (the
    statistics tensor `out` is the caller's); asynchronous."""
    nodes = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64).reshape(-1, problem.dim))
    o = make_opts(**opt)
    _check(lib().pdd_solve_nodes_noalloc(problem.handle, nodes.ctypes.data_as(C.POINTER(C.c_double)), len(nodes),
                                         C.byref(o), C.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def solve_correction(problem: Problem, u_prev: dict, u_prev_t, resid: dict, resid_t, nodes,
                     out=None, stream=None, **opt):
    """pdd_solve_correction with u_prev / residual values in device tensors."""
    nodes = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64).reshape(-1, problem.dim))
    n = len(nodes)
    if out is None:
        out = alloc_stats(n)
    gu, gr = grid_struct(u_prev, u_prev_t), grid_struct(resid, resid_t)
    o = make_opts(**opt)
    _check(lib().pdd_solve_correction(problem.handle, C.byref(gu), C.byref(gr),
                                      nodes.ctypes.data_as(C.POINTER(C.c_double)), n, C.byref(o),
                                      C.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def grid_array(grids, tensors):
    """A C array of Grid structs (the gradient components of an Ito solve)."""
    if len(grids) != len(tensors):
        raise ValueError("one device tensor per grid")
    arr = (Grid * len(grids))()
    for d, (gd, t) in enumerate(zip(grids, tensors)):
        arr[d] = grid_struct(gd, t)
    return arr


def solve_ito(problem: Problem, grad: list, grad_t: list, nodes, out=None, stream=None, **opt):
    """pdd_solve_ito: grad is the list of dim gradient grid dicts, grad_t their
    device tensors."""
    nodes = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64).reshape(-1, problem.dim))
    n = len(nodes)
    if out is None:
        out = alloc_stats(n)
    ga = grid_array(grad, grad_t)
    o = make_opts(**opt)
    _check(lib().pdd_solve_ito(problem.handle, ga, nodes.ctypes.data_as(C.POINTER(C.c_double)), n,
                               C.byref(o), C.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


class Batch:
    """Marshalled pdd_work_item array (and what it points to) of batch-style
    item dicts, reusable across calls."""

    def __init__(self, items):
        self.arr, self.outs, self._keep = _work_items(items)
        self.n = len(items)


def _as_batch(items):
    return items if isinstance(items, Batch) else Batch(items)


def _work_items(items):
    arr = (WorkItem * len(items))()
    keep = []
    outs = []
    for q, it in enumerate(items):
        prob = it["problem"]
        nodes = np.ascontiguousarray(np.asarray(it["nodes"], dtype=np.float64).reshape(-1, prob.dim))
        out = it.get("out")
        if out is None:
            out = alloc_stats(len(nodes))
        o = make_opts(**it["opts"])
        keep += [nodes, o]
        arr[q].problem = prob.handle
        arr[q].nodes = nodes.ctypes.data_as(C.POINTER(C.c_double))
        arr[q].n_nodes = len(nodes)
        arr[q].opts = C.pointer(o)
        if it.get("u_prev") is not None:
            gu = grid_struct(it["u_prev"], it["u_prev_t"])
            gr = grid_struct(it["resid"], it["resid_t"])
            keep += [gu, gr]
            arr[q].u_prev = C.pointer(gu)
            arr[q].resid = C.pointer(gr)
        if it.get("grad") is not None:
            ga = grid_array(it["grad"], it["grad_t"])
            keep.append(ga)
            arr[q].grad = C.cast(ga, C.POINTER(Grid))
        arr[q].out = out.data_ptr()
        outs.append(out)
    return arr, outs, keep


def solve_batch(ctx: Context, items, stream=None):
    """pdd_solve_batch over dicts {problem, nodes, opts(dict), out, [u_prev, u_prev_t, resid,
    resid_t] or [grad, grad_t] (lists: Ito control variate)}; returns the list of stats
    tensors."""
    b = _as_batch(items)
    _check(lib().pdd_solve_batch(ctx.handle, b.arr, b.n, _stream_handle(stream)))
    return b.outs


def plan_paths(pilot: np.ndarray, target_se: float, n_max: int) -> np.ndarray:
    """pdd_plan_paths on host pilot statistics (a STATS_DTYPE array)."""
    pilot = np.ascontiguousarray(pilot, dtype=STATS_DTYPE)
    out = np.zeros(len(pilot), dtype=np.uint64)
    _check(lib().pdd_plan_paths(pilot.ctypes.data_as(C.c_void_p), len(pilot), float(target_se),
                                int(n_max), out.ctypes.data_as(C.POINTER(C.c_uint64))))
    return out


def solve_to_tolerance(ctx: Context, items, target_se, n_pilot, n_max, stream=None):
    """pdd_solve_to_tolerance over batch-style item dicts (their n_paths is ignored);
    target_se is one value or one per item. Returns the stats tensors."""
    b = _as_batch(items)
    se = np.ascontiguousarray(np.broadcast_to(np.asarray(target_se, dtype=np.float64), (b.n,)))
    _check(lib().pdd_solve_to_tolerance(ctx.handle, b.arr, b.n,
                                        se.ctypes.data_as(C.POINTER(C.c_double)), int(n_pilot),
                                        int(n_max), _stream_handle(stream)))
    return b.outs


def glm_fit(x, y, family="normal"):
    """pdd_glm_fit (host only): (coef[2], se[2], iterations) of y = coef[0] + coef[1] x."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    if len(x) != len(y):
        raise ValueError("x and y differ in length")
    coef, se, it = (C.c_double * 2)(), (C.c_double * 2)(), C.c_int32()
    _check(lib().pdd_glm_fit(x.ctypes.data_as(C.POINTER(C.c_double)), y.ctypes.data_as(C.POINTER(C.c_double)),
                             len(x), GLM_FAMILIES[family], coef, se, C.byref(it)))
    return np.array(coef[:]), np.array(se[:]), it.value


def fit_constants(ctx: Context, item: dict, h, n_hat, delta=1.0, stream=None) -> np.ndarray:
    """pdd_fit_constants on a batch-style item dict (its opts need no dt: the
    cloud h sets it): a CONSTANTS_DTYPE array, one per node."""
    opts = dict({"dt": float(h[0])}, **item["opts"])
    b = Batch([dict(item, opts=opts, out=item.get("out", alloc_stats(0)))])
    h = np.ascontiguousarray(h, dtype=np.float64)
    out = np.zeros(b.arr[0].n_nodes, dtype=CONSTANTS_DTYPE)
    _check(lib().pdd_fit_constants(ctx.handle, b.arr, h.ctypes.data_as(C.POINTER(C.c_double)), len(h),
                                   int(n_hat), float(delta), out.ctypes.data_as(C.c_void_p),
                                   _stream_handle(stream)))
    return out


def grid_gradient(ctx: Context, grid: dict, tensor, stream=None):
    """pdd_grid_gradient: (grid dicts, device tensors) of the dim gradient
    components of a grid whose values are in the device tensor `tensor`."""
    import torch
    D = int(grid["dim"])
    g = grid_struct(grid, tensor)
    outs = [torch.empty_like(tensor) for _ in range(D)]
    ptrs = (C.c_void_p * D)(*[o.data_ptr() for o in outs])
    _check(lib().pdd_grid_gradient(ctx.handle, C.byref(g), ptrs, _stream_handle(stream)))
    dicts = [{"dim": D, "n": list(grid["n"]), "lo": list(grid["lo"]), "hi": list(grid["hi"])} for _ in range(D)]
    return dicts, outs


def schedule(K, V, alpha, beta, V_psi, rho_psi, a0, kappa, delta=1.0, a_max=1.0, s_min=1.5, max_levels=8):
    """pdd_schedule (host only): returns (levels a_0 < ... < a_J, predicted
    speedups of the J levels)."""
    n = len(K)
    arr = (SchedNode * n)()
    for i in range(n):
        arr[i] = SchedNode(float(K[i]), float(V[i]), float(alpha[i]), float(beta[i]), float(V_psi[i]),
                           float(rho_psi[i]))
    a = (C.c_double * (max_levels + 1))()
    sp = (C.c_double * max(max_levels, 1))()
    J = C.c_int32()
    _check(lib().pdd_schedule(arr, n, float(a0), float(kappa), float(delta), float(a_max), float(s_min),
                              int(max_levels), a, sp, C.byref(J)))
    return [a[i] for i in range(J.value + 1)], [sp[i] for i in range(J.value)]


def stage2(problem: Problem, n, cuts, nodes, values, rbf_eps, out=None, stream=None):
    """pdd_stage2: u~ on the n[0] x n[1] grid over the problem's box from the
    nodal values (cuts = [axis-0 interface coordinates, axis-1 ones]); returns
    the device FP64 tensor of shape (n[1], n[0])."""
    import torch
    nodes = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64).reshape(-1, 2))
    values = np.ascontiguousarray(np.asarray(values, dtype=np.float64).ravel())
    if out is None:
        out = torch.empty((int(n[1]), int(n[0])), dtype=torch.float64, device="cuda")
    part = Partition()
    keep = []
    for a in range(2):
        part.n[a] = int(n[a])
        c = np.ascontiguousarray(np.asarray(cuts[a], dtype=np.float64).ravel())
        keep.append(c)
        part.n_cuts[a] = len(c)
        part.cuts[a] = c.ctypes.data_as(C.POINTER(C.c_double))
    part.rbf_eps = float(rbf_eps)
    _check(lib().pdd_stage2(problem.handle, C.byref(part), nodes.ctypes.data_as(C.POINTER(C.c_double)),
                            values.ctypes.data_as(C.POINTER(C.c_double)), len(values), C.c_void_p(out.data_ptr()),
                            _stream_handle(stream)))
    return out


def grid_residual(problem: Problem, grid: dict, tensor, stream=None):
    """pdd_grid_residual: (grid dict, device tensor) of r = f - (L + c) u~ for
    the gridded u~ whose values are in the device tensor `tensor`."""
    import torch
    g = grid_struct(grid, tensor)
    out = torch.empty_like(tensor)
    _check(lib().pdd_grid_residual(problem.handle, C.byref(g), C.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return {"dim": int(grid["dim"]), "n": list(grid["n"]), "lo": list(grid["lo"]), "hi": list(grid["hi"])}, out


def kernel_times(ctx: Context, cap=4096):
    """Path-kernel GPU milliseconds of the solves issued with time_kernel=True."""
    buf = (C.c_double * cap)()
    n = C.c_int32()
    _check(lib().pdd_kernel_times(ctx.handle, buf, cap, C.byref(n)))
    return [buf[i] for i in range(n.value)]


def autotune(ctx: Context, item: dict):
    """pdd_autotune on a batch-style item dict; returns the winner's fields (block,
    blocks_per_cu, grab, max_launch_paths, refill, bridge), which the context
    also keeps for later solves of the same key."""
    b = Batch([dict(item, out=item.get("out", alloc_stats(0)))])
    t = Tuning()
    _check(lib().pdd_autotune(ctx.handle, b.arr, C.byref(t)))
    return (t.block, t.blocks_per_cu, t.grab, t.max_launch_paths, t.refill, t.bridge)


def set_tuning(ctx: Context, precision: str, dim: int, correction, tuning=None, generic=False):
    """pdd_set_tuning: (block, blocks_per_cu, grab[, max_launch_paths[, refill[, bridge]]])
    for the key (correction: 0 / False plain, 1 / True correction estimator, 2 Ito
    control variate; generic: the generic rather than the box / bridge / Gaussian
    kernel), or None to remove it."""
    k = TuningKey(PRECISIONS[precision], int(dim), int(correction), 1 if generic else 0)
    t = None if tuning is None else as_tuning(tuning)
    _check(lib().pdd_set_tuning(ctx.handle, C.byref(k), C.byref(t) if t is not None else None))


class Server:
    """pdd_server_*: continuous batching of node-solve requests to a standard
    error. Host result arrays and grid structs are kept here until their
    request completes."""

    def __init__(self, ctx: Context, memory_budget=0, max_inflight=0, max_queued=0, n_pilot=0,
                 n_max=0, chunk_paths=0, epoch_paths=0, pipeline=0):
        self.ctx = ctx
        o = ServerOpts(int(memory_budget), int(max_inflight), int(max_queued), int(n_pilot),
                       int(n_max), int(chunk_paths), int(epoch_paths), int(pipeline), 0)
        h = C.c_void_p()
        _check(lib().pdd_server_create(ctx.handle, C.byref(o), C.byref(h)))
        self.handle = h
        self.pending = {}  # id -> (stats array, kept objects)
        self.results = {}  # id -> (Completion fields, stats array)

    def submit(self, problem: Problem, nodes, dt, target_se, precision="fp32", exit="bridge",
               stream_id=0, u_prev=None, u_prev_t=None, resid=None, resid_t=None, tag=0, grad=None,
               grad_t=None):
        nodes = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64).reshape(-1, problem.dim))
        out = np.zeros(len(nodes), dtype=STATS_DTYPE)
        r = Request()
        r.problem = problem.handle
        r.nodes = nodes.ctypes.data_as(C.POINTER(C.c_double))
        r.n_nodes = len(nodes)
        r.dt = float(dt)
        r.target_se = float(target_se)
        r.precision = PRECISIONS[precision]
        r.exit_mode = EXITS[exit]
        r.stream_id = int(stream_id)
        keep = [nodes, problem]
        if u_prev is not None:
            gu, gr = grid_struct(u_prev, u_prev_t), grid_struct(resid, resid_t)
            keep += [gu, gr, u_prev_t, resid_t]
            r.u_prev = C.pointer(gu)
            r.resid = C.pointer(gr)
        if grad is not None:
            ga = grid_array(grad, grad_t)
            keep += [ga, grad_t]
            r.grad = C.cast(ga, C.POINTER(Grid))
        r.out = out.ctypes.data
        r.user_tag = int(tag)
        rid = C.c_uint64()
        _check(lib().pdd_server_submit(self.handle, C.byref(r), C.byref(rid)))
        self.pending[rid.value] = (out, keep)
        return rid.value

    def poll(self, wait_ms=0, cap=256):
        """Completions since the last poll, as dicts (with 'stats' on success)."""
        buf = (Completion * cap)()
        n = C.c_int32()
        _check(lib().pdd_server_poll(self.handle, buf, cap, C.byref(n), int(wait_ms)))
        got = []
        for i in range(n.value):
            c = buf[i]
            d = {f: getattr(c, f) for f, _ in Completion._fields_ if f != "reserved"}
            out, _ = self.pending.pop(c.id)
            d["stats"] = out if c.status == PDD_OK else None
            self.results[c.id] = d
            got.append(d)
        return got

    def wait_all(self, timeout_s=600.0):
        """Polls until no submitted request is pending (or the timeout)."""
        import time
        t_end = time.time() + timeout_s
        while self.pending and time.time() < t_end:
            self.poll(wait_ms=50)
        return not self.pending

    def report(self) -> dict:
        r = ServerReport()
        _check(lib().pdd_server_report_get(self.handle, C.byref(r)))
        return {f: getattr(r, f) for f, _ in ServerReport._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib().pdd_server_destroy(self.handle)
            self.handle = None
            self.pending.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass
