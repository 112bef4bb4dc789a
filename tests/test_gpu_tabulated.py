"""GPU parity of problems with tabulated coefficients (b, c, f on grids,
pdd_create_problem_tabulated) against the CPU oracle on the same streams,
through the C ABI: FP64 path by path, FP32 within 3 SE; the exact solution
is kept; batches mixing analytic and tabulated problems equal solo solves;
malformed grids are rejected."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1512_02818_amd import pdd  # noqa: E402
from paper_1512_02818_amd import workloads as W  # noqa: E402

from test_gpu_parity import check_fp64_parity, gpu_solve, oracle_solve  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pdd.Context(0)
    yield c
    c.close()


def _tab_2d(fields=("b", "c", "f"), n=65, dtype=np.float64):
    pd = W.unit_square_problem(seed=0)
    return pd, W.tabulated_problem(pd, n=n, fields=fields, amp=0.6, seed=2, dtype=dtype)


@pytest.mark.parametrize("fields", [("b", "c", "f"), ("b",), ("c", "f")])
def test_tabulated_fp64_per_path(ctx, fields):
    pd, tab = _tab_2d(fields)
    nodes = W.unit_square_nodes()[::2]
    n = 3000
    st, rec = gpu_solve(ctx, tab, nodes, n, dt=1e-3, precision="fp64")
    ost, orec = oracle_solve(tab, nodes, n, dt=1e-3)
    check_fp64_parity(st, rec, ost, orec, n)


def test_tabulated_3d_fp64_per_path_and_fp32(ctx):
    rng = np.random.default_rng(4)
    pd = W.random_problem(rng, dim=3)
    tab = W.tabulated_problem(pd, n=17, fields=("b", "c", "f"), amp=0.4, seed=3)
    lo, hi = np.asarray(pd["lo"][:3]), np.asarray(pd["hi"][:3])
    nodes = lo + (hi - lo) * np.array([[0.5, 0.5, 0.5], [0.2, 0.7, 0.4], [0.8, 0.3, 0.6]])
    n = 2000
    st, rec = gpu_solve(ctx, tab, nodes, n, dt=1e-3, precision="fp64")
    ost, orec = oracle_solve(tab, nodes, n, dt=1e-3)
    check_fp64_parity(st, rec, ost, orec, n)
    st32, _ = gpu_solve(ctx, tab, nodes, n, dt=1e-3, precision="fp32")
    assert np.all(np.abs(st32["mean"] - ost["mean"]) <= 3 * ost["stderr"] + 1e-5)


def test_tabulated_fp32_keeps_the_exact_solution(ctx):
    """FP32 paths on FP32 grids: within 3 SE + 1e-5 of the oracle, and the
    exact U within 3 SE + the bias allowance of the oracle's pins."""
    pd, tab = _tab_2d(n=257, dtype=np.float32)
    nodes = W.unit_square_nodes()
    n = 8000
    st, _ = gpu_solve(ctx, tab, nodes, n, dt=1e-3, precision="fp32")
    ost, _ = oracle_solve(tab, nodes, n, dt=1e-3)
    assert np.all(np.abs(st["mean"] - ost["mean"]) <= 3 * ost["stderr"] + 1e-5)
    exact = W.manufactured_u(pd, nodes)
    assert np.all(np.abs(st["mean"] - exact) <= 3 * st["stderr"] + 2e-3)


def test_tabulated_correction_fp64_per_path(ctx):
    pd, tab = _tab_2d()
    gu, gr, _ = W.correction_grids(pd, n=65, seed=1, dtype=np.float64)
    nodes = W.unit_square_nodes()[::3]
    n = 2000
    st, rec = gpu_solve(ctx, tab, nodes, n, grids=(gu, gr), dt=1e-3, precision="fp64", plain_alongside=True)
    ost, orec = oracle_solve(tab, nodes, n, grids=(gu, gr), dt=1e-3)
    check_fp64_parity(st, rec, ost, orec, n, cv=True)


def test_batch_mixing_tabulated_and_analytic_equals_solo(ctx):
    pd, tab = _tab_2d(n=33)
    pa, pt = pdd.Problem(ctx, pd), pdd.Problem(ctx, tab)
    nodes = W.unit_square_nodes()
    items = [{"problem": p, "nodes": nodes[i::3], "opts": dict(dt=1e-3, n_paths=700, precision=prec,
                                                               stream_id=i)}
             for i, (p, prec) in enumerate([(pa, "fp32"), (pt, "fp32"), (pa, "fp64"), (pt, "fp64")])]
    got = [pdd.stats_to_numpy(o) for o in pdd.solve_batch(ctx, items)]
    for it, g in zip(items, got):
        solo = pdd.stats_to_numpy(pdd.solve_nodes(it["problem"], it["nodes"], **it["opts"]))
        assert solo.tobytes() == g.tobytes()
    pa.close()
    pt.close()


def test_malformed_grids_are_rejected(ctx):
    pd, tab = _tab_2d(fields=("c",), n=9)
    L = pdd.lib()
    desc = pdd.problem_desc(pd)
    t = torch.as_tensor(tab["tab"]["c"]["data"]).cuda().contiguous()

    def create(gd, slot="c"):
        g = pdd.grid_struct(gd, t)
        cg = pdd.CoefGrids()
        if slot == "c":
            cg.c = C.pointer(g)
        else:
            cg.b[2] = C.pointer(g)
        h = C.c_void_p()
        st = L.pdd_create_problem_tabulated(ctx.handle, C.byref(desc), C.byref(cg), C.byref(h))
        if st == 0:
            L.pdd_destroy_problem(h)
        return st

    good = tab["tab"]["c"]
    assert create(good) == 0
    assert create(dict(good, lo=[0.1, 0.0])) == -1        # does not contain the domain
    assert b"cover" in L.pdd_last_error()
    assert create(dict(good, n=[1, 9])) == -1             # fewer than 2 points
    assert create(good, slot="b2") == -1                  # b[2] of a 2D problem
    h = C.c_void_p()
    assert L.pdd_create_problem_tabulated(ctx.handle, C.byref(desc), None, C.byref(h)) == -1


def test_tabulated_problem_served_like_solved_to_tolerance(ctx):
    """A tabulated problem through the serving loop and through
    pdd_solve_to_tolerance: the same plan (path counts, steps) and means."""
    pd, tab = _tab_2d(n=33)
    prob = pdd.Problem(ctx, tab)
    nodes = W.unit_square_nodes()[::4]
    se = 3e-3
    sv = pdd.Server(ctx, epoch_paths=1 << 22, chunk_paths=1 << 17)
    rid = sv.submit(prob, nodes, 1e-3, se, precision="fp32", stream_id=9, tag=9)
    assert sv.wait_all(120)
    got = sv.results[rid]
    sv.close()
    assert got["status"] == 0
    item = {"problem": prob, "nodes": nodes, "opts": dict(dt=1e-3, precision="fp32", stream_id=9)}
    (o,) = pdd.solve_to_tolerance(ctx, [item], se, 1000, 1 << 31)
    st = pdd.stats_to_numpy(o)
    assert np.array_equal(st["n"], got["stats"]["n"]) and np.array_equal(st["steps_sum"], got["stats"]["steps_sum"])
    assert np.allclose(st["mean"], got["stats"]["mean"], rtol=1e-12, atol=1e-14)
    assert np.all(st["stderr"] <= 1.3 * se)
    prob.close()
