"""GPU parity of the Ito control variate (Sec. 2.3, eq. F:xiControlVariate)
against the CPU oracle, through the C ABI (pdd_solve_ito, pdd_solve_batch).

FP64 paths: at least 99.99 % of paths end at the oracle's step; phi and
phi + xi of those paths agree to 1e-11 relative, node means to 1e-10 on nodes
where every path matches. FP32 paths: node means within 3 SE + 1e-5 of the
oracle's. Batches: every item equals its own solve bit for bit.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1512_02818_amd import pdd  # noqa: E402
from paper_1512_02818_amd import workloads as W  # noqa: E402

from test_gpu_parity import check_fp64_parity, geometry_case  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pdd.Context(0)
    yield c
    c.close()


def dev(grids, precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    return [torch.as_tensor(np.asarray(g["data"]), dtype=dt).cuda().contiguous() for g in grids]


def gpu_ito(ctx, pd, nodes, n, grad, **opt):
    prob = pdd.Problem(ctx, pd)
    nodes = np.asarray(nodes, dtype=np.float64).reshape(-1, pd["dim"])
    total = len(nodes) * n
    rec = pdd.alloc_records(total, correction=True, plain=True)
    out = pdd.solve_ito(prob, grad, dev(grad, opt.get("precision", "fp32")), nodes, n_paths=n,
                        records=rec, **opt)
    torch.cuda.synchronize()
    st = pdd.stats_to_numpy(out)
    host = {"steps": rec["steps"].cpu().numpy().view(np.uint32), "phi": rec["phi"].cpu().numpy(),
            "e": rec["e"].cpu().numpy()}
    prob.close()
    return st, host


def oracle_ito(pd, nodes, n, grad, **opt):
    from oracle import oracle as O
    kw = {k: v for k, v in opt.items() if k in ("path_offset", "stream", "exit", "law", "max_steps")}
    return O.solve_nodes(pd, nodes, record=True, h=opt["dt"], n_paths=n, grad=grad, **kw)


def check_plain_too(st, rec, ost, orec):
    same = (rec["steps"] & 0x7FFFFFFF) == orec["steps"].astype(np.uint32)
    assert np.all(np.abs(rec["phi"][same] - orec["phi"][same])
                  <= 1e-11 * np.maximum(1.0, np.abs(orec["phi"][same])))
    for f in ("mean_plain", "vr", "rho", "cov"):
        assert np.allclose(st[f], ost[f], rtol=1e-6, atol=1e-9), f


@pytest.mark.parametrize("exit_mode", ["bridge", "shift", "naive"])
def test_ito_fp64_per_path(ctx, exit_mode):
    pd = W.unit_square_problem(seed=13)
    grad = W.gradient_grids(pd, n=129, seed=1, dtype=np.float64)
    nodes = W.unit_square_nodes()
    n = 3000
    st, rec = gpu_ito(ctx, pd, nodes, n, grad, dt=1e-3, precision="fp64", exit=exit_mode)
    ost, orec = oracle_ito(pd, nodes, n, grad, dt=1e-3, exit=exit_mode)
    check_fp64_parity(st, rec, ost, orec, n, cv=True)
    check_plain_too(st, rec, ost, orec)
    assert np.all(st["vr"] > 20) and np.all(st["rho"] < -0.97)


@pytest.mark.parametrize("case", ["box3d", "ball2d_exit"])
def test_ito_other_geometries_fp64(ctx, case):
    """A 3D box with a full drift matrix and gradient grids of different sizes
    per axis (one cell lookup, three trilinear reads per step), and a 2D ball
    (grids over its bounding box), FP64 paths against the oracle path by path."""
    pd, nodes = geometry_case(case)
    n_grid = (9, 13, 11) if case == "box3d" else 33
    grad = W.gradient_grids(pd, n=n_grid, seed=2, dtype=np.float64, amp=1e-2 if case == "box3d" else 0.0)
    n = 2000
    st, rec = gpu_ito(ctx, pd, nodes, n, grad, dt=1e-3, precision="fp64")
    ost, orec = oracle_ito(pd, nodes, n, grad, dt=1e-3)
    check_fp64_parity(st, rec, ost, orec, n, cv=True)
    check_plain_too(st, rec, ost, orec)


@pytest.mark.parametrize("case", ["unit", "box3d"])
def test_ito_fp32_within_3se(ctx, case):
    if case == "unit":
        pd, nodes = W.unit_square_problem(seed=13), W.unit_square_nodes()
        kw = dict(n=257, seed=1)
    else:
        pd, nodes = geometry_case("box3d")
        kw = dict(n=(9, 13, 11), seed=2)
    grad32 = W.gradient_grids(pd, dtype=np.float32, **kw)
    grad64 = W.gradient_grids(pd, dtype=np.float64, **kw)
    n = 4000
    st, rec = gpu_ito(ctx, pd, nodes, n, grad32, dt=1e-3, precision="fp32")
    ost, orec = oracle_ito(pd, nodes, n, grad64, dt=1e-3)
    assert np.all(np.abs(st["mean"] - ost["mean"]) <= 3 * ost["stderr"] + 1e-5), (st["mean"] - ost["mean"], ost["stderr"])
    assert np.all(np.abs(st["mean_plain"] - ost["mean_plain"]) <= 3 * np.sqrt(ost["var_plain"] / n) + 1e-5)
    same = (rec["steps"] & 0x7FFFFFFF) == orec["steps"].astype(np.uint32)
    assert same.mean() > 0.98


def test_ito_exact_gradient_variance_shrinks_with_h(ctx):
    """u~ = u: V[phi + xi] vanishes as h -> 0 (linearly for this scheme), FP32 paths."""
    pd = W.unit_square_problem(seed=13)
    nodes = W.unit_square_nodes()
    exact = W.manufactured_u(pd, nodes)
    grad = W.gradient_grids(pd, n=257, amp=0.0, dtype=np.float32)
    vr = {}
    n = 20000
    # the scheme's own O(h) bias (bridge exit) reaches about 5e-3 at h = 1e-3
    for h, bias in ((1e-3, 6e-3), (2.5e-4, 2e-3)):
        st, _ = gpu_ito(ctx, pd, nodes, n, grad, dt=h, precision="fp32")
        assert np.all(np.abs(st["mean"] - exact) <= 3 * st["stderr"] + bias)
        # E[xi] = 0 on the same paths: mean(phi + xi) - mean(phi) within 3 SE of xi
        var_xi = st["var"] - st["var_plain"] - 2 * st["cov"]
        assert np.all(np.abs(st["mean"] - st["mean_plain"]) <= 3 * np.sqrt(var_xi / n) + 1e-6)
        vr[h] = st["vr"]
    ratio = vr[2.5e-4] / vr[1e-3]
    assert np.all(vr[1e-3] > 30) and np.all((ratio > 2.8) & (ratio < 5.5)), ratio


def test_ito_in_batches_equals_solo(ctx):
    """Plain, correction and Ito items in one pdd_solve_batch (three groups),
    two alike Ito solves merged into one kernel item: every item's statistics
    equal its own solve's bit for bit."""
    pd = W.unit_square_problem(seed=3)
    prob = pdd.Problem(ctx, pd)
    nodes = W.unit_square_nodes()
    gu, gr, _ = W.correction_grids(pd, n=129, seed=1, dtype=np.float32)
    grad = W.gradient_grids(pd, n=129, seed=1, dtype=np.float32)
    gt = dev(grad, "fp32")
    tu, tr = dev([gu, gr], "fp32")
    opts = lambda sid: dict(dt=1e-3, precision="fp32", n_paths=1500, stream_id=sid)  # noqa: E731
    items = [{"problem": prob, "nodes": nodes, "opts": opts(0)},
             {"problem": prob, "nodes": nodes, "opts": opts(1), "u_prev": gu, "u_prev_t": tu,
              "resid": gr, "resid_t": tr},
             {"problem": prob, "nodes": nodes, "opts": opts(2), "grad": grad, "grad_t": gt},
             {"problem": prob, "nodes": nodes[:7], "opts": opts(3), "grad": grad, "grad_t": gt},
             {"problem": prob, "nodes": nodes, "opts": opts(4), "grad": grad, "grad_t": gt}]
    outs = pdd.solve_batch(ctx, items)
    torch.cuda.synchronize()
    got = [pdd.stats_to_numpy(o) for o in outs]
    for q, it in enumerate(items):
        solo = pdd.stats_to_numpy(pdd.solve_batch(ctx, [it])[0])
        for f in ("mean", "var", "mean_plain", "rho", "steps_sum"):
            assert np.array_equal(got[q][f], solo[f], equal_nan=True), (q, f)
    # the Ito item's own entry point gives the same numbers
    st = pdd.stats_to_numpy(pdd.solve_ito(prob, grad, gt, nodes, **opts(2)))
    assert np.array_equal(st["mean"], got[2]["mean"]) and np.array_equal(st["rho"], got[2]["rho"])
    prob.close()


def test_ito_invalid_arguments(ctx):
    pd = W.unit_square_problem(seed=3)
    prob = pdd.Problem(ctx, pd)
    nodes = W.unit_square_nodes()[:2]
    grad = W.gradient_grids(pd, n=33, seed=1, dtype=np.float32)
    gt = dev(grad, "fp32")
    # components of different geometries
    odd = [grad[0], dict(grad[1], n=[33, 33], hi=[1.0, 1.5])]
    with pytest.raises(pdd.PDDError):
        pdd.solve_ito(prob, odd, gt, nodes, dt=1e-3, n_paths=10)
    # dtype of the grids must match the path precision
    with pytest.raises(pdd.PDDError):
        pdd.solve_ito(prob, grad, gt, nodes, dt=1e-3, n_paths=10, precision="fp64")
    # gradient and correction grids together
    gu, gr, _ = W.correction_grids(pd, n=33, seed=1, dtype=np.float32)
    tu, tr = dev([gu, gr], "fp32")
    with pytest.raises(pdd.PDDError):
        pdd.solve_batch(ctx, [{"problem": prob, "nodes": nodes, "opts": dict(dt=1e-3, n_paths=10),
                               "u_prev": gu, "u_prev_t": tu, "resid": gr, "resid_t": tr,
                               "grad": grad, "grad_t": gt}])
    # records need phi as well as phi + xi
    rec = pdd.alloc_records(20, correction=True, plain=False)
    with pytest.raises(pdd.PDDError):
        pdd.solve_ito(prob, grad, gt, nodes, dt=1e-3, n_paths=10, records=rec)
    # a bad estimator in a tuning key
    with pytest.raises(pdd.PDDError):
        pdd.set_tuning(ctx, "fp32", 2, 3, (256, 0, 64))
    pdd.set_tuning(ctx, "fp32", 2, 2, (128, 0, 16))
    st = pdd.stats_to_numpy(pdd.solve_ito(prob, grad, gt, nodes, dt=1e-3, n_paths=500))
    pdd.set_tuning(ctx, "fp32", 2, 2, None)
    st2 = pdd.stats_to_numpy(pdd.solve_ito(prob, grad, gt, nodes, dt=1e-3, n_paths=500))
    assert np.array_equal(st["mean"], st2["mean"])  # the launch shape never changes results
    prob.close()


def test_ito_large_launch_sampled_paths(ctx):
    """The node-solve workload's shape: 500 replicas of the 18 unit-square
    nodes (distinct streams) x 1,000 paths in one batch, FP64, each replica
    with its own records; 1,500 sampled paths recomputed by the oracle one by
    one."""
    from oracle import oracle as O
    pd = W.unit_square_problem(seed=0)
    prob = pdd.Problem(ctx, pd)
    nodes = W.unit_square_nodes()
    grad = W.gradient_grids(pd, n=257, seed=1, dtype=np.float64)
    gt = dev(grad, "fp64")
    R, n = 500, 1000
    recs, items = [], []
    for r in range(R):
        rec = pdd.alloc_records(len(nodes) * n, correction=True, plain=True)
        recs.append(rec)
        items.append({"problem": prob, "nodes": nodes, "grad": grad, "grad_t": gt,
                      "opts": dict(dt=1e-3, precision="fp64", n_paths=n, stream_id=r, records=rec)})
    outs = pdd.solve_batch(ctx, items)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    pick = rng.integers(0, R, size=1500)
    node = rng.integers(0, len(nodes), size=1500)
    path = rng.integers(0, n, size=1500)
    agree = 0
    for r in np.unique(pick):
        sel = pick == r
        orec = O.run_paths(pd, nodes, node[sel], path[sel], h=1e-3, stream=int(r), grad=grad)
        slot = node[sel] * n + path[sel]
        steps = recs[r]["steps"].cpu().numpy().view(np.uint32)[slot] & 0x7FFFFFFF
        e = recs[r]["e"].cpu().numpy()[slot]
        same = steps == orec["steps"].astype(np.uint32)
        agree += int(same.sum())
        assert np.all(np.abs(e[same] - orec["e"][same]) <= 1e-11 * np.maximum(1.0, np.abs(orec["e"][same])))
    assert agree >= 1500 - 2
    st = pdd.stats_to_numpy(outs[0])
    assert np.all(st["n"] == n) and np.all(st["vr"] > 20)
    prob.close()


def test_ito_solved_to_tolerance(ctx):
    """pdd_solve_to_tolerance takes an Ito item like any other: every node
    gets to the target standard error (pilot, plan on V[phi + xi], merged
    continuation), and the result is a merge of the same paths' sums."""
    pd = W.unit_square_problem(seed=3)
    prob = pdd.Problem(ctx, pd)
    nodes = W.unit_square_nodes()
    grad = W.gradient_grids(pd, n=257, seed=1, dtype=np.float32)
    gt = dev(grad, "fp32")
    item = {"problem": prob, "nodes": nodes, "grad": grad, "grad_t": gt,
            "opts": dict(dt=1e-3, precision="fp32", stream_id=5)}
    se = 2e-4
    st = pdd.stats_to_numpy(pdd.solve_to_tolerance(ctx, [item], se, 1000, 1 << 24)[0])
    # the plan uses the pilot's variance (1,000 paths), so the final SE lands
    # near the target, within the pilot's sampling noise
    assert np.all(st["stderr"] < 1.25 * se) and np.median(st["stderr"]) > 0.8 * se, st["stderr"]
    assert np.all(st["n"] > 1000)  # the pilot alone does not reach it
    # the same paths in one solve give the same statistics
    one = pdd.stats_to_numpy(pdd.solve_batch(ctx, [dict(item, opts=dict(item["opts"],
                                                                       n_paths_per_node=st["n"].astype(np.uint64)))])[0])
    assert np.allclose(one["mean"], st["mean"], rtol=1e-12, atol=1e-14)
    assert np.allclose(one["var"], st["var"], rtol=1e-9)
    prob.close()
