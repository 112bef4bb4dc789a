"""Autotuner through the C ABI: the sweep returns a shape of its candidate
set, the context keeps it for later solves, and results do not change."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1512_02818_amd import pdd  # noqa: E402
from paper_1512_02818_amd import tuning as T  # noqa: E402
from paper_1512_02818_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pdd.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("cv", [False, True])
def test_autotune_and_results_unchanged(ctx, prec, cv):
    pd = W.unit_square_problem(seed=1)
    prob = pdd.Problem(ctx, pd)
    nodes = W.unit_square_nodes()
    item = {"problem": prob, "nodes": nodes, "opts": dict(dt=1e-3, precision=prec)}
    if cv:
        gu, gr, _ = W.correction_grids(pd, n=65, seed=2, dtype=np.float32 if prec == "fp32" else np.float64)
        item.update(u_prev=gu, u_prev_t=torch.as_tensor(gu["data"]).cuda().contiguous(),
                    resid=gr, resid_t=torch.as_tensor(gr["data"]).cuda().contiguous())
    pdd.set_tuning(ctx, prec, 2, cv, None)

    def solve():
        (o,) = pdd.solve_batch(ctx, [dict(item, opts=dict(item["opts"], n_paths=2000))])
        return pdd.stats_to_numpy(o)

    before = solve()
    block, bpc, grab, cap, refill, bridge = pdd.autotune(ctx, item)
    assert block in (64, 128, 256) and bpc >= 1 and grab in (16, 64, 256) and cap == 0
    assert refill in (0, 1, 2, 4, 8) and bridge in (0, 1, 2)
    after = solve()  # now with the tuned shape from the context's table
    assert before.tobytes() == after.tobytes()
    prob.close()


def test_set_tuning_validates(ctx):
    with pytest.raises(pdd.PDDError):
        pdd.set_tuning(ctx, "fp32", 4, False, (256, 1, 64))
    with pytest.raises(pdd.PDDError):
        pdd.set_tuning(ctx, "fp32", 2, False, (96, 1, 64))
    pdd.set_tuning(ctx, "fp32", 2, False, (128, 3, 16))
    pdd.set_tuning(ctx, "fp32", 2, False, None)
    pdd.set_tuning(ctx, "fp32", 2, False, (64, 2, 16), generic=True)
    pdd.set_tuning(ctx, "fp32", 2, False, None, generic=True)
    for bad in ((256, 0, 64, 0, 3, 0), (256, 0, 64, 0, 16, 0), (256, 0, 64, 0, 0, 3), (256, 0, 64, 0, 0, -1)):
        with pytest.raises(pdd.PDDError):
            pdd.set_tuning(ctx, "fp32", 2, False, bad)
    pdd.set_tuning(ctx, "fp32", 2, False, (256, 0, 64, 0, 8, 2))
    pdd.set_tuning(ctx, "fp32", 2, False, None)
    k = pdd.TuningKey(0, 2, 0, 2)  # generic must be 0 or 1
    t = pdd.Tuning(128, 1, 64, 0)
    assert pdd.lib().pdd_set_tuning(ctx.handle, pdd.C.byref(k), pdd.C.byref(t)) == -1


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("est", ["plain", "correction", "ito"])
@pytest.mark.parametrize("dim", [2, 3])
def test_refill_and_bridge_form_leave_results_unchanged(ctx, prec, est, dim):
    """Every refill period and both forms of the bridge test give the same
    per-node statistics, bit for bit, as the default (a path's random numbers
    depend only on its indices; the node sums are reduced in a fixed order)."""
    if dim == 2:
        pd = W.unit_square_problem(seed=3)
        nodes = W.unit_square_nodes()
    else:
        rng = np.random.default_rng(5)
        pd = W.random_problem(rng, dim=3)
        nodes = W.face_nodes(rng, pd, 40)
    prob = pdd.Problem(ctx, pd)
    dt = np.float32 if prec == "fp32" else np.float64
    item = {"problem": prob, "nodes": nodes, "opts": dict(dt=1e-3, precision=prec, n_paths=1500)}
    if est == "correction":
        gu, gr, _ = W.correction_grids(pd, n=65 if dim == 2 else 17, seed=2, dtype=dt)
        item.update(u_prev=gu, u_prev_t=torch.as_tensor(gu["data"]).cuda().contiguous(),
                    resid=gr, resid_t=torch.as_tensor(gr["data"]).cuda().contiguous())
    elif est == "ito":
        g = W.gradient_grids(pd, n=65 if dim == 2 else 17, seed=2, dtype=dt)
        item.update(grad=g, grad_t=[torch.as_tensor(x["data"]).cuda().contiguous() for x in g])

    def solve(tuning):
        (o,) = pdd.solve_batch(ctx, [dict(item, opts=dict(item["opts"], tuning=tuning))])
        return pdd.stats_to_numpy(o).tobytes()

    ref = solve(None)
    for refill in (1, 2, 4, 8):
        for bridge in (1, 2):
            assert solve((128, 0, 16, 0, refill, bridge)) == ref, (refill, bridge)
    prob.close()


def test_cache_load(ctx, tmp_path):
    path = str(tmp_path / "c.json")
    arch = T.arch_name()
    T.save_entry(path, T.key(arch, "fp32", 2, False), (128, 4, 64, 0, 4, 2))
    T.save_entry(path, T.key("gfx000", "fp32", 2, False), (64, 1, 16))  # another architecture
    assert T.load(ctx, path) == 1
    prob = pdd.Problem(ctx, W.unit_square_problem())
    st = pdd.stats_to_numpy(pdd.solve_nodes(prob, W.unit_square_nodes(), dt=1e-3, n_paths=500))
    assert np.all(st["n"] == 500)
    pdd.set_tuning(ctx, "fp32", 2, False, None)
    prob.close()
