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
    block, bpc, grab = pdd.autotune(ctx, item)
    assert block in (64, 128, 256) and bpc >= 1 and grab in (16, 64, 256)
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
    k = pdd.TuningKey(0, 2, 0, 2)  # generic must be 0 or 1
    t = pdd.Tuning(128, 1, 64, 0)
    assert pdd.lib().pdd_set_tuning(ctx.handle, pdd.C.byref(k), pdd.C.byref(t)) == -1


def test_cache_load(ctx, tmp_path):
    path = str(tmp_path / "c.json")
    arch = T.arch_name()
    T.save_entry(path, T.key(arch, "fp32", 2, False), (128, 4, 64))
    T.save_entry(path, T.key("gfx000", "fp32", 2, False), (64, 1, 16))  # another architecture
    assert T.load(ctx, path) == 1
    prob = pdd.Problem(ctx, W.unit_square_problem())
    st = pdd.stats_to_numpy(pdd.solve_nodes(prob, W.unit_square_nodes(), dt=1e-3, n_paths=500))
    assert np.all(st["n"] == 500)
    pdd.set_tuning(ctx, "fp32", 2, False, None)
    prob.close()
