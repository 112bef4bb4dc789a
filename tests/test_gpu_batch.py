"""Batched solves: many problems (2D and 3D, plain and correction, FP32 and
FP64, uneven node and path counts) in one pdd_solve_batch call. Every item
must give exactly the statistics of its own solve call (same paths, same
reduction order), and one item is checked against the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1512_02818_amd import pdd  # noqa: E402
from paper_1512_02818_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pdd.Context(0)
    yield c
    c.close()


def _items(ctx):
    wl = W.batch_workload(seed=4, n_problems=12, node_range=(3, 60), path_range=(50, 800))
    items = []
    for q, w in enumerate(wl):
        prob = pdd.Problem(ctx, w["problem"])
        items.append({"problem": prob, "nodes": w["nodes"],
                      "opts": dict(dt=w["dt"] * 10, n_paths=w["n_paths"],
                                   precision="fp64" if q % 3 == 0 else "fp32", stream_id=q)})
    # a correction item and a ragged item on the unit-square problem
    pd = W.unit_square_problem(seed=9)
    prob = pdd.Problem(ctx, pd)
    gu, gr, _ = W.correction_grids(pd, n=65, seed=3, dtype=np.float32)
    tu = torch.as_tensor(gu["data"]).cuda().contiguous()
    tr = torch.as_tensor(gr["data"]).cuda().contiguous()
    items.append({"problem": prob, "nodes": W.unit_square_nodes(),
                  "opts": dict(dt=1e-3, n_paths=700, precision="fp32", plain_alongside=True),
                  "u_prev": gu, "u_prev_t": tu, "resid": gr, "resid_t": tr})
    items.append({"problem": prob, "nodes": W.unit_square_nodes()[:5],
                  "opts": dict(dt=1e-3, n_paths_per_node=np.array([0, 3, 500, 64, 1], dtype=np.uint64),
                               precision="fp64")})
    return items


def test_batch_equals_solo(ctx):
    items = _items(ctx)
    outs = pdd.solve_batch(ctx, items)
    torch.cuda.synchronize()
    batch = [pdd.stats_to_numpy(o) for o in outs]
    for it, b in zip(items, batch):
        if it.get("u_prev") is not None:
            solo = pdd.solve_correction(it["problem"], it["u_prev"], it["u_prev_t"], it["resid"],
                                        it["resid_t"], it["nodes"], **it["opts"])
        else:
            solo = pdd.solve_nodes(it["problem"], it["nodes"], **it["opts"])
        torch.cuda.synchronize()
        s = pdd.stats_to_numpy(solo)
        assert s.tobytes() == b.tobytes()
        assert np.all(s["n_capped"] == 0)


def test_batch_item_matches_oracle(ctx):
    from oracle import oracle as O
    items = _items(ctx)
    outs = pdd.solve_batch(ctx, items)
    torch.cuda.synchronize()
    q = 3  # an FP64 item
    it = items[q]
    st = pdd.stats_to_numpy(outs[q])
    ost = O.solve_nodes(it["problem"].pd, it["nodes"], h=it["opts"]["dt"],
                        n_paths=it["opts"]["n_paths"], stream=it["opts"]["stream_id"])
    assert np.allclose(st["mean"], ost["mean"], rtol=1e-9, atol=1e-10)
    assert np.array_equal(st["steps_sum"], ost["steps_sum"])


def test_batch_chunked_and_empty(ctx):
    items = _items(ctx)[:6]
    items.insert(2, {"problem": items[0]["problem"], "nodes": np.zeros((0, items[0]["problem"].dim)),
                     "opts": dict(dt=1e-3, n_paths=10)})
    ref = [pdd.stats_to_numpy(o) for o in pdd.solve_batch(ctx, items)]
    for it in items:
        it["opts"] = dict(it["opts"], tuning=(128, 2, 16, 3001))
    got = [pdd.stats_to_numpy(o) for o in pdd.solve_batch(ctx, items)]
    for a, b in zip(ref, got):
        assert np.array_equal(a["n"], b["n"]) and np.array_equal(a["steps_sum"], b["steps_sum"])
        assert np.allclose(a["mean"], b["mean"], rtol=1e-13, atol=1e-14, equal_nan=True)


def test_many_small_items_under_any_launch_shape(ctx):
    """Hundreds of small items in one group (empty items and nodes with no
    paths among them), so waves move between the items' queues often: every
    item's statistics equal its solo solve, bit for bit, under every launch
    shape; with launches cut inside items (a node's paths then reach its sums
    in two parts) counts are equal and means agree to rounding."""
    prob = pdd.Problem(ctx, W.unit_square_problem(seed=11))
    rng = np.random.default_rng(7)
    base = W.unit_square_nodes()
    items = []
    for q in range(300):
        nn = int(rng.integers(0, 8))
        counts = rng.integers(0, 400, size=nn).astype(np.uint64)
        if nn and q % 5 == 0:
            counts[0] = 0
        items.append({"problem": prob, "nodes": np.resize(base, (nn, 2)),
                      "opts": dict(dt=1e-3, n_paths_per_node=counts, precision="fp32", stream_id=q)})
    solo = [pdd.stats_to_numpy(pdd.solve_nodes(prob, it["nodes"], **it["opts"])) for it in items]
    for tune in (None, (64, 1, 16, 0), (256, 0, 256, 0), (128, 3, 64, 5003)):
        for it in items:
            it["opts"] = {k: v for k, v in it["opts"].items() if k != "tuning"}
            if tune:
                it["opts"]["tuning"] = tune
        got = [pdd.stats_to_numpy(o) for o in pdd.solve_batch(ctx, items)]
        torch.cuda.synchronize()
        for q, (a, b) in enumerate(zip(solo, got)):
            if tune is None or tune[3] == 0:
                assert a.tobytes() == b.tobytes(), (tune, q)
            else:
                assert np.array_equal(a["n"], b["n"]) and np.array_equal(a["steps_sum"], b["steps_sum"]), q
                assert np.allclose(a["mean"], b["mean"], rtol=1e-13, atol=1e-14, equal_nan=True), q
    prob.close()


@pytest.mark.parametrize("cv", [False, True])
def test_merged_uniform_solves_equal_solo(ctx, cv):
    """Runs of alike uniform solves (same problem and step, distinct streams
    and path offsets) are merged into one kernel item with a per-node RNG
    table; runs are broken by a different path count, step or exit test.
    Every solve's statistics equal its solo solve bit for bit."""
    pd = W.unit_square_problem(seed=21)
    prob = pdd.Problem(ctx, pd)
    nodes = W.unit_square_nodes()
    gu, gr, _ = W.correction_grids(pd, n=65, seed=2, dtype=np.float32)
    tu = torch.as_tensor(gu["data"]).cuda().contiguous()
    tr = torch.as_tensor(gr["data"]).cuda().contiguous()
    items = []
    for q in range(40):
        opts = dict(dt=1e-3, n_paths=300, precision="fp32", stream_id=100 + q, path_offset=7 * q)
        if q in (13, 14):
            opts["n_paths"] = 301          # breaks the run
        if q == 25:
            opts["dt"] = 2e-3              # breaks the run
        if q == 31:
            opts["exit"] = "shift"         # breaks the run (and the kernel variant)
        it = {"problem": prob, "nodes": nodes[q % 5::3], "opts": opts}
        if cv:
            it.update(u_prev=gu, u_prev_t=tu, resid=gr, resid_t=tr)
        items.append(it)
    got = [pdd.stats_to_numpy(o) for o in pdd.solve_batch(ctx, items)]
    torch.cuda.synchronize()
    for q, (it, g) in enumerate(zip(items, got)):
        if cv:
            solo = pdd.solve_correction(prob, gu, tu, gr, tr, it["nodes"], **it["opts"])
        else:
            solo = pdd.solve_nodes(prob, it["nodes"], **it["opts"])
        assert pdd.stats_to_numpy(solo).tobytes() == g.tobytes(), q
    prob.close()
