"""The 64-problem batched workload at its stated size (path counts x 1: 10^3
to 10^6 paths per node, 38,389 nodes, 4.0e9 paths; `bench.py --batch-scale
1.0` runs it whole). A path's random numbers depend only on (problem seed,
stream, node, path index), so sampled paths of every problem, at their
full-size node and path indices, are replayed here through the batch kernel
and by the oracle: two (node, path) pairs per problem, each as a one-path
item of the problem's full node table (per-node path counts, one path at the
sampled node, offset to the sampled path index), with the stream the
benchmark gives the problem. FP64 paths must match the oracle path for path
(same exit step, scores to 1e-10); the FP32 paths of the same pairs are
checked for their exit steps (all but a few equal) and scores within FP32's
reach of the FP64 ones (Sec. 2.3, Alg. 1; the balanced workload of eq.
F:N_y_h)."""
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


def _samples(seed=11, per_problem=2):
    wl = W.batch_workload(seed=4, n_problems=64, scale=1.0)
    rng = np.random.default_rng(seed)
    out = []
    for q, w in enumerate(wl):
        n = len(w["nodes"])
        for _ in range(per_problem):
            out.append((q, int(rng.integers(0, n)), int(rng.integers(0, w["n_paths"]))))
    return wl, out


def _gpu_paths(ctx, wl, samples, precision):
    probs = {}
    items = []
    for q, node, path in samples:
        w = wl[q]
        if q not in probs:
            probs[q] = pdd.Problem(ctx, w["problem"])
        counts = np.zeros(len(w["nodes"]), dtype=np.uint64)
        counts[node] = 1
        items.append({"problem": probs[q], "nodes": w["nodes"],
                      "opts": dict(dt=w["dt"], n_paths_per_node=counts, path_offset=path, precision=precision,
                                   stream_id=q)})
    outs = pdd.solve_batch(ctx, items)
    torch.cuda.synchronize()
    score = np.empty(len(samples))
    steps = np.empty(len(samples), dtype=np.int64)
    for k, ((q, node, path), o) in enumerate(zip(samples, outs)):
        st = pdd.stats_to_numpy(o)
        assert st["n"][node] == 1 and st["n"].sum() == 1
        score[k] = st["mean"][node]
        steps[k] = st["steps_sum"][node]
    for p in probs.values():
        p.close()
    return score, steps


def test_full_size_batch_sampled_paths_match_oracle(ctx):
    from oracle import oracle as O
    wl, samples = _samples()
    assert sum(w["n_paths"] * len(w["nodes"]) for w in wl) > 3e9  # the stated size
    assert max(s[2] for s in samples) > 1e5  # path indices far beyond the reduced batch's
    s64, k64 = _gpu_paths(ctx, wl, samples, "fp64")
    s32, k32 = _gpu_paths(ctx, wl, samples, "fp32")
    o_score = np.empty(len(samples))
    o_steps = np.empty(len(samples), dtype=np.int64)
    for k, (q, node, path) in enumerate(samples):
        w = wl[q]
        rec = O.run_paths(w["problem"], w["nodes"], [node], [path], h=w["dt"], stream=q)
        o_score[k] = rec["phi"][0]
        assert rec["capped"][0] == 0
        o_steps[k] = rec["steps"][0]
    print(f"{len(samples)} paths of 64 problems, {o_steps.sum()} oracle steps, "
          f"longest {o_steps.max()}")
    assert np.array_equal(k64, o_steps), np.nonzero(k64 != o_steps)
    assert np.allclose(s64, o_score, rtol=1e-10, atol=1e-10), np.max(np.abs(s64 - o_score))
    same = k32 == o_steps
    assert same.mean() >= 0.95, same.mean()
    scale = np.maximum(1.0, np.abs(o_score))
    assert np.max(np.abs(s32 - o_score)[same] / scale[same]) < 2e-3
