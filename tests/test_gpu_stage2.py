"""The second stage on the GPU (pdd_stage2: multiquadric interpolation along
the interfaces, finite-difference subdomain solves by banded LU, one
workgroup per subdomain) against the oracle's (numpy interpolation, sparse
direct solves), FP64, to 1e-10: the unit square's four strips and the [0,4]^2
box's 8 x 8 subdomains (crossing interfaces), nodal values = exact u plus
seeded noise of the size of a nodal statistical error; the paper's example
with tabulated coefficients; the argument checks. All calls through the C ABI."""
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


def compare(ctx, pd, part, nodes, vals):
    from oracle import stage2 as S2
    prob = pdd.Problem(ctx, pd)
    u = pdd.stage2(prob, part["n"], part["cuts"], nodes, vals, part["rbf_eps"]).cpu().numpy()
    prob.close()
    ref = S2.stage2(pd, part["n"], part["cuts"], nodes, vals, part["rbf_eps"])
    err = np.max(np.abs(u - ref) / np.maximum(1.0, np.abs(ref)))
    print(f"stage2 {part['n']} {len(part['cuts'][0])}+{len(part['cuts'][1])} cuts: max rel diff {err:.2e}", flush=True)
    assert err <= 1e-10, err
    return u


@pytest.mark.parametrize("n", [65, 257])
def test_unit_square_strips(ctx, n):
    pd = W.unit_square_problem(seed=0)
    nodes = W.unit_square_nodes()
    rng = np.random.default_rng(n)
    vals = W.manufactured_u(pd, nodes) + rng.normal(scale=0.01, size=len(nodes))
    u = compare(ctx, pd, W.unit_square_partition(n), nodes, vals)
    # the exact nodal values give u~ close to u
    u0 = pdd.stage2(pdd.Problem(ctx, pd), (n, n), [[0.25, 0.5, 0.75], []], nodes, W.manufactured_u(pd, nodes),
                    3.0).cpu().numpy()
    g = np.linspace(0, 1, n)
    X, Y = np.meshgrid(g, g)
    U = W.manufactured_u(pd, np.stack([X.ravel(), Y.ravel()], 1)).reshape(n, n)
    assert np.sqrt(np.mean((u0 - U) ** 2)) < 5e-3
    assert np.all(np.isfinite(u))
    import time
    prob = pdd.Problem(ctx, pd)
    t0 = time.perf_counter()
    for _ in range(3):
        pdd.stage2(prob, (n, n), [[0.25, 0.5, 0.75], []], nodes, vals, 3.0)
    torch.cuda.synchronize()
    print(f"stage2 on {n}^2, 4 strips: {(time.perf_counter() - t0) / 3 * 1e3:.2f} ms per call", flush=True)
    prob.close()


def test_big_square_8x8(ctx):
    pd = W.big_square_problem(seed=0)
    nodes = W.big_square_nodes()
    rng = np.random.default_rng(3)
    vals = W.manufactured_u(pd, nodes) + rng.normal(scale=0.003, size=len(nodes))
    compare(ctx, pd, W.big_square_partition(257), nodes, vals)


def test_paper_example_tabulated(ctx):
    pd = W.paper_example_problem(n=129)
    nodes = W.paper_example_nodes()
    vals = W.paper_example_u(nodes)
    part = {"n": (129, 129), "cuts": [[0.5, 1.0, 1.5], []], "rbf_eps": 1.5}
    compare(ctx, pd, part, nodes, vals)


def test_stage2_arguments(ctx):
    pd = W.unit_square_problem(seed=0)
    prob = pdd.Problem(ctx, pd)
    nodes = W.unit_square_nodes()
    vals = W.manufactured_u(pd, nodes)
    with pytest.raises(pdd.PDDError) as e:  # a node on no interface
        pdd.stage2(prob, (65, 65), [[0.25, 0.5, 0.75], []], np.vstack([nodes, [[0.3, 0.3]]]), np.append(vals, 0.0), 3.0)
    assert e.value.status == -1
    with pytest.raises(pdd.PDDError) as e:  # interface off the grid lines
        pdd.stage2(prob, (65, 65), [[0.25, 0.51, 0.75], []], nodes, vals, 3.0)
    assert e.value.status == -1
    with pytest.raises(pdd.PDDError) as e:  # a subdomain 127 points wide on its shorter side
        pdd.stage2(prob, (257, 257), [[0.5], []], nodes[6:12], vals[6:12], 3.0)
    assert e.value.status == -4
    prob.close()
    p3 = pdd.Problem(ctx, W.ball_exit_time_problem(dim=3))
    with pytest.raises(pdd.PDDError) as e:
        pdd.stage2(p3, (33, 33), [[0.0], []], np.zeros((0, 2)), np.zeros(0), 3.0)
    assert e.value.status == -4
    p3.close()


def test_factor_cache_reuse_and_invalidation(ctx):
    """A context keeps the LU factors of the last call's subdomain matrices
    (they depend on the operator, the grid and the interfaces, not on the
    interface data) and each subdomain's response columns (its solution for
    f and for a unit value at each row next to its boundary), so a call with
    the same operator, grid, interfaces and problem only adds up columns.
    Every call of a sequence that hits and misses the cache gives the bits of
    the same call in a fresh context, and the hit matches the oracle: new
    nodal values on the same strips (hit), another drift (miss), other
    interfaces (miss), back to the first (miss, then hit)."""
    from oracle import stage2 as S2
    pd = W.unit_square_problem(seed=0)
    pd2 = dict(pd, b0=[0.3, -0.2])  # another operator on the same grid
    nodes = W.unit_square_nodes()
    rng = np.random.default_rng(3)
    v1 = W.manufactured_u(pd, nodes) + rng.normal(scale=0.01, size=len(nodes))
    v2 = W.manufactured_u(pd, nodes) + rng.normal(scale=0.01, size=len(nodes))
    strips = W.unit_square_partition(129)
    halves = {"n": (129, 129), "cuts": [[0.5], []], "rbf_eps": 3.0}
    half_nodes = nodes[np.abs(nodes[:, 0] - 0.5) < 1e-12]
    half_vals = W.manufactured_u(pd, half_nodes)
    seq = [(pd, strips, nodes, v1), (pd, strips, nodes, v2), (pd2, strips, nodes, v2),
           (pd, halves, half_nodes, half_vals), (pd, strips, nodes, v1), (pd, strips, nodes, v2)]
    probs = {id(pd): pdd.Problem(ctx, pd), id(pd2): pdd.Problem(ctx, pd2)}
    got = [pdd.stage2(probs[id(p)], part["n"], part["cuts"], x, v, part["rbf_eps"]).cpu().numpy()
           for p, part, x, v in seq]
    for p in probs.values():
        p.close()
    for (p, part, x, v), u in zip(seq, got):
        fresh = pdd.Context(0)
        pr = pdd.Problem(fresh, p)
        ref = pdd.stage2(pr, part["n"], part["cuts"], x, v, part["rbf_eps"]).cpu().numpy()
        pr.close()
        fresh.close()
        assert u.tobytes() == ref.tobytes()
    oracle = S2.stage2(pd, strips["n"], strips["cuts"], nodes, v2, strips["rbf_eps"])
    assert np.max(np.abs(got[1] - oracle) / np.maximum(1.0, np.abs(oracle))) <= 1e-10
    assert got[0].tobytes() == got[4].tobytes() and got[1].tobytes() == got[5].tobytes()


def test_substitution_and_response_columns_agree(ctx, monkeypatch):
    """The two ways of solving the subdomains, substituting each call's right
    side with the kept factors (forced here; the library falls back to it
    when the response columns would exceed 2 GiB) and adding up the kept
    response columns, agree to rounding and both match the oracle."""
    from oracle import stage2 as S2
    pd = W.unit_square_problem(seed=0)
    nodes = W.unit_square_nodes()
    vals = W.manufactured_u(pd, nodes) + np.random.default_rng(5).normal(scale=0.01, size=len(nodes))
    part = W.unit_square_partition(129)
    got = {}
    for way in ("0", "1"):
        monkeypatch.setenv("PDD_STAGE2_SUBSTITUTE", way)
        fresh = pdd.Context(0)
        pr = pdd.Problem(fresh, pd)
        got[way] = [pdd.stage2(pr, part["n"], part["cuts"], nodes, vals, part["rbf_eps"]).cpu().numpy()
                    for _ in range(2)]  # the second call reuses what the first kept
        pr.close()
        fresh.close()
    monkeypatch.delenv("PDD_STAGE2_SUBSTITUTE")
    oracle = S2.stage2(pd, part["n"], part["cuts"], nodes, vals, part["rbf_eps"])
    scale = np.maximum(1.0, np.abs(oracle))
    for way in ("0", "1"):
        assert got[way][0].tobytes() == got[way][1].tobytes()
        assert np.max(np.abs(got[way][0] - oracle) / scale) <= 1e-10
    assert np.max(np.abs(got["0"][0] - got["1"][0]) / scale) <= 1e-12
