"""GPU gradient (pdd_grid_gradient) and residual (pdd_grid_residual) of a
gridded u~ against the oracle's second-order differences, and the two control
variates fed with them."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import grid as G  # noqa: E402
from paper_1512_02818_amd import pdd  # noqa: E402
from paper_1512_02818_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pdd.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n", [(3, 3), (7, 5), (257, 129), (5, 6, 3), (33, 17, 9)])
def test_gradient_matches_oracle(ctx, n):
    rng = np.random.default_rng(sum(n))
    D = len(n)
    lo, hi = [0.1, -0.3, 2.0][:D], [0.9, 0.6, 2.5][:D]
    data = rng.normal(size=n[::-1])
    g = {"dim": D, "n": list(n), "lo": lo, "hi": hi, "data": data}
    ref = G.gradient(g)
    for dt, tol in ((torch.float64, 1e-15), (torch.float32, 2e-6)):
        t = torch.as_tensor(data, dtype=dt).cuda().contiguous()
        _, outs = pdd.grid_gradient(ctx, g, t)
        torch.cuda.synchronize()
        scale = max(np.max(np.abs(r["data"])) for r in ref)
        for d in range(D):
            got = outs[d].cpu().numpy().astype(np.float64)
            if dt == torch.float32:  # the oracle on the same rounded values
                ref32 = G.gradient(dict(g, data=data.astype(np.float32)))
                assert np.max(np.abs(got - ref32[d]["data"])) <= tol * scale, (n, d)
            else:
                assert np.max(np.abs(got - ref[d]["data"])) <= tol * scale, (n, d)


def test_ito_with_finite_difference_gradient(ctx):
    """u~ = U + p known only on a 257^2 grid: its FD gradient serves the Ito
    control variate about as well as the exact gradient of the same u~."""
    pd = W.unit_square_problem(seed=13)
    prob = pdd.Problem(ctx, pd)
    nodes = W.unit_square_nodes()
    exact = W.manufactured_u(pd, nodes)
    gu, _, _ = W.correction_grids(pd, n=257, seed=1, dtype=np.float32)
    tu = torch.as_tensor(gu["data"]).cuda().contiguous()
    fd_grids, fd_t = pdd.grid_gradient(ctx, gu, tu)
    ex = W.gradient_grids(pd, n=257, seed=1, dtype=np.float32)
    ex_t = [torch.as_tensor(g["data"]).cuda().contiguous() for g in ex]
    n = 20000
    a = pdd.stats_to_numpy(pdd.solve_ito(prob, fd_grids, fd_t, nodes, dt=1e-3, n_paths=n, precision="fp32"))
    b = pdd.stats_to_numpy(pdd.solve_ito(prob, ex, ex_t, nodes, dt=1e-3, n_paths=n, precision="fp32"))
    assert np.array_equal(a["mean_plain"], b["mean_plain"])  # the same paths
    assert np.all(a["vr"] > 0.8 * b["vr"]), (a["vr"], b["vr"])
    assert np.all(np.abs(a["mean"] - exact) <= 3 * a["stderr"] + 6e-3)
    prob.close()


def test_gradient_rejects_bad_grids(ctx):
    t = torch.zeros((2, 5), dtype=torch.float32).cuda()
    with pytest.raises(pdd.PDDError):
        pdd.grid_gradient(ctx, {"dim": 2, "n": [5, 2], "lo": [0, 0], "hi": [1, 1]}, t)  # n < 3
    t = torch.zeros((5, 5), dtype=torch.float32).cuda()
    with pytest.raises(pdd.PDDError):
        pdd.grid_gradient(ctx, {"dim": 2, "n": [5, 5], "lo": [0, 1], "hi": [1, 1]}, t)  # lo = hi


@pytest.mark.parametrize("case", ["unit", "box3d", "paper"])
def test_residual_matches_oracle(ctx, case):
    from test_gpu_parity import geometry_case
    rng = np.random.default_rng(5)
    if case == "unit":
        pd = W.unit_square_problem(seed=0)
        n = (65, 33)
    elif case == "box3d":
        pd, _ = geometry_case("box3d")
        n = (9, 12, 7)
    else:
        pd = W.paper_example_problem(n=129)
        n = (40, 40)
    D = pd["dim"]
    lo, hi = W.bounding_box(pd)
    u = rng.normal(size=n[::-1]) * 0.1 + 1.0
    g = {"dim": D, "n": list(n), "lo": lo, "hi": hi, "data": u}
    ref = G.residual(pd, g)
    prob = pdd.Problem(ctx, pd)
    for dt, tol in ((torch.float64, 1e-9), (torch.float32, 2e-6)):
        t = torch.as_tensor(u, dtype=dt).cuda().contiguous()
        _, r = pdd.grid_residual(prob, g, t)
        got = r.cpu().numpy().astype(np.float64)
        want = ref if dt == torch.float64 else G.residual(pd, dict(g, data=u.astype(np.float32)))
        scale = np.max(np.abs(want))
        assert np.max(np.abs(got - want)) <= tol * scale, (case, dt, np.max(np.abs(got - want)), scale)
    prob.close()


def test_correction_with_finite_difference_residual(ctx):
    """u~ = U + p known only on a 257^2 grid: its FD residual serves the
    correction estimator about as well as the exact residual."""
    pd = W.unit_square_problem(seed=13)
    prob = pdd.Problem(ctx, pd)
    nodes = W.unit_square_nodes()
    exact = W.manufactured_u(pd, nodes)
    gu, gr, _ = W.correction_grids(pd, n=257, seed=1, dtype=np.float32)
    tu = torch.as_tensor(gu["data"]).cuda().contiguous()
    tr = torch.as_tensor(gr["data"]).cuda().contiguous()
    fd_g, fd_t = pdd.grid_residual(prob, gu, tu)
    n = 20000
    a = pdd.stats_to_numpy(pdd.solve_correction(prob, gu, tu, fd_g, fd_t, nodes, dt=1e-3, n_paths=n,
                                                precision="fp32", plain_alongside=True))
    b = pdd.stats_to_numpy(pdd.solve_correction(prob, gu, tu, gr, tr, nodes, dt=1e-3, n_paths=n,
                                                precision="fp32", plain_alongside=True))
    assert np.array_equal(a["mean_plain"], b["mean_plain"])  # the same paths
    assert np.all(a["vr"] > 0.5 * b["vr"]), (a["vr"], b["vr"])
    assert np.all(np.abs(a["mean"] - exact) <= 3 * a["stderr"] + 1e-3)
    prob.close()


def test_residual_rejects_bad_grids(ctx):
    prob = pdd.Problem(ctx, W.unit_square_problem(seed=0))
    t = torch.zeros((3, 5), dtype=torch.float32).cuda()
    with pytest.raises(pdd.PDDError):
        pdd.grid_residual(prob, {"dim": 2, "n": [5, 3], "lo": [0, 0], "hi": [1, 1]}, t)  # n < 4
    t3 = torch.zeros((4, 4, 4), dtype=torch.float32).cuda()
    with pytest.raises(pdd.PDDError):
        pdd.grid_residual(prob, {"dim": 3, "n": [4, 4, 4], "lo": [0, 0, 0], "hi": [1, 1, 1]}, t3)  # dim mismatch
    prob.close()
