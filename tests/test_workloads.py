"""Synthetic input generators (no method arithmetic): grid layout, the
separable perturbation on grids, the serving request stream."""
import numpy as np

from paper_1512_02818_amd import workloads as W


def test_grid_points_x_fastest():
    p = W.grid_points((3, 2), [0, 0], [1, 1])
    assert np.allclose(p[:4], [[0, 0], [0.5, 0], [1, 0], [0, 1]])
    q = W.grid_points((2, 3, 2), [0, 0, 0], [1, 2, 3])
    assert q.shape == (12, 3)
    assert np.allclose(q[1], [1, 0, 0]) and np.allclose(q[2], [0, 1, 0]) and np.allclose(q[6], [0, 0, 3])


def test_separable_perturbation_matches_pointwise():
    for D, shape in ((2, (9, 7)), (3, (5, 6, 7))):
        lo, hi = [0.1] * D, [1.7] * D
        pert = W.fourier_perturbation(3, dim=D)
        pts = W.grid_points(shape, lo, hi)
        for a, b in zip(W._pert_eval(pert, pts, lo, hi), W._pert_grid(pert, shape, lo, hi)):
            assert np.allclose(a, b, rtol=0, atol=1e-13)


def test_correction_grid_residual_by_finite_differences():
    # r = -(1/2 sigma^2 Lap p + b.grad p + c p) at a grid point (3D), with the
    # derivatives of p taken by central differences of its values
    rng = np.random.default_rng(2)
    pd = W.random_problem(rng, dim=3)
    n = 33
    gu, gr, pert = W.correction_grids(pd, n=n, seed=4, dtype=np.float64)
    L = pd["hi"][0] - pd["lo"][0]
    i = (10, 12, 17)  # z, y, x
    x = np.array([pd["lo"][0] + L / (n - 1) * i[2], pd["lo"][1] + L / (n - 1) * i[1],
                  pd["lo"][2] + L / (n - 1) * i[0]])
    h = 1e-4 * L

    def p(pt):
        return W._pert_eval(pert, np.atleast_2d(pt), pd["lo"], pd["hi"])[0][0]

    E = np.eye(3)
    lap = sum((p(x + h * E[d]) - 2 * p(x) + p(x - h * E[d])) / h ** 2 for d in range(3))
    grad = np.array([(p(x + h * E[d]) - p(x - h * E[d])) / (2 * h) for d in range(3)])
    b = np.asarray(pd["b0"]) + np.asarray(pd["B"]) @ x
    c = pd["c_a"] + pd["c_b"] * x @ x
    r_fd = -(0.5 * pd["sigma"] ** 2 * lap + b @ grad + c * p(x))
    assert abs(r_fd - gr["data"][i]) < 1e-4 * (abs(gr["data"][i]) + 1e-3)
    assert np.isclose(gu["data"][i] - W.manufactured_u(pd, x[None, :])[0], p(x), rtol=0, atol=1e-14)


def test_correction_grids_with_one_size_per_axis():
    # n given per axis: data indexed [z, y, x] with x fastest, the point of
    # index (i, j, k) at lo + (i, j, k) (hi - lo) / (n - 1)
    rng = np.random.default_rng(3)
    pd = W.random_problem(rng, dim=3)
    shape = (9, 13, 11)
    gu, gr, pert = W.correction_grids(pd, n=shape, seed=4, dtype=np.float64)
    assert gu["n"] == list(shape) and gu["data"].shape == shape[::-1] == gr["data"].shape
    lo, hi = np.asarray(pd["lo"]), np.asarray(pd["hi"])
    for idx in ((0, 0, 0), (8, 12, 10), (3, 7, 5)):
        x = lo + np.asarray(idx) * (hi - lo) / (np.asarray(shape) - 1)
        p = W._pert_eval(pert, x[None, :], pd["lo"], pd["hi"])[0][0]
        u = W.manufactured_u(pd, x[None, :])[0]
        assert np.isclose(gu["data"][idx[::-1]], u + p, rtol=0, atol=1e-13)


def test_serving_stream():
    problems, reqs = W.serving_stream(seed=5, rate=200.0, duration=5.0)
    assert 900 < len(reqs) < 1100  # Poisson(1000)
    t = np.array([r["t"] for r in reqs])
    assert np.all(np.diff(t) > 0) and t[-1] <= 5.0
    cv = np.mean([r["cv"] for r in reqs])
    assert 0.25 < cv < 0.35
    n = np.array([len(r["nodes"]) for r in reqs])
    assert n.min() >= 1 and n.max() <= 2000
    for r in reqs[:50]:
        pd = problems[r["problem"]]
        assert np.all(r["nodes"] > pd["lo"][0]) and np.all(r["nodes"] < pd["hi"][0])
        assert np.isclose(r["target_se"], r["tol"] / np.sqrt(2))
        if r["cv"]:
            assert r["grid_n"] in ((129, 257, 513) if pd["dim"] == 2 else (65,))
    assert len({r["stream_id"] for r in reqs}) == len(reqs)
    # same seed, same stream
    _, again = W.serving_stream(seed=5, rate=200.0, duration=5.0)
    assert all(np.array_equal(a["nodes"], b["nodes"]) for a, b in zip(reqs, again))
