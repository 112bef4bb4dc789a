"""GPU edge cases through the C ABI: empty and ragged inputs, single paths,
the step cap, invalid arguments, resume by path offset, independence of the
launch shape (block size, persistent grid, queue grab, launch chunking) and
run-to-run determinism."""
import math

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


@pytest.fixture(scope="module")
def prob(ctx):
    p = pdd.Problem(ctx, W.unit_square_problem(seed=3))
    yield p
    p.close()


def run(prob, nodes, total, **kw):
    rec = pdd.alloc_records(max(total, 1))
    out = pdd.solve_nodes(prob, nodes, records=rec, **kw)
    torch.cuda.synchronize()
    st = pdd.stats_to_numpy(out)
    return st, {k: (v.cpu().numpy()[:total] if v is not None else None) for k, v in rec.items()}


def test_zero_nodes_is_a_noop(prob):
    out = torch.full((pdd.STATS_DTYPE.itemsize,), 7, dtype=torch.uint8, device="cuda")
    pdd.solve_nodes(prob, np.zeros((0, 2)), out=out, dt=1e-3, n_paths=10)
    torch.cuda.synchronize()
    assert torch.all(out == 7)


def test_ragged_counts_match_oracle_paths(prob):
    from oracle import oracle as O
    nodes = W.unit_square_nodes()[:7]
    counts = np.array([0, 1, 63, 64, 65, 0, 300], dtype=np.uint64)
    total = int(counts.sum())
    for prec in ("fp64", "fp32"):
        st, rec = run(prob, nodes, total, dt=1e-3, n_paths_per_node=counts, precision=prec,
                      path_offset=11)
        assert list(st["n"]) == list(counts)
        assert np.isnan(st["mean"][0]) and np.isnan(st["mean"][5])
        assert np.isnan(st["var"][1]) and not np.isnan(st["mean"][1])
        node_idx = np.repeat(np.arange(len(nodes)), counts.astype(np.int64))
        path_idx = np.concatenate([np.arange(c) for c in counts.astype(np.int64)]) + 11
        orec = O.run_paths(prob.pd, nodes, node_idx, path_idx, h=1e-3)
        same = (rec["steps"].view(np.uint32) & 0x7FFFFFFF) == orec["steps"]
        assert same.mean() > (0.999 if prec == "fp64" else 0.98)
        if prec == "fp64":
            assert np.allclose(rec["phi"][same], orec["phi"][same], rtol=1e-11, atol=1e-12)
        for i in np.nonzero(counts > 1)[0]:
            seg = slice(int(counts[:i].sum()), int(counts[:i + 1].sum()))
            assert st["steps_sum"][i] == int((rec["steps"][seg].view(np.uint32) & 0x7FFFFFFF).sum())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_last_path_indices_and_streams_match_oracle(ctx, prob, prec):
    """The highest valid counters: paths 2^32 - 128 .. 2^32 - 1 under the
    stream ids 2^28 - 1 and 2^28 - 2, solved alone and as two merged items of
    one batch (the per-node RNG table), path for path against the oracle; the
    merged records are bitwise those of the solo solves."""
    from oracle import oracle as O
    nodes = W.unit_square_nodes()[:3]
    n = 64
    cases = [((1 << 28) - 1, (1 << 32) - n), ((1 << 28) - 2, (1 << 32) - 2 * n)]
    solo = []
    for stream, off in cases:
        _, rec = run(prob, nodes, 3 * n, dt=1e-3, n_paths=n, path_offset=off, stream_id=stream, precision=prec)
        solo.append(rec)
        orec = O.run_paths(prob.pd, nodes, np.repeat(np.arange(3), n), np.tile(np.arange(n, dtype=np.uint64) + off, 3),
                           h=1e-3, stream=stream)
        steps = rec["steps"].view(np.uint32) & 0x7FFFFFFF
        same = steps == orec["steps"]
        if prec == "fp64":
            assert (~same).sum() <= 1, np.nonzero(~same)
            assert np.allclose(rec["phi"][same], orec["phi"][same], rtol=1e-11, atol=1e-12)
        else:
            assert same.mean() >= 0.95, same.mean()
            scale = np.maximum(1.0, np.abs(orec["phi"][same]))
            assert np.max(np.abs(rec["phi"][same] - orec["phi"][same]) / scale) < 2e-3
    recs = [pdd.alloc_records(3 * n) for _ in cases]
    pdd.solve_batch(ctx, [{"problem": prob, "nodes": nodes,
                           "opts": dict(dt=1e-3, n_paths=n, path_offset=off, stream_id=stream, precision=prec,
                                        records=r)} for (stream, off), r in zip(cases, recs)])
    torch.cuda.synchronize()
    for r, ref in zip(recs, solo):
        assert r["phi"].cpu().numpy()[:3 * n].tobytes() == ref["phi"].tobytes()
        assert r["steps"].cpu().numpy()[:3 * n].tobytes() == ref["steps"].tobytes()


def test_step_cap(prob):
    nodes = W.unit_square_nodes()[:3]
    st, rec = run(prob, nodes, 3 * 500, dt=1e-3, n_paths=500, max_steps=9, precision="fp64")
    steps = rec["steps"].view(np.uint32)
    capped = steps >> 31
    assert np.all((steps & 0x7FFFFFFF) <= 9)
    assert np.all((steps[capped == 1] & 0x7FFFFFFF) == 9)
    assert st["n_capped"].sum() == capped.sum() > 0
    # odd cap lands between the two steps that share a Philox block; same as the oracle
    from oracle import oracle as O
    ost, orec = O.solve_nodes(prob.pd, nodes, record=True, h=1e-3, n_paths=500, max_steps=9)
    assert np.array_equal(steps & 0x7FFFFFFF, orec["steps"].astype(np.uint32))
    assert np.array_equal(capped, orec["capped"].astype(np.uint32))


@pytest.mark.parametrize("bad", ["outside", "on_boundary", "dt", "nan", "grid_dtype", "grid_cover",
                                 "stream", "offset", "tuning"])
def test_invalid_arguments_are_rejected(ctx, prob, bad):
    nodes = W.unit_square_nodes()[:2].copy()
    kw = dict(dt=1e-3, n_paths=10)
    if bad == "outside":
        nodes[1] = [1.2, 0.5]
    elif bad == "on_boundary":
        nodes[0] = [0.0, 0.5]
    elif bad == "dt":
        kw["dt"] = 0.0
    elif bad == "nan":
        nodes[0, 0] = np.nan
    elif bad == "stream":
        kw["stream_id"] = 1 << 28
    elif bad == "offset":
        kw["path_offset"] = (1 << 32) - 5
    elif bad == "tuning":
        kw["tuning"] = (96, 0, 64, 0)
    if bad in ("grid_dtype", "grid_cover"):
        g = W.sampled_grid(prob.pd, lambda p: np.zeros(len(p)), n=9, dtype=np.float64)
        if bad == "grid_cover":
            g["lo"] = [0.1, 0.0]
        t = torch.zeros(81, dtype=torch.float64, device="cuda")
        prec = "fp32" if bad == "grid_dtype" else "fp64"
        with pytest.raises(pdd.PDDError) as ei:
            pdd.solve_correction(prob, g, t, g, t, nodes, precision=prec, **kw)
        assert ei.value.status == (-4 if bad == "grid_dtype" else -1)
        return
    with pytest.raises(pdd.PDDError) as ei:
        pdd.solve_nodes(prob, nodes, **kw)
    assert ei.value.status == -1
    assert pdd.lib().pdd_last_error()


def test_invalid_problems_are_rejected(ctx):
    for mutate in (lambda p: p.update(dim=4), lambda p: p.update(sigma=0.0),
                   lambda p: p.update(lo=[1.0, 0.0], hi=[0.0, 1.0]),
                   lambda p: p["mono"].append({"coef": 1.0, "e": [9, 0]})):
        pd = W.unit_square_problem()
        mutate(pd)
        with pytest.raises(pdd.PDDError):
            pdd.Problem(ctx, pd)


def test_resume_by_path_offset_is_the_same_paths(prob):
    nodes = W.unit_square_nodes()[4:9]
    n, a = 700, 333
    _, full = run(prob, nodes, 5 * n, dt=1e-3, n_paths=n)
    _, r1 = run(prob, nodes, 5 * a, dt=1e-3, n_paths=a)
    _, r2 = run(prob, nodes, 5 * (n - a), dt=1e-3, n_paths=n - a, path_offset=a)
    for i in range(5):
        joined = np.concatenate([r1["phi"][i * a:(i + 1) * a], r2["phi"][i * (n - a):(i + 1) * (n - a)]])
        assert joined.tobytes() == full["phi"][i * n:(i + 1) * n].tobytes()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_launch_shape_does_not_change_results(prob, prec):
    nodes = W.unit_square_nodes()
    n = 3000
    ref_st, ref = run(prob, nodes, 18 * n, dt=1e-3, n_paths=n, precision=prec)
    for tune in ((64, 1, 1, 0), (128, 3, 7, 0), (256, 0, 1024, 0), (256, 2, 64, 0)):
        st, rec = run(prob, nodes, 18 * n, dt=1e-3, n_paths=n, precision=prec, tuning=tune)
        assert rec["phi"].tobytes() == ref["phi"].tobytes(), tune
        assert rec["steps"].tobytes() == ref["steps"].tobytes(), tune
        assert st.tobytes() == ref_st.tobytes(), tune


def test_chunked_launches_and_scratch_records(prob):
    """Without caller records the library keeps records in scratch and may
    cut the solve into several launches; statistics agree with one launch."""
    nodes = W.unit_square_nodes()
    n = 2500
    one = pdd.stats_to_numpy(pdd.solve_nodes(prob, nodes, dt=1e-3, n_paths=n))
    for cap in (4096, 10007, 1 << 20):
        st = pdd.stats_to_numpy(pdd.solve_nodes(prob, nodes, dt=1e-3, n_paths=n,
                                                tuning=(256, 0, 64, cap)))
        assert np.array_equal(st["n"], one["n"]) and np.array_equal(st["steps_sum"], one["steps_sum"])
        assert np.allclose(st["mean"], one["mean"], rtol=1e-14, atol=1e-15)
        assert np.allclose(st["var"], one["var"], rtol=1e-12)


def test_repeat_runs_are_bitwise_identical(prob):
    nodes = W.unit_square_nodes()
    a = pdd.stats_to_numpy(pdd.solve_nodes(prob, nodes, dt=1e-3, n_paths=4000))
    b = pdd.stats_to_numpy(pdd.solve_nodes(prob, nodes, dt=1e-3, n_paths=4000))
    assert a.tobytes() == b.tobytes()


def test_kernel_times_reported(ctx, prob):
    pdd.kernel_times(ctx)
    for _ in range(3):
        pdd.solve_nodes(prob, W.unit_square_nodes(), dt=1e-3, n_paths=500, time_kernel=True)
    pdd.solve_nodes(prob, W.unit_square_nodes(), dt=1e-3, n_paths=500)
    ms = pdd.kernel_times(ctx)
    assert len(ms) == 3 and all(t > 0 for t in ms)
    assert pdd.kernel_times(ctx) == []


def test_long_node_segments_are_reduced_in_chunks(prob):
    """Node segments longer than one reduction chunk (65,536 paths) are summed
    chunk by chunk and merged in chunk order; the sums still agree with the
    per-path records, and scratch and caller records give the same bits."""
    nodes = W.unit_square_nodes()[:3]
    counts = np.array([150_001, 10, 70_000], dtype=np.uint64)
    total = int(counts.sum())
    st, rec = run(prob, nodes, total, dt=1e-3, n_paths_per_node=counts, precision="fp32")
    scratch = pdd.stats_to_numpy(pdd.solve_nodes(prob, nodes, dt=1e-3, n_paths_per_node=counts,
                                                 precision="fp32"))
    assert scratch.tobytes() == st.tobytes()
    ends = np.cumsum(counts.astype(np.int64))
    for i in range(3):
        seg = slice(int(ends[i] - counts[i]), int(ends[i]))
        phi = rec["phi"][seg].astype(np.float64)
        steps = rec["steps"][seg].view(np.uint32)
        assert st["n"][i] == counts[i]
        assert st["steps_sum"][i] == int((steps & 0x7FFFFFFF).astype(np.int64).sum())
        assert st["n_capped"][i] == int((steps >> 31).sum())
        s1 = st["sums"][i][0] + st["sums"][i][1]
        s2 = st["sums"][i][2] + st["sums"][i][3]
        assert abs(s1 - math.fsum(phi)) <= 1e-12 * max(1.0, abs(math.fsum(np.abs(phi))))
        assert abs(s2 - math.fsum(phi * phi)) <= 1e-12 * max(1.0, math.fsum(phi * phi))
    # a launch cap that cuts the long node: same counts, sums to rounding
    cut = pdd.stats_to_numpy(pdd.solve_nodes(prob, nodes, dt=1e-3, n_paths_per_node=counts,
                                             precision="fp32", tuning=(256, 0, 64, 100_003)))
    assert np.array_equal(cut["n"], st["n"]) and np.array_equal(cut["steps_sum"], st["steps_sum"])
    assert np.allclose(cut["mean"], st["mean"], rtol=1e-14, atol=1e-15)


def test_fp32_trig_range_is_checked(ctx):
    """FP32 paths evaluate the trig terms with the hardware sine, whose input
    must stay within +-256 revolutions: a problem whose k x + phase exceeds
    that over the domain is refused for FP32 paths (PDD_E_UNSUPPORTED) and
    solved in FP64; one just inside the range runs in both."""
    base = W.unit_square_problem(seed=0)
    nodes = W.unit_square_nodes()[:2]
    # k x over [0, 1]: 2 pi * 300 revolutions at x = 1
    far = dict(base, trig=[{"amp": 1e-3, "k": [2 * np.pi * 300.0, np.pi], "phase": [0.0, 0.0]}])
    near = dict(base, trig=[{"amp": 1e-3, "k": [2 * np.pi * 200.0, np.pi], "phase": [0.0, 0.0]}])
    p = pdd.Problem(ctx, far)
    with pytest.raises(pdd.PDDError) as e:
        pdd.solve_nodes(p, nodes, dt=1e-3, n_paths=64, precision="fp32")
    assert e.value.status == -4 and "revolutions" in str(e.value)
    st = pdd.stats_to_numpy(pdd.solve_nodes(p, nodes, dt=1e-3, n_paths=64, precision="fp64"))
    assert np.all(st["n"] == 64)
    p.close()
    p = pdd.Problem(ctx, near)
    for prec in ("fp32", "fp64"):
        st = pdd.stats_to_numpy(pdd.solve_nodes(p, nodes, dt=1e-3, n_paths=64, precision=prec))
        assert np.all(st["n"] == 64)
    p.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_paths_ending_before_their_first_step(prob, prec):
    """Nodes inside the shifted test's band (distance <= 0.5826 sigma sqrt(h)
    from the boundary, Alg. 1) end every path before its first step, so whole
    waves end 64 paths at one refill turn (a full batch of ended paths waiting
    to be scored at once) while waves on the other nodes walk. Exit steps and
    scores match the oracle path by path (FP64: scores to 1e-11; FP32: the
    in-band scores are g at the projected point, within FP32 rounding), and
    the records are bitwise the same at refill periods 1 and 8."""
    from oracle import oracle as O
    h = 1e-3
    band = 0.5826 * math.sqrt(h)  # sigma = 1
    nodes = np.array([[0.4 * band, 0.5], [0.3, 0.4], [0.5, 1.0 - 0.7 * band], [0.2 * band, 0.3 * band]])
    n = 640
    recs = []
    for refill in (1, 8):
        st, rec = run(prob, nodes, len(nodes) * n, dt=h, n_paths=n, precision=prec, exit="shift",
                      tuning=(256, 0, 64, 0, refill, 0))
        assert list(st["n"]) == [n] * len(nodes)
        recs.append(rec)
    assert recs[0]["phi"].tobytes() == recs[1]["phi"].tobytes()
    assert recs[0]["steps"].tobytes() == recs[1]["steps"].tobytes()
    ost, orec = O.solve_nodes(prob.pd, nodes, record=True, h=h, n_paths=n, exit="shift")
    steps = recs[0]["steps"].view(np.uint32) & 0x7FFFFFFF
    in_band = np.repeat([True, False, True, True], n)
    assert np.all(steps[in_band] == 0) and np.all(orec["steps"][in_band] == 0)
    same = steps == orec["steps"].astype(np.uint32)
    if prec == "fp64":
        assert same.mean() >= 0.9999, same.mean()
    phi, ophi = recs[0]["phi"], orec["phi"]
    tol = 1e-11 if prec == "fp64" else 1e-5
    ok = same if prec == "fp64" else in_band
    assert np.all(np.abs(phi[ok] - ophi[ok]) <= tol * np.maximum(1.0, np.abs(ophi[ok]))), \
        np.max(np.abs(phi[ok] - ophi[ok]))
