"""The stored oracle records of the [0, 4]^2 workload (paths 0..63 of all
1,792 nodes, h = 1e-4; written by tests/golden/make_c2_golden.py, which calls
only the oracle) still are what the oracle computes: sampled paths are walked
again and must match bit for bit, and the node means of the 64 stored paths
are consistent with the manufactured solution (Sec. 2.2, eq.
F:Statistical_error: the mean lies within q standard errors of u up to the
time-step bias, which at h = 1e-4 is below 1e-3 on this workload)."""
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_paths0_63.npz")


def load():
    z = np.load(GOLDEN)  # allow_pickle stays False
    return {k: z[k] for k in z.files}


def test_golden_matches_the_oracle(orc):
    from paper_1512_02818_amd import workloads as W
    g = load()
    n = int(g["n_paths"])
    pd = W.big_square_problem(seed=int(g["seed"]))
    nodes = W.big_square_nodes()
    assert len(g["steps"]) == len(nodes) * n
    rng = np.random.default_rng(3)
    ni = rng.integers(0, len(nodes), 40)
    pj = rng.integers(0, n, 40)
    rec = orc.run_paths(pd, nodes, ni, pj, h=float(g["h"]))
    slot = ni * n + pj
    assert np.array_equal(rec["steps"].astype(np.uint32), g["steps"][slot])
    assert np.array_equal(rec["phi"], g["phi"][slot])
    assert np.array_equal(rec["capped"].astype(np.uint8), g["capped"][slot])


def test_golden_node_means_against_exact_u():
    from paper_1512_02818_amd import workloads as W
    g = load()
    n = int(g["n_paths"])
    nodes = W.big_square_nodes()
    exact = W.manufactured_u(W.big_square_problem(seed=0), nodes)
    phi = g["phi"].reshape(len(nodes), n)
    mean = np.array([math.fsum(r) / n for r in phi])
    se = phi.std(axis=1, ddof=1) / math.sqrt(n)
    z = np.abs(mean - exact) / se
    assert not g["capped"].any()
    # 64 paths per node: z is roughly |t_63|; 3.5 is exceeded by ~0.1 % of nodes
    assert np.mean(z < 3.5) > 0.99, np.sort(z)[-10:]
    assert np.mean(z) < 1.0
