"""Writes the oracle's per-path records of the [0, 4]^2 throughput workload.

The workload: the unit-square operator (b = (0.5 x, -0.3 y), c = -(1 + |x|^2),
sigma = 1, u = sin(pi x) cos(pi y) + x^2 y) on [0, 4]^2, cut into 8 x 8
subdomains with 16 nodes per interface segment (1,792 nodes), h = 1e-4,
Philox seed 0, RNG stream 0, Brownian-bridge exit test, Gaussian increments
(Sec. 2.3, Alg. 1 and eq. F:E_M). Paths 0 .. 63 of every node are walked by the
CPU oracle alone, in FP64, and their exit steps, capped flags and scores phi
are stored in ``c2_paths0_63.npz`` beside this script. Nothing here touches the
GPU library; the GPU parity test compares its own walks of the same paths
against these records.

Run from the repository root: ``python tests/golden/make_c2_golden.py``
(about 150 s of CPU, spread over the host's cores).
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_paths0_63.npz")
N_PATHS = 64
H = 1e-4
SEED = 0


def _walk(args):
    lo, hi = args
    from oracle import oracle as O
    from paper_1512_02818_amd import workloads as W
    pd = W.big_square_problem(seed=SEED)
    nodes = W.big_square_nodes()
    ni = np.repeat(np.arange(lo, hi, dtype=np.uint32), N_PATHS)
    pj = np.tile(np.arange(N_PATHS, dtype=np.uint64), hi - lo)
    rec = O.run_paths(pd, nodes, ni, pj, h=H)
    return lo, rec["steps"].astype(np.uint32), rec["capped"].astype(np.uint8), rec["phi"].copy()


def main() -> None:
    from oracle import oracle as O
    from paper_1512_02818_amd import workloads as W
    O.build()
    n_nodes = len(W.big_square_nodes())
    chunk = 16
    jobs = [(lo, min(n_nodes, lo + chunk)) for lo in range(0, n_nodes, chunk)]
    steps = np.zeros(n_nodes * N_PATHS, np.uint32)
    capped = np.zeros(n_nodes * N_PATHS, np.uint8)
    phi = np.zeros(n_nodes * N_PATHS, np.float64)
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        for lo, s, c, p in pool.imap_unordered(_walk, jobs):
            sl = slice(lo * N_PATHS, lo * N_PATHS + len(s))
            steps[sl], capped[sl], phi[sl] = s, c, p
            print(f"nodes {lo}..{lo + len(s) // N_PATHS - 1} done", flush=True)
    np.savez_compressed(OUT, steps=steps, capped=capped, phi=phi, n_paths=np.int64(N_PATHS), h=np.float64(H),
                        seed=np.int64(SEED))
    print(f"wrote {OUT}: {len(steps)} paths, {int(steps.sum())} path-steps", flush=True)


if __name__ == "__main__":
    main()
