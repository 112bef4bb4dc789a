"""The library's scheduling algorithm (pdd_schedule, host only: Alg.
A:Scheduling with the sensitivity formula, eq. F:Sensitivity_formula) against
the oracle's brute-force minimisation, and on the closed-form minimiser of a
single uncorrelated node."""
import numpy as np
import pytest

from oracle import stage2 as S2
from paper_1512_02818_amd import pdd


@pytest.fixture(scope="module")
def built():
    import os
    if not os.path.exists(pdd.LIB_PATH):
        from paper_1512_02818_amd import build
        build.build()
    return pdd.lib()


def test_single_node_closed_form(built):
    K, V, Vpsi, kappa, delta, a0 = 2.0, 0.4, 30.0, 1.8, 1.0, 0.01
    p = 2 + 1 / delta
    a_star = (2 * p * V * a0 ** p / (kappa * Vpsi)) ** (1 / (p + 2))
    a, s = pdd.schedule([K], [V], [0.0], [1.0], [Vpsi], [0.0], a0, kappa, delta, a_max=2.0, max_levels=1)
    assert len(a) == 2 and abs(a[1] / a_star - 1) < 1e-6, (a, a_star)
    want_s = K * V / S2.schedule_cost(a_star, a0, [K], [V], [Vpsi], [0.0], [0.0], [1.0], kappa, delta)
    assert abs(s[0] / want_s - 1) < 1e-6


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_matches_the_oracle(built, seed):
    rng = np.random.default_rng(seed)
    n = 18
    K = rng.uniform(0.5, 3.0, n)
    V = rng.uniform(0.1, 1.0, n)
    alpha = rng.uniform(-2, 2, n)
    beta = rng.uniform(0.5, 4, n) * rng.choice([-1, 1], n)
    Vpsi = rng.uniform(0.5, 20, n)
    rho = rng.uniform(-0.5, 0.5, n)
    a0, kappa = 0.0025 * (1 + seed), 1.8
    a, s = pdd.schedule(K, V, alpha, beta, Vpsi, rho, a0, kappa, 1.0, a_max=1.0, s_min=1.5)
    ref = S2.schedule(a0, K, V, Vpsi, rho, alpha, beta, kappa, 1.0, a_max=1.0, s_min=1.5)
    assert len(a) == len(ref) and len(a) >= 2, (a, ref)
    for x, y in zip(a, ref):
        assert abs(x / y - 1) < 4e-3, (a, ref)
    # the library's minimum is at least as low as the brute-force one
    for j in range(1, len(a)):
        f_lib = S2.schedule_cost(a[j], a[j - 1], K, V, Vpsi, rho, alpha, beta, kappa, 1.0)
        f_ref = S2.schedule_cost(ref[j], a[j - 1], K, V, Vpsi, rho, alpha, beta, kappa, 1.0)
        assert f_lib <= f_ref * (1 + 1e-9)


def test_bad_arguments(built):
    with pytest.raises(pdd.PDDError):
        pdd.schedule([1.0], [0.5], [0.0], [0.0], [1.0], [0.0], 0.01, 1.8)  # beta = 0
    with pytest.raises(pdd.PDDError):
        pdd.schedule([1.0], [0.5], [0.0], [1.0], [1.0], [0.0], 2.0, 1.8, a_max=1.0)  # a0 >= a_max
