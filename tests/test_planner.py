"""Path-count planner of the balanced simulation (Sec. 3.1, Def.
D:Balanced_MC_simulation, eq. F:N_y_h), through the C ABI; host only."""
import math

import numpy as np
import pytest

from paper_1512_02818_amd import pdd


@pytest.fixture(scope="module")
def built():
    import os
    if not os.path.exists(pdd.LIB_PATH):
        from paper_1512_02818_amd import build
        build.build()
    return pdd.lib()


def pilot(n, var):
    p = np.zeros(len(var), dtype=pdd.STATS_DTYPE)
    p["n"] = n
    p["var"] = var
    return p


def test_balanced_rule(built):
    # accuracy a at confidence q: q SE = a / 2, so N = 4 q^2 V / a^2
    a, q = 1e-2, 3.0
    var = np.array([0.5, 2.0, 1e-3, 0.0, 7.25])
    got = pdd.plan_paths(pilot(1000, var), a / (2 * q), n_max=1 << 40)
    want = [max(1000, math.ceil(4 * q * q * v / (a * a))) for v in var]
    assert list(got) == want


def test_clamps_and_exact_ceiling(built):
    se = 0.25
    var = np.array([0.0625 * 3, 0.0625 * 3 + 1e-12, 1e6, 1e-9])
    got = pdd.plan_paths(pilot([10, 10, 10, 50], var), se, n_max=10_000)
    assert list(got) == [10, 10, 10_000, 50]  # 3 -> pilot floor 10; huge -> cap; tiny -> pilot n
    got = pdd.plan_paths(pilot([2, 2], [16 * 0.0625, 16 * 0.0625 * (1 + 1e-15)]), se, n_max=100)
    assert list(got) == [16, 17]


@pytest.mark.parametrize("bad", ["n1", "nan", "neg", "se0", "seinf"])
def test_rejects(built, bad):
    p = pilot(100, [1.0, 2.0])
    se = 0.1
    if bad == "n1":
        p["n"][1] = 1
    elif bad == "nan":
        p["var"][0] = np.nan
    elif bad == "neg":
        p["var"][0] = -1.0
    elif bad == "se0":
        se = 0.0
    else:
        se = np.inf
    with pytest.raises(pdd.PDDError) as ei:
        pdd.plan_paths(p, se, n_max=1000)
    assert ei.value.status == -1


def test_empty(built):
    assert len(pdd.plan_paths(pilot(5, np.zeros(0)), 0.1, 10)) == 0
