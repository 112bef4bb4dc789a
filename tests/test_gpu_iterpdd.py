"""The outer iteration (Alg. A:IterPDD) on the unit square's four strips,
through the library: the fitted constants, the schedule (Alg.
A:Scheduling), the levels (plain, then the Ito control variate from the
previous level's u~ built by pdd_stage2) reach the balanced accuracy a0 at
the nodes (eq. F:N_y_h: |error| <= a0 with probability P_q, q = 2), with the
variance reduced at every control-variate level, for fewer path-steps than
PlainPDD(a0)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1512_02818_amd import iterpdd, pdd  # noqa: E402
from paper_1512_02818_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pdd.Context(0)
    yield c
    c.close()


def test_iterpdd_unit_square(ctx):
    pd = W.unit_square_problem(seed=0)
    nodes = W.unit_square_nodes()
    rep = iterpdd.run(ctx, pd, nodes, W.unit_square_partition(129), a0=0.01,
                      exact=lambda p: W.manufactured_u(pd, p), log=print)
    levels = rep["levels"]
    assert len(rep["schedule"]) >= 2, rep["schedule"]
    assert all(b > a for a, b in zip(rep["schedule"], rep["schedule"][1:]))
    assert 1.0 < rep["kappa"] < 4.0
    last = levels[-1]
    assert last["accuracy"] == rep["a0"]
    # balanced accuracy: q SE = a0 / 2 and |bias| ~ a0 / 2 at each node (the
    # plan uses the pilot's variance, so the final SE scatters around its target)
    assert last["max_q_se_over_half_a"] <= 1.5
    assert last["rms_error_nodes"] <= rep["a0"], last
    for r in levels[1:]:
        assert r["control_variate"] and r["mean_vr"] > 1.5, r
    assert rep["speedup_path_steps"] > 1.5, (rep["iterpdd_path_steps"], rep["plainpdd"])
    print({k: rep[k] for k in ("schedule", "kappa", "speedup_path_steps", "speedup_wall")})
