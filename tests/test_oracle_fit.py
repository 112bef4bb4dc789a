"""Pins of the oracle's fast fit of nodal constants (Sec. 5, heuristic H5, Alg. A:Fitting).

* Normal / identity GLM = ordinary least squares: against numpy's lstsq and
  the textbook standard errors.
* Both families reproduce exactly linear data.
* Gamma / identity GLM: at the reported coefficients the likelihood equations
  hold (sum (y - mu) / mu^2 [1, x] = 0) and the gamma log-likelihood is
  larger than at nearby coefficients.
* The paper's noise models (eqs. F:Noisy_model_moment1, F:Noisy_model_moment2)
  simulated with known constants: the fits recover them without bias, and the
  reported standard errors match the spread over repetitions.
"""
import numpy as np
import pytest

from oracle import fit as F


def test_normal_fit_is_least_squares():
    rng = np.random.default_rng(1)
    x = rng.uniform(1e-3, 1e-2, size=50)
    y = 0.7 + 3.0 * x + rng.normal(0, 0.01, size=50)
    coef, se, _ = F.fit_normal(x, y)
    X = np.stack([np.ones_like(x), x], axis=1)
    ref, res, _, _ = np.linalg.lstsq(X, y, rcond=None)
    assert np.allclose(coef, ref, rtol=1e-10, atol=1e-13)
    cov = res[0] / (len(x) - 2) * np.linalg.inv(X.T @ X)
    assert np.allclose(se, np.sqrt(np.diag(cov)), rtol=1e-8)


@pytest.mark.parametrize("fit", [F.fit_normal, F.fit_gamma])
def test_exact_lines_are_reproduced(fit):
    x = np.linspace(1e-3, 1e-2, 30)
    for a, b in ((0.4, 12.0), (2.5, -40.0), (1e-3, 0.0)):
        coef, se, _ = fit(x, a + b * x)
        assert np.allclose(coef, [a, b], rtol=1e-11, atol=1e-13), (fit.__name__, coef)
        assert np.all(se < 1e-9)


def _gamma_loglik(coef, x, y):
    mu = coef[0] + coef[1] * x
    return np.sum(-y / mu - np.log(mu))


def test_gamma_fit_solves_the_likelihood_equations():
    rng = np.random.default_rng(2)
    x = np.linspace(1e-3, 1e-2, 100)
    N = 1000
    mu = 0.3 + 20.0 * x
    y = rng.gamma((N - 1) / 2, 2 * mu / (N - 1))
    coef, _, it = F.fit_gamma(x, y)
    m = coef[0] + coef[1] * x
    r = (y - m) / (m * m)
    scale = np.sum(np.abs(y - m) / (m * m))
    assert abs(np.sum(r)) < 1e-10 * scale and abs(np.sum(r * x)) < 1e-10 * scale * x.max()
    assert 2 <= it < 100
    best = _gamma_loglik(coef, x, y)
    for d in ((1e-3, 0), (-1e-3, 0), (0, 0.1), (0, -0.1), (1e-3, -0.1)):
        assert _gamma_loglik(coef + np.array(d), x, y) < best
    # a plain least-squares line is a different (worse) gamma fit
    ols, _, _ = F.fit_normal(x, y)
    assert _gamma_loglik(ols, x, y) < best


def test_noise_models_recover_known_constants():
    """The cloud of the paper: M = 100 equispaced h in [1e-3, 1e-2], N = 1000
    paths per h; means ~ N(E0 + beta h, V0 / N), variances ~ (V0 + alpha h)
    chi^2_{N-1} / (N - 1)."""
    rng = np.random.default_rng(3)
    h = np.linspace(1e-3, 1e-2, 100)
    N, E0, beta, V0, alpha = 1000, 0.65, 2.2, 0.37, 4.0
    est = []
    for _ in range(400):
        mean = E0 + beta * h + rng.normal(0, np.sqrt((V0 + alpha * h) / N))
        var = (V0 + alpha * h) * rng.chisquare(N - 1, size=len(h)) / (N - 1)
        tau = 0.1 + 1.5 * h + rng.normal(0, 0.01 / np.sqrt(N), size=len(h))
        c = F.fit_node(h, mean, var, tau)
        est.append([c["E_phi"], c["beta"], c["V_phi"], c["alpha"], c["se_E_phi"], c["se_beta"],
                    c["se_V_phi"], c["se_alpha"], c["E_tau"], c["beta_tau"]])
    est = np.array(est)
    m, s = est.mean(axis=0), est.std(axis=0)
    R = len(est)
    for k, truth in ((0, E0), (1, beta), (2, V0), (3, alpha), (8, 0.1), (9, 1.5)):
        assert abs(m[k] - truth) <= 4 * s[k] / np.sqrt(R), (k, m[k], truth)
    # reported standard errors match the spread of the estimates
    for k, k_se in ((0, 4), (1, 5), (2, 6), (3, 7)):
        assert 0.8 < np.mean(est[:, k_se]) / s[k] < 1.25, (k, np.mean(est[:, k_se]), s[k])


# ---------------------------------------------------------------------------
# The library's host fit (pdd_glm_fit, C ABI, no GPU needed) against the oracle
def _lib_or_skip():
    from paper_1512_02818_amd import pdd
    try:
        pdd.lib()
    except Exception as e:  # noqa: BLE001 - the library is not built here
        pytest.skip(f"library not built: {e}")
    return pdd


@pytest.mark.parametrize("family", ["normal", "gamma"])
def test_library_glm_matches_the_oracle(family):
    pdd = _lib_or_skip()
    rng = np.random.default_rng(11)
    for rep in range(20):
        M = int(rng.integers(3, 120))
        h = np.sort(rng.uniform(1e-4, 1e-2, size=M))
        if family == "normal":
            y = rng.normal(0.3, 0.2) + rng.normal(0, 3) * h + rng.normal(0, 1e-3, size=M)
            ref = F.fit_normal(h, y)
        else:
            N = int(rng.integers(10, 5000))
            y = (rng.uniform(0.05, 2.0) + rng.uniform(0, 50) * h) * rng.chisquare(N - 1, size=M) / (N - 1)
            ref = F.fit_gamma(h, y)
        coef, se, it = pdd.glm_fit(h, y, family)
        assert np.allclose(coef, ref[0], rtol=1e-9, atol=1e-12), (rep, coef, ref[0])
        assert np.allclose(se, ref[1], rtol=1e-7, atol=1e-14), (rep, se, ref[1])
        if family == "normal":
            assert it == 1


def test_library_glm_rejects_bad_input():
    pdd = _lib_or_skip()
    x = np.linspace(1e-3, 1e-2, 5)
    with pytest.raises(pdd.PDDError):
        pdd.glm_fit(x[:2], x[:2])  # n < 3
    with pytest.raises(pdd.PDDError):
        pdd.glm_fit(x, -x, "gamma")  # gamma data must be positive
    with pytest.raises(pdd.PDDError):
        pdd.glm_fit(np.full(5, 1e-3), x)  # x does not span a line
