"""Plain reference of the fast fit of nodal constants (paper, Sec. 5 heuristic H5 and
Alg. A:Fitting).

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this module; it shares no code with
the GPU library.

Model of the first moments (eq. F:Noisy_model_moment1): the sample mean of
eta_h over N^ paths at step h is E[eta_0] + B1 h^delta plus Gaussian noise, a
generalised linear model with normal noise and identity link in the regressor
x = h^delta. Model of the second moments (eq. F:Noisy_model_moment2): the
sample variance is B2 h^delta + V[eta_0] chi^2_{N^-1}/(N^-1), i.e. Gamma noise
with the identity link. Each fit returns (intercept, slope), their standard
errors, and the number of scoring iterations.

Both fits are maximum likelihood for their family, written out:
  normal:  least squares through the normal equations of the 2-column design;
  gamma:   iteratively reweighted least squares (Fisher scoring) with the
           gamma variance function V(mu) = mu^2 and the identity link, so the
           working response is y itself and the weights are 1 / mu^2.
Standard errors: sqrt(dispersion * diag((X' W X)^-1)), the dispersion
estimated from the Pearson residuals with n - 2 degrees of freedom.
"""
from __future__ import annotations

import numpy as np


def _weighted_ls(x, y, w):
    """Solves the 2x2 normal equations of sum w (y - a - b x)^2."""
    s0, s1, s2 = np.sum(w), np.sum(w * x), np.sum(w * x * x)
    t0, t1 = np.sum(w * y), np.sum(w * x * y)
    det = s0 * s2 - s1 * s1
    a = (s2 * t0 - s1 * t1) / det
    b = (s0 * t1 - s1 * t0) / det
    inv = np.array([[s2, -s1], [-s1, s0]]) / det
    return np.array([a, b]), inv


def fit_normal(x, y):
    """Normal / identity GLM of y on [1, x]: (coef, se, iterations)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    coef, inv = _weighted_ls(x, y, np.ones_like(x))
    r = y - (coef[0] + coef[1] * x)
    disp = np.sum(r * r) / (len(x) - 2)
    return coef, np.sqrt(disp * np.diag(inv)), 1


def fit_gamma(x, y, max_iter=100, tol=1e-13):
    """Gamma / identity GLM of y > 0 on [1, x] by Fisher scoring, started from
    mu = y: (coef, se, iterations). A step that would make a mean non-positive
    is halved until it does not."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    coef, _ = _weighted_ls(x, y, 1.0 / (y * y))  # the first scoring step from mu = y
    it = 1
    while it < max_iter:
        mu = coef[0] + coef[1] * x
        new, _ = _weighted_ls(x, y, 1.0 / (mu * mu))
        step = 1.0
        while np.any(new[0] + new[1] * x <= 0) and step > 1e-6:
            step *= 0.5
            new = coef + step * (new - coef)
        it += 1
        done = np.all(np.abs(new - coef) <= tol * np.abs(new))
        coef = new
        if done:
            break
    mu = coef[0] + coef[1] * x
    _, inv = _weighted_ls(x, y, 1.0 / (mu * mu))
    disp = np.sum(((y - mu) / mu) ** 2) / (len(x) - 2)
    return coef, np.sqrt(disp * np.diag(inv)), it


def fit_node(h, mean_phi, var_phi, mean_tau, delta=1.0):
    """The nodal constants of Alg. A:Fitting from a cloud of M^ steps h_j and
    the per-step sample mean and variance of phi and mean exit time:
    E[phi_0], beta (normal fit), V[phi_0], alpha (gamma fit), E[tau_0] and its
    slope (normal fit), as a dict."""
    x = np.asarray(h, dtype=np.float64) ** delta
    (e0, beta), se_e, _ = fit_normal(x, mean_phi)
    (v0, alpha), se_v, it = fit_gamma(x, var_phi)
    (t0, bt), se_t, _ = fit_normal(x, mean_tau)
    return {"E_phi": e0, "beta": beta, "se_E_phi": se_e[0], "se_beta": se_e[1],
            "V_phi": v0, "alpha": alpha, "se_V_phi": se_v[0], "se_alpha": se_v[1],
            "E_tau": t0, "beta_tau": bt, "se_E_tau": se_t[0], "iterations": it}
