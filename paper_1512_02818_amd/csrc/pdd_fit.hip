// Fast fit of nodal constants (paper, Sec. 5 heuristic H5 and Alg. A:Fitting): one
// batched launch over a cloud of time steps, then per node a normal /
// identity GLM of the means and a gamma / identity GLM of the variances in
// x = h^delta (eqs. F:Noisy_model_moment1, F:Noisy_model_moment2). The fits
// are host code over a few hundred numbers per node.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "host_runtime.hpp"
#include "pdd.h"

using pdd::fail;

namespace {

// Minimiser of sum w (y - c0 - c1 x)^2 and the inverse of its 2x2 normal
// matrix (for the standard errors). Returns false when the matrix is singular.
bool weighted_line(const double *x, const double *y, const double *w, int n, double c[2], double inv[3])
{
    double s0 = 0, s1 = 0, s2 = 0, t0 = 0, t1 = 0;
    for (int i = 0; i < n; ++i) {
        s0 += w[i];
        s1 += w[i] * x[i];
        s2 += w[i] * x[i] * x[i];
        t0 += w[i] * y[i];
        t1 += w[i] * x[i] * y[i];
    }
    const double det = s0 * s2 - s1 * s1;
    // relative to s0 s2, det is the weighted spread of x; below 1e-12 the x
    // values do not determine a slope
    if (!(std::fabs(det) > 1e-12 * std::fabs(s0 * s2)) || !std::isfinite(det)) return false;
    c[0] = (s2 * t0 - s1 * t1) / det;
    c[1] = (s0 * t1 - s1 * t0) / det;
    inv[0] = s2 / det;  // (0,0)
    inv[1] = -s1 / det; // (0,1)
    inv[2] = s0 / det;  // (1,1)
    return true;
}

pdd_status glm(const double *x, const double *y, int n, int family, double coef[2], double se[2], int *iters)
{
    std::vector<double> w(n, 1.0), mu(n);
    double inv[3];
    int it = 1;
    if (family == PDD_GLM_NORMAL) {
        if (!weighted_line(x, y, w.data(), n, coef, inv)) return fail(PDD_E_INVALID, "the x values do not span a line");
    } else {
        for (int i = 0; i < n; ++i) w[i] = 1.0 / (y[i] * y[i]);  // scoring from mu = y
        if (!weighted_line(x, y, w.data(), n, coef, inv)) return fail(PDD_E_INVALID, "the x values do not span a line");
        bool done = false;
        while (!done && it < 100) {
            for (int i = 0; i < n; ++i) {
                mu[i] = coef[0] + coef[1] * x[i];
                w[i] = 1.0 / (mu[i] * mu[i]);
            }
            double nc[2];
            if (!weighted_line(x, y, w.data(), n, nc, inv)) return fail(PDD_E_INTERNAL, "gamma fit: singular weights");
            // halve a step that would leave a mean outside (0, inf)
            for (int k = 0; k < 20; ++k) {
                bool ok = true;
                for (int i = 0; i < n && ok; ++i) ok = nc[0] + nc[1] * x[i] > 0.0;
                if (ok) break;
                nc[0] = coef[0] + 0.5 * (nc[0] - coef[0]);
                nc[1] = coef[1] + 0.5 * (nc[1] - coef[1]);
            }
            ++it;
            done = std::fabs(nc[0] - coef[0]) <= 1e-13 * std::fabs(nc[0]) &&
                   std::fabs(nc[1] - coef[1]) <= 1e-13 * std::fabs(nc[1]);
            coef[0] = nc[0];
            coef[1] = nc[1];
        }
        // the information matrix at the converged means (the coefficients stay)
        for (int i = 0; i < n; ++i) {
            mu[i] = coef[0] + coef[1] * x[i];
            w[i] = 1.0 / (mu[i] * mu[i]);
        }
        double unused[2];
        if (!weighted_line(x, y, w.data(), n, unused, inv)) return fail(PDD_E_INTERNAL, "gamma fit: singular weights");
    }
    // dispersion from the Pearson residuals, n - 2 degrees of freedom
    double disp = 0.0;
    for (int i = 0; i < n; ++i) {
        const double m = coef[0] + coef[1] * x[i];
        const double r = family == PDD_GLM_NORMAL ? y[i] - m : (y[i] - m) / m;
        disp += r * r;
    }
    disp /= (double)(n - 2);
    se[0] = std::sqrt(disp * inv[0]);
    se[1] = std::sqrt(disp * inv[2]);
    if (iters) *iters = it;
    return PDD_OK;
}

// Objective of the scheduling algorithm at a > a_j (Alg. A:Scheduling with
// the sensitivity formula, eq. F:Sensitivity_formula): sum over nodes of
// K V (kappa (1 - r^2 + |alpha r / beta| a_j) + (a_j / a)^(2 + 1/delta)),
// r^2 = 1 - V[psi] a^2 (1 - rho^2[phi, psi]) / (4 V), kept in [0, 1].
double schedule_objective(const pdd_sched_node *nd, int64_t n, double a, double a_j, double kappa, double delta)
{
    const double p = 2.0 + 1.0 / delta;
    const double tail = std::pow(a_j / a, p);
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double r2 = 1.0 - nd[i].V_psi * a * a * (1.0 - nd[i].rho_psi * nd[i].rho_psi) / (4.0 * nd[i].V);
        r2 = r2 < 0.0 ? 0.0 : (r2 > 1.0 ? 1.0 : r2);
        const double r = std::sqrt(r2);
        acc += nd[i].K * nd[i].V * (kappa * (1.0 - r2 + std::fabs(nd[i].alpha * r / nd[i].beta) * a_j) + tail);
    }
    return acc;
}

}  // namespace

extern "C" {

pdd_status pdd_schedule(const pdd_sched_node *nodes, int64_t n, double a0, double kappa, double delta, double a_max,
                        double s_min, int32_t max_levels, double *a_out, double *speedup, int32_t *n_levels)
{
    if (!nodes || n < 1 || !a_out || !n_levels) return fail(PDD_E_INVALID, "NULL argument or no nodes");
    if (!(a0 > 0.0) || !(a_max > a0) || !(kappa > 0.0) || !(delta > 0.0) || !(s_min > 0.0) || max_levels < 0 ||
        !std::isfinite(a_max) || !std::isfinite(kappa))
        return fail(PDD_E_INVALID, "need 0 < a0 < a_max, kappa > 0, delta > 0, s_min > 0, max_levels >= 0");
    for (int64_t i = 0; i < n; ++i) {
        const pdd_sched_node &q = nodes[i];
        if (!(q.K > 0.0) || !(q.V > 0.0) || !(q.V_psi >= 0.0) || !(std::fabs(q.rho_psi) <= 1.0) || q.beta == 0.0 ||
            !std::isfinite(q.alpha) || !std::isfinite(q.beta) || !std::isfinite(q.K) || !std::isfinite(q.V_psi))
            return fail(PDD_E_INVALID, "node %lld: need K > 0, V > 0, V_psi >= 0, |rho| <= 1, beta != 0, finite values",
                        (long long)i);
    }
    const double p = 2.0 + 1.0 / delta;
    double plain_kv = 0.0;
    for (int64_t i = 0; i < n; ++i) plain_kv += nodes[i].K * nodes[i].V;
    a_out[0] = a0;
    int32_t J = 0;
    while (J < max_levels) {
        const double a_j = a_out[J];
        if (a_j >= a_max) break;
        // coarse log grid over (a_j, a_max], then golden section around the best point
        constexpr int kGrid = 512;
        const double la = std::log(a_j), lb = std::log(a_max);
        int best = 1;
        double best_f = HUGE_VAL;
        for (int k = 1; k <= kGrid; ++k) {
            const double f = schedule_objective(nodes, n, std::exp(la + (lb - la) * k / kGrid), a_j, kappa, delta);
            if (f < best_f) {
                best_f = f;
                best = k;
            }
        }
        double lo = la + (lb - la) * (best - 1) / kGrid, hi = la + (lb - la) * std::min(best + 1, kGrid) / kGrid;
        const double gr = 0.6180339887498949;
        double x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo);
        double f1 = schedule_objective(nodes, n, std::exp(x1), a_j, kappa, delta);
        double f2 = schedule_objective(nodes, n, std::exp(x2), a_j, kappa, delta);
        for (int it = 0; it < 200 && hi - lo > 1e-12; ++it) {
            if (f1 <= f2) {
                hi = x2, x2 = x1, f2 = f1;
                x1 = hi - gr * (hi - lo);
                f1 = schedule_objective(nodes, n, std::exp(x1), a_j, kappa, delta);
            } else {
                lo = x1, x1 = x2, f1 = f2;
                x2 = lo + gr * (hi - lo);
                f2 = schedule_objective(nodes, n, std::exp(x2), a_j, kappa, delta);
            }
        }
        double a = std::exp(0.5 * (lo + hi));
        double f = schedule_objective(nodes, n, a, a_j, kappa, delta);
        if (best_f < f) {  // keep the grid point if the refinement did not improve on it
            a = std::exp(la + (lb - la) * best / kGrid);
            f = best_f;
        }
        // predicted speedup cost(PlainPDD(a_j)) / cost(IterPDD(a_j, a)) (eqs.
        // F:PlainPDD_cost, F:IterPDD_cost without the subdomain terms)
        const double s = plain_kv / f;
        (void)p;
        if (s < s_min) break;
        if (speedup) speedup[J] = s;
        a_out[++J] = a;
    }
    *n_levels = J;
    return PDD_OK;
}

pdd_status pdd_glm_fit(const double *x, const double *y, int32_t n, int32_t family, double *coef, double *se,
                       int32_t *iterations)
{
    if (!x || !y || !coef || !se) return fail(PDD_E_INVALID, "NULL argument");
    if (n < 3) return fail(PDD_E_INVALID, "a line fit with standard errors needs n >= 3");
    if (family != PDD_GLM_NORMAL && family != PDD_GLM_GAMMA) return fail(PDD_E_INVALID, "bad family");
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(x[i]) || !std::isfinite(y[i])) return fail(PDD_E_INVALID, "non-finite data at %d", i);
        if (family == PDD_GLM_GAMMA && !(y[i] > 0.0)) return fail(PDD_E_INVALID, "gamma data must be > 0 (at %d)", i);
    }
    int it = 0;
    pdd_status st = glm(x, y, n, family, coef, se, &it);
    if (st) return st;
    if (iterations) *iterations = it;
    return PDD_OK;
}

pdd_status pdd_fit_constants(pdd_ctx *ctx, const pdd_work_item *item, const double *h, int32_t n_h,
                             uint64_t n_hat, double delta, pdd_node_constants *out, void *stream)
{
    if (!ctx || !item || !h || !out || !item->problem || !item->opts) return fail(PDD_E_INVALID, "NULL argument");
    if (n_h < 3) return fail(PDD_E_INVALID, "the cloud needs at least 3 time steps");
    if (n_hat < 2) return fail(PDD_E_INVALID, "n_hat must be >= 2");
    if (!(delta > 0.0) || !std::isfinite(delta)) return fail(PDD_E_INVALID, "delta must be finite and > 0");
    if (item->n_nodes < 1 || !item->nodes) return fail(PDD_E_INVALID, "the fit needs nodes");
    if (item->opts->rec_steps || item->opts->rec_phi || item->opts->rec_e)
        return fail(PDD_E_UNSUPPORTED, "per-path records are not kept by the fit");
    if ((uint64_t)item->opts->stream_id + (uint64_t)n_h > (1u << 28))
        return fail(PDD_E_INVALID, "stream_id + n_h must be <= 2^28");
    for (int j = 0; j < n_h; ++j)
        if (!(h[j] > 0.0) || !std::isfinite(h[j])) return fail(PDD_E_INVALID, "h[%d] must be finite and > 0", j);
    const int64_t n = item->n_nodes;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipSetDevice(ctx->device));
    pdd_node_stats *dev = nullptr;
    if (hipMalloc(&dev, (size_t)n_h * n * sizeof(pdd_node_stats)) != hipSuccess)
        return fail(PDD_E_NOMEM, "fit statistics (%lld bytes)", (long long)((size_t)n_h * n * sizeof(pdd_node_stats)));
    // the cloud: solve j at step h[j] with its own RNG stream, all in one batch
    std::vector<pdd_solve_opts> opts(n_h, *item->opts);
    std::vector<pdd_work_item> w(n_h, *item);
    for (int j = 0; j < n_h; ++j) {
        opts[j].dt = h[j];
        opts[j].n_paths = n_hat;
        opts[j].n_paths_per_node = nullptr;
        opts[j].stream_id = item->opts->stream_id + (uint32_t)j;
        opts[j].flags &= ~(PDD_ACCUMULATE | PDD_TIME_KERNEL);
        w[j].opts = &opts[j];
        w[j].out = dev + (size_t)j * n;
    }
    pdd_status st = pdd_solve_batch(ctx, w.data(), n_h, stream);
    std::vector<pdd_node_stats> host((size_t)n_h * n);
    if (!st && hipMemcpyAsync(host.data(), dev, host.size() * sizeof(pdd_node_stats), hipMemcpyDeviceToHost, s) != hipSuccess)
        st = fail(PDD_E_HIP, "copying the fit statistics back failed");
    if (!st && hipStreamSynchronize(s) != hipSuccess) st = fail(PDD_E_HIP, "waiting for the fit solves failed");
    (void)hipFree(dev);
    if (st) return st;
    std::vector<double> x(n_h), ym(n_h), yv(n_h), yt(n_h);
    for (int j = 0; j < n_h; ++j) x[j] = std::pow(h[j], delta);
    for (int64_t i = 0; i < n; ++i) {
        pdd_node_constants &c = out[i];
        std::memset(&c, 0, sizeof(c));
        for (int j = 0; j < n_h; ++j) {
            const pdd_node_stats &q = host[(size_t)j * n + i];
            ym[j] = q.mean;
            yv[j] = q.var;
            yt[j] = q.mean_steps * h[j];  // E[tau_h] = h E[exit step]
        }
        double cf[2], se[2];
        int it = 0;
        if ((st = glm(x.data(), ym.data(), n_h, PDD_GLM_NORMAL, cf, se, &it))) return st;
        c.E_phi = cf[0];
        c.beta = cf[1];
        c.se_E_phi = se[0];
        c.se_beta = se[1];
        for (int j = 0; j < n_h; ++j)
            if (!(yv[j] > 0.0)) return fail(PDD_E_INVALID, "node %lld: a zero sample variance cannot be fitted", (long long)i);
        if ((st = glm(x.data(), yv.data(), n_h, PDD_GLM_GAMMA, cf, se, &it))) return st;
        c.V_phi = cf[0];
        c.alpha = cf[1];
        c.se_V_phi = se[0];
        c.se_alpha = se[1];
        c.iterations = it;
        if ((st = glm(x.data(), yt.data(), n_h, PDD_GLM_NORMAL, cf, se, &it))) return st;
        c.E_tau = cf[0];
        c.beta_tau = cf[1];
        c.se_E_tau = se[0];
    }
    return PDD_OK;
}

}  // extern "C"
