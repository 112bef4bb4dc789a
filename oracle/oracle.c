/*
 * Plain FP64 CPU oracle: the first-stage Feynman-Kac nodal solve of
 * probabilistic domain decomposition, written step by step from the paper.
 *
 * THIS IS TEST INFRASTRUCTURE: only the tests, the smoke check and the
 * benchmark's CPU-baseline leg use it. It shares no code with the GPU library.
 * Single-threaded, IEEE double, compiled with floating-point contraction off,
 * glibc transcendentals.
 *
 * Pins (what fixes each part independently of this file; tests/ holds them):
 *   Philox4x32-10        - bit-exact against rocRAND's independent host engine.
 *   Box-Muller / law     - sample moments and a Kolmogorov-Smirnov test.
 *   source f from U      - finite differences of U, and the hand-expanded
 *                          closed form for the unit-square manufactured problem.
 *   integrator + exits   - manufactured solutions, ball exit time, ball killing
 *                          (modified Bessel), harmonic data, rectangle exit
 *                          time (Fourier series), the time-step bias trend.
 *   discrete scheme      - brute-force enumeration of every Rademacher path.
 *   correction estimator - zero-variance invariant for a bilinear solution.
 *   Ito control variate  - E[xi] = 0 over every enumerated Rademacher path;
 *                          the closed form phi + xi = x0 + (Pi(X_K) - X_K)
 *                          for a linear solution; variance that vanishes
 *                          with h for the exact gradient; and agreement, path
 *                          by path, with the correction estimator as h -> 0.
 *   tabulated b, c, f    - affine drift / constant killing on grids walk the
 *                          analytic problem's paths; non-affine tabulated
 *                          coefficients with the matching f keep the
 *                          manufactured solution.
 *   sums / statistics    - math.fsum of the per-path records.
 * No function here is "parity unpinned".
 */
#include "oracle.h"

#include <math.h>
#include <stddef.h>
#include <string.h>

/* ---------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications on a
 * 128-bit counter, the 64-bit key bumped by the Weyl constants between rounds.
 * The paper itself draws with Matlab's randn; the generator and the layout of
 * its counter are a choice of this implementation (same in the GPU code).
 * ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 32-bit word -> uniform strictly inside (0, 1). */
static double unit_open(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

static double sign_of(uint32_t w) { return (w >> 31) ? 1.0 : -1.0; }

static const double TWO_PI = 6.283185307179586476925286766559;

static void philox_at(const orc_problem *p, uint32_t c0, uint32_t path, uint32_t node,
                      uint32_t c3, uint32_t out[4])
{
    uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), (uint32_t)(p->seed >> 32)};
    uint32_t ctr[4] = {c0, path, node, c3};
    orc_philox4x32_10(ctr, key, out);
}

/* The D-dimensional standard normal of step s (the N_D of eq. F:E_M).
 * 2D: one block serves two consecutive steps; step s takes words (0,1) if s is
 * even and (2,3) if odd, of the block with counter (s/2, path, node, stream<<4).
 * 3D: one block per step, counter (s, path, node, stream<<4); words (0,1) give
 * the first two normals by Box-Muller, words (2,3) the third (cosine branch).
 * Box-Muller (1958): r = sqrt(-2 ln u_a), N = r cos(2 pi u_b), r sin(2 pi u_b).
 * Rademacher law (tests only): each normal replaced by +-1 from the top bit
 * of the word that would feed its uniform u_a / u_b. */
void orc_step_normals(const orc_problem *p, const orc_opts *o, uint32_t node,
                      uint64_t path, uint64_t step, double *nrm)
{
    uint32_t w[4];
    uint32_t tag = (o->stream << 4) | 0u;
    if (p->dim == 2) {
        philox_at(p, (uint32_t)(step >> 1), (uint32_t)path, node, tag, w);
        uint32_t a = (step & 1) ? w[2] : w[0];
        uint32_t b = (step & 1) ? w[3] : w[1];
        if (o->law == ORC_LAW_RADEMACHER) {
            nrm[0] = sign_of(a);
            nrm[1] = sign_of(b);
            return;
        }
        double r = sqrt(-2.0 * log(unit_open(a)));
        double th = TWO_PI * unit_open(b);
        nrm[0] = r * cos(th);
        nrm[1] = r * sin(th);
    } else {
        philox_at(p, (uint32_t)step, (uint32_t)path, node, tag, w);
        if (o->law == ORC_LAW_RADEMACHER) {
            nrm[0] = sign_of(w[0]);
            nrm[1] = sign_of(w[1]);
            nrm[2] = sign_of(w[2]);
            return;
        }
        double r = sqrt(-2.0 * log(unit_open(w[0])));
        double th = TWO_PI * unit_open(w[1]);
        nrm[0] = r * cos(th);
        nrm[1] = r * sin(th);
        double r2 = sqrt(-2.0 * log(unit_open(w[2])));
        double th2 = TWO_PI * unit_open(w[3]);
        nrm[2] = r2 * cos(th2);
    }
}

/* The uniform of the Brownian-bridge exit test at step s: word s mod 4 of the
 * block with counter (s/4, path, node, (stream<<4)|1). */
double orc_bridge_uniform(const orc_problem *p, const orc_opts *o, uint32_t node,
                          uint64_t path, uint64_t step)
{
    uint32_t w[4];
    philox_at(p, (uint32_t)(step >> 2), (uint32_t)path, node, (o->stream << 4) | 1u, w);
    return unit_open(w[step & 3]);
}

/* ---------------------------------------------------------------------------
 * Coefficients (Sec. 2.1, eq. F:EllipticBVP with a_ij = sigma^2 delta_ij, so
 * the SDE of eq. F:SDE has sigma times the identity as diffusion matrix).
 * ------------------------------------------------------------------------- */
static double ipow(double x, int n)
{
    double r = 1.0;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
}

/* The analytic drift and killing rate of the descriptor. */
static void drift_analytic(const orc_problem *p, const double *x, double *b)
{
    for (int i = 0; i < p->dim; ++i) {
        double v = p->b0[i];
        for (int j = 0; j < p->dim; ++j) v += p->B[i][j] * x[j];
        b[i] = v;
    }
}

static double kill_analytic(const orc_problem *p, const double *x)
{
    double r2 = 0.0;
    for (int i = 0; i < p->dim; ++i) r2 += x[i] * x[i];
    return p->c_a + p->c_b * r2;
}

/* The coefficients the walk uses: a tabulated component where one is given
 * (its grid interpolant), the analytic one otherwise. */
void orc_drift(const orc_problem *p, const double *x, double *b)
{
    drift_analytic(p, x, b);
    for (int i = 0; i < p->dim; ++i)
        if (p->tab_b[i]) b[i] = orc_interp(p->tab_b[i], x);
}

double orc_kill(const orc_problem *p, const double *x)
{
    return p->tab_c ? orc_interp(p->tab_c, x) : kill_analytic(p, x);
}

static double mono_value(const orc_mono *m, int dim, const double *x)
{
    double v = m->coef;
    for (int d = 0; d < dim; ++d) v *= ipow(x[d], m->e[d]);
    return v;
}

/* U, its gradient and its Laplacian, term by term. */
static void U_full(const orc_problem *p, const double *x, double *U, double *grad, double *lap)
{
    int D = p->dim;
    double u = 0.0, l = 0.0, gr[3] = {0.0, 0.0, 0.0};
    for (int m = 0; m < p->n_trig; ++m) {
        const orc_trig *t = &p->trig[m];
        double s[3], c[3];
        for (int d = 0; d < D; ++d) {
            double arg = t->k[d] * x[d] + t->phase[d];
            s[d] = sin(arg);
            c[d] = cos(arg);
        }
        double val = t->amp;
        for (int d = 0; d < D; ++d) val *= s[d];
        double ksq = 0.0;
        for (int d = 0; d < D; ++d) ksq += t->k[d] * t->k[d];
        u += val;
        l += -ksq * val;
        for (int d = 0; d < D; ++d) {
            double gd = t->amp * t->k[d] * c[d];
            for (int e = 0; e < D; ++e)
                if (e != d) gd *= s[e];
            gr[d] += gd;
        }
    }
    for (int m = 0; m < p->n_mono; ++m) {
        const orc_mono *q = &p->mono[m];
        u += mono_value(q, D, x);
        for (int d = 0; d < D; ++d) {
            int ed = q->e[d];
            if (ed >= 1) {
                double gd = q->coef * (double)ed * ipow(x[d], ed - 1);
                for (int e = 0; e < D; ++e)
                    if (e != d) gd *= ipow(x[e], q->e[e]);
                gr[d] += gd;
            }
            if (ed >= 2) {
                double ld = q->coef * (double)(ed * (ed - 1)) * ipow(x[d], ed - 2);
                for (int e = 0; e < D; ++e)
                    if (e != d) ld *= ipow(x[e], q->e[e]);
                l += ld;
            }
        }
    }
    *U = u;
    *lap = l;
    for (int d = 0; d < D; ++d) grad[d] = gr[d];
}

double orc_U(const orc_problem *p, const double *x)
{
    double u, l, g[3];
    U_full(p, x, &u, g, &l);
    return u;
}

/* f = (1/2) sigma^2 Lap U + b.grad U + c U + sum(fx): the source for which U
 * solves eq. F:EllipticBVP (written L u + c u = f). */
double orc_source(const orc_problem *p, const double *x)
{
    if (p->tab_f) return orc_interp(p->tab_f, x);
    double u, l, g[3], b[3];
    U_full(p, x, &u, g, &l);
    drift_analytic(p, x, b);
    double f = 0.5 * p->sigma * p->sigma * l;
    for (int d = 0; d < p->dim; ++d) f += b[d] * g[d];
    f += kill_analytic(p, x) * u;
    for (int m = 0; m < p->n_fx; ++m) f += mono_value(&p->fx[m], p->dim, x);
    return f;
}

/* g = U + sum(gx) on the boundary. */
double orc_boundary(const orc_problem *p, const double *x)
{
    if (p->tab_g) return orc_interp(p->tab_g, x);
    double v = orc_U(p, x);
    for (int m = 0; m < p->n_gx; ++m) v += mono_value(&p->gx[m], p->dim, x);
    return v;
}

/* Bilinear / trilinear interpolation on a uniform grid, cell index clamped to
 * the grid and the in-cell weight clamped to [0, 1]. */
double orc_interp(const orc_grid *g, const double *x)
{
    int i[3] = {0, 0, 0};
    double w[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < g->dim; ++d) {
        double t = (x[d] - g->lo[d]) * ((double)(g->n[d] - 1) / (g->hi[d] - g->lo[d]));
        double fl = floor(t);
        int id = (int)fl;
        if (fl < 0.0) id = 0;
        if (fl > (double)(g->n[d] - 2)) id = g->n[d] - 2;
        double wd = t - (double)id;
        if (wd < 0.0) wd = 0.0;
        if (wd > 1.0) wd = 1.0;
        i[d] = id;
        w[d] = wd;
    }
    int nx = g->n[0], ny = g->n[1];
    if (g->dim == 2) {
        const double *v = g->data;
        double v00 = v[(size_t)i[1] * nx + i[0]];
        double v10 = v[(size_t)i[1] * nx + i[0] + 1];
        double v01 = v[(size_t)(i[1] + 1) * nx + i[0]];
        double v11 = v[(size_t)(i[1] + 1) * nx + i[0] + 1];
        return (1.0 - w[1]) * ((1.0 - w[0]) * v00 + w[0] * v10) +
               w[1] * ((1.0 - w[0]) * v01 + w[0] * v11);
    }
    double acc = 0.0;
    for (int dz = 0; dz < 2; ++dz) {
        double layer = 0.0;
        for (int dy = 0; dy < 2; ++dy) {
            size_t row = ((size_t)(i[2] + dz) * ny + (i[1] + dy)) * nx + i[0];
            double line = (1.0 - w[0]) * g->data[row] + w[0] * g->data[row + 1];
            layer += (dy ? w[1] : 1.0 - w[1]) * line;
        }
        acc += (dz ? w[2] : 1.0 - w[2]) * layer;
    }
    return acc;
}

/* ---------------------------------------------------------------------------
 * Geometry (the distance map d, the projection Pi and the faces of Alg. 1).
 * Box faces are ordered x-lo, x-hi, y-lo, y-hi, z-lo, z-hi.
 * ------------------------------------------------------------------------- */
static int strictly_inside(const orc_problem *p, const double *x)
{
    if (p->domain == ORC_BOX) {
        for (int d = 0; d < p->dim; ++d)
            if (!(x[d] > p->lo[d] && x[d] < p->hi[d])) return 0;
        return 1;
    }
    double r2 = 0.0;
    for (int d = 0; d < p->dim; ++d) {
        double t = x[d] - p->center[d];
        r2 += t * t;
    }
    return r2 < p->radius * p->radius;
}

static double face_distance(const orc_problem *p, const double *x, int face)
{
    int d = face >> 1;
    return (face & 1) ? p->hi[d] - x[d] : x[d] - p->lo[d];
}

/* Distance to the boundary from inside (minus the signed distance d(x)). */
static double inner_distance(const orc_problem *p, const double *x)
{
    if (p->domain == ORC_BOX) {
        double m = face_distance(p, x, 0);
        for (int f = 1; f < 2 * p->dim; ++f) {
            double t = face_distance(p, x, f);
            if (t < m) m = t;
        }
        return m;
    }
    double r2 = 0.0;
    for (int d = 0; d < p->dim; ++d) {
        double t = x[d] - p->center[d];
        r2 += t * t;
    }
    return p->radius - sqrt(r2);
}

static void radial_projection(const orc_problem *p, const double *x, double *out)
{
    double r2 = 0.0;
    for (int d = 0; d < p->dim; ++d) {
        double t = x[d] - p->center[d];
        r2 += t * t;
    }
    double r = sqrt(r2);
    for (int d = 0; d < p->dim; ++d) {
        if (r > 0.0)
            out[d] = p->center[d] + p->radius * ((x[d] - p->center[d]) / r);
        else
            out[d] = p->center[d] + (d == 0 ? p->radius : 0.0);
    }
}

/* Pi: closest boundary point. Box, strictly inside: move to the nearest face
 * (ties to the lowest face index). Box, otherwise: clamp to the box. */
static void project(const orc_problem *p, const double *x, double *out)
{
    if (p->domain == ORC_BALL) {
        radial_projection(p, x, out);
        return;
    }
    for (int d = 0; d < p->dim; ++d) out[d] = x[d];
    if (strictly_inside(p, x)) {
        int best = 0;
        double bd = face_distance(p, x, 0);
        for (int f = 1; f < 2 * p->dim; ++f) {
            double t = face_distance(p, x, f);
            if (t < bd) { bd = t; best = f; }
        }
        int d = best >> 1;
        out[d] = (best & 1) ? p->hi[d] : p->lo[d];
    } else {
        for (int d = 0; d < p->dim; ++d) {
            if (out[d] < p->lo[d]) out[d] = p->lo[d];
            if (out[d] > p->hi[d]) out[d] = p->hi[d];
        }
    }
}

/* ---------------------------------------------------------------------------
 * The path (Alg. 1 with eq. F:E_M, left-point rule).
 * ------------------------------------------------------------------------- */
static const double GM_SHIFT = 0.5826;          /* Alg. 1, the boundary shift constant */
static const double BRIDGE_SKIP_ARG = 24.953298500158186; /* 36 ln 2: p < 2^-36 skipped */

typedef struct {
    const double *normals; /* given noise, or NULL for Philox */
    const double *unif;
    uint64_t n_given;
    uint32_t node;
    uint64_t path;
} noise_src;

static void draw_normals(const orc_problem *p, const orc_opts *o, const noise_src *ns,
                         uint64_t s, double *nrm)
{
    if (ns->normals) {
        for (int d = 0; d < p->dim; ++d) nrm[d] = ns->normals[s * (uint64_t)p->dim + d];
        return;
    }
    orc_step_normals(p, o, ns->node, ns->path, s, nrm);
}

static double draw_bridge(const orc_problem *p, const orc_opts *o, const noise_src *ns,
                          uint64_t s)
{
    if (ns->normals) return ns->unif[s];
    return orc_bridge_uniform(p, o, ns->node, ns->path, s);
}

static int bad_problem(const orc_problem *p, const orc_opts *o)
{
    if (p->dim != 2 && p->dim != 3) return 1;
    if (!(o->h > 0.0) || !(p->sigma > 0.0)) return 1;
    if ((o->u_prev == NULL) != (o->resid == NULL)) return 1;
    if (o->grad[0]) {
        if (o->u_prev) return 1;
        for (int d = 0; d < p->dim; ++d)
            if (!o->grad[d] || o->grad[d]->dim != p->dim || !o->grad[d]->data) return 1;
    }
    const orc_grid *tab[6] = {p->tab_b[0], p->tab_b[1], p->tab_b[2], p->tab_c, p->tab_f, p->tab_g};
    for (int q = 0; q < 6; ++q) {
        if (!tab[q]) continue;
        if (q < 3 && q >= p->dim) return 1;
        if (tab[q]->dim != p->dim || !tab[q]->data) return 1;
        for (int d = 0; d < p->dim; ++d)
            if (tab[q]->n[d] < 2 || !(tab[q]->hi[d] > tab[q]->lo[d])) return 1;
    }
    return 0;
}

static int run_core(const orc_problem *p, const orc_opts *o, const double *x0,
                    const noise_src *ns, orc_path *out)
{
    int D = p->dim;
    double X[3] = {0, 0, 0}, Xn[3] = {0, 0, 0}, Xt[3] = {0, 0, 0};
    double Y = 1.0, Z = 0.0, R = 0.0, xi = 0.0;
    uint64_t k = 0;
    int capped = 0;
    double h = o->h;
    double sqh = sqrt(h);
    double sig_sqh = p->sigma * sqh;
    double two_over_s2h = 2.0 / (p->sigma * p->sigma * h);
    int cv = o->u_prev != NULL;
    int ito = o->grad[0] != NULL;
    uint64_t cap = o->max_steps;
    if (ns->normals && ns->n_given < cap) cap = ns->n_given;
    for (int d = 0; d < D; ++d) X[d] = x0[d];

    for (;;) {
        /* Alg. 1, shifted-boundary test before the step: stop once the walker
         * is within 0.5826 sigma sqrt(h) of the boundary (or outside). */
        if (o->exit_mode == ORC_EXIT_SHIFT && inner_distance(p, X) <= GM_SHIFT * sig_sqh) {
            project(p, X, Xt);
            break;
        }
        if (k == cap) {
            capped = 1;
            project(p, X, Xt);
            break;
        }
        /* One Euler-Maruyama step (eq. F:E_M) with coefficients at X_k. */
        double nrm[3], b[3];
        draw_normals(p, o, ns, k, nrm);
        orc_drift(p, X, b);
        double c = orc_kill(p, X);
        double f = orc_source(p, X);
        double hY = h * Y;
        Z = Z - hY * f;
        if (cv) R = R + hY * orc_interp(o->resid, X);
        if (ito) {
            /* eq. F:xiControlVariate by its left-point quadrature: the
             * integrand Y sigma grad(u~) at X_k times the increment
             * W_{k+1} - W_k = sqrt(h) N_k of the same step. */
            double gn = 0.0;
            for (int d = 0; d < D; ++d) gn = gn + orc_interp(o->grad[d], X) * nrm[d];
            xi = xi - Y * sig_sqh * gn;
        }
        Y = Y + hY * c;
        for (int d = 0; d < D; ++d) Xn[d] = X[d] + h * b[d] + sig_sqh * nrm[d];
        uint64_t s = k;
        k = k + 1;

        if (o->exit_mode != ORC_EXIT_SHIFT) {
            if (!strictly_inside(p, Xn)) {
                project(p, Xn, Xt);
                break;
            }
            if (o->exit_mode == ORC_EXIT_BRIDGE) {
                /* Brownian bridge between X_k and X_{k+1}: per flat face,
                 * P(cross) = exp(-2 a a' / (sigma^2 h)); faces combined as
                 * independent, P = 1 - prod(1 - p_f), accumulated as
                 * P <- P + p_f (1 - P). */
                double P = 0.0, best_p = -1.0;
                int best_face = -1, live = 0;
                if (p->domain == ORC_BOX) {
                    for (int fc = 0; fc < 2 * D; ++fc) {
                        double a = face_distance(p, X, fc);
                        double an = face_distance(p, Xn, fc);
                        double arg = a * an * two_over_s2h;
                        if (arg <= BRIDGE_SKIP_ARG) {
                            double pf = exp(-arg);
                            P = P + pf * (1.0 - P);
                            live = 1;
                            if (pf > best_p) { best_p = pf; best_face = fc; }
                        }
                    }
                } else {
                    double a = inner_distance(p, X);
                    double an = inner_distance(p, Xn);
                    double arg = a * an * two_over_s2h;
                    if (arg <= BRIDGE_SKIP_ARG) {
                        P = exp(-arg);
                        live = 1;
                    }
                }
                if (live && draw_bridge(p, o, ns, s) < P) {
                    for (int d = 0; d < D; ++d) Xt[d] = Xn[d];
                    if (p->domain == ORC_BOX) {
                        int dd = best_face >> 1;
                        Xt[dd] = (best_face & 1) ? p->hi[dd] : p->lo[dd];
                    } else {
                        radial_projection(p, Xn, Xt);
                    }
                    break;
                }
            }
        }
        for (int d = 0; d < D; ++d) X[d] = Xn[d];
    }

    double gval = orc_boundary(p, Xt);
    out->phi = gval * Y + Z;
    if (cv)
        out->e = (gval - orc_interp(o->u_prev, Xt)) * Y - R;
    else if (ito)
        out->e = out->phi + xi;
    else
        out->e = NAN;
    out->steps = k;
    out->capped = capped;
    out->pad = 0;
    for (int d = 0; d < 3; ++d) out->x_exit[d] = d < D ? Xt[d] : 0.0;
    return 0;
}

int orc_run_path(const orc_problem *p, const orc_opts *o, const double *x0, uint32_t node,
                 uint64_t path, orc_path *out)
{
    if (bad_problem(p, o)) return -1;
    noise_src ns = {NULL, NULL, 0, node, path};
    return run_core(p, o, x0, &ns, out);
}

int orc_run_path_noise(const orc_problem *p, const orc_opts *o, const double *x0,
                       const double *normals, const double *unif, uint64_t n_steps,
                       orc_path *out)
{
    if (bad_problem(p, o) || !normals || !unif) return -1;
    noise_src ns = {normals, unif, n_steps, 0, 0};
    return run_core(p, o, x0, &ns, out);
}

/* ---------------------------------------------------------------------------
 * Statistics (Sec. 2.2, eqs. F:Statistical_error; Sec. 2.3, eqs.
 * F:Variance_Reduction and F:Rho). Neumaier-compensated sums in path order.
 * ------------------------------------------------------------------------- */
typedef struct { double s, c; } nsum;

static void nadd(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double nval(nsum a) { return a.s + a.c; }

int orc_solve_nodes(const orc_problem *p, const orc_opts *o, const double *nodes,
                    int64_t n_nodes, orc_stats *out, orc_path *rec)
{
    if (bad_problem(p, o) || n_nodes < 0) return -1;
    int D = p->dim;
    int ito = o->grad[0] != NULL;
    int cv = o->u_prev != NULL || ito;
    for (int64_t i = 0; i < n_nodes; ++i) {
        const double *x0 = nodes + i * D;
        nsum sp = {0, 0}, sp2 = {0, 0}, se = {0, 0}, se2 = {0, 0}, spe = {0, 0};
        int64_t steps = 0, ncap = 0;
        for (uint64_t jj = 0; jj < o->n_paths; ++jj) {
            orc_path r;
            noise_src ns = {NULL, NULL, 0, (uint32_t)i, o->path_offset + jj};
            run_core(p, o, x0, &ns, &r);
            if (rec) rec[(uint64_t)i * o->n_paths + jj] = r;
            nadd(&sp, r.phi);
            nadd(&sp2, r.phi * r.phi);
            if (cv) {
                nadd(&se, r.e);
                nadd(&se2, r.e * r.e);
                nadd(&spe, r.phi * r.e);
            }
            steps += (int64_t)r.steps;
            ncap += r.capped;
        }
        orc_stats *st = &out[i];
        memset(st, 0, sizeof(*st));
        double n = (double)o->n_paths;
        st->n = (int64_t)o->n_paths;
        st->n_capped = ncap;
        st->steps_sum = steps;
        nsum all[5] = {sp, sp2, se, se2, spe};
        for (int q = 0; q < 5; ++q) {
            st->sums[2 * q] = all[q].s;
            st->sums[2 * q + 1] = all[q].c;
        }
        if (o->n_paths == 0) {
            st->mean = st->var = st->stderr_ = st->mean_steps = NAN;
            st->mean_plain = st->var_plain = st->cov = st->rho = st->vr = st->vr_opt = NAN;
            continue;
        }
        double Sp = nval(sp), Sp2 = nval(sp2);
        st->mean_steps = (double)steps / n;
        st->mean_plain = Sp / n;
        st->var_plain = o->n_paths > 1 ? (Sp2 - Sp * Sp / n) / (n - 1.0) : NAN;
        if (!cv) {
            st->mean = st->mean_plain;
            st->var = st->var_plain;
            st->stderr_ = sqrt(st->var / n);
            st->cov = st->rho = st->vr = st->vr_opt = NAN;
            continue;
        }
        double Se = nval(se), Se2 = nval(se2), Spe = nval(spe);
        /* correction: u_prev(x0) + mean(e); Ito: mean(phi + xi) */
        st->mean = (ito ? 0.0 : orc_interp(o->u_prev, x0)) + Se / n;
        st->var = o->n_paths > 1 ? (Se2 - Se * Se / n) / (n - 1.0) : NAN;
        st->stderr_ = sqrt(st->var / n);
        /* xi = u_prev(x0) + e - phi is the paper's pathwise control variate
         * (Ito: xi = e - phi); the constant does not enter cov or rho. */
        double cpe = o->n_paths > 1 ? (Spe - Sp * Se / n) / (n - 1.0) : NAN;
        double vxi = st->var + st->var_plain - 2.0 * cpe;
        st->cov = cpe - st->var_plain;
        st->rho = st->cov / sqrt(st->var_plain * vxi);
        st->vr = st->var_plain / st->var;
        st->vr_opt = 1.0 / (1.0 - st->rho * st->rho);
    }
    return 0;
}

int orc_run_paths(const orc_problem *p, const orc_opts *o, const double *nodes,
                  const uint32_t *node_idx, const uint64_t *path_idx, int64_t n, orc_path *rec)
{
    if (bad_problem(p, o) || n < 0) return -1;
    for (int64_t q = 0; q < n; ++q) {
        noise_src ns = {NULL, NULL, 0, node_idx[q], path_idx[q]};
        run_core(p, o, nodes + (size_t)node_idx[q] * p->dim, &ns, &rec[q]);
    }
    return 0;
}
