/*
 * Plain FP64 CPU oracle for the first-stage Feynman-Kac nodal solve of
 * probabilistic domain decomposition (Bernal & Acebron, "A multigrid-like
 * algorithm for probabilistic domain decomposition").
 *
 * THIS IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it. It shares no code, header,
 * constant table or helper with the GPU library; the two are written
 * separately from the paper's definitions so that one can check the other.
 *
 * What is computed (paper Sec. 2.1, eq. F:Dynkin, and Sec. 2.3, Alg. 1):
 *   u(x0) = E[ g(X_tau) Y_tau + Z_tau ],  Y = exp(int c),  Z = -int f Y dt,
 * for (1/2) sigma^2 Lap u + b.grad u + c u = f in Omega, u = g on dOmega,
 * discretised with Euler-Maruyama (eq. F:E_M, left-point rule) and one of
 * three exit tests: Brownian-bridge (default), the Gobet-Menozzi shifted
 * boundary of Alg. 1, or the naive test. The correction (control-variate)
 * estimator uses a previous approximation u_prev and the residual
 * r = f - (L + c) u_prev, both given on grids:
 *   u(x0) = u_prev(x0) + E[ (g - u_prev)(X_tau) Y_tau - int r Y dt ],
 * which is phi + xi of eqs. F:Statistics_VR / F:xiControlVariate written
 * without the gradient of u_prev (Ito's formula applied to u_prev). The
 * paper's own form of that control variate is also computed: the pathwise
 * Ito integral xi = -int Y sigma grad(u~) . dW of eq. F:xiControlVariate,
 * accumulated along the same Euler-Maruyama path from grids of the
 * components of grad(u~), with the estimator phi + xi (E[xi] = 0).
 *
 * Parity status of each function is stated in oracle.c beside it.
 */
#ifndef PDD_ORACLE_H
#define PDD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_TRIG 16
#define ORC_MAX_MONO 8

enum { ORC_BOX = 0, ORC_BALL = 1 };
enum { ORC_EXIT_BRIDGE = 0, ORC_EXIT_SHIFT = 1, ORC_EXIT_NAIVE = 2 };
enum { ORC_LAW_GAUSS = 0, ORC_LAW_RADEMACHER = 1 };

/* amp * prod_d sin(k[d] x_d + phase[d]) over the first dim coordinates */
typedef struct { double amp; double k[3]; double phase[3]; } orc_trig;
/* coef * prod_d x_d^e[d] */
typedef struct { double coef; int32_t e[3]; } orc_mono;

struct orc_grid_s;

/* Problem: (1/2) sigma^2 Lap u + b.grad u + c u = f in Omega, u = g on dOmega.
 * b(x) = b0 + B x, c(x) = c_a + c_b |x|^2.
 * U = sum of trig terms + sum of monomials (the manufactured solution);
 * f = (1/2) sigma^2 Lap U + b.grad U + c U + sum(fx),  g = U + sum(gx).
 * Tabulated coefficients: a non-NULL grid replaces the analytic b_d, c or f
 * by its interpolant (f's analytic form always uses the analytic b and c);
 * a tabulated g replaces the boundary data U + sum(gx) by its interpolant at
 * the exit point. */
typedef struct {
    int32_t dim;      /* 2 or 3 */
    int32_t domain;   /* ORC_BOX or ORC_BALL */
    double lo[3], hi[3];
    double center[3], radius;
    double sigma;
    double b0[3];
    double B[3][3];   /* b_i = b0_i + sum_j B[i][j] x_j */
    double c_a, c_b;
    int32_t n_trig, n_mono, n_fx, n_gx;
    orc_trig trig[ORC_MAX_TRIG];
    orc_mono mono[ORC_MAX_MONO];
    orc_mono fx[ORC_MAX_MONO];
    orc_mono gx[ORC_MAX_MONO];
    uint64_t seed;
    const struct orc_grid_s *tab_b[3]; /* drift components, or NULL */
    const struct orc_grid_s *tab_c;    /* killing rate, or NULL */
    const struct orc_grid_s *tab_f;    /* source, or NULL */
    const struct orc_grid_s *tab_g;    /* boundary data, or NULL */
} orc_problem;

/* Values at the n[0] x n[1] (x n[2]) points of a uniform grid on [lo,hi],
 * x fastest. */
typedef struct orc_grid_s {
    int32_t dim;
    int32_t n[3];
    double lo[3], hi[3];
    const double *data;
} orc_grid;

typedef struct {
    double h;             /* time step */
    uint64_t n_paths;     /* paths per node */
    uint64_t path_offset; /* index of the first path of each node */
    uint32_t stream;      /* iterate / request index, part of the RNG counter */
    int32_t exit_mode;    /* ORC_EXIT_* */
    int32_t law;          /* ORC_LAW_* */
    uint64_t max_steps;   /* cap on steps per path */
    const orc_grid *u_prev;  /* both NULL: plain estimator */
    const orc_grid *resid;
    /* Ito control variate (eq. F:xiControlVariate): grad[d] holds the
     * component d of grad(u~) for d < dim; grad[0] == NULL: not used.
     * Exclusive with u_prev / resid. */
    const orc_grid *grad[3];
} orc_opts;

typedef struct {
    double phi;      /* plain score g(X_tau) Y + Z */
    double e;        /* correction score; with the Ito control variate phi + xi
                        (NaN in plain mode) */
    uint64_t steps;  /* exit step k */
    int32_t capped;  /* 1 if stopped by max_steps */
    int32_t pad;
    double x_exit[3];
} orc_path;

typedef struct {
    int64_t n, n_capped;
    int64_t steps_sum;
    double mean, var, stderr_, mean_steps;
    double mean_plain, var_plain, cov, rho, vr, vr_opt;
    /* Neumaier pairs (sum, compensation): phi, phi^2, e, e^2, phi*e */
    double sums[10];
} orc_stats;

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The dim normals and the bridge uniform the scheme uses at step s of path
 * (node i, path j). */
void orc_step_normals(const orc_problem *p, const orc_opts *o, uint32_t node,
                      uint64_t path, uint64_t step, double *out_normals);
double orc_bridge_uniform(const orc_problem *p, const orc_opts *o, uint32_t node,
                          uint64_t path, uint64_t step);

/* Coefficients of the problem at a point. */
void orc_drift(const orc_problem *p, const double *x, double *b);
double orc_kill(const orc_problem *p, const double *x);
double orc_U(const orc_problem *p, const double *x);
double orc_source(const orc_problem *p, const double *x);
double orc_boundary(const orc_problem *p, const double *x);
double orc_interp(const orc_grid *g, const double *x);

/* One path from x0 with the scheme's own Philox draws. Returns 0 on success. */
int orc_run_path(const orc_problem *p, const orc_opts *o, const double *x0,
                 uint32_t node, uint64_t path, orc_path *out);

/* One path driven by given noise: normals[k*dim + d] for step k and the bridge
 * uniform unif[k]; at most n_steps steps (the path is capped after them
 * unless max_steps is smaller). Used by brute-force enumeration tests. */
int orc_run_path_noise(const orc_problem *p, const orc_opts *o, const double *x0,
                       const double *normals, const double *unif, uint64_t n_steps,
                       orc_path *out);

/* All paths of all nodes, node by node, path by path, with compensated sums.
 * rec (nullable) receives n_nodes * n_paths records, node-major. */
int orc_solve_nodes(const orc_problem *p, const orc_opts *o, const double *nodes,
                    int64_t n_nodes, orc_stats *out, orc_path *rec);

/* Same, but for an explicit list of (node, path) pairs; no statistics. */
int orc_run_paths(const orc_problem *p, const orc_opts *o, const double *nodes,
                  const uint32_t *node_idx, const uint64_t *path_idx, int64_t n,
                  orc_path *rec);

#ifdef __cplusplus
}
#endif
#endif
