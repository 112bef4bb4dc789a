/*
 * pdd.h - C ABI of the MI355X (gfx950) first-stage PDD nodal solver.
 *
 * The library estimates, at interfacial nodes x0, the solution of the
 * elliptic Dirichlet problem (paper Sec. 2.1, eq. F:EllipticBVP with
 * a_ij = sigma^2 delta_ij)
 *     (1/2) sigma^2 Lap u + b . grad u + c u = f  in Omega,   u = g on dOmega
 * through its probabilistic representation (eq. F:Dynkin)
 *     u(x0) = E[ g(X_tau) Y_tau + Z_tau ],  Y = exp(int c dt), Z = -int f Y dt,
 * sampling independent Euler-Maruyama paths (Sec. 2.3, Alg. 1, eq. F:E_M)
 * with a Brownian-bridge (default), shifted-boundary (Alg. 1) or naive exit
 * test, and the correction estimator of the multigrid-like iteration, where
 * a previous approximation u_prev is the control variate (eqs. F:Statistics_VR,
 * F:xiControlVariate; Alg. 4, the nodal solves inside the outer loop), or
 * with the paper's pathwise Ito control variate xi itself.
 *
 * Conventions
 *  - All functions return a pdd_status; 0 is success. No exception crosses
 *    the ABI. On failure pdd_last_error() returns a thread-local message.
 *  - Invalid arguments are rejected before anything is enqueued.
 *  - "device" pointers are HIP device memory of the context's GPU; "host"
 *    pointers are ordinary CPU memory. `stream` is a hipStream_t passed as
 *    void* (NULL = the default stream). Solves are asynchronous on `stream`:
 *    outputs are valid once the stream has been synchronised.
 *  - A context owns device scratch; solves issued through one context are
 *    ordered on the device (each waits for the previous one), whatever
 *    stream they use. Use one context per concurrent user.
 *  - Limits: nodes < 2^32, paths per node < 2^32, path_offset + n_paths
 *    <= 2^32, stream_id < 2^28, steps per path < 2^31.
 */
#ifndef PDD_H
#define PDD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pdd_status;
#define PDD_OK 0
#define PDD_E_INVALID (-1)     /* bad argument (node outside Omega, dt <= 0, ...) */
#define PDD_E_NOMEM (-2)       /* device or pinned allocation failed */
#define PDD_E_HIP (-3)         /* a HIP runtime call failed */
#define PDD_E_UNSUPPORTED (-4) /* valid but not implemented combination */
#define PDD_E_BUSY (-5)        /* resource in use */
#define PDD_E_INTERNAL (-6)

typedef struct pdd_ctx pdd_ctx;
typedef struct pdd_problem pdd_problem;

enum { PDD_DOMAIN_BOX = 0, PDD_DOMAIN_BALL = 1 };
/* Exit tests: Brownian bridge between consecutive steps (per flat face
 * p = exp(-2 a a' / (sigma^2 h)), faces combined as independent), the
 * Gobet-Menozzi shifted boundary of Alg. 1 (stop when within
 * 0.5826 sigma sqrt(h) of the boundary), or the naive test (stop when a step
 * lands outside). */
enum { PDD_EXIT_BRIDGE = 0, PDD_EXIT_SHIFT = 1, PDD_EXIT_NAIVE = 2 };
/* Law of the increments: Gaussian (Box-Muller) or +-1 (testing only). */
enum { PDD_LAW_GAUSS = 0, PDD_LAW_RADEMACHER = 1 };
/* Path arithmetic: FP32 (per-path integrals and node sums in FP64) or FP64. */
enum { PDD_FP32 = 0, PDD_FP64 = 1 };
enum { PDD_DTYPE_F32 = 0, PDD_DTYPE_F64 = 1 };

/* Solve flags. */
#define PDD_PLAIN_ALONGSIDE 1u /* correction solve: also score phi, report rho, VR
                                  (Ito solves always do) */
#define PDD_TIME_KERNEL 2u     /* record HIP events around the solve's path-kernel launches */
/* `out` (device) already holds this library's statistics of the same nodes,
 * in the same order, from earlier paths of the same problem, estimator, dt,
 * precision, exit test and stream_id (paths below path_offset); the new
 * paths are merged into those sums, so `out` ends up describing all of them
 * (the pilot-then-continue scheme of the balanced simulation, Sec. 3.1). The
 * caller keeps the path ranges disjoint; nothing checks it. */
#define PDD_ACCUMULATE 4u

#define PDD_MAX_TRIG 16
#define PDD_MAX_MONO 8

/* amp * prod_{d<dim} sin(k[d] x_d + phase[d]) */
typedef struct {
    double amp;
    double k[3];
    double phase[3];
} pdd_trig_term;

/* coef * prod_{d<dim} x_d^e[d], 0 <= e[d] <= 8 */
typedef struct {
    double coef;
    int32_t e[3];
} pdd_mono_term;

/* Problem descriptor (eq. F:EllipticBVP; SDE of eq. F:SDE with diffusion
 * sigma I). The drift is affine, b(x) = b0 + B x (B row-major: b_i = b0_i +
 * sum_j B[i][j] x_j); the killing rate is c(x) = c_a + c_b |x|^2 (c <= 0 keeps
 * the problem well posed). The source and boundary data follow from a
 * manufactured function U (trig + monomial terms):
 *   f = (1/2) sigma^2 Lap U + b.grad U + c U + sum(fx),   g = U + sum(gx),
 * so U is the exact solution when fx and gx are empty. The caller's struct
 * is copied; it is not retained. */
typedef struct {
    int32_t dim;    /* 2 or 3 */
    int32_t domain; /* PDD_DOMAIN_BOX: [lo, hi]; PDD_DOMAIN_BALL: |x - center| < radius */
    double lo[3], hi[3];
    double center[3], radius;
    double sigma; /* > 0 */
    double b0[3];
    double B[3][3];
    double c_a, c_b;
    int32_t n_trig, n_mono, n_fx, n_gx;
    pdd_trig_term trig[PDD_MAX_TRIG];
    pdd_mono_term mono[PDD_MAX_MONO];
    pdd_mono_term fx[PDD_MAX_MONO];
    pdd_mono_term gx[PDD_MAX_MONO];
    uint64_t seed; /* Philox4x32-10 key (lo word, hi word) */
} pdd_problem_desc;

/* Values on a uniform grid of n[0] x n[1] (x n[2]) points spanning [lo, hi],
 * x fastest, in device memory. Interpolated bilinearly (trilinearly): cell
 * index clamped to the grid, in-cell weight clamped to [0, 1]. Borrowed: the
 * caller keeps `data` alive until the solve's stream has completed. The grid
 * must cover the bounding box of Omega. */
typedef struct {
    int32_t dim;
    int32_t dtype; /* PDD_DTYPE_F32 or PDD_DTYPE_F64 */
    int32_t n[3];  /* >= 2 each */
    double lo[3], hi[3];
    const void *data;
} pdd_grid;

/* Launch shape of the path kernel. A solve whose opts give no tuning uses the
 * context's entry for its (precision, dim, estimator) group, set by
 * pdd_autotune or pdd_set_tuning, else the default {256, occupancy, 64, 0,
 * 0, 0}; fields left 0 in a given tuning take the default. Results never
 * depend on the launch shape. */
typedef struct {
    int32_t block;        /* threads per workgroup: 64, 128 or 256 */
    int32_t blocks_per_cu;/* persistent workgroups per compute unit */
    int32_t grab;         /* paths a wavefront takes from the queue at a time */
    int32_t max_launch_paths; /* cap on paths per path-kernel launch (0 = 2^27; records
                                 given by the caller: no cap) */
    int32_t refill;       /* walk-loop iterations between refills of the lanes that
                             ended a path: 1, 2, 4 or 8 (0 = 2 in 2D, 4 in 3D; an
                             iteration is two steps in 2D, one in 3D) */
    int32_t bridge;       /* form of the bridge exit test in the box / bridge /
                             Gaussian kernel: 1 per lane, 2 for the whole wave
                             (boundary-dense walks), 0 = by the walk's boundary density */
} pdd_tuning;

typedef struct {
    double dt;                          /* time step h > 0 */
    uint64_t n_paths;                   /* paths per node (used when n_paths_per_node is NULL) */
    const uint64_t *n_paths_per_node;   /* host, n_nodes counts, or NULL */
    uint64_t path_offset;               /* index of each node's first path */
    uint32_t stream_id;                 /* iterate / request index in the RNG counter */
    int32_t precision;                  /* PDD_FP32 or PDD_FP64 */
    int32_t exit_mode;                  /* PDD_EXIT_* */
    int32_t law;                        /* PDD_LAW_* */
    uint64_t max_steps;                 /* 0 = 2^26 */
    uint32_t flags;                     /* PDD_PLAIN_ALONGSIDE | PDD_TIME_KERNEL | PDD_ACCUMULATE */
    int32_t reserved;
    /* Optional per-path records (device, NULL = not kept). Path jj of node i
     * sits at slot s = sum_{i'<i} N_i' + jj: rec_phi[s] = phi, rec_e[s] = e
     * (correction solves) or phi + xi (Ito solves), rec_steps[s] = exit step
     * | (capped << 31). */
    double *rec_phi;
    double *rec_e;
    uint32_t *rec_steps;
    const pdd_tuning *tuning;           /* NULL = default / tuned */
} pdd_solve_opts;

/* Per-node result (Sec. 2.2 eq. F:Statistical_error; Sec. 2.3 eqs.
 * F:Variance_Reduction, F:Rho). Plain solve: mean/var/stderr of phi.
 * Correction solve: mean = u_prev(x0) + mean(e), var/stderr of e; with
 * PDD_PLAIN_ALONGSIDE also mean_plain/var_plain of phi, cov = Cov[phi, xi]
 * and rho = rho[phi, xi] for the control variate xi = u_prev(x0) + e - phi,
 * vr = var_plain / var and vr_opt = 1 / (1 - rho^2). Ito solve: the same
 * with e = phi + xi and mean = mean(e) (no u_prev term), the plain fields
 * always filled. Unused fields are NaN.
 * sums: Neumaier pairs (sum, compensation) of phi, phi^2, e, e^2, phi*e, so
 * that results of disjoint path ranges can be merged exactly enough. */
typedef struct {
    int64_t n, n_capped, steps_sum;
    double mean, var, stderr_, mean_steps;
    double mean_plain, var_plain, cov, rho, vr, vr_opt;
    double sums[10];
} pdd_node_stats;

/* One item of a batched solve. */
typedef struct {
    pdd_problem *problem;
    const double *nodes;        /* host, n_nodes x dim, row-major */
    int64_t n_nodes;
    const pdd_solve_opts *opts;
    const pdd_grid *u_prev;     /* both NULL: plain estimator */
    const pdd_grid *resid;
    pdd_node_stats *out;        /* device, n_nodes entries */
    const pdd_grid *grad;       /* NULL, or dim gradient grids: Ito control variate
                                   (as pdd_solve_ito; excludes u_prev / resid) */
} pdd_work_item;

/* Creates a context on HIP device `hip_device` (made current for the call). */
pdd_status pdd_init(pdd_ctx **out, int hip_device);
/* Waits for the context's work and frees its scratch. NULL is a no-op. */
void pdd_shutdown(pdd_ctx *ctx);

/* Validates and uploads a problem (eq. F:EllipticBVP). */
pdd_status pdd_create_problem(pdd_ctx *ctx, const pdd_problem_desc *desc, pdd_problem **out);
/* Frees a problem; the caller ensures no solve using it is in flight. */
void pdd_destroy_problem(pdd_problem *problem);

/* Coefficients given on grids (Sec. 2.1, eq. F:EllipticBVP: b, c and f are
 * general functions of x; the analytic family of pdd_problem_desc is a special
 * case). Each non-NULL grid replaces one coefficient of the descriptor by its
 * bilinear / trilinear interpolant (the pdd_grid rule): b[d] the drift
 * component d (d < dim), c the killing rate, f the source, g the boundary
 * data (read at the exit point; without it g = U + sum(gx)). A grid has the
 * problem's dim, n[d] >= 2 points per axis, dtype PDD_DTYPE_F32 or F64, data
 * in device memory (x fastest) and a box [lo, hi] that contains the domain
 * (the box itself, or the ball's bounding box). A NULL f keeps the source's
 * analytic form, which uses the descriptor's analytic b and c. */
typedef struct {
    const pdd_grid *b[3];
    const pdd_grid *c;
    const pdd_grid *f;
    const pdd_grid *g;
} pdd_coef_grids;

/* As pdd_create_problem, with tabulated coefficients. The grids are read
 * during the call: the library keeps its own copies (laid out by cell, in both
 * path precisions) and the caller may free the grids when the call returns.
 * Synchronous on the device. Errors: PDD_E_INVALID for a NULL `grids`, a
 * malformed grid or one that does not contain the domain; PDD_E_NOMEM when
 * the copies cannot be allocated; PDD_E_HIP on a device error. */
pdd_status pdd_create_problem_tabulated(pdd_ctx *ctx, const pdd_problem_desc *desc,
                                        const pdd_coef_grids *grids, pdd_problem **out);

/* Plain estimator phi at n_nodes nodes (Sec. 2.3, Alg. 1: Euler-Maruyama
 * paths of eq. F:E_M from each node, score phi = g(X_tau) Y_tau + Z_tau of eq.
 * F:Dynkin; statistics of Sec. 2.2, eq. F:Statistical_error). `nodes`: host
 * array, n_nodes x dim, row-major; every node strictly inside Omega. `out`:
 * device memory of n_nodes entries, written when the stream reaches the end
 * of the solve. n_nodes == 0 is a no-op. Errors (nothing is enqueued):
 * PDD_E_INVALID for NULL pointers, a node outside Omega, dt <= 0, bad enums
 * or limits; PDD_E_UNSUPPORTED for FP32 paths whose trig terms leave the
 * hardware sine's range; PDD_E_NOMEM / PDD_E_HIP from the device. */
pdd_status pdd_solve_nodes(pdd_problem *problem, const double *nodes, int64_t n_nodes,
                           const pdd_solve_opts *opts, pdd_node_stats *out, void *stream);

/* pdd_solve_nodes for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. Same
 * arguments, results and errors as pdd_solve_nodes, and the same statistics
 * bit for bit whenever the solve's paths fit one launch of this variant
 * (2^21 paths, or tuning->max_launch_paths); above that its launches cut the
 * node sums at other places and the statistics agree to rounding.
 * Limits: one path count for all nodes (n_paths_per_node NULL), at most
 * PDD_NOALLOC_MAX_NODES nodes, no PDD_TIME_KERNEL (PDD_E_UNSUPPORTED
 * otherwise). The call allocates nothing, neither device nor pinned memory:
 * its working memory is a static device array of PDD_NOALLOC_SCRATCH_BYTES
 * per GPU, held from the library's load until the process ends, and the node
 * table and problem reach the device as kernel arguments. Calls on one GPU
 * share that array: two such calls in flight at once on one GPU (other
 * streams, other contexts) race, and the caller must order them; the
 * context's other solves use their own memory and do not conflict. */
#define PDD_NOALLOC_SCRATCH_BYTES (32u << 20)
#define PDD_NOALLOC_MAX_NODES 32768
pdd_status pdd_solve_nodes_noalloc(pdd_problem *problem, const double *nodes, int64_t n_nodes,
                                   const pdd_solve_opts *opts, pdd_node_stats *out, void *stream);

/* Correction estimator of the multigrid-like iteration (Sec. 2.3, eqs.
 * F:Statistics_VR and F:xiControlVariate with gamma = 1, rewritten by Ito's
 * formula so that no gradient is needed): a previous approximation u_prev is
 * the control variate; along each path R = sum h Y_k r(X_k) with the residual
 * r = f - (L + c) u_prev, the score is e = (g - u_prev)(X_tau) Y_tau - R and
 * the node value u_prev(x0) + mean(e). u_prev and r are grids of the
 * problem's dim in the path precision's dtype (borrowed until the stream
 * completes). Arguments, outputs and errors as for pdd_solve_nodes, plus
 * PDD_E_INVALID for a missing or malformed grid or one that does not cover
 * Omega, PDD_E_UNSUPPORTED for a grid dtype other than the path precision's. */
pdd_status pdd_solve_correction(pdd_problem *problem, const pdd_grid *u_prev,
                                const pdd_grid *resid, const double *nodes, int64_t n_nodes,
                                const pdd_solve_opts *opts, pdd_node_stats *out, void *stream);

/* The plain estimator with the paper's pathwise control variate (Sec. 2.3,
 * eqs. F:VR_Milstein_sys with F = -sigma grad(u~), F:xiControlVariate): along
 * each path xi_{k+1} = xi_k - Y_k sigma grad(u~)(X_k) . sqrt(h) N_k, with the
 * normals N_k of the same Euler-Maruyama step (the Alg. 1 xi line read with
 * the Brownian increment, as the Ito integral requires), and the score is
 * phi + xi; E[xi] = 0, so the estimate is unbiased for any u~, and its
 * variance vanishes with h when u~ = u. `grad` points to dim grids, grad[d]
 * holding the component d of grad(u~), all with the same n, lo and hi and
 * the dtype of the path precision (rules of pdd_grid; borrowed until the
 * stream completes). Statistics as described at pdd_node_stats; records need
 * rec_phi and rec_e. Errors as for pdd_solve_nodes, and PDD_E_INVALID for a
 * NULL `grad`, a malformed grid or grids of different geometries. */
pdd_status pdd_solve_ito(pdd_problem *problem, const pdd_grid *grad, const double *nodes, int64_t n_nodes,
                         const pdd_solve_opts *opts, pdd_node_stats *out, void *stream);

/* Many solves at once (the nodal solves of Alg. 1 for several problems, or
 * the iterates of one): items are grouped by (precision, dim, estimator) and
 * each group runs as one persistent launch (work items with their own
 * queues; alike solves merged). Each item's results equal those of its own
 * pdd_solve_nodes / pdd_solve_correction / pdd_solve_ito call bit for bit.
 * Errors as for those calls; the first invalid item fails the whole call
 * before anything is enqueued. */
pdd_status pdd_solve_batch(pdd_ctx *ctx, const pdd_work_item *items, int32_t n_items,
                           void *stream);

/* Path counts of a balanced simulation (Sec. 3.1, Def. D:Balanced_MC_simulation,
 * eq. F:N_y_h): for accuracy a at confidence q the statistical error q SE
 * must equal a/2, i.e. SE = a/(2q) and N = V[phi]/SE^2 = 4 q^2 V[phi]/a^2.
 * Given pilot statistics (host, n_nodes entries, each with n >= 2), writes
 *   n_total[i] = min(n_max, max(pilot[i].n, ceil(pilot[i].var / target_se^2)))
 * to n_total (host). `var` is that of the estimator the pilot ran (phi for
 * the plain solve, e for the correction). Host only; needs no GPU.
 * Errors: NULL pointers, n_nodes < 0, target_se not finite and > 0, a pilot
 * with n < 2 or a non-finite variance. */
pdd_status pdd_plan_paths(const pdd_node_stats *pilot, int64_t n_nodes, double target_se,
                          uint64_t n_max, uint64_t *n_total);

/* Solves items to a standard error: a pilot of n_pilot paths per node (paths
 * path_offset .. path_offset + n_pilot - 1 of each item's opts; the opts'
 * n_paths and n_paths_per_node are ignored), then pdd_plan_paths per item with
 * target_se[q] (host, n_items values), then the missing paths of every node
 * from path_offset + n_pilot on, merged into the pilot's statistics
 * (PDD_ACCUMULATE). Blocks until the pilot has finished; the continuation is
 * asynchronous on `stream`. n_pilot >= 2, n_max >= n_pilot. Items' `out`
 * receive the final statistics. Paths of a node are the same whichever
 * items share the call. */
pdd_status pdd_solve_to_tolerance(pdd_ctx *ctx, const pdd_work_item *items, int32_t n_items,
                                  const double *target_se, uint64_t n_pilot, uint64_t n_max,
                                  void *stream);

/* ------------------------------------------------------------------------
 * Fast fit of nodal constants (Sec. 5, heuristic H5, Alg. A:Fitting). Host only
 * except for the batched solve of pdd_fit_constants.
 * ------------------------------------------------------------------------ */
enum { PDD_GLM_NORMAL = 0, PDD_GLM_GAMMA = 1 };

/* Maximum-likelihood fit of y = coef[0] + coef[1] x (identity link) with normal
 * noise (least squares; the first-moment model of eq. F:Noisy_model_moment1)
 * or gamma noise (Fisher scoring from mu = y, weights 1 / mu^2, a step that
 * would make a mean non-positive is halved; the second-moment model of eq.
 * F:Noisy_model_moment2), n >= 3 points (host arrays). se[k] =
 * sqrt(dispersion * (X'WX)^-1_kk), the dispersion from the Pearson residuals
 * with n - 2 degrees of freedom; iterations (nullable) = scoring passes (1 for
 * the normal family). Errors: NULL pointers, n < 3, non-finite data,
 * non-positive y for the gamma family, x values that do not span a line. */
pdd_status pdd_glm_fit(const double *x, const double *y, int32_t n, int32_t family, double *coef, double *se,
                       int32_t *iterations);

/* Fitted constants of one node. The model in x = h^delta: E[phi_h] = E_phi +
 * beta x (normal fit of the node means; beta is the bias constant of eq.
 * F:Bound_of_error), V[phi_h] = V_phi + alpha x (gamma fit of the sample
 * variances), E[tau_h] = E_tau + beta_tau x (normal fit of h times the mean
 * exit step), with standard errors; iterations of the gamma fit. For a
 * correction or Ito item, phi is that estimator's score and mean its node
 * value. */
typedef struct {
    double E_phi, beta, se_E_phi, se_beta;
    double V_phi, alpha, se_V_phi, se_alpha;
    double E_tau, beta_tau, se_E_tau;
    int32_t iterations, pad;
} pdd_node_constants;

/* Alg. A:Fitting for the nodes of `item`: n_h >= 3 solves of n_hat >= 2
 * paths per node at the steps h[0 .. n_h - 1] (host; the paper takes a cloud
 * of about 100 equispaced steps and n_hat = 1000), solve j with RNG stream
 * item->opts->stream_id + j and otherwise the item's options (its dt,
 * n_paths, records and accumulate flag are ignored), run as one
 * pdd_solve_batch; then per node the three fits of pdd_node_constants in
 * x = h^delta (delta > 0: 1 for the bridge and shifted exits, 1/2 for the
 * naive one). `out`: host, item->n_nodes entries. Synchronous. Errors as for
 * the solve, and PDD_E_INVALID for bad h, n_h, n_hat or delta, or a node whose
 * sample variance is 0 at some step. */
pdd_status pdd_fit_constants(pdd_ctx *ctx, const pdd_work_item *item, const double *h, int32_t n_h,
                             uint64_t n_hat, double delta, pdd_node_constants *out, void *stream);

/* Nodal constants of the scheduling algorithm (Alg. A:Scheduling): K the
 * cost constant of eq. F:Pointwise_cost (4 q^2 E[tau] (2 |beta|)^(1/delta)),
 * V = V[phi], alpha, beta the fitted variance and bias constants
 * (pdd_fit_constants), V_psi = V[psi-bar] and rho_psi = rho[phi, psi-bar]
 * of the auxiliary variate psi-bar of eq. F:Bar_psi. */
typedef struct {
    double K, V, alpha, beta, V_psi, rho_psi;
} pdd_sched_node;

/* Alg. A:Scheduling: from a_0 (the nodal target tolerance), each a_{j+1}
 * minimises over (a_j, a_max] the sum over nodes of
 *   K V (kappa (1 - r^2(a) + |alpha r(a) / beta| a_j) + (a_j / a)^(2 + 1/delta)),
 *   r^2(a) = 1 - V_psi a^2 (1 - rho_psi^2) / (4 V)  (eq. F:Sensitivity_formula,
 * kept in [0, 1]); minimised on a 512-point log grid, then by golden section
 * around its best point. The loop stops when the predicted speedup of the
 * level, (sum K V) / that minimum = cost(PlainPDD(a_j)) / cost(IterPDD(a_j,
 * a_{j+1})) without the subdomain terms (eqs. F:PlainPDD_cost,
 * F:IterPDD_cost), falls below s_min (the paper stops at 1.5, Sec. 6; that
 * level is not taken), when a_j reaches a_max, or after max_levels levels.
 * Writes a_out[0 .. J] = a_0 < a_1 < ... < a_J (host, max_levels + 1 values),
 * the levels' predicted speedups to speedup[0 .. J - 1] (nullable) and J to
 * n_levels. Host only. Errors: NULL pointers, n < 1, a bad constant, or not
 * 0 < a_0 < a_max, kappa > 0, delta > 0, s_min > 0. */
pdd_status pdd_schedule(const pdd_sched_node *nodes, int64_t n, double a0, double kappa, double delta, double a_max,
                        double s_min, int32_t max_levels, double *a_out, double *speedup, int32_t *n_levels);

/* Gradient of a gridded u~ by second-order finite differences (the grad(u~)
 * grids of pdd_solve_ito when only values of u~ on a grid are known, as
 * inside the outer iteration of Sec. 2.3): with dx_d = (hi_d - lo_d) /
 * (n_d - 1), the central difference (u[i+1] - u[i-1]) / (2 dx_d) inside and
 * (-3 u[0] + 4 u[1] - u[2]) / (2 dx_d), (3 u[n-1] - 4 u[n-2] + u[n-3]) /
 * (2 dx_d) at the two ends of each axis; exact for quadratics. `u`: a grid
 * (pdd_grid rules, n_d >= 3, device data); `grad`: host array of dim device
 * pointers, grad[d] receiving the n_0 n_1 (n_2) values of component d in u's
 * dtype and layout (the caller allocates them; with u's n, lo, hi they form
 * the gradient grids). Asynchronous on `stream`. Errors: NULL pointers, a
 * malformed grid, n_d < 3; PDD_E_HIP on a launch failure. */
pdd_status pdd_grid_gradient(pdd_ctx *ctx, const pdd_grid *u, void *const *grad, void *stream);

/* Residual r = f - ((1/2) sigma^2 Lap u~ + b.grad u~ + c u~) of a gridded u~
 * (the residual grid of pdd_solve_correction when only values of u~ are
 * known, as inside the outer iteration), at the grid's points, with the
 * problem's b, c, f (analytic or tabulated, evaluated in FP64) and the
 * derivatives of u~ by second-order differences: those of pdd_grid_gradient
 * for grad u~, (u[i+1] - 2 u[i] + u[i-1]) / dx^2 inside and
 * (2 u[0] - 5 u[1] + 4 u[2] - u[3]) / dx^2 (mirrored) at the ends for the
 * second derivatives; exact for quadratic u~. `u`: a grid of the problem's
 * dim (pdd_grid rules, n_d >= 4, device data); `resid`: device buffer of the
 * same size and dtype (caller-allocated; with u's n, lo, hi it is the residual
 * grid). Asynchronous on `stream`. Errors: NULL pointers, dim mismatch, a
 * malformed grid, n_d < 4; PDD_E_HIP on a launch failure. */
pdd_status pdd_grid_residual(pdd_problem *problem, const pdd_grid *u, void *resid, void *stream);

/* ------------------------------------------------------------------------
 * Second stage of PDD (Sec. 1; Alg. A:IterPDD, the subdomain-BVP step) on a
 * 2D box cut into subdomains by axis-parallel interfaces: the nodal values
 * are interpolated along every interface line and every subdomain is solved,
 * giving the global approximation u~ = (+)_k v_k on a grid.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n[2];          /* grid points per axis over the problem's box (>= 3): u~'s grid */
    int32_t n_cuts[2];     /* interfaces x_0 = c (axis 0) and x_1 = c (axis 1) */
    const double *cuts[2]; /* host: their coordinates; each on an interior grid line */
    double rbf_eps;        /* shape parameter of the multiquadric sqrt(1 + (eps r)^2), > 0 */
} pdd_partition;

/* u~ on the n[0] x n[1] grid over the box (device, FP64, x fastest; written
 * whole). The physical boundary gets the problem's g. Every interface line
 * gets the multiquadric interpolant R (Def. D:Linear_interpolator; the
 * paper's experiment, Sec. 6, uses multiquadric RBFs) of the data on it: the
 * values of the nodes lying on the line and g at the line's two ends on the
 * boundary (s(t) = sum_m lam_m sqrt(1 + (eps (t - t_m))^2), lam from
 * s(t_m) = z_m); where an axis-0 and an axis-1 line cross, the mean of the two.
 * Every subdomain (the grid box between consecutive interfaces) is then solved
 * for (1/2) sigma^2 Lap v + b.grad v + c v = f with the values on its
 * boundary, by second-order finite differences on the grid (central second
 * and first differences, b, c, f of the problem in FP64) and a banded LU
 * factorisation without pivoting, one workgroup per subdomain. The factors
 * depend on the operator (sigma, b, c), the grid and the interfaces only, so
 * the context keeps those of its last call. Since a subdomain's solution is
 * affine in its boundary values, the context also keeps, per subdomain, its
 * solution for f with zero boundary values and its response to a unit value
 * at each row next to the boundary (computed from the factors; at most 2 GiB
 * in all, else every call substitutes): a call with the same operator, grid,
 * interfaces and problem (another set of nodal values) then only adds up
 * those columns, weighted by its boundary values, in a fixed order. The
 * result equals the direct solve to rounding (the same in a fresh context
 * and in a kept one, bit for bit); PDD_STAGE2_SUBSTITUTE=1 in the
 * environment makes every call substitute instead. `nodes` (host,
 * n_nodes x 2) are the interface nodes and `values` (host) their nodal
 * values; a node may lie on several lines. Synchronous (the interpolation
 * weights are solved on the host once the boundary values are on the
 * device); u is complete when the call returns. Errors: PDD_E_INVALID for
 * NULL pointers, a bad grid or shape parameter, an interface off the grid
 * lines or given twice, a node off every interface or outside the box, a
 * singular interpolation system; PDD_E_UNSUPPORTED for a problem that is not
 * a 2D box or a subdomain whose shorter side has more than 64 interior
 * points; PDD_E_NOMEM / PDD_E_HIP from the device. */
pdd_status pdd_stage2(pdd_problem *problem, const pdd_partition *part, const double *nodes, const double *values,
                      int64_t n_nodes, double *u, void *stream);

/* Key of the context's launch-shape table: the path kernel a group of
 * items runs. `generic` selects between the kernel compiled for a box domain
 * with the bridge exit test, Gaussian increments and analytic coefficients
 * (0: used when every item of the group is of that kind) and the generic one
 * (1: ball domains, the shifted or naive exit test, the test law, tabulated
 * coefficients). */
typedef struct {
    int32_t precision;  /* PDD_FP32 or PDD_FP64 */
    int32_t dim;        /* 2 or 3 */
    int32_t correction; /* 0 plain, 1 correction estimator, 2 Ito control variate */
    int32_t generic;    /* 0 or 1, as above */
} pdd_tuning_key;

/* Times samples of `item` (up to 32 of its nodes, about 8 and 16 paths per
 * resident lane in all, its dt, precision, exit test, law, stream and grids;
 * its path counts, records and tuning are ignored) under the launch shapes
 * block {64, 128, 256} x grab {16, 64, 256} at full occupancy, and block 256
 * with 3/4 and 1/2 of the occupancy, twice each after a warm-up; then, with
 * the best shape, the refill periods {1, 2, 4, 8} and, in the box / bridge /
 * Gaussian kernel, both forms of the bridge test. A candidate's cost is the
 * time of the larger sample minus that of the smaller, which leaves out fixed
 * costs and the exit-time tail. The default {256, occupancy, 64} (and the
 * default period and form) is kept unless a candidate is more than 2% faster.
 * The winner is written to `out` (host) and stored in the context's table
 * for the item's key. The tuner takes a work item rather than a problem and
 * options alone because the item also holds what the estimator reads (the
 * u_prev and residual grids, or the gradient grids) and the nodes to sample.
 * Synchronous; uses the context like a solve. Errors as for the solve. */
pdd_status pdd_autotune(pdd_ctx *ctx, const pdd_work_item *item, pdd_tuning *out);

/* Sets (t non-NULL) or removes (t NULL) the context's table entry for `key`,
 * e.g. to restore shapes tuned earlier. PDD_E_INVALID for a bad key (any
 * field out of its range) or shape. */
pdd_status pdd_set_tuning(pdd_ctx *ctx, const pdd_tuning_key *key, const pdd_tuning *t);

/* GPU milliseconds between the first path-kernel launch and the end of the
 * last one, for each solve issued with PDD_TIME_KERNEL since the previous
 * call, oldest first. Waits for those solves. Writes at most `cap` values to
 * `ms` (host) and their count to `n`; the rest are dropped. */
pdd_status pdd_kernel_times(pdd_ctx *ctx, double *ms, int32_t cap, int32_t *n);

/* ------------------------------------------------------------------------
 * Serving loop: continuous batching of node-solve requests, each to its own
 * standard error (pilot, plan by pdd_plan_paths, continuation in chunks).
 *
 * A server owns a host thread and is the only user of its context while it
 * lives. The thread runs epochs: each epoch is one pdd_solve_batch-style
 * launch per (precision, dim, estimator) group over the next chunk of
 * admitted requests (a new request's pilot, or the next slice of its planned
 * paths), pilots first, then the requests with the least remaining work
 * (path-steps estimated from the pilot), up to epoch_paths. Up to `pipeline`
 * epochs are in flight at once, each on its own HIP stream with its own
 * scratch (the first on the server's context, the others on contexts the
 * server creates on the same device): while one epoch finishes its longest
 * paths, the next one, over requests not in flight, already fills the idle
 * compute units, and the host plans finished pilots meanwhile. A request is
 * in at most one epoch in flight, so its chunks run in order. Requests
 * submitted while epochs run wait in a FIFO queue and are admitted at the
 * next epoch boundary when a slot is free and their device memory fits the
 * budget; their chunks then share the launches with those already admitted.
 * A request's chunks depend only on the request and the server options, and
 * each group of an epoch is a single launch, so its results are bitwise the
 * same alone, in any mix, and at any pipeline depth.
 * ------------------------------------------------------------------------ */
typedef struct pdd_server pdd_server;

typedef struct {
    uint64_t memory_budget; /* device bytes for admitted requests and the record scratch (0 = 64 GiB) */
    int32_t max_inflight;   /* requests admitted at once (0 = 1024) */
    int32_t max_queued;     /* submit sheds (PDD_E_BUSY) beyond this many waiting requests (0 = no limit) */
    uint64_t n_pilot;       /* pilot paths per node (0 = 1000) */
    uint64_t n_max;         /* paths per node at most (0 = 2^31) */
    uint64_t chunk_paths;   /* paths of one request per epoch, cut per request (0 = 2^22) */
    uint64_t epoch_paths;   /* paths per epoch launch, <= 2^27 (0 = 2^27) */
    int32_t pipeline;       /* epochs in flight at once, 1 to 4 (0 = 2); each holds a
                               record scratch of epoch_paths paths */
    int32_t reserved;       /* 0 */
} pdd_server_opts;

typedef struct {
    pdd_problem *problem;        /* kept alive by the caller until completion */
    const double *nodes;         /* host, n_nodes x dim; copied by pdd_server_submit */
    int64_t n_nodes;             /* >= 1 */
    double dt;
    double target_se;            /* per-node standard error to reach (> 0) */
    int32_t precision;           /* PDD_FP32 or PDD_FP64 */
    int32_t exit_mode;           /* PDD_EXIT_* */
    uint32_t stream_id;          /* RNG stream of the request */
    int32_t reserved;
    const pdd_grid *u_prev;      /* both NULL: plain estimator; else the correction (structs */
    const pdd_grid *resid;       /* copied, data borrowed until completion) */
    pdd_node_stats *out;         /* host, n_nodes entries; final statistics, written before
                                    the completion is reported */
    uint64_t user_tag;           /* returned in the completion */
    const pdd_grid *grad;        /* NULL, or the problem's dim gradient grids of u~ (one
                                    geometry): the Ito control variate, as pdd_solve_ito;
                                    not with u_prev / resid (structs copied, data borrowed
                                    until completion) */
} pdd_request;

typedef struct {
    uint64_t id, user_tag;
    pdd_status status;           /* PDD_OK, or why the request failed (PDD_E_BUSY: cancelled) */
    int32_t reserved;
    double queued_ms;            /* submit to admission */
    double latency_ms;           /* submit to completion */
    uint64_t paths, path_steps;  /* over all nodes */
    int64_t n_nodes;
} pdd_completion;

/* Latency percentiles count every request that was not shed: a completed
 * one at its latency, and one that was cancelled or has not finished yet at
 * its age (submit to cancellation, or to the report), which is only a lower
 * bound of its latency ("censored"). A percentile is then itself a lower
 * bound when some censored age is at or below it (p50_censored /
 * p99_censored = 1); with no censored request it is exact. Nearest-rank
 * percentiles. */
typedef struct {
    uint64_t submitted, shed, admitted, completed;
    uint64_t failed;                          /* ended with an error other than cancellation */
    uint64_t queued, inflight, epochs;
    uint64_t nodes_completed, path_steps;
    uint64_t mem_in_use, mem_peak, mem_fixed; /* bytes: admitted requests; their peak; record scratch */
    double p50_ms, p99_ms;                    /* latency percentiles of every request not shed (above) */
    double mean_ms;                           /* mean latency of completed requests */
    double wall_s;                            /* first submit to last completion */
    double node_solves_per_s;                 /* nodes_completed / wall_s */
    double epoch_s;                           /* enqueue-to-done time summed over epochs (epochs in
                                                 flight together each count) */
    uint64_t cancelled;                       /* cancelled by pdd_server_destroy */
    uint64_t censored;                        /* requests counted at their age (cancelled or unfinished) */
    int32_t p50_censored, p99_censored;       /* 1: the percentile is a lower bound */
    double p50_done_ms, p99_done_ms;          /* percentiles of completed requests alone */
    double busy_s;                            /* time with at least one epoch in flight */
    uint64_t paths_run;                       /* paths enqueued in epochs (cancelled requests' too) */
} pdd_server_report;

/* Starts a server on `ctx` (NULL opts = defaults). Errors: bad options, a
 * budget smaller than the record scratch (pipeline x epoch_paths x 20 bytes),
 * thread, stream or context creation. */
pdd_status pdd_server_create(pdd_ctx *ctx, const pdd_server_opts *opts, pdd_server **out);
/* Validates and queues a request; writes its id. PDD_E_INVALID: bad request;
 * PDD_E_NOMEM: it can never fit the budget; PDD_E_UNSUPPORTED: its pilot
 * exceeds epoch_paths; PDD_E_BUSY: shed (queue full or server stopping). */
pdd_status pdd_server_submit(pdd_server *server, const pdd_request *req, uint64_t *id);
/* Moves up to `cap` completions (oldest first) to `out` (host) and writes
 * their count to `n`, waiting up to wait_ms (0 = no wait) for the first. */
pdd_status pdd_server_poll(pdd_server *server, pdd_completion *out, int32_t cap, int32_t *n,
                           int32_t wait_ms);
/* Counters and latency percentiles so far (pdd_server_report). */
pdd_status pdd_server_report_get(pdd_server *server, pdd_server_report *out);
/* Stops the server: the epochs in flight end, requests still queued or in
 * flight are cancelled (their `out` is not written), device memory and the
 * server's own contexts are freed. NULL is a no-op. */
void pdd_server_destroy(pdd_server *server);

/* Message of the last failure on this thread ("" if none). */
const char *pdd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PDD_H */
