// Internal structures shared by the host runtime and the HIP kernels of the
// first-stage PDD nodal solver. Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdd.h"

namespace pdd {

constexpr int kMaxTrig = 16;
constexpr int kMaxMono = 8;
constexpr int kExitBridge = 0, kExitShift = 1, kExitNaive = 2;
constexpr int kLawGauss = 0, kLawRademacher = 1;
constexpr int kBox = 0, kBall = 1;
constexpr uint32_t kCappedBit = 0x80000000u;
// Estimators: plain phi; the correction estimator (u_prev and its residual on
// grids); phi + xi with the Ito control variate xi (gradient grids).
constexpr int kEstPlain = 0, kEstCorrection = 1, kEstIto = 2;

// One trig term amp * prod_d sin(k_d x_d + ph_d). In FP32, k and ph are in
// revolutions (k / 2 pi, ph / 2 pi: the hardware sine takes revolutions); in
// FP64 in radians. ak_d = amp * k_d (radians), nhk2a = -(1/2) sigma^2 |k|^2 amp.
template <class T>
struct DevTrig {
    T amp, nhk2a;
    T k[3], ph[3], ak[3];
};

// coef * x^e0 y^e1 z^e2, exponents packed e0 | e1 << 8 | e2 << 16.
template <class T>
struct DevPoly {
    T coef;
    uint32_t e;
};

constexpr int kMaxF = 64;  // terms of the expanded polynomial part of f
constexpr int kMaxG = 16;  // terms of the polynomial part of g
// Dense form of the polynomial part of f, evaluated without loops: total
// degree <= 5 in 2D (21 coefficients), <= 4 in 3D (35 coefficients).
constexpr int kDenseDeg2 = 5, kDenseDeg3 = 4, kMaxDense = 35;
constexpr int kPolyNone = 0, kPolyDense = 1, kPolySparse = 2;

// Problem in the precision of the path arithmetic; passed by value as a kernel
// argument, so every lane reads it through the scalar unit. The manufactured
// function is U = sum(trig) + P with P a sum of monomials; the host expands
// F = (1/2) sigma^2 Lap P + b.grad P + c P + fx and G = P + gx into monomials,
// so that f = F + sum over trig terms of ((1/2) sigma^2 Lap + b.grad + c) T and
// g = G + sum(trig).
// A grid as the kernels read it: value(x) = bilinear / trilinear interpolation.
// The values have the type of the path arithmetic.
template <class T>
struct GridView {
    const T *data;
    const T *cells;  // the same values by cell, corners of a cell together (or null)
    int32_t n[3];
    int32_t pad;
    T lo[3];
    T inv[3];  // (n - 1) / (hi - lo)
    T top[3];  // n - 1
};

template <class T>
struct DevProblem {
    int32_t dim, domain;
    int32_t n_trig, n_f, n_g;
    int32_t f_mode;  // kPolyNone, kPolyDense or kPolySparse
    uint32_t key0, key1;
    T lo[3], hi[3], center[3];
    T radius, radius2;
    T b0[3];
    T B[3][3];
    T c_a, c_b;
    DevTrig<T> trig[kMaxTrig];
    DevPoly<T> fpoly[kMaxF];
    DevPoly<T> gpoly[kMaxG];
    // dense coefficients of F, ordered for nested Horner evaluation: 2D by
    // j (power of y) then i (power of x), i + j <= 5; 3D by k, j, i
    T fdense[kMaxDense];
    // tabulated coefficients: bit q of tab set when tabv[q] replaces the
    // analytic b_0, b_1, b_2, c, f, g (q = 0..5); read through their cell layout
    uint32_t tab;
    int32_t tab_pad;
    GridView<T> tabv[6];
    // bit 6 of tab: b_0 .. b_{dim-1}, c and f are all tabulated on one
    // geometry and interleaved (tabv[q] then keep only the geometry): cell r's
    // record at tab_fused + r (dim + 2) 2^dim holds the 2^dim corners of b_0,
    // ..., c, f in that order; with bit 7 too (2D only), grid point p (x
    // fastest, rows 0 .. n1 - 2) has its record at tab_fused + 8 p: the values
    // of b_0, b_1, c, f at p, then at p + n0 (the point above).
    const T *tab_fused;
};


// Values of a grid gathered by cell: cell (i, j[, k]) at ((k (n1 - 1) + j)
// (n0 - 1) + i) 2^dim, its corners in the order (0,0[,0]), (1,0), (0,1),
// (1,1)[, then the same at k + 1]. One interpolation then reads one aligned
// block instead of 2^dim scattered values.
template <class T>
size_t cell_values(const int32_t *n, int dim)
{
    size_t c = (size_t)1 << dim;
    for (int d = 0; d < dim; ++d) c *= (size_t)(n[d] - 1);
    return c;
}

// One work item: the paths of one solve (one problem, its nodes, its
// estimator and options). Items occupy consecutive ranges of a launch group's
// slot space; slot s of the item belongs to its node i with
// node_start[i] <= s - slot_begin < node_start[i + 1] (or i = (s - slot_begin)
// / uniform_n). Every lane of a wave reads it at the same address, so the
// kernels serve it from the scalar cache.
template <class T>
struct ItemCore {
    int32_t prob;               // index into the problem table (batches)
    int32_t exit_mode, law;
    int32_t score_plain;        // 1: evaluate f and score phi
    uint32_t stream_tag;        // stream_id << 4
    uint32_t max_steps;
    uint32_t n_nodes;
    uint32_t rec_launch;        // 1: scratch records, at group slot - launch start
    int32_t dense_bridge;       // 1: the bridge form for boundary-dense walks (generic kernel)
    int32_t pad_;
    uint64_t slot_begin;        // first slot of the item in the group's slot space
    uint64_t n_slots;
    uint64_t uniform_n;         // paths per node when node_start is null
    uint64_t path_offset;
    uint64_t rec_base;          // record of item slot r at r - rec_base (caller records: 0)
    const double *nodes;        // n_nodes x dim
    const uint64_t *node_start; // n_nodes + 1 item-relative prefix, or null
    double *rec_phi;
    double *rec_e;
    uint32_t *rec_steps;
    T h, sig_sqh, two_over_s2h, gm_thresh, bridge_thresh;
    GridView<T> u_prev, resid;
};

// A work item of the batch kernel: the core fields, plus (per node, 4 words)
// the node index, stream tag and path offset (low word) of the node in the
// solve it belongs to, when several solves that walk alike are merged into
// this item; null: node, stream_tag, path_offset of the core. The
// single-item kernel takes the core alone. Ito items read the components of
// grad(u~) from grad[0 .. dim - 1] (one grid geometry; the components'
// cell layouts interleaved at grad[0].cells: cell r's record of dim x 2^dim
// values at r dim 2^dim, component c's corners at offset c 2^dim).
template <class T>
struct ItemDesc : ItemCore<T> {
    const uint32_t *node_rng;
    GridView<T> grad[3];
};

// One launch of the path kernel: slots [slot_begin, slot_begin + launch_slots)
// of the group's slot space, handed out through *counter.
// The batch kernel keeps one queue per item that the launch touches (items
// item_lo .. item_lo + n_seg - 1: counter[k] for item item_lo + k, whose
// launch-relative slots are [seg[2k], seg[2k+1])); the single-item kernel
// uses counter[0].
struct LaunchArgs {
    uint64_t slot_begin;
    uint32_t launch_slots;
    int32_t n_items;
    int32_t grab;
    int32_t item_lo;
    uint32_t n_seg;
    uint32_t refill_mask;  // lanes are refilled at walk-loop iterations i with (i & refill_mask) == 0
    uint32_t *counter;
    const uint32_t *seg;
};

// Compensated (Neumaier) per-node accumulators: phi, phi^2, e, e^2, phi*e.
struct NodeAcc {
    double s[5];
    double c[5];
    int64_t n, steps, capped, pad;
};

// Per-item entry of the post-processing kernels of a group (nodes are
// numbered across the group's items; node_item maps a node to its item).
struct FinalItem {
    pdd_node_stats *out;  // the item's statistics (device)
    uint64_t gnode;       // first group node of the item
    int32_t has_phi;      // phi is scored (plain solve or PDD_PLAIN_ALONGSIDE)
    int32_t accumulate;   // start from the statistics already in `out`
    int32_t own_reduce;   // caller records: reduced by a launch of its own
    int32_t up_f64;
    // u_prev for the node value u_prev(x0) + mean(e), read in its own dtype;
    // null (Ito items): the node value is mean(e), e = phi + xi
    const void *up_data;
    int32_t up_n[3];
    int32_t pad;
    double up_lo[3], up_inv[3];
};

// One workgroup per node from node_lo on; node i covers slots
// [node_start[i], node_start[i+1]) (or uniform_n each) clipped to
// [slot_begin, slot_end); records of slot q sit at q - rec_base. With
// node_item set, has_phi comes from the node's item and nodes whose item
// reduces on its own are skipped.
struct ReduceArgs {
    const double *rec_phi;
    const double *rec_e;
    const uint32_t *rec_steps;
    uint64_t rec_base;
    const uint64_t *node_start;
    uint64_t uniform_n;
    uint64_t slot_begin, slot_end;
    NodeAcc *acc;
    uint32_t node_lo;
    int32_t has_phi, has_e;
    const uint32_t *node_item;
    const FinalItem *fitems;
    // segments longer than kReduceChunk paths are split: chunk c of node
    // node_lo + b is reduced by workgroup (b, c) into partials[b * n_chunks +
    // c], and the chunks are then merged into acc in chunk order
    NodeAcc *partials;
    uint32_t n_chunks;
};

constexpr uint64_t kReduceChunk = 1ull << 16;

struct FinalizeArgs {
    const NodeAcc *acc;
    const double *nodes;  // group nodes, dim doubles each
    uint32_t n_nodes;     // group nodes
    int32_t dim;
    int32_t has_e;
    const uint32_t *node_item;
    const FinalItem *fitems;
};

// One item's statistics to copy into a contiguous buffer: n entries from src
// to dst + at (so that many items come back to the host in one copy).
struct GatherItem {
    const pdd_node_stats *src;
    uint64_t n;
    uint64_t at;
};

// Kernel arguments of a launch that holds a single item: the item and its
// problem travel by value (scalar loads from the argument segment).
template <class T>
struct OneItemArgs {
    LaunchArgs launch;
    ItemCore<T> item;
    DevProblem<T> prob;
};

// The by-value single-item kernel exists for the FP32 2D plain solve only: it
// fits seven waves per SIMD there without spilling, while with FP64 or the
// correction terms the larger argument block spills and the table kernel is
// as fast. Both kernels give bitwise identical results.
template <class T, int D, int EST>
constexpr bool kOneItemKernel = sizeof(T) == 4 && D == 2 && EST == kEstPlain;

// Kernel kinds: generic (domain, exit test, law and tabulation read at run
// time), or specialised for box problems with the bridge exit test and
// Gaussian increments, in the bridge form for walks with few lanes near a
// face (sparse) or with many (dense). All kinds give the same bits.
constexpr int kKernelGeneric = 0, kKernelSparse = 1, kKernelDense = 2;

// Launchers (defined in the .hip files). EST: kEstPlain, kEstCorrection or
// kEstIto; kind: one of the kernel kinds.
template <class T, int D, int EST>
hipError_t launch_path_kernel(const LaunchArgs &l, const ItemDesc<T> *items,
                              const DevProblem<T> *probs, int grid, int block, int kind, hipStream_t s);
template <class T, int D, int EST>
hipError_t launch_path_kernel_one(const OneItemArgs<T> &a, int grid, int block, int kind, hipStream_t s);
template <class T, int D, int EST>
const void *path_kernel_symbol(bool one, int kind);
// Fills `cells` (cell_values entries) from the point values of a grid,
// converted from S to T.
template <class S, class T, int D>
hipError_t launch_grid_cells(const S *data, const int32_t *n, T *cells, hipStream_t s);
// The same into records of `stride` values per cell, at offset `off` in each.
// out[p stride + off] = data[p] converted from S to T, p < n_points.
template <class S, class T>
hipError_t launch_grid_points_strided(const S *data, uint64_t n_points, T *out, uint32_t stride, uint32_t off,
                                      hipStream_t s);
template <class S, class T, int D>
hipError_t launch_grid_cells_strided(const S *data, const int32_t *n, T *cells, uint32_t stride, uint32_t off,
                                     hipStream_t s);
hipError_t launch_reduce(const ReduceArgs &a, uint32_t n_blocks, hipStream_t s);
// r = f - ((1/2) sigma^2 Lap u + b.grad u + c u) at the points of grid g (u in
// g->data, r in g's dtype and layout), by second-order differences.
hipError_t launch_grid_residual(const DevProblem<double> &P, double sigma, const pdd_grid *g, void *r, hipStream_t s);
// Second stage of PDD on a 2D box cut by axis-parallel interfaces (the
// subdomain-BVP step of Alg. A:IterPDD). u~ lives on a grid of n0 x n1 points
// over the box (x fastest).
struct Stage2Grid {
    double *u;
    int32_t n0, n1;
    double lo0, lo1, span0, span1;  // point i of axis d at lo_d + span_d i / (n_d - 1)
    double dx0, dx1;                 // span_d / (n_d - 1)
    double half_s2;                  // (1/2) sigma^2
};
// One subdomain: the grid box [i0, i1] x [j0, j1] (boundary indices
// included); its interior unknowns in the order r = s w + f, f running along
// the box's shorter interior side (fast_x: along x), s along the other;
// `first`: its first unknown in the stencil / factor tables.
struct SubBox {
    int32_t i0, i1, j0, j1;
    int32_t w, L, fast_x, pad;
    uint64_t first;
};
constexpr int kStage2MaxBand = 64;  // shorter interior side of a subdomain, at most
// One interface line for the interpolation: axis d (the line is x_d = const at
// grid index k), m data points at coordinates t[0..m-1] along the other axis
// with multiquadric weights lam[0..m-1] (at offset `at` in the tables).
struct Stage2Line {
    int32_t d, k, m, pad;
    uint64_t at;
    double eps;
};
// Physical-boundary values g of the grid (every point of the box's edges).
hipError_t launch_stage2_boundary(const DevProblem<double> &P, const Stage2Grid &g, hipStream_t s);
// Interface lines: the multiquadric interpolants at the grid points of each
// line between the box's edges; a point where an axis-0 and an axis-1 line
// cross takes the mean of the two.
hipError_t launch_stage2_lines(const Stage2Grid &g, const Stage2Line *lines, int32_t n_lines, const double *t,
                               const double *lam, hipStream_t s);
// Response of a subdomain's interior to its boundary values: the rows next
// to the box's boundary (nb of them, at rb[rb_at ..]) and, at out_at in the
// response buffer, nb + 1 columns of n values (column q < nb: the solution
// for a unit right side at row rb[rb_at + q]; column nb: the solution for the
// source f with zero boundary values).
struct Stage2Resp {
    uint64_t rb_at, out_at;
    int32_t nb, pad;
};
constexpr int kStage2MaxBoundaryRows = 4096;
// What launch_stage2_solve is to do after the stencils: factor (unless
// `factored`), then either substitute the right side (resp == nullptr) or,
// with the response columns (computed first unless `resp_ready`), add up
// f's column and the boundary values' columns.
struct Stage2Plan {
    bool factored;
    const Stage2Resp *resp_tab;  // device, one per subdomain, or null
    const uint32_t *rb;          // device rows next to the boundary
    double *resp;                // device response columns
    int32_t max_cols;            // largest nb + 1
    bool resp_ready;
};
// Finite-difference stencils of every subdomain's unknowns (6 doubles per
// unknown: slow-1, fast-1, centre, fast+1, slow+1 coefficients and the right
// side with the boundary values moved over; in aux, 2 doubles per unknown:
// the source f alone and the boundary values' part of the right side), then
// (unless plan.factored: factor and lmul already hold the factors of these
// subdomains' matrices) the banded LU factorization of each subdomain, and
// the interior values written into u: by forward elimination and back
// substitution of the right side (one workgroup each), or from the response
// columns. factor: unknowns x (kStage2MaxBand + 2) doubles; lmul: unknowns x
// kStage2MaxBand doubles.
hipError_t launch_stage2_solve(const DevProblem<double> &P, const Stage2Grid &g, const SubBox *boxes,
                               int32_t n_boxes, uint32_t max_unknowns, double *stencil, double *aux, double *factor,
                               double *lmul, const Stage2Plan &plan, hipStream_t s);
hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t s);
hipError_t launch_zero(void *ptr, uint64_t bytes, hipStream_t s);
// Starting sums of every group node: zero, or the statistics already in the
// item's output for an accumulating solve.
hipError_t launch_init_acc(NodeAcc *acc, uint32_t n, const uint32_t *node_item, const FinalItem *fitems,
                           hipStream_t s);
// Copies the statistics of n_items items (table in device memory) into dst.
hipError_t launch_gather_stats(const GatherItem *table, uint32_t n_items, pdd_node_stats *dst, hipStream_t s);

}  // namespace pdd
