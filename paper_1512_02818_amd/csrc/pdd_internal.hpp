// Internal structures shared by the host runtime and the HIP kernels of the
// first-stage PDD nodal solver. Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdd {

constexpr int kMaxTrig = 16;
constexpr int kMaxMono = 8;
constexpr int kExitBridge = 0, kExitShift = 1, kExitNaive = 2;
constexpr int kLawGauss = 0, kLawRademacher = 1;
constexpr int kBox = 0, kBall = 1;
constexpr uint32_t kCappedBit = 0x80000000u;

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
};

// A grid as the kernels read it: value(x) = bilinear / trilinear interpolation.
// The values have the type of the path arithmetic.
template <class T>
struct GridView {
    const T *data;
    int32_t n[3];
    int32_t pad;
    T lo[3];
    T inv[3];  // (n - 1) / (hi - lo)
};

// Arguments of one launch of the path kernel: the slots [slot_begin,
// slot_begin + launch_slots) of the solve's path space. Slot s belongs to the
// node i with node_start[i] <= s < node_start[i + 1] (or i = s / uniform_n).
template <class T>
struct PathArgs {
    DevProblem<T> prob;         // by value: kernel arguments are read with scalar loads
    const double *nodes;        // n_nodes x dim
    const uint64_t *node_start; // n_nodes + 1 prefix, or null (uniform)
    uint64_t uniform_n;
    uint64_t total_slots;
    uint64_t slot_begin;
    uint64_t path_offset;
    uint64_t rec_base;          // records are indexed by slot - rec_base
    double *rec_phi;
    double *rec_e;
    uint32_t *rec_steps;
    uint32_t *counter;          // queue head of this launch
    uint32_t n_nodes;
    uint32_t launch_slots;
    uint32_t stream_tag;        // stream_id << 4
    uint32_t max_steps;
    int32_t exit_mode, law;
    int32_t grab;
    int32_t score_plain;        // 1: evaluate f and score phi
    T h, sig_sqh, two_over_s2h, gm_thresh, bridge_thresh;
    GridView<T> u_prev, resid;
};

// Compensated (Neumaier) per-node accumulators: phi, phi^2, e, e^2, phi*e.
struct NodeAcc {
    double s[5];
    double c[5];
    int64_t n, steps, capped, pad;
};

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
};

struct FinalizeArgs {
    const NodeAcc *acc;
    const double *nodes;
    void *out;  // pdd_node_stats
    uint32_t n_nodes;
    int32_t dim;
    int32_t has_phi, has_e;
    // u_prev for the node value u_prev(x0) + mean(e), read in its own dtype
    const void *up_data;
    int32_t up_f64;
    int32_t up_n[3];
    double up_lo[3], up_inv[3];
};

// Launchers (defined in the .hip files).
template <class T, int D, bool CV>
hipError_t launch_path_kernel(const PathArgs<T> &a, int grid, int block, hipStream_t s);
template <class T, int D, bool CV>
const void *path_kernel_symbol();
hipError_t launch_reduce(const ReduceArgs &a, uint32_t n_blocks, hipStream_t s);
hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t s);
hipError_t launch_zero(void *ptr, uint64_t bytes, hipStream_t s);

}  // namespace pdd
