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

// One trig term amp * prod_d sin(k_d x_d + ph_d). krev / phrev are k / 2pi and
// ph / 2pi (the hardware sine takes revolutions); ksq = |k|^2.
template <class T>
struct DevTrig {
    T amp, ksq;
    T k[3], ph[3];
    T krev[3], phrev[3];
};

template <class T>
struct DevMono {
    T coef;
    int32_t e[3];
};

// Problem in the precision of the path arithmetic. Read by every lane with the
// same address, so the compiler serves it from the scalar cache.
template <class T>
struct DevProblem {
    int32_t dim, domain;
    int32_t n_trig, n_mono, n_fx, n_gx;
    uint32_t key0, key1;
    T lo[3], hi[3], center[3];
    T radius, radius2;
    T half_s2;  // sigma^2 / 2
    T b0[3];
    T B[3][3];
    T c_a, c_b;
    DevTrig<T> trig[kMaxTrig];
    DevMono<T> mono[kMaxMono];
    DevMono<T> fx[kMaxMono];
    DevMono<T> gx[kMaxMono];
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
