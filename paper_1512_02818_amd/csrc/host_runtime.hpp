// Host-side internals shared by the solver runtime and the serving loop
// (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "pdd.h"
#include "pdd_internal.hpp"

namespace pdd {

// Records a thread-local message for pdd_last_error() and returns `code`.
pdd_status fail(pdd_status code, const char *fmt, ...);
extern thread_local std::string g_error;

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::pdd::fail(PDD_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

constexpr double kGmShift = 0.5826;                    // Alg. 1 boundary shift
constexpr double kBridgeSkip = 24.953298500158186;     // 36 ln 2: p < 2^-36 skipped
constexpr uint64_t kDefaultMaxSteps = 1ull << 26;
constexpr uint64_t kScratchSlots = 1ull << 27;         // record slots per launch
constexpr uint64_t kMaxLaunchSlots = 1ull << 31;
constexpr double kHwTrigRevolutions = 256.0;           // input range of the FP32 hardware sine / cosine

struct DeviceBuffer {
    void *ptr = nullptr;
    size_t cap = 0;
};

// One solve (or batch item) after validation.
struct HostItem {
    pdd_problem *prob = nullptr;
    const pdd_grid *u_prev = nullptr, *resid = nullptr;
    const pdd_grid *grad = nullptr;  // dim gradient grids (Ito control variate)
    const double *nodes = nullptr;
    int64_t n_nodes = 0;
    const pdd_solve_opts *o = nullptr;
    pdd_node_stats *out = nullptr;
    int est = kEstPlain;  // kEstPlain, kEstCorrection or kEstIto
    bool score_plain = true, uniform = true, caller_records = false, accumulate = false;
    uint64_t total = 0, max_steps = 0;
    std::vector<uint64_t> starts;  // item-relative prefix (non-uniform counts)
};

// Checks an item's arguments against its problem (nothing is enqueued).
pdd_status validate_item(HostItem &it);
// Key of the launch-shape table: precision, dimension, estimator (kEst*) and
// kernel (specialised box / bridge / Gaussian / analytic, or generic).
inline int tuning_key(int precision, int dim, int est, bool generic)
{
    return precision * 12 + (dim - 2) * 6 + est * 2 + (generic ? 1 : 0);
}
// Whether an item can run in the specialised kernel.
bool specialised(const HostItem &it);
// The launch's refill mask: walk-loop iterations between lane refills, less
// one (the tuning's, else every second iteration in 2D, every fourth in 3D).
template <int D>
inline uint32_t refill_mask(const pdd_tuning &t)
{
    return (uint32_t)((t.refill ? t.refill : (D == 2 ? 2 : 4)) - 1);
}
// Whether many lanes of a wave are near a face at every step of a walk of
// this problem at step dt (then the dense form of the bridge test is the
// faster one).
bool dense_boundary(const pdd_problem_desc &d, double dt);

// Launch shape for a solve: opts->tuning (fields left 0 take the default),
// else the context's table entry for `key` (tuning_key; < 0: none), else
// {256, occupancy, 64, 0}; checked.
pdd_status read_tuning(const pdd_ctx *ctx, const pdd_solve_opts *o, int key, pdd_tuning &tune);
// Resident workgroups per CU of kernel `fn` at `block` threads, from the
// context's table (filled at pdd_init for the plain kernels; `cache`: add a
// missing entry, which allocates host memory).
int occupancy(pdd_ctx *ctx, const void *fn, int block, bool cache = true);
// The allocation-free solve's device scratch on `device` (made current by the
// caller): looked up once per device; PDD_E_HIP if the lookup fails.
pdd_status noalloc_attach(int device);

// Validates items, then enqueues them on `s`, grouped by (precision,
// dimension, estimator); a group of at most kScratchSlots paths without
// caller records is one launch. one_launch: such a group stays one launch
// whatever the tuning's max_launch_paths says (the serving loop, whose
// results must not depend on the tuning table). The items' problems must
// belong to `owner` (NULL: ctx itself), a context on ctx's device whose
// problems ctx's scratch then serves.
pdd_status run_items(pdd_ctx *ctx, std::vector<HostItem> &items, hipStream_t s, bool one_launch = false,
                     const pdd_ctx *owner = nullptr);

}  // namespace pdd

struct pdd_ctx {
    int device = 0;
    int n_cu = 0;
    hipEvent_t done = nullptr;    // end of the last solve
    hipEvent_t staged = nullptr;  // last copy out of the staging buffer
    bool any_done = false, any_staged = false;
    pdd::DeviceBuffer nodes, starts, acc, counters, rec, partials, gather, cells;
    pdd::DeviceBuffer stage2;  // second stage: tables and stencils
    // LU factors of the last second stage's subdomain matrices, and what they
    // factor (the operator, the grid, the interfaces): a call with the same
    // ones only eliminates its right sides
    pdd::DeviceBuffer stage2_lu;
    std::vector<double> stage2_key;
    // the subdomains' response columns to their boundary values (and to f),
    // kept with their key: the factors' key and the problem's serial number
    pdd::DeviceBuffer stage2_resp;
    std::vector<double> stage2_resp_key;
    void *stage = nullptr;
    size_t stage_cap = 0;
    void *readback = nullptr;  // pinned host copy of pilot statistics
    size_t readback_cap = 0;
    std::map<std::tuple<const void *, int>, int> occupancy;
    // timing of path-kernel launches (PDD_TIME_KERNEL)
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timed, spare;
    // launch shapes by (precision, dim, estimator), from pdd_autotune / pdd_set_tuning
    std::map<int, pdd_tuning> tuned;
};

struct pdd_problem {
    pdd_ctx *ctx = nullptr;
    pdd_problem_desc desc{};
    // largest |k_d x_d + phase_d| of a trig term over the domain's bounding
    // box, in revolutions: FP32 paths evaluate sines with the hardware
    // instruction, whose argument must stay within +-256 revolutions
    double trig_rev_max = 0.0;
    pdd::DevProblem<float> pf{};
    pdd::DevProblem<double> pd{};
    pdd::DeviceBuffer tab;  // cell layouts of tabulated coefficients (FP32, then FP64)
    uint64_t serial = 0;    // unique per problem created in the process
};
