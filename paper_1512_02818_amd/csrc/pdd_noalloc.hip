// The plain nodal solve of pdd_solve_nodes without any allocation, for
// callers that cannot allocate (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// Everything the solve needs besides the caller's inputs and outputs lives in
// `scratch`, a file-scope device array of PDD_NOALLOC_SCRATCH_BYTES that each
// GPU holds from the library's load until the process ends. Host code never
// uses the array's name as an address: pdd_init looks its device address up
// once per device (hipGetSymbolAddress, with that device current) and the
// solve passes that address to the kernels. Host inputs (the node table, the
// work item and the problem) reach the device as kernel arguments of a small
// store kernel, so there is no staging buffer and no host-to-device copy.
// Calls on one GPU share its array: two of them in flight at once (on
// different streams, or from different contexts) race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "pdd.h"
#include "host_runtime.hpp"

namespace pdd {
namespace {

static __device__ __align__(256) unsigned char scratch[PDD_NOALLOC_SCRATCH_BYTES];

// Layout of the scratch (byte offsets). Records: FP64 score of every slot of
// a launch, then its exit-step word.
constexpr size_t kNaRecSlots = size_t(1) << 21;
constexpr size_t kNaMaxNodes = PDD_NOALLOC_MAX_NODES;
constexpr size_t kNaOffPhi = 0;
constexpr size_t kNaOffSteps = kNaOffPhi + kNaRecSlots * sizeof(double);
constexpr size_t kNaOffAcc = kNaOffSteps + kNaRecSlots * sizeof(uint32_t);
constexpr size_t kNaOffNodes = kNaOffAcc + kNaMaxNodes * sizeof(NodeAcc);
constexpr size_t kNaOffNitem = kNaOffNodes + kNaMaxNodes * 3 * sizeof(double);
constexpr size_t kNaOffPart = kNaOffNitem + kNaMaxNodes * sizeof(uint32_t);
constexpr size_t kNaPartBytes = size_t(256) << 10;
constexpr size_t kNaOffItem = kNaOffPart + kNaPartBytes;
constexpr size_t kNaOffProb = kNaOffItem + 1024;
constexpr size_t kNaOffFinal = kNaOffProb + 8192;
constexpr size_t kNaOffSeg = kNaOffFinal + 256;
constexpr size_t kNaOffCounter = kNaOffSeg + 256;
constexpr size_t kNaEnd = kNaOffCounter + 256;
static_assert(kNaEnd <= PDD_NOALLOC_SCRATCH_BYTES, "scratch layout exceeds the array");
static_assert(sizeof(ItemDesc<double>) <= 1024 && sizeof(ItemDesc<float>) <= 1024, "item slot");
static_assert(sizeof(DevProblem<double>) <= 8192 && sizeof(FinalItem) <= 256, "problem / final slots");
static_assert(kNaOffAcc % 256 == 0 && kNaOffNodes % 256 == 0 && kNaOffPart % 256 == 0, "alignment");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];        // device address of `scratch` per device (null: not looked up)
hipError_t g_lookup[kMaxDevices];    // result of the lookup, when it failed

// Up to 3,968 bytes that travel as a kernel argument.
struct Blob {
    uint32_t w[992];
};

__global__ void store_kernel(const Blob b, uint32_t n_words, uint32_t *__restrict__ dst)
{
    for (uint32_t i = threadIdx.x; i < n_words; i += blockDim.x) dst[i] = b.w[i];
}

// Copies `bytes` (a multiple of 4) of host memory to device memory through
// kernel arguments, in pieces of one Blob.
pdd_status store(const void *src, size_t bytes, void *dst, hipStream_t s)
{
    const unsigned char *p = static_cast<const unsigned char *>(src);
    unsigned char *q = static_cast<unsigned char *>(dst);
    Blob b;
    for (size_t at = 0; at < bytes; at += sizeof(Blob)) {
        const size_t len = std::min(sizeof(Blob), bytes - at);
        std::memcpy(b.w, p + at, len);
        hipLaunchKernelGGL(store_kernel, dim3(1), dim3(256), 0, s, b, (uint32_t)(len / 4),
                           reinterpret_cast<uint32_t *>(q + at));
        HIP_TRY(hipGetLastError());
    }
    return PDD_OK;
}

template <class T, int D>
pdd_status run_noalloc(pdd_ctx *ctx, const HostItem &it, const pdd_tuning &tune, unsigned char *base,
                       hipStream_t s)
{
    const pdd_solve_opts *o = it.o;
    const uint64_t total = it.total, N = o->n_paths;
    const uint32_t n = (uint32_t)it.n_nodes;
    uint64_t per_launch = std::min<uint64_t>(kNaRecSlots, std::max<uint64_t>(total, 1));
    if (tune.max_launch_paths > 0) per_launch = std::min<uint64_t>(per_launch, (uint64_t)tune.max_launch_paths);
    // chunk partials of one launch: at most (nodes it touches) x (chunks of
    // the longest piece of a node), known before anything is enqueued
    if (N > kReduceChunk) {
        const uint64_t nodes_max = (per_launch - 1) / N + 2;
        const uint64_t chunks_max = (std::min<uint64_t>(N, per_launch) + kReduceChunk - 1) / kReduceChunk;
        if (nodes_max * chunks_max * sizeof(NodeAcc) > kNaPartBytes)
            return fail(PDD_E_INTERNAL, "no-alloc scratch: chunk partials do not fit");
    }
    double *sc_phi = reinterpret_cast<double *>(base + kNaOffPhi);
    uint32_t *sc_steps = reinterpret_cast<uint32_t *>(base + kNaOffSteps);
    NodeAcc *acc = reinterpret_cast<NodeAcc *>(base + kNaOffAcc);
    double *d_nodes = reinterpret_cast<double *>(base + kNaOffNodes);
    uint32_t *nitem = reinterpret_cast<uint32_t *>(base + kNaOffNitem);
    NodeAcc *partials = reinterpret_cast<NodeAcc *>(base + kNaOffPart);
    ItemDesc<T> *d_item = reinterpret_cast<ItemDesc<T> *>(base + kNaOffItem);
    DevProblem<T> *d_prob = reinterpret_cast<DevProblem<T> *>(base + kNaOffProb);
    FinalItem *d_final = reinterpret_cast<FinalItem *>(base + kNaOffFinal);
    uint32_t *d_seg = reinterpret_cast<uint32_t *>(base + kNaOffSeg);
    uint32_t *counter = reinterpret_cast<uint32_t *>(base + kNaOffCounter);

    const pdd_problem_desc &d = it.prob->desc;
    ItemDesc<T> a;
    std::memset(&a, 0, sizeof a);
    a.prob = 0;
    a.exit_mode = o->exit_mode;
    a.law = o->law;
    a.score_plain = 1;
    a.stream_tag = o->stream_id << 4;
    a.max_steps = (uint32_t)it.max_steps;
    a.n_nodes = n;
    a.slot_begin = 0;
    a.n_slots = total;
    a.uniform_n = N;
    a.path_offset = o->path_offset;
    a.nodes = d_nodes;
    if (it.caller_records) {
        a.rec_phi = o->rec_phi;
        a.rec_steps = o->rec_steps;
        a.rec_base = 0;
    } else {
        a.rec_phi = sc_phi;
        a.rec_steps = sc_steps;
        a.rec_launch = 1;
    }
    const double sig_sqh = d.sigma * std::sqrt(o->dt);
    a.h = (T)o->dt;
    a.sig_sqh = (T)sig_sqh;
    a.two_over_s2h = (T)(2.0 / (d.sigma * d.sigma * o->dt));
    a.gm_thresh = (T)(kGmShift * sig_sqh);
    a.bridge_thresh = (T)kBridgeSkip;
    a.dense_bridge = dense_boundary(d, o->dt) ? 1 : 0;
    FinalItem fi;
    std::memset(&fi, 0, sizeof fi);
    fi.out = it.out;
    fi.gnode = 0;
    fi.has_phi = 1;
    fi.accumulate = it.accumulate ? 1 : 0;
    const DevProblem<T> &P = *reinterpret_cast<const DevProblem<T> *>(
        sizeof(T) == 4 ? static_cast<const void *>(&it.prob->pf) : static_cast<const void *>(&it.prob->pd));
    const uint64_t last_len = total ? total - (total - 1) / per_launch * per_launch : 0;
    const uint32_t seg[4] = {0u, (uint32_t)per_launch, 0u, (uint32_t)last_len};

    pdd_status st;
    if ((st = store(it.nodes, (size_t)n * D * sizeof(double), d_nodes, s))) return st;
    if ((st = store(&a, sizeof a, d_item, s))) return st;
    if ((st = store(&P, sizeof P, d_prob, s))) return st;
    if ((st = store(&fi, sizeof fi, d_final, s))) return st;
    if ((st = store(seg, sizeof seg, d_seg, s))) return st;
    HIP_TRY(launch_zero(nitem, ((size_t)n * sizeof(uint32_t) + 7) & ~size_t(7), s));
    HIP_TRY(launch_init_acc(acc, n, nitem, d_final, s));

    const bool one = kOneItemKernel<T, D, kEstPlain>;
    const int kind = !specialised(it)   ? kKernelGeneric
                     : tune.bridge == 1 ? kKernelSparse
                     : tune.bridge == 2 ? kKernelDense
                     : a.dense_bridge   ? kKernelDense
                                        : kKernelSparse;
    const void *fn = path_kernel_symbol<T, D, kEstPlain>(one, kind);
    const int occ = occupancy(ctx, fn, tune.block, false);
    const int bpc = tune.blocks_per_cu > 0 ? std::min(tune.blocks_per_cu, occ) : occ;
    for (uint64_t b = 0; b < total; b += per_launch) {
        const uint64_t len = std::min(per_launch, total - b);
        HIP_TRY(launch_zero(counter, 8, s));
        LaunchArgs L{};
        L.slot_begin = b;
        L.launch_slots = (uint32_t)len;
        L.n_items = 1;
        L.grab = tune.grab;
        L.counter = counter;
        L.item_lo = 0;
        L.n_seg = 1;
        L.refill_mask = refill_mask<D>(tune);
        L.seg = d_seg + (len == per_launch ? 0 : 2);
        const uint64_t blocks_needed = ((len + 63) / 64 * 64 + tune.block - 1) / tune.block;
        const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)ctx->n_cu * bpc, blocks_needed));
        if (one) {
            OneItemArgs<T> A;
            A.launch = L;
            A.item = a;
            A.prob = P;
            if (A.item.rec_launch) A.item.rec_base = b;
            HIP_TRY((launch_path_kernel_one<T, D, kEstPlain>(A, grid, tune.block, kind, s)));
        } else {
            HIP_TRY((launch_path_kernel<T, D, kEstPlain>(L, d_item, d_prob, grid, tune.block, kind, s)));
        }
        // per-node sums of the nodes this launch touched
        // (node i holds slots [i N, (i + 1) N); the longest piece of a node in
        // [b, b + len) sets the chunk count of the reduction)
        const uint64_t e = b + len;
        const uint32_t n_lo = (uint32_t)(b / N), n_hi = (uint32_t)((e - 1) / N);
        uint64_t longest = len;
        if (n_hi > n_lo) {
            longest = std::max((uint64_t)(n_lo + 1) * N - b, e - (uint64_t)n_hi * N);
            if (n_hi > n_lo + 1) longest = std::max(longest, N);
        }
        ReduceArgs r{};
        r.rec_phi = it.caller_records ? o->rec_phi : sc_phi;
        r.rec_steps = it.caller_records ? o->rec_steps : sc_steps;
        r.rec_base = it.caller_records ? 0 : b;
        r.node_start = nullptr;
        r.uniform_n = N;
        r.slot_begin = b;
        r.slot_end = b + len;
        r.acc = acc;
        r.node_lo = n_lo;
        r.has_phi = 1;
        r.has_e = 0;
        r.n_chunks = (uint32_t)std::max<uint64_t>(1, (longest + kReduceChunk - 1) / kReduceChunk);
        r.partials = partials;
        HIP_TRY(launch_reduce(r, n_hi - n_lo + 1, s));
    }
    FinalizeArgs f{};
    f.acc = acc;
    f.nodes = d_nodes;
    f.n_nodes = n;
    f.dim = D;
    f.has_e = 0;
    f.node_item = nitem;
    f.fitems = d_final;
    HIP_TRY(launch_finalize(f, s));
    return PDD_OK;
}

}  // namespace

pdd_status noalloc_attach(int device)
{
    if (device < 0 || device >= kMaxDevices) return fail(PDD_E_UNSUPPORTED, "device index %d out of range", device);
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch[device]) return PDD_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        g_lookup[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
        return fail(PDD_E_HIP, "hipGetSymbolAddress of the no-alloc scratch failed: %s",
                    hipGetErrorString(g_lookup[device]));
    }
    g_scratch[device] = ptr;
    return PDD_OK;
}

}  // namespace pdd

using namespace pdd;

extern "C" pdd_status pdd_solve_nodes_noalloc(pdd_problem *problem, const double *nodes, int64_t n_nodes,
                                              const pdd_solve_opts *opts, pdd_node_stats *out, void *stream)
{
    if (!problem) return fail(PDD_E_INVALID, "problem is NULL");
    if (!opts) return fail(PDD_E_INVALID, "opts is NULL");
    if (opts->n_paths_per_node)
        return fail(PDD_E_UNSUPPORTED, "the no-alloc solve takes one path count for all nodes (n_paths_per_node NULL)");
    if (opts->flags & PDD_TIME_KERNEL) return fail(PDD_E_UNSUPPORTED, "PDD_TIME_KERNEL needs events: not in the no-alloc solve");
    if (n_nodes > (int64_t)kNaMaxNodes)
        return fail(PDD_E_UNSUPPORTED, "the no-alloc solve takes at most %d nodes (got %lld)", PDD_NOALLOC_MAX_NODES,
                    (long long)n_nodes);
    HostItem it;
    it.prob = problem;
    it.nodes = nodes;
    it.n_nodes = n_nodes;
    it.o = opts;
    it.out = out;
    pdd_status st = validate_item(it);
    if (st) return st;
    if (n_nodes == 0) return PDD_OK;
    pdd_ctx *ctx = problem->ctx;
    const int dim = problem->desc.dim;
    pdd_tuning tune;
    if ((st = read_tuning(ctx, opts, tuning_key(opts->precision, dim, kEstPlain, !specialised(it)), tune))) return st;
    void *base = nullptr;
    hipError_t looked = hipSuccess;
    if (ctx->device >= 0 && ctx->device < kMaxDevices) {
        std::lock_guard<std::mutex> lock(g_mu);
        base = g_scratch[ctx->device];
        looked = g_lookup[ctx->device];
    }
    if (!base)
        return fail(PDD_E_HIP, "the no-alloc scratch of device %d has no address (lookup at pdd_init: %s)",
                    ctx->device, hipGetErrorString(looked));
    HIP_TRY(hipSetDevice(ctx->device));
    const hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned char *b = static_cast<unsigned char *>(base);
    if (opts->precision == PDD_FP32)
        return dim == 2 ? run_noalloc<float, 2>(ctx, it, tune, b, s) : run_noalloc<float, 3>(ctx, it, tune, b, s);
    return dim == 2 ? run_noalloc<double, 2>(ctx, it, tune, b, s) : run_noalloc<double, 3>(ctx, it, tune, b, s);
}
