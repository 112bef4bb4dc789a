// Per-node reductions of the per-path records and the node statistics
// (Sec. 2.2, eq. F:Statistical_error; Sec. 2.3, eqs. F:Variance_Reduction and
// F:Rho).
//
// One workgroup per node segment of a launch. Each thread keeps Neumaier
// (sum, compensation) pairs over a fixed stride of the segment; the pairs are
// merged by a butterfly of wave shuffles and then across the waves through
// LDS, always in the same order, and added to the node's accumulator, which
// only this workgroup touches during the launch. The result is therefore the
// same whichever lanes walked which paths.
#include "pdd.h"
#include "pdd_internal.hpp"

namespace pdd {
namespace {

struct Pair {
    double s, c;
};

__device__ __forceinline__ void nadd(Pair &a, double x)
{
    const double t = a.s + x;
    if (fabs(a.s) >= fabs(x))
        a.c += (a.s - t) + x;
    else
        a.c += (x - t) + a.s;
    a.s = t;
}

// Exact-enough merge of two compensated sums; symmetric in its arguments.
__device__ __forceinline__ Pair nmerge(Pair a, Pair b)
{
    const double t = a.s + b.s;
    const double err = fabs(a.s) >= fabs(b.s) ? (a.s - t) + b.s : (b.s - t) + a.s;
    return {t, (a.c + b.c) + err};
}

constexpr int kReduceBlock = 256;

// Node segment [lo, hi) of the launch and its number of chunks.
__device__ __forceinline__ void segment(const ReduceArgs &r, uint32_t node, uint64_t &lo, uint64_t &hi)
{
    uint64_t ns, ne;
    if (r.node_start) {
        ns = r.node_start[node];
        ne = r.node_start[node + 1];
    } else {
        ns = (uint64_t)node * r.uniform_n;
        ne = ns + r.uniform_n;
    }
    lo = ns > r.slot_begin ? ns : r.slot_begin;
    hi = ne < r.slot_end ? ne : r.slot_end;
}

__device__ __forceinline__ uint32_t n_chunks_of(uint64_t lo, uint64_t hi)
{
    return hi > lo ? (uint32_t)((hi - lo + kReduceChunk - 1) / kReduceChunk) : 0u;
}

__global__ void __launch_bounds__(kReduceBlock) reduce_kernel(const ReduceArgs r)
{
    const uint32_t node = r.node_lo + blockIdx.x;
    const uint32_t chunk = blockIdx.y;
    int32_t has_phi = r.has_phi;
    if (r.node_item) {
        const FinalItem &fi = r.fitems[r.node_item[node]];
        if (fi.own_reduce) return;  // whole workgroup: the item is uniform per node
        has_phi = fi.has_phi;
    }
    uint64_t lo, hi;
    segment(r, node, lo, hi);
    const uint32_t nch = n_chunks_of(lo, hi);
    // one chunk (or none): this workgroup merges straight into the node's sums
    const bool direct = nch <= 1;
    if (direct ? chunk != 0 : chunk >= nch) return;  // whole workgroup
    if (!direct) {
        lo += (uint64_t)chunk * kReduceChunk;
        if (hi - lo > kReduceChunk) hi = lo + kReduceChunk;
    }

    Pair acc[5] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
    long long steps = 0, capped = 0;
    for (uint64_t q = lo + threadIdx.x; q < hi; q += kReduceBlock) {
        const uint64_t i = q - r.rec_base;
        const uint32_t sw = r.rec_steps[i];
        steps += sw & ~kCappedBit;
        capped += sw >> 31;
        double phi = 0.0, e = 0.0;
        if (has_phi) {
            phi = r.rec_phi[i];
            nadd(acc[0], phi);
            nadd(acc[1], phi * phi);
        }
        if (r.has_e) {
            e = r.rec_e[i];
            nadd(acc[2], e);
            nadd(acc[3], e * e);
            if (has_phi) nadd(acc[4], phi * e);
        }
    }
    // butterfly across the 64 lanes of the wave
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            Pair o{__shfl_xor(acc[q].s, off), __shfl_xor(acc[q].c, off)};
            acc[q] = nmerge(acc[q], o);
        }
        steps += __shfl_xor(steps, off);
        capped += __shfl_xor(capped, off);
    }
    __shared__ Pair part[kReduceBlock / 64][5];
    __shared__ long long part_i[kReduceBlock / 64][2];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int q = 0; q < 5; ++q) part[wave][q] = acc[q];
        part_i[wave][0] = steps;
        part_i[wave][1] = capped;
    }
    __syncthreads();
    if (threadIdx.x == 0 && !direct) {  // a chunk partial, merged by merge_chunks_kernel
        NodeAcc p;
        Pair tot[5] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
        for (int w = 0; w < kReduceBlock / 64; ++w)
#pragma unroll
            for (int q = 0; q < 5; ++q) tot[q] = nmerge(tot[q], part[w][q]);
        long long st = 0, cp = 0;
        for (int w = 0; w < kReduceBlock / 64; ++w) {
            st += part_i[w][0];
            cp += part_i[w][1];
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            p.s[q] = tot[q].s;
            p.c[q] = tot[q].c;
        }
        p.steps = st;
        p.capped = cp;
        p.n = (long long)(hi - lo);
        p.pad = 0;
        r.partials[(size_t)blockIdx.x * r.n_chunks + chunk] = p;
    }
    if (threadIdx.x == 0 && direct) {
        NodeAcc &A = r.acc[node];
        Pair tot[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) tot[q] = {A.s[q], A.c[q]};
        for (int w = 0; w < kReduceBlock / 64; ++w)
#pragma unroll
            for (int q = 0; q < 5; ++q) tot[q] = nmerge(tot[q], part[w][q]);
        long long st = A.steps, cp = A.capped;
        for (int w = 0; w < kReduceBlock / 64; ++w) {
            st += part_i[w][0];
            cp += part_i[w][1];
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            A.s[q] = tot[q].s;
            A.c[q] = tot[q].c;
        }
        A.steps = st;
        A.capped = cp;
        A.n += (long long)(hi > lo ? hi - lo : 0);
    }
}

// Chunk partials of the split segments, merged into the node sums in chunk
// order (one thread per node of the launch range).
__global__ void merge_chunks_kernel(const ReduceArgs r, uint32_t n_nodes)
{
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_nodes) return;
    const uint32_t node = r.node_lo + b;
    if (r.node_item && r.fitems[r.node_item[node]].own_reduce) return;
    uint64_t lo, hi;
    segment(r, node, lo, hi);
    const uint32_t nch = n_chunks_of(lo, hi);
    if (nch <= 1) return;
    NodeAcc &A = r.acc[node];
    Pair tot[5];
    for (int q = 0; q < 5; ++q) tot[q] = {A.s[q], A.c[q]};
    long long st = A.steps, cp = A.capped, n = A.n;
    for (uint32_t c = 0; c < nch; ++c) {
        const NodeAcc &p = r.partials[(size_t)b * r.n_chunks + c];
        for (int q = 0; q < 5; ++q) tot[q] = nmerge(tot[q], Pair{p.s[q], p.c[q]});
        st += p.steps;
        cp += p.capped;
        n += p.n;
    }
    for (int q = 0; q < 5; ++q) {
        A.s[q] = tot[q].s;
        A.c[q] = tot[q].c;
    }
    A.steps = st;
    A.capped = cp;
    A.n = n;
}

__device__ __forceinline__ double grid_at(const FinalItem &f, size_t i)
{
    return f.up_f64 ? static_cast<const double *>(f.up_data)[i]
                    : (double)static_cast<const float *>(f.up_data)[i];
}

__device__ double interp_node(const FinalItem &g, int dim, const double *x)
{
    int i[3] = {0, 0, 0};
    double w[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) {
        const double t = (x[d] - g.up_lo[d]) * g.up_inv[d];
        const double fl = floor(t);
        int id = (int)fl;
        if (fl < 0.0) id = 0;
        if (fl > (double)(g.up_n[d] - 2)) id = g.up_n[d] - 2;
        double wd = t - (double)id;
        wd = wd < 0.0 ? 0.0 : (wd > 1.0 ? 1.0 : wd);
        i[d] = id;
        w[d] = wd;
    }
    const size_t nx = g.up_n[0], ny = g.up_n[1];
    if (dim == 2) {
        const size_t r0 = (size_t)i[1] * nx + i[0], r1 = r0 + nx;
        return (1.0 - w[1]) * ((1.0 - w[0]) * grid_at(g, r0) + w[0] * grid_at(g, r0 + 1)) +
               w[1] * ((1.0 - w[0]) * grid_at(g, r1) + w[0] * grid_at(g, r1 + 1));
    }
    double acc = 0.0;
    for (int dz = 0; dz < 2; ++dz) {
        double layer = 0.0;
        for (int dy = 0; dy < 2; ++dy) {
            const size_t row = ((size_t)(i[2] + dz) * ny + (i[1] + dy)) * nx + i[0];
            layer += (dy ? w[1] : 1.0 - w[1]) *
                     ((1.0 - w[0]) * grid_at(g, row) + w[0] * grid_at(g, row + 1));
        }
        acc += (dz ? w[2] : 1.0 - w[2]) * layer;
    }
    return acc;
}

__global__ void finalize_kernel(const FinalizeArgs f)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= f.n_nodes) return;
    const NodeAcc &A = f.acc[i];
    const FinalItem &fi = f.fitems[f.node_item[i]];
    const bool has_phi = fi.has_phi != 0;
    pdd_node_stats st;
    const double nan = __builtin_nan("");
    st.n = A.n;
    st.n_capped = A.capped;
    st.steps_sum = A.steps;
    for (int q = 0; q < 5; ++q) {
        st.sums[2 * q] = A.s[q];
        st.sums[2 * q + 1] = A.c[q];
    }
    st.mean = st.var = st.stderr_ = st.mean_steps = nan;
    st.mean_plain = st.var_plain = st.cov = st.rho = st.vr = st.vr_opt = nan;
    if (A.n > 0) {
        const double n = (double)A.n;
        const double Sp = A.s[0] + A.c[0], Sp2 = A.s[1] + A.c[1];
        const double Se = A.s[2] + A.c[2], Se2 = A.s[3] + A.c[3], Spe = A.s[4] + A.c[4];
        st.mean_steps = (double)A.steps / n;
        if (has_phi) {
            st.mean_plain = Sp / n;
            st.var_plain = A.n > 1 ? (Sp2 - Sp * Sp / n) / (n - 1.0) : nan;
        }
        if (!f.has_e) {
            st.mean = st.mean_plain;
            st.var = st.var_plain;
            st.stderr_ = sqrt(st.var / n);
        } else {
            st.mean = (fi.up_data ? interp_node(fi, f.dim, f.nodes + (size_t)i * f.dim) : 0.0) + Se / n;
            st.var = A.n > 1 ? (Se2 - Se * Se / n) / (n - 1.0) : nan;
            st.stderr_ = sqrt(st.var / n);
            if (has_phi) {
                // xi = u_prev(x0) + e - phi is the pathwise control variate
                // (Ito items: xi = e - phi); the constant enters neither cov nor rho
                const double cpe = A.n > 1 ? (Spe - Sp * Se / n) / (n - 1.0) : nan;
                const double vxi = st.var + st.var_plain - 2.0 * cpe;
                st.cov = cpe - st.var_plain;
                st.rho = st.cov / sqrt(st.var_plain * vxi);
                st.vr = st.var_plain / st.var;
                st.vr_opt = 1.0 / (1.0 - st.rho * st.rho);
            }
        }
    }
    fi.out[i - fi.gnode] = st;
}

// Starting sums: zero, or for an accumulating solve the statistics of the
// earlier paths.
__global__ void init_acc_kernel(NodeAcc *acc, uint32_t n, const uint32_t *node_item, const FinalItem *fitems)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const FinalItem &fi = fitems[node_item[i]];
    NodeAcc a;
    if (fi.accumulate) {
        const pdd_node_stats &p = fi.out[i - fi.gnode];
        for (int q = 0; q < 5; ++q) {
            a.s[q] = p.sums[2 * q];
            a.c[q] = p.sums[2 * q + 1];
        }
        a.n = p.n;
        a.steps = p.steps_sum;
        a.capped = p.n_capped;
    } else {
        for (int q = 0; q < 5; ++q) a.s[q] = a.c[q] = 0.0;
        a.n = a.steps = a.capped = 0;
    }
    a.pad = 0;
    acc[i] = a;
}

// One workgroup per item, copying its statistics word by word.
__global__ void gather_stats_kernel(const GatherItem *table, pdd_node_stats *dst)
{
    static_assert(sizeof(pdd_node_stats) % 8 == 0, "statistics are copied in 8-byte words");
    const GatherItem g = table[blockIdx.x];
    const uint64_t words = g.n * (sizeof(pdd_node_stats) / 8);
    const uint64_t *src = reinterpret_cast<const uint64_t *>(g.src);
    uint64_t *out = reinterpret_cast<uint64_t *>(dst + g.at);
    for (uint64_t q = threadIdx.x; q < words; q += blockDim.x) out[q] = src[q];
}

__global__ void zero_kernel(uint64_t *p, uint64_t n_words)
{
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < n_words;
         q += (uint64_t)gridDim.x * blockDim.x)
        p[q] = 0;
}

}  // namespace

hipError_t launch_reduce(const ReduceArgs &a, uint32_t n_blocks, hipStream_t s)
{
    if (n_blocks == 0) return hipSuccess;
    const uint32_t nc = a.n_chunks > 0 ? a.n_chunks : 1;
    hipLaunchKernelGGL(reduce_kernel, dim3(n_blocks, nc), dim3(kReduceBlock), 0, s, a);
    if (nc > 1) {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(merge_chunks_kernel, dim3((n_blocks + 255) / 256), dim3(256), 0, s, a, n_blocks);
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t s)
{
    if (a.n_nodes == 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3((a.n_nodes + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_init_acc(NodeAcc *acc, uint32_t n, const uint32_t *node_item, const FinalItem *fitems,
                           hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(init_acc_kernel, dim3((n + 255) / 256), dim3(256), 0, s, acc, n, node_item, fitems);
    return hipGetLastError();
}

hipError_t launch_gather_stats(const GatherItem *table, uint32_t n_items, pdd_node_stats *dst, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    hipLaunchKernelGGL(gather_stats_kernel, dim3(n_items), dim3(256), 0, s, table, dst);
    return hipGetLastError();
}

// Clears memory with a kernel (a memset node would misbehave in captured graphs).
hipError_t launch_zero(void *ptr, uint64_t bytes, hipStream_t s)
{
    const uint64_t words = bytes / 8;
    if (words == 0) return hipSuccess;
    uint64_t blocks = (words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(zero_kernel, dim3((uint32_t)blocks), dim3(256), 0, s,
                       static_cast<uint64_t *>(ptr), words);
    return hipGetLastError();
}

}  // namespace pdd
