// Issue-rate probe of the VALU instruction classes the path kernel uses, on
// gfx950: how many lane-operations per second (and per compute-unit clock)
// one class sustains when the whole chip issues nothing else. These rates set
// the cost weights and the peak of the path kernel's roofline.
//
// Each lane runs 8 independent dependency chains of one instruction, written
// in inline assembly (so the instruction is exactly the one named and the
// compiler can neither fold nor delete a chain: each asm reads and writes its
// chain's register), 16 times per loop iteration. With 8 chains per lane and
// 8 waves per SIMD every instruction's latency is hidden, so the time is set
// by issue alone. Block 0 records the shader clock counter and the constant
// wall clock around its loop, which gives the clock the chip actually ran at.
//
// Not part of the solver: built as its own library (libpdd_probe.so) for the
// benchmark's --issue-rates mode.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

enum Kind {
    kFmaF32 = 0,    // v_fma_f32
    kMulF32 = 1,    // v_mul_f32
    kAddU32 = 2,    // v_add_u32
    kBitop3 = 3,    // v_bitop3_b32 (three-way XOR)
    kMadU64 = 4,    // v_mad_u64_u32 (32 x 32 -> 64-bit multiply-add)
    kMulHi = 5,     // v_mul_hi_u32
    kExpF32 = 6,    // v_exp_f32
    kLogF32 = 7,    // v_log_f32
    kSinF32 = 8,    // v_sin_f32
    kSqrtF32 = 9,   // v_sqrt_f32
    kCvtF32 = 10,   // v_cvt_f32_u32
    kFmaF64 = 11,   // v_fma_f64
    kMulF64 = 12,   // v_mul_f64
    kFmacF32 = 13,  // v_fmac_f32 (two-operand encoding: d = a b + d)
    kXorB32 = 14,   // v_xor_b32
    kMulLo = 15,    // v_mul_lo_u32
    kMulU24 = 16,   // v_mul_u32_u24
    kMaxI32 = 17,   // v_max_i32
    kAddF64 = 18,   // v_add_f64
    kMovB32 = 19,   // v_mov_b32 (one-operand encoding; chain through a second register)
    // mixes: chains 0-3 run the first instruction, chains 4-7 the second
    kMixFmaMul = 20,   // v_fma_f32 | v_mul_f32
    kMixMadXor = 21,   // v_mad_u64_u32 | v_xor_b32
    kMixExpMul = 22,   // v_exp_f32 | v_mul_f32
    kMixFmacFmac = 23, // v_fmac_f32 | v_fmac_f32 (the same, as a control)
    kMixBitopFmac = 24, // v_bitop3_b32 | v_fmac_f32
    kNumKinds = 25
};

constexpr int kChains = 8;
constexpr int kUnroll = 16;

template <int K>
__device__ __forceinline__ void op(uint32_t (&u)[kChains], float (&f)[kChains], double (&d)[kChains],
                                   uint64_t (&q)[kChains], float fb, uint32_t ub, double db)
{
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        if constexpr (K == kFmaF32) asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(f[c]) : "v"(fb));
        if constexpr (K == kMulF32) asm volatile("v_mul_f32 %0, %0, %1" : "+v"(f[c]) : "v"(fb));
        if constexpr (K == kAddU32) asm volatile("v_add_u32 %0, %0, %1" : "+v"(u[c]) : "v"(ub));
        if constexpr (K == kBitop3) asm volatile("v_bitop3_b32 %0, %0, %1, %1 bitop3:0x96" : "+v"(u[c]) : "v"(ub));
        if constexpr (K == kMadU64) {
            // written in C (the compiler then gives the unused carry a
            // register without hazard padding): q' = lo(q) ub + q, which no
            // rewrite turns into something cheaper; the empty asm pins q
            q[c] = (uint64_t)(uint32_t)q[c] * ub + q[c];
            asm volatile("" : "+v"(q[c]));
        }
        if constexpr (K == kMulHi) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(u[c]) : "v"(ub));
        if constexpr (K == kExpF32) asm volatile("v_exp_f32 %0, %0" : "+v"(f[c]));
        if constexpr (K == kLogF32) asm volatile("v_log_f32 %0, %0" : "+v"(f[c]));
        if constexpr (K == kSinF32) asm volatile("v_sin_f32 %0, %0" : "+v"(f[c]));
        if constexpr (K == kSqrtF32) asm volatile("v_sqrt_f32 %0, %0" : "+v"(f[c]));
        if constexpr (K == kCvtF32) asm volatile("v_cvt_f32_u32 %0, %0" : "+v"(u[c]));
        if constexpr (K == kFmaF64) asm volatile("v_fma_f64 %0, %0, %1, %1" : "+v"(d[c]) : "v"(db));
        if constexpr (K == kMulF64) asm volatile("v_mul_f64 %0, %0, %1" : "+v"(d[c]) : "v"(db));
        if constexpr (K == kFmacF32) asm volatile("v_fmac_f32 %0, %1, %1" : "+v"(f[c]) : "v"(fb));
        if constexpr (K == kXorB32) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(u[c]) : "v"(ub));
        if constexpr (K == kMulLo) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(u[c]) : "v"(ub));
        if constexpr (K == kMulU24) asm volatile("v_mul_u32_u24 %0, %0, %1" : "+v"(u[c]) : "v"(ub));
        if constexpr (K == kMaxI32) asm volatile("v_max_i32 %0, %0, %1" : "+v"(u[c]) : "v"(ub));
        if constexpr (K == kAddF64) asm volatile("v_add_f64 %0, %0, %1" : "+v"(d[c]) : "v"(db));
        if constexpr (K == kMovB32) asm volatile("v_mov_b32 %0, %1" : "=v"(u[c]) : "v"(u[(c + 1) % kChains]));
        if constexpr (K == kMixFmaMul) {
            if (c < kChains / 2)
                asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(f[c]) : "v"(fb));
            else
                asm volatile("v_mul_f32 %0, %0, %1" : "+v"(f[c]) : "v"(fb));
        }
        if constexpr (K == kMixMadXor) {
            if (c < kChains / 2) {
                q[c] = (uint64_t)(uint32_t)q[c] * ub + q[c];
                asm volatile("" : "+v"(q[c]));
            } else {
                asm volatile("v_xor_b32 %0, %0, %1" : "+v"(u[c]) : "v"(ub));
            }
        }
        if constexpr (K == kMixExpMul) {
            if (c < kChains / 2)
                asm volatile("v_exp_f32 %0, %0" : "+v"(f[c]));
            else
                asm volatile("v_mul_f32 %0, %0, %1" : "+v"(f[c]) : "v"(fb));
        }
        if constexpr (K == kMixFmacFmac) asm volatile("v_fmac_f32 %0, %1, %1" : "+v"(f[c]) : "v"(fb));
        if constexpr (K == kMixBitopFmac) {
            if (c < kChains / 2)
                asm volatile("v_bitop3_b32 %0, %0, %1, %1 bitop3:0x96" : "+v"(u[c]) : "v"(ub));
            else
                asm volatile("v_fmac_f32 %0, %1, %1" : "+v"(f[c]) : "v"(fb));
        }
    }
}

template <int K>
__global__ void __launch_bounds__(256) issue_kernel(uint32_t iters, uint32_t never, uint32_t *sink,
                                                    long long *clocks)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t u[kChains];
    float f[kChains];
    double d[kChains];
    uint64_t q[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        u[c] = t * 2654435761u + (uint32_t)c;
        f[c] = 1.0f + 1e-7f * (float)(c + 1);
        d[c] = 1.0 + 1e-15 * (double)(c + 1);
        q[c] = u[c];
    }
    const float fb = 0.999999f + 1e-9f * (float)(t & 7);
    const uint32_t ub = 0x9E3779B9u ^ t;
    const double db = 0.9999999999 + 1e-14 * (double)(t & 7);
    long long c0 = 0, w0 = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c0 = clock64();
        w0 = wall_clock64();
    }
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < kUnroll; ++r) op<K>(u, f, d, q, fb, ub, db);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        clocks[0] = clock64() - c0;
        clocks[1] = wall_clock64() - w0;
    }
    // the chains' values leave the kernel only on a path the host never takes
    if (never == 0x5eed5eedu) {
        uint32_t s = 0;
#pragma unroll
        for (int c = 0; c < kChains; ++c)
            s ^= u[c] ^ __float_as_uint(f[c]) ^ (uint32_t)__double_as_longlong(d[c]) ^ (uint32_t)q[c];
        sink[t] = s;
    }
}

template <int K>
hipError_t launch(int grid, uint32_t iters, uint32_t *sink, long long *clocks, hipStream_t s)
{
    hipLaunchKernelGGL(issue_kernel<K>, dim3(grid), dim3(256), 0, s, iters, 0u, sink, clocks);
    return hipGetLastError();
}

hipError_t launch_kind(int kind, int grid, uint32_t iters, uint32_t *sink, long long *clocks, hipStream_t s)
{
    switch (kind) {
    case kFmaF32: return launch<kFmaF32>(grid, iters, sink, clocks, s);
    case kMulF32: return launch<kMulF32>(grid, iters, sink, clocks, s);
    case kAddU32: return launch<kAddU32>(grid, iters, sink, clocks, s);
    case kBitop3: return launch<kBitop3>(grid, iters, sink, clocks, s);
    case kMadU64: return launch<kMadU64>(grid, iters, sink, clocks, s);
    case kMulHi: return launch<kMulHi>(grid, iters, sink, clocks, s);
    case kExpF32: return launch<kExpF32>(grid, iters, sink, clocks, s);
    case kLogF32: return launch<kLogF32>(grid, iters, sink, clocks, s);
    case kSinF32: return launch<kSinF32>(grid, iters, sink, clocks, s);
    case kSqrtF32: return launch<kSqrtF32>(grid, iters, sink, clocks, s);
    case kCvtF32: return launch<kCvtF32>(grid, iters, sink, clocks, s);
    case kFmaF64: return launch<kFmaF64>(grid, iters, sink, clocks, s);
    case kMulF64: return launch<kMulF64>(grid, iters, sink, clocks, s);
    case kFmacF32: return launch<kFmacF32>(grid, iters, sink, clocks, s);
    case kXorB32: return launch<kXorB32>(grid, iters, sink, clocks, s);
    case kMulLo: return launch<kMulLo>(grid, iters, sink, clocks, s);
    case kMulU24: return launch<kMulU24>(grid, iters, sink, clocks, s);
    case kMaxI32: return launch<kMaxI32>(grid, iters, sink, clocks, s);
    case kAddF64: return launch<kAddF64>(grid, iters, sink, clocks, s);
    case kMovB32: return launch<kMovB32>(grid, iters, sink, clocks, s);
    case kMixFmaMul: return launch<kMixFmaMul>(grid, iters, sink, clocks, s);
    case kMixMadXor: return launch<kMixMadXor>(grid, iters, sink, clocks, s);
    case kMixExpMul: return launch<kMixExpMul>(grid, iters, sink, clocks, s);
    case kMixFmacFmac: return launch<kMixFmacFmac>(grid, iters, sink, clocks, s);
    case kMixBitopFmac: return launch<kMixBitopFmac>(grid, iters, sink, clocks, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

extern "C" {

// Number of instruction classes and the name of class `kind`.
int probe_kinds(void) { return kNumKinds; }

const char *probe_kind_name(int kind)
{
    static const char *names[kNumKinds] = {"v_fma_f32", "v_mul_f32", "v_add_u32", "v_bitop3_b32",
                                           "v_mad_u64_u32", "v_mul_hi_u32", "v_exp_f32", "v_log_f32",
                                           "v_sin_f32", "v_sqrt_f32", "v_cvt_f32_u32", "v_fma_f64",
                                           "v_mul_f64", "v_fmac_f32", "v_xor_b32", "v_mul_lo_u32",
                                           "v_mul_u32_u24", "v_max_i32", "v_add_f64", "v_mov_b32",
                                           "mix v_fma_f32+v_mul_f32", "mix v_mad_u64_u32+v_xor_b32",
                                           "mix v_exp_f32+v_mul_f32", "mix v_fmac_f32+v_fmac_f32",
                                           "mix v_bitop3_b32+v_fmac_f32"};
    return kind >= 0 && kind < kNumKinds ? names[kind] : "";
}

// Times class `kind` on the current device: blocks_per_cu x #CU workgroups
// of 256 threads, `iters` loop iterations of 16 x 8 instructions per lane,
// after one warm-up launch. Writes the launch time (ms), the lane-operations
// it issued, and block 0's shader-clock cycles and wall-clock time (ns) over
// its loop. Returns 0, or a HIP error code.
int probe_issue_rate(int kind, int blocks_per_cu, uint32_t iters, double *ms, double *lane_ops, double *cycles,
                     double *wall_ns)
{
    int dev = 0, n_cu = 0, wall_khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return (int)e;
    const int grid = n_cu * blocks_per_cu;
    uint32_t *sink = nullptr;
    long long *clocks = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    if ((e = hipMalloc(&sink, (size_t)grid * 256 * sizeof(uint32_t))) != hipSuccess) return (int)e;
    if ((e = hipMalloc(&clocks, 2 * sizeof(long long))) != hipSuccess) {
        (void)hipFree(sink);
        return (int)e;
    }
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = launch_kind(kind, grid, iters, sink, clocks, nullptr);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(a, nullptr);
    if (e == hipSuccess) e = launch_kind(kind, grid, iters, sink, clocks, nullptr);
    if (e == hipSuccess) e = hipEventRecord(b, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.f;
    long long host_clk[2] = {0, 0};
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    if (e == hipSuccess) e = hipMemcpy(host_clk, clocks, sizeof host_clk, hipMemcpyDeviceToHost);
    if (e == hipSuccess) {
        const double per_lane = (double)iters * kUnroll * kChains;
        *ms = (double)t;
        *lane_ops = per_lane * (double)grid * 256.0;
        *cycles = (double)host_clk[0];
        *wall_ns = (double)host_clk[1] * 1e6 / (double)wall_khz;
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipFree(sink);
    (void)hipFree(clocks);
    return (int)e;
}

}  // extern "C"
