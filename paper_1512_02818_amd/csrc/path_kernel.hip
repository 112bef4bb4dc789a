// Path kernel of the first-stage PDD nodal solve on gfx950.
//
// One path per lane. A persistent wavefront takes paths from a global queue
// (one atomic per `grab` paths) and refills a lane as soon as its path has
// ended, so waves stay full whatever the spread of exit times. Each path is
// the Euler-Maruyama walk of Alg. 1 (eq. F:E_M, coefficients at the left
// point) with the bridge, shifted-boundary or naive exit test, carrying the
// killing weight Y, the source integral Z and, for the correction estimator,
// the residual integral R (Sec. 2.3; eq. F:Dynkin). Every path writes its
// score and exit step to its own slot; the per-node sums are formed afterwards
// in a fixed order, so results do not depend on scheduling.
//
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) in registers, key =
// problem seed (wave-uniform), counter = (step block, path, node, stream tag).
// In 2D one block gives the two normals of two consecutive steps (words 0,1
// then 2,3), so a lane starts a new path only at an even step; in 3D one block
// per step. The bridge uniform of step s is word s mod 4 of the tag-1 block
// s/4; the block is drawn for every walking lane of the wave at the first step
// of its four-step window at which some lane may have a live face, and cached
// for the rest of the window (drawn per lane inside the rare branch, it would
// be drawn up to four times per window, once for each step at which another
// lane first needs it).
// Box-Muller (1958) on the VALU: in FP32 with the hardware log2, sqrt, sin
// and cos (which take revolutions, so 2 pi u needs no multiply).
#include <type_traits>

#include "pdd_internal.hpp"

namespace pdd {
namespace {

// Device memory that the kernels reach through pointers held in descriptor
// tables (grids, node tables, records). The compiler cannot tell such a
// pointer from an LDS one and would emit flat accesses, which count against
// the same wait counter as the scalar loads of descriptor fields: every wait
// for a field would then also wait for an in-flight grid gather. Casting to
// the global address space gives global loads and stores with their own
// counter.
template <class T>
using Global = __attribute__((address_space(1))) T;
template <class T>
__device__ __forceinline__ T gload(const T *p)
{
    return *(const Global<T> *)p;
}
template <class T>
__device__ __forceinline__ void gstore(T *p, T v)
{
    *(Global<T> *)p = v;
}

constexpr float kLn2f = 0.6931471805599453f;
constexpr float kLog2ef = 1.4426950408889634f;
constexpr double kTwoPi = 6.283185307179586476925286766559;

struct Block4 {
    uint32_t w0, w1, w2, w3;
};

// Philox4x32-10: two 32x32->64 products per round (v_mad_u64_u32) and two
// three-way XORs (v_bitop3_b32 with the XOR3 truth table 0x96), the key bumped
// by the Weyl constants after each round.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// The ten round keys of a (wave-uniform) Philox key, in vector registers: the
// XOR3 takes three vector operands at no extra cost, and keeping twenty
// uniform values out of the scalar register file leaves it to the problem
// constants. Used by the FP32 walks, which are bound by instruction issue:
// recomputing the keys would add scalar instructions to every block.
struct KeySchedule {
    uint32_t k0[10], k1[10];
};

// The key as two scalar words, round keys recomputed by scalar adds in every
// block. Used by the FP64 walks, whose vector registers are the scarce
// resource: twenty fewer live values remove their spills.
struct ScalarKey {
    uint32_t k0, k1;
};

template <class T>
using KeysOf = typename std::conditional<sizeof(T) == 8, ScalarKey, KeySchedule>::type;

template <class K>
__device__ __forceinline__ K key_schedule(uint32_t k0, uint32_t k1);

template <>
__device__ __forceinline__ ScalarKey key_schedule<ScalarKey>(uint32_t k0, uint32_t k1)
{
    return {(uint32_t)__builtin_amdgcn_readfirstlane(k0), (uint32_t)__builtin_amdgcn_readfirstlane(k1)};
}

template <>
__device__ __forceinline__ KeySchedule key_schedule<KeySchedule>(uint32_t k0, uint32_t k1)
{
    KeySchedule ks;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t v0, v1;
        asm volatile("v_mov_b32 %0, %1" : "=v"(v0) : "s"(k0));
        asm volatile("v_mov_b32 %0, %1" : "=v"(v1) : "s"(k1));
        ks.k0[r] = v0;
        ks.k1[r] = v1;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return ks;
}

__device__ __forceinline__ Block4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         const KeySchedule &ks)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, ks.k0[r]);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, ks.k1[r]);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    return {c0, c1, c2, c3};
}

__device__ __forceinline__ Block4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         const ScalarKey &key)
{
    // opaque to the optimiser, so that the round keys are formed here rather
    // than hoisted out of the walk loop into twenty live registers
    uint32_t ka = key.k0, kb = key.k1;
    asm volatile("" : "+s"(ka), "+s"(kb));
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, ka);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, kb);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        ka += 0x9E3779B9u;
        kb += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// Multiply-add with one rounding. The library is built without automatic
// contraction, so every fused operation is written out and all kernels that
// walk the same path round identically.
__device__ __forceinline__ float madd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// x clamped to [lo, hi] (lo <= hi, x not NaN): one median-of-three.
__device__ __forceinline__ float med3(float x, float lo, float hi) { return __builtin_amdgcn_fmed3f(x, lo, hi); }
__device__ __forceinline__ double med3(double x, double lo, double hi) { return fmin(fmax(x, lo), hi); }
__device__ __forceinline__ double madd(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class T>
struct Arith;

// FP32 path arithmetic: 24-bit uniforms, hardware transcendentals.
template <>
struct Arith<float> {
    // (w + 1/2) 2^-32 with w rounded to 24 significant bits: within 2^-24
    // (relative) of the FP64 uniform of the same word, in (0, 1]. It is
    // exactly 1 for the top 128 words (w >= 2^32 - 128, probability 2^-25):
    // such a bridge draw cannot end a path, and Box-Muller gives r = 0.
    __device__ static __forceinline__ float unif(uint32_t w)
    {
        return fmaf((float)w, 0x1.0p-32f, 0x1.0p-33f);
    }
    __device__ static __forceinline__ float unif_bridge(uint32_t w) { return unif(w); }
    __device__ static __forceinline__ float radius(uint32_t w)
    {
        return __builtin_amdgcn_sqrtf(-2.0f * kLn2f * __builtin_amdgcn_logf(unif(w)));
    }
    __device__ static __forceinline__ void box_muller(uint32_t a, uint32_t b, float &n0, float &n1)
    {
        const float r = radius(a);
        const float t = unif(b);  // revolutions
        n0 = r * __builtin_amdgcn_cosf(t);
        n1 = r * __builtin_amdgcn_sinf(t);
    }
    __device__ static __forceinline__ float box_muller_cos(uint32_t a, uint32_t b)
    {
        return radius(a) * __builtin_amdgcn_cosf(unif(b));
    }
    // k and ph are in revolutions; the hardware sine and cosine reduce any
    // argument within +-256 revolutions themselves.
    __device__ static __forceinline__ void trig(const DevTrig<float> &t, int d, float x, float &s,
                                                float &c)
    {
        const float rev = fmaf(t.k[d], x, t.ph[d]);
        s = __builtin_amdgcn_sinf(rev);
        c = __builtin_amdgcn_cosf(rev);
    }
    __device__ static __forceinline__ float sine(const DevTrig<float> &t, int d, float x)
    {
        return __builtin_amdgcn_sinf(fmaf(t.k[d], x, t.ph[d]));
    }
    __device__ static __forceinline__ float exp_neg(float x)
    {
        return __builtin_amdgcn_exp2f(-x * kLog2ef);
    }
    __device__ static __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
};

// FP64 path arithmetic: 32-bit uniforms, correctly rounded-ish library calls.
template <>
struct Arith<double> {
    __device__ static __forceinline__ double unif(uint32_t w)
    {
        return ((double)w + 0.5) * 0x1.0p-32;
    }
    __device__ static __forceinline__ double unif_bridge(uint32_t w) { return unif(w); }
    __device__ static __forceinline__ void box_muller(uint32_t a, uint32_t b, double &n0,
                                                      double &n1)
    {
        const double r = sqrt(-2.0 * log(unif(a)));
        const double th = kTwoPi * unif(b);
        double s, c;
        sincos(th, &s, &c);
        n0 = r * c;
        n1 = r * s;
    }
    __device__ static __forceinline__ double box_muller_cos(uint32_t a, uint32_t b)
    {
        return sqrt(-2.0 * log(unif(a))) * cos(kTwoPi * unif(b));
    }
    __device__ static __forceinline__ void trig(const DevTrig<double> &t, int d, double x,
                                                double &s, double &c)
    {
        sincos(madd(t.k[d], x, t.ph[d]), &s, &c);
    }
    __device__ static __forceinline__ double sine(const DevTrig<double> &t, int d, double x)
    {
        return sin(madd(t.k[d], x, t.ph[d]));
    }
    __device__ static __forceinline__ double exp_neg(double x) { return exp(-x); }
    __device__ static __forceinline__ double sqrt_(double x) { return sqrt(x); }
};

// Sum of monomials coef * x^e0 y^e1 z^e2 (exponents read from a wave-uniform
// packed word, so the power loops are scalar-controlled).
template <class T, int D>
__device__ __forceinline__ T poly_value(const DevPoly<T> *terms, int n, const T *x)
{
    T acc = (T)0;
    for (int m = 0; m < n; ++m) {
        const uint32_t e = terms[m].e;
        T v = terms[m].coef;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int ed = (int)((e >> (8 * d)) & 0xffu);
            for (int i = 0; i < ed; ++i) v *= x[d];
        }
        acc += v;
    }
    return acc;
}

// Dense polynomial in nested Horner form (no loops at run time): in 2D
// sum_j y^j sum_{i <= 5 - j} c_ij x^i, coefficients ordered by j then i;
// in 3D sum_k z^k sum_j y^j sum_{i <= 4 - j - k} c_ijk x^i, ordered by k, j, i.
template <class T, int D>
__device__ __forceinline__ T dense_poly(const T *c, const T *x)
{
    if (D == 2) {
        constexpr int deg = kDenseDeg2;
        T acc = (T)0;
        int off = (deg + 1) * (deg + 2) / 2;
#pragma unroll
        for (int j = deg; j >= 0; --j) {
            off -= deg - j + 1;  // first coefficient of row j
            T p = c[off + deg - j];
#pragma unroll
            for (int i = deg - j - 1; i >= 0; --i) p = madd(p, x[0], c[off + i]);
            acc = (j == deg) ? p : madd(acc, x[1], p);
        }
        return acc;
    }
    constexpr int deg = kDenseDeg3;
    T accz = (T)0;
    int off = kMaxDense;
#pragma unroll
    for (int k = deg; k >= 0; --k) {
        T accy = (T)0;
#pragma unroll
        for (int j = deg - k; j >= 0; --j) {
            off -= deg - j - k + 1;  // row (j, k)
            T p = c[off + deg - j - k];
#pragma unroll
            for (int i = deg - j - k - 1; i >= 0; --i) p = madd(p, x[0], c[off + i]);
            accy = (j == deg - k) ? p : madd(accy, x[1], p);
        }
        accz = (k == deg) ? accy : madd(accz, x[2 % D], accy);
    }
    return accz;
}

template <class T, int D>
__device__ __forceinline__ T interp_cells(const GridView<T> &g, const T *x);
template <class T, int D>
__device__ __forceinline__ void grid_cell(const GridView<T> &g, const T *x, int *i, T *w);
template <class T, int D>
__device__ __forceinline__ size_t cell_index(const GridView<T> &g, const int *i);
template <class T, int D>
__device__ __forceinline__ T interp_corners(const T *p, const T *w);
template <class T>
__device__ __forceinline__ T interp_corner_values(T c00, T c10, T c01, T c11, const T *w);
template <class T, int D>
__device__ __forceinline__ void analytic_source(const DevProblem<T> &P, const T *x, const T *b, T c, T &f,
                                                const T *cf);

// b(x), c(x) and, when asked, f(x) = F(x) + sum over trig terms T of
// (1/2) sigma^2 Lap T + b.grad T + c T, where Lap T = -|k|^2 T and
// d_d T = amp k_d cos(k_d x_d + ph_d) prod_{e != d} sin(k_e x_e + ph_e).
// The dense coefficients of F come from `cf` (a copy of P.fdense in LDS).
// Tabulated coefficients (bit q of `tab`: tabv[q] replaces b_0, b_1, b_2, c,
// f) are interpolated instead; the analytic f always uses the analytic b, c.
template <class T>
using Vec4 = T __attribute__((ext_vector_type(4)));

// The four 16-byte chunks of the pair records that hold a cell's corners
// (p00, p01, p10, p11 at rec[0..3]). Each lane of a quad whose four lanes are
// all active loads chunk m = lane & 3 of every quad member's record, so that a
// load instruction touches 16 cache lines rather than 64 (one per lane: the
// gather of divergent 64-byte records is what bounds these walks), and the
// wave's LDS block `tr` (4 x 64 chunks) hands each lane its own four chunks
// back. Lanes of other quads load their record themselves. The values are
// those of the direct loads, bit for bit.
template <class T>
__device__ __forceinline__ void pair_chunks(const Vec4<T> *base, uint32_t rec, Vec4<T> *tr, Vec4<T> &p00,
                                            Vec4<T> &p01, Vec4<T> &p10, Vec4<T> &p11)
{
    const int lane = __lane_id();
    const uint64_t act = __builtin_amdgcn_read_exec();
    if (tr != nullptr && ((act >> (lane & ~3)) & 0xfull) == 0xfull) {
        const uint32_t m = (uint32_t)lane & 3u;
        // record offset of quad lane k (quad_perm k,k,k,k), chunk m of it
        const uint32_t r0 = (uint32_t)__builtin_amdgcn_mov_dpp((int)rec, 0x00, 0xf, 0xf, false);
        const uint32_t r1 = (uint32_t)__builtin_amdgcn_mov_dpp((int)rec, 0x55, 0xf, 0xf, false);
        const uint32_t r2 = (uint32_t)__builtin_amdgcn_mov_dpp((int)rec, 0xaa, 0xf, 0xf, false);
        const uint32_t r3 = (uint32_t)__builtin_amdgcn_mov_dpp((int)rec, 0xff, 0xf, 0xf, false);
        const Vec4<T> v0 = gload(base + r0 + m), v1 = gload(base + r1 + m), v2 = gload(base + r2 + m),
                      v3 = gload(base + r3 + m);
        tr[0 * 64 + lane] = v0;
        tr[1 * 64 + lane] = v1;
        tr[2 * 64 + lane] = v2;
        tr[3 * 64 + lane] = v3;
        // chunk m of quad lane k sits at tr[k * 64 + quad + m]
        const Vec4<T> *mine = tr + (lane & 3) * 64 + (lane & ~3);
        p00 = mine[0];
        p01 = mine[1];
        p10 = mine[2];
        p11 = mine[3];
    } else {
        p00 = gload(base + rec);
        p01 = gload(base + rec + 1);
        p10 = gload(base + rec + 2);
        p11 = gload(base + rec + 3);
    }
}

template <class T, int D>
__device__ __forceinline__ void coefficients(const DevProblem<T> &P, const T *x, T *b, T &c,
                                             T &f, bool want_f, const T *cf, uint32_t tab,
                                             Vec4<T> *tr = nullptr)
{
#pragma unroll
    for (int i = 0; i < D; ++i) {
        T v = P.b0[i];
#pragma unroll
        for (int j = 0; j < D; ++j) v = madd(P.B[i][j], x[j], v);
        b[i] = v;
    }
    T r2 = (T)0;
#pragma unroll
    for (int d = 0; d < D; ++d) r2 = madd(x[d], x[d], r2);
    c = madd(P.c_b, r2, P.c_a);
    if (tab & 64u) {  // every coefficient tabulated, interleaved
        int i[D];
        T w[D];
        grid_cell<T, D>(P.tabv[3], x, i, w);
        if (D == 2 && (tab & 128u)) {  // pair records of the cell's two lower corners: all four
            const uint32_t n0 = (uint32_t)P.tabv[3].n[0];
            Vec4<T> p00, p01, p10, p11;
            pair_chunks<T>(reinterpret_cast<const Vec4<T> *>(P.tab_fused), 2u * ((uint32_t)i[1] * n0 + (uint32_t)i[0]),
                           tr, p00, p01, p10, p11);
            b[0] = interp_corner_values<T>(p00.x, p10.x, p01.x, p11.x, w);
            b[1 % D] = interp_corner_values<T>(p00.y, p10.y, p01.y, p11.y, w);
            c = interp_corner_values<T>(p00.z, p10.z, p01.z, p11.z, w);
            if (want_f) f = interp_corner_values<T>(p00.w, p10.w, p01.w, p11.w, w);
            return;
        }
        const T *rec = P.tab_fused + cell_index<T, D>(P.tabv[3], i) * (size_t)((D + 2) << D);
#pragma unroll
        for (int d = 0; d < D; ++d) b[d] = interp_corners<T, D>(rec + (d << D), w);
        c = interp_corners<T, D>(rec + (D << D), w);
        if (want_f) f = interp_corners<T, D>(rec + ((D + 1) << D), w);
        return;
    }
    if (tab) {
        if (want_f && (tab & 16u)) {
            f = interp_cells<T, D>(P.tabv[4], x);
            want_f = false;
        }
        if (want_f) analytic_source<T, D>(P, x, b, c, f, cf);
#pragma unroll
        for (int d = 0; d < D; ++d)
            if (tab & (1u << d)) b[d] = interp_cells<T, D>(P.tabv[d], x);
        if (tab & 8u) c = interp_cells<T, D>(P.tabv[3], x);
        return;
    }
    if (want_f) analytic_source<T, D>(P, x, b, c, f, cf);
}

// The analytic source for the analytic b and c.
template <class T, int D>
__device__ __forceinline__ void analytic_source(const DevProblem<T> &P, const T *x, const T *b, T c, T &f,
                                                const T *cf)
{
    T acc = (T)0;
    if (P.f_mode == kPolyDense)
        acc = dense_poly<T, D>(cf, x);
    else if (P.f_mode == kPolySparse)
        acc = poly_value<T, D>(P.fpoly, P.n_f, x);
    for (int m = 0; m < P.n_trig; ++m) {
        const DevTrig<T> &t = P.trig[m];
        T s[D], co[D];
#pragma unroll
        for (int d = 0; d < D; ++d) Arith<T>::trig(t, d, x[d], s[d], co[d]);
        T prod = s[0];
#pragma unroll
        for (int d = 1; d < D; ++d) prod *= s[d];
        acc = madd(madd(c, t.amp, t.nhk2a), prod, acc);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int last = d == D - 1 ? D - 2 : D - 1;  // factor taken by the fused add
            T g = b[d] * t.ak[d] * co[d];
#pragma unroll
            for (int e = 0; e < D; ++e)
                if (e != d && e != last) g *= s[e];
            acc = madd(g, s[last], acc);
        }
    }
    f = acc;
}

// g = G + sum(trig) at a boundary point.
template <class T, int D>
__device__ __forceinline__ T boundary_value(const DevProblem<T> &P, const T *x, uint32_t tab)
{
    if (tab & 32u) return interp_cells<T, D>(P.tabv[5], x);  // tabulated g
    T u = poly_value<T, D>(P.gpoly, P.n_g, x);
    for (int m = 0; m < P.n_trig; ++m) {
        const DevTrig<T> &t = P.trig[m];
        T v = t.amp;
#pragma unroll
        for (int d = 0; d < D; ++d) v *= Arith<T>::sine(t, d, x[d]);
        u += v;
    }
    return u;
}

// Cell of a grid holding x and the weights within it: cell index floor(t)
// clamped to [0, n - 2] and weight t - index clamped to [0, 1], for
// t = (x - lo) inv. Clamping t to [0, n - 1] first gives exactly those values
// (below 0: cell 0, weight 0; from n - 1 up: cell n - 2, weight 1) with one
// truncation and no floor.
template <class T, int D>
__device__ __forceinline__ void grid_cell(const GridView<T> &g, const T *x, int *i, T *w)
{
#pragma unroll
    for (int d = 0; d < D; ++d) {
        T t = (x[d] - g.lo[d]) * g.inv[d];
        t = med3(t, (T)0, g.top[d]);
        int id = (int)t;
        id = id < g.n[d] - 2 ? id : g.n[d] - 2;
        i[d] = id;
        w[d] = t - (T)id;
    }
}

// Bilinear (2D) / trilinear (3D) interpolation of a grid at x.
template <class T, int D>
__device__ __forceinline__ T interp(const GridView<T> &g, const T *x)
{
    int i[D];
    T w[D];
    grid_cell<T, D>(g, x, i, w);
    const int nx = g.n[0];
    if (D == 2) {
        const T *r0 = g.data + (size_t)i[1] * nx + i[0];
        const T *r1 = r0 + nx;
        const T l0 = madd(w[0], gload(r0 + 1), ((T)1 - w[0]) * gload(r0));
        const T l1 = madd(w[0], gload(r1 + 1), ((T)1 - w[0]) * gload(r1));
        return madd(w[1], l1, ((T)1 - w[1]) * l0);
    }
    const int ny = g.n[1];
    T acc = (T)0;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
        T layer = (T)0;
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            const T *row = g.data + ((size_t)(i[2 % D] + dz) * ny + (i[1] + dy)) * nx + i[0];
            const T line = madd(w[0], gload(row + 1), ((T)1 - w[0]) * gload(row));
            layer = madd(dy ? w[1] : (T)1 - w[1], line, layer);
        }
        acc = madd(dz ? w[2 % D] : (T)1 - w[2 % D], layer, acc);
    }
    return acc;
}

// The same interpolation from the grid's cell layout: the corners of the
// cell come in one aligned vector load (two in 3D) instead of 2^D gathers;
// operands and operations are those of interp, so the value is identical.
// interp_cell_at takes the cell and weights already found by grid_cell (for
// several grids of one geometry).
template <class T, int D>
__device__ __forceinline__ size_t cell_index(const GridView<T> &g, const int *i)
{
    const size_t mx = (size_t)(g.n[0] - 1);
    if (D == 2) return (uint32_t)i[1] * (uint32_t)(g.n[0] - 1) + (uint32_t)i[0];
    return ((size_t)i[2 % D] * (size_t)(g.n[1] - 1) + i[1]) * mx + i[0];
}

// Bilinear interpolation from the four corner values of a cell ((0,0),
// (1,0), (0,1), (1,1)), the operations of interp_corners.
template <class T>
__device__ __forceinline__ T interp_corner_values(T c00, T c10, T c01, T c11, const T *w)
{
    const T l0 = madd(w[0], c10, ((T)1 - w[0]) * c00);
    const T l1 = madd(w[0], c11, ((T)1 - w[0]) * c01);
    return madd(w[1], l1, ((T)1 - w[1]) * l0);
}

// Interpolation from the 2^D corner values of one cell, stored together at p.
template <class T, int D>
__device__ __forceinline__ T interp_corners(const T *p, const T *w)
{
    typedef T V4 __attribute__((ext_vector_type(4)));
    if (D == 2) {
        const V4 c = gload(reinterpret_cast<const V4 *>(p));
        const T l0 = madd(w[0], c.y, ((T)1 - w[0]) * c.x);
        const T l1 = madd(w[0], c.w, ((T)1 - w[0]) * c.z);
        return madd(w[1], l1, ((T)1 - w[1]) * l0);
    }
    const V4 *cv = reinterpret_cast<const V4 *>(p);
    T acc = (T)0;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
        const V4 c = gload(cv + dz);
        const T line0 = madd(w[0], c.y, ((T)1 - w[0]) * c.x);
        const T line1 = madd(w[0], c.w, ((T)1 - w[0]) * c.z);
        T layer = madd((T)1 - w[1], line0, (T)0);
        layer = madd(w[1], line1, layer);
        acc = madd(dz ? w[2 % D] : (T)1 - w[2 % D], layer, acc);
    }
    return acc;
}

template <class T, int D>
__device__ __forceinline__ T interp_cell_at(const GridView<T> &g, const int *i, const T *w)
{
    return interp_corners<T, D>(g.cells + (cell_index<T, D>(g, i) << D), w);
}

template <class T, int D>
__device__ __forceinline__ T interp_cells(const GridView<T> &g, const T *x)
{
    int i[D];
    T w[D];
    grid_cell<T, D>(g, x, i, w);
    return interp_cell_at<T, D>(g, i, w);
}

// Cell layout of a grid (see cell_values), values converted from S to T: one
// thread per cell.
template <class S, class T, int D>
__global__ void grid_cells_kernel(const S *__restrict__ data, int n0, int n1, int n2, T *__restrict__ cells,
                                  uint32_t stride, uint32_t off)
{
    const uint64_t m0 = (uint64_t)(n0 - 1), m1 = (uint64_t)(n1 - 1), m2 = D == 3 ? (uint64_t)(n2 - 1) : 1;
    const uint64_t n_cells = m0 * m1 * m2;
    for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < n_cells;
         c += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = c % m0, j = (c / m0) % m1, k = c / (m0 * m1);
        T *out = cells + c * stride + off;
#pragma unroll
        for (int dz = 0; dz < (D == 3 ? 2 : 1); ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx)
                    out[(dz * 2 + dy) * 2 + dx] = (T)data[((k + dz) * (uint64_t)n1 + (j + dy)) * (uint64_t)n0 + i + dx];
    }
}

// Point values of a grid converted from S to T into every stride-th slot (a
// field of interleaved records): one thread per point.
template <class S, class T>
__global__ void grid_points_kernel(const S *__restrict__ data, uint64_t n_points, T *__restrict__ out,
                                   uint32_t stride, uint32_t off)
{
    for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < n_points;
         p += (uint64_t)gridDim.x * blockDim.x)
        out[p * stride + off] = (T)data[p];
}

// Domain, exit test and increment law: read from the problem and item at run
// time, or fixed at compile time for the common box / bridge / Gaussian case,
// which removes their branches and frees the registers of the other cases.
// `dense`: the form of the bridge test for walks in which many lanes of a
// wave are near a face at every step (short paths, a wide step against the
// box), where the per-lane branches of the other form would run at nearly
// every step; both give the same bits.
struct RuntimeMode {
    template <class T>
    __device__ static __forceinline__ int domain(const DevProblem<T> &P) { return P.domain; }
    template <class T>
    __device__ static __forceinline__ bool dense(const ItemCore<T> &a) { return a.dense_bridge != 0; }
    template <class T>
    __device__ static __forceinline__ int exit(const ItemCore<T> &a) { return a.exit_mode; }
    template <class T>
    __device__ static __forceinline__ int law(const ItemCore<T> &a) { return a.law; }
    template <class T>
    __device__ static __forceinline__ uint32_t tab(const DevProblem<T> &P) { return P.tab; }
};
template <bool DENSE>
struct BoxBridgeGaussT {
    template <class T>
    __device__ static constexpr int domain(const DevProblem<T> &) { return kBox; }
    template <class T>
    __device__ static constexpr int exit(const ItemCore<T> &) { return kExitBridge; }
    template <class T>
    __device__ static constexpr int law(const ItemCore<T> &) { return kLawGauss; }
    template <class T>
    __device__ static constexpr uint32_t tab(const DevProblem<T> &) { return 0u; }
    template <class T>
    __device__ static constexpr bool dense(const ItemCore<T> &) { return DENSE; }
};
using BoxBridgeGauss = BoxBridgeGaussT<false>;
using BoxBridgeGaussDense = BoxBridgeGaussT<true>;

template <class T, int D>
__device__ __forceinline__ T inner_distance(const DevProblem<T> &P, int domain, const T *x)
{
    if (domain == kBox) {
        T m = x[0] - P.lo[0];
        m = fmin(m, P.hi[0] - x[0]);
#pragma unroll
        for (int d = 1; d < D; ++d) {
            m = fmin(m, x[d] - P.lo[d]);
            m = fmin(m, P.hi[d] - x[d]);
        }
        return m;
    }
    T r2 = (T)0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const T t = x[d] - P.center[d];
        r2 = madd(t, t, r2);
    }
    return P.radius - Arith<T>::sqrt_(r2);
}

template <class T, int D>
__device__ __forceinline__ void radial(const DevProblem<T> &P, const T *x, T *out)
{
    T r2 = (T)0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const T t = x[d] - P.center[d];
        r2 = madd(t, t, r2);
    }
    const T r = Arith<T>::sqrt_(r2);
#pragma unroll
    for (int d = 0; d < D; ++d)
        out[d] = r > (T)0 ? madd(P.radius, (x[d] - P.center[d]) / r, P.center[d])
                          : P.center[d] + (d == 0 ? P.radius : (T)0);
}

// Closest boundary point: inside a box the nearest face (ties to the lowest
// face index, faces ordered x-lo, x-hi, y-lo, ...), outside the clamp.
template <class T, int D>
__device__ __forceinline__ void project(const DevProblem<T> &P, int domain, const T *x, T *out)
{
    if (domain == kBall) {
        radial<T, D>(P, x, out);
        return;
    }
    bool inside = true;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        out[d] = x[d];
        inside = inside && (x[d] > P.lo[d]) && (x[d] < P.hi[d]);
    }
    if (inside) {
        int best = 0;
        T bd = x[0] - P.lo[0];
#pragma unroll
        for (int f = 1; f < 2 * D; ++f) {
            const int d = f >> 1;
            const T t = (f & 1) ? P.hi[d] - x[d] : x[d] - P.lo[d];
            if (t < bd) {
                bd = t;
                best = f;
            }
        }
#pragma unroll
        for (int d = 0; d < D; ++d)
            if ((best >> 1) == d) out[d] = (best & 1) ? P.hi[d] : P.lo[d];
    } else {
#pragma unroll
        for (int d = 0; d < D; ++d) out[d] = fmin(fmax(out[d], P.lo[d]), P.hi[d]);
    }
}

// State of the path a lane is walking.
// RNG_TABLE: items may be merged solves with a per-node RNG table (batch
// kernel); the single-item kernel takes the stream tag from its item.
// Score of an ended path, written as its record r: phi = g(X_tau) Y + Z
// (plain), e = (g - u_prev)(X_tau) Y - R (correction), phi and phi + xi (Ito),
// and the exit step word.
template <class T, int D, int EST, class M>
__device__ __forceinline__ void score_path(const ItemCore<T> &a, const DevProblem<T> &P, const T *Xt, T Y, double Z,
                                           double R, uint32_t word, uint64_t r)
{
    const T gv = boundary_value<T, D>(P, Xt, M::tab(P));
    if (EST == kEstIto) {  // phi and phi + xi
        const double phi = madd((double)gv, (double)Y, Z);
        gstore(a.rec_phi + r, phi);
        gstore(a.rec_e + r, phi + R);
    } else if (a.score_plain) {
        gstore(a.rec_phi + r, madd((double)gv, (double)Y, Z));
    }
    if (EST == kEstCorrection) {
        const T up = interp<T, D>(a.u_prev, Xt);
        gstore(a.rec_e + r, madd((double)gv - (double)up, (double)Y, -R));
    }
    gstore(a.rec_steps + r, word);
}

// Ended paths of a wave waiting to be scored (batch kernel; dense-bridge and
// generic forms of the single-item kernel): a ring in the wave's LDS (dynamic
// shared memory, one ring per wave).
template <class T, int D>
struct EndedPath {
    T Xt[D];
    T Y;
    uint32_t word;  // exit step | capped bit
    double Z, R;
    uint64_t r;     // record index
};
constexpr uint32_t kEndRing = 128;  // holds a batch of 64 and the up to 64 ended at one turn
template <class T, int D>
struct EndRing {
    EndedPath<T, D> e[kEndRing];
};

template <class T, int D, int EST, class M, bool RNG_TABLE>
struct Walker {
    T X[D], Xt[D];
    T Y;
    T m;  // distance from X to the boundary (inside; cached between steps)
    double Z, R;  // R: sum h Y r (correction estimator) or xi (Ito control variate)
    uint64_t slot;
    uint32_t k, j, node, capped;
    uint32_t tag;  // stream tag of the path's solve (RNG_TABLE)

    // Stream tag of the path: its own with an RNG table, else the item's
    // (a wave-uniform scalar).
    __device__ __forceinline__ uint32_t stream(const ItemCore<T> &a) const { return RNG_TABLE ? tag : a.stream_tag; }
    uint32_t bb_blk;
    uint64_t bw01, bw23;  // cached bridge block, words (0,1) and (2,3)
    KeysOf<T> ks;
    const T *cf;          // dense source coefficients of the problem, in LDS
    Vec4<T> *tr;          // the wave's LDS block for gathering pair records (single-item kernel)

    // Starts path r (slot within the item) of item a. Returns false when it
    // ends before any step (a node inside the shift band of the shifted test).
    __device__ __forceinline__ bool start(const ItemCore<T> &a, const DevProblem<T> &P, uint64_t r, const uint32_t *node_rng)
    {
        slot = r;
        uint64_t jj;
        if (a.node_start == nullptr) {
            if (a.n_slots <= 0xffffffffull) {
                const uint32_t q = (uint32_t)r / (uint32_t)a.uniform_n;
                node = q;
                jj = (uint32_t)r - q * (uint32_t)a.uniform_n;
            } else {
                node = (uint32_t)(r / a.uniform_n);
                jj = r - (uint64_t)node * a.uniform_n;
            }
        } else {
            uint32_t lo = 0, hi = a.n_nodes;  // node_start[lo] <= r < node_start[hi]
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (gload(a.node_start + mid) <= r)
                    lo = mid;
                else
                    hi = mid;
            }
            node = lo;
            jj = r - gload(a.node_start + lo);
        }
        // the path's RNG counter: its node, stream and path index in its own solve
        j = (uint32_t)(a.path_offset + jj);
        uint32_t rnode = node;
        if (RNG_TABLE) {
            tag = a.stream_tag;
            if (node_rng) {
                typedef uint32_t U4 __attribute__((ext_vector_type(4)));
                const U4 v = gload(reinterpret_cast<const U4 *>(node_rng) + node);
                rnode = v.x;
                tag = v.y;
                j = v.z + (uint32_t)jj;
            }
        }
#pragma unroll
        for (int d = 0; d < D; ++d) X[d] = (T)gload(a.nodes + (size_t)node * D + d);
        node = rnode;
        m = inner_distance<T, D>(P, M::domain(P), X);
        Y = (T)1;
        Z = 0.0;
        R = 0.0;
        k = 0;
        capped = 0;
        bb_blk = 0xffffffffu;
        if (M::exit(a) == kExitShift && m <= a.gm_thresh) {
            project<T, D>(P, M::domain(P), X, Xt);
            return false;
        }
        return true;
    }

    // Bridge block of step s for every active lane when some lane needs it
    // and does not hold it (wave-uniform branch).
    __device__ __forceinline__ void bridge_block(const ItemCore<T> &a, uint32_t s, bool need)
    {
        const uint32_t blk = s >> 2;
        if (__ballot(need && blk != bb_blk)) {
            const Block4 q = philox(blk, j, node, stream(a) | 1u, ks);
            bw01 = (uint64_t)q.w0 | ((uint64_t)q.w1 << 32);
            bw23 = (uint64_t)q.w2 | ((uint64_t)q.w3 << 32);
            bb_blk = blk;
        }
    }
    // The bridge uniform of step s: from the block bridge_block has drawn
    // (boundary-dense walks), or drawn here for this lane.
    __device__ __forceinline__ T bridge_uniform(const ItemCore<T> &a, uint32_t s)
    {
        if (!M::dense(a)) {
            const uint32_t blk = s >> 2;
            if (blk != bb_blk) {
                const Block4 q = philox(blk, j, node, stream(a) | 1u, ks);
                bw01 = (uint64_t)q.w0 | ((uint64_t)q.w1 << 32);
                bw23 = (uint64_t)q.w2 | ((uint64_t)q.w3 << 32);
                bb_blk = blk;
            }
        }
        // word s mod 4, picked with a shift (a select chain becomes a stack array)
        const uint32_t w = (uint32_t)(((s & 2) ? bw23 : bw01) >> ((s & 1) << 5));
        return Arith<T>::unif_bridge(w);
    }

    // One step of the walk with the words that feed its normals. Returns
    // false when the path has ended (exit point in Xt). Everything that ends a
    // path (leaving the domain, a live bridge face, the shift band of the next
    // step, the step cap) goes through one rarely taken branch.
    template <class A>
    __device__ __forceinline__ bool step(const A &a, const DevProblem<T> &P, uint32_t wa,
                                         uint32_t wb, uint32_t wc, uint32_t wd)
    {
        T n[D];
        if (M::law(a) == kLawGauss) {
            Arith<T>::box_muller(wa, wb, n[0], n[1]);
            if (D == 3) n[2 % D] = Arith<T>::box_muller_cos(wc, wd);
        } else {
            n[0] = (wa >> 31) ? (T)1 : (T)-1;
            n[1] = (wb >> 31) ? (T)1 : (T)-1;
            if (D == 3) n[2 % D] = (wc >> 31) ? (T)1 : (T)-1;
        }
        T b[D], c, f = (T)0;
        coefficients<T, D>(P, X, b, c, f, EST == kEstIto || a.score_plain != 0, cf, M::tab(P),
                           RNG_TABLE ? nullptr : tr);
        const T hY = a.h * Y;
        if (EST == kEstIto || a.score_plain) Z -= (double)(hY * f);
        if (EST == kEstCorrection) R += (double)(hY * interp_cells<T, D>(a.resid, X));
        if constexpr (EST == kEstIto) {
            // eq. F:xiControlVariate, left-point rule: -Y sigma grad(u~)(X_k)
            // . sqrt(h) N_k, with this step's normals; the gradient grids
            // share one geometry, so the cell is found once, and their cell
            // layouts are interleaved, so its corners of every component are
            // one record (32 bytes in 2D FP32: one L2 request, not two)
            int gi[D];
            T gw[D];
            grid_cell<T, D>(a.grad[0], X, gi, gw);
            const T *rec = a.grad[0].cells + cell_index<T, D>(a.grad[0], gi) * (size_t)(D << D);
            T gn = (T)0;
#pragma unroll
            for (int d = 0; d < D; ++d) gn = madd(interp_corners<T, D>(rec + (d << D), gw), n[d], gn);
            R -= (double)((Y * a.sig_sqh) * gn);
        }
        Y = madd(hY, c, Y);
        T Xn[D];
#pragma unroll
        for (int d = 0; d < D; ++d) Xn[d] = madd(a.sig_sqh, n[d], madd(a.h, b[d], X[d]));
        const uint32_t s = k;
        k = k + 1;

        // distance of the new point to the boundary (negative outside)
        T mn;
        if (M::domain(P) == kBox) {
            mn = Xn[0] - P.lo[0];
            mn = fmin(mn, P.hi[0] - Xn[0]);
#pragma unroll
            for (int d = 1; d < D; ++d) {
                mn = fmin(mn, Xn[d] - P.lo[d]);
                mn = fmin(mn, P.hi[d] - Xn[d]);
            }
        } else {
            T r2n = (T)0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const T t = Xn[d] - P.center[d];
                r2n = madd(t, t, r2n);
            }
            mn = r2n < P.radius2 ? P.radius - Arith<T>::sqrt_(r2n) : (T)-1;
        }
        const bool shift = M::exit(a) == kExitShift;
        // Bridge: a face f is live when a_f a'_f 2/(sigma^2 h) <= 36 ln 2; since
        // a_f >= m and a'_f >= mn, no face is live unless m mn passes that test.
        const bool out = !shift && !(mn > (T)0);
        const bool maybe = M::exit(a) == kExitBridge && m * mn * a.two_over_s2h <= a.bridge_thresh;
        if (M::exit(a) == kExitBridge && M::dense(a)) bridge_block(a, s, maybe);
        const bool next_stop = k == a.max_steps || (shift && mn <= a.gm_thresh);
        if (out || maybe || next_stop) {
            if (out) {  // outside (or on) the boundary: the nearest point is the clamp
                if (M::domain(P) == kBox) {
#pragma unroll
                    for (int d = 0; d < D; ++d) Xt[d] = med3(Xn[d], P.lo[d], P.hi[d]);
                } else {
                    radial<T, D>(P, Xn, Xt);
                }
                return false;
            }
            if (maybe && bridge_exit(a, P, Xn, mn, s)) return false;
            if (shift && mn <= a.gm_thresh) {  // stops before the next step
                project<T, D>(P, M::domain(P), Xn, Xt);
                return false;
            }
            if (k == a.max_steps) {
                capped = 1;
                project<T, D>(P, M::domain(P), Xn, Xt);
                return false;
            }
        }
#pragma unroll
        for (int d = 0; d < D; ++d) X[d] = Xn[d];
        m = mn;
        return true;
    }

    // Brownian-bridge exit between X and Xn (both inside, Xn at distance mn).
    // Per flat face P(cross) = exp(-2 a a' / (sigma^2 h)), faces combined as
    // independent; exit onto the live face with the largest probability.
    __device__ __forceinline__ bool bridge_exit(const ItemCore<T> &a, const DevProblem<T> &P,
                                                const T *Xn, T mn, uint32_t s)
    {
        if (M::domain(P) == kBox && M::dense(a)) {
            // Per axis the face with the smaller argument: unless both faces
            // of the axis are live (a box narrow against the step), it is the
            // only one that can be, so one exponential per axis gives the
            // combined probability and the exit face of the face-by-face rule
            // (live faces combined in face order, the exit face the first of
            // the largest probabilities), with the same operands and
            // roundings. Lanes with both faces of an axis live take every face
            // in turn.
            T alo[D], ahi[D], ad[D];
            bool both = false, live[D], up[D];
            int nlive = 0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                alo[d] = ((X[d] - P.lo[d]) * (Xn[d] - P.lo[d])) * a.two_over_s2h;
                ahi[d] = ((P.hi[d] - X[d]) * (P.hi[d] - Xn[d])) * a.two_over_s2h;
                both = both || (alo[d] <= a.bridge_thresh && ahi[d] <= a.bridge_thresh);
                up[d] = ahi[d] < alo[d];
                ad[d] = up[d] ? ahi[d] : alo[d];
                live[d] = ad[d] <= a.bridge_thresh;
                nlive += live[d] ? 1 : 0;
            }
            // one live axis (the usual case): its face alone
            T amin = ad[0];
            int bestf = up[0] ? 1 : 0;
#pragma unroll
            for (int d = 1; d < D; ++d) {
                amin = live[d] ? ad[d] : amin;
                bestf = live[d] ? 2 * d + (up[d] ? 1 : 0) : bestf;
            }
            T Pe = nlive ? Arith<T>::exp_neg(amin) : (T)0;
            if (nlive > 1) {  // near a corner: the live axes in order
                T bestp = (T)0;
                Pe = (T)0;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const T p = Arith<T>::exp_neg(ad[d]);
                    Pe = live[d] ? madd(p, (T)1 - Pe, Pe) : Pe;
                    const bool better = live[d] && p > bestp;
                    bestp = better ? p : bestp;
                    bestf = better ? 2 * d + (up[d] ? 1 : 0) : bestf;
                }
            }
            if (__builtin_expect(__ballot(both) != 0, 0)) {
                if (both) {  // every live face, in face order
                    Pe = (T)0;
                    T bestp = (T)0;
#pragma unroll
                    for (int q = 0; q < 2 * D; ++q) {
                        const T aq = (q & 1) ? ahi[q >> 1] : alo[q >> 1];
                        const bool live = aq <= a.bridge_thresh;
                        const T p = Arith<T>::exp_neg(aq);
                        Pe = live ? madd(p, (T)1 - Pe, Pe) : Pe;
                        const bool better = live && p > bestp;
                        bestp = better ? p : bestp;
                        bestf = better ? q : bestf;
                    }
                }
            }
            if (bridge_uniform(a, s) < Pe) {
#pragma unroll
                for (int d = 0; d < D; ++d)
                    Xt[d] = (bestf >> 1) == d ? ((bestf & 1) ? P.hi[d] : P.lo[d]) : Xn[d];
                return true;
            }
            return false;
        }
        if (M::domain(P) == kBox) {  // few lanes near a face: per face, one exponential for one live face
            T arg[2 * D];
            T amin = (T)0;
            int fmin = -1, nlive = 0;
#pragma unroll
            for (int q = 0; q < 2 * D; ++q) {
                const int d = q >> 1;
                const T prod = (q & 1) ? (P.hi[d] - X[d]) * (P.hi[d] - Xn[d])
                                       : (X[d] - P.lo[d]) * (Xn[d] - P.lo[d]);
                arg[q] = prod * a.two_over_s2h;
                if (arg[q] <= a.bridge_thresh) {
                    ++nlive;
                    if (fmin < 0 || arg[q] < amin) {
                        amin = arg[q];
                        fmin = q;
                    }
                }
            }
            if (nlive == 0) return false;
            // One live face (the usual case): P is its p and it is the exit
            // face. Several (near a corner): combine them in face order.
            T Pe = Arith<T>::exp_neg(amin);
            int bestf = fmin;
            if (nlive > 1) {
                T bestp = (T)-1;
                Pe = (T)0;
#pragma unroll
                for (int q = 0; q < 2 * D; ++q) {
                    if (arg[q] <= a.bridge_thresh) {
                        const T p = Arith<T>::exp_neg(arg[q]);
                        Pe = madd(p, (T)1 - Pe, Pe);
                        if (p > bestp) {
                            bestp = p;
                            bestf = q;
                        }
                    }
                }
            }
            if (bridge_uniform(a, s) < Pe) {
#pragma unroll
                for (int d = 0; d < D; ++d)
                    Xt[d] = (bestf >> 1) == d ? ((bestf & 1) ? P.hi[d] : P.lo[d]) : Xn[d];
                return true;
            }
            return false;
        }
        const T Pe = Arith<T>::exp_neg(m * mn * a.two_over_s2h);
        if (bridge_uniform(a, s) < Pe) {
            radial<T, D>(P, Xn, Xt);
            return true;
        }
        return false;
    }

    // Score the ended path and write its record at slot - rec_base.
    __device__ __forceinline__ void finish(const ItemCore<T> &a, const DevProblem<T> &P,
                                           uint64_t rec_base)
    {
        score_path<T, D, EST, M>(a, P, Xt, Y, Z, R, k | (capped ? kCappedBit : 0u), slot - rec_base);
    }

    // What scoring the ended path needs, for scoring later from the ring.
    __device__ __forceinline__ void stash(EndedPath<T, D> &e, uint64_t rec_base) const
    {
#pragma unroll
        for (int d = 0; d < D; ++d) e.Xt[d] = Xt[d];
        e.Y = Y;
        e.word = k | (capped ? kCappedBit : 0u);
        e.Z = Z;
        e.R = R;
        e.r = slot - rec_base;
    }
};

// Lanes end paths at any step but take new ones only every few iterations of
// the walk loop (two steps per iteration in 2D, one in 3D; the launch's
// refill_mask, by default every second iteration in 2D and every fourth in
// 3D): every path of a wave then starts at a step count that is the same
// modulo 4 across its lanes, so the bridge uniforms of four consecutive steps
// share one Philox block, which the wave then draws at most once per four
// steps, and the scoring and start of new paths run for several lanes at once.

// Item whose slot range holds group slot s (items are sorted, non-empty
// ranges never overlap). Wave-uniform: a scalar binary search.
template <class T>
__device__ __forceinline__ int find_item(const ItemDesc<T> *__restrict__ items, int n, uint64_t s)
{
    int lo = 0, hi = n;  // items[lo].slot_begin <= s < items[hi].slot_begin
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (items[mid].slot_begin <= s)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Queue of the single-item kernel: a wave takes `grab` slots at a time from
// the launch counter, [next, end) launch-relative, and hands them to its idle
// lanes in order.
struct Pool {
    uint32_t next = 0, end = 0;
    bool exhausted = false;

    __device__ __forceinline__ void refill(const LaunchArgs &L, int lane)
    {
        if (next == end && !exhausted) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(L.counter, (uint32_t)L.grab);
            base = __builtin_amdgcn_readfirstlane(base);
            if (base >= L.launch_slots) {
                exhausted = true;
            } else {
                next = base;
                end = min(base + (uint32_t)L.grab, L.launch_slots);
            }
        }
    }
};

// The single-item kernel scores ended paths from the wave's ring, as the
// batch kernel does, in its dense bridge form (boundary-dense, short walks)
// and its generic form; in the sparse form, for long walks whose lanes seldom
// end at the same turn, each path is scored as it ends (the ring's
// bookkeeping cost the [0,4]^2 launch 2.7 %).
template <class M>
constexpr bool kRingScoreOne = !std::is_same<M, BoxBridgeGaussT<false>>::value;

// Dynamic LDS of a wave of the single-item kernel: the ring of ended paths,
// and in the generic form (the one that walks tabulated problems) the block
// for gathering pair records.
template <class T, int D, class M>
struct OneWaveLds {
    EndRing<T, D> ring;
    Vec4<T> tr[std::is_same<M, RuntimeMode>::value ? 4 * 64 : 1];
};

// One item, passed by value (FP32 2D plain solves). The source polynomial's
// coefficients are staged through LDS once per workgroup: read from there,
// they stay in vector registers for the whole loop (about 96 registers, five
// waves per SIMD) instead of being reloaded by scalar loads at every step,
// which the scalar register file cannot hold next to the other constants.
template <class T, int D, int EST, class M>
__global__ void __launch_bounds__(256) path_kernel_one(const OneItemArgs<T> A)
{
    static_assert(kOneItemKernel<T, D, EST>, "single-item kernel is for FP32 2D plain solves");
    const LaunchArgs &L = A.launch;
    const ItemCore<T> &a = A.item;
    const DevProblem<T> &P = A.prob;
    const int lane = __lane_id();
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    __shared__ T s_cf[kMaxDense];
    extern __shared__ __attribute__((aligned(16))) uint64_t s_one[];  // dynamic: OneWaveLds per wave (ring-scoring forms)
    for (uint32_t i = threadIdx.x; i < (uint32_t)kMaxDense; i += blockDim.x) s_cf[i] = P.fdense[i];
    __syncthreads();
    OneWaveLds<T, D, M> *wl = reinterpret_cast<OneWaveLds<T, D, M> *>(s_one) + (threadIdx.x >> 6);
    EndRing<T, D> *ring = &wl->ring;
    Walker<T, D, EST, M, false> w;
    w.cf = s_cf;
    w.tr = std::is_same<M, RuntimeMode>::value ? wl->tr : nullptr;
    w.ks = key_schedule<KeysOf<T>>(P.key0, P.key1);
    int st = 0;  // 0 idle, 1 walking, 2 ended (to be scored)
    Pool pool;
    uint32_t ring_head = 0, ring_count = 0;

    for (uint32_t iter = 0;; ++iter) {
        if ((iter & L.refill_mask) == 0) {  // refill turn (wave-uniform)
            if constexpr (kRingScoreOne<M>) {
                const uint64_t ended = __ballot(st == 2);
                if (ended) {
                    if (st == 2) {
                        const uint32_t at = (ring_head + ring_count + (uint32_t)__popcll(ended & below)) & (kEndRing - 1);
                        w.stash(ring->e[at], a.rec_base);  // set per launch by the host
                        st = 0;
                    }
                    ring_count += (uint32_t)__popcll(ended);
                }
            } else if (st == 2) {
                w.finish(a, P, a.rec_base);
                st = 0;
            }
            const uint64_t idle = __ballot(st == 0);
            if constexpr (kRingScoreOne<M>) {
                const bool leaving = idle == ~0ull && pool.next == pool.end;  // the wave may stop at this turn
                while (ring_count >= 64u || (leaving && ring_count)) {
                    const uint32_t n = min(ring_count, 64u);
                    if ((uint32_t)lane < n) {
                        const EndedPath<T, D> &e = ring->e[(ring_head + (uint32_t)lane) & (kEndRing - 1)];
                        T Xt[D];
#pragma unroll
                        for (int d = 0; d < D; ++d) Xt[d] = e.Xt[d];
                        score_path<T, D, EST, M>(a, P, Xt, e.Y, e.Z, e.R, e.word, e.r);
                    }
                    ring_head = (ring_head + n) & (kEndRing - 1);
                    ring_count -= n;
                }
            }
            if (idle) {
                pool.refill(L, lane);
                const uint32_t avail = pool.end - pool.next;
                const uint32_t rank = (uint32_t)__popcll(idle & below);
                if (st == 0 && rank < avail) st = w.start(a, P, L.slot_begin + pool.next + rank, nullptr) ? 1 : 2;  // the one item starts at slot 0
                pool.next += min(avail, (uint32_t)__popcll(idle));
            }
            if (__ballot(st != 0) == 0) {
                if (pool.exhausted) break;
                continue;
            }
        }
        if (st == 1) {
            // One Philox block feeds two steps in 2D (words 0,1 then 2,3), one in 3D.
            if (D == 2) {
                const Block4 q = philox(w.k >> 1, w.j, w.node, w.stream(a), w.ks);
                if (!w.step(a, P, q.w0, q.w1, 0u, 0u))
                    st = 2;
                else if (!w.step(a, P, q.w2, q.w3, 0u, 0u))
                    st = 2;
            } else {
                const Block4 q = philox(w.k, w.j, w.node, w.stream(a), w.ks);
                if (!w.step(a, P, q.w0, q.w1, q.w2, q.w3)) st = 2;
            }
        }
    }
}

// Per-item queues of a batch launch. A wave walks the paths of one item at a
// time and may move to another item only once all its lanes are idle, so it
// takes its tickets from its own item's queue for as long as that has slots:
// a single shared queue would hand it the next slots of the whole launch,
// which with many waves lie in another item almost every time and would make
// it wait for its slowest lane at nearly every refill. Waves start spread over
// the items in proportion to their slots; a wave whose item has run dry looks
// for the next item that still has slots (64 candidates per probe).
template <class T>
struct ItemQueue {
    int cur = -1;                     // item of the wave (wave-uniform)
    uint32_t seg_lo = 0, seg_hi = 0;  // its launch-relative slots
    uint32_t next = 0, end = 0;       // the wave's current ticket
    bool dry = true;                  // the current item's queue is used up
    bool done = false;                // every queue of the launch is used up

    // Next ticket of the current item's queue, or dry.
    __device__ __forceinline__ void take(const LaunchArgs &L, int lane)
    {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(L.counter + (cur - L.item_lo), (uint32_t)L.grab);
        base = __builtin_amdgcn_readfirstlane(base);
        if (base < seg_hi - seg_lo) {
            next = seg_lo + base;
            end = min(next + (uint32_t)L.grab, seg_hi);
        } else {
            dry = true;
        }
    }

    // Moves the (idle) wave to an item with slots left, starting with queue k
    // and then probing the ones after it, and takes a ticket there; done when
    // none has slots left. Counters only grow, so every failed attempt means
    // another wave took those slots and the search ends.
    __device__ __forceinline__ void move(const ItemDesc<T> *__restrict__ items, const LaunchArgs &L, int lane,
                                         uint32_t k)
    {
        const uint32_t n = L.n_seg;
        for (;;) {
            cur = __builtin_amdgcn_readfirstlane(L.item_lo + (int)k);
            seg_lo = L.seg[2 * k];
            seg_hi = L.seg[2 * k + 1];
            dry = false;
            take(L, lane);
            if (!dry) return;
            // the probe window nearest after k that has slots left; in it, the
            // item with the most slots left (spreads the waves that move)
            uint32_t found = n;
            for (uint32_t off = 1; off < n && found == n; off += 64) {
                const uint32_t i = off + (uint32_t)lane;
                uint32_t key = 0;  // slots left (capped) << 6 | 63 - lane: the largest wins
                if (i < n) {
                    uint32_t kk = k + i;
                    if (kk >= n) kk -= n;
                    const uint32_t lo = L.seg[2 * kk], hi = L.seg[2 * kk + 1];
                    const uint32_t taken =
                        __hip_atomic_load(L.counter + kk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (taken < hi - lo) key = (min(hi - lo - taken, 0x3ffffffu) << 6) | (uint32_t)(63 - lane);
                }
#pragma unroll
                for (int x = 32; x >= 1; x >>= 1) key = max(key, (uint32_t)__shfl_xor((int)key, x));
                key = __builtin_amdgcn_readfirstlane(key);  // every lane holds the maximum
                if (key) {
                    found = k + off + (63 - (key & 63));
                    if (found >= n) found -= n;
                }
            }
            if (found == n) {
                done = true;
                return;
            }
            k = found;
        }
    }
};

// A batch: items and problems in device tables read at wave-uniform indices.
// Each wave keeps the source coefficients of its current problem in its own
// LDS slot (written when it changes item; a wave's LDS accesses complete in
// order, so no barrier is needed).
// FP64 walks are asked to fit three waves per SIMD (168 registers; the few
// spilled values live outside the step loop), which is faster than two, and
// the FP32 2D box / bridge / Gaussian correction walks five (96 registers:
// one 8-byte value is reloaded at refill turns).
template <class T, int D, int EST, class M>
constexpr int kManyMinWaves = sizeof(T) == 8 ? 3
                              : (D == 2 && EST == kEstCorrection && !std::is_same<M, RuntimeMode>::value) ? 5
                                                                                                          : 1;
template <class T, int D, int EST, class M>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kManyMinWaves<T, D, EST, M>, 8)))
    path_kernel_many(const LaunchArgs L, const ItemDesc<T> *__restrict__ items,
                     const DevProblem<T> *__restrict__ probs)
{
    const int lane = __lane_id();
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    __shared__ T s_cf[256 / 64][kMaxDense];
    extern __shared__ uint64_t s_ring[];  // dynamic: one EndRing per wave
    T *my_cf = s_cf[threadIdx.x >> 6];
    EndRing<T, D> *ring = reinterpret_cast<EndRing<T, D> *>(s_ring) + (threadIdx.x >> 6);
    Walker<T, D, EST, M, true> w;
    w.cf = my_cf;
    w.tr = nullptr;
    int st = 0;
    ItemQueue<T> q;
    // Ended paths are scored 64 at a time, one per lane, from the wave's ring
    // (ring_head, ring_count: wave-uniform): scored as each lane ends, the
    // scoring would run for the whole wave at nearly every refill turn of
    // short walks for the two or three lanes that ended. Every ended path of
    // an item is scored before the wave leaves it.
    uint32_t ring_head = 0, ring_count = 0;

    for (uint32_t iter = 0;; ++iter) {
        if ((iter & L.refill_mask) == 0) {  // refill turn (wave-uniform)
            const uint64_t ended = __ballot(st == 2);
            if (ended) {
                if (st == 2) {
                    const ItemDesc<T> &it = items[q.cur];
                    const uint32_t at = (ring_head + ring_count + (uint32_t)__popcll(ended & below)) & (kEndRing - 1);
                    // scratch records sit at group slot - launch start (modular arithmetic)
                    w.stash(ring->e[at], it.rec_launch ? L.slot_begin - it.slot_begin : it.rec_base);
                    st = 0;
                }
                ring_count += (uint32_t)__popcll(ended);
            }
            const uint64_t idle = __ballot(st == 0);
            const bool leaving = idle == ~0ull && q.next == q.end;  // the wave may move or stop at this turn
            while (ring_count >= 64u || (leaving && ring_count)) {
                const uint32_t n = min(ring_count, 64u);
                if ((uint32_t)lane < n) {
                    const ItemDesc<T> &it = items[q.cur];
                    const EndedPath<T, D> &e = ring->e[(ring_head + (uint32_t)lane) & (kEndRing - 1)];
                    T Xt[D];
#pragma unroll
                    for (int d = 0; d < D; ++d) Xt[d] = e.Xt[d];
                    score_path<T, D, EST, M>(it, probs[it.prob], Xt, e.Y, e.Z, e.R, e.word, e.r);
                }
                ring_head = (ring_head + n) & (kEndRing - 1);
                ring_count -= n;
            }
            if (idle && q.next == q.end && !q.done) {
                if (!q.dry) q.take(L, lane);
                if (q.dry && idle == ~0ull) {
                    const int prev = q.cur;
                    uint32_t k;
                    if (prev < 0) {  // first item: the one holding this wave's share of the launch
                        const uint32_t waves = gridDim.x * (blockDim.x >> 6);
                        const uint32_t gw = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
                        const uint64_t s0 = L.slot_begin + (uint64_t)gw * L.launch_slots / waves;
                        k = (uint32_t)(find_item(items, L.n_items, s0) - L.item_lo);
                        if (k >= L.n_seg) k = 0;
                    } else {
                        k = (uint32_t)(prev - L.item_lo) + 1;
                        if (k >= L.n_seg) k = 0;
                    }
                    q.move(items, L, lane, k);
                    if (!q.done && q.cur != prev) {
                        const ItemDesc<T> &it = items[q.cur];
                        w.ks = key_schedule<KeysOf<T>>(probs[it.prob].key0, probs[it.prob].key1);
                        if (lane < kMaxDense) my_cf[lane] = probs[it.prob].fdense[lane];
                    }
                }
            }
            if (idle && q.next < q.end) {
                const uint32_t avail = q.end - q.next;
                const uint32_t rank = (uint32_t)__popcll(idle & below);
                if (st == 0 && rank < avail) {
                    const ItemDesc<T> &it = items[q.cur];
                    st = w.start(it, probs[it.prob], L.slot_begin + q.next + rank - it.slot_begin, it.node_rng) ? 1 : 2;
                }
                q.next += min(avail, (uint32_t)__popcll(idle));
            }
            if (__ballot(st != 0) == 0) {
                if (q.done) break;
                continue;
            }
        }
        if (st == 1) {
            const ItemDesc<T> &a = items[q.cur];
            const DevProblem<T> &P = probs[a.prob];
            if (D == 2) {
                const Block4 b4 = philox(w.k >> 1, w.j, w.node, w.stream(a), w.ks);
                if (!w.step(a, P, b4.w0, b4.w1, 0u, 0u))
                    st = 2;
                else if (!w.step(a, P, b4.w2, b4.w3, 0u, 0u))
                    st = 2;
            } else {
                const Block4 b4 = philox(w.k, w.j, w.node, w.stream(a), w.ks);
                if (!w.step(a, P, b4.w0, b4.w1, b4.w2, b4.w3)) st = 2;
            }
        }
    }
}

// Residual r = f - ((1/2) sigma^2 Lap u + b.grad u + c u) of a gridded u at
// its points, b, c, f from the problem (FP64), the derivatives of u by
// second-order differences (central inside; three-point one-sided first and
// four-point one-sided second derivatives at the ends of each axis).
template <class S>
__device__ __forceinline__ double fd_first(const S *__restrict__ u, uint64_t p, uint64_t s, int a, int n, double dx)
{
    if (a == 0) return (-3.0 * (double)u[p] + 4.0 * (double)u[p + s] - (double)u[p + 2 * s]) / (2.0 * dx);
    if (a == n - 1) return (3.0 * (double)u[p] - 4.0 * (double)u[p - s] + (double)u[p - 2 * s]) / (2.0 * dx);
    return ((double)u[p + s] - (double)u[p - s]) / (2.0 * dx);
}

template <class S>
__device__ __forceinline__ double fd_second(const S *__restrict__ u, uint64_t p, uint64_t s, int a, int n, double dx)
{
    if (a == 0)
        return (2.0 * (double)u[p] - 5.0 * (double)u[p + s] + 4.0 * (double)u[p + 2 * s] - (double)u[p + 3 * s]) /
               (dx * dx);
    if (a == n - 1)
        return (2.0 * (double)u[p] - 5.0 * (double)u[p - s] + 4.0 * (double)u[p - 2 * s] - (double)u[p - 3 * s]) /
               (dx * dx);
    return ((double)u[p + s] - 2.0 * (double)u[p] + (double)u[p - s]) / (dx * dx);
}

template <class S, int D>
__global__ void __launch_bounds__(256) grid_residual_kernel(const DevProblem<double> P, const S *__restrict__ u,
                                                            int n0, int n1, int n2, double lo0, double lo1,
                                                            double lo2, double dx0, double dx1, double dx2,
                                                            double half_s2, S *__restrict__ r)
{
    __shared__ double s_cf[kMaxDense];
    for (int q = threadIdx.x; q < kMaxDense; q += blockDim.x) s_cf[q] = P.fdense[q];
    __syncthreads();
    const uint64_t m01 = (uint64_t)n0 * n1;
    const uint64_t total = m01 * (D == 3 ? (uint64_t)n2 : 1);
    const int nn[3] = {n0, n1, n2};
    const double lo[3] = {lo0, lo1, lo2}, dx[3] = {dx0, dx1, dx2};
    const uint64_t st[3] = {1, (uint64_t)n0, m01};
    for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < total;
         p += (uint64_t)gridDim.x * blockDim.x) {
        const int idx[3] = {(int)(p % n0), (int)((p / n0) % n1), D == 3 ? (int)(p / m01) : 0};
        double x[D];
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = lo[d] + (double)idx[d] * dx[d];
        double b[D], c, f = 0.0;
        coefficients<double, D>(P, x, b, c, f, true, s_cf, P.tab);
        double lap = 0.0, adv = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lap += fd_second<S>(u, p, st[d], idx[d], nn[d], dx[d]);
            adv += b[d] * fd_first<S>(u, p, st[d], idx[d], nn[d], dx[d]);
        }
        r[p] = (S)(f - (half_s2 * lap + adv + c * (double)u[p]));
    }
}

// Second stage (the subdomain-BVP step of Alg. A:IterPDD) on a 2D box cut by
// axis-parallel interfaces. Grid coordinates are lo + span i / (n - 1), as
// everywhere the grids are sampled.
__device__ __forceinline__ double stage2_coord(double lo, double span, int n, int i)
{
    return lo + span * (double)i / (double)(n - 1);
}

// g at every point of the box's edges.
__global__ void __launch_bounds__(256) stage2_boundary_kernel(const DevProblem<double> P, const Stage2Grid g)
{
    const int n0 = g.n0, n1 = g.n1;
    const int total = 2 * n0 + 2 * (n1 - 2);
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
        int i, j;
        if (q < n0) {
            i = q, j = 0;
        } else if (q < 2 * n0) {
            i = q - n0, j = n1 - 1;
        } else {
            const int r = q - 2 * n0;
            i = (r & 1) ? n0 - 1 : 0;
            j = 1 + (r >> 1);
        }
        const double x[2] = {stage2_coord(g.lo0, g.span0, n0, i), stage2_coord(g.lo1, g.span1, n1, j)};
        g.u[(size_t)j * n0 + i] = boundary_value<double, 2>(P, x, P.tab);
    }
}

__device__ __forceinline__ double multiquadric(const double *t, const double *lam, int m, double eps, double x)
{
    double acc = 0.0;
    for (int q = 0; q < m; ++q) {
        const double e = eps * (x - t[q]);
        acc += lam[q] * sqrt(1.0 + e * e);
    }
    return acc;
}

// One workgroup row per line (blockIdx.y); the points of the line strictly
// between the box's edges.
__global__ void __launch_bounds__(256) stage2_lines_kernel(const Stage2Grid g, const Stage2Line *lines, int32_t n_lines,
                                                           const double *t, const double *lam)
{
    const Stage2Line L = lines[blockIdx.y];
    const int ne = L.d == 0 ? g.n1 : g.n0;  // points along the line
    for (int p = 1 + blockIdx.x * blockDim.x + threadIdx.x; p < ne - 1; p += gridDim.x * blockDim.x) {
        const double tp = L.d == 0 ? stage2_coord(g.lo1, g.span1, g.n1, p) : stage2_coord(g.lo0, g.span0, g.n0, p);
        // a line of the other axis through this point
        int cross = -1;
        for (int q = 0; q < n_lines; ++q)
            if (lines[q].d != L.d && lines[q].k == p) cross = q;
        if (cross >= 0 && L.d == 1) continue;  // the crossing axis-0 line writes the point
        double v = multiquadric(t + L.at, lam + L.at, L.m, L.eps, tp);
        if (cross >= 0) {
            const Stage2Line C = lines[cross];
            const double tc = stage2_coord(g.lo0, g.span0, g.n0, L.k);
            v = 0.5 * (v + multiquadric(t + C.at, lam + C.at, C.m, C.eps, tc));
        }
        const size_t at = L.d == 0 ? (size_t)p * g.n0 + L.k : (size_t)L.k * g.n0 + p;
        g.u[at] = v;
    }
}

// Grid point of unknown r of a subdomain.
__device__ __forceinline__ void stage2_point(const SubBox &b, uint64_t r, int &i, int &j)
{
    const int s = (int)(r / (uint64_t)b.w), f = (int)(r % (uint64_t)b.w);
    if (b.fast_x) {
        i = b.i0 + 1 + f;
        j = b.j0 + 1 + s;
    } else {
        i = b.i0 + 1 + s;
        j = b.j0 + 1 + f;
    }
}

// Stencil of every unknown: (1/2) sigma^2 Lap v + b.grad v + c v = f by
// second-order differences; neighbours on the subdomain's boundary move to
// the right side with their grid values. Slots: 0 slow-1, 1 fast-1,
// 2 centre, 3 fast+1, 4 slow+1, 5 right side; aux: f, and the boundary
// neighbours' part of the right side (the same products, summed from zero).
__global__ void __launch_bounds__(256) stage2_stencil_kernel(const DevProblem<double> P, const Stage2Grid g,
                                                             const SubBox *boxes, double *stencil, double *aux)
{
    __shared__ double s_cf[kMaxDense];
    for (int q = threadIdx.x; q < kMaxDense; q += blockDim.x) s_cf[q] = P.fdense[q];
    __syncthreads();
    const SubBox b = boxes[blockIdx.y];
    const uint64_t n = (uint64_t)b.w * (uint64_t)b.L;
    const double cx = g.half_s2 / (g.dx0 * g.dx0), cy = g.half_s2 / (g.dx1 * g.dx1);
    for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < n; r += (uint64_t)gridDim.x * blockDim.x) {
        int i, j;
        stage2_point(b, r, i, j);
        const double x[2] = {stage2_coord(g.lo0, g.span0, g.n0, i), stage2_coord(g.lo1, g.span1, g.n1, j)};
        double bb[2], c, f = 0.0;
        coefficients<double, 2>(P, x, bb, c, f, true, s_cf, P.tab);
        const double aW = cx - bb[0] / (2.0 * g.dx0), aE = cx + bb[0] / (2.0 * g.dx0);
        const double aS = cy - bb[1] / (2.0 * g.dx1), aN = cy + bb[1] / (2.0 * g.dx1);
        double out[6] = {0.0, 0.0, -2.0 * cx - 2.0 * cy + c, 0.0, 0.0, f};
        double yb = 0.0;
        // neighbours: west, east, south, north with their band slots
        const int ni[4] = {i - 1, i + 1, i, i};
        const int nj[4] = {j, j, j - 1, j + 1};
        const double a[4] = {aW, aE, aS, aN};
        const int slot[4] = {b.fast_x ? 1 : 0, b.fast_x ? 3 : 4, b.fast_x ? 0 : 1, b.fast_x ? 4 : 3};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool inside = ni[q] > b.i0 && ni[q] < b.i1 && nj[q] > b.j0 && nj[q] < b.j1;
            if (inside) {
                out[slot[q]] = a[q];
            } else {
                const double t = a[q] * g.u[(size_t)nj[q] * g.n0 + ni[q]];
                out[5] -= t;
                yb -= t;
            }
        }
        double *o = stencil + (b.first + r) * 6;
#pragma unroll
        for (int q = 0; q < 6; ++q) o[q] = out[q];
        aux[(b.first + r) * 2] = f;
        aux[(b.first + r) * 2 + 1] = yb;
    }
}

// Entry e (column r - w + e) of unknown r's row of a subdomain's band matrix.
__device__ __forceinline__ double stage2_entry(const double *st, int w, int e)
{
    double v = 0.0;
    if (e == 0) v += st[0];
    if (e == w - 1) v += st[1];
    if (e == w) v += st[2];
    if (e == w + 1) v += st[3];
    if (e == 2 * w) v += st[4];
    return v;
}

// A lane's double, read by every lane (wave-uniform result).
__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Banded LU without pivoting (the stencil matrices are diagonally dominant
// once h is small enough for the drift) of one subdomain per workgroup: the
// rows of the active window (the pivot row and the w rows below it) stay in
// LDS in a ring of w + 1 slots; a retired pivot row goes to `factor` (its w + 1
// upper entries; stride kStage2MaxBand + 2, the last slot left for the
// eliminated right side), the multipliers l(k + 1 + t, k) of pivot k to
// lmul[k w + t], and the row w + 1 below it takes its slot. The factors depend
// on the operator, the grid and the subdomains only, not on the data on the
// interfaces, so a context keeps them for the next call with the same ones.
constexpr int kStage2LuThreads = 1024;

__global__ void __launch_bounds__(kStage2LuThreads) stage2_lu_kernel(const SubBox *boxes, const double *stencil,
                                                                     double *factor, double *lmul)
{
    constexpr int MW = kStage2MaxBand;
    constexpr int ROW = 2 * MW + 1;
    constexpr int FS = MW + 2;  // factor stride
    constexpr int CH = 64;      // back-substitution chunk
    __shared__ double A[(MW + 1) * ROW];
    __shared__ double lcol[MW];
    __shared__ double S[CH * 6];  // stencils of the rows that the next CH pivots bring into the window
    const SubBox bx = boxes[blockIdx.x];
    const int w = bx.w, R = w + 1;
    const uint64_t n = (uint64_t)w * (uint64_t)bx.L;
    const double *st = stencil + bx.first * 6;
    double *U = factor + bx.first * FS;
    double *Lm = lmul + bx.first * MW;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < R * (2 * w + 1); idx += blockDim.x) {
        const int rr = idx / (2 * w + 1), e = idx % (2 * w + 1);
        A[rr * ROW + e] = (uint64_t)rr < n ? stage2_entry(st + (size_t)rr * 6, w, e) : 0.0;
    }
    // this thread's (row, column) offsets of the w x w update, the same at
    // every pivot: pair m is update idx = tid + T m (T threads), row offset
    // idx / w and column offset idx % w (no division inside the pivot loop)
    constexpr int T = kStage2LuThreads;
    constexpr int kPairs = MW * MW / T;
    static_assert(MW * MW % T == 0, "whole pairs per thread");
    int prr[kPairs], pcc[kPairs];
#pragma unroll
    for (int m = 0; m < kPairs; ++m) {
        const int idx = tid + T * m;
        prr[m] = idx < w * w ? idx / w : -1;
        pcc[m] = idx < w * w ? idx % w : 0;
    }
    int sk = 0;  // slot of pivot row k: k mod R
    for (uint64_t k = 0; k < n; ++k) {
        __syncthreads();
        if (k % CH == 0) {  // rows k + R .. k + R + CH - 1, entering at pivots k .. k + CH - 1
            for (int idx = tid; idx < CH * 6; idx += blockDim.x) {
                const uint64_t q = (k + R) * 6 + idx;
                S[idx] = q < n * 6 ? st[q] : 0.0;
            }
            __syncthreads();
        }
        if (tid < w) {
            const uint64_t r = k + 1 + tid;
            double l = 0.0;
            if (r < n) {
                int sr = sk + 1 + tid;
                if (sr >= R) sr -= R;
                l = A[sr * ROW + (w - 1 - tid)] / A[sk * ROW + w];  // column k of row r: offset k - r + w
            }
            lcol[tid] = l;
            Lm[k * w + tid] = l;
        }
        __syncthreads();
        const uint64_t left = n - 1 - k;  // unknowns after k: rows and columns k + 1 + o exist for o < left
        // all reads first, then the stores: each pair writes its own entry, and
        // the pivot row and multipliers are not written in this phase
        int at[kPairs];
        double upd[kPairs];
#pragma unroll
        for (int m = 0; m < kPairs; ++m) {
            const int rr = prr[m], cc = pcc[m];
            at[m] = -1;
            if (rr >= 0 && (uint64_t)rr < left && (uint64_t)cc < left) {
                int sr = sk + 1 + rr;
                if (sr >= R) sr -= R;
                at[m] = sr * ROW + (cc - rr + w);
                upd[m] = A[at[m]] - lcol[rr] * A[sk * ROW + (cc + 1 + w)];
            }
        }
#pragma unroll
        for (int m = 0; m < kPairs; ++m)
            if (at[m] >= 0) A[at[m]] = upd[m];
        __syncthreads();
        // retire row k (its columns k .. k + w) and load row k + R into its slot
        const uint64_t nr = k + R;
        const double *sn = S + (k % CH) * 6;  // row nr's stencil
        for (int e = tid; e < 2 * w + 1; e += blockDim.x) {
            if (e >= w) U[k * FS + (e - w)] = A[sk * ROW + e];
            A[sk * ROW + e] = nr < n ? stage2_entry(sn, w, e) : 0.0;
        }
        if (++sk == R) sk = 0;
    }
}

// Forward elimination of the right sides (column 5 of the stencils) with the
// stored multipliers, then back substitution, one subdomain per workgroup,
// both in wave 0 with the pending rows in registers: row r's value lives in
// lane r mod w (n = w L, so the w rows of a window fill the lanes). Forward,
// pivot k: its value y_k (final) is broadcast from lane k mod w, that lane
// takes row k + w, and every lane subtracts l(r, k) y_k from its row r in
// k + 1 .. k + w: the products and differences of eliminating the right side
// alongside the factorization, in its order. y_k goes to the right-side slot
// of factor row k. Back, from k = n - 1 down: x_k = (its value) / u(k, k) is
// broadcast, written to u, its lane takes row k - w's y, and every row j in
// k - w .. k - 1 subtracts u(j, k) x_k. Multipliers, entering right sides and
// U rows are staged through LDS in chunks.
constexpr int kStage2SubstThreads = 256;

// dst[i] = src[i] for i < count (count <= PER x the block's threads): each
// thread issues its PER global loads before any LDS store, so that they are
// in flight together rather than one after another.
template <int PER>
__device__ __forceinline__ void stage_chunk(double *dst, const double *src, int count, int tid)
{
    double t[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int i = tid + u * kStage2SubstThreads;
        t[u] = i < count ? gload(src + i) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int i = tid + u * kStage2SubstThreads;
        if (i < count) dst[i] = t[u];
    }
}

__global__ void __launch_bounds__(kStage2SubstThreads) stage2_subst_kernel(const Stage2Grid g, const SubBox *boxes,
                                                                           const double *stencil, double *factor,
                                                                           const double *lmul)
{
    constexpr int MW = kStage2MaxBand;
    constexpr int FS = MW + 2;  // factor stride
    constexpr int CH = 64;      // pivots (rows) per chunk
    constexpr int PF = 8;       // steps whose operands are read ahead
    __shared__ double Lc[CH * MW];          // forward: multipliers of the chunk's pivots
    __shared__ double Bc[CH];               // forward: right sides entering the window
    __shared__ double Uc[(CH + MW) * FS];   // back: U rows lo - w .. hi - 1
    const SubBox bx = boxes[blockIdx.x];
    const int w = bx.w;
    const uint64_t n = (uint64_t)w * (uint64_t)bx.L;
    const double *st = stencil + bx.first * 6;
    double *U = factor + bx.first * FS;
    const double *Lm = lmul + bx.first * MW;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    double v = tid < 64 && lane < w ? st[(size_t)lane * 6 + 5] : 0.0;  // rows 0 .. w - 1
    int s = 0;  // lane of pivot k: k mod w
    for (uint64_t k0 = 0; k0 < n; k0 += CH) {
        const int m = n - k0 < (uint64_t)CH ? (int)(n - k0) : CH;
        __syncthreads();
        stage_chunk<CH * MW / kStage2SubstThreads>(Lc, Lm + k0 * w, m * w, tid);
        for (int idx = tid; idx < m; idx += blockDim.x) {
            const uint64_t q = k0 + idx + w;  // the row entering the window at pivot k0 + idx
            Bc[idx] = q < n ? st[q * 6 + 5] : 0.0;
        }
        __syncthreads();
        if (tid < 64) {
            double ybuf = 0.0;  // lane i keeps y of pivot k0 + i
            for (int i0 = 0; i0 < m; i0 += PF) {
                // this lane's multipliers and the entering right sides of the
                // next PF pivots, read ahead of the dependent chain
                double lv[PF], bv[PF];
                int su = s;
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    int d = lane - su - 1;  // this lane's row at pivot k0 + i0 + u: k + 1 + d
                    if (d < 0) d += w;
                    const bool ok = i0 + u < m && lane < w && k0 + i0 + u + 1 + d < n;
                    lv[u] = ok ? Lc[(i0 + u) * w + d] : 0.0;
                    bv[u] = i0 + u < m ? Bc[i0 + u] : 0.0;
                    if (++su == w) su = 0;
                }
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    if (i0 + u >= m) break;
                    const double yk = readlane_f64(v, s);
                    ybuf = lane == i0 + u ? yk : ybuf;
                    v = lane == s ? bv[u] : v;
                    const double nv = v - lv[u] * yk;
                    v = lv[u] != 0.0 ? nv : v;  // rows in pivot k's reach (a zero multiplier changes nothing)
                    if (++s == w) s = 0;
                }
            }
            if (lane < m) U[(k0 + lane) * FS + MW + 1] = ybuf;
        }
    }
    // back substitution; rows n - w .. n - 1 fill lanes 0 .. w - 1
    s = w - 1;  // lane of row n - 1
    for (uint64_t hi = n; hi > 0;) {
        const uint64_t lo = hi > CH ? hi - CH : 0;
        const uint64_t base = lo > (uint64_t)w ? lo - w : 0;  // rows base .. hi - 1 staged
        __syncthreads();
        stage_chunk<((CH + MW) * FS + kStage2SubstThreads - 1) / kStage2SubstThreads>(Uc, U + base * FS,
                                                                                      (int)(hi - base) * FS, tid);
        __syncthreads();
        if (tid < 64) {
            if (hi == n) v = lane < w ? Uc[(n - w + lane - base) * FS + MW + 1] : 0.0;
            const int cnt = (int)(hi - lo);
            double xbuf = 0.0;  // lane i keeps x of row hi - 1 - i
            for (int i0 = 0; i0 < cnt; i0 += PF) {
                // rows hi - 1 - i0 - u: the divisor's reciprocal, this lane's
                // entry of the row it updates and the right side entering the
                // window
                double rv[PF], uv[PF], yv[PF];
                int su = s;
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    const uint64_t k = hi - 1 - (uint64_t)(i0 + u);
                    const bool in = i0 + u < cnt;
                    int d = su - 1 - lane;  // this lane's row: k - 1 - d
                    if (d < 0) d += w;
                    rv[u] = 1.0 / (in ? Uc[(k - base) * FS] : 1.0);
                    uv[u] = in && lane < w && k >= (uint64_t)(d + 1) ? Uc[(k - 1 - d - base) * FS + (d + 1)] : 0.0;
                    yv[u] = in && k >= (uint64_t)w ? Uc[(k - w - base) * FS + MW + 1] : 0.0;
                    if (--su < 0) su = w - 1;
                }
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    if (i0 + u >= cnt) break;
                    const double xk = readlane_f64(v, s) * rv[u];
                    xbuf = lane == i0 + u ? xk : xbuf;
                    v = lane == s ? yv[u] : v;
                    const double nv = v - uv[u] * xk;
                    v = uv[u] != 0.0 ? nv : v;
                    if (--s < 0) s = w - 1;
                }
            }
            if (lane < cnt) {
                int i, j;
                stage2_point(bx, hi - 1 - (uint64_t)lane, i, j);
                g.u[(size_t)j * g.n0 + i] = xbuf;
            }
        }
        hi = lo;
    }
}

// Response columns of the subdomains (one workgroup per subdomain and four
// columns, a wave per column): the solution for a unit right side at each
// row next to the box's boundary, and for the source f with zero boundary
// values, by the substitution of stage2_subst_kernel with the stored factors
// (the chunks of multipliers and U rows staged once for the four waves). The
// forward pass leaves y in the column, the backward pass overwrites it with
// the solution.
constexpr int kStage2RespWaves = kStage2SubstThreads / 64;
__global__ void __launch_bounds__(kStage2SubstThreads) stage2_resp_kernel(const SubBox *boxes, const double *aux,
                                                                          const double *factor, const double *lmul,
                                                                          const Stage2Resp *tab, const uint32_t *rb,
                                                                          double *resp)
{
    constexpr int MW = kStage2MaxBand;
    constexpr int FS = MW + 2;
    constexpr int CH = 64;
    constexpr int PF = 8;
    constexpr int NW = kStage2RespWaves;
    __shared__ double Lc[CH * MW];
    __shared__ double Bc[NW][CH];
    __shared__ double Uc[(CH + MW) * FS];
    __shared__ double Yc[NW][CH + MW];
    const SubBox bx = boxes[blockIdx.x];
    const Stage2Resp rt = tab[blockIdx.x];
    const int w = bx.w;
    const uint64_t n = (uint64_t)w * (uint64_t)bx.L;
    const double *U = factor + bx.first * FS;
    const double *Lm = lmul + bx.first * MW;
    const double *fa = aux + bx.first * 2;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int col = (int)blockIdx.y * NW + wv;
    const bool act = col <= rt.nb;
    const bool src = col == rt.nb;  // the source column
    const uint64_t rc = act && !src ? rb[rt.rb_at + col] : ~0ull;
    double *out = resp + rt.out_at + (uint64_t)(act ? col : 0) * n;
    auto rhs = [&](uint64_t q) { return src ? fa[q * 2] : (q == rc ? 1.0 : 0.0); };
    double v = act && lane < w ? rhs((uint64_t)lane) : 0.0;
    int s = 0;
    for (uint64_t k0 = 0; k0 < n; k0 += CH) {
        const int m = n - k0 < (uint64_t)CH ? (int)(n - k0) : CH;
        __syncthreads();
        stage_chunk<CH * MW / kStage2SubstThreads>(Lc, Lm + k0 * w, m * w, tid);
        for (int idx = lane; idx < m; idx += 64) {
            const uint64_t q = k0 + idx + w;
            Bc[wv][idx] = act && q < n ? rhs(q) : 0.0;
        }
        __syncthreads();
        if (act) {
            double ybuf = 0.0;
            for (int i0 = 0; i0 < m; i0 += PF) {
                double lv[PF], bv[PF];
                int su = s;
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    int d = lane - su - 1;
                    if (d < 0) d += w;
                    const bool ok = i0 + u < m && lane < w && k0 + i0 + u + 1 + d < n;
                    lv[u] = ok ? Lc[(i0 + u) * w + d] : 0.0;
                    bv[u] = i0 + u < m ? Bc[wv][i0 + u] : 0.0;
                    if (++su == w) su = 0;
                }
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    if (i0 + u >= m) break;
                    const double yk = readlane_f64(v, s);
                    ybuf = lane == i0 + u ? yk : ybuf;
                    v = lane == s ? bv[u] : v;
                    const double nv = v - lv[u] * yk;
                    v = lv[u] != 0.0 ? nv : v;
                    if (++s == w) s = 0;
                }
            }
            if (lane < m) out[k0 + lane] = ybuf;
        }
    }
    s = w - 1;
    for (uint64_t hi = n; hi > 0;) {
        const uint64_t lo = hi > CH ? hi - CH : 0;
        const uint64_t base = lo > (uint64_t)w ? lo - w : 0;
        __syncthreads();
        stage_chunk<((CH + MW) * FS + kStage2SubstThreads - 1) / kStage2SubstThreads>(Uc, U + base * FS,
                                                                                      (int)(hi - base) * FS, tid);
        for (int idx = lane; idx < (int)(hi - base); idx += 64) Yc[wv][idx] = act ? gload(out + base + idx) : 0.0;
        __syncthreads();
        if (act) {
            if (hi == n) v = lane < w ? Yc[wv][n - w + lane - base] : 0.0;
            const int cnt = (int)(hi - lo);
            double xbuf = 0.0;
            for (int i0 = 0; i0 < cnt; i0 += PF) {
                double rv[PF], uv[PF], yv[PF];
                int su = s;
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    const uint64_t k = hi - 1 - (uint64_t)(i0 + u);
                    const bool in = i0 + u < cnt;
                    int d = su - 1 - lane;
                    if (d < 0) d += w;
                    rv[u] = 1.0 / (in ? Uc[(k - base) * FS] : 1.0);
                    uv[u] = in && lane < w && k >= (uint64_t)(d + 1) ? Uc[(k - 1 - d - base) * FS + (d + 1)] : 0.0;
                    yv[u] = in && k >= (uint64_t)w ? Yc[wv][k - w - base] : 0.0;
                    if (--su < 0) su = w - 1;
                }
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    if (i0 + u >= cnt) break;
                    const double xk = readlane_f64(v, s) * rv[u];
                    xbuf = lane == i0 + u ? xk : xbuf;
                    v = lane == s ? yv[u] : v;
                    const double nv = v - uv[u] * xk;
                    v = uv[u] != 0.0 ? nv : v;
                    if (--s < 0) s = w - 1;
                }
            }
            if (lane < cnt) out[hi - 1 - lane] = xbuf;
        }
        hi = lo;
    }
}

// Interior values from the response columns: u = (f's column) + sum over the
// rows next to the boundary of (that row's column) x (its boundary part of
// the right side), in row order; one thread per unknown.
__global__ void __launch_bounds__(256) stage2_apply_kernel(const Stage2Grid g, const SubBox *boxes, const double *aux,
                                                           const Stage2Resp *tab, const uint32_t *rb,
                                                           const double *resp)
{
    __shared__ double yb[kStage2MaxBoundaryRows];
    const SubBox bx = boxes[blockIdx.y];
    const Stage2Resp rt = tab[blockIdx.y];
    const uint64_t n = (uint64_t)bx.w * (uint64_t)bx.L;
    for (int c = threadIdx.x; c < rt.nb; c += blockDim.x) yb[c] = aux[(bx.first + rb[rt.rb_at + c]) * 2 + 1];
    __syncthreads();
    for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < n; r += (uint64_t)gridDim.x * blockDim.x) {
        const double *col = resp + rt.out_at + r;
        double acc = col[(uint64_t)rt.nb * n];
        for (int c = 0; c < rt.nb; ++c) acc = fma(col[(uint64_t)c * n], yb[c], acc);
        int i, j;
        stage2_point(bx, r, i, j);
        g.u[(size_t)j * g.n0 + i] = acc;
    }
}

}  // namespace

hipError_t launch_grid_residual(const DevProblem<double> &P, double sigma, const pdd_grid *g, void *r, hipStream_t s)
{
    const int D = g->dim;
    const int n2 = D == 3 ? g->n[2] : 1;
    const uint64_t total = (uint64_t)g->n[0] * g->n[1] * n2;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((total + 255) / 256, 16384);
    double dx[3] = {0, 0, 0};
    for (int d = 0; d < D; ++d) dx[d] = (g->hi[d] - g->lo[d]) / (g->n[d] - 1);
    const double h2 = 0.5 * sigma * sigma;
    if (g->dtype == PDD_DTYPE_F32) {
        const float *u = static_cast<const float *>(g->data);
        float *out = static_cast<float *>(r);
        if (D == 2)
            hipLaunchKernelGGL((grid_residual_kernel<float, 2>), dim3(blocks), dim3(256), 0, s, P, u, g->n[0], g->n[1],
                               n2, g->lo[0], g->lo[1], 0.0, dx[0], dx[1], 0.0, h2, out);
        else
            hipLaunchKernelGGL((grid_residual_kernel<float, 3>), dim3(blocks), dim3(256), 0, s, P, u, g->n[0], g->n[1],
                               n2, g->lo[0], g->lo[1], g->lo[2], dx[0], dx[1], dx[2], h2, out);
    } else {
        const double *u = static_cast<const double *>(g->data);
        double *out = static_cast<double *>(r);
        if (D == 2)
            hipLaunchKernelGGL((grid_residual_kernel<double, 2>), dim3(blocks), dim3(256), 0, s, P, u, g->n[0],
                               g->n[1], n2, g->lo[0], g->lo[1], 0.0, dx[0], dx[1], 0.0, h2, out);
        else
            hipLaunchKernelGGL((grid_residual_kernel<double, 3>), dim3(blocks), dim3(256), 0, s, P, u, g->n[0],
                               g->n[1], n2, g->lo[0], g->lo[1], g->lo[2], dx[0], dx[1], dx[2], h2, out);
    }
    return hipGetLastError();
}

hipError_t launch_stage2_boundary(const DevProblem<double> &P, const Stage2Grid &g, hipStream_t s)
{
    const int total = 2 * g.n0 + 2 * (g.n1 - 2);
    hipLaunchKernelGGL(stage2_boundary_kernel, dim3((total + 255) / 256), dim3(256), 0, s, P, g);
    return hipGetLastError();
}

hipError_t launch_stage2_lines(const Stage2Grid &g, const Stage2Line *lines, int32_t n_lines, const double *t,
                               const double *lam, hipStream_t s)
{
    if (n_lines == 0) return hipSuccess;
    const int len = g.n0 > g.n1 ? g.n0 : g.n1;
    hipLaunchKernelGGL(stage2_lines_kernel, dim3((len + 255) / 256, n_lines), dim3(256), 0, s, g, lines, n_lines, t,
                       lam);
    return hipGetLastError();
}

hipError_t launch_stage2_solve(const DevProblem<double> &P, const Stage2Grid &g, const SubBox *boxes,
                               int32_t n_boxes, uint32_t max_unknowns, double *stencil, double *aux, double *factor,
                               double *lmul, const Stage2Plan &plan, hipStream_t s)
{
    if (n_boxes == 0) return hipSuccess;
    hipLaunchKernelGGL(stage2_stencil_kernel, dim3((max_unknowns + 255) / 256, n_boxes), dim3(256), 0, s, P, g,
                       boxes, stencil, aux);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!plan.factored) {
        hipLaunchKernelGGL(stage2_lu_kernel, dim3(n_boxes), dim3(kStage2LuThreads), 0, s, boxes, stencil, factor,
                           lmul);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!plan.resp) {
        hipLaunchKernelGGL(stage2_subst_kernel, dim3(n_boxes), dim3(kStage2SubstThreads), 0, s, g, boxes, stencil,
                           factor, lmul);
        return hipGetLastError();
    }
    if (!plan.resp_ready) {
        const uint32_t groups = (uint32_t)(plan.max_cols + kStage2RespWaves - 1) / kStage2RespWaves;
        hipLaunchKernelGGL(stage2_resp_kernel, dim3(n_boxes, groups), dim3(kStage2SubstThreads), 0, s, boxes, aux,
                           factor, lmul, plan.resp_tab, plan.rb, plan.resp);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((max_unknowns + 255) / 256, 1024);
    hipLaunchKernelGGL(stage2_apply_kernel, dim3(blocks, n_boxes), dim3(256), 0, s, g, boxes, aux, plan.resp_tab,
                       plan.rb, plan.resp);
    return hipGetLastError();
}

template <class T, int D, int EST>
hipError_t launch_path_kernel(const LaunchArgs &l, const ItemDesc<T> *items,
                              const DevProblem<T> *probs, int grid, int block, int kind, hipStream_t s)
{
    const size_t lds = (size_t)(block / 64) * sizeof(EndRing<T, D>);
    if (kind == kKernelDense)
        hipLaunchKernelGGL((path_kernel_many<T, D, EST, BoxBridgeGaussDense>), dim3(grid), dim3(block), lds, s, l,
                           items, probs);
    else if (kind == kKernelSparse)
        hipLaunchKernelGGL((path_kernel_many<T, D, EST, BoxBridgeGauss>), dim3(grid), dim3(block), lds, s, l,
                           items, probs);
    else
        hipLaunchKernelGGL((path_kernel_many<T, D, EST, RuntimeMode>), dim3(grid), dim3(block), lds, s, l, items,
                           probs);
    return hipGetLastError();
}

template <class T, int D, int EST>
hipError_t launch_path_kernel_one(const OneItemArgs<T> &a, int grid, int block, int kind, hipStream_t s)
{
    if constexpr (kOneItemKernel<T, D, EST>) {
        static_assert(sizeof(OneItemArgs<T>) <= 4096, "kernel arguments exceed 4 KiB");
        const size_t waves = (size_t)(block / 64);
        if (kind == kKernelDense)
            hipLaunchKernelGGL((path_kernel_one<T, D, EST, BoxBridgeGaussDense>), dim3(grid), dim3(block),
                               waves * sizeof(OneWaveLds<T, D, BoxBridgeGaussDense>), s, a);
        else if (kind == kKernelSparse)
            hipLaunchKernelGGL((path_kernel_one<T, D, EST, BoxBridgeGauss>), dim3(grid), dim3(block), 0, s, a);
        else
            hipLaunchKernelGGL((path_kernel_one<T, D, EST, RuntimeMode>), dim3(grid), dim3(block),
                               waves * sizeof(OneWaveLds<T, D, RuntimeMode>), s, a);
        return hipGetLastError();
    } else {
        return hipErrorInvalidDeviceFunction;
    }
}

template <class T, int D, int EST>
const void *path_kernel_symbol(bool one, int kind)
{
    if constexpr (kOneItemKernel<T, D, EST>)
        if (one)
            return kind == kKernelDense    ? reinterpret_cast<const void *>(&path_kernel_one<T, D, EST, BoxBridgeGaussDense>)
                   : kind == kKernelSparse ? reinterpret_cast<const void *>(&path_kernel_one<T, D, EST, BoxBridgeGauss>)
                                           : reinterpret_cast<const void *>(&path_kernel_one<T, D, EST, RuntimeMode>);
    return kind == kKernelDense    ? reinterpret_cast<const void *>(&path_kernel_many<T, D, EST, BoxBridgeGaussDense>)
           : kind == kKernelSparse ? reinterpret_cast<const void *>(&path_kernel_many<T, D, EST, BoxBridgeGauss>)
                                   : reinterpret_cast<const void *>(&path_kernel_many<T, D, EST, RuntimeMode>);
}

template <class S, class T, int D>
hipError_t launch_grid_cells_strided(const S *data, const int32_t *n, T *cells, uint32_t stride, uint32_t off,
                                     hipStream_t s)
{
    const uint64_t n_cells = cell_values<T>(n, D) >> D;
    if (n_cells == 0) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((n_cells + 255) / 256, 4096);
    hipLaunchKernelGGL((grid_cells_kernel<S, T, D>), dim3((uint32_t)blocks), dim3(256), 0, s, data, n[0], n[1],
                       D == 3 ? n[2] : 2, cells, stride, off);
    return hipGetLastError();
}

template <class S, class T, int D>
hipError_t launch_grid_cells(const S *data, const int32_t *n, T *cells, hipStream_t s)
{
    return launch_grid_cells_strided<S, T, D>(data, n, cells, 1u << D, 0u, s);
}

template <class S, class T>
hipError_t launch_grid_points_strided(const S *data, uint64_t n_points, T *out, uint32_t stride, uint32_t off,
                                      hipStream_t s)
{
    if (n_points == 0) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((n_points + 255) / 256, 4096);
    hipLaunchKernelGGL((grid_points_kernel<S, T>), dim3((uint32_t)blocks), dim3(256), 0, s, data, n_points, out,
                       stride, off);
    return hipGetLastError();
}
template hipError_t launch_grid_points_strided<float, float>(const float *, uint64_t, float *, uint32_t, uint32_t,
                                                             hipStream_t);
template hipError_t launch_grid_points_strided<float, double>(const float *, uint64_t, double *, uint32_t,
                                                              uint32_t, hipStream_t);
template hipError_t launch_grid_points_strided<double, float>(const double *, uint64_t, float *, uint32_t,
                                                              uint32_t, hipStream_t);
template hipError_t launch_grid_points_strided<double, double>(const double *, uint64_t, double *, uint32_t,
                                                               uint32_t, hipStream_t);

#define PDD_GRID_CELLS(S, T, D) \
    template hipError_t launch_grid_cells<S, T, D>(const S *, const int32_t *, T *, hipStream_t); \
    template hipError_t launch_grid_cells_strided<S, T, D>(const S *, const int32_t *, T *, uint32_t, uint32_t, \
                                                            hipStream_t);
PDD_GRID_CELLS(float, float, 2)
PDD_GRID_CELLS(float, float, 3)
PDD_GRID_CELLS(double, double, 2)
PDD_GRID_CELLS(double, double, 3)
PDD_GRID_CELLS(float, double, 2)
PDD_GRID_CELLS(float, double, 3)
PDD_GRID_CELLS(double, float, 2)
PDD_GRID_CELLS(double, float, 3)

#define PDD_INSTANTIATE(T, D, EST)                                                              \
    template hipError_t launch_path_kernel<T, D, EST>(const LaunchArgs &, const ItemDesc<T> *, \
                                                     const DevProblem<T> *, int, int, int, hipStream_t); \
    template hipError_t launch_path_kernel_one<T, D, EST>(const OneItemArgs<T> &, int, int, int, hipStream_t); \
    template const void *path_kernel_symbol<T, D, EST>(bool, int);

PDD_INSTANTIATE(float, 2, kEstPlain)
PDD_INSTANTIATE(float, 2, kEstCorrection)
PDD_INSTANTIATE(float, 2, kEstIto)
PDD_INSTANTIATE(float, 3, kEstPlain)
PDD_INSTANTIATE(float, 3, kEstCorrection)
PDD_INSTANTIATE(float, 3, kEstIto)
PDD_INSTANTIATE(double, 2, kEstPlain)
PDD_INSTANTIATE(double, 2, kEstCorrection)
PDD_INSTANTIATE(double, 2, kEstIto)
PDD_INSTANTIATE(double, 3, kEstPlain)
PDD_INSTANTIATE(double, 3, kEstCorrection)
PDD_INSTANTIATE(double, 3, kEstIto)

}  // namespace pdd
