// Host runtime of the first-stage PDD nodal solver: the C ABI of pdd.h.
//
// A solve turns its nodes and path counts into a path space of slots (node
// after node, path after path), cuts it into launches that fit the record
// scratch, and per launch runs the persistent path kernel and the per-node
// reduction; a finalize kernel turns the node accumulators into statistics.
// Everything is enqueued on the caller's stream; host inputs travel through a
// pinned staging buffer owned by the context.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "pdd.h"
#include "host_runtime.hpp"

using namespace pdd;

namespace pdd {

thread_local std::string g_error;

pdd_status fail(pdd_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

}  // namespace pdd

namespace {

pdd_status ensure(pdd_ctx *ctx, DeviceBuffer &b, size_t bytes)
{
    if (bytes <= b.cap) return PDD_OK;
    // the previous solve may still read the old buffer
    if (ctx->any_done) HIP_TRY(hipEventSynchronize(ctx->done));
    if (b.ptr) HIP_TRY(hipFree(b.ptr));
    b.ptr = nullptr;
    b.cap = 0;
    size_t want = std::max<size_t>(bytes, 4096);
    if (hipMalloc(&b.ptr, want) != hipSuccess) {
        b.ptr = nullptr;
        return fail(PDD_E_NOMEM, "hipMalloc of %zu bytes failed", want);
    }
    b.cap = want;
    return PDD_OK;
}

pdd_status ensure_stage(pdd_ctx *ctx, size_t bytes)
{
    if (ctx->any_staged) HIP_TRY(hipEventSynchronize(ctx->staged));
    if (bytes <= ctx->stage_cap) return PDD_OK;
    if (ctx->stage) HIP_TRY(hipHostFree(ctx->stage));
    ctx->stage = nullptr;
    ctx->stage_cap = 0;
    size_t want = std::max<size_t>(bytes, 1 << 16);
    if (hipHostMalloc(&ctx->stage, want, hipHostMallocDefault) != hipSuccess) {
        ctx->stage = nullptr;
        return fail(PDD_E_NOMEM, "pinned allocation of %zu bytes failed", want);
    }
    ctx->stage_cap = want;
    return PDD_OK;
}

// Monomials keyed by packed exponents (e0 | e1 << 8 | e2 << 16).
using PolyMap = std::map<uint32_t, double>;

uint32_t pack_exp(const int e[3]) { return (uint32_t)e[0] | ((uint32_t)e[1] << 8) | ((uint32_t)e[2] << 16); }

void poly_add(PolyMap &p, const int e[3], double coef)
{
    if (coef != 0.0) p[pack_exp(e)] += coef;
}

// F = (1/2) sigma^2 Lap P + b.grad P + c P + fx for P = sum of the monomials,
// b = b0 + B x, c = c_a + c_b |x|^2, expanded into monomials.
PolyMap expand_source(const pdd_problem_desc &d)
{
    PolyMap F;
    const double hs2 = 0.5 * d.sigma * d.sigma;
    for (int m = 0; m < d.n_mono; ++m) {
        const pdd_mono_term &q = d.mono[m];
        int e[3] = {q.e[0], q.e[1], q.e[2]};
        for (int i = 0; i < d.dim; ++i) {
            if (e[i] >= 2) {  // (1/2) sigma^2 d_ii
                int t[3] = {e[0], e[1], e[2]};
                t[i] -= 2;
                poly_add(F, t, hs2 * q.coef * e[i] * (e[i] - 1));
            }
            if (e[i] >= 1) {  // b_i d_i = (b0_i + sum_j B_ij x_j) d_i
                int t[3] = {e[0], e[1], e[2]};
                t[i] -= 1;
                const double g = q.coef * e[i];
                poly_add(F, t, d.b0[i] * g);
                for (int j = 0; j < d.dim; ++j) {
                    int u[3] = {t[0], t[1], t[2]};
                    u[j] += 1;
                    poly_add(F, u, d.B[i][j] * g);
                }
            }
        }
        poly_add(F, e, d.c_a * q.coef);  // c P
        for (int j = 0; j < d.dim; ++j) {
            int u[3] = {e[0], e[1], e[2]};
            u[j] += 2;
            poly_add(F, u, d.c_b * q.coef);
        }
    }
    for (int m = 0; m < d.n_fx; ++m) poly_add(F, d.fx[m].e, d.fx[m].coef);
    return F;
}

PolyMap expand_boundary(const pdd_problem_desc &d)
{
    PolyMap G;
    for (int m = 0; m < d.n_mono; ++m) poly_add(G, d.mono[m].e, d.mono[m].coef);
    for (int m = 0; m < d.n_gx; ++m) poly_add(G, d.gx[m].e, d.gx[m].coef);
    return G;
}

template <class T>
int fill_poly(const PolyMap &src, DevPoly<T> *dst, int cap)
{
    int n = 0;
    for (const auto &kv : src) {
        if (kv.second == 0.0) continue;
        if (n == cap) return -1;
        dst[n].coef = (T)kv.second;
        dst[n].e = kv.first;
        ++n;
    }
    return n;
}

// Dense Horner table of F when every monomial fits (2D: total degree <= 5,
// 3D: <= 4), in the order the kernel reads it (3D: k, then j, then i).
template <class T>
bool fill_dense(const PolyMap &F, int dim, T *c)
{
    const int deg = dim == 2 ? kDenseDeg2 : kDenseDeg3;
    for (int q = 0; q < kMaxDense; ++q) c[q] = (T)0;
    for (const auto &kv : F) {
        const int e0 = kv.first & 0xff, e1 = (kv.first >> 8) & 0xff, e2 = (kv.first >> 16) & 0xff;
        if (e0 + e1 + e2 > deg) return false;
    }
    int off = 0;
    for (int k = 0; k <= (dim == 3 ? deg : 0); ++k)
        for (int j = 0; j <= deg - k; ++j)
            for (int i = 0; i <= deg - j - k; ++i, ++off) {
                const int e[3] = {i, j, k};
                auto it = F.find(pack_exp(e));
                if (it != F.end()) c[off] = (T)it->second;
            }
    return true;
}

template <class T>
pdd_status fill_problem(const pdd_problem_desc &d, DevProblem<T> &p, bool revolutions)
{
    std::memset(&p, 0, sizeof p);
    p.dim = d.dim;
    p.domain = d.domain;
    p.n_trig = d.n_trig;
    p.key0 = (uint32_t)(d.seed & 0xffffffffu);
    p.key1 = (uint32_t)(d.seed >> 32);
    for (int i = 0; i < 3; ++i) {
        p.lo[i] = (T)d.lo[i];
        p.hi[i] = (T)d.hi[i];
        p.center[i] = (T)d.center[i];
        p.b0[i] = (T)d.b0[i];
        for (int j = 0; j < 3; ++j) p.B[i][j] = (T)d.B[i][j];
    }
    p.radius = (T)d.radius;
    p.radius2 = (T)(d.radius * d.radius);
    p.c_a = (T)d.c_a;
    p.c_b = (T)d.c_b;
    const double inv2pi = 0.15915494309189533577;
    const double hs2 = 0.5 * d.sigma * d.sigma;
    for (int m = 0; m < d.n_trig; ++m) {
        const pdd_trig_term &t = d.trig[m];
        DevTrig<T> &q = p.trig[m];
        double ksq = 0.0;
        for (int k = 0; k < d.dim; ++k) ksq += t.k[k] * t.k[k];
        q.amp = (T)t.amp;
        q.nhk2a = (T)(-hs2 * ksq * t.amp);
        for (int k = 0; k < 3; ++k) {
            q.k[k] = (T)(revolutions ? t.k[k] * inv2pi : t.k[k]);
            q.ph[k] = (T)(revolutions ? t.phase[k] * inv2pi : t.phase[k]);
            q.ak[k] = (T)(t.amp * t.k[k]);
        }
    }
    const PolyMap F = expand_source(d);
    const int nf = fill_poly(F, p.fpoly, kMaxF);
    const int ng = fill_poly(expand_boundary(d), p.gpoly, kMaxG);
    if (nf < 0 || ng < 0)
        return fail(PDD_E_UNSUPPORTED, "polynomial part too large: f needs <= %d and g <= %d monomials",
                    kMaxF, kMaxG);
    p.n_f = nf;
    p.n_g = ng;
    p.f_mode = nf == 0 ? kPolyNone : (fill_dense(F, d.dim, p.fdense) ? kPolyDense : kPolySparse);
    return PDD_OK;
}

bool finite3(const double *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

pdd_status check_desc(const pdd_problem_desc *d)
{
    if (!d) return fail(PDD_E_INVALID, "desc is NULL");
    if (d->dim != 2 && d->dim != 3) return fail(PDD_E_INVALID, "dim must be 2 or 3 (got %d)", d->dim);
    if (d->domain == PDD_DOMAIN_BOX) {
        for (int i = 0; i < d->dim; ++i)
            if (!(d->lo[i] < d->hi[i]) || !std::isfinite(d->lo[i]) || !std::isfinite(d->hi[i]))
                return fail(PDD_E_INVALID, "box needs finite lo < hi on axis %d", i);
    } else if (d->domain == PDD_DOMAIN_BALL) {
        if (!(d->radius > 0.0) || !std::isfinite(d->radius) || !finite3(d->center, d->dim))
            return fail(PDD_E_INVALID, "ball needs a finite center and radius > 0");
    } else {
        return fail(PDD_E_INVALID, "unknown domain %d", d->domain);
    }
    if (!(d->sigma > 0.0) || !std::isfinite(d->sigma)) return fail(PDD_E_INVALID, "sigma must be > 0");
    if (d->n_trig < 0 || d->n_trig > PDD_MAX_TRIG || d->n_mono < 0 || d->n_mono > PDD_MAX_MONO ||
        d->n_fx < 0 || d->n_fx > PDD_MAX_MONO || d->n_gx < 0 || d->n_gx > PDD_MAX_MONO)
        return fail(PDD_E_INVALID, "term counts out of range");
    auto mono_ok = [&](const pdd_mono_term *m, int n) {
        for (int q = 0; q < n; ++q) {
            if (!std::isfinite(m[q].coef)) return false;
            for (int k = 0; k < 3; ++k)
                if (m[q].e[k] < 0 || m[q].e[k] > 8 || (k >= d->dim && m[q].e[k] != 0)) return false;
        }
        return true;
    };
    if (!mono_ok(d->mono, d->n_mono) || !mono_ok(d->fx, d->n_fx) || !mono_ok(d->gx, d->n_gx))
        return fail(PDD_E_INVALID, "monomial exponents must be 0..8 (and 0 beyond dim)");
    for (int q = 0; q < d->n_trig; ++q)
        if (!std::isfinite(d->trig[q].amp) || !finite3(d->trig[q].k, d->dim) ||
            !finite3(d->trig[q].phase, d->dim))
            return fail(PDD_E_INVALID, "trig term %d is not finite", q);
    if (!finite3(d->b0, d->dim) || !std::isfinite(d->c_a) || !std::isfinite(d->c_b))
        return fail(PDD_E_INVALID, "drift / killing coefficients must be finite");
    for (int i = 0; i < d->dim; ++i)
        if (!finite3(d->B[i], d->dim)) return fail(PDD_E_INVALID, "drift matrix must be finite");
    return PDD_OK;
}

// Largest |k_d x_d + phase_d| / (2 pi) of the trig terms over the bounding
// box of the domain (a corner maximises |k_d x_d|).
double trig_revolutions(const pdd_problem_desc &d)
{
    double mx = 0.0;
    for (int m = 0; m < d.n_trig; ++m)
        for (int i = 0; i < d.dim; ++i) {
            const double lo = d.domain == PDD_DOMAIN_BOX ? d.lo[i] : d.center[i] - d.radius;
            const double hi = d.domain == PDD_DOMAIN_BOX ? d.hi[i] : d.center[i] + d.radius;
            const double k = d.trig[m].k[i], ph = d.trig[m].phase[i];
            mx = std::max(mx, std::max(std::fabs(k * lo + ph), std::fabs(k * hi + ph)));
        }
    return mx * 0.15915494309189533577;
}

bool strictly_inside(const pdd_problem_desc &d, const double *x)
{
    if (d.domain == PDD_DOMAIN_BOX) {
        for (int i = 0; i < d.dim; ++i)
            if (!(x[i] > d.lo[i] && x[i] < d.hi[i])) return false;
        return true;
    }
    double r2 = 0.0;
    for (int i = 0; i < d.dim; ++i) {
        const double t = x[i] - d.center[i];
        r2 += t * t;
    }
    return r2 < d.radius * d.radius;
}

pdd_status check_grid(const pdd_problem_desc &d, const pdd_grid *g, int precision, const char *name)
{
    if (!g) return fail(PDD_E_INVALID, "%s grid is NULL", name);
    if (g->dim != d.dim) return fail(PDD_E_INVALID, "%s grid dim %d != problem dim %d", name, g->dim, d.dim);
    if (!g->data) return fail(PDD_E_INVALID, "%s grid has no data", name);
    if (precision < 0) {  // any supported dtype (converted by the library)
        if (g->dtype != PDD_DTYPE_F32 && g->dtype != PDD_DTYPE_F64)
            return fail(PDD_E_INVALID, "%s grid has an unknown dtype %d", name, g->dtype);
    } else {
        const int want = precision == PDD_FP64 ? PDD_DTYPE_F64 : PDD_DTYPE_F32;
        if (g->dtype != want)
            return fail(PDD_E_UNSUPPORTED, "%s grid dtype must match the path precision (%s)", name,
                        precision == PDD_FP64 ? "f64" : "f32");
    }
    for (int i = 0; i < d.dim; ++i) {
        if (g->n[i] < 2) return fail(PDD_E_INVALID, "%s grid needs >= 2 points per axis", name);
        if (!(g->lo[i] < g->hi[i])) return fail(PDD_E_INVALID, "%s grid needs lo < hi", name);
        const double blo = d.domain == PDD_DOMAIN_BOX ? d.lo[i] : d.center[i] - d.radius;
        const double bhi = d.domain == PDD_DOMAIN_BOX ? d.hi[i] : d.center[i] + d.radius;
        if (g->lo[i] > blo || g->hi[i] < bhi)
            return fail(PDD_E_INVALID, "%s grid does not cover the domain on axis %d", name, i);
    }
    return PDD_OK;
}

template <class T>
GridView<T> make_view(const pdd_grid *g, int dim)
{
    GridView<T> v{};
    if (!g) return v;
    v.data = static_cast<const T *>(g->data);
    for (int i = 0; i < 3; ++i) {
        v.n[i] = i < dim ? g->n[i] : 1;
        v.lo[i] = (T)g->lo[i];
        v.inv[i] = i < dim ? (T)((double)(g->n[i] - 1) / (g->hi[i] - g->lo[i])) : (T)0;
        v.top[i] = (T)(v.n[i] - 1);
    }
    return v;
}

}  // namespace

int pdd::occupancy(pdd_ctx *ctx, const void *fn, int block, bool cache)
{
    auto key = std::make_tuple(fn, block);
    auto it = ctx->occupancy.find(key);
    if (it != ctx->occupancy.end()) return it->second;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, block, 0) != hipSuccess || n < 1) n = 1;
    if (cache) ctx->occupancy[key] = n;
    return n;
}

// Largest FP32 cell-record layout of a 2D tabulated problem (about half an
// XCD's L2); larger grids are interleaved by pairs of points.
constexpr size_t kCellRecordMaxBytes = 8u << 20;

uint64_t next_problem_serial()
{
    static std::atomic<uint64_t> next{1};
    return next.fetch_add(1);
}

bool pdd::specialised(const HostItem &it)
{
    return it.prob->desc.domain == PDD_DOMAIN_BOX && it.o->exit_mode == PDD_EXIT_BRIDGE &&
           it.o->law == PDD_LAW_GAUSS && it.prob->pf.tab == 0;
}

// A face can be live within about 3.5 sigma sqrt(dt) of it (2 a a' / (sigma^2
// dt) <= 36 ln 2), so the share of lanes in such a band is about 7 sigma
// sqrt(dt) / width per axis. Above 15 % nearly every lane of a wave meets a
// live face within a few steps and the dense form wins (the unit square at dt
// = 1e-3: 0.89, 15 % faster); the [0, 4]^2 box at dt = 1e-4 (0.035) keeps the
// per-lane form, 1.5 % faster there.
bool pdd::dense_boundary(const pdd_problem_desc &d, double dt)
{
    const double band = 7.0 * d.sigma * std::sqrt(dt);
    double share = 0.0;
    for (int i = 0; i < d.dim; ++i)
        share += band / (d.domain == PDD_DOMAIN_BOX ? d.hi[i] - d.lo[i] : 2.0 * d.radius);
    return share > 0.15;
}

pdd_status pdd::validate_item(HostItem &it)
{
    const pdd_solve_opts *o = it.o;
    if (!it.prob) return fail(PDD_E_INVALID, "problem is NULL");
    if (!o) return fail(PDD_E_INVALID, "opts is NULL");
    if (it.n_nodes < 0) return fail(PDD_E_INVALID, "n_nodes < 0");
    if (it.n_nodes >= (1ll << 32)) return fail(PDD_E_INVALID, "too many nodes");
    if (it.n_nodes > 0 && !it.nodes) return fail(PDD_E_INVALID, "nodes is NULL");
    if (it.n_nodes > 0 && !it.out) return fail(PDD_E_INVALID, "out is NULL");
    const pdd_problem_desc &d = it.prob->desc;
    const int dim = d.dim;
    const bool cv = it.u_prev || it.resid;
    if (cv && (!it.u_prev || !it.resid)) return fail(PDD_E_INVALID, "correction needs u_prev and residual grids");
    if (cv && it.grad) return fail(PDD_E_INVALID, "an item takes the correction grids or the gradient grids, not both");
    it.est = cv ? kEstCorrection : (it.grad ? kEstIto : kEstPlain);
    if (!(o->dt > 0.0) || !std::isfinite(o->dt)) return fail(PDD_E_INVALID, "dt must be > 0");
    if (o->precision != PDD_FP32 && o->precision != PDD_FP64) return fail(PDD_E_INVALID, "bad precision");
    if (o->exit_mode < PDD_EXIT_BRIDGE || o->exit_mode > PDD_EXIT_NAIVE) return fail(PDD_E_INVALID, "bad exit mode");
    if (o->law != PDD_LAW_GAUSS && o->law != PDD_LAW_RADEMACHER) return fail(PDD_E_INVALID, "bad law");
    if (o->stream_id >= (1u << 28)) return fail(PDD_E_INVALID, "stream_id must be < 2^28");
    if (o->precision == PDD_FP32 && it.prob->trig_rev_max > kHwTrigRevolutions)
        return fail(PDD_E_UNSUPPORTED,
                    "FP32 paths: a trig term's argument reaches %.1f revolutions over the domain, beyond the "
                    "+-%.0f of the hardware sine (use FP64 paths)",
                    it.prob->trig_rev_max, kHwTrigRevolutions);
    it.max_steps = o->max_steps ? o->max_steps : kDefaultMaxSteps;
    if (it.max_steps >= (1ull << 31)) return fail(PDD_E_INVALID, "max_steps must be < 2^31");
    if (cv) {
        pdd_status st = check_grid(d, it.u_prev, o->precision, "u_prev");
        if (st) return st;
        st = check_grid(d, it.resid, o->precision, "residual");
        if (st) return st;
    }
    if (it.est == kEstIto) {
        for (int q = 0; q < dim; ++q) {
            pdd_status st = check_grid(d, &it.grad[q], o->precision, "gradient");
            if (st) return st;
            for (int i = 0; i < dim; ++i)
                if (it.grad[q].n[i] != it.grad[0].n[i] || it.grad[q].lo[i] != it.grad[0].lo[i] ||
                    it.grad[q].hi[i] != it.grad[0].hi[i])
                    return fail(PDD_E_INVALID, "gradient grids must share one geometry (n, lo, hi)");
        }
    }
    if ((o->rec_phi || o->rec_e) && !o->rec_steps) return fail(PDD_E_INVALID, "per-path records need rec_steps");
    if (o->rec_steps && it.est != kEstPlain && !o->rec_e) return fail(PDD_E_INVALID, "correction and Ito records need rec_e");
    // the Ito control variate rides on phi, which is therefore always scored
    it.score_plain = it.est != kEstCorrection || (o->flags & PDD_PLAIN_ALONGSIDE);
    if (o->rec_steps && it.score_plain && !o->rec_phi) return fail(PDD_E_INVALID, "records need rec_phi");
    it.caller_records = o->rec_steps != nullptr;
    it.accumulate = (o->flags & PDD_ACCUMULATE) != 0;
    for (int64_t i = 0; i < it.n_nodes; ++i) {
        const double *x = it.nodes + i * dim;
        if (!finite3(x, dim) || !strictly_inside(d, x))
            return fail(PDD_E_INVALID, "node %lld is not strictly inside the domain", (long long)i);
    }
    it.uniform = o->n_paths_per_node == nullptr;
    it.total = 0;
    if (it.uniform) {
        if (o->path_offset + o->n_paths > (1ull << 32))
            return fail(PDD_E_INVALID, "path_offset + n_paths must be <= 2^32");
        if (o->n_paths && (uint64_t)it.n_nodes > UINT64_MAX / o->n_paths) return fail(PDD_E_INVALID, "too many paths");
        it.total = (uint64_t)it.n_nodes * o->n_paths;
    } else {
        it.starts.resize(it.n_nodes + 1);
        for (int64_t i = 0; i < it.n_nodes; ++i) {
            const uint64_t c = o->n_paths_per_node[i];
            if (o->path_offset + c > (1ull << 32))
                return fail(PDD_E_INVALID, "path_offset + paths of node %lld exceed 2^32", (long long)i);
            it.starts[i] = it.total;
            it.total += c;
        }
        it.starts[it.n_nodes] = it.total;
    }
    if (it.caller_records && it.total > kMaxLaunchSlots)
        return fail(PDD_E_UNSUPPORTED, "per-path records are limited to 2^31 paths per solve");
    return PDD_OK;
}

namespace {

pdd_status check_tuning(const pdd_tuning &tune)
{
    if (tune.block != 64 && tune.block != 128 && tune.block != 256)
        return fail(PDD_E_INVALID, "tuning.block must be 64, 128 or 256");
    if (tune.grab < 1 || tune.grab > 4096 || tune.blocks_per_cu < 0 || tune.blocks_per_cu > 64 ||
        tune.max_launch_paths < 0)
        return fail(PDD_E_INVALID, "tuning out of range");
    if (tune.refill != 0 && tune.refill != 1 && tune.refill != 2 && tune.refill != 4 && tune.refill != 8)
        return fail(PDD_E_INVALID, "tuning.refill must be 0, 1, 2, 4 or 8");
    if (tune.bridge < 0 || tune.bridge > 2) return fail(PDD_E_INVALID, "tuning.bridge must be 0, 1 or 2");
    return PDD_OK;
}

}  // namespace

// Launch shape of a group: the caller's (fields left 0 take the default),
// else the context's table entry for the group's key, else the default.
pdd_status pdd::read_tuning(const pdd_ctx *ctx, const pdd_solve_opts *o, int key, pdd_tuning &tune)
{
    tune = pdd_tuning{256, 0, 64, 0, 0, 0};
    if (!o->tuning && key >= 0) {
        auto f = ctx->tuned.find(key);
        if (f != ctx->tuned.end()) tune = f->second;
    }
    if (o->tuning) {
        if (o->tuning->block) tune.block = o->tuning->block;
        if (o->tuning->blocks_per_cu) tune.blocks_per_cu = o->tuning->blocks_per_cu;
        if (o->tuning->grab) tune.grab = o->tuning->grab;
        tune.max_launch_paths = o->tuning->max_launch_paths;
        if (o->tuning->refill) tune.refill = o->tuning->refill;
        if (o->tuning->bridge) tune.bridge = o->tuning->bridge;
    }
    return check_tuning(tune);
}

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Runs a group of items that share precision, dimension and estimator: one
// slot space, launches of the persistent path kernel over it, per-item
// reductions and statistics.
template <class T, int D, int EST>
pdd_status run_group(pdd_ctx *ctx, std::vector<HostItem *> &items, const pdd_tuning &tune,
                     bool timed, bool one_launch, hipStream_t s)
{
    const int n_items = (int)items.size();
    // problems used by the group
    std::vector<pdd_problem *> probs;
    std::vector<int> prob_of(n_items);
    for (int q = 0; q < n_items; ++q) {
        auto f = std::find(probs.begin(), probs.end(), items[q]->prob);
        prob_of[q] = (int)(f - probs.begin());
        if (f == probs.end()) probs.push_back(items[q]->prob);
    }
    // slot space and node tables
    std::vector<uint64_t> slot_begin(n_items), gnode(n_items + 1);
    uint64_t total = 0, n_nodes_all = 0, n_starts = 0;
    for (int q = 0; q < n_items; ++q) {
        slot_begin[q] = total;
        total += items[q]->total;
        gnode[q] = n_nodes_all;
        n_nodes_all += items[q]->n_nodes;
        if (!items[q]->uniform) n_starts += items[q]->n_nodes + 1;
    }
    gnode[n_items] = n_nodes_all;
    if (n_nodes_all == 0) return PDD_OK;
    bool any_scratch = false;
    for (auto *it : items) any_scratch |= !it->caller_records;

    // Kernel items: runs of consecutive items that walk alike (same problem,
    // step, exit test, law, max steps, scoring, grids, the same number of
    // paths for every node, and records in the scratch) are merged into one
    // kernel item whose nodes carry their own RNG node index, stream and path
    // offset. A wave can then take paths of the whole run without waiting for
    // its lanes at every item boundary; every path still draws the numbers of
    // its own solve. (Ragged items are not merged: finding a path's node in a
    // long ragged table costs more than the boundaries.)
    auto alike = [&](const HostItem *x, const HostItem *y) {
        if (x->prob != y->prob || x->caller_records || y->caller_records) return false;
        if (!x->uniform || !y->uniform || x->o->n_paths != y->o->n_paths) return false;
        const pdd_solve_opts *a = x->o, *b = y->o;
        if (a->dt != b->dt || a->exit_mode != b->exit_mode || a->law != b->law || x->max_steps != y->max_steps ||
            x->score_plain != y->score_plain)
            return false;
        if (EST == kEstPlain) return true;
        auto same = [](const pdd_grid *g, const pdd_grid *h) {
            if (g->data != h->data || g->dtype != h->dtype) return false;
            for (int i = 0; i < D; ++i)
                if (g->n[i] != h->n[i] || g->lo[i] != h->lo[i] || g->hi[i] != h->hi[i]) return false;
            return true;
        };
        if (EST == kEstIto) {
            for (int d = 0; d < D; ++d)
                if (!same(&x->grad[d], &y->grad[d])) return false;
            return true;
        }
        return same(x->u_prev, y->u_prev) && same(x->resid, y->resid);
    };
    std::vector<int> kfirst;  // first item of each kernel item, then n_items
    for (int q = 0; q < n_items; ++q)
        if (q == 0 || !alike(items[q - 1], items[q])) kfirst.push_back(q);
    const int n_k = (int)kfirst.size();
    kfirst.push_back(n_items);
    std::vector<uint64_t> kslot(n_k + 1);  // slot ranges of the kernel items
    bool any_merged = false;
    for (int k = 0; k < n_k; ++k) {
        kslot[k] = slot_begin[kfirst[k]];
        any_merged |= kfirst[k + 1] - kfirst[k] > 1;
    }
    kslot[n_k] = total;

    uint64_t per_launch = std::min(kScratchSlots, std::max<uint64_t>(total, 1));
    if (tune.max_launch_paths > 0 && !one_launch) per_launch = std::min<uint64_t>(per_launch, tune.max_launch_paths);
    const uint64_t n_launch = total ? (total + per_launch - 1) / per_launch : 0;

    // queue counters: one per launch for the single-item kernel, one per item
    // a launch touches for the batch kernel (items are sorted by slot), with
    // that item's launch-relative slot range
    std::vector<uint32_t> ctr_at(n_launch + 1, 0), seg_lo(n_launch, 0), seg_n(n_launch, 0);
    for (uint64_t l = 0; l < n_launch; ++l) {
        const uint64_t b = l * per_launch, e = std::min(total, b + per_launch);
        const auto first = std::upper_bound(kslot.begin(), kslot.begin() + n_k, b) - kslot.begin() - 1;
        const auto last = std::upper_bound(kslot.begin(), kslot.begin() + n_k, e - 1) - kslot.begin() - 1;
        seg_lo[l] = (uint32_t)first;
        seg_n[l] = (uint32_t)(last - first + 1);
        ctr_at[l + 1] = ctr_at[l] + std::max<uint32_t>(seg_n[l], 1);
    }
    const size_t n_ctr = (size_t)ctr_at[n_launch] + 2;
    const size_t ctr_bytes = (n_ctr * sizeof(uint32_t) + 7) & ~size_t(7);  // cleared in 8-byte words

    // staged upload: nodes | global node starts | item node starts | kernel
    // items | problems | node -> item | per-item post-processing entries |
    // queue ranges | per-node RNG table of merged items
    const size_t off_nodes = 0;
    const size_t off_gstart = align_up(off_nodes + n_nodes_all * D * sizeof(double), 256);
    const size_t off_istart = align_up(off_gstart + (n_nodes_all + 1) * sizeof(uint64_t), 256);
    const size_t off_items = align_up(off_istart + n_starts * sizeof(uint64_t), 256);
    const size_t off_probs = align_up(off_items + n_k * sizeof(ItemDesc<T>), 256);
    const size_t off_nitem = align_up(off_probs + probs.size() * sizeof(DevProblem<T>), 256);
    const size_t off_fitems = align_up(off_nitem + n_nodes_all * sizeof(uint32_t), 256);
    const size_t off_seg = align_up(off_fitems + n_items * sizeof(FinalItem), 256);
    const size_t off_rng = align_up(off_seg + n_ctr * 2 * sizeof(uint32_t), 256);
    const size_t bytes = align_up(off_rng + (any_merged ? n_nodes_all * 4 * sizeof(uint32_t) : 0), 256);

    pdd_status st;
    if ((st = ensure(ctx, ctx->nodes, bytes))) return st;
    if ((st = ensure(ctx, ctx->acc, n_nodes_all * sizeof(NodeAcc)))) return st;
    if ((st = ensure(ctx, ctx->counters, ctr_bytes))) return st;
    const bool need_phi = std::any_of(items.begin(), items.end(), [](HostItem *i) { return i->score_plain && !i->caller_records; });
    constexpr bool HAS_E = EST != kEstPlain;
    const size_t per_slot = sizeof(uint32_t) + (need_phi ? 8 : 0) + (HAS_E ? 8 : 0);
    double *sc_phi = nullptr, *sc_e = nullptr;
    uint32_t *sc_steps = nullptr;
    if (any_scratch && total) {
        if ((st = ensure(ctx, ctx->rec, per_launch * per_slot))) return st;
        char *base = static_cast<char *>(ctx->rec.ptr);
        sc_phi = need_phi ? reinterpret_cast<double *>(base) : nullptr;
        sc_e = HAS_E ? reinterpret_cast<double *>(base + (need_phi ? per_launch * 8 : 0)) : nullptr;
        sc_steps = reinterpret_cast<uint32_t *>(base + per_launch * ((need_phi ? 8 : 0) + (HAS_E ? 8 : 0)));
    }
    // grids the path kernel reads at every step, in cell layout: the residual
    // of a correction item, the gradient components of an Ito item (grid c of
    // item q at cell_at[3 q + c]); one copy per distinct grid, rebuilt per
    // solve since the caller may change a grid's values between solves
    // (an Ito item's D components are interleaved: one record of D x 2^D
    // values per cell, component c at offset c 2^D, keyed by its first grid)
    std::vector<const pdd_grid *> cell_grid;
    std::vector<size_t> cell_off, cell_at(3 * (size_t)n_items, 0);
    if (HAS_E) {
        size_t used = 0;
        for (int q = 0; q < n_items; ++q) {
            const pdd_grid *g = EST == kEstIto ? &items[q]->grad[0] : items[q]->resid;
            auto same = [&](const pdd_grid *o) {
                if (!std::equal(g->n, g->n + D, o->n)) return false;
                if (EST != kEstIto) return o->data == g->data;
                for (int c = 0; c < D; ++c)
                    if ((&items[q]->grad[0])[c].data != o[c].data) return false;
                return true;
            };
            size_t k = 0;
            while (k < cell_grid.size() && !same(cell_grid[k])) ++k;
            if (k == cell_grid.size()) {
                cell_grid.push_back(g);
                cell_off.push_back(used);
                used += align_up(cell_values<T>(g->n, D) * (EST == kEstIto ? D : 1), 64);
            }
            cell_at[3 * (size_t)q] = cell_off[k];
        }
        if ((st = ensure(ctx, ctx->cells, used * sizeof(T)))) return st;
    }
    T *d_cells = static_cast<T *>(ctx->cells.ptr);

    if ((st = ensure_stage(ctx, bytes))) return st;
    char *h = static_cast<char *>(ctx->stage);
    char *dv = static_cast<char *>(ctx->nodes.ptr);
    uint64_t *h_gstart = reinterpret_cast<uint64_t *>(h + off_gstart);
    uint64_t *h_istart = reinterpret_cast<uint64_t *>(h + off_istart);
    ItemDesc<T> *h_items = reinterpret_cast<ItemDesc<T> *>(h + off_items);
    DevProblem<T> *h_probs = reinterpret_cast<DevProblem<T> *>(h + off_probs);
    uint32_t *h_nitem = reinterpret_cast<uint32_t *>(h + off_nitem);
    FinalItem *h_fitems = reinterpret_cast<FinalItem *>(h + off_fitems);
    uint32_t *h_seg = reinterpret_cast<uint32_t *>(h + off_seg);
    for (uint64_t l = 0; l < n_launch; ++l) {
        const uint64_t b = l * per_launch, e = std::min(total, b + per_launch);
        for (uint32_t k = 0; k < seg_n[l]; ++k) {
            const int q = (int)(seg_lo[l] + k);
            const uint64_t lo = std::max(kslot[q], b), hi = std::min(kslot[q + 1], e);
            h_seg[2 * (ctr_at[l] + k)] = (uint32_t)(lo - b);
            h_seg[2 * (ctr_at[l] + k) + 1] = (uint32_t)(std::max(lo, hi) - b);
        }
    }
    std::vector<ItemDesc<T>> oitems(n_items);  // one per item, before merging
    std::memset(oitems.data(), 0, n_items * sizeof(ItemDesc<T>));
    std::memset(h_fitems, 0, n_items * sizeof(FinalItem));
    size_t istart_used = 0;
    for (int q = 0; q < n_items; ++q) {
        HostItem &it = *items[q];
        const pdd_solve_opts *o = it.o;
        std::memcpy(h + off_nodes + gnode[q] * D * sizeof(double), it.nodes, it.n_nodes * D * sizeof(double));
        for (int64_t i = 0; i < it.n_nodes; ++i) {
            h_gstart[gnode[q] + i] = slot_begin[q] + (it.uniform ? (uint64_t)i * o->n_paths : it.starts[i]);
            h_nitem[gnode[q] + i] = (uint32_t)q;
        }
        FinalItem &fi = h_fitems[q];
        fi.out = it.out;
        fi.gnode = gnode[q];
        fi.has_phi = it.score_plain ? 1 : 0;
        fi.accumulate = it.accumulate ? 1 : 0;
        fi.own_reduce = it.caller_records ? 1 : 0;
        if (EST == kEstCorrection) {
            fi.up_data = it.u_prev->data;
            fi.up_f64 = it.u_prev->dtype == PDD_DTYPE_F64;
            for (int i = 0; i < 3; ++i) {
                fi.up_n[i] = i < D ? it.u_prev->n[i] : 1;
                fi.up_lo[i] = it.u_prev->lo[i];
                fi.up_inv[i] = i < D ? (double)(it.u_prev->n[i] - 1) / (it.u_prev->hi[i] - it.u_prev->lo[i]) : 0.0;
            }
        }
        ItemDesc<T> &a = oitems[q];
        a.prob = prob_of[q];
        a.exit_mode = o->exit_mode;
        a.law = o->law;
        a.score_plain = it.score_plain ? 1 : 0;
        a.stream_tag = o->stream_id << 4;
        a.max_steps = (uint32_t)it.max_steps;
        a.n_nodes = (uint32_t)it.n_nodes;
        a.slot_begin = slot_begin[q];
        a.n_slots = it.total;
        a.uniform_n = o->n_paths;
        a.path_offset = o->path_offset;
        a.nodes = reinterpret_cast<const double *>(dv + off_nodes + gnode[q] * D * sizeof(double));
        if (!it.uniform) {
            std::memcpy(h_istart + istart_used, it.starts.data(), it.starts.size() * sizeof(uint64_t));
            a.node_start = reinterpret_cast<const uint64_t *>(dv + off_istart) + istart_used;
            istart_used += it.starts.size();
        }
        if (it.caller_records) {  // records of item slot r at r
            a.rec_phi = o->rec_phi;
            a.rec_e = o->rec_e;
            a.rec_steps = o->rec_steps;
            a.rec_base = 0;
        } else {
            a.rec_phi = sc_phi;
            a.rec_e = sc_e;
            a.rec_steps = sc_steps;
            a.rec_launch = 1;
        }
        const pdd_problem_desc &d = it.prob->desc;
        const double hh = o->dt;
        const double sig_sqh = d.sigma * std::sqrt(hh);
        a.h = (T)hh;
        a.sig_sqh = (T)sig_sqh;
        a.two_over_s2h = (T)(2.0 / (d.sigma * d.sigma * hh));
        a.gm_thresh = (T)(kGmShift * sig_sqh);
        a.bridge_thresh = (T)kBridgeSkip;
        a.dense_bridge = dense_boundary(d, hh) ? 1 : 0;
        a.u_prev = make_view<T>(it.u_prev, D);
        a.resid = make_view<T>(it.resid, D);
        if (EST == kEstCorrection) a.resid.cells = d_cells + cell_at[3 * (size_t)q];
        if (EST == kEstIto)
            for (int c = 0; c < D; ++c) {
                a.grad[c] = make_view<T>(&it.grad[c], D);
                a.grad[c].cells = d_cells + cell_at[3 * (size_t)q];
            }
    }
    h_gstart[n_nodes_all] = total;
    // kernel items: a merged one walks the nodes of its items in order, each
    // node with its own RNG node index, stream tag and path offset
    uint32_t *h_rng = reinterpret_cast<uint32_t *>(h + off_rng);
    for (int k = 0; k < n_k; ++k) {
        const int q0 = kfirst[k], q1 = kfirst[k + 1];
        h_items[k] = oitems[q0];
        if (q1 - q0 == 1) continue;
        ItemDesc<T> &a = h_items[k];
        for (int q = q0; q < q1; ++q)
            for (uint64_t i = gnode[q]; i < gnode[q + 1]; ++i) {
                h_rng[4 * i] = (uint32_t)(i - gnode[q]);
                h_rng[4 * i + 1] = oitems[q].stream_tag;
                h_rng[4 * i + 2] = (uint32_t)oitems[q].path_offset;
                h_rng[4 * i + 3] = 0;
            }
        a.n_nodes = (uint32_t)(gnode[q1] - gnode[q0]);
        a.n_slots = kslot[k + 1] - kslot[k];
        a.node_rng = reinterpret_cast<const uint32_t *>(dv + off_rng) + 4 * gnode[q0];
        a.path_offset = 0;
        a.stream_tag = 0;
    }
    for (size_t p = 0; p < probs.size(); ++p)
        std::memcpy(&h_probs[p], sizeof(T) == 4 ? (const void *)&probs[p]->pf : (const void *)&probs[p]->pd,
                    sizeof(DevProblem<T>));

    // chunk partials of long node segments (reduce kernel): sized for the
    // longest node of the group before anything of the group is enqueued
    uint64_t longest = 0;
    for (uint64_t i = 0; i < n_nodes_all; ++i) longest = std::max(longest, h_gstart[i + 1] - h_gstart[i]);
    const uint64_t max_chunks = std::max<uint64_t>(1, (longest + kReduceChunk - 1) / kReduceChunk);
    if (max_chunks > 1 && (st = ensure(ctx, ctx->partials, n_nodes_all * max_chunks * sizeof(NodeAcc)))) return st;
    // chunks needed by nodes [n_lo, n_hi] of gs restricted to slots [a, b)
    auto chunks_in = [&](const uint64_t *gs, uint32_t n_lo, uint32_t n_hi, uint64_t a, uint64_t b) {
        uint64_t mx = 0;
        for (uint32_t i = n_lo; i <= n_hi; ++i) {
            const uint64_t x = std::max(gs[i], a), y = std::min(gs[i + 1], b);
            if (y > x) mx = std::max(mx, y - x);
        }
        return (uint32_t)std::max<uint64_t>(1, (mx + kReduceChunk - 1) / kReduceChunk);
    };

    HIP_TRY(hipMemcpyAsync(dv, h, bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(ctx->staged, s));
    ctx->any_staged = true;
    const uint32_t *d_nitem = reinterpret_cast<const uint32_t *>(dv + off_nitem);
    const FinalItem *d_fitems = reinterpret_cast<const FinalItem *>(dv + off_fitems);
    NodeAcc *d_acc = static_cast<NodeAcc *>(ctx->acc.ptr);
    // zero sums, or the earlier paths' sums of accumulating items
    HIP_TRY(launch_init_acc(d_acc, (uint32_t)n_nodes_all, d_nitem, d_fitems, s));
    HIP_TRY(launch_zero(ctx->counters.ptr, ctr_bytes, s));
    for (size_t k = 0; k < cell_grid.size(); ++k) {
        if (EST == kEstIto) {
            for (int c = 0; c < D; ++c)
                HIP_TRY((launch_grid_cells_strided<T, T, D>(static_cast<const T *>(cell_grid[k][c].data),
                                                             cell_grid[k]->n, d_cells + cell_off[k],
                                                             (uint32_t)(D << D), (uint32_t)(c << D), s)));
        } else {
            HIP_TRY((launch_grid_cells<T, T, D>(static_cast<const T *>(cell_grid[k]->data), cell_grid[k]->n,
                                             d_cells + cell_off[k], s)));
        }
    }

    const int block = tune.block;
    // (the single-item kernel has no per-node RNG table)
    const bool one = n_k == 1 && kOneItemKernel<T, D, EST> && kfirst[1] == 1;
    // box / bridge / Gaussian / analytic throughout: the specialised kernel,
    // in the bridge form of the walks that hold most of the group's slots
    const bool spec = std::all_of(items.begin(), items.end(), [](const HostItem *i) { return specialised(*i); });
    uint64_t dense_slots = 0;
    for (int q = 0; q < n_items; ++q)
        if (oitems[q].dense_bridge) dense_slots += oitems[q].n_slots;
    const int kind = !spec                ? kKernelGeneric
                     : tune.bridge == 1     ? kKernelSparse
                     : tune.bridge == 2     ? kKernelDense
                     : 2 * dense_slots >= total ? kKernelDense
                                            : kKernelSparse;
    const void *fn = path_kernel_symbol<T, D, EST>(one, kind);
    // more workgroups than fit at once only queue behind the resident ones
    const int occ = occupancy(ctx, fn, block);
    const int bpc = tune.blocks_per_cu > 0 ? std::min(tune.blocks_per_cu, occ) : occ;
    const ItemDesc<T> *d_items = reinterpret_cast<const ItemDesc<T> *>(dv + off_items);
    const DevProblem<T> *d_probs = reinterpret_cast<const DevProblem<T> *>(dv + off_probs);
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (timed && total) {
        if (!ctx->spare.empty()) {
            ev = ctx->spare.back();
            ctx->spare.pop_back();
        } else {
            HIP_TRY(hipEventCreate(&ev.first));
            HIP_TRY(hipEventCreate(&ev.second));
        }
    }
    uint32_t launch = 0;
    for (uint64_t b = 0; b < total; b += per_launch, ++launch) {
        const uint64_t len = std::min(per_launch, total - b);
        LaunchArgs L{};
        L.slot_begin = b;
        L.launch_slots = (uint32_t)len;
        L.n_items = n_k;
        L.grab = tune.grab;
        L.counter = static_cast<uint32_t *>(ctx->counters.ptr) + ctr_at[launch];
        L.item_lo = (int32_t)seg_lo[launch];
        L.n_seg = seg_n[launch];
        L.refill_mask = refill_mask<D>(tune);
        L.seg = reinterpret_cast<const uint32_t *>(dv + off_seg) + 2 * ctr_at[launch];
        const uint64_t waves_needed = (len + 63) / 64;
        const uint64_t blocks_needed = (waves_needed * 64 + block - 1) / block;
        const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)ctx->n_cu * bpc, blocks_needed));
        if (timed && b == 0) HIP_TRY(hipEventRecord(ev.first, s));
        if (one) {  // the item and its problem travel as kernel arguments
            OneItemArgs<T> A;
            A.launch = L;
            A.item = h_items[0];
            A.prob = h_probs[0];
            // the single item starts at slot 0; scratch records of this launch
            // start at slot b
            if (A.item.rec_launch) A.item.rec_base = b;
            HIP_TRY((launch_path_kernel_one<T, D, EST>(A, grid, block, kind, s)));
        } else {
            HIP_TRY((launch_path_kernel<T, D, EST>(L, d_items, d_probs, grid, block, kind, s)));
        }
        if (timed && b + per_launch >= total) HIP_TRY(hipEventRecord(ev.second, s));
        // reduction of the nodes this launch touched: one launch for the items
        // whose records are in the scratch, one per item with caller records
        const uint64_t *d_gstart = reinterpret_cast<const uint64_t *>(dv + off_gstart);
        if (any_scratch) {
            const uint32_t n_lo = (uint32_t)(std::upper_bound(h_gstart, h_gstart + n_nodes_all + 1, b) - h_gstart - 1);
            const uint32_t n_hi =
                (uint32_t)(std::upper_bound(h_gstart, h_gstart + n_nodes_all + 1, b + len - 1) - h_gstart - 1);
            ReduceArgs r{};
            r.rec_phi = sc_phi;
            r.rec_e = sc_e;
            r.rec_steps = sc_steps;
            r.rec_base = b;
            r.node_start = d_gstart;
            r.slot_begin = b;
            r.slot_end = b + len;
            r.acc = d_acc;
            r.node_lo = n_lo;
            r.has_e = HAS_E;
            r.node_item = d_nitem;
            r.fitems = d_fitems;
            r.n_chunks = chunks_in(h_gstart, n_lo, n_hi, b, b + len);
            r.partials = static_cast<NodeAcc *>(ctx->partials.ptr);
            HIP_TRY(launch_reduce(r, n_hi - n_lo + 1, s));
        }
        for (int q = 0; q < n_items; ++q) {
            HostItem &it = *items[q];
            if (!it.caller_records) continue;
            const uint64_t lo = std::max(b, slot_begin[q]);
            const uint64_t hi = std::min(b + len, slot_begin[q] + it.total);
            if (lo >= hi) continue;
            const uint64_t *gs = h_gstart + gnode[q];
            const uint32_t n_lo = (uint32_t)(std::upper_bound(gs, gs + it.n_nodes + 1, lo) - gs - 1);
            const uint32_t n_hi = (uint32_t)(std::upper_bound(gs, gs + it.n_nodes + 1, hi - 1) - gs - 1);
            ReduceArgs r{};
            r.rec_phi = it.o->rec_phi;
            r.rec_e = it.o->rec_e;
            r.rec_steps = it.o->rec_steps;
            r.rec_base = slot_begin[q];
            r.node_start = d_gstart + gnode[q];
            r.slot_begin = lo;
            r.slot_end = hi;
            r.acc = d_acc + gnode[q];
            r.node_lo = n_lo;
            r.has_phi = it.score_plain;
            r.has_e = HAS_E;
            r.n_chunks = chunks_in(gs, n_lo, n_hi, lo, hi);
            r.partials = static_cast<NodeAcc *>(ctx->partials.ptr);
            HIP_TRY(launch_reduce(r, n_hi - n_lo + 1, s));
        }
    }
    if (timed && total) ctx->timed.push_back(ev);
    FinalizeArgs f{};
    f.acc = d_acc;
    f.nodes = reinterpret_cast<const double *>(dv + off_nodes);
    f.n_nodes = (uint32_t)n_nodes_all;
    f.dim = D;
    f.has_e = HAS_E;
    f.node_item = d_nitem;
    f.fitems = d_fitems;
    HIP_TRY(launch_finalize(f, s));
    return PDD_OK;
}

template <class T, int D>
pdd_status run_group_est(int est, pdd_ctx *ctx, std::vector<HostItem *> &g, const pdd_tuning &tune, bool timed,
                         bool one_launch, hipStream_t s)
{
    if (est == kEstCorrection) return run_group<T, D, kEstCorrection>(ctx, g, tune, timed, one_launch, s);
    if (est == kEstIto) return run_group<T, D, kEstIto>(ctx, g, tune, timed, one_launch, s);
    return run_group<T, D, kEstPlain>(ctx, g, tune, timed, one_launch, s);
}

}  // namespace

// Validates items, then runs them grouped by (precision, dim, estimator).
pdd_status pdd::run_items(pdd_ctx *ctx, std::vector<HostItem> &items, hipStream_t s, bool one_launch,
                          const pdd_ctx *owner)
{
    if (!owner) owner = ctx;
    for (auto &it : items) {
        pdd_status st = validate_item(it);
        if (st) return st;
        if (it.prob->ctx != owner) return fail(PDD_E_INVALID, "problem belongs to another context");
    }
    if (items.empty()) return PDD_OK;
    pdd_tuning tune;
    pdd_status st = read_tuning(ctx, items[0].o, -1, tune);  // the caller's shape, checked up front
    if (st) return st;
    bool timed = false;
    for (auto &it : items) timed |= (it.o->flags & PDD_TIME_KERNEL) != 0;
    HIP_TRY(hipSetDevice(ctx->device));
    if (ctx->any_done) HIP_TRY(hipStreamWaitEvent(s, ctx->done, 0));
    for (int prec = 0; prec < 2; ++prec)
        for (int dim = 2; dim <= 3; ++dim)
            for (int est = kEstPlain; est <= kEstIto; ++est) {
                std::vector<HostItem *> g;
                for (auto &it : items)
                    if (it.o->precision == prec && it.prob->desc.dim == dim && it.est == est && it.n_nodes > 0)
                        g.push_back(&it);
                if (g.empty()) continue;
                const bool generic = !std::all_of(g.begin(), g.end(), [](const HostItem *i) { return specialised(*i); });
                if ((st = read_tuning(ctx, items[0].o, tuning_key(prec, dim, est, generic), tune))) return st;
                if (prec == PDD_FP32)
                    st = dim == 2 ? run_group_est<float, 2>(est, ctx, g, tune, timed, one_launch, s)
                                  : run_group_est<float, 3>(est, ctx, g, tune, timed, one_launch, s);
                else
                    st = dim == 2 ? run_group_est<double, 2>(est, ctx, g, tune, timed, one_launch, s)
                                  : run_group_est<double, 3>(est, ctx, g, tune, timed, one_launch, s);
                if (st) return st;
                // the next group reuses the staging buffer and the scratch
                HIP_TRY(hipEventRecord(ctx->done, s));
                ctx->any_done = true;
            }
    return PDD_OK;
}

extern "C" {

const char *pdd_last_error(void) { return g_error.c_str(); }

pdd_status pdd_init(pdd_ctx **out, int hip_device)
{
    if (!out) return fail(PDD_E_INVALID, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (hip_device < 0 || hip_device >= n) return fail(PDD_E_INVALID, "no HIP device %d (have %d)", hip_device, n);
    HIP_TRY(hipSetDevice(hip_device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, hip_device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(PDD_E_UNSUPPORTED, "built for gfx950, device is %s", prop.gcnArchName);
    pdd_ctx *ctx = new pdd_ctx();
    ctx->device = hip_device;
    ctx->n_cu = prop.multiProcessorCount;
    if (hipEventCreateWithFlags(&ctx->done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->staged, hipEventDisableTiming) != hipSuccess) {
        delete ctx;
        return fail(PDD_E_HIP, "event creation failed");
    }
    // the allocation-free solve's scratch on this device, and the occupancy of
    // every plain path kernel, so that pdd_solve_nodes_noalloc only looks
    // things up; a failed lookup is reported by that entry point alone (and
    // cleared here, so that no later launch check mistakes it for its own)
    if (noalloc_attach(hip_device) != PDD_OK) (void)hipGetLastError();
    for (int block : {64, 128, 256})
        for (int kind : {kKernelGeneric, kKernelSparse, kKernelDense}) {
            for (bool one : {false, true}) {
                occupancy(ctx, path_kernel_symbol<float, 2, kEstPlain>(one, kind), block);
                occupancy(ctx, path_kernel_symbol<float, 3, kEstPlain>(one, kind), block);
                occupancy(ctx, path_kernel_symbol<double, 2, kEstPlain>(one, kind), block);
                occupancy(ctx, path_kernel_symbol<double, 3, kEstPlain>(one, kind), block);
            }
        }
    *out = ctx;
    return PDD_OK;
}

void pdd_shutdown(pdd_ctx *ctx)
{
    if (!ctx) return;
    // best effort: errors cannot be reported from here
    (void)hipSetDevice(ctx->device);
    if (ctx->any_done) (void)hipEventSynchronize(ctx->done);
    if (ctx->any_staged) (void)hipEventSynchronize(ctx->staged);
    for (DeviceBuffer *b : {&ctx->nodes, &ctx->starts, &ctx->acc, &ctx->counters, &ctx->rec, &ctx->partials,
                            &ctx->gather, &ctx->cells, &ctx->stage2, &ctx->stage2_lu, &ctx->stage2_resp})
        if (b->ptr) (void)hipFree(b->ptr);
    if (ctx->stage) (void)hipHostFree(ctx->stage);
    if (ctx->readback) (void)hipHostFree(ctx->readback);
    (void)hipEventDestroy(ctx->done);
    (void)hipEventDestroy(ctx->staged);
    for (auto *v : {&ctx->timed, &ctx->spare})
        for (auto &e : *v) {
            (void)hipEventSynchronize(e.second);
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    delete ctx;
}

pdd_status pdd_create_problem(pdd_ctx *ctx, const pdd_problem_desc *desc, pdd_problem **out)
{
    if (!ctx || !out) return fail(PDD_E_INVALID, "ctx and out must not be NULL");
    *out = nullptr;
    pdd_status st = check_desc(desc);
    if (st) return st;
    pdd_problem *p = new pdd_problem();
    p->serial = next_problem_serial();
    p->ctx = ctx;
    p->desc = *desc;
    p->trig_rev_max = trig_revolutions(*desc);
    if ((st = fill_problem(*desc, p->pf, true)) || (st = fill_problem(*desc, p->pd, false))) {
        delete p;
        return st;
    }
    *out = p;
    return PDD_OK;
}

void pdd_destroy_problem(pdd_problem *problem)
{
    if (!problem) return;
    if (problem->tab.ptr) {
        (void)hipSetDevice(problem->ctx->device);
        (void)hipFree(problem->tab.ptr);
    }
    delete problem;
}

pdd_status pdd_create_problem_tabulated(pdd_ctx *ctx, const pdd_problem_desc *desc, const pdd_coef_grids *grids,
                                        pdd_problem **out)
{
    if (!ctx || !out) return fail(PDD_E_INVALID, "ctx and out must not be NULL");
    *out = nullptr;
    if (!grids) return fail(PDD_E_INVALID, "grids is NULL");
    pdd_status st = check_desc(desc);
    if (st) return st;
    const pdd_grid *g[6] = {grids->b[0], grids->b[1], grids->b[2], grids->c, grids->f, grids->g};
    static const char *names[6] = {"b[0]", "b[1]", "b[2]", "c", "f", "g"};
    const int D = desc->dim;
    if (D == 2 && g[2]) return fail(PDD_E_INVALID, "b[2] grid given for a 2D problem");
    // both precisions' cell layouts of every given grid, in one allocation
    uint32_t tab = 0;
    for (int q = 0; q < 6; ++q) {
        if (!g[q]) continue;
        if ((st = check_grid(*desc, g[q], -1, names[q]))) return st;
        tab |= 1u << q;
    }
    // b_0 .. b_{D-1}, c and f all given on one geometry: interleaved (slot 6),
    // so a step reads all of them at once, in one record of the (D + 2) values'
    // 2^D corners per cell (one 64-byte read per step in 2D FP32). A 2D grid
    // whose cell records would outgrow an XCD's 4 MB L2 takes, per grid point,
    // one record of the four values at the point and at the point above it
    // instead (half the bytes; a cell's four corners are the records of two
    // adjacent points, 64 contiguous bytes, mostly one L2 request): at 513^2
    // the cell records (16.8 MB) hit L2 55 % of the time and the launch waits
    // on the memory fabric; records of single points (4.2 MB; a step then
    // reads two rows, about 2.2 L2 requests) were 7.5 % faster, these pair
    // records (8.4 MB) 6 % faster again.
    auto in_record = [&](int q) { return q < D || q == 3 || q == 4; };
    bool fused = g[3] != nullptr;  // the geometry is compared with c's grid
    for (int q = 0; q < 5; ++q)
        if (in_record(q)) {
            fused = fused && g[q];
            for (int i = 0; fused && i < D; ++i)
                fused = g[q]->n[i] == g[3]->n[i] && g[q]->lo[i] == g[3]->lo[i] && g[q]->hi[i] == g[3]->hi[i];
        }
    const bool by_point =
        fused && D == 2 && (size_t)(g[3]->n[0] - 1) * (size_t)(g[3]->n[1] - 1) * 16 * sizeof(float) > kCellRecordMaxBytes;
    const uint32_t rec_vals = by_point ? 8u : (uint32_t)((D + 2) << D);
    size_t off32[7] = {}, off64[7] = {}, n32 = 0, n64 = 0;
    for (int q = 0; q < 6; ++q)
        if ((tab & (1u << q)) && !(fused && in_record(q))) {
            off32[q] = n32;
            n32 += align_up(cell_values<float>(g[q]->n, D), 64);
            off64[q] = n64;
            n64 += align_up(cell_values<double>(g[q]->n, D), 64);
        }
    if (fused) {
        const size_t recs = by_point ? (size_t)g[3]->n[0] * (g[3]->n[1] - 1) : cell_values<float>(g[3]->n, D) >> D;
        off32[6] = n32;
        n32 += align_up(recs * rec_vals, 64);
        off64[6] = n64;
        n64 += align_up(recs * rec_vals, 64);
        tab |= by_point ? 64u | 128u : 64u;
    }
    pdd_problem *p = new pdd_problem();
    p->serial = next_problem_serial();
    p->ctx = ctx;
    p->desc = *desc;
    p->trig_rev_max = trig_revolutions(*desc);
    if ((st = fill_problem(*desc, p->pf, true)) || (st = fill_problem(*desc, p->pd, false))) {
        delete p;
        return st;
    }
    if (tab) {
        auto bail = [&](pdd_status s2) {
            pdd_destroy_problem(p);
            return s2;
        };
        if (hipSetDevice(ctx->device) != hipSuccess) return bail(fail(PDD_E_HIP, "hipSetDevice failed"));
        const size_t bytes = align_up(n32 * sizeof(float), 256) + n64 * sizeof(double);
        if (hipMalloc(&p->tab.ptr, bytes) != hipSuccess) {
            p->tab.ptr = nullptr;
            return bail(fail(PDD_E_NOMEM, "hipMalloc of %zu bytes for tabulated coefficients failed", bytes));
        }
        p->tab.cap = bytes;
        float *c32 = static_cast<float *>(p->tab.ptr);
        double *c64 = reinterpret_cast<double *>(static_cast<char *>(p->tab.ptr) + align_up(n32 * sizeof(float), 256));
        for (int q = 0; q < 6; ++q) {
            if (!(tab & (1u << q))) continue;
            const pdd_grid *gq = g[q];
            // own cell layout, or field k of the interleaved records
            const bool rec = fused && in_record(q);
            const uint32_t k = q < 3 ? (uint32_t)q : (uint32_t)(q - 3 + D);
            const uint32_t stride = rec ? rec_vals : (1u << D), off = rec ? (by_point ? k : k << D) : 0u;
            float *d32 = c32 + (rec ? off32[6] : off32[q]);
            double *d64 = c64 + (rec ? off64[6] : off64[q]);
            hipError_t e1, e2;
            if (rec && by_point) {  // field k of the pair records: point p, then p + n0
                const uint64_t np = (uint64_t)gq->n[0] * (gq->n[1] - 1);
                const uint64_t n0 = (uint64_t)gq->n[0];
                if (gq->dtype == PDD_DTYPE_F32) {
                    const float *src = static_cast<const float *>(gq->data);
                    e1 = launch_grid_points_strided<float, float>(src, np, d32, 8u, k, nullptr);
                    if (e1 == hipSuccess) e1 = launch_grid_points_strided<float, float>(src + n0, np, d32, 8u, 4u + k, nullptr);
                    e2 = launch_grid_points_strided<float, double>(src, np, d64, 8u, k, nullptr);
                    if (e2 == hipSuccess) e2 = launch_grid_points_strided<float, double>(src + n0, np, d64, 8u, 4u + k, nullptr);
                } else {
                    const double *src = static_cast<const double *>(gq->data);
                    e1 = launch_grid_points_strided<double, float>(src, np, d32, 8u, k, nullptr);
                    if (e1 == hipSuccess) e1 = launch_grid_points_strided<double, float>(src + n0, np, d32, 8u, 4u + k, nullptr);
                    e2 = launch_grid_points_strided<double, double>(src, np, d64, 8u, k, nullptr);
                    if (e2 == hipSuccess) e2 = launch_grid_points_strided<double, double>(src + n0, np, d64, 8u, 4u + k, nullptr);
                }
            } else if (gq->dtype == PDD_DTYPE_F32) {
                const float *src = static_cast<const float *>(gq->data);
                e1 = D == 2 ? launch_grid_cells_strided<float, float, 2>(src, gq->n, d32, stride, off, nullptr)
                            : launch_grid_cells_strided<float, float, 3>(src, gq->n, d32, stride, off, nullptr);
                e2 = D == 2 ? launch_grid_cells_strided<float, double, 2>(src, gq->n, d64, stride, off, nullptr)
                            : launch_grid_cells_strided<float, double, 3>(src, gq->n, d64, stride, off, nullptr);
            } else {
                const double *src = static_cast<const double *>(gq->data);
                e1 = D == 2 ? launch_grid_cells_strided<double, float, 2>(src, gq->n, d32, stride, off, nullptr)
                            : launch_grid_cells_strided<double, float, 3>(src, gq->n, d32, stride, off, nullptr);
                e2 = D == 2 ? launch_grid_cells_strided<double, double, 2>(src, gq->n, d64, stride, off, nullptr)
                            : launch_grid_cells_strided<double, double, 3>(src, gq->n, d64, stride, off, nullptr);
            }
            if (e1 != hipSuccess || e2 != hipSuccess)
                return bail(fail(PDD_E_HIP, "cell layout of the %s grid: %s", names[q],
                                 hipGetErrorString(e1 != hipSuccess ? e1 : e2)));
            p->pf.tabv[q] = make_view<float>(gq, D);
            p->pf.tabv[q].data = nullptr;
            p->pf.tabv[q].cells = rec ? nullptr : d32;
            p->pd.tabv[q] = make_view<double>(gq, D);
            p->pd.tabv[q].data = nullptr;
            p->pd.tabv[q].cells = rec ? nullptr : d64;
        }
        if (fused) {
            p->pf.tab_fused = c32 + off32[6];
            p->pd.tab_fused = c64 + off64[6];
        }
        const hipError_t e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) return bail(fail(PDD_E_HIP, "tabulated coefficients: %s", hipGetErrorString(e)));
        p->pf.tab = p->pd.tab = tab;
    }
    *out = p;
    return PDD_OK;
}

pdd_status pdd_solve_nodes(pdd_problem *problem, const double *nodes, int64_t n_nodes,
                           const pdd_solve_opts *opts, pdd_node_stats *out, void *stream)
{
    if (!problem) return fail(PDD_E_INVALID, "problem is NULL");
    std::vector<HostItem> items(1);
    items[0].prob = problem;
    items[0].nodes = nodes;
    items[0].n_nodes = n_nodes;
    items[0].o = opts;
    items[0].out = out;
    return run_items(problem->ctx, items, static_cast<hipStream_t>(stream));
}

pdd_status pdd_solve_correction(pdd_problem *problem, const pdd_grid *u_prev, const pdd_grid *resid,
                                const double *nodes, int64_t n_nodes, const pdd_solve_opts *opts,
                                pdd_node_stats *out, void *stream)
{
    if (!problem) return fail(PDD_E_INVALID, "problem is NULL");
    if (!u_prev || !resid) return fail(PDD_E_INVALID, "correction solve needs u_prev and residual grids");
    std::vector<HostItem> items(1);
    items[0].prob = problem;
    items[0].u_prev = u_prev;
    items[0].resid = resid;
    items[0].nodes = nodes;
    items[0].n_nodes = n_nodes;
    items[0].o = opts;
    items[0].out = out;
    return run_items(problem->ctx, items, static_cast<hipStream_t>(stream));
}

pdd_status pdd_solve_ito(pdd_problem *problem, const pdd_grid *grad, const double *nodes, int64_t n_nodes,
                         const pdd_solve_opts *opts, pdd_node_stats *out, void *stream)
{
    if (!problem) return fail(PDD_E_INVALID, "problem is NULL");
    if (!grad) return fail(PDD_E_INVALID, "the Ito control variate needs the gradient grids");
    std::vector<HostItem> items(1);
    items[0].prob = problem;
    items[0].grad = grad;
    items[0].nodes = nodes;
    items[0].n_nodes = n_nodes;
    items[0].o = opts;
    items[0].out = out;
    return run_items(problem->ctx, items, static_cast<hipStream_t>(stream));
}

pdd_status pdd_solve_batch(pdd_ctx *ctx, const pdd_work_item *witems, int32_t n_items, void *stream)
{
    if (!ctx) return fail(PDD_E_INVALID, "ctx is NULL");
    if (n_items < 0 || (n_items > 0 && !witems)) return fail(PDD_E_INVALID, "bad items");
    std::vector<HostItem> items(n_items);
    for (int32_t q = 0; q < n_items; ++q) {
        const pdd_work_item &w = witems[q];
        if (!w.problem) return fail(PDD_E_INVALID, "item %d: problem is NULL", q);
        if ((w.u_prev == nullptr) != (w.resid == nullptr))
            return fail(PDD_E_INVALID, "item %d: correction needs u_prev and residual grids", q);
        items[q].prob = w.problem;
        items[q].u_prev = w.u_prev;
        items[q].resid = w.resid;
        items[q].grad = w.grad;
        items[q].nodes = w.nodes;
        items[q].n_nodes = w.n_nodes;
        items[q].o = w.opts;
        items[q].out = w.out;
    }
    return run_items(ctx, items, static_cast<hipStream_t>(stream));
}

pdd_status pdd_plan_paths(const pdd_node_stats *pilot, int64_t n_nodes, double target_se,
                          uint64_t n_max, uint64_t *n_total)
{
    if (n_nodes < 0 || (n_nodes > 0 && (!pilot || !n_total))) return fail(PDD_E_INVALID, "bad arguments");
    if (!(target_se > 0.0) || !std::isfinite(target_se)) return fail(PDD_E_INVALID, "target_se must be finite and > 0");
    const double inv2 = 1.0 / (target_se * target_se);
    for (int64_t i = 0; i < n_nodes; ++i) {
        const pdd_node_stats &p = pilot[i];
        if (p.n < 2 || !std::isfinite(p.var) || p.var < 0.0)
            return fail(PDD_E_INVALID, "pilot of node %lld has n < 2 or no finite variance", (long long)i);
        const double want = std::ceil(p.var * inv2);  // N = V / SE^2
        uint64_t n = want >= 1.8e19 ? UINT64_MAX : (uint64_t)want;
        n = std::max<uint64_t>(n, (uint64_t)p.n);
        n_total[i] = std::min(n, n_max);
    }
    return PDD_OK;
}

pdd_status pdd_solve_to_tolerance(pdd_ctx *ctx, const pdd_work_item *witems, int32_t n_items,
                                  const double *target_se, uint64_t n_pilot, uint64_t n_max,
                                  void *stream)
{
    if (!ctx) return fail(PDD_E_INVALID, "ctx is NULL");
    if (n_items < 0 || (n_items > 0 && (!witems || !target_se))) return fail(PDD_E_INVALID, "bad items");
    if (n_pilot < 2 || n_max < n_pilot) return fail(PDD_E_INVALID, "need 2 <= n_pilot <= n_max");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<pdd_solve_opts> opts(n_items);
    std::vector<HostItem> items(n_items);
    for (int32_t q = 0; q < n_items; ++q) {
        const pdd_work_item &w = witems[q];
        if (!w.problem || !w.opts) return fail(PDD_E_INVALID, "item %d: problem or opts is NULL", q);
        if ((w.u_prev == nullptr) != (w.resid == nullptr))
            return fail(PDD_E_INVALID, "item %d: correction needs u_prev and residual grids", q);
        if (w.opts->rec_steps || w.opts->rec_phi || w.opts->rec_e)
            return fail(PDD_E_UNSUPPORTED, "item %d: per-path records are not kept by solves to a tolerance", q);
        if (!(target_se[q] > 0.0) || !std::isfinite(target_se[q]))
            return fail(PDD_E_INVALID, "item %d: target_se must be finite and > 0", q);
        opts[q] = *w.opts;
        opts[q].n_paths = n_pilot;
        opts[q].n_paths_per_node = nullptr;
        opts[q].flags &= ~PDD_ACCUMULATE;
        HostItem &it = items[q];
        it.prob = w.problem;
        it.u_prev = w.u_prev;
        it.resid = w.resid;
        it.grad = w.grad;
        it.nodes = w.nodes;
        it.n_nodes = w.n_nodes;
        it.o = &opts[q];
        it.out = w.out;
    }
    pdd_status st = run_items(ctx, items, s);  // pilot
    if (st) return st;
    // all pilot statistics back in one copy into pinned memory, after a
    // kernel has gathered the items' outputs into one device buffer (the
    // gather table travels in the same pinned buffer, behind the statistics)
    size_t total_nodes = 0, n_live = 0;
    for (int32_t q = 0; q < n_items; ++q) {
        total_nodes += (size_t)std::max<int64_t>(0, witems[q].n_nodes);
        n_live += witems[q].n_nodes > 0;
    }
    const size_t stats_bytes = align_up(std::max<size_t>(total_nodes, 1) * sizeof(pdd_node_stats), 256);
    const size_t rb_bytes = stats_bytes + std::max<size_t>(n_live, 1) * sizeof(GatherItem);
    if ((st = ensure(ctx, ctx->gather, rb_bytes))) return st;
    if (rb_bytes > ctx->readback_cap) {
        if (ctx->readback) HIP_TRY(hipHostFree(ctx->readback));
        ctx->readback = nullptr;
        ctx->readback_cap = 0;
        if (hipHostMalloc(&ctx->readback, rb_bytes, hipHostMallocDefault) != hipSuccess) {
            ctx->readback = nullptr;
            return fail(PDD_E_NOMEM, "pinned allocation of %zu bytes failed", rb_bytes);
        }
        ctx->readback_cap = rb_bytes;
    }
    pdd_node_stats *pilot = static_cast<pdd_node_stats *>(ctx->readback);
    GatherItem *table = reinterpret_cast<GatherItem *>(static_cast<char *>(ctx->readback) + stats_bytes);
    std::vector<size_t> at(n_items, 0);
    size_t used = 0, k = 0;
    for (int32_t q = 0; q < n_items; ++q) {
        const int64_t n = witems[q].n_nodes;
        at[q] = used;
        if (n <= 0) continue;
        table[k++] = GatherItem{static_cast<const pdd_node_stats *>(witems[q].out), (uint64_t)n, (uint64_t)used};
        used += (size_t)n;
    }
    char *dg = static_cast<char *>(ctx->gather.ptr);
    HIP_TRY(hipMemcpyAsync(dg + stats_bytes, table, k * sizeof(GatherItem), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_gather_stats(reinterpret_cast<const GatherItem *>(dg + stats_bytes), (uint32_t)k,
                                reinterpret_cast<pdd_node_stats *>(dg), s));
    HIP_TRY(hipMemcpyAsync(pilot, dg, used * sizeof(pdd_node_stats), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    // plan; items whose pilot already meets the target are done
    std::vector<std::vector<uint64_t>> counts(n_items);
    std::vector<HostItem> cont;
    cont.reserve(n_items);
    for (int32_t q = 0; q < n_items; ++q) {
        const int64_t n = witems[q].n_nodes;
        if (n <= 0) continue;
        counts[q].resize(n);
        if ((st = pdd_plan_paths(pilot + at[q], n, target_se[q], n_max, counts[q].data()))) return st;
        bool more = false;
        for (auto &c : counts[q]) {
            c -= n_pilot;
            more |= c > 0;
        }
        if (!more) continue;
        opts[q].n_paths_per_node = counts[q].data();
        opts[q].path_offset += n_pilot;
        opts[q].flags |= PDD_ACCUMULATE;
        HostItem it;
        it.prob = witems[q].problem;
        it.u_prev = witems[q].u_prev;
        it.resid = witems[q].resid;
        it.grad = witems[q].grad;
        it.nodes = witems[q].nodes;
        it.n_nodes = n;
        it.o = &opts[q];
        it.out = witems[q].out;
        cont.push_back(std::move(it));
    }
    if (cont.empty()) return PDD_OK;
    return run_items(ctx, cont, s);  // continuation
}

pdd_status pdd_kernel_times(pdd_ctx *ctx, double *ms, int32_t cap, int32_t *n)
{
    if (!ctx || !n || cap < 0 || (cap > 0 && !ms)) return fail(PDD_E_INVALID, "bad arguments");
    HIP_TRY(hipSetDevice(ctx->device));
    int32_t k = 0;
    for (auto &e : ctx->timed) {
        HIP_TRY(hipEventSynchronize(e.second));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, e.first, e.second));
        if (k < cap) ms[k++] = (double)t;
        ctx->spare.push_back(e);
    }
    ctx->timed.clear();
    *n = k;
    return PDD_OK;
}

pdd_status pdd_autotune(pdd_ctx *ctx, const pdd_work_item *item, pdd_tuning *out)
{
    if (!ctx || !item || !out || !item->problem || !item->opts) return fail(PDD_E_INVALID, "NULL argument");
    if (item->problem->ctx != ctx) return fail(PDD_E_INVALID, "problem belongs to another context");
    if (item->n_nodes < 1 || !item->nodes) return fail(PDD_E_INVALID, "autotuning needs nodes");
    if ((item->u_prev == nullptr) != (item->resid == nullptr))
        return fail(PDD_E_INVALID, "correction needs u_prev and residual grids");
    if (item->u_prev && item->grad)
        return fail(PDD_E_INVALID, "an item takes the correction grids or the gradient grids, not both");
    const int dim = item->problem->desc.dim;
    const int est = item->u_prev ? kEstCorrection : (item->grad ? kEstIto : kEstPlain);
    const int prec = item->opts->precision;
    if (prec != PDD_FP32 && prec != PDD_FP64) return fail(PDD_E_INVALID, "bad precision");
    HIP_TRY(hipSetDevice(ctx->device));
    // the kernel this group launches for a single item, and its occupancy
    const bool spec = item->problem->desc.domain == PDD_DOMAIN_BOX && item->problem->pf.tab == 0 &&
                      item->opts->exit_mode == PDD_EXIT_BRIDGE && item->opts->law == PDD_LAW_GAUSS;
    const int kind = !spec ? kKernelGeneric
                     : dense_boundary(item->problem->desc, item->opts->dt) ? kKernelDense : kKernelSparse;
    auto symbol = [&](auto tag) -> const void * {
        using T = decltype(tag);
        if (dim == 2)
            return est == kEstCorrection ? path_kernel_symbol<T, 2, kEstCorrection>(true, kind)
                   : est == kEstIto      ? path_kernel_symbol<T, 2, kEstIto>(true, kind)
                                         : path_kernel_symbol<T, 2, kEstPlain>(true, kind);
        return est == kEstCorrection ? path_kernel_symbol<T, 3, kEstCorrection>(true, kind)
               : est == kEstIto      ? path_kernel_symbol<T, 3, kEstIto>(true, kind)
                                     : path_kernel_symbol<T, 3, kEstPlain>(true, kind);
    };
    const void *fn = prec == PDD_FP32 ? symbol(0.0f) : symbol(0.0);
    const int occ256 = occupancy(ctx, fn, 256);
    // sample: up to 32 nodes spread over the item's, about 8 (then 16) paths
    // per resident lane of the default shape
    const int64_t ns = std::min<int64_t>(32, item->n_nodes);
    const uint64_t lanes = (uint64_t)ctx->n_cu * occ256 * 256;
    std::vector<double> nodes((size_t)ns * dim);
    for (int64_t i = 0; i < ns; ++i) {
        const int64_t src = i * item->n_nodes / ns;
        std::memcpy(&nodes[(size_t)i * dim], item->nodes + src * dim, dim * sizeof(double));
    }
    pdd_solve_opts o = *item->opts;
    o.n_paths = std::max<uint64_t>(64, (8 * lanes + ns - 1) / ns);
    o.n_paths_per_node = nullptr;
    o.path_offset = 0;
    o.flags &= PDD_PLAIN_ALONGSIDE;
    o.rec_phi = o.rec_e = nullptr;
    o.rec_steps = nullptr;
    pdd_tuning cand{};
    o.tuning = &cand;
    pdd_node_stats *dev = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    pdd_status st = PDD_OK;
    auto cleanup = [&] {
        if (s) (void)hipStreamSynchronize(s);
        if (dev) (void)hipFree(dev);
        if (s) (void)hipStreamDestroy(s);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (hipMalloc(&dev, (size_t)ns * sizeof(pdd_node_stats)) != hipSuccess ||
        hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(PDD_E_HIP, "autotune could not allocate its sample");
    }
    const uint64_t base_paths = o.n_paths;
    auto time_one = [&](const pdd_tuning &t, uint64_t paths, float &ms) -> pdd_status {
        cand = t;
        o.n_paths = paths;
        std::vector<HostItem> items(1);
        items[0].prob = item->problem;
        items[0].u_prev = item->u_prev;
        items[0].resid = item->resid;
        items[0].grad = item->grad;
        items[0].nodes = nodes.data();
        items[0].n_nodes = ns;
        items[0].o = &o;
        items[0].out = dev;
        HIP_TRY(hipEventRecord(e0, s));
        pdd_status r = run_items(ctx, items, s);
        if (r) return r;
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        return PDD_OK;
    };
    float ms = 0.f;
    const pdd_tuning dflt{256, occ256, 64, 0, 0, 0};
    st = time_one(dflt, 2 * base_paths, ms);  // warm-up (code load, scratch growth)
    // candidates: every block size and grab at full occupancy, and the
    // default block with fewer workgroups per CU
    std::vector<pdd_tuning> cands{dflt};
    for (int block : {64, 128, 256}) {
        const int occ = occupancy(ctx, fn, block);
        for (int grab : {16, 64, 256})
            if (!(block == 256 && grab == 64)) cands.push_back(pdd_tuning{block, occ, grab, 0, 0, 0});
    }
    if (occ256 * 3 / 4 >= 1 && occ256 * 3 / 4 != occ256)
        cands.push_back(pdd_tuning{256, occ256 * 3 / 4, 64, 0, 0, 0});
    if (occ256 / 2 >= 1 && occ256 / 2 != occ256 * 3 / 4) cands.push_back(pdd_tuning{256, occ256 / 2, 64, 0, 0, 0});
    pdd_tuning best = dflt;
    float best_ms = 1e30f;
    // the cost of a shape is the marginal time of the second P paths, t(2P) -
    // t(P): it cancels the fixed costs and the exit-time tail, which a whole
    // short run would weigh far more than a real solve does
    auto sweep = [&](const std::vector<pdd_tuning> &cs, bool first) {
        for (size_t c = 0; c < cs.size() && !st; ++c) {
            float t1 = 1e30f, t2 = 1e30f;
            for (int rep = 0; rep < 2 && !st; ++rep) {
                st = time_one(cs[c], base_paths, ms);
                t1 = std::min(t1, ms);
                if (!st) st = time_one(cs[c], 2 * base_paths, ms);
                t2 = std::min(t2, ms);
            }
            const float m = t2 - t1;
            // the default stands unless a candidate is more than 2% faster
            if (!st && ((first && c == 0) || m < 0.98f * best_ms)) {
                best_ms = m;
                best = cs[c];
            }
        }
    };
    sweep(cands, true);
    // then, with the best shape: the refill period, and in the box / bridge /
    // Gaussian kernel the form of the bridge test
    std::vector<pdd_tuning> more;
    for (int r : {1, 2, 4, 8})
        if (r != (dim == 2 ? 2 : 4)) {
            pdd_tuning t = best;
            t.refill = r;
            more.push_back(t);
        }
    if (spec)
        for (int b : {1, 2})
            if (b != (kind == kKernelDense ? 2 : 1)) {
                pdd_tuning t = best;
                t.bridge = b;
                more.push_back(t);
            }
    sweep(more, false);
    cleanup();
    if (st) return st;
    ctx->tuned[tuning_key(prec, dim, est, !spec)] = best;
    *out = best;
    return PDD_OK;
}

pdd_status pdd_stage2(pdd_problem *problem, const pdd_partition *part, const double *nodes, const double *values,
                      int64_t n_nodes, double *u, void *stream)
{
    if (!problem || !part || !u || (n_nodes > 0 && (!nodes || !values)))
        return fail(PDD_E_INVALID, "NULL argument");
    if (n_nodes < 0) return fail(PDD_E_INVALID, "n_nodes < 0");
    const pdd_problem_desc &d = problem->desc;
    if (d.dim != 2 || d.domain != PDD_DOMAIN_BOX)
        return fail(PDD_E_UNSUPPORTED, "the second stage takes 2D box domains");
    if (part->n[0] < 3 || part->n[1] < 3) return fail(PDD_E_INVALID, "the grid needs >= 3 points per axis");
    if (!(part->rbf_eps > 0.0) || !std::isfinite(part->rbf_eps))
        return fail(PDD_E_INVALID, "rbf_eps must be finite and > 0");
    const int n[2] = {part->n[0], part->n[1]};
    // interfaces: grid indices on each axis
    std::vector<int> cut_idx[2];
    std::vector<double> cut_pos[2];
    for (int a = 0; a < 2; ++a) {
        if (part->n_cuts[a] < 0 || (part->n_cuts[a] > 0 && !part->cuts[a]))
            return fail(PDD_E_INVALID, "bad interface list on axis %d", a);
        for (int q = 0; q < part->n_cuts[a]; ++q) {
            const double c = part->cuts[a][q];
            const double t = (c - d.lo[a]) * (double)(n[a] - 1) / (d.hi[a] - d.lo[a]);
            const double r = std::round(t);
            if (!std::isfinite(c) || std::fabs(t - r) > 1e-9 || r <= 0.0 || r >= (double)(n[a] - 1))
                return fail(PDD_E_INVALID, "interface %g on axis %d is not on an interior grid line", c, a);
            if (std::find(cut_idx[a].begin(), cut_idx[a].end(), (int)r) != cut_idx[a].end())
                return fail(PDD_E_INVALID, "interface %g on axis %d given twice", c, a);
            cut_idx[a].push_back((int)r);
            cut_pos[a].push_back(c);
        }
    }
    // nodes: each on at least one interface line
    auto on_line = [](double x, double c) { return std::fabs(x - c) <= 1e-9 * std::max(1.0, std::fabs(c)); };
    for (int64_t i = 0; i < n_nodes; ++i) {
        const double *x = nodes + 2 * i;
        if (!finite3(x, 2) || !strictly_inside(d, x) || !std::isfinite(values[i]))
            return fail(PDD_E_INVALID, "node %lld is not strictly inside the domain or its value is not finite",
                        (long long)i);
        bool any = false;
        for (int a = 0; a < 2 && !any; ++a)
            for (double c : cut_pos[a]) any = any || on_line(x[a], c);
        if (!any) return fail(PDD_E_INVALID, "node %lld lies on no interface", (long long)i);
    }
    // subdomains: the grid boxes between consecutive interfaces
    std::vector<int> ix = cut_idx[0], iy = cut_idx[1];
    std::sort(ix.begin(), ix.end());
    std::sort(iy.begin(), iy.end());
    ix.insert(ix.begin(), 0);
    ix.push_back(n[0] - 1);
    iy.insert(iy.begin(), 0);
    iy.push_back(n[1] - 1);
    std::vector<SubBox> boxes;
    uint64_t unknowns = 0, max_unknowns = 0;
    for (size_t a = 0; a + 1 < ix.size(); ++a)
        for (size_t b = 0; b + 1 < iy.size(); ++b) {
            SubBox bx{};
            bx.i0 = ix[a], bx.i1 = ix[a + 1], bx.j0 = iy[b], bx.j1 = iy[b + 1];
            const int mx = bx.i1 - bx.i0 - 1, my = bx.j1 - bx.j0 - 1;
            if (mx < 1 || my < 1) continue;
            bx.fast_x = mx <= my;
            bx.w = bx.fast_x ? mx : my;
            bx.L = bx.fast_x ? my : mx;
            if (bx.w > kStage2MaxBand)
                return fail(PDD_E_UNSUPPORTED, "subdomain of %d x %d interior points: the shorter side must be <= %d",
                            mx, my, kStage2MaxBand);
            bx.first = unknowns;
            unknowns += (uint64_t)mx * my;
            max_unknowns = std::max<uint64_t>(max_unknowns, (uint64_t)mx * my);
            boxes.push_back(bx);
        }
    pdd_ctx *ctx = problem->ctx;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipSetDevice(ctx->device));
    if (ctx->any_done) HIP_TRY(hipStreamWaitEvent(s, ctx->done, 0));
    Stage2Grid g{};
    g.u = u;
    g.n0 = n[0], g.n1 = n[1];
    g.lo0 = d.lo[0], g.lo1 = d.lo[1];
    g.span0 = d.hi[0] - d.lo[0], g.span1 = d.hi[1] - d.lo[1];
    g.dx0 = g.span0 / (n[0] - 1), g.dx1 = g.span1 / (n[1] - 1);
    g.half_s2 = 0.5 * d.sigma * d.sigma;
    // physical boundary first: the ends of every interface line carry g
    HIP_TRY(launch_stage2_boundary(problem->pd, g, s));
    const size_t grid_bytes = (size_t)n[0] * n[1] * sizeof(double);
    pdd_status st;
    if ((st = ensure_stage(ctx, grid_bytes))) return st;
    double *hg = static_cast<double *>(ctx->stage);
    HIP_TRY(hipMemcpyAsync(hg, u, grid_bytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    // multiquadric weights of every line (host: small dense systems)
    std::vector<Stage2Line> lines;
    std::vector<double> t_all, lam_all;
    for (int a = 0; a < 2; ++a)
        for (size_t q = 0; q < cut_pos[a].size(); ++q) {
            const int e = 1 - a, k = cut_idx[a][q];
            std::vector<double> t, z;
            t.push_back(d.lo[e]);
            z.push_back(a == 0 ? hg[k] : hg[(size_t)k * n[0]]);
            for (int64_t i = 0; i < n_nodes; ++i)
                if (on_line(nodes[2 * i + a], cut_pos[a][q])) {
                    t.push_back(nodes[2 * i + e]);
                    z.push_back(values[i]);
                }
            t.push_back(d.hi[e]);
            z.push_back(a == 0 ? hg[(size_t)(n[1] - 1) * n[0] + k] : hg[(size_t)k * n[0] + n[0] - 1]);
            const int m = (int)t.size();
            // Phi lam = z by Gaussian elimination with partial pivoting
            std::vector<double> M((size_t)m * m);
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < m; ++c) {
                    const double ee = part->rbf_eps * (t[r] - t[c]);
                    M[(size_t)r * m + c] = std::sqrt(1.0 + ee * ee);
                }
            std::vector<double> lam = z;
            for (int c = 0; c < m; ++c) {
                int p = c;
                for (int r = c + 1; r < m; ++r)
                    if (std::fabs(M[(size_t)r * m + c]) > std::fabs(M[(size_t)p * m + c])) p = r;
                if (M[(size_t)p * m + c] == 0.0)
                    return fail(PDD_E_INVALID, "interpolation system of interface %g is singular (repeated nodes?)",
                                cut_pos[a][q]);
                if (p != c) {
                    for (int cc = 0; cc < m; ++cc) std::swap(M[(size_t)p * m + cc], M[(size_t)c * m + cc]);
                    std::swap(lam[p], lam[c]);
                }
                for (int r = c + 1; r < m; ++r) {
                    const double l = M[(size_t)r * m + c] / M[(size_t)c * m + c];
                    for (int cc = c; cc < m; ++cc) M[(size_t)r * m + cc] -= l * M[(size_t)c * m + cc];
                    lam[r] -= l * lam[c];
                }
            }
            for (int r = m - 1; r >= 0; --r) {
                double acc = lam[r];
                for (int cc = r + 1; cc < m; ++cc) acc -= M[(size_t)r * m + cc] * lam[cc];
                lam[r] = acc / M[(size_t)r * m + r];
            }
            Stage2Line L{};
            L.d = a, L.k = k, L.m = m, L.at = t_all.size(), L.eps = part->rbf_eps;
            lines.push_back(L);
            t_all.insert(t_all.end(), t.begin(), t.end());
            lam_all.insert(lam_all.end(), lam.begin(), lam.end());
        }
    // the rows of every subdomain next to its boundary, and the layout of its
    // response columns (nb + 1 columns of its unknowns)
    std::vector<Stage2Resp> resp_tab(boxes.size());
    std::vector<uint32_t> rb;
    uint64_t resp_values = 0;
    int32_t max_cols = 0;
    bool use_resp = true;
    for (size_t q = 0; q < boxes.size(); ++q) {
        const SubBox &bx = boxes[q];
        const uint64_t nq = (uint64_t)bx.w * bx.L;
        resp_tab[q].rb_at = rb.size();
        for (uint64_t r = 0; r < nq; ++r) {
            const int sl = (int)(r / bx.w), f = (int)(r % bx.w);
            const int i = bx.i0 + 1 + (bx.fast_x ? f : sl), j = bx.j0 + 1 + (bx.fast_x ? sl : f);
            if (i - 1 == bx.i0 || i + 1 == bx.i1 || j - 1 == bx.j0 || j + 1 == bx.j1) rb.push_back((uint32_t)r);
        }
        resp_tab[q].nb = (int32_t)(rb.size() - resp_tab[q].rb_at);
        resp_tab[q].out_at = resp_values;
        resp_values += (uint64_t)(resp_tab[q].nb + 1) * nq;
        max_cols = std::max(max_cols, resp_tab[q].nb + 1);
        use_resp = use_resp && resp_tab[q].nb <= kStage2MaxBoundaryRows;
    }
    // response columns up to 2 GiB; beyond, every call substitutes (as every
    // call does with PDD_STAGE2_SUBSTITUTE=1 in the environment, which the
    // tests use to check the two ways against each other)
    const char *force_subst = std::getenv("PDD_STAGE2_SUBSTITUTE");
    use_resp = use_resp && resp_values * sizeof(double) <= (2ull << 30) &&
               !(force_subst && force_subst[0] == '1');
    // device tables: lines | t | lam | boxes | response layout | boundary rows | stencils | aux
    const size_t off_lines = 0;
    const size_t off_t = align_up(off_lines + lines.size() * sizeof(Stage2Line), 256);
    const size_t off_lam = align_up(off_t + t_all.size() * sizeof(double), 256);
    const size_t off_boxes = align_up(off_lam + lam_all.size() * sizeof(double), 256);
    const size_t off_resp = align_up(off_boxes + boxes.size() * sizeof(SubBox), 256);
    const size_t off_rb = align_up(off_resp + resp_tab.size() * sizeof(Stage2Resp), 256);
    const size_t table_bytes = align_up(off_rb + rb.size() * sizeof(uint32_t), 256);
    const size_t off_stencil = table_bytes;
    const size_t off_aux = align_up(off_stencil + unknowns * 6 * sizeof(double), 256);
    const size_t bytes = off_aux + unknowns * 2 * sizeof(double);
    if ((st = ensure(ctx, ctx->stage2, bytes))) return st;
    // the subdomain matrices depend on the operator (sigma, b, c), the grid
    // and the interfaces: factored already when the last call had the same
    std::vector<double> key = {(double)d.dim, d.lo[0], d.lo[1], d.hi[0], d.hi[1], d.sigma, d.b0[0], d.b0[1],
                               d.B[0][0], d.B[0][1], d.B[1][0], d.B[1][1], d.c_a, d.c_b,
                               (problem->pd.tab & 15u) ? (double)problem->serial : -1.0, (double)n[0], (double)n[1]};
    for (int a = 0; a < 2; ++a) {
        key.push_back((double)cut_pos[a].size());
        key.insert(key.end(), cut_pos[a].begin(), cut_pos[a].end());
    }
    const size_t lu_bytes = unknowns * (2 * kStage2MaxBand + 2) * sizeof(double);
    const bool factored = ctx->stage2_key == key && ctx->stage2_lu.ptr && ctx->stage2_lu.cap >= lu_bytes;
    if (!factored) {
        ctx->stage2_key.clear();
        if ((st = ensure(ctx, ctx->stage2_lu, lu_bytes))) return st;
    }
    double *d_factor = static_cast<double *>(ctx->stage2_lu.ptr);
    double *d_lmul = d_factor + unknowns * (kStage2MaxBand + 2);
    // the response columns depend on the factors and on f: the factors' key
    // and the problem
    std::vector<double> resp_key = key;
    resp_key.push_back((double)problem->serial);
    const size_t resp_bytes = resp_values * sizeof(double);
    bool resp_ready = false;
    if (use_resp) {
        resp_ready = factored && ctx->stage2_resp_key == resp_key && ctx->stage2_resp.ptr &&
                     ctx->stage2_resp.cap >= resp_bytes;
        if (!resp_ready) {
            ctx->stage2_resp_key.clear();
            if ((st = ensure(ctx, ctx->stage2_resp, resp_bytes))) return st;
        }
    }
    if ((st = ensure_stage(ctx, table_bytes))) return st;
    char *h = static_cast<char *>(ctx->stage);
    std::memcpy(h + off_lines, lines.data(), lines.size() * sizeof(Stage2Line));
    std::memcpy(h + off_t, t_all.data(), t_all.size() * sizeof(double));
    std::memcpy(h + off_lam, lam_all.data(), lam_all.size() * sizeof(double));
    std::memcpy(h + off_boxes, boxes.data(), boxes.size() * sizeof(SubBox));
    std::memcpy(h + off_resp, resp_tab.data(), resp_tab.size() * sizeof(Stage2Resp));
    std::memcpy(h + off_rb, rb.data(), rb.size() * sizeof(uint32_t));
    char *dv = static_cast<char *>(ctx->stage2.ptr);
    HIP_TRY(hipMemcpyAsync(dv, h, table_bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(ctx->staged, s));
    ctx->any_staged = true;
    HIP_TRY(launch_stage2_lines(g, reinterpret_cast<const Stage2Line *>(dv + off_lines), (int32_t)lines.size(),
                                reinterpret_cast<const double *>(dv + off_t),
                                reinterpret_cast<const double *>(dv + off_lam), s));
    Stage2Plan plan{};
    plan.factored = factored;
    if (use_resp) {
        plan.resp_tab = reinterpret_cast<const Stage2Resp *>(dv + off_resp);
        plan.rb = reinterpret_cast<const uint32_t *>(dv + off_rb);
        plan.resp = static_cast<double *>(ctx->stage2_resp.ptr);
        plan.max_cols = max_cols;
        plan.resp_ready = resp_ready;
    }
    HIP_TRY(launch_stage2_solve(problem->pd, g, reinterpret_cast<const SubBox *>(dv + off_boxes), (int32_t)boxes.size(),
                                (uint32_t)max_unknowns, reinterpret_cast<double *>(dv + off_stencil),
                                reinterpret_cast<double *>(dv + off_aux), d_factor, d_lmul, plan, s));
    ctx->stage2_key = key;
    if (use_resp) ctx->stage2_resp_key = resp_key;
    HIP_TRY(hipEventRecord(ctx->done, s));
    ctx->any_done = true;
    return PDD_OK;
}

pdd_status pdd_set_tuning(pdd_ctx *ctx, const pdd_tuning_key *key, const pdd_tuning *t)
{
    if (!ctx || !key) return fail(PDD_E_INVALID, "NULL argument");
    if ((key->precision != PDD_FP32 && key->precision != PDD_FP64) || key->dim < 2 || key->dim > 3 ||
        key->correction < 0 || key->correction > 2 || (key->generic != 0 && key->generic != 1))
        return fail(PDD_E_INVALID, "bad tuning key");
    const int k = tuning_key(key->precision, key->dim, key->correction, key->generic != 0);
    if (!t) {
        ctx->tuned.erase(k);
        return PDD_OK;
    }
    pdd_tuning v = *t;
    if (!v.block) v.block = 256;
    if (!v.grab) v.grab = 64;
    pdd_status st = check_tuning(v);
    if (st) return st;
    ctx->tuned[k] = v;
    return PDD_OK;
}

}  // extern "C"
