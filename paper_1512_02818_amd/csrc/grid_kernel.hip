// Gradient of a gridded function by second-order finite differences: the
// grad(u~) grids of the pathwise control variate (eq. F:xiControlVariate) when
// only values of u~ on a grid are known, as inside the outer iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "host_runtime.hpp"
#include "pdd.h"

using pdd::fail;

namespace {

// Derivative along one axis at a point whose index along that axis is a (of
// n): central inside, three-point one-sided at the two ends; s is the
// point's stride along the axis, two_dx twice the spacing.
template <class S>
__device__ __forceinline__ S axis_derivative(const S *__restrict__ u, uint64_t p, uint64_t s, int a, int n, S two_dx)
{
    if (a == 0) return ((S)-3 * u[p] + (S)4 * u[p + s] - u[p + 2 * s]) / two_dx;
    if (a == n - 1) return ((S)3 * u[p] - (S)4 * u[p - s] + u[p - 2 * s]) / two_dx;
    return (u[p + s] - u[p - s]) / two_dx;
}

// One thread per grid point (x fastest, so neighbouring threads read
// neighbouring values), all dim components.
template <class S, int D>
__global__ void grid_gradient_kernel(const S *__restrict__ u, int n0, int n1, int n2, S dx0, S dx1, S dx2,
                                     S *__restrict__ g0, S *__restrict__ g1, S *__restrict__ g2)
{
    const uint64_t m01 = (uint64_t)n0 * n1;
    const uint64_t total = m01 * (D == 3 ? (uint64_t)n2 : 1);
    for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < total;
         p += (uint64_t)gridDim.x * blockDim.x) {
        const int i = (int)(p % n0), j = (int)((p / n0) % n1);
        g0[p] = axis_derivative<S>(u, p, 1, i, n0, dx0);
        g1[p] = axis_derivative<S>(u, p, (uint64_t)n0, j, n1, dx1);
        if (D == 3) g2[p] = axis_derivative<S>(u, p, m01, (int)(p / m01), n2, dx2);
    }
}

template <class S, int D>
hipError_t launch_gradient(const pdd_grid *g, void *const *out, hipStream_t s)
{
    const int n2 = D == 3 ? g->n[2] : 1;
    const uint64_t total = (uint64_t)g->n[0] * g->n[1] * n2;
    const uint64_t blocks = std::min<uint64_t>((total + 255) / 256, 16384);
    S two_dx[3] = {0, 0, 0};
    for (int d = 0; d < D; ++d) two_dx[d] = (S)(2.0 * ((g->hi[d] - g->lo[d]) / (g->n[d] - 1)));
    hipLaunchKernelGGL((grid_gradient_kernel<S, D>), dim3((uint32_t)blocks), dim3(256), 0, s,
                       static_cast<const S *>(g->data), g->n[0], g->n[1], n2, two_dx[0], two_dx[1], two_dx[2],
                       static_cast<S *>(out[0]), static_cast<S *>(out[1]), static_cast<S *>(D == 3 ? out[2] : out[1]));
    return hipGetLastError();
}

}  // namespace

extern "C" pdd_status pdd_grid_residual(pdd_problem *problem, const pdd_grid *u, void *resid, void *stream)
{
    if (!problem || !u || !resid) return fail(PDD_E_INVALID, "NULL argument");
    const int D = u->dim;
    if (D != problem->desc.dim) return fail(PDD_E_INVALID, "grid dim %d != problem dim %d", D, problem->desc.dim);
    if (!u->data) return fail(PDD_E_INVALID, "grid has no data");
    if (u->dtype != PDD_DTYPE_F32 && u->dtype != PDD_DTYPE_F64) return fail(PDD_E_INVALID, "bad grid dtype");
    for (int d = 0; d < D; ++d) {
        if (u->n[d] < 4) return fail(PDD_E_INVALID, "second derivatives at the edges need n >= 4 per axis");
        if (!(u->hi[d] > u->lo[d]) || !std::isfinite(u->hi[d] - u->lo[d]))
            return fail(PDD_E_INVALID, "grid needs finite lo < hi");
    }
    if ((uint64_t)u->n[0] * u->n[1] * (D == 3 ? (uint64_t)u->n[2] : 1) >= (1ull << 40))
        return fail(PDD_E_INVALID, "grid too large");
    HIP_TRY(hipSetDevice(problem->ctx->device));
    const hipError_t e = pdd::launch_grid_residual(problem->pd, problem->desc.sigma, u, resid,
                                                   static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(PDD_E_HIP, "grid residual launch: %s", hipGetErrorString(e));
    return PDD_OK;
}

extern "C" pdd_status pdd_grid_gradient(pdd_ctx *ctx, const pdd_grid *u, void *const *grad, void *stream)
{
    if (!ctx || !u || !grad) return fail(PDD_E_INVALID, "NULL argument");
    const int D = u->dim;
    if (D != 2 && D != 3) return fail(PDD_E_INVALID, "grid dim must be 2 or 3");
    if (!u->data) return fail(PDD_E_INVALID, "grid has no data");
    if (u->dtype != PDD_DTYPE_F32 && u->dtype != PDD_DTYPE_F64) return fail(PDD_E_INVALID, "bad grid dtype");
    for (int d = 0; d < D; ++d) {
        if (u->n[d] < 3) return fail(PDD_E_INVALID, "second-order differences need n >= 3 per axis");
        if (!(u->hi[d] > u->lo[d]) || !std::isfinite(u->hi[d] - u->lo[d]))
            return fail(PDD_E_INVALID, "grid needs finite lo < hi");
        if (!grad[d]) return fail(PDD_E_INVALID, "gradient buffer %d is NULL", d);
    }
    if ((uint64_t)u->n[0] * u->n[1] * (D == 3 ? (uint64_t)u->n[2] : 1) >= (1ull << 40))
        return fail(PDD_E_INVALID, "grid too large");
    HIP_TRY(hipSetDevice(ctx->device));
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (u->dtype == PDD_DTYPE_F32)
        e = D == 2 ? launch_gradient<float, 2>(u, grad, s) : launch_gradient<float, 3>(u, grad, s);
    else
        e = D == 2 ? launch_gradient<double, 2>(u, grad, s) : launch_gradient<double, 3>(u, grad, s);
    if (e != hipSuccess) return fail(PDD_E_HIP, "grid gradient launch: %s", hipGetErrorString(e));
    return PDD_OK;
}
