// k_kk.hip -- the Kramers-Kronig route (Sec. II: Re and Im of chi0 are connected by the
// Kramers-Kronig transformation; the usual practice computes Im alone and recovers Re from it on
// a frequency grid wide enough to hold the whole spectrum).
//
// Im chi0 on a uniform grid w'_k = lo + k h (k = 0..K-1) is taken as the piecewise-linear
// interpolant, zero one spacing beyond each end.  For it the principal value
//   Re chi0(w) = (1/pi) P int Im chi0(w') / (w' - w) dw'
// is exact: each tent k contributes Im_k L_k(w) with
//   L_k(w) = [phi(x + h) - 2 phi(x) + phi(x - h)] / h,   x = w'_k - w,   phi(x) = x ln|x|,
// evaluated for |x| > 2h as log1p(-t^2)/t + log1p(t) - log1p(-t), t = h/x (no cancellation).
#include "chi0_internal.h"

#include <math.h>

namespace chi0 {

namespace {

__device__ __forceinline__ double phi(double x) { return x == 0.0 ? 0.0 : x * log(fabs(x)); }

__device__ __forceinline__ double tent_kernel(double x, double h)
{
    if (fabs(x) > 2.0 * h) {
        const double t = h / x;
        return log1p(-t * t) / t + log1p(t) - log1p(-t);
    }
    return (phi(x + h) - 2.0 * phi(x) + phi(x - h)) / h;
}

__global__ __launch_bounds__(256) void kk_grid_kernel(double lo, double h, int K, const double *__restrict__ omega,
                                                      int nw, double *__restrict__ omega_all)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < K) omega_all[i] = lo + (double)i * h;
    else if (i < K + nw) omega_all[i] = omega[i - K];
}

__global__ __launch_bounds__(256) void kk_transform_kernel(const double *__restrict__ im_all, int K, int nw, double lo,
                                                           double h, const double *__restrict__ omega,
                                                           double *__restrict__ out, int64_t out_stride)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (i >= nw) return;
    const double w = omega[i];
    const double *im = im_all + (int64_t)q * (K + nw) * 2;
    double re = 0.0;
    for (int k = 0; k < K; ++k) {
        const double v = im[2 * k + 1];
        if (v != 0.0) re = fma(v, tent_kernel(lo + (double)k * h - w, h), re);
    }
    out[(int64_t)q * out_stride + 2 * i] = re * (1.0 / 3.14159265358979323846);
    out[(int64_t)q * out_stride + 2 * i + 1] = im[2 * (K + i) + 1];
}

}  // namespace

hipError_t launch_kk_grid(double lo, double h, int K, const double *omega, int nw, double *omega_all, hipStream_t s)
{
    if (K < 2 || nw < 1) return hipErrorInvalidValue;
    const int n = K + nw;
    hipLaunchKernelGGL(kk_grid_kernel, dim3((n + 255) / 256), dim3(256), 0, s, lo, h, K, omega, nw, omega_all);
    return hipGetLastError();
}

hipError_t launch_kk_transform(const double *im_all, int nq, int K, int nw, double lo, double h, const double *omega,
                               double *out, int64_t out_stride, hipStream_t s)
{
    if (K < 2 || nw < 1 || nq < 1) return hipErrorInvalidValue;
    dim3 grid((nw + 255) / 256, nq), block(256);
    hipLaunchKernelGGL(kk_transform_kernel, grid, block, 0, s, im_all, K, nw, lo, h, omega, out, out_stride);
    return hipGetLastError();
}

}  // namespace chi0
