// k_reduce.hip -- deterministic final reduction (K_R).
// out[q * out_stride + v] = scale * sum_b partial[(q * nblocks + b) * nvals + v], with the
// blocks added in increasing order, so repeated runs give bitwise-identical chi0.
#include "chi0_internal.h"

namespace chi0 {

namespace {

__global__ __launch_bounds__(256) void reduce_kernel(const double *__restrict__ partial, int nblocks, int nvals,
                                                     double scale, double *__restrict__ out, int64_t out_stride)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (v >= nvals) return;
    const double *p = partial + (int64_t)q * nblocks * nvals + v;
    // four independent running sums (fixed assignment b % 4) combined in a fixed order
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int b = 0;
    for (; b + 4 <= nblocks; b += 4) {
        s0 += p[(int64_t)(b + 0) * nvals];
        s1 += p[(int64_t)(b + 1) * nvals];
        s2 += p[(int64_t)(b + 2) * nvals];
        s3 += p[(int64_t)(b + 3) * nvals];
    }
    for (; b < nblocks; ++b) s0 += p[(int64_t)b * nvals];
    out[(int64_t)q * out_stride + v] = scale * ((s0 + s1) + (s2 + s3));
}

}  // namespace

hipError_t launch_reduce(const double *partial, int nq, int nblocks, int nvals, double scale, double *out,
                         int64_t out_stride, hipStream_t s)
{
    if (nq < 1 || nblocks < 1 || nvals < 1) return hipErrorInvalidValue;
    dim3 grid((nvals + 255) / 256, nq), block(256);
    hipLaunchKernelGGL(reduce_kernel, grid, block, 0, s, partial, nblocks, nvals, scale, out, out_stride);
    return hipGetLastError();
}

}  // namespace chi0
