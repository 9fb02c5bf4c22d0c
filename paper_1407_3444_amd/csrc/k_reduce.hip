// k_reduce.hip -- deterministic final reduction (K_R).
// out[q * out_stride + v] = scale * sum_b partial[(q * nblocks + b) * nvals + v], with the
// blocks added in a fixed order (four quarters of the block range, each in increasing order),
// so repeated runs give bitwise-identical chi0.  A sum over
// a group of q-entries (the point-group loop) is the same sum over the group's consecutive
// blocks, added to the earlier launches' result when a group spans several launches.
#include "chi0_internal.h"

namespace chi0 {

namespace {

__device__ __forceinline__ double ordered_sum(const double *__restrict__ p, int nblocks, int nvals)
{
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
    return (s0 + s1) + (s2 + s3);
}

__global__ __launch_bounds__(256) void reduce_batch_kernel(const BatchItemDev *__restrict__ items,
                                                           const int32_t *__restrict__ block_item)
{
    const BatchItemDev it = items[block_item[blockIdx.x]];
    const int nvals = 2 * it.nw;
    const int v = (blockIdx.x - it.kr_begin) * blockDim.x + threadIdx.x;
    if (v >= nvals) return;
    it.out[v] = it.scale * ordered_sum(it.partial + v, it.nblocks, nvals);
}

// A workgroup takes 64 consecutive values of one q; its 4 waves sum the quarters of the block
// range (each in block order, four running sums), and wave 0 adds the quarters in order.
// accumulate: add to what out holds (the earlier parts of a sum split over launches) instead of
// overwriting it.
constexpr int kReduceVals = 64;
constexpr int kReduceSlices = 4;

__global__ __launch_bounds__(kReduceVals * kReduceSlices) void reduce_kernel(
    const double *__restrict__ partial, int nblocks, int nvals, double scale, double *__restrict__ out,
    int64_t out_stride, int accumulate)
{
    __shared__ double quarter[kReduceSlices][kReduceVals];
    const int lane = threadIdx.x % kReduceVals, slice = threadIdx.x / kReduceVals;
    const int v = blockIdx.x * kReduceVals + lane;
    const int q = blockIdx.y;
    const int per = (nblocks + kReduceSlices - 1) / kReduceSlices;
    const int b0 = min(nblocks, slice * per), b1 = min(nblocks, b0 + per);
    double s = 0.0;
    if (v < nvals && b1 > b0)
        s = ordered_sum(partial + ((int64_t)q * nblocks + b0) * nvals + v, b1 - b0, nvals);
    quarter[slice][lane] = s;
    __syncthreads();
    if (slice != 0 || v >= nvals) return;
    const double t = scale * ((quarter[0][lane] + quarter[1][lane]) + (quarter[2][lane] + quarter[3][lane]));
    double *o = out + (int64_t)q * out_stride + v;
    *o = accumulate ? *o + t : t;
}

}  // namespace

hipError_t launch_reduce_batch(const BatchItemDev *items, const int32_t *block_item, int nblocks_total,
                               hipStream_t s)
{
    if (nblocks_total < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(reduce_batch_kernel, dim3(nblocks_total), dim3(256), 0, s, items, block_item);
    return hipGetLastError();
}

hipError_t launch_reduce(const double *partial, int nq, int nblocks, int nvals, double scale, double *out,
                         int64_t out_stride, hipStream_t s, bool accumulate)
{
    if (nq < 1 || nblocks < 1 || nvals < 1) return hipErrorInvalidValue;
    dim3 grid((nvals + kReduceVals - 1) / kReduceVals, nq), block(kReduceVals * kReduceSlices);
    hipLaunchKernelGGL(reduce_kernel, grid, block, 0, s, partial, nblocks, nvals, scale, out, out_stride,
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

}  // namespace chi0
