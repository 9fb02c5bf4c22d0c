// k_tetra_batch.hip -- the fused tetrahedron launch of the batched form (K_B over a table of
// (instance, q, frequency-chunk) items).
#include "k_tetra.h"

namespace chi0 {

namespace {

// Fused launch over the (instance, q) items of a batch: workgroup -> item from a table, then the
// item's own frequency count and precision select the instantiation.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void tetra_batch_kernel(const BatchItemDev *__restrict__ items,
                                                         const int32_t *__restrict__ block_item)
{
    // one list buffer for both forms, sized for the larger FP64 record
    __shared__ __attribute__((aligned(16))) unsigned char lbuf[kCapDyn * sizeof(DynRec<false>)];
    __shared__ __attribute__((aligned(16))) uint16_t queue[kQCap][kWave];
    static_assert(sizeof(DynRec<true>) <= sizeof(DynRec<false>), "mixed records fit the FP64 buffer");
    DynRec<false> *list = reinterpret_cast<DynRec<false> *>(lbuf);
    DynRec<true> *list32 = reinterpret_cast<DynRec<true> *>(lbuf);
    const BatchItemDev it = items[block_item[blockIdx.x]];
    const int blk = blockIdx.x - it.kb_begin;
    double *part = it.partial + (int64_t)blk * it.nw * 2;
    const int slots = (it.nw + kWave - 1) / kWave;
    switch (slots * 2 + (it.precision != 0 ? 1 : 0)) {
#define C0_CASE(S)                                                                                        \
    case 2 * S:                                                                                           \
        dynamic_body<S, false, false>(it.M, it.Q, it.nblocks, blk, it.omega, it.nw, part, list, queue);          \
        break;                                                                                            \
    case 2 * S + 1:                                                                                       \
        dynamic_body<S, true, false>(it.M, it.Q, it.nblocks, blk, it.omega, it.nw, part, list32, queue);         \
        break;
        C0_CASE(1) C0_CASE(2) C0_CASE(3) C0_CASE(4) C0_CASE(5) C0_CASE(6) C0_CASE(7) C0_CASE(8)
#undef C0_CASE
    default: break;
    }
}

}  // namespace

hipError_t launch_tetra_batch(const BatchItemDev *items, const int32_t *block_item, int nblocks_total, hipStream_t s)
{
    if (nblocks_total < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(tetra_batch_kernel, dim3(nblocks_total), dim3(kWave), 0, s, items, block_item);
    return hipGetLastError();
}

}  // namespace chi0
