// k_tetra_list.hip -- the dynamic tetrahedron kernel (K_B) instantiated for tetrahedron-list plans.
#include "k_tetra.h"

namespace chi0 {

hipError_t launch_tetra_dynamic_list(const MeshDev &mesh, const BatchDev &batch, int nq, int nblocks,
                                     const double *omega, int nw, double *partial, bool mixed, hipStream_t s)
{
    if (nw < 1 || nw > kMaxOmegaPerLaunch || nq < 1 || nq > kMaxQBatch || !mesh.tets) return hipErrorInvalidValue;
    dim3 grid(nblocks, nq), block(kWave);
    int slots = (nw + kWave - 1) / kWave;
    // slot counts 1, 2, 4, 8 (a kernel with more slots than frequencies idles the extra ones)
    slots = slots <= 1 ? 1 : slots <= 2 ? 2 : slots <= 4 ? 4 : 8;
    switch (slots * 2 + (mixed ? 1 : 0)) {
#define C0_LIST(S)                                                                                        \
    case 2 * S:                                                                                           \
        hipLaunchKernelGGL((tetra_dynamic_kernel<S, false, true>), grid, block, 0, s, mesh, batch, nblocks, \
                           omega, nw, partial);                                                           \
        break;                                                                                            \
    case 2 * S + 1:                                                                                       \
        hipLaunchKernelGGL((tetra_dynamic_kernel<S, true, true>), grid, block, 0, s, mesh, batch, nblocks,  \
                           omega, nw, partial);                                                           \
        break;
        C0_LIST(1) C0_LIST(2) C0_LIST(4) C0_LIST(8)
#undef C0_LIST
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace chi0
