// k_tetra_dyn.hip -- the dynamic tetrahedron kernel (K_B) instantiated for mesh plans, and its
// launcher (list plans are instantiated in k_tetra_list.hip).
#include "k_tetra.h"

namespace chi0 {

hipError_t launch_tetra_dynamic(const MeshDev &mesh, const BatchDev &batch, int nq, int nblocks,
                                const double *omega, int nw, double *partial, bool mixed, hipStream_t s)
{
    if (nw < 1 || nw > kMaxOmegaPerLaunch || nq < 1 || nq > kMaxQBatch) return hipErrorInvalidValue;
    if (hipError_t e = launch_band_range(mesh, batch, nq, s); e != hipSuccess) return e;
    dim3 grid(nblocks, nq), block(kWave);
    int slots = (nw + kWave - 1) / kWave;
    if (mesh.tets) return launch_tetra_dynamic_list(mesh, batch, nq, nblocks, omega, nw, partial, mixed, s);
    switch (slots * 2 + (mixed ? 1 : 0)) {
#define C0_CASE(S)                                                                                        \
    case 2 * S:                                                                                           \
        hipLaunchKernelGGL((tetra_dynamic_kernel<S, false, false>), grid, block, 0, s, mesh, batch, nblocks, \
                           omega, nw, partial);                                                           \
        break;                                                                                            \
    case 2 * S + 1:                                                                                       \
        hipLaunchKernelGGL((tetra_dynamic_kernel<S, true, false>), grid, block, 0, s, mesh, batch, nblocks,  \
                           omega, nw, partial);                                                           \
        break;
        C0_CASE(1) C0_CASE(2) C0_CASE(3) C0_CASE(4) C0_CASE(5) C0_CASE(6) C0_CASE(7) C0_CASE(8)
#undef C0_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_tetra_dynamic_pairs(const MeshDev &mesh, const BatchDev &batch, int nq, int nblk,
                                      const double *omega, int nw, double *partial, bool mixed, hipStream_t s)
{
    if (nw < 1 || nw > kMaxOmegaPerLaunch || nq < 1 || nq > kMaxQBatch || nblk < 1 || mesh.tets)
        return hipErrorInvalidValue;
    if (hipError_t e = launch_band_range(mesh, batch, nq, s); e != hipSuccess) return e;
    const int64_t nx = (int64_t)mesh.nbw * mesh.nbw * nblk;
    if (nx >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    dim3 grid((unsigned)nx, nq), block(kWave);
    const int slots = (nw + kWave - 1) / kWave;
    switch (slots * 2 + (mixed ? 1 : 0)) {
#define C0_CASE(S)                                                                                        \
    case 2 * S:                                                                                           \
        hipLaunchKernelGGL((tetra_dynamic_pairs_kernel<S, false>), grid, block, 0, s, mesh, batch, nblk, omega, nw, \
                           partial);                                                                      \
        break;                                                                                            \
    case 2 * S + 1:                                                                                       \
        hipLaunchKernelGGL((tetra_dynamic_pairs_kernel<S, true>), grid, block, 0, s, mesh, batch, nblk, omega, nw, \
                           partial);                                                                      \
        break;
        C0_CASE(1) C0_CASE(2) C0_CASE(3) C0_CASE(4) C0_CASE(5) C0_CASE(6) C0_CASE(7) C0_CASE(8)
#undef C0_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace chi0
