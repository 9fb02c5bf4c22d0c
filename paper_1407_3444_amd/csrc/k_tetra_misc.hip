// k_tetra_misc.hip -- the static, pair-resolved static, imaginary-part (Kramers-Kronig route) and
// census instantiations of the tetrahedron kernel (K_B).
#include "k_tetra.h"

namespace chi0 {

namespace {

// Three waves per SIMD: the static evaluation fits 168 VGPRs with a few spills outside its loops,
// and its 12 KiB list leaves LDS for twelve workgroups per CU (12% faster than two waves).
template <bool LIST>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void tetra_static_kernel(MeshDev M, BatchDev B, int nblocks,
                                                          double *__restrict__ partial)
{
    __shared__ StatRec list[kCapStat];
    const int qi = blockIdx.y;
    const int64_t n_units = tets_per_pair(M) * M.nbw * M.nbw;
    const double acc = static_body<LIST>(M, B.q[qi], 0, n_units, blockIdx.x, nblocks, list);
    if (threadIdx.x == 0) partial[(int64_t)qi * nblocks + blockIdx.x] = acc;
}

// Imaginary part alone (tetrahedron delta weights, for the Kramers-Kronig route): every
// (final tetrahedron, frequency) pair with the frequency strictly inside the tetrahedron's range
// of D values is queued and evaluated without logarithms (near_im); outside that range the
// imaginary part vanishes exactly, so nothing else is evaluated.  Up to 16 slots (1024
// frequencies) per launch.
struct ImRec {
    double y[4];                // D at the corners (sorted ascending after the prep pass)
    double w[4];                // sign * volume * W
    double inv[6];              // reciprocals of the node spans (prep pass, im_span_rcp)
};
constexpr int kCapIm = 64;      // final tetrahedra per LDS list
static_assert(kCapIm >= kMaxRecsPerUnit, "a list must hold a whole unit");
constexpr int kQCapIm = 64;     // work items queued per lane

template <int NSLOT>
__device__ __forceinline__ void drain_im(const ImRec *list, uint16_t (*queue)[kWave], int &qn, int lane,
                                         const double *__restrict__ omega, double *acc)
{
    while (__any(qn > 0)) {
        if (qn > 0) {
            --qn;
            const int e = queue[qn][lane];
            const int r = e >> 5, s = e & 31;
            double y[4], w[4], inv[6];
#pragma unroll
            for (int k = 0; k < 4; ++k) { y[k] = list[r].y[k]; w[k] = list[r].w[k]; }
#pragma unroll
            for (int k = 0; k < 6; ++k) inv[k] = list[r].inv[k];
            const double v = near_im_spans(y, w, inv, omega[lane + kWave * s]);
            // into the accumulator of slot s: an FMA with a factor 1 or 0 per slot (exactly acc + v or
            // acc; only frequencies strictly inside a tetrahedron's range are queued, so v is finite)
#pragma unroll
            for (int ss = 0; ss < NSLOT; ++ss) acc[ss] = fma(s == ss ? 1.0 : 0.0, v, acc[ss]);
        }
    }
}

template <int NSLOT, bool LIST>
__global__ __launch_bounds__(64) void tetra_im_kernel(MeshDev M, BatchDev B, int nblocks,
                                                      const double *__restrict__ omega, int nw,
                                                      double *__restrict__ partial)
{
    __shared__ ImRec list[kCapIm];
    __shared__ uint16_t queue[kQCapIm][kWave];
    const int qi = blockIdx.y;
    const QDev Q = B.q[qi];
    const int lane = threadIdx.x;
    const int blk = blockIdx.x;
    const int64_t n_units = tets_per_pair(M) * M.nbw * M.nbw;
    double om[NSLOT], acc[NSLOT];
    bool live[NSLOT];
    double wlo = omega[nw - 1], whi = wlo;
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
        const int idx = lane + kWave * s;
        live[s] = idx < nw;
        om[s] = omega[live[s] ? idx : nw - 1];
        acc[s] = 0.0;
        wlo = fmin(wlo, om[s]);
        whi = fmax(whi, om[s]);
    }
    wlo = wave_min(wlo);
    whi = wave_max(whi);
    int qn = 0;
    const PairMask pm = pair_mask(M, Q, lane);
    for (int64_t base = (int64_t)blk * kWave; base < n_units; base += (int64_t)nblocks * kWave) {
        const UnitIdx b0 = decode_unit<LIST>(M, base);
        if (round_inert<LIST>(M, pm, b0)) continue;
        const UnitIdx ux = round_unit<LIST>(M, b0, lane);
        const bool valid = base + lane < n_units;
        int cnt = 0;
        if (valid) {
            Vtx t[4];
            load_unit<LIST>(M, Q, ux, t);
            cnt = count_unit(t, M.form);
        }
        int start = 0;
        while (start < kWave) {
            int next;
            const int nrec = fill_list<ImRec, kCapIm, LIST>(M, Q, ux, valid, cnt, start, lane, list, next);
            start = next;
            if (nrec == 0) continue;
            __syncthreads();
            for (int r = lane; r < nrec; r += kWave) {
                double y[4] = {list[r].y[0], list[r].y[1], list[r].y[2], list[r].y[3]};
                double w[4] = {list[r].w[0], list[r].w[1], list[r].w[2], list[r].w[3]};
                sort4(y, w);
                double inv[6];
                im_span_rcp(y, inv);
#pragma unroll
                for (int k = 0; k < 4; ++k) { list[r].y[k] = y[k]; list[r].w[k] = w[k]; }
#pragma unroll
                for (int k = 0; k < 6; ++k) list[r].inv[k] = inv[k];
            }
            __syncthreads();
            for (int r = 0; r < nrec; ++r) {
                const double y0 = list[r].y[0], y3 = list[r].y[3];
                // wave-uniform: the tetrahedron's D range misses every frequency of the launch
                if (__builtin_amdgcn_readfirstlane(y0 < whi && y3 > wlo ? 1 : 0) == 0) continue;
#pragma unroll
                for (int s = 0; s < NSLOT; ++s) {
                    if (live[s] && y0 < om[s] && om[s] < y3) {
                        queue[qn][lane] = (uint16_t)((r << 5) | s);
                        ++qn;
                    }
                }
                if (__any(qn > kQCapIm - NSLOT)) drain_im<NSLOT>(list, queue, qn, lane, omega, acc);
            }
            drain_im<NSLOT>(list, queue, qn, lane, omega, acc);
            __syncthreads();
        }
    }
    double *part = partial + ((int64_t)qi * nblocks + blk) * nw * 2;
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
        const int idx = lane + kWave * s;
        if (idx < nw) {
            part[2 * idx] = 0.0;
            part[2 * idx + 1] = acc[s];
        }
    }
}

// Band-pair resolved static evaluation: workgroup x = p * nblk + j takes the units of pair p
// (its tetrahedra: consecutive units) as part j of nblk; partial[q][j][pair].
template <bool LIST>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void tetra_static_pairs_kernel(MeshDev M, BatchDev B, int nblk,
                                                                double *__restrict__ partial)
{
    __shared__ StatRec list[kCapStat];
    const int qi = blockIdx.y;
    const int npairs = M.nbw * M.nbw;
    const int p = blockIdx.x / nblk, j = blockIdx.x - p * nblk;
    const int64_t per_pair = tets_per_pair(M);
    const double acc = static_body<LIST>(M, B.q[qi], (int64_t)p * per_pair, (int64_t)(p + 1) * per_pair, j, nblk, list);
    if (threadIdx.x == 0) partial[((int64_t)qi * nblk + j) * npairs + p] = acc;
}

// Work census (diagnostic, untimed): the dynamic evaluation itself (8 slots, so up to
// kMaxOmegaPerLaunch frequencies), instantiated with counters: units with a non-empty carved
// region, final tetrahedra, (final tetrahedron, frequency) evaluations of the near branch, far
// evaluations (one per tetrahedron and frequency on the per-tetrahedron path, one per list and
// frequency where a whole list is evaluated as one series), the series terms they use, and the
// near evaluations repeated in full because an entry's nodes cluster (FP64 form).
template <bool MIXED, bool LIST>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void census_kernel(
    MeshDev M, BatchDev B, int nblocks, const double *__restrict__ omega, int nw, double *__restrict__ partial,
    int count_tets, unsigned long long *__restrict__ counts)
{
    __shared__ DynRec<MIXED> list[kCapDyn];
    __shared__ __attribute__((aligned(16))) uint16_t queue[kQCap][kWave];
    const int qi = blockIdx.y;
    WorkCount wc = {0, 0, 0, 0, 0, 0, 0};
    dynamic_body<8, MIXED, LIST, true>(M, B.q[qi], nblocks, blockIdx.x, omega, nw,
                                       partial + ((int64_t)qi * nblocks + blockIdx.x) * nw * 2, list, queue, &wc,
                                       count_tets != 0);
    if (threadIdx.x == 0) {
        atomicAdd(&counts[0], wc.units);
        atomicAdd(&counts[1], wc.tets);
        atomicAdd(&counts[2], wc.near);
        atomicAdd(&counts[3], wc.far);
        atomicAdd(&counts[4], wc.terms);
        atomicAdd(&counts[5], wc.redo);
        atomicAdd(&counts[6], wc.coef);
    }
}

// Minimum and maximum of each window band's energies over all k-points of the arrays: workgroup
// (b, 0) reduces band b of e(k) into rng_k, workgroup (b, 1 + i) band b of q i's e(k+q) into its
// rng_kq (a mesh shift reads the plan's own energies).  NaN values are passed over.
constexpr int kRangeThreads = 256;

// out[0..1] = (min, max) of e[0..nk) by one workgroup of kRangeThreads.
__device__ __forceinline__ void band_range_one(const double *__restrict__ e, int64_t nk, double *out)
{
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t k = threadIdx.x; k < nk; k += kRangeThreads) {
        const double v = e[k];
        lo = fmin(lo, v);
        hi = fmax(hi, v);
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    __shared__ double slo[kRangeThreads / kWave], shi[kRangeThreads / kWave];
    const int w = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0) {
        slo[w] = lo;
        shi[w] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kRangeThreads / kWave; ++i) {
            lo = fmin(lo, slo[i]);
            hi = fmax(hi, shi[i]);
        }
        out[0] = lo;
        out[1] = hi;
    }
}

__global__ __launch_bounds__(kRangeThreads) void band_range_kernel(MeshDev M, BatchDev B)
{
    const int b = blockIdx.x, src = blockIdx.y;
    const double *e = (src == 0 ? M.eps_k : B.q[src - 1].eps_kq) + (int64_t)(M.lo + b) * M.nk;
    band_range_one(e, M.nk, (src == 0 ? B.q[0].rng_k : B.q[src - 1].rng_kq) + 2 * b);
}

// Batched form: workgroup (2 g + src, b) takes band b of group g's e(k) (src 0) or e(k+q) (src 1).
__global__ __launch_bounds__(kRangeThreads) void band_range_batch_kernel(const BatchItemDev *__restrict__ items,
                                                                         const int32_t *__restrict__ group_item)
{
    const int b = blockIdx.y, src = blockIdx.x & 1;
    const BatchItemDev &it = items[group_item[blockIdx.x >> 1]];
    if (b >= it.M.nbw) return;           // the whole workgroup: before any barrier
    const double *e = (src == 0 ? it.M.eps_k : it.Q.eps_kq) + (int64_t)(it.M.lo + b) * it.M.nk;
    band_range_one(e, it.M.nk, (src == 0 ? it.Q.rng_k : it.Q.rng_kq) + 2 * b);
}

}  // namespace

hipError_t launch_band_range(const MeshDev &mesh, const BatchDev &batch, int nq, hipStream_t s)
{
    if (!batch.q[0].rng_k) return hipSuccess;
    if (nq < 1 || nq > kMaxQBatch || mesh.nbw < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(band_range_kernel, dim3(mesh.nbw, nq + 1), dim3(kRangeThreads), 0, s, mesh, batch);
    return hipGetLastError();
}

hipError_t launch_band_range_batch(const BatchItemDev *items, const int32_t *group_item, int ngroups, int max_nbw,
                                   hipStream_t s)
{
    if (ngroups < 1 || max_nbw < 1 || max_nbw > 65535 || ngroups > (1 << 30)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(band_range_batch_kernel, dim3(2 * ngroups, max_nbw), dim3(kRangeThreads), 0, s, items,
                       group_item);
    return hipGetLastError();
}

hipError_t launch_census(const MeshDev &mesh, const BatchDev &batch, int nq, int nblocks, const double *omega,
                         int nw, double *partial, bool mixed, bool first_chunk, unsigned long long *counts,
                         hipStream_t s)
{
    if (nq < 1 || nq > kMaxQBatch || nw < 1 || nw > kMaxOmegaPerLaunch || nblocks < 1) return hipErrorInvalidValue;
    if (hipError_t e = launch_band_range(mesh, batch, nq, s); e != hipSuccess) return e;
    dim3 grid(nblocks, nq), block(kWave);
    const int ct = first_chunk ? 1 : 0;
    if (mesh.tets) {
        if (mixed)
            hipLaunchKernelGGL((census_kernel<true, true>), grid, block, 0, s, mesh, batch, nblocks, omega, nw, partial,
                               ct, counts);
        else
            hipLaunchKernelGGL((census_kernel<false, true>), grid, block, 0, s, mesh, batch, nblocks, omega, nw,
                               partial, ct, counts);
    } else {
        if (mixed)
            hipLaunchKernelGGL((census_kernel<true, false>), grid, block, 0, s, mesh, batch, nblocks, omega, nw,
                               partial, ct, counts);
        else
            hipLaunchKernelGGL((census_kernel<false, false>), grid, block, 0, s, mesh, batch, nblocks, omega, nw,
                               partial, ct, counts);
    }
    return hipGetLastError();
}

hipError_t launch_tetra_im(const MeshDev &mesh, const BatchDev &batch, int nq, int nblocks, const double *omega,
                           int nw, double *partial, hipStream_t s)
{
    if (nw < 1 || nw > kMaxOmegaIm || nq < 1 || nq > kMaxQBatch || nblocks < 1) return hipErrorInvalidValue;
    if (hipError_t e = launch_band_range(mesh, batch, nq, s); e != hipSuccess) return e;
    dim3 grid(nblocks, nq), block(kWave);
    const bool list = mesh.tets != nullptr;
    if (nw <= 8 * kWave) {
        if (list)
            hipLaunchKernelGGL((tetra_im_kernel<8, true>), grid, block, 0, s, mesh, batch, nblocks, omega, nw, partial);
        else
            hipLaunchKernelGGL((tetra_im_kernel<8, false>), grid, block, 0, s, mesh, batch, nblocks, omega, nw, partial);
    } else {
        if (list)
            hipLaunchKernelGGL((tetra_im_kernel<16, true>), grid, block, 0, s, mesh, batch, nblocks, omega, nw, partial);
        else
            hipLaunchKernelGGL((tetra_im_kernel<16, false>), grid, block, 0, s, mesh, batch, nblocks, omega, nw, partial);
    }
    return hipGetLastError();
}

hipError_t launch_tetra_static_pairs(const MeshDev &mesh, const BatchDev &batch, int nq, int nblk, double *partial,
                                     hipStream_t s)
{
    if (nq < 1 || nq > kMaxQBatch || nblk < 1) return hipErrorInvalidValue;
    if (hipError_t e = launch_band_range(mesh, batch, nq, s); e != hipSuccess) return e;
    dim3 grid(nblk * mesh.nbw * mesh.nbw, nq), block(kWave);
    if (mesh.tets)
        hipLaunchKernelGGL(tetra_static_pairs_kernel<true>, grid, block, 0, s, mesh, batch, nblk, partial);
    else
        hipLaunchKernelGGL(tetra_static_pairs_kernel<false>, grid, block, 0, s, mesh, batch, nblk, partial);
    return hipGetLastError();
}

hipError_t launch_tetra_static(const MeshDev &mesh, const BatchDev &batch, int nq, int nblocks, double *partial,
                               hipStream_t s)
{
    if (nq < 1 || nq > kMaxQBatch) return hipErrorInvalidValue;
    if (hipError_t e = launch_band_range(mesh, batch, nq, s); e != hipSuccess) return e;
    dim3 grid(nblocks, nq), block(kWave);
    if (mesh.tets)
        hipLaunchKernelGGL(tetra_static_kernel<true>, grid, block, 0, s, mesh, batch, nblocks, partial);
    else
        hipLaunchKernelGGL(tetra_static_kernel<false>, grid, block, 0, s, mesh, batch, nblocks, partial);
    return hipGetLastError();
}

}  // namespace chi0
