// chi0_internal.h -- launch interfaces shared by the host library and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace chi0 {

constexpr int kMaxQBatch = 16;     // q-points handled by one launch of each kernel
constexpr int kWave = 64;
constexpr int kSlots = 8;          // frequencies per lane in the dynamic kernel (8 x 64 = 512)
constexpr int kMaxOmegaPerLaunch = kSlots * kWave;
constexpr int kMaxOmegaIm = 16 * kWave;   // frequencies per launch of the imaginary-part kernel
constexpr int kMaxOrbSmall = 64;          // orbital bases up to this size use the 16-k matrix-element tiles
constexpr int kMaxOrb = 16384;            // largest basis (plane waves) of the matrix elements

// Per-q data of one batch.
struct QDev {
    const double *eps_kq;   // [nb][Nk]: explicit k+q energies, or the mesh energies (shift mode)
    const double *c_kq;     // [Nk][no][nb] complex: explicit k+q eigenvectors, or the mesh ones
    double *W;              // [nbw][nbw][Nk] matrix elements of this q (null under CMA)
    int32_t shift[3];       // mesh shift (0 in explicit mode)
    int32_t explicit_kq;
    // Band ranges over all k-points of the arrays, [nbw][2] = (min, max) of the window's bands:
    // e(k) (shared by the q of a batch) and this q's e(k+q); filled by launch_band_range ahead of
    // the tetrahedron kernels, which then skip rounds of band pairs with no carved region.  Null:
    // no skipping.
    double *rng_k;
    double *rng_kq;
};

struct BatchDev {
    QDev q[kMaxQBatch];
};

struct MeshDev {
    int32_t n1, n2, n3;
    int32_t nb, no, lo, nbw;
    int32_t cma, form;
    int64_t nk;             // k-points of the arrays (the mesh, or the points of a tetrahedron list)
    double mu;
    const double *eps_k;    // [nb][Nk]
    const double *c_k;      // [Nk][no][nb] complex
    // Tetrahedra per band pair = nperm * ncell: the mesh's 6 Kuhn tetrahedra per cell (nperm 6,
    // ncell Nk, tets null) or an explicit list (nperm 1, ncell n_tet, tets [n_tet][4] corner
    // indices into the k-points).
    int64_t ncell;
    int32_t nperm;
    const int32_t *tets;
    // mixed form: near-degenerate final tetrahedra (two sorted corner values of e'-e closer than
    // max(degen_tol, degen_rel * span)) keep the FP64 near branch
    double degen_tol, degen_rel;
};

// Tetrahedra per band pair.
__host__ __device__ inline int64_t tets_per_pair(const MeshDev &M) { return (int64_t)M.nperm * M.ncell; }

// One (instance, q) item of a fused batch launch (device table entry).
struct BatchItemDev {
    MeshDev M;
    QDev Q;
    const double *omega;   // [nw]
    double *partial;       // this item's K_B partial sums [nblocks][nw][2]
    double *out;           // chi of this q: [nw][2]
    double scale;          // g_s / (6 Nk)
    int32_t nw, precision;
    int32_t nblocks;       // K_B workgroups of this item
    int32_t kb_begin;      // first K_B workgroup of the item in the fused grid
    int32_t ka_begin;      // first K_A workgroup (16 k each), -1 under CMA
    int32_t kr_begin;      // first K_R workgroup (256 values each)
};

// Fused launches over a batch table: matrix elements, tetrahedron weights, reduction.
hipError_t launch_contract_batch(const BatchItemDev *items, const int32_t *block_item, int nblocks_total,
                                 hipStream_t s);
hipError_t launch_tetra_batch(const BatchItemDev *items, const int32_t *block_item, int nblocks_total,
                              hipStream_t s);
hipError_t launch_reduce_batch(const BatchItemDev *items, const int32_t *block_item, int nblocks_total,
                               hipStream_t s);
// Band ranges of a batch stage: group_item[g] is the first item of (instance, q) group g, whose
// QDev range pointers (shared by the group's items) receive e(k) and e(k+q); max_nbw bounds the
// groups' band windows.
hipError_t launch_band_range_batch(const BatchItemDev *items, const int32_t *group_item, int ngroups, int max_nbw,
                                   hipStream_t s);

// K_A: W_nm(k) = |sum_o conj(c_{o,n}(k)) c_{o,m}(k+q)|^2 for nq q-points of a batch.
// precision 0: FP64 MFMA; 1: BF16 hi+lo split MFMA; 2: FP16 hi+lo split MFMA (FP32 accumulate).
// Split operands of the plan's eigenvectors in the workspace (pack_bytes(mesh)); ptr null: none.
// A split-precision plane-wave launch of at least kPackMinQ q, all given by mesh shifts, fills them
// unless valid is set (an earlier launch of the same call did) and reads them instead of the FP64
// eigenvectors.
struct PackState {
    void *ptr;
    bool valid;
};
hipError_t launch_contract(const MeshDev &mesh, const BatchDev &batch, int nq, int precision, PackState *pack,
                           hipStream_t s);
constexpr int kPackMinQ = 3;
size_t pack_bytes(const MeshDev &mesh);

// Band ranges of a batch (see QDev::rng_k): nothing when the batch carries no range pointers.
// Every K_B launcher below calls it before its kernel.
hipError_t launch_band_range(const MeshDev &mesh, const BatchDev &batch, int nq, hipStream_t s);

// K_B static: per-block partial sums of Re chi0(q, 0) (unnormalised) into partial[nq][nblocks].
hipError_t launch_tetra_static(const MeshDev &mesh, const BatchDev &batch, int nq, int nblocks, double *partial,
                               hipStream_t s);

// K_B imaginary part alone (delta weights): partial sums partial[nq][nblocks][nw][2] with Re = 0,
// nw <= kMaxOmegaIm.
hipError_t launch_tetra_im(const MeshDev &mesh, const BatchDev &batch, int nq, int nblocks, const double *omega,
                           int nw, double *partial, hipStream_t s);

// Kramers-Kronig route: omega_all[k] = lo + k h (k < K), omega_all[K + i] = omega[i] (i < nw).
hipError_t launch_kk_grid(double lo, double h, int K, const double *omega, int nw, double *omega_all, hipStream_t s);

// Kramers-Kronig route: out[q][i] = (Re, Im), Re = (1/pi) sum_k im_all[q][k].im L_k(omega_i) over the
// K grid points (tents of the piecewise-linear interpolant, zero one spacing beyond each end),
// Im = im_all[q][K + i].im; im_all is [nq][K + nw][2].
hipError_t launch_kk_transform(const double *im_all, int nq, int K, int nw, double lo, double h, const double *omega,
                               double *out, int64_t out_stride, hipStream_t s);

// K_B static resolved by band pair: nblk workgroups per pair, partial sums partial[nq][nblk][nbw^2].
hipError_t launch_tetra_static_pairs(const MeshDev &mesh, const BatchDev &batch, int nq, int nblk, double *partial,
                                     hipStream_t s);

// K_B dynamic: per-block partial sums into partial[nq][nblocks][nw][2], nw <= kMaxOmegaPerLaunch.
// mixed: far-branch series in FP32 (FP64 near branch and accumulation).
hipError_t launch_tetra_dynamic(const MeshDev &mesh, const BatchDev &batch, int nq, int nblocks,
                                const double *omega, int nw, double *partial, bool mixed, hipStream_t s);
hipError_t launch_tetra_dynamic_list(const MeshDev &mesh, const BatchDev &batch, int nq, int nblocks,
                                     const double *omega, int nw, double *partial, bool mixed, hipStream_t s);
// K_B dynamic resolved by band pair (mesh plans): partial[nq][nbw*nbw][nblk][nw][2].
hipError_t launch_tetra_dynamic_pairs(const MeshDev &mesh, const BatchDev &batch, int nq, int nblk,
                                      const double *omega, int nw, double *partial, bool mixed, hipStream_t s);

// Census of the work of a dynamic call (nw <= kMaxOmegaPerLaunch), by the dynamic evaluation
// itself with counters (it also writes the call's partial sums): counts[0..5] += active units,
// final tetrahedra, near-branch evaluations, far-branch evaluations (per final tetrahedron and
// frequency, or per list of final tetrahedra and frequency where a list is one series), the
// series terms of the far evaluations (FP32 series when mixed), and the near evaluations repeated
// in full (FP64 form: an entry's nodes cluster).  Units and final tetrahedra are
// counted only when first_chunk is set (the first frequency chunk of a call).
hipError_t launch_census(const MeshDev &mesh, const BatchDev &batch, int nq, int nblocks, const double *omega,
                         int nw, double *partial, bool mixed, bool first_chunk, unsigned long long *counts,
                         hipStream_t s);

// Content scan of device inputs: clear the verdict word, then OR bits into it for non-finite
// values of a float64 array, and for eigenvectors c[Nk][no][nb] (complex) with non-finite
// coefficients or a squared norm off 1 by more than tol.
constexpr unsigned kScanEps = 1u, kScanEig = 2u, kScanOmega = 4u, kScanNorm = 8u;
hipError_t launch_scan_clear(unsigned *flag, hipStream_t s);
hipError_t launch_scan_finite(const double *p, int64_t n, unsigned bit, unsigned *flag, hipStream_t s);
hipError_t launch_scan_eigvec(const double *c, int64_t nk, int no, int nb, unsigned bit_nonfinite, unsigned bit_norm,
                              double tol, unsigned *flag, hipStream_t s);

// K_R: out[q * out_stride + v] = scale * sum_b partial[(q * nblocks + b) * nvals + v], fixed order.
hipError_t launch_reduce(const double *partial, int nq, int nblocks, int nvals, double scale,
                         double *out, int64_t out_stride, hipStream_t s, bool accumulate = false);

}  // namespace chi0
