// k_contract.hip -- matrix elements on the FP64 matrix cores (K_A).
//
// For every mesh point k of a q:  M_nm = sum_o conj(c_{o,n}(k)) c_{o,m}(k+q)  and
// W_nm(k) = |M_nm|^2 (the tight-binding matrix element of the footnote in Sec. III).
// Per k this is a small complex GEMM (bands x orbitals) x (orbitals x bands); it
// runs as real 16x16x4 FP64 MFMAs (v_mfma_f64_16x16x4f64), four per step of 4
// orbitals:  Re M = Cr^T Br + Ci^T Bi,  Im M = Cr^T Bi - Ci^T Br.
// A workgroup is one wave that handles 16 consecutive k; |M|^2 of a 16x16 band
// tile is staged in LDS as [n][m][k] and written out pair-major, so each store
// covers 16 consecutive k of one band pair (the layout the tetrahedron kernel
// reads with consecutive lanes on consecutive cells).
#include "chi0_internal.h"

namespace chi0 {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kKPerBlock = 16;

typedef double Tile[16][kKPerBlock + 1];

// One workgroup of FP64 matrix elements: k = k0 .. k0+15 of one q.
__device__ __forceinline__ void contract_f64_body(const MeshDev &M, const QDev &Q, int64_t k0, Tile *tile)
{
    const int lane = threadIdx.x;
    const int row = lane & 15;      // A row (band n) / B column (band m) of this lane
    const int kk = lane >> 4;       // orbital within the step of 4
    const int64_t nk = M.nk;
    const int ntile = (M.nbw + 15) / 16;
    const int nb = M.nb, no = M.no;

    for (int tn = 0; tn < ntile; ++tn) {
        for (int tm = 0; tm < ntile; ++tm) {
            const int n = tn * 16 + row;
            const int m = tm * 16 + row;
            for (int kl = 0; kl < kKPerBlock; ++kl) {
                const int64_t k = k0 + kl;
                if (k >= nk) break;
                int64_t kq = k;
                if (!Q.explicit_kq) {
                    int i2 = (int)(k % M.n3);
                    const int64_t t = k / M.n3;
                    int i1 = (int)(t % M.n2);
                    int i0 = (int)(t / M.n2);
                    i0 += Q.shift[0]; i0 -= i0 >= M.n1 ? M.n1 : 0;
                    i1 += Q.shift[1]; i1 -= i1 >= M.n2 ? M.n2 : 0;
                    i2 += Q.shift[2]; i2 -= i2 >= M.n3 ? M.n3 : 0;
                    kq = ((int64_t)i0 * M.n2 + i1) * M.n3 + i2;
                }
                dbl4 accr = {0.0, 0.0, 0.0, 0.0};
                dbl4 acci = {0.0, 0.0, 0.0, 0.0};
                for (int o0 = 0; o0 < no; o0 += 4) {
                    const int o = o0 + kk;
                    double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
                    if (o < no && n < M.nbw) {
                        const double *p = M.c_k + 2 * ((k * no + o) * nb + M.lo + n);
                        ar = p[0];
                        ai = p[1];
                    }
                    if (o < no && m < M.nbw) {
                        const double *p = Q.c_kq + 2 * ((kq * no + o) * nb + M.lo + m);
                        br = p[0];
                        bi = p[1];
                    }
                    accr = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, accr, 0, 0, 0);
                    accr = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, accr, 0, 0, 0);
                    acci = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, acci, 0, 0, 0);
                    acci = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, br, acci, 0, 0, 0);
                }
                // accumulator element v of this lane is D[kk + 4 v][row] (row index = band n,
                // column = band m) for the FP64 16x16x4 MFMA
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    tile[kk + 4 * v][row][kl] = accr[v] * accr[v] + acci[v] * acci[v];
            }
            __syncthreads();
            for (int e = lane; e < 16 * 16 * kKPerBlock; e += 64) {
                const int kl = e % kKPerBlock;
                const int pj = e / kKPerBlock;
                const int i = pj / 16, j = pj % 16;
                const int nn = tn * 16 + i, mm = tm * 16 + j;
                const int64_t k = k0 + kl;
                if (nn < M.nbw && mm < M.nbw && k < nk)
                    Q.W[((int64_t)nn * M.nbw + mm) * nk + k] = tile[i][j][kl];
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Split-precision form: 16-bit MFMA with FP32 accumulation and hi + lo operands.
// Every FP64 operand x is split as x = hi + lo with hi = round16(x) and
// lo = round16((x - hi) * S) / S (S = 2^11 for FP16, whose exponent range would flush
// small remainders; S = 1 for BF16), and a product is taken as
// hi*hi + (hi*lo + lo*hi) / S: three MFMAs, the dropped lo*lo term is below the FP32
// accumulation error.  The complex product is folded into real GEMMs over a doubled
// reduction axis:  Re M = [Cr Ci] . [Br; Bi],  Im M = [Cr Ci] . [Bi; -Br].
// ---------------------------------------------------------------------------

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float f)
{
    // round to nearest even (finite inputs)
    const unsigned u = __float_as_uint(f);
    return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float from_bf16(short h) { return __uint_as_float(((unsigned)(unsigned short)h) << 16); }

template <bool FP16>
struct Split4 {
    half4 hh, hl;
    bf16x4 bh, bl;
};

template <bool FP16>
__device__ __forceinline__ void split_value(double x, int j, Split4<FP16> &s)
{
    if (FP16) {
        const _Float16 hi = (_Float16)x;
        const _Float16 lo = (_Float16)((x - (double)hi) * 2048.0);
        s.hh[j] = hi;
        s.hl[j] = lo;
    } else {
        const short hi = to_bf16((float)x);
        const short lo = to_bf16((float)(x - (double)from_bf16(hi)));
        s.bh[j] = hi;
        s.bl[j] = lo;
    }
}

template <bool FP16>
__device__ __forceinline__ flt4 mfma16(const Split4<FP16> &a, bool a_lo, const Split4<FP16> &b, bool b_lo, flt4 c)
{
    if (FP16)
        return __builtin_amdgcn_mfma_f32_16x16x16f16(a_lo ? a.hl : a.hh, b_lo ? b.hl : b.hh, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a_lo ? a.bl : a.bh, b_lo ? b.bl : b.bh, c, 0, 0, 0);
}

// One workgroup of split-precision matrix elements: k = k0 .. k0+15 of one q.
template <bool FP16>
__device__ __forceinline__ void contract_split_body(const MeshDev &M, const QDev &Q, int64_t k0, Tile *tile)
{
    const int lane = threadIdx.x;
    const int row = lane & 15;      // A row (band n) / B column (band m)
    const int kq4 = lane >> 4;      // which 4 of the 16 reduction indices of a step
    const int64_t nk = M.nk;
    const int ntile = (M.nbw + 15) / 16;
    const int nb = M.nb, no = M.no;
    const int kred = 2 * no;        // reduction axis: orbitals (real parts), then orbitals (imaginary)
    const float inv_s = FP16 ? 1.0f / 2048.0f : 1.0f;

    for (int tn = 0; tn < ntile; ++tn) {
        for (int tm = 0; tm < ntile; ++tm) {
            const int n = tn * 16 + row;
            const int m = tm * 16 + row;
            for (int kl = 0; kl < kKPerBlock; ++kl) {
                const int64_t k = k0 + kl;
                if (k >= nk) break;
                int64_t kq = k;
                if (!Q.explicit_kq) {
                    int i2 = (int)(k % M.n3);
                    const int64_t t = k / M.n3;
                    int i1 = (int)(t % M.n2);
                    int i0 = (int)(t / M.n2);
                    i0 += Q.shift[0]; i0 -= i0 >= M.n1 ? M.n1 : 0;
                    i1 += Q.shift[1]; i1 -= i1 >= M.n2 ? M.n2 : 0;
                    i2 += Q.shift[2]; i2 -= i2 >= M.n3 ? M.n3 : 0;
                    kq = ((int64_t)i0 * M.n2 + i1) * M.n3 + i2;
                }
                flt4 re_main = {0.f, 0.f, 0.f, 0.f}, re_corr = {0.f, 0.f, 0.f, 0.f};
                flt4 im_main = {0.f, 0.f, 0.f, 0.f}, im_corr = {0.f, 0.f, 0.f, 0.f};
                for (int r0 = 0; r0 < kred; r0 += 16) {
                    Split4<FP16> a, bre, bim;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int r = r0 + 4 * kq4 + j;
                        const bool imag = r >= no;
                        const int o = imag ? r - no : r;
                        double av = 0.0, brv = 0.0, biv = 0.0;
                        if (r < kred && n < M.nbw) {
                            const double *p = M.c_k + 2 * ((k * no + o) * nb + M.lo + n);
                            av = imag ? p[1] : p[0];                // [Cr Ci]
                        }
                        if (r < kred && m < M.nbw) {
                            const double *p = Q.c_kq + 2 * ((kq * no + o) * nb + M.lo + m);
                            brv = imag ? p[1] : p[0];               // [Br; Bi]
                            biv = imag ? -p[0] : p[1];              // [Bi; -Br]
                        }
                        split_value<FP16>(av, j, a);
                        split_value<FP16>(brv, j, bre);
                        split_value<FP16>(biv, j, bim);
                    }
                    re_main = mfma16<FP16>(a, false, bre, false, re_main);
                    re_corr = mfma16<FP16>(a, false, bre, true, re_corr);
                    re_corr = mfma16<FP16>(a, true, bre, false, re_corr);
                    im_main = mfma16<FP16>(a, false, bim, false, im_main);
                    im_corr = mfma16<FP16>(a, false, bim, true, im_corr);
                    im_corr = mfma16<FP16>(a, true, bim, false, im_corr);
                }
                // accumulator element v of this lane is D[4 kq4 + v][row] for the 16x16x16 MFMA
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float mr = fmaf(re_corr[v], inv_s, re_main[v]);
                    const float mi = fmaf(im_corr[v], inv_s, im_main[v]);
                    tile[4 * kq4 + v][row][kl] = (double)(mr * mr + mi * mi);
                }
            }
            __syncthreads();
            for (int e = lane; e < 16 * 16 * kKPerBlock; e += 64) {
                const int kl = e % kKPerBlock;
                const int pj = e / kKPerBlock;
                const int i = pj / 16, j = pj % 16;
                const int nn = tn * 16 + i, mm = tm * 16 + j;
                const int64_t k = k0 + kl;
                if (nn < M.nbw && mm < M.nbw && k < nk) Q.W[((int64_t)nn * M.nbw + mm) * nk + k] = tile[i][j][kl];
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(64) void contract_f64_kernel(MeshDev M, BatchDev B)
{
    __shared__ double tile[16][16][kKPerBlock + 1];
    contract_f64_body(M, B.q[blockIdx.y], (int64_t)blockIdx.x * kKPerBlock, tile);
}

template <bool FP16>
__global__ __launch_bounds__(64) void contract_split_kernel(MeshDev M, BatchDev B)
{
    __shared__ double tile[16][16][kKPerBlock + 1];
    contract_split_body<FP16>(M, B.q[blockIdx.y], (int64_t)blockIdx.x * kKPerBlock, tile);
}

// ---------------------------------------------------------------------------
// Large bases (plane waves): the contraction length n_orb runs to thousands, so one k is a
// genuine complex GEMM (nbw x n_orb)^H (n_orb x nbw).  One workgroup of four waves per (k, q):
// with nbw > 16 each wave owns one 16x16 band tile over the whole reduction; with nbw <= 16 the
// single tile's reduction is split four ways and summed through LDS.  Operands are read
// straight from HBM (16 consecutive bands of one orbital: 256 contiguous bytes per load), the
// waves of a workgroup sharing them through the caches.
// ---------------------------------------------------------------------------
constexpr int kPwWaves = 4;

__global__ __launch_bounds__(256) void contract_pw_kernel(MeshDev M, BatchDev B)
{
    __shared__ double red[kPwWaves][8][64];
    const QDev Q = B.q[blockIdx.y];
    const int64_t k = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = lane & 15, kk = lane >> 4;
    const int nb = M.nb, no = M.no;
    const int ntile = M.nbw > 16 ? 2 : 1;
    const int ntiles = ntile * ntile;            // 4 or 1
    const int nsplit = kPwWaves / ntiles;        // 1 or 4 reduction slices
    const int tile = wave % ntiles, slice = wave / ntiles;
    const int tn = tile / ntile, tm = tile % ntile;
    int64_t kq = k;
    if (!Q.explicit_kq) {
        int i2 = (int)(k % M.n3);
        const int64_t t = k / M.n3;
        int i1 = (int)(t % M.n2);
        int i0 = (int)(t / M.n2);
        i0 += Q.shift[0]; i0 -= i0 >= M.n1 ? M.n1 : 0;
        i1 += Q.shift[1]; i1 -= i1 >= M.n2 ? M.n2 : 0;
        i2 += Q.shift[2]; i2 -= i2 >= M.n3 ? M.n3 : 0;
        kq = ((int64_t)i0 * M.n2 + i1) * M.n3 + i2;
    }
    const int n = tn * 16 + row, m = tm * 16 + row;
    const bool an = n < M.nbw, bm = m < M.nbw;
    const double *pa = M.c_k + 2 * ((k * no) * nb + M.lo + (an ? n : 0));
    const double *pb = Q.c_kq + 2 * ((kq * no) * nb + M.lo + (bm ? m : 0));
    // reduction slice of this wave: orbitals [o_begin, o_end) in steps of 4
    const int steps = (no + 3) / 4;
    const int per = (steps + nsplit - 1) / nsplit;
    const int o_begin = slice * per * 4, o_end = min(no, (slice + 1) * per * 4);
    dbl4 accr = {0.0, 0.0, 0.0, 0.0};
    dbl4 acci = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int o0 = o_begin; o0 < o_end; o0 += 4) {
        const int o = o0 + kk;
        double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
        if (o < o_end) {
            const int64_t off = 2 * (int64_t)o * nb;
            if (an) { ar = pa[off]; ai = pa[off + 1]; }
            if (bm) { br = pb[off]; bi = pb[off + 1]; }
        }
        accr = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, accr, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, acci, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, br, acci, 0, 0, 0);
    }
    if (nsplit > 1) {
        // sum the reduction slices in a fixed order (wave 0 + 1 + 2 + 3)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            red[wave][v][lane] = accr[v];
            red[wave][4 + v][lane] = acci[v];
        }
        __syncthreads();
        if (wave != 0) return;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double sr = red[0][v][lane], si = red[0][4 + v][lane];
            for (int w2 = 1; w2 < kPwWaves; ++w2) {
                sr += red[w2][v][lane];
                si += red[w2][4 + v][lane];
            }
            accr[v] = sr;
            acci[v] = si;
        }
    }
    // accumulator element v of this lane is D[kk + 4 v][row]: band n = tn*16 + kk + 4v, m = tm*16 + row
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int nn = tn * 16 + kk + 4 * v, mm = tm * 16 + row;
        if (nn < M.nbw && mm < M.nbw)
            Q.W[((int64_t)nn * M.nbw + mm) * M.nk + k] = accr[v] * accr[v] + acci[v] * acci[v];
    }
}

// Fused launch over the (instance, q) items of a batch: workgroup -> item from a table.
__global__ __launch_bounds__(64) void contract_batch_kernel(const BatchItemDev *__restrict__ items,
                                                            const int32_t *__restrict__ block_item)
{
    __shared__ double tile[16][16][kKPerBlock + 1];
    const BatchItemDev it = items[block_item[blockIdx.x]];
    const int64_t k0 = (int64_t)(blockIdx.x - it.ka_begin) * kKPerBlock;
    if (it.precision == 1)
        contract_split_body<false>(it.M, it.Q, k0, tile);
    else if (it.precision == 2)
        contract_split_body<true>(it.M, it.Q, k0, tile);
    else
        contract_f64_body(it.M, it.Q, k0, tile);
}

}  // namespace

hipError_t launch_contract_batch(const BatchItemDev *items, const int32_t *block_item, int nblocks_total,
                                 hipStream_t s)
{
    if (nblocks_total < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(contract_batch_kernel, dim3(nblocks_total), dim3(64), 0, s, items, block_item);
    return hipGetLastError();
}

hipError_t launch_contract(const MeshDev &mesh, const BatchDev &batch, int nq, int precision, hipStream_t s)
{
    if (nq < 1 || nq > kMaxQBatch) return hipErrorInvalidValue;
    if (mesh.no > kMaxOrbSmall) {
        // large (plane-wave) bases: one four-wave workgroup per (k, q), FP64 in every precision
        if (mesh.nbw > 32) return hipErrorInvalidValue;
        dim3 grid((unsigned)mesh.nk, nq), block(64 * kPwWaves);
        hipLaunchKernelGGL(contract_pw_kernel, grid, block, 0, s, mesh, batch);
        return hipGetLastError();
    }
    const int64_t nblk = (mesh.nk + kKPerBlock - 1) / kKPerBlock;
    dim3 grid((unsigned)nblk, nq), block(64);
    if (precision == 1)
        hipLaunchKernelGGL(contract_split_kernel<false>, grid, block, 0, s, mesh, batch);
    else if (precision == 2)
        hipLaunchKernelGGL(contract_split_kernel<true>, grid, block, 0, s, mesh, batch);
    else
        hipLaunchKernelGGL(contract_f64_kernel, grid, block, 0, s, mesh, batch);
    return hipGetLastError();
}

}  // namespace chi0
