// k_contract.hip -- matrix elements on the FP64 matrix cores (K_A).
//
// For every mesh point k of a q:  M_nm = sum_o conj(c_{o,n}(k)) c_{o,m}(k+q)  and
// W_nm(k) = |M_nm|^2 (the tight-binding matrix element of the footnote in Sec. III).
// Per k this is a small complex GEMM (bands x orbitals) x (orbitals x bands); it
// runs as real 16x16x4 FP64 MFMAs (v_mfma_f64_16x16x4f64), four per step of 4
// orbitals:  Re M = Cr^T Br + Ci^T Bi,  Im M = Cr^T Bi - Ci^T Br.
// A workgroup is one wave that handles 16 consecutive k, two at a time (their loads
// in flight together); |M|^2 of a band tile (min(nbw, 16) squared pairs) is staged in
// LDS as [pair][k] and written out pair-major, so each store covers 16 consecutive k
// of one band pair (the layout the tetrahedron kernel reads with consecutive lanes on
// consecutive cells).  The staging tile is sized for the band window at launch, so a
// 10-band window holds 11 workgroups per CU rather than 4.
#include "chi0_internal.h"

namespace chi0 {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kKPerBlock = 16;
constexpr int kHalfBlock = kKPerBlock / 2;   // the two k of one iteration: kl and kl + kHalfBlock
constexpr int kTileLd = kKPerBlock + 1;      // staged values per pair (odd: no bank conflicts)
constexpr int kXcd = 8;                      // XCDs; workgroup b is dispatched to XCD b % kXcd

// Band tile edge of the staging tile: the window itself up to 16 bands, else 16.
__host__ __device__ inline int tile_dim(int nbw) { return nbw < 16 ? nbw : 16; }

// Mesh index of k + q: the shifted mesh point, or k itself when the k+q data are given explicitly.
__device__ __forceinline__ int64_t shifted_k(const MeshDev &M, const QDev &Q, int64_t k)
{
    if (Q.explicit_kq) return k;
    int i2 = (int)(k % M.n3);
    const int64_t t = k / M.n3;
    int i1 = (int)(t % M.n2);
    int i0 = (int)(t / M.n2);
    i0 += Q.shift[0]; i0 -= i0 >= M.n1 ? M.n1 : 0;
    i1 += Q.shift[1]; i1 -= i1 >= M.n2 ? M.n2 : 0;
    i2 += Q.shift[2]; i2 -= i2 >= M.n3 ? M.n3 : 0;
    return ((int64_t)i0 * M.n2 + i1) * M.n3 + i2;
}

// Stage |M|^2 of one k: accumulator element i of lane (g = lane / 16, row = lane % 16) is
// D[g + 4 i][row] for the FP64 16x16x4 MFMA (F64) and D[4 g + i][row] for the 16x16x32 FP32-
// accumulating ones (row index = band n, column = band m); pairs outside the T x T tile are padding.
template <bool F64>
__device__ __forceinline__ void stage_k(double *tile, int T, int g, int row, int kl, const double (&v)[4])
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int n = F64 ? g + 4 * i : 4 * g + i;
        if (n < T && row < T) tile[(n * T + row) * kTileLd + kl] = v[i];
    }
}

// Write the staged tile (band tiles tn, tm) of k0 .. k0+15 pair-major into W: 16 consecutive
// lanes store the 16 k of one pair.
__device__ __forceinline__ void write_tile(const MeshDev &M, const QDev &Q, const double *tile, int T, int tn,
                                           int tm, int64_t k0, int lane)
{
    for (int e = lane; e < T * T * kKPerBlock; e += 64) {
        const int kl = e % kKPerBlock;
        const int pj = e / kKPerBlock;
        const int i = pj / T, j = pj - i * T;
        const int nn = tn * 16 + i, mm = tm * 16 + j;
        const int64_t k = k0 + kl;
        if (nn < M.nbw && mm < M.nbw && k < M.nk) Q.W[((int64_t)nn * M.nbw + mm) * M.nk + k] = tile[pj * kTileLd + kl];
    }
}

// One workgroup of FP64 matrix elements: k = k0 .. k0+15 of one q, as the pairs (kl, kl + 8).
__device__ __forceinline__ void contract_f64_body(const MeshDev &M, const QDev &Q, int64_t k0, double *tile)
{
    const int lane = threadIdx.x;
    const int row = lane & 15;      // A row (band n) / B column (band m) of this lane
    const int kk = lane >> 4;       // orbital within the step of 4
    const int64_t nk = M.nk;
    const int ntile = (M.nbw + 15) / 16, T = tile_dim(M.nbw);
    const int nb = M.nb, no = M.no;

    for (int tn = 0; tn < ntile; ++tn) {
        for (int tm = 0; tm < ntile; ++tm) {
            const int n = tn * 16 + row;
            const int m = tm * 16 + row;
            for (int kl = 0; kl < kHalfBlock; ++kl) {
                const int64_t ka = k0 + kl, kb = ka + kHalfBlock;
                if (ka >= nk) break;
                const bool vb = kb < nk;
                const int64_t kqa = shifted_k(M, Q, ka), kqb = vb ? shifted_k(M, Q, kb) : kqa;
                dbl4 ra = {0.0, 0.0, 0.0, 0.0}, ia = ra, rb = ra, ib = ra;
                for (int o0 = 0; o0 < no; o0 += 4) {
                    const int o = o0 + kk;
                    double2 a0 = {0.0, 0.0}, a1 = a0, b0 = a0, b1 = a0;
                    if (o < no && n < M.nbw) {
                        a0 = *reinterpret_cast<const double2 *>(M.c_k + 2 * ((ka * no + o) * nb + M.lo + n));
                        if (vb) a1 = *reinterpret_cast<const double2 *>(M.c_k + 2 * ((kb * no + o) * nb + M.lo + n));
                    }
                    if (o < no && m < M.nbw) {
                        b0 = *reinterpret_cast<const double2 *>(Q.c_kq + 2 * ((kqa * no + o) * nb + M.lo + m));
                        if (vb) b1 = *reinterpret_cast<const double2 *>(Q.c_kq + 2 * ((kqb * no + o) * nb + M.lo + m));
                    }
                    ra = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.x, b0.x, ra, 0, 0, 0);
                    rb = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.x, b1.x, rb, 0, 0, 0);
                    ra = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.y, b0.y, ra, 0, 0, 0);
                    rb = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.y, b1.y, rb, 0, 0, 0);
                    ia = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.x, b0.y, ia, 0, 0, 0);
                    ib = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.x, b1.y, ib, 0, 0, 0);
                    ia = __builtin_amdgcn_mfma_f64_16x16x4f64(-a0.y, b0.x, ia, 0, 0, 0);
                    ib = __builtin_amdgcn_mfma_f64_16x16x4f64(-a1.y, b1.x, ib, 0, 0, 0);
                }
                double va[4], vv[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    va[v] = ra[v] * ra[v] + ia[v] * ia[v];
                    vv[v] = rb[v] * rb[v] + ib[v] * ib[v];
                }
                stage_k<true>(tile, T, kk, row, kl, va);
                if (vb) stage_k<true>(tile, T, kk, row, kl + kHalfBlock, vv);
            }
            __syncthreads();
            write_tile(M, Q, tile, T, tn, tm, k0, lane);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Split-precision forms: 16-bit MFMA with FP32 accumulation and hi + lo operands, on the gfx950
// 16x16x32 instructions (v_mfma_f32_16x16x32_{bf16,f16}).  Every FP64 operand x is taken to FP32
// and split as x = hi + lo with hi = round16(x) and lo = round16((x - hi) * S) / S (S = 2^11 for
// FP16, whose exponent range would flush small remainders; S = 1 for BF16); a product is taken as
// hi*hi + (hi*lo + lo*hi) / S: three MFMAs.  hi and lo together carry 2 x 8 significant bits for
// BF16 and 2 x 11 for FP16, so the dropped lo*lo term and the rounding of lo leave a relative error
// of about 2^-16 per product for BF16 (well above the FP32 accumulation's 2^-24) and about 2^-22
// for FP16.
//
// The complex product is folded into two real GEMMs over a doubled reduction axis.  One MFMA
// covers 16 orbitals: lane (row, g) holds the real parts of orbitals 4g .. 4g+3 of the step and
// then their imaginary parts, so with a = C(k), b = C(k+q)
//     A = [ar; ai],  B_re = [br; bi],  B_im = [bi; -br],   Re M = A . B_re,  Im M = A . B_im.
// B_im is B_re with its two halves exchanged and the second negated: a register permutation and a
// sign flip of packed 16-bit values, so every coefficient is split once.  Which reduction slot the
// hardware gives each of a lane's eight values does not matter: A and B use the same assignment.
// Per 16 orbitals and 16x16 tile pair: six MFMAs (hi.hi, hi.lo, lo.hi for Re and for Im).
// ---------------------------------------------------------------------------

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef float flt2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr unsigned kSign2 = 0x80008000u;   // sign bits of two packed 16-bit values

// Two FP64 values -> packed 16-bit high parts and low parts (round to nearest even; the low parts
// scaled by 2^11 for FP16).
template <bool FP16>
__device__ __forceinline__ void split2(double x, double y, unsigned &hi, unsigned &lo)
{
    const flt2 f = {(float)x, (float)y};
    if (FP16) {
        const f16x2 h = __builtin_convertvector(f, f16x2);
        const flt2 r = (f - __builtin_convertvector(h, flt2)) * 2048.0f;
        hi = __builtin_bit_cast(unsigned, h);
        lo = __builtin_bit_cast(unsigned, __builtin_convertvector(r, f16x2));
    } else {
        const bf16x2 h = __builtin_convertvector(f, bf16x2);
        const flt2 r = f - __builtin_convertvector(h, flt2);
        hi = __builtin_bit_cast(unsigned, h);
        lo = __builtin_bit_cast(unsigned, __builtin_convertvector(r, bf16x2));
    }
}

template <bool FP16>
__device__ __forceinline__ flt4 mfma32(u32x4 a, u32x4 b, flt4 c)
{
    if (FP16)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                      0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

// The split operand of 4 orbitals of one lane: hi and lo of [re0..re3, im0..im3].
template <bool FP16>
__device__ __forceinline__ void split_op(const double2 (&v)[4], u32x4 &hi, u32x4 &lo)
{
    unsigned h[4], l[4];
    split2<FP16>(v[0].x, v[1].x, h[0], l[0]);
    split2<FP16>(v[2].x, v[3].x, h[1], l[1]);
    split2<FP16>(v[0].y, v[1].y, h[2], l[2]);
    split2<FP16>(v[2].y, v[3].y, h[3], l[3]);
    hi = u32x4{h[0], h[1], h[2], h[3]};
    lo = u32x4{l[0], l[1], l[2], l[3]};
}

// [br; bi] -> [bi; -br]
__device__ __forceinline__ u32x4 rot_op(u32x4 b) { return u32x4{b[2], b[3], b[0] ^ kSign2, b[1] ^ kSign2}; }

// Re and Im accumulators of one 16x16 tile pair (main hi.hi products and the scaled corrections).
struct SplitAcc {
    flt4 re, re_c, im, im_c;
};

template <bool FP16>
__device__ __forceinline__ void split_step(SplitAcc &c, u32x4 ah, u32x4 al, u32x4 bh, u32x4 bl)
{
    c.re = mfma32<FP16>(ah, bh, c.re);
    c.re_c = mfma32<FP16>(ah, bl, c.re_c);
    c.re_c = mfma32<FP16>(al, bh, c.re_c);
    const u32x4 ih = rot_op(bh), il = rot_op(bl);
    c.im = mfma32<FP16>(ah, ih, c.im);
    c.im_c = mfma32<FP16>(ah, il, c.im_c);
    c.im_c = mfma32<FP16>(al, ih, c.im_c);
}

// |M|^2 of accumulator element v
template <bool FP16>
__device__ __forceinline__ double split_abs2(const SplitAcc &c, int v)
{
    const float inv_s = FP16 ? 1.0f / 2048.0f : 1.0f;
    const double mr = (double)fmaf(c.re_c[v], inv_s, c.re[v]);
    const double mi = (double)fmaf(c.im_c[v], inv_s, c.im[v]);
    return mr * mr + mi * mi;
}

// One workgroup of split-precision matrix elements: k = k0 .. k0+15 of one q, as the pairs
// (kl, kl + 8).
template <bool FP16>
__device__ __forceinline__ void contract_split_body(const MeshDev &M, const QDev &Q, int64_t k0, double *tile)
{
    const int lane = threadIdx.x;
    const int row = lane & 15;      // A row (band n) / B column (band m)
    const int g = lane >> 4;        // orbitals 4g .. 4g+3 of a step of 16
    const int64_t nk = M.nk;
    const int ntile = (M.nbw + 15) / 16, T = tile_dim(M.nbw);
    const int nb = M.nb, no = M.no;

    for (int tn = 0; tn < ntile; ++tn) {
        for (int tm = 0; tm < ntile; ++tm) {
            const int n = tn * 16 + row;
            const int m = tm * 16 + row;
            for (int kl = 0; kl < kHalfBlock; ++kl) {
                const int64_t ka = k0 + kl, kb = ka + kHalfBlock;
                if (ka >= nk) break;
                const bool vb = kb < nk;
                const int64_t kqa = shifted_k(M, Q, ka), kqb = vb ? shifted_k(M, Q, kb) : kqa;
                SplitAcc acc0, acc1;
                acc0.re = acc0.re_c = acc0.im = acc0.im_c = flt4{0.f, 0.f, 0.f, 0.f};
                acc1 = acc0;
                for (int o0 = 0; o0 < no; o0 += 16) {
                    double2 av0[4], bv0[4], av1[4], bv1[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int o = o0 + 4 * g + i;
                        av0[i] = bv0[i] = av1[i] = bv1[i] = double2{0.0, 0.0};
                        if (o < no && n < M.nbw) {
                            av0[i] = *reinterpret_cast<const double2 *>(M.c_k + 2 * ((ka * no + o) * nb + M.lo + n));
                            if (vb) av1[i] = *reinterpret_cast<const double2 *>(M.c_k + 2 * ((kb * no + o) * nb + M.lo + n));
                        }
                        if (o < no && m < M.nbw) {
                            bv0[i] = *reinterpret_cast<const double2 *>(Q.c_kq + 2 * ((kqa * no + o) * nb + M.lo + m));
                            if (vb) bv1[i] = *reinterpret_cast<const double2 *>(Q.c_kq + 2 * ((kqb * no + o) * nb + M.lo + m));
                        }
                    }
                    u32x4 ah, al, bh, bl;
                    split_op<FP16>(av0, ah, al);
                    split_op<FP16>(bv0, bh, bl);
                    split_step<FP16>(acc0, ah, al, bh, bl);
                    split_op<FP16>(av1, ah, al);
                    split_op<FP16>(bv1, bh, bl);
                    split_step<FP16>(acc1, ah, al, bh, bl);
                }
                double va[4], vv[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    va[v] = split_abs2<FP16>(acc0, v);
                    vv[v] = split_abs2<FP16>(acc1, v);
                }
                stage_k<false>(tile, T, g, row, kl, va);
                if (vb) stage_k<false>(tile, T, g, row, kl + kHalfBlock, vv);
            }
            __syncthreads();
            write_tile(M, Q, tile, T, tn, tm, k0, lane);
            __syncthreads();
        }
    }
}

// The (k-block, q) of a small-basis workgroup.  The launch is 1-D; workgroup b runs on XCD
// b % kXcd, each XCD takes a contiguous range of k-blocks, and the q of one k-block sit on
// consecutive slots of one XCD, so C(k) is fetched from HBM once and shared by the q in that XCD's
// L2.  False past the last k-block (the whole workgroup returns before any barrier).
__device__ __forceinline__ bool small_item(const MeshDev &M, int nq, int64_t &k0, int &qi)
{
    const int64_t nkb = (M.nk + kKPerBlock - 1) / kKPerBlock;
    const int64_t b = blockIdx.x;
    const int xcd = (int)(b % kXcd);
    const int64_t slot = b / kXcd;
    const int64_t per_xcd = (nkb + kXcd - 1) / kXcd;
    const int64_t kb = xcd * per_xcd + slot / nq;
    qi = (int)(slot % nq);
    k0 = kb * kKPerBlock;
    return kb < nkb;
}

// Dynamic LDS: the staging tile, tile_dim(nbw)^2 * kTileLd doubles.
__global__ __launch_bounds__(64) void contract_f64_kernel(MeshDev M, BatchDev B, int nq)
{
    extern __shared__ double tile[];
    int64_t k0;
    int qi;
    if (!small_item(M, nq, k0, qi)) return;
    contract_f64_body(M, B.q[qi], k0, tile);
}

template <bool FP16>
__global__ __launch_bounds__(64) void contract_split_kernel(MeshDev M, BatchDev B, int nq)
{
    extern __shared__ double tile[];
    int64_t k0;
    int qi;
    if (!small_item(M, nq, k0, qi)) return;
    contract_split_body<FP16>(M, B.q[qi], k0, tile);
}

// ---------------------------------------------------------------------------
// Large bases (plane waves): the contraction length n_orb runs to thousands, so one k is a
// genuine complex GEMM (nbw x n_orb)^H (n_orb x nbw) per q, and the q of one launch all share
// the k operand.  A workgroup is one k and up to kPwQ q (fewer when the launch has fewer), one wave
// per q; each wave computes the
// whole nbw x nbw block (NT x NT tiles of 16x16, NT = 1 or 2) over the whole reduction, so the
// k operand is fetched from HBM once and reaches the other waves through the caches.
//
// The complex product takes three real MFMAs instead of four (Gauss): with a = C(k) and
// b = C(k+q) per orbital,
//     P = sum (ar + ai)(br + bi),  R = sum ar bi,  S = sum ai br,
//     Re M = sum (ar br + ai bi) = P - R - S,   Im M = sum (ar bi - ai br) = R - S,
// and |M|^2 is formed from the three accumulators at the end.
//
// Workgroups are dispatched round-robin over the 8 XCDs.  The launch is 1-D and block b runs
// (k, qgroup) with xcd = b % 8, and each XCD takes a contiguous range of k: the q-groups of one k
// sit on consecutive slots of the same XCD, so their k operand is shared in that XCD's L2, and
// consecutive k of a band pair (adjacent 8-byte entries of W) are written through the same L2,
// which merges them into whole sectors.
// ---------------------------------------------------------------------------
constexpr int kPwQ = 8;      // q (waves) per workgroup
constexpr int kPwDepth = 4;  // steps of operands in flight per wave

// The (k, q) of this wave; false past the mesh or the last q.  blockDim.x / 64 q per workgroup
// (kPwQ, or nq when the launch has fewer).
__device__ __forceinline__ bool pw_item(const MeshDev &M, int nq, int n_qgroups, int64_t &k, int &qi)
{
    const int64_t b = blockIdx.x;
    const int xcd = (int)(b % kXcd);
    const int64_t slot = b / kXcd;
    const int64_t k_per_xcd = (M.nk + kXcd - 1) / kXcd;
    k = xcd * k_per_xcd + slot / n_qgroups;
    qi = (int)(slot % n_qgroups) * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6);
    return k < M.nk && qi < nq;
}

template <int NT>
__global__ __launch_bounds__(64 * kPwQ) void contract_pw_kernel(MeshDev M, BatchDev B, int nq, int n_qgroups)
{
    const int lane = threadIdx.x & 63;
    int64_t k;
    int qi;
    if (!pw_item(M, nq, n_qgroups, k, qi)) return;      // no barriers below: a wave may leave on its own
    const QDev Q = B.q[qi];
    const int64_t kq = shifted_k(M, Q, k);
    const int row = lane & 15, kk = lane >> 4;
    const int nb = M.nb, no = M.no;
    // operand rows of this lane: band t*16 + row of C(k) (A) and of C(k+q) (B), orbital o0 + kk
    const double *pa[NT];
    const double *pb[NT];
    bool ok[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int n = t * 16 + row;
        ok[t] = n < M.nbw;
        pa[t] = M.c_k + 2 * ((k * no) * nb + M.lo + (ok[t] ? n : 0));
        pb[t] = Q.c_kq + 2 * ((kq * no) * nb + M.lo + (ok[t] ? n : 0));
    }
    // one accumulator set per tile pair; with a single tile, two sets over alternating steps
    constexpr int NS = NT == 1 ? 2 : 1;
    dbl4 accP[NS][NT][NT], accR[NS][NT][NT], accS[NS][NT][NT];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int tn = 0; tn < NT; ++tn)
#pragma unroll
            for (int tm = 0; tm < NT; ++tm) {
                accP[s][tn][tm] = dbl4{0.0, 0.0, 0.0, 0.0};
                accR[s][tn][tm] = dbl4{0.0, 0.0, 0.0, 0.0};
                accS[s][tn][tm] = dbl4{0.0, 0.0, 0.0, 0.0};
            }
    // operands of kPwDepth steps of 4 orbitals in flight: the slot of a step is refilled with
    // the step kPwDepth later as soon as its MFMAs have been issued
    double ar[kPwDepth][NT], ai[kPwDepth][NT], br[kPwDepth][NT], bi[kPwDepth][NT];
    // Loads are unconditional (past the last orbital the address is clamped to it and the value
    // replaced by zero), so no branch separates a load from its use and the wait counters can let
    // the later steps' loads stay in flight.
    auto fetch = [&](int d, int o) {
        const int64_t off = 2 * (int64_t)min(o, no - 1) * nb;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const bool use = o < no && ok[t];
            const double2 a = *reinterpret_cast<const double2 *>(pa[t] + off);
            const double2 b = *reinterpret_cast<const double2 *>(pb[t] + off);
            ar[d][t] = use ? a.x : 0.0;
            ai[d][t] = use ? a.y : 0.0;
            br[d][t] = use ? b.x : 0.0;
            bi[d][t] = use ? b.y : 0.0;
        }
    };
#pragma unroll
    for (int d = 0; d < kPwDepth; ++d) fetch(d, 4 * d + kk);
    for (int o0 = 0; o0 < no; o0 += 4 * kPwDepth) {
#pragma unroll
        for (int d = 0; d < kPwDepth; ++d) {
            const int s = d % NS;
#pragma unroll
            for (int tn = 0; tn < NT; ++tn) {
                const double as = ar[d][tn] + ai[d][tn];
#pragma unroll
                for (int tm = 0; tm < NT; ++tm) {
                    const double bs = br[d][tm] + bi[d][tm];
                    accP[s][tn][tm] = __builtin_amdgcn_mfma_f64_16x16x4f64(as, bs, accP[s][tn][tm], 0, 0, 0);
                    accR[s][tn][tm] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[d][tn], bi[d][tm], accR[s][tn][tm], 0, 0, 0);
                    accS[s][tn][tm] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[d][tn], br[d][tm], accS[s][tn][tm], 0, 0, 0);
                }
            }
            fetch(d, o0 + 4 * (d + kPwDepth) + kk);
        }
    }
    // accumulator element v of this lane is D[kk + 4 v][row]: band n = tn*16 + kk + 4v, m = tm*16 + row
#pragma unroll
    for (int tn = 0; tn < NT; ++tn)
#pragma unroll
        for (int tm = 0; tm < NT; ++tm)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double P = accP[0][tn][tm][v], R = accR[0][tn][tm][v], S = accS[0][tn][tm][v];
#pragma unroll
                for (int s = 1; s < NS; ++s) {
                    P += accP[s][tn][tm][v];
                    R += accR[s][tn][tm][v];
                    S += accS[s][tn][tm][v];
                }
                const double re = P - R - S, im = R - S;
                const int nn = tn * 16 + kk + 4 * v, mm = tm * 16 + row;
                if (nn < M.nbw && mm < M.nbw)
                    Q.W[((int64_t)nn * M.nbw + mm) * M.nk + k] = re * re + im * im;
            }
}

// Split-precision forms for large bases: the workgroup and XCD layout of contract_pw_kernel, the
// folded two-GEMM product and hi/lo split of the small-basis form (16 orbitals per MFMA step).
// Coefficients arrive as FP64 and are split as they are used; each lane keeps pw_split_depth(NT)
// steps of its operands in flight (two for one tile, one for 2 x 2 tiles, whose operands and
// accumulators would otherwise not fit in 256 registers).
constexpr int pw_split_depth(int nt) { return nt == 1 ? 2 : 1; }

template <int NT, bool FP16>
__global__ __launch_bounds__(64 * kPwQ) void contract_pw_split_kernel(MeshDev M, BatchDev B, int nq, int n_qgroups)
{
    const int lane = threadIdx.x & 63;
    int64_t k;
    int qi;
    if (!pw_item(M, nq, n_qgroups, k, qi)) return;      // no barriers below: a wave may leave on its own
    const QDev Q = B.q[qi];
    const int64_t kq = shifted_k(M, Q, k);
    const int row = lane & 15, g = lane >> 4;
    const int nb = M.nb, no = M.no;
    const double *pa[NT];
    const double *pb[NT];
    bool ok[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int n = t * 16 + row;
        ok[t] = n < M.nbw;
        pa[t] = M.c_k + 2 * ((k * no) * nb + M.lo + (ok[t] ? n : 0));
        pb[t] = Q.c_kq + 2 * ((kq * no) * nb + M.lo + (ok[t] ? n : 0));
    }
    SplitAcc acc[NT][NT];
#pragma unroll
    for (int tn = 0; tn < NT; ++tn)
#pragma unroll
        for (int tm = 0; tm < NT; ++tm) acc[tn][tm].re = acc[tn][tm].re_c = acc[tn][tm].im = acc[tn][tm].im_c = flt4{0.f, 0.f, 0.f, 0.f};
    constexpr int D = pw_split_depth(NT);
    double2 av[D][NT][4], bv[D][NT][4];
    // unconditional loads, clamped to the last orbital and zeroed past it (as in contract_pw_kernel)
    auto fetch = [&](int d, int o0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = o0 + 4 * g + i;
            const int64_t off = 2 * (int64_t)min(o, no - 1) * nb;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const bool use = o < no && ok[t];
                const double2 a = *reinterpret_cast<const double2 *>(pa[t] + off);
                const double2 b = *reinterpret_cast<const double2 *>(pb[t] + off);
                av[d][t][i] = use ? a : double2{0.0, 0.0};
                bv[d][t][i] = use ? b : double2{0.0, 0.0};
            }
        }
    };
#pragma unroll
    for (int d = 0; d < D; ++d) fetch(d, 16 * d);
    for (int o0 = 0; o0 < no; o0 += 16 * D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            u32x4 ah[NT], al[NT], bh[NT], bl[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                split_op<FP16>(av[d][t], ah[t], al[t]);
                split_op<FP16>(bv[d][t], bh[t], bl[t]);
            }
            fetch(d, o0 + 16 * (d + D));
#pragma unroll
            for (int tn = 0; tn < NT; ++tn)
#pragma unroll
                for (int tm = 0; tm < NT; ++tm) split_step<FP16>(acc[tn][tm], ah[tn], al[tn], bh[tm], bl[tm]);
        }
    }
    // accumulator element v of this lane is D[4 g + v][row]: band n = tn*16 + 4g + v, m = tm*16 + row
#pragma unroll
    for (int tn = 0; tn < NT; ++tn)
#pragma unroll
        for (int tm = 0; tm < NT; ++tm)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int nn = tn * 16 + 4 * g + v, mm = tm * 16 + row;
                if (nn < M.nbw && mm < M.nbw) Q.W[((int64_t)nn * M.nbw + mm) * M.nk + k] = split_abs2<FP16>(acc[tn][tm], v);
            }
}

// Packed split operands.  When every q of a launch is a mesh shift, all its k+q operands are rows
// of the plan's own eigenvector array, so the split is done once per launch: pack_split_kernel
// writes, for every (k, block of 4 orbitals, band n of the window), the 32 bytes a lane loads for
// one MFMA step (hi of [re o..o+3, im o..o+3], then lo), and contract_pw_packed_kernel reads them
// for both operands: 8 bytes per coefficient instead of 16, and no conversion in the loop.
constexpr int kPackThreads = 256;

template <bool FP16>
__global__ __launch_bounds__(kPackThreads) void pack_split_kernel(MeshDev M, u32x4 *__restrict__ pack)
{
    const int nb4 = (M.no + 3) / 4;
    const int64_t total = M.nk * (int64_t)nb4 * M.nbw;
    for (int64_t e = (int64_t)blockIdx.x * kPackThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kPackThreads) {
        const int n = (int)(e % M.nbw);
        const int64_t t = e / M.nbw;
        const int blk = (int)(t % nb4);
        const int64_t k = t / nb4;
        double2 v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = 4 * blk + i;
            v[i] = o < M.no ? *reinterpret_cast<const double2 *>(M.c_k + 2 * ((k * M.no + o) * M.nb + M.lo + n))
                            : double2{0.0, 0.0};
        }
        u32x4 hi, lo;
        split_op<FP16>(v, hi, lo);
        pack[2 * e] = hi;
        pack[2 * e + 1] = lo;
    }
}

// Steps of packed operands in flight per wave: four (measured 3% faster than two for 2 x 2 tiles,
// 238 registers).
constexpr int kPwPackedDepth = 4;

template <int NT, bool FP16>
__global__ __launch_bounds__(64 * kPwQ) void contract_pw_packed_kernel(MeshDev M, BatchDev B, int nq, int n_qgroups,
                                                                        const u32x4 *__restrict__ pack)
{
    const int lane = threadIdx.x & 63;
    int64_t k;
    int qi;
    if (!pw_item(M, nq, n_qgroups, k, qi)) return;      // no barriers below: a wave may leave on its own
    const QDev Q = B.q[qi];
    const int64_t kq = shifted_k(M, Q, k);
    const int row = lane & 15, g = lane >> 4;
    const int nb4 = (M.no + 3) / 4;
    const int nsteps = (nb4 + 3) / 4;      // steps of 16 orbitals (4 blocks of 4)
    const u32x4 *pa[NT];
    const u32x4 *pb[NT];
    bool ok[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int n = t * 16 + row;
        ok[t] = n < M.nbw;
        pa[t] = pack + 2 * ((k * nb4) * M.nbw + (ok[t] ? n : 0));
        pb[t] = pack + 2 * ((kq * nb4) * M.nbw + (ok[t] ? n : 0));
    }
    SplitAcc acc[NT][NT];
#pragma unroll
    for (int tn = 0; tn < NT; ++tn)
#pragma unroll
        for (int tm = 0; tm < NT; ++tm) acc[tn][tm].re = acc[tn][tm].re_c = acc[tn][tm].im = acc[tn][tm].im_c = flt4{0.f, 0.f, 0.f, 0.f};
    constexpr int D = kPwPackedDepth;
    u32x4 ah[D][NT], al[D][NT], bh[D][NT], bl[D][NT];
    const u32x4 zero = {0u, 0u, 0u, 0u};
    // unconditional loads, clamped to the last block and zeroed past it
    auto fetch = [&](int d, int step) {
        const int blk = 4 * step + g;
        const int64_t off = 2 * (int64_t)min(blk, nb4 - 1) * M.nbw;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const bool use = blk < nb4 && ok[t];
            const u32x4 a0 = pa[t][off], a1 = pa[t][off + 1];
            const u32x4 b0 = pb[t][off], b1 = pb[t][off + 1];
            ah[d][t] = use ? a0 : zero;
            al[d][t] = use ? a1 : zero;
            bh[d][t] = use ? b0 : zero;
            bl[d][t] = use ? b1 : zero;
        }
    };
#pragma unroll
    for (int d = 0; d < D; ++d) fetch(d, d);
    for (int s0 = 0; s0 < nsteps; s0 += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            u32x4 xh[NT], xl[NT], yh[NT], yl[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                xh[t] = ah[d][t];
                xl[t] = al[d][t];
                yh[t] = bh[d][t];
                yl[t] = bl[d][t];
            }
            fetch(d, s0 + d + D);
#pragma unroll
            for (int tn = 0; tn < NT; ++tn)
#pragma unroll
                for (int tm = 0; tm < NT; ++tm) split_step<FP16>(acc[tn][tm], xh[tn], xl[tn], yh[tm], yl[tm]);
        }
    }
#pragma unroll
    for (int tn = 0; tn < NT; ++tn)
#pragma unroll
        for (int tm = 0; tm < NT; ++tm)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int nn = tn * 16 + 4 * g + v, mm = tm * 16 + row;
                if (nn < M.nbw && mm < M.nbw) Q.W[((int64_t)nn * M.nbw + mm) * M.nk + k] = split_abs2<FP16>(acc[tn][tm], v);
            }
}

// Fused launch over the (instance, q) items of a batch: workgroup -> item from a table.
__global__ __launch_bounds__(64) void contract_batch_kernel(const BatchItemDev *__restrict__ items,
                                                            const int32_t *__restrict__ block_item)
{
    __shared__ double tile[16 * 16 * kTileLd];
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

size_t pack_bytes(const MeshDev &mesh)
{
    return (size_t)mesh.nk * (size_t)((mesh.no + 3) / 4) * (size_t)mesh.nbw * 2 * sizeof(u32x4);
}

hipError_t launch_contract(const MeshDev &mesh, const BatchDev &batch, int nq, int precision, PackState *pack,
                           hipStream_t s)
{
    if (nq < 1 || nq > kMaxQBatch) return hipErrorInvalidValue;
    if (mesh.no > kMaxOrbSmall) {
        // large (plane-wave) bases: one workgroup per (k, group of up to kPwQ q)
        if (mesh.nbw > 32) return hipErrorInvalidValue;
        const int gq = nq < kPwQ ? nq : kPwQ;           // q (waves) per workgroup
        const int ng = (nq + gq - 1) / gq;
        const int64_t k_per_xcd = (mesh.nk + kXcd - 1) / kXcd;
        const int64_t nblk = k_per_xcd * kXcd * ng;
        if (nblk >= (int64_t(1) << 31)) return hipErrorInvalidValue;
        const dim3 grid((unsigned)nblk), block(64 * gq);
        const bool two = mesh.nbw > 16;
        bool shifts = true;
        for (int i = 0; i < nq; ++i) shifts = shifts && !batch.q[i].explicit_kq;
        if (precision != 0 && pack && pack->ptr && shifts && nq >= kPackMinQ) {
            u32x4 *pk = static_cast<u32x4 *>(pack->ptr);
            const int64_t total = mesh.nk * (int64_t)((mesh.no + 3) / 4) * mesh.nbw;
            const unsigned pblk = (unsigned)std::min<int64_t>((total + kPackThreads - 1) / kPackThreads, 65536);
            const bool fill = !pack->valid;
            pack->valid = true;
            if (precision == 1) {
                if (fill) hipLaunchKernelGGL(pack_split_kernel<false>, dim3(pblk), dim3(kPackThreads), 0, s, mesh, pk);
                if (two) hipLaunchKernelGGL((contract_pw_packed_kernel<2, false>), grid, block, 0, s, mesh, batch, nq, ng, pk);
                else hipLaunchKernelGGL((contract_pw_packed_kernel<1, false>), grid, block, 0, s, mesh, batch, nq, ng, pk);
            } else {
                if (fill) hipLaunchKernelGGL(pack_split_kernel<true>, dim3(pblk), dim3(kPackThreads), 0, s, mesh, pk);
                if (two) hipLaunchKernelGGL((contract_pw_packed_kernel<2, true>), grid, block, 0, s, mesh, batch, nq, ng, pk);
                else hipLaunchKernelGGL((contract_pw_packed_kernel<1, true>), grid, block, 0, s, mesh, batch, nq, ng, pk);
            }
            return hipGetLastError();
        }
        if (precision == 1) {
            if (two) hipLaunchKernelGGL((contract_pw_split_kernel<2, false>), grid, block, 0, s, mesh, batch, nq, ng);
            else hipLaunchKernelGGL((contract_pw_split_kernel<1, false>), grid, block, 0, s, mesh, batch, nq, ng);
        } else if (precision == 2) {
            if (two) hipLaunchKernelGGL((contract_pw_split_kernel<2, true>), grid, block, 0, s, mesh, batch, nq, ng);
            else hipLaunchKernelGGL((contract_pw_split_kernel<1, true>), grid, block, 0, s, mesh, batch, nq, ng);
        } else {
            if (two) hipLaunchKernelGGL(contract_pw_kernel<2>, grid, block, 0, s, mesh, batch, nq, ng);
            else hipLaunchKernelGGL(contract_pw_kernel<1>, grid, block, 0, s, mesh, batch, nq, ng);
        }
        return hipGetLastError();
    }
    const int64_t nkb = (mesh.nk + kKPerBlock - 1) / kKPerBlock;
    const int64_t nblk = (nkb + kXcd - 1) / kXcd * kXcd * nq;
    if (nblk >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    const int T = tile_dim(mesh.nbw);
    const size_t lds = (size_t)T * T * kTileLd * sizeof(double);
    const dim3 grid((unsigned)nblk), block(64);
    if (precision == 1)
        hipLaunchKernelGGL(contract_split_kernel<false>, grid, block, lds, s, mesh, batch, nq);
    else if (precision == 2)
        hipLaunchKernelGGL(contract_split_kernel<true>, grid, block, lds, s, mesh, batch, nq);
    else
        hipLaunchKernelGGL(contract_f64_kernel, grid, block, lds, s, mesh, batch, nq);
    return hipGetLastError();
}

}  // namespace chi0
