// chi0_math.h -- per-tetrahedron arithmetic of the chi0 path: double carving of a
// mesh tetrahedron and the analytic integral of W/(w - D + i0) over a final
// tetrahedron (Heil et al., arXiv:1407.3444, Sec. II).
//
// Everything here is header-only and compiles for the GPU and for the host, so
// the same code can be exercised on the CPU by the host-side checks.
//
// Integral over a final tetrahedron S with corner values D_j, weights W_j:
//   (1/|S|) int_S W / (w - D + i0) = sum_j W_j J_j,   J_j = dG/dD_j,
//   G(D_1..D_4) = h[D_1, D_2, D_3, D_4],   h(x) = (w - x)^3 Log(w - x + i0),
// the third divided difference of h (Hermite-Genocchi: h''' = -6 Log, and a
// derivative with respect to a node doubles that node).  The W-weighted sum
// is therefore the directional derivative of G along (W_1..W_4), evaluated
// here by forward-mode differentiation of the divided-difference computation.
//
//  * far branch (all nodes within rho * |w - c| of their centre c; rho = kRhoFar for the FP64
//    series of the multi-frequency kernels, kRhoFar32 for their FP32 series, kRhoOne for a
//    single frequency):
//    G = sum_m h^(3+m)(c)/(3+m)! H_m(D - c), H_m the complete homogeneous
//    symmetric polynomial.  Its W-derivative is a power series in
//    t = 1/(w - c) whose coefficients depend only on the tetrahedron, so they
//    are computed once per tetrahedron and each frequency costs one Horner
//    evaluation.  No logarithm, and Im = 0 (w lies outside the D range).
//  * near branch: Newton recursion on the sorted nodes from the four
//    logarithms, where an entry whose nodes cluster tightly compared with
//    their distance from w is summed as a short Taylor series about its
//    farther end node (exact for tied nodes).
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define C0_HD __host__ __device__ __forceinline__
#else
#define C0_HD inline
#endif

namespace chi0 {

constexpr double kPi = 3.14159265358979323846;
#ifndef CHI0_FAR_TERMS
#define CHI0_FAR_TERMS 50
#define CHI0_RHO_FAR 0.5
#endif
#ifndef CHI0_THETA_ENTRY
#define CHI0_THETA_ENTRY 0.1
#endif
constexpr int kFarTerms = CHI0_FAR_TERMS;          // series terms kept in the far branch
constexpr double kRhoFar = CHI0_RHO_FAR;           // far branch when half-span <= kRhoFar * |w - c|
constexpr double kThetaEntry = CHI0_THETA_ENTRY;   // series sub-entry when span <= kThetaEntry * |w - x_end|
// Mixed-precision form: the far series in FP32 with kFarTerms32 terms at the ratio kRhoFar32
// (0.4^20 ~ 1e-8, the FP32 resolution); its near branch runs in FP32 and is cheap enough that
// the smaller ratio pays.  Near-degenerate tetrahedra keep the FP64 near evaluation.
#ifndef CHI0_FAR_TERMS32
#define CHI0_FAR_TERMS32 20
#define CHI0_RHO_FAR32 0.4
#endif
constexpr int kFarTerms32 = CHI0_FAR_TERMS32;
constexpr double kRhoFar32 = CHI0_RHO_FAR32;

struct cplx {
    double re, im;
};

C0_HD cplx cmk(double r, double i) { cplx z; z.re = r; z.im = i; return z; }

// 1/d: on the GPU the hardware estimate (relative error below 5e-8 on gfx950) refined by one
// third-order step t (1 + e + e^2), e = 1 - d t, which leaves e^3 < 1e-22: within an ulp or two
// of the correctly rounded quotient, without the division's scaling and fix-up sequence
C0_HD double rcp(double d)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const double t = __builtin_amdgcn_rcp(d);
    const double e = fma(-d, t, 1.0);
    return fma(t, fma(e, e, e), t);
#else
    return 1.0 / d;
#endif
}
C0_HD cplx cadd(cplx a, cplx b) { return cmk(a.re + b.re, a.im + b.im); }
C0_HD cplx csub(cplx a, cplx b) { return cmk(a.re - b.re, a.im - b.im); }
C0_HD cplx cscale(cplx a, double s) { return cmk(a.re * s, a.im * s); }
C0_HD cplx cfma(cplx acc, cplx a, double s) { return cmk(fma(a.re, s, acc.re), fma(a.im, s, acc.im)); }

// ---------------------------------------------------------------------------
// Carving (Sec. II: first carving by e = mu, second carving by e' = mu)
// ---------------------------------------------------------------------------

// Corner attributes carried through the carving: a = e - mu, b = e' - mu,
// D = e' - e, W = |M|^2.  All four are linear on a tetrahedron.
struct Vtx {
    double a, b, D, W;
};

C0_HD Vtx vlerp(const Vtx &p, const Vtx &q, double t)
{
    Vtx r;
    r.a = fma(t, q.a - p.a, p.a);
    r.b = fma(t, q.b - p.b, p.b);
    r.D = fma(t, q.D - p.D, p.D);
    r.W = fma(t, q.W - p.W, p.W);
    return r;
}

C0_HD void vswap_if(bool c, Vtx &x, Vtx &y, double &fx, double &fy)
{
    if (c) {
        Vtx t = x; x = y; y = t;
        double g = fx; fx = fy; fy = g;
    }
}

// The clipping function f of a vertex: which attribute and with which sign.
// KEEP_NEG_A: keep a < 0;  KEEP_POS_A: keep a > 0;  same for b.
enum ClipKind { KEEP_NEG_A = 0, KEEP_POS_A = 1, KEEP_NEG_B = 2, KEEP_POS_B = 3 };

C0_HD double clip_value(const Vtx &v, int kind)
{
    switch (kind) {
    case KEEP_NEG_A: return v.a;
    case KEEP_POS_A: return -v.a;
    case KEEP_NEG_B: return v.b;
    default: return -v.b;
    }
}

// Keep the part of tetrahedron (t0..t3, volume fraction vol) where f < 0 and
// hand each resulting tetrahedron to sink(v0, v1, v2, v3, vol).  0, 1 or 3 pieces.
// Volume fractions are products of the edge parameters, never determinants.
template <class Sink>
C0_HD void clip_neg(Vtx t0, Vtx t1, Vtx t2, Vtx t3, double vol, int kind, Sink &sink)
{
    double f0 = clip_value(t0, kind), f1 = clip_value(t1, kind);
    double f2 = clip_value(t2, kind), f3 = clip_value(t3, kind);
    // partition: inside (f < 0) vertices first (a sorting network on the key f >= 0)
    vswap_if(f0 >= 0.0 && f1 < 0.0, t0, t1, f0, f1);
    vswap_if(f2 >= 0.0 && f3 < 0.0, t2, t3, f2, f3);
    vswap_if(f0 >= 0.0 && f2 < 0.0, t0, t2, f0, f2);
    vswap_if(f1 >= 0.0 && f3 < 0.0, t1, t3, f1, f3);
    vswap_if(f1 >= 0.0 && f2 < 0.0, t1, t2, f1, f2);
    const int nin = (f0 < 0.0) + (f1 < 0.0) + (f2 < 0.0) + (f3 < 0.0);
    if (nin == 0) return;
    if (nin == 4) { sink(t0, t1, t2, t3, vol); return; }
    if (nin == 1) {
        // corner tetrahedron at t0; s_k = fraction of edge t0->tk
        const double s1 = f0 / (f0 - f1), s2 = f0 / (f0 - f2), s3 = f0 / (f0 - f3);
        sink(t0, vlerp(t0, t1, s1), vlerp(t0, t2, s2), vlerp(t0, t3, s3), vol * s1 * s2 * s3);
        return;
    }
    if (nin == 3) {
        // tetrahedron minus the corner at t3: prism (t0,t1,t2 | P0,P1,P2), P_i on edge t_i->t3
        const double s0 = f0 / (f0 - f3), s1 = f1 / (f1 - f3), s2 = f2 / (f2 - f3);
        const double r0 = f3 / (f3 - f0), r1 = f3 / (f3 - f1);   // 1 - s_i without cancellation
        const Vtx P0 = vlerp(t0, t3, s0), P1 = vlerp(t1, t3, s1), P2 = vlerp(t2, t3, s2);
        sink(t0, t1, t2, P0, vol * s0);
        sink(t1, t2, P0, P1, vol * r0 * s1);
        sink(t2, P0, P1, P2, vol * r0 * r1 * s2);
        return;
    }
    // nin == 2: prism with ends (t0, P02, P03) and (t1, P12, P13)
    const double s02 = f0 / (f0 - f2), s03 = f0 / (f0 - f3);
    const double s12 = f1 / (f1 - f2), s13 = f1 / (f1 - f3);
    const double r02 = f2 / (f2 - f0), r03 = f3 / (f3 - f0);       // 1 - s02, 1 - s03
    const Vtx P02 = vlerp(t0, t2, s02), P03 = vlerp(t0, t3, s03);
    const Vtx P12 = vlerp(t1, t2, s12), P13 = vlerp(t1, t3, s13);
    sink(t0, P02, P03, t1, vol * s02 * s03);
    sink(P02, P03, t1, P12, vol * s03 * s12 * r02);
    sink(P03, t1, P12, P13, vol * r03 * s12 * s13);
}

// Second carving stage: forwards every piece clipped by the second function.
template <class Sink>
struct SecondClip {
    int kind;
    Sink *out;
    C0_HD void operator()(const Vtx &v0, const Vtx &v1, const Vtx &v2, const Vtx &v3, double vol)
    {
        clip_neg(v0, v1, v2, v3, vol, kind, *out);
    }
};

// Region 1 = {e < mu < e'} (n occupied at k, m empty at k+q); region 2 = {e' < mu < e}.
template <class Sink>
C0_HD void carve_region(const Vtx &t0, const Vtx &t1, const Vtx &t2, const Vtx &t3, int region,
                        Sink &sink)
{
    SecondClip<Sink> second;
    second.kind = region == 1 ? KEEP_POS_B : KEEP_NEG_B;
    second.out = &sink;
    clip_neg(t0, t1, t2, t3, 1.0, region == 1 ? KEEP_NEG_A : KEEP_POS_A, second);
}

// Quick tests on the corner values before any carving.
C0_HD bool region_empty(const Vtx &t0, const Vtx &t1, const Vtx &t2, const Vtx &t3, int region)
{
    if (region == 1)
        return (t0.a >= 0.0 && t1.a >= 0.0 && t2.a >= 0.0 && t3.a >= 0.0) ||
               (t0.b <= 0.0 && t1.b <= 0.0 && t2.b <= 0.0 && t3.b <= 0.0);
    return (t0.a <= 0.0 && t1.a <= 0.0 && t2.a <= 0.0 && t3.a <= 0.0) ||
           (t0.b >= 0.0 && t1.b >= 0.0 && t2.b >= 0.0 && t3.b >= 0.0);
}

// ---------------------------------------------------------------------------
// Final-tetrahedron weights
// ---------------------------------------------------------------------------

// Sort the four (D, W) pairs by D ascending (5 compare-exchanges).
C0_HD void sort4(double y[4], double w[4])
{
#define C0_CX(i, j)                                                         \
    if (y[j] < y[i]) {                                                      \
        double ty = y[i]; y[i] = y[j]; y[j] = ty;                           \
        double tw = w[i]; w[i] = w[j]; w[j] = tw;                           \
    }
    C0_CX(0, 1) C0_CX(2, 3) C0_CX(0, 2) C0_CX(1, 3) C0_CX(1, 2)
#undef C0_CX
}

// Far-branch coefficients: sum_j W_j J_j = sum_{m=1..K} a[m-1] t^m, t = 1/(w - c),
// a_m = 6/(m(m+1)(m+2)(m+3)) * d/dW H_m(D - c)   (valid for half-span < |w - c|).
template <int K = kFarTerms>
C0_HD void far_coeffs(const double y[4], const double w[4], double c, double *a)
{
    double z0 = y[0] - c, z1 = y[1] - c, z2 = y[2] - c, z3 = y[3] - c;
    double P0 = 1.0, P1 = 1.0, P2 = 1.0, P3 = 1.0;      // H_{m-1} over growing variable sets
    double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;      // their W-derivatives
#pragma unroll
    for (int m = 1; m <= K; ++m) {
        double n0 = z0 * P0;
        double e0 = fma(w[0], P0, z0 * d0);
        double n1 = fma(z1, P1, n0);
        double e1 = fma(w[1], P1, fma(z1, d1, e0));
        double n2 = fma(z2, P2, n1);
        double e2 = fma(w[2], P2, fma(z2, d2, e1));
        double n3 = fma(z3, P3, n2);
        double e3 = fma(w[3], P3, fma(z3, d3, e2));
        P0 = n0; P1 = n1; P2 = n2; P3 = n3;
        d0 = e0; d1 = e1; d2 = e2; d3 = e3;
        const double mm = (double)m;
        a[m - 1] = 6.0 / (mm * (mm + 1.0) * (mm + 2.0) * (mm + 3.0)) * e3;
    }
}

// The same coefficients in blocks of K / NB terms, only the first nblocks blocks (the terms a
// class-cut Horner sum reads); a[] past them is left untouched.
template <int K, int NB>
C0_HD void far_coeffs_blocks(const double y[4], const double w[4], double c, double *a, int nblocks)
{
    constexpr int S = K / NB;
    double z0 = y[0] - c, z1 = y[1] - c, z2 = y[2] - c, z3 = y[3] - c;
    double P0 = 1.0, P1 = 1.0, P2 = 1.0, P3 = 1.0;
    double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (b >= nblocks) continue;        // (not break: the loop stays unrolled)
#pragma unroll
        for (int j = 1; j <= S; ++j) {
            const int m = b * S + j;
            double n0 = z0 * P0;
            double e0 = fma(w[0], P0, z0 * d0);
            double n1 = fma(z1, P1, n0);
            double e1 = fma(w[1], P1, fma(z1, d1, e0));
            double n2 = fma(z2, P2, n1);
            double e2 = fma(w[2], P2, fma(z2, d2, e1));
            double n3 = fma(z3, P3, n2);
            double e3 = fma(w[3], P3, fma(z3, d3, e2));
            P0 = n0; P1 = n1; P2 = n2; P3 = n3;
            d0 = e0; d1 = e1; d2 = e2; d3 = e3;
            const double mm = (double)m;
            a[m - 1] = 6.0 / (mm * (mm + 1.0) * (mm + 2.0) * (mm + 3.0)) * e3;
        }
    }
}

template <int K = kFarTerms>
C0_HD double far_horner(const double *a, double t)
{
    double s = a[K - 1];
#pragma unroll
    for (int m = K - 2; m >= 0; --m) s = fma(s, t, a[m]);
    return s * t;
}

// Truncation of the far series for a group of frequencies (all frequencies one wave evaluates
// together, i.e. those of one launch).  A frequency of the group that takes the far branch has
// |w - c| >= max(dist, hs / rho), dist = distance from c to the group's frequency interval and
// rho the form's far ratio, so its ratio hs / |w - c| is at most rho_g = min(rho, hs / dist).  The
// remainder after n terms is bounded by a factor polynomial in n times rho_g^n |t|, so n <= K terms
// with rho_g^n <= rho^K keep the error bound of the full K-term series at the largest ratio rho.
// The group gets class
// j = 1..kFarClasses (n = j K / kFarClasses terms), the smallest j with
// j >= kFarClasses ln(rho) / ln(rho_g); class 0 when every frequency of the group is near.
constexpr int kFarClasses = 10;

// (rho is the far ratio of the form: kRhoFar, or kRhoFar32 for the FP32 series.)
C0_HD int far_class(double hs, double dist, double dfar, double rho = kRhoFar)
{
    if (!(hs <= rho * dfar)) return 0;              // the farthest frequency is near too
    if (!(hs < rho * dist)) return kFarClasses;     // rho_g = rho (also dist = 0)
    // j = ceil(kFarClasses log2(1/rho) / log2(dist/hs)) with a small upward margin; a huge
    // ratio (hs = 0 included) gives log2 = inf and class 1
    const float lx = log2f((float)(dist / hs));
    const float q = (float)kFarClasses * log2f((float)(1.0 / rho)) * 1.00001f / lx;
    const int j = (int)ceilf(q);
    return j < 1 ? 1 : (j > kFarClasses ? kFarClasses : j);
}

C0_HD double fmaT(double a, double b, double c) { return fma(a, b, c); }
C0_HD float fmaT(float a, float b, float c) { return fmaf(a, b, c); }

// Horner sum over the first cls * K / kFarClasses coefficients (highest first), without the
// final factor t: sum_{m < n} a[m] t^m.  Class 0 gives 0.  cls is uniform over the wave in the
// kernels, so every block test is a scalar branch.
template <int K, class T>
C0_HD T far_horner_cls(const T *a, T t, int cls)
{
    constexpr int S = K / kFarClasses;
    static_assert(S * kFarClasses == K, "term count must be a multiple of the class count");
    T s = T(0);
#pragma unroll
    for (int j = kFarClasses; j >= 1; --j) {
        if (j <= cls) {
#pragma unroll
            for (int m = j * S - 1; m >= (j - 1) * S; --m) s = fmaT(s, t, a[m]);
        }
    }
    return s;
}

// ---------------------------------------------------------------------------
// Near branch, in FP64 or (mixed form) FP32.  Node values, weights and frequency come in as
// FP64; differences of them (u = w - y_i, spans, offsets) are formed in FP64 and only then
// rounded to the working type T, so no difference is taken in T.
// ---------------------------------------------------------------------------
template <class T>
struct cx {
    T re, im;
};

template <class T> C0_HD cx<T> cxm(T r, T i) { cx<T> z; z.re = r; z.im = i; return z; }
template <class T> C0_HD cx<T> cxsub(cx<T> a, cx<T> b) { return cxm<T>(a.re - b.re, a.im - b.im); }
template <class T> C0_HD cx<T> cxscale(cx<T> a, T s) { return cxm<T>(a.re * s, a.im * s); }
template <class T> C0_HD cx<T> cxfma(cx<T> acc, cx<T> a, T s) { return cxm<T>(fmaT(a.re, s, acc.re), fmaT(a.im, s, acc.im)); }
template <class T> C0_HD cx<T> cxsel(bool c, cx<T> a, cx<T> b) { return cxm<T>(c ? a.re : b.re, c ? a.im : b.im); }

// Natural logarithm of a positive finite x (the near branch's leaves): x = m 2^e with m in
// [1/sqrt2, sqrt2), log x = e ln2 + 2 atanh(f), f = (m - 1)/(m + 1), |f| <= 3 - 2 sqrt2 < 0.1716,
// and atanh(f)/f = sum_k f^(2k)/(2k + 1) summed to k = 11 (f^24 < 4e-19).  m - 1 is exact, f carries
// the error of one reciprocal, ln2 is split so that e ln2_hi is exact: within a few ulp of the
// correctly rounded value, at a third of the instructions of the library logarithm (which keeps
// extra precision through double-double sums).
C0_HD double log_pos(double x)
{
    int e;
    double m = frexp(x, &e);                       // m in [0.5, 1)
    const bool lo = m < 0.70710678118654752440;
    m = lo ? 2.0 * m : m;
    e = lo ? e - 1 : e;
    const double f = (m - 1.0) * rcp(m + 1.0);
    const double f2 = f * f;
    double p = 1.0 / 23.0;
    p = fma(p, f2, 1.0 / 21.0);
    p = fma(p, f2, 1.0 / 19.0);
    p = fma(p, f2, 1.0 / 17.0);
    p = fma(p, f2, 1.0 / 15.0);
    p = fma(p, f2, 1.0 / 13.0);
    p = fma(p, f2, 1.0 / 11.0);
    p = fma(p, f2, 1.0 / 9.0);
    p = fma(p, f2, 1.0 / 7.0);
    p = fma(p, f2, 1.0 / 5.0);
    p = fma(p, f2, 1.0 / 3.0);
    const double twof = 2.0 * f;
    const double ed = (double)e;
    // ln 2 = kLn2Hi + kLn2Lo, kLn2Hi with 32 significant bits (e ln2_hi exact for |e| < 2^21)
    constexpr double kLn2Hi = 0.693147180369123816490;
    constexpr double kLn2Lo = 1.90821492927058770002e-10;
    return fma(ed, kLn2Hi, fma(ed, kLn2Lo, fma(twof * f2, p, twof)));
}

C0_HD double logT(double x) { return log_pos(x); }
C0_HD float logT(float x) { return logf(x); }
C0_HD double absT(double x) { return fabs(x); }
C0_HD float absT(float x) { return fabsf(x); }
C0_HD float rcp(float d)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const float t = __builtin_amdgcn_rcpf(d);
    return fmaf(t, fmaf(-d, t, 1.0f), t);
#else
    return 1.0f / d;
#endif
}

// Entry series: kEntryTerms terms in FP64; in FP32 the series is selected up to the wider
// kThetaEntry32 (so the Newton recursion loses at most a factor 1/kThetaEntry32 per level) and
// needs kEntryTerms32 terms for the FP32 resolution.
#ifndef CHI0_ENTRY_TERMS
#define CHI0_ENTRY_TERMS 12
#endif
#ifndef CHI0_ENTRY_TERMS32
#define CHI0_ENTRY_TERMS32 10
#endif
#ifndef CHI0_THETA_ENTRY32
#define CHI0_THETA_ENTRY32 0.3
#endif
#ifndef CHI0_DEFER_PAIR_SERIES
#define CHI0_DEFER_PAIR_SERIES 1
#endif
// 2-node entries in FP64: the series is selected below the smaller ratio kThetaPair, with
// kPairTerms terms; between kThetaPair and kThetaEntry the recursion loses at most a factor
// 1/kThetaPair of relative accuracy on the entry.
#ifndef CHI0_THETA_PAIR
#define CHI0_THETA_PAIR 0.02
#endif
#ifndef CHI0_PAIR_TERMS
#define CHI0_PAIR_TERMS 8
#endif
constexpr double kThetaPair = CHI0_THETA_PAIR;
constexpr int kPairTerms = CHI0_PAIR_TERMS;
constexpr int kEntryTerms = CHI0_ENTRY_TERMS;
constexpr int kEntryTerms32 = CHI0_ENTRY_TERMS32;
constexpr double kThetaEntry32 = CHI0_THETA_ENTRY32;

template <class T> struct NearParams;
template <> struct NearParams<double> {
    static constexpr int terms = kEntryTerms;
    static constexpr double theta = kThetaEntry;
    static constexpr int pair_terms = kPairTerms;
    static constexpr double theta_pair = kThetaPair;
};
template <> struct NearParams<float> {
    static constexpr int terms = kEntryTerms32;
    static constexpr double theta = kThetaEntry32;
    static constexpr int pair_terms = kEntryTerms32;
    static constexpr double theta_pair = kThetaEntry32;
};

C0_HD double entry_coef(int n) { return 6.0 / ((double)n * (n - 1) * (n - 2) * (n - 3)); }

// h^(n)/n! (x-derivatives of h(x) = u^3 L, u = w - x, L = Log(u + i0)) for n <= 3.
template <class T>
C0_HD cx<T> hder_low(int n, T u, cx<T> L)
{
    switch (n) {
    case 0: { T u3 = u * u * u; return cxm<T>(u3 * L.re, u3 * L.im); }
    case 1: { T u2 = u * u; return cxm<T>(-(T(3) * u2 * L.re + u2), -T(3) * u2 * L.im); }
    case 2: return cxm<T>(T(3) * u * L.re + T(2.5) * u, T(3) * u * L.im);
    default: return cxm<T>(-(L.re + T(11.0 / 6.0)), -L.im);
    }
}

// Value and W-derivative of a divided difference of h over P+1 nodes (P = 1, 2) as a
// Taylor series about one of its nodes, e (u = w - y_e, L = Log(u)):
//   h[..] = sum_m h^(P+m)(y_e)/(P+m)! H_m(y - y_e),
// H_m the complete homogeneous symmetric polynomial of the offsets, scaled by 1/u.  The
// offset of e itself is exactly 0, so H_m only runs over the other P offsets z (with
// W-derivatives dz) and dH_m gains dz_e H_{m-1}.  Exact to rounding when the nodes lie within
// theta |u| of y_e; computed for every lane (no data-dependent trip count).

// P = 1: nodes y_e and y_o (offset yo_ye = y_o - y_e).  H_m = z^m, dH_m = z^(m-1) (dz_e + m dz_o).
template <class T>
C0_HD void taylor_pair(T yo_ye, T we, T wo, T u, cx<T> L, cx<T> &val, cx<T> &tan)
{
    const T inv = rcp(u);
    const T z = yo_ye * inv, dze = we * inv, dzo = wo * inv;
    // m = 0, 1, 2: the first, second and third derivative terms (logarithmic, complex)
    const cx<T> h1 = hder_low<T>(1, u, L), h2 = hder_low<T>(2, u, L), h3 = hder_low<T>(3, u, L);
    val = h1;
    tan = cxm<T>(T(0), T(0));
    val = cxfma(val, h2, u * z);
    tan = cxfma(tan, h2, u * (dze + dzo));
    val = cxfma(val, h3, u * u * z * z);
    tan = cxfma(tan, h3, u * u * z * (dze + T(2) * dzo));
    // m >= 3: real coefficients 6/(n(n-1)(n-2)(n-3)) u^2, n = m + 1
    T zprev = z * z, sv = T(0), st = T(0);
#pragma unroll
    for (int m = 3; m < NearParams<T>::pair_terms; ++m) {
        const T zm = zprev * z;
        const T cf = T(entry_coef(m + 1));
        sv = fmaT(cf, zm, sv);
        st = fmaT(cf * zprev, fmaT(T(m), dzo, dze), st);
        zprev = zm;
    }
    const T u2 = u * u;
    val.re = fmaT(sv, u2, val.re);
    tan.re = fmaT(st, u2, tan.re);
}

// P = 2: nodes y_e, y_1, y_2 (offsets from y_e).  H_m = H_m(z1, z2) by the recurrence over the
// two offsets.
template <class T>
C0_HD void taylor_triple(T y1_ye, T y2_ye, T we, T w1, T w2, T u, cx<T> L, cx<T> &val, cx<T> &tan)
{
    const T inv = rcp(u);
    const T z1 = y1_ye * inv, z2 = y2_ye * inv;
    const T dze = we * inv, dz1 = w1 * inv, dz2 = w2 * inv;
    T A = T(1), dA = T(0), Bv = T(1), dB = T(0);      // H_m(z1), H_m(z1, z2) and derivatives
    // m = 0, 1: the second and third derivative terms (logarithmic, complex)
    const cx<T> h2 = hder_low<T>(2, u, L), h3 = hder_low<T>(3, u, L);
    val = h2;
    tan = cxm<T>(T(0), T(0));
    {
        const T nA = A * z1, ndA = dz1 * A + z1 * dA;
        const T nB = fmaT(z2, Bv, nA), ndB = fmaT(dz2, Bv, fmaT(z2, dB, ndA));
        const T dH = fmaT(dze, Bv, ndB);
        val = cxfma(val, h3, u * nB);
        tan = cxfma(tan, h3, u * dH);
        A = nA; dA = ndA; Bv = nB; dB = ndB;
    }
    T sv = T(0), st = T(0);
#pragma unroll
    for (int m = 2; m < NearParams<T>::terms; ++m) {
        const T nA = A * z1, ndA = fmaT(dz1, A, z1 * dA);
        const T nB = fmaT(z2, Bv, nA), ndB = fmaT(dz2, Bv, fmaT(z2, dB, ndA));
        const T dH = fmaT(dze, Bv, ndB);
        const T cf = T(entry_coef(m + 2));
        sv = fmaT(cf, nB, sv);
        st = fmaT(cf, dH, st);
        A = nA; dA = ndA; Bv = nB; dB = ndB;
    }
    val.re = fmaT(sv, u, val.re);
    tan.re = fmaT(st, u, tan.re);
}

// One Newton entry over nodes y[0..P] (P = 1, 2) from its two children A = [y_1..y_P] and
// B = [y_0..y_{P-1}], or, when its nodes cluster within theta of their distance to w, from the
// Taylor series about its end node farther from w.  y: FP64 node values; u: w - y in T.
// SERIES = false: the series is not evaluated; *need is set when it would have been selected, and
// the entry then holds the (inaccurate) recursion value.
template <int P, class T, bool SERIES = true>
C0_HD void newton_entry(const double *y, const T *w, const T *u, const cx<T> *L, cx<T> A, cx<T> dA, cx<T> B,
                        cx<T> dB, cx<T> &V, cx<T> &Tg, bool *need = nullptr)
{
    const T span = T(y[P] - y[0]);
    const T inv = rcp(span);
    const cx<T> E = cxscale(cxsub(A, B), inv);
    const T dspan = (w[P] - w[0]) * inv;
    cx<T> dE = cxscale(cxsub(dA, dB), inv);
    dE = cxm<T>(fmaT(-E.re, dspan, dE.re), fmaT(-E.im, dspan, dE.im));
    const T d0 = absT(u[0]), dP = absT(u[P]);
    const bool first = d0 >= dP;
    const T far = first ? d0 : dP;
    const bool use_series = span <= T(P == 1 ? NearParams<T>::theta_pair : NearParams<T>::theta) * far;
    if (!SERIES) {
        *need = *need || use_series;
        V = E;
        Tg = dE;
        return;
    }
    const bool at_w = far == T(0);                 // every node at w: h[..] and its derivative vanish
    const T ue = at_w ? T(1) : (first ? u[0] : u[P]);
    const cx<T> Le = cxsel(first, L[0], L[P]);
    cx<T> Vt, Tt;
    if (P == 1) {
        taylor_pair<T>(T(first ? y[1] - y[0] : y[0] - y[1]), first ? w[0] : w[1], first ? w[1] : w[0], ue, Le, Vt,
                       Tt);
    } else {
        // expansion node y[0] or y[2]; the other two in order
        const double ye = first ? y[0] : y[P];
        taylor_triple<T>(T((first ? y[1] : y[0]) - ye), T((first ? y[P] : y[1]) - ye), first ? w[0] : w[P],
                         first ? w[1] : w[0], first ? w[P] : w[1], ue, Le, Vt, Tt);
    }
    if (at_w) { Vt = cxm<T>(T(0), T(0)); Tt = cxm<T>(T(0), T(0)); }
    V = cxsel(use_series, Vt, E);
    Tg = cxsel(use_series, Tt, dE);
}

// Near branch: sum_j W_j J_j at frequency om for sorted nodes y with weights w, as the
// W-derivative of the Newton table of h over the 4 nodes (leaves from 4 logarithms).
// h is taken with Log(u) - log(s), s the span of the nodes: the dropped part log(s) u^3 is a
// cubic, whose third divided difference is a constant, so the W-derivative is unchanged while
// the logarithms stay O(1) (no cancellation of a large common log(s) between the leaves).
// SERIES = false: no entry evaluates its series; *need reports whether any would have used it (the
// result is then to be discarded and the full evaluation done instead).  The series are needed
// only where nodes cluster relative to their distance from w, so most items skip them.
template <class T, bool SERIES = true>
C0_HD cplx near_eval_t(const double y[4], const double wd[4], double om, bool *need = nullptr)
{
    T u[4], w[4];
    cx<T> L[4], V0[4], T0[4];
    const T inv_s = rcp(T(y[3] - y[0]));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        u[i] = T(om - y[i]);
        w[i] = T(wd[i]);
        const bool zero = u[i] == T(0);             // h and h' vanish at u = 0
        L[i] = cxm<T>(zero ? T(0) : logT(absT(u[i]) * inv_s), u[i] < T(0) ? T(kPi) : T(0));
        V0[i] = hder_low<T>(0, u[i], L[i]);
        T0[i] = cxscale(hder_low<T>(1, u[i], L[i]), w[i]);
    }
    cx<T> V1[3], T1[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        newton_entry<1, T, SERIES || !CHI0_DEFER_PAIR_SERIES>(y + i, w + i, u + i, L + i, V0[i + 1], T0[i + 1], V0[i],
                                                               T0[i], V1[i], T1[i], need);
    cx<T> V2[2], T2[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
        newton_entry<2, T, SERIES>(y + i, w + i, u + i, L + i, V1[i + 1], T1[i + 1], V1[i], T1[i], V2[i], T2[i],
                                   need);
    // the top entry spans all nodes; in the near branch its span exceeds its distance to w
    const T inv = inv_s;
    const cx<T> E = cxscale(cxsub(V2[1], V2[0]), inv);
    const T dspan = (w[3] - w[0]) * inv;
    const cx<T> dE = cxscale(cxsub(T2[1], T2[0]), inv);
    // for w <= every node all leaves carry the same Im Log = pi (u <= 0), the imaginary part is
    // the divided difference of a cubic and its W-derivative vanishes: set it exactly (for
    // w >= every node it is exactly 0 already)
    const bool below = om <= y[0];
    return cmk((double)fmaT(-E.re, dspan, dE.re), below ? 0.0 : (double)fmaT(-E.im, dspan, dE.im));
}

C0_HD cplx near_eval(const double y[4], const double w[4], double om) { return near_eval_t<double>(y, w, om); }

// Mixed form: the near branch in FP32 (see near_eval_t); the kernels keep FP64 for
// near-degenerate tetrahedra (near_degenerate below).
C0_HD cplx near_eval32(const double y[4], const double w[4], double om) { return near_eval_t<float>(y, w, om); }

// The near branch without the entry series, for callers that evaluate the items whose entries
// cluster (need = true) again with near_eval / near_eval32.
C0_HD cplx near_eval_fast(const double y[4], const double w[4], double om, bool &need)
{
    need = false;
    return near_eval_t<double, false>(y, w, om, &need);
}
C0_HD cplx near_eval32_fast(const double y[4], const double w[4], double om, bool &need)
{
    need = false;
    return near_eval_t<float, false>(y, w, om, &need);
}

// ---------------------------------------------------------------------------
// Imaginary part alone (the tetrahedron delta weights, Sec. II, Eq. (2)):
// Im h(x) = pi (w - x)^3 for x > w and 0 for x <= w, i.e. -pi v^3 [v > 0] with v = x - w.  An
// entry of the Newton table whose nodes all lie on one side of w is the divided difference of 0 or
// of the plain cubic -pi v^3, known in closed form; only entries whose nodes straddle w use the
// recursion, whose span then separates nodes on both sides of w.  No logarithm, no series.
// Returns Im sum_j W_j J_j for sorted nodes y with weights w at frequency om.
// ---------------------------------------------------------------------------
struct RD {
    double v, t;   // value and W-derivative
};

template <int P>
C0_HD RD im_entry_poly(const double *v, const double *w)
{
    RD r;
    if (P == 0) { r.v = -kPi * v[0] * v[0] * v[0]; r.t = -3.0 * kPi * v[0] * v[0] * w[0]; }
    if (P == 1) {
        r.v = -kPi * (v[0] * v[0] + v[0] * v[1] + v[1] * v[1]);
        r.t = -kPi * ((2.0 * v[0] + v[1]) * w[0] + (v[0] + 2.0 * v[1]) * w[1]);
    }
    if (P == 2) { r.v = -kPi * (v[0] + v[1] + v[2]); r.t = -kPi * (w[0] + w[1] + w[2]); }
    if (P == 3) { r.v = -kPi; r.t = 0.0; }
    return r;
}

// entry over nodes i..i+P from its children B = [i..i+P-1], A = [i+1..i+P]; inv = 1/(y[P] - y[0])
// (read only when the nodes straddle w, so a span of zero never enters)
template <int P>
C0_HD RD im_entry(const double *v, const double *w, RD A, RD B, double inv)
{
    RD r;
    if (v[P] <= 0.0) {                 // every node at or below w: Im h vanishes on all of them
        r.v = 0.0;
        r.t = 0.0;
    } else if (v[0] >= 0.0) {          // every node at or above w: the plain cubic
        r = im_entry_poly<P>(v, w);
    } else {                           // nodes on both sides of w
        r.v = (A.v - B.v) * inv;
        r.t = fma(-r.v, (w[P] - w[0]) * inv, (A.t - B.t) * inv);
    }
    return r;
}

// Reciprocals of the node spans of sorted nodes y that the straddling entries divide by, which
// depend on the tetrahedron only: pairs (0,1), (1,2), (2,3), triples (0,2), (1,3), all (0,3).
C0_HD void im_span_rcp(const double y[4], double inv[6])
{
    inv[0] = rcp(y[1] - y[0]);
    inv[1] = rcp(y[2] - y[1]);
    inv[2] = rcp(y[3] - y[2]);
    inv[3] = rcp(y[2] - y[0]);
    inv[4] = rcp(y[3] - y[1]);
    inv[5] = rcp(y[3] - y[0]);
}

// Im sum_j W_j J_j for sorted nodes y with weights w at frequency om, given the span reciprocals
// of im_span_rcp (computed once per tetrahedron by callers that evaluate many frequencies).
C0_HD double near_im_spans(const double y[4], const double w[4], const double inv[6], double om)
{
    double v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = y[i] - om;
    RD L0[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const RD z = {0.0, 0.0};
        L0[i] = im_entry<0>(v + i, w + i, z, z, 0.0);
    }
    RD L1[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) L1[i] = im_entry<1>(v + i, w + i, L0[i + 1], L0[i], inv[i]);
    RD L2[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) L2[i] = im_entry<2>(v + i, w + i, L1[i + 1], L1[i], inv[3 + i]);
    return im_entry<3>(v, w, L2[1], L2[0], inv[5]).t;
}

C0_HD double near_im(const double y[4], const double w[4], double om)
{
    double inv[6];
    im_span_rcp(y, inv);
    return near_im_spans(y, w, inv, om);
}

// Mixed form: a final tetrahedron whose sorted corner values have two neighbours closer than
// max(tol, rel * span) (or that is flat) keeps the FP64 near branch; tol in the energy unit of the
// band arrays (default kDegenerateTol, 1e-6: eV for the supplied models).
constexpr double kDegenerateTol = 1e-6;
C0_HD bool near_degenerate(const double y[4], double tol, double rel = 0.0)
{
    const double t = fmax(tol, rel * (y[3] - y[0]));
    return !(y[1] - y[0] >= t && y[2] - y[1] >= t && y[3] - y[2] >= t);
}

// sum_j W_j J_j for one final tetrahedron (unsorted input) at one frequency.  With a single
// frequency the coefficient recurrence is not shared, so a far evaluation costs about as much per
// term as the recurrence; the far branch is taken at the smaller ratio kRhoOne with kTermsOne
// terms (kRhoOne^kTermsOne ~ 1e-16), where the near branch is cheaper than a longer series.
constexpr double kRhoOne = 0.4;
constexpr int kTermsOne = 40;

C0_HD cplx tetra_weight_sum(const double D[4], const double Wt[4], double om)
{
    double y[4] = {D[0], D[1], D[2], D[3]}, w[4] = {Wt[0], Wt[1], Wt[2], Wt[3]};
    sort4(y, w);
    const double c = 0.5 * (y[0] + y[3]), r = 0.5 * (y[3] - y[0]);
    const double d = om - c;
    if (r <= kRhoOne * fabs(d)) {
        double a[kTermsOne];
        far_coeffs<kTermsOne>(y, w, c, a);
        return cmk(far_horner<kTermsOne>(a, 1.0 / d), 0.0);
    }
    return near_eval(y, w, om);
}

}  // namespace chi0
