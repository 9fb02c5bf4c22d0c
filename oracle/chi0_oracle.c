/*
 * chi0_oracle.c -- plain, slow, CPU FP64 oracle for the bare susceptibility
 * chi0(q, omega) by the linear tetrahedron method with double occupation
 * carving (Heil et al., arXiv:1407.3444, Sec. II).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the GPU path.
 *
 * What is computed (Sec. II, Eqs. (1)-(3) and the carving condition, Eq. (4)):
 *
 *   chi0(q,w) = g_s/(6 Nk) sum_T sum_{n,m in window} [ I_R1(T) - I_R2(T) ]
 *   I_R(T)    = (1/|T|) int_{T cap R} W(k) / (w - D(k) + i0) dk
 *
 * with, on each mesh tetrahedron T, the band energies e = eps_n(k),
 * e' = eps_m(k+q), D = e' - e and the matrix-element weight
 * W = |sum_o conj(c_{o,n}(k)) c_{o,m}(k+q)|^2 (W = 1 under the constant
 * matrix-element approximation) all interpolated linearly from the corners
 * ("on equal footing", Sec. II).  R1 = {e < mu < e'} (occupied n at k, empty m
 * at k+q) and R2 = {e' < mu < e}; their difference is the occupation factor
 * f(e) - f(e') of the retarded Lindhard function.  Only the regions where the
 * product of Heaviside functions equals one are integrated: each tetrahedron
 * is cut once by the plane e = mu and each piece again by e' = mu (Sec. II,
 * the "second carving"), giving fully occupied final tetrahedra.
 *
 * On a final tetrahedron S with corner values D_1..D_4, W_1..W_4 and volume
 * fraction v_S, the integral is v_S sum_j W_j J_j with
 *
 *   J_j = 6 int_simplex lambda_j / (w - lambda.D + i0) dlambda
 *       = h[D_1, D_2, D_3, D_4, D_j],   h(x) = (w - x)^3 Log(w - x + i0),
 *
 * the 5-node divided difference with node j doubled (Hermite-Genocchi; the
 * paper only says that simpler formulas become usable on
 * the final tetrahedra and does not print them).  Re is the principal value,
 * Im = -pi delta.  Divided differences are evaluated by the Newton recursion on
 * sorted nodes, except that any entry whose nodes cluster tightly compared with
 * their distance from w is summed as a Taylor series about one of its nodes
 * (exact for tied nodes, free of the cancellation of the recursion).
 *
 * form = 1 evaluates the paper's own one-sided expression, Eq. (1)/(2): only
 * R1 is carved and each piece contributes 1/(w - D + i0) - 1/(w + D + i0).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* An entry whose node span is at most THETA times the distance of the
 * expansion node from w is summed as a Taylor series. */
#define THETA 0.5
#define TAYLOR_MAX_TERMS 400

/* Operation count of the last mesh evaluation (for the benchmark's op-count figure; it changes
 * no value).  Every floating-point operation of the carving and of the weight evaluation is
 * tallied in a per-thread counter with these weights: real add, subtract, multiply, divide 1;
 * complex add 2, complex multiply 6, complex divide 11; modulus 5; complex logarithm 87 (the
 * modulus plus two real transcendental functions, log and arg, at 41 each).  Units (mesh
 * tetrahedron, band pair) whose carved regions are not empty are counted beside it. */
enum { OP_CADD = 2, OP_CMUL = 6, OP_CDIV = 11, OP_CABS = 5, OP_CLOG = 87 };
static _Thread_local unsigned long long t_ops, t_units;
static unsigned long long g_ops, g_units;
#define OPS(n) (t_ops += (unsigned long long)(n))

/* ------------------------------------------------------------------------- */
/* The function h(x) = (w-x)^3 Log(w-x+i0) and its derivatives               */
/* ------------------------------------------------------------------------- */

/* The frequency is complex, z = w + i eta with eta >= 0 (Eq. (1): the retarded response is the
 * limit eta -> 0+ of the response at z).  u = z - x then lies in the closed upper half plane and
 * Log is the principal branch: on the real axis (eta = 0, stored as +0) it is log|u| for u > 0 and
 * log|u| + i pi for u < 0, the branch of w + i0. */
static cplx log_upper(cplx u) { return clog(u); }

/* u^k for a small integer k (negative k: 1/u^|k|), by repeated multiplication */
static cplx cpowi(cplx u, int k)
{
    OPS((k < 0 ? -k : k) * OP_CMUL + (k < 0 ? OP_CDIV : 0));
    cplx r = 1.0;
    for (int i = 0; i < (k < 0 ? -k : k); ++i) r *= u;
    return k < 0 ? 1.0 / r : r;
}

/* h^{(n)}(x) / n!  at a point with u = z - x (x-derivatives).
 *   h      =  u^3 L
 *   h'     = -(3 u^2 L + u^2)
 *   h''    =  6 u L + 5 u
 *   h'''   = -(6 L + 11)
 *   h^(n)  =  6 (n-4)! / u^(n-3)      (n >= 4)
 * At u = 0 the first three vanish and the rest diverge (NaN is returned). */
static cplx hder_fact(int n, cplx u)
{
    if (u == 0.0) {
        if (n <= 2) return 0.0;
        return NAN;
    }
    if (n >= 4) {
        double nn = (double)n;
        OPS(6 + 2 + OP_CDIV);
        return 6.0 / (nn * (nn - 1.0) * (nn - 2.0) * (nn - 3.0) * cpowi(u, n - 3));
    }
    cplx L = log_upper(u);
    OPS(OP_CLOG + (n == 0 ? 3 * OP_CMUL : n == 1 ? 3 * OP_CMUL + 2 + OP_CADD + 2 : n == 2 ? OP_CMUL + 6 + OP_CADD : 7));
    switch (n) {
    case 0: return u * u * u * L;
    case 1: return -(3.0 * u * u * L + u * u);
    case 2: return (6.0 * u * L + 5.0 * u) / 2.0;
    default: return -(6.0 * L + 11.0) / 6.0;
    }
}

/* Taylor sum  f[x_i..x_j] = sum_m h^{(p+m)}(c)/(p+m)! H_m(x_i - c, ..., x_j - c)
 * about the node c, H_m the complete homogeneous symmetric polynomial. */
static cplx dd_taylor(const double *x, int i, int j, double c, cplx z)
{
    int p = j - i;
    cplx u = z - c;
    cplx y[5];                         /* offsets from c, in units of u */
    double rho = 0.0;
    for (int v = 0; v <= p; ++v) {
        y[v] = (x[i + v] - c) / u;
        if (cabs(y[v]) > rho) rho = cabs(y[v]);
    }
    OPS(1 + (p + 1) * (1 + OP_CDIV + OP_CABS));
    if (rho == 0.0) return hder_fact(p, u);      /* all nodes equal: h^(p)(c)/p! */
    /* number of terms: the bound C(m+p,p) rho^m falls below 1e-18 (at least 4 terms) */
    int M = 0;
    for (double b = 1.0; M < TAYLOR_MAX_TERMS && (M < 4 || b > 1e-18); ++M)
        b *= (double)(M + p + 1) / (double)(M + 1) * rho;
    OPS(5 * M + (p + 1) * M * (OP_CMUL + OP_CADD));
    /* H[m] = H_m(y) of the scaled offsets, built up one variable at a time */
    cplx H[TAYLOR_MAX_TERMS + 1];
    H[0] = 1.0;
    for (int m = 1; m <= M; ++m) H[m] = 0.0;
    for (int v = 0; v <= p; ++v)
        for (int m = 1; m <= M; ++m) H[m] += y[v] * H[m - 1];
    /* h^{(n)}(c)/n! (x-c)^m-terms: for n = p+m >= 4 the coefficient is
     * 6/(n(n-1)(n-2)(n-3)) u^(3-n), and u^(3-n) u^m = u^(3-p). */
    cplx s = 0.0;
    cplx up = cpowi(u, 3 - p);
    for (int m = M; m >= 0; --m) {
        int n = p + m;
        if (n >= 4) {
            double nn = (double)n;
            OPS(7 + 2 + OP_CMUL + OP_CADD);
            s += 6.0 / (nn * (nn - 1.0) * (nn - 2.0) * (nn - 3.0)) * up * H[m];
        } else {
            OPS(2 * OP_CMUL + OP_CADD);
            s += hder_fact(n, u) * cpowi(u, m) * H[m];
        }
    }
    return s;
}

/* Divided difference h[x_i..x_j] over sorted nodes, memoised in tab/done. */
static cplx dd_entry(const double *x, int i, int j, cplx z, cplx tab[5][5], int done[5][5])
{
    if (done[i][j]) return tab[i][j];
    cplx v;
    if (i == j) {
        v = hder_fact(0, z - x[i]);
    } else {
        double span = x[j] - x[i];
        double di = cabs(z - x[i]), dj = cabs(z - x[j]);
        double far = di > dj ? di : dj;
        OPS(1 + 2 * (1 + OP_CABS) + 1);
        if (span <= THETA * far) {
            v = dd_taylor(x, i, j, di >= dj ? x[i] : x[j], z);
        } else {
            v = (dd_entry(x, i + 1, j, z, tab, done) - dd_entry(x, i, j - 1, z, tab, done)) / span;
            OPS(OP_CADD + 2);
        }
    }
    tab[i][j] = v;
    done[i][j] = 1;
    return v;
}

/* 5-node divided difference of h over arbitrary (unsorted) nodes. */
static cplx dd5(const double nodes[5], cplx z)
{
    double x[5];
    memcpy(x, nodes, sizeof x);
    for (int a = 1; a < 5; ++a) {          /* insertion sort */
        double t = x[a];
        int b = a - 1;
        while (b >= 0 && x[b] > t) { x[b + 1] = x[b]; --b; }
        x[b + 1] = t;
    }
    cplx tab[5][5];
    int done[5][5];
    memset(done, 0, sizeof done);
    return dd_entry(x, 0, 4, z, tab, done);
}

/* Corner weights J_j = h[D1,D2,D3,D4,D_j] of 1/(z - D) on a simplex (z = w + i0 on the real
 * axis). */
static void corner_weights(const double D[4], cplx z, cplx J[4])
{
    for (int j = 0; j < 4; ++j) {
        double nodes[5] = {D[0], D[1], D[2], D[3], D[j]};
        J[j] = dd5(nodes, z);
    }
}

/* ------------------------------------------------------------------------- */
/* Carving                                                                   */
/* ------------------------------------------------------------------------- */

/* A tetrahedron given by its four vertices in barycentric coordinates of the
 * mesh tetrahedron: b[v][i] is coordinate i of vertex v. */
typedef struct { double b[4][4]; } btet;

static double det4(const double m[4][4])
{
    OPS(4 + 3 * (1 + 2 * 4) + 2 * (1 + 2 * 3) + (1 + 2 * 2));   /* pivot products, eliminations */
    double a[4][4];
    memcpy(a, m, sizeof a);
    double det = 1.0;
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int r = c + 1; r < 4; ++r)
            if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        if (a[piv][c] == 0.0) return 0.0;
        if (piv != c) {
            for (int k = 0; k < 4; ++k) { double t = a[c][k]; a[c][k] = a[piv][k]; a[piv][k] = t; }
            det = -det;
        }
        det *= a[c][c];
        for (int r = c + 1; r < 4; ++r) {
            double f = a[r][c] / a[c][c];
            for (int k = c; k < 4; ++k) a[r][k] -= f * a[c][k];
        }
    }
    return det;
}

/* volume of t as a fraction of the mesh tetrahedron */
static double btet_volume(const btet *t) { return fabs(det4(t->b)); }

static void set_vertex(btet *t, int v, const double *p) { memcpy(t->b[v], p, 4 * sizeof(double)); }

/* point on the edge from vertex p (f<0) to vertex q (f>=0) where the linear f vanishes */
static void cut_point(const btet *t, int p, int q, const double *fv, double *out)
{
    OPS(2 + 4 * 3);
    double s = fv[p] / (fv[p] - fv[q]);
    for (int i = 0; i < 4; ++i) out[i] = t->b[p][i] + s * (t->b[q][i] - t->b[p][i]);
}

/* Keep the part of tetrahedron t where the linear function with mesh-corner
 * values f is strictly negative.  Writes 0, 1 or 3 tetrahedra. */
static int clip_negative(const btet *t, const double f[4], btet out[3])
{
    double fv[4];
    int in[4], ot[4], nin = 0, nout = 0;
    OPS(4 * 4 * 2);
    for (int v = 0; v < 4; ++v) {
        fv[v] = 0.0;
        for (int i = 0; i < 4; ++i) fv[v] += t->b[v][i] * f[i];
        if (fv[v] < 0.0) in[nin++] = v; else ot[nout++] = v;
    }
    if (nin == 0) return 0;
    if (nin == 4) { out[0] = *t; return 1; }
    if (nin == 1) {
        /* corner tetrahedron at the single inside vertex */
        double P[3][4];
        for (int k = 0; k < 3; ++k) cut_point(t, in[0], ot[k], fv, P[k]);
        set_vertex(&out[0], 0, t->b[in[0]]);
        for (int k = 0; k < 3; ++k) set_vertex(&out[0], k + 1, P[k]);
        return 1;
    }
    if (nin == 3) {
        /* the tetrahedron minus the corner at the outside vertex l: a prism
         * (i,j,k | Pi,Pj,Pk) split into three tetrahedra */
        int l = ot[0];
        double P[3][4];
        for (int k = 0; k < 3; ++k) cut_point(t, in[k], l, fv, P[k]);
        const double *A0 = t->b[in[0]], *A1 = t->b[in[1]], *A2 = t->b[in[2]];
        set_vertex(&out[0], 0, A0); set_vertex(&out[0], 1, A1); set_vertex(&out[0], 2, A2); set_vertex(&out[0], 3, P[0]);
        set_vertex(&out[1], 0, A1); set_vertex(&out[1], 1, A2); set_vertex(&out[1], 2, P[0]); set_vertex(&out[1], 3, P[1]);
        set_vertex(&out[2], 0, A2); set_vertex(&out[2], 1, P[0]); set_vertex(&out[2], 2, P[1]); set_vertex(&out[2], 3, P[2]);
        return 3;
    }
    /* nin == 2: prism with end triangles (i, Pik, Pil) and (j, Pjk, Pjl) */
    {
        int i = in[0], j = in[1], k = ot[0], l = ot[1];
        double Pik[4], Pil[4], Pjk[4], Pjl[4];
        cut_point(t, i, k, fv, Pik);
        cut_point(t, i, l, fv, Pil);
        cut_point(t, j, k, fv, Pjk);
        cut_point(t, j, l, fv, Pjl);
        set_vertex(&out[0], 0, t->b[i]); set_vertex(&out[0], 1, Pik); set_vertex(&out[0], 2, Pil); set_vertex(&out[0], 3, t->b[j]);
        set_vertex(&out[1], 0, Pik); set_vertex(&out[1], 1, Pil); set_vertex(&out[1], 2, t->b[j]); set_vertex(&out[1], 3, Pjk);
        set_vertex(&out[2], 0, Pil); set_vertex(&out[2], 1, t->b[j]); set_vertex(&out[2], 2, Pjk); set_vertex(&out[2], 3, Pjl);
        return 3;
    }
}

/* Carve the mesh tetrahedron into final tetrahedra of region 1 ({a<0, b>0})
 * or region 2 ({a>0, b<0}), a = e - mu, b = e' - mu at the corners.
 * Returns the count (at most 9); zero-volume pieces are kept. */
static int carve_region(const double a[4], const double b[4], int region, btet out[9])
{
    btet T, first[3];
    memset(&T, 0, sizeof T);
    for (int v = 0; v < 4; ++v) T.b[v][v] = 1.0;
    double fa[4], fb[4];
    for (int i = 0; i < 4; ++i) {
        fa[i] = region == 1 ? a[i] : -a[i];   /* first carving: Theta(mu - e) (region 1) */
        fb[i] = region == 1 ? -b[i] : b[i];   /* second carving: Theta(e' - mu) (region 1) */
    }
    int n1 = clip_negative(&T, fa, first), n = 0;
    for (int p = 0; p < n1; ++p) n += clip_negative(&first[p], fb, out + n);
    return n;
}

/* ------------------------------------------------------------------------- */
/* Mesh                                                                      */
/* ------------------------------------------------------------------------- */

/* Six tetrahedra per mesh cell along the (1,1,1) index diagonal: for each
 * permutation (p0,p1,p2) of the axes the corners are c, c+e_p0, c+e_p0+e_p1,
 * c+(1,1,1). */
static const int PERMS[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

static long long flat_index(const int n[3], long long i1, long long i2, long long i3)
{
    i1 = ((i1 % n[0]) + n[0]) % n[0];
    i2 = ((i2 % n[1]) + n[1]) % n[1];
    i3 = ((i3 % n[2]) + n[2]) % n[2];
    return (i1 * n[1] + i2) * n[2] + i3;
}

static void tet_corners(const int n[3], long long cell, int t, long long idx[4])
{
    long long i3 = cell % n[2], i2 = (cell / n[2]) % n[1], i1 = cell / ((long long)n[1] * n[2]);
    long long c[3] = {i1, i2, i3};
    idx[0] = flat_index(n, c[0], c[1], c[2]);
    c[PERMS[t][0]] += 1;
    idx[1] = flat_index(n, c[0], c[1], c[2]);
    c[PERMS[t][1]] += 1;
    idx[2] = flat_index(n, c[0], c[1], c[2]);
    c[PERMS[t][2]] += 1;
    idx[3] = flat_index(n, c[0], c[1], c[2]);
}

/* ------------------------------------------------------------------------- */
/* Driver                                                                    */
/* ------------------------------------------------------------------------- */

typedef struct {
    int n[3], nb, no, lo, nbw;
    long long nk;
    const double *eps_k, *c_k, *eps_kq, *c_kq;
    int shift[3];
    double mu;
    int cma, form;
    int single_carving; /* comparison only: first carving alone (see tet_contribution_at) */
    double eta;         /* imaginary part of the frequency (0: the retarded limit on the real axis) */
    double *W; /* [nbw][nbw][nk] */
} problem;

/* index of the k+q data for mesh point k */
static long long kq_index(const problem *P, long long k)
{
    if (P->eps_kq) return k;
    long long i3 = k % P->n[2], i2 = (k / P->n[2]) % P->n[1], i1 = k / ((long long)P->n[1] * P->n[2]);
    return flat_index(P->n, i1 + P->shift[0], i2 + P->shift[1], i3 + P->shift[2]);
}

/* W_nm(k) = |sum_o conj(c_{o,n}(k)) c_{o,m}(k+q)|^2  (footnote of Sec. III, with the
 * conjugate so that it is the modulus of an overlap) */
static void build_W(problem *P)
{
    long long nk = P->nk;
    int nbw = P->nbw;
    P->W = (double *)malloc(sizeof(double) * (size_t)nbw * nbw * nk);
    const double *ckq = P->c_kq ? P->c_kq : P->c_k;
#pragma omp parallel for schedule(static)
    for (long long k = 0; k < nk; ++k) {
        long long kq = kq_index(P, k);
        for (int n = 0; n < nbw; ++n)
            for (int m = 0; m < nbw; ++m) {
                double re = 0.0, im = 0.0;
                for (int o = 0; o < P->no; ++o) {
                    const double *a = P->c_k + 2 * (((size_t)k * P->no + o) * P->nb + (P->lo + n));
                    const double *b = ckq + 2 * (((size_t)kq * P->no + o) * P->nb + (P->lo + m));
                    /* conj(a) * b */
                    re += a[0] * b[0] + a[1] * b[1];
                    im += a[0] * b[1] - a[1] * b[0];
                }
                P->W[((size_t)n * nbw + m) * nk + k] = re * re + im * im;
            }
    }
}

/* Accumulate the contribution of one final tetrahedron (vertices in barycentric
 * coordinates) with sign s into acc[nw]. */
static void add_piece(const btet *S, const double Dc[4], const double Wc[4], double s,
                      int form, int nw, const double *omega, double eta, cplx *acc)
{
    double v = btet_volume(S);
    if (v == 0.0) return;
    OPS(4 * 4 * 4 + (unsigned long long)nw * (4 * (2 + OP_CADD) * (form == 1 ? 2 : 1) + 5));
    double D[4], Wv[4], Dm[4];
    for (int q = 0; q < 4; ++q) {
        D[q] = 0.0; Wv[q] = 0.0;
        for (int i = 0; i < 4; ++i) { D[q] += S->b[q][i] * Dc[i]; Wv[q] += S->b[q][i] * Wc[i]; }
        Dm[q] = -D[q];
    }
    for (int iw = 0; iw < nw; ++iw) {
        cplx J[4], sum = 0.0;
        const cplx z = omega[iw] + I * eta;
        corner_weights(D, z, J);
        for (int j = 0; j < 4; ++j) sum += Wv[j] * J[j];
        if (form == 1) {
            /* Eq. (1): 1/(w - D) + 1/(-w - D)  ==  1/(w - D) - 1/(w + D), both retarded (on the
             * real axis only: the complex-frequency entry point takes form 0) */
            corner_weights(Dm, z, J);
            for (int j = 0; j < 4; ++j) sum -= Wv[j] * J[j];
        }
        acc[iw] += s * v * sum;
    }
}

/* Contributions of one tetrahedron whose corners are the k-points idx[4] (k+q data at
 * idq[4]), all band pairs.  Pair (n, m) adds into acc + (n * nbw + m) * pair_stride
 * (pair_stride = 0: every pair into acc). */
static void tet_contribution_at(const problem *P, const long long idx[4], const long long idq[4], int nw,
                                const double *omega, cplx *acc, long long pair_stride)
{
    const double *ekq = P->eps_kq ? P->eps_kq : P->eps_k;
    for (int n = 0; n < P->nbw; ++n)
        for (int m = 0; m < P->nbw; ++m) {
            double a[4], b[4], Dc[4], Wc[4];
            for (int c = 0; c < 4; ++c) {
                double e = P->eps_k[(size_t)(P->lo + n) * P->nk + idx[c]];
                double ep = ekq[(size_t)(P->lo + m) * P->nk + idq[c]];
                a[c] = e - P->mu;
                b[c] = ep - P->mu;
                Dc[c] = ep - e;
                Wc[c] = P->cma ? 1.0 : P->W[((size_t)n * P->nbw + m) * P->nk + idx[c]];
            }
            cplx *pacc = acc + (size_t)(n * P->nbw + m) * pair_stride;
            btet S[9];
            if (P->single_carving) {
                /* The treatment the second carving replaces (Sec. II): only the occupied part
                 * e < mu is carved out; the final-state factor Theta(e' - mu) is taken at the
                 * corners of the tetrahedron and interpolated linearly with W.  Eq. (1) form. */
                double Wv[4], fa[4];
                for (int c = 0; c < 4; ++c) {
                    Wv[c] = b[c] > 0.0 ? Wc[c] : 0.0;
                    fa[c] = a[c];
                }
                btet T;
                memset(&T, 0, sizeof T);
                for (int v = 0; v < 4; ++v) T.b[v][v] = 1.0;
                int n1 = clip_negative(&T, fa, S);
                for (int s = 0; s < n1; ++s) add_piece(&S[s], Dc, Wv, +1.0, 1, nw, omega, P->eta, pacc);
                continue;
            }
            OPS(4 * 3);
            int ns = carve_region(a, b, 1, S), active = ns > 0;
            for (int s = 0; s < ns; ++s) add_piece(&S[s], Dc, Wc, +1.0, P->form, nw, omega, P->eta, pacc);
            if (P->form == 0) {
                ns = carve_region(a, b, 2, S);
                active = active || ns > 0;
                for (int s = 0; s < ns; ++s) add_piece(&S[s], Dc, Wc, -1.0, 0, nw, omega, P->eta, pacc);
            }
            t_units += (unsigned long long)active;
        }
}

/* Contributions of one mesh tetrahedron (cell, Kuhn tetrahedron t), all band pairs. */
static void tet_contribution(const problem *P, long long cell, int t, int nw, const double *omega, cplx *acc,
                             long long pair_stride)
{
    long long idx[4], idq[4];
    tet_corners(P->n, cell, t, idx);
    for (int c = 0; c < 4; ++c) idq[c] = kq_index(P, idx[c]);
    tet_contribution_at(P, idx, idq, nw, omega, acc, pair_stride);
}

static int setup(problem *P, int n1, int n2, int n3, int nb, int no,
                 const double *eps_k, const double *c_k, const double *eps_kq, const double *c_kq,
                 int s1, int s2, int s3, double mu, int band_lo, int band_hi, int cma, int form)
{
    memset(P, 0, sizeof *P);
    if (n1 <= 0 || n2 <= 0 || n3 <= 0 || nb <= 0) return -2;
    if (band_hi < 0) band_hi = nb;
    if (band_lo < 0 || band_lo >= band_hi || band_hi > nb) return -2;
    if (!eps_k || (!cma && !c_k) || (form != 0 && form != 1)) return -1;
    if ((eps_kq == NULL) != (c_kq == NULL) && !cma) return -1;
    P->n[0] = n1; P->n[1] = n2; P->n[2] = n3;
    P->nk = (long long)n1 * n2 * n3;
    P->nb = nb; P->no = no; P->lo = band_lo; P->nbw = band_hi - band_lo;
    P->eps_k = eps_k; P->c_k = c_k; P->eps_kq = eps_kq; P->c_kq = c_kq;
    P->shift[0] = s1; P->shift[1] = s2; P->shift[2] = s3;
    P->mu = mu; P->cma = cma; P->form = form;
    if (!cma) build_W(P);
    return 0;
}

/*
 * chi0 at one q for nw frequencies.  eps_k: [nb][Nk]; c_k: complex [Nk][no][nb]
 * (re, im interleaved), may be NULL under CMA.  If eps_kq is NULL the k+q data
 * is the mesh data shifted by the integer vector (s1,s2,s3); otherwise eps_kq
 * [nb][Nk] and c_kq [Nk][no][nb] hold it for every mesh point.  Only mesh cells
 * [cell_begin, cell_end) are summed (cell_end < 0: all), with the full-mesh
 * normalisation.  out: [nw][2] = (Re, Im).  Returns 0 on success.
 */
static int oracle_mesh(int n1, int n2, int n3, int nb, int no,
                       const double *eps_k, const double *c_k,
                       const double *eps_kq, const double *c_kq,
                       int s1, int s2, int s3,
                       double mu, double spin_factor, int band_lo, int band_hi,
                       int cma, int form, int nw, const double *omega, double eta,
                       long long cell_begin, long long cell_end, int nthreads, double *out)
{
    problem P;
    if (!(eta >= 0.0) || (eta > 0.0 && form != 0)) return -1;
    int rc = setup(&P, n1, n2, n3, nb, no, eps_k, c_k, eps_kq, c_kq, s1, s2, s3, mu,
                   band_lo, band_hi, cma, form);
    if (rc) return rc;
    P.eta = eta;
    long long ncell = P.nk;
    if (cell_end < 0 || cell_end > ncell) cell_end = ncell;
    if (cell_begin < 0) cell_begin = 0;
    int nt = 1;
#ifdef _OPENMP
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    cplx *acc = (cplx *)calloc((size_t)nt * nw, sizeof(cplx));
    g_ops = 0;
    g_units = 0;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        cplx *my = acc + (size_t)tid * nw;
        t_ops = 0;
        t_units = 0;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (long long cell = cell_begin; cell < cell_end; ++cell)
            for (int t = 0; t < 6; ++t) tet_contribution(&P, cell, t, nw, omega, my, 0);
#ifdef _OPENMP
#pragma omp critical
#endif
        {
            g_ops += t_ops;
            g_units += t_units;
        }
    }
    double pref = spin_factor / (6.0 * (double)P.nk);
    for (int iw = 0; iw < nw; ++iw) {
        cplx s = 0.0;
        for (int t = 0; t < nt; ++t) s += acc[(size_t)t * nw + iw];   /* fixed order */
        out[2 * iw] = pref * creal(s);
        out[2 * iw + 1] = pref * cimag(s);
    }
    free(acc);
    free(P.W);
    return 0;
}

int chi0_oracle(int n1, int n2, int n3, int nb, int no,
                const double *eps_k, const double *c_k,
                const double *eps_kq, const double *c_kq,
                int s1, int s2, int s3,
                double mu, double spin_factor, int band_lo, int band_hi,
                int cma, int form, int nw, const double *omega,
                long long cell_begin, long long cell_end, int nthreads, double *out)
{
    return oracle_mesh(n1, n2, n3, nb, no, eps_k, c_k, eps_kq, c_kq, s1, s2, s3, mu, spin_factor, band_lo,
                       band_hi, cma, form, nw, omega, 0.0, cell_begin, cell_end, nthreads, out);
}

/*
 * The same integral of the linear interpolant at the complex frequencies z = omega + i eta
 * (eta >= 0, difference form only): sum W (f - f') / (z - D) integrated exactly over the carved
 * final tetrahedra.  It is analytic in z in the upper half plane and tends to chi0_oracle's
 * retarded result as eta -> 0+ (Eq. (1)); at finite eta it can be compared with plain k sums of
 * the same Lorentzian-broadened expression, which converge without extrapolation in eta.
 */
int chi0_oracle_z(int n1, int n2, int n3, int nb, int no,
                  const double *eps_k, const double *c_k,
                  const double *eps_kq, const double *c_kq,
                  int s1, int s2, int s3,
                  double mu, double spin_factor, int band_lo, int band_hi,
                  int cma, int nw, const double *omega, double eta, int nthreads, double *out)
{
    return oracle_mesh(n1, n2, n3, nb, no, eps_k, c_k, eps_kq, c_kq, s1, s2, s3, mu, spin_factor, band_lo,
                       band_hi, cma, 0, nw, omega, eta, 0, -1, nthreads, out);
}

/*
 * chi0 at one q summed over an explicit list of tetrahedra instead of the mesh's Kuhn
 * tetrahedra: the irreducible wedge of Sec. II decomposed into tetrahedra, or any other set.
 * tets[n_tet][4] are corner indices into n_kp k-points; eps_k [nb][n_kp] and c_k
 * [n_kp][no][nb] hold the data at those points, eps_kq [nb][n_kp] and c_kq [n_kp][no][nb]
 * (c_kq may be NULL under CMA) the data at the same points shifted by q.  Every tetrahedron
 * is the fraction `volume` of the zone.  single_carving = 1 (with form 1 only) replaces the
 * second carving by the corner-interpolated final-state factor, the treatment the paper compares
 * its method with.  out: [nw][2] = (Re, Im).  Returns 0 on success.
 */
int chi0_oracle_list(int n_kp, int nb, int no,
                     const double *eps_k, const double *c_k,
                     const double *eps_kq, const double *c_kq,
                     long long n_tet, const int *tets, double volume,
                     double mu, double spin_factor, int band_lo, int band_hi,
                     int cma, int form, int single_carving, int nw, const double *omega, int nthreads,
                     double *out)
{
    if (!eps_kq || !tets || n_tet < 0 || !(volume > 0.0)) return -1;
    if (single_carving && form != 1) return -1;
    for (long long t = 0; t < 4 * n_tet; ++t)
        if (tets[t] < 0 || tets[t] >= n_kp) return -2;
    problem P;
    int rc = setup(&P, n_kp, 1, 1, nb, no, eps_k, c_k, eps_kq, cma ? NULL : c_kq, 0, 0, 0, mu,
                   band_lo, band_hi, cma, form);
    if (rc) return rc;
    P.single_carving = single_carving;
    int nt = 1;
#ifdef _OPENMP
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    cplx *acc = (cplx *)calloc((size_t)nt * nw, sizeof(cplx));
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        cplx *my = acc + (size_t)tid * nw;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (long long t = 0; t < n_tet; ++t) {
            long long idx[4];
            for (int c = 0; c < 4; ++c) idx[c] = tets[4 * t + c];
            tet_contribution_at(&P, idx, idx, nw, omega, my, 0);
        }
    }
    double pref = spin_factor * volume;
    for (int iw = 0; iw < nw; ++iw) {
        cplx s = 0.0;
        for (int t = 0; t < nt; ++t) s += acc[(size_t)t * nw + iw];   /* fixed order */
        out[2 * iw] = pref * creal(s);
        out[2 * iw + 1] = pref * cimag(s);
    }
    free(acc);
    free(P.W);
    return 0;
}

/*
 * The same sum resolved by band pair (the band-transition histogram of Sec. III): out
 * [nbw][nbw][nw][2] receives, for n, m relative to band_lo, the terms of pair (n, m) alone, so
 * that the sum over all pairs is chi0_oracle's result.  Other arguments as for chi0_oracle.
 */
int chi0_oracle_pairs(int n1, int n2, int n3, int nb, int no,
                      const double *eps_k, const double *c_k,
                      const double *eps_kq, const double *c_kq,
                      int s1, int s2, int s3,
                      double mu, double spin_factor, int band_lo, int band_hi,
                      int cma, int form, int nw, const double *omega, int nthreads, double *out)
{
    problem P;
    int rc = setup(&P, n1, n2, n3, nb, no, eps_k, c_k, eps_kq, c_kq, s1, s2, s3, mu,
                   band_lo, band_hi, cma, form);
    if (rc) return rc;
    const long long npair = (long long)P.nbw * P.nbw, per = npair * nw;
    int nt = 1;
#ifdef _OPENMP
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    cplx *acc = (cplx *)calloc((size_t)nt * per, sizeof(cplx));
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        cplx *my = acc + (size_t)tid * per;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (long long cell = 0; cell < P.nk; ++cell)
            for (int t = 0; t < 6; ++t) tet_contribution(&P, cell, t, nw, omega, my, nw);
    }
    double pref = spin_factor / (6.0 * (double)P.nk);
    for (long long i = 0; i < per; ++i) {
        cplx s = 0.0;
        for (int t = 0; t < nt; ++t) s += acc[(size_t)t * per + i];   /* fixed order */
        out[2 * i] = pref * creal(s);
        out[2 * i + 1] = pref * cimag(s);
    }
    free(acc);
    free(P.W);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Exact polynomial moments of the same carved integrand                     */
/* ------------------------------------------------------------------------- */

static double factd(int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; }

/* (1/|S|) int_S lambda_j (lambda.D)^p  =  6 sum_{|alpha|=p} p!/alpha! D^alpha (alpha+e_j)!/(p+4)!
 * (Dirichlet integral over the simplex). */
static double simplex_moment(const double D[4], int j, int p)
{
    double s = 0.0;
    for (int a0 = 0; a0 <= p; ++a0)
        for (int a1 = 0; a0 + a1 <= p; ++a1)
            for (int a2 = 0; a0 + a1 + a2 <= p; ++a2) {
                int al[4] = {a0, a1, a2, p - a0 - a1 - a2};
                double mono = 1.0, inv = 1.0, num = 1.0;
                for (int i = 0; i < 4; ++i) {
                    mono *= pow(D[i], al[i]);
                    inv *= factd(al[i]);
                    num *= factd(al[i] + (i == j));
                }
                s += factd(p) / inv * mono * num;
            }
    return 6.0 * s / factd(p + 4);
}

/*
 * mom[p] = g_s/(6Nk) sum [ int_R1 W D^p - int_R2 W D^p ] / |T|  for p = 0..pmax, over the
 * same carved regions (difference form).  Then chi0(q,w) = sum_p mom[p] / w^(p+1) for
 * |w| above the spectrum of D.
 */
int chi0_oracle_moments(int n1, int n2, int n3, int nb, int no,
                        const double *eps_k, const double *c_k,
                        const double *eps_kq, const double *c_kq,
                        int s1, int s2, int s3, double mu, double spin_factor,
                        int band_lo, int band_hi, int cma, int pmax, double *mom)
{
    problem P;
    int rc = setup(&P, n1, n2, n3, nb, no, eps_k, c_k, eps_kq, c_kq, s1, s2, s3, mu,
                   band_lo, band_hi, cma, 0);
    if (rc) return rc;
    for (int p = 0; p <= pmax; ++p) mom[p] = 0.0;
    const double *ekq = P.eps_kq ? P.eps_kq : P.eps_k;
    for (long long cell = 0; cell < P.nk; ++cell)
        for (int t = 0; t < 6; ++t) {
            long long idx[4], idq[4];
            tet_corners(P.n, cell, t, idx);
            for (int c = 0; c < 4; ++c) idq[c] = kq_index(&P, idx[c]);
            for (int n = 0; n < P.nbw; ++n)
                for (int m = 0; m < P.nbw; ++m) {
                    double a[4], b[4], Dc[4], Wc[4];
                    for (int c = 0; c < 4; ++c) {
                        double e = P.eps_k[(size_t)(P.lo + n) * P.nk + idx[c]];
                        double ep = ekq[(size_t)(P.lo + m) * P.nk + idq[c]];
                        a[c] = e - mu; b[c] = ep - mu; Dc[c] = ep - e;
                        Wc[c] = P.cma ? 1.0 : P.W[((size_t)n * P.nbw + m) * P.nk + idx[c]];
                    }
                    for (int region = 1; region <= 2; ++region) {
                        btet S[9];
                        int ns = carve_region(a, b, region, S);
                        for (int s = 0; s < ns; ++s) {
                            double v = btet_volume(&S[s]);
                            double D[4], Wv[4];
                            for (int q = 0; q < 4; ++q) {
                                D[q] = 0.0; Wv[q] = 0.0;
                                for (int i = 0; i < 4; ++i) { D[q] += S[s].b[q][i] * Dc[i]; Wv[q] += S[s].b[q][i] * Wc[i]; }
                            }
                            for (int p = 0; p <= pmax; ++p) {
                                double acc = 0.0;
                                for (int j = 0; j < 4; ++j) acc += Wv[j] * simplex_moment(D, j, p);
                                mom[p] += (region == 1 ? 1.0 : -1.0) * v * acc;
                            }
                        }
                    }
                }
        }
    double pref = spin_factor / (6.0 * (double)P.nk);
    for (int p = 0; p <= pmax; ++p) mom[p] *= pref;
    free(P.W);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Pieces exported for the oracle's own tests                                */
/* ------------------------------------------------------------------------- */

/* J[j] (re, im interleaved) for one simplex with corner values D at frequency w */
void chi0_oracle_weights(const double *D, double w, double *J)
{
    cplx Jc[4];
    corner_weights(D, w + 0.0 * I, Jc);
    for (int j = 0; j < 4; ++j) { J[2 * j] = creal(Jc[j]); J[2 * j + 1] = cimag(Jc[j]); }
}

/* 5-node divided difference of h(x) = (w-x)^3 Log(w-x+i0) */
void chi0_oracle_dd5(const double *nodes, double w, double *out)
{
    cplx v = dd5(nodes, w + 0.0 * I);
    out[0] = creal(v);
    out[1] = cimag(v);
}

/* Final tetrahedra of region 1 or 2 for corner values a = e - mu, b = e' - mu:
 * verts[s][v][i] barycentric coordinates, vols[s] volume fractions. Returns count. */
int chi0_oracle_carve(const double *a, const double *b, int region, double *verts, double *vols)
{
    btet S[9];
    int ns = carve_region(a, b, region, S);
    for (int s = 0; s < ns; ++s) {
        memcpy(verts + 16 * s, S[s].b, 16 * sizeof(double));
        vols[s] = btet_volume(&S[s]);
    }
    return ns;
}

/* Corner mesh indices of tetrahedron t of a cell (for the oracle's tests) */
void chi0_oracle_tet_corners(int n1, int n2, int n3, long long cell, int t, long long *idx)
{
    int n[3] = {n1, n2, n3};
    tet_corners(n, cell, t, idx);
}

/* The matrix-element weights the integration interpolates (footnote of Sec. III, with n at k
 * and m at k+q): W[(n*nbw + m)*Nk + k] = |sum_o conj(c_{o,n}(k)) c_{o,m}(k+q)|^2 for n, m
 * relative to band_lo.  Arguments as for chi0_oracle (not under CMA).  Returns 0 on success. */
int chi0_oracle_W(int n1, int n2, int n3, int nb, int no,
                  const double *eps_k, const double *c_k,
                  const double *eps_kq, const double *c_kq,
                  int s1, int s2, int s3, int band_lo, int band_hi, double *W)
{
    problem P;
    int rc = setup(&P, n1, n2, n3, nb, no, eps_k, c_k, eps_kq, c_kq, s1, s2, s3, 0.0,
                   band_lo, band_hi, 0, 0);
    if (rc) return rc;
    memcpy(W, P.W, sizeof(double) * (size_t)P.nbw * P.nbw * P.nk);
    free(P.W);
    return 0;
}

/* The operation and active-unit counts of the last mesh evaluation (chi0_oracle or
 * chi0_oracle_z). */
void chi0_oracle_last_count(unsigned long long *ops, unsigned long long *units)
{
    *ops = g_ops;
    *units = g_units;
}
