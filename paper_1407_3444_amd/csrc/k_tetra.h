// k_tetra.h -- device code of the tetrahedron kernel of the chi0 path (K_B), shared by the
// translation units that instantiate its kernels (k_tetra_*.hip).
//
// One work unit is one (mesh tetrahedron, band pair) of one q.  A workgroup is
// one 64-lane wave; rounds of 64 consecutive units are dealt to the workgroups
// round-robin, so every workgroup sees the same mix of band pairs (the work of
// a pair depends strongly on where its bands lie relative to mu).  Each round,
// every lane takes one unit, loads the 4 corner values of e = eps_n(k),
// e' = eps_m(k+q) and W_nm(k) (coalesced: consecutive lanes hold consecutive
// cells), carves it into final tetrahedra -- first by e = mu, then by
// e' = mu (Sec. II) -- and appends them to a list in LDS at an offset from a
// wave prefix sum (so the order, and with it every FP64 sum, is fixed).
//
//  * dynamic: every final tetrahedron is then evaluated by all 64 lanes, each
//    lane owning up to 8 frequencies (lane + 64 s).  Far-cluster tetrahedra
//    cost one Horner evaluation per frequency from coefficients computed once
//    (spread over the lanes) and stored with the tetrahedron in LDS; only
//    frequencies inside a tetrahedron's near window pay for logarithms.
//    Lanes accumulate their own frequencies, so no cross-lane reduction.
//  * static (w = 0): lanes split the list instead, and the wave reduces its
//    lane sums with a fixed butterfly at the end.
//
// Each workgroup writes its partial sums; the reduce kernel (K_R) adds them in
// block order.
#pragma once

#include "chi0_internal.h"
#include "chi0_math.h"

namespace chi0 {

namespace {

constexpr int kCapDyn = 32;     // final tetrahedra per LDS list (dynamic)
constexpr int kCapStat = 192;   // final tetrahedra per LDS list (static)
// Near-branch work items queued per lane.  36 rows keep the FP64 form's list and queue within
// 20 KiB, so that eight one-wave workgroups (two per SIMD, the register limit) fit in the 160 KiB
// of LDS of a CU.
constexpr int kQCap = 36;
// One unit yields at most 18 final tetrahedra (each region: at most 3 pieces from the first
// carving, each cut into at most 3 by the second; form 1 stores every piece twice), and a list
// must hold a whole unit, or filling it would never advance.
constexpr int kMaxRecsPerUnit = 18;
static_assert(kCapDyn >= kMaxRecsPerUnit && kCapStat >= kMaxRecsPerUnit, "a list must hold a whole unit");

// A final tetrahedron of a dynamic list.  The series storage is sized for the form, so the mixed
// form's shorter FP32 series keeps its lists small in LDS.
template <bool MIXED>
struct DynRec {
    double y[4];                // D at the corners (sorted ascending after the prep pass)
    double w[4];                // sign * volume * W at the same corners
    double c, hs;               // centre and half-span of the D values (prep pass)
    int32_t cls;                // far-series class against the frequency interval (prep pass)
    int32_t flags;              // prep pass: 1 = no frequency of the interval is near,
                                // 2 = near-degenerate (kept FP64 in the mixed form)
    union {
        alignas(16) double a[MIXED ? kFarTerms32 / 2 : kFarTerms];      // series coefficients (FP64 form)
        alignas(16) float a32[MIXED ? kFarTerms32 : 2 * kFarTerms];     // the FP32 series (mixed form)
    };
};

static_assert(kCapDyn * sizeof(DynRec<false>) + kQCap * kWave * sizeof(uint16_t) <= 160 * 1024 / 8,
              "eight FP64 dynamic workgroups fit the LDS of a CU");
static_assert(kQCap * kWave * sizeof(uint16_t) >= kFarTerms * sizeof(double),
              "a list's summed series fits the near queue's memory");
static_assert(kFarTerms32 % 4 == 0 && kFarTerms32 <= 2 * kFarTerms, "FP32 series read four at a time, inside the union");

struct StatRec {
    double D[4];
    double w[4];
};
static_assert(kCapStat * sizeof(StatRec) <= 160 * 1024 / 12, "twelve static workgroups fit the LDS of a CU");

constexpr int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

__device__ __forceinline__ int wrap_inc(int i, int n) { return i + 1 == n ? 0 : i + 1; }

// Corner values of unit u (pair-major, then tetrahedron permutation, then cell).
// A unit = (band pair, tetrahedron of a cell, cell): unit index u = (pair * nperm + perm) * ncell + cell;
// a tetrahedron list is one "permutation" whose cells are the listed tetrahedra.
struct UnitIdx {
    int pair, perm, cell;
};

// Tetrahedra of a cell: the 6 Kuhn tetrahedra of a mesh cell, or one listed tetrahedron
// (LIST: the kernels are compiled for mesh plans and list plans separately, so the mesh path
// carries nothing of the list path).
template <bool LIST>
__device__ __forceinline__ int64_t n_cells(const MeshDev &M) { return LIST ? M.ncell : M.nk; }
template <bool LIST>
constexpr int n_perm() { return LIST ? 1 : 6; }

// General decomposition of a unit index (64-bit divisions).
template <bool LIST>
__device__ __forceinline__ UnitIdx decode_unit(const MeshDev &M, int64_t u)
{
    UnitIdx x;
    const int64_t nc = n_cells<LIST>(M);
    const int64_t q = u / nc;
    x.cell = (int)(u - q * nc);
    x.pair = (int)(q / n_perm<LIST>());
    x.perm = (int)(q - (int64_t)x.pair * n_perm<LIST>());
    return x;
}

// Unit base + lane of a round of 64 consecutive units: the round's base is decomposed once
// (wave-uniform, scalar arithmetic) and every lane carries its offset into the cell index.
template <bool LIST>
__device__ __forceinline__ UnitIdx round_unit(const MeshDev &M, const UnitIdx &b, int lane)
{
    UnitIdx x = b;
    x.cell += lane;
    const int nc = (int)n_cells<LIST>(M);
    while (x.cell >= nc) {        // at most once unless there are fewer than 64 cells
        x.cell -= nc;
        if (++x.perm == n_perm<LIST>()) {
            x.perm = 0;
            ++x.pair;
        }
    }
    return x;
}

template <bool LIST>
__device__ __forceinline__ void load_unit(const MeshDev &M, const QDev &Q, const UnitIdx &x, Vtx t[4])
{
    const int64_t nk = M.nk;
    const int pair = x.pair, perm = x.perm;
    const int n = pair / M.nbw, m = pair - n * M.nbw;
    const double *ek = M.eps_k + (int64_t)(M.lo + n) * nk;
    const double *ekq = Q.eps_kq + (int64_t)(M.lo + m) * nk;
    const double *Wp = M.cma ? nullptr : Q.W + (int64_t)pair * nk;
    auto put = [&](int c, int64_t idx, int64_t idq) {
        const double e = ek[idx], ep = ekq[idq];
        t[c].a = e - M.mu;
        t[c].b = ep - M.mu;
        t[c].D = ep - e;
        t[c].W = M.cma ? 1.0 : Wp[idx];
    };
    if (LIST) {
        // explicit tetrahedron (list plans): corner k-points from the list, k+q data at the same points
        const int4 c4 = reinterpret_cast<const int4 *>(M.tets)[x.cell];
        put(0, c4.x, c4.x);
        put(1, c4.y, c4.y);
        put(2, c4.z, c4.z);
        put(3, c4.w, c4.w);
        return;
    }
    int i[3];
    const unsigned c12 = (unsigned)x.cell / (unsigned)M.n3;
    i[2] = x.cell - (int)(c12 * (unsigned)M.n3);
    i[0] = (int)(c12 / (unsigned)M.n2);
    i[1] = (int)c12 - i[0] * M.n2;
    const int nn[3] = {M.n1, M.n2, M.n3};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (c > 0) {
            const int ax = kPerm[perm][c - 1];
            i[ax] = wrap_inc(i[ax], nn[ax]);
        }
        const int64_t idx = ((int64_t)i[0] * M.n2 + i[1]) * M.n3 + i[2];
        int64_t idq = idx;
        if (!Q.explicit_kq) {
            int j0 = i[0] + Q.shift[0], j1 = i[1] + Q.shift[1], j2 = i[2] + Q.shift[2];
            j0 -= j0 >= M.n1 ? M.n1 : 0;
            j1 -= j1 >= M.n2 ? M.n2 : 0;
            j2 -= j2 >= M.n3 ? M.n3 : 0;
            idq = ((int64_t)j0 * M.n2 + j1) * M.n3 + j2;
        }
        put(c, idx, idq);
    }
}

struct CountSink {
    int n;
    int mult;
    __device__ void operator()(const Vtx &, const Vtx &, const Vtx &, const Vtx &, double vol)
    {
        n += (vol != 0.0) ? mult : 0;
    }
};

// Appends final tetrahedra as (D, sign*vol*W); with form 1 also (-D, -sign*vol*W).
template <class Rec>
struct WriteSink {
    Rec *list;
    int pos;
    int limit;     // one past the last slot counted for this unit: never written beyond
    double sign;
    int form;
    __device__ void put(const Vtx &v0, const Vtx &v1, const Vtx &v2, const Vtx &v3, double s, bool neg)
    {
        if (pos >= limit) return;
        Rec &r = list[pos++];
        const double g = neg ? -1.0 : 1.0;
        r.y[0] = g * v0.D; r.y[1] = g * v1.D; r.y[2] = g * v2.D; r.y[3] = g * v3.D;
        r.w[0] = s * v0.W; r.w[1] = s * v1.W; r.w[2] = s * v2.W; r.w[3] = s * v3.W;
    }
    __device__ void operator()(const Vtx &v0, const Vtx &v1, const Vtx &v2, const Vtx &v3, double vol)
    {
        if (vol == 0.0) return;
        put(v0, v1, v2, v3, sign * vol, false);
        if (form == 1) put(v0, v1, v2, v3, -sign * vol, true);
    }
};

template <>
__device__ void WriteSink<StatRec>::put(const Vtx &v0, const Vtx &v1, const Vtx &v2, const Vtx &v3,
                                        double s, bool neg)
{
    if (pos >= limit) return;
    StatRec &r = list[pos++];
    const double g = neg ? -1.0 : 1.0;
    r.D[0] = g * v0.D; r.D[1] = g * v1.D; r.D[2] = g * v2.D; r.D[3] = g * v3.D;
    r.w[0] = s * v0.W; r.w[1] = s * v1.W; r.w[2] = s * v2.W; r.w[3] = s * v3.W;
}

__device__ __forceinline__ int count_unit(const Vtx t[4], int form)
{
    CountSink cs;
    cs.n = 0;
    cs.mult = form == 1 ? 2 : 1;
    if (!region_empty(t[0], t[1], t[2], t[3], 1)) carve_region(t[0], t[1], t[2], t[3], 1, cs);
    if (form == 0) {
        cs.mult = 1;
        if (!region_empty(t[0], t[1], t[2], t[3], 2)) carve_region(t[0], t[1], t[2], t[3], 2, cs);
    }
    return cs.n;
}

template <class Rec>
__device__ __forceinline__ void write_unit(const Vtx t[4], int form, Rec *list, int pos, int limit)
{
    WriteSink<Rec> ws;
    ws.list = list;
    ws.pos = pos;
    ws.limit = limit;
    ws.form = form;
    ws.sign = 1.0;
    if (!region_empty(t[0], t[1], t[2], t[3], 1)) carve_region(t[0], t[1], t[2], t[3], 1, ws);
    if (form == 0) {
        ws.sign = -1.0;
        if (!region_empty(t[0], t[1], t[2], t[3], 2)) carve_region(t[0], t[1], t[2], t[3], 2, ws);
    }
}

__device__ __forceinline__ int wave_inclusive_scan(int x, int lane)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

// Fill the LDS list with the final tetrahedra of lanes [start, next) of this round.
// Returns the number of records; next_out receives the first lane left for a later pass.
// The unit's corner values are loaded again here (cache hits) rather than kept in
// registers across the evaluation of the list.
template <class Rec, int CAP, bool LIST>
__device__ __forceinline__ int fill_list(const MeshDev &M, const QDev &Q, const UnitIdx &ux, bool valid, int cnt,
                                         int start, int lane, Rec *list, int &next_out)
{
    const int c = (lane >= start) ? cnt : 0;
    const int incl = wave_inclusive_scan(c, lane);
    const int excl = incl - c;
    const bool fits = lane >= start && incl <= CAP;
    const unsigned long long mask = __ballot(fits);
    const int next = start + __popcll(mask);
    const int nrec = __shfl(incl, next - 1, kWave);
    if (fits && valid && cnt > 0) {
        Vtx t[4];
        load_unit<LIST>(M, Q, ux, t);
        write_unit<Rec>(t, M.form, list, excl, incl);
    }
    next_out = next;
    return nrec;
}

__device__ __forceinline__ double wave_min(double x)
{
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) x = fmin(x, __shfl_xor(x, d, kWave));
    return x;
}

__device__ __forceinline__ double wave_max(double x)
{
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) x = fmax(x, __shfl_xor(x, d, kWave));
    return x;
}

// Band pairs with a carved region somewhere on the mesh, one bit per pair index p = n nbw + m < 256:
// region 1 = {e < mu < e'} needs some e_n < mu and some e'_m > mu, region 2 the reverse, and the
// band ranges run over every k-point of the arrays.  Without ranges, or with more than 256 pairs,
// every pair is marked.  Built once per workgroup (one ballot per 64 pairs).
struct PairMask {
    uint64_t bits[4];
    __device__ __forceinline__ bool active(int p) const
    {
        const int w = p >> 6;
        const uint64_t b = w == 0 ? bits[0] : w == 1 ? bits[1] : w == 2 ? bits[2] : bits[3];
        return ((b >> (p & 63)) & 1) != 0;
    }
};

__device__ __forceinline__ PairMask pair_mask(const MeshDev &M, const QDev &Q, int lane)
{
    PairMask pm;
    const int npairs = M.nbw * M.nbw;
    const bool use = Q.rng_k != nullptr && npairs <= 4 * kWave;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int p = lane + kWave * j;
        bool a = true;
        if (use && p < npairs) {
            const int n = p / M.nbw, m = p - n * M.nbw;
            a = (Q.rng_k[2 * n] < M.mu && Q.rng_kq[2 * m + 1] > M.mu) ||
                (Q.rng_k[2 * n + 1] > M.mu && Q.rng_kq[2 * m] < M.mu);
        }
        pm.bits[j] = __ballot(a);
    }
    return pm;
}

// True when the round of 64 units starting at b0 touches only pairs with no carved region: its
// own pair and, when it runs past that pair's last unit, the next one (a pair holds at least 64
// units, else nothing is skipped).  Such units count no final tetrahedron, so skipping the round,
// its loads included, leaves every result unchanged.  Wave-uniform.
template <bool LIST>
__device__ __forceinline__ bool round_inert(const MeshDev &M, const PairMask &pm, const UnitIdx &b0)
{
    if (b0.pair >= 4 * kWave || pm.active(b0.pair)) return false;
    const int64_t per_pair = tets_per_pair(M);
    const int64_t off = (int64_t)b0.perm * n_cells<LIST>(M) + b0.cell;     // unit offset in the pair
    if (off + kWave <= per_pair) return true;
    if (per_pair < kWave || b0.pair + 1 >= 4 * kWave) return false;
    return !pm.active(b0.pair + 1);
}

__device__ __forceinline__ int wave_sum(int x)
{
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}


// 1/d in FP32: hardware estimate + one Newton step
__device__ __forceinline__ float recip32(float d)
{
    const float t = __builtin_amdgcn_rcpf(d);
    return fmaf(t, fmaf(-d, t, 1.0f), t);
}

// NSLOT independent Horner chains sum_{m < n} a[m] t_s^m over the first n = cls K / kFarClasses
// coefficients (cls wave-uniform: one scalar branch per block of terms).
template <int K, int NSLOT, class T>
__device__ __forceinline__ void horner_slots(const T *a, const T *tt, int cls, T *f)
{
    constexpr int S = K / kFarClasses;
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) f[s] = T(0);
#pragma unroll
    for (int j = kFarClasses; j >= 1; --j) {
        if (j <= cls) {
#pragma unroll
            for (int m = j * S - 1; m >= (j - 1) * S; --m) {
#pragma unroll
                for (int s = 0; s < NSLOT; ++s) f[s] = fmaT(f[s], tt[s], a[m]);
            }
        }
    }
}

// The same FP64 sums with the coefficients read from LDS (broadcast reads) one block of terms at
// a time, the next block fetched while the current one is summed, so that only two blocks are
// held in registers rather than the whole series.  The block loop runs cls times (wave-uniform).
template <int K, int NSLOT>
__device__ __forceinline__ void horner_slots_lds(const double *a, const double *tt, int cls, double *f)
{
    constexpr int S = K / kFarClasses;
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) f[s] = 0.0;
    if (cls <= 0) return;
    double b[S];
#pragma unroll
    for (int m = 0; m < S; ++m) b[m] = a[(cls - 1) * S + m];
    for (int j = cls; j >= 1; --j) {
        double nb[S];
        const int nj = j > 1 ? j - 2 : 0;     // next block (clamped: always inside the series)
#pragma unroll
        for (int m = 0; m < S; ++m) nb[m] = a[nj * S + m];
#pragma unroll
        for (int m = S - 1; m >= 0; --m) {
#pragma unroll
            for (int s = 0; s < NSLOT; ++s) f[s] = fma(f[s], tt[s], b[m]);
        }
#pragma unroll
        for (int m = 0; m < S; ++m) b[m] = nb[m];
    }
}

// Evaluate this lane's queued near-branch items (tetrahedron r, slot s), newest first.  Each
// lane's queue has two ends: items of the FP64 evaluation at the bottom (rows 0, 1, ...), and,
// in the mixed form, items of the FP32 evaluation at the top (rows kQCap-1, kQCap-2, ...).
// Lanes with an empty end idle; the loop ends when that end is empty in every lane.
// Evaluates the lane's queued near items (tetrahedron r, slot s) and empties the queue.  With
// TWO_PASS (the FP64 form) a first pass skips the Taylor series of the Newton entries, which few
// items need (the entry's nodes must cluster within theta of their distance from w) but which
// would otherwise cost every wave that holds one such item; those items are set aside in queue
// positions already consumed and evaluated in full by a second pass.  The FP32 near branch is
// cheap enough that the second pass does not pay; it takes one pass.  With a counter (census),
// the items evaluated by the second pass are counted.
template <int NSLOT, bool F32, bool TWO_PASS = false, class Rec>
__device__ __forceinline__ void drain_near(const Rec *list, uint16_t (*queue)[kWave], int &qn, int lane,
                                           const double *__restrict__ omega, cplx *acc,
                                           unsigned long long *redo_count = nullptr)
{
    const int top = qn;
    int nredo = 0;
    auto slot = [&](int p) -> uint16_t & { return queue[F32 ? kQCap - 1 - p : p][lane]; };
    // the item's result goes to the accumulator of its slot s (a lane-dependent index, so every
    // slot takes an FMA with a factor 1 or 0: exactly acc + z or acc for a finite result)
    auto add = [&](int s, cplx z) {
#pragma unroll
        for (int ss = 0; ss < NSLOT; ++ss) {
            const double m = s == ss ? 1.0 : 0.0;
            acc[ss].re = fma(m, z.re, acc[ss].re);
            acc[ss].im = fma(m, z.im, acc[ss].im);
        }
    };
    while (__any(qn > 0)) {
        if (qn > 0) {
            --qn;
            const int e = slot(qn);
            const int r = e >> 3, s = e & 7;
            double y[4], w[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) { y[k] = list[r].y[k]; w[k] = list[r].w[k]; }
            // the frequency is read again (a cached load) rather than picked out of the
            // lane's register array, which would be indexed dynamically
            const double o = omega[lane + kWave * s];
            bool need = false;
            const cplx z = !TWO_PASS ? (F32 ? near_eval32(y, w, o) : near_eval(y, w, o))
                                     : (F32 ? near_eval32_fast(y, w, o, need) : near_eval_fast(y, w, o, need));
            if (need) {
                // positions top - 1 - nredo >= qn have been consumed already
                slot(top - 1 - nredo) = (uint16_t)e;
                ++nredo;
            } else {
                add(s, z);
            }
        }
    }
    if (TWO_PASS && redo_count) *redo_count += (unsigned long long)wave_sum(nredo);
    while (TWO_PASS && __any(nredo > 0)) {
        if (nredo > 0) {
            --nredo;
            const int e = slot(top - 1 - nredo);
            const int r = e >> 3, s = e & 7;
            double y[4], w[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) { y[k] = list[r].y[k]; w[k] = list[r].w[k]; }
            const double o = omega[lane + kWave * s];
            add(s, F32 ? near_eval32(y, w, o) : near_eval(y, w, o));
        }
    }
}

// Work counted by the census instantiation (COUNT) of the dynamic body, wave totals.
struct WorkCount {
    unsigned long long units, tets, near, far, terms, redo, coef;
};

// One workgroup of the dynamic evaluation of one q: workgroup blk of nblocks, writing its
// partial sums for every frequency to part[nw][2].  The units are [u0, u1) (u1 < 0: all of them;
// a band pair's units are consecutive, for the pair-resolved call).  With COUNT the same evaluation also counts
// its work into *wc (units with a non-empty carved region and final tetrahedra only when
// count_tets is set, so that a frequency grid split over launches counts them once).
template <int NSLOT, bool MIXED, bool LIST, bool COUNT = false>
__device__ __forceinline__ void dynamic_body(const MeshDev &M, const QDev &Q, int nblocks, int blk,
                                             const double *__restrict__ omega, int nw, double *__restrict__ part,
                                             DynRec<MIXED> *list, uint16_t (*queue)[kWave], WorkCount *wc = nullptr,
                                             bool count_tets = false, int64_t u0 = 0, int64_t u1 = -1)
{
    const int lane = threadIdx.x;
    const int64_t n_units = u1 < 0 ? tets_per_pair(M) * M.nbw * M.nbw : u1;
    constexpr double kRho = MIXED ? kRhoFar32 : kRhoFar;     // far ratio of the series in use

    // frequencies of this lane (slot s holds w[lane + 64 s]; dead lanes repeat the last one)
    // and their interval [wlo, whi] over the wave, from which each tetrahedron's far-series
    // class follows
    double om[NSLOT];
    bool live[NSLOT];
    cplx acc[NSLOT];
    double wlo = omega[nw - 1], whi = wlo;
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
        const int idx = lane + kWave * s;
        live[s] = idx < nw;
        om[s] = omega[live[s] ? idx : nw - 1];
        acc[s] = cmk(0.0, 0.0);
        wlo = fmin(wlo, om[s]);
        whi = fmax(whi, om[s]);
    }
    wlo = wave_min(wlo);
    whi = wave_max(whi);
    const PairMask pm = pair_mask(M, Q, lane);
    int qn = 0, qn32 = 0;      // this lane's FP64 and FP32 near items queued

    // rounds of 64 consecutive units, dealt to the workgroups round-robin: every workgroup
    // samples all band pairs, so the work per workgroup is even
    for (int64_t base = u0 + (int64_t)blk * kWave; base < n_units; base += (int64_t)nblocks * kWave) {
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
        if (COUNT && count_tets) wc->units += __popcll(__ballot(cnt > 0));
        int start = 0;
        while (start < kWave) {
            int next;
            const int nrec = fill_list<DynRec<MIXED>, kCapDyn, LIST>(M, Q, ux, valid, cnt, start, lane, list, next);
            start = next;
            if (nrec == 0) continue;
            if (COUNT && count_tets) wc->tets += nrec;
            __syncthreads();
            // per-tetrahedron preparation, one lane per tetrahedron (nrec <= kCapDyn < kWave)
            const bool mine = lane < nrec;
            double y[4] = {0.0, 0.0, 0.0, 0.0}, w[4] = {0.0, 0.0, 0.0, 0.0};
            double c0 = 0.0, hs0 = 0.0;     // centre and half-span of this lane's D values
            if (mine) {
#pragma unroll
                for (int k = 0; k < 4; ++k) { y[k] = list[lane].y[k]; w[k] = list[lane].w[k]; }
                sort4(y, w);
                c0 = 0.5 * (y[0] + y[3]);
                hs0 = 0.5 * (y[3] - y[0]);
            }
            // The list as one cluster: when every frequency of the interval is far from the span
            // [C - R, C + R] of all its D values, the weights of all its tetrahedra are one series
            // in 1/(w - C) whose coefficients are the sums of the tetrahedra's coefficients about
            // C (each converges at the same ratio R/|w - C| <= kRho, so the truncation bound is
            // that of a single tetrahedron), and the frequencies pay one Horner evaluation for
            // the whole list.  Such a frequency is far from every tetrahedron of the list, so no
            // near item arises.
            const double clo = wave_min(mine ? c0 - hs0 : INFINITY), chi = wave_max(mine ? c0 + hs0 : -INFINITY);
            const double C = 0.5 * (clo + chi), R = 0.5 * (chi - clo);
            const double distC = fmax(fmax(wlo - C, C - whi), 0.0);
            const bool cluster = R < kRho * distC;
            const int clsC = far_class(R, distC, fmax(fabs(wlo - C), fabs(whi - C)), kRho);
            if (COUNT && count_tets) {
                // coefficients computed below (blocks of kFarTerms / kFarClasses terms)
                int nb = 0;
                if (mine) {
                    const double dist = fmax(fmax(wlo - c0, c0 - whi), 0.0);
                    nb = cluster ? clsC : far_class(hs0, dist, fmax(fabs(wlo - c0), fabs(whi - c0)), kRho);
                }
                wc->coef += (unsigned long long)wave_sum(nb) * ((MIXED ? kFarTerms32 : kFarTerms) / kFarClasses);
            }
            if (mine) {
                const double dist = fmax(fmax(wlo - c0, c0 - whi), 0.0);
                const double cc = cluster ? C : c0;
                const int cls = far_class(hs0, dist, fmax(fabs(wlo - c0), fabs(whi - c0)), kRho);
                // only the blocks of terms a Horner sum reads: the tetrahedron's own class, or the
                // list's when the list is summed as one series (later ones stay unread)
                if constexpr (MIXED) {
                    double a[kFarTerms32] = {};
                    far_coeffs_blocks<kFarTerms32, kFarClasses>(y, w, cc, a, cluster ? clsC : cls);
#pragma unroll
                    for (int m = 0; m < kFarTerms32; ++m) list[lane].a32[m] = (float)a[m];
                } else {
                    far_coeffs_blocks<kFarTerms, kFarClasses>(y, w, cc, list[lane].a, cluster ? clsC : cls);
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) { list[lane].y[k] = y[k]; list[lane].w[k] = w[k]; }
                list[lane].c = c0;
                list[lane].hs = hs0;
                list[lane].cls = cls;
                list[lane].flags = (hs0 < kRho * dist ? 1 : 0) | (near_degenerate(y, M.degen_tol, M.degen_rel) ? 2 : 0);
            }
            __syncthreads();
            if (cluster) {
                // coefficients of the list about C, summed over the tetrahedra in list order into
                // the (empty) near queue's memory, then one Horner evaluation per frequency
                double *acl = reinterpret_cast<double *>(&queue[0][0]);
                constexpr int KC = MIXED ? kFarTerms32 : kFarTerms;
                if (lane < KC) {
                    double sum = 0.0;
                    for (int r = 0; r < nrec; ++r) {
                        if constexpr (MIXED) sum += (double)list[r].a32[lane];
                        else sum += list[r].a[lane];
                    }
                    acl[lane] = sum;
                }
                __syncthreads();
                if (MIXED) {
                    float a[kFarTerms32], tt[NSLOT], f[NSLOT];
#pragma unroll
                    for (int m = 0; m < kFarTerms32; ++m) a[m] = (float)acl[m];
#pragma unroll
                    for (int s = 0; s < NSLOT; ++s) tt[s] = recip32((float)(om[s] - C));
                    horner_slots<kFarTerms32, NSLOT>(a, tt, clsC, f);
#pragma unroll
                    for (int s = 0; s < NSLOT; ++s) acc[s].re += (double)(f[s] * tt[s]);
                    if (COUNT) {
                        wc->far += nw;
                        wc->terms += (unsigned long long)nw * (clsC * kFarTerms32 / kFarClasses);
                    }
                } else {
                    double tt[NSLOT], f[NSLOT];
#pragma unroll
                    for (int s = 0; s < NSLOT; ++s) tt[s] = rcp(om[s] - C);
                    horner_slots_lds<kFarTerms, NSLOT>(acl, tt, clsC, f);
#pragma unroll
                    for (int s = 0; s < NSLOT; ++s) acc[s].re = fma(f[s], tt[s], acc[s].re);
                    if (COUNT) {
                        wc->far += nw;
                        wc->terms += (unsigned long long)nw * (clsC * kFarTerms / kFarClasses);
                    }
                }
            }
            for (int r = 0; r < (cluster ? 0 : nrec); ++r) {
                // far branch: all slots at once, 8 independent Horner chains on coefficients
                // read from LDS (broadcast) into registers; the series is cut to the terms the
                // distance between this tetrahedron and the frequency interval needs (a
                // wave-uniform class, so the cut is a scalar branch per block of terms).  When
                // the whole interval is far from the tetrahedron no frequency can take the near
                // branch, and the per-frequency tests are skipped.
                const double c = list[r].c, hs = list[r].hs;
                const int cls = __builtin_amdgcn_readfirstlane(list[r].cls);
                const int flags = __builtin_amdgcn_readfirstlane(list[r].flags);
                const bool allfar = (flags & 1) != 0;
                // mixed form: near items of non-degenerate tetrahedra go to the FP32 end
                const bool f32 = MIXED && (flags & 2) == 0;
                bool nearb[NSLOT];
#pragma unroll
                for (int s = 0; s < NSLOT; ++s) nearb[s] = allfar ? false : !(hs <= kRho * fabs(om[s] - c));
                if (COUNT) {
                    unsigned long long nn = 0, nf = 0;
#pragma unroll
                    for (int s = 0; s < NSLOT; ++s) {
                        nn += __popcll(__ballot(live[s] && nearb[s]));
                        nf += __popcll(__ballot(live[s] && !nearb[s]));
                    }
                    if (cls == 0) {      // every frequency near: the far Horner is skipped
                        nn += nf;
                        nf = 0;
                    }
                    wc->near += nn;
                    wc->far += nf;
                    wc->terms += nf * (unsigned long long)(cls * (MIXED ? kFarTerms32 : kFarTerms) / kFarClasses);
                }
                if (cls != 0 && MIXED) {
                    float a[kFarTerms32];
#pragma unroll
                    for (int m = 0; m < kFarTerms32; m += 4) {
                        const float4 v = *reinterpret_cast<const float4 *>(&list[r].a32[m]);
                        a[m] = v.x; a[m + 1] = v.y; a[m + 2] = v.z; a[m + 3] = v.w;
                    }
                    float tt[NSLOT], f[NSLOT];
                    if (allfar) {
#pragma unroll
                        for (int s = 0; s < NSLOT; ++s) tt[s] = recip32((float)(om[s] - c));
                        horner_slots<kFarTerms32, NSLOT>(a, tt, cls, f);
#pragma unroll
                        for (int s = 0; s < NSLOT; ++s) acc[s].re += (double)(f[s] * tt[s]);
                    } else {
#pragma unroll
                        for (int s = 0; s < NSLOT; ++s) tt[s] = recip32((float)(nearb[s] ? 1.0 : om[s] - c));
                        horner_slots<kFarTerms32, NSLOT>(a, tt, cls, f);
#pragma unroll
                        for (int s = 0; s < NSLOT; ++s)
                            if (!nearb[s]) acc[s].re += (double)(f[s] * tt[s]);
                    }
                } else if (!MIXED && cls != 0) {
                    const double *a = list[r].a;
                    double tt[NSLOT], f[NSLOT];
                    if (allfar) {
#pragma unroll
                        for (int s = 0; s < NSLOT; ++s) tt[s] = rcp(om[s] - c);
                        horner_slots_lds<kFarTerms, NSLOT>(a, tt, cls, f);
#pragma unroll
                        for (int s = 0; s < NSLOT; ++s) acc[s].re = fma(f[s], tt[s], acc[s].re);
                    } else {
#pragma unroll
                        for (int s = 0; s < NSLOT; ++s) tt[s] = rcp(nearb[s] ? 1.0 : om[s] - c);
                        horner_slots_lds<kFarTerms, NSLOT>(a, tt, cls, f);
#pragma unroll
                        for (int s = 0; s < NSLOT; ++s)
                            if (!nearb[s]) acc[s].re = fma(f[s], tt[s], acc[s].re);
                    }
                }
                if (!allfar) {
#pragma unroll
                    for (int s = 0; s < NSLOT; ++s) {
                        if (nearb[s] && live[s]) {
                            if (f32) {
                                queue[kQCap - 1 - qn32][lane] = (uint16_t)((r << 3) | s);
                                ++qn32;
                            } else {
                                queue[qn][lane] = (uint16_t)((r << 3) | s);
                                ++qn;
                            }
                        }
                    }
                }
                // one drain site (the near evaluations are long; one inlined copy keeps the kernel
                // within the instruction cache): when a queue may not hold the next tetrahedron's
                // items, and after the list's last tetrahedron
                if (r == nrec - 1 || __any(qn + qn32 > kQCap - NSLOT)) {
                    drain_near<NSLOT, false, !MIXED>(list, queue, qn, lane, omega, acc, COUNT ? &wc->redo : nullptr);
                    if (MIXED) drain_near<NSLOT, true>(list, queue, qn32, lane, omega, acc);
                }
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
        const int idx = lane + kWave * s;
        if (idx < nw) {
            part[2 * idx] = acc[s].re;
            part[2 * idx + 1] = acc[s].im;
        }
    }
}

template <int NSLOT, bool MIXED, bool LIST>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void tetra_dynamic_kernel(MeshDev M, BatchDev B, int nblocks,
                                                           const double *__restrict__ omega, int nw,
                                                           double *__restrict__ partial)
{
    __shared__ DynRec<MIXED> list[kCapDyn];
    __shared__ __attribute__((aligned(16))) uint16_t queue[kQCap][kWave];
    const int qi = blockIdx.y;
    dynamic_body<NSLOT, MIXED, LIST>(M, B.q[qi], nblocks, blockIdx.x, omega, nw,
                               partial + ((int64_t)qi * nblocks + blockIdx.x) * nw * 2, list, queue);
}

// Band-pair resolved dynamic evaluation (mesh plans): workgroup x = p * nblk + j takes the units of
// pair p as part j of nblk; partial[q][pair][j][nw][2].
template <int NSLOT, bool MIXED>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void tetra_dynamic_pairs_kernel(
    MeshDev M, BatchDev B, int nblk, const double *__restrict__ omega, int nw, double *__restrict__ partial)
{
    __shared__ DynRec<MIXED> list[kCapDyn];
    __shared__ __attribute__((aligned(16))) uint16_t queue[kQCap][kWave];
    const int qi = blockIdx.y;
    const int npairs = M.nbw * M.nbw;
    const int p = blockIdx.x / nblk, j = blockIdx.x - p * nblk;
    const int64_t per_pair = tets_per_pair(M);
    dynamic_body<NSLOT, MIXED, false>(M, B.q[qi], nblk, j, omega, nw,
                                      partial + (((int64_t)qi * npairs + p) * nblk + j) * nw * 2, list, queue, nullptr,
                                      false, (int64_t)p * per_pair, (int64_t)(p + 1) * per_pair);
}

// Static evaluation (w = 0, Re only) of units [u0, u1) by workgroup blk of nblocks: rounds of
// 64 consecutive units dealt round-robin; each lane evaluates its own final tetrahedra.
// Returns the workgroup's sum (valid in every lane).
template <bool LIST>
__device__ __forceinline__ double static_body(const MeshDev &M, const QDev &Q, int64_t u0, int64_t u1, int blk,
                                              int nblocks, StatRec *list)
{
    const int lane = threadIdx.x;
    double acc = 0.0;
    const PairMask pm = pair_mask(M, Q, lane);
    for (int64_t base = u0 + (int64_t)blk * kWave; base < u1; base += (int64_t)nblocks * kWave) {
        const UnitIdx b0 = decode_unit<LIST>(M, base);
        if (round_inert<LIST>(M, pm, b0)) continue;
        const UnitIdx ux = round_unit<LIST>(M, b0, lane);
        const bool valid = base + lane < u1;
        int cnt = 0;
        if (valid) {
            Vtx t[4];
            load_unit<LIST>(M, Q, ux, t);
            cnt = count_unit(t, M.form);
        }
        int start = 0;
        while (start < kWave) {
            int next;
            const int nrec = fill_list<StatRec, kCapStat, LIST>(M, Q, ux, valid, cnt, start, lane, list, next);
            start = next;
            if (nrec == 0) continue;
            __syncthreads();
            for (int r = lane; r < nrec; r += kWave) {
                const double D[4] = {list[r].D[0], list[r].D[1], list[r].D[2], list[r].D[3]};
                const double w[4] = {list[r].w[0], list[r].w[1], list[r].w[2], list[r].w[3]};
                acc += tetra_weight_sum(D, w, 0.0).re;
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, kWave);
    return acc;
}

}  // namespace
}  // namespace chi0
