// chi0_api.cpp -- the C ABI of libchi0: argument checks, workspace layout and the
// launch sequence per batch of q-points:
//   K_A  matrix elements W_nm(k) for every q of the batch (skipped under CMA)
//   K_B  carving + tetrahedron weights -> per-workgroup partial sums
//   K_R  ordered reduction of the partial sums -> chi0(q, w)
// Every check is done on the host before anything is enqueued.
#include "../../include/chi0.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "chi0_host.h"
#include "chi0_internal.h"
#include "chi0_math.h"

using namespace chi0;

struct TimedLaunch {
    int kind;
    hipEvent_t start, stop;
};

// Verdict slots of the asynchronous input scans: each call's verdict word is copied from the
// workspace into one pinned host word, whose event says when it has landed.
constexpr int kScanSlots = 8;

struct chi0_plan_s {
    chi0_desc d;
    MeshDev mesh;
    bool list = false;      // tetrahedron-list plan: explicit q only, prefactor spin_factor * volume
    double volume = 0.0;
    int qbatch = kMaxQBatch;   // q-points per launch sequence (batch_hint)
    hipStream_t stream;
    std::string err;
    bool profiling = false;
    std::vector<TimedLaunch> events;
    // input scans (allocated at plan creation when a device is present)
    unsigned *scan_host = nullptr;          // pinned [kScanSlots]
    hipEvent_t scan_ev[kScanSlots] = {};
    bool scan_pending[kScanSlots] = {};
    int scan_next = 0;
    unsigned scan_bits = 0;                 // verdicts landed and not yet reported
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

chi0_status fail(chi0_plan_t p, chi0_status st, const char *msg)
{
    if (p) p->err = msg;
    return st;
}

chi0_status device_fail(chi0_plan_t p, hipError_t e, const char *where)
{
    if (p) {
        p->err = std::string(where) + ": " + hipGetErrorString(e);
    }
    return CHI0_E_DEVICE;
}

// Pinned verdict words and their events; without a device the plan simply has none (every
// computing call then fails at its first launch anyway).
void scan_setup(chi0_plan_s *p)
{
    if (p->d.skip_input_scan) return;
    void *h = nullptr;
    if (hipHostMalloc(&h, sizeof(unsigned) * kScanSlots, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    for (int i = 0; i < kScanSlots; ++i) {
        if (hipEventCreateWithFlags(&p->scan_ev[i], hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(p->scan_ev[j]);
            (void)hipHostFree(h);
            return;
        }
    }
    p->scan_host = static_cast<unsigned *>(h);
}

void scan_release(chi0_plan_s *p)
{
    if (!p->scan_host) return;
    for (int i = 0; i < kScanSlots; ++i) (void)hipEventDestroy(p->scan_ev[i]);
    (void)hipHostFree(p->scan_host);
    p->scan_host = nullptr;
}

// Collect the verdicts that have landed (all of them, waiting, when block is set).
void scan_collect(chi0_plan_s *p, bool block)
{
    if (!p->scan_host) return;
    for (int k = 0; k < kScanSlots; ++k) {
        const int i = (p->scan_next + k) % kScanSlots;     // oldest first
        if (!p->scan_pending[i]) continue;
        const hipError_t e = block ? hipEventSynchronize(p->scan_ev[i]) : hipEventQuery(p->scan_ev[i]);
        if (e == hipErrorNotReady) continue;
        p->scan_pending[i] = false;
        if (e == hipSuccess) p->scan_bits |= p->scan_host[i];
    }
}

// The status for collected verdicts (consumed), CHI0_OK if none.
chi0_status scan_report(chi0_plan_s *p)
{
    const unsigned b = p->scan_bits;
    if (!b) return CHI0_OK;
    p->scan_bits = 0;
    std::string what;
    if (b & kScanEps) what += " band energies;";
    if (b & kScanEig) what += " eigenvector coefficients;";
    if (b & kScanOmega) what += " frequencies;";
    if (b & (kScanEps | kScanEig | kScanOmega)) {
        p->err = "input scan of an earlier call: non-finite" + what;
        if (b & kScanNorm) p->err += " and eigenvectors not normalised";
        return CHI0_E_NONFINITE;
    }
    p->err = "input scan of an earlier call: an eigenvector's squared norm differs from 1 by more than 1e-6";
    return CHI0_E_NOT_NORMALIZED;
}

// Start of every computing call: report a verdict of an earlier scan that has landed.
chi0_status begin_call(chi0_plan_s *p)
{
    scan_collect(p, false);
    return scan_report(p);
}

// Enqueue the scan of the inputs of one call: mesh arrays, the explicit k+q arrays of qs (each
// distinct array once) and omega; the verdict word sits in the workspace at flag.
chi0_status enqueue_scan(chi0_plan_s *p, int nq, const chi0_q *qs, const double *omega, int nw, unsigned *flag)
{
    if (p->d.skip_input_scan || !p->scan_host) return CHI0_OK;
    const int slot = p->scan_next;
    if (p->scan_pending[slot]) {           // the ring is full: wait for its oldest verdict
        const hipError_t e = hipEventSynchronize(p->scan_ev[slot]);
        if (e != hipSuccess) return device_fail(p, e, "input scan");
        p->scan_pending[slot] = false;
        p->scan_bits |= p->scan_host[slot];
    }
    const MeshDev &M = p->mesh;
    const double tol = 1e-6;
    hipError_t e = launch_scan_clear(flag, p->stream);
    if (e == hipSuccess) e = launch_scan_finite(M.eps_k, (int64_t)M.nb * M.nk, kScanEps, flag, p->stream);
    if (e == hipSuccess && !M.cma)
        e = launch_scan_eigvec(M.c_k, M.nk, M.no, M.nb, kScanEig, kScanNorm, tol, flag, p->stream);
    // each distinct explicit array once (an array repeated in several entries, as in a group
    // call, is scanned at its first entry; no host allocation on this path)
    auto first_use = [&](int i, bool eps) {
        const void *a = eps ? (const void *)qs[i].eps_kq : (const void *)qs[i].c_kq;
        for (int j = 0; j < i; ++j)
            if (qs[j].explicit_kq == 1 && (eps ? (const void *)qs[j].eps_kq : (const void *)qs[j].c_kq) == a)
                return false;
        return true;
    };
    for (int i = 0; i < nq && e == hipSuccess; ++i) {
        if (qs[i].explicit_kq != 1) continue;
        if (first_use(i, true)) e = launch_scan_finite(qs[i].eps_kq, (int64_t)M.nb * M.nk, kScanEps, flag, p->stream);
        if (e == hipSuccess && !M.cma && qs[i].c_kq && first_use(i, false))
            e = launch_scan_eigvec(qs[i].c_kq, M.nk, M.no, M.nb, kScanEig, kScanNorm, tol, flag, p->stream);
    }
    if (e == hipSuccess && omega) e = launch_scan_finite(omega, nw, kScanOmega, flag, p->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&p->scan_host[slot], flag, sizeof(unsigned), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipEventRecord(p->scan_ev[slot], p->stream);
    if (e != hipSuccess) return device_fail(p, e, "input scan");
    p->scan_pending[slot] = true;
    p->scan_next = (slot + 1) % kScanSlots;
    return CHI0_OK;
}

int64_t n_units(const chi0_plan_s *p)
{
    return tets_per_pair(p->mesh) * p->mesh.nbw * p->mesh.nbw;
}

// Prefactor of the tetrahedron sum: g_s times the zone fraction of one tetrahedron.
double prefactor(const chi0_plan_s *p)
{
    return p->list ? p->d.spin_factor * p->volume : p->d.spin_factor / (6.0 * (double)p->mesh.nk);
}

// Workgroups per q: up to 1024, each taking at least 4 rounds of 64 units.
int n_blocks(const chi0_plan_s *p)
{
    const int64_t rounds = (n_units(p) + kWave - 1) / kWave;
    return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (rounds + 3) / 4));
}

// Workgroups per band pair of the pair-resolved static call: up to 64, each at least 4 rounds.
int n_blocks_pair(const chi0_plan_s *p)
{
    const int64_t rounds = (tets_per_pair(p->mesh) + kWave - 1) / kWave;
    return (int)std::max<int64_t>(1, std::min<int64_t>(64, (rounds + 3) / 4));
}

struct Layout {
    size_t w_off, w_bytes_per_q, part_off, part_bytes_per_q, pack_off, pack_bytes, count_off, flag_off, rng_off,
        rng_bytes, total;
    int qbatch;
};

// The band ranges of a q batch (e(k), then each q's e(k+q)): [1 + qbatch][nbw][2] doubles.
size_t range_bytes(const chi0_plan_s *p, int qbatch)
{
    return align_up(sizeof(double) * 2 * (size_t)p->mesh.nbw * (size_t)(1 + qbatch));
}

// qcap > 0 caps the q-points per launch sequence below the plan's own (the no-allocation call);
// packed: room for the split operands of a split-precision plane-wave plan whose launches take
// at least kPackMinQ q (not in the no-allocation call, whose scratch is too small for them).
Layout layout(const chi0_plan_s *p, int nq, int nvals, int qcap = 0, bool packed = true)
{
    Layout L;
    L.qbatch = std::min(nq, qcap > 0 ? std::min(qcap, p->qbatch) : p->qbatch);
    L.w_bytes_per_q = p->d.cma ? 0 : align_up(sizeof(double) * (size_t)p->mesh.nbw * p->mesh.nbw * p->mesh.nk);
    // the partial sums of a dynamic or static call, or of a pair-resolved static call
    const size_t npairs = (size_t)p->mesh.nbw * p->mesh.nbw;
    L.part_bytes_per_q = align_up(sizeof(double) * std::max((size_t)n_blocks(p) * nvals,
                                                           (size_t)n_blocks_pair(p) * npairs));
    L.w_off = 0;
    L.part_off = L.w_bytes_per_q * L.qbatch;
    L.pack_off = L.part_off + L.part_bytes_per_q * L.qbatch;
    L.pack_bytes = packed && L.qbatch >= kPackMinQ && !p->d.cma && p->d.precision != 0 && p->mesh.no > kMaxOrbSmall
                       ? align_up(pack_bytes(p->mesh))
                       : 0;
    L.count_off = L.pack_off + L.pack_bytes;
    L.flag_off = L.count_off + 128;       // census counters (56 bytes), then the scan verdict
    L.rng_off = L.count_off + kAlign;
    L.rng_bytes = range_bytes(p, L.qbatch);
    L.total = L.rng_off + L.rng_bytes;
    return L;
}

// The split-operand region of a call's workspace, not yet filled.
PackState pack_state(void *ws, const Layout &L)
{
    return PackState{L.pack_bytes ? static_cast<char *>(ws) + L.pack_off : nullptr, false};
}

unsigned *scan_flag(void *ws, const Layout &L)
{
    return reinterpret_cast<unsigned *>(static_cast<char *>(ws) + L.flag_off);
}

// Workspace of the Kramers-Kronig route: W and the partial sums as for a dynamic call (up to
// kMaxOmegaIm frequencies per launch), then the frequency list (grid and requested) and the
// imaginary part on it for one batch of q.
struct KKLayout {
    size_t w_off, w_bytes_per_q, part_off, part_bytes_per_q, om_off, im_off, flag_off, rng_off, rng_bytes, total;
    int qbatch, n_all;
};

KKLayout kk_layout(const chi0_plan_s *p, int nq, int nw, int K)
{
    KKLayout L;
    L.qbatch = std::min(nq, p->qbatch);
    L.n_all = K + nw;
    L.w_bytes_per_q = p->d.cma ? 0 : align_up(sizeof(double) * (size_t)p->mesh.nbw * p->mesh.nbw * p->mesh.nk);
    L.part_bytes_per_q = align_up(sizeof(double) * (size_t)n_blocks(p) * 2 * std::min(L.n_all, kMaxOmegaIm));
    L.w_off = 0;
    L.part_off = L.w_bytes_per_q * L.qbatch;
    L.om_off = L.part_off + L.part_bytes_per_q * L.qbatch;
    L.im_off = L.om_off + align_up(sizeof(double) * (size_t)L.n_all);
    L.flag_off = L.im_off + align_up(sizeof(double) * 2 * (size_t)L.n_all * L.qbatch);
    L.rng_off = L.flag_off + kAlign;
    L.rng_bytes = range_bytes(p, L.qbatch);
    L.total = L.rng_off + L.rng_bytes;
    return L;
}

// Workspace of the pair-resolved dynamic call: W of one q batch, then the partial sums
// [q][pair][nblk][2 nwc] (nblk workgroups per pair), then the scan verdict.
struct PairsLayout {
    size_t w_off, w_bytes_per_q, part_off, part_bytes_per_q, flag_off, rng_off, rng_bytes, total;
    int qbatch, nblk;
};

PairsLayout dpairs_layout(const chi0_plan_s *p, int nq, int nvals)
{
    PairsLayout L;
    L.qbatch = std::min(nq, p->qbatch);
    const int64_t rounds = (tets_per_pair(p->mesh) + kWave - 1) / kWave;
    // up to 64 workgroups per pair (16 measured 1.7x slower on the 100-pair workload: a pair's work
    // is uneven and lands on too few workgroups), at most 8192 per q so the partial sums stay
    // within 64 MiB per q at 512 frequencies, each at least 4 rounds
    const int64_t npairs = (int64_t)p->mesh.nbw * p->mesh.nbw;
    const int64_t cap = std::min<int64_t>(64, std::max<int64_t>(4, 8192 / npairs));
    L.nblk = (int)std::max<int64_t>(1, std::min<int64_t>(cap, (rounds + 3) / 4));
    L.w_bytes_per_q = p->d.cma ? 0 : align_up(sizeof(double) * (size_t)p->mesh.nbw * p->mesh.nbw * p->mesh.nk);
    L.part_bytes_per_q =
        align_up(sizeof(double) * (size_t)p->mesh.nbw * p->mesh.nbw * (size_t)L.nblk * (size_t)nvals);
    L.w_off = 0;
    L.part_off = L.w_bytes_per_q * L.qbatch;
    L.flag_off = L.part_off + L.part_bytes_per_q * L.qbatch;
    L.rng_off = L.flag_off + kAlign;
    L.rng_bytes = range_bytes(p, L.qbatch);
    L.total = L.rng_off + L.rng_bytes;
    return L;
}

chi0_status check_qs(chi0_plan_t p, int32_t nq, const chi0_q *qs)
{
    if (nq < 1 || !qs) return fail(p, CHI0_E_INVALID_ARG, "nq must be >= 1 and qs non-null");
    for (int i = 0; i < nq; ++i) {
        const char *msg = "";
        const chi0_status st = check_q(p->d, qs[i], &msg);
        if (st) return fail(p, st, msg);
        if (p->list && qs[i].explicit_kq != 1)
            return fail(p, CHI0_E_INVALID_ARG, "a tetrahedron-list plan takes explicit k+q data only");
    }
    return CHI0_OK;
}

// Launches of a group call: entries [e0, e0 + ne) of groups [g0, g0 + ng); a group of more than
// kMaxQBatch entries is split over launches whose results are added to the first one's.
struct GroupLaunch {
    int e0, ne, g0, ng;
    bool accumulate;
};

std::vector<GroupLaunch> group_launches(int nq, int n_group, int qbatch)
{
    std::vector<GroupLaunch> out;
    if (n_group <= qbatch) {
        const int per = qbatch / n_group;
        for (int g0 = 0; g0 < nq; g0 += per) {
            const int ng = std::min(per, nq - g0);
            out.push_back({g0 * n_group, ng * n_group, g0, ng, false});
        }
    } else {
        for (int g = 0; g < nq; ++g)
            for (int c0 = 0; c0 < n_group; c0 += qbatch)
                out.push_back({g * n_group + c0, std::min(qbatch, n_group - c0), g, 1, c0 > 0});
    }
    return out;
}

// The device descriptors of q0 .. q0 + nqb - 1: W of q i in the workspace's W region, and, when the
// layout has one, the band ranges in its range region (e(k) first, then q i's e(k+q)).
void fill_batch(const chi0_plan_s *p, const chi0_q *qs, int q0, int nqb, void *ws, const Layout &L, BatchDev &B)
{
    std::memset(&B, 0, sizeof B);
    double *rng = L.rng_bytes ? reinterpret_cast<double *>(static_cast<char *>(ws) + L.rng_off) : nullptr;
    for (int i = 0; i < nqb; ++i) {
        double *W = p->d.cma ? nullptr
                             : reinterpret_cast<double *>(static_cast<char *>(ws) + L.w_off + L.w_bytes_per_q * i);
        B.q[i] = make_qdev(p->mesh, qs[q0 + i], W);
        if (rng) {
            B.q[i].rng_k = rng;
            B.q[i].rng_kq = rng + 2 * (size_t)p->mesh.nbw * (1 + i);
        }
    }
}

// Run one launch, bracketed by events when profiling.
// (no_alloc: the no-allocation call records no profile events, whose creation allocates)
template <class F>
hipError_t timed(chi0_plan_s *p, int kind, F &&launch, bool no_alloc = false)
{
    if (!p->profiling || no_alloc) return launch();
    TimedLaunch t;
    t.kind = kind;
    hipError_t e = hipEventCreate(&t.start);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&t.stop)) != hipSuccess) return e;
    if ((e = hipEventRecord(t.start, p->stream)) != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(t.stop, p->stream)) != hipSuccess) return e;
    p->events.push_back(t);
    return hipSuccess;
}

}  // namespace

namespace chi0 {

chi0_status check_desc(const chi0_desc *d, const double *eps_k, const double *c_k)
{
    if (!d) return CHI0_E_INVALID_ARG;
    for (int i = 0; i < 3; ++i)
        if (d->nk[i] < 1) return CHI0_E_SHAPE;
    const int64_t nk = (int64_t)d->nk[0] * d->nk[1] * d->nk[2];
    if (nk >= (int64_t(1) << 31)) return CHI0_E_SHAPE;
    if (d->n_bands < 1 || d->n_bands > 64) return CHI0_E_SHAPE;
    const int hi = d->band_hi <= 0 ? d->n_bands : d->band_hi;
    if (d->band_lo < 0 || d->band_lo >= hi || hi > d->n_bands) return CHI0_E_SHAPE;
    if (hi - d->band_lo > 32) return CHI0_E_SHAPE;
    if (d->cma != 0 && d->cma != 1) return CHI0_E_INVALID_ARG;
    if (!d->cma && (d->n_orb < 1 || d->n_orb > kMaxOrb)) return CHI0_E_SHAPE;
    if (d->form != 0 && d->form != 1) return CHI0_E_INVALID_ARG;
    for (int i = 0; i < 3; ++i)
        if (d->reserved[i] != 0) return CHI0_E_INVALID_ARG;
    if (d->batch_hint < 0 || d->batch_hint > kMaxQBatch) return CHI0_E_INVALID_ARG;
    if (d->skip_input_scan != 0 && d->skip_input_scan != 1) return CHI0_E_INVALID_ARG;
    if (!std::isfinite(d->mu) || !std::isfinite(d->spin_factor) || !std::isfinite(d->degen_tol_ev) ||
        !std::isfinite(d->degen_rel_tol))
        return CHI0_E_NONFINITE;
    if (d->degen_tol_ev < 0.0 || d->degen_rel_tol < 0.0) return CHI0_E_INVALID_ARG;
    if (d->precision < 0 || d->precision > 2) return CHI0_E_INVALID_ARG;
    if (!eps_k) return CHI0_E_INVALID_ARG;
    if (!d->cma && !c_k) return CHI0_E_INVALID_ARG;
    return CHI0_OK;
}

MeshDev make_mesh(const chi0_desc &d, const double *eps_k, const double *c_k)
{
    MeshDev M;
    std::memset(&M, 0, sizeof M);
    const int hi = d.band_hi <= 0 ? d.n_bands : d.band_hi;
    M.n1 = d.nk[0];
    M.n2 = d.nk[1];
    M.n3 = d.nk[2];
    M.nk = (int64_t)d.nk[0] * d.nk[1] * d.nk[2];
    M.nb = d.n_bands;
    M.no = d.cma ? 1 : d.n_orb;
    M.lo = d.band_lo;
    M.nbw = hi - d.band_lo;
    M.cma = d.cma;
    M.form = d.form;
    M.mu = d.mu;
    M.eps_k = eps_k;
    M.c_k = c_k;
    M.ncell = M.nk;
    M.nperm = 6;
    M.tets = nullptr;
    M.degen_tol = d.degen_tol_ev > 0.0 ? d.degen_tol_ev : kDegenerateTol;
    M.degen_rel = d.degen_rel_tol;
    return M;
}

// Mesh shift of a q given by q_frac: q_frac[a] * N_a rounded, when it is an integer to 1e-9
// relative; false otherwise.
bool shift_from_frac(const chi0_desc &d, const chi0_q &q, int32_t shift[3])
{
    for (int a = 0; a < 3; ++a) {
        const double x = q.q_frac[a] * (double)d.nk[a];
        const double r = std::nearbyint(x);
        if (!(std::fabs(x - r) <= 1e-9 * std::max(1.0, std::fabs(x)))) return false;
        const double m = std::fmod(r, (double)d.nk[a]);
        shift[a] = (int32_t)(m < 0 ? m + d.nk[a] : m);
    }
    return true;
}

chi0_status check_q(const chi0_desc &d, const chi0_q &q, const char **msg)
{
    if (q.explicit_kq < 0 || q.explicit_kq > 2) {
        *msg = "explicit_kq must be 0, 1 or 2";
        return CHI0_E_INVALID_ARG;
    }
    if (q.explicit_kq == 2) {
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(q.q_frac[a])) {
                *msg = "q_frac not finite";
                return CHI0_E_NONFINITE;
            }
        int32_t s[3];
        if (!shift_from_frac(d, q, s)) {
            *msg = "q_frac is not a vector of the mesh";
            return CHI0_E_NOT_COMMENSURATE;
        }
    }
    if (q.explicit_kq == 1) {
        if (!q.eps_kq) {
            *msg = "explicit q without eps_kq";
            return CHI0_E_INVALID_ARG;
        }
        if (!d.cma && !q.c_kq) {
            *msg = "explicit q without c_kq";
            return CHI0_E_INVALID_ARG;
        }
    }
    return CHI0_OK;
}

QDev make_qdev(const MeshDev &M, const chi0_q &q, double *W)
{
    QDev d;
    std::memset(&d, 0, sizeof d);
    const int n[3] = {M.n1, M.n2, M.n3};
    d.explicit_kq = q.explicit_kq == 1 ? 1 : 0;
    if (q.explicit_kq == 1) {
        d.eps_kq = q.eps_kq;
        d.c_kq = q.c_kq;
    } else {
        d.eps_kq = M.eps_k;
        d.c_kq = M.c_k;
        int32_t s[3] = {q.shift[0], q.shift[1], q.shift[2]};
        if (q.explicit_kq == 2) {
            chi0_desc dd;
            std::memset(&dd, 0, sizeof dd);
            dd.nk[0] = M.n1; dd.nk[1] = M.n2; dd.nk[2] = M.n3;
            shift_from_frac(dd, q, s);     // validated by check_q
        }
        d.explicit_kq = 0;
        for (int a = 0; a < 3; ++a) d.shift[a] = ((s[a] % n[a]) + n[a]) % n[a];
    }
    d.W = M.cma ? nullptr : W;
    return d;
}

}  // namespace chi0

extern "C" {

const char *chi0_status_string(chi0_status s)
{
    switch (s) {
    case CHI0_OK: return "ok";
    case CHI0_E_INVALID_ARG: return "invalid argument";
    case CHI0_E_SHAPE: return "shape out of range";
    case CHI0_E_NONFINITE: return "non-finite input";
    case CHI0_E_WORKSPACE: return "workspace too small";
    case CHI0_E_DEVICE: return "device error";
    case CHI0_E_UNSUPPORTED: return "unsupported";
    case CHI0_E_NOT_COMMENSURATE: return "q not commensurate with the mesh";
    case CHI0_E_NOT_NORMALIZED: return "eigenvectors not normalised";
    }
    return "unknown status";
}

const char *chi0_last_error(chi0_plan_t p) { return p ? p->err.c_str() : ""; }

chi0_status chi0_plan(chi0_plan_t *out, const chi0_desc *d, const double *eps_k, const double *c_k, void *stream)
{
    if (!out) return CHI0_E_INVALID_ARG;
    *out = nullptr;
    const chi0_status st = check_desc(d, eps_k, c_k);
    if (st) return st;
    chi0_plan_s *p = new (std::nothrow) chi0_plan_s();
    if (!p) return CHI0_E_INVALID_ARG;
    p->d = *d;
    p->mesh = make_mesh(*d, eps_k, c_k);
    p->d.band_hi = p->mesh.lo + p->mesh.nbw;
    p->qbatch = d->batch_hint > 0 ? d->batch_hint : kMaxQBatch;
    p->stream = static_cast<hipStream_t>(stream);
    scan_setup(p);
    *out = p;
    return CHI0_OK;
}

chi0_status chi0_plan_list(chi0_plan_t *out, const chi0_desc *d, const chi0_tetra_list *list, const double *eps_k,
                           const double *c_k, void *stream)
{
    if (!out) return CHI0_E_INVALID_ARG;
    *out = nullptr;
    if (!d || !list || !list->tets) return CHI0_E_INVALID_ARG;
    if (list->n_kp < 1 || list->n_kp >= (int64_t(1) << 31) || list->n_tet < 1 || list->n_tet >= (int64_t(1) << 31))
        return CHI0_E_SHAPE;
    if (!(list->volume > 0.0) || !std::isfinite(list->volume)) return CHI0_E_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(list->tets) % 16 != 0) return CHI0_E_INVALID_ARG;
    // the band arrays are a one-dimensional "mesh" of n_kp points
    chi0_desc dl = *d;
    dl.nk[0] = (int32_t)list->n_kp;
    dl.nk[1] = dl.nk[2] = 1;
    const chi0_status st = check_desc(&dl, eps_k, c_k);
    if (st) return st;
    // every corner index must address a k-point: checked once on the host
    std::vector<int32_t> h((size_t)list->n_tet * 4);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(h.data(), list->tets, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost, hs) != hipSuccess ||
        hipStreamSynchronize(hs) != hipSuccess)
        return CHI0_E_DEVICE;
    for (int32_t v : h)
        if (v < 0 || v >= list->n_kp) return CHI0_E_SHAPE;
    chi0_plan_s *p = new (std::nothrow) chi0_plan_s();
    if (!p) return CHI0_E_INVALID_ARG;
    p->d = dl;
    p->mesh = make_mesh(dl, eps_k, c_k);
    p->mesh.ncell = list->n_tet;
    p->mesh.nperm = 1;
    p->mesh.tets = list->tets;
    p->list = true;
    p->volume = list->volume;
    p->d.band_hi = p->mesh.lo + p->mesh.nbw;
    p->qbatch = d->batch_hint > 0 ? d->batch_hint : kMaxQBatch;
    p->stream = hs;
    scan_setup(p);
    *out = p;
    return CHI0_OK;
}

chi0_status chi0_destroy(chi0_plan_t p)
{
    if (p) {
        for (auto &t : p->events) {
            (void)hipEventDestroy(t.start);
            (void)hipEventDestroy(t.stop);
        }
        scan_collect(p, true);
        scan_release(p);
    }
    delete p;
    return CHI0_OK;
}

chi0_status chi0_sync(chi0_plan_t p)
{
    if (!p) return CHI0_E_INVALID_ARG;
    const hipError_t e = hipStreamSynchronize(p->stream);
    scan_collect(p, true);
    if (e != hipSuccess) return device_fail(p, e, "stream");
    return scan_report(p);
}

chi0_status chi0_profile_enable(chi0_plan_t p, int32_t enable)
{
    if (!p || (enable != 0 && enable != 1)) return CHI0_E_INVALID_ARG;
    p->profiling = enable == 1;
    return CHI0_OK;
}

chi0_status chi0_profile_read(chi0_plan_t p, chi0_profile *out)
{
    if (!p || !out) return CHI0_E_INVALID_ARG;
    std::memset(out, 0, sizeof *out);
    chi0_status st = CHI0_OK;
    for (auto &t : p->events) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(t.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.start, t.stop);
        if (e != hipSuccess) st = device_fail(p, e, "profile events");
        out->ms[t.kind] += ms;
        out->launches[t.kind] += 1;
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    p->events.clear();
    return st;
}

chi0_status chi0_census(chi0_plan_t p, int32_t nq, const chi0_q *qs, int32_t nw, const double *omega, void *ws,
                        size_t ws_bytes, uint64_t *counts)
{
    if (!p) return CHI0_E_INVALID_ARG;
    chi0_status st = begin_call(p);
    if (st) return st;
    st = check_qs(p, nq, qs);
    if (st) return st;
    if (nw < 1 || !omega || !counts) return fail(p, CHI0_E_INVALID_ARG, "nw >= 1, omega and counts required");
    const Layout L = layout(p, nq, 2 * std::min(nw, kMaxOmegaPerLaunch));
    if (!ws || ws_bytes < L.total) return fail(p, CHI0_E_WORKSPACE, "workspace too small");
    auto *dc = reinterpret_cast<unsigned long long *>(static_cast<char *>(ws) + L.count_off);
    double *partial = reinterpret_cast<double *>(static_cast<char *>(ws) + L.part_off);
    if ((st = enqueue_scan(p, nq, qs, omega, nw, scan_flag(ws, L))) != CHI0_OK) return st;
    hipError_t e = hipMemsetAsync(dc, 0, 7 * sizeof(unsigned long long), p->stream);
    if (e != hipSuccess) return device_fail(p, e, "census clear");
    for (int q0 = 0; q0 < nq; q0 += L.qbatch) {
        const int nqb = std::min(L.qbatch, nq - q0);
        BatchDev B;
        fill_batch(p, qs, q0, nqb, ws, L, B);
        for (int w0 = 0; w0 < nw; w0 += kMaxOmegaPerLaunch) {
            const int nwc = std::min(kMaxOmegaPerLaunch, nw - w0);
            if ((e = launch_census(p->mesh, B, nqb, n_blocks(p), omega + w0, nwc, partial, p->d.precision != 0,
                                   w0 == 0, dc, p->stream)) !=
                hipSuccess)
                return device_fail(p, e, "census kernel");
        }
    }
    unsigned long long h[7];
    if ((e = hipMemcpyAsync(h, dc, sizeof h, hipMemcpyDeviceToHost, p->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(p->stream)) != hipSuccess)
        return device_fail(p, e, "census copy");
    for (int i = 0; i < 7; ++i) counts[i] = h[i];
    return CHI0_OK;
}

chi0_status chi0_workspace_size(chi0_plan_t p, int32_t nq, int32_t nw, size_t *bytes)
{
    if (!p || !bytes) return CHI0_E_INVALID_ARG;
    if (nq < 1 || nw < 1) return fail(p, CHI0_E_INVALID_ARG, "nq and nw must be >= 1");
    *bytes = layout(p, nq, 2 * std::min(nw, kMaxOmegaPerLaunch)).total;
    return CHI0_OK;
}

chi0_status chi0_static(chi0_plan_t p, int32_t nq, const chi0_q *qs, void *ws, size_t ws_bytes, double *chi)
{
    if (!p) return CHI0_E_INVALID_ARG;
    chi0_status st = begin_call(p);
    if (st) return st;
    st = check_qs(p, nq, qs);
    if (st) return st;
    if (!chi) return fail(p, CHI0_E_INVALID_ARG, "chi is null");
    const Layout L = layout(p, nq, 1);
    size_t need = 0;
    chi0_workspace_size(p, nq, 1, &need);
    if (!ws || ws_bytes < need || ws_bytes < L.total) return fail(p, CHI0_E_WORKSPACE, "workspace too small");
    if ((st = enqueue_scan(p, nq, qs, nullptr, 0, scan_flag(ws, L))) != CHI0_OK) return st;
    const int nblk = n_blocks(p);
    double *partial = reinterpret_cast<double *>(static_cast<char *>(ws) + L.part_off);
    const double scale = prefactor(p);
    PackState pk = pack_state(ws, L);
    for (int q0 = 0; q0 < nq; q0 += L.qbatch) {
        const int nqb = std::min(L.qbatch, nq - q0);
        BatchDev B;
        fill_batch(p, qs, q0, nqb, ws, L, B);
        hipError_t e;
        if (!p->d.cma && (e = timed(p, 0, [&] {
                              return launch_contract(p->mesh, B, nqb, p->d.precision, &pk, p->stream);
                          })) != hipSuccess)
            return device_fail(p, e, "matrix-element kernel");
        if ((e = timed(p, 1, [&] { return launch_tetra_static(p->mesh, B, nqb, nblk, partial, p->stream); })) !=
            hipSuccess)
            return device_fail(p, e, "tetrahedron kernel");
        if ((e = timed(p, 2, [&] { return launch_reduce(partial, nqb, nblk, 1, scale, chi + q0, 1, p->stream); })) !=
            hipSuccess)
            return device_fail(p, e, "reduce kernel");
    }
    return CHI0_OK;
}

chi0_status chi0_static_pairs(chi0_plan_t p, int32_t nq, const chi0_q *qs, void *ws, size_t ws_bytes, double *chi)
{
    if (!p) return CHI0_E_INVALID_ARG;
    chi0_status st = begin_call(p);
    if (st) return st;
    st = check_qs(p, nq, qs);
    if (st) return st;
    if (!chi) return fail(p, CHI0_E_INVALID_ARG, "chi is null");
    const Layout L = layout(p, nq, 1);
    if (!ws || ws_bytes < L.total) return fail(p, CHI0_E_WORKSPACE, "workspace too small");
    if ((st = enqueue_scan(p, nq, qs, nullptr, 0, scan_flag(ws, L))) != CHI0_OK) return st;
    const int nblk = n_blocks_pair(p);
    const int npairs = p->mesh.nbw * p->mesh.nbw;
    double *partial = reinterpret_cast<double *>(static_cast<char *>(ws) + L.part_off);
    const double scale = prefactor(p);
    PackState pk = pack_state(ws, L);
    for (int q0 = 0; q0 < nq; q0 += L.qbatch) {
        const int nqb = std::min(L.qbatch, nq - q0);
        BatchDev B;
        fill_batch(p, qs, q0, nqb, ws, L, B);
        hipError_t e;
        if (!p->d.cma && (e = timed(p, 0, [&] {
                              return launch_contract(p->mesh, B, nqb, p->d.precision, &pk, p->stream);
                          })) != hipSuccess)
            return device_fail(p, e, "matrix-element kernel");
        if ((e = timed(p, 1, [&] { return launch_tetra_static_pairs(p->mesh, B, nqb, nblk, partial, p->stream); })) !=
            hipSuccess)
            return device_fail(p, e, "tetrahedron kernel");
        if ((e = timed(p, 2, [&] {
                 return launch_reduce(partial, nqb, nblk, npairs, scale, chi + (int64_t)q0 * npairs, npairs, p->stream);
             })) != hipSuccess)
            return device_fail(p, e, "reduce kernel");
    }
    return CHI0_OK;
}

}  // extern "C"

namespace {

// The dynamic call on a given workspace, at most qcap q-points per launch sequence (0: the
// plan's own); no_alloc: no profile events.
chi0_status dynamic_run(chi0_plan_t p, int32_t nq, const chi0_q *qs, int32_t nw, const double *omega, void *ws,
                        size_t ws_bytes, double *chi, int qcap, bool no_alloc)
{
    chi0_status st = begin_call(p);
    if (st) return st;
    st = check_qs(p, nq, qs);
    if (st) return st;
    if (nw < 1 || !omega || !chi) return fail(p, CHI0_E_INVALID_ARG, "nw >= 1, omega and chi non-null required");
    const int nwc_max = std::min(nw, kMaxOmegaPerLaunch);
    const Layout L = layout(p, nq, 2 * nwc_max, qcap, !no_alloc);
    if (!ws || ws_bytes < L.total) return fail(p, CHI0_E_WORKSPACE, "workspace too small");
    if ((st = enqueue_scan(p, nq, qs, omega, nw, scan_flag(ws, L))) != CHI0_OK) return st;
    const int nblk = n_blocks(p);
    double *partial = reinterpret_cast<double *>(static_cast<char *>(ws) + L.part_off);
    const double scale = prefactor(p);
    PackState pk = pack_state(ws, L);
    for (int q0 = 0; q0 < nq; q0 += L.qbatch) {
        const int nqb = std::min(L.qbatch, nq - q0);
        BatchDev B;
        fill_batch(p, qs, q0, nqb, ws, L, B);
        hipError_t e;
        if (!p->d.cma && (e = timed(p, 0, [&] {
                              return launch_contract(p->mesh, B, nqb, p->d.precision, &pk, p->stream);
                          }, no_alloc)) != hipSuccess)
            return device_fail(p, e, "matrix-element kernel");
        for (int w0 = 0; w0 < nw; w0 += kMaxOmegaPerLaunch) {
            const int nwc = std::min(kMaxOmegaPerLaunch, nw - w0);
            if ((e = timed(p, 1, [&] {
                     return launch_tetra_dynamic(p->mesh, B, nqb, nblk, omega + w0, nwc, partial, p->d.precision != 0,
                                                 p->stream);
                 }, no_alloc)) != hipSuccess)
                return device_fail(p, e, "tetrahedron kernel");
            if ((e = timed(p, 2, [&] {
                     return launch_reduce(partial, nqb, nblk, 2 * nwc, scale, chi + ((int64_t)q0 * nw + w0) * 2,
                                          (int64_t)nw * 2, p->stream);
                 }, no_alloc)) != hipSuccess)
                return device_fail(p, e, "reduce kernel");
        }
    }
    return CHI0_OK;
}

}  // namespace

namespace chi0 {

chi0_status dynamic_scratch(chi0_plan_t p, int32_t nq, const chi0_q *qs, int32_t nw, const double *omega,
                            void *scratch, size_t scratch_bytes, double *chi)
{
    if (!p) return CHI0_E_INVALID_ARG;
    if (nq < 1 || nw < 1) return fail(p, CHI0_E_INVALID_ARG, "nq and nw must be >= 1");
    const int nvals = 2 * std::min(nw, kMaxOmegaPerLaunch);
    int qcap = p->qbatch;
    while (qcap > 1 && layout(p, nq, nvals, qcap, false).total > scratch_bytes) --qcap;
    if (layout(p, nq, nvals, qcap, false).total > scratch_bytes)
        return fail(p, CHI0_E_WORKSPACE, "the no-allocation call's fixed scratch cannot hold the workspace of one q of "
                                         "this plan (use chi0_dynamic with a caller workspace)");
    return dynamic_run(p, nq, qs, nw, omega, scratch, scratch_bytes, chi, qcap, true);
}

chi0_status plan_device_error(chi0_plan_t p, hipError_t e, const char *where) { return device_fail(p, e, where); }

}  // namespace chi0

extern "C" {

chi0_status chi0_dynamic(chi0_plan_t p, int32_t nq, const chi0_q *qs, int32_t nw, const double *omega, void *ws,
                         size_t ws_bytes, double *chi)
{
    if (!p) return CHI0_E_INVALID_ARG;
    // the workspace chi0_workspace_size reports is exactly the layout of the plan's own batch
    return dynamic_run(p, nq, qs, nw, omega, ws, ws_bytes, chi, 0, false);
}

chi0_status chi0_dynamic_pairs_workspace_size(chi0_plan_t p, int32_t nq, int32_t nw, size_t *bytes)
{
    if (!p || !bytes) return CHI0_E_INVALID_ARG;
    if (nq < 1 || nw < 1) return fail(p, CHI0_E_INVALID_ARG, "nq and nw must be >= 1");
    *bytes = dpairs_layout(p, nq, 2 * std::min(nw, kMaxOmegaPerLaunch)).total;
    return CHI0_OK;
}

chi0_status chi0_dynamic_pairs(chi0_plan_t p, int32_t nq, const chi0_q *qs, int32_t nw, const double *omega,
                               void *ws, size_t ws_bytes, double *chi)
{
    if (!p) return CHI0_E_INVALID_ARG;
    chi0_status st = begin_call(p);
    if (st) return st;
    if (p->list) return fail(p, CHI0_E_UNSUPPORTED, "the pair-resolved dynamic call takes mesh plans");
    st = check_qs(p, nq, qs);
    if (st) return st;
    if (nw < 1 || !omega || !chi) return fail(p, CHI0_E_INVALID_ARG, "nw >= 1, omega and chi non-null required");
    const int nwc_max = std::min(nw, kMaxOmegaPerLaunch);
    const PairsLayout L = dpairs_layout(p, nq, 2 * nwc_max);
    if (!ws || ws_bytes < L.total) return fail(p, CHI0_E_WORKSPACE, "workspace too small");
    unsigned *flag = reinterpret_cast<unsigned *>(static_cast<char *>(ws) + L.flag_off);
    if ((st = enqueue_scan(p, nq, qs, omega, nw, flag)) != CHI0_OK) return st;
    const int npairs = p->mesh.nbw * p->mesh.nbw;
    double *partial = reinterpret_cast<double *>(static_cast<char *>(ws) + L.part_off);
    const double scale = prefactor(p);
    Layout Lw = {};   // W of the batch at the start of the workspace, as for chi0_dynamic
    Lw.w_off = L.w_off;
    Lw.w_bytes_per_q = L.w_bytes_per_q;
    Lw.rng_off = L.rng_off;
    Lw.rng_bytes = L.rng_bytes;
    PackState pk = {nullptr, false};
    for (int q0 = 0; q0 < nq; q0 += L.qbatch) {
        const int nqb = std::min(L.qbatch, nq - q0);
        BatchDev B;
        fill_batch(p, qs, q0, nqb, ws, Lw, B);
        hipError_t e;
        if (!p->d.cma && (e = timed(p, 0, [&] {
                              return launch_contract(p->mesh, B, nqb, p->d.precision, &pk, p->stream);
                          })) != hipSuccess)
            return device_fail(p, e, "matrix-element kernel");
        for (int w0 = 0; w0 < nw; w0 += kMaxOmegaPerLaunch) {
            const int nwc = std::min(kMaxOmegaPerLaunch, nw - w0);
            if ((e = timed(p, 1, [&] {
                     return launch_tetra_dynamic_pairs(p->mesh, B, nqb, L.nblk, omega + w0, nwc, partial,
                                                       p->d.precision != 0, p->stream);
                 })) != hipSuccess)
                return device_fail(p, e, "tetrahedron kernel");
            // groups (q, pair) in order: out[((q0 + q) npairs + pair) nw + w][2]
            if ((e = timed(p, 2, [&] {
                     return launch_reduce(partial, nqb * npairs, L.nblk, 2 * nwc, scale,
                                          chi + ((int64_t)q0 * npairs * nw + w0) * 2, (int64_t)nw * 2, p->stream);
                 })) != hipSuccess)
                return device_fail(p, e, "reduce kernel");
        }
    }
    return CHI0_OK;
}

chi0_status chi0_kk_workspace_size(chi0_plan_t p, int32_t nq, int32_t nw, int32_t n_spec, size_t *bytes)
{
    if (!p || !bytes) return CHI0_E_INVALID_ARG;
    if (nq < 1 || nw < 1 || n_spec < 2) return fail(p, CHI0_E_INVALID_ARG, "nq, nw >= 1 and n_spec >= 2 required");
    if ((int64_t)nw + n_spec > (int64_t)INT32_MAX / 4) return fail(p, CHI0_E_SHAPE, "too many frequencies");
    *bytes = kk_layout(p, nq, nw, n_spec).total;
    return CHI0_OK;
}

chi0_status chi0_dynamic_kk(chi0_plan_t p, int32_t nq, const chi0_q *qs, int32_t nw, const double *omega,
                            int32_t n_spec, double spec_lo, double spec_hi, void *ws, size_t ws_bytes, double *chi)
{
    if (!p) return CHI0_E_INVALID_ARG;
    chi0_status st = begin_call(p);
    if (st) return st;
    st = check_qs(p, nq, qs);
    if (st) return st;
    if (nw < 1 || !omega || !chi || n_spec < 2)
        return fail(p, CHI0_E_INVALID_ARG, "nw >= 1, n_spec >= 2, omega and chi non-null required");
    if (!std::isfinite(spec_lo) || !std::isfinite(spec_hi)) return fail(p, CHI0_E_NONFINITE, "spectral range");
    if (!(spec_hi > spec_lo)) return fail(p, CHI0_E_INVALID_ARG, "spec_hi must exceed spec_lo");
    size_t need = 0;
    if ((st = chi0_kk_workspace_size(p, nq, nw, n_spec, &need)) != CHI0_OK) return st;
    const KKLayout L = kk_layout(p, nq, nw, n_spec);
    if (!ws || ws_bytes < need) return fail(p, CHI0_E_WORKSPACE, "workspace too small");
    char *base = static_cast<char *>(ws);
    if ((st = enqueue_scan(p, nq, qs, omega, nw, reinterpret_cast<unsigned *>(base + L.flag_off))) != CHI0_OK)
        return st;
    double *partial = reinterpret_cast<double *>(base + L.part_off);
    double *om_all = reinterpret_cast<double *>(base + L.om_off);
    double *im_all = reinterpret_cast<double *>(base + L.im_off);
    const double h = (spec_hi - spec_lo) / (double)(n_spec - 1);
    const int nblk = n_blocks(p);
    const double scale = prefactor(p);
    hipError_t e = launch_kk_grid(spec_lo, h, n_spec, omega, nw, om_all, p->stream);
    if (e != hipSuccess) return device_fail(p, e, "frequency grid kernel");
    Layout Lw = {};   // W of the batch sits at the start of the workspace, as for chi0_dynamic
    Lw.w_off = L.w_off;
    Lw.w_bytes_per_q = L.w_bytes_per_q;
    Lw.rng_off = L.rng_off;
    Lw.rng_bytes = L.rng_bytes;
    PackState pk = pack_state(ws, Lw);
    for (int q0 = 0; q0 < nq; q0 += L.qbatch) {
        const int nqb = std::min(L.qbatch, nq - q0);
        BatchDev B;
        fill_batch(p, qs, q0, nqb, ws, Lw, B);
        if (!p->d.cma && (e = timed(p, 0, [&] {
                              return launch_contract(p->mesh, B, nqb, p->d.precision, &pk, p->stream);
                          })) != hipSuccess)
            return device_fail(p, e, "matrix-element kernel");
        for (int w0 = 0; w0 < L.n_all; w0 += kMaxOmegaIm) {
            const int nwc = std::min(kMaxOmegaIm, L.n_all - w0);
            if ((e = timed(p, 1, [&] {
                     return launch_tetra_im(p->mesh, B, nqb, nblk, om_all + w0, nwc, partial, p->stream);
                 })) != hipSuccess)
                return device_fail(p, e, "imaginary-part kernel");
            if ((e = timed(p, 2, [&] {
                     return launch_reduce(partial, nqb, nblk, 2 * nwc, scale, im_all + 2 * (int64_t)w0,
                                          2 * (int64_t)L.n_all, p->stream);
                 })) != hipSuccess)
                return device_fail(p, e, "reduce kernel");
        }
        if ((e = launch_kk_transform(im_all, nqb, n_spec, nw, spec_lo, h, omega, chi + (int64_t)q0 * nw * 2,
                                     2 * (int64_t)nw, p->stream)) != hipSuccess)
            return device_fail(p, e, "Kramers-Kronig kernel");
    }
    return CHI0_OK;
}

chi0_status chi0_static_group(chi0_plan_t p, int32_t nq, int32_t n_group, const chi0_q *qs, void *ws,
                              size_t ws_bytes, double *chi)
{
    if (!p) return CHI0_E_INVALID_ARG;
    if (nq < 1 || n_group < 1 || (int64_t)nq * n_group >= (int64_t(1) << 31))
        return fail(p, CHI0_E_INVALID_ARG, "nq and n_group must be >= 1");
    const int ne = nq * n_group;
    chi0_status st = begin_call(p);
    if (st) return st;
    st = check_qs(p, ne, qs);
    if (st) return st;
    if (!chi) return fail(p, CHI0_E_INVALID_ARG, "chi is null");
    const Layout L = layout(p, ne, 1);
    if (!ws || ws_bytes < L.total) return fail(p, CHI0_E_WORKSPACE, "workspace too small");
    if ((st = enqueue_scan(p, ne, qs, nullptr, 0, scan_flag(ws, L))) != CHI0_OK) return st;
    const int nblk = n_blocks(p);
    double *partial = reinterpret_cast<double *>(static_cast<char *>(ws) + L.part_off);
    const double scale = prefactor(p);
    PackState pk = pack_state(ws, L);
    for (const GroupLaunch &G : group_launches(nq, n_group, p->qbatch)) {
        BatchDev B;
        fill_batch(p, qs, G.e0, G.ne, ws, L, B);
        const int per_group = G.ne / G.ng;
        hipError_t e;
        if (!p->d.cma && (e = timed(p, 0, [&] {
                              return launch_contract(p->mesh, B, G.ne, p->d.precision, &pk, p->stream);
                          })) != hipSuccess)
            return device_fail(p, e, "matrix-element kernel");
        if ((e = timed(p, 1, [&] { return launch_tetra_static(p->mesh, B, G.ne, nblk, partial, p->stream); })) !=
            hipSuccess)
            return device_fail(p, e, "tetrahedron kernel");
        if ((e = timed(p, 2, [&] {
                 return launch_reduce(partial, G.ng, per_group * nblk, 1, scale, chi + G.g0, 1, p->stream,
                                      G.accumulate);
             })) != hipSuccess)
            return device_fail(p, e, "reduce kernel");
    }
    return CHI0_OK;
}

chi0_status chi0_dynamic_group(chi0_plan_t p, int32_t nq, int32_t n_group, const chi0_q *qs, int32_t nw,
                               const double *omega, void *ws, size_t ws_bytes, double *chi)
{
    if (!p) return CHI0_E_INVALID_ARG;
    if (nq < 1 || n_group < 1 || (int64_t)nq * n_group >= (int64_t(1) << 31))
        return fail(p, CHI0_E_INVALID_ARG, "nq and n_group must be >= 1");
    const int ne = nq * n_group;
    chi0_status st = begin_call(p);
    if (st) return st;
    st = check_qs(p, ne, qs);
    if (st) return st;
    if (nw < 1 || !omega || !chi) return fail(p, CHI0_E_INVALID_ARG, "nw >= 1, omega and chi non-null required");
    const int nwc_max = std::min(nw, kMaxOmegaPerLaunch);
    const Layout L = layout(p, ne, 2 * nwc_max);
    if (!ws || ws_bytes < L.total) return fail(p, CHI0_E_WORKSPACE, "workspace too small");
    if ((st = enqueue_scan(p, ne, qs, omega, nw, scan_flag(ws, L))) != CHI0_OK) return st;
    const int nblk = n_blocks(p);
    double *partial = reinterpret_cast<double *>(static_cast<char *>(ws) + L.part_off);
    const double scale = prefactor(p);
    PackState pk = pack_state(ws, L);
    for (const GroupLaunch &G : group_launches(nq, n_group, p->qbatch)) {
        BatchDev B;
        fill_batch(p, qs, G.e0, G.ne, ws, L, B);
        const int per_group = G.ne / G.ng;
        hipError_t e;
        if (!p->d.cma && (e = timed(p, 0, [&] {
                              return launch_contract(p->mesh, B, G.ne, p->d.precision, &pk, p->stream);
                          })) != hipSuccess)
            return device_fail(p, e, "matrix-element kernel");
        for (int w0 = 0; w0 < nw; w0 += kMaxOmegaPerLaunch) {
            const int nwc = std::min(kMaxOmegaPerLaunch, nw - w0);
            if ((e = timed(p, 1, [&] {
                     return launch_tetra_dynamic(p->mesh, B, G.ne, nblk, omega + w0, nwc, partial, p->d.precision != 0,
                                                 p->stream);
                 })) != hipSuccess)
                return device_fail(p, e, "tetrahedron kernel");
            if ((e = timed(p, 2, [&] {
                     return launch_reduce(partial, G.ng, per_group * nblk, 2 * nwc, scale,
                                          chi + ((int64_t)G.g0 * nw + w0) * 2, (int64_t)nw * 2, p->stream,
                                          G.accumulate);
                 })) != hipSuccess)
                return device_fail(p, e, "reduce kernel");
        }
    }
    return CHI0_OK;
}

chi0_status chi0_matrix_elements(chi0_plan_t p, const chi0_q *q, double *W)
{
    if (!p) return CHI0_E_INVALID_ARG;
    if (p->d.cma) return fail(p, CHI0_E_UNSUPPORTED, "no matrix elements under cma");
    chi0_status st = begin_call(p);
    if (st) return st;
    st = check_qs(p, 1, q);
    if (st) return st;
    if (!W) return fail(p, CHI0_E_INVALID_ARG, "W is null");
    Layout L = {};    // W itself is the W region of q 0 (no other region)
    L.w_bytes_per_q = layout(p, 1, 1).w_bytes_per_q;
    BatchDev B;
    fill_batch(p, q, 0, 1, W, L, B);
    hipError_t e = launch_contract(p->mesh, B, 1, p->d.precision, nullptr, p->stream);
    if (e != hipSuccess) return device_fail(p, e, "matrix-element kernel");
    return CHI0_OK;
}

}  // extern "C"
