/*
 * chi0.h -- C ABI of libchi0, the MI355X (gfx950) library for the bare
 * (Lindhard) susceptibility chi0(q, omega) by the linear tetrahedron method
 * with double occupation carving (Heil et al., arXiv:1407.3444, Sec. II).
 *
 * What one call computes (Sec. II, Eqs. (1)-(3), carving condition Eq. (4)):
 *
 *   chi0(q,w) = g_s/(6 Nk) sum_T sum_{n,m in [band_lo, band_hi)}
 *               (1/|T|) int_T W_nm(k) [f(e) - f(e')] / (w - (e' - e) + i0) dk
 *
 * e = eps_n(k), e' = eps_m(k+q), W_nm(k) = |sum_o conj(c_{o,n}(k)) c_{o,m}(k+q)|^2
 * (the tight-binding matrix element of the footnote in Sec. III; W = 1 under the
 * constant matrix-element approximation), all three interpolated linearly on
 * each of the 6 tetrahedra of every mesh cell.  T = 0, f = step function at mu.
 * Each tetrahedron is carved twice -- first by e = mu, then by e' = mu -- and
 * only the final tetrahedra where the product of occupation factors is one
 * are integrated, analytically.  The result is the retarded response (+i0),
 * per unit cell, in states per energy unit: Re chi0(q -> 0, 0) = -N(E_F).
 *
 * Conventions shared by every entry point
 *   * Mesh: Gamma-centred N1 x N2 x N3, k = (i1/N1, i2/N2, i3/N3) in fractional
 *     reciprocal coordinates, flat index k = (i1*N2 + i2)*N3 + i3.  Cell (i1,i2,i3)
 *     holds the tetrahedra {c, c+e_p0, c+e_p0+e_p1, c+(1,1,1)} for the six axis
 *     permutations (p0,p1,p2); indices wrap periodically.
 *   * Band energies: float64, band-major [n_bands][Nk].
 *   * Eigenvectors: complex128 as interleaved (re, im) float64, [Nk][n_orb][n_bands];
 *     entry (k, o, n) is orbital o of the eigenvector of band n at k.
 *   * All array pointers passed to the library are DEVICE pointers (HIP), except
 *     the chi0_desc and chi0_q structures themselves, which live in host memory.
 *   * The caller owns all device memory, inputs, workspace and outputs.  The
 *     library allocates no device memory.  Inputs must stay valid and unmodified
 *     until the stream work that reads them has completed.
 *   * Work is enqueued on the HIP stream given to chi0_plan and runs
 *     asynchronously; outputs are valid once that stream has been synchronised.
 *   * Errors: every call returns a chi0_status; descriptor and argument checks are
 *     done on the host before anything is enqueued.  A failure reported by the HIP
 *     runtime is returned as CHI0_E_DEVICE.  No exception crosses the ABI.
 *   * Content checks (Sec. II takes band energies and normalised eigenvectors as inputs): unless
 *     the descriptor sets skip_input_scan, every computing call of a plan first enqueues a scan
 *     of the device arrays it reads -- eps_k, c_k, the explicit k+q arrays of its q-points and
 *     omega -- for non-finite values and for eigenvectors whose squared norm
 *     sum_o |c_{o,n}(k)|^2 differs from 1 by more than 1e-6.  The scan runs on the stream
 *     ahead of the computation and does not stop it; its verdict is reported asynchronously:
 *     by the plan's next call once the scan has completed (that call then returns
 *     CHI0_E_NONFINITE or CHI0_E_NOT_NORMALIZED and enqueues nothing), or by chi0_sync.  The
 *     outputs of a call whose scan failed are not meaningful.  chi0_matrix_elements and the
 *     batched form do not scan.
 *   * A plan is not thread safe: use one plan per host thread.
 *   * If a final tetrahedron has a whole face on which e' - e equals w (e.g. an
 *     exactly nested tetrahedron at w = 0), the integral diverges and the output
 *     for that (q, w) is not finite.
 */
#ifndef CHI0_H
#define CHI0_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum chi0_status {
    CHI0_OK = 0,
    CHI0_E_INVALID_ARG = -1,   /* null pointer, bad enum value, a count below its minimum (an empty q
                                  list or frequency grid included): nothing is enqueued */
    CHI0_E_SHAPE = -2,         /* mesh, band, orbital or window sizes out of range */
    CHI0_E_NONFINITE = -3,     /* host values (mu, the spin factor, the degeneracy tolerances, q_frac,
                                  a spectral range) not finite; or, from the device scan, a
                                  non-finite band energy, eigenvector coefficient or frequency */
    CHI0_E_NOT_COMMENSURATE = -4, /* a q given by q_frac alone (explicit_kq = 2) is not a mesh vector */
    CHI0_E_WORKSPACE = -5,     /* workspace null or smaller than chi0_workspace_size */
    CHI0_E_DEVICE = -6,        /* the HIP runtime reported an error */
    CHI0_E_UNSUPPORTED = -7,   /* valid request outside what this build implements */
    CHI0_E_NOT_NORMALIZED = -8 /* device scan: an eigenvector's squared norm differs from 1 by more
                                  than 1e-6 */
} chi0_status;

/* Problem description, copied by chi0_plan. */
typedef struct chi0_desc {
    int32_t nk[3];          /* mesh N1, N2, N3 (each >= 1, Nk < 2^31) */
    int32_t n_bands;        /* bands stored in the energy/eigenvector arrays (1..64) */
    int32_t n_orb;          /* basis functions per eigenvector: orbitals (1..64), or up to 16384
                               plane waves (a basis above 64 takes the plane-wave MFMA contraction,
                               one wave per q sharing the k operand, in the precision below);
                               ignored under cma */
    int32_t band_lo;        /* first band of the summation window (Sec. III band truncation) */
    int32_t band_hi;        /* one past the last band; <= 0 means n_bands; window <= 32 bands */
    int32_t cma;            /* 1: constant matrix elements W = 1 (Sec. III), eigenvectors unused */
    int32_t form;           /* 0: occupation difference f(e)-f(e') (regions e<mu<e' minus e'<mu<e);
                               1: the paper's Eq. (1)/(2): region e<mu<e' only, with
                                  1/(w-D+i0) - 1/(w+D+i0)  (equal to form 0 under time reversal) */
    int32_t precision;      /* 0: FP64 everywhere.
                               1: mixed: matrix elements from BF16 MFMA with hi+lo split operands
                                  and FP32 accumulation (orbital and plane-wave bases alike); dynamic weights of final tetrahedra in
                                  FP32 (far series and near branch), except that near-degenerate
                                  final tetrahedra (degen_tol_ev, degen_rel_tol below) keep the
                                  FP64 near branch; carving, differences of energies and the chi0
                                  accumulation stay FP64.
                               2: as 1 with FP16 (low part scaled by 2^11) instead of BF16. */
    int32_t batch_hint;     /* q-points per launch sequence, 1..16 (0 = 16): the workspace holds the
                               matrix elements and partial sums of that many q at once, so a
                               smaller value trades launches for memory */
    int32_t skip_input_scan; /* 0: scan the device inputs of every call (see Content checks);
                               1: do not scan */
    int32_t reserved[3];    /* must be zero */
    double mu;              /* Fermi level (energy units of the band arrays) */
    double spin_factor;     /* g_s, 2 for spin-degenerate bands */
    double degen_tol_ev;    /* mixed form: a final tetrahedron whose sorted corner values of e'-e
                               have two neighbours closer than max(degen_tol_ev, degen_rel_tol x
                               their span) is near-degenerate and keeps the FP64 near branch.
                               Energy units of the band arrays; >= 0, 0 selects 1e-6 */
    double degen_rel_tol;   /* the relative part of the rule above, >= 0 (0: absolute rule only) */
} chi0_desc;

/* One q.  Either an integer mesh shift (k+q data = mesh data at (i + shift) mod N),
 * or explicit band data at k+q for every mesh point k. */
typedef struct chi0_q {
    int32_t shift[3];       /* used when explicit_kq == 0 */
    int32_t explicit_kq;    /* 0: mesh shift `shift`;
                               1: eps_kq / c_kq below hold the k+q data;
                               2: mesh shift derived from q_frac: q_frac[a] * N_a must be an integer
                                  to 1e-9 relative (else CHI0_E_NOT_COMMENSURATE) */
    const double *eps_kq;   /* device [n_bands][Nk] float64, energies at k+q */
    const double *c_kq;     /* device [Nk][n_orb][n_bands] complex128 (re,im), eigenvectors at
                               k+q; may be NULL under cma */
    double q_frac[3];       /* q in fractional reciprocal coordinates: defines the shift when
                               explicit_kq = 2, informational otherwise (not read) */
} chi0_q;

typedef struct chi0_plan_s *chi0_plan_t;

/* Create a plan.  eps_k: device [n_bands][Nk]; c_k: device [Nk][n_orb][n_bands] complex128,
 * may be NULL under cma.  hip_stream: a hipStream_t (NULL = default stream).  On success
 * *out receives the plan, which borrows eps_k and c_k. */
chi0_status chi0_plan(chi0_plan_t *out, const chi0_desc *desc, const double *eps_k,
                      const double *c_k, void *hip_stream);

/* Device workspace (bytes) needed by chi0_static / chi0_dynamic for nq q-points and nw
 * frequencies (nw = 1 for the static call).  It holds the matrix elements and partial sums of
 * the q of one launch sequence (batch_hint) and, for a split-precision plan with a basis above 64
 * whose launches take 3 or more q, the eigenvectors of the band window split once into 16-bit
 * high and low parts (8 bytes per coefficient): launches whose q are all mesh shifts read those
 * instead of the FP64 coefficients.  It also holds each window band's energy range over the
 * k-points (e(k) and every e(k+q) of a launch), from which the tetrahedron kernels skip the band
 * pairs that have no carved region anywhere (no change to any result). */
chi0_status chi0_workspace_size(chi0_plan_t plan, int32_t nq, int32_t nw, size_t *bytes);

/* Static chi0(q, 0) (Sec. III uses Eq. (1) at w = 0, where Im vanishes).
 * qs: host array of nq chi0_q; chi: device float64 [nq] receives Re chi0(q, 0). */
chi0_status chi0_static(chi0_plan_t plan, int32_t nq, const chi0_q *qs, void *workspace,
                        size_t workspace_bytes, double *chi);

/* Static chi0(q, 0) resolved by band pair (the band-transition histogram of Sec. III, Fig. 8):
 * chi: device float64 [nq][nbw][nbw]; entry (q, n, m), n and m relative to band_lo, holds the
 * terms of band n at k and band m at k+q, so the sum over (n, m) is chi0_static's result.
 * Workspace as for chi0_static (chi0_workspace_size with nw = 1). */
chi0_status chi0_static_pairs(chi0_plan_t plan, int32_t nq, const chi0_q *qs, void *workspace,
                              size_t workspace_bytes, double *chi);

/* Dynamic chi0(q, w) on a frequency grid (Sec. IV; Re by the analytic tetrahedron formula,
 * Im by the tetrahedron delta weights, both exact for the linear interpolant).
 * omega: device float64 [nw] (any real values, any order); chi: device float64
 * [nq][nw][2] receives (Re, Im). */
chi0_status chi0_dynamic(chi0_plan_t plan, int32_t nq, const chi0_q *qs, int32_t nw,
                         const double *omega, void *workspace, size_t workspace_bytes,
                         double *chi);

/* Dynamic chi0(q, w) resolved by band pair (the per-pair analysis of Sec. III at every
 * frequency): chi: device float64 [nq][nbw][nbw][nw][2]; entry (q, n, m, w) holds the terms of
 * band n at k and band m at k+q, so the sum over (n, m) is chi0_dynamic's result (to the rounding
 * of the different summation order).  Each band pair's units are evaluated by workgroups of their
 * own.  Mesh plans only (a tetrahedron-list plan returns CHI0_E_UNSUPPORTED).  The workspace is
 * given by chi0_dynamic_pairs_workspace_size: the matrix elements of one q batch and up to
 * min(64 nbw^2, 8192) partial sums per q and frequency. */
chi0_status chi0_dynamic_pairs(chi0_plan_t plan, int32_t nq, const chi0_q *qs, int32_t nw,
                               const double *omega, void *workspace, size_t workspace_bytes, double *chi);

/* Device workspace (bytes) of chi0_dynamic_pairs for nq q-points and nw frequencies. */
chi0_status chi0_dynamic_pairs_workspace_size(chi0_plan_t plan, int32_t nq, int32_t nw, size_t *bytes);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): chi0_dynamic with its workspace in a fixed device array
 * of the library, 128 MiB per device (held from the first call on a device until the process
 * ends), instead of a caller buffer.  Arguments and results as for chi0_dynamic.  Each launch
 * sequence takes as many q-points as the array holds (at most the plan's batch_hint); a plan whose
 * workspace for a single q exceeds 128 MiB is rejected with CHI0_E_WORKSPACE.  Allocates nothing
 * (no device or pinned memory, no profile events even while profiling is enabled).  Every call on
 * a device shares that device's array: calls that overlap on one device (any plans, any streams)
 * race, so they must be serialised by the caller. */
chi0_status chi0_dynamic_noalloc(chi0_plan_t plan, int32_t nq, const chi0_q *qs, int32_t nw,
                                 const double *omega, double *chi);

/* The Kramers-Kronig route (Sec. II: the common practice is to compute Im chi0 alone and to
 * recover Re chi0 by a Kramers-Kronig transform, which needs a frequency grid over the whole
 * spectrum).
 * Im chi0 is computed exactly (tetrahedron delta weights, no logarithms) at the requested
 * frequencies omega (device float64 [nw]) and on the uniform spectral grid
 * w'_k = spec_lo + k (spec_hi - spec_lo)/(n_spec - 1), k < n_spec; Re chi0 at omega is the exact
 * principal-value transform (1/pi) P int Im(w')/(w' - w) dw' of the piecewise-linear interpolant
 * of Im on that grid (taken as zero one spacing beyond each end), so it approximates the analytic
 * Re to the accuracy of that interpolant: the grid must cover every e' - e of the band window.
 * chi: device float64 [nq][nw][2] receives (Re, Im).  Workspace: chi0_kk_workspace_size. */
chi0_status chi0_kk_workspace_size(chi0_plan_t plan, int32_t nq, int32_t nw, int32_t n_spec, size_t *bytes);
chi0_status chi0_dynamic_kk(chi0_plan_t plan, int32_t nq, const chi0_q *qs, int32_t nw, const double *omega,
                            int32_t n_spec, double spec_lo, double spec_hi, void *workspace,
                            size_t workspace_bytes, double *chi);

/* Matrix elements of one q, the weights the tetrahedron integration interpolates:
 * W[(n*nbw + m)*Nk + k] = |sum_o conj(c_{o,n}(k)) c_{o,m}(k+q)|^2 (footnote of Sec. III),
 * n, m relative to band_lo, nbw = band_hi - band_lo.  W: device float64 [nbw][nbw][Nk].
 * CHI0_E_UNSUPPORTED under cma. */
chi0_status chi0_matrix_elements(chi0_plan_t plan, const chi0_q *q, double *W);

/* ------------------------------------------------------------------------------------------
 * Irreducible wedge and point-group loop (Sec. II).  The paper integrates over the irreducible
 * wedge (IW) of the zone decomposed into tetrahedra and repeats the second carving for every
 * point-group element g of the crystal.  For bands and matrix elements invariant under the group,
 * the zone integral at q equals the sum over g of the wedge integral with the k+q data taken at
 * k + g^-1 q.  A list plan integrates over an explicit tetrahedron list (the wedge); the group
 * calls sum the results of groups of q-entries (one entry per g) inside the reduction kernel.
 * ------------------------------------------------------------------------------------------ */

/* An explicit set of tetrahedra replacing the mesh's Kuhn tetrahedra. */
typedef struct chi0_tetra_list {
    int64_t n_kp;           /* k-points of the band arrays: eps_k [n_bands][n_kp] and c_k
                               [n_kp][n_orb][n_bands]; 1 <= n_kp < 2^31 */
    int64_t n_tet;          /* tetrahedra, 1 <= n_tet < 2^31 */
    const int32_t *tets;    /* device int32 [n_tet][4], 16-byte aligned: the corner k-point
                               indices of every tetrahedron; chi0_plan_list copies them to the
                               host once and rejects any index outside [0, n_kp) (CHI0_E_SHAPE) */
    double volume;          /* fraction of the zone one tetrahedron covers (> 0); the result is
                               spin_factor * volume * (sum over tetrahedra), so 1/(6 N1 N2 N3)
                               for tetrahedra of an N1 x N2 x N3 mesh */
} chi0_tetra_list;

/* Create a plan over a tetrahedron list.  desc as for chi0_plan except that desc->nk is not used;
 * eps_k: device [n_bands][n_kp]; c_k: device [n_kp][n_orb][n_bands] complex128 (NULL under cma).
 * Every q given to this plan must be explicit (explicit_kq = 1, eps_kq [n_bands][n_kp] and c_kq
 * [n_kp][n_orb][n_bands] at the list's k-points shifted by q); a mesh shift is rejected with
 * CHI0_E_INVALID_ARG.  All calls of a mesh plan are available except the batched form.  The
 * plan borrows list->tets as it borrows eps_k and c_k.  Synchronises the stream once (the index
 * check). */
chi0_status chi0_plan_list(chi0_plan_t *out, const chi0_desc *desc, const chi0_tetra_list *list,
                           const double *eps_k, const double *c_k, void *hip_stream);

/* Group sums (the point-group loop): qs holds nq * n_group entries, group i being entries
 * i * n_group .. i * n_group + n_group - 1 (one per point-group element, each with its k+q data);
 * chi receives, per group, the sum of the group's chi0 values: device float64 [nq] (static) or
 * [nq][nw][2] (dynamic).  Each group is summed in entry order inside the reduction kernel (groups
 * of more than 16 entries over several launches, each added to the previous total).  Workspace:
 * chi0_workspace_size(plan, nq * n_group, nw). */
chi0_status chi0_static_group(chi0_plan_t plan, int32_t nq, int32_t n_group, const chi0_q *qs, void *workspace,
                              size_t workspace_bytes, double *chi);
chi0_status chi0_dynamic_group(chi0_plan_t plan, int32_t nq, int32_t n_group, const chi0_q *qs, int32_t nw,
                               const double *omega, void *workspace, size_t workspace_bytes, double *chi);

/* The irreducible wedge 0 <= z <= y <= x <= 1/2 (fractional coordinates) of a Gamma-centred
 * n x n x n simple-cubic mesh (n even, 2..1024) under the 48-element cubic group O_h, as
 * tetrahedra: every mesh cube i >= j >= l >= 0 in the wedge split into the six tetrahedra of the
 * three axis orders from its corner (0,0,0) to (1,1,1), keeping those inside the wedge (Fig. 1(a)).
 * Host memory.  *n_kp receives the (n/2+1)(n/2+2)(n/2+3)/6 wedge points, *n_tet the (n/2)^3
 * tetrahedra, *volume 1/(6 n^3); when non-NULL, kfrac [n_kp][3] receives the points, tets
 * [n_tet][4] the corner indices and ops [48][3][3] the group's integer matrices acting on
 * fractional coordinates (signed permutations, identity first).  Call first with NULL arrays for
 * the sizes. */
chi0_status chi0_iw_cubic(int32_t n, int64_t *n_kp, int64_t *n_tet, double *volume, double *kfrac,
                          int32_t *tets, int32_t *ops);

/* Wait for the plan's stream and report the verdict of every input scan enqueued since the last
 * report (see Content checks): CHI0_OK, CHI0_E_NONFINITE or CHI0_E_NOT_NORMALIZED (chi0_last_error
 * names the input), or CHI0_E_DEVICE if the stream failed. */
chi0_status chi0_sync(chi0_plan_t plan);

/* Kernel timing of the plan's launches, measured with HIP events on the plan's stream
 * while profiling is enabled.  Index 0: matrix-element kernel, 1: tetrahedron kernel,
 * 2: reduction kernel. */
typedef struct chi0_profile {
    double ms[3];           /* summed kernel time in milliseconds */
    int64_t launches[3];    /* number of launches */
} chi0_profile;

/* Start (enable = 1) or stop (0) recording events around every launch of this plan. */
chi0_status chi0_profile_enable(chi0_plan_t plan, int32_t enable);

/* Wait for the recorded events, return the sums since the last read (host struct) and reset. */
chi0_status chi0_profile_read(chi0_plan_t plan, chi0_profile *out);

/* Work census of chi0_dynamic(plan, nq, qs, nw, omega) (diagnostic): the same evaluation with
 * counters, its result discarded.  counts (host uint64 [7]) receives the number of (tetrahedron,
 * band pair, q) units whose carved region is non-empty, the number of final tetrahedra, the
 * number of (final tetrahedron, frequency) evaluations taking the near branch, the number of
 * far-branch series evaluations (one per final tetrahedron and frequency, or one per list of up
 * to 32 final tetrahedra and frequency where every frequency is far from the whole list and the
 * list's series are summed into one), the series terms summed over those evaluations (each cut
 * to the terms its distance from the frequencies needs), and the near evaluations that the FP64
 * form repeats in full because a divided-difference entry's nodes cluster (its first pass skips
 * every entry's Taylor series), and the far-series coefficients computed for the final
 * tetrahedra (only the blocks of terms their series class, or their list's, reads).  Uses the
 * same workspace as chi0_dynamic and synchronises the stream. */
chi0_status chi0_census(chi0_plan_t plan, int32_t nq, const chi0_q *qs, int32_t nw,
                        const double *omega, void *workspace, size_t workspace_bytes,
                        uint64_t *counts);

/* ------------------------------------------------------------------------------------------
 * Batched form: many independent instances (each a plan-like problem with its own mesh, bands,
 * q-list and frequency grid) run as one fused sequence of three launches -- matrix elements,
 * tetrahedron weights, reduction -- over a flat table of (instance, q, frequency-chunk) items,
 * optionally captured once into a HIP graph and replayed.  Each item computes exactly what
 * chi0_dynamic computes for that instance and q (same kernels, same summation order for a given
 * number of workgroups per item), so the batched result equals the per-instance calls to
 * rounding of the block partition.
 * ------------------------------------------------------------------------------------------ */

typedef struct chi0_instance {
    chi0_desc desc;         /* as for chi0_plan (validated the same way) */
    const double *eps_k;    /* device [n_bands][Nk] float64 */
    const double *c_k;      /* device [Nk][n_orb][n_bands] complex128; NULL under cma */
    int32_t nq;             /* q-points of this instance, >= 1 */
    int32_t nw;             /* frequencies, >= 1 (static problems: nw = 1, omega = {0}) */
    const chi0_q *qs;       /* host [nq]; copied by chi0_batch_create */
    const double *omega;    /* device [nw] float64 */
    double *chi;            /* device [nq][nw][2] float64 output (Re, Im) */
} chi0_instance;

typedef struct chi0_batch_opts {
    int64_t workgroups;     /* tetrahedron-kernel workgroups of the whole batch, spread over the
                               items in proportion to their estimated cost (each item gets
                               1..1024 and at most one per 64 units); 0 = 32768.  The workspace
                               is sized for this value and both frequency tiles;
                               chi0_batch_tune only tries smaller counts. */
    uint64_t stage_w_bytes; /* most bytes of matrix elements W resident at once: (instance, q)
                               groups are run in stages whose W fits (a group larger than the
                               limit runs alone); 0 = one stage */
    int32_t use_graph;      /* 1: capture the launch sequence into a HIP graph on the first run
                               and replay it afterwards; 0: launch directly every run */
    int32_t reserved[5];    /* must be zero */
} chi0_batch_opts;

typedef struct chi0_batch_s *chi0_batch_t;

/* Device workspace (bytes) a batch of n_inst instances needs (opts may be NULL = defaults). */
chi0_status chi0_batch_workspace_size(int32_t n_inst, const chi0_instance *inst,
                                      const chi0_batch_opts *opts, size_t *bytes);

/* Validate the instances, schedule the items and write the item tables into the workspace
 * (a synchronous upload on hip_stream).  The batch borrows every device pointer of every
 * instance and the workspace; they must stay valid while the batch exists.  Nothing is
 * computed until chi0_batch_run. */
chi0_status chi0_batch_create(chi0_batch_t *out, int32_t n_inst, const chi0_instance *inst,
                              const chi0_batch_opts *opts, void *workspace, size_t workspace_bytes,
                              void *hip_stream);

/* Compute chi0 of every instance into its chi array, asynchronously on hip_stream (NULL = the
 * default stream).  Runs that overlap on different streams race on the workspace. */
chi0_status chi0_batch_run(chi0_batch_t batch, void *hip_stream);

/* Autotune the schedule: after one warm-up run, time reps runs for every combination of the
 * tetrahedron-kernel workgroup count (the one the batch was created with, and 1/2, 1/4, 1/8 of
 * it, not below one per item) and the frequency tile of an item (512 or 256 frequencies: 8 or 4
 * frequencies per lane), keep the fastest (synchronises hip_stream; leaves valid results in the
 * outputs).  *chosen (may be NULL) receives the workgroup count; chi0_batch_info_get the tile. */
chi0_status chi0_batch_tune(chi0_batch_t batch, void *hip_stream, int32_t reps, int64_t *chosen);

/* Schedule summary of a batch (host struct). */
typedef struct chi0_batch_info {
    int64_t items;          /* (instance, q, frequency chunk) items */
    int64_t stages;         /* W-budget stages (launch triples) */
    int64_t workgroups[3];  /* workgroups of the matrix-element, tetrahedron and reduction
                               launches, summed over stages */
    int64_t nominal_units;  /* sum over instances of nq * 6 Nk * nbw^2 * nw */
    int64_t omega_tile;     /* most frequencies of one item (512 unless the tuner chose 256) */
} chi0_batch_info;

chi0_status chi0_batch_info_get(chi0_batch_t batch, chi0_batch_info *info);

/* Release a batch (host memory and its graph, if any).  NULL is accepted. */
chi0_status chi0_batch_destroy(chi0_batch_t batch);

/* Text of the last error recorded on this batch ("" if none). */
const char *chi0_batch_last_error(chi0_batch_t batch);

/* Release a plan (host memory only).  NULL is accepted. */
chi0_status chi0_destroy(chi0_plan_t plan);

/* Static description of a status code. */
const char *chi0_status_string(chi0_status status);

/* Text of the last error recorded on this plan ("" if none). */
const char *chi0_last_error(chi0_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* CHI0_H */
