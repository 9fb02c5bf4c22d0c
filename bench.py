"""Benchmark of the chi0 hot path on one MI355X.

Default workload (the precision-study configuration of the 10-orbital model): the
seeded two-site tetragonal tight-binding model (10 d-like orbitals, seed 2) on a
64 x 64 x 8 mesh (196,608 tetrahedra), all 100 band pairs, 64 q at the arc-length
midpoints of Gamma-X-M-Gamma (explicit k+q eigenpairs), 512 frequencies on [0, 2] eV,
dynamic chi0 (analytic Re, delta-weight Im), FP64, with the mixed-precision forms
timed beside it.

One step = one chi0_dynamic call over all q x w: matrix elements (MFMA), carving +
tetrahedron weights, ordered reduction.  Inputs are resident in HBM before the timed
region.  Prints one JSON line.

--workload selects the other seeded configurations: bcc_dynamic (9-orbital bcc, 48^3,
64 q x 512 w, --n-keep band window), tetra_static (the 10-orbital model, 256 q, static),
sc_cma (single-band cubic, 16^3, 8 q, static), batch (16 heterogeneous instances in one
fused launch sequence) and pw_static (plane-wave basis: 4096 coefficients per band, 32 bands,
12^3 mesh, 16 q, static; the matrix-element contraction against the FP64 MFMA roofline) and
iw_cubic (the irreducible wedge of a 48^3 cubic mesh with the 48-element point-group loop, beside
the full mesh at the same q).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def _metrics():
    """The parity metric shared with the tests (tests/metrics.py)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("tests_metrics", os.path.join(ROOT, "tests", "metrics.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    sys.modules["tests_metrics"] = mod
    return mod

# Flops of the formulas as the tetrahedron kernel executes them, counted from the source: an FMA
# counts 2, an add, subtract or multiply 1, the hardware reciprocal estimate 1 (the reciprocal
# routine is the estimate plus three FMAs: 7), frexp, compares and selects 0.  Work a kernel computes
# and then discards is not counted.  FP64 form:
#   far evaluation (final tetrahedron, w; or a list of final tetrahedra summed into one series, w):
#        w - c 1, reciprocal 7, final accumulate 2 -> 10, plus 2 per series term (one Horner FMA);
#        the census counts the terms each evaluation uses
#   near evaluation, first pass (every near item): leaves 4 x (u 1, |u|/span 1, logarithm 41, u^3 L
#        4, W h' 8) = 220; span reciprocal 8; five Newton entries (span 1, reciprocal 7, value and
#        W-derivative 14, series test 1) = 115; top entry 14; accumulate 2 -> 359
#   near evaluation repeated in full (items whose entries cluster, counted by the census):
#        359 + three 2-node entry series of 8 terms (95 each) + two 3-node entry series of 12 terms
#        (205 each) -> 1054
#   per final tetrahedron: centre and half-span 4, offsets 4, class and flags 12 -> 20; carving
#        (edge parameters and interpolated corners of the written pieces) about 40; plus 23 per
#        series coefficient with its W-derivative, computed for the blocks of terms the series
#        class reads (the census counts them; 50 for every tetrahedron in earlier kernels)
#   the logarithm (own routine): range reduction 3, reciprocal 7, 11-term atanh series 23, scale
#        and ln2 terms 8 -> 41
FLOPS_FAR_BASE = 10
FLOPS_PER_TERM = 2
FLOPS_NEAR_FIRST = 359
FLOPS_NEAR_FULL = 1054
FLOPS_PER_FINAL_TET = 20 + 40
FLOPS_PER_COEF = 23
# Mixed form: the series in FP32 (20 terms at ratio 0.4), the near branch in FP32 except near-
# degenerate tetrahedra; the same formulas with the FP32 logarithm (hardware, 3) and 10-term
# entry series, one pass: 886 per near evaluation; coefficients still computed in FP64 and
# rounded to FP32 (24 each, the blocks the class reads, counted by the census).
FLOPS_NEAR_FULL_FP32 = 886
FLOPS_PER_FINAL_TET_MIXED = 16 + 40
FLOPS_PER_COEF_MIXED = 24
FP64_PEAK_TFLOPS = 78.6      # 256 CUs x 2.4 GHz x 128 FP64 flop/clk (vector)
FP32_PEAK_TFLOPS = 157.3     # published FP32 vector peak (packed FP32; this library is built without it)
HBM_PEAK_GBS = 8000.0        # published HBM3E bandwidth
METRIC = "chi0 band-pair*tetra*omega updates/s, mixed vs FP64 GPU, at stated rel error"
VALUE_FORM = "FP64 path; the mixed forms, their speed-up over it and their error per q are under 'mixed'"

# HBM bytes per launch of the tetrahedron kernel on the default workload (16 q per launch), from
# rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (scale factors from a plain 1 GiB copy), valid for
# the kernel sources with this hash only (see the counter summary under profiles/).
TRAFFIC_KERNEL_SHA = "c97c6df10c9b3c23"
TRAFFIC_BYTES_PER_LAUNCH = (337496.9 * 2.0 + 155647.3 * 1.0) * 1024


def census_flops(census: dict, mixed: bool = False) -> int:
    """Flops of a dynamic call from its work census (the counts above)."""
    if mixed:
        return (census["far_evals"] * FLOPS_FAR_BASE + census["far_terms"] * FLOPS_PER_TERM
                + census["near_evals"] * FLOPS_NEAR_FULL_FP32
                + census["final_tetrahedra"] * FLOPS_PER_FINAL_TET_MIXED + census["coef_terms"] * FLOPS_PER_COEF_MIXED)
    return (census["far_evals"] * FLOPS_FAR_BASE + census["far_terms"] * FLOPS_PER_TERM
            + census["near_evals"] * FLOPS_NEAR_FIRST + census.get("near_redo", 0) * FLOPS_NEAR_FULL
            + census["final_tetrahedra"] * FLOPS_PER_FINAL_TET + census["coef_terms"] * FLOPS_PER_COEF)


def host_cores() -> dict:
    """The host cores this process may use (the CPU baseline runs on all of them), and the CPU."""
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = os.environ.get("OMP_NUM_THREADS")
    threads = min(avail, int(omp)) if omp and omp.isdigit() and int(omp) > 0 else avail
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"threads": threads, "nproc": os.cpu_count(), "affinity": avail, "cpu_model": model}


def input_manifest(wl) -> str:
    """SHA-256 over every input array of a workload (energies, eigenvectors, k+q data, omega), in a
    fixed order: the GPU run and the CPU baseline read these same bytes."""
    import hashlib
    h = hashlib.sha256()
    for a in (wl.eps_k, wl.c_k, wl.omega):
        if a is not None:
            h.update(np.ascontiguousarray(a).tobytes())
    for q in wl.qs:
        for a in (q.eps_kq, q.c_kq):
            if a is not None:
                h.update(np.ascontiguousarray(a).tobytes())
        if q.shift is not None:
            h.update(np.asarray(q.shift, dtype=np.int64).tobytes())
    return h.hexdigest()


def timed_median(fn, reps: int = 3):
    """Median wall time of reps calls of fn (and the last result)."""
    times, out = [], None
    for _ in range(reps):
        t = time.time()
        out = fn()
        times.append(time.time() - t)
    return float(np.median(times)), out


# The same for the plane-wave contraction kernel on the pw_static workload (16 q per launch), and
# for the split forms' pair of kernels (the split into packed operands, then the packed-operand
# contraction; figures of the BF16x3 pair, FP16x3 reads 5% less).
PW_TRAFFIC_KERNEL_SHA = "34b23f18bec6d0d5"
PW_TRAFFIC_BYTES_PER_LAUNCH = (33183559 * 2.0 + 700292 * 1.0) * 1024
PW_PACKED_TRAFFIC_BYTES_PER_LAUNCH = ((1769503 + 16849096) * 2.0 + (1769824 + 754128) * 1.0) * 1024


def kernel_sha(files=("k_tetra.h", "k_tetra_dyn.hip", "chi0_math.h")) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1407_3444_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def upload(wl, dev):
    import torch
    import paper_1407_3444_amd as lib
    eps = torch.from_numpy(wl.eps_k).to(dev)
    ck = None if wl.c_k is None else torch.from_numpy(wl.c_k).to(dev)
    qs = []
    for q in wl.qs:
        if q.shift is not None:
            qs.append(lib.Q(shift=q.shift))
        else:
            c = None if (q.c_kq is None or wl.cma) else torch.from_numpy(q.c_kq).to(dev)
            qs.append(lib.Q(eps_kq=torch.from_numpy(q.eps_kq).to(dev), c_kq=c))
    return eps, ck, qs


def bench_static(args, wl, desc):
    """Static chi0 over all q of a static workload: one chi0_static call per step."""
    import torch
    import paper_1407_3444_amd as lib
    dev = torch.device("cuda:0")
    eps, ck, qs = upload(wl, dev)
    lo, hi = wl.window()
    nbw = hi - lo
    plan = lib.Chi0Plan(wl.nk, eps, ck, mu=wl.mu, spin_factor=wl.spin_factor, band_lo=lo, band_hi=hi,
                        cma=wl.cma)
    ws = plan.workspace(len(qs), 1)
    if args.pairs:
        out = torch.empty((len(qs), nbw, nbw), dtype=torch.float64, device=dev)
        call = lambda: plan.static_pairs(qs, workspace=ws, out=out)
        desc = desc.replace(", FP64", ", resolved by band pair, FP64")
    else:
        out = torch.empty(len(qs), dtype=torch.float64, device=dev)
        call = lambda: plan.static(qs, workspace=ws, out=out)
    for _ in range(max(1, args.warmup)):
        call()
    torch.cuda.synchronize()
    plan.profile(True)
    plan.read_profile()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        call()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    prof = plan.read_profile()
    units = len(qs) * 6 * wl.n_k * nbw * nbw
    result = {"metric": METRIC, "value_form": VALUE_FORM, "value": units / (ms * 1e-3),
              "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
              "data": "synthetic (seeded tight-binding model, eigenpairs by numpy eigh)",
              "config": {"workload": desc, "mesh": list(wl.nk), "n_q": len(qs), "n_omega": 1,
                         "band_pairs": nbw * nbw, "units_per_step": units, "parallelism": "single GPU"},
              "roofline": None,
              "kernel_ms_per_step": {k: round(v["ms"] / args.steps, 3) for k, v in prof.items()}}
    if args.pairs:
        # band-pair analysis (Sec. III, Fig. 8): the share of each (n at k, m at k+q) pair in chi0 at the
        # q of largest |chi0|, and the band-truncation convergence: chi0 of the window of n_keep bands
        # nearest the Fermi level (mean energy closest to mu) is the sum of its (n, m) block
        pr = out.cpu().numpy()
        tot = pr.sum(axis=(1, 2))
        qmax = int(np.argmax(np.abs(tot)))
        conv = {}
        for n_keep in range(1, nbw + 1):
            wlo, whi = synth_band_window(wl.eps_k[lo:hi], n_keep, wl.mu)
            sub = pr[:, wlo:whi, wlo:whi].sum(axis=(1, 2))
            rel = np.abs(sub - tot) / np.abs(tot)
            conv[str(n_keep)] = {"window": [lo + wlo, lo + whi], "rel_diff_vs_all_max": float(rel.max()),
                                 "rel_diff_vs_all_mean": float(rel.mean())}
        result["band_pairs"] = {"q_index_of_max": qmax, "chi0_at_q": float(tot[qmax]),
                                "pair_share_at_q": np.round(pr[qmax] / tot[qmax], 4).tolist(),
                                "truncation": conv}
        log("band truncation", {k: round(v["rel_diff_vs_all_max"], 4) for k, v in conv.items()})
    if not args.no_cpu_baseline:
        import oracle
        threads = host_cores()["threads"]
        t1 = time.time()
        if args.pairs:
            ref = oracle.chi0_pairs(wl, 0, nthreads=threads)[:, :, 0].real
            err = float(np.max(np.abs(out[0].cpu().numpy() - ref)) / np.max(np.abs(ref)))
        else:
            ref = oracle.chi0(wl, 0, nthreads=threads)[0].real
            err = abs(float(out[0].item()) - ref) / abs(ref)
        dt = time.time() - t1
        result["cpu_baseline"] = {"value": 6 * wl.n_k * nbw * nbw / dt, "unit": "updates/s", "cores": threads,
                                  "kind": "oracle", "sample": f"q index 0 of {len(qs)}, full mesh, {dt:.1f} s"}
        result["parity_sample"] = {"rel_err_vs_oracle": err, "q": 0}
    print(json.dumps(result), flush=True)


def synth_band_window(eps, n_keep, mu):
    import synth
    return synth.band_window(eps, n_keep, mu)


def bench_pw(args):
    """Plane-wave-basis workload: static chi0 over 16 q with matrix elements summed over 4096
    plane-wave coefficients per band (Sec. III), so the contraction dominates the step.  The
    roofline is that of the contraction kernel against the FP64 MFMA peak; a batched complex GEMM
    from the vendor BLAS (torch.matmul) on the same operands of one q is timed as a yardstick."""
    import torch
    import paper_1407_3444_amd as lib
    import synth
    t0 = time.time()
    nk, n_pw, nb, nq = (12, 12, 12), 4096, 32, 16
    wl = synth.plane_wave_workload(nk, n_pw, nb, nq, 1, seed=11)
    wl.static = True
    log(f"plane-wave inputs built in {time.time() - t0:.1f}s: {wl.c_k.nbytes / 2**30:.2f} GiB of coefficients")
    dev = torch.device("cuda:0")
    eps, ck, qs = upload(wl, dev)
    lo, hi = wl.window()
    nbw = hi - lo
    plan = lib.Chi0Plan(wl.nk, eps, ck, mu=wl.mu, spin_factor=wl.spin_factor, band_lo=lo, band_hi=hi)
    ws = plan.workspace(len(qs), 1)
    out = torch.empty(len(qs), dtype=torch.float64, device=dev)
    for _ in range(max(1, args.warmup)):
        plan.static(qs, workspace=ws, out=out)
    torch.cuda.synchronize()
    plan.profile(True)
    plan.read_profile()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        plan.static(qs, workspace=ws, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    prof = plan.read_profile()
    plan.profile(False)
    log("timed", args.steps, "steps:", f"{ms:.2f} ms/step", prof)
    units = len(qs) * 6 * wl.n_k * nbw * nbw
    con = prof["contract"]
    avg_ms = con["ms"] / con["launches"]
    q_per_launch = len(qs) * args.steps / con["launches"]
    # per (k, q): nbw^2 complex dot products of length n_pw, 8 real flops per complex term (the
    # usual complex-GEMM count; the kernel issues three real products per term, 6 flops)
    flops_launch = 8.0 * n_pw * nbw * nbw * wl.n_k * q_per_launch
    mfma_flops_launch = 6.0 * n_pw * nbw * nbw * wl.n_k * q_per_launch
    # per launch: the window's coefficients at every k once (shared by the q of the launch), at
    # k+q once per (k, q), 16 bytes each, and the nbw^2 results per (k, q)
    bytes_launch = (n_pw * nbw * 16.0 * (1 + q_per_launch) + nbw * nbw * 8.0 * q_per_launch) * wl.n_k
    # the roofline counts the flops of the three-product form, the ones the matrix cores must do
    achieved = mfma_flops_launch / (avg_ms * 1e-3) / 1e12
    pw_sha_ok = kernel_sha(("k_contract.hip",)) == PW_TRAFFIC_KERNEL_SHA
    result = {"metric": METRIC, "value_form": VALUE_FORM, "value": units / (ms * 1e-3),
              "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
              "data": "synthetic (seeded 32-orbital tight-binding energies, seeded orthonormal plane-wave "
                      "coefficients)",
              "config": {"workload": "plane-wave basis, 12^3 mesh, 4096 plane waves, 32 bands (all pairs), "
                                     "16 q, static, FP64",
                         "mesh": list(wl.nk), "n_pw": n_pw, "n_q": len(qs), "band_pairs": nbw * nbw,
                         "units_per_step": units, "parallelism": "single GPU"},
              "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                           "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                           "traffic": PW_TRAFFIC_BYTES_PER_LAUNCH if len(qs) == 16 and pw_sha_ok else None,
                           "kernel": "contract_pw_kernel", "avg_launch_ms": round(avg_ms, 3),
                           "algorithmic_bytes_per_launch": bytes_launch,
                           "hbm_bound_ms": round(bytes_launch / 8e12 * 1e3, 3),
                           "mfma_bound_ms": round(mfma_flops_launch / (FP64_PEAK_TFLOPS * 1e12) * 1e3, 3),
                           "complex_gemm_equivalent_tflops": round(flops_launch / (avg_ms * 1e-3) / 1e12, 3)},
              "kernel_ms_per_step": {k: round(v["ms"] / args.steps, 3) for k, v in prof.items()}}

    # yardstick: vendor batched ZGEMM of one q (k+q coefficients gathered beforehand, untimed)
    sh = wl.qs[0].shift
    c5 = (ck if ck.is_complex() else torch.view_as_complex(ck)).view(*nk, n_pw, nb)[..., lo:hi]
    a_h = c5.reshape(wl.n_k, n_pw, nbw).transpose(1, 2).conj().contiguous()
    b = torch.roll(c5, shifts=tuple(-int(v) for v in sh), dims=(0, 1, 2)).reshape(wl.n_k, n_pw, nbw).contiguous()
    m = torch.matmul(a_h, b)
    torch.cuda.synchronize()
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record(stream)
    for _ in range(args.steps):
        m = torch.matmul(a_h, b)
    g1.record(stream)
    torch.cuda.synchronize()
    gms = g0.elapsed_time(g1) / args.steps
    w_lib = (m.abs() ** 2).permute(1, 2, 0).contiguous()
    w_ours = plan.matrix_elements(qs[0])
    torch.cuda.synchronize()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record(stream)
    for _ in range(args.steps):
        plan.matrix_elements(qs[0], out=w_ours)
    s1.record(stream)
    torch.cuda.synchronize()
    single_ms = s0.elapsed_time(s1) / args.steps
    diff = float((w_ours - w_lib).abs().max() / w_lib.abs().max())
    gflops = 8.0 * n_pw * nbw * nbw * wl.n_k
    result["vendor_zgemm_one_q"] = {"ms": gms, "tflops": gflops / (gms * 1e-3) / 1e12,
                                    "ours_ms_per_q": avg_ms / q_per_launch, "ours_single_q_call_ms": single_ms,
                                    "max_rel_diff_of_W": diff}
    log(f"vendor batched zgemm: {gms:.3f} ms/q; ours {avg_ms / q_per_launch:.3f} ms/q; W rel diff {diff:.2e}")
    del a_h, b, m, w_lib

    # split-precision forms of the same step: time, matrix-element and chi0 errors against this run's
    # FP64 result, and the roofline of their contraction (HBM).  With 16 q given by mesh shifts the
    # library splits the window's coefficients once per launch into packed 8-byte operands (read 16
    # bytes, write 8 per coefficient) and the contraction kernel reads those, at every k once and at
    # every k+q once per q; the matrix cores do 24 flops per band pair and basis function (two real
    # GEMMs of doubled depth, three products each).
    packed_bytes = (n_pw * nbw * (16.0 + 8.0 + 8.0 * (1 + q_per_launch)) + nbw * nbw * 8.0 * q_per_launch) * wl.n_k
    ref64 = out.clone()
    mixed = {}
    for prec, name in ((1, "bf16x3"), (2, "fp16x3")):
        mplan = lib.Chi0Plan(wl.nk, eps, ck, mu=wl.mu, spin_factor=wl.spin_factor, band_lo=lo, band_hi=hi,
                             precision=prec)
        mout = torch.empty_like(out)
        mws = mplan.workspace(len(qs), 1)      # with room for the packed split operands
        for _ in range(max(1, args.warmup)):
            mplan.static(qs, workspace=mws, out=mout)
        torch.cuda.synchronize()
        mplan.profile(True)
        mplan.read_profile()
        m0, m1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        m0.record(stream)
        for _ in range(args.steps):
            mplan.static(qs, workspace=mws, out=mout)
        m1.record(stream)
        torch.cuda.synchronize()
        mms = m0.elapsed_time(m1) / args.steps
        mprof = mplan.read_profile()
        mplan.profile(False)
        mcon = mprof["contract"]
        m_avg = mcon["ms"] / mcon["launches"]
        w_split = mplan.matrix_elements(qs[0])
        torch.cuda.synchronize()
        w_err = float((w_split - w_ours).abs().max() / w_ours.abs().max())
        chi_err = float(((mout - ref64).abs() / ref64.abs()).max())
        hbm = packed_bytes / (m_avg * 1e-3) / 1e9
        split_flops = 24.0 * n_pw * nbw * nbw * wl.n_k * q_per_launch
        mixed[name] = {"ms_per_step": round(mms, 3), "speedup_vs_fp64": round(ms / mms, 3),
                       "contract_ms_per_launch": round(m_avg, 3),
                       "contract_speedup_vs_fp64": round(avg_ms / m_avg, 3),
                       "max_rel_err_of_W_vs_fp64": w_err, "max_rel_err_of_chi0_vs_fp64": chi_err,
                       "roofline": {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS,
                                    "unit": "GB/s", "frac": round(hbm / HBM_PEAK_GBS, 4),
                                    "traffic": (PW_PACKED_TRAFFIC_BYTES_PER_LAUNCH
                                                if len(qs) == 16 and pw_sha_ok else None),
                                    "kernel": "pack_split_kernel + contract_pw_packed_kernel",
                                    "algorithmic_bytes_per_launch": packed_bytes,
                                    "mfma_tflops": round(split_flops / (m_avg * 1e-3) / 1e12, 1)}}
        log(f"{name}: {mms:.2f} ms/step, contraction {m_avg:.3f} ms/launch ({hbm:.0f} GB/s), "
            f"W err {w_err:.2e}, chi0 err {chi_err:.2e}")
        del mplan, mout, mws, w_split
    result["mixed"] = mixed

    if not args.no_cpu_baseline:
        import oracle
        threads = host_cores()["threads"]
        t1 = time.time()
        ref = oracle.chi0(wl, 0, nthreads=threads)[0].real
        dt = time.time() - t1
        err = abs(float(out[0].item()) - ref) / abs(ref)
        result["cpu_baseline"] = {"value": 6 * wl.n_k * nbw * nbw / dt, "unit": "updates/s", "cores": threads,
                                  "kind": "oracle", "sample": f"q index 0 of {len(qs)}, full mesh, {dt:.1f} s"}
        result["parity_sample"] = {"rel_err_vs_oracle": err, "q": 0}
        log(f"oracle sample {dt:.1f}s, rel err {err:.2e}")
    print(json.dumps(result), flush=True)


def bench_iw(args):
    """Irreducible wedge with the point-group loop (Sec. II): a 6-orbital O_h-symmetric cubic model,
    the wedge of the 48^3 mesh (13,824 tetrahedra, 2,925 points), 48 group elements per q, 4 q,
    256 frequencies, dynamic, FP64; the full 48^3 Kuhn mesh at the same q is timed beside it (the
    same number of tetrahedron units; the two triangulations differ, so the values agree to the
    discretisation error)."""
    import torch
    import paper_1407_3444_amd as lib
    import synth
    dev = torch.device("cuda:0")
    t0 = time.time()
    n, nw = 48, 256
    model = synth.cubic_s_model(5, 6)
    q_list = [np.array(v) for v in ([0.1, 0.0, 0.0], [0.23, 0.0, 0.0], [0.1, 0.1, 0.0], [0.19, 0.07, 0.03])]
    omega = synth.omega_grid(nw)
    mu = 0.0
    kf, tets, vol, ops = lib.iw_cubic(n)
    e, c = synth.eigensystem(model, kf)
    opsf = ops.astype(np.float64)
    entries = []
    for q in q_list:
        for g in opsf:
            entries.append(synth.eigensystem(model, kf + q @ g))
    log(f"wedge inputs built in {time.time() - t0:.1f}s: {len(kf)} points, {len(tets)} tetrahedra, "
        f"{len(entries)} (q, g) entries")
    om = torch.from_numpy(omega).to(dev)
    eps_d, c_d = torch.from_numpy(e).to(dev), torch.from_numpy(c).to(dev)
    plan = lib.Chi0Plan(None, eps_d, c_d, mu=mu, tetrahedra=(torch.from_numpy(tets).to(dev), vol))
    qs = [lib.Q(eps_kq=torch.from_numpy(a).to(dev), c_kq=torch.from_numpy(b).to(dev)) for a, b in entries]
    ws = plan.workspace(len(qs), nw)
    out = torch.empty((len(q_list), nw, 2), dtype=torch.float64, device=dev)
    census = {}
    for i in range(0, len(qs), 16):
        for k, v in plan.census(qs[i:i + 16], om, workspace=ws).items():
            census[k] = census.get(k, 0) + v
    stream = torch.cuda.current_stream()

    def timed(fn, steps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    plan.profile(True)
    plan.read_profile()
    ms = timed(lambda: plan.dynamic_group(qs, 48, om, workspace=ws, out=out), args.steps)
    prof = plan.read_profile()
    plan.profile(False)
    log(f"wedge + point-group loop: {ms:.1f} ms/step", prof)
    got = torch.view_as_complex(out).cpu().numpy()

    # the full Kuhn mesh at the same q (explicit k+q)
    nk = (n, n, n)
    kfm = synth.mesh_kfrac(nk)
    em, cm = synth.eigensystem(model, kfm)
    mplan = lib.Chi0Plan(nk, torch.from_numpy(em).to(dev), torch.from_numpy(cm).to(dev), mu=mu)
    mqs = []
    for q in q_list:
        a, b = synth.eigensystem(model, kfm + q)
        mqs.append(lib.Q(eps_kq=torch.from_numpy(a).to(dev), c_kq=torch.from_numpy(b).to(dev)))
    mws = mplan.workspace(len(mqs), nw)
    mout = torch.empty((len(q_list), nw, 2), dtype=torch.float64, device=dev)
    mcensus = mplan.census(mqs, om, workspace=mws)
    mms = timed(lambda: mplan.dynamic(mqs, om, workspace=mws, out=mout), args.steps)
    mesh_val = torch.view_as_complex(mout).cpu().numpy()
    diff = float(np.max(np.abs(got - mesh_val)) / np.max(np.abs(mesh_val)))
    log(f"full mesh: {mms:.1f} ms/step; wedge vs mesh max rel difference {diff:.2e}")

    nbw = 6
    units = len(entries) * len(tets) * nbw * nbw * nw
    tet = prof["tetra"]
    avg_ms = tet["ms"] / tet["launches"]
    achieved = census_flops(census) / (tet["ms"] / args.steps * 1e-3) / 1e12
    result = {"metric": METRIC, "value_form": VALUE_FORM, "value": units / (ms * 1e-3), "unit": "updates/s",
              "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": ms, "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "dtype": "f64",
              "data": "synthetic (seeded 6-orbital O_h-symmetric cubic tight-binding model)",
              "config": {"workload": "irreducible wedge of a 48^3 simple-cubic mesh (13,824 tetrahedra) with the "
                                     "48-element point-group loop, 6 orbitals (36 band pairs), 4 q x 256 w, dynamic, "
                                     "FP64",
                         "wedge_points": int(len(kf)), "wedge_tetrahedra": int(len(tets)), "group_order": 48,
                         "n_q": len(q_list), "n_omega": nw, "units_per_step": units, "parallelism": "single GPU"},
              "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                           "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": None,
                           "kernel": "tetra_dynamic_kernel (list form), all launches of a step",
                           "avg_launch_ms": round(avg_ms, 3),
                           "launches_per_step": tet["launches"] / args.steps},
              "census": census,
              "kernel_ms_per_step": {k: round(v["ms"] / args.steps, 3) for k, v in prof.items()},
              "full_mesh_same_q": {"ms_per_step": mms, "value": units / (mms * 1e-3),
                                   "max_rel_difference_vs_wedge": diff, "census": mcensus}}
    if not args.no_cpu_baseline:
        import oracle
        threads = host_cores()["threads"]
        sample_g, sample_w = list(range(0, 48, 4)), [0, 36, 73, 109, 146, 182, 219, 255]
        t1 = time.time()
        ref = oracle.chi0_iw(e, c, [entries[g] for g in sample_g], tets, vol, omega[sample_w], mu=mu,
                             nthreads=threads)
        dt = time.time() - t1
        u = len(sample_g) * len(tets) * nbw * nbw * len(sample_w)
        # parity on the same sample: the GPU sum over the same six group elements of q 0
        sub = [qs[g] for g in sample_g]
        part = plan.dynamic_group(sub, len(sub), om).cpu().numpy()[0][sample_w]
        err = float(np.max(np.abs(part - ref)) / np.max(np.abs(ref)))
        result["cpu_baseline"] = {"value": u / dt, "unit": "updates/s", "cores": threads, "kind": "oracle",
                                  "sample": f"q 0, {len(sample_g)} of 48 group elements, {len(sample_w)} w, "
                                            f"{dt:.1f} s"}
        result["parity_sample"] = {"max_rel_err_vs_oracle": err, "q": 0, "group_elements": sample_g,
                                   "omega_index": sample_w}
        log(f"oracle sample {dt:.1f}s, rel err {err:.2e}")
    print(json.dumps(result), flush=True)


def bench_batch(args):
    """The 16-instance heterogeneous batch: one fused, graph-captured launch sequence per step
    (FP64 and mixed), against the same instances as 16 sequential chi0_dynamic calls (FP64)."""
    import torch
    import paper_1407_3444_amd as lib
    import synth
    t0 = time.time()
    wls = synth.batch_workloads(nq_div=args.batch_nq_div)
    dev = torch.device("cuda:0")
    log(f"batch inputs built in {time.time() - t0:.1f}s: {len(wls)} instances")
    insts, plans = [], []
    for wl, _ in wls:
        eps, ck, qs = upload(wl, dev)
        om = torch.from_numpy(wl.omega).to(dev)
        insts.append(lib.Instance(nk=wl.nk, eps_k=eps, c_k=ck, qs=qs, omega=om, mu=wl.mu,
                                  spin_factor=wl.spin_factor))
        plans.append(lib.Chi0Plan(wl.nk, eps, ck, mu=wl.mu, spin_factor=wl.spin_factor))
    units = sum(len(w.qs) * 6 * w.n_k * w.n_bands ** 2 * len(w.omega) for w, _ in wls)
    stream = torch.cuda.current_stream()

    def timed(fn, steps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    # sequential FP64: one chi0_dynamic call per instance, one shared workspace
    ws_bytes = max(p.workspace_bytes(len(i.qs), int(i.omega.shape[0])) for p, i in zip(plans, insts))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    seq_out = [torch.empty((len(i.qs), int(i.omega.shape[0]), 2), dtype=torch.float64, device=dev)
               for i in insts]
    census = {}
    for p, i in zip(plans, insts):
        for k, v in p.census(i.qs, i.omega, workspace=ws).items():
            census[k] = census.get(k, 0) + v
    log("census", census)

    def seq():
        for p, i, o in zip(plans, insts, seq_out):
            p.dynamic(i.qs, i.omega, workspace=ws, out=o)
    seq_ms = timed(seq, args.steps)
    log(f"sequential FP64: {seq_ms:.1f} ms/step")
    del ws

    batch = lib.Chi0Batch(insts, workgroups=args.batch_workgroups, use_graph=True)
    chosen = batch.tune(reps=1) if args.tune else None
    info = batch.info()
    log("batch", info, "tuned workgroups", chosen)
    b_ms = timed(batch.run, args.steps)
    log(f"batched FP64 (graph): {b_ms:.1f} ms/step")
    seq_np = [torch.view_as_complex(o).cpu().numpy() for o in seq_out]
    b_np = [torch.view_as_complex(i.chi).cpu().numpy() for i in insts]
    rel_b = max(float(np.max(np.abs(a - b)) / np.max(np.abs(b))) for a, b in zip(b_np, seq_np))
    batch.close()
    del batch

    m_insts = [lib.Instance(nk=i.nk, eps_k=i.eps_k, c_k=i.c_k, qs=i.qs, omega=i.omega, mu=i.mu,
                            spin_factor=i.spin_factor, precision=1) for i in insts]
    mbatch = lib.Chi0Batch(m_insts, workgroups=args.batch_workgroups, use_graph=True)
    m_ms = timed(mbatch.run, args.steps)
    m_np = [torch.view_as_complex(i.chi).cpu().numpy() for i in m_insts]
    _per_result = _metrics().per_result
    per_q = np.concatenate([_per_result(a, b).max(axis=1) for a, b in zip(m_np, seq_np)])
    log(f"batched mixed (graph): {m_ms:.1f} ms/step, max rel err {per_q.max():.2e}")
    mbatch.close()

    flops = census_flops(census)
    achieved = flops / (b_ms * 1e-3) / 1e12
    result = {
        "metric": METRIC, "value_form": VALUE_FORM,
        "value": units / (b_ms * 1e-3), "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": b_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (16 seeded tight-binding models, eigenpairs by numpy eigh)",
        "config": {"workload": "heterogeneous batch of 16 TB models (tetragonal/bcc/sc, 4-32 orbitals, "
                               f"24^3-48^3 meshes, 32-128 q / {args.batch_nq_div}, 128-512 w), one fused "
                               "graph-captured launch sequence, FP64",
                   "instances": [w.meta for w, _ in wls], "units_per_step": units,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": None,
                     "kernel": "tetra_batch_kernel (whole step: K_A + K_B + K_R)"},
        "census": census, "batch_info": info, "tuned_workgroups": chosen,
        "sequential_fp64": {"value": units / (seq_ms * 1e-3), "ms_per_step": seq_ms,
                            "batched_speedup": seq_ms / b_ms, "batched_max_rel_diff": rel_b},
        "mixed": {"bf16x3_batched": {"value": units / (m_ms * 1e-3), "ms_per_step": m_ms,
                                     "speedup_vs_sequential_fp64": seq_ms / m_ms,
                                     "speedup_vs_batched_fp64": b_ms / m_ms,
                                     "rel_err_vs_fp64_gpu_per_q_max": float(per_q.max()),
                                     "rel_err_vs_fp64_gpu_per_q_mean": float(per_q.mean()),
                                     "metric": "per result: |d| / max(|ref|, 1e-3 max_w |ref|)"}},
    }
    if not args.no_cpu_baseline:
        import oracle
        threads = host_cores()["threads"]
        wl = wls[15][0]
        sample_w = list(range(0, len(wl.omega), max(1, len(wl.omega) // 4)))
        t1 = time.time()
        ref = oracle.chi0(wl, 0, omega=wl.omega[sample_w], nthreads=threads)
        dt = time.time() - t1
        u = 6 * wl.n_k * wl.n_bands ** 2 * len(sample_w)
        err = float(np.max(np.abs(b_np[15][0][sample_w] - ref)) / np.max(np.abs(ref)))
        result["cpu_baseline"] = {"value": u / dt, "unit": "updates/s", "cores": threads, "kind": "oracle",
                                  "sample": f"instance 15 (32 orbitals, 24^3), q index 0, {len(sample_w)} w, "
                                            f"{dt:.1f} s"}
        result["parity_sample"] = {"max_rel_err_vs_oracle": err, "instance": 15, "q": 0, "omega_index": sample_w}
        log(f"oracle sample {dt:.1f}s, rel err {err:.2e}")
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nq", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--workload", default="tetra_dynamic",
                    choices=["tetra_dynamic", "bcc_dynamic", "tetra_static", "sc_cma", "batch", "pw_static",
                             "iw_cubic"])
    ap.add_argument("--batch-nq-div", type=int, default=1,
                    help="batch workload: divide every instance's q count by this (1 = full size)")
    ap.add_argument("--batch-workgroups", type=int, default=0, help="batch workload: K_B workgroups (0 = default)")
    ap.add_argument("--tune", action="store_true", help="batch workload: autotune the workgroups first")
    ap.add_argument("--kk", type=int, default=0, metavar="N_SPEC",
                    help="dynamic workloads: also time the Kramers-Kronig route with N_SPEC spectral points")
    ap.add_argument("--pairs", action="store_true",
                    help="time the band-pair resolved call (chi0_static_pairs, or chi0_dynamic_pairs for "
                         "dynamic workloads)")
    ap.add_argument("--n-keep", type=int, default=9, help="band window of bcc_dynamic")
    ap.add_argument("--sweep", action="store_true",
                    help="bcc_dynamic with all 9 bands: also time the 7- and 5-band windows and report "
                         "their difference from the all-band result per q")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = args.copy_probe // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import synth
    t0 = time.time()
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "pw_static":
        return bench_pw(args)
    if args.workload == "iw_cubic":
        return bench_iw(args)
    if args.workload == "tetra_dynamic":
        wl = synth.make_workload("tetra_dynamic", nq=64, q_subset=list(range(min(args.nq, 64))),
                                 workers=args.workers)
        desc = ("tetragonal two-site 10-orbital TB, 64x64x8 mesh, 64 q x 512 w, dynamic, all 100 band "
                "pairs, FP64")
    elif args.workload == "bcc_dynamic":
        wl = synth.make_workload("bcc_dynamic", nq=64, q_subset=list(range(min(args.nq, 64))),
                                 n_keep=args.n_keep, workers=args.workers)
        desc = f"bcc 9-orbital TB, 48^3 mesh, 64 q x 512 w, dynamic, {args.n_keep}-band window, FP64"
    elif args.workload == "tetra_static":
        nq = 256 if args.nq == 64 else args.nq
        wl = synth.make_workload("tetra_static", nq=256, q_subset=list(range(min(nq, 256))),
                                 workers=args.workers)
        desc = "tetragonal two-site 10-orbital TB, 64x64x8 mesh, 256 q, static, all 100 band pairs, FP64"
    else:
        wl = synth.make_workload("sc_cma")
        desc = "single-band simple-cubic NN TB, CMA, 16^3 mesh, 8 q on Gamma-R, static, FP64"
    log(f"inputs built in {time.time() - t0:.1f}s: mesh {wl.nk}, {len(wl.qs)} q, {len(wl.omega)} w")
    if wl.static:
        return bench_static(args, wl, desc)

    import torch
    import paper_1407_3444_amd as lib
    dev = torch.device("cuda:0")
    eps, ck, qs = upload(wl, dev)
    om = torch.from_numpy(wl.omega).to(dev)
    lo, hi = wl.window()
    nbw = hi - lo
    plan = lib.Chi0Plan(wl.nk, eps, ck, mu=wl.mu, spin_factor=wl.spin_factor, band_lo=lo, band_hi=hi)
    ws = plan.workspace(len(qs), len(wl.omega))
    out = torch.empty((len(qs), len(wl.omega), 2), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    log(f"resident on device; workspace {ws.numel() / 2**20:.1f} MiB")

    census = plan.census(qs, om, workspace=ws)
    log("census", census)

    for _ in range(args.warmup):
        plan.dynamic(qs, om, workspace=ws, out=out)
    torch.cuda.synchronize()
    log("warmup done")

    plan.profile(True)
    plan.read_profile()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for i in range(args.steps):
        plan.dynamic(qs, om, workspace=ws, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    prof = plan.read_profile()
    plan.profile(False)
    log("timed", args.steps, "steps:", f"{ms_total:.1f} ms", prof)

    nw = len(wl.omega)
    units_per_step = len(qs) * 6 * wl.n_k * nbw * nbw * nw
    ms_step = ms_total / args.steps
    value = units_per_step * args.steps / (ms_total * 1e-3)

    tet = prof["tetra"]
    launches_per_step = tet["launches"] / args.steps
    avg_ms = tet["ms"] / tet["launches"]
    flops_per_step = census_flops(census)
    flops_per_launch = flops_per_step / launches_per_step
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
    traffic = None
    if args.workload == "tetra_dynamic" and len(qs) == 64 and kernel_sha() == TRAFFIC_KERNEL_SHA:
        traffic = TRAFFIC_BYTES_PER_LAUNCH
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": traffic,
                "kernel": "tetra_dynamic_kernel", "avg_launch_ms": round(avg_ms, 3),
                "launches_per_step": launches_per_step,
                "flops_per_launch": flops_per_launch,
                "count": "census x flops of the formulas as executed (bench.py constants)"}

    result = {
        "metric": METRIC, "value_form": VALUE_FORM,
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded tight-binding model, eigenpairs by numpy eigh)",
        "config": {"workload": desc,
                   "mesh": list(wl.nk), "n_q": len(qs), "n_omega": nw, "band_pairs": nbw * nbw,
                   "tetrahedra": 6 * wl.n_k, "units_per_step": units_per_step,
                   "active_units_per_step": census["active_units"] * nw,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "census": census,
        "kernel_ms_per_step": {k: round(v["ms"] / args.steps, 3) for k, v in prof.items()},
    }

    # the oracle sample: q index 0 at 8 frequencies on the full mesh; it checks the FP64 and mixed
    # results and times the CPU baseline
    sample_w = [0, 73, 146, 219, 292, 365, 438, 511] if nw == 512 else list(range(0, nw, max(1, nw // 8)))[:8]
    ref_sample = None
    if not args.no_cpu_baseline:
        import oracle
        _m = _metrics()
        _max_err, _mean_err = _m.max_err, _m.mean_err
        cores = host_cores()
        dt, ref_sample = timed_median(lambda: oracle.chi0(wl, 0, omega=wl.omega[sample_w],
                                                          nthreads=cores["threads"]), reps=3)
        units = 6 * wl.n_k * nbw * nbw * len(sample_w)
        got = torch.view_as_complex(out[0]).cpu().numpy()[sample_w]
        result["cpu_baseline"] = {"value": units / dt, "unit": "updates/s", "cores": cores["threads"],
                                  "kind": "oracle",
                                  "sample": f"q index 0, {len(sample_w)} of {nw} w, full "
                                            f"{'x'.join(map(str, wl.nk))} mesh, median of 3 runs "
                                            f"({dt:.1f} s each)",
                                  "cpu_model": cores["cpu_model"], "nproc": cores["nproc"],
                                  "affinity_cores": cores["affinity"],
                                  "inputs_sha256": input_manifest(wl)}
        result["parity_sample"] = {"max_rel_err_vs_oracle": _max_err(got, ref_sample),
                                   "mean_rel_err_vs_oracle": _mean_err(got, ref_sample),
                                   "q": 0, "omega_index": sample_w,
                                   "metric": "per result: |d| / max(|ref|, 1e-3 max_w |ref|)"}
        log(f"oracle sample {dt:.1f}s (median of 3, {cores['threads']} threads), "
            f"max rel err {result['parity_sample']['max_rel_err_vs_oracle']:.2e}")
        # The second op count: the oracle's own tally of floating-point operations on its sample
        # (weights in chi0_oracle.c), per active unit and frequency, times the launch's active units
        # and frequencies.  The oracle evaluates every (final tetrahedron, frequency) pair by full
        # divided differences with complex logarithms and no far series, so this figure measures
        # how much work the kernel's formulation saves, not how well it uses the ALUs; `frac`
        # above is the census count.
        o_ops, o_units = oracle.last_count()
        per_unit_w = o_ops / max(1, o_units * len(sample_w))
        o_flops_launch = per_unit_w * census["active_units"] * nw / launches_per_step
        o_rate = o_flops_launch / (avg_ms * 1e-3) / 1e12
        roofline["oracle_count"] = {"flops_per_active_unit_and_w": round(per_unit_w, 1),
                                    "sample_active_units": o_units, "flops_per_launch": o_flops_launch,
                                    "achieved": round(o_rate, 1), "frac": round(o_rate / FP64_PEAK_TFLOPS, 2),
                                    "note": "oracle formulation (full divided differences for every pair); "
                                            "frac above uses the census count"}
        log(f"oracle op count: {per_unit_w:.0f} flops per active unit and w; "
            f"{o_rate:.0f} TFLOP/s oracle-equivalent ({o_rate / FP64_PEAK_TFLOPS:.1f}x the FP64 peak)")

    if args.pairs:
        # the same step resolved by band pair (one output per q, pair and frequency)
        pws = torch.empty(plan.dynamic_pairs_workspace_bytes(len(qs), nw), dtype=torch.uint8, device=dev)
        pout = torch.empty((len(qs), nbw, nbw, nw, 2), dtype=torch.float64, device=dev)
        plan.dynamic_pairs(qs, om, workspace=pws, out=pout)
        torch.cuda.synchronize()
        p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p0.record(stream)
        for i in range(args.steps):
            plan.dynamic_pairs(qs, om, workspace=pws, out=pout)
        p1.record(stream)
        torch.cuda.synchronize()
        pms = p0.elapsed_time(p1) / args.steps
        psum = pout.sum(dim=(1, 2))
        pdiff = float((psum - out).abs().max() / out.abs().max())
        result["pairs"] = {"ms_per_step": pms, "time_vs_dynamic": pms / ms_step,
                           "workspace_bytes": pws.numel(), "max_rel_diff_of_pair_sum_vs_dynamic": pdiff}
        log(f"pair-resolved dynamic: {pms:.1f} ms/step ({pms / ms_step:.2f}x), pair sum vs dynamic {pdiff:.1e}")
        del pws, pout

    if not args.no_mixed:
        # mixed forms: split BF16 / FP16 MFMA matrix elements, FP32 weights with the FP64 near branch
        # for near-degenerate tetrahedra, FP64 accumulation.  Errors per result (|d| / max(|ref|,
        # 1e-3 max_w |ref|)): against the FP64 oracle on its sample, and against this run's FP64 GPU
        # result over every q and frequency.
        _per_result = _metrics().per_result
        ref64 = torch.view_as_complex(out).cpu().numpy()
        res = {}
        for prec, name in ((1, "bf16x3"), (2, "fp16x3")):
            mplan = lib.Chi0Plan(wl.nk, eps, ck, mu=wl.mu, spin_factor=wl.spin_factor, band_lo=lo,
                                 band_hi=hi, precision=prec)
            mout = torch.empty_like(out)
            mcensus = mplan.census(qs, om, workspace=ws) if name == "bf16x3" else None
            mplan.dynamic(qs, om, workspace=ws, out=mout)
            torch.cuda.synchronize()
            mplan.profile(True)
            mplan.read_profile()
            m0, m1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            m0.record(stream)
            for i in range(args.steps):
                mplan.dynamic(qs, om, workspace=ws, out=mout)
            m1.record(stream)
            torch.cuda.synchronize()
            mprof = mplan.read_profile()
            mplan.profile(False)
            mms = m0.elapsed_time(m1) / args.steps
            got = torch.view_as_complex(mout).cpu().numpy()
            err_gpu = _per_result(got, ref64)
            entry = {"value": units_per_step / (mms * 1e-3), "ms_per_step": mms,
                     "speedup_vs_fp64": ms_step / mms,
                     "rel_err_vs_fp64_gpu_per_q_max": float(err_gpu.max(axis=1).max()),
                     "rel_err_vs_fp64_gpu_per_q_mean": float(err_gpu.mean(axis=1).mean()),
                     "kernel_ms_per_step": {k: round(v["ms"] / args.steps, 3) for k, v in mprof.items()}}
            if ref_sample is not None:
                e = _per_result(got[0][sample_w], ref_sample)
                entry["rel_err_vs_oracle_sample_max"] = float(e.max())
                entry["rel_err_vs_oracle_sample_mean"] = float(e.mean())
            if mcensus is not None:
                mt = mprof["tetra"]
                m_avg = mt["ms"] / mt["launches"]
                m_ach = census_flops(mcensus, mixed=True) / (mt["launches"] / args.steps) / (m_avg * 1e-3) / 1e12
                entry["roofline"] = {"bound": "alu", "achieved": round(m_ach, 3), "peak": FP32_PEAK_TFLOPS,
                                     "unit": "TFLOP/s", "frac": round(m_ach / FP32_PEAK_TFLOPS, 4),
                                     "traffic": None, "kernel": "tetra_dynamic_kernel (mixed form)",
                                     "avg_launch_ms": round(m_avg, 3),
                                     "count": "FP32 + FP64 flops from the census (bench.py constants)"}
                entry["census"] = mcensus
            res[name] = entry
            log(f"mixed {name}: {mms:.1f} ms/step, per-result err vs FP64 GPU max {err_gpu.max():.2e}"
                + (f", vs oracle sample {entry['rel_err_vs_oracle_sample_max']:.2e}" if ref_sample is not None else ""))
            del mplan
        result["mixed"] = res

    if args.kk:
        # Kramers-Kronig route: Im by delta weights on a spectral grid covering every e' - e of the
        # window, Re by the principal-value transform; error against this run's analytic FP64 result
        ref64 = torch.view_as_complex(out).cpu().numpy()
        e = eps[lo:hi]
        emin, emax = float(e.min()), float(e.max())
        ekq_min = min(float(q.eps_kq[lo:hi].min()) if q.eps_kq is not None else emin for q in qs)
        ekq_max = max(float(q.eps_kq[lo:hi].max()) if q.eps_kq is not None else emax for q in qs)
        spec_lo, spec_hi = ekq_min - emax - 0.01, ekq_max - emin + 0.01
        kout = torch.empty_like(out)
        plan.dynamic_kk(qs, om, args.kk, spec_lo, spec_hi, out=kout)
        torch.cuda.synchronize()
        k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        k0.record(stream)
        for i in range(args.steps):
            plan.dynamic_kk(qs, om, args.kk, spec_lo, spec_hi, out=kout)
        k1.record(stream)
        torch.cuda.synchronize()
        kms = k0.elapsed_time(k1) / args.steps
        got = torch.view_as_complex(kout).cpu().numpy()
        err_re = np.max(np.abs(got.real - ref64.real), axis=1) / np.max(np.abs(ref64.real), axis=1)
        err_im = np.max(np.abs(got.imag - ref64.imag), axis=1) / np.max(np.abs(ref64), axis=1)
        result["kk_route"] = {"value": units_per_step / (kms * 1e-3), "ms_per_step": kms,
                              "speedup_vs_fp64": ms_step / kms, "n_spec": args.kk,
                              "spectral_range": [spec_lo, spec_hi],
                              "re_rel_err_vs_analytic_per_q_max": float(err_re.max()),
                              "re_rel_err_vs_analytic_per_q_mean": float(err_re.mean()),
                              "im_rel_err_vs_analytic_max": float(err_im.max())}
        log(f"KK route: {kms:.1f} ms/step, Re rel err {err_re.max():.2e}, Im rel err {err_im.max():.2e}")

    if args.sweep and args.workload == "bcc_dynamic" and (lo, hi) == (0, wl.n_bands):
        # band truncation (Sec. III): the 7- and 5-band windows nearest the Fermi level (mean energy
        # closest to mu) against the sum over all 9 bands, per q: max_w |chi_n - chi_9| / max_w |chi_9|
        import synth
        ref_all = torch.view_as_complex(out).cpu().numpy()
        sweep = {}
        for n_keep in (7, 5):
            wlo, whi = synth.band_window(wl.eps_k, n_keep, wl.mu)
            splan = lib.Chi0Plan(wl.nk, eps, ck, mu=wl.mu, spin_factor=wl.spin_factor, band_lo=wlo, band_hi=whi)
            sout = torch.empty_like(out)
            splan.dynamic(qs, om, workspace=ws, out=sout)
            torch.cuda.synchronize()
            s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s0.record(stream)
            for i in range(args.steps):
                splan.dynamic(qs, om, workspace=ws, out=sout)
            s1.record(stream)
            torch.cuda.synchronize()
            sms = s0.elapsed_time(s1) / args.steps
            got = torch.view_as_complex(sout).cpu().numpy()
            rel = np.max(np.abs(got - ref_all), axis=1) / np.max(np.abs(ref_all), axis=1)
            su = len(qs) * 6 * wl.n_k * (whi - wlo) ** 2 * nw
            sweep[str(n_keep)] = {"window": [wlo, whi], "ms_per_step": sms, "value": su / (sms * 1e-3),
                                  "rel_diff_vs_all_bands_per_q_max": float(rel.max()),
                                  "rel_diff_vs_all_bands_per_q_mean": float(rel.mean()),
                                  "rel_diff_vs_all_bands_per_q": [round(float(v), 4) for v in rel]}
            log(f"band window {n_keep} {wlo}..{whi}: {sms:.1f} ms/step, max rel diff vs all bands {rel.max():.3f}")
            splan.sync()
            del splan
        result["band_truncation"] = sweep

    plan.sync()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
