"""GPU parity: libchi0 (HIP, gfx950) against the CPU FP64 oracle on the same seeded inputs.

Bar for the all-FP64 path: every result within 1e-10 of the oracle's, relative to the result
(per q and frequency, |got - ref| / max(|ref|, 1e-3 max_w |ref|), see tests/metrics.py); 1e-5 for
the mixed-precision forms.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from metrics import max_err, mean_err

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _plan(wl, **kw):
    torch = _torch()
    import paper_1407_3444_amd as lib
    dev = torch.device("cuda:0")
    eps = torch.from_numpy(np.ascontiguousarray(wl.eps_k)).to(dev)
    ck = None if wl.c_k is None else torch.from_numpy(np.ascontiguousarray(wl.c_k)).to(dev)
    lo, hi = wl.window()
    plan = lib.Chi0Plan(wl.nk, eps, ck, mu=wl.mu, spin_factor=wl.spin_factor, band_lo=lo, band_hi=hi,
                        cma=wl.cma, form=kw.get("form", wl.form), precision=kw.get("precision", 0),
                        batch_hint=kw.get("batch_hint", 0))
    qs = []
    for q in wl.qs:
        if q.shift is not None:
            qs.append(lib.Q(shift=q.shift))
        else:
            e = torch.from_numpy(np.ascontiguousarray(q.eps_kq)).to(dev)
            c = None if (q.c_kq is None or wl.cma) else torch.from_numpy(np.ascontiguousarray(q.c_kq)).to(dev)
            qs.append(lib.Q(eps_kq=e, c_kq=c))
    return plan, qs


def _relerr(got, ref):
    """Largest per-result error (tests/metrics.py)."""
    return max_err(got, ref)


def _say(*a):
    print(*a, flush=True)


def test_matrix_elements_match_plain_contraction():
    """K_A (FP64 MFMA) against |conj(C(k))^T C(k+q)|^2 computed with numpy."""
    torch = _torch()
    m = synth.tetragonal_two_site_model(2)
    wl = synth.model_workload(m, (8, 8, 4), [np.array([0.13, 0.31, 0.07])], np.zeros(1), static=True)
    wl.band_lo, wl.band_hi = 1, 9
    plan, qs = _plan(wl)
    _say("matrix elements 8x8x4, window [1,9)")
    W = plan.matrix_elements(qs[0]).cpu().numpy()
    ck = wl.c_k[:, :, 1:9]
    ckq = wl.qs[0].c_kq[:, :, 1:9]
    M = np.einsum("kon,kom->nmk", ck.conj(), ckq)
    ref = np.abs(M) ** 2
    assert np.max(np.abs(W - ref)) < 1e-13


def test_matrix_elements_shift_mode_and_wide_window():
    """Commensurate shift, 20 orbitals / 20 bands (two 16-wide band tiles, 5 orbital steps)."""
    torch = _torch()
    m = synth.random_model("tetragonal", 9, 20)
    wl = synth.model_workload(m, (4, 4, 3), None, np.zeros(1), shifts=[(1, 3, 2)], static=True)
    plan, qs = _plan(wl)
    _say("matrix elements shift mode 20 bands")
    W = plan.matrix_elements(qs[0]).cpu().numpy()
    n = wl.nk
    idx = np.arange(wl.n_k).reshape(n)
    kq = np.roll(idx, shift=(-1, -3, -2), axis=(0, 1, 2)).ravel()
    M = np.einsum("kon,kom->nmk", wl.c_k.conj(), wl.c_k[kq])
    assert np.max(np.abs(W - np.abs(M) ** 2)) < 1e-13


def test_static_sc_cma_full_config():
    """Single-band SC model, CMA, 16^3 mesh, all 8 q (7 mesh shifts + 1 explicit)."""
    wl = synth.make_workload("sc_cma")
    plan, qs = _plan(wl)
    _say("static sc_cma 16^3, 8 q")
    got = plan.static(qs).cpu().numpy()
    ref = np.array([oracle.chi0(wl, i)[0].real for i in range(len(wl.qs))])
    for i in range(len(ref)):
        assert abs(got[i] - ref[i]) <= TOL * abs(ref[i]), (i, got[i], ref[i])


@pytest.mark.parametrize("form", [0, 1])
def test_static_tetragonal_matrix_elements(form):
    """10-orbital two-site model, all 100 band pairs, explicit k+q, ragged mesh 12x10x3."""
    wl = synth.make_workload("tetra_static", nk=(12, 10, 3), nq=16, q_subset=[0, 5, 11, 15])
    wl.form = form
    plan, qs = _plan(wl)
    _say("static tetragonal 12x10x3 form", form)
    got = plan.static(qs).cpu().numpy()
    for i in range(len(wl.qs)):
        ref = oracle.chi0(wl, i)[0].real
        assert abs(got[i] - ref) <= TOL * abs(ref), (i, got[i], ref)


@pytest.mark.parametrize("form", [0, 1])
def test_dynamic_tetragonal(form):
    torch = _torch()
    wl = synth.make_workload("tetra_dynamic", nk=(8, 8, 3), nq=8, q_subset=[1, 6], nw=80)
    wl.form = form
    om = np.concatenate([wl.omega, [-0.7, -0.05, 3.5, 25.0]])
    plan, qs = _plan(wl)
    _say("dynamic tetragonal 8x8x3 form", form, "nw", len(om))
    got = plan.dynamic(qs, torch.from_numpy(om).cuda()).cpu().numpy()
    for i in range(len(wl.qs)):
        ref = oracle.chi0(wl, i, omega=om)
        assert _relerr(got[i], ref) <= TOL, (i, _relerr(got[i], ref))


def test_dynamic_bcc_band_window():
    """9-orbital bcc model with a 7-band window (band truncation), explicit k+q."""
    torch = _torch()
    wl = synth.make_workload("bcc_dynamic", nk=(6, 6, 6), nq=8, q_subset=[2, 5], nw=64, n_keep=7)
    plan, qs = _plan(wl)
    _say("dynamic bcc 6^3 window", wl.window())
    got = plan.dynamic(qs, torch.from_numpy(wl.omega).cuda()).cpu().numpy()
    for i in range(len(wl.qs)):
        ref = oracle.chi0(wl, i)
        assert _relerr(got[i], ref) <= TOL


def test_dynamic_more_than_512_frequencies_and_shift_mode():
    """nw = 600 (two frequency launches), commensurate shift, 3-orbital model."""
    torch = _torch()
    m = synth.random_model("sc", 4, 3)
    wl = synth.model_workload(m, (5, 4, 3), None, np.linspace(-1.0, 3.0, 600), shifts=[(2, 1, 1)])
    plan, qs = _plan(wl)
    _say("dynamic 600 omega shift mode")
    got = plan.dynamic(qs, torch.from_numpy(wl.omega).cuda()).cpu().numpy()
    ref = oracle.chi0(wl, 0)
    assert _relerr(got[0], ref) <= TOL


def test_static_equals_dynamic_at_zero_and_determinism():
    torch = _torch()
    wl = synth.make_workload("tetra_static", nk=(8, 8, 2), nq=8, q_subset=[3])
    plan, qs = _plan(wl)
    _say("static vs dynamic at w=0, determinism")
    s1 = plan.static(qs).cpu().numpy()
    s2 = plan.static(qs).cpu().numpy()
    assert np.array_equal(s1, s2)
    om = torch.tensor([0.0, 0.5], dtype=torch.float64, device="cuda")
    d1 = plan.dynamic(qs, om).cpu().numpy()
    d2 = plan.dynamic(qs, om).cpu().numpy()
    assert np.array_equal(d1, d2)
    assert abs(d1[0, 0].real - s1[0]) <= 1e-13 * abs(s1[0])
    assert abs(d1[0, 0].imag) <= 1e-13 * abs(s1[0])


def test_fully_occupied_window_gives_zero():
    """A window of bands that are all below mu everywhere has no carved region: chi0 == 0."""
    torch = _torch()
    wl = synth.make_workload("tetra_static", nk=(4, 4, 2), nq=8, q_subset=[2])
    assert wl.eps_k[:3].max() < wl.mu - 0.01 and wl.qs[0].eps_kq[:3].max() < wl.mu - 0.01
    wl.band_lo, wl.band_hi = 0, 3
    plan, qs = _plan(wl)
    assert plan.static(qs).cpu().numpy()[0] == 0.0


def test_full_size_dynamic_sampled_outputs():
    """The benchmark's configuration (10-orbital model, 64x64x8 mesh, 512 w, batch launch) on
    2 of its 64 q; the oracle checks 3 sampled frequencies of each."""
    torch = _torch()
    wl = synth.make_workload("tetra_dynamic", q_subset=[7, 40], workers=8)
    plan, qs = _plan(wl)
    _say("full-size dynamic 64x64x8, 2 q x 512 w")
    got = plan.dynamic(qs, torch.from_numpy(wl.omega).cuda()).cpu().numpy()
    for i, sample in enumerate([[5, 200, 470], [64, 333, 511]]):
        ref = oracle.chi0(wl, i, omega=wl.omega[sample])
        assert _relerr(got[i][sample], ref) <= TOL, (i, got[i][sample], ref)


def test_full_size_static_sampled_q():
    """Static chi0 of the 10-orbital model on the full 64x64x8 mesh, 2 of its 256 q."""
    wl = synth.make_workload("tetra_static", q_subset=[31, 200], workers=8)
    plan, qs = _plan(wl)
    _say("full-size static 64x64x8, 2 q")
    got = plan.static(qs).cpu().numpy()
    for i in range(2):
        ref = oracle.chi0(wl, i)[0].real
        assert abs(got[i] - ref) <= TOL * abs(ref), (i, got[i], ref)


@pytest.mark.parametrize("precision,tol", [(1, 2e-5), (2, 1e-6)])
def test_matrix_elements_split_precision(precision, tol):
    """BF16x3 (1) and FP16x3 (2) split-product MFMA against the plain contraction."""
    torch = _torch()
    import paper_1407_3444_amd as lib
    m = synth.tetragonal_two_site_model(2)
    wl = synth.model_workload(m, (8, 8, 4), [np.array([0.13, 0.31, 0.07])], np.zeros(1), static=True)
    dev = torch.device("cuda:0")
    plan = lib.Chi0Plan(wl.nk, torch.from_numpy(wl.eps_k).to(dev), torch.from_numpy(wl.c_k).to(dev),
                        precision=precision)
    q = wl.qs[0]
    _say("split-precision matrix elements, precision", precision)
    W = plan.matrix_elements(lib.Q(eps_kq=torch.from_numpy(q.eps_kq).to(dev),
                                   c_kq=torch.from_numpy(q.c_kq).to(dev))).cpu().numpy()
    ref = np.abs(np.einsum("kon,kom->nmk", wl.c_k.conj(), q.c_kq)) ** 2
    err = np.max(np.abs(W - ref))
    _say("max abs W error", err)
    assert err < tol


@pytest.mark.parametrize("precision", [1, 2])
def test_dynamic_mixed_precision_error(precision):
    """Mixed form (split MFMA matrix elements, FP32 far-branch weights, FP64 fallback and
    accumulation) against the FP64 oracle: max relative error per q <= 1e-5."""
    torch = _torch()
    import paper_1407_3444_amd as lib
    wl = synth.make_workload("tetra_dynamic", nk=(10, 10, 4), nq=8, q_subset=[2, 5], nw=128)
    dev = torch.device("cuda:0")
    plan = lib.Chi0Plan(wl.nk, torch.from_numpy(wl.eps_k).to(dev), torch.from_numpy(wl.c_k).to(dev),
                        precision=precision)
    qs = [lib.Q(eps_kq=torch.from_numpy(q.eps_kq).to(dev), c_kq=torch.from_numpy(q.c_kq).to(dev)) for q in wl.qs]
    _say("dynamic mixed precision", precision)
    got = plan.dynamic(qs, torch.from_numpy(wl.omega).to(dev)).cpu().numpy()
    for i in range(len(wl.qs)):
        ref = oracle.chi0(wl, i)
        err = _relerr(got[i], ref)
        _say(f"q {i}: per-result rel err max {err:.2e}, mean {mean_err(got[i], ref):.2e}")
        assert err <= 1e-5


@pytest.mark.parametrize("precision", [1, 2])
def test_full_size_mixed_precision_sampled(precision):
    """The mixed forms in the benchmark's configuration (64x64x8 mesh, 512 w, 16-q launch) on one
    q: four sampled frequencies against the FP64 oracle, per result <= 1e-5."""
    torch = _torch()
    wl = synth.make_workload("tetra_dynamic", q_subset=[52], workers=8)
    plan, qs = _plan(wl, precision=precision)
    _say("full-size dynamic mixed precision", precision)
    got = plan.dynamic(qs, torch.from_numpy(wl.omega).cuda()).cpu().numpy()[0]
    sample = [3, 150, 301, 499]
    ref = oracle.chi0(wl, 0, omega=wl.omega[sample])
    err = _relerr(got[sample], ref)
    _say(f"per-result error {err:.2e}")
    assert err <= 1e-5


def test_dynamic_mixed_precision_degenerate_model():
    """Mixed form on the single-band cubic model (CMA, explicit k+q): its symmetric mesh makes many
    final tetrahedra with tied or nearly tied corner values, which take the FP64 fallback of the
    near branch; error against the FP64 oracle <= 1e-5 per q."""
    torch = _torch()
    import paper_1407_3444_amd as lib
    wl = synth.make_workload("sc_cma", nk=(12, 12, 12))
    wl.qs = [q for q in wl.qs if q.eps_kq is not None][:1] + [
        synth.model_workload(synth.sc_nn_model(1.0), (12, 12, 12), [np.array([0.21, 0.17, 0.07])],
                             np.zeros(1), static=True).qs[0]]
    # (w = 0 is left out: at q = (j/16)(1,1,1) some final tetrahedra have e' - e = 0 on a face)
    om = np.linspace(0.05, 6.0, 96)
    dev = torch.device("cuda:0")
    plan = lib.Chi0Plan(wl.nk, torch.from_numpy(wl.eps_k).to(dev), None, cma=True, precision=1)
    qs = [lib.Q(eps_kq=torch.from_numpy(q.eps_kq).to(dev)) for q in wl.qs]
    _say("dynamic mixed precision, cubic CMA model")
    got = plan.dynamic(qs, torch.from_numpy(om).cuda()).cpu().numpy()
    for i in range(len(wl.qs)):
        ref = oracle.chi0(wl, i, omega=om)
        err = _relerr(got[i], ref)
        _say(f"q {i}: per-result rel err max {err:.2e}, mean {mean_err(got[i], ref):.2e}")
        assert err <= 1e-5


@pytest.mark.parametrize("n_keep", [9, 7, 5])
def test_full_size_bcc_band_windows_sampled(n_keep):
    """The 9-orbital bcc model on the full 48^3 mesh (663,552 tetrahedra), one q of the (010)
    path, 512 w, with the 9-band sum and the 7- and 5-band truncations (Sec. III); the oracle
    checks 2 frequencies."""
    torch = _torch()
    wl = synth.make_workload("bcc_dynamic", q_subset=[20], n_keep=n_keep, workers=8)
    plan, qs = _plan(wl)
    _say("full-size bcc 48^3, window", wl.window())
    got = plan.dynamic(qs, torch.from_numpy(wl.omega).cuda()).cpu().numpy()
    sample = [37, 290]
    ref = oracle.chi0(wl, 0, omega=wl.omega[sample])
    assert _relerr(got[0][sample], ref) <= TOL, (got[0][sample], ref)


@pytest.mark.parametrize("nk,window", [((7, 6, 3), (1, 9)), ((64, 64, 8), (0, 10))])
def test_static_band_pairs(nk, window):
    """Static chi0 resolved by band pair against the oracle's pair-resolved sum (every pair,
    relative to the largest pair of the q) and against chi0_static (sum over pairs); the second
    case is the full 64x64x8 mesh of the 10-orbital model at the path's M-point neighbourhood."""
    torch = _torch()
    qi = [70] if nk[0] == 64 else [0, 3]
    wl = synth.make_workload("tetra_static", nk=nk, nq=256 if nk[0] == 64 else 8, q_subset=qi)
    wl.band_lo, wl.band_hi = window
    plan, qs = _plan(wl)
    _say("static band pairs", nk, window)
    got = plan.static_pairs(qs).cpu().numpy()
    tot = plan.static(qs).cpu().numpy()
    for i in range(len(wl.qs)):
        ref = oracle.chi0_pairs(wl, i)[:, :, 0].real
        err = max_err(got[i].ravel(), ref.ravel())        # per pair, floor 1e-3 of the largest pair
        _say(f"q {i}: max per-pair error {err:.2e}")
        assert err <= TOL
        assert abs(got[i].sum() - tot[i]) <= 1e-12 * abs(tot[i])


@pytest.mark.parametrize("n_spec", [300, 1500])
def test_dynamic_kk_route(n_spec):
    """The Kramers-Kronig route against the oracle's: Im (delta weights, no logarithms) against the
    analytic oracle at every requested frequency, Re against the oracle's principal-value transform
    of the same spectral grid; 1500 grid points make two imaginary-part launches (1024 + 776 with
    the 300 requested frequencies)."""
    torch = _torch()
    wl = synth.make_workload("tetra_dynamic", nk=(8, 8, 3), nq=8, q_subset=[1, 6], nw=300)
    lo_b, hi_b = 2, 8
    wl.band_lo, wl.band_hi = lo_b, hi_b
    e = wl.eps_k[lo_b:hi_b]
    ekq = np.concatenate([q.eps_kq[lo_b:hi_b] for q in wl.qs], axis=1)
    dmin, dmax = float(ekq.min() - e.max() - 0.05), float(ekq.max() - e.min() + 0.05)
    plan, qs = _plan(wl)
    om = torch.from_numpy(wl.omega).cuda()
    _say("dynamic KK route, n_spec", n_spec)
    got = plan.dynamic_kk(qs, om, n_spec, dmin, dmax).cpu().numpy()
    for i in range(len(wl.qs)):
        ref = oracle.chi0_kk(wl, i, wl.omega, n_spec, dmin, dmax)
        exact = oracle.chi0(wl, i)
        e_im = max_err(got[i].imag, exact.imag)
        e_re = max_err(got[i].real, ref.real)
        kk_vs_exact = np.max(np.abs(got[i].real - exact.real)) / np.max(np.abs(exact.real))
        _say(f"q {i}: Im err {e_im:.2e}, Re vs oracle KK {e_re:.2e}, KK Re vs analytic {kk_vs_exact:.2e}")
        assert e_im <= TOL and e_re <= TOL


@pytest.mark.parametrize("n_pw,nb,nq", [(1001, 24, 2), (998, 10, 11)])
def test_plane_wave_matrix_elements(n_pw, nb, nq):
    """Large (plane-wave) basis: the MFMA contraction (one wave per q, three real products per
    complex product) against numpy's |conj(C(k))^T C(k+q)|^2; 24 bands make 2x2 16x16 tiles (the
    last ones partial), 10 bands one partial tile; basis sizes not divisible by 4 or 8; 11 q fill
    one workgroup of q and part of a second, on a mesh (36 points) that is not a multiple of the
    8 XCDs.  Static chi0 of all q in one call (one launch of the contraction) must equal the
    calls with one q each (to rounding of the reduction partition) and the oracle within the FP64
    bar."""
    torch = _torch()
    wl = synth.plane_wave_workload((4, 3, 3), n_pw, nb, nq=nq, nw=4)
    plan, qs = _plan(wl)
    _say("plane-wave matrix elements", n_pw, nb, nq)
    n = wl.nk
    idx = np.arange(wl.n_k).reshape(n)
    for i, q in enumerate(wl.qs):
        W = plan.matrix_elements(qs[i]).cpu().numpy()
        s = q.shift
        kq = np.roll(idx, shift=(-s[0], -s[1], -s[2]), axis=(0, 1, 2)).ravel()
        M = np.einsum("kon,kom->nmk", wl.c_k.conj(), wl.c_k[kq])
        assert np.max(np.abs(W - np.abs(M) ** 2)) < 1e-13
    # all q in one launch (q-groups of one workgroup) against one q per call, and the oracle
    together = plan.static(qs).cpu().numpy()
    for i in range(nq):
        alone = plan.static([qs[i]]).cpu().numpy()
        assert abs(alone[0] - together[i]) <= 1e-13 * abs(together[i]), i
        ref = oracle.chi0(wl, i, omega=np.zeros(1))[0].real
        assert abs(together[i] - ref) <= TOL * abs(ref), (i, together[i], ref)


@pytest.mark.parametrize("precision", [1, 2])
@pytest.mark.parametrize("n_pw,nb,nq", [(1001, 24, 2), (998, 10, 11)])
def test_plane_wave_matrix_elements_split_precision(precision, n_pw, nb, nq):
    """Split-product plane-wave contraction (BF16x3 = 1, FP16x3 = 2 on the 16x16x32 MFMAs) against
    numpy's FP64 |M|^2, element by element.  With S = sum_o (|ar|+|ai|)(|br|+|bi|) over the basis,
    each real product is exact to about 2^-16 (BF16: hi and lo keep 8 bits each, the dropped lo*lo
    term is 2^-18 of the product) or 2^-21 (FP16) of its magnitude, so |dM| <= c S with c = 2^-14
    or 2^-19 (a factor 4 left for the FP32 accumulation), and |dW| <= 2|M| c S + (c S)^2."""
    torch = _torch()
    wl = synth.plane_wave_workload((4, 3, 3), n_pw, nb, nq=nq, nw=4)
    plan, qs = _plan(wl, precision=precision)
    c_eps = 2.0 ** -14 if precision == 1 else 2.0 ** -19
    _say("plane-wave split matrix elements", precision, n_pw, nb, nq)
    idx = np.arange(wl.n_k).reshape(wl.nk)
    a = np.abs(wl.c_k.real) + np.abs(wl.c_k.imag)
    worst = 0.0
    for i, q in enumerate(wl.qs):
        W = plan.matrix_elements(qs[i]).cpu().numpy()
        s = q.shift
        kq = np.roll(idx, shift=(-s[0], -s[1], -s[2]), axis=(0, 1, 2)).ravel()
        M = np.einsum("kon,kom->nmk", wl.c_k.conj(), wl.c_k[kq])
        e = c_eps * np.einsum("kon,kom->nmk", a, a[kq])
        bound = 2 * np.abs(M) * e + e * e
        ratio = np.max(np.abs(W - np.abs(M) ** 2) / bound)
        worst = max(worst, ratio)
    _say(f"largest |dW| / bound {worst:.3f}")
    assert worst <= 1.0


@pytest.mark.parametrize("precision", [1, 2])
@pytest.mark.parametrize("n_pw,nb", [(1001, 24), (998, 10)])
def test_plane_wave_packed_operands(precision, n_pw, nb):
    """A split-precision launch of 3 or more q given by mesh shifts splits the eigenvectors once into
    packed operands and reads those; a launch of fewer q splits them as it reads.  Both give the same
    operands and MFMA sequence, so the pair-resolved static chi0 of 7 q in one launch, of launches of
    3, 3 and 1 q (the packed operands filled once and reused) and of one q per call must agree to
    the rounding of the FP64 sums, and all within the mixed-form bar of the oracle."""
    torch = _torch()
    wl = synth.plane_wave_workload((4, 3, 3), n_pw, nb, nq=7, nw=4)
    plan, qs = _plan(wl, precision=precision)
    plan3, _ = _plan(wl, precision=precision, batch_hint=3)
    _say("plane-wave packed operands", precision, n_pw, nb)
    together = plan.static_pairs(qs).cpu().numpy()
    in_threes = plan3.static_pairs(qs).cpu().numpy()
    alone = np.stack([plan.static_pairs([q]).cpu().numpy()[0] for q in qs])
    scale = np.max(np.abs(alone))
    assert np.max(np.abs(together - alone)) <= 1e-13 * scale
    assert np.max(np.abs(in_threes - alone)) <= 1e-13 * scale
    for i in range(len(qs)):
        ref = oracle.chi0(wl, i, omega=np.zeros(1))[0].real
        got = together[i].sum()
        assert abs(got - ref) <= 1e-5 * abs(ref), (i, got, ref)


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_plane_wave_static(precision):
    """The plane-wave configuration at full size (12^3 mesh, 4096 plane waves, 32 bands, 16 q by
    mesh shift in one launch; the split form reads packed operands): static chi0 of two of the
    q against the oracle, within the FP64 bar (FP64) or the mixed-form bar (BF16x3)."""
    torch = _torch()
    wl = synth.plane_wave_workload((12, 12, 12), 4096, 32, 16, 1, seed=11)
    wl.static = True
    plan, qs = _plan(wl, precision=precision)
    _say("full-size plane-wave static, precision", precision)
    got = plan.static(qs).cpu().numpy()
    plan.sync()
    for i in (0, 13):
        ref = oracle.chi0(wl, i, omega=np.zeros(1))[0].real
        err = abs(got[i] - ref) / abs(ref)
        _say(f"q {i}: rel err {err:.2e}")
        assert err <= (TOL if precision == 0 else 1e-5), (i, got[i], ref)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_plane_wave_dynamic_chi0(precision):
    """chi0 with plane-wave matrix elements (300 plane waves, 6 bands) against the oracle: FP64
    within the FP64 bar, the split forms within the mixed-form bar."""
    torch = _torch()
    wl = synth.plane_wave_workload((4, 4, 3), 300, 6, nq=2, nw=40)
    plan, qs = _plan(wl, precision=precision)
    _say("plane-wave dynamic chi0, precision", precision)
    got = plan.dynamic(qs, torch.from_numpy(wl.omega).cuda()).cpu().numpy()
    for i in range(len(wl.qs)):
        ref = oracle.chi0(wl, i)
        err = _relerr(got[i], ref)
        _say(f"q {i}: per-result error {err:.2e}")
        assert err <= (TOL if precision == 0 else 1e-5)


def _host_carving_lib():
    """The kernels' carving and weight arithmetic (chi0_math.h) compiled for the host."""
    import ctypes
    import os
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    src = os.path.join(here, "hostcheck", "chi0_hostcheck.cpp")
    lib = os.path.join(here, "hostcheck", "libchi0_hostcheck_gpu.so")
    tmp = lib + ".tmp%d" % os.getpid()
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", src, "-o", tmp])
    os.replace(tmp, lib)
    hc = ctypes.CDLL(lib)
    dp = ctypes.POINTER(ctypes.c_double)
    hc.hc_unit.argtypes = [dp, dp, dp, ctypes.c_double, ctypes.c_int, dp]
    hc.hc_unit.restype = ctypes.c_int
    return hc, dp


def test_census_counts_the_evaluation():
    """chi0_census: the units with a non-empty carved region equal the oracle's (a count that does
    not depend on how a carved region is cut into tetrahedra); the final tetrahedra equal those of
    the kernels' own carving compiled for the host; every (final tetrahedron, frequency) pair is
    evaluated near, far on its own, or far as part of a list series, so near + far evaluations
    never exceed final tetrahedra x frequencies, and each far evaluation uses at least one term."""
    torch = _torch()
    hc, dp = _host_carving_lib()
    wl = synth.make_workload("tetra_dynamic", nk=(6, 6, 2), nq=8, q_subset=[3], nw=40)
    plan, qs = _plan(wl)
    om = torch.from_numpy(wl.omega).cuda()
    got = plan.census(qs, om)
    _say("census", got)
    q = wl.qs[0]
    lo, hi = wl.window()
    units = host_tets = 0
    ones = np.ones(4)
    out = np.zeros(2)
    for cell in range(wl.n_k):
        for t in range(6):
            idx = oracle.tet_corners(wl.nk, cell, t)
            for n in range(lo, hi):
                for m in range(lo, hi):
                    a = np.ascontiguousarray(wl.eps_k[n][idx] - wl.mu)
                    b = np.ascontiguousarray(q.eps_kq[m][idx] - wl.mu)
                    k = 0
                    for region in (1, 2):
                        _, vols = oracle.carve(a, b, region)
                        k += int(np.sum(vols != 0.0))
                    units += k > 0
                    host_tets += hc.hc_unit(a.ctypes.data_as(dp), b.ctypes.data_as(dp), ones.ctypes.data_as(dp),
                                            0.5, 0, out.ctypes.data_as(dp))
    assert got["active_units"] == units
    assert got["final_tetrahedra"] == host_tets
    nw = len(wl.omega)
    assert 0 < got["near_evals"] and 0 < got["far_evals"]
    assert got["near_evals"] + got["far_evals"] <= host_tets * nw
    assert got["far_terms"] >= got["far_evals"]
    # series coefficients: whole blocks of 5 terms, at most the 50 of the series per tetrahedron
    assert got["coef_terms"] % 5 == 0 and 0 < got["coef_terms"] <= 50 * host_tets


@pytest.mark.parametrize("precision,nw", [(0, 40), (0, 600), (1, 40)])
def test_dynamic_pairs_match_oracle_and_the_pair_sum(precision, nw):
    """chi0_dynamic_pairs: chi0(q, w) of every band pair (n at k, m at k+q) against the oracle's
    pair-resolved evaluation, per result against max(|ref|, 1e-3 of the largest |ref| of any pair);
    the sum over pairs equals chi0_dynamic's result to rounding in FP64 (another summation order)
    and within the mixed-form bar in the mixed form (whose FP32 series are cut and summed per list,
    and the lists differ when each pair has lists of its own); 600 frequencies take two launches."""
    torch = _torch()
    import paper_1407_3444_amd as lib
    wl = synth.make_workload("tetra_dynamic", nk=(6, 6, 2), nq=8, q_subset=[3], nw=nw)
    wl.band_lo, wl.band_hi = 2, 8
    plan, qs = _plan(wl, precision=precision)
    om = torch.from_numpy(wl.omega).cuda()
    _say("dynamic pairs, precision", precision, "nw", nw)
    got = plan.dynamic_pairs(qs, om).cpu().numpy()[0]            # [nbw][nbw][nw]
    ref = oracle.chi0_pairs(wl, 0)
    scale = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    err = np.max(np.abs(got - ref) / scale)
    _say(f"per-pair per-result error {err:.2e}")
    assert err <= (TOL if precision == 0 else 1e-5)
    total = plan.dynamic(qs, om).cpu().numpy()[0]
    bound = 1e-13 if precision == 0 else 1e-5
    assert np.max(np.abs(got.sum(axis=(0, 1)) - total)) <= bound * np.max(np.abs(total))


def test_full_size_dynamic_pairs_sampled():
    """The pair-resolved dynamic call in the benchmark's configuration (10-orbital model, 64x64x8
    mesh, 512 w, all 100 band pairs) on one q: three sampled frequencies of every pair against the
    oracle's pair-resolved evaluation, per result against max(|ref|, 1e-3 of the largest |ref|);
    the pair sum against chi0_dynamic at every frequency."""
    torch = _torch()
    wl = synth.make_workload("tetra_dynamic", q_subset=[21], workers=8)
    plan, qs = _plan(wl)
    om = torch.from_numpy(wl.omega).cuda()
    _say("full-size dynamic pairs 64x64x8, 1 q x 512 w")
    got = plan.dynamic_pairs(qs, om).cpu().numpy()[0]            # [nbw][nbw][nw]
    sample = [17, 256, 490]
    ref = oracle.chi0_pairs(wl, 0, omega=wl.omega[sample])
    g = got[:, :, sample]
    scale = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    err = np.max(np.abs(g - ref) / scale)
    _say(f"per-pair per-result error {err:.2e}")
    assert err <= TOL
    total = plan.dynamic(qs, om).cpu().numpy()[0]
    assert np.max(np.abs(got.sum(axis=(0, 1)) - total)) <= 1e-13 * np.max(np.abs(total))


def test_dynamic_pairs_rejects_list_plans():
    torch = _torch()
    import paper_1407_3444_amd as lib
    dev = torch.device("cuda:0")
    eps = torch.zeros((1, 4), dtype=torch.float64, device=dev)
    tets = torch.tensor([[0, 1, 2, 3]], dtype=torch.int32, device=dev)
    plan = lib.Chi0Plan(None, eps, None, cma=True, tetrahedra=(tets, 1.0))
    q = lib.Q(eps_kq=eps.clone())
    with pytest.raises(lib.Chi0Error) as e:
        plan.dynamic_pairs([q], torch.zeros(4, dtype=torch.float64, device=dev))
    assert e.value.status == -7


def test_nonfinite_frequency_only_affects_itself():
    """A NaN or infinite frequency does not stop the call: a NaN gives NaN at its own frequency and
    leaves every other one bit for bit unchanged; an infinite frequency (whose own value is not
    meaningful) widens the frequency interval the series are cut for, and the other frequencies
    keep the FP64 bar.  The input scan reports both at the next synchronisation."""
    torch = _torch()
    import paper_1407_3444_amd as lib
    wl = synth.make_workload("tetra_dynamic", nk=(6, 6, 2), nq=8, q_subset=[3], nw=40)
    plan, qs = _plan(wl)
    om = wl.omega.copy()
    ref = plan.dynamic(qs, torch.from_numpy(om).cuda()).cpu().numpy()[0]
    plan.sync()
    keep = np.ones(len(om), bool)
    keep[7] = False
    bad = om.copy()
    bad[7] = np.nan
    got = plan.dynamic(qs, torch.from_numpy(bad).cuda()).cpu().numpy()[0]
    with pytest.raises(lib.Chi0Error) as e:
        plan.sync()
    assert e.value.status == -3 and "frequencies" in str(e.value)
    assert np.array_equal(got[keep], ref[keep])
    assert np.isnan(got[7].real)
    bad[7] = np.inf
    got = plan.dynamic(qs, torch.from_numpy(bad).cuda()).cpu().numpy()[0]
    with pytest.raises(lib.Chi0Error) as e:
        plan.sync()
    assert e.value.status == -3
    assert np.max(np.abs(got[keep] - ref[keep])) <= TOL * np.max(np.abs(ref[keep]))


def test_frequencies_on_corner_values_and_widest_window():
    """Frequencies equal to corner values e' - e of the mesh (a node of the divided differences at
    w exactly), and the widest band window (32 bands of a 32-orbital model: 2x2 tiles of the
    matrix elements, 1024 band pairs), against the oracle."""
    torch = _torch()
    wl = synth.make_workload("tetra_dynamic", nk=(6, 6, 2), nq=8, q_subset=[3], nw=8)
    q = wl.qs[0]
    rng = np.random.default_rng(5)
    D = (q.eps_kq[:, None, :] - wl.eps_k[None, :, :]).ravel()
    on = np.sort(rng.choice(D[(D > 0.05) & (D < 2.0)], 12, replace=False))
    wl.omega = np.concatenate([on, [0.0]])
    plan, qs = _plan(wl)
    got = plan.dynamic(qs, torch.from_numpy(wl.omega).cuda()).cpu().numpy()[0]
    ref = oracle.chi0(wl, 0)
    assert np.all(np.isfinite(got))
    assert _relerr(got, ref) <= TOL
    m = synth.random_model("tetragonal", 77, 32)
    wl = synth.model_workload(m, (4, 4, 3), [np.array([0.13, 0.07, 0.21])], synth.omega_grid(24))
    assert wl.window() == (0, 32)
    plan, qs = _plan(wl)
    got = plan.dynamic(qs, torch.from_numpy(wl.omega).cuda()).cpu().numpy()[0]
    ref = oracle.chi0(wl, 0)
    assert _relerr(got, ref) <= TOL


def _lindhard_static(q, kf):
    """Free-electron static Lindhard function (m = hbar = 1, g_s = 2, per unit volume)."""
    x = q / (2 * kf)
    return -kf / np.pi ** 2 * (0.5 + (1 - x * x) / (4 * x) * np.log(abs((1 + x) / (1 - x))))


def test_free_electron_gamma_r_static_against_oracle_and_lindhard():
    """The free-electron variant of the single-band configuration: eps = k^2/2 on the 16^3 index
    mesh spanning [-pi, pi)^3, k_F = pi/2, the Eq. (1) form (region e < mu < e' only, so the
    Fermi sphere at k+q never needs to fit the box), explicit k+q data at the 8 points
    q_j = (j/16)(1,1,1) of Gamma-R (reciprocal lattice 2 pi).  Every value within 1e-10 of the
    oracle; both within the linear-tetrahedron discretisation error of the Lindhard closed form
    (the oracle's own pin shows it falling as h^2)."""
    torch = _torch()
    import paper_1407_3444_amd as lib
    nk = (16, 16, 16)
    kf = np.pi / 2
    e = synth.free_electron_eps(nk)
    dev = torch.device("cuda:0")
    plan = lib.Chi0Plan(nk, torch.from_numpy(e).to(dev), None, mu=kf ** 2 / 2, cma=True, form=1)
    qs, qcart = [], []
    for j in range(1, 9):
        qc = np.full(3, j / 16 * 2 * np.pi)
        qcart.append(qc)
        qs.append(lib.Q(eps_kq=torch.from_numpy(synth.free_electron_eps(nk, qc)).to(dev)))
    _say("free electrons 16^3, Gamma-R, form 1")
    got = plan.static(qs).cpu().numpy()
    for j, qc in enumerate(qcart):
        ref = oracle.chi0_raw(nk, e, None, [0.0], eps_kq=synth.free_electron_eps(nk, qc), mu=kf ** 2 / 2,
                              cma=True, form=1)[0].real
        lind = _lindhard_static(np.linalg.norm(qc), kf)
        _say(f"q {j + 1}: gpu {got[j]:.12e} oracle {ref:.12e} Lindhard {lind:.6e}")
        assert abs(got[j] - ref) <= TOL * abs(ref), (j, got[j], ref)
        # 16^3 discretisation error: 1.5% near q = 0, up to 6% past 2 k_F (the kink of the Lindhard
        # function); the oracle pin shows it falling as h^2 on finer meshes
        assert abs(got[j] - lind) <= 0.07 * abs(lind), (j, got[j], lind)


def test_full_size_dynamic_q_in_the_last_launch():
    """The benchmark's configuration with 20 q: two launch sequences (16 + 4 q); a q of the second
    one is checked against the oracle at 3 frequencies, a q of the first at 1."""
    torch = _torch()
    wl = synth.make_workload("tetra_dynamic", q_subset=list(range(44, 64)), workers=8)
    plan, qs = _plan(wl)
    _say("full-size dynamic 64x64x8, 20 q x 512 w (launches of 16 + 4 q)")
    got = plan.dynamic(qs, torch.from_numpy(wl.omega).cuda()).cpu().numpy()
    for i, sample in ((18, [3, 257, 508]), (5, [130])):
        ref = oracle.chi0(wl, i, omega=wl.omega[sample])
        err = _relerr(got[i][sample], ref)
        _say(f"q index {44 + i}: max per-result error {err:.2e}")
        assert err <= TOL, (i, got[i][sample], ref)


def test_band_truncation_sub_windows_from_pair_resolved_output():
    """Band truncation (Sec. III: sums over the bands near the Fermi level): the pair-resolved static
    chi0 of the full 9-band window of the bcc model, summed over the (n, m) block of a narrower
    window, is chi0 of that window; checked against the oracle for the 5- and 7-band windows of the
    window rule (mean energy closest to mu) and two off-centre windows."""
    torch = _torch()
    wl = synth.make_workload("bcc_dynamic", nk=(8, 8, 8), nq=8, q_subset=[1, 5], nw=8, n_keep=9)
    wl.static = True
    plan, qs = _plan(wl)
    _say("band-truncation windows from pairs, bcc 8^3")
    pairs = plan.static_pairs(qs).cpu().numpy()
    windows = [synth.band_window(wl.eps_k, 5, wl.mu), synth.band_window(wl.eps_k, 7, wl.mu), (0, 4), (6, 9)]
    for i in range(len(wl.qs)):
        for lo, hi in windows:
            got = pairs[i, lo:hi, lo:hi].sum()
            wl.band_lo, wl.band_hi = lo, hi
            ref = oracle.chi0(wl, i, omega=[0.0])[0].real
            wl.band_lo, wl.band_hi = 0, 9
            assert abs(got - ref) <= TOL * max(abs(ref), 1e-3 * abs(pairs[i].sum())), (i, lo, hi, got, ref)
