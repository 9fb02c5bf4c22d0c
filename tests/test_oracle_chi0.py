"""Pins for the whole oracle chi0(q, omega) (CPU only).

Each test ties the oracle to something the paper or the mathematics fixes:
the free-electron Lindhard function, the q -> 0 limit -N(E_F) (the paper's
"stringent test", Sec. III), exact large-omega moments, the sum rules and the
Kramers-Kronig relation between Re and Im (Sec. II), the antisymmetry of
Im chi0 in omega (Eq. (3)), the equivalence of the paper's one-sided Eq. (1)
with the occupation-difference form, G-periodicity under the constant
matrix-element approximation (Sec. III) and brute-force k sums.
"""
import numpy as np
import pytest
from scipy import integrate
from scipy.interpolate import CubicSpline

import oracle
import synth


KF = np.pi / 2


def _lindhard_static(q):
    """Free-electron static Lindhard function (m = hbar = 1, g_s = 2, per unit volume)."""
    x = q / (2 * KF)
    nf = KF / np.pi ** 2
    return -nf * (0.5 + (1 - x * x) / (4 * x) * np.log(abs((1 + x) / (1 - x))))


def _free_electron_chi0(N, qvec, omega, form=1):
    nk = (N, N, N)
    e = synth.free_electron_eps(nk)
    ekq = synth.free_electron_eps(nk, qvec)
    return oracle.chi0_raw(nk, e, None, omega, eps_kq=ekq, mu=KF ** 2 / 2, cma=True, form=form)


@pytest.mark.parametrize("q", [0.3, 1.0, 2.5])
def test_free_electron_static_lindhard_converges(q):
    """Eq. (1) form on eps = k^2/2: error against the Lindhard closed form falls as h^2."""
    errs = []
    for N in (16, 32):
        val = _free_electron_chi0(N, np.array([q, 0.0, 0.0]), [0.0])[0].real
        errs.append(abs(val - _lindhard_static(q)))
    assert errs[1] < errs[0] / 3.0
    assert errs[1] < 1e-3


def _free_electron_im(q, w):
    """Im chi0 of free electrons for w > 0 (Eq. (2)): -pi g_s/(2pi)^3 int d^3k delta(w - q k_z - q^2/2)
    over |k| < kF < |k + q|, i.e. (1/q) times the area of the allowed disk at k_z = (w - q^2/2)/q."""
    kz = (w - q * q / 2) / q
    area = np.pi * (max(0.0, KF ** 2 - kz ** 2) - max(0.0, KF ** 2 - (kz + q) ** 2))
    area = max(area, 0.0)
    return -np.pi * 2.0 / (2 * np.pi) ** 3 * area / q


def test_free_electron_dynamic_im_converges():
    q = 0.8
    ws = np.array([0.2, 0.6, 1.1, 1.6])
    ref = np.array([_free_electron_im(q, w) for w in ws])
    errs = []
    for N in (16, 32):
        val = _free_electron_chi0(N, np.array([0.0, q, 0.0]), ws).imag
        errs.append(np.max(np.abs(val - ref)))
    assert errs[1] < errs[0] / 2.5
    assert errs[1] < 0.05 * np.max(np.abs(ref))


def _tet_dos(nk, eps, mu, spin=2.0):
    """Textbook linear-tetrahedron density of states at mu (Lehmann-Taut form)."""
    nb = eps.shape[0]
    Nk = int(np.prod(nk))
    tot = 0.0
    for cell in range(Nk):
        for t in range(6):
            idx = oracle.tet_corners(nk, cell, t)
            for n in range(nb):
                e1, e2, e3, e4 = np.sort(eps[n, idx])
                E = mu
                if E <= e1 or E >= e4:
                    continue
                if E < e2:
                    g = 3 * (E - e1) ** 2 / ((e2 - e1) * (e3 - e1) * (e4 - e1))
                elif E < e3:
                    g = (3 * (e2 - e1) + 6 * (E - e2)
                         - 3 * (e3 - e1 + e4 - e2) * (E - e2) ** 2 / ((e3 - e2) * (e4 - e2))) / ((e3 - e1) * (e4 - e1))
                else:
                    g = 3 * (e4 - E) ** 2 / ((e4 - e1) * (e4 - e2) * (e4 - e3))
                tot += g
    return spin * tot / (6 * Nk)


def test_q_to_zero_gives_minus_dos():
    """chi0(h q_hat, 0) -> -N(E_F) of the same tetrahedron mesh (with matrix elements)."""
    nk = (6, 6, 4)
    m = synth.tetragonal_two_site_model(2)
    kf = synth.mesh_kfrac(nk)
    eps, c = synth.eigensystem(m, kf)
    N = _tet_dos(nk, eps, 0.0)
    assert N > 0.1
    qhat = np.array([0.6, 0.3, 0.1]) / np.linalg.norm([0.6, 0.3, 0.1])
    errs = []
    for h in (1e-3, 1e-4):
        ekq, ckq = synth.eigensystem(m, kf + h * qhat)
        errs.append(abs(oracle.chi0_raw(nk, eps, c, [0.0], eps_kq=ekq, c_kq=ckq)[0].real + N))
    assert errs[1] < errs[0] / 5
    assert errs[1] < 1e-4 * N


def _small_tr_workload(nk=(4, 4, 3), shift=(1, 2, 1), omega=(0.0,), seed=7, n_orb=3):
    m = synth.random_model("tetragonal", seed, n_orb)
    return synth.model_workload(m, nk, None, np.asarray(omega, float), shifts=[shift])


def test_large_omega_moments():
    """At |w| far above the spectrum of D: chi0 = sum_p mom[p] / w^(p+1), with the moments
    integrated exactly (polynomials on the carved tetrahedra)."""
    wl = _small_tr_workload(omega=(-300.0, 250.0, 400.0))
    mom = oracle.moments(wl, 0, pmax=7)
    val = oracle.chi0(wl, 0)
    for w, v in zip(wl.omega, val):
        series = sum(mom[p] / w ** (p + 1) for p in range(8))
        assert abs(v.real - series) < 1e-12 * abs(series)
        assert abs(v.imag) < 1e-14 * abs(series)


def test_eq1_form_equals_difference_form_under_time_reversal():
    """Real hoppings, commensurate q, centrally symmetric triangulation: the paper's one-sided
    Eq. (1)/(2) and the occupation-difference form agree exactly."""
    wl = _small_tr_workload(omega=(-1.3, -0.2, 0.0, 0.35, 1.7))
    d = oracle.chi0(wl, 0, form=0)
    e = oracle.chi0(wl, 0, form=1)
    np.testing.assert_allclose(e, d, rtol=1e-11, atol=1e-13 * np.max(np.abs(d)))


def test_eq3_im_odd_re_even_in_omega():
    """Eq. (3): Im chi0(q,-w) = -Im chi0(q,w) (and Re is even) under time reversal."""
    ws = np.array([0.15, 0.6, 1.1, 2.3])
    wl = _small_tr_workload(omega=np.concatenate([ws, -ws]))
    v = oracle.chi0(wl, 0)
    pos, neg = v[:4], v[4:]
    scale = np.max(np.abs(v))
    np.testing.assert_allclose(neg.imag, -pos.imag, atol=1e-12 * scale)
    np.testing.assert_allclose(neg.real, pos.real, atol=1e-12 * scale)
    assert np.all(pos.imag <= 1e-15 * scale)


def _fine_grid_workload():
    m = synth.random_model("sc", 21, 2)
    return synth.model_workload(m, (4, 4, 3), [np.array([0.13, 0.27, 0.05])], np.zeros(1))


def test_sum_rules_zeroth_and_first_moment():
    """int Im chi0 dw = -pi mom[0] and the f-sum int w Im chi0 dw = -pi mom[1]."""
    wl = _fine_grid_workload()
    mom = oracle.moments(wl, 0, pmax=1)
    lo = float(np.min(wl.eps_k) - np.max(wl.qs[0].eps_kq)) - 0.01
    hi = float(np.max(wl.qs[0].eps_kq) - np.min(wl.eps_k)) + 0.01
    ws = np.linspace(lo, hi, 4001)
    im = oracle.chi0(wl, 0, omega=ws).imag
    i0 = integrate.simpson(im, x=ws)
    i1 = integrate.simpson(ws * im, x=ws)
    assert abs(i0 + np.pi * mom[0]) < 3e-5 * abs(np.pi * mom[0])
    assert abs(i1 + np.pi * mom[1]) < 3e-5 * abs(np.pi * mom[1])


def test_kramers_kronig():
    """Re chi0(w0) = -(1/pi) PV int Im chi0(w') / (w0 - w') dw' (retarded response)."""
    wl = _fine_grid_workload()
    lo = float(np.min(wl.eps_k) - np.max(wl.qs[0].eps_kq)) - 0.01
    hi = float(np.max(wl.qs[0].eps_kq) - np.min(wl.eps_k)) + 0.01
    ws = np.linspace(lo, hi, 4001)
    im = oracle.chi0(wl, 0, omega=ws).imag
    spl = CubicSpline(ws, im)
    for w0 in [lo + 0.31 * (hi - lo), lo + 0.55 * (hi - lo), hi + 0.7]:
        re = oracle.chi0(wl, 0, omega=[w0])[0].real
        if lo < w0 < hi:
            pv = integrate.quad(spl, lo, hi, weight="cauchy", wvar=w0, limit=400)[0]
        else:
            pv = integrate.quad(lambda x: spl(x) / (x - w0), lo, hi, limit=400)[0]
        kk = (1.0 / np.pi) * pv      # -(1/pi) PV int Im/(w0 - w') = (1/pi) PV int Im/(w' - w0)
        assert abs(re - kk) < 2e-4 * max(abs(re), 1e-3)


def test_cma_is_g_periodic_and_matrix_elements_are_gauge_free():
    """Under CMA chi0(q + G) = chi0(q) (Sec. III); with matrix elements the eigenpairs at k+q+G
    equal those at k+q in the periodic gauge, so chi0 is unchanged too."""
    m = synth.random_model("tetragonal", 5, 3)
    nk = (4, 4, 2)
    q = np.array([0.21, 0.37, 0.11])
    a = synth.model_workload(m, nk, [q, q + np.array([1.0, 0.0, 0.0]), q + np.array([0.0, -1.0, 1.0])],
                             np.array([0.0, 0.8]))
    ref = oracle.chi0(a, 0)
    for i in (1, 2):
        np.testing.assert_allclose(oracle.chi0(a, i), ref, rtol=1e-10, atol=1e-13)
    a.cma = True
    ref = oracle.chi0(a, 0)
    for i in (1, 2):
        np.testing.assert_allclose(oracle.chi0(a, i), ref, rtol=1e-10, atol=1e-13)


def test_static_signs():
    """Re chi0(q, 0) <= 0 for every q (both regions contribute negatively at w = 0)."""
    wl = synth.make_workload("sc_cma", nk=(8, 8, 8), nq=3)
    for i in range(len(wl.qs)):
        v = oracle.chi0(wl, i)[0]
        assert v.real < 0 and abs(v.imag) < 1e-14


def _fermi(x, T):
    return 0.5 * (1.0 - np.tanh(x / (2.0 * T)))


def _brute_static_sc(q, M, T):
    """(g_s/M) sum_k (f(e_k) - f(e_k+q)) / (e_k - e_k+q) on an M^3 offset grid at temperature T
    (the ratio stays bounded, so the plain k sum converges)."""
    g = (np.arange(M) + 0.5) / M
    k1, k2 = np.meshgrid(g, g, indexing="ij")
    tot = 0.0
    for k3 in g:
        e = -2 * (np.cos(2 * np.pi * k1) + np.cos(2 * np.pi * k2) + np.cos(2 * np.pi * k3))
        ep = -2 * (np.cos(2 * np.pi * (k1 + q[0])) + np.cos(2 * np.pi * (k2 + q[1]))
                   + np.cos(2 * np.pi * (k3 + q[2])))
        D = ep - e
        tiny = np.abs(D) < 1e-9
        ratio = np.where(tiny, -1.0 / (4 * T * np.cosh(e / (2 * T)) ** 2),
                         (_fermi(e, T) - _fermi(ep, T)) / np.where(tiny, 1.0, e - ep))
        tot += ratio.sum()
    return 2.0 * tot / M ** 3


def test_brute_force_dense_k_sum():
    """Single-band SC model, static, CMA: dense k sums at T = 0.1 and 0.05, extrapolated to
    T = 0 in T^2 (Sommerfeld), against the tetrahedron result: the error falls with the
    mesh and is below 2e-3 on 48^3."""
    q = np.array([0.23, 0.11, 0.03])
    b1, b2 = _brute_static_sc(q, 160, 0.1), _brute_static_sc(q, 160, 0.05)
    brute = b2 + (b2 - b1) / 3.0
    m = synth.sc_nn_model(1.0)
    errs = []
    for N in (24, 48):
        wl = synth.model_workload(m, (N, N, N), [q], np.zeros(1), static=True)
        wl.cma = True
        errs.append(abs(oracle.chi0(wl, 0)[0].real - brute))
    assert errs[1] < errs[0] / 3.0
    assert errs[1] < 2e-3 * abs(brute)


def test_band_pair_resolution_sums_to_chi0_and_matches_band_windows():
    """chi0 resolved by band pair (the band-transition histogram of Sec. III): the pairs sum to
    the total, every diagonal pair (n, n) equals chi0 over the one-band window [n, n+1), every
    2x2 block equals chi0 over the two-band window, and every static pair is <= 0 (both carved
    regions give negative terms at w = 0)."""
    m = synth.tetragonal_two_site_model(2)
    wl = synth.model_workload(m, (6, 6, 3), [np.array([0.17, 0.05, 0.11])], np.array([0.0, 0.4, 1.3]))
    wl.band_lo, wl.band_hi = 2, 8
    P = oracle.chi0_pairs(wl, 0)
    tot = oracle.chi0(wl, 0)
    assert np.max(np.abs(P.sum(axis=(0, 1)) - tot)) <= 1e-13 * np.max(np.abs(tot))
    for n in range(6):
        wl1 = synth.model_workload(m, (6, 6, 3), [np.array([0.17, 0.05, 0.11])], wl.omega)
        wl1.band_lo, wl1.band_hi = 2 + n, 3 + n
        ref = oracle.chi0(wl1, 0)
        assert np.max(np.abs(P[n, n] - ref)) <= 1e-13 * max(np.max(np.abs(ref)), 1e-300)
    wl2 = synth.model_workload(m, (6, 6, 3), [np.array([0.17, 0.05, 0.11])], wl.omega)
    wl2.band_lo, wl2.band_hi = 4, 6
    ref = oracle.chi0(wl2, 0)
    assert np.max(np.abs(P[2:4, 2:4].sum(axis=(0, 1)) - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert np.all(P[:, :, 0].real <= 1e-15)


def test_band_pair_orientation_n_at_k_m_at_k_plus_q():
    """Pair (n, m) takes band n at k and band m at k+q.  With a gapped two-band model (band 0
    filled, band 1 empty) only transitions 0 -> 1 absorb at w > 0: Im chi0_01 < 0 there while
    Im chi0_10 vanishes identically (its region e'_0 < mu < e_1 has D = e'_0 - e_1 < 0)."""
    hop = {}
    synth._add_pair(hop, (0, 0, 0), np.diag([-1.5, 1.5]))
    synth._add_pair(hop, (1, 0, 0), np.array([[-0.2, 0.05], [0.05, 0.25]]))
    synth._add_pair(hop, (0, 1, 0), np.array([[-0.15, 0.0], [0.03, 0.2]]))
    synth._add_pair(hop, (0, 0, 1), np.array([[-0.1, 0.02], [0.0, 0.15]]))
    model = synth.TBModel("gapped2", 2, hop)
    om = np.linspace(0.5, 5.0, 40)
    wl = synth.model_workload(model, (6, 6, 6), [np.array([0.13, 0.21, 0.07])], om)
    assert wl.eps_k[0].max() < 0.0 < wl.eps_k[1].min()
    P = oracle.chi0_pairs(wl, 0)
    assert np.all(P[1, 0].imag == 0.0) and np.all(P[0, 0] == 0.0) and np.all(P[1, 1] == 0.0)
    assert P[0, 1].imag.min() < -1e-3 * np.abs(P[0, 1]).max()


def test_kk_tent_transform_of_the_semicircle():
    """The discrete principal-value transform of the Kramers-Kronig route against a closed-form
    Hilbert pair: G(w) = 2 (w - sqrt(w^2 - 1)) has Im G = -2 sqrt(1 - w^2) on |w| < 1 and
    Re G = 2 w there, 2 (w - sign(w) sqrt(w^2 - 1)) outside; the error falls with the spacing."""
    om = np.array([-1.7, -0.8, -0.3, 0.0, 0.45, 0.9, 1.3, 2.5])
    ref = np.where(np.abs(om) < 1, 2 * om, 2 * (om - np.sign(om) * np.sqrt(np.maximum(om * om - 1, 0))))
    errs = []
    for n in (201, 801, 3201):
        grid = np.linspace(-1.0, 1.0, n)
        im = -2.0 * np.sqrt(np.maximum(1.0 - grid ** 2, 0.0))
        re = oracle.kk_tent_matrix(om, -1.0, 1.0, n) @ im / np.pi
        errs.append(np.max(np.abs(re - ref)))
    assert errs[2] < 2e-3 and errs[2] < errs[1] / 3 < errs[0] / 9


def test_kk_route_converges_to_the_analytic_real_part():
    """Re chi0 from the Kramers-Kronig route on a grid covering the whole spectrum against the
    analytic Re of the same oracle: the difference is the interpolation error of Im and falls
    as the spectral grid is refined."""
    m = synth.tetragonal_two_site_model(2)
    wl = synth.model_workload(m, (6, 6, 2), [np.array([0.21, 0.08, 0.0])], np.zeros(1))
    wl.band_lo, wl.band_hi = 3, 7
    lo, hi = wl.window()
    e = wl.eps_k[lo:hi]
    ekq = wl.qs[0].eps_kq[lo:hi]
    dmin, dmax = ekq.min() - e.max() - 0.05, ekq.max() - e.min() + 0.05
    om = np.linspace(-0.5, 1.5, 9)
    exact = oracle.chi0(wl, 0, omega=om)
    errs = []
    for n in (400, 1600):
        kk = oracle.chi0_kk(wl, 0, om, n, dmin, dmax)
        assert np.max(np.abs(kk.imag - exact.imag)) <= 1e-13 * np.max(np.abs(exact))
        errs.append(np.max(np.abs(kk.real - exact.real)) / np.max(np.abs(exact.real)))
    assert errs[1] < 2e-2 and errs[1] < errs[0] / 2
