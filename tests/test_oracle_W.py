"""Pins of the oracle's matrix-element weights W_nm(k) = |<n,k|m,k+q>|^2 (the tight-binding
matrix element of the footnote in Sec. III, taken as the modulus of an overlap, with n at k and m at
k+q as in Eq. (1)).

What fixes W independently of the oracle's own formula:
  * with every band kept, U = C(k)^H C(k+q) is unitary, so W = |U|^2 is unistochastic: every row
    and every column sums to one (a wrong orbital or band stride, or a missing modulus, breaks it);
  * at q = 0 (mod G) U = C(k)^H C(k) = 1, so W is the identity for non-degenerate bands (a dropped
    complex conjugate breaks it: C^T C is not the identity for complex eigenvectors);
  * a single orbital has unit-modulus eigenvectors, so W = 1 and chi0 equals its constant
    matrix-element value exactly;
  * the orientation (n at k, m at k+q) is fixed by a hand-built three-orbital case whose W is not
    symmetric: with C(k) = 1 and C(k+q) a cyclic permutation with phases, W = |P|^2 exactly, and the
    chi0 of flat bands is then a closed form that the swapped orientation misses.  (With two
    orbitals and both bands kept W is doubly stochastic and 2 x 2, hence symmetric, so the
    orientation needs three.)
"""
import numpy as np
import pytest

import oracle
import synth


def _tetragonal(nk, q):
    model = synth.tetragonal_two_site_model(2)
    kf = synth.mesh_kfrac(nk)
    e, c = synth.eigensystem(model, kf)
    ekq, ckq = synth.eigensystem(model, kf + np.asarray(q)[None, :])
    return e, c, ekq, ckq


def test_W_is_unistochastic_with_all_bands():
    nk = (4, 4, 2)
    _, c, _, ckq = _tetragonal(nk, [0.137, -0.291, 0.412])
    W = oracle.matrix_elements_raw(nk, c, c_kq=ckq)
    assert W.shape == (10, 10, 32)
    assert np.all(W >= 0.0) and np.all(W <= 1.0 + 1e-12)
    np.testing.assert_allclose(W.sum(axis=1), 1.0, rtol=0, atol=1e-12)   # rows: sum over m at k+q
    np.testing.assert_allclose(W.sum(axis=0), 1.0, rtol=0, atol=1e-12)   # columns: sum over n at k
    # a generic q mixes the bands: W is far from a permutation
    assert W.max(axis=1).min() < 0.99


def test_W_window_is_a_block_of_the_full_W():
    nk = (3, 3, 2)
    _, c, _, ckq = _tetragonal(nk, [0.3, 0.1, 0.2])
    full = oracle.matrix_elements_raw(nk, c, c_kq=ckq)
    win = oracle.matrix_elements_raw(nk, c, c_kq=ckq, band_lo=3, band_hi=7)
    np.testing.assert_array_equal(win, full[3:7, 3:7])
    # a window loses weight to the bands outside it: rows sum to at most one
    assert np.all(win.sum(axis=1) <= 1.0 + 1e-12)


@pytest.mark.parametrize("shift", [(0, 0, 0), (4, 0, 0), (0, 8, 2)])
def test_W_is_identity_at_q_equivalent_to_zero(shift):
    nk = (4, 4, 2)
    model = synth.tetragonal_two_site_model(2)
    e, c = synth.eigensystem(model, synth.mesh_kfrac(nk))
    assert np.min(np.diff(e, axis=0)) > 1e-6          # non-degenerate bands at every k
    W = oracle.matrix_elements_raw(nk, c, shift=shift)
    eye = np.broadcast_to(np.eye(10)[:, :, None], W.shape)
    np.testing.assert_allclose(W, eye, rtol=0, atol=1e-12)


def test_single_orbital_W_is_one_and_chi0_equals_the_constant_matrix_element_value():
    nk = (6, 6, 6)
    model = synth.sc_nn_model(1.0)
    kf = synth.mesh_kfrac(nk)
    q = np.array([0.21, 0.07, 0.33])
    e, _ = synth.eigensystem(model, kf)
    ekq, _ = synth.eigensystem(model, kf + q[None, :])
    rng = np.random.default_rng(4)
    # arbitrary gauge phases: the single-orbital eigenvector is a phase
    c = np.exp(2j * np.pi * rng.random((kf.shape[0], 1, 1)))
    ckq = np.exp(2j * np.pi * rng.random((kf.shape[0], 1, 1)))
    W = oracle.matrix_elements_raw(nk, c, c_kq=ckq)
    np.testing.assert_allclose(W, 1.0, rtol=0, atol=1e-14)
    om = np.array([0.0, 0.4, 1.3, 3.0])
    with_me = oracle.chi0_raw(nk, e, c, om, eps_kq=ekq, c_kq=ckq, mu=0.3)
    cma = oracle.chi0_raw(nk, e, None, om, eps_kq=ekq, mu=0.3, cma=True)
    np.testing.assert_allclose(with_me, cma, rtol=1e-13, atol=1e-15)


def _cyclic_case(nk=(2, 2, 2)):
    """Three flat bands; C(k) = 1 and C(k+q) = P with P[o, m] = phase_m if o = (m - 1) mod 3, so that
    <n,k|m,k+q> = P[n, m] and W[n, m] = 1 exactly for (n, m) in {(0, 1), (1, 2), (2, 0)}."""
    nkt = int(np.prod(nk))
    e = np.array([-1.0, 0.5, 2.0])          # at k: band 0 occupied, bands 1 and 2 empty
    ep = np.array([-0.7, 1.0, -2.0])        # at k+q: bands 0 and 2 occupied, band 1 empty
    P = np.zeros((3, 3), dtype=np.complex128)
    for m, ph in zip(range(3), (np.exp(0.3j), np.exp(-1.1j), np.exp(2.0j))):
        P[(m - 1) % 3, m] = ph
    c = np.broadcast_to(np.eye(3, dtype=np.complex128), (nkt, 3, 3)).copy()
    ckq = np.broadcast_to(P, (nkt, 3, 3)).copy()
    eps = np.repeat(e[:, None], nkt, axis=1)
    epsq = np.repeat(ep[:, None], nkt, axis=1)
    return nk, eps, c, epsq, ckq, e, ep, np.abs(P) ** 2


def test_W_orientation_n_at_k_m_at_k_plus_q_closed_form():
    nk, eps, c, epsq, ckq, e, ep, absP2 = _cyclic_case()
    W = oracle.matrix_elements_raw(nk, c, c_kq=ckq)
    np.testing.assert_allclose(W, np.broadcast_to(absP2[:, :, None], W.shape), rtol=0, atol=1e-15)
    assert W[0, 1, 0] == pytest.approx(1.0) and W[1, 0, 0] == 0.0


def test_chi0_orientation_closed_form_for_flat_bands():
    """Flat bands make every tetrahedron a single point of the spectrum: chi0(w) =
    g_s sum_nm W_nm (f(e_n) - f(e'_m)) / (w - (e'_m - e_n) + i0), with f the T = 0 occupation
    at mu = 0 (Eq. (1) with the occupation difference written out)."""
    nk, eps, c, epsq, ckq, e, ep, absP2 = _cyclic_case()
    om = np.array([0.0, 0.9, -1.7, 3.3])
    got = oracle.chi0_raw(nk, eps, c, om, eps_kq=epsq, c_kq=ckq)
    f, fp = (e < 0).astype(float), (ep < 0).astype(float)

    def closed(Wm):
        out = np.zeros(om.size, dtype=complex)
        for n in range(3):
            for m in range(3):
                out += 2.0 * Wm[n, m] * (f[n] - fp[m]) / (om - (ep[m] - e[n]))
        return out

    np.testing.assert_allclose(got, closed(absP2), rtol=1e-13, atol=1e-14)
    # the swapped orientation (m at k, n at k+q) gives a different chi0
    assert np.max(np.abs(closed(absP2.T) - got)) > 0.5 * np.max(np.abs(got))
