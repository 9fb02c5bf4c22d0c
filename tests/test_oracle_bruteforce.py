"""The oracle's whole dynamic chi0 with matrix elements against the continuum, by brute force.

The retarded chi0 of Eq. (1) is the boundary value at eta -> 0+ of the function of the complex
frequency z = w + i eta,

    chi0(q, z) = (g_s / V_BZ) int dk sum_nm W_nm(k) [f(e_n(k)) - f(e_m(k+q))] / (z - e_m(k+q) + e_n(k)),

which is analytic in the upper half plane.  At finite eta the integrand is smooth in k except for
the Fermi steps; with the Fermi function at a small temperature T it is smooth everywhere, so a plain
k sum on an M^3 grid converges exponentially in M, and the temperature error vanishes as T -> 0.
The oracle evaluates the same tetrahedron integral as on the real axis with z in place of w + i0
(the complex-frequency entry point shares every step of the real-axis one), so at equal eta its
result must converge to the brute-force sum as h^2 when the mesh is refined.  The brute force here
is plain numpy: a closed-form 2 x 2 eigensolver, the Fermi function and the Lorentzian-broadened
sum; nothing of the oracle.  The real-axis limit is tied to the complex one by continuity at
vanishing eta.
"""
import numpy as np

import oracle
import synth


def _two_band_model():
    """Two orbitals on a simple-cubic lattice with real hoppings t(-R) = t(R)^T: the orbital mixing
    varies with k, so W_nm(k, q) is far from 0 and 1."""
    hop = {}
    synth._add_pair(hop, (0, 0, 0), np.array([[-0.3, 0.15], [0.15, 0.4]]))
    synth._add_pair(hop, (1, 0, 0), np.array([[-0.25, 0.12], [-0.05, 0.18]]))
    synth._add_pair(hop, (0, 1, 0), np.array([[-0.25, 0.04], [0.10, 0.18]]))
    synth._add_pair(hop, (0, 0, 1), np.array([[-0.20, 0.0], [0.07, 0.15]]))
    return synth.TBModel("two_band", 2, hop)


def _eig2(H):
    """Eigenpairs of Hermitian 2 x 2 matrices [k][2][2] in closed form: energies [2][k] ascending,
    eigenvectors [k][orbital][band] (the coupling H01 is non-zero for this model)."""
    a, d, b = H[:, 0, 0].real, H[:, 1, 1].real, H[:, 0, 1]
    m = 0.5 * (a + d)
    r = np.sqrt(0.25 * (a - d) ** 2 + np.abs(b) ** 2)
    vecs = []
    for lam in (m - r, m + r):
        v0, v1 = b, lam - a
        nrm = np.sqrt(np.abs(v0) ** 2 + np.abs(v1) ** 2)
        vecs.append(np.stack([v0 / nrm, v1 / nrm], axis=1))
    return np.stack([m - r, m + r], axis=0), np.stack(vecs, axis=2)


def _brute(model, q, M, T, eta, omegas, mu=0.0):
    """(g_s / M^3) sum_k sum_nm W_nm (f_n(k) - f_m(k+q)) / (w + i eta - e_m(k+q) + e_n(k)) on the
    offset M^3 grid, Fermi function at temperature T."""
    g = (np.arange(M) + 0.5) / M
    k1, k2 = np.meshgrid(g, g, indexing="ij")
    out = np.zeros(len(omegas), dtype=complex)
    for k3 in g:
        kf = np.stack([k1.ravel(), k2.ravel(), np.full(k1.size, k3)], axis=1)
        e, c = _eig2(model.hk(kf))
        ep, cp = _eig2(model.hk(kf + q[None, :]))
        f = 1.0 / (np.exp((e - mu) / T) + 1.0)
        fp = 1.0 / (np.exp((ep - mu) / T) + 1.0)
        for n in range(2):
            for m in range(2):
                W = np.abs(np.sum(np.conj(c[:, :, n]) * cp[:, :, m], axis=1)) ** 2
                num = W * (f[n] - fp[m])
                D = ep[m] - e[n]
                for i, w in enumerate(omegas):
                    out[i] += np.sum(num / (w + 1j * eta - D))
    return 2.0 * out / M ** 3


def _tetra(model, N, q, omegas, eta, mu):
    nk = (N, N, N)
    kf = synth.mesh_kfrac(nk)
    e, c = synth.eigensystem(model, kf)
    ekq, ckq = synth.eigensystem(model, kf + q[None, :])
    return oracle.chi0_z_raw(nk, e, c, omegas, eta, eps_kq=ekq, c_kq=ckq, mu=mu)


def test_dynamic_chi0_with_matrix_elements_converges_to_the_dense_k_sum():
    model = _two_band_model()
    q = np.array([0.21, 0.13, 0.05])
    om = np.array([0.05, 0.3, 0.6])        # inside the particle-hole continuum: Im chi0 != 0
    eta = 0.1
    # mu = -0.5 lies inside the lower band, away from its upper edge near 0 (a band edge at the
    # Fermi level would make the temperature error fall only slowly).  All four band pairs
    # contribute: the lower band crosses mu, the upper one is empty.
    mu = -0.5
    # brute force: converged in M (128 and 160 agree to 3e-6 at T = 0.0075); the temperature
    # error at T = 0.005 is a few 1e-4 (the step from T = 0.0075 is checked)
    b1 = _brute(model, q, 128, 0.0075, eta, om, mu=mu)
    b2 = _brute(model, q, 160, 0.005, eta, om, mu=mu)
    ref = b2
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(b2 - b1)) < 1e-3 * scale
    errs = [np.max(np.abs(_tetra(model, N, q, om, eta, mu) - ref)) / scale for N in (12, 24, 48)]
    # second-order convergence of the linear tetrahedron interpolant: each halving of h cuts the
    # error by about 4 (asserted with margin), down to a few 1e-3 at 48^3
    assert errs[1] < 0.4 * errs[0]
    assert errs[2] < 0.4 * errs[1]
    assert errs[2] < 4e-3
    assert np.min(np.abs(ref.imag)) > 0.05 * scale     # the absorptive part is really tested


def test_complex_frequency_tends_to_the_retarded_real_axis_result():
    model = _two_band_model()
    q = np.array([0.21, 0.13, 0.05])
    nk = (6, 6, 6)
    kf = synth.mesh_kfrac(nk)
    e, c = synth.eigensystem(model, kf)
    ekq, ckq = synth.eigensystem(model, kf + q[None, :])
    om = np.array([-0.4, 0.0, 0.05, 0.3, 0.6, 2.5])
    real_axis = oracle.chi0_raw(nk, e, c, om, eps_kq=ekq, c_kq=ckq)
    at_zero = oracle.chi0_z_raw(nk, e, c, om, 0.0, eps_kq=ekq, c_kq=ckq)
    np.testing.assert_array_equal(at_zero, real_axis)
    near = oracle.chi0_z_raw(nk, e, c, om, 1e-9, eps_kq=ekq, c_kq=ckq)
    np.testing.assert_allclose(near, real_axis, rtol=0, atol=1e-6 * np.max(np.abs(real_axis)))
