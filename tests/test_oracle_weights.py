"""Pins for the oracle's tetrahedron corner weights J_j (CPU only).

J_j(w; D) = 6 int_simplex lambda_j / (w - lambda.D + i0) dlambda is the integral
over a final tetrahedron (Sec. II: linear interpolation of energies and matrix
elements on each tetrahedron, Eqs. (1)-(2) for the integrand).  Each test checks
it against something other than the oracle's own divided-difference code:
direct cubature of the definition, a 60-digit evaluation, the B-spline density
of lambda.D (scipy) with Cauchy principal-value quadrature, and textbook closed
forms.
"""
import numpy as np
import mpmath as mp
import pytest
from scipy import integrate
from scipy.interpolate import BSpline

import oracle


def _tplquad_weight(D, w, j):
    """6 * int over the unit simplex of lambda_j / (w - lambda.D) (w outside the D range)."""
    D = np.asarray(D, dtype=float)

    def f(l3, l2, l1):
        lam = np.array([l1, l2, l3, 1.0 - l1 - l2 - l3])
        return lam[j] / (w - lam @ D)

    val, _ = integrate.tplquad(f, 0.0, 1.0, lambda l1: 0.0, lambda l1: 1.0 - l1,
                               lambda l1, l2: 0.0, lambda l1, l2: 1.0 - l1 - l2,
                               epsabs=1e-13, epsrel=1e-12)
    return 6.0 * val


@pytest.mark.parametrize("D,w", [
    ([0.3, 0.7, 1.1, 1.9], 2.6),
    ([0.3, 0.7, 1.1, 1.9], -0.4),
    ([-0.2, 0.05, 0.4, 0.41], 0.9),
    ([1.0, 1.0, 1.2, 1.5], 0.1),
])
def test_weights_match_cubature_of_definition(D, w):
    J = oracle.weights(D, w)
    for j in range(4):
        ref = _tplquad_weight(D, w, j)
        assert abs(J[j].imag) < 1e-13 * abs(J[j].real)
        assert abs(J[j].real - ref) < 1e-9 * abs(ref)


def _mp_weights(D, w, dps=240):
    """J_j at high precision from the Lagrange form of the divided difference of
    h(x) = (w-x)^3 Log(w-x+i0) with node j doubled (d/dD_j of the 4-node sum).
    Tied nodes are separated by 1e-40 (far below double resolution)."""
    with mp.workdps(dps):
        y = [mp.mpf(float(v)) + mp.mpf(10) ** -40 * (k + 1) * (k + 2) * (1 if k % 2 else -1)
             for k, v in enumerate(D)]
        W = mp.mpf(float(w))

        def L(u):
            return mp.log(abs(u)) + (1j * mp.pi if u < 0 else 0)

        def h(x):
            u = W - x
            return mp.mpc(0) if u == 0 else u ** 3 * L(u)

        def hp(x):
            u = W - x
            return mp.mpc(0) if u == 0 else -(3 * u ** 2 * L(u) + u ** 2)

        out = []
        for j in range(4):
            J = mp.mpc(0)
            for i in range(4):
                if i == j:
                    continue
                P = y[i] - y[j]
                for k in range(4):
                    if k != i:
                        P *= y[i] - y[k]
                J += h(y[i]) / P
            Pj, S = mp.mpf(1), mp.mpf(0)
            for k in range(4):
                if k != j:
                    Pj *= y[j] - y[k]
                    S += 1 / (y[j] - y[k])
            J += hp(y[j]) / Pj - h(y[j]) * S / Pj
            out.append(complex(J))
        return np.array(out)


def _stress_cases():
    rng = np.random.default_rng(11)
    cases = []
    for _ in range(12):   # spread nodes, w anywhere
        cases.append((rng.uniform(0, 2, 4), rng.uniform(-1, 3)))
    for _ in range(12):   # tight clusters far from w
        c = rng.uniform(0.5, 1.5)
        cases.append((c + rng.uniform(0, 1, 4) * 10 ** rng.uniform(-9, -2), rng.uniform(-1, 3)))
    for _ in range(8):    # one near-tied pair among spread nodes
        y = rng.uniform(0, 2, 4)
        y[1] = y[0] + 10 ** rng.uniform(-12, -4)
        cases.append((y, rng.uniform(-1, 3)))
    for _ in range(6):    # exact triple tie
        y = rng.uniform(0, 2, 4)
        y[1] = y[0]
        y[2] = y[0]
        cases.append((y, rng.uniform(-1, 3)))
    for _ in range(8):    # w very close to a node
        y = rng.uniform(0, 2, 4)
        cases.append((y, y[rng.integers(4)] + rng.choice([-1, 1]) * 10 ** rng.uniform(-12, -3)))
    cases.append((np.array([0.0, 0.3, 0.5, 0.9]), 0.0))      # w exactly on a node
    cases.append((np.array([0.0, 0.0, 0.5, 0.9]), 0.0))      # doubled node at w
    return cases


@pytest.mark.parametrize("case", range(48))
def test_weights_match_high_precision(case):
    D, w = _stress_cases()[case]
    J = oracle.weights(D, w)
    ref = _mp_weights(D, w)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(J - ref)) <= 2e-13 * scale, (D, w, J, ref)


def _bspline_M(D, j):
    """Normalised cubic B-spline M(x) (integral 1) with knots D u {D_j}: the density of
    lambda.D under the weight 4 lambda_j on the simplex."""
    t = np.sort(np.concatenate([np.asarray(D, float), [D[j]]]))
    B = BSpline.basis_element(t, extrapolate=False)
    scale = 4.0 / (t[-1] - t[0])

    def M(x):
        v = B(np.atleast_1d(x))
        v = np.nan_to_num(v, nan=0.0)
        return scale * v
    return M, t


@pytest.mark.parametrize("seed", range(6))
def test_weights_match_bspline_density(seed):
    """Im J_j = -(pi/4) M(w) and Re J_j = (1/4) PV int M(x)/(w-x) dx."""
    rng = np.random.default_rng(100 + seed)
    D = rng.uniform(0.0, 1.0, 4)
    if seed == 5:
        D[2] = D[1]    # tied knots
    for j in range(4):
        M, t = _bspline_M(D, j)
        total = sum(integrate.quad(lambda x: M(x)[0], t[i], t[i + 1])[0]
                    for i in range(4) if t[i + 1] > t[i])
        assert abs(total - 1.0) < 1e-10
        for w in [t[0] + 0.37 * (t[-1] - t[0]), t[0] + 0.81 * (t[-1] - t[0])]:
            J = oracle.weights(D, w)[j]
            assert abs(J.imag - (-np.pi / 4.0) * M(w)[0]) < 1e-12 * max(1.0, abs(J.imag))
            # principal value: pieces without w plainly, the piece holding w with a Cauchy weight
            pv = 0.0
            for i in range(4):
                a, b = t[i], t[i + 1]
                if b <= a:
                    continue
                if a < w < b:
                    pv += integrate.quad(lambda x: M(x)[0], a, b, weight="cauchy", wvar=w,
                                         epsabs=1e-13, epsrel=1e-12, limit=200)[0]
                else:
                    pv += integrate.quad(lambda x: M(x)[0] / (x - w), a, b, epsabs=1e-13,
                                         epsrel=1e-12)[0]
            # quad's Cauchy weight integrates f/(x - w); J has 1/(w - x)
            assert abs(J.real - (-0.25 * pv)) < 1e-8 * max(1.0, abs(J.real))


def test_flat_band_limit():
    """All corners equal: J_j = 1/(4 (w - D0))."""
    for D0, w in [(0.5, 1.5), (1.2, -0.3), (-0.7, 0.2)]:
        J = oracle.weights([D0] * 4, w)
        np.testing.assert_allclose(J.real, 1.0 / (4.0 * (w - D0)), rtol=1e-15)
        assert np.all(J.imag == 0.0)


def test_sum_of_weights_is_static_textbook_formula():
    """At w = 0 with positive distinct D: sum_j J_j = -<1/D> and
    <1/D> = 3 sum_i D_i^2 ln D_i / prod_{k!=i} (D_i - D_k) (tetrahedron average of 1/D)."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        D = rng.uniform(0.1, 2.0, 4)
        ref = 0.0
        for i in range(4):
            P = np.prod([D[i] - D[k] for k in range(4) if k != i])
            ref += 3.0 * D[i] ** 2 * np.log(D[i]) / P
        J = oracle.weights(D, 0.0)
        np.testing.assert_allclose(-J.sum().real, ref, rtol=1e-9)


def test_translation_and_scaling():
    """J(w; D) depends on w - D only, and J(a w; a D) = J(w; D) / a for a > 0."""
    D = np.array([0.2, 0.9, 0.45, 1.3])
    for w in [-0.5, 0.6, 2.0]:
        J = oracle.weights(D, w)
        np.testing.assert_allclose(oracle.weights(D + 0.75, w + 0.75), J, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(oracle.weights(3.0 * D, 3.0 * w), J / 3.0, rtol=1e-12, atol=1e-14)
