"""Pins for the oracle's double carving of a tetrahedron (CPU only).

Sec. II: the first carving keeps the part of a tetrahedron where band n at k
is occupied (e < mu), the second keeps the part of that where band m at k+q is
empty (e' > mu); the final tetrahedra fill exactly the region where the
product of Heaviside functions is one (the carving condition, Eq. (4)).
"""
import numpy as np
import pytest

import oracle


def _region_volume(a, b, sa, sb):
    """volume fraction of {sa*a < 0, sb*b < 0} via the oracle's carving of region 1
    with sign-flipped corner values (region 1 keeps {a < 0, b > 0})."""
    _, vols = oracle.carve(sa * np.asarray(a), -sb * np.asarray(b), 1)
    return vols.sum()


def test_four_regions_partition_the_tetrahedron():
    """{a<0,b<0} + {a<0,b>0} + {a>0,b<0} + {a>0,b>0} fill the tetrahedron exactly."""
    rng = np.random.default_rng(3)
    for _ in range(500):
        a = rng.normal(size=4)
        b = rng.normal(size=4)
        tot = (_region_volume(a, b, 1, 1) + _region_volume(a, b, 1, -1)
               + _region_volume(a, b, -1, 1) + _region_volume(a, b, -1, -1))
        assert abs(tot - 1.0) < 1e-13


def test_region_volumes_match_monte_carlo():
    rng = np.random.default_rng(4)
    lam = rng.dirichlet(np.ones(4), size=400000)        # uniform in the tetrahedron
    for _ in range(20):
        a = rng.normal(size=4)
        b = rng.normal(size=4)
        fa, fb = lam @ a, lam @ b
        for region, mask in [(1, (fa < 0) & (fb > 0)), (2, (fa > 0) & (fb < 0))]:
            _, vols = oracle.carve(a, b, region)
            p = mask.mean()
            sigma = np.sqrt(max(p * (1 - p), 1e-12) / lam.shape[0])
            assert abs(vols.sum() - p) < 5 * sigma + 1e-12


def test_final_tetrahedra_lie_in_the_region():
    """Every vertex of a final tetrahedron satisfies e <= mu <= e' (region 1) and the
    volume of each piece equals the determinant of its barycentric vertices."""
    rng = np.random.default_rng(8)
    for _ in range(300):
        a = rng.normal(size=4)
        b = rng.normal(size=4)
        verts, vols = oracle.carve(a, b, 1)
        assert len(vols) <= 9
        for V, v in zip(verts, vols):
            assert np.all(V @ a <= 1e-12) and np.all(V @ b >= -1e-12)
            np.testing.assert_allclose(V.sum(axis=1), 1.0, atol=1e-14)
            assert abs(abs(np.linalg.det(V)) - v) < 1e-13


def test_full_and_empty_tetrahedra():
    a = np.array([-1.0, -2.0, -0.5, -0.1])
    b = np.array([0.3, 0.2, 1.0, 0.01])
    verts, vols = oracle.carve(a, b, 1)
    assert len(vols) == 1 and vols[0] == 1.0
    assert len(oracle.carve(a, b, 2)[1]) == 0
    assert len(oracle.carve(-a, b, 1)[1]) == 0


def test_carved_integral_is_continuous_in_the_corner_values():
    """Moving a corner across mu changes the carved volume and the weighted integral
    continuously (no jump from the case split)."""
    rng = np.random.default_rng(12)
    D = np.array([0.4, 0.9, 0.6, 1.2])
    Wc = np.array([0.3, 0.8, 0.5, 0.1])
    b = np.array([0.5, -0.2, 0.7, 0.3])

    def integral(a):
        verts, vols = oracle.carve(a, b, 1)
        tot = 0.0
        for V, v in zip(verts, vols):
            J = oracle.weights(V @ D, 2.5)
            tot += v * np.dot(V @ Wc, J.real)
        return tot

    for eps in [1e-6, 1e-9]:
        a_lo = np.array([-0.3, 0.4, -eps, 0.2])
        a_hi = np.array([-0.3, 0.4, +eps, 0.2])
        assert abs(integral(a_lo) - integral(a_hi)) < 50 * eps
