"""Pins for the oracle's irreducible-wedge integration with the point-group loop (Sec. II)
(CPU only).

The wedge and the group are pinned geometrically (the 48 images of the wedge's tetrahedra tile
the zone exactly once, by brute-force point location) and the loop by an exact identity: summing
the wedge integral over the group with the k+q data taken at k + g^-1 q equals the integral over
the whole zone triangulated by the images of the wedge's tetrahedra, for models whose bands and
matrix elements are invariant under the group.  The free-electron Lindhard function pins the
result against the continuum.
"""
import numpy as np
import pytest

import oracle
import synth

KF = np.pi / 2


def _in_tet(p, v):
    """Barycentric coordinates of points p [n][3] in the tetrahedron with vertices v [4][3]."""
    T = (v[1:] - v[0]).T
    lam = np.linalg.solve(T, (p - v[0]).T).T
    return np.concatenate([1.0 - lam.sum(axis=1, keepdims=True), lam], axis=1)


def test_point_group_is_oh():
    ops = oracle.cubic_point_group()
    assert ops.shape == (48, 3, 3)
    assert np.array_equal(ops[0], np.eye(3, dtype=ops.dtype))
    keys = {g.tobytes() for g in ops}
    assert len(keys) == 48
    for g in ops:
        assert np.array_equal(g @ g.T, np.eye(3, dtype=ops.dtype))
    for a in ops[::5]:
        for b in ops[::3]:
            assert (a @ b).tobytes() in keys
    # the simple-cubic nearest-neighbour band is invariant under every element
    m = synth.sc_nn_model(1.0)
    k = np.random.default_rng(1).random((20, 3)) - 0.5
    e0, _ = synth.eigensystem(m, k)
    for g in ops:
        e1, _ = synth.eigensystem(m, k @ g.T)
        assert np.max(np.abs(e1 - e0)) < 1e-13


@pytest.mark.parametrize("n", [2, 4, 6])
def test_wedge_tetrahedra_tile_the_zone(n):
    kf, tets, vol = oracle.iw_cubic(n)
    m = n // 2
    assert tets.shape == (m ** 3, 4)
    assert kf.shape[0] == (m + 1) * (m + 2) * (m + 3) // 6
    assert abs(48 * tets.shape[0] * vol - 1.0) < 1e-15
    # every tetrahedron has the volume of a Kuhn tetrahedron and lies in 0 <= z <= y <= x <= 1/2
    for t in tets:
        v = kf[t]
        assert abs(abs(np.linalg.det(v[1:] - v[0])) / 6.0 - vol) < 1e-15
        c = v.mean(axis=0)
        assert 0.0 < c[2] < c[1] < c[0] < 0.5
    # the images under O_h cover the cube [-1/2, 1/2]^3 exactly once (generic sample points)
    pts = np.random.default_rng(n).random((400, 3)) - 0.5
    count = np.zeros(len(pts), dtype=int)
    for g in oracle.cubic_point_group():
        for t in tets:
            lam = _in_tet(pts, kf[t] @ g.T)
            count += np.all(lam > 0.0, axis=1)
    assert np.all(count == 1), np.bincount(count)


def _full_zone(kf, tets, ops):
    """The zone triangulated by the images g T of the wedge's tetrahedra: points and tetrahedra."""
    n_iw = kf.shape[0]
    scale = 1
    while not np.allclose(kf * scale, np.round(kf * scale)):
        scale += 1
    where, pts, out = {}, [], []
    for g in ops:
        img = np.round((kf @ g.T) * scale).astype(np.int64)
        idx = np.empty(n_iw, dtype=np.int64)
        for i, p in enumerate(map(tuple, img)):
            if p not in where:
                where[p] = len(pts)
                pts.append(p)
            idx[i] = where[p]
        out.append(idx[tets])
    return np.array(pts, dtype=np.float64) / scale, np.concatenate(out).astype(np.int32)


def _model_entries(model, kf, q, ops):
    """Energies and eigenvectors at the wedge's points and, per g, at k + g^-1 q."""
    e, c = synth.eigensystem(model, kf)
    entries = []
    for g in ops:
        ekq, ckq = synth.eigensystem(model, kf + q @ g)     # g^-1 q = g^T q for orthogonal g
        entries.append((ekq, ckq))
    return e, c, entries


@pytest.mark.parametrize("kind", ["sc_cma", "cubic_s"])
def test_point_group_loop_equals_full_zone(kind):
    ops = oracle.cubic_point_group()
    kf, tets, vol = oracle.iw_cubic(6)
    q = np.array([0.137, 0.052, -0.021])
    omega = np.array([0.0, 0.35, 1.2, 2.9])
    if kind == "sc_cma":
        model, cma, kw = synth.sc_nn_model(1.0), True, {"mu": 0.3}
    else:
        model, cma, kw = synth.cubic_s_model(5, 3), False, {"mu": 0.1}
    e, c, entries = _model_entries(model, kf, q, ops)
    if cma:
        c, entries = None, [(ekq, None) for ekq, _ in entries]
    for form in (0, 1):
        iw = oracle.chi0_iw(e, c, entries, tets, vol, omega, cma=cma, form=form, **kw)
        pts, ftets = _full_zone(kf, tets, ops)
        ef, cf = synth.eigensystem(model, pts)
        efq, cfq = synth.eigensystem(model, pts + q)
        full = oracle.chi0_list(ef, None if cma else cf, efq, None if cma else cfq, ftets, vol, omega,
                                cma=cma, form=form, **kw)
        assert np.max(np.abs(iw - full)) <= 1e-12 * np.max(np.abs(full)), (form, iw, full)
        assert abs(full[0].imag) < 1e-14 and full[0].real < 0.0


def test_wedge_loop_is_sensitive_to_the_group():
    """A plausible mistake, the 24 proper rotations counted twice instead of all 48 elements,
    must not reproduce the full-zone integral (the identity above is not trivially satisfied)."""
    ops = oracle.cubic_point_group()
    proper = [i for i, g in enumerate(ops) if round(np.linalg.det(g)) == 1]
    assert len(proper) == 24
    kf, tets, vol = oracle.iw_cubic(6)
    q = np.array([0.137, 0.052, -0.021])
    model = synth.cubic_s_model(5, 3)
    e, c, entries = _model_entries(model, kf, q, ops)
    full = oracle.chi0_iw(e, c, entries, tets, vol, [0.4], mu=0.1)
    twice = 2.0 * oracle.chi0_iw(e, c, [entries[i] for i in proper], tets, vol, [0.4], mu=0.1)
    assert abs(twice[0] - full[0]) > 1e-4 * abs(full[0]), (twice, full)


def _lindhard_static(q):
    x = q / (2 * KF)
    nf = KF / np.pi ** 2
    return -nf * (0.5 + (1 - x * x) / (4 * x) * np.log(abs((1 + x) / (1 - x))))


def _free_electron_iw(n, qvec, omega, form=1):
    ops = oracle.cubic_point_group()
    kf, tets, vol = oracle.iw_cubic(n)
    e = synth.free_electron_eps_at(kf)
    entries = [(synth.free_electron_eps_at(kf, qvec @ g), None) for g in ops]
    return oracle.chi0_iw(e, None, entries, tets, vol, omega, mu=KF ** 2 / 2, cma=True, form=form)


@pytest.mark.parametrize("q", [0.3, 1.0, 2.5])
def test_free_electron_wedge_lindhard_converges(q):
    """Eq. (1) form over the wedge with the point-group loop: error against Lindhard ~ h^2."""
    errs = []
    for n in (16, 32):
        val = _free_electron_iw(n, np.array([q, 0.0, 0.0]), [0.0])[0].real
        errs.append(abs(val - _lindhard_static(q)))
    assert errs[1] < errs[0] / 3.0
    assert errs[1] < 1e-3


def test_single_carving_reduces_to_double_when_final_states_are_all_empty():
    """The comparison treatment (first carving only, final-state factor at the corners) equals the
    double carving exactly when every k+q state is empty, and vanishes when every one is full."""
    ops = oracle.cubic_point_group()
    kf, tets, vol = oracle.iw_cubic(8)
    m = synth.sc_nn_model(1.0)
    e, _ = synth.eigensystem(m, kf)
    omega = np.array([0.0, 0.7, 3.1])
    for shift, zero in ((20.0, False), (-20.0, True)):
        ents = [(synth.eigensystem(m, kf + np.array([0.1, 0.05, 0.0]) @ g)[0] + shift, None) for g in ops[:6]]
        d = oracle.chi0_iw(e, None, ents, tets, vol, omega, mu=0.2, cma=True, form=1)
        s = oracle.chi0_iw(e, None, ents, tets, vol, omega, mu=0.2, cma=True, form=1, single_carving=True)
        if zero:
            assert np.all(d == 0) and np.all(s == 0)
        else:
            assert np.max(np.abs(s - d)) <= 1e-13 * np.max(np.abs(d))


def test_second_carving_needs_fewer_wedge_points():
    """Re-test of the Sec. II claim (about 500 wedge k-points with the second carving against more
    than 2000 without) on free electrons against Lindhard: over q = 0.4, 1.2, 2.6 (k_F = pi/2) the
    double carving on the 24^3 wedge (455 points) is more accurate than the single carving on the
    48^3 wedge (2925 points)."""
    worst_double, worst_single = 0.0, 0.0
    for q in (0.4, 1.2, 2.6):
        ref = _lindhard_static(q)
        d = _free_electron_iw(24, np.array([q, 0.0, 0.0]), [0.0])[0].real
        ops = oracle.cubic_point_group()
        kf, tets, vol = oracle.iw_cubic(48)
        e = synth.free_electron_eps_at(kf)
        ents = [(synth.free_electron_eps_at(kf, np.array([q, 0.0, 0.0]) @ g), None) for g in ops]
        s = oracle.chi0_iw(e, None, ents, tets, vol, [0.0], mu=KF ** 2 / 2, cma=True, form=1,
                           single_carving=True)[0].real
        worst_double = max(worst_double, abs(d - ref) / abs(ref))
        worst_single = max(worst_single, abs(s - ref) / abs(ref))
    assert worst_double < 0.02
    assert worst_double < worst_single / 2, (worst_double, worst_single)
