"""CPU checks of the GPU path's per-tetrahedron arithmetic against the oracle.

``paper_1407_3444_amd/csrc/chi0_math.h`` (carving and the far-series /
near-branch weight evaluation the kernels use) is compiled for the host here
and compared with the oracle's independent carving and divided differences on
random and adversarial tetrahedra.  This runs without a GPU.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hostcheck", "chi0_hostcheck.cpp")
LIB = os.path.join(HERE, "hostcheck", "libchi0_hostcheck.so")


@pytest.fixture(scope="module")
def hc():
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", SRC, "-o", tmp])
    os.replace(tmp, LIB)
    lib = ctypes.CDLL(LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.hc_weight_sum.argtypes = [dp, dp, ctypes.c_double, dp]
    lib.hc_rho_far.argtypes = [ctypes.c_int]
    lib.hc_rho_far.restype = ctypes.c_double
    lib.hc_unit.argtypes = [dp, dp, dp, ctypes.c_double, ctypes.c_int, dp]
    lib.hc_unit.restype = ctypes.c_int
    lib.hc_group.argtypes = [dp, dp, dp, ctypes.c_int, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int)]
    lib.hc_group.restype = ctypes.c_int
    lib.hc_cluster.argtypes = [dp, dp, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int, dp]
    lib.hc_cluster.restype = ctypes.c_int
    lib.hc_near_fast.argtypes = [dp, dp, ctypes.c_double, ctypes.c_int, dp]
    lib.hc_near_fast.restype = ctypes.c_int
    lib.hc_near.argtypes = [dp, dp, ctypes.c_double, ctypes.c_int, dp]
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _weight_sum(hc, D, W, w):
    D = np.ascontiguousarray(D, float)
    W = np.ascontiguousarray(W, float)
    out = np.zeros(2)
    hc.hc_weight_sum(_p(D), _p(W), float(w), _p(out))
    return complex(out[0], out[1])


def _cases():
    rng = np.random.default_rng(17)
    out = []
    for _ in range(300):
        out.append((rng.uniform(0, 2, 4), rng.uniform(0, 1, 4), rng.uniform(-1, 3)))
    for _ in range(200):   # clustered, far and near
        c = rng.uniform(0.2, 1.8)
        out.append((c + rng.uniform(0, 1, 4) * 10 ** rng.uniform(-8, -1), rng.uniform(0, 1, 4),
                    c + rng.choice([-1, 1]) * 10 ** rng.uniform(-3, 0.5)))
    for _ in range(100):   # ties and near ties
        y = rng.uniform(0, 2, 4)
        y[1] = y[0] + (0.0 if rng.random() < 0.5 else 10 ** rng.uniform(-13, -5))
        if rng.random() < 0.3:
            y[3] = y[2]
        out.append((y, rng.uniform(0, 1, 4), rng.uniform(-1, 3)))
    for _ in range(100):   # w close to or at a node
        y = rng.uniform(0, 2, 4)
        j = rng.integers(4)
        w = y[j] if rng.random() < 0.3 else y[j] + rng.choice([-1, 1]) * 10 ** rng.uniform(-12, -2)
        out.append((y, rng.uniform(0, 1, 4), w))
    return out


def test_weight_sum_matches_oracle(hc):
    worst = 0.0
    for D, W, w in _cases():
        ref = np.dot(W, oracle.weights(D, w))
        got = _weight_sum(hc, D, W, w)
        scale = np.sum(np.abs(W) * np.abs(oracle.weights(D, w)))
        err = abs(got - ref) / scale
        worst = max(worst, err)
        assert err < 5e-12, (D, W, w, got, ref)
    print("worst relative error", worst)


def test_static_weight_sum_matches_oracle(hc):
    """w = 0 with nodes on both sides, at zero and near zero (the static kernel's cases)."""
    rng = np.random.default_rng(23)
    for _ in range(400):
        D = rng.uniform(0, 1.5, 4) * (10 ** rng.uniform(-4, 0))
        if rng.random() < 0.3:
            D[rng.integers(4)] = 0.0
        W = rng.uniform(0, 1, 4)
        ref = np.dot(W, oracle.weights(D, 0.0))
        got = _weight_sum(hc, D, W, 0.0)
        scale = np.sum(np.abs(W) * np.abs(oracle.weights(D, 0.0)))
        assert abs(got - ref) < 5e-12 * scale


def _oracle_unit(a, b, Wc, w, form):
    """contribution of one (tetrahedron, band pair) from the oracle's carving and weights"""
    D = b - a
    tot = 0j
    regions = [(1, 1.0)] if form == 1 else [(1, 1.0), (2, -1.0)]
    for region, sign in regions:
        verts, vols = oracle.carve(a, b, region)
        for V, v in zip(verts, vols):
            if v == 0.0:
                continue
            Dv, Wv = V @ D, V @ Wc
            tot += sign * v * np.dot(Wv, oracle.weights(Dv, w))
            if form == 1:
                tot -= sign * v * np.dot(Wv, oracle.weights(-Dv, w))
    return tot


@pytest.mark.parametrize("form", [0, 1])
def test_carved_unit_matches_oracle(hc, form):
    rng = np.random.default_rng(31 + form)
    for it in range(400):
        a = rng.normal(size=4)
        b = rng.normal(size=4) + (0.5 if it % 3 == 0 else 0.0)
        if it % 7 == 0:
            a[rng.integers(4)] = 0.0
        Wc = rng.uniform(0, 1, 4)
        w = 0.0 if it % 2 == 0 else rng.uniform(-2, 3)
        ref = _oracle_unit(a, b, Wc, w, form)
        out = np.zeros(2)
        hc.hc_unit(_p(a), _p(b), _p(Wc), float(w), form, _p(out))
        got = complex(out[0], out[1])
        assert abs(got - ref) <= 1e-11 * max(1.0, abs(ref)), (it, a, b, w, got, ref)


def _group_cases():
    """(D, W, omega group of 64): groups of 64 equally spaced frequencies at every distance from
    the tetrahedron's values, spans from ties to wide."""
    rng = np.random.default_rng(23)
    out = []
    for _ in range(250):
        c = rng.uniform(0.0, 2.0)
        hs = 10 ** rng.uniform(-6, -0.5) if rng.random() < 0.9 else 0.0
        D = c + hs * rng.uniform(-1, 1, 4)
        D[rng.integers(4)] = c - hs
        D[rng.integers(4)] = c + hs
        width = 10 ** rng.uniform(-2, 0)
        start = c + rng.choice([-1, 1]) * 10 ** rng.uniform(-3, 1) - (width if rng.random() < 0.5 else 0.0)
        out.append((D, rng.uniform(0, 1, 4), np.linspace(start, start + width, 64)))
    return out


def _group(hc, D, W, om, fp32):
    D = np.ascontiguousarray(D, float)
    W = np.ascontiguousarray(W, float)
    om = np.ascontiguousarray(om, float)
    out = np.zeros(2 * len(om))
    far = (ctypes.c_int * len(om))()
    cls = hc.hc_group(_p(D), _p(W), _p(om), len(om), int(fp32), _p(out), far)
    return cls, out[0::2] + 1j * out[1::2], np.array(list(far), dtype=bool)


@pytest.mark.parametrize("fp32,bound", [(0, 5e-12), (1, 1e-6)])
def test_series_cut_per_frequency_group_keeps_accuracy(hc, fp32, bound):
    """The far series cut to the class of a group of 64 frequencies (the terms the group's
    distance from the tetrahedron needs) matches the oracle's weights at every frequency."""
    worst, classes = 0.0, []
    for D, W, om in _group_cases():
        cls, got, far = _group(hc, D, W, om, fp32)
        classes.append(cls)
        assert (cls == 0) == (not far.any())
        for i in range(len(om)):
            J = oracle.weights(D, om[i])
            ref = np.dot(W, J)
            scale = np.sum(np.abs(W) * np.abs(J))
            err = abs(got[i] - ref) / scale
            worst = max(worst, err)
            assert err < bound, (D, W, om[i], cls, got[i], ref)
    # the cases exercise short, intermediate and full series
    assert min(c for c in classes if c > 0) <= 2 and max(classes) == 10 and 0 in classes
    print("worst relative error", worst, "classes", np.bincount(classes))


@pytest.mark.parametrize("fp32,bound", [(0, 5e-12), (1, 2e-6)])
def test_list_as_one_series_matches_oracle(hc, fp32, bound):
    """A list of final tetrahedra far from every frequency of a group, evaluated as one series about
    the centre of its span (the sum of the tetrahedra's coefficients about that centre), matches
    the sum of the oracle's weights; lists whose span reaches a frequency are refused."""
    rng = np.random.default_rng(23)
    used = refused = 0
    worst = 0.0
    for trial in range(120):
        nt = int(rng.integers(1, 33))
        c = rng.uniform(-1.0, 3.0)
        spread = 10 ** rng.uniform(-4, -0.5)
        D = c + rng.uniform(-spread, spread, (nt, 4))
        if trial % 10 == 0:
            D[:, 1] = D[:, 0]                      # tied corners
        W = rng.uniform(-1, 1, (nt, 4))
        om = np.sort(rng.uniform(0.0, 2.0, 64))
        out = np.zeros(2 * len(om))
        ok = hc.hc_cluster(_p(np.ascontiguousarray(D)), _p(np.ascontiguousarray(W)), nt, _p(om), len(om), fp32,
                           _p(out))
        span = (D.min(), D.max())
        far = (0.5 * (span[1] - span[0])) < hc.hc_rho_far(fp32) * max(0.0, om[0] - 0.5 * sum(span), 0.5 * sum(span) - om[-1])
        assert bool(ok) == far
        if not ok:
            refused += 1
            continue
        used += 1
        for i in range(len(om)):
            J = [oracle.weights(D[r], om[i]) for r in range(nt)]
            ref = sum(np.dot(W[r], J[r]) for r in range(nt))
            scale = sum(np.sum(np.abs(W[r]) * np.abs(J[r])) for r in range(nt))
            err = abs(out[2 * i] - ref.real) / scale
            worst = max(worst, err)
            assert err < bound, (trial, nt, i, out[2 * i], ref)
    assert used > 30 and refused > 10, (used, refused)
    print("worst relative error", worst, "lists as one series", used, "refused", refused)


@pytest.mark.parametrize("fp32", [0, 1])
def test_near_first_pass_equals_full_unless_flagged(hc, fp32):
    """The near drain's first pass (no entry series) gives bit for bit the full near evaluation
    whenever it does not flag the item; flagged items (2- or 3-node entries whose nodes cluster
    relative to their distance from w) are exactly those re-evaluated in full."""
    rng = np.random.default_rng(31)
    flagged = 0
    for _ in range(3000):
        y = np.sort(rng.uniform(0.0, 1.0, 4))
        if rng.random() < 0.3:
            k = int(rng.integers(0, 2))
            y[k + 1] = y[k] + 10 ** rng.uniform(-8, -1) * (y[3] - y[0] + 1e-3)
            y[k + 2] = y[k + 1] + 10 ** rng.uniform(-8, -1) * (y[3] - y[0] + 1e-3)
            y = np.sort(y)
        w = rng.uniform(-1, 1, 4)
        # frequencies of the near branch: within hs / rho of the centre (rho = 0.5 FP64, 0.4 FP32)
        c, hs = 0.5 * (y[0] + y[3]), 0.5 * (y[3] - y[0])
        om = rng.uniform(c - 2.5 * hs, c + 2.5 * hs)
        fast, full = np.zeros(2), np.zeros(2)
        need = hc.hc_near_fast(_p(y), _p(w), float(om), fp32, _p(fast))
        hc.hc_near(_p(y), _p(w), float(om), fp32, _p(full))
        if need:
            flagged += 1
        else:
            assert np.array_equal(fast, full), (y, w, om, fast, full)
    print("flagged", flagged, "of 3000")
    assert 30 < flagged < 2900, flagged
