"""GPU checks of the device build of the kernels' per-tetrahedron arithmetic (chi0_math.h, built
by tests/devcheck for gfx950 with the library's flags): the hardware reciprocal with its
third-order step, the library's own FP64 logarithm, the FP32 forms and the compiler's
contractions, checked on the GPU against numpy, the oracle's divided differences (Sec. II corner
weights) and the host build of the same source."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
DEVLIB = os.path.join(HERE, "devcheck", "libchi0_devcheck.so")
HOSTSRC = os.path.join(HERE, "hostcheck", "chi0_hostcheck.cpp")


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(DEVLIB):
        raise RuntimeError("tests/devcheck/libchi0_devcheck.so is missing: run __graft_entry__.build()")
    lib = ctypes.CDLL(DEVLIB)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.dc_eval.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_int)]
    lib.dc_eval.restype = ctypes.c_int
    return lib


@pytest.fixture(scope="module")
def host():
    lib_path = os.path.join(HERE, "hostcheck", "libchi0_hostcheck_dev.so")
    tmp = lib_path + ".tmp%d" % os.getpid()
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", HOSTSRC, "-o", tmp])
    os.replace(tmp, lib_path)
    lib = ctypes.CDLL(lib_path)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.hc_near_fast.argtypes = [dp, dp, ctypes.c_double, ctypes.c_int, dp]
    lib.hc_near_fast.restype = ctypes.c_int
    lib.hc_near.argtypes = [dp, dp, ctypes.c_double, ctypes.c_int, dp]
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _run(dev, what, x=None, D=None, W=None, om=None):
    n = len(x) if x is not None else len(om)
    x = np.ascontiguousarray(np.zeros(n) if x is None else x, dtype=np.float64)
    D = np.ascontiguousarray(np.zeros((n, 4)) if D is None else D, dtype=np.float64)
    W = np.ascontiguousarray(np.zeros((n, 4)) if W is None else W, dtype=np.float64)
    om = np.ascontiguousarray(np.zeros(n) if om is None else om, dtype=np.float64)
    out = np.zeros((n, 2))
    flag = np.zeros(n, dtype=np.int32)
    rc = dev.dc_eval(what, n, _p(x), _p(D), _p(W), _p(om), _p(out),
                     flag.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    assert rc == 0, "dc_eval failed with HIP error %d" % rc
    return out[:, 0] + 1j * out[:, 1], flag


def _cases(seed=17):
    """Final tetrahedra and frequencies of the near branch: random, clustered nodes near and far,
    ties and near ties, frequencies at and next to a node."""
    rng = np.random.default_rng(seed)
    D, W, om = [], [], []
    for _ in range(300):
        D.append(rng.uniform(0, 2, 4)); W.append(rng.uniform(0, 1, 4)); om.append(rng.uniform(-1, 3))
    for _ in range(200):
        c = rng.uniform(0.2, 1.8)
        D.append(c + rng.uniform(0, 1, 4) * 10 ** rng.uniform(-8, -1)); W.append(rng.uniform(0, 1, 4))
        om.append(c + rng.choice([-1, 1]) * 10 ** rng.uniform(-3, 0.5))
    for _ in range(100):
        y = rng.uniform(0, 2, 4)
        y[1] = y[0] + (0.0 if rng.random() < 0.5 else 10 ** rng.uniform(-13, -5))
        if rng.random() < 0.3:
            y[3] = y[2]
        D.append(y); W.append(rng.uniform(0, 1, 4)); om.append(rng.uniform(-1, 3))
    for _ in range(100):
        y = rng.uniform(0, 2, 4)
        j = rng.integers(4)
        om.append(y[j] if rng.random() < 0.3 else y[j] + rng.choice([-1, 1]) * 10 ** rng.uniform(-12, -2))
        D.append(y); W.append(rng.uniform(0, 1, 4))
    return np.array(D), np.array(W), np.array(om)


def _oracle(D, W, om):
    ref = np.empty(len(om), dtype=complex)
    scale = np.empty(len(om))
    for i in range(len(om)):
        J = oracle.weights(D[i], om[i])
        ref[i] = np.dot(W[i], J)
        scale[i] = np.sum(np.abs(W[i]) * np.abs(J))
    return ref, scale


def test_reciprocal_within_two_ulp(dev):
    """rcp on the GPU (hardware estimate and one third-order step) against the correctly rounded
    quotient, over 300 decades, both signs, powers of two and values next to 1; the FP32 form
    against the FP32 quotient."""
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.choice([-1.0, 1.0], 20000) * 10 ** rng.uniform(-150, 150, 20000),
                        2.0 ** np.arange(-60, 61), 1.0 + rng.uniform(-1e-6, 1e-6, 2000)])
    got, _ = _run(dev, 0, x=x)
    ulps = np.abs(got.real - 1.0 / x) / np.spacing(np.abs(1.0 / x))
    _say(f"rcp: worst {ulps.max():.2f} ulp")
    assert ulps.max() <= 2.0
    xf = (rng.choice([-1.0, 1.0], 20000) * 10 ** rng.uniform(-30, 30, 20000)).astype(np.float32)
    gotf, _ = _run(dev, 6, x=xf.astype(np.float64))
    reff = (np.float32(1.0) / xf).astype(np.float64)
    ulpf = np.abs(gotf.real - reff) / np.spacing(np.abs(reff).astype(np.float32)).astype(np.float64)
    _say(f"rcp (FP32): worst {ulpf.max():.2f} ulp")
    assert ulpf.max() <= 2.0


def test_own_logarithm_within_two_ulp(dev):
    """log_pos on the GPU against numpy's logarithm: 600 decades, both sides of the range
    reduction's edges (sqrt 2 and its halvings), and arguments next to 1 where the result is
    small."""
    rng = np.random.default_rng(7)
    edges = np.sqrt(2.0) * 2.0 ** np.arange(-20, 21)
    x = np.concatenate([10 ** rng.uniform(-300, 300, 20000), edges, np.nextafter(edges, 0), np.nextafter(edges, 4),
                        1.0 + rng.uniform(-1e-3, 1e-3, 3000), 1.0 + 10 ** rng.uniform(-15, -4, 2000),
                        rng.uniform(0.5, 2.0, 5000)])
    got, _ = _run(dev, 1, x=x)
    ref = np.log(x)
    ulps = np.abs(got.real - ref) / np.spacing(np.maximum(np.abs(ref), 1e-300))
    _say(f"log_pos: worst {ulps.max():.2f} ulp")
    assert ulps.max() <= 2.0


def test_near_branch_matches_oracle_and_host_build(dev, host):
    """The FP64 near branch on the GPU against the oracle's weights (the bound of the host check)
    and against the host build, within 2e-12 of the weights' scale: the size of the branch's own
    rounding error (its error against the oracle reaches 9e-13 on the host), which the device's
    contractions and hardware reciprocal reorder; the first pass without entry series takes the same
    decisions on the GPU as on the host, and where it needs no series agrees with the full
    evaluation to the same rounding bound.  Cases are taken where the kernels call the near branch: the frequency inside the
    near window (half-span above 0.5 times the distance from the centre)."""
    D, W, om = _cases()
    Ds = np.sort(D, axis=1)
    c, hs = 0.5 * (Ds[:, 0] + Ds[:, 3]), 0.5 * (Ds[:, 3] - Ds[:, 0])
    keep = hs > 0.5 * np.abs(om - c)
    D, W, om, Ds = D[keep], W[keep], om[keep], Ds[keep]
    assert len(om) > 300
    order = np.argsort(D, axis=1)
    Ws = np.take_along_axis(W, order, axis=1)
    got, _ = _run(dev, 2, D=D, W=W, om=om)
    fast, need = _run(dev, 3, D=D, W=W, om=om)
    ref, scale = _oracle(D, W, om)
    err = np.abs(got - ref) / scale
    _say(f"near_eval: worst {err.max():.2e} of the weights' scale vs the oracle")
    assert err.max() < 5e-12
    for i in range(len(om)):
        out = np.zeros(2)
        yi, wi = np.ascontiguousarray(Ds[i]), np.ascontiguousarray(Ws[i])
        host.hc_near(_p(yi), _p(wi), float(om[i]), 0, _p(out))
        assert abs(got[i] - complex(out[0], out[1])) <= 2e-12 * scale[i], i
        hneed = host.hc_near_fast(_p(yi), _p(wi), float(om[i]), 0, _p(out))
        assert bool(hneed) == bool(need[i]), i
    ok = need == 0
    assert ok.sum() > 100 and (~ok).sum() > 50
    # equal to rounding: the two instantiations are compiled separately, so the device's
    # contractions may differ between them
    assert np.all(np.abs(fast[ok] - got[ok]) <= 2e-12 * scale[ok])


def test_one_frequency_weights_match_oracle(dev):
    """tetra_weight_sum (the one-frequency far series or near branch of the static kernel) on the
    GPU against the oracle at w = 0 and at other frequencies."""
    rng = np.random.default_rng(23)
    n = 800
    D = rng.uniform(0, 1.5, (n, 4)) * 10 ** rng.uniform(-4, 0, (n, 1))
    D[rng.random(n) < 0.3, 0] = 0.0
    D[n // 2:] += rng.uniform(-2, 2, (n - n // 2, 1))
    W = rng.uniform(0, 1, (n, 4))
    om = np.where(np.arange(n) < n // 2, 0.0, rng.uniform(-1, 1, n))
    got, _ = _run(dev, 5, D=D, W=W, om=om)
    ref, scale = _oracle(D, W, om)
    err = np.abs(got - ref) / scale
    _say(f"tetra_weight_sum: worst {err.max():.2e}")
    assert err.max() < 5e-12


def test_fp32_near_branch_matches_oracle(dev):
    """The mixed form's FP32 near branch (device FP32 logarithm and reciprocal) where the mixed
    kernel uses it — tetrahedra that are not near-degenerate (sorted neighbours at least the
    default 1e-6 apart) at frequencies inside the near window of the FP32 series (half-span above
    0.4 times the distance from the centre) — against the oracle.  The host build of the same code
    stays within 2e-5 of the weights' scale on these cases; the bound leaves room for the device's
    FP32 functions."""
    D, W, om = _cases(seed=29)
    Ds = np.sort(D, axis=1)
    gaps = np.min(np.diff(Ds, axis=1), axis=1)
    c, hs = 0.5 * (Ds[:, 0] + Ds[:, 3]), 0.5 * (Ds[:, 3] - Ds[:, 0])
    keep = (gaps >= 1e-6) & (hs > 0.4 * np.abs(om - c))
    D, W, om = D[keep], W[keep], om[keep]
    assert len(om) > 200
    got, _ = _run(dev, 4, D=D, W=W, om=om)
    ref, scale = _oracle(D, W, om)
    err = np.abs(got - ref) / scale
    _say(f"near_eval32: worst {err.max():.2e} over {len(om)} cases")
    assert err.max() < 1e-4
