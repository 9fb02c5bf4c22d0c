"""CPU FP64 oracle for chi0(q, omega) -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it.  The arithmetic lives in ``chi0_oracle.c`` (plain C,
FP64, OpenMP over mesh cells); this module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chi0_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_chi0.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-shared", "-fPIC",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i, d, ll = ctypes.c_int, ctypes.c_double, ctypes.c_longlong
        lib.chi0_oracle.argtypes = [i, i, i, i, i, dp, dp, dp, dp, i, i, i, d, d, i, i, i, i, i, dp,
                                    ll, ll, i, dp]
        lib.chi0_oracle.restype = i
        lib.chi0_oracle_pairs.argtypes = [i, i, i, i, i, dp, dp, dp, dp, i, i, i, d, d, i, i, i, i, i, dp, i, dp]
        lib.chi0_oracle_pairs.restype = i
        lib.chi0_oracle_moments.argtypes = [i, i, i, i, i, dp, dp, dp, dp, i, i, i, d, d, i, i, i, i, dp]
        lib.chi0_oracle_moments.restype = i
        lib.chi0_oracle_weights.argtypes = [dp, d, dp]
        lib.chi0_oracle_weights.restype = None
        lib.chi0_oracle_dd5.argtypes = [dp, d, dp]
        lib.chi0_oracle_dd5.restype = None
        lib.chi0_oracle_carve.argtypes = [dp, dp, i, dp, dp]
        lib.chi0_oracle_carve.restype = i
        lib.chi0_oracle_list.argtypes = [i, i, i, dp, dp, dp, dp, ll, ctypes.POINTER(ctypes.c_int), d, d, d, i, i,
                                         i, i, i, i, dp, i, dp]
        lib.chi0_oracle_list.restype = i
        lib.chi0_oracle_z.argtypes = [i, i, i, i, i, dp, dp, dp, dp, i, i, i, d, d, i, i, i, i, dp, d, i, dp]
        lib.chi0_oracle_z.restype = i
        ull = ctypes.POINTER(ctypes.c_ulonglong)
        lib.chi0_oracle_last_count.argtypes = [ull, ull]
        lib.chi0_oracle_last_count.restype = None
        lib.chi0_oracle_W.argtypes = [i, i, i, i, i, dp, dp, dp, dp, i, i, i, i, i, dp]
        lib.chi0_oracle_W.restype = i
        lib.chi0_oracle_tet_corners.argtypes = [i, i, i, ll, i, ctypes.POINTER(ctypes.c_longlong)]
        lib.chi0_oracle_tet_corners.restype = None
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _c128_as_f64(a):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a.view(np.float64)


def chi0_raw(nk, eps_k, c_k, omega, *, eps_kq=None, c_kq=None, shift=(0, 0, 0), mu=0.0,
             spin_factor=2.0, band_lo=0, band_hi=-1, cma=False, form=0,
             cells: Optional[Sequence[int]] = None, nthreads: int = 0) -> np.ndarray:
    """chi0 at one q for all omega: complex array [nw]."""
    lib = _load()
    eps_k = _f64(eps_k)
    nb = eps_k.shape[0]
    no = 1 if c_k is None else c_k.shape[1]
    ck = _c128_as_f64(c_k)
    ekq = _f64(eps_kq)
    ckq = _c128_as_f64(c_kq)
    omega = _f64(np.atleast_1d(omega))
    out = np.zeros((omega.size, 2))
    c0, c1 = (0, -1) if cells is None else (int(cells[0]), int(cells[1]))
    rc = lib.chi0_oracle(int(nk[0]), int(nk[1]), int(nk[2]), nb, no, _ptr(eps_k), _ptr(ck), _ptr(ekq),
                         _ptr(ckq), int(shift[0]), int(shift[1]), int(shift[2]), float(mu),
                         float(spin_factor), int(band_lo), int(band_hi), int(bool(cma)), int(form),
                         omega.size, _ptr(omega), c0, c1, int(nthreads), _ptr(out))
    if rc != 0:
        raise ValueError("chi0_oracle failed with code %d" % rc)
    return out[:, 0] + 1j * out[:, 1]


def chi0_z_raw(nk, eps_k, c_k, omega, eta: float, *, eps_kq=None, c_kq=None, shift=(0, 0, 0), mu=0.0,
               spin_factor=2.0, band_lo=0, band_hi=-1, cma=False, nthreads: int = 0) -> np.ndarray:
    """The same tetrahedron integral (difference form) at complex frequencies z = omega + i eta,
    eta >= 0: complex array [nw].  eta = 0 is chi0_raw's retarded result."""
    lib = _load()
    eps_k = _f64(eps_k)
    nb = eps_k.shape[0]
    no = 1 if c_k is None else c_k.shape[1]
    omega = _f64(np.atleast_1d(omega))
    out = np.zeros((omega.size, 2))
    rc = lib.chi0_oracle_z(int(nk[0]), int(nk[1]), int(nk[2]), nb, no, _ptr(eps_k), _ptr(_c128_as_f64(c_k)),
                           _ptr(_f64(eps_kq)), _ptr(_c128_as_f64(c_kq)), int(shift[0]), int(shift[1]),
                           int(shift[2]), float(mu), float(spin_factor), int(band_lo), int(band_hi),
                           int(bool(cma)), omega.size, _ptr(omega), float(eta), int(nthreads), _ptr(out))
    if rc != 0:
        raise ValueError("chi0_oracle_z failed with code %d" % rc)
    return out[:, 0] + 1j * out[:, 1]


def chi0_list(eps_k, c_k, eps_kq, c_kq, tets, volume: float, omega, *, mu=0.0, spin_factor=2.0, band_lo=0,
              band_hi=-1, cma=False, form=0, single_carving=False, nthreads: int = 0) -> np.ndarray:
    """chi0 at one q over an explicit list of tetrahedra (corner indices tets [n_tet][4] into the
    k-points of eps_k [nb][n_kp]; eps_kq/c_kq hold the data at the same points shifted by q; each
    tetrahedron is the fraction `volume` of the zone): complex array [nw].  single_carving (form 1
    only) is the comparison treatment without the second carving."""
    lib = _load()
    eps_k = _f64(eps_k)
    nb, n_kp = eps_k.shape
    no = 1 if c_k is None else c_k.shape[1]
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    omega = _f64(np.atleast_1d(omega))
    out = np.zeros((omega.size, 2))
    ck, ckq = (None, None) if cma else (_c128_as_f64(c_k), _c128_as_f64(c_kq))
    rc = lib.chi0_oracle_list(int(n_kp), nb, no, _ptr(eps_k), _ptr(ck), _ptr(_f64(eps_kq)), _ptr(ckq),
                              tets.shape[0], tets.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), float(volume),
                              float(mu), float(spin_factor), int(band_lo), int(band_hi), int(bool(cma)), int(form),
                              int(bool(single_carving)), omega.size, _ptr(omega), int(nthreads), _ptr(out))
    if rc != 0:
        raise ValueError("chi0_oracle_list failed with code %d" % rc)
    return out[:, 0] + 1j * out[:, 1]


def cubic_point_group() -> np.ndarray:
    """The 48 operations of O_h as integer matrices acting on fractional coordinates of a simple
    cubic reciprocal lattice (signed permutation matrices), identity first."""
    import itertools
    ops = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            g = np.zeros((3, 3), dtype=np.int64)
            for r in range(3):
                g[r, perm[r]] = signs[r]
            ops.append(g)
    ops.sort(key=lambda g: (not np.array_equal(g, np.eye(3, dtype=np.int64)),))
    return np.array(ops)


def iw_cubic(n: int):
    """Irreducible wedge of a Gamma-centred n x n x n simple-cubic mesh (n even) under O_h,
    decomposed into tetrahedra (Sec. II, Fig. 1(a)).

    The wedge is 0 <= z <= y <= x <= 1/2 (fractional).  A cube of the mesh with integer corner
    (i, j, l), i >= j >= l, splits into six tetrahedra by the order in which the three axes are
    stepped from its corner to the opposite one; a tetrahedron lies in the wedge unless the cube
    sits on the plane x = y (i == j) and the tetrahedron steps y before x, or on y = z (j == l)
    and it steps z before y.  Returns (kfrac [n_kp][3], tets [n_tet][4] int32, volume of one
    tetrahedron as a fraction of the zone)."""
    import itertools
    if n < 2 or n % 2:
        raise ValueError("n must be even and >= 2")
    m = n // 2
    pts = [(i, j, l) for i in range(m + 1) for j in range(i + 1) for l in range(j + 1)]
    where = {p: t for t, p in enumerate(pts)}
    tets = []
    for i in range(m):
        for j in range(i + 1):
            for l in range(j + 1):
                for order in itertools.permutations(range(3)):
                    rank = {ax: r for r, ax in enumerate(order)}
                    if i == j and rank[0] > rank[1]:
                        continue
                    if j == l and rank[1] > rank[2]:
                        continue
                    c = [i, j, l]
                    corners = [where[tuple(c)]]
                    for ax in order:
                        c[ax] += 1
                        corners.append(where[tuple(c)])
                    tets.append(corners)
    kfrac = np.array(pts, dtype=np.float64) / n
    return kfrac, np.array(tets, dtype=np.int32), 1.0 / (6.0 * n ** 3)


def chi0_iw(eps_k, c_k, entries, tets, volume: float, omega, **kw) -> np.ndarray:
    """The point-group loop of Sec. II: the second carving is repeated for every point-group
    element g, each with the k+q data of the wedge's points taken at k + g^-1 q; entries is the
    list of (eps_kq, c_kq) per g and the result the sum of the per-g wedge integrals."""
    total = None
    for eps_kq, c_kq in entries:
        part = chi0_list(eps_k, c_k, eps_kq, c_kq, tets, volume, omega, **kw)
        total = part if total is None else total + part
    return total


def chi0(wl, q_index: int, omega=None, cells=None, nthreads: int = 0, form: Optional[int] = None) -> np.ndarray:
    """chi0 of a synth.Workload at one of its q for the given omegas (default: all)."""
    q = wl.qs[q_index]
    om = (np.zeros(1) if wl.static else wl.omega) if omega is None else np.atleast_1d(omega)
    lo, hi = wl.window()
    return chi0_raw(wl.nk, wl.eps_k, wl.c_k, om, eps_kq=q.eps_kq, c_kq=q.c_kq,
                    shift=q.shift if q.shift is not None else (0, 0, 0), mu=wl.mu,
                    spin_factor=wl.spin_factor, band_lo=lo, band_hi=hi, cma=wl.cma,
                    form=wl.form if form is None else form, cells=cells, nthreads=nthreads)


def last_count():
    """(operations, active units) of the last chi0 / chi0_raw / chi0_z_raw call: the oracle's own
    floating-point operation tally (weights in chi0_oracle.c) and the (mesh tetrahedron, band pair)
    units with a non-empty carved region."""
    lib = _load()
    ops, units = ctypes.c_ulonglong(0), ctypes.c_ulonglong(0)
    lib.chi0_oracle_last_count(ctypes.byref(ops), ctypes.byref(units))
    return int(ops.value), int(units.value)


def chi0_pairs(wl, q_index: int, omega=None, nthreads: int = 0, form: Optional[int] = None) -> np.ndarray:
    """chi0 resolved by band pair: complex array [nbw][nbw][nw] whose sum over pairs is chi0()."""
    lib = _load()
    q = wl.qs[q_index]
    om = _f64(np.atleast_1d((np.zeros(1) if wl.static else wl.omega) if omega is None else omega))
    lo, hi = wl.window()
    nbw = hi - lo
    eps_k = _f64(wl.eps_k)
    ck = _c128_as_f64(wl.c_k)
    ekq = _f64(q.eps_kq)
    ckq = _c128_as_f64(q.c_kq)
    s = q.shift if q.shift is not None else (0, 0, 0)
    out = np.zeros((nbw, nbw, om.size, 2))
    rc = lib.chi0_oracle_pairs(int(wl.nk[0]), int(wl.nk[1]), int(wl.nk[2]), wl.n_bands, wl.n_orb,
                               _ptr(eps_k), _ptr(ck), _ptr(ekq), _ptr(ckq), int(s[0]), int(s[1]), int(s[2]),
                               float(wl.mu), float(wl.spin_factor), lo, hi, int(bool(wl.cma)),
                               int(wl.form if form is None else form), om.size, _ptr(om), int(nthreads),
                               _ptr(out))
    if rc != 0:
        raise ValueError("chi0_oracle_pairs failed with code %d" % rc)
    return out[..., 0] + 1j * out[..., 1]


def kk_tent_matrix(omega, lo: float, hi: float, n_spec: int) -> np.ndarray:
    """L[i, k] = P int hat_k(w') / (w' - omega_i) dw' for the tents hat_k of the uniform grid
    w'_k = lo + k h on [lo, hi] (n_spec points), written out from the antiderivative
    phi(x) = x ln|x| of the integrand: L = [phi(x + h) - 2 phi(x) + phi(x - h)] / h, x = w'_k - omega_i
    (Sec. II: Re and Im of chi0 are connected by the Kramers-Kronig transformation)."""
    om = np.atleast_1d(np.asarray(omega, dtype=np.float64))
    h = (hi - lo) / (n_spec - 1)
    x = (lo + h * np.arange(n_spec))[None, :] - om[:, None]

    def phi(z):
        out = np.zeros_like(z)
        nz = z != 0.0
        out[nz] = z[nz] * np.log(np.abs(z[nz]))
        return out
    direct = (phi(x + h) - 2.0 * phi(x) + phi(x - h)) / h
    with np.errstate(divide="ignore", invalid="ignore"):
        t = h / x
        series = np.log1p(-t * t) / t + np.log1p(t) - np.log1p(-t)
    return np.where(np.abs(x) > 2.0 * h, series, direct)


def chi0_kk(wl, q_index: int, omega, n_spec: int, lo: float, hi: float, nthreads: int = 0) -> np.ndarray:
    """The Kramers-Kronig route: Im chi0 exactly at omega, Re chi0 at omega as the principal-value
    transform (1/pi) P int Im(w')/(w' - w) dw' of the piecewise-linear interpolant of Im on the
    uniform grid of n_spec points over [lo, hi] (zero one spacing beyond each end)."""
    om = np.atleast_1d(np.asarray(omega, dtype=np.float64))
    grid = lo + (hi - lo) / (n_spec - 1) * np.arange(n_spec)
    im_grid = chi0(wl, q_index, omega=grid, nthreads=nthreads).imag
    im_direct = chi0(wl, q_index, omega=om, nthreads=nthreads).imag
    re = kk_tent_matrix(om, lo, hi, n_spec) @ im_grid / np.pi
    return re + 1j * im_direct


def matrix_elements_raw(nk, c_k, *, c_kq=None, shift=(0, 0, 0), band_lo=0, band_hi=-1) -> np.ndarray:
    """W[n, m, k] = |sum_o conj(c_{o,n}(k)) c_{o,m}(k+q)|^2 (n at k, m at k+q, relative to band_lo)
    for eigenvectors c_k [Nk][no][nb] and the k+q data c_kq (same layout) or the mesh shift."""
    lib = _load()
    ck = _c128_as_f64(c_k)
    nkt, no, nb = c_k.shape
    lo, hi = int(band_lo), (nb if band_hi is None or band_hi < 0 else int(band_hi))
    eps = np.zeros((nb, nkt))          # energies do not enter W
    ckq = _c128_as_f64(c_kq)
    out = np.zeros((hi - lo, hi - lo, nkt))
    rc = lib.chi0_oracle_W(int(nk[0]), int(nk[1]), int(nk[2]), nb, no, _ptr(eps), _ptr(ck),
                           _ptr(eps if c_kq is not None else None), _ptr(ckq), int(shift[0]), int(shift[1]),
                           int(shift[2]), lo, hi, _ptr(out))
    if rc != 0:
        raise ValueError("chi0_oracle_W failed with code %d" % rc)
    return out


def matrix_elements(wl, q_index: int) -> np.ndarray:
    """W of a synth.Workload at one of its q over its band window: [nbw][nbw][Nk]."""
    q = wl.qs[q_index]
    lo, hi = wl.window()
    return matrix_elements_raw(wl.nk, wl.c_k, c_kq=q.c_kq, shift=q.shift if q.shift is not None else (0, 0, 0),
                               band_lo=lo, band_hi=hi)


def moments(wl, q_index: int, pmax: int = 6) -> np.ndarray:
    """Exact moments mom[p] of the carved integrand: chi0(w) = sum_p mom[p]/w^(p+1) at large w."""
    lib = _load()
    q = wl.qs[q_index]
    lo, hi = wl.window()
    eps_k = _f64(wl.eps_k)
    ck = _c128_as_f64(wl.c_k)
    ekq = _f64(q.eps_kq)
    ckq = _c128_as_f64(q.c_kq)
    s = q.shift if q.shift is not None else (0, 0, 0)
    out = np.zeros(pmax + 1)
    rc = lib.chi0_oracle_moments(int(wl.nk[0]), int(wl.nk[1]), int(wl.nk[2]), wl.n_bands, wl.n_orb,
                                 _ptr(eps_k), _ptr(ck), _ptr(ekq), _ptr(ckq), int(s[0]), int(s[1]),
                                 int(s[2]), float(wl.mu), float(wl.spin_factor), lo, hi,
                                 int(bool(wl.cma)), pmax, _ptr(out))
    if rc != 0:
        raise ValueError("chi0_oracle_moments failed with code %d" % rc)
    return out


def weights(D: Sequence[float], w: float) -> np.ndarray:
    """Corner weights J_j (complex, 4) of 1/(w - D + i0) on a simplex with corner values D."""
    lib = _load()
    D = np.ascontiguousarray(D, dtype=np.float64)
    out = np.zeros(8)
    lib.chi0_oracle_weights(_ptr(D), float(w), _ptr(out))
    return out[0::2] + 1j * out[1::2]


def dd5(nodes: Sequence[float], w: float) -> complex:
    lib = _load()
    x = np.ascontiguousarray(nodes, dtype=np.float64)
    out = np.zeros(2)
    lib.chi0_oracle_dd5(_ptr(x), float(w), _ptr(out))
    return complex(out[0], out[1])


def carve(a: Sequence[float], b: Sequence[float], region: int):
    """Final tetrahedra (barycentric vertices [n][4][4], volume fractions [n]) of a region."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    verts = np.zeros((9, 4, 4))
    vols = np.zeros(9)
    n = lib.chi0_oracle_carve(_ptr(a), _ptr(b), int(region), _ptr(verts), _ptr(vols))
    return verts[:n].copy(), vols[:n].copy()


def tet_corners(nk, cell: int, t: int) -> np.ndarray:
    lib = _load()
    out = (ctypes.c_longlong * 4)()
    lib.chi0_oracle_tet_corners(int(nk[0]), int(nk[1]), int(nk[2]), int(cell), int(t), out)
    return np.array(list(out), dtype=np.int64)
