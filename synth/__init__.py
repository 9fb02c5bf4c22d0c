"""Seeded synthetic inputs for the bare-susceptibility path.

This module only prepares inputs: tight-binding Hamiltonians, their band
energies and orbital eigenvectors on a k-mesh and at k+q, q-lists and
omega-grids.  It holds none of the susceptibility arithmetic (no matrix
elements, no carving, no weights), so the CPU oracle and the GPU library can
both consume exactly the same bytes from it.

Conventions (all fixed here, used by both sides):

* k is in fractional reciprocal coordinates.  Mesh point (i1, i2, i3) of an
  N1 x N2 x N3 Gamma-centred mesh is k = (i1/N1, i2/N2, i3/N3) and has the
  flat index (i1*N2 + i2)*N3 + i3.
* H(k) = sum_R t(R) exp(i 2 pi k.R) with integer lattice vectors R and real
  hoppings t(-R) = t(R)^T, so H is Hermitian, time-reversal symmetric
  (H(-k) = conj H(k)) and periodic in k (no orbital-position phases).
* Band energies are returned band-major, ``eps[nb][Nk]`` (float64), and the
  eigenvectors as ``c[Nk][no][nb]`` (complex128): column n of the no x nb
  block is the eigenvector of band n, bands in ascending energy.
* Energies are in eV (in units of t for the single-band cubic model); the
  Fermi level is mu = 0 and the spin factor 2 unless a config says otherwise.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "TBModel", "mesh_kfrac", "eigensystem", "sc_nn_model", "tetragonal_two_site_model",
    "bcc_spd_model", "random_model", "free_electron_eps", "Workload", "QPoint",
    "make_workload", "gamma_x_m_gamma_midpoints", "bcc_gamma_h_gamma_path", "omega_grid",
    "band_window", "random_commensurate_shifts", "batch_workloads", "plane_wave_workload",
    "cubic_s_model", "free_electron_eps_at",
]


# ---------------------------------------------------------------------------
# k-meshes
# ---------------------------------------------------------------------------

def mesh_kfrac(nk: Sequence[int]) -> np.ndarray:
    """Fractional coordinates (Nk, 3) of the Gamma-centred mesh, flat order i3 fastest."""
    n1, n2, n3 = (int(v) for v in nk)
    i1, i2, i3 = np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij")
    return np.stack([i1.ravel() / n1, i2.ravel() / n2, i3.ravel() / n3], axis=1).astype(np.float64)


# ---------------------------------------------------------------------------
# tight-binding models
# ---------------------------------------------------------------------------

@dataclass
class TBModel:
    """Real-space hoppings t(R) (no x no, real) for integer lattice vectors R."""
    name: str
    n_orb: int
    hoppings: Dict[Tuple[int, int, int], np.ndarray]
    meta: dict = field(default_factory=dict)

    def hk(self, kfrac: np.ndarray) -> np.ndarray:
        """H(k) for k of shape (Nk, 3): complex128 (Nk, no, no)."""
        kfrac = np.asarray(kfrac, dtype=np.float64)
        out = np.zeros((kfrac.shape[0], self.n_orb, self.n_orb), dtype=np.complex128)
        for R, t in self.hoppings.items():
            phase = np.exp(2j * np.pi * (kfrac @ np.asarray(R, dtype=np.float64)))
            out += phase[:, None, None] * t[None, :, :]
        return out


def _add_pair(hop: dict, R, t):
    """Insert t(R) and t(-R) = t(R)^T."""
    R = tuple(int(v) for v in R)
    mR = tuple(-v for v in R)
    if R == (0, 0, 0):
        hop[R] = hop.get(R, 0) + 0.5 * (t + t.T)
        return
    hop[R] = hop.get(R, 0) + t
    hop[mR] = hop.get(mR, 0) + t.T


def sc_nn_model(t: float = 1.0) -> TBModel:
    """Single-band simple-cubic nearest-neighbour model, eps = -2t sum_i cos(2 pi k_i)."""
    hop: dict = {}
    for R in [(1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        _add_pair(hop, R, np.array([[-t]]))
    return TBModel("sc_nn", 1, hop, {"t": t})


def cubic_s_model(seed: int, n_orb: int = 3, sigma: float = 0.5) -> TBModel:
    """Simple-cubic model with n_orb s-like orbitals per site: a seeded symmetric onsite matrix
    and one symmetric hopping matrix per shell (the 6 nearest and the 12 next-nearest neighbours),
    the same for every bond of the shell, so H(g k) = H(k) for every cubic point-group operation g
    and the bands and |<n k|m k+q>|^2 are invariant under the whole group."""
    rng = np.random.default_rng(seed)
    hop: dict = {}

    def sym(scale):
        a = rng.normal(0.0, scale, (n_orb, n_orb))
        return 0.5 * (a + a.T)

    _add_pair(hop, (0, 0, 0), np.diag(rng.uniform(-1.0, 1.0, n_orb)) + sym(0.3 * sigma))
    t1, t2 = sym(sigma), sym(0.5 * sigma)
    for R in [(1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        _add_pair(hop, R, t1)
    for R in [(1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)]:
        _add_pair(hop, R, t2)
    return TBModel("cubic_s", n_orb, hop, {"seed": seed, "sigma": sigma})


def tetragonal_two_site_model(seed: int, sigma: float = 0.3) -> TBModel:
    """Two-site tetragonal cell with 5 d-like orbitals per site (10 orbitals).

    Onsite levels U(-1, 1) eV; the R = 0 inter-site block and full 10 x 10
    blocks for the shells (1,0,0), (0,1,0), (1,1,0), (1,-1,0), (0,0,1) (and
    their negatives) are i.i.d. N(0, sigma^2) eV.
    """
    rng = np.random.default_rng(seed)
    no = 10
    hop: dict = {}
    t0 = np.zeros((no, no))
    t0[np.arange(no), np.arange(no)] = rng.uniform(-1.0, 1.0, no)
    inter = rng.normal(0.0, sigma, (5, 5))
    t0[:5, 5:] = inter
    t0[5:, :5] = inter.T
    hop[(0, 0, 0)] = t0
    for R in [(1, 0, 0), (0, 1, 0), (1, 1, 0), (1, -1, 0), (0, 0, 1)]:
        _add_pair(hop, R, rng.normal(0.0, sigma, (no, no)))
    return TBModel("tetragonal_two_site", no, hop, {"seed": seed, "sigma": sigma, "a": 1.0, "c": 1.5})


# bcc primitive vectors a1 = (-1,1,1)/2, a2 = (1,-1,1)/2, a3 = (1,1,-1)/2; a Cartesian
# lattice vector R_cart has integer coordinates n = [[0,1,1],[1,0,1],[1,1,0]] R_cart.
_BCC_TO_PRIM = np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=np.float64)


def _bcc_prim(Rcart) -> Tuple[int, int, int]:
    n = _BCC_TO_PRIM @ np.asarray(Rcart, dtype=np.float64)
    r = np.rint(n)
    assert np.allclose(n, r)
    return tuple(int(v) for v in r)


def bcc_spd_model(seed: int, n_orb: int = 9, sigma: float = 0.5) -> TBModel:
    """bcc lattice (a = 1), n_orb s,p,d-like orbitals, hoppings to 2nd neighbours.

    Onsite levels U(-1, 1) eV; each of the 8 first-neighbour vectors (+-1,+-1,+-1)/2
    and 6 second-neighbour vectors (+-1,0,0)... carries an i.i.d. N(0, sigma^2)
    block (one draw per +-R pair, t(-R) = t(R)^T).
    """
    rng = np.random.default_rng(seed)
    hop: dict = {(0, 0, 0): np.diag(rng.uniform(-1.0, 1.0, n_orb))}
    shells = [(0.5, 0.5, 0.5), (0.5, 0.5, -0.5), (0.5, -0.5, 0.5), (-0.5, 0.5, 0.5),
              (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    for Rc in shells:
        _add_pair(hop, _bcc_prim(Rc), rng.normal(0.0, sigma, (n_orb, n_orb)))
    return TBModel("bcc_spd", n_orb, hop, {"seed": seed, "sigma": sigma})


def random_model(kind: str, seed: int, n_orb: int) -> TBModel:
    """Model families used by the batched workload: 'tetragonal', 'bcc' or 'sc'."""
    rng = np.random.default_rng(seed)
    if kind == "bcc":
        return bcc_spd_model(seed, n_orb=n_orb, sigma=0.5)
    hop: dict = {(0, 0, 0): np.diag(rng.uniform(-1.0, 1.0, n_orb))}
    if kind == "tetragonal":
        shells = [(1, 0, 0), (0, 1, 0), (1, 1, 0), (1, -1, 0), (0, 0, 1)]
        sigma = 0.3
    elif kind == "sc":
        shells = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
        sigma = 0.4
    else:
        raise ValueError(kind)
    for R in shells:
        _add_pair(hop, R, rng.normal(0.0, sigma, (n_orb, n_orb)))
    return TBModel(kind, n_orb, hop, {"seed": seed, "sigma": sigma})


def eigensystem(model: TBModel, kfrac: np.ndarray, chunk: int = 65536):
    """Band energies eps[nb][Nk] (float64) and eigenvectors c[Nk][no][nb] (complex128)."""
    nk = kfrac.shape[0]
    no = model.n_orb
    eps = np.empty((no, nk), dtype=np.float64)
    c = np.empty((nk, no, no), dtype=np.complex128)
    for s in range(0, nk, chunk):
        e, v = np.linalg.eigh(model.hk(kfrac[s:s + chunk]))
        eps[:, s:s + chunk] = e.T
        c[s:s + chunk] = v
    return eps, c


def free_electron_eps(nk: Sequence[int], q_cart=(0.0, 0.0, 0.0)) -> np.ndarray:
    """eps = |k + q|^2 / 2 on the index mesh spanning [-pi, pi)^3 (a = 1), shape (1, Nk)."""
    n = np.asarray(nk)
    frac = mesh_kfrac(nk)
    k = 2.0 * np.pi * frac - np.pi + np.asarray(q_cart, dtype=np.float64)[None, :]
    return (0.5 * np.sum(k * k, axis=1))[None, :].copy()


def free_electron_eps_at(kfrac: np.ndarray, q_cart=(0.0, 0.0, 0.0)) -> np.ndarray:
    """eps = |k + q|^2 / 2 at k = 2 pi kfrac (Gamma-centred fractional points, a = 1), shape (1, n)."""
    k = 2.0 * np.pi * np.asarray(kfrac, dtype=np.float64) + np.asarray(q_cart, dtype=np.float64)[None, :]
    return (0.5 * np.sum(k * k, axis=1))[None, :].copy()


# ---------------------------------------------------------------------------
# q-lists and omega grids
# ---------------------------------------------------------------------------

def gamma_x_m_gamma_midpoints(nq: int) -> np.ndarray:
    """nq points at arc-length midpoints of Gamma-X-M-Gamma at kz = 0 (fractional)."""
    corners = np.array([[0, 0, 0], [0.5, 0, 0], [0.5, 0.5, 0], [0, 0, 0]], dtype=np.float64)
    seg = np.linalg.norm(np.diff(corners, axis=0), axis=1)
    total = seg.sum()
    s = (np.arange(nq) + 0.5) * total / nq
    out = np.empty((nq, 3))
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    for i, si in enumerate(s):
        j = min(int(np.searchsorted(cum, si, side="right")) - 1, 2)
        f = (si - cum[j]) / seg[j]
        out[i] = corners[j] + f * (corners[j + 1] - corners[j])
    return out


def bcc_gamma_h_gamma_path(nq: int) -> np.ndarray:
    """q = y (0,1,0) 2pi/a, y_j = 2(j - 1/2)/nq, as bcc fractional coordinates y (1/2, -1/2, 1/2)."""
    y = 2.0 * (np.arange(1, nq + 1) - 0.5) / nq
    return y[:, None] * np.array([[0.5, -0.5, 0.5]])


def omega_grid(nw: int, w_max: float = 2.0) -> np.ndarray:
    return np.linspace(0.0, w_max, nw)


def random_commensurate_shifts(rng: np.random.Generator, nk: Sequence[int], nq: int) -> np.ndarray:
    """nq random non-zero integer mesh shifts (shift not congruent to 0)."""
    out = []
    while len(out) < nq:
        s = [int(rng.integers(0, n)) for n in nk]
        if any(v != 0 for v in s):
            out.append(s)
    return np.asarray(out, dtype=np.int32)


def band_window(eps: np.ndarray, n_keep: int, mu: float = 0.0) -> Tuple[int, int]:
    """Contiguous window of n_keep bands whose mean mesh energy is closest to mu (ties: lower)."""
    nb = eps.shape[0]
    if n_keep >= nb:
        return 0, nb
    best, best_lo = None, 0
    for lo in range(0, nb - n_keep + 1):
        d = abs(float(eps[lo:lo + n_keep].mean()) - mu)
        if best is None or d < best:
            best, best_lo = d, lo
    return best_lo, best_lo + n_keep


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

@dataclass
class QPoint:
    """One q: either an integer mesh shift, or explicit k+q band data on the same mesh."""
    q_frac: np.ndarray
    shift: Optional[Tuple[int, int, int]] = None
    eps_kq: Optional[np.ndarray] = None   # [nb][Nk]
    c_kq: Optional[np.ndarray] = None     # [Nk][no][nb]


@dataclass
class Workload:
    name: str
    nk: Tuple[int, int, int]
    eps_k: np.ndarray                 # [nb][Nk] float64
    c_k: Optional[np.ndarray]         # [Nk][no][nb] complex128, None under CMA
    qs: List[QPoint]
    omega: np.ndarray                 # [nw]
    mu: float = 0.0
    spin_factor: float = 2.0
    cma: bool = False
    form: int = 0
    band_lo: int = 0
    band_hi: int = -1
    static: bool = False
    meta: dict = field(default_factory=dict)

    @property
    def n_bands(self) -> int:
        return self.eps_k.shape[0]

    @property
    def n_orb(self) -> int:
        return 1 if self.c_k is None else self.c_k.shape[1]

    @property
    def n_k(self) -> int:
        return int(np.prod(self.nk))

    def window(self) -> Tuple[int, int]:
        hi = self.n_bands if self.band_hi < 0 else self.band_hi
        return self.band_lo, hi

    def nominal_units(self) -> int:
        lo, hi = self.window()
        nw = 1 if self.static else len(self.omega)
        return len(self.qs) * 6 * self.n_k * (hi - lo) ** 2 * nw


def _explicit_q(model: TBModel, kf: np.ndarray, q: np.ndarray) -> QPoint:
    e, c = eigensystem(model, kf + q[None, :])
    return QPoint(q_frac=np.asarray(q, dtype=np.float64), eps_kq=e, c_kq=c)


def _explicit_qs(model: TBModel, kf: np.ndarray, qlist, workers: int = 1) -> List[QPoint]:
    """Explicit k+q eigensystems for every q (optionally in worker processes; same bytes)."""
    qlist = [np.asarray(q, dtype=np.float64) for q in qlist]
    if workers <= 1 or len(qlist) <= 1:
        return [_explicit_q(model, kf, q) for q in qlist]
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        return list(ex.map(_explicit_q, [model] * len(qlist), [kf] * len(qlist), qlist))


def make_workload(name: str, nk=None, nq: Optional[int] = None, nw: Optional[int] = None,
                  q_subset: Optional[Sequence[int]] = None, n_keep: Optional[int] = None,
                  workers: int = 1) -> Workload:
    """Build one of the seeded workloads.

    name:
      'sc_cma'        single-band SC NN model (t=1, mu=0), CMA, static, q_j = (j/N)(1,1,1), j=1..8
                      (commensurate mesh shift (j,j,j)); default mesh 16^3.
      'tetra_static'  10-orbital two-site tetragonal model (seed 2), static, q at midpoints of
                      Gamma-X-M-Gamma (explicit k+q); default mesh 64x64x8, 256 q.
      'bcc_dynamic'   9-orbital bcc model (seed 3), q along (010) Gamma-H-Gamma (explicit k+q),
                      omega on [0, 2] eV; default mesh 48^3, 64 q x 512 omega, band window n_keep.
      'tetra_dynamic' the 'tetra_static' model at 64 q (midpoints of the same path) x 512 omega.
    nk / nq / nw override the mesh, number of q on the path and omega count (smaller test sizes);
    q_subset keeps only those indices of the q-list (the k+q eigensystems are only built for them);
    workers > 1 builds the k+q eigensystems in that many processes (identical results).
    """
    if name == "sc_cma":
        nk = tuple(nk or (16, 16, 16))
        model = sc_nn_model(1.0)
        kf = mesh_kfrac(nk)
        eps, _ = eigensystem(model, kf)
        nq = nq or 8
        qs = []
        # q_j = (j/16)(1,1,1) for j < 8 as mesh shifts; the R point itself (j = 8) is the exact
        # nesting eps(k+q) = -eps(k) of the half-filled band, where the tetrahedron integral
        # diverges logarithmically, so the last point is (15/32)(1,1,1) with explicit k+q.
        for j in range(1, nq + 1):
            if j < 8 and all(n % 16 == 0 for n in nk):
                s = tuple(j * n // 16 for n in nk)
                qs.append(QPoint(q_frac=np.array(s, dtype=np.float64) / np.array(nk), shift=s))
            else:
                qf = np.full(3, (j / 16.0) if j < 8 else 15.0 / 32.0)
                e_kq, _ = eigensystem(model, kf + qf[None, :])
                qs.append(QPoint(q_frac=qf, eps_kq=e_kq))
        if q_subset is not None:
            qs = [qs[i] for i in q_subset]
        return Workload(name, nk, eps, None, qs, np.zeros(1), cma=True, static=True,
                        meta={"model": "sc_nn", "t": 1.0})
    if name in ("tetra_static", "tetra_dynamic"):
        dyn = name == "tetra_dynamic"
        nk = tuple(nk or (64, 64, 8))
        model = tetragonal_two_site_model(2)
        kf = mesh_kfrac(nk)
        eps, c = eigensystem(model, kf)
        qlist = gamma_x_m_gamma_midpoints(nq or (64 if dyn else 256))
        idx = range(len(qlist)) if q_subset is None else q_subset
        qs = _explicit_qs(model, kf, [qlist[i] for i in idx], workers)
        omega = omega_grid(nw or 512) if dyn else np.zeros(1)
        return Workload(name, nk, eps, c, qs, omega, static=not dyn,
                        meta={"model": "tetragonal_two_site", "seed": 2, "q_index": list(idx)})
    if name == "bcc_dynamic":
        nk = tuple(nk or (48, 48, 48))
        model = bcc_spd_model(3)
        kf = mesh_kfrac(nk)
        eps, c = eigensystem(model, kf)
        qlist = bcc_gamma_h_gamma_path(nq or 64)
        idx = range(len(qlist)) if q_subset is None else q_subset
        qs = _explicit_qs(model, kf, [qlist[i] for i in idx], workers)
        lo, hi = band_window(eps, n_keep or 9)
        return Workload(name, nk, eps, c, qs, omega_grid(nw or 512), band_lo=lo, band_hi=hi,
                        meta={"model": "bcc_spd", "seed": 3, "q_index": list(idx), "n_keep": n_keep or 9})
    raise ValueError(f"unknown workload {name!r}")


def model_workload(model: TBModel, nk, q_fracs: Sequence, omega: np.ndarray, static: bool = False,
                   shifts: Optional[Sequence] = None, **kw) -> Workload:
    """A workload for an arbitrary model: explicit k+q for q_fracs, or integer mesh shifts."""
    nk = tuple(int(v) for v in nk)
    kf = mesh_kfrac(nk)
    eps, c = eigensystem(model, kf)
    qs = []
    if shifts is not None:
        for s in shifts:
            s = tuple(int(v) for v in s)
            qs.append(QPoint(q_frac=np.array(s, dtype=np.float64) / np.array(nk), shift=s))
    else:
        for q in q_fracs:
            qs.append(_explicit_q(model, kf, np.asarray(q, dtype=np.float64)))
    return Workload(model.name, nk, eps, c, qs, np.asarray(omega, dtype=np.float64), static=static, **kw)


def batch_workloads(nq_div: int = 1, precision: int = 0) -> List[Tuple[Workload, int]]:
    """The 16-instance heterogeneous batch (seeds 500..515).

    Instance i: lattice family tetragonal / bcc / sc in turn, n_orb = 4 + round(28 i / 15) orbitals
    (all bands kept), an L^3 mesh with L = 48, 40, 32, 24 for i in blocks of four, nq = 128 -
    round(96 i / 15) random non-zero commensurate mesh shifts (divided by nq_div, at least 1) and
    nw = 512 - round(384 i / 15) frequencies on [0, 2] eV.  Large meshes pair with few orbitals
    and many q and frequencies, so the per-instance work stays within a factor of a few.
    Returns (workload, precision) pairs.
    """
    kinds = ("tetragonal", "bcc", "sc")
    out = []
    for i in range(16):
        seed = 500 + i
        n_orb = 4 + int(round(28 * i / 15))
        L = (48, 40, 32, 24)[i // 4]
        nq = max(1, (128 - int(round(96 * i / 15))) // nq_div)
        nw = 512 - int(round(384 * i / 15))
        model = random_model(kinds[i % 3], seed, n_orb)
        rng = np.random.default_rng(seed)
        shifts = random_commensurate_shifts(rng, (L, L, L), nq)
        wl = model_workload(model, (L, L, L), None, omega_grid(nw), shifts=shifts)
        wl.name = "batch%02d_%s" % (i, model.name)
        wl.meta = {"model": model.name, "seed": seed, "n_orb": n_orb, "mesh": L, "nq": nq, "nw": nw}
        out.append((wl, precision))
    return out


def plane_wave_workload(nk, n_pw: int, nb: int, nq: int, nw: int, seed: int = 7) -> Workload:
    """Large-basis (plane-wave) stand-in: band energies of a seeded nb-orbital tetragonal model,
    and at every k nb orthonormal eigenvector columns in an n_pw-dimensional plane-wave space
    (Cholesky QR of a seeded complex Gaussian matrix), so matrix elements are sums over n_pw coefficients
    (Sec. III: about 4000 plane waves).  q: nq random non-zero commensurate shifts.  The
    coefficients are not smooth in k; they exercise the contraction, not the physics."""
    nk = tuple(int(v) for v in nk)
    model = random_model("tetragonal", seed, nb)
    kf = mesh_kfrac(nk)
    eps, _ = eigensystem(model, kf)
    rng = np.random.default_rng(seed + 1000)
    nkt = kf.shape[0]
    c = np.empty((nkt, n_pw, nb), dtype=np.complex128)
    for k0 in range(0, nkt, 64):
        k1 = min(nkt, k0 + 64)
        a = rng.standard_normal((k1 - k0, n_pw, nb)) + 1j * rng.standard_normal((k1 - k0, n_pw, nb))
        # orthonormal columns by Cholesky QR (a Gaussian block is well conditioned)
        g = np.matmul(a.conj().transpose(0, 2, 1), a)
        r_inv = np.linalg.inv(np.linalg.cholesky(g).conj().transpose(0, 2, 1))
        c[k0:k1] = np.matmul(a, r_inv)
    shifts = random_commensurate_shifts(rng, nk, nq)
    qs = [QPoint(q_frac=np.array(sh, dtype=np.float64) / np.array(nk), shift=tuple(int(v) for v in sh)) for sh in shifts]
    return Workload("plane_wave", nk, eps, c, qs, omega_grid(nw),
                    meta={"model": "tetragonal", "seed": seed, "n_pw": n_pw, "nb": nb})
