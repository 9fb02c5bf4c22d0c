"""Python binding of libchi0 (MI355X / gfx950 bare-susceptibility library).

Argument marshalling only: every step of the computation (matrix elements,
carving, tetrahedron weights, reduction) runs in the HIP kernels of
``libchi0.so``; PyTorch provides device memory and the stream.  There is no
CPU fallback: if the library is missing, or no GPU is present, the calls raise.

    plan = Chi0Plan(nk, eps_k, c_k, mu=0.0)          # device tensors
    chi_static = plan.static([Q(shift=(1, 1, 1))])  # float64 [nq]
    chi = plan.dynamic([Q(eps_kq=e, c_kq=c)], omega) # complex128 [nq, nw]
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

# The counts of chi0_census, in the order of its counts[] array.
CENSUS_KEYS = ("active_units", "final_tetrahedra", "near_evals", "far_evals", "far_terms", "near_redo",
               "coef_terms")

__all__ = ["Chi0Plan", "Chi0Batch", "Instance", "Q", "Chi0Error", "load_library", "LIB_PATH", "iw_cubic",
           "EXPORTED_SYMBOLS"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libchi0.so")

EXPORTED_SYMBOLS = ["chi0_plan", "chi0_workspace_size", "chi0_static", "chi0_static_pairs", "chi0_dynamic",
                    "chi0_dynamic_noalloc", "chi0_dynamic_pairs", "chi0_dynamic_pairs_workspace_size",
                    "chi0_kk_workspace_size", "chi0_dynamic_kk", "chi0_plan_list", "chi0_static_group",
                    "chi0_dynamic_group", "chi0_iw_cubic",
                    "chi0_matrix_elements", "chi0_profile_enable", "chi0_profile_read", "chi0_census",
                    "chi0_sync", "chi0_destroy", "chi0_status_string", "chi0_last_error", "chi0_batch_workspace_size",
                    "chi0_batch_create", "chi0_batch_run", "chi0_batch_tune", "chi0_batch_info_get",
                    "chi0_batch_destroy", "chi0_batch_last_error"]

STATUS = {0: "CHI0_OK", -1: "CHI0_E_INVALID_ARG", -2: "CHI0_E_SHAPE", -3: "CHI0_E_NONFINITE",
          -4: "CHI0_E_NOT_COMMENSURATE", -5: "CHI0_E_WORKSPACE", -6: "CHI0_E_DEVICE", -7: "CHI0_E_UNSUPPORTED",
          -8: "CHI0_E_NOT_NORMALIZED"}


class Chi0Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Desc(ctypes.Structure):
    _fields_ = [("nk", ctypes.c_int32 * 3), ("n_bands", ctypes.c_int32), ("n_orb", ctypes.c_int32),
                ("band_lo", ctypes.c_int32), ("band_hi", ctypes.c_int32), ("cma", ctypes.c_int32),
                ("form", ctypes.c_int32), ("precision", ctypes.c_int32), ("batch_hint", ctypes.c_int32),
                ("skip_input_scan", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3),
                ("mu", ctypes.c_double), ("spin_factor", ctypes.c_double), ("degen_tol_ev", ctypes.c_double),
                ("degen_rel_tol", ctypes.c_double)]


class _Q(ctypes.Structure):
    _fields_ = [("shift", ctypes.c_int32 * 3), ("explicit_kq", ctypes.c_int32),
                ("eps_kq", ctypes.c_void_p), ("c_kq", ctypes.c_void_p), ("q_frac", ctypes.c_double * 3)]


class _Instance(ctypes.Structure):
    _fields_ = [("desc", _Desc), ("eps_k", ctypes.c_void_p), ("c_k", ctypes.c_void_p), ("nq", ctypes.c_int32),
                ("nw", ctypes.c_int32), ("qs", ctypes.POINTER(_Q)), ("omega", ctypes.c_void_p),
                ("chi", ctypes.c_void_p)]


class _BatchOpts(ctypes.Structure):
    _fields_ = [("workgroups", ctypes.c_int64), ("stage_w_bytes", ctypes.c_uint64), ("use_graph", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 5)]


class _BatchInfo(ctypes.Structure):
    _fields_ = [("items", ctypes.c_int64), ("stages", ctypes.c_int64), ("workgroups", ctypes.c_int64 * 3),
                ("nominal_units", ctypes.c_int64), ("omega_tile", ctypes.c_int64)]


class _TetraList(ctypes.Structure):
    _fields_ = [("n_kp", ctypes.c_int64), ("n_tet", ctypes.c_int64), ("tets", ctypes.c_void_p),
                ("volume", ctypes.c_double)]


class _Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 3), ("launches", ctypes.c_int64 * 3)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libchi0.so and declare its C ABI (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"libchi0 not built: {path} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    lib.chi0_plan.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_Desc), vp, vp, vp]
    lib.chi0_workspace_size.argtypes = [vp, i32, i32, ctypes.POINTER(sz)]
    lib.chi0_static.argtypes = [vp, i32, ctypes.POINTER(_Q), vp, sz, vp]
    lib.chi0_static_pairs.argtypes = [vp, i32, ctypes.POINTER(_Q), vp, sz, vp]
    lib.chi0_kk_workspace_size.argtypes = [vp, i32, i32, i32, ctypes.POINTER(sz)]
    lib.chi0_dynamic_kk.argtypes = [vp, i32, ctypes.POINTER(_Q), i32, vp, i32, ctypes.c_double, ctypes.c_double,
                                    vp, sz, vp]
    lib.chi0_dynamic.argtypes = [vp, i32, ctypes.POINTER(_Q), i32, vp, vp, sz, vp]
    lib.chi0_dynamic_noalloc.argtypes = [vp, i32, ctypes.POINTER(_Q), i32, vp, vp]
    lib.chi0_dynamic_pairs.argtypes = [vp, i32, ctypes.POINTER(_Q), i32, vp, vp, sz, vp]
    lib.chi0_dynamic_pairs_workspace_size.argtypes = [vp, i32, i32, ctypes.POINTER(sz)]
    lib.chi0_matrix_elements.argtypes = [vp, ctypes.POINTER(_Q), vp]
    lib.chi0_profile_enable.argtypes = [vp, i32]
    lib.chi0_profile_read.argtypes = [vp, ctypes.POINTER(_Profile)]
    lib.chi0_census.argtypes = [vp, i32, ctypes.POINTER(_Q), i32, vp, vp, sz, ctypes.POINTER(ctypes.c_uint64)]
    lib.chi0_plan_list.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_Desc), ctypes.POINTER(_TetraList), vp, vp, vp]
    lib.chi0_static_group.argtypes = [vp, i32, i32, ctypes.POINTER(_Q), vp, sz, vp]
    lib.chi0_dynamic_group.argtypes = [vp, i32, i32, ctypes.POINTER(_Q), i32, vp, vp, sz, vp]
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.chi0_iw_cubic.argtypes = [i32, i64p, i64p, ctypes.POINTER(ctypes.c_double), vp, vp, vp]
    lib.chi0_sync.argtypes = [vp]
    lib.chi0_destroy.argtypes = [vp]
    lib.chi0_status_string.argtypes = [i32]
    lib.chi0_status_string.restype = ctypes.c_char_p
    lib.chi0_last_error.argtypes = [vp]
    lib.chi0_last_error.restype = ctypes.c_char_p
    lib.chi0_batch_workspace_size.argtypes = [i32, ctypes.POINTER(_Instance), ctypes.POINTER(_BatchOpts),
                                              ctypes.POINTER(sz)]
    lib.chi0_batch_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(_Instance), ctypes.POINTER(_BatchOpts),
                                      vp, sz, vp]
    lib.chi0_batch_run.argtypes = [vp, vp]
    lib.chi0_batch_tune.argtypes = [vp, vp, i32, ctypes.POINTER(ctypes.c_int64)]
    lib.chi0_batch_info_get.argtypes = [vp, ctypes.POINTER(_BatchInfo)]
    lib.chi0_batch_destroy.argtypes = [vp]
    lib.chi0_batch_last_error.argtypes = [vp]
    lib.chi0_batch_last_error.restype = ctypes.c_char_p
    for name in ("chi0_plan", "chi0_workspace_size", "chi0_static", "chi0_static_pairs", "chi0_dynamic",
                 "chi0_dynamic_noalloc", "chi0_dynamic_pairs", "chi0_dynamic_pairs_workspace_size",
                 "chi0_kk_workspace_size", "chi0_dynamic_kk",
                 "chi0_matrix_elements", "chi0_profile_enable", "chi0_profile_read", "chi0_census",
                 "chi0_sync", "chi0_destroy", "chi0_batch_workspace_size", "chi0_batch_create", "chi0_batch_run",
                 "chi0_batch_tune", "chi0_batch_info_get", "chi0_batch_destroy", "chi0_plan_list",
                 "chi0_static_group", "chi0_dynamic_group", "chi0_iw_cubic"):
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


@dataclass
class Q:
    """One q: an integer mesh shift, explicit device band data at k+q, or (from_frac) the mesh shift
    of the fractional vector q_frac, which must be commensurate with the mesh."""
    shift: Sequence[int] = (0, 0, 0)
    eps_kq: Optional[object] = None    # torch float64 [nb][Nk] on the device
    c_kq: Optional[object] = None      # torch complex128 [Nk][no][nb] on the device
    q_frac: Optional[Sequence[float]] = None
    from_frac: bool = False


def _dev_ptr(t, dtype_name: str, shape=None, what: str = "tensor"):
    """Device pointer of a contiguous device tensor of the given dtype (and exact shape, if given)."""
    if t is None:
        return None
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{what}: libchi0 takes device tensors")
    if str(t.dtype) != dtype_name:
        raise ValueError(f"{what}: expected {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensors must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(int(v) for v in shape):
        raise ValueError(f"{what}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _out_f64(t, shape, what: str):
    """An output tensor as float64 of the exact shape (a complex128 tensor of shape[:-1] when the last
    axis is the (Re, Im) pair is viewed as real)."""
    import torch
    if t is not None and t.dtype == torch.complex128 and shape[-1] == 2:
        if tuple(t.shape) != tuple(shape[:-1]):
            raise ValueError(f"{what}: expected shape {tuple(shape[:-1])}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{what}: tensors must be contiguous")
        t = torch.view_as_real(t)
    _dev_ptr(t, "torch.float64", shape, what)
    return t


def _workspace_ptr(ws):
    """(pointer, bytes) of a workspace tensor: contiguous device memory of any dtype."""
    if not getattr(ws, "is_cuda", False):
        raise ValueError("workspace: libchi0 takes device tensors")
    if not ws.is_contiguous():
        raise ValueError("workspace: tensors must be contiguous")
    return ctypes.c_void_p(ws.data_ptr()), int(ws.numel() * ws.element_size())


def _check_band_arrays(eps_k, c_k, n_kp: int, cma: bool):
    """eps_k float64 [nb][n_kp]; c_k complex128 [n_kp][no][nb] unless cma."""
    if eps_k is None or eps_k.dim() != 2 or int(eps_k.shape[1]) != int(n_kp):
        raise ValueError(f"eps_k must have shape [n_bands, {n_kp}], got "
                         f"{None if eps_k is None else tuple(eps_k.shape)}")
    _dev_ptr(eps_k, "torch.float64", what="eps_k")
    if not cma:
        if c_k is None:
            raise ValueError("c_k is required unless cma")
        if c_k.dim() != 3 or int(c_k.shape[0]) != int(n_kp) or int(c_k.shape[2]) != int(eps_k.shape[0]):
            raise ValueError(f"c_k must have shape [{n_kp}, n_orb, {int(eps_k.shape[0])}], got {tuple(c_k.shape)}")
        _dev_ptr(c_k, "torch.complex128", what="c_k")


def _make_desc(nk, eps_k, c_k, mu, spin_factor, band_lo, band_hi, cma, form, precision, batch_hint=0,
               skip_input_scan=False, degen_tol_ev=0.0, degen_rel_tol=0.0) -> _Desc:
    d = _Desc()
    for i in range(3):
        d.nk[i] = int(nk[i])
    d.n_bands = int(eps_k.shape[0])
    d.n_orb = 1 if c_k is None else int(c_k.shape[1])
    d.band_lo, d.band_hi = int(band_lo), int(band_hi)
    d.cma, d.form, d.precision = int(bool(cma)), int(form), int(precision)
    d.batch_hint, d.skip_input_scan = int(batch_hint), int(bool(skip_input_scan))
    d.mu, d.spin_factor = float(mu), float(spin_factor)
    d.degen_tol_ev, d.degen_rel_tol = float(degen_tol_ev), float(degen_rel_tol)
    return d


def _q_struct(q: "Q", dst: _Q, eps_k=None, c_k=None, cma: bool = False):
    """Fill a chi0_q; explicit k+q arrays must match the shapes of the plan's eps_k / c_k."""
    if q.q_frac is not None:
        for a in range(3):
            dst.q_frac[a] = float(q.q_frac[a])
    if q.eps_kq is not None:
        dst.explicit_kq = 1
        shp_e = None if eps_k is None else tuple(eps_k.shape)
        dst.eps_kq = _dev_ptr(q.eps_kq, "torch.float64", shp_e, "eps_kq")
        if not cma:
            if q.c_kq is None:
                raise ValueError("c_kq is required with eps_kq unless cma")
            shp_c = None if c_k is None else tuple(c_k.shape)
            dst.c_kq = _dev_ptr(q.c_kq, "torch.complex128", shp_c, "c_kq")
    elif q.from_frac:
        if q.q_frac is None:
            raise ValueError("from_frac needs q_frac")
        dst.explicit_kq = 2
    else:
        for a in range(3):
            dst.shift[a] = int(q.shift[a])


class Chi0Plan:
    """A chi0 plan over fixed mesh band data (eps_k [nb][Nk], c_k [Nk][no][nb] on the device).

    With tetrahedra=(tets, volume) the plan integrates over that explicit list instead of the
    mesh's Kuhn tetrahedra (tets: int32 device tensor [n_tet][4] of corner indices into the
    k-points of eps_k [nb][n_kp]; volume: zone fraction of one tetrahedron); nk is then unused
    and every q must carry explicit k+q data.

    Every tensor argument is checked here (device, dtype, contiguity and exact shape) before its
    pointer reaches the library, which cannot check device extents itself."""

    def __init__(self, nk, eps_k, c_k=None, *, mu: float = 0.0, spin_factor: float = 2.0,
                 band_lo: int = 0, band_hi: int = 0, cma: bool = False, form: int = 0,
                 precision: int = 0, stream=None, tetrahedra=None, batch_hint: int = 0,
                 skip_input_scan: bool = False, degen_tol_ev: float = 0.0, degen_rel_tol: float = 0.0):
        import torch
        self._lib = load_library()
        self.eps_k = eps_k
        self.c_k = c_k
        self.cma = bool(cma)
        if tetrahedra is not None:
            nk = (int(eps_k.shape[1]), 1, 1)
        self.nk = tuple(int(v) for v in nk)
        n_kp = self.nk[0] * self.nk[1] * self.nk[2]
        _check_band_arrays(eps_k, c_k, n_kp, self.cma)
        d = _make_desc(self.nk, eps_k, c_k, mu, spin_factor, band_lo, band_hi, cma, form, precision, batch_hint,
                       skip_input_scan, degen_tol_ev, degen_rel_tol)
        self.nbw = (d.n_bands if band_hi <= 0 else band_hi) - band_lo
        self.n_kp = n_kp
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        handle = ctypes.c_void_p()
        ck_ptr = None if self.cma else _dev_ptr(c_k, "torch.complex128", what="c_k")
        if tetrahedra is None:
            st = self._lib.chi0_plan(ctypes.byref(handle), ctypes.byref(d), _dev_ptr(eps_k, "torch.float64"),
                                     ck_ptr, ctypes.c_void_p(self._stream.cuda_stream))
        else:
            tets, volume = tetrahedra
            if tets.dim() != 2 or int(tets.shape[1]) != 4:
                raise ValueError(f"tetrahedra: expected shape [n_tet, 4], got {tuple(tets.shape)}")
            self._tets = tets
            tl = _TetraList(n_kp, int(tets.shape[0]), _dev_ptr(tets, "torch.int32", what="tetrahedra"),
                            float(volume))
            st = self._lib.chi0_plan_list(ctypes.byref(handle), ctypes.byref(d), ctypes.byref(tl),
                                          _dev_ptr(eps_k, "torch.float64"), ck_ptr,
                                          ctypes.c_void_p(self._stream.cuda_stream))
        if st != 0:
            raise Chi0Error(st, "chi0_plan rejected the description")
        self._h = handle

    def close(self):
        if getattr(self, "_h", None):
            self._lib.chi0_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, what: str):
        if st != 0:
            raise Chi0Error(st, f"{what}: {self._lib.chi0_last_error(self._h).decode()}")

    def _qarray(self, qs: Sequence[Q]):
        arr = (_Q * len(qs))()
        for i, q in enumerate(qs):
            _q_struct(q, arr[i], self.eps_k, self.c_k, self.cma)
        return arr

    def _ws(self, workspace, nq: int, nw: int):
        ws = workspace if workspace is not None else self.workspace(nq, nw)
        return ws, _workspace_ptr(ws)

    def _omega(self, omega):
        if omega is None or omega.dim() != 1:
            raise ValueError("omega must be a 1-D float64 device tensor")
        return int(omega.shape[0]), _dev_ptr(omega, "torch.float64", what="omega")

    def _new(self, shape):
        import torch
        return torch.empty(shape, dtype=torch.float64, device=self.eps_k.device)

    def workspace_bytes(self, nq: int, nw: int) -> int:
        n = ctypes.c_size_t()
        self._check(self._lib.chi0_workspace_size(self._h, nq, nw, ctypes.byref(n)), "chi0_workspace_size")
        return int(n.value)

    def workspace(self, nq: int, nw: int):
        import torch
        return torch.empty(self.workspace_bytes(nq, nw), dtype=torch.uint8, device=self.eps_k.device)

    def sync(self):
        """Wait for the plan's stream; raises Chi0Error if an input scan found non-finite values or
        unnormalised eigenvectors in a call since the last report."""
        self._check(self._lib.chi0_sync(self._h), "chi0_sync")

    def static(self, qs: Sequence[Q], workspace=None, out=None):
        """Re chi0(q, 0) for each q: float64 tensor [nq]."""
        nq = len(qs)
        arr = self._qarray(qs)
        ws, (wp, wn) = self._ws(workspace, nq, 1)
        chi = _out_f64(out if out is not None else self._new((nq,)), (nq,), "out")
        self._check(self._lib.chi0_static(self._h, nq, arr, wp, wn, ctypes.c_void_p(chi.data_ptr())), "chi0_static")
        return chi

    def static_pairs(self, qs: Sequence[Q], workspace=None, out=None):
        """Re chi0(q, 0) resolved by band pair: float64 tensor [nq, nbw, nbw] (n at k, m at k+q)."""
        nq = len(qs)
        arr = self._qarray(qs)
        ws, (wp, wn) = self._ws(workspace, nq, 1)
        shape = (nq, self.nbw, self.nbw)
        chi = _out_f64(out if out is not None else self._new(shape), shape, "out")
        self._check(self._lib.chi0_static_pairs(self._h, nq, arr, wp, wn, ctypes.c_void_p(chi.data_ptr())),
                    "chi0_static_pairs")
        return chi

    def dynamic(self, qs: Sequence[Q], omega, workspace=None, out=None):
        """chi0(q, w): complex128 tensor [nq, nw] (omega: float64 device tensor [nw]; out: float64
        [nq, nw, 2] or complex128 [nq, nw])."""
        import torch
        nq = len(qs)
        nw, op = self._omega(omega)
        arr = self._qarray(qs)
        ws, (wp, wn) = self._ws(workspace, nq, nw)
        chi = _out_f64(out if out is not None else self._new((nq, nw, 2)), (nq, nw, 2), "out")
        self._check(self._lib.chi0_dynamic(self._h, nq, arr, nw, op, wp, wn, ctypes.c_void_p(chi.data_ptr())),
                    "chi0_dynamic")
        return torch.view_as_complex(chi)

    def dynamic_pairs_workspace_bytes(self, nq: int, nw: int) -> int:
        n = ctypes.c_size_t()
        self._check(self._lib.chi0_dynamic_pairs_workspace_size(self._h, nq, nw, ctypes.byref(n)),
                    "chi0_dynamic_pairs_workspace_size")
        return int(n.value)

    def dynamic_pairs(self, qs: Sequence[Q], omega, workspace=None, out=None):
        """chi0(q, w) resolved by band pair: complex128 tensor [nq, nbw, nbw, nw] (n at k, m at k+q;
        out: float64 [nq, nbw, nbw, nw, 2] or complex128 [nq, nbw, nbw, nw]).  Mesh plans only."""
        import torch
        nq = len(qs)
        nw, op = self._omega(omega)
        arr = self._qarray(qs)
        if workspace is None:
            workspace = torch.empty(self.dynamic_pairs_workspace_bytes(nq, nw), dtype=torch.uint8,
                                    device=self.eps_k.device)
        wp, wn = _workspace_ptr(workspace)
        shape = (nq, self.nbw, self.nbw, nw, 2)
        chi = _out_f64(out if out is not None else self._new(shape), shape, "out")
        self._check(self._lib.chi0_dynamic_pairs(self._h, nq, arr, nw, op, wp, wn, ctypes.c_void_p(chi.data_ptr())),
                    "chi0_dynamic_pairs")
        return torch.view_as_complex(chi)

    def dynamic_noalloc(self, qs: Sequence[Q], omega, out):
        """chi0_dynamic_noalloc: as dynamic() with the library's fixed device scratch as workspace; the
        output tensor must be supplied (float64 [nq, nw, 2] or complex128 [nq, nw]), so nothing is
        allocated on this path."""
        import torch
        nq = len(qs)
        nw, op = self._omega(omega)
        arr = self._qarray(qs)
        chi = _out_f64(out, (nq, nw, 2), "out")
        self._check(self._lib.chi0_dynamic_noalloc(self._h, nq, arr, nw, op, ctypes.c_void_p(chi.data_ptr())),
                    "chi0_dynamic_noalloc")
        return torch.view_as_complex(chi)

    def static_group(self, qs: Sequence[Q], n_group: int, workspace=None, out=None):
        """Point-group loop, static: qs holds groups of n_group entries; float64 tensor
        [len(qs) // n_group] of the per-group sums of Re chi0(q, 0)."""
        if n_group < 1 or len(qs) % n_group:
            raise ValueError("len(qs) must be a multiple of n_group")
        nq = len(qs) // n_group
        arr = self._qarray(qs)
        ws, (wp, wn) = self._ws(workspace, len(qs), 1)
        chi = _out_f64(out if out is not None else self._new((nq,)), (nq,), "out")
        self._check(self._lib.chi0_static_group(self._h, nq, int(n_group), arr, wp, wn,
                                                ctypes.c_void_p(chi.data_ptr())), "chi0_static_group")
        return chi

    def dynamic_group(self, qs: Sequence[Q], n_group: int, omega, workspace=None, out=None):
        """Point-group loop, dynamic: per-group sums of chi0(q, w), complex128 tensor [nq, nw]."""
        import torch
        if n_group < 1 or len(qs) % n_group:
            raise ValueError("len(qs) must be a multiple of n_group")
        nq = len(qs) // n_group
        nw, op = self._omega(omega)
        arr = self._qarray(qs)
        ws, (wp, wn) = self._ws(workspace, len(qs), nw)
        chi = _out_f64(out if out is not None else self._new((nq, nw, 2)), (nq, nw, 2), "out")
        self._check(self._lib.chi0_dynamic_group(self._h, nq, int(n_group), arr, nw, op, wp, wn,
                                                 ctypes.c_void_p(chi.data_ptr())), "chi0_dynamic_group")
        return torch.view_as_complex(chi)

    def dynamic_kk(self, qs: Sequence[Q], omega, n_spec: int, spec_lo: float, spec_hi: float, workspace=None,
                   out=None):
        """chi0(q, w) by the Kramers-Kronig route: Im exact, Re from Im on the uniform spectral grid
        of n_spec points over [spec_lo, spec_hi]; complex128 tensor [nq, nw]."""
        import torch
        nq = len(qs)
        nw, op = self._omega(omega)
        arr = self._qarray(qs)
        if workspace is None:
            n = ctypes.c_size_t()
            self._check(self._lib.chi0_kk_workspace_size(self._h, nq, nw, int(n_spec), ctypes.byref(n)),
                        "chi0_kk_workspace_size")
            workspace = torch.empty(int(n.value), dtype=torch.uint8, device=self.eps_k.device)
        wp, wn = _workspace_ptr(workspace)
        chi = _out_f64(out if out is not None else self._new((nq, nw, 2)), (nq, nw, 2), "out")
        self._check(self._lib.chi0_dynamic_kk(self._h, nq, arr, nw, op, int(n_spec), float(spec_lo), float(spec_hi),
                                              wp, wn, ctypes.c_void_p(chi.data_ptr())), "chi0_dynamic_kk")
        return torch.view_as_complex(chi)

    def matrix_elements(self, q: Q, out=None):
        """W_nm(k) of one q: float64 tensor [nbw, nbw, Nk]."""
        shape = (self.nbw, self.nbw, self.n_kp)
        W = _out_f64(out if out is not None else self._new(shape), shape, "out")
        arr = self._qarray([q])
        self._check(self._lib.chi0_matrix_elements(self._h, arr, ctypes.c_void_p(W.data_ptr())),
                    "chi0_matrix_elements")
        return W

    def profile(self, enable: bool = True):
        """Record HIP events around every launch of this plan (see read_profile)."""
        self._check(self._lib.chi0_profile_enable(self._h, int(bool(enable))), "chi0_profile_enable")

    def read_profile(self) -> dict:
        """Kernel times (ms) and launch counts since the last read: keys contract/tetra/reduce."""
        prof = _Profile()
        self._check(self._lib.chi0_profile_read(self._h, ctypes.byref(prof)), "chi0_profile_read")
        names = ("contract", "tetra", "reduce")
        return {n: {"ms": prof.ms[i], "launches": int(prof.launches[i])} for i, n in enumerate(names)}

    def census(self, qs: Sequence[Q], omega, workspace=None) -> dict:
        """Work census of dynamic(qs, omega) (diagnostic; synchronises)."""
        nq = len(qs)
        nw, op = self._omega(omega)
        arr = self._qarray(qs)
        ws, (wp, wn) = self._ws(workspace, nq, nw)
        counts = (ctypes.c_uint64 * len(CENSUS_KEYS))()
        self._check(self._lib.chi0_census(self._h, nq, arr, nw, op, wp, wn, counts), "chi0_census")
        return {k: int(counts[i]) for i, k in enumerate(CENSUS_KEYS)}


def iw_cubic(n: int):
    """The irreducible wedge of a Gamma-centred n^3 simple-cubic mesh under O_h in tetrahedra
    (host arrays from chi0_iw_cubic): (kfrac float64 [n_kp][3], tets int32 [n_tet][4],
    volume of one tetrahedron, ops int32 [48][3][3])."""
    import numpy as np
    lib = load_library()
    n_kp, n_tet, vol = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
    st = lib.chi0_iw_cubic(int(n), ctypes.byref(n_kp), ctypes.byref(n_tet), ctypes.byref(vol), None, None, None)
    if st != 0:
        raise Chi0Error(st, f"chi0_iw_cubic({n})")
    kfrac = np.zeros((n_kp.value, 3))
    tets = np.zeros((n_tet.value, 4), dtype=np.int32)
    ops = np.zeros((48, 3, 3), dtype=np.int32)
    st = lib.chi0_iw_cubic(int(n), ctypes.byref(n_kp), ctypes.byref(n_tet), ctypes.byref(vol),
                           kfrac.ctypes.data_as(ctypes.c_void_p), tets.ctypes.data_as(ctypes.c_void_p),
                           ops.ctypes.data_as(ctypes.c_void_p))
    if st != 0:
        raise Chi0Error(st, f"chi0_iw_cubic({n})")
    return kfrac, tets, vol.value, ops


@dataclass
class Instance:
    """One problem of a batch: mesh band data, its q-list and frequency grid (device tensors).

    chi (complex128 [nq, nw], allocated by Chi0Batch when None) receives chi0(q, w)."""
    nk: Sequence[int]
    eps_k: object
    c_k: Optional[object]
    qs: Sequence[Q]
    omega: object
    mu: float = 0.0
    spin_factor: float = 2.0
    band_lo: int = 0
    band_hi: int = 0
    cma: bool = False
    form: int = 0
    precision: int = 0
    chi: Optional[object] = None


class Chi0Batch:
    """Many instances run as one fused launch sequence (optionally a replayed HIP graph)."""

    def __init__(self, instances: Sequence[Instance], *, workgroups: int = 0, stage_w_bytes: int = 0,
                 use_graph: bool = True, stream=None):
        import torch
        self._lib = load_library()
        self.instances = list(instances)
        n = len(self.instances)
        self._inst = (_Instance * n)()
        self._qarrs = []
        dev = self.instances[0].eps_k.device
        for i, ins in enumerate(self.instances):
            if ins.omega is None or ins.omega.dim() != 1:
                raise ValueError(f"instance {i}: omega must be a 1-D float64 device tensor")
            nw = int(ins.omega.shape[0])
            _check_band_arrays(ins.eps_k, ins.c_k, int(ins.nk[0]) * int(ins.nk[1]) * int(ins.nk[2]), bool(ins.cma))
            shape = (len(ins.qs), nw, 2)
            ins.chi = _out_f64(ins.chi if ins.chi is not None else
                               torch.empty(shape, dtype=torch.float64, device=dev), shape, f"instance {i}: chi")
            qa = (_Q * len(ins.qs))()
            for j, q in enumerate(ins.qs):
                _q_struct(q, qa[j], ins.eps_k, ins.c_k, bool(ins.cma))
            self._qarrs.append(qa)
            s = self._inst[i]
            s.desc = _make_desc(ins.nk, ins.eps_k, ins.c_k, ins.mu, ins.spin_factor, ins.band_lo, ins.band_hi,
                                ins.cma, ins.form, ins.precision)
            s.eps_k = _dev_ptr(ins.eps_k, "torch.float64")
            s.c_k = None if ins.cma else _dev_ptr(ins.c_k, "torch.complex128")
            s.nq, s.nw = len(ins.qs), nw
            s.qs = ctypes.cast(qa, ctypes.POINTER(_Q))
            s.omega = _dev_ptr(ins.omega, "torch.float64", what=f"instance {i}: omega")
            s.chi = _dev_ptr(ins.chi, "torch.float64")
        self._opts = _BatchOpts()
        self._opts.workgroups = int(workgroups)
        self._opts.stage_w_bytes = int(stage_w_bytes)
        self._opts.use_graph = int(bool(use_graph))
        nbytes = ctypes.c_size_t()
        st = self._lib.chi0_batch_workspace_size(n, self._inst, ctypes.byref(self._opts), ctypes.byref(nbytes))
        if st != 0:
            raise Chi0Error(st, "chi0_batch_workspace_size rejected the instances")
        self.workspace = torch.empty(max(1, int(nbytes.value)), dtype=torch.uint8, device=dev)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        handle = ctypes.c_void_p()
        st = self._lib.chi0_batch_create(ctypes.byref(handle), n, self._inst, ctypes.byref(self._opts),
                                         ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                         ctypes.c_void_p(self._stream.cuda_stream))
        if st != 0:
            raise Chi0Error(st, "chi0_batch_create failed")
        self._h = handle

    def close(self):
        if getattr(self, "_h", None):
            self._lib.chi0_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, what: str):
        if st != 0:
            raise Chi0Error(st, f"{what}: {self._lib.chi0_batch_last_error(self._h).decode()}")

    def run(self, stream=None):
        """Enqueue the whole batch; returns the instances' chi as complex128 views."""
        import torch
        s = stream if stream is not None else self._stream
        self._check(self._lib.chi0_batch_run(self._h, ctypes.c_void_p(s.cuda_stream)), "chi0_batch_run")
        return [torch.view_as_complex(ins.chi) for ins in self.instances]

    def tune(self, reps: int = 2, stream=None) -> int:
        s = stream if stream is not None else self._stream
        chosen = ctypes.c_int64()
        self._check(self._lib.chi0_batch_tune(self._h, ctypes.c_void_p(s.cuda_stream), int(reps),
                                              ctypes.byref(chosen)), "chi0_batch_tune")
        return int(chosen.value)

    def info(self) -> dict:
        inf = _BatchInfo()
        self._check(self._lib.chi0_batch_info_get(self._h, ctypes.byref(inf)), "chi0_batch_info_get")
        return {"items": int(inf.items), "stages": int(inf.stages),
                "workgroups": {"contract": int(inf.workgroups[0]), "tetra": int(inf.workgroups[1]),
                               "reduce": int(inf.workgroups[2])},
                "nominal_units": int(inf.nominal_units), "omega_tile": int(inf.omega_tile)}
