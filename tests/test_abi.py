"""The C ABI without a GPU: the library loads, exports every entry point the header
declares, and rejects bad descriptors and arguments on the host with the documented
status codes (no device call is made on these paths)."""
import ctypes
import os
import re

import pytest

import paper_1407_3444_amd as lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chi0.h")


def _header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(chi0_\w+)\s*\(", text, re.M)))


def test_header_declares_the_binding_symbols():
    assert sorted(lib.EXPORTED_SYMBOLS) == _header_functions()


def test_library_exports_every_declared_symbol():
    so = lib.load_library()
    for name in _header_functions():
        assert hasattr(so, name), name


def _desc(**kw):
    d = lib._Desc()
    d.nk[0], d.nk[1], d.nk[2] = kw.get("nk", (4, 4, 4))
    d.n_bands = kw.get("n_bands", 4)
    d.n_orb = kw.get("n_orb", 4)
    d.band_lo = kw.get("band_lo", 0)
    d.band_hi = kw.get("band_hi", 0)
    d.cma = kw.get("cma", 0)
    d.form = kw.get("form", 0)
    d.precision = kw.get("precision", 0)
    d.mu = kw.get("mu", 0.0)
    d.spin_factor = kw.get("spin_factor", 2.0)
    return d


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced by chi0_plan


def _plan(d, eps=FAKE, ck=FAKE):
    so = lib.load_library()
    h = ctypes.c_void_p()
    st = so.chi0_plan(ctypes.byref(h), ctypes.byref(d), eps, ck, None)
    return st, h


@pytest.mark.parametrize("kw,status", [
    (dict(nk=(0, 4, 4)), -2),
    (dict(n_bands=0), -2),
    (dict(n_bands=65), -2),
    (dict(band_lo=3, band_hi=2), -2),
    (dict(band_lo=-1), -2),
    (dict(band_hi=5), -2),
    (dict(n_bands=40, band_lo=0, band_hi=40), -2),
    (dict(n_orb=0), -2),
    (dict(form=2), -1),
    (dict(cma=3), -1),
    (dict(mu=float("nan")), -3),
    (dict(spin_factor=float("inf")), -3),
    (dict(precision=3), -1),
    (dict(precision=-1), -1),
])
def test_plan_rejects_bad_descriptors(kw, status):
    st, h = _plan(_desc(**kw))
    assert st == status
    assert not h.value


def test_plan_rejects_null_pointers():
    assert _plan(_desc(), eps=None)[0] == -1
    assert _plan(_desc(), ck=None)[0] == -1
    assert _plan(_desc(cma=1), ck=None)[0] == 0


def test_calls_validate_before_any_device_work():
    so = lib.load_library()
    st, h = _plan(_desc(nk=(3, 5, 2), n_bands=6, n_orb=6, band_lo=1, band_hi=5))
    assert st == 0
    try:
        size = ctypes.c_size_t()
        assert so.chi0_workspace_size(h, 3, 700, ctypes.byref(size)) == 0 and size.value > 0
        assert so.chi0_workspace_size(h, 0, 1, ctypes.byref(size)) == -1
        q = (lib._Q * 2)()
        q[1].explicit_kq = 1                       # explicit without arrays
        out = ctypes.c_void_p(0x2000)
        ws = ctypes.c_void_p(0x3000)
        assert so.chi0_static(h, 2, q, ws, 1 << 40, out) == -1
        assert b"eps_kq" in so.chi0_last_error(h)
        q[1].explicit_kq = 0
        assert so.chi0_static(h, 0, q, ws, 1 << 40, out) == -1
        assert so.chi0_static(h, 2, q, ws, 16, out) == -5          # workspace too small
        assert so.chi0_static(h, 2, q, None, 1 << 40, out) == -5
        assert so.chi0_dynamic(h, 2, q, 0, out, ws, 1 << 40, out) == -1
        assert so.chi0_dynamic(h, 2, q, 4, None, ws, 1 << 40, out) == -1
        assert so.chi0_dynamic(h, 2, q, 4, out, ws, 8, out) == -5
        assert so.chi0_status_string(-5) == b"workspace too small"
    finally:
        so.chi0_destroy(h)
    assert so.chi0_destroy(None) == 0


def test_workspace_grows_with_frequencies_up_to_one_launch():
    so = lib.load_library()
    st, h = _plan(_desc(nk=(8, 8, 8), n_bands=4, n_orb=4))
    try:
        sizes = []
        for nw in (1, 64, 512, 2048):
            s = ctypes.c_size_t()
            so.chi0_workspace_size(h, 1, nw, ctypes.byref(s))
            sizes.append(s.value)
        assert sizes[0] < sizes[1] < sizes[2] == sizes[3]
    finally:
        so.chi0_destroy(h)


def _instance(nq=3, nw=100, **kw):
    ins = lib._Instance()
    ins.desc = _desc(**kw)
    ins.eps_k = FAKE
    ins.c_k = None if kw.get("cma") else FAKE
    qa = (lib._Q * max(nq, 1))()
    for j in range(max(nq, 1)):
        qa[j].shift[0] = j + 1
    ins.nq, ins.nw = nq, nw
    ins.qs = ctypes.cast(qa, ctypes.POINTER(lib._Q))
    ins.omega = ctypes.c_void_p(0x4000)
    ins.chi = ctypes.c_void_p(0x5000)
    return ins, qa


def _batch_size(insts, **opt):
    so = lib.load_library()
    arr = (lib._Instance * len(insts))(*insts)
    o = lib._BatchOpts()
    o.workgroups = opt.get("workgroups", 0)
    o.stage_w_bytes = opt.get("stage_w_bytes", 0)
    o.use_graph = opt.get("use_graph", 0)
    if "reserved" in opt:
        o.reserved[0] = opt["reserved"]
    n = ctypes.c_size_t()
    st = so.chi0_batch_workspace_size(len(insts), arr, ctypes.byref(o), ctypes.byref(n))
    return st, n.value


def test_batch_validates_instances_on_the_host():
    a, qa = _instance(nk=(8, 8, 8))
    b, qb = _instance(nq=2, nw=700, nk=(6, 6, 6), n_bands=6, n_orb=5, band_lo=1, band_hi=5)
    st, n = _batch_size([a, b])
    assert st == 0 and n > 0
    bad, qbad = _instance(nk=(8, 0, 8))
    assert _batch_size([a, bad])[0] == -2
    assert _batch_size([_instance(nq=0)[0]])[0] == -1
    assert _batch_size([_instance(nw=0)[0]])[0] == -1
    assert _batch_size([a], reserved=1)[0] == -1
    assert _batch_size([a], use_graph=2)[0] == -1
    c, qc = _instance()
    c.qs = None
    assert _batch_size([c])[0] == -1
    d, qd = _instance()
    qd[1].explicit_kq = 1                     # explicit q without its arrays
    assert _batch_size([d])[0] == -1
    so = lib.load_library()
    assert so.chi0_batch_workspace_size(0, None, None, ctypes.byref(ctypes.c_size_t())) == -1
    assert so.chi0_batch_destroy(None) == 0


def test_batch_workspace_follows_workgroups_and_stage_budget():
    insts = [_instance(nq=4, nw=300, nk=(12, 12, 12), n_bands=8, n_orb=8)[0] for _ in range(3)]
    w_bytes = 8 * 8 * 8 * 12 ** 3                       # W of one q
    sizes = [_batch_size(insts, workgroups=g)[1] for g in (256, 1024, 4096)]
    assert sizes[0] <= sizes[1] <= sizes[2]
    one_stage = _batch_size(insts)[1]
    staged = _batch_size(insts, stage_w_bytes=2 * w_bytes)[1]
    # one stage holds W of all 12 (instance, q) groups; budgeted stages hold two at a time
    assert one_stage - staged >= 9 * w_bytes


def test_batch_create_checks_the_workspace_before_device_work():
    so = lib.load_library()
    a, qa = _instance(nk=(8, 8, 8))
    arr = (lib._Instance * 1)(a)
    h = ctypes.c_void_p()
    st, need = _batch_size([a])
    assert st == 0
    assert so.chi0_batch_create(ctypes.byref(h), 1, arr, None, None, need, None) == -5
    assert so.chi0_batch_create(ctypes.byref(h), 1, arr, None, ctypes.c_void_p(0x6000), need - 256, None) == -5
    assert not h.value


def test_plane_wave_basis_sizes():
    assert _plan(_desc(n_orb=4096, n_bands=8))[0] == 0
    assert _plan(_desc(n_orb=16384, n_bands=8))[0] == 0
    assert _plan(_desc(n_orb=16385, n_bands=8))[0] == -2


def test_iw_cubic_host_builder():
    """The wedge builder is host code: sizes, the O_h matrices, and the same wedge as the oracle's
    own construction (compared as sets of corner coordinates)."""
    import numpy as np
    import oracle
    so = lib.load_library()
    n_kp, n_tet, vol = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
    for bad in (0, 3, 7, 1026):
        assert so.chi0_iw_cubic(bad, ctypes.byref(n_kp), ctypes.byref(n_tet), ctypes.byref(vol), None, None,
                                None) == -2
    assert so.chi0_iw_cubic(8, None, ctypes.byref(n_tet), ctypes.byref(vol), None, None, None) == -1
    for n in (2, 6, 12):
        kf, tets, v, ops = lib.iw_cubic(n)
        m = n // 2
        assert kf.shape == ((m + 1) * (m + 2) * (m + 3) // 6, 3) and tets.shape == (m ** 3, 4)
        assert v == 1.0 / (6 * n ** 3)
        assert np.array_equal(ops[0], np.eye(3, dtype=np.int32))
        assert len({g.tobytes() for g in ops}) == 48
        for g in ops:
            assert np.array_equal(g @ g.T, np.eye(3, dtype=np.int32))
        kf2, tets2, v2 = oracle.iw_cubic(n)
        key = lambda k, t: sorted(tuple(sorted(map(tuple, np.round(k[c] * n).astype(int)))) for c in t)
        assert key(kf, tets) == key(kf2, tets2)


def test_list_plan_validates_on_the_host():
    so = lib.load_library()
    d = _desc(cma=1)
    h = ctypes.c_void_p()

    def make(n_kp=5, n_tet=1, tets=4096, volume=0.1):
        tl = lib._TetraList(n_kp, n_tet, tets, volume)
        return so.chi0_plan_list(ctypes.byref(h), ctypes.byref(d), ctypes.byref(tl), FAKE, None, None)

    assert make(n_kp=0) == -2
    assert make(n_tet=0) == -2
    assert make(n_kp=1 << 31) == -2
    assert make(tets=None) == -1
    assert make(tets=4100) == -1          # not 16-byte aligned
    assert make(volume=0.0) == -1
    assert make(volume=float("nan")) == -1
    assert so.chi0_plan_list(ctypes.byref(h), ctypes.byref(d), None, FAKE, None, None) == -1


@pytest.mark.parametrize("field,value,status", [
    ("batch_hint", 17, -1), ("batch_hint", -1, -1), ("skip_input_scan", 2, -1),
    ("degen_tol_ev", float("nan"), -3), ("degen_rel_tol", float("inf"), -3),
    ("degen_tol_ev", -1e-6, -1), ("degen_rel_tol", -0.1, -1),
])
def test_plan_rejects_bad_new_descriptor_fields(field, value, status):
    d = _desc()
    setattr(d, field, value)
    st, h = _plan(d)
    assert st == status and not h.value


def test_plan_rejects_nonzero_reserved():
    d = _desc()
    d.reserved[2] = 1
    assert _plan(d)[0] == -1


def test_q_from_fraction_is_checked_on_the_host():
    so = lib.load_library()
    st, h = _plan(_desc(nk=(4, 4, 8)))
    assert st == 0
    try:
        q = (lib._Q * 1)()
        q[0].explicit_kq = 2
        ws, out = ctypes.c_void_p(0x3000), ctypes.c_void_p(0x2000)
        q[0].q_frac[0], q[0].q_frac[1], q[0].q_frac[2] = 0.3, 0.0, 0.0     # 0.3 * 4 is not an integer
        assert so.chi0_static(h, 1, q, ws, 1 << 40, out) == -4
        assert b"not a vector of the mesh" in so.chi0_last_error(h)
        q[0].q_frac[0] = float("nan")
        assert so.chi0_static(h, 1, q, ws, 1 << 40, out) == -3
        # commensurate (and periodic images) pass the q check and stop at the workspace check
        for frac in ((0.25, -0.5, 0.125), (1.75, 3.0, -0.875)):
            q[0].q_frac[0], q[0].q_frac[1], q[0].q_frac[2] = frac
            assert so.chi0_static(h, 1, q, ws, 16, out) == -5
        q[0].explicit_kq = 3
        assert so.chi0_static(h, 1, q, ws, 1 << 40, out) == -1
        assert so.chi0_status_string(-4) == b"q not commensurate with the mesh"
        assert so.chi0_status_string(-8) == b"eigenvectors not normalised"
    finally:
        so.chi0_destroy(h)
    assert so.chi0_sync(None) == -1


def test_batch_hint_bounds_the_workspace():
    so = lib.load_library()
    sizes = []
    for hint in (0, 16, 4, 1):
        d = _desc(nk=(16, 16, 16), n_bands=8, n_orb=8)
        d.batch_hint = hint
        st, h = _plan(d)
        assert st == 0
        s = ctypes.c_size_t()
        assert so.chi0_workspace_size(h, 64, 512, ctypes.byref(s)) == 0
        sizes.append(s.value)
        so.chi0_destroy(h)
    w_per_q = 8 * 8 * 8 * 16 ** 3
    assert sizes[0] == sizes[1] > sizes[2] > sizes[3]
    assert sizes[1] - sizes[2] >= 12 * w_per_q and sizes[2] - sizes[3] >= 3 * w_per_q


def test_batch_rejects_plane_wave_bases():
    a, qa = _instance(nk=(4, 4, 4), n_bands=8, n_orb=128)
    assert _batch_size([a])[0] == -7
    b, qb = _instance(nk=(4, 4, 4), n_bands=8, n_orb=64)
    assert _batch_size([b])[0] == 0


class _FakeDev:
    """Stands in for a device tensor in the binding's host-side checks (never dereferenced)."""

    def __init__(self, shape, dtype):
        import torch
        self.shape = tuple(shape)
        self.dtype = getattr(torch, dtype)
        self.is_cuda = True

    def dim(self):
        return len(self.shape)

    def is_contiguous(self):
        return True

    def data_ptr(self):
        return 0x1000


def test_binding_checks_shapes_before_passing_pointers():
    eps = _FakeDev((10, 64), "float64")
    ck = _FakeDev((64, 10, 10), "complex128")
    lib._check_band_arrays(eps, ck, 64, False)
    with pytest.raises(ValueError, match="eps_k"):
        lib._check_band_arrays(_FakeDev((10, 63), "float64"), ck, 64, False)
    with pytest.raises(ValueError, match="c_k"):
        lib._check_band_arrays(eps, _FakeDev((64, 10, 9), "complex128"), 64, False)
    with pytest.raises(ValueError, match="expected torch.complex128"):
        lib._check_band_arrays(eps, _FakeDev((64, 10, 10), "float64"), 64, False)
    lib._check_band_arrays(eps, None, 64, True)
    q = lib._Q()
    lib._q_struct(lib.Q(eps_kq=_FakeDev((10, 64), "float64"), c_kq=_FakeDev((64, 10, 10), "complex128")), q,
                  eps, ck, False)
    assert q.explicit_kq == 1
    with pytest.raises(ValueError, match="eps_kq"):
        lib._q_struct(lib.Q(eps_kq=_FakeDev((10, 32), "float64"), c_kq=ck), lib._Q(), eps, ck, False)
    with pytest.raises(ValueError, match="c_kq"):
        lib._q_struct(lib.Q(eps_kq=eps, c_kq=_FakeDev((32, 10, 10), "complex128")), lib._Q(), eps, ck, False)
    with pytest.raises(ValueError, match="c_kq is required"):
        lib._q_struct(lib.Q(eps_kq=eps), lib._Q(), eps, ck, False)
    qf = lib._Q()
    lib._q_struct(lib.Q(q_frac=(0.25, 0.0, 0.5), from_frac=True), qf)
    assert qf.explicit_kq == 2 and qf.q_frac[2] == 0.5
    lib._out_f64(_FakeDev((3, 8, 2), "float64"), (3, 8, 2), "out")
    with pytest.raises(ValueError, match="out"):
        lib._out_f64(_FakeDev((3, 7, 2), "float64"), (3, 8, 2), "out")
    with pytest.raises(ValueError, match="out"):
        lib._out_f64(_FakeDev((3,), "float32"), (3,), "out")
