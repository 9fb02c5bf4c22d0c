"""GPU tests of the boundary's content checks and descriptor options: the asynchronous input scan
(non-finite band energies, eigenvector coefficients and frequencies; eigenvectors that are not
normalised, Sec. II takes normalised eigenvectors as input), q given by its fractional coordinates,
the q-points per launch sequence, and the degeneracy tolerances of the mixed form."""
import numpy as np
import pytest

import oracle
import synth
from metrics import max_err

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print(*a, flush=True)


def _setup(nk=(6, 6, 2), q_subset=(3,), nw=24, **kw):
    torch = _torch()
    import paper_1407_3444_amd as lib
    wl = synth.make_workload("tetra_dynamic", nk=nk, nq=8, q_subset=list(q_subset), nw=nw)
    dev = torch.device("cuda:0")
    eps = torch.from_numpy(wl.eps_k).to(dev)
    ck = torch.from_numpy(wl.c_k).to(dev)
    plan = lib.Chi0Plan(wl.nk, eps, ck, mu=wl.mu, **kw)
    qs = [lib.Q(eps_kq=torch.from_numpy(q.eps_kq).to(dev), c_kq=torch.from_numpy(q.c_kq).to(dev)) for q in wl.qs]
    om = torch.from_numpy(wl.omega).to(dev)
    return lib, torch, wl, plan, qs, om, eps, ck


def test_scan_reports_nonfinite_band_energy_at_sync_and_at_the_next_call():
    lib, torch, wl, plan, qs, om, eps, ck = _setup()
    _say("scan: NaN in the k+q energies")
    plan.dynamic(qs, om)
    plan.sync()                                    # clean inputs: nothing to report
    bad = qs[0].eps_kq.clone()
    bad[4, 11] = float("nan")
    qbad = lib.Q(eps_kq=bad, c_kq=qs[0].c_kq)
    plan.dynamic([qbad], om)
    with pytest.raises(lib.Chi0Error) as e:
        plan.sync()
    assert e.value.status == -3 and "band energies" in str(e.value)
    plan.sync()                                    # reported once
    # the verdict also reaches the next call once the scan has completed
    plan.static([qbad])
    torch.cuda.synchronize()
    with pytest.raises(lib.Chi0Error) as e:
        plan.static(qs)
    assert e.value.status == -3
    got = plan.static(qs).cpu().numpy()           # nothing pending: computes again
    plan.sync()
    ref = oracle.chi0(wl, 0, omega=[0.0])[0].real
    assert abs(got[0] - ref) <= 1e-10 * abs(ref)


def test_scan_reports_unnormalised_and_nonfinite_eigenvectors():
    lib, torch, wl, plan, qs, om, eps, ck = _setup()
    _say("scan: eigenvector norms")
    c = qs[0].c_kq.clone()
    c[5, :, 2] *= 1.001                            # squared norm 1.002
    plan.static([lib.Q(eps_kq=qs[0].eps_kq, c_kq=c)])
    with pytest.raises(lib.Chi0Error) as e:
        plan.sync()
    assert e.value.status == -8
    c = qs[0].c_kq.clone()
    c[0, 3, 1] = complex(float("inf"), 0.0)
    plan.static([lib.Q(eps_kq=qs[0].eps_kq, c_kq=c)])
    with pytest.raises(lib.Chi0Error) as e:
        plan.sync()
    assert e.value.status == -3 and "eigenvector" in str(e.value)


def test_scan_of_plane_wave_eigenvectors():
    """Large bases take the workgroup-per-k scan: 300 plane waves and 6 bands (a band count that
    does not divide the workgroup, so some threads idle); clean inputs pass, one coefficient of one
    column scaled (squared norm off by about 1e-3) and one non-finite coefficient are reported."""
    torch = _torch()
    import paper_1407_3444_amd as lib
    wl = synth.plane_wave_workload((4, 4, 3), 300, 6, nq=2, nw=4)
    dev = torch.device("cuda:0")
    eps = torch.from_numpy(wl.eps_k).to(dev)
    plan = lib.Chi0Plan(wl.nk, eps, torch.from_numpy(wl.c_k).to(dev), mu=wl.mu)
    qs = [lib.Q(shift=q.shift) for q in wl.qs]
    _say("scan: plane-wave eigenvectors")
    plan.static(qs)
    plan.sync()
    c = wl.c_k.copy()
    c[17, :, 4] *= np.sqrt(1.001)
    bad = lib.Chi0Plan(wl.nk, eps, torch.from_numpy(c).to(dev), mu=wl.mu)
    bad.static(qs)
    with pytest.raises(lib.Chi0Error) as e:
        bad.sync()
    assert e.value.status == -8
    c = wl.c_k.copy()
    c[46, 299, 5] = complex(float("nan"), 0.0)
    bad = lib.Chi0Plan(wl.nk, eps, torch.from_numpy(c).to(dev), mu=wl.mu)
    bad.static(qs)
    with pytest.raises(lib.Chi0Error) as e:
        bad.sync()
    assert e.value.status == -3 and "eigenvector" in str(e.value)


def test_scan_can_be_skipped():
    lib, torch, wl, plan, qs, om, eps, ck = _setup(skip_input_scan=True)
    bad = om.clone()
    bad[3] = float("nan")
    got = plan.dynamic(qs, bad).cpu().numpy()
    plan.sync()
    assert np.isnan(got[0, 3].real)


def test_q_from_fraction_equals_the_mesh_shift():
    torch = _torch()
    import paper_1407_3444_amd as lib
    m = synth.random_model("sc", 4, 3)
    nk = (6, 4, 3)
    wl = synth.model_workload(m, nk, None, np.linspace(-0.5, 2.5, 40), shifts=[(2, 1, 2)])
    dev = torch.device("cuda:0")
    plan = lib.Chi0Plan(nk, torch.from_numpy(wl.eps_k).to(dev), torch.from_numpy(wl.c_k).to(dev))
    om = torch.from_numpy(wl.omega).to(dev)
    _say("q from q_frac")
    a = plan.dynamic([lib.Q(shift=(2, 1, 2))], om).cpu().numpy()
    b = plan.dynamic([lib.Q(q_frac=(2 / 6, 1 / 4, 2 / 3), from_frac=True),
                      lib.Q(q_frac=(1 + 2 / 6, -3 / 4, -1 / 3), from_frac=True)], om).cpu().numpy()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[0], b[1])
    with pytest.raises(lib.Chi0Error) as e:
        plan.static([lib.Q(q_frac=(0.1, 0.0, 0.0), from_frac=True)])
    assert e.value.status == -4
    ref = oracle.chi0(wl, 0)
    assert max_err(a[0], ref) <= 1e-10


def test_batch_hint_changes_launches_not_results():
    lib, torch, wl, plan, qs, om, eps, ck = _setup(nk=(5, 4, 3), q_subset=range(7))
    small = lib.Chi0Plan(wl.nk, eps, ck, mu=wl.mu, batch_hint=3)
    assert small.workspace_bytes(7, 24) < plan.workspace_bytes(7, 24)
    _say("batch_hint 3 vs 16")
    a = plan.dynamic(qs, om).cpu().numpy()
    b = small.dynamic(qs, om).cpu().numpy()
    assert np.array_equal(a, b)
    small.profile(True)
    small.read_profile()
    small.static(qs)
    prof = small.read_profile()
    assert prof["tetra"]["launches"] == 3           # 3 + 3 + 1 q


def test_degeneracy_tolerance_selects_the_fp64_near_branch():
    """Mixed form: a tolerance wider than every gap sends every near evaluation to the FP64 branch;
    both settings stay within the mixed-form bar of the oracle and give different results."""
    lib, torch, wl, plan, qs, om, eps, ck = _setup(nk=(6, 6, 3), nw=64, precision=1)
    wide = lib.Chi0Plan(wl.nk, eps, ck, mu=wl.mu, precision=1, degen_tol_ev=100.0)
    rel = lib.Chi0Plan(wl.nk, eps, ck, mu=wl.mu, precision=1, degen_rel_tol=2.0)
    _say("degeneracy tolerances")
    a = plan.dynamic(qs, om).cpu().numpy()[0]
    b = wide.dynamic(qs, om).cpu().numpy()[0]
    c = rel.dynamic(qs, om).cpu().numpy()[0]
    ref = oracle.chi0(wl, 0)
    for got in (a, b, c):
        assert max_err(got, ref) <= 1e-5
    assert not np.array_equal(a, b)
    assert np.array_equal(b, c)        # both rules mark every final tetrahedron


def test_empty_q_list_and_frequency_grid_are_rejected_at_every_entry_point():
    """An empty q list or frequency grid is an invalid argument (CHI0_E_INVALID_ARG) at every entry
    point that takes one: nothing is enqueued, the output keeps its contents, and the plan computes
    as before afterwards."""
    import ctypes
    lib, torch, wl, plan, qs, om, eps, ck = _setup()
    L, h = plan._lib, plan._h
    nw = len(om)
    ref = plan.dynamic(qs, om).cpu().numpy()
    plan.sync()
    arr = plan._qarray(qs)
    ws = plan.workspace(1, nw)
    wsp = plan.dynamic_pairs_workspace_bytes(1, nw)
    ws = torch.empty(max(ws.numel(), wsp) + (1 << 20), dtype=torch.uint8, device=om.device)
    wp, wn = ctypes.c_void_p(ws.data_ptr()), int(ws.numel())
    nbw = plan.nbw
    out = torch.full((nbw * nbw * nw * 2,), 7.0, dtype=torch.float64, device=om.device)
    op, cp = ctypes.c_void_p(om.data_ptr()), ctypes.c_void_p(out.data_ptr())
    sz = ctypes.c_size_t()
    counts = (ctypes.c_uint64 * 7)(*([5] * 7))
    calls = {
        "workspace_size, nq = 0": lambda: L.chi0_workspace_size(h, 0, nw, ctypes.byref(sz)),
        "workspace_size, nw = 0": lambda: L.chi0_workspace_size(h, 1, 0, ctypes.byref(sz)),
        "pairs workspace_size, nw = 0": lambda: L.chi0_dynamic_pairs_workspace_size(h, 1, 0, ctypes.byref(sz)),
        "kk workspace_size, nq = 0": lambda: L.chi0_kk_workspace_size(h, 0, nw, 64, ctypes.byref(sz)),
        "static, nq = 0": lambda: L.chi0_static(h, 0, arr, wp, wn, cp),
        "static_pairs, nq = 0": lambda: L.chi0_static_pairs(h, 0, arr, wp, wn, cp),
        "dynamic, nq = 0": lambda: L.chi0_dynamic(h, 0, arr, nw, op, wp, wn, cp),
        "dynamic, nw = 0": lambda: L.chi0_dynamic(h, 1, arr, 0, op, wp, wn, cp),
        "dynamic_pairs, nq = 0": lambda: L.chi0_dynamic_pairs(h, 0, arr, nw, op, wp, wn, cp),
        "dynamic_pairs, nw = 0": lambda: L.chi0_dynamic_pairs(h, 1, arr, 0, op, wp, wn, cp),
        "dynamic_noalloc, nq = 0": lambda: L.chi0_dynamic_noalloc(h, 0, arr, nw, op, cp),
        "dynamic_noalloc, nw = 0": lambda: L.chi0_dynamic_noalloc(h, 1, arr, 0, op, cp),
        "dynamic_kk, nw = 0": lambda: L.chi0_dynamic_kk(h, 1, arr, 0, op, 64, -20.0, 20.0, wp, wn, cp),
        "static_group, nq = 0": lambda: L.chi0_static_group(h, 0, 1, arr, wp, wn, cp),
        "dynamic_group, nw = 0": lambda: L.chi0_dynamic_group(h, 1, 1, arr, 0, op, wp, wn, cp),
        "census, nw = 0": lambda: L.chi0_census(h, 1, arr, 0, op, wp, wn, counts),
    }
    for what, call in calls.items():
        _say("empty input:", what)
        assert call() == -1, what
    torch.cuda.synchronize()
    assert bool((out == 7.0).all()) and list(counts) == [5] * 7
    got = plan.dynamic(qs, om).cpu().numpy()
    plan.sync()
    assert np.array_equal(got, ref)


def test_plan_follows_band_energies_changed_in_place():
    """A plan borrows its band energies; the band ranges from which the tetrahedron kernels skip
    inert band pairs are taken anew by every call, so a band moved across the Fermi level in place
    between two calls contributes in the second, which matches the oracle on the changed data."""
    lib, torch, wl, plan, qs, om, eps, ck = _setup(q_subset=(3, 5))
    first = plan.dynamic(qs, om).cpu().numpy()
    plan.sync()
    below = [b for b in range(wl.eps_k.shape[0]) if wl.eps_k[b].max() < wl.mu]
    assert below, "the model needs a band entirely below the Fermi level"
    b = below[-1]
    shift = float(wl.mu - wl.eps_k[b].mean())
    _say("band", b, "moved by", shift)
    eps[b] += shift
    wl.eps_k[b] += shift
    for q in wl.qs:                      # explicit k+q energies of the same bands move alike
        q.eps_kq[b] += shift
    qs2 = [lib.Q(eps_kq=torch.from_numpy(q.eps_kq).to(eps.device), c_kq=q2.c_kq) for q, q2 in zip(wl.qs, qs)]
    got = plan.dynamic(qs2, om).cpu().numpy()
    plan.sync()
    for j in range(len(qs2)):
        ref = oracle.chi0(wl, j)
        e = max_err(got[j], ref)
        _say("q", j, "after the move: err", e)
        assert e <= 1e-10
    assert max_err(got[0], first[0]) > 1e-6
