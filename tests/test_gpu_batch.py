"""GPU: the batched entry point against the single-plan calls and the CPU FP64 oracle.

A batch of heterogeneous instances (three lattice families, 1..14 orbitals, band windows, CMA,
both forms, mixed precision, more than 512 frequencies, shift and explicit q) must give, per
instance and q, the same chi0 as chi0_dynamic (to rounding of the block partition) and the
oracle within the FP64 bar; the graph replays, the W-budget stages and the tuner must not change
the result.
"""
import numpy as np
import pytest

import oracle
import synth
from metrics import max_err

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print(*a, flush=True)


def _relerr(got, ref):
    """Normwise difference of two GPU results (consistency of two launch schedules)."""
    return np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300)


def _workloads():
    """Seeded small instances; every q either a mesh shift or explicit k+q data."""
    wls = []
    m = synth.random_model("tetragonal", 501, 6)
    wl = synth.model_workload(m, (6, 6, 4), None, synth.omega_grid(96), shifts=[(1, 2, 1), (3, 0, 2), (5, 5, 3)])
    wls.append((wl, {}))
    m = synth.random_model("bcc", 502, 9)
    wl = synth.model_workload(m, (6, 6, 6), [np.array([0.0, 0.29, 0.0])], np.linspace(-0.5, 3.0, 600))
    wl.band_lo, wl.band_hi = synth.band_window(wl.eps_k, 5)
    wls.append((wl, {}))
    m = synth.random_model("sc", 503, 4)
    wl = synth.model_workload(m, (5, 7, 4), None, synth.omega_grid(40), shifts=[(2, 3, 1), (1, 1, 1)])
    wl.form = 1
    wls.append((wl, {}))
    m = synth.sc_nn_model(1.0)
    wl = synth.model_workload(m, (8, 8, 8), None, synth.omega_grid(130), shifts=[(1, 1, 1), (3, 3, 3)])
    wl.c_k, wl.cma = None, True
    wls.append((wl, {}))
    m = synth.random_model("tetragonal", 505, 14)
    wl = synth.model_workload(m, (4, 4, 6), None, synth.omega_grid(64), shifts=[(1, 3, 2)])
    wls.append((wl, {"precision": 1}))
    return wls


def _instance(wl, precision=0):
    torch = _torch()
    import paper_1407_3444_amd as lib
    dev = torch.device("cuda:0")
    eps = torch.from_numpy(np.ascontiguousarray(wl.eps_k)).to(dev)
    ck = None if (wl.c_k is None or wl.cma) else torch.from_numpy(np.ascontiguousarray(wl.c_k)).to(dev)
    qs = []
    for q in wl.qs:
        if q.shift is not None:
            qs.append(lib.Q(shift=q.shift))
        else:
            e = torch.from_numpy(np.ascontiguousarray(q.eps_kq)).to(dev)
            c = None if wl.cma else torch.from_numpy(np.ascontiguousarray(q.c_kq)).to(dev)
            qs.append(lib.Q(eps_kq=e, c_kq=c))
    lo, hi = wl.window()
    om = torch.from_numpy(np.ascontiguousarray(wl.omega)).to(dev)
    return lib.Instance(nk=wl.nk, eps_k=eps, c_k=ck, qs=qs, omega=om, mu=wl.mu, spin_factor=wl.spin_factor,
                        band_lo=lo, band_hi=hi, cma=wl.cma, form=wl.form, precision=precision)


def _single(ins):
    import paper_1407_3444_amd as lib
    plan = lib.Chi0Plan(ins.nk, ins.eps_k, ins.c_k, mu=ins.mu, spin_factor=ins.spin_factor, band_lo=ins.band_lo,
                        band_hi=ins.band_hi, cma=ins.cma, form=ins.form, precision=ins.precision)
    return plan.dynamic(ins.qs, ins.omega).cpu().numpy()


@pytest.fixture(scope="module")
def batch_setup():
    wls = _workloads()
    insts = [_instance(wl, **kw) for wl, kw in wls]
    return wls, insts


def test_batch_equals_single_plans_and_oracle(batch_setup):
    torch = _torch()
    import paper_1407_3444_amd as lib
    wls, insts = batch_setup
    _say("batch of", len(insts), "instances, direct launches")
    b = lib.Chi0Batch(insts, workgroups=512, use_graph=False)
    info = b.info()
    _say("batch info", info)
    assert info["items"] == sum(len(w.qs) * ((len(w.omega) + 511) // 512) for w, _ in wls)
    out = [c.cpu().numpy() for c in b.run()]
    torch.cuda.synchronize()
    for i, ((wl, kw), ins) in enumerate(zip(wls, insts)):
        ref_plan = _single(ins)
        err = _relerr(out[i], ref_plan)
        _say("instance", i, "batch vs plan", err)
        assert err <= 1e-13, (i, err)
        if kw.get("precision", 0) == 0:
            for j in range(len(wl.qs)):
                ref = oracle.chi0(wl, j)
                e = max_err(out[i][j], ref)
                assert e <= TOL, (i, j, e)


def test_batch_graph_replays_and_stages(batch_setup):
    torch = _torch()
    import paper_1407_3444_amd as lib
    wls, insts = batch_setup
    _say("batch graph replays")
    eager = lib.Chi0Batch(insts, workgroups=512, use_graph=False)
    ref = [c.cpu().numpy().copy() for c in eager.run()]
    torch.cuda.synchronize()
    eager.close()
    g = lib.Chi0Batch(insts, workgroups=512, use_graph=True)
    for rep in range(3):
        for ins in insts:
            ins.chi.fill_(float("nan"))
        # eager work of the program between replays
        x = torch.randn(1 << 16, device="cuda:0", dtype=torch.float64)
        float((x * x).sum())
        got = [c.cpu().numpy() for c in g.run()]
        torch.cuda.synchronize()
        for i in range(len(insts)):
            assert np.array_equal(got[i], ref[i]), (rep, i)
    g.close()
    # a W budget of one group per stage: same per-item partition, bitwise equal results
    w_max = max(8 * (ins.band_hi - ins.band_lo) ** 2 * int(np.prod(ins.nk)) for ins in insts if not ins.cma)
    s = lib.Chi0Batch(insts, workgroups=512, stage_w_bytes=w_max, use_graph=True)
    assert s.info()["stages"] > 1
    got = [c.cpu().numpy() for c in s.run()]
    torch.cuda.synchronize()
    for i in range(len(insts)):
        assert np.array_equal(got[i], ref[i]), i


def test_batch_tune_keeps_results(batch_setup):
    torch = _torch()
    import paper_1407_3444_amd as lib
    wls, insts = batch_setup
    _say("batch tune")
    b = lib.Chi0Batch(insts, workgroups=2048, use_graph=True)
    chosen = b.tune(reps=1)
    assert chosen in (2048, 1024, 512, 256)
    tile = b.info()["omega_tile"]
    _say("tuned workgroups", chosen, "frequency tile", tile)
    assert tile in (256, 512)
    tuned = [c.cpu().numpy().copy() for c in b.run()]
    torch.cuda.synchronize()
    for i, ins in enumerate(insts):
        ref = _single(ins)
        assert _relerr(tuned[i], ref) <= 1e-13, i


def test_graph_replay_follows_band_energies_changed_in_place():
    """The batched K_B skips band pairs whose energy ranges rule out a carved region; the ranges
    are taken inside the captured launch sequence, so a replay after the band energies changed in
    place must see the new ranges: a band moved from below the Fermi level to across it adds its
    pairs' contributions, equal to a fresh single-plan call on the changed data."""
    torch = _torch()
    import paper_1407_3444_amd as lib
    m = synth.random_model("tetragonal", 511, 6)
    wl = synth.model_workload(m, (6, 6, 4), None, synth.omega_grid(96), shifts=[(1, 2, 1), (3, 0, 2)])
    below = [b for b in range(wl.eps_k.shape[0]) if wl.eps_k[b].max() < wl.mu]
    assert below, "the model needs a band entirely below the Fermi level"
    ins = _instance(wl)
    g = lib.Chi0Batch([ins], workgroups=256, use_graph=True)
    first = g.run()[0].cpu().numpy().copy()
    torch.cuda.synchronize()
    assert _relerr(first, _single(ins)) <= 1e-13
    b = below[0]
    shift = float(wl.mu - wl.eps_k[b].mean())
    _say("band", b, "moved by", shift, "eV across the Fermi level")
    ins.eps_k[b] += shift                        # in place: the captured graph reads the same memory
    torch.cuda.synchronize()
    again = g.run()[0].cpu().numpy().copy()
    torch.cuda.synchronize()
    ref = _single(ins)
    assert _relerr(again, ref) <= 1e-13
    assert _relerr(again, first) > 1e-6          # the band's new pairs contribute
    g.close()
