"""chi0_dynamic_noalloc: the dynamic call with the library's fixed device scratch as workspace (for
callers that cannot allocate), against chi0_dynamic with a caller workspace on the same inputs, on
two calls in a row (the second smaller), and its rejection of a plan too large for the scratch."""
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


def test_no_alloc_call_equals_the_workspace_call_on_two_calls_in_a_row():
    torch = _torch()
    import paper_1407_3444_amd as lib
    # 15 MB of workspace per q: the 128 MiB scratch holds 8 q per launch sequence, so the 12 q of the
    # first call run as 8 + 4 there against one sequence of 12 with a caller workspace
    wl = synth.make_workload("tetra_dynamic", nk=(32, 32, 8), nq=16, q_subset=list(range(2, 14)), nw=600,
                             workers=8)
    dev = torch.device("cuda:0")
    plan = lib.Chi0Plan(wl.nk, torch.from_numpy(wl.eps_k).to(dev), torch.from_numpy(wl.c_k).to(dev), mu=wl.mu)
    assert 12 * 15e6 > (128 << 20) > 8 * 15e6
    qs = [lib.Q(eps_kq=torch.from_numpy(q.eps_kq).to(dev), c_kq=torch.from_numpy(q.c_kq).to(dev)) for q in wl.qs]
    om = torch.from_numpy(wl.omega).to(dev)
    _say("no-alloc call 1: 12 q x 600 w on 32x32x8")
    ref = plan.dynamic(qs, om).cpu().numpy()
    out = torch.empty((len(qs), len(wl.omega), 2), dtype=torch.float64, device=dev)
    got = plan.dynamic_noalloc(qs, om, out).cpu().numpy()
    plan.sync()
    assert np.array_equal(got, ref)
    for i in (0, 11):
        assert max_err(got[i], ref[i]) <= 1e-10
    # second call, smaller: 3 q, 70 frequencies (new values over the scratch left by call 1)
    sub = [qs[9], qs[4], qs[0]]
    om2 = om[100:170].contiguous()
    _say("no-alloc call 2: 3 q x 70 w")
    ref2 = plan.dynamic(sub, om2).cpu().numpy()
    out2 = torch.empty((3, 70), dtype=torch.complex128, device=dev)
    got2 = plan.dynamic_noalloc(sub, om2, out2).cpu().numpy()
    plan.sync()
    assert np.array_equal(got2, ref2)
    # and the oracle, at the FP64 bar, on one q of the second call
    sample = [0, 33, 69]
    r = oracle.chi0(wl, 4, omega=wl.omega[100:170][sample])
    assert max_err(got2[1][sample], r) <= 1e-10


def test_no_alloc_call_rejects_a_plan_too_large_for_the_scratch():
    torch = _torch()
    import paper_1407_3444_amd as lib
    dev = torch.device("cuda:0")
    nk = (64, 64, 8)                                  # 32 bands: W of one q is 268 MB > 128 MiB
    eps = torch.zeros((32, 32768), dtype=torch.float64, device=dev)
    ck = torch.zeros((32768, 1, 32), dtype=torch.complex128, device=dev)
    plan = lib.Chi0Plan(nk, eps, ck, skip_input_scan=True)
    om = torch.zeros(4, dtype=torch.float64, device=dev)
    out = torch.empty((1, 4, 2), dtype=torch.float64, device=dev)
    with pytest.raises(lib.Chi0Error) as e:
        plan.dynamic_noalloc([lib.Q(shift=(1, 0, 0))], om, out)
    assert e.value.status == -5 and "scratch" in str(e.value)
