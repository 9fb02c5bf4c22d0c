"""The oracle's operation and active-unit counts, which give the benchmark's second op-count figure
(operations per active unit and frequency in the oracle's own formulation)."""
import numpy as np
from scipy.optimize import linprog

import oracle
import synth


def _region_nonempty(a, b):
    """Whether {a < 0 < b} meets the tetrahedron in a set of positive volume (Sec. II carving
    regions, a = e - mu, b = e' - mu linear on the simplex): max t subject to a.l + t <= 0,
    -b.l + t <= 0 over barycentric l, by linear programming."""
    c = np.zeros(5)
    c[4] = -1.0
    A = np.array([list(a) + [1.0], list(-np.asarray(b)) + [1.0]])
    res = linprog(c, A_ub=A, b_ub=[0.0, 0.0], A_eq=[[1.0, 1.0, 1.0, 1.0, 0.0]], b_eq=[1.0],
                  bounds=[(0.0, None)] * 4 + [(None, 1.0)], method="highs")
    return res.status == 0 and -res.fun > 1e-12


def _workload():
    wl = synth.make_workload("tetra_dynamic", nk=(3, 3, 2), nq=8, q_subset=[3], nw=8)
    wl.band_lo, wl.band_hi = 3, 7            # 16 band pairs around mu
    return wl


def test_active_units_equal_a_linear_programming_count():
    """Units (mesh tetrahedron, band pair) with a non-empty region e < mu < e' or e' < mu < e,
    counted by the oracle while it evaluates, against linear programs on every unit."""
    wl = _workload()
    oracle.chi0(wl, 0, omega=wl.omega[:1])
    _, units = oracle.last_count()
    q = wl.qs[0]
    lo, hi = wl.window()
    expect = 0
    for cell in range(wl.n_k):
        for t in range(6):
            idx = oracle.tet_corners(wl.nk, cell, t)
            for n in range(lo, hi):
                for m in range(lo, hi):
                    a = wl.eps_k[n][idx] - wl.mu
                    b = q.eps_kq[m][idx] - wl.mu
                    expect += int(_region_nonempty(a, b) or _region_nonempty(-a, -b))
    assert units == expect and units > 0


def test_operation_count_is_per_frequency_and_thread_independent():
    """The tally does not depend on the thread count, and its frequency-independent part (the
    carving) is the same for every split of the frequencies: ops(A) + ops(B) - ops(A u B)."""
    wl = _workload()
    om = wl.omega

    def ops(idx, threads=0):
        oracle.chi0(wl, 0, omega=om[idx], nthreads=threads)
        return oracle.last_count()[0]

    full = ops(list(range(8)))
    assert full == ops(list(range(8)), threads=1) == ops(list(range(8)), threads=3)
    fixed1 = ops([0, 1, 2]) + ops([3, 4, 5, 6, 7]) - full
    fixed2 = ops([0, 5]) + ops([1, 2, 3, 4, 6, 7]) - full
    assert fixed1 == fixed2 and 0 < fixed1 < full / 8
