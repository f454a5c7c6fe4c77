"""Whole-loop invariants of the column-generation oracle.

* F never increases from one round to the next (adding an aperture with
  y = 0 keeps the previous point feasible);
* the DAO objective is bounded below by the fluence-map optimum over
  beamlet intensities x >= 0 (the DAO model is the same model with its
  variables restricted to sums of aperture indicators; Section 2.2), found
  here with scipy's L-BFGS-B;
* every aperture in the pool is deliverable (one contiguous run per row of
  its beam) and distinct;
* plan metrics D95 and Dmax against their definitions on hand-made doses.
"""
import math

import numpy as np
import pytest
import scipy.optimize as so

import oracle
from conftest import cached_phantom, oracle_problem


@pytest.fixture(scope="module")
def mini_solution():
    ph = cached_phantom("mini")
    P = oracle_problem(ph)
    return ph, P, oracle.solve(P, 6, eps=1e-8, max_steps=3000)


def test_objective_decreases_over_rounds(mini_solution):
    ph, P, res = mini_solution
    Fs = [1.0 * oracle.objective(P, np.zeros(P.n_vox))] + [r["F"] for r in res["log"]]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(Fs[:-1], Fs[1:]))
    assert res["log"][0]["rc"] < 0


def test_fmo_lower_bound(mini_solution):
    ph, P, res = mini_solution

    def fg(x):
        z = oracle.dose(P, x)
        return oracle.objective(P, z), oracle.prices(P, oracle.grad_objective(P, z))

    r = so.minimize(fg, np.full(P.n_blt, 0.01), jac=True, method="L-BFGS-B",
                    bounds=[(0, None)] * P.n_blt,
                    options=dict(ftol=1e-15, gtol=1e-12, maxiter=20000))
    assert r.fun <= res["F"] * (1 + 1e-9)
    assert res["F"] < 5 * r.fun + 1e-3    # a 6-aperture plan is in the same range


def test_pool_deliverable_and_distinct(mini_solution):
    ph, P, res = mini_solution
    assert len(set(res["pool"])) == len(res["pool"])
    for ap in res["pool"]:
        r0, r1 = P.beam_row_range(ap.beam)
        assert len(ap.leaves) == r1 - r0
        for r, (L, R) in zip(range(r0, r1), ap.leaves):
            assert 0 <= L <= R <= P.row_len[r]
            assert (L < R) or (L, R) == (0, 0)
    x = oracle.beamlet_intensity(P, res["pool"], res["y"])
    np.testing.assert_allclose(oracle.dose(P, x), res["d"], rtol=1e-10, atol=1e-14)


def test_optimal_stop_when_nothing_prices_negative():
    ph = cached_phantom("mini")
    pres = [dict(p) for p in ph.prescriptions]
    pres[0].update(t_under=0.0, w_under=0.0)     # no dose wanted anywhere
    P = oracle.make_problem(ph.csr(), ph.rows_per_beam, ph.row_len, ph.vox_struct, pres)
    res = oracle.solve(P, 5)
    assert res["status"] == "optimal" and res["pool"] == []


def test_d95_dmax_definitions():
    z = np.arange(100, dtype=float)[::-1]
    m = np.ones(100, bool)
    assert oracle.d95(z, m) == 5.0
    assert oracle.dmax(z, m) == 99.0
    m2 = np.zeros(100, bool)
    m2[[3, 50, 70]] = True
    assert oracle.dmax(z, m2) == 96.0
    assert oracle.d95(z, m2) == 29.0
    # D95 is the largest dose that at least 95 % of the voxels reach
    rng = np.random.default_rng(0)
    for n in (1, 3, 19, 20, 21, 1000):
        v = rng.normal(size=n)
        best = max(c for c in v if np.count_nonzero(v >= c) >= 0.95 * n)
        assert oracle.d95(v, np.ones(n, bool)) == best
