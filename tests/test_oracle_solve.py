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


def _micro_problem(seed=0, n_vox=40):
    """Two beams of two MLC rows of three beamlets each, a random sparse
    non-negative D, a target (first half of the voxels: T- = T+ = 1,
    weights 1) and an organ (second half: T+ = 0.3, weight 0.5)."""
    rng = np.random.default_rng(seed)
    n_blt = 12
    dense = rng.uniform(0.0, 1.0, (n_vox, n_blt)) * (rng.uniform(size=(n_vox, n_blt)) < 0.5)
    import scipy.sparse as sp
    D = sp.csr_matrix(dense)
    vs = np.zeros(n_vox, dtype=np.int16)
    vs[n_vox // 2:] = 1
    pres = [dict(is_target=1, t_under=1.0, t_over=1.0, w_under=1.0, w_over=1.0),
            dict(is_target=0, t_under=0.0, t_over=0.3, w_under=0.0, w_over=0.5)]
    return oracle.make_problem(D, [2, 2], [3, 3, 3, 3], vs, pres)


def _fmo_optimum(P):
    def fg(x):
        z = oracle.dose(P, x)
        return oracle.objective(P, z), oracle.prices(P, oracle.grad_objective(P, z))

    r = so.minimize(fg, np.full(P.n_blt, 0.1), jac=True, method="L-BFGS-B", bounds=[(0, None)] * P.n_blt,
                    options=dict(ftol=1e-16, gtol=1e-14, maxiter=100000, maxcor=30))
    return r.fun


@pytest.mark.parametrize("seed", range(3))
def test_optimal_stop_reaches_fmo_optimum(seed):
    """When the loop ends because no aperture prices below -tau, the plan is
    optimal over every deliverable aperture, and since every fluence map
    x >= 0 is a non-negative sum of aperture indicators (each row's profile
    splits into intervals), that optimum is the fluence-map optimum of
    Section 2.2's equivalence (found here by L-BFGS-B over x >= 0)."""
    P = _micro_problem(seed)
    res = oracle.solve(P, 200, eps=1e-12, max_steps=200000, tau_rel=1e-10)
    assert res["status"] == "optimal", res["status"]
    f_fmo = _fmo_optimum(P)
    assert f_fmo > 1e-4                        # a non-trivial optimum
    assert abs(res["F"] - f_fmo) <= 1e-9 * f_fmo, (res["F"], f_fmo, len(res["pool"]))


def _one_voxel_problem():
    """One target voxel (T- = T+ = 1, weights 1) reached by the two beamlets
    of a single MLC row with D = [1, 1]: F(y) = (1 - 2 y)^2 for the aperture
    opening both, whose reduced cost at y = 0 is -4."""
    import scipy.sparse as sp
    D = sp.csr_matrix(np.array([[1.0, 1.0]]))
    pres = [dict(is_target=1, t_under=1.0, t_over=1.0, w_under=1.0, w_over=1.0)]
    return oracle.make_problem(D, [1], [2], np.zeros(1, np.int16), pres)


def test_duplicate_aperture_tightens_then_succeeds():
    """eps = 10: the master stops at once (KKT residual 4 <= 10 * |rc_1|), so
    pricing returns the pooled aperture again; the tolerance is divided by 10
    (residual 4 <= 4 still stops it), again by 10 (0.4 < 4: one exact step
    reaches y = 1/2), after which nothing prices negative."""
    P = _one_voxel_problem()
    res = oracle.solve(P, 5, eps=10.0, max_steps=100, max_tighten=3)
    assert res["rc1"] == -4.0
    assert res["status"] == "optimal"
    assert len(res["pool"]) == 1 and res["pool"][0].leaves == ((0, 2),)
    assert res["eps"] == pytest.approx(0.1, rel=1e-15)
    assert res["y"][0] == 0.5 and res["F"] == 0.0


def test_duplicate_aperture_stalls_after_max_tighten():
    """The same problem with one tightening allowed: the second duplicate ends
    the loop as stalled, with the pool and the (unmoved) intensity kept."""
    P = _one_voxel_problem()
    res = oracle.solve(P, 5, eps=10.0, max_steps=100, max_tighten=1)
    assert res["status"] == "stalled"
    assert len(res["pool"]) == 1 and res["y"][0] == 0.0
    assert res["eps"] == pytest.approx(1.0, rel=1e-15)
    assert res["F"] == 1.0
