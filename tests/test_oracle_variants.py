"""Pins for the method variants of the oracle.

Nested targets (Section 3's head-and-neck cases: PTV1 inside PTV2, each
with its own prescription; eq. 10 sums the terms of every structure that
contains a voxel):
* the objective equals eq. 9 + eq. 10 summed structure by structure over
  each structure's voxel set (a direct transcription, independent of the
  per-voxel term arrays), with and without per-voxel threshold shifts;
* the gradient matches central finite differences of F(D x);
* the exact line search matches a sort of every breakpoint of every term.

Re-optimization mode (Discussion: eq. 3 and eq. 4 with alpha_j = beta_j = 1
and T_j the deformed dose of the original plan):
* at zero dose the prices are w = -2 D^T (T on the target) (closed form);
* when T is the dose of a pool at known intensities y0, the master over that
  pool reaches F = 0 and y = y0 (D_K of full column rank);
* the column-generation loop never increases F.

Several apertures per round:
* the beam ranking's values equal each beam's optimum found by enumerating
  every interval of every row (brute force), in value order with ties to the
  lowest beam, and each ranked aperture attains its value;
* the loop fills the budget with distinct apertures in fewer rounds and never
  increases F.
"""
import math

import numpy as np
import pytest

import oracle
from conftest import cached_phantom
from oracle.master import MasterState, solve_master


def _nested_problem(ph, shift=None):
    return oracle.make_problem(ph.csr(), ph.rows_per_beam, ph.row_len, ph.vox_struct, ph.prescriptions,
                               vox_struct2=ph.vox_struct2, vox_shift=shift)


def _direct_objective(ph, z, shift=None):
    """eq. 9 + eq. 10 structure by structure, thresholds shifted per voxel."""
    tau = np.zeros(ph.n_vox) if shift is None else np.asarray(shift)
    total = []
    for s, pr in enumerate(ph.prescriptions):
        members = ph.vox_struct == s
        if ph.vox_struct2 is not None:
            members = members | (ph.vox_struct2 == s)
        n = int(members.sum())
        if n == 0:
            continue
        zs, ts = z[members], tau[members]
        if pr["is_target"]:
            total.append(pr["w_under"] / n * math.fsum((np.maximum(0.0, pr["t_under"] + ts - zs) ** 2).tolist()))
        total.append(pr["w_over"] / n * math.fsum((np.maximum(0.0, zs - pr["t_over"] - ts) ** 2).tolist()))
    return math.fsum(total)


@pytest.mark.parametrize("shifted", [False, True])
def test_nested_objective_equals_per_structure_sum(shifted):
    ph = cached_phantom("mini", nested_targets=True)
    assert "PTV1" in ph.struct_names and np.any(ph.vox_struct2 >= 0)
    rng = np.random.default_rng(3)
    shift = rng.uniform(-0.2, 0.2, ph.n_vox) if shifted else None
    P = _nested_problem(ph, shift)
    assert P.extra is not None
    for k in range(4):
        z = rng.uniform(0.0, 1.3, ph.n_vox)
        F = oracle.objective(P, z)
        ref = _direct_objective(ph, z, shift)
        assert abs(F - ref) <= 1e-12 * ref, (k, F, ref)
    # a PTV1 voxel's objective has both targets' under-dose terms
    j = int(np.flatnonzero(ph.vox_struct2 >= 0)[0])
    z = np.full(ph.n_vox, 0.5)
    f = oracle.model.objective_terms(P, z)[j]
    n1 = int(np.sum((ph.vox_struct == 0) | (ph.vox_struct2 == 0)))
    n2 = int(np.sum((ph.vox_struct == 1) | (ph.vox_struct2 == 1)))
    t1, t2 = ph.prescriptions[0]["t_under"], ph.prescriptions[1]["t_under"]
    tau = 0.0 if shift is None else shift[j]
    expect = (max(0.0, t1 + tau - 0.5) ** 2 / n1 + max(0.0, t2 + tau - 0.5) ** 2 / n2
              + max(0.0, 0.5 - 1.0 - tau) ** 2 * (1.0 / n1 + 1.0 / n2))
    assert abs(f - expect) <= 1e-15 + 1e-12 * expect


def test_nested_gradient_finite_differences():
    ph = cached_phantom("mini", nested_targets=True)
    P = _nested_problem(ph)
    rng = np.random.default_rng(4)
    x = rng.uniform(0.0, 0.08, ph.n_blt)
    g = oracle.prices(P, oracle.grad_objective(P, oracle.dose(P, x)))
    for i in rng.choice(ph.n_blt, 8, replace=False):
        h = 1e-6
        e = np.zeros(ph.n_blt)
        e[i] = h
        fd = (oracle.objective(P, oracle.dose(P, x + e)) - oracle.objective(P, oracle.dose(P, x - e))) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-8, np.max(np.abs(g))), (i, fd, g[i])


def _phi_prime(P, d, q, t):
    return math.fsum((q * oracle.grad_objective(P, d + t * q)).tolist())


@pytest.mark.parametrize("seed", range(4))
def test_nested_line_search_against_breakpoint_sort(seed):
    ph = cached_phantom("mini", nested_targets=True)
    P = _nested_problem(ph)
    rng = np.random.default_rng(seed)
    d = oracle.dose(P, rng.uniform(0.0, 0.05, ph.n_blt))
    q = oracle.dose(P, -oracle.prices(P, oracle.grad_objective(P, d)) * rng.uniform(0.5, 1.5, ph.n_blt))
    assert _phi_prime(P, d, q, 0.0) < 0
    bps = []
    for a, tu, b, to in P.terms():
        for T, w in ((tu, a), (to, b)):
            m = (q != 0) & (w > 0)
            bps.append((T - d)[m] / q[m])
    bps = np.concatenate(bps)
    cand = np.unique(np.concatenate([[0.0], bps[bps > 0]]))
    ref = None
    for ta, tb in zip(cand[:-1], cand[1:]):
        ga, gb = _phi_prime(P, d, q, ta), _phi_prime(P, d, q, tb)
        if gb >= 0:
            ref = ta - ga * (tb - ta) / (gb - ga)
            break
    if ref is None:
        ta = cand[-1]
        ga, gb = _phi_prime(P, d, q, ta), _phi_prime(P, d, q, ta + 1.0)
        ref = ta - ga / (gb - ga)
    t, _ = oracle.line_search(P, d, q, math.inf)
    assert abs(t - ref) <= 1e-9 * ref


def _reopt_problem(ph, T):
    reached = np.diff(ph.row_ptr) > 0
    labels, pres = oracle.reoptimization_structures(ph.vox_struct == 0, reached)
    return oracle.make_problem(ph.csr(), ph.rows_per_beam, ph.row_len, labels, pres, vox_shift=T), labels


def test_reoptimization_weights_are_one_and_first_prices_closed_form():
    ph = cached_phantom("mini")
    rng = np.random.default_rng(5)
    T = rng.uniform(0.2, 1.0, ph.n_vox)
    P, labels = _reopt_problem(ph, T)
    tgt = labels == 0
    assert np.all(P.a[tgt] == 1.0) and np.all(P.a[~tgt] == 0.0)
    assert np.all(P.b[labels >= 0] == 1.0)
    np.testing.assert_array_equal(P.t_under[tgt], T[tgt])
    np.testing.assert_array_equal(P.t_over[labels >= 0], T[labels >= 0])
    # at zero dose only the target's under-dose terms are active
    st = MasterState.empty(P)
    w_ref = -2.0 * (ph.csr().T @ np.where(tgt, T, 0.0))
    np.testing.assert_allclose(st.g, w_ref, rtol=1e-13, atol=1e-15)
    # F(0) = sum over target voxels of T_j^2
    assert abs(oracle.objective(P, np.zeros(ph.n_vox)) - math.fsum((T[tgt] ** 2).tolist())) <= 1e-12


def test_reoptimization_recovers_a_reachable_plan():
    ph = cached_phantom("mini")
    P0 = oracle.make_problem(ph.csr(), ph.rows_per_beam, ph.row_len, ph.vox_struct, ph.prescriptions)
    pool = oracle.solve(P0, 4, eps=1e-4, max_steps=60)["pool"]
    y0 = np.array([0.03, 0.02, 0.04, 0.01])
    T = oracle.dose(P0, oracle.beamlet_intensity(P0, pool, y0))
    P, _ = _reopt_problem(ph, T)
    DK = np.stack([oracle.dose(P, oracle.beamlet_intensity(P, [ap], [1.0])) for ap in pool], axis=1)
    assert np.linalg.matrix_rank(DK) == len(pool)
    st = MasterState.empty(P)
    for ap in pool:
        st.add(ap)
    F0 = oracle.objective(P, st.d)
    log = solve_master(P, st, tol=1e-14 * F0, max_steps=5000)
    F = oracle.objective(P, st.d)
    assert F <= 1e-16 * F0, (F, F0, log["steps"])
    np.testing.assert_allclose(st.y, y0, rtol=1e-6)


def test_reoptimization_loop_decreases_objective():
    ph = cached_phantom("mini")
    rng = np.random.default_rng(6)
    T = oracle.dose(oracle.make_problem(ph.csr(), ph.rows_per_beam, ph.row_len, ph.vox_struct, ph.prescriptions),
                    rng.uniform(0.0, 0.05, ph.n_blt))
    # the deformed dose: the original dose moved by one voxel along x
    T = np.roll(T.reshape(ph.shape[::-1]), 1, axis=2).reshape(-1)
    P, _ = _reopt_problem(ph, T)
    res = oracle.solve(P, 5, eps=1e-8, max_steps=2000)
    Fs = [oracle.objective(P, np.zeros(ph.n_vox))] + [r["F"] for r in res["log"]]
    assert res["log"][0]["rc"] < 0
    assert all(b <= a * (1 + 1e-12) for a, b in zip(Fs[:-1], Fs[1:]))


# --- several apertures per round --------------------------------------------

def _beam_optimum_brute(P, g, b):
    """Smallest sum over every deliverable aperture of beam b (each row: closed
    or any contiguous run), by enumeration of each row's intervals."""
    r0, r1 = P.beam_row_range(b)
    starts = P.row_start()
    total = 0.0
    for r in range(r0, r1):
        w = g[starts[r]:starts[r] + P.row_len[r]]
        n = len(w)
        best = min([0.0] + [math.fsum(w[l:q].tolist()) for q in range(1, n + 1) for l in range(q)])
        total += best
    return total


def test_ranked_apertures_order_and_values():
    ph = cached_phantom("mini")
    P = oracle.make_problem(ph.csr(), ph.rows_per_beam, ph.row_len, ph.vox_struct, ph.prescriptions)
    rng = np.random.default_rng(8)
    for k in range(3):
        d = oracle.dose(P, rng.uniform(0.0, 0.06, ph.n_blt))
        g = oracle.prices(P, oracle.grad_objective(P, d))
        pr = oracle.price(P, g)
        ranked = oracle.ranked_apertures(P, pr)
        assert ranked[0][1] == pr["aperture"] and ranked[0][0] == pr["rc"]
        brute = sorted((_beam_optimum_brute(P, g, b), b) for b in range(len(ph.rows_per_beam)))
        assert [ap.beam for _, ap in ranked] == [b for _, b in brute]
        for (v, ap), (vb, _) in zip(ranked, brute):
            assert abs(v - vb) <= 1e-14 * max(1.0, abs(vb))
            # each beam's aperture attains its value
            assert abs(math.fsum(g[ap.open_beamlets(P)].tolist()) - v) <= 1e-14 * max(1.0, abs(v))


def test_several_apertures_per_round_loop():
    ph = cached_phantom("mini")
    P = oracle.make_problem(ph.csr(), ph.rows_per_beam, ph.row_len, ph.vox_struct, ph.prescriptions)
    res = oracle.solve(P, 7, eps=1e-8, max_steps=3000, per_round=3)
    assert len(res["pool"]) == 7 and len(set(res["pool"])) == 7
    assert len(res["log"]) < 7          # some round added more than one
    assert any(r["extra"] for r in res["log"])
    Fs = [oracle.objective(P, np.zeros(ph.n_vox))] + [r["F"] for r in res["log"]]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(Fs[:-1], Fs[1:]))
    # the same budget one aperture at a time ends at a comparable objective
    one = oracle.solve(P, 7, eps=1e-8, max_steps=3000)
    assert res["F"] < 3.0 * one["F"] and one["F"] < 3.0 * res["F"]
