"""Pins for the restricted master (gradient projection, Section 2.3).

* Exact line search against brute force: every breakpoint of the piecewise
  quadratic phi(t) = F(d + t q) is sorted, phi' is evaluated at each, and the
  root is interpolated inside the piece where phi' changes sign.
* NNLS special case: with every voxel in one target whose under- and
  over-dose thresholds and weights coincide, F is a scaled least-squares
  objective ||D_K y - T||^2, so the converged master must agree with
  scipy.optimize.nnls on the aperture dose matrix.
* General master against scipy's L-BFGS-B with bounds y >= 0.
* Invariants: F never increases from one step to the next, and the KKT
  conditions hold at exit.
* Conjugate gradient projection: on the NNLS special case (F one quadratic)
  started on the optimum's face, the conjugate direction must reach the
  NNLS optimum in K steps (the finite termination of conjugate gradients
  with exact line searches), which plain projected steepest descent does
  not; after a blocking step the next direction is the projected negative
  gradient again.
The pins on the converged master run in both direction modes.
"""
import math

import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp

import oracle
from conftest import cached_phantom, oracle_problem
from oracle.master import MasterState, kkt_residual, solve_master


def _phi_prime(P, d, q, t):
    return math.fsum((q * oracle.grad_objective(P, d + t * q)).tolist())


def _brute_line_search(P, d, q, t_max):
    nz = q != 0
    bps = []
    for T, wgt in ((P.t_under, P.a), (P.t_over, P.b)):
        m = nz & (wgt > 0)
        bps.append((T - d)[m] / q[m])
    bps = np.concatenate(bps)
    cand = np.unique(np.concatenate([[0.0], bps[(bps > 0) & (bps < t_max)]]))
    ends = list(cand) + ([t_max] if math.isfinite(t_max) else [cand[-1] * 2 + 1.0])
    for ta, tb in zip(ends[:-1], ends[1:]):
        ga, gb = _phi_prime(P, d, q, ta), _phi_prime(P, d, q, tb)
        if gb >= 0:
            return ta - ga * (tb - ta) / (gb - ga)
    if not math.isfinite(t_max):
        # root beyond the last breakpoint: phi' is linear there
        ta = ends[-1]
        ga, gb = _phi_prime(P, d, q, ta), _phi_prime(P, d, q, ta + 1.0)
        return ta - ga / (gb - ga)
    return t_max


@pytest.mark.parametrize("seed", range(8))
def test_line_search_against_breakpoint_sort(seed):
    ph = cached_phantom("mini")
    P = oracle_problem(ph)
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 0.05, P.n_blt)
    d = oracle.dose(P, x)
    u = oracle.grad_objective(P, d)
    # a descent direction in beamlet space
    dx = -oracle.prices(P, u) * rng.uniform(0.5, 1.5, P.n_blt)
    q = oracle.dose(P, dx)
    assert _phi_prime(P, d, q, 0.0) < 0
    t_max = math.inf if seed % 2 == 0 else float(rng.uniform(0.1, 2.0)) * 1e-3
    t, evals = oracle.line_search(P, d, q, t_max)
    ref = _brute_line_search(P, d, q, t_max)
    assert abs(t - ref) <= 1e-9 * max(abs(ref), 1e-300), (t, ref, evals)
    assert evals <= 20


def test_line_search_blocking_step():
    ph = cached_phantom("mini")
    P = oracle_problem(ph)
    rng = np.random.default_rng(11)
    d = oracle.dose(P, rng.uniform(0, 0.02, P.n_blt))
    q = oracle.dose(P, -oracle.prices(P, oracle.grad_objective(P, d)))
    t_free, _ = oracle.line_search(P, d, q, math.inf)
    t, _ = oracle.line_search(P, d, q, 0.5 * t_free)
    assert t == 0.5 * t_free


def _single_target_problem(ph):
    """Every voxel that any beamlet reaches is one target, T- = T+ = 0.3, alpha = beta."""
    reached = np.diff(ph.row_ptr) > 0
    vs = np.where(reached, 0, -1).astype(np.int16)
    pres = [dict(is_target=1, t_under=0.3, t_over=0.3, w_under=2.0, w_over=2.0)]
    return oracle.make_problem(ph.csr(), ph.rows_per_beam, ph.row_len, vs, pres), reached


def _pool(P, k, seed):
    rng = np.random.default_rng(seed)
    pool = []
    for _ in range(k):
        b = int(rng.integers(P.rows_per_beam.shape[0]))
        r0, r1 = P.beam_row_range(b)
        leaves = []
        for r in range(r0, r1):
            n = int(P.row_len[r])
            L = int(rng.integers(0, n))
            R = int(rng.integers(L + 1, n + 1))
            leaves.append((L, R))
        pool.append(oracle.Aperture(b, tuple(leaves)))
    return pool


def _dk(P, pool):
    cols = []
    for ap in pool:
        x = np.zeros(P.n_blt)
        x[ap.open_beamlets(P)] = 1.0
        cols.append(oracle.dose(P, x))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("conjugate", [True, False])
def test_master_matches_nnls_special_case(conjugate):
    ph = cached_phantom("mini")
    P, reached = _single_target_problem(ph)
    pool = _pool(P, 5, 0)
    st = MasterState.empty(P)
    for ap in pool:
        st.add(ap)
    log = solve_master(P, st, tol=1e-13, max_steps=20000, conjugate=conjugate)
    assert log["kkt"] <= 1e-13
    DK = _dk(P, pool)[reached]
    y_ref, _ = so.nnls(DK, np.full(DK.shape[0], 0.3), maxiter=10000)
    F_ref = 2.0 / reached.sum() * float(np.sum((DK @ y_ref - 0.3) ** 2))
    F = oracle.objective(P, st.d)
    assert abs(F - F_ref) <= 1e-9 * F_ref
    np.testing.assert_allclose(st.y, y_ref, rtol=1e-5, atol=1e-7)


@pytest.mark.parametrize("conjugate", [True, False])
@pytest.mark.parametrize("seed", [1, 2])
def test_master_matches_lbfgsb(seed, conjugate):
    ph = cached_phantom("mini")
    P = oracle_problem(ph)
    pool = _pool(P, 6, seed)
    st = MasterState.empty(P)
    for ap in pool:
        st.add(ap)
    log = solve_master(P, st, tol=1e-12, max_steps=50000, track_F=True, conjugate=conjugate)
    assert log["kkt"] <= 1e-12
    DK = sp.csr_matrix(_dk(P, pool))

    def fg(y):
        z = DK @ y
        return oracle.objective(P, z), DK.T @ oracle.grad_objective(P, z)

    r = so.minimize(fg, np.full(len(pool), 0.01), jac=True, method="L-BFGS-B",
                    bounds=[(0, None)] * len(pool),
                    options=dict(ftol=1e-16, gtol=1e-14, maxiter=20000, maxcor=30))
    F = oracle.objective(P, st.d)
    assert F <= r.fun * (1 + 1e-9)
    assert abs(F - r.fun) <= 1e-9 * r.fun
    pi = oracle.grad_objective(P, st.d)
    pi_ref = oracle.grad_objective(P, DK @ r.x)
    assert np.max(np.abs(pi - pi_ref)) <= 1e-6 * np.max(np.abs(pi_ref))
    # F never increases along the iteration
    Fs = np.array(log["F_trace"])
    assert np.all(np.diff(Fs) <= 1e-15 * Fs[0])
    # KKT at exit
    grad = oracle.aperture_gradient(P, pool, st.g)
    assert np.all(st.y >= 0)
    assert np.all(np.abs(grad[st.y > 0]) <= 1e-12)
    assert np.all(grad[st.y == 0] >= -1e-12)
    assert kkt_residual(st.y, grad) == log["kkt"]


def test_line_search_pure_quadratic_clamps_to_t_max():
    # every reached voxel in one target with T- = T+: phi is one quadratic with
    # no breakpoints, so the line search must stop at t_max when t_max is short
    ph = cached_phantom("mini")
    P, reached = _single_target_problem(ph)
    rng = np.random.default_rng(5)
    d = oracle.dose(P, rng.uniform(0, 0.01, P.n_blt))
    q = oracle.dose(P, -oracle.prices(P, oracle.grad_objective(P, d)))
    t_free, ev = oracle.line_search(P, d, q, math.inf)
    # exact minimiser of the quadratic: -phi'(0) / phi''
    g0 = _phi_prime(P, d, q, 0.0)
    curv = 2.0 * float(np.sum(q * q * P.a))      # one side active at a time, a = b
    assert abs(t_free - (-g0 / curv)) <= 1e-12 * t_free
    t, _ = oracle.line_search(P, d, q, 0.3 * t_free)
    assert t == 0.3 * t_free


@pytest.mark.parametrize("conjugate", [True, False])
def test_blocking_apertures_land_exactly_on_zero(conjugate):
    from oracle.master import master_step
    ph = cached_phantom("mini")
    P = oracle_problem(ph)
    blocked = 0
    for seed in range(6):
        st = MasterState.empty(P)
        for ap in _pool(P, 6, 100 + seed):
            st.add(ap)
        st.y = np.random.default_rng(seed).uniform(0.0, 0.05, 6)
        st.refresh(P)
        for _ in range(40):
            y_before = st.y.copy()
            rec = master_step(P, st, conjugate)
            if rec is None:
                break
            if rec["t"] == rec["t_max"]:
                was_pos = y_before > 0
                assert np.any(st.y[was_pos] == 0.0)
                # a block ends the conjugate sequence
                assert st.p_prev is None and st.r_prev is None
                blocked += 1
    assert blocked >= 3


def test_take_step_blocking_exactly_zero():
    from oracle.master import max_step, take_step
    rng = np.random.default_rng(3)
    residual_nonzero = 0
    for _ in range(2000):
        y = rng.uniform(0.0, 1.0, 4)
        p = rng.normal(size=4)
        if not np.any(p < 0):
            continue
        t = max_step(y, p)
        k = int(np.argmin(np.where(p < 0, y / np.where(p < 0, -p, 1.0), np.inf)))
        if y[k] + t * p[k] != 0.0:
            residual_nonzero += 1          # plain arithmetic would miss zero here
        out = take_step(y, p, t)
        assert out[k] == 0.0 and np.all(out >= 0.0)
        # a shorter step blocks nothing
        assert np.all(take_step(y, p, 0.5 * t) > 0.0)
    assert residual_nonzero > 0


def test_line_search_returns_t_max_inside_first_piece():
    # under-dose only (T- = 50) and a uniform direction: phi is one quadratic
    # up to t = 50, where every voxel reaches its threshold at once, so the
    # first Newton point is the exact minimiser; a shorter t_max must win
    ph = cached_phantom("mini")
    reached = np.diff(ph.row_ptr) > 0
    vs = np.where(reached, 0, -1).astype(np.int16)
    # alpha = |v| makes every per-voxel weight exactly 1, so all sums are exact
    pres = [dict(is_target=1, t_under=50.0, t_over=1e9, w_under=float(reached.sum()),
                 w_over=0.0)]
    P = oracle.make_problem(ph.csr(), ph.rows_per_beam, ph.row_len, vs, pres)
    assert np.all(P.a[reached] == 1.0)
    d = np.zeros(P.n_vox)
    q = reached.astype(float)
    t_free, ev = oracle.line_search(P, d, q, math.inf)
    assert ev == 1 and abs(t_free - 50.0) < 1e-12
    t, ev = oracle.line_search(P, d, q, 12.5)
    assert t == 12.5 and ev == 1


@pytest.mark.parametrize("seed", [0, 3, 5, 7, 10])
def test_conjugate_projection_terminates_on_a_face(seed):
    # F = c ||D_K y - T||^2 exactly (one target, T- = T+, alpha = beta) and a
    # pool whose NNLS optimum is strictly positive; started inside the
    # positive orthant near it, no step blocks, so the face never changes and
    # conjugate gradients with exact line searches reach the minimiser in K
    # steps.  Projected steepest descent from the same point does not.
    from oracle.master import master_step
    ph = cached_phantom("mini")
    P, reached = _single_target_problem(ph)
    K = 5
    pool = _pool(P, K, seed)
    DK = _dk(P, pool)[reached]
    y_ref, _ = so.nnls(DK, np.full(DK.shape[0], 0.3))
    assert np.min(y_ref) > 0
    res = {}
    for conjugate in (True, False):
        st = MasterState.empty(P)
        for ap in pool:
            st.add(ap)
        st.y = y_ref * np.random.default_rng(seed).uniform(0.5, 1.5, K)
        st.refresh(P)
        g0 = np.max(np.abs(oracle.aperture_gradient(P, pool, st.g)))
        for _ in range(K):
            rec = master_step(P, st, conjugate)
            assert rec is not None and rec["t"] < rec["t_max"]
        grad = oracle.aperture_gradient(P, pool, st.g)
        res[conjugate] = (kkt_residual(st.y, grad) / g0, np.max(np.abs(st.y - y_ref) / y_ref))
    assert res[True][0] <= 1e-10 and res[True][1] <= 1e-9, res
    assert res[False][0] >= 1e-4, res


def test_conjugate_direction_first_step_and_restart_rule():
    # the first step of a pool, and any step whose free set differs from the
    # last one's, move along the projected negative gradient r
    from oracle.master import direction
    ph = cached_phantom("mini")
    P = oracle_problem(ph)
    st = MasterState.empty(P)
    for ap in _pool(P, 4, 7):
        st.add(ap)
    st.y = np.array([0.0, 0.02, 0.01, 0.0])
    st.refresh(P)
    grad = np.array([1.0, -2.0, 0.5, -1.0])
    p, r, free = direction(st, grad)
    np.testing.assert_array_equal(free, [False, True, True, True])
    np.testing.assert_array_equal(p, [0.0, 2.0, -0.5, 1.0])
    np.testing.assert_array_equal(p, r)
    # same free set: r + beta p_prev with the truncated Polak-Ribiere beta
    st.p_prev, st.r_prev, st.free_prev = np.array([0.0, 1.0, 1.0, 1.0]), np.array([0.0, 1.0, -1.0, 1.0]), free
    p2, r2, _ = direction(st, grad)
    beta = (2 * (2 - 1) + (-0.5) * (-0.5 + 1) + 1 * (1 - 1)) / 3.0
    np.testing.assert_allclose(p2, r2 + beta * st.p_prev, rtol=0, atol=1e-15)
    # negative beta is truncated to 0
    st.r_prev = np.array([0.0, 4.0, 0.0, 0.0])
    p3, r3, _ = direction(st, grad)
    np.testing.assert_array_equal(p3, r3)
    # different free set: restart
    st.r_prev, st.free_prev = np.array([0.0, 1.0, -1.0, 1.0]), np.array([True, True, True, True])
    p4, r4, _ = direction(st, grad)
    np.testing.assert_array_equal(p4, r4)
    # plain projected steepest descent ignores the memory
    st.free_prev = free
    p5, r5, _ = direction(st, grad, conjugate=False)
    np.testing.assert_array_equal(p5, r5)
