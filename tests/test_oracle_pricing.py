"""Pins for the pricing oracle (eq. 8 and the row scan of Section 2.3).

* A prefix-sum formulation of the row minimum (interval sum = difference of
  two prefix sums; exact rational arithmetic) must give the same leaves and
  value as the oracle's enumeration on random rows, on integer rows with
  constructed exact ties and on all-non-negative rows.
* Brute force over every deliverable aperture of small beams
  ((n(n+1)/2 + 1)^rows apertures) must reach the same beam value, and the
  same aperture when the minimum is unique.
* Closed form of the first round: at zero dose every price is <= 0, so each
  row opens from its first position to just past its last negative beamlet,
  and the chosen beam is the one with the largest PTV dose per unit fluence.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from conftest import cached_phantom, oracle_problem
from oracle.aperture import Aperture


def prefix_row_min(w):
    """Minimum-sum interval of a row from prefix sums, in exact rational
    arithmetic.  With P[0] = 0 and P[k] = w_0 + ... + w_{k-1}, the interval
    [l, r) sums to P[r] - P[l]; for each right end r the best interval ends
    there and starts at the earliest l < r with the largest P[l]; over right
    ends in increasing order only a strictly smaller value replaces the best,
    which starts at 0 with the row closed.  Independent of the oracle's
    enumeration (no interval sums are formed one by one)."""
    from fractions import Fraction
    P = [Fraction(0)]
    for v in w:
        P.append(P[-1] + Fraction(float(v)))
    best, L, R = Fraction(0), 0, 0
    for r in range(1, len(w) + 1):
        lmax = max(range(r), key=lambda l: (P[l], -l))
        if P[r] - P[lmax] < best:
            best, L, R = P[r] - P[lmax], lmax, r
    return L, R, float(best)


def _rows(rng):
    for n in range(1, 13):
        for _ in range(30):
            yield rng.normal(size=n)
            yield rng.integers(-3, 4, size=n).astype(float)       # many exact ties
            yield rng.integers(0, 4, size=n).astype(float)        # never negative
            yield -rng.integers(0, 2, size=n).astype(float)       # zero / negative runs


def test_scan_equals_enumeration():
    rng = np.random.default_rng(0)
    for w in _rows(rng):
        L, R, best, second = oracle.price_row(w)
        l2, r2, v2 = prefix_row_min(list(w))
        if R == L:
            assert (l2, r2) in [(0, 0)] and v2 == 0.0
        else:
            assert (L, R) == (l2, r2), (w, (L, R), (l2, r2))
        assert abs(best - v2) <= 1e-12 * (1 + np.abs(w).sum())
        assert second >= best


def test_row_gap_and_closed_row():
    # all non-negative: closed, gap = smallest single entry
    L, R, best, second = oracle.price_row([3.0, 1.0, 2.0])
    assert (L, R, best, second) == (0, 0, 0.0, 1.0)
    # unique best [1, 3) = -5; runner-up [1, 2) = -4
    L, R, best, second = oracle.price_row([1.0, -4.0, -1.0, 2.0])
    assert (L, R, best, second) == (1, 3, -5.0, -4.0)
    # tie: [0, 1) and [2, 3) both -2 -> smallest right end wins, gap 0
    L, R, best, second = oracle.price_row([-2.0, 3.0, -2.0])
    assert (L, R, best, second) == (0, 1, -2.0, -2.0)
    # leading zeros are included (earliest maximal prefix), trailing excluded
    L, R, best, _ = oracle.price_row([0.0, 0.0, -1.0, -2.0, 0.0])
    assert (L, R, best) == (0, 4, -3.0)


def _tiny_problem(rows, n, seed, integer):
    rng = np.random.default_rng(seed)
    N = rows * n * 2
    import scipy.sparse as sp
    D = sp.csr_matrix((1, N))
    P = oracle.make_problem(D, [rows, rows], [n] * (2 * rows), np.array([-1]), [])
    g = rng.integers(-4, 4, size=N).astype(float) if integer else rng.normal(size=N)
    return P, g


def _brute_force(P, g):
    starts = P.row_start()
    best = (math.inf, None)
    values = []
    for b in range(P.rows_per_beam.shape[0]):
        r0, r1 = P.beam_row_range(b)
        choices = []
        for r in range(r0, r1):
            n = int(P.row_len[r])
            choices.append([(0, 0)] + [(l, rr) for rr in range(1, n + 1) for l in range(rr)])
        for leaves in itertools.product(*choices):
            ap = Aperture(b, tuple(leaves))
            v = math.fsum(g[ap.open_beamlets(P)].tolist())
            values.append((v, ap))
            if v < best[0]:
                best = (v, ap)
    return best, values


@pytest.mark.parametrize("rows,n,seed,integer", [(3, 4, 0, False), (3, 4, 1, True),
                                                 (4, 5, 2, False), (2, 5, 3, True)])
def test_pricing_equals_brute_force(rows, n, seed, integer):
    P, g = _tiny_problem(rows, n, seed, integer)
    res = oracle.price(P, g)
    (bv, bap), values = _brute_force(P, g)
    expect_count = 2 * (n * (n + 1) // 2 + 1) ** rows
    assert len(values) == expect_count
    assert abs(res["rc"] - bv) <= 1e-12 * (1 + np.abs(g).sum())
    minima = [ap for v, ap in values if v == bv]
    if len(minima) == 1:
        assert res["aperture"] == bap
        assert res["gap"] > 0
    else:
        assert res["aperture"] in minima
        assert res["gap"] == 0.0
    # the oracle's gap is a true lower bound on how far any other aperture is
    others = sorted(v for v, ap in values if ap != res["aperture"])
    assert others[0] - res["rc"] >= res["gap"] - 1e-12


def test_first_round_closed_form():
    ph = cached_phantom("tiny")
    P = oracle_problem(ph)
    u0 = oracle.grad_objective(P, np.zeros(P.n_vox))
    w = oracle.prices(P, u0)
    assert np.all(w <= 0.0)
    ptv = ph.structure_mask("PTV")
    ptv_dose = np.asarray(ph.csr()[ptv].sum(axis=0)).ravel()   # sum_{j in PTV} D_ij
    res = oracle.price(P, w)
    starts = P.row_start()
    # beam with the largest total PTV dose per unit fluence over its
    # negative-priced beamlets
    totals = [ptv_dose[ph.beamlet_beam == b].sum() for b in range(ph.n_beams)]
    assert res["aperture"].beam == int(np.argmax(totals))
    r0, r1 = P.beam_row_range(res["aperture"].beam)
    for r, (L, R) in zip(range(r0, r1), res["aperture"].leaves):
        wr = w[starts[r]:starts[r] + P.row_len[r]]
        neg = np.flatnonzero(wr < 0)
        if neg.size == 0:
            assert (L, R) == (0, 0)
        else:
            assert (L, R) == (0, int(neg.max()) + 1)
    n_ptv = int(ptv.sum())
    assert abs(res["rc"] - (-2.0 / n_ptv) * max(totals)) <= 1e-12 * abs(res["rc"])


def test_beam_tie_goes_to_lowest_index():
    # both beams see the same prices: equal values, beam 0 wins, gap 0
    P, g = _tiny_problem(3, 4, 5, False)
    half = g.shape[0] // 2
    g[half:] = g[:half]
    res = oracle.price(P, g)
    assert res["beam_values"][0] == res["beam_values"][1]
    assert res["aperture"].beam == 0 and res["gap"] == 0.0
    # make beam 1 strictly better by one unit on an open beamlet of its best row
    g2 = g.copy()
    g2[half + int(np.argmin(g[:half]))] -= 1.0
    assert oracle.price(P, g2)["aperture"].beam == 1
