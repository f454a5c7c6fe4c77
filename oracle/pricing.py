"""Pricing sub-problem (eq. 8, Section 2.3) by direct enumeration (test infrastructure).

For beam b the sub-problem asks for the deliverable aperture of b that
minimises sum_{i in A_k} w_i.  Under the consecutiveness constraint the rows
are independent, so each MLC row picks the contiguous run of beamlets with
the smallest sum, or stays closed (sum 0) when no run is negative; the
aperture's value is the sum over its rows, and the beam with the smallest
value supplies the new aperture (Section 2.3).

The paper solves each row with a single left-to-right scan.  The oracle uses
the plain definition instead -- every interval is enumerated and summed
exactly -- and adopts the scan's tie rule so that both agree on which of
several equal intervals is chosen:
* the scan replaces its best only on a strictly smaller value, visiting right
  ends in increasing order, so among equal sums the smallest right end wins;
* for a fixed right end it measures from the earliest maximal prefix (strict
  improvement of the running maximum), so the earliest left end wins;
* the best value starts at 0 with the row closed, so a row without a negative
  interval stays closed.
Beams with equal values go to the lowest beam index.

Several apertures per round (a variant of the loop): the beams ranked by
value (ties to the lowest index) each supply their own best aperture, so the
m best beams give m apertures, the first being the usual entering one.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

from .aperture import Aperture
from .model import Problem


def price_row(w) -> Tuple[int, int, float, float]:
    """Best leaf interval of one row.

    Returns ``(L, R, best, second)``: the chosen half-open interval [L, R)
    (``(0, 0)`` when closed), its exact sum, and the smallest sum among all
    other candidates (the closed row counts as a candidate of value 0).
    ``second - best`` is the row's decision gap.
    """
    w = [float(v) for v in w]
    n = len(w)
    best, L, R = 0.0, 0, 0
    cands = [(0.0, 0, 0)]
    for r in range(1, n + 1):           # right end, increasing
        for l in range(0, r):           # left end, increasing
            s = math.fsum(w[l:r])
            cands.append((s, l, r))
            if s < best:
                best, L, R = s, l, r
    second = min((c[0] for c in cands if (c[1], c[2]) != (L, R)), default=math.inf)
    return L, R, best, second


def price(P: Problem, g: np.ndarray) -> Dict:
    """Solve the sub-problem for every beam and pick the entering aperture.

    Returns a dict with the chosen ``aperture``, its reduced cost ``rc``
    (the beam value), the per-beam values, and the decision ``gap``: the
    smaller of (second-best beam value - best beam value) and the smallest
    row gap among the chosen beam's rows.
    """
    g = np.asarray(g, dtype=np.float64)
    starts = P.row_start()
    row_res = []
    for r, n in enumerate(P.row_len):
        row_res.append(price_row(g[starts[r]:starts[r] + n]))
    beam_vals = []
    for b in range(P.rows_per_beam.shape[0]):
        r0, r1 = P.beam_row_range(b)
        beam_vals.append(math.fsum(row_res[r][2] for r in range(r0, r1)))
    best_b = 0
    for b in range(1, len(beam_vals)):
        if beam_vals[b] < beam_vals[best_b]:
            best_b = b
    r0, r1 = P.beam_row_range(best_b)
    leaves = tuple((row_res[r][0], row_res[r][1]) for r in range(r0, r1))
    others = [v for b, v in enumerate(beam_vals) if b != best_b]
    beam_gap = (min(others) - beam_vals[best_b]) if others else math.inf
    row_gap = min((row_res[r][3] - row_res[r][2] for r in range(r0, r1)), default=math.inf)
    return dict(aperture=Aperture(best_b, leaves), rc=beam_vals[best_b],
                beam_values=beam_vals, gap=min(beam_gap, row_gap),
                rows=row_res)


def ranked_apertures(P: Problem, pr: Dict) -> List[Tuple[float, Aperture]]:
    """Every beam's best aperture with its value, from a :func:`price`
    result, ordered by value and then beam index."""
    out = []
    for b in range(P.rows_per_beam.shape[0]):
        r0, r1 = P.beam_row_range(b)
        leaves = tuple((pr["rows"][r][0], pr["rows"][r][1]) for r in range(r0, r1))
        out.append((pr["beam_values"][b], b, Aperture(b, leaves)))
    out.sort(key=lambda t: (t[0], t[1]))
    return [(v, ap) for v, _, ap in out]
