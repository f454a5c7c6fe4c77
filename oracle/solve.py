"""Column-generation loop (Section 2.2 and Section 2.3) -- test infrastructure.

Each round solves the pricing sub-problem at the current dual multipliers
(pi = grad F at the master's dose), and the aperture it returns enters the
pool with intensity 0; the master is then re-solved over the enlarged pool
(Section 2.3: one aperture is added per iteration).  The paper fixes the
number of apertures at 50 for its timings (Section 3); the flowchart that
would give the exact loop order is missing from the text, so this reading is
used:

* round 1 prices at y = 0 (zero dose);  rc_1 is its reduced cost;
* a round stops the loop when the best reduced cost is >= -tau,
  tau = tau_rel * |rc_1| (no improving aperture: the current plan is optimal);
* if pricing returns an aperture already in the pool, the master was not
  solved tightly enough: its tolerance is divided by 10 (at most
  ``max_tighten`` times over the solve), the master is re-solved and the
  round is priced again; after that the loop stops;
* otherwise the aperture enters and the master runs to KKT residual
  <= eps * |rc_1| (or ``max_steps`` steps), by conjugate gradient projection
  unless ``conjugate=False`` (see :mod:`oracle.master`);
* the loop ends when the pool holds ``n_apertures`` apertures.

With ``per_round = m > 1`` (a variant: several apertures per round), after
the entering aperture the beams ranked 2..m by value (ties to the lowest
index) add their own best apertures too, each only if its value is below
-tau, it is not already pooled and the budget allows; then the master runs
once over the enlarged pool.
"""
from __future__ import annotations

from typing import Callable, Dict, List, Optional

import numpy as np

from .master import MasterState, solve_master
from .model import Problem, objective
from .pricing import price, ranked_apertures


def solve(P: Problem, n_apertures: int, eps: float = 1e-6, max_steps: int = 500,
          tau_rel: float = 1e-10, max_tighten: int = 3, track_F: bool = False,
          conjugate: bool = True, per_round: int = 1, on_round: Optional[Callable[[int, Dict, MasterState], None]] = None) -> Dict:
    st = MasterState.empty(P)
    log: List[Dict] = []
    rc1 = None
    tighten = 0
    status = "budget"
    while len(st.pool) < n_apertures:
        pr = price(P, st.g)
        if rc1 is None:
            rc1 = pr["rc"]
            if rc1 >= 0.0:
                status = "optimal"
                break
        scale = abs(rc1)
        if pr["rc"] >= -tau_rel * scale:
            status = "optimal"
            break
        if pr["aperture"] in st.pool:
            if tighten >= max_tighten:
                status = "stalled"
                break
            tighten += 1
            eps /= 10.0
            solve_master(P, st, eps * scale, max_steps, conjugate=conjugate)
            continue
        st.add(pr["aperture"])
        extra = []
        if per_round > 1:
            for v, ap in ranked_apertures(P, pr)[1:per_round]:
                if len(st.pool) >= n_apertures or not v < -tau_rel * scale:
                    break
                if ap in st.pool:
                    continue
                st.add(ap)
                extra.append(ap)
        mlog = solve_master(P, st, eps * scale, max_steps, track_F=track_F, conjugate=conjugate)
        rec = dict(round=len(st.pool), beam=pr["aperture"].beam, rc=pr["rc"], gap=pr["gap"], extra=extra,
                   steps=mlog["steps"], ls_evals=mlog["ls_evals"], kkt=mlog["kkt"],
                   F=objective(P, st.d), F_trace=mlog["F_trace"])
        log.append(rec)
        if on_round is not None:
            on_round(len(st.pool), pr, st)
    return dict(pool=list(st.pool), y=st.y.copy(), d=st.d.copy(), F=objective(P, st.d),
                rc1=rc1, status=status, log=log, eps=eps, state=st)
