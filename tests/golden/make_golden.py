"""Writes the oracle's column-generation trajectories used as parity fixtures.

Calls only ``oracle/`` (and the seeded phantom generator for its inputs), so
every stored value is the FP64 oracle's.  For phantoms whose dose matrix is
stored in FP32 the oracle solves the problem with D rounded to FP32 (exact in
FP64), which is the problem an FP32 context holds.  For each phantom it records, per
round: the entering aperture (beam, leaves), its reduced cost, the decision
gap, the master's step count, line-search evaluations, KKT residual at exit,
whether the master stopped at the step cap, the objective after the master
and the pool intensities y after the master.  The final dose is not stored:
it is D (A y) of the last round's pool and intensities, which the tests
recompute with the oracle.

Usage::

    python tests/golden/make_golden.py prostate 50      # all 50 rounds
    python tests/golden/make_golden.py headneck 10      # first 10 rounds

The solve parameters are the library defaults (KKT tolerance 1e-6 |rc_1|,
500 master steps per round, entry threshold 1e-10 |rc_1|, three tightenings,
conjugate gradient projection).
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from phantom import make_phantom  # noqa: E402

EPS, MAX_STEPS, TAU_REL, MAX_TIGHTEN = 1e-6, 500, 1e-10, 3


def golden_path(name: str, seed: int, rounds: int) -> str:
    return os.path.join(HERE, f"{name}_seed{seed}_r{rounds}.json")


def main(name: str, rounds: int, seed: int = 0) -> str:
    ph = make_phantom(name, seed)
    D = ph.csr()
    if ph.dtype == "f32":
        # an FP32 context stores D rounded to FP32; the oracle solves that
        # same problem (the rounded values are exact in FP64)
        D = D.copy()
        D.data = D.data.astype(np.float32).astype(np.float64)
    P = oracle.make_problem(D, ph.rows_per_beam, ph.row_len, ph.vox_struct, ph.prescriptions)
    recs = []
    t0 = time.perf_counter()

    def on_round(k, pr, st):
        recs.append(dict(y=[float(v) for v in st.y]))
        print(f"[golden] {name} round {k} rc={pr['rc']:.6e} gap={pr['gap']:.3e} "
              f"t={time.perf_counter() - t0:.0f}s", flush=True)

    res = oracle.solve(P, rounds, eps=EPS, max_steps=MAX_STEPS, tau_rel=TAU_REL,
                       max_tighten=MAX_TIGHTEN, on_round=on_round)
    out_rounds = []
    for rec, extra, ap in zip(res["log"], recs, res["pool"]):
        out_rounds.append(dict(round=rec["round"], beam=ap.beam, leaves=[list(p) for p in ap.leaves],
                               rc=rec["rc"], gap=rec["gap"], F=rec["F"], steps=rec["steps"],
                               ls_evals=rec["ls_evals"], kkt=rec["kkt"],
                               capped=bool(rec["steps"] >= MAX_STEPS), y=extra["y"]))
    ptv = ph.vox_struct == 0
    metrics = dict(ptv_d95=oracle.d95(res["d"], ptv))
    for s, nm in enumerate(ph.struct_names):
        if s > 0:
            metrics[f"dmax_{nm}"] = oracle.dmax(res["d"], ph.vox_struct == s)
    doc = dict(phantom=name, seed=seed, n_vox=ph.n_vox, n_blt=ph.n_blt, nnz=ph.nnz,
               d_dtype=ph.dtype, direction="conjugate", eps=EPS, max_steps=MAX_STEPS, tau_rel=TAU_REL,
               max_tighten=MAX_TIGHTEN, rounds_requested=rounds, status=res["status"],
               rc1=res["rc1"], F=res["F"], final_eps=res["eps"], metrics=metrics,
               dose_sum=math.fsum(res["d"].tolist()), dose_max=float(np.max(res["d"])),
               oracle_seconds=time.perf_counter() - t0, rounds=out_rounds)
    path = golden_path(name, seed, rounds)
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"[golden] wrote {path} F={res['F']:.10e} status={res['status']}", flush=True)
    return path


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]), int(sys.argv[3]) if len(sys.argv) > 3 else 0)
