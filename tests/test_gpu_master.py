"""GPU parity of the restricted master and the column-generation loop.

* Step by step: the same pool, from y = 0, one gradient-projection step at a
  time on both sides (conjugate and steepest directions); objective, KKT
  residual and step length compared after every step (FP64: 1e-9 relative
  after up to 30 steps; FP32: 1e-5) until the KKT residual falls to 1e-7
  (FP64) or 1e-3 (FP32) of its first value, where the gradient is rounding
  noise and the next direction is arbitrary on both sides.
* Converged master: same pool, tight tolerance: objective, intensities and
  dose against the oracle.
* Free-running solve in FP64 (32^3 phantom, 10 apertures): the same aperture
  in every round whose decision gap exceeds 1e-9, and the final dose within
  1e-9 relative.
* Teacher-forced rounds in FP32 at the prostate-shaped size: the GPU prices
  on its own master point; wherever the oracle's gap exceeds the FP32
  decision bound the leaves must agree; the oracle's aperture is then added
  on both sides so the trajectories stay in lockstep.
"""
import math

import numpy as np
import pytest

import oracle
from conftest import cached_phantom, oracle_problem
from gpu_util import ctx_for, relerr, torch_cuda
from oracle.master import MasterState, kkt_residual, master_step, solve_master

pytestmark = pytest.mark.gpu

# the ways the master can run: aperture dose matrix as one persistent
# cooperative launch per solve (rows held in LDS, or streamed from device
# memory), aperture dose matrix with one launch per phase, beamlet matrix
# with the pool map
MASTER_OPTS = {"ap-persistent": dict(master=0, persistent=2), "ap-stream": dict(master=0, persistent=1),
               "ap-launches": dict(master=0, persistent=0),
               "beamlet": dict(master=1)}
MASTERS = pytest.mark.parametrize("master", list(MASTER_OPTS))


def _oracle_pool(P, n, seed=0):
    """First n apertures of an oracle solve (a realistic pool)."""
    res = oracle.solve(P, n, eps=1e-4, max_steps=60)
    return res["pool"]


@MASTERS
@pytest.mark.parametrize("direction", [1, 0], ids=["conjugate", "steepest"])
@pytest.mark.parametrize("name,dtype,steps,tol", [("mini", "f64", 30, 1e-9), ("tiny", "f64", 20, 1e-9),
                                                   ("tiny", "f32", 10, 1e-5)])
def test_master_steps_parity(name, dtype, steps, tol, master, direction):
    ph = cached_phantom(name)
    P = oracle_problem(ph, dtype)
    pool = _oracle_pool(P, 4)
    ctx = ctx_for(ph, dtype=dtype, direction=direction, **MASTER_OPTS[master])
    try:
        ctx.reset()
        st = MasterState.empty(P)
        for ap in pool:
            ctx.add_aperture(ap.beam, ap.leaves)
            st.add(ap)
        # once the KKT residual is down to the rounding level of the
        # gradient, the next direction is rounding noise on both sides
        kr = kr0 = kkt_residual(st.y, oracle.aperture_gradient(P, st.pool, st.g))
        floor = (1e-7 if dtype == "f64" else 1e-3) * kr0
        for s in range(steps):
            if kr <= floor:
                break
            print(f"[step] {name} {dtype} {s} kkt {kr:.3e}", flush=True)
            F, kkt, t = ctx.master_step()
            rec = master_step(P, st, conjugate=bool(direction))
            if rec is None:
                assert t == 0.0
                break
            Fr = oracle.objective(P, st.d)
            kr = kkt_residual(st.y, oracle.aperture_gradient(P, st.pool, st.g))
            assert abs(F - Fr) <= tol * Fr, (s, F, Fr)
            assert abs(t - rec["t"]) <= tol * 10 * rec["t"], (s, t, rec["t"])
            assert abs(kkt - kr) <= tol * 100 * max(kr, 1e-3 * abs(F)), (s, kkt, kr)
        _, y = ctx.get_pool()
        np.testing.assert_allclose(y, st.y, rtol=tol * 100, atol=tol * 1e-3)
    finally:
        ctx.close()


@MASTERS
@pytest.mark.parametrize("name,dtype,tol", [("mini", "f64", 1e-9), ("tiny", "f64", 1e-9), ("tiny", "f32", 1e-5)])
def test_master_converged_parity(name, dtype, tol, master):
    torch = torch_cuda()
    ph = cached_phantom(name)
    P = oracle_problem(ph, dtype)
    pool = _oracle_pool(P, 5)
    st = MasterState.empty(P)
    for ap in pool:
        st.add(ap)
    ktol = 1e-9 if dtype == "f64" else 1e-6
    log = solve_master(P, st, tol=ktol, max_steps=20000)
    ctx = ctx_for(ph, dtype=dtype, **MASTER_OPTS[master])
    try:
        ctx.reset()
        for ap in pool:
            ctx.add_aperture(ap.beam, ap.leaves)
        steps, kkt, F = ctx.master_solve(ktol, 20000)
        Fr = oracle.objective(P, st.d)
        assert abs(F - Fr) <= tol * Fr, (F, Fr, steps, log["steps"])
        d = torch.empty(ph.n_vox, dtype=torch.float64, device="cuda:0")
        F2 = ctx.get_dose(d)
        assert F2 == F
        assert relerr(d.cpu().numpy(), st.d) <= (1e-8 if dtype == "f64" else 1e-4)
        if dtype == "f64":
            assert kkt <= ktol and steps == log["steps"]
    finally:
        ctx.close()


_TINY_REF = {}


@MASTERS
def test_solve_tiny_f64_free_running(master):
    torch = torch_cuda()
    ph = cached_phantom("tiny")
    P = oracle_problem(ph)
    if "ref" not in _TINY_REF:
        _TINY_REF["ref"] = oracle.solve(P, ph.n_apertures, eps=1e-6)
    ref = _TINY_REF["ref"]
    ctx = ctx_for(ph, dtype="f64", **MASTER_OPTS[master])
    try:
        out = ctx.solve(ph.n_apertures)
        pool, y = ctx.get_pool()
        assert out["rounds"] == len(ref["log"])
        for k, (rec, ap) in enumerate(zip(ref["log"], ref["pool"])):
            print(f"[round] {k} gap={rec['gap']:.3e} steps gpu={out['round_steps'][k]} cpu={rec['steps']}",
                  flush=True)
            if rec["gap"] > 1e-9:
                assert pool[k] == (ap.beam, ap.leaves), k
            assert abs(out["round_rc"][k] - rec["rc"]) <= 1e-9 * abs(rec["rc"])
            assert abs(out["round_F"][k] - rec["F"]) <= 1e-9 * rec["F"]
        d = torch.empty(ph.n_vox, dtype=torch.float64, device="cuda:0")
        F = ctx.get_dose(d)
        assert abs(F - ref["F"]) <= 1e-9 * ref["F"]
        assert relerr(d.cpu().numpy(), ref["d"]) <= 1e-8
        np.testing.assert_allclose(y, ref["y"], rtol=1e-6, atol=1e-9)
    finally:
        ctx.close()


@MASTERS
def test_prostate_f32_teacher_forced_rounds(master):
    ph = cached_phantom("prostate")
    P = oracle_problem(ph)
    ctx = ctx_for(ph, dtype="f32", **MASTER_OPTS[master])
    rounds = 3
    try:
        ctx.reset()
        st = MasterState.empty(P)
        rc1 = None
        for k in range(rounds):
            ref = oracle.price(P, st.g)
            got = ctx.price_current()
            rc1 = rc1 if rc1 is not None else ref["rc"]
            # FP32 decision bound: the GPU's master point differs from the
            # oracle's by the FP32 rounding of its products
            bound = max(1e-9, 1e-5 * abs(ref["rc"]))
            print(f"[round] {k} rc={ref['rc']:.6e} gap={ref['gap']:.3e} bound={bound:.1e}", flush=True)
            if ref["gap"] > bound:
                assert (got["beam"], got["leaves"]) == (ref["aperture"].beam, ref["aperture"].leaves)
            assert abs(got["rc"] - ref["rc"]) <= 1e-5 * abs(ref["rc"])
            ap = ref["aperture"]
            st.add(ap)
            ctx.add_aperture(ap.beam, ap.leaves)
            tol = 1e-6 * abs(rc1)
            log = solve_master(P, st, tol=tol, max_steps=80)
            steps, kkt, F = ctx.master_solve(tol, 80)
            Fr = oracle.objective(P, st.d)
            print(f"[round] {k} F gpu={F:.10e} cpu={Fr:.10e} steps {steps}/{log['steps']}", flush=True)
            assert abs(F - Fr) <= 1e-5 * Fr
    finally:
        ctx.close()


def test_prostate_plan_runs_on_chip():
    """At the benchmark's size (prostate-shaped phantom, FP32, pool of 50) every
    workgroup's rows fit in LDS, so the persistent master takes the on-chip form."""
    ph = cached_phantom("prostate")
    ctx = ctx_for(ph, dtype="f32", max_apertures=64)
    try:
        inf = ctx.info()
        if inf["onchip_lds_bytes"] == 0:
            pytest.fail("the on-chip form is unavailable on this device")
        out = ctx.solve(ph.n_apertures)
        assert out["rounds"] >= 1
        assert ctx.info()["last_master_form"] == 2
    finally:
        ctx.close()
