"""GPU parity of the 16-bit storage of D: FP16 or BF16 values over a
per-beamlet FP32 scale, with or without the FP16 residual.

Two FP64 oracle references:
* the quantized matrix s_i (hi + lo) that the device multiplies with, built
  independently in tests/quant.py (numpy rounding).  The products must match
  it to the FP32 bar (1e-5 of the max norm), which checks the kernels, the
  scale handling and the residual path.
* the original D.  Per entry, the stored value is within 2^-12 (FP16) or
  2^-9 (BF16) of D_ij relative to its column maximum, and within ~2^-23 with
  the residual; with non-negative terms the max-norm error of a product is
  at most that bound.  The bars below are those bounds rounded up.
The converged master on the same pool is compared the same two ways, plus
the plan metrics PTV D95 and OAR Dmax against the FP64 master on the
original D.  The precision form of the head-and-neck-shaped plan (16-bit D
and an FP16 aperture dose matrix) is checked teacher-forced against the
oracle's stored trajectory: objective after every round, final dose, PTV D95
and organ Dmax within 1e-3.  The prostate-shaped plan, whose master keeps D_K
on chip, is checked the same way with an FP16 aperture dose matrix.
"""
import numpy as np
import pytest

import oracle
import paper_1003_5402_amd as dao
from conftest import cached_phantom, oracle_problem
from gpu_util import ctx_for, dev, relerr, torch_cuda
from oracle.master import MasterState, solve_master
from oracle.metrics import d95, dmax
from quant import quantized

pytestmark = pytest.mark.gpu

FMT = {"native": dao.DAO_DFMT_NATIVE, "f16": dao.DAO_DFMT_F16, "bf16": dao.DAO_DFMT_BF16}
FORMATS = [("f16", 0), ("f16", 1), ("bf16", 0), ("bf16", 1)]
# max-norm relative error against the original D
BOUND = {("f16", 0): 3e-4, ("bf16", 0): 2e-3, ("f16", 1): 1e-5, ("bf16", 1): 1e-5}


def _problems(ph, fmt, res):
    import oracle as o
    P = oracle_problem(ph)            # original D, FP64
    Dq = quantized(ph.csr(), fmt, res)
    Pq = o.make_problem(Dq, ph.rows_per_beam, ph.row_len, ph.vox_struct, ph.prescriptions)
    return P, Pq


@pytest.mark.parametrize("name", ["tiny", "prostate"])
@pytest.mark.parametrize("fmt,res", FORMATS)
def test_products_with_16bit_storage(name, fmt, res):
    torch = torch_cuda()
    ph = cached_phantom(name)
    P, Pq = _problems(ph, fmt, res)
    print(f"[precision] {name} {fmt} residual={res}", flush=True)
    ctx = ctx_for(ph, dtype="f32", d_format=FMT[fmt], d_residual=res)
    try:
        info = ctx.info()
        assert info["d_format"] == FMT[fmt] and info["d_residual"] == res
        rng = np.random.default_rng(11)
        for trial in range(2):
            x = rng.uniform(0.0, 0.05, ph.n_blt).astype(np.float32).astype(np.float64)
            d = torch.full((ph.n_vox,), float("nan"), dtype=torch.float32, device="cuda:0")
            ctx.dose(dev(x, torch.float32), d)
            torch.cuda.synchronize()
            got = d.double().cpu().numpy()
            assert relerr(got, oracle.dose(Pq, x)) <= 1e-5, trial
            assert relerr(got, oracle.dose(P, x)) <= BOUND[(fmt, res)], (trial, relerr(got, oracle.dose(P, x)))
            z = oracle.dose(P, x).astype(np.float32).astype(np.float64)
            g = torch.full((ph.n_blt,), float("nan"), dtype=torch.float32, device="cuda:0")
            F = ctx.gradient(dev(z, torch.float32), g)
            torch.cuda.synchronize()
            gg = g.double().cpu().numpy()
            assert relerr(gg, oracle.prices(Pq, oracle.grad_objective(Pq, z))) <= 1e-5, trial
            assert relerr(gg, oracle.prices(P, oracle.grad_objective(P, z))) <= BOUND[(fmt, res)], trial
            assert abs(F - oracle.objective(P, z)) <= 1e-12 * oracle.objective(P, z)
    finally:
        ctx.close()


@pytest.mark.parametrize("fmt,res", FORMATS)
def test_converged_master_with_16bit_storage(fmt, res):
    """Same pool (the oracle's first five apertures on the original D): the
    GPU master matches the FP64 master on the quantized D to the FP32 bars
    (F 1e-5, dose 1e-4) and the FP64 master on the original D to the format's
    bound (F, dose, PTV D95, OAR Dmax)."""
    torch = torch_cuda()
    ph = cached_phantom("tiny")
    P, Pq = _problems(ph, fmt, res)
    pool = oracle.solve(P, 5, eps=1e-4, max_steps=60)["pool"]
    refs = {}
    for key, PP in (("q", Pq), ("d", P)):
        st = MasterState.empty(PP)
        for ap in pool:
            st.add(ap)
        solve_master(PP, st, tol=1e-7, max_steps=20000)
        refs[key] = (oracle.objective(PP, st.d), st.d)
    ctx = ctx_for(ph, dtype="f32", d_format=FMT[fmt], d_residual=res)
    try:
        ctx.reset()
        for ap in pool:
            ctx.add_aperture(ap.beam, ap.leaves)
        steps, kkt, F = ctx.master_solve(1e-7, 20000)
        d = torch.empty(ph.n_vox, dtype=torch.float64, device="cuda:0")
        ctx.get_dose(d)
        z = d.cpu().numpy()
        Fq, zq = refs["q"]
        F0, z0 = refs["d"]
        assert abs(F - Fq) <= 1e-5 * Fq, (F, Fq)
        assert relerr(z, zq) <= 1e-4
        bound = max(BOUND[(fmt, res)], 1e-4)
        errs = dict(F=abs(F - F0) / F0, dose=relerr(z, z0))
        ptv = np.asarray(ph.vox_struct) == 0
        oar = np.asarray(ph.vox_struct) == 1
        errs["D95"] = abs(d95(z, ptv) - d95(z0, ptv)) / d95(z0, ptv)
        errs["Dmax"] = abs(dmax(z, oar) - dmax(z0, oar)) / dmax(z0, oar)
        print(f"[precision] {fmt} residual={res} errors vs FP64 on the original D: {errs}", flush=True)
        for k, v in errs.items():
            assert v <= 10 * bound, (k, v)
    finally:
        ctx.close()


def _golden(name):
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"{name}_seed0_r50.json")
    if not os.path.exists(path):
        pytest.skip(f"no stored trajectory {path}")
    with open(path) as f:
        return json.load(f)


# the precision form of the head-and-neck-shaped plan (streaming master):
# 16-bit D (with and without the FP16 residual) and an FP16 aperture dose
# matrix; the prostate-shaped plan's master keeps D_K on chip
PLAN_FORMATS = [("headneck", "f16", 0, 1), ("headneck", "f16", 1, 1), ("headneck", "bf16", 1, 1),
                ("headneck", "f16", 0, 0), ("prostate", "native", 0, 1), ("prostate", "f16", 0, 1)]


@pytest.mark.parametrize("name,fmt,res,dk16", PLAN_FORMATS)
def test_precision_plan_teacher_forced(name, fmt, res, dk16):
    """Teacher-forced against the FP64 oracle's stored 50-aperture trajectory
    (the oracle on the FP32 matrix): every round starts from the oracle's
    pool and intensities; the objective after the round's master and, at the
    end, the dose, PTV D95 and organ Dmax agree with the oracle's to 1e-3.
    Pricing decisions are compared where the gap exceeds the reduced-cost
    error of the format (1e-3 |rc|); closer ones are counted."""
    torch = torch_cuda()
    doc = _golden(name)
    ph = cached_phantom(name)
    rc1 = doc["rc1"]
    tol = doc["eps"] * abs(rc1)
    ctx = ctx_for(ph, dtype="f32", d_format=FMT[fmt], d_residual=res, dk_format=FMT["f16"] if dk16 else 0)
    worst_F, near = 0.0, 0
    try:
        for k, rec in enumerate(doc["rounds"]):
            pool = [(r["beam"], tuple(tuple(p) for p in r["leaves"])) for r in doc["rounds"][:k]]
            ctx.set_state(pool, doc["rounds"][k - 1]["y"] if k else [], rc1=rc1 if k else float("nan"),
                          eps=doc["eps"])
            got = ctx.price_current()
            if rec["gap"] > 1e-3 * abs(rec["rc"]):
                assert (got["beam"], got["leaves"]) == (rec["beam"], tuple(tuple(p) for p in rec["leaves"])), k
            else:
                near += 1
            ctx.add_aperture(rec["beam"], rec["leaves"])
            steps, kkt, F = ctx.master_solve(tol, doc["max_steps"])
            worst_F = max(worst_F, abs(F - rec["F"]) / rec["F"])
            assert abs(F - rec["F"]) <= 1e-3 * rec["F"], (k, F, rec["F"])
        # the last round's plan against the oracle's
        P = oracle_problem(ph, "f32")
        ap = [oracle.Aperture(r["beam"], tuple(tuple(p) for p in r["leaves"])) for r in doc["rounds"]]
        z0 = oracle.dose(P, oracle.beamlet_intensity(P, ap, doc["rounds"][-1]["y"]))
        d = torch.empty(ph.n_vox, dtype=torch.float64, device="cuda:0")
        ctx.get_dose(d)
        z = d.cpu().numpy()
        ptv = np.asarray(ph.vox_struct) == 0
        errs = dict(F=worst_F, dose=relerr(z, z0), D95=abs(d95(z, ptv) - d95(z0, ptv)) / d95(z0, ptv))
        for s, nm in enumerate(ph.struct_names):
            if s > 0:
                m = np.asarray(ph.vox_struct) == s
                errs[f"Dmax_{nm}"] = abs(dmax(z, m) - dmax(z0, m)) / dmax(z0, m)
        print(f"[precision] {name} {fmt} residual={res} dk16={dk16}: {errs}, near decisions {near}", flush=True)
        for key, v in errs.items():
            assert v <= 1e-3, (key, v)
    finally:
        ctx.close()


def test_selective_residual_plan():
    """d_residual 2 on the head-and-neck-shaped plan (FP16 D and D_K): the
    early rounds run on the 16-bit values, near-tie decisions are priced
    again with the residual, and the last rounds run with the residual and an
    FP32 D_K.  The final plan is then accurate to the FP32 bar: the GPU's
    dose and objective equal the FP64 oracle's dose D (A y) and F at the
    GPU's own final pool and intensities to 1e-5, and the objective is within
    1e-3 of the oracle's stored plan.  A second plan on the same context
    (which goes back to the FP16 D_K) repeats the first bit for bit."""
    torch = torch_cuda()
    doc = _golden("headneck")
    ph = cached_phantom("headneck")
    P = oracle_problem(ph, "f32")
    ctx = ctx_for(ph, dtype="f32", d_format=FMT["f16"], d_residual=2, dk_format=FMT["f16"], residual_rounds=5)
    try:
        assert ctx.info()["dk_format"] == FMT["f16"]
        out = ctx.solve(len(doc["rounds"]))
        info = ctx.info()
        assert out["rounds"] == len(doc["rounds"])
        assert info["dk_format"] == 0          # the final rounds switched D_K to FP32
        pool, y = ctx.get_pool()
        ap = [oracle.Aperture(b, lv) for b, lv in pool]
        z0 = oracle.dose(P, oracle.beamlet_intensity(P, ap, y))
        d = torch.empty(ph.n_vox, dtype=torch.float64, device="cuda:0")
        F = ctx.get_dose(d)
        z = d.cpu().numpy()
        F0 = oracle.objective(P, z0)
        print(f"[precision] selective residual: reprices {info['residual_reprices']}, F {F:.10e} "
              f"oracle at the same y {F0:.10e}, stored plan {doc['F']:.10e}, dose err {relerr(z, z0):.2e}",
              flush=True)
        assert relerr(z, z0) <= 1e-5
        assert abs(F - F0) <= 1e-5 * F0
        assert abs(F - doc["F"]) <= 1e-3 * doc["F"]
        again = ctx.solve(len(doc["rounds"]))
        print(f"[precision] selective residual, second plan: F {again['F']:.10e}", flush=True)
        assert again["rounds"] == out["rounds"] and again["F"] == out["F"]
        assert list(again["round_beam"]) == list(out["round_beam"])
        pool2, y2 = ctx.get_pool()
        assert pool2 == pool and np.array_equal(np.asarray(y2), np.asarray(y))
    finally:
        ctx.close()


@pytest.mark.parametrize("name,expect", [("headneck", "f16"), ("prostate", "native")])
def test_automatic_dk_storage(name, expect):
    """dk_format = DAO_DFMT_AUTO: a plan starts with D_K in FP32 and moves it
    to FP16 once the pool outgrows the master's on-chip form.  The
    head-and-neck-shaped matrix does so after a few apertures, and its plan
    stays within the FP16 bar (1e-3) of the FP32 plan; the prostate-shaped
    one stays on chip in FP32, so its plan equals the FP32 plan bit for bit.
    A second plan on the same context (back to FP32 storage, the buffer
    cleared) repeats the first bit for bit."""
    ph = cached_phantom(name)
    n = 12
    auto = ctx_for(ph, dtype="f32", dk_format=dao.DAO_DFMT_AUTO)
    ref = ctx_for(ph, dtype="f32")
    try:
        assert auto.info()["dk_format"] == FMT["native"]
        a, b = auto.solve(n), ref.solve(n)
        got = auto.info()["dk_format"]
        print(f"[precision] {name} auto D_K: {got}, F {a['F']:.12e} FP32 {b['F']:.12e}", flush=True)
        assert got == FMT[expect] and a["rounds"] == b["rounds"] == n
        if expect == "native":
            assert a["F"] == b["F"] and list(a["round_beam"]) == list(b["round_beam"])
            assert list(a["round_steps"]) == list(b["round_steps"])
        else:
            assert abs(a["F"] - b["F"]) <= 1e-3 * b["F"]
        again = auto.solve(n)
        assert again["F"] == a["F"] and list(again["round_beam"]) == list(a["round_beam"])
    finally:
        auto.close()
        ref.close()
