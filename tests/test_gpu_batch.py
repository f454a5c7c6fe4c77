"""Several solves in one batched master launch per round (dao_solve_batch):
each plan is the one its solve gives alone.

The batched launch gives each solve only part of the grid, so its FP64
partial sums are grouped differently from the solo launch; decisions are
unchanged where they are not near-ties.  FP64 contexts: identical apertures
and F within 1e-9.  FP32 contexts: identical apertures and F within the FP32
bar 1e-5 on the phantoms and budgets used here.
"""
import numpy as np
import pytest

import paper_1003_5402_amd as dao
from gpu_util import ctx_for, torch_cuda
from phantom import make_phantom

pytestmark = pytest.mark.gpu


def _phantoms(specs):
    return [make_phantom(name, seed) for name, seed in specs]


def _alone(ph, dtype, n_ap):
    ctx = ctx_for(ph, dtype=dtype)
    try:
        out = ctx.solve(n_ap)
        pool, y = ctx.get_pool()
        return out, pool, y
    finally:
        ctx.close()


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-9), ("f32", 1e-5)])
def test_batch_equals_alone(dtype, tol):
    torch_cuda()
    specs = [("mini", 0), ("tiny", 0), ("tiny", 1)]
    budgets = [6, 8, 6]
    phs = _phantoms(specs)
    alone = [_alone(ph, dtype, n) for ph, n in zip(phs, budgets)]
    ctxs = [ctx_for(ph, dtype=dtype) for ph in phs]
    try:
        outs = dao.solve_batch(ctxs, budgets)
        for i, (out, ctx) in enumerate(zip(outs, ctxs)):
            ref, pool_ref, y_ref = alone[i]
            pool, y = ctx.get_pool()
            print(f"[batch] {specs[i]} rounds {out['rounds']} F {out['F']:.12e} alone {ref['F']:.12e}", flush=True)
            assert out["rounds"] == ref["rounds"] and out["stop"] == ref["stop"]
            assert pool == pool_ref, i
            assert abs(out["F"] - ref["F"]) <= tol * ref["F"], (i, out["F"], ref["F"])
            np.testing.assert_allclose(y, y_ref, rtol=100 * tol, atol=tol * max(1e-12, float(np.max(y_ref))))
    finally:
        for c in ctxs:
            c.close()


def test_batch_of_different_sizes_and_budgets_fp32():
    """A prostate-shaped solve beside two small ones, budgets that end at
    different rounds: every plan as alone."""
    torch_cuda()
    specs = [("prostate", 0), ("tiny", 2), ("mini", 1)]
    budgets = [6, 4, 3]
    phs = _phantoms(specs)
    alone = [_alone(ph, "f32", n) for ph, n in zip(phs, budgets)]
    ctxs = [ctx_for(ph, dtype="f32") for ph in phs]
    try:
        outs = dao.solve_batch(ctxs, budgets)
        for i, (out, ctx) in enumerate(zip(outs, ctxs)):
            ref, pool_ref, _ = alone[i]
            pool, _ = ctx.get_pool()
            assert pool == pool_ref, i
            assert abs(out["F"] - ref["F"]) <= 1e-5 * ref["F"], (i, out["F"], ref["F"])
            assert np.array_equal(out["round_beam"], ref["round_beam"])
    finally:
        for c in ctxs:
            c.close()


def test_batch_with_streamed_aperture_matrix_fp32():
    """A head-and-neck-shaped solve beside a prostate-shaped one: past a few
    apertures the head-and-neck D_K no longer fits on chip, so the batched
    launch takes the hybrid form (D_K streamed, each workgroup's rows of d,
    q and classes on chip, row batches dealt over its share of the grid);
    every plan as alone."""
    torch_cuda()
    specs = [("headneck", 0), ("prostate", 0)]
    budgets = [9, 9]   # equal budgets: every round, both solves share the launch
    phs = _phantoms(specs)
    alone = [_alone(ph, "f32", n) for ph, n in zip(phs, budgets)]
    ctxs = [ctx_for(ph, dtype="f32") for ph in phs]
    try:
        outs = dao.solve_batch(ctxs, budgets)
        forms = [c.info()["last_master_form"] for c in ctxs]
        print(f"[batch] head-and-neck + prostate: last forms {forms}", flush=True)
        assert forms == [6, 6]
        for i, (out, ctx) in enumerate(zip(outs, ctxs)):
            ref, pool_ref, _ = alone[i]
            pool, _ = ctx.get_pool()
            print(f"[batch] {specs[i]} F {out['F']:.12e} alone {ref['F']:.12e}", flush=True)
            assert pool == pool_ref, i
            assert abs(out["F"] - ref["F"]) <= 1e-5 * ref["F"], (i, out["F"], ref["F"])
    finally:
        for c in ctxs:
            c.close()


def test_batch_rejects_bad_arguments():
    torch_cuda()
    ph = make_phantom("mini", 0)
    a = ctx_for(ph, dtype="f64")
    b = ctx_for(ph, dtype="f32")
    try:
        with pytest.raises(dao.DaoError):
            dao.solve_batch([a, a], [2, 2])      # the same context twice
        with pytest.raises(dao.DaoError):
            dao.solve_batch([a, b], [2, 2])      # mixed dtypes
        with pytest.raises(dao.DaoError):
            dao.solve_batch([a], [10 ** 6])      # budget above max_apertures
    finally:
        a.close()
        b.close()
