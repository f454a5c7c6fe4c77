"""dao_price_noalloc (the pricing call that allocates nothing) against dao_price.

Both take the same prices; the allocation-free call keeps its launch's
scratch in the library's static device array.  Two calls in a row on one
device share that array, the second with a smaller input (fewer MLC rows, a
different context), and each must return exactly what dao_price returns:
leaves and beam identical, reduced cost and gap bit for bit (same kernel,
same order of sums).  A context with more rows than the array holds is
refused with DAO_EINVAL.
"""
import numpy as np
import pytest

import oracle
import paper_1003_5402_amd as dao
from conftest import cached_phantom, oracle_problem
from gpu_util import ctx_for, torch_cuda

pytestmark = pytest.mark.gpu


def _prices(ph, seed):
    """Oracle prices at a random fluence (a realistic sign pattern)."""
    P = oracle_problem(ph, ph.dtype if ph.dtype == "f32" else None)
    x = np.random.default_rng(seed).uniform(0.0, 0.05, ph.n_blt)
    return oracle.prices(P, oracle.grad_objective(P, oracle.dose(P, x)))


def _same(a, b):
    assert a["beam"] == b["beam"]
    assert a["leaves"] == b["leaves"]
    assert a["rc"] == b["rc"] and a["gap"] == b["gap"]


def test_noalloc_pricing_matches_dao_price_twice_shrinking():
    torch = torch_cuda()
    big, small = cached_phantom("prostate"), cached_phantom("mini")
    assert int(small.rows_per_beam.sum()) < int(big.rows_per_beam.sum())
    for ph, seed in ((big, 1), (small, 2)):
        g = torch.tensor(_prices(ph, seed), dtype=torch.float64, device="cuda:0")
        ctx = ctx_for(ph, dtype="f64" if ph.dtype == "f64" else "f32")
        try:
            ref = ctx.price(g)
            got = ctx.price_noalloc(g)
            print(f"[noalloc] {ph.name} rows {int(ph.rows_per_beam.sum())} beam {got['beam']} rc {got['rc']:.6e}",
                  flush=True)
            _same(got, ref)
            # a second call on the same context, after dao_price used the
            # context's own scratch, still agrees
            _same(ctx.price_noalloc(g), ref)
        finally:
            ctx.close()


def test_noalloc_pricing_integer_ties():
    # integer prices with exact ties: the tie rules must hold through the
    # static scratch too
    torch = torch_cuda()
    ph = cached_phantom("tiny")
    rng = np.random.default_rng(5)
    w = rng.integers(-3, 3, ph.n_blt).astype(np.float64)
    g = torch.tensor(w, dtype=torch.float64, device="cuda:0")
    ctx = ctx_for(ph, dtype="f64")
    try:
        _same(ctx.price_noalloc(g), ctx.price(g))
        P = oracle_problem(ph)
        ref = oracle.price(P, w)
        got = ctx.price_noalloc(g)
        assert (got["beam"], got["leaves"]) == (ref["aperture"].beam, ref["aperture"].leaves)
    finally:
        ctx.close()


def test_noalloc_rejects_more_rows_than_the_scratch_holds():
    # 8 beams of 520 one-beamlet rows: 4160 rows, above the 4096-row limit
    torch = torch_cuda()
    B, R = 8, 520
    n = B * R
    V = 4
    row_ptr = np.array([0, n, 2 * n, 2 * n, 2 * n], dtype=np.int64)
    col = np.concatenate([np.arange(n), np.arange(n)]).astype(np.int32)
    val = np.full(2 * n, 0.5)
    vs = np.array([0, 0, -1, -1], dtype=np.int16)
    pres = [dict(is_target=1, t_under=1.0, t_over=1.0, w_under=1.0, w_over=1.0)]
    ctx = dao.DaoContext(row_ptr, col, val, n, np.full(B, R), np.ones(B * R), vs, pres, dtype="f64",
                         stream=torch.cuda.current_stream().cuda_stream)
    try:
        g = torch.full((n,), -1.0, dtype=torch.float64, device="cuda:0")
        ctx.price(g)
        with pytest.raises(dao.DaoError) as e:
            ctx.price_noalloc(g)
        assert e.value.status == dao.binding.DAO_EINVAL
        assert "4096" in str(e.value)
    finally:
        ctx.close()
