"""GPU parity of the single products against the FP64 oracle, through the C ABI.

Tolerances (max-norm error relative to the oracle's max-norm):
* FP64 contexts: 1e-12.  Both sides accumulate in FP64; only the order of
  the sums differs.
* FP32 contexts: 1e-5 (the dose/objective bar of the method's FP32 path).
  A dose row has at most ~130 non-negative terms, so its FP32 sum is within
  130 * 2^-24 < 1e-5 of the exact sum; the transposed product sums ~3-6e3
  terms per beamlet in 256 short sequential runs plus a 8-level tree, so
  its error is ~(15 + 8) * 2^-24 of the absolute sum.
The objective F is summed in FP64 on both sides: 1e-12 for both types.
Inputs the GPU reads in FP32 (x, d) are rounded to FP32 first and the oracle
gets the same rounded values.
"""
import numpy as np
import pytest

import oracle
from conftest import cached_phantom, oracle_problem
from gpu_util import ctx_for, dev, relerr, tdtype, torch_cuda

pytestmark = pytest.mark.gpu

CASES = [("mini", "f64"), ("tiny", "f64"), ("tiny", "f32"), ("prostate", "f32"), ("headneck", "f32")]


def _tol(dtype):
    return 1e-12 if dtype == "f64" else 1e-5


def _np_dtype(dtype):
    return np.float64 if dtype == "f64" else np.float32


@pytest.fixture(scope="module")
def contexts():
    out = {}
    yield out
    for c in out.values():
        c[2].close()


def _get(contexts, name, dtype):
    key = (name, dtype)
    if key not in contexts:
        ph = cached_phantom(name)
        print(f"[ctx] {name} {dtype}", flush=True)
        contexts[key] = (ph, oracle_problem(ph, dtype), ctx_for(ph, dtype=dtype))
    return contexts[key]


@pytest.mark.parametrize("name,dtype", CASES)
def test_dose_parity(contexts, name, dtype):
    torch = torch_cuda()
    ph, P, ctx = _get(contexts, name, dtype)
    rng = np.random.default_rng(1)
    for trial in range(3):
        x = rng.uniform(0.0, 0.05, ph.n_blt).astype(_np_dtype(dtype)).astype(np.float64)
        if trial == 1:
            x[:] = 0.0
            x[ph.n_blt // 3] = 1.0      # one open beamlet
        xd = dev(x, tdtype(ctx))
        d = torch.full((ph.n_vox,), float("nan"), dtype=tdtype(ctx), device="cuda:0")
        ctx.dose(xd, d)
        torch.cuda.synchronize()
        ref = oracle.dose(P, x)
        got = d.double().cpu().numpy()
        assert np.all(np.isfinite(got))
        assert relerr(got, ref) <= _tol(dtype), (trial, relerr(got, ref))
        # voxels no beamlet reaches get exactly 0
        empty = np.diff(ph.row_ptr) == 0
        assert np.all(got[empty] == 0.0)
    # zero fluence gives zero dose everywhere
    z = torch.zeros(ph.n_blt, dtype=tdtype(ctx), device="cuda:0")
    d = torch.ones(ph.n_vox, dtype=tdtype(ctx), device="cuda:0")
    ctx.dose(z, d)
    assert float(d.abs().max()) == 0.0


@pytest.mark.parametrize("name,dtype", CASES)
def test_gradient_and_objective_parity(contexts, name, dtype):
    torch = torch_cuda()
    ph, P, ctx = _get(contexts, name, dtype)
    rng = np.random.default_rng(2)
    for scale in (0.0, 0.02, 0.06):
        x = rng.uniform(0.0, 1.0, ph.n_blt) * scale
        d = oracle.dose(P, x).astype(_np_dtype(dtype)).astype(np.float64)
        g = torch.full((ph.n_blt,), float("nan"), dtype=tdtype(ctx), device="cuda:0")
        F = ctx.gradient(dev(d, tdtype(ctx)), g)
        torch.cuda.synchronize()
        Fref = oracle.objective(P, d)
        gref = oracle.prices(P, oracle.grad_objective(P, d))
        assert abs(F - Fref) <= 1e-12 * Fref, (scale, F, Fref)
        assert relerr(g.double().cpu().numpy(), gref) <= _tol(dtype), scale


@pytest.mark.parametrize("name,dtype", CASES)
def test_price_on_oracle_prices(contexts, name, dtype):
    """FP64 prices from the oracle: identical beam and leaves always."""
    ph, P, ctx = _get(contexts, name, dtype)
    rng = np.random.default_rng(3)
    states = [np.zeros(ph.n_blt), rng.uniform(0, 0.03, ph.n_blt), rng.uniform(0, 0.08, ph.n_blt)]
    for x in states:
        w = oracle.prices(P, oracle.grad_objective(P, oracle.dose(P, x)))
        res = ctx.price(dev(w, torch_cuda().float64))
        ref = oracle.price(P, w)
        assert res["beam"] == ref["aperture"].beam
        assert res["leaves"] == ref["aperture"].leaves
        assert abs(res["rc"] - ref["rc"]) <= 1e-12 * abs(ref["rc"])
        assert abs(res["gap"] - ref["gap"]) <= 1e-12 * max(abs(ref["rc"]), abs(ref["gap"]))


def test_price_exact_ties_and_closed_rows(contexts):
    """Integer prices with many exact ties, all-positive rows, zero runs."""
    ph, P, ctx = _get(contexts, "mini", "f64")
    rng = np.random.default_rng(4)
    for trial in range(40):
        w = rng.integers(-3, 4, size=ph.n_blt).astype(np.float64)
        if trial % 4 == 1:
            w = np.abs(w)                     # nothing negative: all rows closed
        if trial % 4 == 2:
            w = -rng.integers(0, 2, size=ph.n_blt).astype(np.float64)
        res = ctx.price(dev(w, torch_cuda().float64))
        ref = oracle.price(P, w)
        assert (res["beam"], res["leaves"]) == (ref["aperture"].beam, ref["aperture"].leaves), trial
        assert res["rc"] == ref["rc"] and res["gap"] == ref["gap"]


@pytest.mark.parametrize("name,dtype", CASES)
def test_products_are_deterministic(contexts, name, dtype):
    torch = torch_cuda()
    ph, P, ctx = _get(contexts, name, dtype)
    x = dev(np.random.default_rng(5).uniform(0, 0.05, ph.n_blt), tdtype(ctx))
    d1 = torch.empty(ph.n_vox, dtype=tdtype(ctx), device="cuda:0")
    d2 = torch.empty_like(d1)
    ctx.dose(x, d1)
    ctx.dose(x, d2)
    g1 = torch.empty(ph.n_blt, dtype=tdtype(ctx), device="cuda:0")
    g2 = torch.empty_like(g1)
    F1 = ctx.gradient(d1, g1)
    F2 = ctx.gradient(d1, g2)
    assert torch.equal(d1, d2) and torch.equal(g1, g2) and F1 == F2


@pytest.mark.parametrize("name,dtype", CASES)
def test_price_own_prices_at_zero_dose(contexts, name, dtype):
    """Round 1 prices on the GPU's own FP64 prices.  Beamlets that reach no
    target voxel are priced exactly 0, which makes exact ties between leaf
    intervals with and without them; the row scan's rule (leading zeros in,
    trailing zeros out) must resolve them as the oracle does."""
    ph, P, ctx = _get(contexts, name, dtype)
    ctx.reset()
    got = ctx.price_current()
    w = oracle.prices(P, oracle.grad_objective(P, np.zeros(P.n_vox)))
    ref = oracle.price(P, w)
    assert (got["beam"], got["leaves"]) == (ref["aperture"].beam, ref["aperture"].leaves)
    assert abs(got["rc"] - ref["rc"]) <= 1e-12 * abs(ref["rc"])


# Every variant of the two products (loads in flight per thread, x staged on
# chip or read from device memory, slices per workgroup, whole rows per lane
# on a grid of 1, 2 or 4 workgroups per compute unit) adds the same terms in
# the same order: results agree bit for bit with the plain variant, in every
# value format.
VARIANTS = [(0, 4), (1, 8), (2, 16), (3, 4), (4, 8), (5, 4), (6, 16), (7, 8), (8, 16)]


@pytest.mark.parametrize("name,dtype,fmt", [("tiny", "f64", 0), ("prostate", "f32", 0), ("prostate", "f32", 1),
                                            ("headneck", "f32", 0)])
def test_product_variants_identical(name, dtype, fmt):
    torch = torch_cuda()
    ph = cached_phantom(name)
    rng = np.random.default_rng(11)
    x = dev(rng.uniform(0.0, 0.05, ph.n_blt), torch.float64 if dtype == "f64" else torch.float32)
    outs = []
    for dv, gd in VARIANTS:
        if dv == 2 and fmt != 0:
            continue
        print(f"[variant] {name} {dtype} fmt={fmt} dose={dv} depth={gd}", flush=True)
        ctx = ctx_for(ph, dtype=dtype, d_format=fmt, product_tune=0, dose_variant=dv, gradient_depth=gd)
        try:
            inf = ctx.info()
            assert (inf["dose_variant"], inf["gradient_depth"]) == (dv, gd)
            d = torch.full((ph.n_vox,), float("nan"), dtype=x.dtype, device="cuda:0")
            ctx.dose(x, d)
            g = torch.full((ph.n_blt,), float("nan"), dtype=x.dtype, device="cuda:0")
            F = ctx.gradient(d, g)
            torch.cuda.synchronize()
            outs.append((d.cpu(), g.cpu(), F))
        finally:
            ctx.close()
    d0, g0, F0 = outs[0]
    assert torch.isfinite(d0).all() and torch.isfinite(g0).all()
    for d, g, F in outs[1:]:
        assert torch.equal(d, d0) and torch.equal(g, g0) and F == F0


def test_tuned_variant_reported():
    ph = cached_phantom("tiny")
    ctx = ctx_for(ph, dtype="f32")
    try:
        inf = ctx.info()
        assert 0 <= inf["dose_variant"] <= 8 and inf["gradient_depth"] in (4, 8, 16)
    finally:
        ctx.close()


def test_product_timing_calls():
    """The measurement entry points run, return positive times and leave the
    products' results unchanged; bad arguments are rejected."""
    import paper_1003_5402_amd as dao
    torch = torch_cuda()
    ph = cached_phantom("tiny")
    ctx = ctx_for(ph, dtype="f32")
    try:
        x = dev(np.random.default_rng(3).uniform(0, 0.05, ph.n_blt), torch.float32)
        d0 = torch.empty(ph.n_vox, dtype=torch.float32, device="cuda:0")
        ctx.dose(x, d0)
        scrub = torch.zeros(4 << 20, dtype=torch.uint8, device="cuda:0")
        assert ctx.time_product(0, 3) > 0 and ctx.time_product(1, 3) > 0
        assert ctx.time_product_cold(0, 2, scrub) > 0 and ctx.time_product_cold(1, 2, scrub) > 0
        assert int(scrub.count_nonzero()) == 0
        d1 = torch.empty_like(d0)
        ctx.dose(x, d1)
        torch.cuda.synchronize()
        assert torch.equal(d0, d1)
        with pytest.raises(dao.DaoError):
            ctx.time_product(2, 3)
        with pytest.raises(dao.DaoError):
            ctx.time_product_cold(0, 2, scrub[: 1 << 19])
        # the streaming-read reference: positive, buffers untouched, sizes checked
        buf = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda:0")
        assert ctx.time_read_cold(buf, 1 << 20, 2, scrub) > 0
        assert int(buf.count_nonzero()) == 0 and int(scrub.count_nonzero()) == 0
        for nbytes in (8, 1000):
            with pytest.raises(dao.DaoError):
                ctx.time_read_cold(buf, nbytes, 2, scrub)
    finally:
        ctx.close()
