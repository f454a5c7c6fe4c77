"""Host encoder of the 16-bit storage of D (dao_encode_values), pinned to
numpy's FP16 rounding and to the definition of round-to-nearest-even BF16."""
import numpy as np
import pytest

import paper_1003_5402_amd as dao
from quant import round_bf16, round_f16

# the inputs include values past FP16's range on purpose (they encode to
# infinity, as numpy's cast does)
pytestmark = [pytest.mark.filterwarnings("ignore:overflow encountered in cast"),
              pytest.mark.filterwarnings("ignore:invalid value encountered in add")]


def _ratios(seed=0):
    rng = np.random.default_rng(seed)
    r = np.concatenate([
        10.0 ** rng.uniform(-9, 0, 20000),                         # spans FP16 subnormals to 1
        rng.uniform(0, 1, 5000),
        np.arange(1, 2049) / 2048.0,                               # exact FP16 values
        (np.arange(1024, 2048) + 0.5) / 2048.0,                    # FP16 ties (even rounding)
        (np.arange(128, 256) + 0.5) / 256.0,                       # BF16 ties
        np.array([0.0, 1.0, 6.103515625e-05, 5.960464477539063e-08, 2.98e-08, 1.0000001]),
        (np.arange(0, 1024) + 0.5) * 2.0 ** -24,                   # FP16 subnormal ties
        np.array([2.0 ** -25, 2.0 ** -25 * (1 + 2.0 ** -40), 2.0 ** -26, 1e-300, 5e-324,
                  65504.0, 65519.99, 65520.0, 1e5, 3.0e38]),       # half-unit edge, tiny, FP16 overflow
    ])
    return r


def _dec_f16(h):
    return h.view(np.float16).astype(np.float64)


def _dec_bf16(h):
    return (h.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def test_f16_hi_is_numpy_rounding_and_lo_the_residual():
    r = _ratios()
    hi, lo = dao.encode_values(dao.DAO_DFMT_F16, r)
    assert np.array_equal(_dec_f16(hi), round_f16(r))
    assert np.array_equal(hi, r.astype(np.float16).view(np.uint16))
    assert np.array_equal(_dec_f16(lo), round_f16(r - _dec_f16(hi)))
    # hi + lo: for r in [0, 1] the residual |r - hi| <= 2^-12 is rounded to
    # FP16 with at most 2^-11 relative or 2^-25 absolute (subnormal) error
    rec = _dec_f16(hi) + _dec_f16(lo)
    inside = r <= 1.0
    assert np.max(np.abs(rec[inside] - r[inside])) <= 2.0 ** -23
    big = (r > 0.25) & inside
    assert np.max(np.abs(rec[big] - r[big]) / r[big]) < 2.0 ** -21


def test_bf16_hi_is_nearest_even():
    r = _ratios(1)
    hi, lo = dao.encode_values(dao.DAO_DFMT_BF16, r)
    got = _dec_bf16(hi)
    assert np.array_equal(got, round_bf16(r))
    # nearest: no neighbouring BF16 value is closer; ties go to an even pattern
    for step in (-1, 1):
        nb = hi.astype(np.int64) + step
        ok = (nb >= 0) & (nb < 0x7F80)            # finite, non-negative neighbours
        alt = _dec_bf16(nb[ok].astype(np.uint16))
        d0, d1 = np.abs(got[ok] - r[ok]), np.abs(alt - r[ok])
        assert np.all(d0 <= d1)
        tie = d0 == d1
        assert np.all(hi[ok][tie] % 2 == 0)
    assert np.array_equal(_dec_f16(lo), round_f16(r - got))


def test_encoder_rejects_bad_arguments():
    with pytest.raises(dao.DaoError):
        dao.encode_values(dao.DAO_DFMT_NATIVE, np.array([0.5]))
    with pytest.raises(dao.DaoError):
        dao.encode_values(dao.DAO_DFMT_F16, np.array([-0.5]))
    with pytest.raises(dao.DaoError):
        dao.encode_values(dao.DAO_DFMT_BF16, np.array([np.nan]))
