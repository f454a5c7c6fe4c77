"""Test-side reference of the 16-bit storage of D (numpy only).

Round-to-nearest-even to FP16 comes from numpy's float64 -> float16
conversion; BF16 (8 exponent bits, 7 stored mantissa bits) is rounded here
from the binary definition with np.rint (half to even).  The per-beamlet
scale is the column maximum rounded to FP32, and a stored value is
s_i * (hi + lo) with lo the FP16 rounding of D_ij / s_i - hi.
"""
import numpy as np


def round_bf16(r):
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros_like(r)
    nz = r != 0
    a = np.abs(r[nz])
    m, e = np.frexp(a)                 # a = m 2^e, m in [0.5, 1)
    E = np.maximum(e - 1, -126)        # exponent of the binade (subnormals share -126)
    q = np.rint(np.ldexp(a, 7 - E))    # units of the last stored bit
    out[nz] = np.sign(r[nz]) * np.ldexp(q, E - 7)
    return out


def round_f16(r):
    return np.asarray(r, dtype=np.float64).astype(np.float16).astype(np.float64)


def col_scales(D):
    """FP32 column maxima of a CSR matrix (1 for empty columns)."""
    Dc = D.tocsc()
    s = np.ones(D.shape[1])
    for i in range(D.shape[1]):
        v = Dc.data[Dc.indptr[i]:Dc.indptr[i + 1]]
        if v.size and v.max() > 0:
            s[i] = v.max()
    return s.astype(np.float32).astype(np.float64)


def quantized(D, fmt, residual):
    """The matrix the device multiplies with: s_i (hi + lo) per entry."""
    s = col_scales(D)
    Q = D.tocsr(copy=True)
    r = Q.data / s[Q.indices]
    hi = round_f16(r) if fmt == "f16" else round_bf16(r)
    val = hi + (round_f16(r - hi) if residual else 0.0)
    Q.data = s[Q.indices] * val
    return Q
