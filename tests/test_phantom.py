"""Input generator checks and the closed-form single-beamlet dose pin.

The pin: with one beamlet open at unit intensity (x = e_i) the dose is column
i of D, and that column must equal the pencil-beam formula evaluated straight
from the beam geometry -- with the body entry point found here by bisection
on the outline, not by the generator's analytic ray intersection.  The same
test drives the oracle's dose routine (eq. 1, eq. 2, eq. 7 with one open
beamlet), so it pins both the matrix assembly and the oracle's D x.
"""
import math

import numpy as np
import pytest

from conftest import cached_phantom, oracle_problem
from phantom import make_phantom
from phantom.generator import BEAMLET_MM, MU_PER_MM, TRUNC_MM


def _inside(ph, x, y):
    cx, cy = ph.body.center
    hx, hy = ph.body.half
    if ph.body.kind == "box":
        return abs(x - cx) <= hx and abs(y - cy) <= hy
    return ((x - cx) / hx) ** 2 + ((y - cy) / hy) ** 2 <= 1.0


def _entry_by_bisection(ph, p0, dv):
    """First s with p0 + s dv inside the body, found by marching then bisecting."""
    s = -2000.0
    step = 0.25
    while not _inside(ph, p0[0] + s * dv[0], p0[1] + s * dv[1]):
        s += step
        if s > 2000.0:
            return math.nan
    lo, hi = s - step, s
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _inside(ph, p0[0] + mid * dv[0], p0[1] + mid * dv[1]):
            hi = mid
        else:
            lo = mid
    return hi


def _column_from_geometry(ph, i):
    th, uc, zr = ph.beamlet_axis(i)
    e = np.array([math.cos(th), math.sin(th)])
    lat = np.array([-math.sin(th), math.cos(th)])
    s_in = _entry_by_bisection(ph, ph.iso[:2] + uc * lat, -e)
    P = ph.voxel_centers()
    rel = P - ph.iso
    s = -(rel[:, :2] @ e)
    u = rel[:, :2] @ lat
    zz = rel[:, 2]
    rho2 = (u - uc) ** 2 + (zz - zr) ** 2
    depth = s - s_in
    inside = np.array([_inside(ph, x, y) for x, y in P[:, :2]]) if ph.body.kind != "box" else \
        (np.abs(P[:, 0] - ph.body.center[0]) <= ph.body.half[0]) & \
        (np.abs(P[:, 1] - ph.body.center[1]) <= ph.body.half[1])
    val = np.exp(-MU_PER_MM * depth) * np.exp(-rho2 / (2 * ph.sigma_mm ** 2))
    keep = (rho2 <= TRUNC_MM ** 2) & (depth >= -1e-9) & inside
    return np.where(keep, val, 0.0)


@pytest.mark.parametrize("name,beamlets", [("tiny", [0, 37, 163, 319]), ("mini", [0, 47])])
def test_single_beamlet_dose_matches_formula(name, beamlets):
    import oracle
    ph = cached_phantom(name)
    P = oracle_problem(ph)
    for i in beamlets:
        ref = _column_from_geometry(ph, i)
        x = np.zeros(ph.n_blt)
        x[i] = 1.0
        d = oracle.dose(P, x)
        assert np.count_nonzero(ref) > 100
        np.testing.assert_allclose(d, ref, rtol=1e-9, atol=1e-12)


@pytest.mark.slow
def test_single_beamlet_dose_prostate_f32():
    import oracle
    ph = cached_phantom("prostate")
    P = oracle_problem(ph)
    for i in [0, ph.n_blt // 2, ph.n_blt - 1]:
        ref = _column_from_geometry(ph, i)
        x = np.zeros(ph.n_blt)
        x[i] = 1.0
        d = oracle.dose(P, x)
        # D is stored at FP32: one rounding of each coefficient
        np.testing.assert_allclose(d, ref, rtol=2 ** -23, atol=1e-12)
        assert np.all(d.astype(np.float32).astype(np.float64) == d)


def test_deterministic_per_seed():
    a = make_phantom("mini", 3)
    b = make_phantom("mini", 3)
    c = make_phantom("mini", 4)
    for f in ["row_ptr", "col", "val", "vox_struct", "row_len", "rows_per_beam"]:
        assert np.array_equal(getattr(a, f), getattr(b, f))
    assert not np.array_equal(a.iso, c.iso)


def test_tiny_shape_and_csr_invariants():
    ph = cached_phantom("tiny")
    s = ph.summary()
    assert s["n_vox"] == 32 ** 3
    assert s["n_blt"] == 320 and s["n_rows"] == 40 and s["max_row_len"] == 8
    assert 4.0e5 <= s["nnz"] <= 7.0e5
    assert np.all(np.diff(ph.row_ptr) >= 0) and ph.row_ptr[0] == 0 and ph.row_ptr[-1] == ph.nnz
    for r in range(0, ph.n_vox, 997):
        c = ph.col[ph.row_ptr[r]:ph.row_ptr[r + 1]]
        assert np.all(np.diff(c) > 0)
    assert np.all(ph.val > 0) and np.all(np.isfinite(ph.val))
    assert int(ph.row_len.sum()) == ph.n_blt
    assert int(ph.rows_per_beam.sum()) == ph.n_rows
    # beamlets are numbered beam -> row -> position
    assert np.all(np.diff(ph.beamlet_beam) >= 0)
    # one PTV (sphere r = 15 mm, about 905 voxels) and one organ at risk
    assert abs(s["struct_sizes"]["PTV"] - 4 / 3 * math.pi * 15 ** 3 / 2.5 ** 3) < 40


@pytest.mark.slow
def test_paper_scale_configs_in_range():
    p = cached_phantom("prostate").summary()
    assert 1000 <= p["n_blt"] <= 1300 and 0.7 * 3e6 <= p["nnz"] <= 1.3 * 3e6
    assert p["n_beams"] == 9 and p["dtype"] == "f32" and p["n_apertures"] == 50
    h = cached_phantom("headneck").summary()
    assert h["n_beams"] == 5 and h["n_blt"] >= 1500 and h["nnz"] >= 0.7e7
    assert len(h["struct_sizes"]) == 8   # PTV, 6 organs at risk, normal tissue
