"""Pins for the oracle's objective (eq. 9, eq. 10), gradient and prices (eq. 8).

* closed form at zero dose: F(0) = sum over targets of alpha_s (T_s^-)^2 and
  dF/dz_j = -2 alpha_s T_s^- / |v_s| on targets, 0 elsewhere;
* closed form for a single voxel moved off its threshold;
* central finite differences of F(D x) against D^T grad F (chain rule);
* the adjoint identity <D x, u> = <x, D^T u> (a transposed operand fails it).
"""
import math

import numpy as np
import pytest

import oracle
from conftest import cached_phantom, oracle_problem


def test_objective_at_zero_dose_closed_form():
    ph = cached_phantom("tiny")
    P = oracle_problem(ph)
    F0 = oracle.objective(P, np.zeros(P.n_vox))
    # one target: alpha = 1, T^- = 1, so F(0) = 1 exactly up to rounding of 1/|v|
    assert abs(F0 - 1.0) < 1e-14
    g0 = oracle.grad_objective(P, np.zeros(P.n_vox))
    ptv = ph.structure_mask("PTV")
    n = int(ptv.sum())
    np.testing.assert_allclose(g0[ptv], -2.0 / n, rtol=1e-15)
    assert np.all(g0[~ptv] == 0.0)


def test_objective_general_prescriptions_zero_dose():
    ph = cached_phantom("mini")
    pres = [dict(p) for p in ph.prescriptions]
    pres[0].update(t_under=0.8, t_over=1.1, w_under=3.0, w_over=2.0)
    P = oracle.make_problem(ph.csr(), ph.rows_per_beam, ph.row_len, ph.vox_struct, pres)
    assert abs(oracle.objective(P, np.zeros(P.n_vox)) - 3.0 * 0.8 ** 2) < 1e-14


def test_single_voxel_offsets_closed_form():
    ph = cached_phantom("mini")
    P = oracle_problem(ph)
    sizes = {k: int(np.sum(ph.vox_struct == k)) for k in range(len(ph.struct_names))}
    z = np.zeros(P.n_vox)
    # put every target voxel at its prescription and every other voxel at 0:
    z[ph.vox_struct == 0] = 1.0
    assert oracle.objective(P, z) == 0.0
    j_t = int(np.flatnonzero(ph.vox_struct == 0)[5])
    j_o = int(np.flatnonzero(ph.vox_struct == 1)[7])
    z2 = z.copy()
    z2[j_t] = 1.0 - 0.25          # under-dose a target voxel by 0.25
    z2[j_o] = 0.5 + 0.3           # over-dose an organ voxel by 0.3 above T+ = 0.5
    expect = 1.0 / sizes[0] * 0.25 ** 2 + 0.5 / sizes[1] * 0.3 ** 2
    assert abs(oracle.objective(P, z2) - expect) < 1e-15
    g = oracle.grad_objective(P, z2)
    assert abs(g[j_t] - (-2.0 / sizes[0] * 0.25)) < 1e-15
    assert abs(g[j_o] - (2.0 * 0.5 / sizes[1] * 0.3)) < 1e-15
    z3 = z.copy()
    z3[j_t] = 1.2                 # target over-dose, T+ = 1, beta = 1
    assert abs(oracle.objective(P, z3) - 1.0 / sizes[0] * 0.2 ** 2) < 1e-15


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_finite_differences(seed):
    ph = cached_phantom("mini")
    P = oracle_problem(ph)
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 0.04, P.n_blt)
    e = rng.normal(size=P.n_blt)
    z = oracle.dose(P, x)
    g = oracle.prices(P, oracle.grad_objective(P, z))
    h = 1e-6
    fp = oracle.objective(P, oracle.dose(P, x + h * e))
    fm = oracle.objective(P, oracle.dose(P, x - h * e))
    fd = (fp - fm) / (2 * h)
    an = float(np.dot(g, e))
    assert abs(fd - an) <= 1e-7 * max(abs(an), 1e-12)


def test_adjoint_identity():
    ph = cached_phantom("tiny")
    P = oracle_problem(ph)
    rng = np.random.default_rng(7)
    x = rng.normal(size=P.n_blt)
    u = rng.normal(size=P.n_vox)
    lhs = math.fsum((oracle.dose(P, x) * u).tolist())
    rhs = math.fsum((x * oracle.prices(P, u)).tolist())
    assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + 1.0)


def test_structure_size_normalisation():
    ph = cached_phantom("tiny")
    (a, tu, b, to), second = oracle.voxel_coefficients(ph.vox_struct, ph.prescriptions)
    assert second is None
    for s, pr in enumerate(ph.prescriptions):
        m = ph.vox_struct == s
        assert abs(math.fsum(b[m].tolist()) - pr["w_over"]) < 1e-12
        if pr["is_target"]:
            assert abs(math.fsum(a[m].tolist()) - pr["w_under"]) < 1e-12
        else:
            assert np.all(a[m] == 0.0)
    assert np.all(b[ph.vox_struct < 0] == 0.0) and np.all(a[ph.vox_struct < 0] == 0.0)
