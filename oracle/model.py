"""Objective, dose and prices of the DAO model in FP64 (test infrastructure).

Paper passages followed:
* Section 2.1, eq. 1 and eq. 2: aperture dose z = sum_k D_kj y_k with
  D_kj = sum_{i in A_k} D_ij.  With beamlet intensities x_i = sum_{k in K_i} y_k
  (eq. 7) this is z = D x, which is how the dose is evaluated here.
* Discussion, eq. 9 and eq. 10: the per-structure one-sided quadratic
  penalties.  Under-dose on targets with weight alpha_s / |v_s| below T_s^-,
  over-dose on every structure with weight beta_s / |v_s| above T_s^+.
  Structures may overlap (eq. 10 sums over all structures containing a
  voxel): a voxel may carry a second structure label, whose terms are added
  to those of its first (nested targets such as the head-and-neck cases'
  PTV1 inside PTV2, Section 3).
* eq. 3 to eq. 5 with per-voxel thresholds T_j: each voxel's thresholds may
  be shifted by a per-voxel amount tau_j (T^-_s + tau_j, T^+_s + tau_j).  The
  re-optimization mode of the Discussion (alpha_j = beta_j = 1, T_j the
  deformed dose of the original plan) is the special case of one target
  structure and one structure for all other voxels, thresholds 0, weights
  equal to the structure sizes (so alpha_s / |v_s| = 1) and tau = T.
* Section 2.3, eq. 8: beamlet prices w_i = sum_j D_ij pi_j.  The dual
  multiplier of the dose-definition constraint (eq. 6) at a stationary point
  of the Lagrangian is pi_j = dF/dz_j, so w = D^T grad F(z).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Problem:
    """Everything the method needs, as plain FP64 arrays.

    ``D`` is the voxel x beamlet dose matrix (CSR).  ``rows_per_beam`` and
    ``row_len`` give the MLC geometry: beamlets are numbered beam by beam,
    row by row, position by position.  The per-voxel arrays hold the
    coefficients of eq. 9 and eq. 10 after dividing the structure weights by
    the structure size.
    """

    D: sp.csr_matrix
    rows_per_beam: np.ndarray
    row_len: np.ndarray
    a: np.ndarray        # under-dose weight alpha_s/|v_s| (0 off targets)
    t_under: np.ndarray  # T_s^- (+ tau_j)
    b: np.ndarray        # over-dose weight beta_s/|v_s|
    t_over: np.ndarray   # T_s^+ (+ tau_j)
    # the terms of each voxel's second structure (same four arrays), or None
    extra: Optional[tuple] = None

    def terms(self):
        """Every (a, T^-, b, T^+) term set: the first structure's, then the
        second structure's if any voxel has one."""
        t = [(self.a, self.t_under, self.b, self.t_over)]
        if self.extra is not None:
            t.append(self.extra)
        return t

    @property
    def n_vox(self) -> int:
        return self.D.shape[0]

    @property
    def n_blt(self) -> int:
        return self.D.shape[1]

    def row_start(self) -> np.ndarray:
        """First beamlet index of every MLC row."""
        return np.concatenate([[0], np.cumsum(self.row_len)[:-1]]).astype(np.int64)

    def beam_row_range(self, beam: int):
        """Half-open range of global MLC row indices belonging to ``beam``."""
        first = int(np.sum(self.rows_per_beam[:beam]))
        return first, first + int(self.rows_per_beam[beam])


def structure_sizes(vox_struct: np.ndarray, n_struct: int, vox_struct2: Optional[np.ndarray] = None):
    """|v_s|: the number of voxels carrying label s as first or second structure."""
    size = np.zeros(n_struct, dtype=np.int64)
    for labels in (vox_struct, vox_struct2):
        if labels is None:
            continue
        for s in range(n_struct):
            size[s] += int(np.count_nonzero(np.asarray(labels) == s))
    return size


def _coefficients(labels: np.ndarray, prescriptions: Sequence[Dict], size: np.ndarray):
    V = labels.shape[0]
    a = np.zeros(V)
    tu = np.zeros(V)
    b = np.zeros(V)
    to = np.zeros(V)
    for s, pr in enumerate(prescriptions):
        m = labels == s
        if size[s] == 0 or not np.any(m):
            continue
        if pr["is_target"]:
            a[m] = pr["w_under"] / size[s]
            tu[m] = pr["t_under"]
        b[m] = pr["w_over"] / size[s]
        to[m] = pr["t_over"]
    return a, tu, b, to


def voxel_coefficients(vox_struct: np.ndarray, prescriptions: Sequence[Dict],
                       vox_struct2: Optional[np.ndarray] = None):
    """Per-voxel (a, T^-, b, T^+) from eq. 9 and eq. 10 for the first label,
    and for the second label when given (``None`` when absent).

    Label ``-1`` means none.  |v_s| counts the voxels carrying s as either
    label.  Targets get both terms, other structures the over-dose term only.
    """
    size = structure_sizes(vox_struct, len(prescriptions), vox_struct2)
    first = _coefficients(np.asarray(vox_struct), prescriptions, size)
    second = None
    if vox_struct2 is not None and np.any(np.asarray(vox_struct2) >= 0):
        second = _coefficients(np.asarray(vox_struct2), prescriptions, size)
    return first, second


def make_problem(D: sp.csr_matrix, rows_per_beam, row_len, vox_struct, prescriptions,
                 vox_struct2=None, vox_shift=None) -> Problem:
    """The problem of eq. 9 and eq. 10 on dose matrix D.  ``vox_struct2``:
    optional second structure label per voxel; ``vox_shift``: optional
    per-voxel threshold shift tau_j (both thresholds of every term of voxel j
    move by tau_j)."""
    (a, tu, b, to), second = voxel_coefficients(np.asarray(vox_struct), prescriptions, vox_struct2)
    if vox_shift is not None:
        tau = np.asarray(vox_shift, dtype=np.float64)
        tu, to = tu + tau, to + tau
        if second is not None:
            second = (second[0], second[1] + tau, second[2], second[3] + tau)
    return Problem(D=sp.csr_matrix(D, dtype=np.float64),
                   rows_per_beam=np.asarray(rows_per_beam, dtype=np.int64),
                   row_len=np.asarray(row_len, dtype=np.int64),
                   a=a, t_under=tu, b=b, t_over=to, extra=second)


def reoptimization_structures(target: np.ndarray, reached: np.ndarray):
    """Labels and prescriptions of the re-optimization mode (eq. 3 and eq. 4
    with alpha_j = beta_j = 1 and per-voxel T_j): structure 0 = target voxels
    (under- and over-dose, thresholds 0 before the shift), structure 1 = every
    other voxel in ``reached`` (over-dose only); weights equal to the
    structure sizes so that every per-voxel weight is exactly 1.  Pair with
    ``vox_shift = T``."""
    target = np.asarray(target, dtype=bool)
    rest = np.asarray(reached, dtype=bool) & ~target
    labels = np.full(target.shape[0], -1, dtype=np.int16)
    labels[target] = 0
    labels[rest] = 1
    nt, nr = int(target.sum()), int(rest.sum())
    pres = [dict(is_target=1, t_under=0.0, t_over=0.0, w_under=float(nt), w_over=float(nt)),
            dict(is_target=0, t_under=0.0, t_over=0.0, w_under=0.0, w_over=float(max(nr, 1)))]
    return labels, pres


def dose(P: Problem, x: np.ndarray) -> np.ndarray:
    """z = D x (eq. 1 and eq. 2 with x from eq. 7)."""
    return P.D @ np.asarray(x, dtype=np.float64)


def objective_terms(P: Problem, z: np.ndarray) -> np.ndarray:
    """f_j = sum over the voxel's terms of a_j max(0, T^-_j - z_j)^2 + b_j max(0, z_j - T^+_j)^2."""
    f = np.zeros_like(np.asarray(z, dtype=np.float64))
    for a, tu, b, to in P.terms():
        under = np.maximum(0.0, tu - z)
        over = np.maximum(0.0, z - to)
        f = f + a * under * under + b * over * over
    return f


def objective(P: Problem, z: np.ndarray) -> float:
    """F(z) = sum over structures of eq. 9 and eq. 10, summed exactly (fsum)."""
    return math.fsum(objective_terms(P, z).tolist())


def grad_objective(P: Problem, z: np.ndarray) -> np.ndarray:
    """dF/dz_j = sum over the voxel's terms of -2 a_j max(0, T^-_j - z_j) + 2 b_j max(0, z_j - T^+_j)."""
    g = np.zeros_like(np.asarray(z, dtype=np.float64))
    for a, tu, b, to in P.terms():
        g = g + (-2.0 * a * np.maximum(0.0, tu - z) + 2.0 * b * np.maximum(0.0, z - to))
    return g


def prices(P: Problem, u: np.ndarray) -> np.ndarray:
    """w = D^T u: with u = grad F(z) these are the w_i of eq. 8."""
    return P.D.T @ np.asarray(u, dtype=np.float64)
