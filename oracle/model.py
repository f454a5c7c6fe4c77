"""Objective, dose and prices of the DAO model in FP64 (test infrastructure).

Paper passages followed:
* Section 2.1, eq. 1 and eq. 2: aperture dose z = sum_k D_kj y_k with
  D_kj = sum_{i in A_k} D_ij.  With beamlet intensities x_i = sum_{k in K_i} y_k
  (eq. 7) this is z = D x, which is how the dose is evaluated here.
* Discussion, eq. 9 and eq. 10: the per-structure one-sided quadratic
  penalties.  Under-dose on targets with weight alpha_s / |v_s| below T_s^-,
  over-dose on every structure with weight beta_s / |v_s| above T_s^+.
  eq. 3 to eq. 5 are the per-voxel special case.
* Section 2.3, eq. 8: beamlet prices w_i = sum_j D_ij pi_j.  The dual
  multiplier of the dose-definition constraint (eq. 6) at a stationary point
  of the Lagrangian is pi_j = dF/dz_j, so w = D^T grad F(z).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Sequence

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
    t_under: np.ndarray  # T_s^-
    b: np.ndarray        # over-dose weight beta_s/|v_s|
    t_over: np.ndarray   # T_s^+

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


def voxel_coefficients(vox_struct: np.ndarray, prescriptions: Sequence[Dict]):
    """Per-voxel (a, T^-, b, T^+) from eq. 9 and eq. 10.

    Each voxel belongs to at most one structure (label ``-1``: none).  |v_s|
    is the number of voxels carrying label s.  Targets get both terms,
    other structures the over-dose term only.
    """
    V = vox_struct.shape[0]
    a = np.zeros(V)
    tu = np.zeros(V)
    b = np.zeros(V)
    to = np.zeros(V)
    for s, pr in enumerate(prescriptions):
        m = vox_struct == s
        size = int(np.count_nonzero(m))
        if size == 0:
            continue
        if pr["is_target"]:
            a[m] = pr["w_under"] / size
            tu[m] = pr["t_under"]
        b[m] = pr["w_over"] / size
        to[m] = pr["t_over"]
    return a, tu, b, to


def make_problem(D: sp.csr_matrix, rows_per_beam, row_len, vox_struct, prescriptions) -> Problem:
    a, tu, b, to = voxel_coefficients(np.asarray(vox_struct), prescriptions)
    return Problem(D=sp.csr_matrix(D, dtype=np.float64),
                   rows_per_beam=np.asarray(rows_per_beam, dtype=np.int64),
                   row_len=np.asarray(row_len, dtype=np.int64),
                   a=a, t_under=tu, b=b, t_over=to)


def dose(P: Problem, x: np.ndarray) -> np.ndarray:
    """z = D x (eq. 1 and eq. 2 with x from eq. 7)."""
    return P.D @ np.asarray(x, dtype=np.float64)


def objective_terms(P: Problem, z: np.ndarray) -> np.ndarray:
    """f_j = a_j max(0, T^-_j - z_j)^2 + b_j max(0, z_j - T^+_j)^2."""
    under = np.maximum(0.0, P.t_under - z)
    over = np.maximum(0.0, z - P.t_over)
    return P.a * under * under + P.b * over * over


def objective(P: Problem, z: np.ndarray) -> float:
    """F(z) = sum over structures of eq. 9 and eq. 10, summed exactly (fsum)."""
    return math.fsum(objective_terms(P, z).tolist())


def grad_objective(P: Problem, z: np.ndarray) -> np.ndarray:
    """dF/dz_j = -2 a_j max(0, T^-_j - z_j) + 2 b_j max(0, z_j - T^+_j)."""
    return (-2.0 * P.a * np.maximum(0.0, P.t_under - z)
            + 2.0 * P.b * np.maximum(0.0, z - P.t_over))


def prices(P: Problem, u: np.ndarray) -> np.ndarray:
    """w = D^T u: with u = grad F(z) these are the w_i of eq. 8."""
    return P.D.T @ np.asarray(u, dtype=np.float64)
