"""Apertures and the aperture <-> beamlet maps (test infrastructure).

An aperture (Section 2.1: the set A_k of open beamlets of one beam) is stored
as its beam and one half-open leaf interval [L, R) per MLC row of that beam,
positions counted from 0 within the row; a closed row is (0, 0).  The
consecutiveness constraint of Section 2.3 (one contiguous open run per row)
is built into this form.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

from .model import Problem


@dataclasses.dataclass(frozen=True)
class Aperture:
    beam: int
    leaves: Tuple[Tuple[int, int], ...]   # one (L, R) per row of the beam

    def open_beamlets(self, P: Problem) -> np.ndarray:
        r0, r1 = P.beam_row_range(self.beam)
        assert len(self.leaves) == r1 - r0
        starts = P.row_start()
        idx = [np.arange(starts[r] + L, starts[r] + R)
               for r, (L, R) in zip(range(r0, r1), self.leaves) if R > L]
        return np.concatenate(idx) if idx else np.zeros(0, dtype=np.int64)


def beamlet_intensity(P: Problem, pool: Sequence[Aperture], y: Sequence[float]) -> np.ndarray:
    """x_i = sum over apertures k containing beamlet i of y_k (eq. 7)."""
    x = np.zeros(P.n_blt)
    for ap, yk in zip(pool, y):
        x[ap.open_beamlets(P)] += float(yk)
    return x


def aperture_gradient(P: Problem, pool: Sequence[Aperture], g: np.ndarray) -> np.ndarray:
    """dF/dy_k = sum_{i in A_k} g_i (chain rule through eq. 1 and eq. 2).

    With g = w = D^T grad F this is the reduced cost of every pool aperture:
    the objective of the sub-problem (eq. 8) evaluated at aperture k.
    """
    return np.array([math.fsum(g[ap.open_beamlets(P)].tolist()) for ap in pool])
