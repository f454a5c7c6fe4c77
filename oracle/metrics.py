"""Plan metrics used to state dose error (test infrastructure).

D95 of a target: the dose that 95 % of its voxels receive at least, taken as
the value at 0-based position floor(0.05 |v|) of the target doses sorted in
ascending order.  Dmax of an organ: the largest voxel dose in it.
"""
from __future__ import annotations

import math

import numpy as np


def d95(z: np.ndarray, mask: np.ndarray) -> float:
    v = np.sort(np.asarray(z, dtype=np.float64)[np.asarray(mask, dtype=bool)])
    if v.size == 0:
        return math.nan
    return float(v[int(math.floor(0.05 * v.size))])


def dmax(z: np.ndarray, mask: np.ndarray) -> float:
    v = np.asarray(z, dtype=np.float64)[np.asarray(mask, dtype=bool)]
    return float(v.max()) if v.size else math.nan
