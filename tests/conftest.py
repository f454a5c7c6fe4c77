import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


_PH_CACHE = {}


def cached_phantom(name, seed=0, **kw):
    """Phantoms are deterministic per (name, seed, options); build each once per session."""
    from phantom import make_phantom
    key = (name, seed, tuple(sorted(kw.items())))
    if key not in _PH_CACHE:
        _PH_CACHE[key] = make_phantom(name, seed, **kw)
    return _PH_CACHE[key]


def oracle_problem(ph, dtype=None):
    """Oracle problem on the phantom's data.  With dtype="f32" the dose
    matrix is first rounded to FP32, which is what an FP32 context stores, so
    both sides solve the same problem."""
    import numpy as np
    import oracle
    D = ph.csr()
    if dtype == "f32":
        D = D.copy()
        D.data = D.data.astype(np.float32).astype(np.float64)
    return oracle.make_problem(D, ph.rows_per_beam, ph.row_len, ph.vox_struct, ph.prescriptions)
