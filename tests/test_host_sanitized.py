"""The library's host code (input validation, layout construction, 16-bit
encoders: csrc/layout.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer by g++ and run on phantom inputs (no GPU).

tests/host_layout_check.cpp reads every array the layout builder writes and
checks it against the CSR input (forward sliced-ELL entries in order with
zero padding, transposed entries, row permutation, objective classes, MLC
geometry), feeds malformed inputs to the validator, checks the encoders'
rounding, and checks that the persistent master's dealing of row batches to
workgroups (dao_common.h) is a bijection within the LDS sizing, and that the
forward product's balanced slice lists hold every slice once.  A sanitizer
report or a failed check ends the run non-zero.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from conftest import ROOT, cached_phantom

SRC = os.path.join(ROOT, "paper_1003_5402_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("asan") / "host_layout_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", SRC, os.path.join(SRC, "layout.cpp"),
           os.path.join(ROOT, "tests", "host_layout_check.cpp"), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return str(out)


def _write(ph, path):
    with open(path, "wb") as f:
        V, N, nnz = ph.n_vox, ph.n_blt, int(ph.row_ptr[-1])
        f.write(struct.pack("<5q", V, N, nnz, len(ph.rows_per_beam), len(ph.prescriptions)))
        f.write(np.ascontiguousarray(ph.row_ptr, dtype="<i8").tobytes())
        f.write(np.ascontiguousarray(ph.col, dtype="<i4").tobytes())
        f.write(np.ascontiguousarray(ph.val, dtype="<f8").tobytes())
        f.write(np.ascontiguousarray(ph.rows_per_beam, dtype="<i4").tobytes())
        f.write(np.ascontiguousarray(ph.row_len, dtype="<i4").tobytes())
        f.write(np.ascontiguousarray(ph.vox_struct, dtype="<i2").tobytes())
        for p in ph.prescriptions:
            f.write(struct.pack("<i4d", int(p["is_target"]), p["t_under"], p["t_over"], p["w_under"], p["w_over"]))


@pytest.mark.parametrize("name", ["mini", "tiny"])
def test_layout_under_sanitizers(checker, name, tmp_path):
    ph = cached_phantom(name)
    path = tmp_path / f"{name}.bin"
    _write(ph, path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([checker, str(path)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.startswith("OK"), r.stdout
