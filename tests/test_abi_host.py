"""Host-side checks of the C ABI (no GPU needed).

* libdao.so loads and exports every function include/dao.h declares, and the
  binding declares exactly those;
* dao_create rejects every malformed input with DAO_EINVAL before any device
  call, and an over-cap footprint with DAO_ENOMEM.
"""
import os
import re

import numpy as np
import pytest

import paper_1003_5402_amd as dao
from conftest import ROOT, cached_phantom


def _declared():
    src = open(os.path.join(ROOT, "include", "dao.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dao_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = dao.load_library()
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert names == dao.symbols()


def test_library_links_hip_runtime():
    # the product path is the HIP library itself: no Python fallback exists
    import subprocess
    out = subprocess.run(["ldd", dao.binding.LIB_PATH], capture_output=True, text=True).stdout
    assert "amdhip64" in out


def _args(ph):
    return dict(row_ptr=ph.row_ptr.copy(), col=ph.col.copy(), val=ph.val.copy(), n_blt=ph.n_blt,
                rows_per_beam=ph.rows_per_beam.copy(), row_len=ph.row_len.copy(),
                vox_struct=ph.vox_struct.copy(), prescriptions=[dict(p) for p in ph.prescriptions])


def _expect(status, **kw):
    with pytest.raises(dao.DaoError) as e:
        a = kw.pop("_a")
        opts = kw.pop("_opts", {})
        dao.DaoContext(**a, **opts)
    assert e.value.status == status, str(e.value)
    return str(e.value)


def test_create_rejects_malformed_inputs():
    ph = cached_phantom("mini")
    cases = []
    a = _args(ph); a["row_ptr"][10] = a["row_ptr"][9] - 1; cases.append(("decreases", a))
    a = _args(ph); a["col"][3] = ph.n_blt; cases.append(("out of range", a))
    r = int(np.flatnonzero(np.diff(ph.row_ptr) >= 2)[0])
    a = _args(ph); e = a["row_ptr"][r]; a["col"][e + 1] = a["col"][e]
    cases.append(("strictly increasing", a))
    a = _args(ph); a["val"][7] = np.nan; cases.append(("non-finite", a))
    a = _args(ph); a["val"][7] = -1.0; cases.append(("negative value", a))
    a = _args(ph); a["row_len"][0] += 1; cases.append(("sum of row_len", a))
    a = _args(ph); a["row_len"][0] = 65; a["row_len"][1] -= 61; cases.append(("row_len", a))
    a = _args(ph); a["vox_struct"][4] = len(ph.prescriptions); cases.append(("structure id", a))
    a = _args(ph); a["prescriptions"][1]["w_over"] = -0.5; cases.append(("negative weight", a))
    a = _args(ph); a["prescriptions"][0]["t_under"] = 2.0; cases.append(("t_under > t_over", a))
    a = _args(ph); a["rows_per_beam"][0] = 0; cases.append(("rows_per_beam", a))
    a = _args(ph); a["n_blt"] = 70000; cases.append(("65535", a))
    for needle, a in cases:
        msg = _expect(dao.DAO_EINVAL, _a=a)
        assert needle in msg, (needle, msg)
    msg = _expect(dao.DAO_EINVAL, _a=_args(ph), _opts=dict(max_apertures=0))
    assert "max_apertures" in msg
    msg = _expect(dao.DAO_EINVAL, _a=_args(ph), _opts=dict(ls_slots=0))
    assert "ls_slots" in msg
    msg = _expect(dao.DAO_EINVAL, _a=_args(ph), _opts=dict(persistent=3))
    assert "persistent" in msg
    for opts, needle in [(dict(d_format=3), "d_format"), (dict(d_residual=1), "d_residual"),
                         (dict(d_format=1, d_residual=3), "d_residual"),
                         (dict(d_format=1, d_residual=2, residual_rounds=-1), "residual_rounds"),
                         (dict(direction=2), "direction"), (dict(apertures_per_round=0), "apertures_per_round"),
                         (dict(apertures_per_round=17), "apertures_per_round"), (dict(dk_format=2), "dk_format"), (dict(dk_format=4), "dk_format"),
                         (dict(dk_format=1, dtype="f64"), "DAO_F32"), (dict(dk_format=1, master=1), "aperture"),
                         (dict(d_format=1, dtype="f64"), "DAO_F32"), (dict(d_format=2, master=1), "aperture"),
                         (dict(product_tune=2), "product_tune"), (dict(dose_variant=9), "dose_variant"),
                         (dict(dose_variant=2, d_format=1), "native"), (dict(gradient_depth=6), "gradient_depth")]:
        msg = _expect(dao.DAO_EINVAL, _a=_args(ph), _opts=opts)
        assert needle in msg, (opts, msg)


def test_create_rejects_malformed_structure_extras():
    ph = cached_phantom("mini", nested_targets=True)
    v2 = ph.vox_struct2.copy()
    j = int(np.flatnonzero(v2 >= 0)[0])
    bad = v2.copy(); bad[j] = ph.vox_struct[j]
    msg = _expect(dao.DAO_EINVAL, _a=_args(ph), _opts=dict(vox_struct2=bad))
    assert "same structure twice" in msg
    bad = v2.copy(); bad[j] = len(ph.prescriptions)
    msg = _expect(dao.DAO_EINVAL, _a=_args(ph), _opts=dict(vox_struct2=bad))
    assert "second structure id" in msg
    a = _args(ph); a["vox_struct"][j] = -1
    msg = _expect(dao.DAO_EINVAL, _a=a, _opts=dict(vox_struct2=v2))
    assert "no first" in msg
    shift = np.zeros(ph.n_vox); shift[3] = np.inf
    msg = _expect(dao.DAO_EINVAL, _a=_args(ph), _opts=dict(vox_shift=shift))
    assert "threshold shift" in msg


def test_create_enforces_memory_cap():
    ph = cached_phantom("mini")
    msg = _expect(dao.DAO_ENOMEM, _a=_args(ph), _opts=dict(mem_cap_bytes=10000))
    assert "exceeds mem_cap_bytes" in msg


def test_server_rejects_bad_options():
    """dao_server_create checks its options before touching the device."""
    for kw in (dict(max_live=0), dict(max_live=65), dict(hbm_cap_bytes=-1), dict(workers=-1), dict(workers=17)):
        with pytest.raises(dao.DaoError):
            dao.Server(**kw)
