"""ctypes declarations of include/dao.h and a small context wrapper."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int16, c_int32, c_int64, c_void_p
from typing import Dict, Optional, Sequence

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdao.so")

DAO_OK, DAO_EOPTIMAL, DAO_ESTALLED, DAO_ENOTCONV = 0, 1, 2, 3
DAO_EINVAL, DAO_ENOMEM, DAO_EDEVICE, DAO_ESTATE = -1, -2, -3, -4
DAO_F64, DAO_F32 = 0, 1
DAO_MASTER_APERTURE, DAO_MASTER_BEAMLET = 0, 1
DAO_DFMT_NATIVE, DAO_DFMT_F16, DAO_DFMT_BF16, DAO_DFMT_AUTO = 0, 1, 2, 3
DAO_DIR_STEEPEST, DAO_DIR_CONJUGATE = 0, 1
_NAMES = {0: "DAO_OK", 1: "DAO_EOPTIMAL", 2: "DAO_ESTALLED", 3: "DAO_ENOTCONV", -1: "DAO_EINVAL",
          -2: "DAO_ENOMEM",
          -3: "DAO_EDEVICE", -4: "DAO_ESTATE"}


class DaoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class dao_matrix(ctypes.Structure):
    _fields_ = [("n_vox", c_int64), ("n_blt", c_int64), ("nnz", c_int64),
                ("row_ptr", POINTER(c_int64)), ("col", POINTER(c_int32)), ("val", POINTER(c_double))]


class dao_beams(ctypes.Structure):
    _fields_ = [("n_beams", c_int32), ("rows_per_beam", POINTER(c_int32)), ("row_len", POINTER(c_int32))]


class dao_structures(ctypes.Structure):
    _fields_ = [("n_struct", c_int32), ("vox_struct", POINTER(c_int16)), ("vox_struct2", POINTER(c_int16)),
                ("vox_shift", POINTER(c_double))]


class dao_prescription(ctypes.Structure):
    _fields_ = [("is_target", c_int32), ("t_under", c_double), ("t_over", c_double),
                ("w_under", c_double), ("w_over", c_double)]


class dao_options(ctypes.Structure):
    _fields_ = [("dtype", c_int32), ("max_apertures", c_int32), ("eps", c_double),
                ("max_steps", c_int32), ("tau_rel", c_double), ("max_tighten", c_int32),
                ("refresh_every", c_int32), ("ls_slots", c_int32), ("mem_cap_bytes", c_int64),
                ("master", c_int32), ("d_format", c_int32), ("d_residual", c_int32),
                ("persistent", c_int32), ("product_tune", c_int32), ("dose_variant", c_int32),
                ("gradient_depth", c_int32), ("direction", c_int32), ("apertures_per_round", c_int32),
                ("dk_format", c_int32), ("residual_rounds", c_int32),
                ("graphs", c_int32)]


class dao_info_t(ctypes.Structure):
    _fields_ = [("n_vox", c_int64), ("n_vox_nonempty", c_int64), ("n_blt", c_int64), ("nnz", c_int64),
                ("n_rows", c_int64), ("n_beams", c_int32), ("max_rows_per_beam", c_int32),
                ("dtype", c_int32), ("n_slices", c_int32), ("sell_entries", c_int64),
                ("device_bytes", c_int64), ("d_format", c_int32), ("d_residual", c_int32),
                ("bytes_dose", c_int64), ("bytes_gradient", c_int64),
                ("dose_variant", c_int32), ("gradient_depth", c_int32), ("last_master_form", c_int32),
                ("onchip_lds_bytes", c_int32), ("dk_format", c_int32), ("residual_reprices", c_int32)]


class dao_server_options(ctypes.Structure):
    _fields_ = [("max_live", c_int32), ("batch_masters", c_int32), ("hbm_cap_bytes", c_int64),
                ("workers", c_int32)]


class dao_plan(ctypes.Structure):
    _fields_ = [("rounds", c_int32), ("stop", c_int32), ("F", c_double), ("rc1", c_double),
                ("total_steps", c_int64), ("total_ls_evals", c_int64),
                ("round_beam", POINTER(c_int32)), ("round_rc", POINTER(c_double)),
                ("round_gap", POINTER(c_double)), ("round_steps", POINTER(c_int32)),
                ("round_kkt", POINTER(c_double)), ("round_F", POINTER(c_double)),
                ("price_s", c_double), ("master_s", c_double),
                ("round_stop", POINTER(c_int32)), ("capped_rounds", c_int32)]


class dao_state_info(ctypes.Structure):
    _fields_ = [("n", c_int32), ("tighten", c_int32), ("rc1", c_double), ("eps", c_double),
                ("last_step", c_double), ("prev_step", c_double)]


# name -> (restype, argtypes); every symbol include/dao.h declares
_SIGS = {
    "dao_default_options": (None, [POINTER(dao_options)]),
    "dao_create": (c_int32, [POINTER(dao_matrix), POINTER(dao_beams), POINTER(dao_structures),
                             POINTER(dao_prescription), POINTER(dao_options), c_void_p, POINTER(c_void_p)]),
    "dao_destroy": (None, [c_void_p]),
    "dao_last_error": (c_char_p, [c_void_p]),
    "dao_create_error": (c_char_p, []),
    "dao_info": (c_int32, [c_void_p, POINTER(dao_info_t)]),
    "dao_dose": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "dao_gradient": (c_int32, [c_void_p, c_void_p, c_void_p, POINTER(c_double)]),
    "dao_price": (c_int32, [c_void_p, c_void_p, POINTER(c_int32), POINTER(c_int16),
                            POINTER(c_double), POINTER(c_double)]),
    "dao_price_noalloc": (c_int32, [c_void_p, c_void_p, POINTER(c_int32), POINTER(c_int16),
                                    POINTER(c_double), POINTER(c_double)]),
    "dao_reset": (c_int32, [c_void_p]),
    "dao_add_aperture": (c_int32, [c_void_p, c_int32, POINTER(c_int16)]),
    "dao_master_step": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_double), POINTER(c_double)]),
    "dao_master_solve": (c_int32, [c_void_p, c_double, c_int32, POINTER(c_int32), POINTER(c_double),
                                   POINTER(c_double)]),
    "dao_price_current": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int16), POINTER(c_double),
                                    POINTER(c_double)]),
    "dao_get_pool": (c_int32, [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int32), POINTER(c_int16),
                               POINTER(c_double)]),
    "dao_get_dose": (c_int32, [c_void_p, c_void_p, POINTER(c_double)]),
    "dao_solve": (c_int32, [c_void_p, c_int32, POINTER(dao_plan)]),
    "dao_solve_resume": (c_int32, [c_void_p, c_int32, POINTER(dao_plan)]),
    "dao_get_state": (c_int32, [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int16), POINTER(c_double),
                                POINTER(dao_state_info)]),
    "dao_set_state": (c_int32, [c_void_p, POINTER(dao_state_info), POINTER(c_int32), POINTER(c_int16),
                                POINTER(c_double)]),
    "dao_solve_batch": (c_int32, [POINTER(c_void_p), c_int32, POINTER(c_int32), POINTER(dao_plan)]),
    "dao_server_create": (c_int32, [c_void_p, c_void_p, POINTER(c_void_p)]),
    "dao_server_destroy": (None, [c_void_p]),
    "dao_server_submit": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32,
                                    POINTER(c_int64)]),
    "dao_server_step": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32)]),
    "dao_server_poll": (c_int32, [c_void_p, c_int64, POINTER(c_int32), POINTER(dao_plan)]),
    "dao_server_info": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int64)]),
    "dao_time_product": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_double)]),
    "dao_profile_phases": (c_int32, [c_void_p, POINTER(c_double)]),
    "dao_encode_values": (c_int32, [c_int32, c_int64, POINTER(c_double), POINTER(ctypes.c_uint16),
                                    POINTER(ctypes.c_uint16)]),
    "dao_time_product_cold": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_int64, POINTER(c_double)]),
    "dao_time_read_cold": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_void_p, c_int64, POINTER(c_double)]),
    "dao_profile_start": (c_int32, [c_void_p, c_int32]),
    "dao_profile_stop": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int64), POINTER(c_double),
                                   POINTER(c_double)]),
}

_lib = None


def symbols():
    return sorted(_SIGS)


def load_library(path: str = LIB_PATH):
    """Load libdao.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_1003_5402_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a, ctype):
    return a.ctypes.data_as(POINTER(ctype))


def encode_values(d_format: int, r, residual: bool = True):
    """The library's host encoder of 16-bit D storage: (hi, lo) uint16 patterns
    of the ratios r (lo None without residual)."""
    lib = load_library()
    r = np.ascontiguousarray(r, dtype=np.float64)
    hi = np.zeros(r.shape, dtype=np.uint16)
    lo = np.zeros(r.shape, dtype=np.uint16) if residual else None
    st = lib.dao_encode_values(int(d_format), r.size, _ptr(r, c_double), _ptr(hi, ctypes.c_uint16),
                               _ptr(lo, ctypes.c_uint16) if lo is not None else None)
    if st != DAO_OK:
        raise DaoError(st, "dao_encode_values rejected its arguments")
    return hi, lo


def _addr(v) -> int:
    """Device address of a torch tensor (or an int address)."""
    if isinstance(v, int):
        return v
    return int(v.data_ptr())


def _plan_arrays(n):
    n = max(1, int(n))
    arr = dict(round_beam=np.zeros(n, np.int32), round_rc=np.zeros(n), round_gap=np.zeros(n),
               round_steps=np.zeros(n, np.int32), round_kkt=np.zeros(n), round_F=np.zeros(n),
               round_stop=np.zeros(n, np.int32))
    P = dao_plan()
    for k, a in arr.items():
        setattr(P, k, _ptr(a, c_int32 if a.dtype == np.int32 else c_double))
    return P, arr


def _plan_dict(P, arr, st):
    r = P.rounds
    return dict(status=st, rounds=r, stop=P.stop, F=P.F, rc1=P.rc1, total_steps=P.total_steps,
                total_ls_evals=P.total_ls_evals, price_s=P.price_s, master_s=P.master_s,
                capped_rounds=P.capped_rounds, **{k: v[:r].copy() for k, v in arr.items()})


STOP_NAMES = {1: "kkt", 2: "step_cap", 3: "zero_direction"}


def write_round_log(plan: Dict, out, **meta) -> int:
    """One JSON line per round of a plan dict (from solve / solve_batch /
    the server): round, entering beam, reduced cost, decision gap, objective
    after the master, master steps, KKT residual and the master's stop
    reason.  `out` is a path (appended to) or a text file; `meta` is copied
    into every line.  Returns the number of lines written."""
    import json
    lines = []
    for k in range(int(plan["rounds"])):
        rec = dict(meta)
        rec.update(round=k, beam=int(plan["round_beam"][k]), rc=float(plan["round_rc"][k]),
                   gap=float(plan["round_gap"][k]), F=float(plan["round_F"][k]),
                   steps=int(plan["round_steps"][k]), kkt=float(plan["round_kkt"][k]),
                   stop=STOP_NAMES.get(int(plan["round_stop"][k]), int(plan["round_stop"][k])))
        lines.append(json.dumps(rec))
    text = "".join(line + "\n" for line in lines)
    if isinstance(out, (str, os.PathLike)):
        with open(out, "a") as f:
            f.write(text)
    else:
        out.write(text)
    return len(lines)


def solve_batch(ctxs, n_apertures) -> list:
    """dao_solve_batch over DaoContexts: one plan dict per context."""
    lib = load_library()
    n = len(ctxs)
    H = (c_void_p * n)(*[c._h for c in ctxs])
    na = np.ascontiguousarray(n_apertures, dtype=np.int32)
    plans = (dao_plan * n)()
    keep = []
    for i in range(n):
        P, arr = _plan_arrays(na[i])
        plans[i] = P
        keep.append(arr)
    st = lib.dao_solve_batch(H, n, _ptr(na, c_int32), plans)
    if st < 0:
        raise DaoError(st, lib.dao_last_error(ctxs[0]._h).decode())
    return [_plan_dict(plans[i], keep[i], int(plans[i].stop)) for i in range(n)]


def _structures(n_struct, vs, vox_struct2, vox_shift, keep):
    """dao_structures with the optional second labels and threshold shifts
    (NULL when absent); the arrays are appended to ``keep``."""
    S = dao_structures()
    S.n_struct = int(n_struct)
    S.vox_struct = _ptr(vs, c_int16)
    if vox_struct2 is not None:
        v2 = np.ascontiguousarray(vox_struct2, dtype=np.int16)
        keep.append(v2)
        S.vox_struct2 = _ptr(v2, c_int16)
    if vox_shift is not None:
        sh = np.ascontiguousarray(vox_shift, dtype=np.float64)
        keep.append(sh)
        S.vox_shift = _ptr(sh, c_double)
    return S


class DaoContext:
    """One plan's device state: dose matrix, structures, pool and master."""

    def __init__(self, row_ptr, col, val, n_blt: int, rows_per_beam, row_len, vox_struct,
                 prescriptions: Sequence[Dict], dtype: str = "f32", stream: int = 0, vox_struct2=None,
                 vox_shift=None, **opts):
        lib = load_library()
        self._lib = lib
        self._keep = []
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        vl = np.ascontiguousarray(val, dtype=np.float64)
        rpb = np.ascontiguousarray(rows_per_beam, dtype=np.int32)
        rl = np.ascontiguousarray(row_len, dtype=np.int32)
        vs = np.ascontiguousarray(vox_struct, dtype=np.int16)
        self._keep += [rp, cl, vl, rpb, rl, vs]
        M = dao_matrix(rp.shape[0] - 1, int(n_blt), cl.shape[0], _ptr(rp, c_int64), _ptr(cl, c_int32),
                       _ptr(vl, c_double))
        Bm = dao_beams(rpb.shape[0], _ptr(rpb, c_int32), _ptr(rl, c_int32))
        S = _structures(len(prescriptions), vs, vox_struct2, vox_shift, self._keep)
        PA = (dao_prescription * max(1, len(prescriptions)))()
        for i, p in enumerate(prescriptions):
            PA[i] = dao_prescription(int(p["is_target"]), p["t_under"], p["t_over"], p["w_under"], p["w_over"])
        O = dao_options()
        lib.dao_default_options(byref(O))
        O.dtype = DAO_F64 if dtype == "f64" else DAO_F32
        names = {f for f, _ in dao_options._fields_}
        for k, v in opts.items():
            if k not in names:
                raise TypeError(f"unknown option {k!r}")
            setattr(O, k, v)
        h = c_void_p()
        st = lib.dao_create(byref(M), byref(Bm), byref(S), PA, byref(O), c_void_p(stream), byref(h))
        if st != DAO_OK:
            raise DaoError(st, lib.dao_create_error().decode())
        self._h = h
        self.dtype = dtype
        self.n_vox = int(M.n_vox)
        self.n_blt = int(n_blt)
        self.rows_per_beam = rpb.copy()
        self.max_rows_per_beam = int(rpb.max())
        self.opts = O

    @classmethod
    def from_phantom(cls, ph, dtype: Optional[str] = None, stream: int = 0, **opts) -> "DaoContext":
        return cls(ph.row_ptr, ph.col, ph.val, ph.n_blt, ph.rows_per_beam, ph.row_len, ph.vox_struct,
                   ph.prescriptions, dtype=dtype or ph.dtype, stream=stream,
                   vox_struct2=getattr(ph, "vox_struct2", None), **opts)

    # -- helpers -------------------------------------------------------------
    def _check(self, st):
        if st < 0:
            raise DaoError(st, self._lib.dao_last_error(self._h).decode())
        return st

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dao_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls -----------------------------------------------------------------
    def info(self) -> Dict:
        i = dao_info_t()
        self._check(self._lib.dao_info(self._h, byref(i)))
        return {f: getattr(i, f) for f, _ in dao_info_t._fields_}

    def dose(self, x, d) -> None:
        self._check(self._lib.dao_dose(self._h, c_void_p(_addr(x)), c_void_p(_addr(d))))

    def gradient(self, d, g) -> float:
        F = c_double()
        self._check(self._lib.dao_gradient(self._h, c_void_p(_addr(d)), c_void_p(_addr(g)), byref(F)))
        return F.value

    def _price_out(self):
        beam = c_int32()
        lv = np.zeros(2 * self.max_rows_per_beam, dtype=np.int16)
        rc, gap = c_double(), c_double()
        return beam, lv, rc, gap

    def _price_result(self, beam, lv, rc, gap):
        nr = int(self.rows_per_beam[beam.value])
        leaves = tuple((int(lv[2 * i]), int(lv[2 * i + 1])) for i in range(nr))
        return dict(beam=beam.value, leaves=leaves, rc=rc.value, gap=gap.value)

    def price(self, g64) -> Dict:
        beam, lv, rc, gap = self._price_out()
        self._check(self._lib.dao_price(self._h, c_void_p(_addr(g64)), byref(beam), _ptr(lv, c_int16),
                                        byref(rc), byref(gap)))
        return self._price_result(beam, lv, rc, gap)

    def price_noalloc(self, g64) -> Dict:
        """dao_price_noalloc: dao_price with the library's static scratch."""
        beam, lv, rc, gap = self._price_out()
        self._check(self._lib.dao_price_noalloc(self._h, c_void_p(_addr(g64)), byref(beam), _ptr(lv, c_int16),
                                                byref(rc), byref(gap)))
        return self._price_result(beam, lv, rc, gap)

    def price_current(self) -> Dict:
        beam, lv, rc, gap = self._price_out()
        self._check(self._lib.dao_price_current(self._h, byref(beam), _ptr(lv, c_int16), byref(rc),
                                                byref(gap)))
        return self._price_result(beam, lv, rc, gap)

    def reset(self) -> None:
        self._check(self._lib.dao_reset(self._h))

    def add_aperture(self, beam: int, leaves) -> None:
        lv = np.zeros(2 * self.max_rows_per_beam, dtype=np.int16)
        flat = np.asarray(leaves, dtype=np.int16).reshape(-1)
        lv[:flat.shape[0]] = flat
        self._check(self._lib.dao_add_aperture(self._h, int(beam), _ptr(lv, c_int16)))

    def master_step(self):
        F, kkt, step = c_double(), c_double(), c_double()
        self._check(self._lib.dao_master_step(self._h, byref(F), byref(kkt), byref(step)))
        return F.value, kkt.value, step.value

    def master_solve(self, tol: float, max_steps: int):
        """(steps, kkt, F); ``self.last_master_capped`` tells whether the step
        cap ended the solve (DAO_ENOTCONV)."""
        steps, kkt, F = c_int32(), c_double(), c_double()
        st = self._check(self._lib.dao_master_solve(self._h, float(tol), int(max_steps), byref(steps),
                                                    byref(kkt), byref(F)))
        self.last_master_capped = st == DAO_ENOTCONV
        return steps.value, kkt.value, F.value

    def get_state(self, cap: int = 256) -> Dict:
        """Pool, intensities and loop scalars (dao_get_state)."""
        beams = np.zeros(cap, dtype=np.int32)
        lv = np.zeros(cap * 2 * self.max_rows_per_beam, dtype=np.int16)
        y = np.zeros(cap, dtype=np.float64)
        info = dao_state_info()
        self._check(self._lib.dao_get_state(self._h, cap, _ptr(beams, c_int32), _ptr(lv, c_int16),
                                            _ptr(y, c_double), byref(info)))
        n = info.n
        lv = lv.reshape(cap, self.max_rows_per_beam, 2)
        pool = [(int(beams[i]), tuple((int(a), int(b)) for a, b in lv[i, :int(self.rows_per_beam[beams[i]])]))
                for i in range(n)]
        return dict(pool=pool, y=y[:n].copy(), rc1=info.rc1, eps=info.eps, tighten=info.tighten,
                    last_step=info.last_step, prev_step=info.prev_step)

    def set_state(self, pool, y, rc1: float = float("nan"), eps: Optional[float] = None, tighten: int = 0,
                  last_step: float = 0.0, prev_step: float = 0.0) -> None:
        """Restore a pool [(beam, ((L, R), ...)), ...] and intensities (dao_set_state)."""
        n = len(pool)
        m = max(1, n)
        beams = np.zeros(m, dtype=np.int32)
        lv = np.zeros((m, self.max_rows_per_beam, 2), dtype=np.int16)
        for i, (b, leaves) in enumerate(pool):
            beams[i] = int(b)
            fl = np.asarray(leaves, dtype=np.int16).reshape(-1, 2)
            lv[i, :fl.shape[0]] = fl
        yv = np.zeros(m, dtype=np.float64)
        yv[:n] = np.asarray(y, dtype=np.float64)[:n]
        info = dao_state_info(n, int(tighten), float(rc1), float(eps if eps is not None else self.opts.eps),
                              float(last_step), float(prev_step))
        self._check(self._lib.dao_set_state(self._h, byref(info), _ptr(beams, c_int32),
                                            _ptr(lv.reshape(-1), c_int16), _ptr(yv, c_double)))

    def get_pool(self, cap: int = 256):
        n = c_int32()
        beams = np.zeros(cap, dtype=np.int32)
        lv = np.zeros(cap * 2 * self.max_rows_per_beam, dtype=np.int16)
        y = np.zeros(cap, dtype=np.float64)
        self._check(self._lib.dao_get_pool(self._h, cap, byref(n), _ptr(beams, c_int32), _ptr(lv, c_int16),
                                           _ptr(y, c_double)))
        k = min(n.value, cap)
        lv = lv.reshape(cap, self.max_rows_per_beam, 2)
        pool = []
        for i in range(k):
            nr = int(self.rows_per_beam[beams[i]])
            pool.append((int(beams[i]), tuple((int(a), int(b)) for a, b in lv[i, :nr])))
        return pool, y[:k].copy()

    def get_dose(self, d64=None) -> float:
        F = c_double()
        self._check(self._lib.dao_get_dose(self._h, c_void_p(_addr(d64) if d64 is not None else 0),
                                           byref(F)))
        return F.value

    def time_product(self, kernel: int, iters: int) -> float:
        """Mean microseconds per launch of product kernel 0 (D x) or 1 (D^T u)."""
        us = c_double()
        self._check(self._lib.dao_time_product(self._h, int(kernel), int(iters), byref(us)))
        return us.value

    def time_product_cold(self, kernel: int, iters: int, scrub) -> float:
        """As time_product, with a read of the device tensor `scrub` (its
        whole size) before every timed launch to evict the caches."""
        us = c_double()
        nbytes = scrub.numel() * scrub.element_size()
        self._check(self._lib.dao_time_product_cold(self._h, int(kernel), int(iters), c_void_p(_addr(scrub)),
                                                    c_int64(nbytes), byref(us)))
        return us.value

    def time_read_cold(self, buf, nbytes: int, iters: int, scrub) -> float:
        """dao_time_read_cold: a plain streaming read of the first `nbytes`
        bytes of device tensor `buf`, timed cold as time_product_cold."""
        us = c_double()
        sbytes = scrub.numel() * scrub.element_size()
        self._check(self._lib.dao_time_read_cold(self._h, c_void_p(_addr(buf)), c_int64(nbytes), int(iters),
                                                 c_void_p(_addr(scrub)), c_int64(sbytes), byref(us)))
        return us.value

    def profile_phases(self) -> Dict:
        """Persistent master: microseconds per phase in the last profiling window."""
        us = (c_double * 7)()
        self._check(self._lib.dao_profile_phases(self._h, us))
        names = ["update", "update_reduce", "direction", "ls_first_pass", "ls_reduce", "decide_step",
                 "ls_later_passes"]
        return {n: float(us[i]) for i, n in enumerate(names)}

    def profile_start(self, kernel: int) -> None:
        self._check(self._lib.dao_profile_start(self._h, int(kernel)))

    def profile_stop(self) -> Dict:
        n, w, us, b = c_int64(), c_int64(), c_double(), c_double()
        self._check(self._lib.dao_profile_stop(self._h, byref(n), byref(w), byref(us), byref(b)))
        return dict(launches=n.value, working_launches=w.value, total_us=us.value, total_bytes=b.value)

    def solve(self, n_apertures: int, round_log=None) -> Dict:
        """dao_solve; with `round_log` (a path or text file) the per-round
        records are appended to it as JSON lines (write_round_log)."""
        P, arr = _plan_arrays(n_apertures)
        st = self._check(self._lib.dao_solve(self._h, int(n_apertures), byref(P)))
        plan = _plan_dict(P, arr, st)
        if round_log is not None:
            write_round_log(plan, round_log)
        return plan

    def solve_resume(self, n_apertures: int) -> Dict:
        """Column generation continued from the current pool (dao_solve_resume)."""
        P, arr = _plan_arrays(n_apertures)
        st = self._check(self._lib.dao_solve_resume(self._h, int(n_apertures), byref(P)))
        return _plan_dict(P, arr, st)


class Server:
    """The library's serving loop (dao_server_*): queue requests, step rounds,
    poll results.  Keeps each request's host arrays alive until it is done."""

    def __init__(self, max_live: int = 8, hbm_cap_bytes: int = 0, stream: int = 0, batch_masters: bool = True,
                 workers: int = 0):
        self._lib = load_library()
        o = dao_server_options(int(max_live), int(bool(batch_masters)), int(hbm_cap_bytes), int(workers))
        h = c_void_p()
        st = self._lib.dao_server_create(byref(o), c_void_p(stream), byref(h))
        if st != DAO_OK:
            raise DaoError(st, "dao_server_create rejected its options")
        self._h = h
        self._keep = {}
        self._n_ap = {}

    def submit(self, ph, n_apertures: int, dtype: Optional[str] = None, **opts) -> int:
        rp = np.ascontiguousarray(ph.row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(ph.col, dtype=np.int32)
        vl = np.ascontiguousarray(ph.val, dtype=np.float64)
        rpb = np.ascontiguousarray(ph.rows_per_beam, dtype=np.int32)
        rl = np.ascontiguousarray(ph.row_len, dtype=np.int32)
        vs = np.ascontiguousarray(ph.vox_struct, dtype=np.int16)
        M = dao_matrix(rp.shape[0] - 1, int(ph.n_blt), cl.shape[0], _ptr(rp, c_int64), _ptr(cl, c_int32),
                       _ptr(vl, c_double))
        Bm = dao_beams(rpb.shape[0], _ptr(rpb, c_int32), _ptr(rl, c_int32))
        extra = []
        S = _structures(len(ph.prescriptions), vs, getattr(ph, "vox_struct2", None), None, extra)
        PA = (dao_prescription * max(1, len(ph.prescriptions)))()
        for i, p in enumerate(ph.prescriptions):
            PA[i] = dao_prescription(int(p["is_target"]), p["t_under"], p["t_over"], p["w_under"], p["w_over"])
        O = dao_options()
        self._lib.dao_default_options(byref(O))
        O.dtype = DAO_F64 if (dtype or ph.dtype) == "f64" else DAO_F32
        names = {f for f, _ in dao_options._fields_}
        for k, v in opts.items():
            if k not in names:
                raise TypeError(f"unknown option {k!r}")
            setattr(O, k, v)
        t = c_int64()
        st = self._lib.dao_server_submit(self._h, byref(M), byref(Bm), byref(S), PA, byref(O), int(n_apertures),
                                         byref(t))
        if st != DAO_OK:
            raise DaoError(st, "dao_server_submit rejected the request")
        self._keep[t.value] = (rp, cl, vl, rpb, rl, vs, M, Bm, S, PA, O, extra)
        self._n_ap[t.value] = int(n_apertures)
        return t.value

    def step(self):
        nl, nd = c_int32(), c_int32()
        st = self._lib.dao_server_step(self._h, byref(nl), byref(nd))
        if st < 0:
            raise DaoError(st, "dao_server_step failed")
        return nl.value, nd.value

    def poll(self, ticket: int):
        """(state, plan dict or None): state 0 queued, 1 live, 2 done."""
        P, arr = _plan_arrays(self._n_ap.get(ticket, 1))
        state = c_int32()
        st = self._lib.dao_server_poll(self._h, int(ticket), byref(state), byref(P))
        if state.value != 2:
            if st < 0:
                raise DaoError(st, "unknown ticket")
            return state.value, None
        self._keep.pop(ticket, None)
        self._n_ap.pop(ticket, None)
        return 2, _plan_dict(P, arr, int(st))

    def info(self):
        q, l, u = c_int32(), c_int32(), c_int64()
        self._lib.dao_server_info(self._h, byref(q), byref(l), byref(u))
        return dict(queued=q.value, live=l.value, used_bytes=u.value)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dao_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

