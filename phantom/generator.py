"""Synthetic anatomy, beams and pencil-beam dose matrix (inputs only).

Geometry and conventions
------------------------
* Voxel grid ``(nx, ny, nz)`` of cubic voxels with edge ``h`` mm.  Voxel
  ``j = (iz * ny + iy) * nx + ix`` has its centre at
  ``((ix + 0.5) h, (iy + 0.5) h, (iz + 0.5) h)``.  Every grid voxel is a row of
  D, so rows of voxels outside the body (or outside every beam) are empty.
* Beams are coplanar, parallel, in the axial (x, y) plane.  Beam ``b`` has
  gantry angle ``theta_b = b * 360 / B`` degrees.  With
  ``e = (cos theta, sin theta)`` pointing from the isocentre to the source, a
  point ``p`` has travel coordinate ``s = -(p - iso).e`` (grows along the
  beam), lateral coordinate ``u = (p - iso).(-sin theta, cos theta)`` and axial
  coordinate ``zz = p_z - iso_z``.
* Each beam is cut into 5 mm x 5 mm beamlets on a grid centred on the
  isocentre.  Grid row ``r`` (an MLC leaf pair) sits at
  ``zz_r = (r + 0.5 - nrows / 2) * 5`` and grid column ``c`` at
  ``u_c = (c + 0.5 - ncols / 2) * 5``.  Leaves move along ``u``.
* Beamlets are numbered beam-major, then leaf row, then position within the
  row, so each MLC row is a contiguous run of beamlet indices (the per-row
  pricing of Section 2.3 scans such runs).
* Active beamlets: either the whole grid, or (when ``active='ptv'``) every
  beamlet whose central ray passes within 5 mm of a PTV voxel centre, with
  each row then filled to the convex span of its active beamlets so that rows
  are contiguous; rows without an active beamlet are dropped.

Pencil-beam kernel (stand-in for the dose engine the paper uses)::

    D_ij = exp(-0.005 * depth) * exp(-rho^2 / (2 sigma^2))
           if rho <= 10 mm, depth >= 0 and voxel j lies in the body, else 0

where ``rho`` is the distance from voxel centre j to the central ray of
beamlet i and ``depth = s_j - s_in(i)`` is measured along the beam from the
point where beamlet i's central ray enters the body.

Structures carry one label per voxel (PTV first, then organs at risk in the
listed order, then normal tissue = rest of the body); ``-1`` marks voxels
outside the body.  With ``nested_targets`` the target is split as in the
paper's head-and-neck cases: a boost target PTV1 inside a larger PTV2; PTV1
voxels carry PTV1 as first label and PTV2 as second label
(``vox_struct2``), the rest of PTV2 carries PTV2.  Prescriptions follow the per-structure objective of the
Discussion (eq. 9 and eq. 10): targets have under- and over-dose thresholds
and weights, other structures over-dose only.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np
import scipy.sparse as sp

BEAMLET_MM = 5.0
TRUNC_MM = 10.0
MU_PER_MM = 0.005


# --------------------------------------------------------------------------
# body outline (z-invariant)
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Body:
    """A z-invariant body: an axis-aligned box or an axis-aligned ellipse."""

    kind: str                 # "box" or "ellipse"
    center: np.ndarray        # (2,) mm, x and y
    half: np.ndarray          # (2,) mm, half extents (box) or semi-axes

    def contains(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        dx = x - self.center[0]
        dy = y - self.center[1]
        if self.kind == "box":
            return (np.abs(dx) <= self.half[0]) & (np.abs(dy) <= self.half[1])
        return (dx / self.half[0]) ** 2 + (dy / self.half[1]) ** 2 <= 1.0

    def entry(self, p0: np.ndarray, dv: np.ndarray) -> float:
        """Smallest s with p0 + s*dv inside the outline (nan if the line misses)."""
        q = np.asarray(p0, dtype=np.float64) - self.center
        dv = np.asarray(dv, dtype=np.float64)
        if self.kind == "box":
            lo, hi = -math.inf, math.inf
            for a in range(2):
                if abs(dv[a]) < 1e-15:
                    if abs(q[a]) > self.half[a]:
                        return math.nan
                    continue
                t1 = (-self.half[a] - q[a]) / dv[a]
                t2 = (self.half[a] - q[a]) / dv[a]
                lo = max(lo, min(t1, t2))
                hi = min(hi, max(t1, t2))
            return lo if lo <= hi else math.nan
        ax, ay = self.half
        a = (dv[0] / ax) ** 2 + (dv[1] / ay) ** 2
        b = 2.0 * (q[0] * dv[0] / ax ** 2 + q[1] * dv[1] / ay ** 2)
        c = (q[0] / ax) ** 2 + (q[1] / ay) ** 2 - 1.0
        disc = b * b - 4 * a * c
        if disc < 0:
            return math.nan
        return (-b - math.sqrt(disc)) / (2 * a)


# --------------------------------------------------------------------------
# the phantom record
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Phantom:
    name: str
    seed: int
    shape: tuple              # (nx, ny, nz)
    h: float                  # voxel edge, mm
    iso: np.ndarray           # (3,) isocentre, mm
    body: Body
    sigma_mm: float
    beam_angles: np.ndarray   # (B,) radians
    grid_rows: int            # beamlet grid size per beam
    grid_cols: int
    # beamlet table, in beamlet-number order
    beamlet_beam: np.ndarray  # (N,) int32
    beamlet_grow: np.ndarray  # (N,) int32 grid row
    beamlet_gcol: np.ndarray  # (N,) int32 grid column
    rows_per_beam: np.ndarray  # (B,) int32
    row_len: np.ndarray       # (R,) int32
    # dose matrix, CSR over all grid voxels
    row_ptr: np.ndarray       # (V+1,) int64
    col: np.ndarray           # (nnz,) int32, sorted within each row
    val: np.ndarray           # (nnz,) float64 (float32-representable if dtype=f32)
    dtype: str                # "f64" or "f32": storage precision of D
    # structures and prescriptions
    vox_struct: np.ndarray    # (V,) int16, -1 = none
    struct_names: List[str]
    prescriptions: List[Dict]  # per structure: is_target, t_under, t_over, w_under, w_over
    n_apertures: int
    vox_struct2: Optional[np.ndarray] = None   # (V,) int16 second label (nested targets), -1 = none

    @property
    def n_vox(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def n_blt(self) -> int:
        return int(self.beamlet_beam.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def n_beams(self) -> int:
        return int(self.rows_per_beam.shape[0])

    @property
    def n_rows(self) -> int:
        return int(self.row_len.shape[0])

    def csr(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr),
                             shape=(self.n_vox, self.n_blt))

    def voxel_centers(self, idx: Optional[np.ndarray] = None) -> np.ndarray:
        nx, ny, nz = self.shape
        if idx is None:
            idx = np.arange(nx * ny * nz, dtype=np.int64)
        ix = idx % nx
        iy = (idx // nx) % ny
        iz = idx // (nx * ny)
        return np.stack([(ix + 0.5) * self.h, (iy + 0.5) * self.h,
                         (iz + 0.5) * self.h], axis=1)

    def beamlet_axis(self, i: int):
        """(angle, u_c, zz_r) of beamlet i's central ray."""
        b = int(self.beamlet_beam[i])
        u_c = (self.beamlet_gcol[i] + 0.5 - self.grid_cols / 2.0) * BEAMLET_MM
        z_r = (self.beamlet_grow[i] + 0.5 - self.grid_rows / 2.0) * BEAMLET_MM
        return float(self.beam_angles[b]), float(u_c), float(z_r)

    def row_beam(self) -> np.ndarray:
        return np.repeat(np.arange(self.n_beams, dtype=np.int32), self.rows_per_beam)

    def structure_mask(self, name: str) -> np.ndarray:
        return self.vox_struct == self.struct_names.index(name)

    def summary(self) -> Dict:
        nz_rows = int(np.count_nonzero(np.diff(self.row_ptr)))
        return dict(name=self.name, seed=self.seed, shape=list(self.shape),
                    n_vox=self.n_vox, n_vox_nonempty=nz_rows, n_blt=self.n_blt,
                    n_beams=self.n_beams, n_rows=self.n_rows,
                    max_row_len=int(self.row_len.max()), nnz=self.nnz,
                    dtype=self.dtype, n_apertures=self.n_apertures,
                    struct_sizes={n: int(np.count_nonzero(self.vox_struct == k))
                                  for k, n in enumerate(self.struct_names)})


# --------------------------------------------------------------------------
# shapes evaluated at voxel centres
# --------------------------------------------------------------------------
def _ellipsoid(P, c, semi):
    return (((P[:, 0] - c[0]) / semi[0]) ** 2 + ((P[:, 1] - c[1]) / semi[1]) ** 2
            + ((P[:, 2] - c[2]) / semi[2]) ** 2) <= 1.0


def _cylinder_z(P, cxy, r):
    return (P[:, 0] - cxy[0]) ** 2 + (P[:, 1] - cxy[1]) ** 2 <= r * r


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------
CONFIGS: Dict[str, Dict] = {
    # reduced case for fast CPU tests: not a benchmark workload
    "mini": dict(shape=(20, 20, 12), h=2.5, n_beams=3, grid=(4, 4), active="all",
                 sigma=4.0, body=("box", None), anatomy="sphere_cyl",
                 ptv_r=9.0, oar_r=5.0, oar_off=15.0, dtype="f64", n_apertures=6),
    # 32^3 at 2.5 mm, sphere PTV r=15 mm, cylinder OAR r=8 mm, 5 beams of 8x8
    "tiny": dict(shape=(32, 32, 32), h=2.5, n_beams=5, grid=(8, 8), active="all",
                 sigma=4.0, body=("box", None), anatomy="sphere_cyl",
                 ptv_r=15.0, oar_r=8.0, oar_off=25.5, dtype="f64", n_apertures=10),
    # prostate-shaped: 150x100x60, ellipsoid PTV, bladder + rectum, 9 beams
    "prostate": dict(shape=(150, 100, 60), h=2.5, n_beams=9, grid=(16, 24),
                     active="ptv", sigma=4.0, body=("ellipse", (90.0, 80.0)),
                     anatomy="prostate", dtype="f32", n_apertures=50),
    # head-and-neck-shaped: 200x200x100, 3-ellipsoid PTV, 6 OARs, 5 beams
    "headneck": dict(shape=(200, 200, 100), h=2.5, n_beams=5, grid=(50, 44),
                     active="ptv", sigma=3.5, body=("ellipse", (160.0, 140.0)),
                     anatomy="headneck", dtype="f32", n_apertures=50),
}

NT_T_OVER = 0.5
NT_W_OVER = 0.1


def _presc(is_target, t_under, t_over, w_under, w_over):
    return dict(is_target=int(is_target), t_under=float(t_under), t_over=float(t_over),
                w_under=float(w_under), w_over=float(w_over))


# nested targets: PTV1 (boost) prescription 1.0, PTV2 54/73.8 of it
# (Section 3's head-and-neck prescriptions, normalised to PTV1); PTV2 also
# contains PTV1, so its over-dose threshold is PTV1's
PTV2_T_UNDER = 54.0 / 73.8
PTV1_SCALE = 0.6


def _nest(out):
    """Split the first (target) entry into PTV1 (a shrunk copy of its first
    component, passed as out[0][3]) and PTV2 (the whole target)."""
    name, ptv, pr, ptv1 = out[0]
    return [("PTV1", ptv1 & ptv, _presc(1, 1.0, 1.0, 1.0, 1.0)),
            ("PTV2", ptv, _presc(1, PTV2_T_UNDER, 1.0, 1.0, 1.0))] + [o[:3] for o in out[1:]]


def _anatomy(kind, cfg, P, iso, rng, shift, ptv_scale):
    """Return (list of (name, mask, prescription, boost mask)) in priority
    order; the boost mask (a shrunk copy of the target's first component) is
    used only for nested targets."""
    out = []
    c = iso + shift
    if kind == "sphere_cyl":
        ptv = _ellipsoid(P, c, [cfg["ptv_r"] * ptv_scale] * 3)
        boost = _ellipsoid(P, c, [cfg["ptv_r"] * ptv_scale * PTV1_SCALE] * 3)
        # organ-at-risk cylinder along z, posterior (+y) of the isocentre
        oar = _cylinder_z(P, (iso[0], iso[1] + cfg["oar_off"]), cfg["oar_r"])
        out.append(("PTV", ptv, _presc(1, 1.0, 1.0, 1.0, 1.0), boost))
        out.append(("OAR", oar, _presc(0, 0.0, 0.5, 0.0, 0.5), None))
    elif kind == "prostate":
        semi = np.array([35.0, 25.0, 25.0]) * ptv_scale
        ptv = _ellipsoid(P, c, semi)
        # bladder tangent anteriorly (-y), rectum tangent posteriorly (+y)
        bl_semi = np.array([30.0, 25.0, 25.0])
        re_semi = np.array([15.0, 15.0, 30.0])
        bladder = _ellipsoid(P, c + np.array([0.0, -(semi[1] + bl_semi[1]), 0.0]), bl_semi)
        rectum = _ellipsoid(P, c + np.array([0.0, semi[1] + re_semi[1], 0.0]), re_semi)
        out.append(("PTV", ptv, _presc(1, 1.0, 1.0, 1.0, 1.0), _ellipsoid(P, c, semi * PTV1_SCALE)))
        out.append(("bladder", bladder, _presc(0, 0.0, 0.5, 0.0, 0.5), None))
        out.append(("rectum", rectum, _presc(0, 0.0, 0.5, 0.0, 0.5), None))
    elif kind == "headneck":
        ptv = np.zeros(P.shape[0], dtype=bool)
        boost = None
        for _ in range(3):
            # lateral semi-axes U[20, 40] mm; elongated along z (nodal chains run
            # superior-inferior) with a z semi-axis U[40, 75] mm; centres within
            # 20 mm of the isocentre in the axial plane and U[-40, 40] mm in z
            semi = np.array([rng.uniform(20.0, 40.0), rng.uniform(20.0, 40.0),
                             rng.uniform(40.0, 75.0)]) * ptv_scale
            d2 = rng.normal(size=2)
            d2 *= rng.uniform(0.0, 20.0) / max(np.linalg.norm(d2), 1e-12)
            d = np.array([d2[0], d2[1], rng.uniform(-40.0, 40.0)])
            ptv |= _ellipsoid(P, c + d, semi)
            if boost is None:
                boost = _ellipsoid(P, c + d, semi * PTV1_SCALE)
        out.append(("PTV", ptv, _presc(1, 1.0, 1.0, 1.0, 1.0), boost))
        thr = rng.uniform(0.4, 0.7, size=6)
        cord = _cylinder_z(P, (iso[0], iso[1] + 60.0), 6.0)
        stem = _ellipsoid(P, iso + np.array([0.0, 45.0, 70.0]), [12.0, 12.0, 20.0])
        lpar = _ellipsoid(P, iso + np.array([-45.0, 10.0, 25.0]), [12.0, 15.0, 20.0])
        rpar = _ellipsoid(P, iso + np.array([45.0, 10.0, 25.0]), [12.0, 15.0, 20.0])
        oars = [("cord", cord), ("brainstem", stem), ("parotid_l", lpar),
                ("parotid_r", rpar)]
        for k in range(2):
            for _ in range(1000):
                r = rng.uniform(6.0, 15.0)
                cc = iso + rng.uniform([-70.0, -70.0, -60.0], [70.0, 70.0, 60.0])
                m = _ellipsoid(P, cc, [r, r, r])
                if not np.any(m & ptv):
                    break
            oars.append((f"sphere{k}", m))
        for (name, m), t in zip(oars, thr):
            out.append((name, m, _presc(0, 0.0, t, 0.0, 0.5), None))
    else:
        raise ValueError(kind)
    return out


def make_phantom(name: str = "tiny", seed: int = 0, *, shift_mm=(0.0, 0.0, 0.0),
                 ptv_scale: float = 1.0, n_apertures: Optional[int] = None,
                 dtype: Optional[str] = None, body_half: Optional[Sequence[float]] = None,
                 normal_tissue: bool = True, nested_targets: bool = False) -> Phantom:
    """Build a seeded phantom.

    ``name`` picks an entry of :data:`CONFIGS`.  ``shift_mm`` rigidly moves the
    target (not the beams), ``ptv_scale`` scales it; both serve re-planning
    variants.  ``normal_tissue`` adds the over-dose term on the body outside
    all listed structures.  ``nested_targets`` splits the target into PTV1
    inside PTV2 (see the module docstring).
    """
    cfg = CONFIGS[name]
    rng = np.random.default_rng(seed)
    nx, ny, nz = cfg["shape"]
    h = float(cfg["h"])
    V = nx * ny * nz
    center = np.array([nx * h / 2, ny * h / 2, nz * h / 2])
    iso = center + rng.uniform(-0.5, 0.5, size=3) * h
    kind, half = cfg["body"]
    if body_half is not None:
        half = tuple(body_half)
    if kind == "box":
        body = Body("box", center[:2].copy(), np.array([nx * h / 2, ny * h / 2]))
    else:
        body = Body("ellipse", center[:2].copy(), np.array(half, dtype=np.float64))

    # ---- voxel centres and labels --------------------------------------
    idx = np.arange(V, dtype=np.int64)
    ix = idx % nx
    iy = (idx // nx) % ny
    iz = idx // (nx * ny)
    P = np.stack([(ix + 0.5) * h, (iy + 0.5) * h, (iz + 0.5) * h], axis=1)
    inside = body.contains(P[:, 0], P[:, 1])
    structs = _anatomy(cfg["anatomy"], cfg, P, iso, rng,
                       np.asarray(shift_mm, dtype=np.float64), float(ptv_scale))
    structs = _nest(structs) if nested_targets else [o[:3] for o in structs]
    vox_struct = np.full(V, -1, dtype=np.int16)
    names, prescs = [], []
    for k, (nm, m, pr) in enumerate(structs):
        sel = m & inside & (vox_struct < 0)
        vox_struct[sel] = k
        names.append(nm)
        prescs.append(pr)
    vox_struct2 = None
    if nested_targets:
        # PTV1 voxels also belong to PTV2 (structure 1)
        vox_struct2 = np.full(V, -1, dtype=np.int16)
        vox_struct2[(vox_struct == 0) & structs[1][1]] = 1
    if normal_tissue:
        k = len(names)
        vox_struct[inside & (vox_struct < 0)] = k
        names.append("NT")
        prescs.append(_presc(0, 0.0, NT_T_OVER, 0.0, NT_W_OVER))
    targets = [k for k, pr in enumerate(prescs) if pr["is_target"]]
    ptv_idx = np.flatnonzero(np.isin(vox_struct, targets))

    # ---- beams and active beamlets -------------------------------------
    B = int(cfg["n_beams"])
    grows, gcols = cfg["grid"]
    angles = np.arange(B) * (2.0 * math.pi / B)
    ucs = (np.arange(gcols) + 0.5 - gcols / 2.0) * BEAMLET_MM
    zrs = (np.arange(grows) + 0.5 - grows / 2.0) * BEAMLET_MM
    bl_map = []            # per beam: (grows, gcols) -> global beamlet index or -1
    bl_beam, bl_grow, bl_gcol, rows_per_beam, row_len = [], [], [], [], []
    n = 0
    for b, th in enumerate(angles):
        if cfg["active"] == "all":
            act = np.ones((grows, gcols), dtype=bool)
        else:
            rel = P[ptv_idx] - iso
            u = -rel[:, 0] * math.sin(th) + rel[:, 1] * math.cos(th)
            zz = rel[:, 2]
            act = np.zeros((grows, gcols), dtype=bool)
            for r in range(grows):
                dz2 = (zz - zrs[r]) ** 2
                near = dz2 <= BEAMLET_MM ** 2
                if not near.any():
                    continue
                un, dzn = u[near], dz2[near]
                for cc in range(gcols):
                    act[r, cc] = bool(np.any((un - ucs[cc]) ** 2 + dzn <= BEAMLET_MM ** 2))
        m = np.full((grows, gcols), -1, dtype=np.int64)
        nrows_b = 0
        for r in range(grows):
            cs = np.flatnonzero(act[r])
            if cs.size == 0:
                continue
            lo, hi = int(cs.min()), int(cs.max()) + 1
            m[r, lo:hi] = np.arange(n, n + hi - lo)
            bl_beam += [b] * (hi - lo)
            bl_grow += [r] * (hi - lo)
            bl_gcol += list(range(lo, hi))
            row_len.append(hi - lo)
            n += hi - lo
            nrows_b += 1
        rows_per_beam.append(nrows_b)
        bl_map.append(m)

    # ---- pencil-beam dose matrix ---------------------------------------
    sigma = float(cfg["sigma"])
    rows_l, cols_l, vals_l = [], [], []
    body_idx = np.flatnonzero(inside)
    Pb = P[body_idx] - iso
    for b, th in enumerate(angles):
        ct, st = math.cos(th), math.sin(th)
        e = np.array([ct, st])
        lat = np.array([-st, ct])
        s_in = np.array([body.entry(iso[:2] + uc * lat, -e) for uc in ucs])
        s = -(Pb[:, 0] * ct + Pb[:, 1] * st)
        u = -Pb[:, 0] * st + Pb[:, 1] * ct
        zz = Pb[:, 2]
        c0 = np.floor(u / BEAMLET_MM + gcols / 2.0).astype(np.int64)
        r0 = np.floor(zz / BEAMLET_MM + grows / 2.0).astype(np.int64)
        m = bl_map[b]
        for dr in range(-2, 3):
            rr = r0 + dr
            okr = (rr >= 0) & (rr < grows)
            for dc in range(-2, 3):
                cc = c0 + dc
                ok = okr & (cc >= 0) & (cc < gcols)
                sel = np.flatnonzero(ok)
                if sel.size == 0:
                    continue
                gi = m[rr[sel], cc[sel]]
                ok2 = gi >= 0
                sel, gi = sel[ok2], gi[ok2]
                du = u[sel] - ucs[cc[sel]]
                dz = zz[sel] - zrs[rr[sel]]
                rho2 = du * du + dz * dz
                depth = s[sel] - s_in[cc[sel]]
                keep = (rho2 <= TRUNC_MM * TRUNC_MM) & (depth >= 0.0) & np.isfinite(depth)
                sel, gi, rho2, depth = sel[keep], gi[keep], rho2[keep], depth[keep]
                v = np.exp(-MU_PER_MM * depth) * np.exp(-rho2 / (2.0 * sigma * sigma))
                rows_l.append(body_idx[sel])
                cols_l.append(gi)
                vals_l.append(v)
    rows = np.concatenate(rows_l) if rows_l else np.zeros(0, np.int64)
    cols = np.concatenate(cols_l) if cols_l else np.zeros(0, np.int64)
    vals = np.concatenate(vals_l) if vals_l else np.zeros(0)
    dtype = dtype or cfg["dtype"]
    if dtype == "f32":
        vals = vals.astype(np.float32).astype(np.float64)
    A = sp.coo_matrix((vals, (rows, cols)), shape=(V, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return Phantom(
        name=name, seed=seed, shape=(nx, ny, nz), h=h, iso=iso, body=body,
        sigma_mm=sigma, beam_angles=angles, grid_rows=grows, grid_cols=gcols,
        beamlet_beam=np.asarray(bl_beam, np.int32), beamlet_grow=np.asarray(bl_grow, np.int32),
        beamlet_gcol=np.asarray(bl_gcol, np.int32),
        rows_per_beam=np.asarray(rows_per_beam, np.int32), row_len=np.asarray(row_len, np.int32),
        row_ptr=A.indptr.astype(np.int64), col=A.indices.astype(np.int32),
        val=A.data.astype(np.float64), dtype=dtype, vox_struct=vox_struct,
        struct_names=names, prescriptions=prescs,
        n_apertures=int(n_apertures if n_apertures is not None else cfg["n_apertures"]),
        vox_struct2=vox_struct2)
