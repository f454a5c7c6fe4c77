"""Restricted master problem by gradient projection (test infrastructure).

Section 2.3 solves the master -- the objective over the current pool of
apertures with y >= 0 -- by the gradient projection method: move along the
negative gradient, projected so that the intensities stay non-negative.  The
paper takes the method from its earlier fluence-map work and gives no step
rule, tolerance or iteration cap; Section 2.2 and Section 2.3 only require
that the master find the optimal intensities of the pool.  This module fixes
one reading of those details, and the HIP path follows the same reading:

* gradient over the pool:   grad_k = sum_{i in A_k} g_i,  g = D^T grad F(d)
* projected negative gradient r: r_k = -grad_k, except r_k = 0 where y_k = 0
  and grad_k >= 0 (moving would leave the feasible set); the apertures with
  r_k allowed to be non-zero form the free set
* direction p (``conjugate=True``, the default): p = r + beta p_prev with
  beta = max(0, r.(r - r_prev) / r_prev.r_prev) (Polak-Ribiere, truncated at
  0), taken only when the previous step of this pool exists, did not block
  (t < t_max) and had the same free set, and only if it is a descent
  direction (grad.p < 0); otherwise p = r.  This is Polyak's conjugate
  gradient projection: on a fixed face of the constraints and a fixed piece
  of F it is the conjugate gradient method, which reaches the face's minimum
  in at most |free set| steps, while the plain projected steepest descent
  (``conjugate=False``: always p = r) zig-zags and may need thousands.
* longest feasible step:    t_max = min over p_k < 0 of y_k / (-p_k)
* exact line search of the convex piecewise quadratic phi(t) = F(d + t q),
  q = D (A p), on [0, t_max]   (see :func:`line_search`)
* update y += t p (apertures that block at t = t_max are set to exactly 0)
  and d += t q; every 50 steps d is recomputed as D (A y)
* stop when the KKT residual max_k |min(y_k, grad_k)| <= tol, or after
  ``max_steps`` steps.

The memory of the conjugate direction (previous p, r and free set) belongs
to the master state: it is cleared when an aperture enters the pool and after
a step that blocks, and kept across the 50-step dose recomputation and
across consecutive solves of the same pool.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from .aperture import Aperture, aperture_gradient, beamlet_intensity
from .model import Problem, dose, grad_objective, objective, prices

REFRESH_EVERY = 50
LS_MAX_ITER = 60


def _slopes(P: Problem, z: np.ndarray, q: np.ndarray):
    """phi''(t) just right and just left of t: sum_j q_j^2 times the active curvature."""
    q2 = q * q
    s_r = s_l = 0.0
    for a, tu, b, to in P.terms():
        ua = a > 0
        ob = b > 0
        under_r = ua & ((z < tu) | ((z == tu) & (q < 0)))
        over_r = ob & ((z > to) | ((z == to) & (q > 0)))
        under_l = ua & ((z < tu) | ((z == tu) & (q > 0)))
        over_l = ob & ((z > to) | ((z == to) & (q < 0)))
        s_r += 2.0 * float(np.sum(q2 * (a * under_r + b * over_r)))
        s_l += 2.0 * float(np.sum(q2 * (a * under_l + b * over_l)))
    return s_r, s_l


def _breakpoints(P: Problem, d: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Values of t at which some voxel's dose d_j + t q_j meets one of its thresholds."""
    nz = q != 0
    out = []
    for a, tu, b, to in P.terms():
        out.append((tu - d)[nz & (a > 0)] / q[nz & (a > 0)])
        out.append((to - d)[nz & (b > 0)] / q[nz & (b > 0)])
    return np.concatenate(out)


def line_search(P: Problem, d: np.ndarray, q: np.ndarray, t_max: float,
                max_iter: int = LS_MAX_ITER):
    """Exact minimiser of phi(t) = F(d + t q) over 0 <= t <= t_max.

    phi is convex and piecewise quadratic, so phi' is continuous, monotone
    and piecewise linear, with kinks only where a voxel's dose crosses one of
    its thresholds.  Safeguarded Newton on phi':
      evaluate phi'(t), the slopes of phi' on both sides of t and the nearest
      breakpoints on both sides; if the Newton point from t stays inside the
      current linear piece it is the exact root and is returned; otherwise it
      becomes the next trial point (bisecting the bracket if it falls
      outside).  The result is t_max when phi' < 0 all the way to t_max.
    Returns ``(t, evaluations)``.  Requires phi'(0) < 0.
    """
    bps = _breakpoints(P, d, q)
    lo, hi = 0.0, float(t_max)
    hi_known = False           # has phi'(hi) > 0 been seen?
    t = 0.0
    for it in range(1, max_iter + 1):
        z = d + t * q
        gphi = float(np.sum(q * grad_objective(P, z)))
        s_r, s_l = _slopes(P, z, q)
        right = bps[bps > t]
        left = bps[bps < t]
        nb = float(right.min()) if right.size else math.inf
        pb = float(left.max()) if left.size else -math.inf
        if gphi == 0.0:
            return t, it
        if gphi < 0.0:
            if t >= t_max:
                return float(t_max), it
            lo = t
            tn = t - gphi / s_r if s_r > 0.0 else math.inf
            if tn <= nb:                       # root inside the current piece
                return min(tn, float(t_max)), it
            if nb >= t_max:                    # phi' < 0 all the way to t_max
                return float(t_max), it
            if tn < hi:
                nxt = tn
            elif not hi_known:
                nxt = hi                       # try the blocking step itself
            else:
                nxt = 0.5 * (lo + hi)
            if math.isinf(nxt):                # flat piece, open bracket
                nxt = nb
        else:
            hi, hi_known = t, True
            tn = t - gphi / s_l if s_l > 0.0 else -math.inf
            if tn >= pb:                       # root inside the current piece
                return max(tn, lo), it
            nxt = tn if tn > lo else 0.5 * (lo + hi)
        t = nxt
    return lo, max_iter


@dataclasses.dataclass
class MasterState:
    pool: List[Aperture]
    y: np.ndarray
    d: np.ndarray
    u: np.ndarray
    g: np.ndarray
    # conjugate-direction memory: direction, projected gradient and free set
    # of the last step (None: the next step starts from r)
    p_prev: Optional[np.ndarray] = None
    r_prev: Optional[np.ndarray] = None
    free_prev: Optional[np.ndarray] = None

    def forget_direction(self) -> None:
        self.p_prev = self.r_prev = self.free_prev = None

    @classmethod
    def empty(cls, P: Problem) -> "MasterState":
        d = np.zeros(P.n_vox)
        u = grad_objective(P, d)
        return cls(pool=[], y=np.zeros(0), d=d, u=u, g=prices(P, u))

    def refresh(self, P: Problem) -> None:
        """Recompute d, grad F and g from y (removes incremental drift in d)."""
        self.d = dose(P, beamlet_intensity(P, self.pool, self.y))
        self.u = grad_objective(P, self.d)
        self.g = prices(P, self.u)

    def add(self, ap: Aperture) -> None:
        self.pool.append(ap)
        self.y = np.append(self.y, 0.0)
        self.forget_direction()


def kkt_residual(y: np.ndarray, grad: np.ndarray) -> float:
    """max_k |min(y_k, grad_k)|: zero exactly at a KKT point of min F, y >= 0."""
    if y.size == 0:
        return 0.0
    return float(np.max(np.abs(np.minimum(y, grad))))


def _ratios(y: np.ndarray, p: np.ndarray) -> np.ndarray:
    r = np.full(p.shape, math.inf)
    neg = p < 0.0
    r[neg] = y[neg] / (-p[neg])
    return r


def max_step(y: np.ndarray, p: np.ndarray) -> float:
    """Longest step keeping y + t p >= 0: min over p_k < 0 of y_k / (-p_k)."""
    return float(_ratios(y, p).min()) if p.size else math.inf


def take_step(y: np.ndarray, p: np.ndarray, t: float) -> np.ndarray:
    """y + t p, with the apertures that block at t = t_max set to exactly 0."""
    r = _ratios(y, p)
    out = y + t * p
    if p.size and t == float(r.min()):
        out[r == t] = 0.0
    return np.maximum(out, 0.0)


def direction(st: MasterState, grad: np.ndarray, conjugate: bool = True):
    """Search direction p and the projected negative gradient r and free set
    it came from (see the module docstring)."""
    free = ~((st.y == 0.0) & (grad >= 0.0))
    r = np.where(free, -grad, 0.0)
    p = r
    if (conjugate and st.r_prev is not None and st.r_prev.shape == r.shape
            and np.array_equal(free, st.free_prev)):
        beta = max(0.0, float(np.dot(r, r - st.r_prev)) / float(np.dot(st.r_prev, st.r_prev)))
        cand = r + beta * st.p_prev
        if float(np.dot(grad, cand)) < 0.0:
            p = cand
    return p, r, free


def master_step(P: Problem, st: MasterState, conjugate: bool = True) -> Optional[dict]:
    """One gradient-projection iteration in place.  Returns its record, or
    None when the projected negative gradient is zero (an exact KKT point)."""
    grad = aperture_gradient(P, st.pool, st.g)
    p, r, free = direction(st, grad, conjugate)
    if not np.any(r != 0.0):
        return None
    t_max = max_step(st.y, p)
    q = dose(P, beamlet_intensity(P, st.pool, p))
    t, evals = line_search(P, st.d, q, t_max)
    st.y = take_step(st.y, p, t)
    st.d = st.d + t * q
    st.u = grad_objective(P, st.d)
    st.g = prices(P, st.u)
    if t == t_max:
        st.forget_direction()
    else:
        st.p_prev, st.r_prev, st.free_prev = p, r, free
    return dict(t=t, t_max=t_max, ls_evals=evals, gphi0=float(np.dot(grad, p)))


def solve_master(P: Problem, st: MasterState, tol: float, max_steps: int = 500,
                 track_F: bool = False, conjugate: bool = True):
    """Iterate :func:`master_step` until the KKT residual is at most ``tol``
    or ``max_steps`` steps were taken.  Returns a log dict."""
    Fs = [objective(P, st.d)] if track_F else []
    steps, evals = 0, 0
    kkt = kkt_residual(st.y, aperture_gradient(P, st.pool, st.g))
    while kkt > tol and steps < max_steps:
        rec = master_step(P, st, conjugate)
        if rec is None:
            break
        steps += 1
        evals += rec["ls_evals"]
        if steps % REFRESH_EVERY == 0:
            st.refresh(P)
        if track_F:
            Fs.append(objective(P, st.d))
        kkt = kkt_residual(st.y, aperture_gradient(P, st.pool, st.g))
    return dict(steps=steps, kkt=kkt, ls_evals=evals, F_trace=Fs)
