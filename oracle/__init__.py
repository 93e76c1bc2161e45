"""FP64 CPU oracle for the per-projection PCA solve -- TEST INFRASTRUCTURE.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package; the product path never does.
It shares no code with the HIP library.

The primitives (projection P, its transpose, Eq. 1, the warp of Eqs. A.3/A.5,
the Jacobian of Eq. A.8, the tumour-position inversion) are plain C in
``pcas_oracle.c``; this module adds the intensity fit (Eq. A.1), the objective
(Eq. 2), the gradient chain of the Appendix, and the two solvers:

* ``solve_paper`` -- the Appendix algorithm: alternate the closed-form (a, b)
  of Eq. A.1 with a normalised gradient step (Eq. A.2) whose step size comes
  from Armijo backtracking (mu0, alpha, beta as stated there), stopping when
  the step falls below mu_min or after max_iter iterations.
* ``solve_cg`` -- the nonlinear conjugate-gradient variant (not in the paper):
  Polak-Ribiere+ directions on the reduced objective min_{a,b} J, with the
  same Armijo rule.
* ``solve_bfgs`` -- a quasi-Newton variant (not in the paper): BFGS updates of
  a dense K x K inverse-Hessian estimate on the same reduced objective, with
  the same Armijo rule and the unit quasi-Newton step tried first.

All arithmetic is float64.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")

# ---------------------------------------------------------------------------
# ctypes plumbing
# ---------------------------------------------------------------------------


class _Vol(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("spacing", ctypes.c_double * 3),
                ("origin", ctypes.c_double * 3)]


class _Proj(ctypes.Structure):
    _fields_ = [("angle", ctypes.c_double), ("sad", ctypes.c_double), ("sid", ctypes.c_double),
                ("nu", ctypes.c_int32), ("nv", ctypes.c_int32),
                ("pitch_u", ctypes.c_double), ("pitch_v", ctypes.c_double),
                ("offset_u", ctypes.c_double), ("offset_v", ctypes.c_double),
                ("step", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b  # type: ignore
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        VP, PP = ctypes.POINTER(_Vol), ctypes.POINTER(_Proj)
        L.orc_drr_forward.argtypes = [VP, PP, P, P]
        L.orc_drr_pixels.argtypes = [VP, PP, P, ctypes.c_int64, P, P]
        L.orc_drr_adjoint.argtypes = [VP, PP, P, P]
        L.orc_pca_dvf.argtypes = [ctypes.c_int64, ctypes.c_int32, P, P, P, P]
        L.orc_warp.argtypes = [VP, P, P, P]
        L.orc_warp_jacobian.argtypes = [VP, P, P, P]
        L.orc_grad_chain.argtypes = [ctypes.c_int64, ctypes.c_int32, P, P, P, P]
        L.orc_locate.argtypes = [VP, ctypes.c_int32, P, P, P, P, ctypes.c_double, ctypes.c_int32, P]
        L.orc_locate.restype = ctypes.c_int32
        L.orc_ray_table.argtypes = [VP, PP, P, P, P, P]
        L.orc_siddon_forward.argtypes = [VP, PP, P, P]
        _lib = L
    return _lib


def _vol(vol) -> _Vol:
    v = _Vol()
    for c in range(3):
        v.n[c] = int(vol.n[c])
        v.spacing[c] = float(vol.spacing[c])
        v.origin[c] = float(vol.origin[c])
    return v


def _proj(pr) -> _Proj:
    return _Proj(float(pr.angle), float(pr.sad), float(pr.sid), int(pr.nu), int(pr.nv),
                 float(pr.pitch_u), float(pr.pitch_v), float(getattr(pr, "offset_u", 0.0)),
                 float(getattr(pr, "offset_v", 0.0)), float(pr.step))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _nvox(vol) -> int:
    return int(vol.n[0]) * int(vol.n[1]) * int(vol.n[2])


# ---------------------------------------------------------------------------
# primitives
# ---------------------------------------------------------------------------

def drr_forward(vol, proj, f) -> np.ndarray:
    """P f (Eq. 2), shape [nv][nu]."""
    f = _f64(f).reshape(-1)
    assert f.size == _nvox(vol)
    p = np.empty((int(proj.nv), int(proj.nu)))
    lib().orc_drr_forward(ctypes.byref(_vol(vol)), ctypes.byref(_proj(proj)), _ptr(f), _ptr(p))
    return p


def drr_pixels(vol, proj, f, pix) -> np.ndarray:
    """Selected entries (flat pixel indices iu + nu*iv) of P f."""
    f = _f64(f).reshape(-1)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    out = np.empty(pix.size)
    lib().orc_drr_pixels(ctypes.byref(_vol(vol)), ctypes.byref(_proj(proj)), _ptr(f),
                         int(pix.size), _ptr(pix), _ptr(out))
    return out


def drr_adjoint(vol, proj, r) -> np.ndarray:
    """P^T r, shape [n3][n2][n1]."""
    r = _f64(r).reshape(-1)
    assert r.size == int(proj.nu) * int(proj.nv)
    bp = np.empty(tuple(int(v) for v in (vol.n[2], vol.n[1], vol.n[0])))
    lib().orc_drr_adjoint(ctypes.byref(_vol(vol)), ctypes.byref(_proj(proj)), _ptr(r), _ptr(bp))
    return bp


def pca_dvf(vol, mean, U, w) -> np.ndarray:
    """Eq. 1, shape [3][n3][n2][n1] (mm)."""
    N = _nvox(vol)
    U = _f64(U)
    K = U.size // (3 * N)
    mean = None if mean is None else _f64(mean)
    w = _f64(w).reshape(-1)
    assert w.size == K
    x = np.empty((3,) + tuple(int(v) for v in (vol.n[2], vol.n[1], vol.n[0])))
    lib().orc_pca_dvf(N, K, _ptr(mean), _ptr(U), _ptr(w), _ptr(x))
    return x


def warp(vol, f0, x) -> np.ndarray:
    """Eqs. A.3 / A.5: f = f0 at (index + x / spacing), zero outside."""
    f0 = _f64(f0)
    x = _f64(x)
    f = np.empty(tuple(int(v) for v in (vol.n[2], vol.n[1], vol.n[0])))
    lib().orc_warp(ctypes.byref(_vol(vol)), _ptr(f0), _ptr(x), _ptr(f))
    return f


def warp_jacobian(vol, f0, x) -> np.ndarray:
    """Eq. A.8 and analogues, per mm, shape [3][n3][n2][n1]."""
    f0 = _f64(f0)
    x = _f64(x)
    jac = np.empty((3,) + tuple(int(v) for v in (vol.n[2], vol.n[1], vol.n[0])))
    lib().orc_warp_jacobian(ctypes.byref(_vol(vol)), _ptr(f0), _ptr(x), _ptr(jac))
    return jac


def grad_chain(vol, U, jac, bp) -> np.ndarray:
    """dJ/dw = 2 U^T (df/dx) P^T r (Appendix), given jac = df/dx, bp = P^T r."""
    N = _nvox(vol)
    U = _f64(U)
    K = U.size // (3 * N)
    g = np.empty(K)
    lib().orc_grad_chain(N, K, _ptr(U), _ptr(_f64(jac)), _ptr(_f64(bp)), _ptr(g))
    return g


def grad_w(vol, f0, mean, U, w, bp) -> np.ndarray:
    """The K-vector 2 U^T (df/dx) bp at coefficients w."""
    x = pca_dvf(vol, mean, U, w)
    return grad_chain(vol, U, warp_jacobian(vol, f0, x), bp)


def locate(vol, mean, U, w, c0, tol: float = 1e-9, max_iter: int = 100):
    """Tumour position: fixed point y = c0 - x(y) at one point (mm)."""
    N = _nvox(vol)
    U = _f64(U)
    K = U.size // (3 * N)
    mean = None if mean is None else _f64(mean)
    out = np.empty(3)
    it = lib().orc_locate(ctypes.byref(_vol(vol)), K, _ptr(mean), _ptr(U), _ptr(_f64(w)),
                          _ptr(_f64(c0)), float(tol), int(max_iter), _ptr(out))
    return out, int(it)


def siddon_forward(vol, proj, f) -> np.ndarray:
    """Exact-path projection of the voxel-constant volume (Siddon's method),
    shape [nv][nu]."""
    p = np.empty(int(proj.nu) * int(proj.nv))
    lib().orc_siddon_forward(ctypes.byref(_vol(vol)), ctypes.byref(_proj(proj)), _ptr(_f64(f)),
                             _ptr(p))
    return p.reshape(int(proj.nv), int(proj.nu))


def ray_table(vol, proj):
    """(t_in, length, nsamp, dt) per pixel, each shaped [nv][nu]."""
    M = int(proj.nu) * int(proj.nv)
    t_in, length, dt = np.empty(M), np.empty(M), np.empty(M)
    ns = np.empty(M, dtype=np.int64)
    lib().orc_ray_table(ctypes.byref(_vol(vol)), ctypes.byref(_proj(proj)), _ptr(t_in),
                        _ptr(length), _ptr(ns), _ptr(dt))
    sh = (int(proj.nv), int(proj.nu))
    return t_in.reshape(sh), length.reshape(sh), ns.reshape(sh), dt.reshape(sh)


def total_samples(vol, proj) -> int:
    return int(ray_table(vol, proj)[2].sum())


# ---------------------------------------------------------------------------
# Eq. A.1 and Eq. 2
# ---------------------------------------------------------------------------

class SingularFit(ValueError):
    pass


def intensity_fit(p, y):
    """Eq. A.1: (a, b) = (Y^T Y)^{-1} Y^T p with Y = [y, 1]."""
    p = _f64(p).reshape(-1)
    y = _f64(y).reshape(-1)
    M = float(y.size)
    syy, sy = float(y @ y), float(y.sum())
    syp, sp = float(y @ p), float(p.sum())
    det = syy * M - sy * sy
    if not (abs(det) > 1e-12 * syy * M):
        raise SingularFit("Y^T Y is singular (constant measured projection)")
    a = (M * syp - sy * sp) / det
    b = (syy * sp - sy * syp) / det
    return a, b


# ---------------------------------------------------------------------------
# solvers
# ---------------------------------------------------------------------------

STOP_CONVERGED, STOP_MAXITER, STOP_LINESEARCH = 0, 1, 2


@dataclass
class SolveOptions:
    """method 0: the Appendix algorithm (Eq. A.1 alternated with Eq. A.2 and
    Armijo); method 1: PR+ nonlinear CG on the reduced objective; method 2:
    BFGS on the reduced objective.

    The Appendix states mu0 = 2, alpha = 0.1, beta = 0.5, a stop when the step
    drops below 0.1, and at most 10 iterations, for coefficients scaled to a
    standard deviation of 10.  Our modes carry unit-variance coefficients, so
    the paper-mode step sizes are scaled by 1/10 (mu0 = 0.2, mu_min = 0.01).

    In CG and BFGS modes the line search (_line_search) shrinks a failed
    Armijo trial to the minimiser of the quadratic through phi(0), phi'(0)
    and phi(t), kept within [beta_lo * t, beta * t], and may lengthen an
    accepted first trial once (ls_extrap); mu_min is unused there.

    polish: when a CG or BFGS solve ends at the noise floor (the noise or
    decrement stop, or a failed search), one more step w - H g is tried with
    an inverse-Hessian estimate H (BFGS's own; CG keeps one from its steps by
    the same updates) and kept if it lowers ||g||.  The gradient stays
    accurate far below the noise of J, so this reaches the minimiser more
    closely than comparisons of J can."""
    method: int = 1
    max_iter: int = 30
    fit_intensity: bool = True
    max_backtracks: int = 12
    mu0: float = 1.0
    alpha: float = 0.1
    beta: float = 0.5
    mu_min: float = 0.01
    gtol_rel: float = 1e-9
    beta_lo: float = 0.1
    xtol: float = 1e-10
    ftol_rel: float = 1e-14
    ls_extrap: float = 10.0
    polish: bool = False

    @staticmethod
    def paper() -> "SolveOptions":
        return SolveOptions(method=0, max_iter=10, mu0=0.2, alpha=0.1, beta=0.5, mu_min=0.01)


@dataclass
class SolveReport:
    status: int = STOP_MAXITER
    iters: int = 0
    n_fevals: int = 0
    n_grads: int = 0
    J0: float = float("nan")
    J: float = float("nan")
    a: float = 1.0
    b: float = 0.0
    gnorm: float = float("nan")
    J_trace: List[float] = field(default_factory=list)


class Problem:
    """One projection: reference image, motion model, geometry, measurement."""

    def __init__(self, vol, proj, f0, mean, U, y, fit_intensity: bool = True):
        self.vol, self.proj = vol, proj
        self.f0 = _f64(f0)
        self.mean = None if mean is None else _f64(mean)
        self.U = _f64(U)
        self.K = self.U.size // (3 * _nvox(vol))
        self.y = _f64(y).reshape(int(proj.nv), int(proj.nu))
        self.fit = bool(fit_intensity)

    def project(self, w):
        """f = warp(f0, xbar + U w) and p = P f."""
        x = pca_dvf(self.vol, self.mean, self.U, w)
        f = warp(self.vol, self.f0, x)
        return f, drr_forward(self.vol, self.proj, f)

    def fit_ab(self, p):
        return intensity_fit(p, self.y) if self.fit else (1.0, 0.0)

    def objective(self, w, ab=None):
        """J at w.  With ab=None, (a, b) is refitted (Eq. A.1) first; returns
        (J, a, b, residual)."""
        _, p = self.project(w)
        a, b = self.fit_ab(p) if ab is None else ab
        r = p - a * self.y - b
        return float(np.sum(r * r)), a, b, r

    def gradient(self, w, r):
        """dJ/dw at fixed (a, b) for the residual r (Appendix)."""
        bp = drr_adjoint(self.vol, self.proj, r)
        return grad_w(self.vol, self.f0, self.mean, self.U, w, bp)


def solve_paper(prob: Problem, w0, opts: Optional[SolveOptions] = None):
    """The Appendix algorithm (Eqs. A.1, A.2 and Armijo's rule)."""
    o = opts or SolveOptions.paper()
    w = _f64(w0).copy()
    rep = SolveReport()
    _, p = prob.project(w)
    rep.n_fevals += 1
    for it in range(o.max_iter):
        a, b = prob.fit_ab(p)                          # step 1 (Eq. A.1)
        r = p - a * prob.y - b
        J = float(np.sum(r * r))
        if it == 0:
            rep.J0 = J
        rep.J_trace.append(J)
        rep.a, rep.b, rep.J = a, b, J
        g = prob.gradient(w, r)
        rep.n_grads += 1
        gn = float(np.linalg.norm(g))
        rep.gnorm = gn
        if gn == 0.0 or J == 0.0:
            rep.status = STOP_CONVERGED
            return w, rep
        d = g / gn                                     # step 2 (Eq. A.2)
        mu = o.mu0
        while True:
            w_try = w - mu * d
            J_try, _, _, _ = prob.objective(w_try, ab=(a, b))
            rep.n_fevals += 1
            if J_try <= J - o.alpha * mu * gn:        # Armijo, directional slope -||g||
                break
            mu *= o.beta
            if mu < o.mu_min:                         # step too small: stop, no update
                rep.status = STOP_CONVERGED
                rep.iters = it
                return w, rep
        w = w_try
        rep.iters = it + 1
        _, p = prob.project(w)
    a, b = prob.fit_ab(p)
    r = p - a * prob.y - b
    rep.a, rep.b, rep.J = a, b, float(np.sum(r * r))
    rep.J_trace.append(rep.J)
    rep.status = STOP_MAXITER
    return w, rep


def _line_search(prob, o, w, phi, d, gd, t):
    """Armijo search along d from w (phi = J(w), gd = g.d < 0), first trial
    step t, shared by solve_cg and solve_bfgs.

    A trial with phi_t <= phi + alpha t gd is accepted.  A rejected one moves
    t to the minimiser of the quadratic through phi(0), phi'(0) = gd and
    phi(t), kept within [beta_lo t, beta t]; a rejected trial whose change is
    within ftol_rel of phi ends the search at the noise floor, and a step
    shorter than xtol (in units of w) or max_backtracks trials fail it.

    When the first trial is accepted and that quadratic puts its minimiser
    beyond twice the trial step, one more trial is made there (capped at
    ls_extrap times the step; ls_extrap = 0 turns this off) and the lower of
    the two points is kept: backtracking can only shorten a step, so a first
    guess that is too short would otherwise stay short.

    Returns (status, t, w_t, phi_t, a_t, b_t, r_t, n_evals) with status
    "ok", "noise" or "fail"."""
    dn = float(np.linalg.norm(d))
    n = 0
    for trial in range(o.max_backtracks):
        if t * dn < o.xtol:                            # step too short to matter
            break
        w_t = w + t * d
        phi_t, a_t, b_t, r_t = prob.objective(w_t)
        n += 1
        if phi_t <= phi + o.alpha * t * gd:
            if trial == 0 and o.ls_extrap > 0.0:
                t_q = -gd * t * t / (2.0 * (phi_t - phi - gd * t))
                if t_q > 2.0 * t:
                    t_x = min(t_q, o.ls_extrap * t)
                    w_x = w + t_x * d
                    phi_x, a_x, b_x, r_x = prob.objective(w_x)
                    n += 1
                    if phi_x < phi_t:
                        return "ok", t_x, w_x, phi_x, a_x, b_x, r_x, n
            return "ok", t, w_t, phi_t, a_t, b_t, r_t, n
        if abs(phi_t - phi) <= o.ftol_rel * phi:       # change below rounding noise
            return "noise", t, None, None, None, None, None, n
        t_q = -gd * t * t / (2.0 * (phi_t - phi - gd * t))
        t = min(max(t_q, o.beta_lo * t), o.beta * t)
    return "fail", t, None, None, None, None, None, n


def curvature_update(B, s, y):
    """Direct BFGS update of a Hessian estimate (Nocedal and Wright,
    Numerical Optimization, Eq. 6.19): B+ = B - (B s)(B s)^T / (s.B s) +
    y y^T / (y.s).  B+ satisfies the secant equation B+ s = y and stays
    symmetric positive definite when y.s > 0."""
    Bs = B @ s
    return B - np.outer(Bs, Bs) / float(s @ Bs) + np.outer(y, y) / float(y @ s)


def _curvature_estimate(B, s_k, y_k):
    """solve_cg's curvature estimate after an accepted step: (y.y / y.s) I at
    the first usable pair (the reciprocal of Eq. 6.20's scaling), then
    curvature_update; pairs with y.s <= 1e-12 |s| |y| skipped."""
    sy = float(s_k @ y_k)
    if sy > 1e-12 * float(np.linalg.norm(s_k)) * float(np.linalg.norm(y_k)):
        if B is None:
            B = (float(y_k @ y_k) / sy) * np.eye(s_k.size)
        B = curvature_update(B, s_k, y_k)
    return B


def solve_cg(prob: Problem, w0, opts: Optional[SolveOptions] = None):
    """PR+ nonlinear CG on phi(w) = min_{a,b} J(w, a, b).

    phi's gradient is dJ/dw at the fitted (a, b) (the fit is an exact
    minimiser, Eq. A.1).  The directions are PR+ CG's; each is searched
    with _line_search.  Its first trial step minimises the quadratic model
    along d: t = -(g.d) / (d.B d), with B the curvature estimate that
    _curvature_estimate builds from the accepted steps s and gradient
    changes y.  Before B exists the first trial is mu0/||d|| on the first
    iteration, else t = -(g.d) / (c ||d||^2) with the curvature c =
    (s.y) / (s.s) the last accepted step measured, or, when s.y <= 0,
    t_prev (g_prev.d_prev) / (g.d).

    With the model's first trial, its predicted decrease -(g.d) t / 2 within
    ftol_rel of phi ends the solve as converged when the model is trusted:
    the last accepted decrease was within ftol_rel of phi too, or, for a
    step accepted at the model's first trial, within a factor 2 of the
    decrease predicted for it (solve_bfgs's stop).  A failed search restarts
    along -g once; a second failure ends the solve."""
    o = opts or SolveOptions()
    w = _f64(w0).copy()
    rep = SolveReport()
    phi, a, b, r = prob.objective(w)
    rep.n_fevals += 1
    g = prob.gradient(w, r)
    rep.n_grads += 1
    rep.J0 = phi
    rep.J_trace.append(phi)
    g0 = float(np.linalg.norm(g))
    d = -g
    restart, first = True, True
    t_prev = gd_prev = 0.0
    curv = 0.0                                         # (s.y) / (s.s) of the last accepted step
    B = None                                           # curvature estimate
    H = None                                           # for the polish step only
    last_drop, last_pred = float("inf"), -1.0
    floor = False                                      # ended at the noise floor
    it = 0
    rep.status = STOP_MAXITER
    while it < o.max_iter:
        gn = float(np.linalg.norm(g))
        if gn <= o.gtol_rel * g0 or phi == 0.0:
            rep.status = STOP_CONVERGED
            break
        gd = float(g @ d)
        if gd >= 0.0:                                  # not a descent direction
            d = -g
            gd = -gn * gn
            restart = True
        dbd = float(d @ (B @ d)) if B is not None else 0.0
        pred = -1.0
        if dbd > 0.0:
            t = -gd / dbd
            pred = -0.5 * gd * t
            if pred <= o.ftol_rel * phi and (
                    last_drop <= o.ftol_rel * phi or 0.5 * last_pred <= last_drop <= 2.0 * last_pred):
                rep.status = STOP_CONVERGED
                floor = True
                break
        elif first:
            t = o.mu0 / float(np.linalg.norm(d))
        elif curv > 0.0:
            t = -gd / (curv * float(d @ d))
        else:
            t = t_prev * gd_prev / gd
        t0 = t
        st, t, w_t, phi_t, a_t, b_t, r_t, n = _line_search(prob, o, w, phi, d, gd, t)
        rep.n_fevals += n
        if st == "noise":
            rep.status = STOP_CONVERGED
            floor = True
            break
        if st == "fail":
            if restart:
                rep.status = STOP_LINESEARCH
                floor = True
                break
            d = -g
            restart = True
            continue
        g_new = prob.gradient(w_t, r_t)
        rep.n_grads += 1
        s_k, y_k = w_t - w, g_new - g
        ss = float(s_k @ s_k)
        curv = float(s_k @ y_k) / ss if ss > 0.0 else 0.0
        B = _curvature_estimate(B, s_k, y_k)
        if o.polish:
            H = _hessian_update(H, s_k, y_k)
        last_pred = pred if t == t0 else -1.0
        last_drop = phi - phi_t
        w, phi, a, b, r = w_t, phi_t, a_t, b_t, r_t
        beta_pr = max(0.0, float(g_new @ (g_new - g)) / float(g @ g))
        d = -g_new + beta_pr * d
        t_prev, gd_prev = t, gd
        g = g_new
        restart, first = False, False
        it += 1
        rep.J_trace.append(phi)
    if floor and o.polish:
        w, phi, a, b, g = _polish(prob, H, w, phi, a, b, g, rep)
    rep.iters = it
    rep.J, rep.a, rep.b = phi, a, b
    rep.gnorm = float(np.linalg.norm(g))
    return w, rep


def bfgs_update(H, s, y):
    """Inverse-Hessian BFGS update (Nocedal and Wright, Numerical
    Optimization, Eq. 6.17): H+ = (I - rho s y^T) H (I - rho y s^T) +
    rho s s^T with rho = 1 / (y.s).  H+ satisfies the secant equation
    H+ y = s and stays symmetric positive definite when y.s > 0."""
    n = s.size
    rho = 1.0 / float(y @ s)
    L = np.eye(n) - rho * np.outer(s, y)
    return L @ H @ L.T + rho * np.outer(s, s)


def _hessian_update(H, s_k, y_k):
    """The estimate's update after an accepted step (solve_bfgs's rule; also
    kept by solve_cg for the polish step): scaled identity at the first
    usable pair, then bfgs_update; pairs with y.s <= 1e-12 |s| |y| skipped."""
    sy = float(s_k @ y_k)
    if sy > 1e-12 * float(np.linalg.norm(s_k)) * float(np.linalg.norm(y_k)):
        if H is None:
            H = (sy / float(y_k @ y_k)) * np.eye(s_k.size)
        H = bfgs_update(H, s_k, y_k)
    return H


def _polish(prob, H, w, phi, a, b, g, rep):
    """One step w - H g, kept if ||g|| drops (SolveOptions.polish)."""
    if H is None:
        return w, phi, a, b, g
    d = -(H @ g)
    if float(g @ d) >= 0.0:
        return w, phi, a, b, g
    w_p = w + d
    phi_p, a_p, b_p, r_p = prob.objective(w_p)
    rep.n_fevals += 1
    g_p = prob.gradient(w_p, r_p)
    rep.n_grads += 1
    if float(np.linalg.norm(g_p)) < float(np.linalg.norm(g)):
        return w_p, phi_p, a_p, b_p, g_p
    return w, phi, a, b, g


def solve_bfgs(prob: Problem, w0, opts: Optional[SolveOptions] = None):
    """BFGS on phi(w) = min_{a,b} J(w, a, b), the reduced objective of
    solve_cg.

    The first iteration, and any after a reset, steps along -g with trial
    length mu0/||g||; the others along d = -H g with unit trial step.  Both
    are searched with _line_search.  After the first accepted step H starts
    as (y.s / y.y) I (Nocedal and Wright, Eq. 6.20) before its first update.
    An update is skipped when y.s <= 1e-12 ||s|| ||y||.  A failed search
    with an estimate resets it and retries along -g; a failed search along
    -g ends the solve.  With an estimate, the solve also ends (converged)
    when the decrease the quadratic model predicts, g.H g / 2, is within
    ftol_rel of J and the model is trusted: the last accepted step's decrease
    was within ftol_rel of J as well, or, for a unit quasi-Newton step, within
    a factor 2 of the g.H g / 2 predicted for it.  (The prediction alone can
    be far too small while H still underestimates flat directions.)"""
    o = opts or SolveOptions()
    w = _f64(w0).copy()
    rep = SolveReport()
    phi, a, b, r = prob.objective(w)
    rep.n_fevals += 1
    g = prob.gradient(w, r)
    rep.n_grads += 1
    rep.J0 = phi
    rep.J_trace.append(phi)
    g0 = float(np.linalg.norm(g))
    H = None
    H_last = None                                      # last estimate, for the polish step
    last_drop = float("inf")                           # J decrease of the last accepted step
    last_pred = -1.0                                   # the model's prediction of it (< 0: none)
    floor = False
    it = 0
    rep.status = STOP_MAXITER
    while it < o.max_iter:
        gn = float(np.linalg.norm(g))
        if gn <= o.gtol_rel * g0 or phi == 0.0:
            rep.status = STOP_CONVERGED
            break
        if H is not None:
            d = -(H @ g)
            gd = float(g @ d)
            t = 1.0
            if gd >= 0.0:                                  # estimate lost definiteness
                H = None
            elif -0.5 * gd <= o.ftol_rel * phi and (
                    last_drop <= o.ftol_rel * phi or 0.5 * last_pred <= last_drop <= 2.0 * last_pred):
                # the decrease the model still predicts is below the noise, and
                # the model is trusted: the last step's decrease was below the
                # noise too, or within a factor 2 of the model's prediction
                rep.status = STOP_CONVERGED
                floor = True
                break
        if H is None:
            d = -g
            gd = -gn * gn
            t = o.mu0 / gn
        st, t, w_t, phi_t, a_t, b_t, r_t, n = _line_search(prob, o, w, phi, d, gd, t)
        rep.n_fevals += n
        if st == "noise":
            rep.status = STOP_CONVERGED
            floor = True
            break
        if st == "fail":
            if H is None:
                rep.status = STOP_LINESEARCH
                floor = True
                break
            H_last, H = H, None
            continue
        g_new = prob.gradient(w_t, r_t)
        rep.n_grads += 1
        # the quadratic model's decrease at the accepted step, when it took
        # the unit quasi-Newton step (phi(w + d) ~ phi + g.d - g.d / 2)
        last_pred = -0.5 * gd if (H is not None and t == 1.0) else -1.0
        H = _hessian_update(H, w_t - w, g_new - g)
        last_drop = phi - phi_t
        w, phi, a, b, g = w_t, phi_t, a_t, b_t, g_new
        it += 1
        rep.J_trace.append(phi)
    if floor and o.polish:
        w, phi, a, b, g = _polish(prob, H if H is not None else H_last, w, phi, a, b, g, rep)
    rep.iters = it
    rep.J, rep.a, rep.b = phi, a, b
    rep.gnorm = float(np.linalg.norm(g))
    return w, rep


def solve(prob: Problem, w0, opts: Optional[SolveOptions] = None):
    o = opts or SolveOptions()
    return {0: solve_paper, 1: solve_cg, 2: solve_bfgs}[o.method](prob, w0, o)


def measured_projection(vol, proj, f0, mean, U, w_star, xi, noise_level):
    """y = P f(w*) + noise_level * RMS(P f(w*)) * xi (the synthetic measurement)."""
    x = pca_dvf(vol, mean, U, w_star)
    p = drr_forward(vol, proj, warp(vol, f0, x))
    rms = float(np.sqrt(np.mean(p * p)))
    return p + noise_level * rms * _f64(xi).reshape(p.shape)
