"""FP64 CPU oracle for the per-projection PCA solve -- TEST INFRASTRUCTURE.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package; the product path never does.
It shares no code with the HIP library.

The primitives (projection P, its transpose, Eq. 1, the warp of Eqs. A.3/A.5,
the Jacobian of Eq. A.8, the tumour-position inversion) are plain C in
``pcas_oracle.c``; this module adds the intensity fit (Eq. A.1), the objective
(Eq. 2), the gradient chain of the Appendix, and the solvers:

* ``solve_paper`` -- the Appendix algorithm: alternate the closed-form (a, b)
  of Eq. A.1 with a normalised gradient step (Eq. A.2) whose step size comes
  from Armijo backtracking (mu0, alpha, beta as stated there), stopping when
  the step falls below mu_min or after max_iter iterations.
* ``solve_cg`` -- plain Polak-Ribiere+ nonlinear CG with Armijo backtracking
  on the reduced objective min_{a,b} J (not in the paper; the workload's CG).
* ``minimise`` -- the reference minimiser that converged solves are compared
  with: solve_cg, then Newton's method on the gradient with a Hessian from
  central differences of the gradient, then, where the gradient cannot
  vanish (a minimum on a kink of the trilinear interpolant), compass search
  on the objective.

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
        L.orc_set_threads.argtypes = [ctypes.c_int32]
        L.orc_set_threads.restype = ctypes.c_int32
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


def set_threads(n: int) -> int:
    """Thread count of the C primitives' parallel loops (results do not
    depend on it); returns the count in force."""
    return int(lib().orc_set_threads(int(n)))


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
    Armijo's rule); method 1: Polak-Ribiere+ nonlinear CG with Armijo
    backtracking on the reduced objective min_{a,b} J (the workload's "CG
    iterations"; not in the paper).

    The Appendix states mu0 = 2, alpha = 0.1, beta = 0.5, a stop once the
    step drops below 0.1, and at most 10 iterations, for coefficients scaled
    to a standard deviation of 10.  Our modes carry unit-variance
    coefficients, so the paper-mode step sizes are scaled by 1/10 (mu0 = 0.2,
    mu_min = 0.01).  CG keeps the paper's alpha and beta, starts a search
    along a fresh steepest-descent direction with a step of length mu0, and
    stops when ||g|| <= gtol_rel ||g0||."""
    method: int = 1
    max_iter: int = 30
    max_backtracks: int = 40
    mu0: float = 1.0
    alpha: float = 0.1
    beta: float = 0.5
    mu_min: float = 0.01
    gtol_rel: float = 1e-6

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
    mu_trace: List[float] = field(default_factory=list)


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
    """The Appendix algorithm (Eqs. A.1, A.2 and Armijo's rule).  The accepted
    step lengths are recorded in rep.mu_trace."""
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
        rep.mu_trace.append(mu)
        rep.iters = it + 1
        _, p = prob.project(w)
    a, b = prob.fit_ab(p)
    r = p - a * prob.y - b
    rep.a, rep.b, rep.J = a, b, float(np.sum(r * r))
    rep.J_trace.append(rep.J)
    rep.status = STOP_MAXITER
    return w, rep


def solve_cg(prob: Problem, w0, opts: Optional[SolveOptions] = None):
    """Polak-Ribiere+ nonlinear CG on phi(w) = min_{a,b} J(w, a, b).

    (a, b) is refitted by Eq. A.1 inside every evaluation; the fit is an exact
    minimiser, so phi's gradient is dJ/dw at the fitted (a, b).  Each
    iteration searches along d with Armijo backtracking, phi(w + t d) <=
    phi(w) + alpha t g.d, shrinking t by beta up to max_backtracks times.
    The first trial is mu0 / ||d|| on a steepest-descent direction (the first
    iteration and every restart), else t_prev (g_prev.d_prev) / (g.d) (the
    previous step's first-order decrease carried over; Nocedal and Wright,
    Numerical Optimization, Sec. 3.5).  A first trial that passes is
    lengthened by 1/beta for as long as the longer step still passes and
    lowers phi.  Then beta_PR+ = max(0, g+.(g+ - g) /
    g.g) and d+ = -g+ + beta_PR+ d (their Eq. 5.45); a direction that is not
    a descent direction is replaced by -g.  A failed search restarts along
    -g once; a failed search along -g ends the solve."""
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
    restart = True
    t_prev = gd_prev = 0.0
    it = 0
    rep.status = STOP_MAXITER
    while it < o.max_iter:
        gn = float(np.linalg.norm(g))
        if gn <= o.gtol_rel * g0 or phi == 0.0:
            rep.status = STOP_CONVERGED
            break
        gd = float(g @ d)
        if gd >= 0.0:
            d = -g
            gd = -gn * gn
            restart = True
        t = o.mu0 / float(np.linalg.norm(d)) if restart else t_prev * gd_prev / gd
        ok = False
        for trial in range(o.max_backtracks):
            w_t = w + t * d
            phi_t, a_t, b_t, r_t = prob.objective(w_t)
            rep.n_fevals += 1
            if phi_t <= phi + o.alpha * t * gd:
                ok = True
                break
            t *= o.beta
        # a first trial that passed: lengthen by 1/beta while the longer step
        # still passes and lowers phi (backtracking alone never lengthens a
        # step, and this carried-over first trial can start too short)
        while ok and trial == 0:
            t_x = t / o.beta
            w_x = w + t_x * d
            phi_x, a_x, b_x, r_x = prob.objective(w_x)
            rep.n_fevals += 1
            if not (phi_x <= phi + o.alpha * t_x * gd and phi_x < phi_t):
                break
            t, w_t, phi_t, a_t, b_t, r_t = t_x, w_x, phi_x, a_x, b_x, r_x
        if not ok:
            if restart:
                rep.status = STOP_LINESEARCH
                break
            d = -g
            restart = True
            continue
        g_new = prob.gradient(w_t, r_t)
        rep.n_grads += 1
        beta_pr = max(0.0, float(g_new @ (g_new - g)) / float(g @ g))
        d = -g_new + beta_pr * d
        t_prev, gd_prev = t, gd
        w, phi, a, b, r, g = w_t, phi_t, a_t, b_t, r_t, g_new
        restart = False
        it += 1
        rep.J_trace.append(phi)
    rep.iters = it
    rep.J, rep.a, rep.b = phi, a, b
    rep.gnorm = float(np.linalg.norm(g))
    return w, rep


def fd_hessian(prob: Problem, w, h: float = 1e-3):
    """Hessian of phi at w by central differences of its gradient: column k
    is (grad phi(w + h e_k) - grad phi(w - h e_k)) / (2 h), then symmetrised.
    Each gradient is taken at its own fitted (a, b), i.e. it is phi's."""
    K = w.size
    H = np.empty((K, K))
    for k in range(K):
        e = np.zeros(K)
        e[k] = h
        _, _, _, rp = prob.objective(w + e)
        _, _, _, rm = prob.objective(w - e)
        H[:, k] = (prob.gradient(w + e, rp) - prob.gradient(w - e, rm)) / (2.0 * h)
    return 0.5 * (H + H.T)


def compass_search(prob: Problem, w, phi: float, h0: float, h_min: float, max_evals: int = 4000,
                   rtol: float = 1e-15):
    """Direct search on phi with a fixed positive spanning set of directions
    (Kolda, Lewis and Torczon, Optimization by direct search, SIAM Review 45
    (2003), Secs. 2.2 and 3): the 2K coordinate directions +-e_k, then the
    2^K diagonals (+-1, ..., +-1)/sqrt(K).  From w, try w + h d for each
    direction in turn and move to the first point that lowers phi by more
    than rtol |phi| (its rounding); when none does, halve h; stop once
    h < h_min.  It compares values of phi only, so it reaches a local
    minimiser where the gradient jumps as well (the diagonals let it follow a
    crease that no coordinate direction descends).
    Returns (w, phi, evaluations)."""
    w = _f64(w).copy()
    K = w.size
    dirs = [sgn * e for e in np.eye(K) for sgn in (1.0, -1.0)]
    for signs in range(1 << K):
        dirs.append(np.array([1.0 if (signs >> k) & 1 else -1.0 for k in range(K)]) / np.sqrt(K))
    h, n = h0, 0
    while h >= h_min and n < max_evals:
        moved = False
        for dvec in dirs:
            w_t = w + h * dvec
            phi_t = prob.objective(w_t)[0]
            n += 1
            if phi_t < phi - rtol * abs(phi):
                w, phi, moved = w_t, phi_t, True
                break
        if not moved:
            h *= 0.5
    return w, phi, n


def minimise(prob: Problem, w0, gtol_rel: float = 1e-10, max_newton: int = 60,
             h: float = 1e-3, cg_opts: Optional[SolveOptions] = None,
             h_compass: float = 1e-3, h_min: float = 1e-9):
    """The oracle's minimiser of phi(w) = min_{a,b} J near w0: the reference
    that every converged solve is compared with.

    Textbook stages, sharing nothing with the library's solvers:
      1. solve_cg from w0 (monotone in phi), which settles the basin and
         lands near its minimiser;
      2. Newton's method for grad phi = 0 from there, w <- w - H^-1 g, with
         H from fd_hessian (recomputed whenever a step shrinks ||g|| by less
         than half), each step kept only while ||g|| decreases and phi does
         not rise beyond its rounding (near the minimiser differences of phi
         fall below its rounding, the gradient does not), until ||g|| <=
         gtol_rel ||g0||;
      3. compass_search on phi from there, steps h_compass down to h_min
         (in units of w).
    Trilinear interpolation makes phi piecewise smooth: its gradient jumps
    where a voxel's warp position crosses a grid plane.  With many small
    jumps the gradient is effectively smooth and stage 2 converges (the
    difference Hessian over +-h is an average curvature, so linearly) and
    stage 3 finds nothing to improve; when the minimum sits on jumps (coarse
    voxels, small displacements) no point has a small gradient, or a point
    with a vanishing one-sided gradient is not a minimum, and stage 3's
    comparisons of phi go on from there.
    Returns (w, info) with info = {"gnorm0", "gnorm", "newton_steps",
    "compass_evals", "hessian_eigs", "J", "a", "b", "cg": the stage-1
    report}.  Positive eigenvalues of the difference Hessian at the end mean
    phi curves upward around the point."""
    w0 = _f64(w0)
    w, rep = solve_cg(prob, w0, cg_opts or SolveOptions())
    _, _, _, r = prob.objective(w0)
    g0 = float(np.linalg.norm(prob.gradient(w0, r)))
    phi, a, b, r = prob.objective(w)
    g = prob.gradient(w, r)
    H = fd_hessian(prob, w, h)
    steps = 0
    for _ in range(max_newton):
        gn = float(np.linalg.norm(g))
        if gn <= gtol_rel * g0 or phi == 0.0:
            break
        w_n = w - np.linalg.solve(H, g)
        phi_n, a_n, b_n, r_n = prob.objective(w_n)
        g_n = prob.gradient(w_n, r_n)
        gn_n = float(np.linalg.norm(g_n))
        if not (gn_n < gn and phi_n <= phi * (1.0 + 1e-13)):
            break
        w, phi, a, b, g = w_n, phi_n, a_n, b_n, g_n
        steps += 1
        if gn_n > 0.5 * gn:
            H = fd_hessian(prob, w, h)
    n_compass = 0
    if phi > 0.0:
        w, phi, n_compass = compass_search(prob, w, phi, h_compass, h_min)
        phi, a, b, r = prob.objective(w)
        g = prob.gradient(w, r)
    eigs = np.linalg.eigvalsh(fd_hessian(prob, w, h))
    info = {"gnorm0": g0, "gnorm": float(np.linalg.norm(g)), "newton_steps": steps,
            "compass_evals": n_compass, "hessian_eigs": eigs, "J": phi, "a": a, "b": b,
            "cg": rep}
    return w, info


def solve(prob: Problem, w0, opts: Optional[SolveOptions] = None):
    o = opts or SolveOptions()
    return {0: solve_paper, 1: solve_cg}[o.method](prob, w0, o)


def measured_projection(vol, proj, f0, mean, U, w_star, xi, noise_level):
    """y = P f(w*) + noise_level * RMS(P f(w*)) * xi (the synthetic measurement)."""
    x = pca_dvf(vol, mean, U, w_star)
    p = drr_forward(vol, proj, warp(vol, f0, x))
    rms = float(np.sqrt(np.mean(p * p)))
    return p + noise_level * rms * _f64(xi).reshape(p.shape)
