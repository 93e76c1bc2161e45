"""Step-for-step specification of the solver state machine in
paper_1102_1712_amd/csrc/solver.h -- TEST INFRASTRUCTURE, NOT THE ORACLE.

The library's CG and BFGS solves add engineering the paper does not define:
a first trial from a quadratic model of phi along d, one extrapolated trial,
a noise band of J with a decrement stop, and a polish step.  This module
restates those rules in numpy so that tests/test_solver_machine.py can check,
on the CPU, that the C++ machine takes exactly these steps (same accepted
points, evaluation and gradient counts, stop status).  It is a specification
of the product's host logic, written beside it and changed with it; it proves
nothing about the method.  Parity of the method is judged against the
oracle's own minimiser (oracle.minimise), which shares none of these rules.

The problem interface is the oracle's: prob.objective(w) -> (phi, a, b, r)
with (a, b) refitted, prob.gradient(w, r) -> dJ/dw.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

STOP_CONVERGED, STOP_MAXITER, STOP_LINESEARCH = 0, 1, 2


@dataclass
class MachineOptions:
    """Options of the machine's CG (method 1) and BFGS (method 2), the
    library's pcas_opts fields of the same names.

    The line search (_line_search) shrinks a failed Armijo trial to the
    minimiser of the quadratic through phi(0), phi'(0) and phi(t), kept
    within [beta_lo * t, beta * t], and may lengthen an accepted first trial
    once (ls_extrap).

    polish: when a solve ends at the noise floor (the noise or decrement
    stop, or a failed search), one more step w - H g is tried with an
    inverse-Hessian estimate H (BFGS's own; CG keeps one from its steps by
    the same updates) and kept if it lowers ||g||.

    precond (machine_cg): each gradient comes with the Gauss-Newton matrix H
    of its point (prob.gauss_newton(w, r)); CG is preconditioned by it."""
    method: int = 1
    max_iter: int = 30
    max_backtracks: int = 12
    mu0: float = 1.0
    alpha: float = 0.1
    beta: float = 0.5
    gtol_rel: float = 1e-9
    beta_lo: float = 0.1
    xtol: float = 1e-10
    ftol_rel: float = 1e-14
    ls_extrap: float = 10.0
    polish: bool = False
    precond: bool = False


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


def _line_search(prob, o, w, phi, d, gd, t):
    """Armijo search along d from w (phi = J(w), gd = g.d < 0), first trial
    step t, shared by machine_cg and machine_bfgs.

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
    """machine_cg's curvature estimate after an accepted step: (y.y / y.s) I at
    the first usable pair (the reciprocal of Eq. 6.20's scaling), then
    curvature_update; pairs with y.s <= 1e-12 |s| |y| skipped."""
    sy = float(s_k @ y_k)
    if sy > 1e-12 * float(np.linalg.norm(s_k)) * float(np.linalg.norm(y_k)):
        if B is None:
            B = (float(y_k @ y_k) / sy) * np.eye(s_k.size)
        B = curvature_update(B, s_k, y_k)
    return B


def _precondition(H, g):
    """z = H^-1 g by Cholesky factors; (g, False) when H is missing or not
    positive definite."""
    if H is None:
        return g.copy(), False
    try:
        L = np.linalg.cholesky(H)
    except np.linalg.LinAlgError:
        return g.copy(), False
    return np.linalg.solve(L.T, np.linalg.solve(L, g)), True


def machine_cg(prob, w0, opts: Optional[MachineOptions] = None):
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
    decrease predicted for it (machine_bfgs's stop).  A failed search restarts
    along -g once; a second failure ends the solve.

    Preconditioned (opts.precond): with z = H^-1 g for the Gauss-Newton
    matrix H of the current point, the directions are -z + beta d with the
    PR+ rule in preconditioned inner products, beta = max(0, z+.(g+ - g) /
    (z.g)); a direction that is not downhill restarts along -z; H replaces B
    as the model of the first trial and of the stop; and the polish step is
    the Gauss-Newton step -z.  An H that is not positive definite falls back
    to z = g and to B."""
    o = opts or MachineOptions()
    w = np.asarray(w0, dtype=np.float64).copy()
    rep = SolveReport()
    phi, a, b, r = prob.objective(w)
    rep.n_fevals += 1
    g = prob.gradient(w, r)
    rep.n_grads += 1
    rep.J0 = phi
    rep.J_trace.append(phi)
    g0 = float(np.linalg.norm(g))
    pre = o.precond
    Hg, z, have_hg = None, None, False
    if pre:
        Hg = prob.gauss_newton(w, r)
        z, have_hg = _precondition(Hg, g)
    d = -z if pre else -g
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
            if pre and have_hg:
                d = -z
                gd = -float(g @ z)
            else:
                d = -g
                gd = -gn * gn
            restart = True
        if pre and have_hg:
            dbd = float(d @ (Hg @ d))
        else:
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
        if pre:
            zg = float(z @ g)
            Hg = prob.gauss_newton(w_t, r_t)
            zn, have_hg = _precondition(Hg, g_new)
            beta_pr = max(0.0, float(zn @ (g_new - g)) / zg if zg > 0.0 else 0.0)
            d = -zn + beta_pr * d
            z = zn
        else:
            beta_pr = max(0.0, float(g_new @ (g_new - g)) / float(g @ g))
            d = -g_new + beta_pr * d
        w, phi, a, b, r = w_t, phi_t, a_t, b_t, r_t
        t_prev, gd_prev = t, gd
        g = g_new
        restart, first = False, False
        it += 1
        rep.J_trace.append(phi)
    if floor and o.polish:
        w, phi, a, b, g = _polish(prob, H, w, phi, a, b, g, rep,
                                  step=z if pre and have_hg else None)
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
    """The estimate's update after an accepted step (machine_bfgs's rule; also
    kept by machine_cg for the polish step): scaled identity at the first
    usable pair, then bfgs_update; pairs with y.s <= 1e-12 |s| |y| skipped."""
    sy = float(s_k @ y_k)
    if sy > 1e-12 * float(np.linalg.norm(s_k)) * float(np.linalg.norm(y_k)):
        if H is None:
            H = (sy / float(y_k @ y_k)) * np.eye(s_k.size)
        H = bfgs_update(H, s_k, y_k)
    return H


def _polish(prob, H, w, phi, a, b, g, rep, step=None):
    """One step w - H g (or w - step), kept if ||g|| drops
    (MachineOptions.polish)."""
    if H is None and step is None:
        return w, phi, a, b, g
    d = -step if step is not None else -(H @ g)
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


def machine_bfgs(prob, w0, opts: Optional[MachineOptions] = None):
    """BFGS on phi(w) = min_{a,b} J(w, a, b), the reduced objective of
    machine_cg.

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
    o = opts or MachineOptions()
    w = np.asarray(w0, dtype=np.float64).copy()
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


def machine_solve(prob, w0, opts: MachineOptions):
    return {1: machine_cg, 2: machine_bfgs}[opts.method](prob, w0, opts)
