"""Pins for the FP64 oracle: closed forms, invariants, brute force and the
paper's stated constants -- nothing here re-types the oracle's formulas.

Each test names the passage it pins and the class of mistake it would catch.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_1102_1712_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# independent geometry: rotate a canonical (angle 0) source/pixel pair and
# find the chord through the box by bisection on an inside/outside test.
# ---------------------------------------------------------------------------

def _rays_by_rotation(proj, pix):
    th = proj.angle
    R = np.array([[np.cos(th), -np.sin(th), 0.0], [np.sin(th), np.cos(th), 0.0], [0.0, 0.0, 1.0]])
    S0 = np.array([0.0, -proj.sad, 0.0])
    iu, iv = pix % proj.nu, pix // proj.nu
    u = (iu - (proj.nu - 1) / 2.0) * proj.pitch_u + proj.offset_u
    v = (iv - (proj.nv - 1) / 2.0) * proj.pitch_v + proj.offset_v
    P0 = np.stack([u, np.full_like(u, proj.sid - proj.sad, dtype=float), v], axis=-1)
    return R @ S0, P0 @ R.T


def _inside(vol, X):
    lo = np.array(vol.origin)
    hi = lo + (np.array(vol.n) - 1) * np.array(vol.spacing)
    return np.all((X >= lo) & (X <= hi), axis=-1)


def _chord_bisect(vol, S, P):
    """Entry/exit points of the segment line S->P through the box, by dense
    search for an inside point then bisection.  Returns (length, midpoint)."""
    d = P - S
    ts = np.linspace(0.0, 2.0, 20001)
    X = S[None, :] + ts[:, None] * d[None, :]
    ins = _inside(vol, X)
    if not ins.any():
        return 0.0, None
    idx = np.nonzero(ins)[0]
    t_first, t_last = ts[idx[0]], ts[idx[-1]]

    def bis(a, b):  # a outside, b inside
        for _ in range(200):
            m = 0.5 * (a + b)
            if _inside(vol, S + m * d):
                b = m
            else:
                a = m
        return b

    t_in = bis(ts[idx[0] - 1], t_first)
    t_out = bis(ts[idx[-1] + 1], t_last)
    A, B = S + t_in * d, S + t_out * d
    return float(np.linalg.norm(B - A)), 0.5 * (A + B)


def _geom_case():
    vol = synth.centred_volume((12, 10, 9), (5.0, 6.0, 7.0))
    proj = synth.Projection(angle=0.7, sad=400.0, sid=600.0, nu=15, nv=11,
                            pitch_u=9.0, pitch_v=9.5, step=2.5, offset_u=3.0, offset_v=-2.0)
    return vol, proj


def test_chord_uniform_box():
    """Sec. II.A (P) -- f = mu on the grid gives mu times the chord length
    through the box for every ray (midpoint rule, interpolation weights sum
    to one).  Catches wrong source/detector placement, slab bugs, a wrong
    step count or a dropped interpolation weight."""
    vol, proj = _geom_case()
    mu = 0.0173
    f = np.full(vol.shape_zyx, mu)
    p = O.drr_forward(vol, proj, f).reshape(-1)
    pix = np.arange(proj.npix)
    S, P = _rays_by_rotation(proj, pix)
    L = np.array([_chord_bisect(vol, S, P[t])[0] for t in pix])
    assert (L > 0).sum() > 20 and (L == 0).sum() > 5     # both hits and misses
    np.testing.assert_allclose(p, mu * L, rtol=1e-12, atol=1e-12)


def test_chord_linear_ramp_midpoint():
    """Sec. II.A (P) with Eq. A.5 -- trilinear interpolation reproduces a
    linear field and the midpoint rule integrates it exactly, so each ray
    gives (chord length) x (field at the chord midpoint).  Catches swapped
    or mis-paired interpolation weights and off-centre samples."""
    vol, proj = _geom_case()
    al, be, ga, de = 0.37, -0.21, 0.55, 9.0
    k, j, i = np.meshgrid(*[np.arange(n) for n in vol.shape_zyx], indexing="ij")
    f = al * i + be * j + ga * k + de
    p = O.drr_forward(vol, proj, f).reshape(-1)
    pix = np.arange(proj.npix)
    S, P = _rays_by_rotation(proj, pix)
    o, s = np.array(vol.origin), np.array(vol.spacing)
    for t in pix:
        L, mid = _chord_bisect(vol, S, P[t])
        if L == 0.0:
            assert p[t] == 0.0
            continue
        q = (mid - o) / s
        expect = L * (al * q[0] + be * q[1] + ga * q[2] + de)
        assert abs(p[t] - expect) <= 1e-11 * abs(expect)


def test_rotation_symmetry():
    """Sec. II.A (P changes with gantry angle) -- on a centred cubic grid the
    projection at angle+90deg of f equals the projection at angle of f
    rotated by 90deg about the SI axis.  Catches a wrong rotation sense,
    detector-axis orientation or source position."""
    vol = synth.centred_volume((20, 20, 12), (5.0, 5.0, 6.0))
    rng = np.random.default_rng(3)
    f = rng.uniform(0.0, 1.0, vol.shape_zyx)
    n = vol.n[0]
    g = np.empty_like(f)
    for jj in range(n):            # g(i, j, k) = f(n-1-j, i, k)
        for ii in range(n):
            g[:, jj, ii] = f[:, ii, n - 1 - jj]
    base = synth.Projection(angle=0.4, sad=500.0, sid=800.0, nu=21, nv=13, pitch_u=7.0,
                            pitch_v=8.0, step=1.7)
    rot = synth.Projection(angle=0.4 + np.pi / 2, sad=500.0, sid=800.0, nu=21, nv=13,
                           pitch_u=7.0, pitch_v=8.0, step=1.7)
    np.testing.assert_allclose(O.drr_forward(vol, rot, f), O.drr_forward(vol, base, g),
                               rtol=1e-10, atol=1e-12)


def test_adjoint_identity():
    """Appendix (P^T in dJ/dw) -- <P x, y> = <x, P^T y> to 1e-12."""
    c = synth.small(seed=21)
    rng = np.random.default_rng(4)
    x = rng.normal(size=c.vol.shape_zyx)
    y = rng.normal(size=(c.proj.nv, c.proj.nu))
    lhs = float(np.sum(O.drr_forward(c.vol, c.proj, x) * y))
    rhs = float(np.sum(x * O.drr_adjoint(c.vol, c.proj, y)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_adjoint_dense_bruteforce():
    """Appendix (P^T) -- build the dense P column by column on a 5x6x7
    volume and a 3x4 detector and check P^T y = A^T y.  Catches any
    asymmetry between the scatter and the gather (a missed corner, a wrong
    voxel index)."""
    vol = synth.centred_volume((5, 6, 7), (10.0, 9.0, 8.0))
    proj = synth.Projection(angle=2.1, sad=300.0, sid=450.0, nu=3, nv=4, pitch_u=15.0,
                            pitch_v=14.0, step=3.3)
    N, M = vol.nvox, proj.npix
    A = np.zeros((M, N))
    for v in range(N):
        e = np.zeros(N)
        e[v] = 1.0
        A[:, v] = O.drr_forward(vol, proj, e.reshape(vol.shape_zyx)).reshape(-1)
    assert np.count_nonzero(A) > 50
    y = np.random.default_rng(5).normal(size=M)
    bp = O.drr_adjoint(vol, proj, y).reshape(-1)
    np.testing.assert_allclose(bp, A.T @ y, rtol=1e-13, atol=1e-14)


# ---------------------------------------------------------------------------
# Eq. 1, Eqs. A.3 / A.5, Eq. A.8
# ---------------------------------------------------------------------------

def _small_fields(seed=7, K=3, with_mean=True):
    c = synth.small(seed=seed, K=K, with_mean=with_mean)
    return c


def test_pca_dvf_basis_vectors():
    """Eq. 1 -- w = e_k gives xbar + u_k exactly; w = 0 gives xbar; the
    field is affine in w.  Catches a transposed mode/component index."""
    c = _small_fields()
    for k in range(c.K):
        w = np.zeros(c.K)
        w[k] = 1.0
        assert np.array_equal(O.pca_dvf(c.vol, c.mean, c.U, w), c.mean + c.U[k])
    assert np.array_equal(O.pca_dvf(c.vol, c.mean, c.U, np.zeros(c.K)), c.mean)
    w1, w2 = np.array([0.3, -1.2, 0.7]), np.array([-0.4, 0.1, 2.0])
    lhs = O.pca_dvf(c.vol, None, c.U, w1 + w2)
    rhs = O.pca_dvf(c.vol, None, c.U, w1) + O.pca_dvf(c.vol, None, c.U, w2)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-13)


def test_identity_warp_bitwise():
    """Eq. A.3 -- a zero field reproduces the reference image bitwise."""
    c = _small_fields()
    x = O.pca_dvf(c.vol, None, c.U, np.zeros(c.K))
    assert np.array_equal(O.warp(c.vol, c.f0, x), c.f0)


def test_integer_shift_warp():
    """Eq. A.3 -- a constant field of whole voxels pulls f0 from the shifted
    voxel, with zeros where the source lies outside the grid.  Catches an
    axis mix-up or a sign error in the pull-back."""
    c = _small_fields()
    s = c.vol.spacing
    x = np.empty((3,) + c.vol.shape_zyx)
    x[0], x[1], x[2] = 2 * s[0], -1 * s[1], 3 * s[2]
    f = O.warp(c.vol, c.f0, x)
    expect = np.zeros_like(c.f0)
    # f(i, j, k) = f0(i+2, j-1, k+3); arrays are [k][j][i]
    expect[:-3, 1:, :-2] = c.f0[3:, :-1, 2:]
    assert np.array_equal(f, expect)


def test_ramp_warp_and_jacobian():
    """Eqs. A.5 and A.8 -- on a linear reference image a*i + b*j + c*k + d the
    warp gives f0 + (a x1/s1 + b x2/s2 + c x3/s3) and the Jacobian is
    (a/s1, b/s2, c/s3), wherever all eight neighbours are inside."""
    c = _small_fields()
    al, be, ga, de = 0.31, -0.17, 0.23, 5.0
    k, j, i = np.meshgrid(*[np.arange(n) for n in c.vol.shape_zyx], indexing="ij")
    f0 = al * i + be * j + ga * k + de
    x = O.pca_dvf(c.vol, c.mean, c.U, np.array([0.8, -0.5, 0.6]))
    s = c.vol.spacing
    q = [i + x[0] / s[0], j + x[1] / s[1], k + x[2] / s[2]]
    inner = np.ones(f0.shape, bool)
    for a, n in zip(q, c.vol.n):
        inner &= (a >= 0) & (a < n - 1)
    assert inner.mean() > 0.5
    f = O.warp(c.vol, f0, x)
    expect = f0 + al * x[0] / s[0] + be * x[1] / s[1] + ga * x[2] / s[2]
    np.testing.assert_allclose(f[inner], expect[inner], rtol=1e-13, atol=1e-12)
    jac = O.warp_jacobian(c.vol, f0, x)
    for comp, val in enumerate((al / s[0], be / s[1], ga / s[2])):
        np.testing.assert_allclose(jac[comp][inner], val, rtol=1e-12, atol=1e-14)


def test_jacobian_matches_central_difference():
    """Eq. A.8 is the exact derivative of Eq. A.5 away from grid crossings:
    compare with a central difference of the warp under a uniform shift of
    one component.  Catches a wrong neighbour pairing or weight."""
    c = _small_fields()
    x = O.pca_dvf(c.vol, c.mean, c.U, np.array([1.1, 0.4, -0.9]))
    jac = O.warp_jacobian(c.vol, c.f0, x)
    s = np.array(c.vol.spacing)
    k, j, i = np.meshgrid(*[np.arange(n) for n in c.vol.shape_zyx], indexing="ij")
    idx = (i, j, k)
    for comp in range(3):
        h = 1e-5 * s[comp]
        xp, xm = x.copy(), x.copy()
        xp[comp] += h
        xm[comp] -= h
        fd = (O.warp(c.vol, c.f0, xp) - O.warp(c.vol, c.f0, xm)) / (2 * h)
        q = idx[comp] + x[comp] / s[comp]
        frac = q - np.floor(q)
        ok = (frac > 1e-3) & (frac < 1 - 1e-3)
        scale = np.abs(jac[comp]).max()
        assert np.max(np.abs(fd[ok] - jac[comp][ok])) <= 1e-7 * scale


def test_jacobian_right_derivative_at_grid_points():
    """Appendix (remarks after Eq. A.8) -- at integer positions the formula
    is the right-side derivative: with x = 0 it is the forward difference
    f0(i+1) - f0(i) (zero beyond the last voxel), per mm."""
    c = _small_fields()
    x = np.zeros((3,) + c.vol.shape_zyx)
    jac = O.warp_jacobian(c.vol, c.f0, x)
    s = c.vol.spacing
    pad = np.zeros(tuple(n + 1 for n in c.f0.shape))
    pad[:-1, :-1, :-1] = c.f0
    fwd_i = (pad[:-1, :-1, 1:] - c.f0) / s[0]
    fwd_j = (pad[:-1, 1:, :-1] - c.f0) / s[1]
    fwd_k = (pad[1:, :-1, :-1] - c.f0) / s[2]
    np.testing.assert_allclose(jac[0], fwd_i, rtol=1e-14, atol=1e-17)
    np.testing.assert_allclose(jac[1], fwd_j, rtol=1e-14, atol=1e-17)
    np.testing.assert_allclose(jac[2], fwd_k, rtol=1e-14, atol=1e-17)


# ---------------------------------------------------------------------------
# Eq. A.1, Eq. 2, gradient
# ---------------------------------------------------------------------------

def test_intensity_fit_matches_lstsq_and_special_cases():
    """Eq. A.1 -- the unique minimiser over (a, b): agrees with a library
    least-squares solve; y = Pf gives (1, 0); y = 2 Pf + 3 gives
    (0.5, -1.5); a constant y is singular."""
    rng = np.random.default_rng(8)
    p = rng.uniform(0, 5, 300)
    y = 0.7 * p + rng.normal(0, 0.3, 300) - 0.2
    a, b = O.intensity_fit(p, y)
    sol = np.linalg.lstsq(np.stack([y, np.ones_like(y)], 1), p, rcond=None)[0]
    np.testing.assert_allclose([a, b], sol, rtol=1e-12)
    np.testing.assert_allclose(O.intensity_fit(p, p), [1.0, 0.0], atol=1e-12)
    np.testing.assert_allclose(O.intensity_fit(p, 2 * p + 3), [0.5, -1.5], atol=1e-12)
    with pytest.raises(O.SingularFit):
        O.intensity_fit(p, np.full_like(p, 4.0))


def _problem(case, fit=True):
    y = O.measured_projection(case.vol, case.proj, case.f0, case.mean, case.U, case.w_star,
                              case.xi, case.noise_level)
    return O.Problem(case.vol, case.proj, case.f0, case.mean, case.U, y, fit_intensity=fit), y


def _kink_free_step(case, w, k, candidates=(1e-6, 3e-7, 1e-7, 3e-8, 1e-8)):
    """Largest FD step for which no voxel's warp position crosses a grid line
    between w - h e_k and w + h e_k (trilinear interpolation has kinks there;
    the Appendix notes Eq. A.8 is then a one-sided derivative)."""
    s = np.array(case.vol.spacing)
    for h in candidates:
        e = np.zeros(case.K)
        e[k] = h * max(1.0, abs(w[k]))
        xp = O.pca_dvf(case.vol, case.mean, case.U, w + e)
        xm = O.pca_dvf(case.vol, case.mean, case.U, w - e)
        if all(np.array_equal(np.floor(xp[c] / s[c]), np.floor(xm[c] / s[c])) for c in range(3)):
            return e[k]
    pytest.skip("no kink-free finite-difference step")


@pytest.mark.parametrize("where", ["zero", "offset"])
def test_gradient_central_difference(where):
    """Appendix -- dJ/dw = 2 U^T (df/dx) P^T r agrees with a central
    difference of J at fixed (a, b) to 1e-6.  Catches a sign error, a
    dropped factor 2, a transposed U or a wrong adjoint."""
    c = synth.small(seed=9)
    prob, _ = _problem(c)
    w = np.zeros(c.K) if where == "zero" else c.w_star + 0.3 * np.array([0.5, -0.7, 0.2])
    J, a, b, r = prob.objective(w)
    g = prob.gradient(w, r)
    fd = np.zeros(c.K)
    for k in range(c.K):
        h = _kink_free_step(c, w, k)
        e = np.zeros(c.K)
        e[k] = h
        fd[k] = (prob.objective(w + e, ab=(a, b))[0] - prob.objective(w - e, ab=(a, b))[0]) / (2 * h)
    assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(fd)


def test_gradient_taylor_slope_two():
    """J(w + h d) - J(w) - h g.d = O(h^2): the log-log slope is about 2."""
    c = synth.small(seed=12)
    prob, _ = _problem(c)
    w = c.w_star + np.array([0.4, -0.3, 0.5])
    J, a, b, r = prob.objective(w)
    g = prob.gradient(w, r)
    d = np.array([0.6, 0.2, -0.77])
    hs = np.array([1e-1, 5e-2, 2.5e-2, 1.25e-2])
    rem = np.array([abs(prob.objective(w + h * d, ab=(a, b))[0] - J - h * (g @ d)) for h in hs])
    slope = np.polyfit(np.log(hs), np.log(rem), 1)[0]
    assert 1.8 < slope < 2.2


def test_reduced_objective_gradient_envelope():
    """With (a, b) refitted at every w (Eq. A.1 is the exact minimiser), the
    gradient at the fitted (a, b) is the gradient of min_{a,b} J."""
    c = synth.small(seed=13)
    prob, _ = _problem(c)
    w = c.w_star + np.array([-0.5, 0.3, 0.2])
    J, a, b, r = prob.objective(w)
    g = prob.gradient(w, r)
    fd = np.zeros(c.K)
    for k in range(c.K):
        h = _kink_free_step(c, w, k)
        e = np.zeros(c.K)
        e[k] = h
        fd[k] = (prob.objective(w + e)[0] - prob.objective(w - e)[0]) / (2 * h)
    assert np.linalg.norm(g - fd) <= 1e-5 * np.linalg.norm(fd)


# ---------------------------------------------------------------------------
# solvers
# ---------------------------------------------------------------------------

def test_paper_constants_golden():
    """Appendix (after Eq. A.2): mu0 = 2, alpha = 0.1, beta = 0.5, stop below
    0.1, at most 10 iterations, coefficients scaled to std 10.  The paper
    mode keeps alpha, beta and the cap, and scales the step sizes by our
    coefficient std (1) over the paper's (10)."""
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    o = O.SolveOptions.paper()
    scale = 1.0 / g["coefficient_std"]
    assert o.method == 0
    assert o.alpha == g["armijo_alpha"] and o.beta == g["armijo_beta"]
    assert o.max_iter == g["max_iter"]
    assert abs(o.mu0 - g["armijo_mu0"] * scale) < 1e-15
    assert abs(o.mu_min - g["stop_step"] * scale) < 1e-15


def test_paper_solver_monotone_and_stops():
    """Appendix -- every accepted step decreases J (alternating exact fit and
    Armijo step), and the solve ends on a small step or the 10-iteration cap."""
    c = synth.small(seed=14)
    prob, _ = _problem(c)
    w, rep = O.solve_paper(prob, np.zeros(c.K))
    tr = np.array(rep.J_trace)
    assert np.all(np.diff(tr) <= 1e-15 * tr[0])
    assert tr[-1] < 0.2 * tr[0]
    assert rep.iters <= 10
    assert rep.status in (O.STOP_CONVERGED, O.STOP_MAXITER)


class _Scalar:
    """A one-pixel, one-coefficient problem in the oracle's interface:
    p(w) = [w], y = [c], no intensity fit, so J(w) = (w - c)^2 and
    dJ/dw = 2 (w - c)."""

    def __init__(self, c):
        self.y = np.array([[c]])
        self.fit = False
        self.calls = []

    def project(self, w):
        return None, np.array([[float(w[0])]])

    def fit_ab(self, p):
        return 1.0, 0.0

    def objective(self, w, ab=None):
        self.calls.append(("J", float(w[0]), ab))
        a, b = (1.0, 0.0) if ab is None else ab
        r = np.array([[float(w[0])]]) - a * self.y - b
        return float(np.sum(r * r)), a, b, r

    def gradient(self, w, r):
        return np.array([2.0 * float(r[0, 0])])


def test_paper_solver_armijo_sequence_by_hand():
    """Appendix, Eq. A.2 and the Armijo rule after it, with the paper's own
    constants (mu0 = 2, alpha = 0.1, beta = 0.5, stop below 0.1) on
    J(w) = (w - 2.3)^2 from w = 0, worked by hand:
      it 1: J 5.29, g -4.6, d = -1: mu 2 -> w 2, J 0.09 <= 5.29 - 0.92.
      it 2: J 0.09, g -0.6: mu 2 (w 4, J 2.89) and 1 (w 3, J 0.49) fail;
            mu 0.5 -> w 2.5, J 0.04 <= 0.09 - 0.03.
      it 3: J 0.04, g 0.4, d = +1: mu 2, 1, 0.5 (w 0.5, 1.5, 2: J 3.24,
            0.64, 0.09) fail; mu 0.25 -> w 2.25, J 0.0025 <= 0.04 - 0.01.
      it 4: J 0.0025, g -0.1: mu 2, 1, 0.5, 0.25, 0.125 (w 4.25, 3.25, 2.75,
            2.5, 2.375) all fail; 0.0625 < 0.1: stop without the step.
    So mu = (2, 0.5, 0.25), w = 2.25 after 3 iterations, 1 + 1 + 3 + 4 + 5 =
    14 evaluations and 4 gradients.  Catches a wrong alpha or beta, a test
    against g instead of ||g||, a step taken below mu_min, or mu not
    restarting at mu0."""
    q = _Scalar(2.3)
    o = O.SolveOptions(method=0, max_iter=10, mu0=2.0, alpha=0.1, beta=0.5, mu_min=0.1)
    w, rep = O.solve_paper(q, np.zeros(1), o)
    assert rep.mu_trace == [2.0, 0.5, 0.25]
    assert w[0] == 2.25
    assert (rep.iters, rep.n_fevals, rep.n_grads, rep.status) == (3, 14, 4, O.STOP_CONVERGED)
    np.testing.assert_allclose(rep.J_trace, [5.29, 0.09, 0.04, 0.0025], rtol=1e-12)
    # the ten-iteration cap: J = (w - 40)^2 moves by mu0 = 2 every time
    w, rep = O.solve_paper(_Scalar(40.0), np.zeros(1), o)
    assert (rep.iters, rep.status, w[0]) == (10, O.STOP_MAXITER, 20.0)
    assert rep.mu_trace == [2.0] * 10


def test_paper_solver_fixes_the_fit_during_the_search():
    """Appendix: step 1 fits (a, b) (Eq. A.1) at the current w; step 2's
    Armijo trials then compare J at that fixed (a, b).  The trials of one
    iteration all carry one (a, b), the fit at the iterate they start from;
    that iterate is w0 for the first iteration and the previous iteration's
    last (accepted) trial afterwards."""
    c = synth.small(seed=19)
    prob, y = _problem(c)
    seen = []
    orig = prob.objective

    def spy(w, ab=None):
        seen.append((np.array(w), ab))
        return orig(w, ab)

    prob.objective = spy
    w, rep = O.solve_paper(prob, np.zeros(c.K))
    assert seen and all(ab is not None for _, ab in seen)
    groups = []
    for wt, ab in seen:
        if not groups or groups[-1][0] != ab:
            groups.append((ab, []))
        groups[-1][1].append(wt)
    assert len(groups) in (rep.iters, rep.iters + 1)
    start = np.zeros(c.K)
    for ab, trials in groups:
        _, p = prob.project(start)
        assert ab == pytest.approx(O.intensity_fit(p, y), rel=1e-13)
        start = trials[-1]
    assert np.array_equal(w, groups[rep.iters - 1][1][-1])


def test_cg_second_direction_is_conjugate():
    """PR+ CG (Nocedal and Wright, Eq. 5.45): on a quadratic, after an exact
    first line search the next direction is A-conjugate to the first, so the
    second step s1 satisfies s1.A s0 = 0.  mu0 is set so that the first trial
    is the exact minimiser along -g0 (Armijo accepts it).  Catches a wrong
    sign or index in beta or in the new direction."""
    rng = np.random.default_rng(45)
    for K in (2, 3, 5):
        A, _ = _spd(rng, K, 30.0)
        cvec = 3.0 * rng.normal(size=K)
        q = _Quadratic(A, cvec)
        g0 = -cvec                                     # gradient at w = 0
        t_star = float(g0 @ g0) / float(g0 @ A @ g0)
        mu0 = t_star * float(np.linalg.norm(g0))
        w1, _ = O.solve_cg(q, np.zeros(K), O.SolveOptions(mu0=mu0, max_iter=1, gtol_rel=0.0))
        w2, _ = O.solve_cg(q, np.zeros(K), O.SolveOptions(mu0=mu0, max_iter=2, gtol_rel=0.0))
        s0, s1 = w1, w2 - w1
        np.testing.assert_allclose(w1, -t_star * g0, rtol=1e-13)
        assert abs(float(s1 @ A @ s0)) <= 1e-12 * np.linalg.norm(A @ s0) * np.linalg.norm(s1)
        assert np.linalg.norm(s1) > 0.0


@pytest.mark.parametrize("solver", ["paper", "cg"])
def test_solver_monotone(solver):
    c = synth.small(seed=15)
    prob, _ = _problem(c)
    w, rep = getattr(O, "solve_" + solver)(prob, np.zeros(c.K))
    assert np.all(np.diff(rep.J_trace) <= 0.0)


def test_planted_w_exact_recovery_32():
    """Noise-free 32^3 FP64 volume: the oracle's minimiser recovers the
    planted w to 1e-8 relative (the measured image is exactly P f(w*), so w*
    is a zero-residual minimiser with (a, b) = (1, 0)); plain CG alone, which
    stops at ||g|| <= 1e-6 ||g0||, to 1e-5."""
    c = synth.recovery32()
    prob, _ = _problem(c)
    w, info = O.minimise(prob, np.zeros(c.K))
    assert np.linalg.norm(w - c.w_star) <= 1e-8 * np.linalg.norm(c.w_star)
    np.testing.assert_allclose([info["a"], info["b"]], [1.0, 0.0], atol=1e-8)
    assert np.all(info["hessian_eigs"] > 0.0)
    w_cg, rep = O.solve_cg(prob, np.zeros(c.K))
    assert rep.status == O.STOP_CONVERGED
    assert np.linalg.norm(w_cg - c.w_star) <= 1e-5 * np.linalg.norm(c.w_star)


class _Quadratic:
    """phi(w) = (w - w*).A (w - w*) / 2 + 10 with w* = A^-1 c, in the solvers'
    problem interface, with (a, b) reported as (1, 0): its minimiser is
    A^-1 c in closed form, its gradient A w - c, and phi >= 10 > 0."""

    def __init__(self, A, c):
        self.A, self.c = A, c
        self.ws = np.linalg.solve(A, c)

    def objective(self, w, ab=None):
        e = w - self.ws
        return float(0.5 * e @ self.A @ e + 10.0), 1.0, 0.0, None

    def gradient(self, w, r):
        return self.A @ w - self.c


def _spd(rng, K, kappa):
    Q, _ = np.linalg.qr(rng.normal(size=(K, K)))
    return Q @ np.diag(np.geomspace(1.0, kappa, K)) @ Q.T, Q


def test_solvers_reach_quadratic_minimiser():
    """Plain CG and the reference minimiser end at A^-1 c on ill-conditioned
    quadratics; the difference Hessian of a quadratic is A itself, so the
    minimiser's Newton stage lands there to rounding."""
    rng = np.random.default_rng(42)
    for K, kappa in ((3, 10.0), (5, 1e2), (8, 1e3)):
        A, _ = _spd(rng, K, kappa)
        c = 3.0 * rng.normal(size=K)
        ws = np.linalg.solve(A, c)
        w, rep = O.solve_cg(_Quadratic(A, c), np.zeros(K), O.SolveOptions(max_iter=400))
        assert rep.status == O.STOP_CONVERGED
        assert np.linalg.norm(w - ws) <= 1e-5 * kappa * np.linalg.norm(ws), (K, kappa, rep)
        wm, info = O.minimise(_Quadratic(A, c), np.zeros(K), cg_opts=O.SolveOptions(max_iter=5))
        assert np.linalg.norm(wm - ws) <= 1e-12 * kappa * np.linalg.norm(ws), (K, kappa, info)
        np.testing.assert_allclose(np.sort(info["hessian_eigs"]), np.geomspace(1.0, kappa, K),
                                   rtol=1e-9)


def test_fd_hessian_of_quadratic_is_exact():
    """Central differences of a linear gradient are exact: fd_hessian
    returns A (to rounding) at any point and for any step."""
    rng = np.random.default_rng(46)
    A, _ = _spd(rng, 4, 50.0)
    q = _Quadratic(A, rng.normal(size=4))
    for h in (1e-1, 1e-3):
        np.testing.assert_allclose(O.fd_hessian(q, rng.normal(size=4), h), A, rtol=0,
                                   atol=1e-9 * np.abs(A).max())


def test_cg_and_minimiser_agree_on_noisy_small():
    """With 1% noise the minimiser is not w*, but plain CG from w0 = 0 and
    the reference minimiser find the same point, and it is a minimum: J
    rises along every axis at +-1e-3 (no gradient involved)."""
    c = synth.small(seed=17)
    prob, _ = _problem(c)
    w_cg, r_cg = O.solve_cg(prob, np.zeros(c.K))
    w_m, info = O.minimise(prob, np.zeros(c.K))
    assert np.linalg.norm(w_cg - w_m) <= 1e-4 * np.linalg.norm(w_m)
    assert info["J"] <= r_cg.J
    assert info["gnorm"] <= 1e-6 * info["gnorm0"]
    assert np.all(info["hessian_eigs"] > 0.0)
    J = prob.objective(w_m)[0]
    for k in range(c.K):
        e = np.zeros(c.K)
        e[k] = 1e-3
        assert prob.objective(w_m + e)[0] > J and prob.objective(w_m - e)[0] > J


def test_k1_matches_bruteforce_line_search():
    """K = 1 with (a, b) fixed to (1, 0): the minimiser agrees with a dense
    grid search refined by golden-section search on J itself (no gradient
    involved), and so does plain CG."""
    c = synth.small(seed=16, K=1)
    prob, y = _problem(c, fit=False)
    w_m, _ = O.minimise(prob, np.zeros(1))
    w_cg, rep = O.solve_cg(prob, np.zeros(1))

    def J(v):
        return prob.objective(np.array([v]))[0]

    grid = np.linspace(c.w_star[0] - 2.0, c.w_star[0] + 2.0, 201)
    vals = [J(v) for v in grid]
    i = int(np.argmin(vals))
    lo, hi = grid[max(i - 1, 0)], grid[min(i + 1, grid.size - 1)]
    gr = (np.sqrt(5) - 1) / 2
    a, b = lo, hi
    c1, c2 = b - gr * (b - a), a + gr * (b - a)
    f1, f2 = J(c1), J(c2)
    for _ in range(80):
        if f1 < f2:
            b, c2, f2 = c2, c1, f1
            c1 = b - gr * (b - a)
            f1 = J(c1)
        else:
            a, c1, f1 = c1, c2, f2
            c2 = a + gr * (b - a)
            f2 = J(c2)
    w_gs = 0.5 * (a + b)
    assert abs(w_m[0] - w_gs) <= 1e-5 * max(1.0, abs(w_gs))
    assert abs(w_cg[0] - w_gs) <= 1e-5 * max(1.0, abs(w_gs))


def test_tiny_config_minimiser():
    """64^3 FP64 with 1% noise (the tiny workload): the reference minimiser is
    a strict local minimum (||g|| <= 1e-10 ||g0||, positive definite
    difference Hessian) whose J does not exceed J at the planted w, near w*;
    plain CG's 30 iterations get within 1e-3 of it."""
    c = synth.tiny()
    prob, _ = _problem(c)
    w, info = O.minimise(prob, np.zeros(c.K))
    assert info["gnorm"] <= 1e-10 * info["gnorm0"]
    assert np.all(info["hessian_eigs"] > 0.0)
    assert info["J"] <= prob.objective(c.w_star)[0]
    assert np.linalg.norm(w - c.w_star) <= 0.1 * np.linalg.norm(c.w_star)
    w_cg = info["cg"]
    assert w_cg.iters == 30 or w_cg.status == O.STOP_CONVERGED


# ---------------------------------------------------------------------------
# tumour position
# ---------------------------------------------------------------------------

def test_locate_rigid_translation():
    """Sec. II.A (pull-back inversion at one point) -- for a rigid field x = t
    the tumour moves to c0 - t."""
    vol = synth.centred_volume((20, 18, 16), (4.0, 5.0, 6.0))
    t = np.array([3.2, -1.7, 4.4])
    mean = np.empty((3,) + vol.shape_zyx)
    for c in range(3):
        mean[c] = t[c]
    U = np.zeros((1, 3) + vol.shape_zyx)
    c0 = np.array([5.0, -7.0, 3.0])
    y, it = O.locate(vol, mean, U, np.zeros(1), c0)
    assert it > 0
    np.testing.assert_allclose(y, c0 - t, atol=1e-12)


def test_locate_affine_field():
    """For an affine field x(p) = A p + t (reproduced exactly by trilinear
    interpolation) the fixed point is (I + A)^{-1} (c0 - t)."""
    vol = synth.centred_volume((24, 22, 20), (4.0, 4.0, 5.0))
    A = np.array([[0.05, -0.02, 0.01], [0.03, 0.04, -0.02], [-0.01, 0.02, 0.06]])
    t = np.array([1.5, -2.0, 0.7])
    k, j, i = np.meshgrid(*[np.arange(n) for n in vol.shape_zyx], indexing="ij")
    P = np.stack([vol.origin[0] + i * vol.spacing[0], vol.origin[1] + j * vol.spacing[1],
                  vol.origin[2] + k * vol.spacing[2]])
    mean = np.einsum("ab,b...->a...", A, P) + t[:, None, None, None]
    U = np.zeros((1, 3) + vol.shape_zyx)
    c0 = np.array([10.0, -6.0, 4.0])
    y, it = O.locate(vol, mean, U, np.zeros(1), c0, tol=1e-12)
    assert it > 0
    np.testing.assert_allclose(y, np.linalg.solve(np.eye(3) + A, c0 - t), atol=1e-9)


# ---------------------------------------------------------------------------
# Siddon's exact-path projector (the simulator of Sec. II.B): the volume as
# constant over voxel cells [centre - s/2, centre + s/2], the ray from the
# source to the pixel centre.
# ---------------------------------------------------------------------------

def _cell_box(vol, lo_idx=None, hi_idx=None):
    s = np.array(vol.spacing)
    o = np.array(vol.origin)
    lo_idx = np.zeros(3) if lo_idx is None else np.asarray(lo_idx, float)
    hi_idx = np.array(vol.n) - 1.0 if hi_idx is None else np.asarray(hi_idx, float)
    return o + (lo_idx - 0.5) * s, o + (hi_idx + 0.5) * s


def _segment_in_box(S, P, lo, hi, n=4001):
    """Length of the segment S->P inside [lo, hi]: dense search + bisection."""
    d = P - S
    ts = np.linspace(0.0, 1.0, n)
    X = S[None, :] + ts[:, None] * d[None, :]
    ins = np.all((X >= lo) & (X <= hi), axis=-1)
    if not ins.any():
        return 0.0

    def inside(t):
        x = S + t * d
        return bool(np.all((x >= lo) & (x <= hi)))

    def bis(a, b):   # a outside, b inside
        for _ in range(200):
            m = 0.5 * (a + b)
            if inside(m):
                b = m
            else:
                a = m
        return b

    idx = np.nonzero(ins)[0]
    t_in = bis(ts[idx[0] - 1], ts[idx[0]]) if idx[0] > 0 else 0.0
    t_out = bis(ts[idx[-1] + 1], ts[idx[-1]]) if idx[-1] < n - 1 else 1.0
    return float((t_out - t_in) * np.linalg.norm(d))


def test_siddon_uniform_volume_is_chord_of_cell_box():
    """f = mu: the path lengths through all cells add up to the chord through
    the grid's outer box (catches dropped or doubled cell intervals)."""
    vol, proj = _geom_case()
    mu = 0.037
    p = O.siddon_forward(vol, proj, np.full(vol.shape_zyx, mu))
    pix = np.arange(proj.nu * proj.nv)
    S, P = _rays_by_rotation(proj, pix)
    lo, hi = _cell_box(vol)
    L = np.array([_segment_in_box(S, P[r], lo, hi) for r in pix])
    assert (L > 0).sum() > 20 and (L == 0).sum() > 0          # hits and misses
    np.testing.assert_allclose(p.reshape(-1), mu * L, rtol=1e-9, atol=1e-9)


def test_siddon_single_cell_is_its_segment_length():
    """One non-zero voxel: each ray's value is the length of the ray inside
    that voxel's cell (catches a wrong cell index or a shifted cell grid)."""
    vol, proj = _geom_case()
    rng = np.random.default_rng(5)
    pix = np.arange(proj.nu * proj.nv)
    S, P = _rays_by_rotation(proj, pix)
    for _ in range(4):
        v = [int(rng.integers(2, vol.n[c] - 2)) for c in range(3)]
        f = np.zeros(vol.shape_zyx)
        f[v[2], v[1], v[0]] = 2.0
        p = O.siddon_forward(vol, proj, f).reshape(-1)
        lo, hi = _cell_box(vol, v, v)
        L = np.array([_segment_in_box(S, P[r], lo, hi, n=20001) for r in pix])
        assert (L > 0).any()
        np.testing.assert_allclose(p, 2.0 * L, rtol=1e-7, atol=1e-7)


def test_siddon_matches_fine_riemann_sum():
    """A random voxel-constant volume: Siddon equals the limit of a fine
    midpoint sum of the nearest-cell value along the ray."""
    vol, proj = _geom_case()
    rng = np.random.default_rng(6)
    f = rng.uniform(0.0, 1.0, vol.shape_zyx)
    p = O.siddon_forward(vol, proj, f).reshape(-1)
    pix = np.arange(0, proj.nu * proj.nv, 7)
    S, P = _rays_by_rotation(proj, pix)
    s, o, n = np.array(vol.spacing), np.array(vol.origin), np.array(vol.n)
    m = 400000
    t = (np.arange(m) + 0.5) / m
    for k, r in enumerate(pix):
        d = P[k] - S
        X = S[None, :] + t[:, None] * d[None, :]
        q = np.floor((X - (o - 0.5 * s)) / s).astype(np.int64)
        ok = np.all((q >= 0) & (q < n), axis=1)
        vals = np.zeros(m)
        vals[ok] = f[q[ok, 2], q[ok, 1], q[ok, 0]]
        riemann = vals.sum() * np.linalg.norm(d) / m
        assert abs(riemann - p[r]) <= 1e-3 * max(abs(p[r]), 1e-9) + 1e-6


@pytest.mark.slow
def test_clinical_golden_is_stationary():
    """tests/golden/clinical_minimiser.json (the GPU full-size solve parity
    reference) is a minimiser of the current oracle's clinical objective:
    its gradient is below 1e-5 of the gradient at w = 0, for both fit modes."""
    gold = json.load(open(os.path.join(GOLDEN, "clinical_minimiser.json")))
    c = synth.clinical()
    assert gold["workload"] == c.name and gold["angle"] == c.proj.angle
    y = O.measured_projection(c.vol, c.proj, c.f0, c.mean, c.U, c.w_star, c.xi, c.noise_level)
    y = y.astype(np.float32).astype(np.float64)
    for key, fit in (("fit", True), ("nofit", False)):
        prob = O.Problem(c.vol, c.proj, c.f0, c.mean, c.U, y, fit_intensity=fit)
        g = prob.gradient(np.array(gold[key]["w"]), prob.objective(np.array(gold[key]["w"]))[3])
        g0 = prob.gradient(np.zeros(c.K), prob.objective(np.zeros(c.K))[3])
        assert np.linalg.norm(g) <= 1e-5 * np.linalg.norm(g0), key
