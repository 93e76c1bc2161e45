"""Autograd form: the hand-written backward (back-projection + Jacobian
chain) against central finite differences of the forward and against the
FP64 oracle gradient, including the K = 5 clinical-size workload."""
import numpy as np
import pytest

import oracle as O
from paper_1102_1712_amd import autograd as AG
from paper_1102_1712_amd import synth

from gpu_common import Dev, say, to_dev, to_np, torch_or_skip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_or_skip()


def _loss_and_grad(torch, d, w_np, r):
    c = d.case
    w = torch.tensor(w_np, dtype=torch.float64, requires_grad=True)
    p = AG.project(w, c.vol, c.proj, d.rays, d.f0, d.mean, d.U)
    L = (p.double() * r.double()).sum()
    L.backward()
    return float(L.detach()), w.grad.numpy().copy()


def _fd_grad(torch, d, f0, w0, r, h):
    c = d.case
    fd = np.zeros(c.K)
    for k in range(c.K):
        e = np.zeros(c.K)
        e[k] = h
        with torch.no_grad():
            Lp = float((AG.project(torch.tensor(w0 + e), c.vol, c.proj, d.rays, f0, d.mean, d.U)
                        .double() * r.double()).sum())
            Lm = float((AG.project(torch.tensor(w0 - e), c.vol, c.proj, d.rays, f0, d.mean, d.U)
                        .double() * r.double()).sum())
        fd[k] = (Lp - Lm) / (2 * h)
    return fd


def _smooth_case():
    c = synth.small(dtype="f64", seed=5)
    d = Dev(c)
    k, j, i = np.meshgrid(*[np.arange(n) for n in c.vol.shape_zyx], indexing="ij")
    smooth = (np.exp(-((i - 18) ** 2 + (j - 20) ** 2 + (k - 12) ** 2) / 60.0)
              + 0.5 * np.exp(-((i - 25) ** 2 + (j - 12) ** 2 + (k - 15) ** 2) / 30.0))
    d.f0 = to_dev(smooth, d.dt)
    return c, d, smooth


def test_backward_exact_against_kink_free_difference(torch):
    """FP64: with a step small enough that no voxel's warp position crosses a
    grid line (so the trilinear warp is linear over the stencil) the central
    difference equals the backward to rounding."""
    c, d, smooth = _smooth_case()
    r = torch.randn((c.proj.nv, c.proj.nu), device="cuda", dtype=torch.float64,
                    generator=torch.Generator(device="cuda").manual_seed(2))
    w0 = c.w_star + np.array([0.2, -0.1, 0.3])
    say("autograd kink-free FD")
    _, g = _loss_and_grad(torch, d, w0, r)
    s = np.array(c.vol.spacing)
    fd = np.zeros(c.K)
    for k in range(c.K):
        for h in (1e-6, 3e-7, 1e-7, 3e-8):
            e = np.zeros(c.K)
            e[k] = h
            xp, xm = O.pca_dvf(c.vol, c.mean, c.U, w0 + e), O.pca_dvf(c.vol, c.mean, c.U, w0 - e)
            if all(np.array_equal(np.floor(xp[q] / s[q]), np.floor(xm[q] / s[q])) for q in range(3)):
                break
        fd[k] = _fd_grad(torch, d, d.f0, w0, r, h)[k]
    assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(fd)


def test_backward_against_central_difference_h1e3(torch):
    """h = 1e-3 on w.  The GPU forward's differences equal the FP64 oracle's
    differences of the same discrete function; the backward differs from
    them only by the trilinear kinks the stencil crosses (O(h))."""
    c, d, smooth = _smooth_case()
    rng = np.random.default_rng(2)
    r_np = rng.normal(size=(c.proj.nv, c.proj.nu))
    r = to_dev(r_np, d.dt)
    w0 = c.w_star + np.array([0.2, -0.1, 0.3])
    say("autograd FD h=1e-3")
    _, g = _loss_and_grad(torch, d, w0, r)
    fd = _fd_grad(torch, d, d.f0, w0, r, 1e-3)
    fd_o = np.zeros(c.K)
    for k in range(c.K):
        e = np.zeros(c.K)
        e[k] = 1e-3
        Lp = np.sum(O.drr_forward(c.vol, c.proj, O.warp(c.vol, smooth, O.pca_dvf(c.vol, c.mean, c.U, w0 + e))) * r_np)
        Lm = np.sum(O.drr_forward(c.vol, c.proj, O.warp(c.vol, smooth, O.pca_dvf(c.vol, c.mean, c.U, w0 - e))) * r_np)
        fd_o[k] = (Lp - Lm) / 2e-3
    say("g", g, "fd", fd, "fd oracle", fd_o)
    assert np.linalg.norm(fd - fd_o) <= 1e-8 * np.linalg.norm(fd_o)
    assert np.linalg.norm(g - fd) <= 5e-3 * np.linalg.norm(fd)


def test_clinical_k5_central_difference(torch):
    """256x256x128 FP32, K = 5, h = 1e-3: backward vs central differences;
    with the phantom's sharp edges the kinks crossed by the stencil bound
    the agreement to about 1e-2."""
    c = synth.clinical_k5()
    d = Dev(c)
    r = torch.randn((c.proj.nv, c.proj.nu), device="cuda", dtype=torch.float32,
                    generator=torch.Generator(device="cuda").manual_seed(4))
    w0 = 0.5 * c.w_star
    say("autograd FD clinical K=5")
    _, g = _loss_and_grad(torch, d, w0, r)
    fd = _fd_grad(torch, d, d.f0, w0, r, 1e-3)
    say("g", g, "fd", fd)
    assert np.linalg.norm(g - fd) <= 2e-2 * np.linalg.norm(fd)


def test_backward_matches_oracle_gradient(torch):
    c = synth.small(dtype="f64", seed=7)
    d = Dev(c)
    rng = np.random.default_rng(9)
    r_np = rng.normal(size=(c.proj.nv, c.proj.nu))
    w0 = np.array([0.3, -0.6, 0.9])
    say("autograd vs oracle f64")
    _, g = _loss_and_grad(torch, d, w0, to_dev(r_np, d.dt))
    bp = O.drr_adjoint(c.vol, c.proj, r_np)
    g_ref = 0.5 * O.grad_w(c.vol, c.f0, c.mean, c.U, w0, bp)
    assert np.linalg.norm(g - g_ref) <= 1e-10 * np.linalg.norm(g_ref)


def test_clinical_k5_gradient(torch):
    """256x256x128 FP32, K = 5, 512x384 detector: autograd gradient of
    <p, r> vs the FP64 oracle within 1e-4."""
    c = synth.clinical_k5()
    d = Dev(c)
    rng = np.random.default_rng(10)
    r_np = rng.normal(size=(c.proj.nv, c.proj.nu)).astype(np.float32).astype(np.float64)
    w0 = 0.5 * c.w_star
    say("autograd clinical K=5")
    _, g = _loss_and_grad(torch, d, w0, to_dev(r_np, d.dt))
    bp = O.drr_adjoint(c.vol, c.proj, r_np)
    g_ref = 0.5 * O.grad_w(c.vol, c.f0, c.mean, c.U, w0, bp)
    say("g", g, "ref", g_ref)
    assert np.linalg.norm(g - g_ref) <= 1e-4 * np.linalg.norm(g_ref)


def test_module_and_store_warp_agree(torch):
    c = synth.small(dtype="f32", seed=6)
    d = Dev(c)
    say("PCAProjector store/recompute")
    r = torch.randn((c.proj.nv, c.proj.nu), device="cuda", dtype=torch.float32)
    grads = []
    for store in (False, True):
        m = AG.PCAProjector(c.vol, c.proj, d.f0, d.mean, d.U, store_warp=store)
        w = torch.tensor(c.w_star, dtype=torch.float64, requires_grad=True)
        (m(w).double() * r.double()).sum().backward()
        grads.append(w.grad.clone())
    assert torch.equal(grads[0], grads[1])


def test_set_projection_between_forward_and_backward(torch):
    """A graph recorded at angle A keeps A's ray table: switching the module
    to angle B before backward leaves the gradient equal to a fresh one at
    A, and overwriting the saved table in place raises instead."""
    c = synth.small(dtype="f64", seed=5)
    d = Dev(c)
    r = torch.randn((c.proj.nv, c.proj.nu), device="cuda", dtype=torch.float64,
                    generator=torch.Generator(device="cuda").manual_seed(12))
    say("autograd: set_projection before backward")
    m = AG.PCAProjector(c.vol, c.proj, d.f0, d.mean, d.U)
    w = torch.tensor(0.5 * c.w_star, dtype=torch.float64, requires_grad=True)
    loss = (m(w) * r).sum()
    m.set_projection(synth.with_angle(c, c.proj.angle + 0.7).proj)
    loss.backward()
    fresh = AG.PCAProjector(c.vol, c.proj, d.f0, d.mean, d.U)
    w2 = torch.tensor(0.5 * c.w_star, dtype=torch.float64, requires_grad=True)
    (fresh(w2) * r).sum().backward()
    assert torch.equal(w.grad, w2.grad)
    # an in-place change of the saved table is caught by autograd
    w3 = torch.tensor(0.5 * c.w_star, dtype=torch.float64, requires_grad=True)
    loss3 = (fresh(w3) * r).sum()
    fresh.rays.add_(0)
    with pytest.raises(RuntimeError):
        loss3.backward()
