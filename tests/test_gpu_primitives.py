"""Primitive parity: each C-ABI entry point against the FP64 oracle on the
same inputs, at sizes spanning several tiles / bricks with ragged edges.

Tolerances: FP64 paths agree to rounding (1e-11 .. 1e-12 relative); FP32
paths use the projection bound of 1e-5 relative L2 (and 1e-4 for the
gradient), with FP64 accumulation inside every reduction."""
import numpy as np
import pytest

import oracle as O
from paper_1102_1712_amd import binding as B
from paper_1102_1712_amd import synth

from gpu_common import (Dev, measured, rays_np, rel_l2, say, small, tdt, to_dev, to_np,
                        torch_or_skip)

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-11, "f32": 1e-5}


@pytest.fixture(scope="module")
def torch():
    return torch_or_skip()


@pytest.fixture(scope="module", params=["f64", "f32"])
def sm(request, torch):
    case = small(dtype=request.param, seed=5 if request.param == "f64" else 6)
    say("small case", request.param, case.vol.n, (case.proj.nu, case.proj.nv))
    return Dev(case)


def test_ray_table_matches_oracle(sm):
    c = sm.case
    torch = __import__("torch")
    torch.cuda.synchronize()
    rec = rays_np(sm.rays, c.dtype).reshape(c.proj.nv, c.proj.nu)
    t_in, L, ns, dt = O.ray_table(c.vol, c.proj)
    assert np.array_equal(rec["n"], ns), "sample counts differ"
    assert (ns == 0).sum() > 0 and (ns > 0).sum() > 100       # misses and hits both present
    hit = ns > 0
    tol = 1e-6 if c.dtype == "f32" else 1e-14
    np.testing.assert_allclose(rec["dt"][hit], dt[hit], rtol=tol)


def test_drr_forward(sm):
    c = sm.case
    rng = np.random.default_rng(11)
    f = c.f0 + 0.003 * rng.uniform(size=c.f0.shape)
    f = f.astype(np.float32 if c.dtype == "f32" else np.float64).astype(np.float64)
    say("drr_forward", c.dtype)
    p = to_np(B.drr_forward(c.vol, c.proj, sm.rays, to_dev(f, sm.dt)))
    ref = O.drr_forward(c.vol, c.proj, f)
    assert rel_l2(p, ref) <= TOL[c.dtype]
    assert np.all(p[ref == 0] == 0)


def test_drr_adjoint(sm):
    c = sm.case
    rng = np.random.default_rng(12)
    r = rng.normal(size=(c.proj.nv, c.proj.nu))
    r = r.astype(np.float32 if c.dtype == "f32" else np.float64).astype(np.float64)
    say("drr_adjoint", c.dtype)
    bp = to_np(B.drr_adjoint(c.vol, c.proj, sm.rays, to_dev(r, sm.dt)))
    ref = O.drr_adjoint(c.vol, c.proj, r)
    assert rel_l2(bp, ref) <= TOL[c.dtype]


def test_adjoint_identity_on_gpu(sm, torch):
    """<P x, y> = <x, P^T y> for the GPU pair itself (same ray table)."""
    c = sm.case
    g = torch.Generator(device="cuda").manual_seed(3)
    x = torch.rand(c.vol.shape_zyx, generator=g, device="cuda", dtype=sm.dt)
    y = torch.randn((c.proj.nv, c.proj.nu), generator=g, device="cuda", dtype=sm.dt)
    say("adjoint identity", c.dtype)
    Px = B.drr_forward(c.vol, c.proj, sm.rays, x)
    PTy = B.drr_adjoint(c.vol, c.proj, sm.rays, y)
    lhs = float((Px.double() * y.double()).sum())
    rhs = float((x.double() * PTy.double()).sum())
    tol = 1e-12 if c.dtype == "f64" else 1e-5
    assert abs(lhs - rhs) <= tol * abs(lhs)


def test_adjoint_bitwise_reproducible(sm, torch):
    c = sm.case
    r = torch.randn((c.proj.nv, c.proj.nu), device="cuda", dtype=sm.dt)
    say("adjoint repeat", c.dtype)
    a = B.drr_adjoint(c.vol, c.proj, sm.rays, r)
    b = B.drr_adjoint(c.vol, c.proj, sm.rays, r)
    assert torch.equal(a, b)


def test_pca_dvf_and_warps(sm):
    c = sm.case
    w = np.array([0.7, -1.1, 0.4])
    say("pca_dvf / warp", c.dtype)
    dvf = B.pca_dvf(sm.mean, sm.U, w)
    ref_x = O.pca_dvf(c.vol, c.mean, c.U, w)
    tol = 1e-6 if c.dtype == "f32" else 1e-14
    assert rel_l2(to_np(dvf), ref_x) <= tol
    f_a = to_np(B.warp_trilinear(c.vol, sm.f0, dvf))
    f_b = to_np(B.warp_pca(c.vol, sm.f0, sm.mean, sm.U, w))
    # the oracle warps with the GPU's (rounded) field, isolating the warp
    ref_f = O.warp(c.vol, c.f0, to_np(dvf))
    tolw = 2e-6 if c.dtype == "f32" else 1e-12
    assert rel_l2(f_a, ref_f) <= tolw
    assert rel_l2(f_b, O.warp(c.vol, c.f0, ref_x)) <= tolw


def test_identity_warp_bitwise(sm, torch):
    c = sm.case
    say("identity warp", c.dtype)
    f = B.warp_pca(c.vol, sm.f0, None, sm.U, np.zeros(c.K))
    assert torch.equal(f, sm.f0)
    zero = torch.zeros((3,) + c.vol.shape_zyx, device="cuda", dtype=sm.dt)
    assert torch.equal(B.warp_trilinear(c.vol, sm.f0, zero), sm.f0)


def test_integer_shift_warp(sm, torch):
    c = sm.case
    s = c.vol.spacing
    x = np.empty((3,) + c.vol.shape_zyx)
    x[0], x[1], x[2] = -2 * s[0], 3 * s[1], 1 * s[2]
    say("integer shift", c.dtype)
    f = to_np(B.warp_trilinear(c.vol, sm.f0, to_dev(x, sm.dt)))
    expect = np.zeros_like(c.f0)
    expect[:-1, :-3, 2:] = c.f0[1:, 3:, :-2]     # f(i,j,k) = f0(i-2, j+3, k+1)
    bad = np.argwhere(f != expect)
    if bad.size:
        say("mismatches", len(bad), "first (k,j,i):", bad[:6].tolist())
        for k, j, i in bad[:6]:
            say("  got", repr(f[k, j, i]), "expected", repr(expect[k, j, i]))
    assert bad.size == 0


def test_grad_w(sm, torch):
    c = sm.case
    rng = np.random.default_rng(13)
    bp = rng.normal(size=c.vol.shape_zyx)
    bp = bp.astype(np.float32 if c.dtype == "f32" else np.float64).astype(np.float64)
    for w in (np.zeros(c.K), c.w_star + np.array([0.3, -0.2, 0.25])):
        say("grad_w", c.dtype, w)
        g = to_np(B.grad_w(c.vol, sm.f0, sm.mean, sm.U, w, to_dev(bp, sm.dt)))
        ref = O.grad_w(c.vol, c.f0, c.mean, c.U, w, bp)
        tol = 1e-4 if c.dtype == "f32" else 1e-10
        assert np.linalg.norm(g - ref) <= tol * np.linalg.norm(ref)


def test_grad_w_bitwise_reproducible(sm, torch):
    c = sm.case
    bp = torch.randn(c.vol.shape_zyx, device="cuda", dtype=sm.dt)
    say("grad repeat", c.dtype)
    a = B.grad_w(c.vol, sm.f0, sm.mean, sm.U, c.w_star, bp)
    b = B.grad_w(c.vol, sm.f0, sm.mean, sm.U, c.w_star, bp)
    assert torch.equal(a, b)


@pytest.mark.parametrize("fit", [True, False])
def test_residual_fit(sm, fit):
    c = sm.case
    rng = np.random.default_rng(14)
    y = rng.uniform(0.5, 3.0, (c.proj.nv, c.proj.nu))
    p = 0.8 * y + 0.3 + rng.normal(0, 0.05, y.shape)
    np_dt = np.float32 if c.dtype == "f32" else np.float64
    y, p = y.astype(np_dt).astype(np.float64), p.astype(np_dt).astype(np.float64)
    say("residual_fit", c.dtype, fit)
    r, stats = B.residual_fit(to_dev(p, sm.dt), to_dev(y, sm.dt), fit_intensity=fit)
    st = to_np(stats)
    a, b = O.intensity_fit(p, y) if fit else (1.0, 0.0)
    rr = p - a * y - b
    np.testing.assert_allclose(st[1:3], [a, b], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(st[0], np.sum(rr * rr), rtol=1e-10)
    np.testing.assert_allclose(st[3:], [p.sum(), (p * y).sum(), (p * p).sum(), y.sum(),
                                        (y * y).sum()], rtol=1e-12)
    tolr = 1e-6 if c.dtype == "f32" else 1e-12
    assert rel_l2(to_np(r), rr) <= tolr


def test_residual_fit_singular(torch):
    y = torch.full((37, 41), 2.5, device="cuda", dtype=torch.float64)
    p = torch.rand((37, 41), device="cuda", dtype=torch.float64)
    say("residual_fit singular")
    _, st = B.residual_fit(p, y, fit_intensity=True)
    assert np.isnan(to_np(st)[:3]).all()


def test_tumour_position(sm):
    c = sm.case
    w = c.w_star
    say("tumour_position", c.dtype)
    out = to_np(B.tumour_position(c.vol, sm.mean, sm.U, w, c.tumour_c0))
    ref, it = O.locate(c.vol, c.mean, c.U, w, c.tumour_c0)
    assert it > 0 and out[3] > 0
    tol = 1e-5 if c.dtype == "f32" else 1e-9
    np.testing.assert_allclose(out[:3], ref, atol=tol)


def test_tiny_config_primitives(torch):
    """64^3 FP64 at 4 mm with the 128x128 detector (the tiny workload)."""
    c = synth.tiny()
    d = Dev(c)
    say("tiny primitives")
    w = c.w_star
    f = to_np(B.warp_pca(c.vol, d.f0, d.mean, d.U, w))
    x = O.pca_dvf(c.vol, c.mean, c.U, w)
    f_ref = O.warp(c.vol, c.f0, x)
    assert rel_l2(f, f_ref) <= 1e-12
    p = to_np(B.drr_forward(c.vol, c.proj, d.rays, to_dev(f_ref, d.dt)))
    p_ref = O.drr_forward(c.vol, c.proj, f_ref)
    assert rel_l2(p, p_ref) <= 1e-12
    r = p_ref - measured(c)
    bp = to_np(B.drr_adjoint(c.vol, c.proj, d.rays, to_dev(r, d.dt)))
    bp_ref = O.drr_adjoint(c.vol, c.proj, r)
    assert rel_l2(bp, bp_ref) <= 1e-12
    g = to_np(B.grad_w(c.vol, d.f0, d.mean, d.U, w, to_dev(bp_ref, d.dt)))
    g_ref = O.grad_w(c.vol, c.f0, c.mean, c.U, w, bp_ref)
    assert np.linalg.norm(g - g_ref) <= 1e-10 * np.linalg.norm(g_ref)
