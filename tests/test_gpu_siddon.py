"""The exact-path (Siddon) projector against the oracle's independent
merged-crossings implementation, the half-fan detector offset for the
ray-march pair, and a solve whose measurement the solve's own P did not
make, against the oracle's solve of the same data."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_1102_1712_amd import binding as B
from paper_1102_1712_amd import synth

from gpu_common import Dev, rel_l2, say, to_dev, to_np, torch_or_skip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_or_skip()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("angle", [None, 0.0, np.pi / 4, 2.2])
def test_siddon_matches_oracle(torch, dtype, angle):
    c = synth.small(dtype=dtype, seed=31)
    if angle is not None:
        c = synth.with_angle(c, angle)
    d = Dev(c)
    say("siddon", dtype, angle)
    p = to_np(B.drr_siddon(c.vol, c.proj, d.f0))
    ref = O.siddon_forward(c.vol, c.proj, c.f0)
    assert (ref == 0).any() and (ref > 0).sum() > 100
    assert rel_l2(p, ref) <= (1e-13 if dtype == "f64" else 1e-6)
    assert np.all(p[ref == 0] == 0)


def test_siddon_clinical_f32(torch):
    """256x256x128, 512x384 detector: every pixel against the oracle."""
    c = synth.clinical()
    d = Dev(c)
    p = to_np(B.drr_siddon(c.vol, c.proj, d.f0))
    ref = O.siddon_forward(c.vol, c.proj, c.f0)
    assert rel_l2(p, ref) <= 1e-6


def test_siddon_half_fan_offset(torch):
    """A detector shifted by a third of its width (half-fan acquisition)."""
    c = synth.small(dtype="f64", seed=32)
    proj = dataclasses.replace(c.proj, offset_u=c.proj.nu * c.proj.pitch_u / 3.0)
    d = Dev(c)
    p = to_np(B.drr_siddon(c.vol, proj, d.f0))
    assert rel_l2(p, O.siddon_forward(c.vol, proj, c.f0)) <= 1e-13


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ray_march_pair_half_fan(torch, dtype):
    """The trilinear projection and its transpose with the offset detector."""
    c = synth.small(dtype=dtype, seed=33)
    proj = dataclasses.replace(c.proj, offset_u=-c.proj.nu * c.proj.pitch_u / 3.0,
                               offset_v=c.proj.pitch_v * 2.5)
    d = Dev(c)
    rays = B.ray_table(c.vol, proj, d.dt)
    tol = 1e-12 if dtype == "f64" else 1e-5
    p = to_np(B.drr_forward(c.vol, proj, rays, d.f0))
    assert rel_l2(p, O.drr_forward(c.vol, proj, c.f0)) <= tol
    r = np.random.default_rng(4).normal(size=(proj.nv, proj.nu))
    r = r.astype(np.float32 if dtype == "f32" else np.float64).astype(np.float64)
    bp = to_np(B.drr_adjoint(c.vol, proj, rays, to_dev(r, d.dt)))
    assert rel_l2(bp, O.drr_adjoint(c.vol, proj, r)) <= tol


def test_solve_with_exact_path_measurement(torch):
    """FP64: y from Siddon's projector (+1% noise), solved with the
    ray-march P (no inverse crime): the GPU solve's minimiser equals the
    oracle's on the same data."""
    c = synth.small(dtype="f64", seed=34)
    d = Dev(c)
    x = O.pca_dvf(c.vol, c.mean, c.U, c.w_star)
    f = O.warp(c.vol, c.f0, x)
    p = O.siddon_forward(c.vol, c.proj, f)
    y = p + 0.01 * np.sqrt(np.mean(p ** 2)) * c.xi
    w, rep = B.solve_projection(c.vol, c.proj, d.f0, d.mean, d.U, to_dev(y, d.dt), np.zeros(c.K),
                                B.default_opts())
    prob = O.Problem(c.vol, c.proj, c.f0, c.mean, c.U, y)
    w_o, _ = O.minimise(prob, np.zeros(c.K))
    say("exact-path data: gpu", w, rep["status"], "oracle", w_o, "planted", c.w_star)
    assert rep["status"] in ("converged", "line_search")
    assert np.linalg.norm(w - w_o) <= 1e-4 * np.linalg.norm(w_o)
