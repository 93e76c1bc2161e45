"""Element-wise parity of P and P^T at the benchmark's full size: the
clinical workload (256x256x128 FP32 at 1.5 x 1.5 x 2.5 mm, 512x384 detector
at 0.8 mm, step 0.75 mm) through the C ABI against the FP64 oracle.

Both sides take the same inputs (float32 values, upcast exactly for the
oracle), so each comparison isolates one operator: the projection (Sec.
II.A, Eq. 2) and its transpose, the back-projection of the Appendix's
gradient, in both accumulator widths (64-bit drr_adjoint, and the 32-bit
accumulation of drr_adjoint32, which the solver's fused FP32 gradient
uses).  Three gantry angles: the benchmark's, whose rays travel mostly along
x; a quarter turn away, along y, so the projection's slab plan runs along
each in-plane axis; and 45 degrees, where rays cross both in-plane axes
alike and the staged boxes are largest.  Bar: relative L2 <= 1e-5."""
import numpy as np
import pytest

import oracle as O
from paper_1102_1712_amd import binding as B
from paper_1102_1712_amd import synth

from gpu_common import rel_l2, say, to_dev, to_np, torch_or_skip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def clinical():
    torch = torch_or_skip()
    say("building the clinical workload")
    c = synth.clinical()
    # the oracle's warped volume at half the planted coefficients, rounded to
    # float32: the projector's input on both sides
    x = O.pca_dvf(c.vol, c.mean, c.U, 0.5 * c.w_star)
    f = O.warp(c.vol, c.f0, x).astype(np.float32)
    rng = np.random.default_rng(71)
    r_noise = rng.normal(size=(c.proj.nv, c.proj.nu)).astype(np.float32)
    return torch, c, f, r_noise


def _angles(c):
    return {"bench": c.proj.angle, "quarter": c.proj.angle + 0.5 * np.pi,
            "diagonal": 0.25 * np.pi}


def _sample_pixels(proj):
    """Every border pixel (the cone's edge rays), an 8 x 8 lattice over the
    detector, and 1024 seeded random pixels: 5,856 of the 196,608 at the
    clinical size."""
    nu, nv = proj.nu, proj.nv
    iu, iv = np.meshgrid(np.arange(nu), np.arange(nv))
    border = (iu == 0) | (iu == nu - 1) | (iv == 0) | (iv == nv - 1)
    lattice = (iu % 8 == 3) & (iv % 8 == 5)
    flat = np.flatnonzero(border | lattice)
    rng = np.random.default_rng(72)
    extra = rng.choice(nu * nv, size=1024, replace=False)
    return np.unique(np.concatenate([flat, extra]))


@pytest.mark.parametrize("which", ["bench", "quarter", "diagonal"])
def test_clinical_forward_pixels(clinical, which):
    torch, c, f, _ = clinical
    proj = synth.with_angle(c, _angles(c)[which]).proj
    say("clinical forward parity", which, "angle", proj.angle)
    rays = B.ray_table(c.vol, proj, torch.float32)
    p = to_np(B.drr_forward(c.vol, proj, rays, to_dev(f, torch.float32))).reshape(-1)
    pix = _sample_pixels(proj)
    assert pix.size >= 4096
    ref = O.drr_pixels(c.vol, proj, f.astype(np.float64), pix)
    err = rel_l2(p[pix], ref)
    worst = float(np.max(np.abs(p[pix] - ref)) / np.max(np.abs(ref)))
    say("pixels", pix.size, "rel L2", err, "max |diff| / max |p|", worst)
    assert err <= 1e-5
    assert worst <= 1e-5


@pytest.mark.parametrize("acc32", [False, True])
@pytest.mark.parametrize("which", ["bench", "quarter", "diagonal"])
def test_clinical_adjoint_whole_volume(clinical, which, acc32):
    torch, c, _, r = clinical
    proj = synth.with_angle(c, _angles(c)[which]).proj
    say("clinical adjoint parity", which, "acc32", acc32)
    rays = B.ray_table(c.vol, proj, torch.float32)
    bp = to_np(B.drr_adjoint(c.vol, proj, rays, to_dev(r, torch.float32), acc32=acc32))
    ref = O.drr_adjoint(c.vol, proj, r.astype(np.float64))
    err = rel_l2(bp, ref)
    say("rel L2", err)
    assert err <= 1e-5
    # a voxel no sample reaches stays exactly zero
    assert np.all(bp[ref == 0.0] == 0.0)


def test_clinical_adjoint32_is_reproducible(clinical):
    """Fixed-point sums are order-independent: two launches give the same
    bits (the 32-bit accumulators included)."""
    torch, c, _, r = clinical
    rays = B.ray_table(c.vol, c.proj, torch.float32)
    rd = to_dev(r, torch.float32)
    a = B.drr_adjoint(c.vol, c.proj, rays, rd, acc32=True)
    b = B.drr_adjoint(c.vol, c.proj, rays, rd, acc32=True)
    assert torch.equal(a, b)
