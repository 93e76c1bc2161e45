"""The largest volume the library accepts: the kernels address a volume with
32-bit byte offsets, so an FP32 volume must stay below 2 GiB.  At
1024 x 1024 x 511 voxels (2 GiB - 4 MiB) the projection of every pixel of a
detector that covers the whole volume, and the whole back-projection in both
accumulator widths, match the FP64 oracle (the projection to 1e-5, the
back-projection to 1e-4, see below); the far slices, whose byte
offsets come within 4 MiB of 2^31, are reached; and a volume one slice
larger is refused before any GPU work.

The detector is coarse (64 x 48 pixels at 12 x 8 mm, magnification 1.5), so
that the oracle's samples stay few while its rays span every part of the
grid.  Inputs are seeded uniform values drawn on the GPU; both sides read
the same float32 values."""
import numpy as np
import pytest

import oracle as O
from paper_1102_1712_amd import binding as B
from paper_1102_1712_amd import synth

from gpu_common import rel_l2, say, to_np, torch_or_skip

pytestmark = pytest.mark.gpu

N_MAX = (1024, 1024, 511)


def _geometry(n):
    vol = synth.centred_volume(n, (0.5, 0.5, 0.5))
    proj = synth.Projection(angle=0.3, sad=1000.0, sid=1500.0, nu=64, nv=48, pitch_u=12.0,
                            pitch_v=8.0, step=0.25)
    return vol, proj


@pytest.fixture(scope="module")
def big():
    torch = torch_or_skip()
    vol, proj = _geometry(N_MAX)
    assert np.prod(vol.n) * 4 == (1 << 31) - (4 << 20)
    say("drawing the 2 GiB volume on the GPU")
    g = torch.Generator(device="cuda").manual_seed(91)
    f = torch.rand((N_MAX[2], N_MAX[1], N_MAX[0]), generator=g, device="cuda", dtype=torch.float32)
    rays = B.ray_table(vol, proj, torch.float32)
    return torch, vol, proj, f, rays


def test_max_size_forward_every_pixel(big):
    torch, vol, proj, f, rays = big
    say("max-size forward projection")
    p = to_np(B.drr_forward(vol, proj, rays, f)).reshape(-1)
    f64 = f.cpu().numpy().astype(np.float64)
    pix = np.arange(proj.nu * proj.nv)
    ref = O.drr_pixels(vol, proj, f64, pix)
    del f64
    err = rel_l2(p, ref)
    say("rel L2", err, "pixels hit", int((ref > 0).sum()))
    assert (ref > 0).sum() > 0.5 * pix.size
    assert err <= 1e-5


@pytest.mark.parametrize("acc32", [False, True])
def test_max_size_adjoint_whole_volume(big, acc32):
    torch, vol, proj, f, rays = big
    rng = np.random.default_rng(92)
    r = rng.normal(size=(proj.nv, proj.nu)).astype(np.float32)
    say("max-size back-projection, acc32", acc32)
    bp = to_np(B.drr_adjoint(vol, proj, rays, torch.from_numpy(r).cuda(), acc32=acc32))
    ref = O.drr_adjoint(vol, proj, r.astype(np.float64)).reshape(bp.shape)
    # the last slices (byte offsets within 4 MiB of 2^31) are reached and right
    far = slice(N_MAX[2] - 8, N_MAX[2])
    assert np.count_nonzero(ref[far]) > 1000
    err_far = rel_l2(bp[far], ref[far])
    err = rel_l2(bp, ref)
    say("rel L2", err, "far slices", err_far)
    # FP32 sample positions at index coordinates near 1024 are rounded to
    # about 2^-24 * 1024 = 6e-5 voxel, which moves every trilinear weight by
    # as much; the scatter keeps those per-sample errors (a ray sum averages
    # them), so the bar is the gradient's 1e-4 rather than the projection's
    # 1e-5.  A wrong byte offset would show as an O(1) error in the far slices.
    assert err <= 1e-4 and err_far <= 1e-4
    assert np.all(bp[ref == 0.0] == 0.0)


def test_one_slice_more_is_refused(big):
    torch = big[0]
    vol, proj = _geometry((N_MAX[0], N_MAX[1], N_MAX[2] + 1))   # exactly 2 GiB in FP32
    # the size check comes first, so the (small) buffers are never touched
    rays = torch.zeros(64, dtype=torch.uint8, device="cuda")
    f = torch.zeros(16, dtype=torch.float32, device="cuda")
    with pytest.raises(B.PcasError):
        B.drr_forward(vol, proj, rays, f)
    with pytest.raises(B.PcasError):
        B.drr_adjoint(vol, proj, rays, torch.zeros((proj.nv, proj.nu), device="cuda"),
                      out=torch.zeros(16, dtype=torch.float32, device="cuda"))
