"""The back-projection's per-voxel weight bound (host logic, CPU).

The GPU back-projection sizes its fixed-point accumulators from
pcas_backprojection_bound: a brick's voxel totals must stay below
step * max|r| * B.  Here the bound is checked against the exact
back-projection of an all-ones image computed by the oracle, (P^T 1)(v) =
sum over rays and samples of dt * weight, on geometries chosen to stress it:
high magnification (source close to the volume), fine detector pitch,
detector offsets, anisotropic voxels, steep cone angles and steps above and
below the voxel size.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_1102_1712_amd import binding as B
from paper_1102_1712_amd import synth


def _geom(n, spacing, det, pitch, step, sad=1000.0, sid=1500.0, angle=0.3, offset=(0.0, 0.0)):
    vol = synth.centred_volume(n, spacing)
    proj = synth.Projection(angle=angle, sad=sad, sid=sid, nu=det[0], nv=det[1], pitch_u=pitch[0],
                            pitch_v=pitch[1], offset_u=offset[0], offset_v=offset[1], step=step)
    return vol, proj


GEOMS = {
    "tiny": _geom((64, 64, 64), (4.0, 4.0, 4.0), (128, 128), (3.0, 3.0), 2.0),
    "ragged_aniso": _geom((40, 36, 28), (5.0, 6.0, 7.0), (48, 40), (7.0, 8.0), 2.5),
    "fine_pitch": _geom((24, 24, 16), (2.0, 2.0, 3.0), (160, 120), (0.25, 0.25), 1.0),
    "close_source": _geom((32, 32, 24), (4.0, 4.0, 4.0), (200, 160), (1.0, 1.0), 2.0,
                          sad=120.0, sid=300.0, angle=0.9),
    "steep_cone": _geom((20, 20, 60), (3.0, 3.0, 3.0), (64, 200), (1.5, 1.5), 1.5,
                        sad=150.0, sid=400.0, angle=2.2),
    "half_fan": _geom((32, 32, 20), (4.0, 4.0, 5.0), (96, 64), (1.2, 1.2), 2.0,
                      offset=(40.0, -10.0), angle=4.0),
    "long_step": _geom((30, 30, 30), (1.0, 1.0, 1.0), (80, 80), (0.5, 0.5), 3.5),
    "short_step": _geom((30, 26, 22), (3.0, 2.0, 4.0), (64, 48), (2.0, 2.0), 0.3),
}


@pytest.mark.parametrize("name", sorted(GEOMS))
def test_backprojection_bound_holds(oracle_lib, name):
    vol, proj = GEOMS[name]
    bound = B.backprojection_bound(vol, proj)
    bp = O.drr_adjoint(vol, proj, np.ones(proj.nu * proj.nv))
    peak = float(bp.max())
    assert peak > 0.0
    assert peak <= proj.step * bound, (name, peak / (proj.step * bound))
    # not vacuous: within a modest factor of the exact peak
    assert proj.step * bound <= 200.0 * peak, (name, peak / (proj.step * bound))


def test_backprojection_bound_rejects_invalid():
    vol, proj = GEOMS["tiny"]
    with pytest.raises(B.PcasError):
        B.backprojection_bound(vol, dataclasses.replace(proj, step=0.0))
    with pytest.raises(B.PcasError):
        B.backprojection_bound(vol, dataclasses.replace(proj, sad=100.0))   # source inside


def _brick_halo_max(vol, bp, brick):
    """Largest value of bp over a 32 x 16 x 8 brick and its one-voxel halo
    (clipped to the grid); bricks numbered x fastest, then y, then z."""
    n1, n2, n3 = vol.n
    nbx, nby = -(-n1 // 32), -(-n2 // 16)
    bx, by, bz = brick % nbx, (brick // nbx) % nby, brick // (nbx * nby)
    lo = (bx * 32, by * 16, bz * 8)
    hi = (min(lo[0] + 32, n1) - 1, min(lo[1] + 16, n2) - 1, min(lo[2] + 8, n3) - 1)
    sl = bp[max(lo[2] - 1, 0):min(hi[2] + 1, n3 - 1) + 1,
            max(lo[1] - 1, 0):min(hi[1] + 1, n2 - 1) + 1,
            max(lo[0] - 1, 0):min(hi[0] + 1, n1 - 1) + 1]
    return float(sl.max())


@pytest.mark.parametrize("name", sorted(GEOMS))
def test_brick_bounds_hold(oracle_lib, name):
    """The per-brick bound that sizes every back-projection's fixed-point
    accumulators covers the exact (P^T 1) over each brick and its halo, on
    every stress geometry; and it is the tighter of the two bounds."""
    vol, proj = GEOMS[name]
    bp = O.drr_adjoint(vol, proj, np.ones(proj.nu * proj.nv))
    nb = B.backprojection_brick_count(vol)
    ratios = []
    for brick in range(nb):
        peak = _brick_halo_max(vol, bp, brick)
        bound = proj.step * B.backprojection_brick_bound(vol, proj, brick)
        assert peak <= bound, (name, brick, peak, bound)
        assert bound <= proj.step * B.backprojection_bound(vol, proj) * (1 + 1e-12)
        if peak > 0.0:
            ratios.append(bound / peak)
    assert ratios and min(ratios) >= 1.0
    with pytest.raises(B.PcasError):
        B.backprojection_brick_bound(vol, proj, nb)


def _live_bricks(vol, proj):
    """The liveness rule restated: a brick is live unless the images of the
    eight corners of its box with a one-voxel halo (clipped to the grid) all
    fall more than a pixel off the detector on one side (or one corner lies
    at or behind the source's plane)."""
    t = proj.angle
    src = np.array([proj.sad * np.sin(t), -proj.sad * np.cos(t), 0.0])
    eu, ev = np.array([np.cos(t), np.sin(t), 0.0]), np.array([0.0, 0.0, 1.0])
    en = np.array([-np.sin(t), np.cos(t), 0.0])
    n, s, o = np.array(vol.n), np.array(vol.spacing), np.array(vol.origin)
    ext = np.array([32, 16, 8])
    nb = -(-n // ext)
    live = np.zeros(nb[::-1], dtype=bool)          # [bz][by][bx]
    for bz in range(nb[2]):
        for by in range(nb[1]):
            for bx in range(nb[0]):
                lo = np.array([bx, by, bz]) * ext
                hi = np.minimum(lo + ext, n) - 1
                a, b = np.maximum(lo - 1, 0), np.minimum(hi + 1, n - 1)
                us, vs, behind = [], [], False
                for corner in range(8):
                    idx = np.where([(corner >> c) & 1 for c in range(3)], b, a)
                    rel = o + idx * s - src
                    depth = rel @ en
                    if not depth > 0.0:
                        behind = True
                        continue
                    us.append((rel @ eu) * proj.sid / depth - proj.offset_u)
                    vs.append((rel @ ev) * proj.sid / depth - proj.offset_v)
                u = np.array(us) / proj.pitch_u + 0.5 * (proj.nu - 1)
                v = np.array(vs) / proj.pitch_v + 0.5 * (proj.nv - 1)
                hit = len(us) > 0 and u.max() >= -1 and u.min() <= proj.nu and \
                    v.max() >= -1 and v.min() <= proj.nv
                live[bz, by, bx] = behind or hit
    return live


@pytest.mark.parametrize("name", sorted(GEOMS))
def test_live_bricks_hold_every_sampled_voxel(oracle_lib, name):
    """The warp inside a solve writes only the voxels of live bricks.  That
    is safe when every voxel a sample's cell touches -- every voxel where
    the oracle's P^T 1 is nonzero -- lies in a live brick; the library's
    count of live voxels follows the same rule."""
    vol, proj = GEOMS[name]
    live = _live_bricks(vol, proj)
    n = np.array(vol.n)
    mask = np.repeat(np.repeat(np.repeat(live, 8, 0), 16, 1), 32, 2)[:n[2], :n[1], :n[0]]
    assert B.live_voxels(vol, proj) == int(mask.sum())
    bp = O.drr_adjoint(vol, proj, np.ones(proj.nu * proj.nv)).reshape(n[2], n[1], n[0])
    assert np.all(mask[bp > 0.0])
    assert (bp > 0.0).sum() > 0


def test_clinical_live_fraction():
    """At the benchmark's geometry a little over half the bricks are live."""
    c = synth.clinical()
    frac = B.live_voxels(c.vol, c.proj) / np.prod(c.vol.n)
    assert 0.5 < frac < 0.7
