"""Seeded synthetic inputs for the per-projection PCA solve.

This module only *draws* inputs: geometry records, a lung phantom, smooth
orthonormal motion modes, a planted coefficient vector, unit Gaussian noise
and a gantry angle.  It holds none of the method's arithmetic (no deformation
synthesis, no warp, no projection): both the HIP path and the FP64 oracle take
these arrays as given, and whoever needs a measured projection forms it with
its own forward model and then adds ``noise_level * rms(p) * xi``.

Recipe (the paper's data -- NCAT phantom, patient 4DCT -- is not available, so
these phantoms stand in for it; see Sec. II.B-II.D of the paper for the real
workloads):

* reference volume f0 (Sec. II.A, the reference image of Eq. 2): body
  ellipsoid 0.02/mm with semi-axes (0.45, 0.35, 0.48) x extent, two lung
  ellipsoids 0.005/mm centred at (+-0.20 E1, 0, 0) with semi-axes
  (0.15 E1, 0.22 E2, 0.30 E3), a 10 mm diameter tumour sphere 0.02/mm at
  (-0.20 E1, 0.05 E2, 0.10 E3); voxel centres are point-sampled; Gaussian
  texture sigma 0.001/mm is added inside the body only and the result is
  clamped at 0, so air is exactly 0.
* PCA eigenvectors u_k (Eq. 1): each is a sum of 8 Gaussian bumps (centre
  uniform in the body, sigma U(20, 50) mm, vector amplitude U(0, 10) mm along
  a random direction), then modified Gram-Schmidt in FP64 under the inner
  product <u, v> = (1/N) sum_voxels sum_c u_c v_c, so each mode has 1 mm RMS.
* mean DVF x-bar (Eq. 1): one more bump field scaled to 0.5 mm RMS (or None).
* planted w*: N(0, 1)^K, redrawn from the same stream until a Lipschitz bound
  guarantees the pull-back field does not fold:
  ||grad xbar|| + sum_k |w_k| ||grad u_k|| <= 0.5 (finite differences, mm/mm).
* measurement noise: xi ~ N(0, 1) per detector pixel (unit; scaled by caller).
* gantry angle: U[0, 2 pi).

Layouts: volumes are C-ordered ``[n3][n2][n1]`` (index i along axis 1 --
lateral -- fastest); vector fields ``[3][n3][n2][n1]`` with components
(lateral, AP, SI); modes ``[K][3][n3][n2][n1]``; detector images
``[nv][nu]`` with u fastest.  All lengths are in mm.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

__all__ = [
    "Volume", "Projection", "Case", "centred_volume", "make_case",
    "tiny", "recovery32", "clinical", "clinical_k5", "small",
]


@dataclass(frozen=True)
class Volume:
    """Regular voxel grid.  Voxel (i, j, k) has its centre at
    ``origin + (i, j, k) * spacing`` (mm); i is the fastest index."""

    n: Tuple[int, int, int]
    spacing: Tuple[float, float, float]
    origin: Tuple[float, float, float]

    @property
    def nvox(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def shape_zyx(self) -> Tuple[int, int, int]:
        return (int(self.n[2]), int(self.n[1]), int(self.n[0]))


@dataclass(frozen=True)
class Projection:
    """Circular cone-beam geometry for one projection.

    Source at (SAD sin t, -SAD cos t, 0); flat detector at distance SID from
    the source, u axis (cos t, sin t, 0), v axis (0, 0, 1) (the rotation /
    SI axis).  Pixel (iu, iv) centre sits at
    ``u = (iu - (nu-1)/2) * pitch_u + offset_u`` and likewise for v.
    ``step`` is the ray-march sample spacing in mm."""

    angle: float
    sad: float
    sid: float
    nu: int
    nv: int
    pitch_u: float
    pitch_v: float
    step: float
    offset_u: float = 0.0
    offset_v: float = 0.0

    @property
    def npix(self) -> int:
        return int(self.nu) * int(self.nv)


def centred_volume(n, spacing) -> Volume:
    n = tuple(int(v) for v in n)
    s = tuple(float(v) for v in spacing)
    origin = tuple(-(n[c] - 1) / 2.0 * s[c] for c in range(3))
    return Volume(n=n, spacing=s, origin=origin)


@dataclass
class Case:
    name: str
    vol: Volume
    proj: Projection
    dtype: str                       # "f32" or "f64": the GPU compute type
    K: int
    f0: np.ndarray                   # [n3][n2][n1] float64 (already rounded to dtype)
    mean: Optional[np.ndarray]       # [3][n3][n2][n1] or None
    U: np.ndarray                    # [K][3][n3][n2][n1]
    w_star: np.ndarray               # [K] float64
    xi: np.ndarray                   # [nv][nu] float64, unit normal
    tumour_c0: np.ndarray            # [3] mm, tumour centre in the reference image
    noise_level: float
    meta: dict = field(default_factory=dict)

    def arrays(self, np_dtype=None):
        """f0, mean, U cast to ``np_dtype`` (default: the case's dtype)."""
        if np_dtype is None:
            np_dtype = np.float32 if self.dtype == "f32" else np.float64
        f0 = np.ascontiguousarray(self.f0, dtype=np_dtype)
        mean = None if self.mean is None else np.ascontiguousarray(self.mean, dtype=np_dtype)
        U = np.ascontiguousarray(self.U, dtype=np_dtype)
        return f0, mean, U


# --------------------------------------------------------------------------
# drawing helpers
# --------------------------------------------------------------------------

def _axes(vol: Volume):
    return [vol.origin[c] + np.arange(vol.n[c]) * vol.spacing[c] for c in range(3)]


def _extent(vol: Volume) -> np.ndarray:
    return np.array(vol.n, dtype=np.float64) * np.array(vol.spacing, dtype=np.float64)


def _ellipsoid_mask(ax, centre, semi):
    x = ((ax[0] - centre[0]) / semi[0]) ** 2
    y = ((ax[1] - centre[1]) / semi[1]) ** 2
    z = ((ax[2] - centre[2]) / semi[2]) ** 2
    return (z[:, None, None] + y[None, :, None] + x[None, None, :]) <= 1.0


def phantom(vol: Volume, rng: np.random.Generator, texture_sigma: float = 0.001) -> np.ndarray:
    """Lung phantom in 1/mm, float64, [n3][n2][n1]."""
    ax = _axes(vol)
    E = _extent(vol)
    body_semi = np.array([0.45, 0.35, 0.48]) * E
    body = _ellipsoid_mask(ax, (0.0, 0.0, 0.0), body_semi)
    f = np.where(body, 0.02, 0.0)
    lung_semi = np.array([0.15, 0.22, 0.30]) * E
    for sgn in (+1.0, -1.0):
        lung = _ellipsoid_mask(ax, (sgn * 0.20 * E[0], 0.0, 0.0), lung_semi)
        f = np.where(lung & body, 0.005, f)
    c_t = np.array([-0.20 * E[0], 0.05 * E[1], 0.10 * E[2]])
    tumour = _ellipsoid_mask(ax, c_t, (5.0, 5.0, 5.0))
    f = np.where(tumour, 0.02, f)
    tex = rng.normal(0.0, texture_sigma, size=f.shape)
    f = np.where(body, np.maximum(f + tex, 0.0), 0.0)
    return f


def tumour_centre(vol: Volume) -> np.ndarray:
    E = _extent(vol)
    return np.array([-0.20 * E[0], 0.05 * E[1], 0.10 * E[2]])


def _bump_field(vol: Volume, rng: np.random.Generator, n_bumps: int = 8,
                sigma_range=(20.0, 50.0), amp_max: float = 10.0) -> np.ndarray:
    ax = _axes(vol)
    E = _extent(vol)
    semi = np.array([0.45, 0.35, 0.48]) * E
    out = np.zeros((3,) + vol.shape_zyx)
    for _ in range(n_bumps):
        while True:
            c = rng.uniform(-1.0, 1.0, 3) * semi
            if np.sum((c / semi) ** 2) <= 1.0:
                break
        sig = rng.uniform(*sigma_range)
        amp = rng.uniform(0.0, amp_max)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        g = [np.exp(-((ax[q] - c[q]) ** 2) / (2.0 * sig * sig)) for q in range(3)]
        G = g[2][:, None, None] * g[1][None, :, None] * g[0][None, None, :]
        for comp in range(3):
            out[comp] += (amp * d[comp]) * G
    return out


def _rms(v: np.ndarray, nvox: int) -> float:
    return float(np.sqrt(np.sum(v * v) / nvox))


def modes(vol: Volume, K: int, rng: np.random.Generator, progress=None) -> np.ndarray:
    """K orthonormal (1 mm RMS) smooth vector fields, [K][3][n3][n2][n1]."""
    N = vol.nvox
    fields = []
    for k in range(K):
        fields.append(_bump_field(vol, rng))
        if progress:
            progress(f"mode {k + 1}/{K} drawn")
    U = np.stack(fields)
    del fields
    for k in range(K):          # modified Gram-Schmidt
        for j in range(k):
            U[k] -= (np.sum(U[k] * U[j]) / N) * U[j]
        U[k] /= _rms(U[k], N)
    return U


def mean_field(vol: Volume, rng: np.random.Generator, rms_mm: float = 0.5) -> np.ndarray:
    m = _bump_field(vol, rng)
    return m * (rms_mm / _rms(m, vol.nvox))


def _max_jacobian_norm(field3: np.ndarray, vol: Volume) -> float:
    """max over voxels of the Frobenius norm of the finite-difference
    Jacobian of a 3-component field (mm per mm)."""
    s = vol.spacing
    acc = np.zeros(vol.shape_zyx)
    for comp in range(3):
        grads = np.gradient(field3[comp], s[2], s[1], s[0])
        for g in grads:
            acc += g * g
    return float(np.sqrt(acc.max()))


def planted_w(K: int, rng: np.random.Generator, mode_bounds, mean_bound: float,
              limit: float = 0.5, max_draws: int = 10000) -> np.ndarray:
    for _ in range(max_draws):
        w = rng.normal(0.0, 1.0, K)
        if mean_bound + float(np.sum(np.abs(w) * np.asarray(mode_bounds))) <= limit:
            return w
    raise RuntimeError("could not draw a non-folding planted w")


# --------------------------------------------------------------------------
# cases
# --------------------------------------------------------------------------

def make_case(name: str, n, spacing, det, pitch, step, K: int, dtype: str, seed: int,
              noise_level: float = 0.01, with_mean: bool = True, angle=None,
              sad: float = 1000.0, sid: float = 1500.0, offset_u: float = 0.0,
              progress=None) -> Case:
    """progress: optional callable told each finished stage (large volumes
    take minutes to draw)."""
    vol = centred_volume(n, spacing)
    ss = np.random.SeedSequence(seed).spawn(6)
    r_tex, r_modes, r_mean, r_w, r_noise, r_angle = (np.random.default_rng(s) for s in ss)
    f0 = phantom(vol, r_tex)
    if progress:
        progress(f"{name}: phantom drawn")
    U = modes(vol, K, r_modes, progress)
    mean = mean_field(vol, r_mean) if with_mean else None
    if progress:
        progress(f"{name}: modes and mean field done")
    np_dt = np.float32 if dtype == "f32" else np.float64
    # round to the compute type once; every consumer sees the same discrete problem
    f0 = f0.astype(np_dt).astype(np.float64)
    U = U.astype(np_dt).astype(np.float64)
    if mean is not None:
        mean = mean.astype(np_dt).astype(np.float64)
    mb = []
    for k in range(K):
        mb.append(_max_jacobian_norm(U[k], vol))
        if progress:
            progress(f"{name}: mode {k + 1}/{K} gradient bound")
    meanb = 0.0 if mean is None else _max_jacobian_norm(mean, vol)
    w_star = planted_w(K, r_w, mb, meanb)
    theta = float(r_angle.uniform(0.0, 2.0 * np.pi)) if angle is None else float(angle)
    proj = Projection(angle=theta, sad=sad, sid=sid, nu=int(det[0]), nv=int(det[1]),
                      pitch_u=float(pitch[0]), pitch_v=float(pitch[1]), step=float(step),
                      offset_u=float(offset_u))
    xi = r_noise.normal(0.0, 1.0, (proj.nv, proj.nu))
    return Case(name=name, vol=vol, proj=proj, dtype=dtype, K=K, f0=f0, mean=mean, U=U,
                w_star=w_star, xi=xi, tumour_c0=tumour_centre(vol), noise_level=noise_level,
                meta={"seed": seed, "mode_grad_bounds": mb, "mean_grad_bound": meanb})


def tiny(seed: int = 0, **kw) -> Case:
    """64^3 FP64 at 4 mm, K=3, 128x128 detector at 3 mm, step 2 mm, 1% noise."""
    return make_case("tiny-64^3-f64", (64, 64, 64), (4.0, 4.0, 4.0), (128, 128), (3.0, 3.0),
                     2.0, 3, "f64", seed, **kw)


def recovery32(seed: int = 10, **kw) -> Case:
    """32^3 FP64 at 8 mm, K=3, 64x64 detector at 6 mm, step 4 mm, noise-free."""
    kw.setdefault("noise_level", 0.0)
    return make_case("recovery-32^3-f64", (32, 32, 32), (8.0, 8.0, 8.0), (64, 64), (6.0, 6.0),
                     4.0, 3, "f64", seed, **kw)


def clinical(seed: int = 1, K: int = 3, **kw) -> Case:
    """256x256x128 FP32 at 1.5x1.5x2.5 mm, K=3, 512x384 detector at 0.8 mm,
    step 0.75 mm (half the smallest voxel spacing), 1% noise."""
    return make_case(f"clinical-256x256x128-K{K}-f32", (256, 256, 128), (1.5, 1.5, 2.5),
                     (512, 384), (0.8, 0.8), 0.75, K, "f32", seed, **kw)


def clinical_k5(seed: int = 2, **kw) -> Case:
    return clinical(seed=seed, K=5, **kw)


def small(n=(40, 36, 28), spacing=(5.0, 6.0, 7.0), det=(48, 40), pitch=(7.0, 8.0), step=2.5,
          K: int = 3, dtype: str = "f64", seed: int = 5, **kw) -> Case:
    """Ragged anisotropic case for parity tests (no dimension a tile multiple)."""
    return make_case("small", n, spacing, det, pitch, step, K, dtype, seed, **kw)


def with_angle(case: Case, angle: float) -> Case:
    return replace(case, proj=replace(case.proj, angle=float(angle)))


def serve_small(seed: int = 40, **kw) -> Case:
    """Serving mix, small requests: 128x128x96 FP32 at 3 x 3 x 3.33 mm, K=3,
    512x384 detector at 0.4 mm, step 1.5 mm."""
    return make_case("serve-128x128x96-K3-f32", (128, 128, 96), (3.0, 3.0, 10.0 / 3.0),
                     (512, 384), (0.4, 0.4), 1.5, 3, "f32", seed, **kw)


def serve_large(seed: int = 41, **kw) -> Case:
    """Serving mix, large requests: 512x512x256 FP32 at 0.75 x 0.75 x 1.25 mm,
    K=5, 1024x768 detector at 0.4 mm, step 0.375 mm."""
    return make_case("serve-512x512x256-K5-f32", (512, 512, 256), (0.75, 0.75, 1.25),
                     (1024, 768), (0.4, 0.4), 0.375, 5, "f32", seed, **kw)
