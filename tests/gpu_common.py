"""Shared helpers for the GPU tests (HIP path through the C ABI vs the oracle)."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1102_1712_amd import binding as B
from paper_1102_1712_amd import synth


def torch_or_skip():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    B.lib()      # fail loudly if the HIP library is missing
    return torch


def say(*msg):
    print("[gpu-test]", *msg, flush=True)
    sys.stdout.flush()


def tdt(case_or_dtype):
    import torch
    d = case_or_dtype if isinstance(case_or_dtype, str) else case_or_dtype.dtype
    return torch.float32 if d == "f32" else torch.float64


def to_dev(a, dtype):
    import torch
    if a is None:
        return None
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


RAY_DTYPES = {
    "f32": np.dtype([("e", "<f4", 3), ("d", "<f4", 3), ("dt", "<f4"), ("n", "<i4")]),
    "f64": np.dtype([("e", "<f8", 3), ("d", "<f8", 3), ("dt", "<f8"), ("n", "<i4"),
                     ("pad", "<i4")]),
}


def rays_np(rays_t, dtype: str):
    return rays_t.cpu().numpy().view(RAY_DTYPES[dtype])


class Dev:
    """A case's arrays on the GPU in its compute dtype."""

    def __init__(self, case):
        self.case = case
        self.dt = tdt(case)
        f0, mean, U = case.arrays()
        self.f0 = to_dev(f0, self.dt)
        self.mean = to_dev(mean, self.dt)
        self.U = to_dev(U, self.dt)
        self.rays = B.ray_table(case.vol, case.proj, self.dt)


def measured(case):
    """Measured projection from the oracle (FP64), rounded to the case dtype."""
    y = O.measured_projection(case.vol, case.proj, case.f0, case.mean, case.U, case.w_star,
                              case.xi, case.noise_level)
    np_dt = np.float32 if case.dtype == "f32" else np.float64
    return y.astype(np_dt).astype(np.float64)


SMALL_F64 = dict(dtype="f64", seed=5)
SMALL_F32 = dict(dtype="f32", seed=6)


def small(**kw):
    return synth.small(**kw)


def oracle_gauss_newton(case, y, w, fit=True):
    """The Gauss-Newton matrix of the reduced objective at w in oracle
    arithmetic: Q = [P J_1 .. P J_K] from the oracle's projections of the
    Jacobian volumes J_k = sum_c U_kc df/dx_c (Eq. A.8), then
    2 (Q^T Q - Q^T Y (Y^T Y)^-1 Y^T Q) with Y = [y, 1] (2 Q^T Q without the
    fit)."""
    c = case
    N = c.vol.nvox
    U = np.asarray(c.U, dtype=np.float64).reshape(c.K, 3, N)
    x = O.pca_dvf(c.vol, c.mean, c.U, w).reshape(3, N)
    jac = O.warp_jacobian(c.vol, c.f0, x).reshape(3, N)
    Q = np.stack([O.drr_forward(c.vol, c.proj, (U[k] * jac).sum(0)).ravel() for k in range(c.K)], 1)
    if not fit:
        return 2.0 * Q.T @ Q
    yv = np.asarray(y, dtype=np.float64).ravel()
    Y = np.stack([yv, np.ones_like(yv)], 1)
    QY = Q.T @ Y
    return 2.0 * (Q.T @ Q - QY @ np.linalg.solve(Y.T @ Y, QY.T))
