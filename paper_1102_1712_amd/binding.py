"""Thin Python binding over the libpcasolve C ABI (``include/pcasolve.h``).

Argument marshalling only: every step runs in the HIP library.  Device
arrays are ``torch`` tensors on a ROCm device (PyTorch supplies memory and
the current stream, nothing else); geometry is any object with the
attributes of ``synth.Volume`` / ``synth.Projection``.  There is no CPU
fallback: if the shared library is missing the first call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpcasolve.so")

PCAS_F32, PCAS_F64 = 0, 1
STATUS = {0: "ok", -1: "invalid argument", -2: "invalid geometry", -3: "singular intensity fit",
          -4: "non-finite input or objective", -5: "workspace", -6: "HIP runtime error"}
STOP = {0: "converged", 1: "max_iter", 2: "line_search"}
EXPORTS = ("pcas_abi_version", "pcas_status_string", "pcas_last_error", "pcas_default_opts",
           "pcas_paper_opts", "pcas_ray_table_bytes", "ray_table", "pca_dvf", "warp_trilinear",
           "warp_pca", "drr_forward", "drr_siddon", "drr_adjoint", "drr_adjoint32",
           "pcas_backprojection_bound", "pcas_backprojection_brick_bound",
           "backprojection_brick_count", "pcas_live_voxels",
           "residual_fit_workspace_bytes",
           "residual_fit", "grad_w_workspace_bytes", "grad_w", "tumour_position",
           "objective_gradient", "solve_projection_workspace", "solve_projection",
           "pcas_server_reserved_bytes", "pcas_server_create", "pcas_server_destroy",
           "pcas_server_add_model", "pcas_server_request_bytes", "pcas_server_submit",
           "pcas_server_step", "pcas_server_set_substep_share", "pcas_server_poll",
           "pcas_server_stats", "pcas_predict", "pcas_fit_predictor",
           "grad_w_noalloc_scratch_bytes", "grad_w_noalloc")


class PcasError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        self.code = code
        msg = f"{where}: {STATUS.get(code, 'unknown')} ({code})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


class Vol(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("spacing", ctypes.c_double * 3),
                ("origin", ctypes.c_double * 3)]


class Proj(ctypes.Structure):
    _fields_ = [("angle", ctypes.c_double), ("sad", ctypes.c_double), ("sid", ctypes.c_double),
                ("nu", ctypes.c_int32), ("nv", ctypes.c_int32),
                ("pitch_u", ctypes.c_double), ("pitch_v", ctypes.c_double),
                ("offset_u", ctypes.c_double), ("offset_v", ctypes.c_double),
                ("step", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("fit_intensity", ctypes.c_int32), ("max_backtracks", ctypes.c_int32),
                ("mu0", ctypes.c_double), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("mu_min", ctypes.c_double), ("gtol_rel", ctypes.c_double),
                ("beta_lo", ctypes.c_double), ("xtol", ctypes.c_double),
                ("locate", ctypes.c_int32), ("locate_max_iter", ctypes.c_int32),
                ("locate_tol", ctypes.c_double), ("c0_mm", ctypes.c_double * 3),
                ("profile", ctypes.c_int32), ("grad_mode", ctypes.c_int32),
                ("ftol_rel", ctypes.c_double), ("ls_extrap", ctypes.c_double),
                ("polish", ctypes.c_int32), ("speculate", ctypes.c_int32),
                ("precond", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("n_fevals", ctypes.c_int32), ("n_grads", ctypes.c_int32),
                ("J0", ctypes.c_double), ("J", ctypes.c_double), ("a", ctypes.c_double),
                ("b", ctypes.c_double), ("gnorm0", ctypes.c_double), ("gnorm", ctypes.c_double),
                ("tumour_mm", ctypes.c_double * 3), ("locate_iters", ctypes.c_int32),
                ("spec_grads", ctypes.c_int32), ("kernel_ms", ctypes.c_double * 13),
                ("kernel_launches", ctypes.c_int32 * 13), ("host_ms", ctypes.c_double),
                ("wait_ms", ctypes.c_double)]


# report.kernel_ms classes; in a solve class 4 is the back-projection with the
# Jacobian chain fused into it, class 10 a speculative launch of it whose gate
# was shut (it exited at once), classes 11 and 12 the two launches of a fused
# evaluation (grad_mode 2)
KERNEL_CLASSES = ("ray_table", "warp_pca", "drr_forward", "residual", "drr_adjoint_chain",
                  "grad_w", "tumour_position", "y_sums", "jacobian", "drr_forward_dot",
                  "spec_skipped", "warp_jac", "drr_forward_eval")
PROFILE_ALL = (1 << len(KERNEL_CLASSES)) - 1


def profile_mask(*classes: str) -> int:
    """opts.profile value that times the named kernel classes (all if none)."""
    if not classes:
        return PROFILE_ALL
    return sum(1 << KERNEL_CLASSES.index(c) for c in set(classes))


_lib = None


def lib():
    """Load libpcasolve.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; run `python -m paper_1102_1712_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, SZ, D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t,
                              ctypes.c_double)
        VP, PP = ctypes.POINTER(Vol), ctypes.POINTER(Proj)
        DP = ctypes.POINTER(ctypes.c_double)
        sig = {
            "pcas_abi_version": (I32, []),
            "pcas_status_string": (ctypes.c_char_p, [I32]),
            "pcas_last_error": (ctypes.c_char_p, []),
            "pcas_default_opts": (None, [ctypes.POINTER(Opts)]),
            "pcas_paper_opts": (None, [ctypes.POINTER(Opts)]),
            "pcas_ray_table_bytes": (SZ, [I32, PP]),
            "ray_table": (I32, [I32, VP, PP, P, P]),
            "pca_dvf": (I32, [I32, I64, I32, P, P, DP, P, P]),
            "warp_trilinear": (I32, [I32, VP, P, P, P, P]),
            "warp_pca": (I32, [I32, VP, I32, P, P, P, DP, P, P]),
            "drr_forward": (I32, [I32, VP, PP, P, P, P, P]),
            "drr_adjoint": (I32, [I32, VP, PP, P, P, P, P]),
            "drr_adjoint32": (I32, [I32, VP, PP, P, P, P, P]),
            "drr_siddon": (I32, [I32, VP, PP, P, P, P]),
            "pcas_backprojection_bound": (D, [VP, PP]),
            "pcas_backprojection_brick_bound": (D, [VP, PP, I32]),
            "backprojection_brick_count": (I32, [VP]),
            "pcas_live_voxels": (I64, [VP, PP]),
            "residual_fit_workspace_bytes": (SZ, [I64]),
            "residual_fit": (I32, [I32, I64, P, P, I32, P, P, P, SZ, P]),
            "grad_w_workspace_bytes": (SZ, [I32, VP, I32]),
            "grad_w": (I32, [I32, VP, I32, P, P, P, DP, P, P, P, SZ, P]),
            "tumour_position": (I32, [I32, VP, I32, P, P, DP, DP, D, I32, P, P]),
            "objective_gradient": (I32, [I32, VP, PP, I32, P, P, P, P, DP, I32, I32, P, SZ, DP,
                                         P]),
            "pcas_server_reserved_bytes": (SZ, [I32]),
            "pcas_server_create": (I32, [P, SZ, I32, P, ctypes.POINTER(P)]),
            "pcas_server_destroy": (I32, [P]),
            "pcas_server_add_model": (I32, [P, I32, VP, I32, P, P, P, ctypes.POINTER(I32)]),
            "pcas_server_request_bytes": (SZ, [P, I32, PP, ctypes.POINTER(Opts)]),
            "pcas_server_submit": (I32, [P, I32, PP, P, DP, ctypes.POINTER(Opts),
                                         ctypes.POINTER(I64)]),
            "pcas_server_set_substep_share": (I32, [P, D]),
            "pcas_server_step": (I32, [P, ctypes.POINTER(I32)]),
            "pcas_server_poll": (I32, [P, I64, DP, ctypes.POINTER(Report), ctypes.POINTER(I32)]),
            "pcas_server_stats": (I32, [P, ctypes.POINTER(I32), ctypes.POINTER(I32),
                                        ctypes.POINTER(SZ)]),
            "pcas_predict": (I32, [I32, I32, DP, DP, I32, DP]),
            "grad_w_noalloc_scratch_bytes": (SZ, []),
            "grad_w_noalloc": (I32, [I32, VP, I32, P, P, P, DP, P, P, P]),
            "pcas_fit_predictor": (I32, [I32, I32, I32, DP, DP]),
            "solve_projection_workspace": (SZ, [I32, VP, PP, I32]),
            "solve_projection": (I32, [I32, VP, PP, I32, P, P, P, P, DP, ctypes.POINTER(Opts), P,
                                       SZ, DP, ctypes.POINTER(Report), P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def c_vol(vol) -> Vol:
    v = Vol()
    for c in range(3):
        v.n[c] = int(vol.n[c])
        v.spacing[c] = float(vol.spacing[c])
        v.origin[c] = float(vol.origin[c])
    return v


def c_proj(pr) -> Proj:
    return Proj(float(pr.angle), float(pr.sad), float(pr.sid), int(pr.nu), int(pr.nv),
                float(pr.pitch_u), float(pr.pitch_v), float(getattr(pr, "offset_u", 0.0)),
                float(getattr(pr, "offset_v", 0.0)), float(pr.step))


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return PCAS_F32
    if t.dtype == torch.float64:
        return PCAS_F64
    raise TypeError(f"unsupported dtype {t.dtype} (float32 or float64)")


def _dev(t, name: str, dtype=None):
    """Check a device tensor argument and return its pointer."""
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _host_doubles(w, n: Optional[int] = None):
    torch = _torch()
    if isinstance(w, torch.Tensor):
        w = w.detach().to("cpu", torch.float64).numpy()
    a = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(-1))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} coefficients, got {a.size}")
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check(code: int, where: str):
    if code != 0:
        detail = lib().pcas_last_error().decode() if code == -6 else ""
        raise PcasError(code, where, detail)


def _nvox(vol) -> int:
    return int(vol.n[0]) * int(vol.n[1]) * int(vol.n[2])


def _vshape(vol):
    return (int(vol.n[2]), int(vol.n[1]), int(vol.n[0]))


def _K_of(U, vol) -> int:
    N = _nvox(vol)
    if U.numel() % (3 * N):
        raise ValueError("U must hold K x 3 x N values")
    return U.numel() // (3 * N)


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def ray_table(vol, proj, dtype, out=None, stream=None):
    """a1: per-pixel ray records as a byte tensor on the current device."""
    torch = _torch()
    code = PCAS_F32 if dtype == torch.float32 else PCAS_F64
    cp = c_proj(proj)
    nbytes = lib().pcas_ray_table_bytes(code, ctypes.byref(cp))
    if out is None:
        out = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    elif out.numel() < nbytes:
        raise ValueError("ray table buffer too small")
    _check(lib().ray_table(code, ctypes.byref(c_vol(vol)), ctypes.byref(cp), _dev(out, "rays"),
                           _stream(stream)), "ray_table")
    out._pcas_dtype = code
    return out


def pca_dvf(mean, U, w, out=None, stream=None):
    """a2 (Eq. 1): x = mean + sum_k w_k U_k, shape like mean ([3][...])."""
    torch = _torch()
    K = U.shape[0]
    N = U[0].numel() // 3
    if out is None:
        out = torch.empty(U.shape[1:], dtype=U.dtype, device=U.device)
    _, wp = _host_doubles(w, K)
    _check(lib().pca_dvf(_dtype_code(U), N, K, _dev(mean, "mean", U.dtype), _dev(U, "U"), wp,
                         _dev(out, "dvf", U.dtype), _stream(stream)), "pca_dvf")
    return out


def warp_trilinear(vol, f0, dvf, out=None, stream=None):
    """a3 (Eqs. A.3, A.5): f0 pulled back through dvf (mm)."""
    torch = _torch()
    if out is None:
        out = torch.empty_like(f0)
    _check(lib().warp_trilinear(_dtype_code(f0), ctypes.byref(c_vol(vol)), _dev(f0, "f0"),
                                _dev(dvf, "dvf", f0.dtype), _dev(out, "f", f0.dtype),
                                _stream(stream)), "warp_trilinear")
    return out


def warp_pca(vol, f0, mean, U, w, out=None, stream=None):
    """a2 + a3 fused: f = f0 pulled back through mean + U w."""
    torch = _torch()
    K = _K_of(U, vol)
    if out is None:
        out = torch.empty_like(f0)
    _, wp = _host_doubles(w, K)
    _check(lib().warp_pca(_dtype_code(f0), ctypes.byref(c_vol(vol)), K, _dev(f0, "f0"),
                          _dev(mean, "mean", f0.dtype), _dev(U, "U", f0.dtype), wp,
                          _dev(out, "f", f0.dtype), _stream(stream)), "warp_pca")
    return out


def drr_forward(vol, proj, rays, f, out=None, stream=None):
    """a4 (Eq. 2): p = P f, shape [nv][nu]."""
    torch = _torch()
    if out is None:
        out = torch.empty((int(proj.nv), int(proj.nu)), dtype=f.dtype, device=f.device)
    _check(lib().drr_forward(_dtype_code(f), ctypes.byref(c_vol(vol)), ctypes.byref(c_proj(proj)),
                             _dev(rays, "rays"), _dev(f, "f"), _dev(out, "p", f.dtype),
                             _stream(stream)), "drr_forward")
    return out


def drr_siddon(vol, proj, f, out=None, stream=None):
    """Exact-path (Siddon) projection of the voxel-constant volume, [nv][nu]."""
    torch = _torch()
    if out is None:
        out = torch.empty((int(proj.nv), int(proj.nu)), dtype=f.dtype, device=f.device)
    _check(lib().drr_siddon(_dtype_code(f), ctypes.byref(c_vol(vol)), ctypes.byref(c_proj(proj)),
                            _dev(f, "f"), _dev(out, "out", f.dtype), _stream(stream)),
           "drr_siddon")
    return out


def drr_adjoint(vol, proj, rays, r, out=None, stream=None, acc32=False):
    """a6: bp = P^T r, shape [n3][n2][n1].  acc32 (float32 only): the
    32-bit-accumulator form (drr_adjoint32)."""
    torch = _torch()
    if out is None:
        out = torch.empty(_vshape(vol), dtype=r.dtype, device=r.device)
    name = "drr_adjoint32" if acc32 else "drr_adjoint"
    _check(getattr(lib(), name)(_dtype_code(r), ctypes.byref(c_vol(vol)),
                                ctypes.byref(c_proj(proj)), _dev(rays, "rays"), _dev(r, "r"),
                                _dev(out, "bp", r.dtype), _stream(stream)), name)
    return out


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def predict(history, coeffs) -> np.ndarray:
    """Eq. 3 (pcas_predict): history [L', K], most recent last; coeffs [K, L]
    with coeffs[k, l-1] = c_kl.  Host-only."""
    h = np.ascontiguousarray(history, dtype=np.float64)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    K, L = c.shape
    if h.ndim != 2 or h.shape[1] != K:
        raise ValueError("history must be [n, K]")
    out = np.empty(K)
    _check(lib().pcas_predict(K, L, _dp(c), _dp(h), h.shape[0], _dp(out)), "pcas_predict")
    return out


def fit_predictor(w_train, L: int = 2) -> np.ndarray:
    """Least-squares c_kl of Eq. 3 on w_train [T, K] (pcas_fit_predictor);
    returns [K, L].  Host-only."""
    w = np.ascontiguousarray(w_train, dtype=np.float64)
    T, K = w.shape
    out = np.empty((K, int(L)))
    _check(lib().pcas_fit_predictor(T, K, int(L), _dp(w), _dp(out)), "pcas_fit_predictor")
    return out


def backprojection_bound(vol, proj) -> float:
    """B with (P^T 1)(v) <= step * B for every voxel (host-only query)."""
    b = lib().pcas_backprojection_bound(ctypes.byref(c_vol(vol)), ctypes.byref(c_proj(proj)))
    if b < 0:
        raise PcasError(-1, "backprojection_bound: invalid volume or projection")
    return b


def backprojection_brick_bound(vol, proj, brick: int) -> float:
    """B_brick with (P^T 1)(v) <= step * B_brick over the brick and its halo
    (host-only query)."""
    b = lib().pcas_backprojection_brick_bound(ctypes.byref(c_vol(vol)), ctypes.byref(c_proj(proj)),
                                              int(brick))
    if b < 0:
        raise PcasError(-1, "backprojection_brick_bound: invalid volume, projection or brick")
    return b


def live_voxels(vol, proj) -> int:
    """Voxels of the bricks the projection can read (the solve's warp writes
    only these; host-only query)."""
    n = int(lib().pcas_live_voxels(ctypes.byref(c_vol(vol)), ctypes.byref(c_proj(proj))))
    if n < 0:
        raise PcasError(-1, "live_voxels: invalid volume or projection")
    return n


def backprojection_brick_count(vol) -> int:
    """Number of back-projection bricks of a volume (host-only query)."""
    n = int(lib().backprojection_brick_count(ctypes.byref(c_vol(vol))))
    if n < 0:
        raise PcasError(-1, "backprojection_brick_count: invalid volume")
    return n


def residual_fit(p, y, fit_intensity: bool = True, r_out=None, want_r: bool = True, stream=None):
    """a5 (Eq. A.1, Eq. 2): returns (r, stats) with stats a float64 device
    tensor [J, a, b, sum p, sum p y, sum p p, sum y, sum y y]."""
    torch = _torch()
    M = p.numel()
    if want_r and r_out is None:
        r_out = torch.empty_like(p)
    stats = torch.empty(8, dtype=torch.float64, device=p.device)
    ws = torch.empty(lib().residual_fit_workspace_bytes(M), dtype=torch.uint8, device=p.device)
    _check(lib().residual_fit(_dtype_code(p), M, _dev(p, "p"), _dev(y, "y", p.dtype),
                              1 if fit_intensity else 0, _dev(r_out, "r", p.dtype) if want_r else None,
                              _dev(stats, "stats"), _dev(ws, "workspace"), ws.numel(),
                              _stream(stream)), "residual_fit")
    return r_out, stats


def grad_w(vol, f0, mean, U, w, bp, out=None, workspace=None, stream=None):
    """a7: g = 2 U^T (df/dx) bp as a float64 device tensor [K]."""
    torch = _torch()
    K = _K_of(U, vol)
    code = _dtype_code(f0)
    cv = c_vol(vol)
    if out is None:
        out = torch.empty(K, dtype=torch.float64, device=f0.device)
    nb = lib().grad_w_workspace_bytes(code, ctypes.byref(cv), K)
    if workspace is None:
        workspace = torch.empty(nb, dtype=torch.uint8, device=f0.device)
    _, wp = _host_doubles(w, K)
    _check(lib().grad_w(code, ctypes.byref(cv), K, _dev(f0, "f0"), _dev(mean, "mean", f0.dtype),
                        _dev(U, "U", f0.dtype), wp, _dev(bp, "bp", f0.dtype),
                        _dev(out, "g", torch.float64), _dev(workspace, "workspace"),
                        workspace.numel(), _stream(stream)), "grad_w")
    return out


def grad_w_noalloc(vol, f0, mean, U, w, bp, out, stream=None):
    """grad_w with the library's static scratch instead of a workspace
    (grad_w_noalloc): out is a caller-provided float64 device tensor [K];
    nothing is allocated."""
    torch = _torch()
    K = _K_of(U, vol)
    _, wp = _host_doubles(w, K)
    _check(lib().grad_w_noalloc(_dtype_code(f0), ctypes.byref(c_vol(vol)), K, _dev(f0, "f0"),
                                _dev(mean, "mean", f0.dtype), _dev(U, "U", f0.dtype), wp,
                                _dev(bp, "bp", f0.dtype), _dev(out, "g", torch.float64),
                                _stream(stream)), "grad_w_noalloc")
    return out


def tumour_position(vol, mean, U, w, c0_mm: Sequence[float], tol: float = 1e-9,
                    max_iter: int = 100, out=None, stream=None):
    """a9: float64 device tensor [y1, y2, y3 (mm), iterations or -1]."""
    torch = _torch()
    K = _K_of(U, vol)
    if out is None:
        out = torch.empty(4, dtype=torch.float64, device=U.device)
    _, wp = _host_doubles(w, K)
    _, cp = _host_doubles(c0_mm, 3)
    _check(lib().tumour_position(_dtype_code(U), ctypes.byref(c_vol(vol)), K,
                                 _dev(mean, "mean", U.dtype), _dev(U, "U"), wp, cp, float(tol),
                                 int(max_iter), _dev(out, "out", torch.float64), _stream(stream)),
           "tumour_position")
    return out


def default_opts(**overrides) -> Opts:
    o = Opts()
    lib().pcas_default_opts(ctypes.byref(o))
    return _apply(o, overrides)


def paper_opts(**overrides) -> Opts:
    o = Opts()
    lib().pcas_paper_opts(ctypes.byref(o))
    return _apply(o, overrides)


def _apply(o: Opts, overrides) -> Opts:
    for k, v in overrides.items():
        if k == "c0_mm":
            for c in range(3):
                o.c0_mm[c] = float(v[c])
        elif k in ("method", "max_iter", "fit_intensity", "max_backtracks", "locate",
                   "locate_max_iter", "profile", "grad_mode", "polish", "speculate", "precond"):
            setattr(o, k, int(v))
        else:
            setattr(o, k, float(v))
    return o


def report_dict(r: Report) -> dict:
    return {"status": STOP.get(r.status, r.status), "iters": r.iters, "n_fevals": r.n_fevals,
            "n_grads": r.n_grads, "J0": r.J0, "J": r.J, "a": r.a, "b": r.b,
            "gnorm0": r.gnorm0, "gnorm": r.gnorm, "tumour_mm": list(r.tumour_mm),
            "locate_iters": r.locate_iters, "spec_grads": r.spec_grads, "host_ms": r.host_ms,
            "wait_ms": r.wait_ms,
            "kernel_ms": {k: r.kernel_ms[i] for i, k in enumerate(KERNEL_CLASSES)},
            "kernel_launches": {k: r.kernel_launches[i] for i, k in enumerate(KERNEL_CLASSES)}}


def solve_projection_workspace(vol, proj, K: int, dtype) -> int:
    torch = _torch()
    code = PCAS_F32 if dtype == torch.float32 else PCAS_F64
    return int(lib().solve_projection_workspace(code, ctypes.byref(c_vol(vol)),
                                                ctypes.byref(c_proj(proj)), int(K)))


def solve_projection(vol, proj, f0, mean, U, y, w0, opts: Optional[Opts] = None, workspace=None,
                     stream=None):
    """a1-a9: solve one projection; returns (w as float64 numpy [K], report dict).
    Synchronous (the library waits for its own stream)."""
    torch = _torch()
    K = _K_of(U, vol)
    code = _dtype_code(f0)
    cv, cp = c_vol(vol), c_proj(proj)
    need = lib().solve_projection_workspace(code, ctypes.byref(cv), ctypes.byref(cp), K)
    if workspace is None:
        workspace = torch.empty(max(int(need), 1), dtype=torch.uint8, device=f0.device)
    o = default_opts() if opts is None else opts
    _, w0p = _host_doubles(w0, K)
    w_out = np.zeros(K)
    rep = Report()
    _check(lib().solve_projection(code, ctypes.byref(cv), ctypes.byref(cp), K, _dev(f0, "f0"),
                                  _dev(mean, "mean", f0.dtype), _dev(U, "U", f0.dtype),
                                  _dev(y, "y", f0.dtype), w0p, ctypes.byref(o),
                                  _dev(workspace, "workspace"), workspace.numel(),
                                  w_out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  ctypes.byref(rep), _stream(stream)), "solve_projection")
    return w_out, report_dict(rep)


def objective_gradient(vol, proj, f0, mean, U, y, w, fit_intensity: bool = True,
                       grad_mode: int = 1, workspace=None, stream=None, gauss_newton=False):
    """a5 + a6 + a7 at one point: (J, a, b, g as float64 numpy [K]) exactly as
    the solver forms them (grad_mode 1: back-projection + Jacobian chain; 0:
    projected Jacobian volumes; 2: the fused evaluation), and with
    gauss_newton (grad_mode 2) also the Gauss-Newton matrix [K, K] of the
    reduced objective.  Synchronous."""
    torch = _torch()
    K = _K_of(U, vol)
    code = _dtype_code(f0)
    cv, cp = c_vol(vol), c_proj(proj)
    need = lib().solve_projection_workspace(code, ctypes.byref(cv), ctypes.byref(cp), K)
    if workspace is None:
        workspace = torch.empty(max(int(need), 1), dtype=torch.uint8, device=f0.device)
    _, wp = _host_doubles(w, K)
    out = np.zeros(3 + K + (K * K if int(grad_mode) == 2 else 0))
    _check(lib().objective_gradient(code, ctypes.byref(cv), ctypes.byref(cp), K, _dev(f0, "f0"),
                                    _dev(mean, "mean", f0.dtype), _dev(U, "U", f0.dtype),
                                    _dev(y, "y", f0.dtype), wp, int(bool(fit_intensity)),
                                    int(grad_mode), _dev(workspace, "workspace"),
                                    workspace.numel(),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    _stream(stream)), "objective_gradient")
    if gauss_newton:
        return (float(out[0]), float(out[1]), float(out[2]), out[3:3 + K].copy(),
                out[3 + K:].reshape(K, K).copy())
    return float(out[0]), float(out[1]), float(out[2]), out[3:3 + K].copy()


class Server:
    """Serving loop over the C ABI: requests of different models (volume
    sizes, K) solved concurrently with their work batched into shared
    launches; admission by the footprint each request needs in the arena.

    The arena is one device byte tensor owned by this object; registered
    models' tensors and submitted measurements are kept alive here until
    the request has been polled."""

    def __init__(self, arena_bytes: int, max_active: int = 16, device="cuda", stream=None):
        torch = _torch()
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        self._stream = stream
        h = ctypes.c_void_p()
        _check(lib().pcas_server_create(_dev(self.arena, "arena"), self.arena.numel(),
                                        int(max_active), _stream(stream), ctypes.byref(h)),
               "pcas_server_create")
        self._h = h
        self._models = []          # (vol, K, dtype, tensors)
        self._inflight = {}        # request id -> (model id, y tensor)

    @staticmethod
    def reserved_bytes(max_active: int) -> int:
        return int(lib().pcas_server_reserved_bytes(int(max_active)))

    def add_model(self, vol, f0, mean, U) -> int:
        K = _K_of(U, vol)
        mid = ctypes.c_int32()
        _check(lib().pcas_server_add_model(self._h, _dtype_code(f0), ctypes.byref(c_vol(vol)), K,
                                           _dev(f0, "f0"), _dev(mean, "mean", f0.dtype),
                                           _dev(U, "U", f0.dtype), ctypes.byref(mid)),
               "pcas_server_add_model")
        self._models.append((vol, K, f0.dtype, (f0, mean, U)))
        return int(mid.value)

    def request_bytes(self, model_id: int, proj, opts: Optional[Opts] = None) -> int:
        o = default_opts() if opts is None else opts
        return int(lib().pcas_server_request_bytes(self._h, int(model_id),
                                                   ctypes.byref(c_proj(proj)), ctypes.byref(o)))

    def submit(self, model_id: int, proj, y, w0, opts: Optional[Opts] = None) -> int:
        vol, K, dt, _ = self._models[model_id]
        o = default_opts() if opts is None else opts
        _, w0p = _host_doubles(w0, K)
        rid = ctypes.c_int64()
        _check(lib().pcas_server_submit(self._h, int(model_id), ctypes.byref(c_proj(proj)),
                                        _dev(y, "y", dt), w0p, ctypes.byref(o),
                                        ctypes.byref(rid)), "pcas_server_submit")
        self._inflight[int(rid.value)] = (model_id, y)
        return int(rid.value)

    def step(self) -> int:
        n = ctypes.c_int32()
        _check(lib().pcas_server_step(self._h, ctypes.byref(n)), "pcas_server_step")
        return int(n.value)

    def set_substep_share(self, share: float) -> None:
        """Extra passes for cheap requests per step, as a share of the main
        pass's estimated cost (0 = one pass per step)."""
        _check(lib().pcas_server_set_substep_share(self._h, float(share)),
               "pcas_server_set_substep_share")

    def poll(self, request_id: int):
        """(done, status, w, report dict); status is 0 or the request's error
        code.  A completed request is returned once."""
        mid, _ = self._inflight[request_id]
        K = self._models[mid][1]
        w = np.zeros(K)
        rep = Report()
        done = ctypes.c_int32()
        st = lib().pcas_server_poll(self._h, int(request_id),
                                    w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    ctypes.byref(rep), ctypes.byref(done))
        if not done.value:
            if st != 0:
                _check(st, "pcas_server_poll")
            return False, 0, None, None
        del self._inflight[request_id]
        return True, int(st), w, report_dict(rep)

    def stats(self):
        p, a, u = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
        _check(lib().pcas_server_stats(self._h, ctypes.byref(p), ctypes.byref(a), ctypes.byref(u)),
               "pcas_server_stats")
        return {"pending": int(p.value), "active": int(a.value), "arena_used": int(u.value)}

    def close(self):
        if self._h is not None and self._h.value:
            lib().pcas_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
