"""Streaming per-projection solve: a projection sequence at changing gantry
angles, each solve warm-started from a linear prediction of its coefficients.

Sec. II.A (Eq. 3): the initial guess of coefficient k for the current
projection is a linear combination of its last L optimised values,
w_k0(t) = sum_{l=1..L} c_kl w*_k(t - l), with one prediction model per
coefficient (they have different dynamics).  The paper fits the c_kl on the
training 4DCT after resampling to the projection rate, and notes that the
first breathing cycles of the scan itself may be used instead; here they are
fitted by least squares on the first frames of the stream (L = 2 as in the
paper).  Until L solutions exist the previous solution (or w0) is used --
the paper's earlier warm start.

The loop keeps f0, xbar and U resident on the GPU, builds nothing per frame
but the measured image handed in by the caller, and calls solve_projection
(which builds the frame's ray table) with the tumour localisation enabled.
Latency per frame is measured on the host around the synchronous call.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field, replace
from typing import Callable, List, Optional

import numpy as np

from . import binding as B


# ---------------------------------------------------------------------------
# Eq. 3: per-coefficient linear prediction
# ---------------------------------------------------------------------------

def predict(history: np.ndarray, coeffs: np.ndarray) -> np.ndarray:
    """Eq. 3: history [L', K] with the most recent solution last; coeffs
    [K, L] with coeffs[k, l-1] = c_kl.  Needs L' >= L.  Runs in the library
    (pcas_predict)."""
    return B.predict(history, coeffs)


def fit_predictor(w_train: np.ndarray, L: int = 2) -> np.ndarray:
    """Least-squares fit of c_kl, separately for every coefficient, on a
    training sequence w_train [T, K] (T > L).  Runs in the library
    (pcas_fit_predictor)."""
    return B.fit_predictor(w_train, L)


# ---------------------------------------------------------------------------
# synthetic breathing trace (input generation; no method arithmetic)
# ---------------------------------------------------------------------------

def breathing_trace(n_frames: int, fps: float, seed: int, period=(3.0, 6.0), amp=(5.0, 20.0),
                    drift_mm_per_min: float = 2.0) -> np.ndarray:
    """Irregular breathing signal in mm, one value per frame: cycles of
    random period and amplitude (1 - cos shape, 0 at end-of-exhale) plus a
    linear baseline drift."""
    rng = np.random.default_rng(seed)
    t = np.arange(n_frames) / fps
    s = np.zeros(n_frames)
    t0 = 0.0
    while t0 < t[-1] + 1e-9:
        P = rng.uniform(*period)
        A = rng.uniform(*amp)
        m = (t >= t0) & (t < t0 + P)
        s[m] = 0.5 * A * (1.0 - np.cos(2.0 * np.pi * (t[m] - t0) / P))
        t0 += P
    return s + drift_mm_per_min / 60.0 * t


def planted_trajectory(trace_mm: np.ndarray, K: int, seed: int, scale: float) -> np.ndarray:
    """Coefficient trajectories driven by the trace, with a per-coefficient
    gain and lag (hysteresis): w_k(t) = scale * g_k * trace(t - lag_k)."""
    rng = np.random.default_rng(seed)
    gains = rng.uniform(0.5, 1.0, K) * rng.choice([-1.0, 1.0], K)
    lags = rng.integers(0, 4, K)
    T = trace_mm.size
    w = np.zeros((T, K))
    for k in range(K):
        src = np.concatenate([np.full(lags[k], trace_mm[0]), trace_mm])[:T]
        w[:, k] = scale * gains[k] * src
    return w


# ---------------------------------------------------------------------------
# the loop
# ---------------------------------------------------------------------------

@dataclass
class FrameResult:
    w: np.ndarray
    tumour_mm: np.ndarray
    latency_ms: float
    iters: int
    n_fevals: int
    n_grads: int
    status: str


@dataclass
class StreamReport:
    frames: List[FrameResult] = field(default_factory=list)

    def latencies(self) -> np.ndarray:
        return np.array([f.latency_ms for f in self.frames])

    def summary(self) -> dict:
        lat = self.latencies()
        return {"frames": len(self.frames), "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
                "mean_iters": float(np.mean([f.iters for f in self.frames])),
                "mean_fevals": float(np.mean([f.n_fevals for f in self.frames]))}


class StreamSolver:
    """Solves a sequence of projections of one patient model (resident f0,
    mean, U) at changing gantry angles with warm starts.

    init: "predict" (Eq. 3 once L solutions exist and coefficients are
    set), "previous" (last solution) or "zero"."""

    def __init__(self, vol, proj_template, f0, mean, U, opts: Optional[B.Opts] = None,
                 c0_mm=None, init: str = "predict", predictor: Optional[np.ndarray] = None):
        import torch
        self.vol, self.proj = vol, proj_template
        self.f0, self.mean, self.U = f0, mean, U
        self.K = B._K_of(U, vol)
        self.init = init
        self.coeffs = predictor
        base = opts if opts is not None else B.default_opts()
        self.opts = base
        if c0_mm is not None:
            self.opts.locate = 1
            for c in range(3):
                self.opts.c0_mm[c] = float(c0_mm[c])
        self.ws = torch.empty(B.solve_projection_workspace(vol, proj_template, self.K, f0.dtype),
                              dtype=torch.uint8, device=f0.device)
        self.history: List[np.ndarray] = []
        self.report = StreamReport()

    def initial_guess(self) -> np.ndarray:
        if not self.history or self.init == "zero":
            return np.zeros(self.K)
        if self.init == "predict" and self.coeffs is not None and len(self.history) >= self.coeffs.shape[1]:
            return predict(np.array(self.history), self.coeffs)
        return self.history[-1].copy()

    def step(self, angle: float, y) -> FrameResult:
        proj = replace(self.proj, angle=float(angle))
        w0 = self.initial_guess()
        t0 = time.perf_counter()
        w, rep = B.solve_projection(self.vol, proj, self.f0, self.mean, self.U, y, w0, self.opts,
                                    workspace=self.ws)
        dt = (time.perf_counter() - t0) * 1e3
        self.history.append(w.copy())
        fr = FrameResult(w=w, tumour_mm=np.array(rep["tumour_mm"]), latency_ms=dt,
                         iters=rep["iters"], n_fevals=rep["n_fevals"], n_grads=rep["n_grads"],
                         status=rep["status"])
        self.report.frames.append(fr)
        return fr

    def run(self, angles, measurement: Callable[[int, float], object]) -> StreamReport:
        for t, ang in enumerate(angles):
            self.step(ang, measurement(t, ang))
        return self.report


def localisation_errors(located: np.ndarray, truth: np.ndarray) -> dict:
    """Sec. I: mean absolute 3D error and its 95th percentile (mm)."""
    e = np.linalg.norm(np.asarray(located) - np.asarray(truth), axis=1)
    return {"e_mean_mm": float(e.mean()), "e95_mm": float(np.percentile(e, 95)),
            "e_max_mm": float(e.max())}
