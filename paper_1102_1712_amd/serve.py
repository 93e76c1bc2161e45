"""Serving driver: a persistent request loop over the batching server.

Projections of several resident models (different volume sizes and K)
arrive as a Poisson stream at changing gantry angles; each is submitted to
a :class:`binding.Server` when it arrives, warm-started from the latest
completed solution of its model, and the loop keeps stepping the server
(one batched operation of every admitted solve per step) while polling for
completions.  Latency is arrival to completion on the host clock.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import binding as B


@dataclass
class Arrival:
    t: float                  # seconds after the start
    model: int
    proj: object              # Projection at this request's angle
    y: object                 # device measurement
    w_true: Optional[np.ndarray] = None


@dataclass
class Done:
    index: int
    model: int
    arrival: float
    submitted: float
    completed: float
    status: int
    w: Optional[np.ndarray]
    report: Optional[dict]

    @property
    def latency_ms(self) -> float:
        return (self.completed - self.arrival) * 1e3


def poisson_times(rate_hz: float, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n))


def run(server: B.Server, arrivals: List[Arrival], opts_by_model: Dict[int, B.Opts],
        K_by_model: Dict[int, int], warm: bool = True, time_limit_s: float = 600.0) -> List[Done]:
    """Feeds arrivals (sorted by t) to the server in real time and runs it
    until every request has completed.  Returns one Done per arrival."""
    order = sorted(range(len(arrivals)), key=lambda i: arrivals[i].t)
    latest: Dict[int, np.ndarray] = {}
    inflight: Dict[int, tuple] = {}
    out: List[Optional[Done]] = [None] * len(arrivals)
    nxt = 0
    t0 = time.perf_counter()
    while nxt < len(order) or inflight:
        now = time.perf_counter() - t0
        if now > time_limit_s:
            raise TimeoutError("serving run exceeded its time limit")
        while nxt < len(order) and arrivals[order[nxt]].t <= now:
            i = order[nxt]
            a = arrivals[i]
            K = K_by_model[a.model]
            w0 = latest[a.model] if (warm and a.model in latest) else np.zeros(K)
            rid = server.submit(a.model, a.proj, a.y, w0, opts_by_model[a.model])
            inflight[rid] = (i, time.perf_counter() - t0)
            nxt += 1
        if not inflight:
            # idle until the next arrival
            wait = arrivals[order[nxt]].t - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.001))
            continue
        server.step()
        now = time.perf_counter() - t0
        for rid in list(inflight):
            done, status, w, rep = server.poll(rid)
            if not done:
                continue
            i, ts = inflight.pop(rid)
            a = arrivals[i]
            out[i] = Done(index=i, model=a.model, arrival=a.t, submitted=ts, completed=now,
                          status=status, w=w, report=rep)
            if status == 0:
                latest[a.model] = w
    return [d for d in out if d is not None]


def summary(done: List[Done]) -> dict:
    lat = np.array([d.latency_ms for d in done])
    span = max(d.completed for d in done) - min(d.arrival for d in done)
    return {"requests": len(done), "solves_s": len(done) / span if span > 0 else None,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "failed": int(sum(d.status != 0 for d in done))}
