#!/usr/bin/env python3
"""Benchmark of the per-projection PCA solve on one MI355X.

One step = one call of solve_projection on the clinical-size workload: ray
table, then CG iterations of evaluations, then the tumour-position
inversion.  By default an evaluation is the fused one (grad_mode 2): DVF
synthesis, warp and the K Jacobian volumes in one voxel pass, then one
cone-beam projection of all K + 1 volumes whose sums give the intensity
fit, the objective, the gradient and the Gauss-Newton matrix that
preconditions CG (precond 1).  The same solve by plain CG and by the other
two gradient routes (back-projection of the residual + Jacobian chain;
projections of the Jacobian volumes after the evaluation), and by BFGS, is
reported beside it.  Inputs (reference volume, mean field and K = 3 modes, measured
projection) are resident in HBM before the timed region.

Prints ONE JSON line (see the keys below).  Kernel durations come from HIP
events recorded by the library on the solve's stream around its launches:
the warmup steps time every kernel class, which names the dominant one, and
the timed steps time that class alone (opts.profile is a class mask; each
timed launch adds two event records), so the roofline's duration is measured
inside the timed region at the cost of one kernel's events.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METHODS = {"paper": 0, "cg": 1, "bfgs": 2}
METRIC = "per-projection solve latency p50/p99 ms; DRR+adjoint Gsamples/s; % HBM peak"
HBM_PEAK_GBS = 8000.0
# fp32 vector peak without packed math: 256 CUs x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
VALU_F32_PEAK_TFLOPS = 78.6
# Algorithmic flops per projection sample.  Forward: position e + sh d
# (3 fma = 6), fractions (3), trilinear value as 7 lerps of 3 flops (21),
# accumulation (1) = 31.  Back-projection: position (6), fractions (3),
# corner weights (9), 8 weighted accumulations (16) = 34.  Projection of nv
# volumes at once: position and fractions once (9), then either 22 per volume
# (lerps) or the eight corner weights once (15) and 16 per volume (eight
# products and the accumulation), whichever is fewer; the fused evaluation
# projects K + 1 volumes.
def proj_flops(nv: int) -> float:
    return float(min(9 + 22 * nv, 24 + 16 * nv))


def flops_per_sample(kernel: str, K: int) -> float:
    return {"drr_forward": proj_flops(1), "drr_adjoint": 34.0, "drr_adjoint_chain": 34.0,
            "drr_forward_dot": proj_flops(K), "drr_forward_eval": proj_flops(K + 1)}[kernel]


# Jacobian chain per voxel: field 6K, displacement split 6, Eq. A.8 and its
# two analogues 3 x 13, per-mm and bp scaling 6, mode sums 5K + K.
def chain_flops_per_voxel(K: int) -> float:
    return 12.0 * K + 51.0


# solver configurations reported beside the timed one: (label, grad_mode, precond)
SOLVER_VARIANTS = (("cg_route0", 0, 0), ("cg_route1", 1, 0), ("cg_route2", 2, 0),
                   ("pcg_route2", 2, 1))

SAMPLE_KERNELS = ("drr_forward", "drr_adjoint", "drr_adjoint_chain", "drr_forward_dot",
                  "drr_forward_eval")
KERNEL_SOURCES = {"drr_forward": "k_drr.hip", "drr_adjoint": "k_drr.hip",
                  "drr_adjoint_chain": "k_drr.hip", "drr_forward_dot": "k_drr.hip",
                  "drr_forward_eval": "k_drr.hip", "warp_pca": "k_warp.hip",
                  "warp_jac": "k_warp.hip", "grad_w": "k_grad.hip", "jacobian": "k_grad.hip"}
HBM_KERNELS = ("warp_pca", "warp_jac", "grad_w", "jacobian")


def kernel_digest(kernel: str) -> str:
    """sha256[:16] of the kernel's source file and every header it includes,
    directly or through other headers (device code only: host-side files
    such as the solver's state machine, which the shared header pulls in for
    its gradient rule, do not change a kernel's traffic)."""
    import hashlib
    import re

    csrc = os.path.join(ROOT, "paper_1102_1712_amd", "csrc")
    files, todo = [], [KERNEL_SOURCES[kernel]]
    while todo:
        f = todo.pop(0)
        if f in files or f == "solver.h" or not os.path.exists(os.path.join(csrc, f)):
            continue
        files.append(f)
        with open(os.path.join(csrc, f)) as fh:
            todo += re.findall(r'#include "([A-Za-z0-9_]+\.h)"', fh.read())
    h = hashlib.sha256()
    for f in [files[0]] + sorted(files[1:]):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if that summary is for another workload or the kernel's source has
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.txt")
    if kernel not in KERNEL_SOURCES or not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) == 4 and parts[0] == kernel:
                if parts[3] != kernel_digest(kernel):
                    return None
                return int(parts[1]) + int(parts[2])
    return None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def build_inputs(workload: str, seed: int):
    import torch

    from paper_1102_1712_amd import binding as B
    from paper_1102_1712_amd import synth

    t0 = time.time()
    if workload == "clinical":
        case = synth.clinical(seed=seed)
    elif workload == "clinical_k5":
        case = synth.clinical_k5()
    else:
        case = synth.tiny(seed=seed)
    dt = torch.float32 if case.dtype == "f32" else torch.float64
    f0, mean, U = case.arrays()
    dev = dict(f0=torch.from_numpy(f0).cuda(), mean=torch.from_numpy(mean).cuda(),
               U=torch.from_numpy(U).cuda())
    # measured projection: P f(w*) plus 1% Gaussian noise (formed on the GPU)
    rays = B.ray_table(case.vol, case.proj, dt)
    f = B.warp_pca(case.vol, dev["f0"], dev["mean"], dev["U"], case.w_star)
    p = B.drr_forward(case.vol, case.proj, rays, f)
    rms = torch.sqrt(torch.mean(p.double() ** 2))
    xi = torch.from_numpy(case.xi).cuda()
    dev["y"] = (p.double() + case.noise_level * rms * xi).to(dt).contiguous()
    dev["rays"] = rays
    torch.cuda.synchronize()
    log(f"inputs for {case.name} ready in {time.time() - t0:.1f} s")
    return case, dev, dt


def samples_per_drr(rays, dtype: str) -> int:
    rec = rays.cpu().numpy()
    if dtype == "f32":
        n = rec.view(np.int32).reshape(-1, 8)[:, 7]
    else:
        n = rec.view(np.int32).reshape(-1, 16)[:, 14]
    return int(n.astype(np.int64).sum())


def solver_opts(args, method: int, **kw):
    """The benchmark's solver options for a method: the gradient route of
    --grad-mode and, for CG on the fused evaluation, the Gauss-Newton
    preconditioner of --precond."""
    from paper_1102_1712_amd import binding as B
    pre = args.precond if (method == 1 and args.grad_mode == 2) else 0
    return B.default_opts(method=method, grad_mode=args.grad_mode, precond=pre, **kw)


def reached_voxels(case, dev) -> int:
    """Voxels that at least one projection sample touches (P^T 1 > 0): the
    gradient's chain has work only there, since it skips voxels where the
    back-projected residual is zero."""
    import torch

    from paper_1102_1712_amd import binding as B

    ones = torch.ones((case.proj.nv, case.proj.nu), dtype=dev["f0"].dtype, device="cuda")
    bp = B.drr_adjoint(case.vol, case.proj, dev["rays"], ones)
    return int((bp > 0).sum().item())


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def host_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))


def _oracle_problem(case):
    import oracle as O
    # the oracle's measured image comes from its own forward model
    y = O.measured_projection(case.vol, case.proj, case.f0, case.mean, case.U, case.w_star,
                              case.xi, case.noise_level)
    return O.Problem(case.vol, case.proj, case.f0, case.mean, case.U, y)


def cpu_baseline(case, samples: int, tiny_runs: int = 3):
    """The FP64 oracle as it stands (test infrastructure, never tuned for
    this), timed on the host cores:
      * one full solve of the benchmark's workload from w0 = 0 with the
        oracle's plain PR+ CG (at most 30 iterations, stop at ||g|| <= 1e-6
        ||g0||), on all cores: `value`, in solves/s;
      * the tiny workload's full solve, median of tiny_runs, on all cores and
        on one core;
      * one forward evaluation of the benchmark's workload (forward samples/s).
    """
    import oracle as O
    from paper_1102_1712_amd import synth

    n_all = host_threads()
    O.set_threads(n_all)
    prob = _oracle_problem(case)
    w0 = np.zeros(case.K)
    t0 = time.perf_counter()
    prob.objective(w0)
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    w, rep = O.solve_cg(prob, w0)
    t_solve = time.perf_counter() - t0
    log(f"oracle clinical solve: {t_solve:.1f} s ({rep.iters} iterations, {rep.n_fevals} "
        f"evaluations, {rep.n_grads} gradients)")
    tiny = synth.tiny()
    tprob = _oracle_problem(tiny)
    tiny_t = {}
    for label, n in (("all_cores", n_all), ("one_core", 1)):
        O.set_threads(n)
        ts = []
        for _ in range(tiny_runs):
            t0 = time.perf_counter()
            _, trep = O.solve_cg(tprob, np.zeros(tiny.K))
            ts.append(time.perf_counter() - t0)
        tiny_t[label] = {"threads": n, "median_s": float(np.median(ts)),
                         "runs_s": [float(t) for t in ts]}
        log(f"oracle tiny solve, {n} threads: median {np.median(ts):.2f} s")
    O.set_threads(n_all)
    return {
        "value": 1.0 / t_solve, "unit": "solves/s", "cores": n_all, "kind": "oracle",
        "cpu_model": cpu_model(),
        "solve_s": t_solve, "iters": rep.iters, "n_fevals": rep.n_fevals, "n_grads": rep.n_grads,
        "forward_s": t_fwd,
        "forward_gsamples_s": samples / t_fwd / 1e9 if samples else None,
        "tiny_solve": tiny_t,
        "sample": (f"one full FP64 oracle solve of the {case.name} workload from w0 = 0 (plain "
                   f"PR+ CG: {rep.iters} iterations, {rep.n_fevals} evaluations, "
                   f"{rep.n_grads} gradients) on {n_all} host threads; the tiny workload's "
                   f"full solve, median of {tiny_runs}, on {n_all} threads and on 1"),
    }


def kernels_mode(case, dev, dt, reps: int) -> int:
    """Each hot kernel alone, `reps` times, plus a device copy of known size
    (the calibration kernel for HBM byte counters).  Prints one JSON line of
    HIP-event timings."""
    import torch

    from paper_1102_1712_amd import binding as B

    vol, proj = case.vol, case.proj
    w = case.w_star * 0.5
    f = B.warp_pca(vol, dev["f0"], dev["mean"], dev["U"], w)
    p = B.drr_forward(vol, proj, dev["rays"], f)
    r = (p - dev["y"]).contiguous()
    bp = B.drr_adjoint(vol, proj, dev["rays"], r)
    g = B.grad_w(vol, dev["f0"], dev["mean"], dev["U"], w, bp)
    copy_bytes = 256 << 20
    src = torch.empty(copy_bytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    calls = {
        "warp_pca": lambda: B.warp_pca(vol, dev["f0"], dev["mean"], dev["U"], w, out=f),
        "drr_forward": lambda: B.drr_forward(vol, proj, dev["rays"], f, out=p),
        "drr_adjoint": lambda: B.drr_adjoint(vol, proj, dev["rays"], r, out=bp),
        "grad_w": lambda: B.grad_w(vol, dev["f0"], dev["mean"], dev["U"], w, bp, out=g),
        "copy_256MiB": lambda: dst.copy_(src),
    }
    out = {}
    for name, fn in calls.items():
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        out[name] = {"median_ms": float(np.median(ts)), "min_ms": float(np.min(ts))}
        log(f"{name}: median {out[name]['median_ms']:.4f} ms")
    out["copy_256MiB"]["bytes"] = 2 * copy_bytes
    print(json.dumps({"mode": "kernels", "workload": case.name, "reps": reps, "kernels": out}),
          flush=True)
    return 0


def stream_mode(case, dev, dt, args) -> int:
    """A sequence of projections over one rotation (15 frames/s): the planted
    coefficients follow a seeded irregular breathing trace; the sequence is
    solved twice, each solve warm-started by the Eq. 3 prediction, then by
    the previous solution, and the located tumour is compared with the
    planted trajectory's."""
    import dataclasses

    import torch

    from paper_1102_1712_amd import binding as B
    from paper_1102_1712_amd import stream as S

    n = args.frames
    fps = 15.0
    trace = S.breathing_trace(n + 60, fps, seed=args.seed + 100)
    w_all = S.planted_trajectory(trace, case.K, seed=args.seed + 101, scale=0.05)
    coeffs = S.fit_predictor(w_all[:60], L=2)
    w_true = w_all[60:]
    angles = case.proj.angle + np.arange(n) * (2 * np.pi / n)
    gen = torch.Generator(device="cuda").manual_seed(args.seed + 102)
    xtol = 1e-7 if case.dtype == "f32" else 1e-10
    # measured projections (same forward model, 1% noise) and true positions
    truth = np.zeros((n, 3))
    loc = torch.empty(4, dtype=torch.float64, device="cuda")
    ys = []
    for t in range(n):
        pj = dataclasses.replace(case.proj, angle=float(angles[t]))
        rays = B.ray_table(case.vol, pj, dt, out=dev["rays"])
        f = B.warp_pca(case.vol, dev["f0"], dev["mean"], dev["U"], w_true[t])
        p = B.drr_forward(case.vol, pj, rays, f)
        rms = torch.sqrt(torch.mean(p.double() ** 2))
        ys.append((p.double() + 0.01 * rms * torch.randn(p.shape, generator=gen, device="cuda",
                                                          dtype=torch.float64)).to(dt).contiguous())
        B.tumour_position(case.vol, dev["mean"], dev["U"], w_true[t], case.tumour_c0, out=loc)
        truth[t] = loc.cpu().numpy()[:3]
    log(f"stream: {n} measured projections made")
    out = {"mode": "stream", "workload": case.name, "frames": n, "fps": fps, "method": args.method,
           "grad_mode": args.grad_mode, "precond": args.precond if args.method == "cg" else 0,
           "data": "synthetic (measured images from the same forward model, 1% noise)"}
    for init in ("predict", "previous"):
        solver = S.StreamSolver(case.vol, case.proj, dev["f0"], dev["mean"], dev["U"],
                                opts=solver_opts(args, METHODS[args.method], xtol=xtol),
                                c0_mm=case.tumour_c0,
                                predictor=coeffs, init=init)
        for t in range(n):
            solver.step(angles[t], ys[t])
            if (t + 1) % 200 == 0:
                log(f"stream {init} frame {t + 1}/{n}: p50 so far "
                    f"{np.median(solver.report.latencies()):.2f} ms")
        located = np.array([fr.tumour_mm for fr in solver.report.frames])
        out[init] = {**solver.report.summary(), **S.localisation_errors(located, truth)}
        frames = solver.report.frames
        slow = sorted(range(n), key=lambda t: -frames[t].latency_ms)[:6]
        out[init]["slowest_frames"] = [
            {"frame": t, "ms": frames[t].latency_ms, "iters": frames[t].iters,
             "n_fevals": frames[t].n_fevals, "status": frames[t].status} for t in slow]
    out["predict"]["init"] = "Eq. 3 prediction (L = 2, fitted on 60 earlier frames)"
    out["previous"]["init"] = "previous frame's solution"
    print(json.dumps(out), flush=True)
    return 0


def serve_mode(args) -> int:
    """Batched mixed-size serving: Poisson arrivals (200 requests/s) of
    projections of two resident models -- 128x128x96 K=3 with a 512x384
    detector and 512x512x256 K=5 with a 1024x768 detector, 0.4 mm pitch --
    at random angles through the batching server (16 slots, admission by
    footprint, warm starts per model); the same requests solved one after
    another by solve_projection for comparison."""
    import dataclasses

    import torch

    from paper_1102_1712_amd import binding as B
    from paper_1102_1712_amd import serve as SV
    from paper_1102_1712_amd import synth

    t_build = time.perf_counter()
    cases = [synth.serve_small(progress=log), synth.serve_large(progress=log)]
    devs = []
    for c in cases:
        f0, mean, U = c.arrays(np.float32)
        devs.append({k: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
                     for k, a in (("f0", f0), ("mean", mean), ("U", U))})
    log(f"serve: models built in {time.perf_counter() - t_build:.1f} s")
    rng = np.random.default_rng(args.seed + 200)
    n = args.requests
    times = SV.poisson_times(args.rate, n, seed=args.seed + 201)
    gen = torch.Generator(device="cuda").manual_seed(args.seed + 202)
    arrivals = []
    for j in range(n):
        m = int(rng.integers(0, 2))
        c, d = cases[m], devs[m]
        pj = dataclasses.replace(c.proj, angle=float(rng.uniform(0.0, 2 * np.pi)))
        # a breathing-like planted state per request
        w_true = c.w_star * (1.0 + 0.3 * np.sin(2 * np.pi * times[j] / 4.0))
        rays = B.ray_table(c.vol, pj, torch.float32)
        f = B.warp_pca(c.vol, d["f0"], d["mean"], d["U"], w_true)
        p = B.drr_forward(c.vol, pj, rays, f)
        rms = torch.sqrt(torch.mean(p.double() ** 2))
        y = (p.double() + 0.01 * rms * torch.randn(p.shape, generator=gen, device="cuda",
                                                    dtype=torch.float64)).float().contiguous()
        arrivals.append(SV.Arrival(t=float(times[j]), model=m, proj=pj, y=y, w_true=w_true))
        del rays, f, p
    torch.cuda.synchronize()
    Ks = {m: cases[m].K for m in range(2)}
    # gradient route per model: the faster of the back-projection route and
    # the fused evaluation (with CG preconditioned by its Gauss-Newton matrix
    # unless --precond 0) on one of the model's own requests (the fused
    # evaluation projects K + 1 volumes, which can lose on the large K = 5
    # model when it does not save evaluations)
    pre = args.precond if args.method == "cg" else 0
    route_ms = {}
    for m in range(2):
        a = next(x for x in arrivals if x.model == m)
        d = devs[m]
        ws_m = torch.empty(B.solve_projection_workspace(cases[m].vol, a.proj, Ks[m], torch.float32),
                           dtype=torch.uint8, device="cuda")
        for gm in (1, 2):
            o = B.default_opts(xtol=1e-7, method=METHODS[args.method], grad_mode=gm,
                               precond=pre if gm == 2 else 0)
            B.solve_projection(cases[m].vol, a.proj, d["f0"], d["mean"], d["U"], a.y, np.zeros(Ks[m]),
                               o, workspace=ws_m)
            ts = []
            for _ in range(3):
                t0 = time.perf_counter()
                B.solve_projection(cases[m].vol, a.proj, d["f0"], d["mean"], d["U"], a.y,
                                   np.zeros(Ks[m]), o, workspace=ws_m)
                ts.append((time.perf_counter() - t0) * 1e3)
            route_ms[(m, gm)] = float(np.median(ts))
        del ws_m
    route = {m: min((1, 2), key=lambda gm: route_ms[(m, gm)]) for m in range(2)}
    log(f"serve: route per model {route} from {route_ms}")
    opts = {m: B.default_opts(xtol=1e-7, method=METHODS[args.method], grad_mode=route[m],
                              precond=pre if route[m] == 2 else 0)
            for m in range(2)}

    def new_server(share=args.substep_share):
        srv0 = B.Server(B.Server.reserved_bytes(args.slots) + (64 << 20), max_active=args.slots)
        for c, d in zip(cases, devs):
            srv0.add_model(c.vol, d["f0"], d["mean"], d["U"])
        need = max(srv0.request_bytes(m, cases[m].proj, opts[m]) for m in range(2))
        srv0.close()
        srv = B.Server(B.Server.reserved_bytes(args.slots) + args.slots * need + (1 << 20),
                       max_active=args.slots)
        srv.set_substep_share(share)
        for c, d in zip(cases, devs):
            srv.add_model(c.vol, d["f0"], d["mean"], d["U"])
        return srv, need

    out = {"mode": "serve", "requests": n, "rate_hz": args.rate, "slots": args.slots,
           "grad_mode_per_model": [route[m] for m in range(2)], "precond": pre,
           "solve_ms_per_model_and_route": {f"model{m}_route{gm}": v for (m, gm), v in route_ms.items()},
           "substep_share": args.substep_share,
           "models": [{"workload": c.name, "volume": list(c.vol.n), "K": c.K,
                       "detector": [c.proj.nu, c.proj.nv], "pitch_mm": c.proj.pitch_u,
                       "step_mm": c.proj.step} for c in cases],
           "data": "synthetic (measured images from the same forward model, 1% noise)"}
    # warm-started serving run (the configuration), then the zero-start pair
    runs = {}
    for label, warm, share in (("served_warm", True, args.substep_share),
                               ("served_zero", False, args.substep_share),
                               ("served_warm_one_pass", True, 0.0)):
        srv, need = new_server(share)
        out["arena_bytes"] = int(srv.arena.numel())
        out["request_bytes_max"] = int(need)
        SV.run(srv, arrivals[:2], opts, Ks, warm=warm)          # warm the kernels up
        done = SV.run(srv, arrivals, opts, Ks, warm=warm)
        srv.close()
        runs[label] = done
        summ = SV.summary(done)
        for m in range(2):
            lat = [d.latency_ms for d in done if d.model == m]
            summ[f"model{m}_p50_ms"] = float(np.percentile(lat, 50))
            summ[f"model{m}_p99_ms"] = float(np.percentile(lat, 99))
        out[label] = summ
        log(f"serve {label}: {summ}")
    # the same requests one after another, each alone (zero start)
    ws = {m: torch.empty(B.solve_projection_workspace(cases[m].vol, cases[m].proj, cases[m].K,
                                                      torch.float32), dtype=torch.uint8,
                         device="cuda") for m in range(2)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = []
    for a in arrivals:
        d = devs[a.model]
        w, rep = B.solve_projection(cases[a.model].vol, a.proj, d["f0"], d["mean"], d["U"], a.y,
                                    np.zeros(Ks[a.model]), opts[a.model], workspace=ws[a.model])
        plain.append(w)
    t_plain = time.perf_counter() - t0
    zero = {dn.index: dn.w for dn in runs["served_zero"]}
    out["plain_sequential"] = {"solves_s": n / t_plain, "total_s": t_plain}
    out["served_zero_equals_plain_bitwise"] = bool(all(np.array_equal(zero[i], plain[i])
                                                       for i in range(n)))
    for label, done in runs.items():
        for m in range(2):
            err = [np.linalg.norm(dn.w - arrivals[dn.index].w_true) /
                   np.linalg.norm(arrivals[dn.index].w_true) for dn in done if dn.model == m]
            out[label][f"model{m}_w_rel_err_vs_planted_median"] = float(np.median(err))
            out[label][f"model{m}_w_rel_err_vs_planted_max"] = float(np.max(err))
    # small requests only, all submitted at once (a burst, so that the
    # server's throughput and not the arrival process sets the rate): where
    # one request leaves the GPU idle between launches, batching pays most
    small = [dataclasses.replace(a, t=0.0) for a in arrivals if a.model == 0]
    srv, _ = new_server()
    SV.run(srv, small[:2], opts, Ks, warm=False)
    done = SV.run(srv, small, opts, Ks, warm=False)
    srv.close()
    t0 = time.perf_counter()
    for a in small:
        d = devs[0]
        B.solve_projection(cases[0].vol, a.proj, d["f0"], d["mean"], d["U"], a.y,
                           np.zeros(Ks[0]), opts[0], workspace=ws[0])
    t_small = time.perf_counter() - t0
    out["small_only"] = {"served": SV.summary(done),
                         "plain_sequential_solves_s": len(small) / t_small}
    log(f"serve small only: {out['small_only']}")
    print(json.dumps(out), flush=True)
    return 0


def resolution_mode(case, dev, dt, args) -> int:
    """Detector-resolution sweep (the synthetic analogue of the paper's
    downsampling study): one measurement made with the exact-path (Siddon)
    projector at 1024x768 and 0.4 mm pitch plus 1% noise, binned by 1, 2,
    ..., 32 (pixel means, pitch times the factor), each solved with the
    ray-march P on the clinical volume; latency, evaluations and the error
    against the planted coefficients and tumour position per resolution."""
    import dataclasses

    import torch

    from paper_1102_1712_amd import binding as B

    fine = dataclasses.replace(case.proj, nu=1024, nv=768, pitch_u=0.4, pitch_v=0.4)
    f = B.warp_pca(case.vol, dev["f0"], dev["mean"], dev["U"], case.w_star)
    p = B.drr_siddon(case.vol, fine, f).double()
    gen = torch.Generator(device="cuda").manual_seed(args.seed + 300)
    p = p + 0.01 * torch.sqrt(torch.mean(p ** 2)) * torch.randn(p.shape, generator=gen,
                                                                  device="cuda",
                                                                  dtype=torch.float64)
    loc = torch.empty(4, dtype=torch.float64, device="cuda")
    B.tumour_position(case.vol, dev["mean"], dev["U"], case.w_star, case.tumour_c0, out=loc)
    truth = loc.cpu().numpy()[:3]
    xtol = 1e-7 if case.dtype == "f32" else 1e-10
    opts = solver_opts(args, METHODS[args.method], xtol=xtol, locate=1,
                       c0_mm=tuple(case.tumour_c0))
    rows = []
    for b in (1, 2, 4, 8, 16, 32):
        pj = dataclasses.replace(fine, nu=fine.nu // b, nv=fine.nv // b, pitch_u=fine.pitch_u * b,
                                 pitch_v=fine.pitch_v * b)
        y = p.reshape(pj.nv, b, pj.nu, b).mean(dim=(1, 3)).to(dt).contiguous()
        ws = torch.empty(B.solve_projection_workspace(case.vol, pj, case.K, dt),
                         dtype=torch.uint8, device="cuda")
        w0 = np.zeros(case.K)
        B.solve_projection(case.vol, pj, dev["f0"], dev["mean"], dev["U"], y, w0, opts,
                           workspace=ws)
        ts = []
        for _ in range(max(3, args.steps // 10)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            w, rep = B.solve_projection(case.vol, pj, dev["f0"], dev["mean"], dev["U"], y, w0,
                                        opts, workspace=ws)
            ts.append((time.perf_counter() - t0) * 1e3)
        rows.append({"detector": [pj.nu, pj.nv], "pitch_mm": pj.pitch_u, "bin": b,
                     "p50_ms": float(np.median(ts)), "iters": rep["iters"],
                     "n_fevals": rep["n_fevals"], "status": rep["status"],
                     "w_rel_err_vs_planted": float(np.linalg.norm(w - case.w_star) /
                                                   np.linalg.norm(case.w_star)),
                     "tumour_err_mm": float(np.linalg.norm(np.array(rep["tumour_mm"]) - truth))})
        log(f"resolution {pj.nu}x{pj.nv}: {rows[-1]}")
    print(json.dumps({"mode": "resolution", "workload": case.name,
                      "measurement": "Siddon exact path at 1024x768, 0.4 mm, 1% noise, binned",
                      "rows": rows}), flush=True)
    return 0


def autograd_mode(args) -> int:
    """The differentiation form against the plain solve (clinical volume,
    K = 5, 512x384): the same objective minimised by torch.optim.LBFGS
    (strong-Wolfe line search) over the autograd projector -- whose backward
    is the back-projection + Jacobian chain -- with the intensity fit done in
    torch, and by solve_projection; p50/p99 latency per projection and the
    agreement of the two minimisers."""
    import torch

    from paper_1102_1712_amd import autograd as AG
    from paper_1102_1712_amd import binding as B

    case, dev, dt = build_inputs("clinical_k5", args.seed)
    y = dev["y"]
    yd = y.double()
    M = float(yd.numel())
    sy, syy = float(yd.sum()), float((yd * yd).sum())
    det = syy * M - sy * sy
    model = AG.PCAProjector(case.vol, case.proj, dev["f0"], dev["mean"], dev["U"])

    def objective(w):
        p = model(w).double()
        sp, spy = p.sum(), (p * yd).sum()
        a = (M * spy - sy * sp) / det           # Eq. A.1 (an exact minimiser: the
        b = (syy * sp - sy * spy) / det         # envelope gradient is the fixed-(a, b) one)
        r = p - a * yd - b
        return (r * r).sum()

    def solve_autograd():
        w = torch.zeros(case.K, dtype=torch.float64, requires_grad=True)
        opt = torch.optim.LBFGS([w], lr=1.0, max_iter=60, tolerance_grad=1e-10,
                                tolerance_change=1e-12, history_size=10,
                                line_search_fn="strong_wolfe")
        nev = [0]

        def closure():
            opt.zero_grad()
            J = objective(w)
            J.backward()
            nev[0] += 1
            return J

        opt.step(closure)
        with torch.no_grad():
            J = float(objective(w))
        return w.detach().numpy().copy(), J, nev[0]

    xtol = 1e-7 if case.dtype == "f32" else 1e-10
    ws = torch.empty(B.solve_projection_workspace(case.vol, case.proj, case.K, dt),
                     dtype=torch.uint8, device="cuda")

    def plain(method):
        opts = solver_opts(args, method, xtol=xtol)

        def solve_plain():
            w, rep = B.solve_projection(case.vol, case.proj, dev["f0"], dev["mean"], dev["U"], y,
                                        np.zeros(case.K), opts, workspace=ws)
            return w, rep["J"], rep["n_fevals"] + rep["n_grads"]
        return solve_plain

    out = {"mode": "autograd", "workload": case.name, "K": case.K, "grad_mode": args.grad_mode,
           "precond_of_plain_cg": args.precond if args.grad_mode == 2 else 0,
           "autograd_optimizer": "torch.optim.LBFGS, strong Wolfe, history 10"}
    for label, fn in (("plain", plain(1)), ("plain_bfgs", plain(2)), ("autograd", solve_autograd)):
        fn()
        ts = []
        for _ in range(max(5, args.steps // 5)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            w, J, nev = fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        out[label] = {"p50_ms": float(np.percentile(ts, 50)), "p99_ms": float(np.percentile(ts, 99)),
                      "J": J, "evaluations": nev, "w": list(map(float, w)),
                      "w_rel_err_vs_planted": float(np.linalg.norm(w - case.w_star) /
                                                    np.linalg.norm(case.w_star))}
        log(f"autograd mode {label}: {out[label]}")
    wa, wp = np.array(out["autograd"]["w"]), np.array(out["plain"]["w"])
    out["w_rel_diff"] = float(np.linalg.norm(wa - wp) / np.linalg.norm(wp))
    out["J_rel_diff"] = float(abs(out["autograd"]["J"] - out["plain"]["J"]) / out["plain"]["J"])
    wq = np.array(out["plain_bfgs"]["w"])
    out["bfgs_w_rel_diff"] = float(np.linalg.norm(wa - wq) / np.linalg.norm(wq))
    out["bfgs_J_rel_diff"] = float(abs(out["autograd"]["J"] - out["plain_bfgs"]["J"]) /
                                   out["plain_bfgs"]["J"])
    print(json.dumps(out), flush=True)
    return 0


def random_angles(case, dev, dt, args, base: dict) -> dict:
    """p50/p99 of solves at args.angles seeded random angles in [0, 2 pi),
    CG and BFGS, each angle with its own measured projection."""
    import dataclasses

    import torch

    from paper_1102_1712_amd import binding as B

    rng = np.random.default_rng(args.seed + 400)
    gen = torch.Generator(device="cuda").manual_seed(args.seed + 401)
    angles = rng.uniform(0.0, 2.0 * np.pi, args.angles)
    probs = []
    for th in angles:
        pj = dataclasses.replace(case.proj, angle=float(th))
        rays = B.ray_table(case.vol, pj, dt)
        f = B.warp_pca(case.vol, dev["f0"], dev["mean"], dev["U"], case.w_star)
        p = B.drr_forward(case.vol, pj, rays, f)
        rms = torch.sqrt(torch.mean(p.double() ** 2))
        y = (p.double() + case.noise_level * rms * torch.randn(p.shape, generator=gen, device="cuda",
                                                              dtype=torch.float64)).to(dt)
        probs.append((pj, y.contiguous()))
        del rays, f, p
    ws = torch.empty(B.solve_projection_workspace(case.vol, case.proj, case.K, dt),
                     dtype=torch.uint8, device="cuda")
    out = {"angles": int(args.angles)}
    for label, method in (("cg", 1), ("bfgs", 2)):
        o = B.default_opts(**{**base, "method": method,
                              "precond": base.get("precond", 0) if method == 1 else 0})
        ts, ev, err = [], [], []
        for pj, y in probs:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            w, rep = B.solve_projection(case.vol, pj, dev["f0"], dev["mean"], dev["U"], y,
                                        np.zeros(case.K), o, workspace=ws)
            ts.append((time.perf_counter() - t0) * 1e3)
            ev.append(rep["n_fevals"] + rep["n_grads"])
            err.append(np.linalg.norm(w - case.w_star) / np.linalg.norm(case.w_star))
        out[label] = {"p50_ms": float(np.percentile(ts, 50)), "p99_ms": float(np.percentile(ts, 99)),
                      "mean_ms": float(np.mean(ts)), "mean_evaluations": float(np.mean(ev)),
                      "w_rel_err_vs_planted_median": float(np.median(err))}
    return out


def adjoint_alone(case, dev, S: int, acc32: bool = False) -> dict:
    """The back-projection on its own (in the solve it runs fused with the
    Jacobian chain), HIP events on the current stream, for the DRR+adjoint
    figure; acc32: the 32-bit-accumulator form (drr_adjoint32)."""
    import torch

    from paper_1102_1712_amd import binding as B

    es = 4 if case.dtype == "f32" else 8
    r = dev["y"].clone()
    bp = B.drr_adjoint(case.vol, case.proj, dev["rays"], r, acc32=acc32)
    torch.cuda.synchronize()
    ts = []
    for _ in range(10):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        B.drr_adjoint(case.vol, case.proj, dev["rays"], r, out=bp, acc32=acc32)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    a = float(np.median(ts))
    return {"avg_ms": a, "launches": len(ts), "Gsamples_s": S / (a * 1e-3) / 1e9,
            "effective_GBs": 8 * es * S / (a * 1e-3) / 1e9, "timed": "alone",
            "accumulator_bits": 32 if acc32 else 64}


def drr_alone(case, dev, S: int) -> dict:
    """The one-volume projection p = P f on its own (drr_forward: no
    moments), HIP events on the current stream, for the DRR figure; the
    timed solve projects f with its Jacobian volumes instead."""
    import torch

    from paper_1102_1712_amd import binding as B

    es = 4 if case.dtype == "f32" else 8
    f = B.warp_pca(case.vol, dev["f0"], dev["mean"], dev["U"], case.w_star)
    p = B.drr_forward(case.vol, case.proj, dev["rays"], f)
    torch.cuda.synchronize()
    ts = []
    for _ in range(10):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        B.drr_forward(case.vol, case.proj, dev["rays"], f, out=p)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    a = float(np.median(ts))
    return {"avg_ms": a, "launches": len(ts), "Gsamples_s": S / (a * 1e-3) / 1e9,
            "effective_GBs": 8 * es * S / (a * 1e-3) / 1e9, "timed": "alone"}


def tiny_latency(args) -> dict:
    """The tiny workload (64^3 FP64, 128x128 detector, K = 3) solved with
    the same options as the benchmark's solve, one call at a time: p50/p99
    latency of solve_projection (launch- and read-back-bound at this size)."""
    import torch

    from paper_1102_1712_amd import binding as B

    case, dev, dt = build_inputs("tiny", 0)
    ws = torch.empty(B.solve_projection_workspace(case.vol, case.proj, case.K, dt),
                     dtype=torch.uint8, device="cuda")
    w0 = np.zeros(case.K)

    def run(speculate, n, grad_mode=args.grad_mode, precond=None):
        kw = {"grad_mode": grad_mode}
        kw["precond"] = (args.precond if grad_mode == 2 else 0) if precond is None else precond
        o = B.default_opts(locate=1, c0_mm=tuple(case.tumour_c0), speculate=speculate, **kw)
        for _ in range(3):
            B.solve_projection(case.vol, case.proj, dev["f0"], dev["mean"], dev["U"], dev["y"],
                               w0, o, workspace=ws)
        ts, hs = [], []
        for _ in range(n):
            t0 = time.perf_counter()
            w, rep = B.solve_projection(case.vol, case.proj, dev["f0"], dev["mean"], dev["U"],
                                        dev["y"], w0, o, workspace=ws)
            ts.append((time.perf_counter() - t0) * 1e3)
            hs.append((rep["host_ms"], rep["host_ms"] - rep["wait_ms"]))
        return w, rep, ts, np.array(hs)

    w, rep, ts, hs = run(1, max(20, args.tiny_steps))
    _, rep0, ts0, _ = run(0, 20, 1)
    others = {label: float(np.percentile(run(1, 20, gm, pc)[2], 50))
              for label, gm, pc in SOLVER_VARIANTS}
    return {"workload": case.name, "solves": len(ts), "p50_ms": float(np.percentile(ts, 50)),
            "grad_mode": args.grad_mode, "precond": args.precond if args.grad_mode == 2 else 0,
            "p50_ms_by_solver": others,
            "p99_ms": float(np.percentile(ts, 99)), "mean_ms": float(np.mean(ts)),
            "library_p50_ms": float(np.percentile(hs[:, 0], 50)),
            "host_work_p50_ms": float(np.percentile(hs[:, 1], 50)),
            "route1_no_speculation_p50_ms": float(np.percentile(ts0, 50)),
            "iters": rep["iters"], "n_fevals": rep["n_fevals"], "n_grads": rep["n_grads"],
            "spec_grads": rep["spec_grads"],
            "w_rel_err_vs_planted": float(np.linalg.norm(w - case.w_star) /
                                          np.linalg.norm(case.w_star))}


def oracle_minimiser(case):
    """The FP64 oracle's minimiser of this workload stored beside the tests
    (written by a script that calls the oracle alone), or None when the
    workload is not the stored one."""
    path = os.path.join(ROOT, "tests", "golden", "clinical_minimiser.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        g = json.load(fh)
    if g.get("workload") != case.name or g.get("angle") != case.proj.angle:
        return None
    return g["fit"]


def measured_hbm_frac(kernel: str, workload: str, avg_ms):
    """Measured HBM bytes per launch (profiles/, when current) over the
    launch's duration, as a fraction of the 8 TB/s peak."""
    t = measured_traffic(kernel, workload)
    if t is None or not avg_ms:
        return None
    return t / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS


def host_time(step, base, args):
    """The solve with no timing events at all: wall time of the Python call,
    the library's own wall time of the C call (report.host_ms) and its host
    work outside read-back waits, with and without speculative gradients.  Busy time of the kernels is not taken
    from events here: an event pair around every kernel stretches each one
    by the marker's dispatch, so their sum exceeds the event-free solve."""
    from paper_1102_1712_amd import binding as B
    out = {}
    for name, spec in (("", 1), ("no_speculation_", 0)):
        o = B.default_opts(profile=0, speculate=spec, **base)
        step(o)
        ts, hs, ws = [], [], []
        for _ in range(max(10, args.steps // 2)):
            t0 = time.perf_counter()
            _, r = step(o)
            ts.append((time.perf_counter() - t0) * 1e3)
            hs.append(r["host_ms"])
            ws.append(r["host_ms"] - r["wait_ms"])
        out[name + "p50_ms"] = float(np.percentile(ts, 50))
        out[name + "library_p50_ms"] = float(np.percentile(hs, 50))
        # host work in the library outside its read-back waits (an upper
        # bound of what the GPU waits for the host: launches queued behind a
        # running kernel cost it nothing)
        out[name + "host_work_p50_ms"] = float(np.percentile(ws, 50))
        out[name + "spec_grads"] = r["spec_grads"]
    out["n_grads"] = r["n_grads"]
    log(f"host time: {out}")
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="clinical", choices=["clinical", "tiny"])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--tiny-steps", type=int, default=50,
                    help="solve mode: tiny-workload solves timed for its p50/p99 (0: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="time the steps without per-kernel HIP events")
    ap.add_argument("--mode", default="solve",
                    choices=["solve", "kernels", "stream", "serve", "resolution", "autograd"],
                    help="solve: the contract line; kernels: each hot kernel alone plus a "
                         "copy of known size (for profiler counters); stream: a warm-started "
                         "projection sequence; serve: batched mixed-size serving; "
                         "resolution: detector-binning sweep on exact-path data; autograd: "
                         "the differentiation form against the plain solve")
    ap.add_argument("--grad-mode", type=int, default=2, choices=[0, 1, 2],
                    help="gradient route of the timed solve (opts.grad_mode)")
    ap.add_argument("--precond", type=int, default=1, choices=[0, 1],
                    help="CG preconditioned by the Gauss-Newton matrix (opts.precond; "
                         "grad_mode 2 and cg only)")
    ap.add_argument("--method", default="cg", choices=list(METHODS),
                    help="solver: PR+ CG (the configured one), BFGS, or the Appendix algorithm")
    ap.add_argument("--angles", type=int, default=100,
                    help="solve mode: seeded random angles timed besides the fixed one (0: none)")
    ap.add_argument("--frames", type=int, default=600)
    ap.add_argument("--requests", type=int, default=32)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--substep-share", type=float, default=0.25,
                    help="serving: extra passes for cheap requests, share of the main pass")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the per-projection solve runs on a single "
              "MI355X (multi-GPU sharding is a design note, not built); use --gpus 1",
              file=sys.stderr)
        return 2

    import torch

    from paper_1102_1712_amd import binding as B

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    B.lib()
    if args.mode == "serve":
        return serve_mode(args)
    if args.mode == "autograd":
        return autograd_mode(args)
    case, dev, dt = build_inputs(args.workload, args.seed)
    if args.mode == "kernels":
        return kernels_mode(case, dev, dt, max(args.steps, 1))
    if args.mode == "stream":
        return stream_mode(case, dev, dt, args)
    if args.mode == "resolution":
        return resolution_mode(case, dev, dt, args)
    S = samples_per_drr(dev["rays"], case.dtype)
    # voxels the solve's warp writes (live bricks) and the chain works on
    live = B.live_voxels(case.vol, case.proj)
    reach = reached_voxels(case, dev)
    ws = torch.empty(B.solve_projection_workspace(case.vol, case.proj, case.K, dt),
                     dtype=torch.uint8, device="cuda")
    xtol = 1e-7 if case.dtype == "f32" else 1e-10
    base = dict(locate=1, c0_mm=tuple(case.tumour_c0), xtol=xtol)
    base["method"] = METHODS[args.method]
    base["grad_mode"] = args.grad_mode
    base["precond"] = args.precond if (args.grad_mode == 2 and args.method == "cg") else 0
    timed = ("pcg" if base["precond"] else args.method) + f"_route{args.grad_mode}"
    opts_warm = B.default_opts(profile=0 if args.no_profile else B.PROFILE_ALL, **base)
    w0 = np.zeros(case.K)

    def step(o):
        return B.solve_projection(case.vol, case.proj, dev["f0"], dev["mean"], dev["U"], dev["y"],
                                  w0, o, workspace=ws)

    wms, wn = {}, {}
    for i in range(args.warmup):
        w, rep = step(opts_warm)
        for k, v in rep["kernel_ms"].items():
            wms[k] = wms.get(k, 0.0) + v
            wn[k] = wn.get(k, 0) + rep["kernel_launches"][k]
        log(f"warmup {i}: iters {rep['iters']} fevals {rep['n_fevals']} grads {rep['n_grads']} "
            f"status {rep['status']}")
    # the timed steps carry events around the dominant kernel class only
    # (every class when there was no warmup to name it)
    warm_dominant = max((k for k in wms if wn.get(k)), key=lambda k: wms[k], default=None)
    if args.no_profile:
        mask = 0
    elif warm_dominant is None:
        mask = B.PROFILE_ALL
    else:
        mask = B.profile_mask(warm_dominant)
    opts_timed = B.default_opts(profile=mask, **base)

    times, kms, kn = [], {}, {}
    torch.cuda.synchronize()
    t_begin = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        w, rep = step(opts_timed)
        times.append(time.perf_counter() - t0)
        for k, v in rep["kernel_ms"].items():
            kms[k] = kms.get(k, 0.0) + v
            kn[k] = kn.get(k, 0) + rep["kernel_launches"][k]
    torch.cuda.synchronize()
    total = time.perf_counter() - t_begin
    log(f"timed {args.steps} steps in {total:.3f} s")

    ms = np.array(times) * 1e3
    host = host_time(step, base, args)
    werr = float(np.linalg.norm(w - case.w_star) / np.linalg.norm(case.w_star))
    N, M = case.vol.nvox, case.proj.npix
    es = 4 if case.dtype == "f32" else 8
    K = case.K
    avg = {k: (kms[k] / kn[k] if kn.get(k) else None) for k in kms}
    # algorithmic bytes per launch ("Roofline accounting");
    # the solve's warp writes only live bricks, its chain reads the fields
    # only where P^T r can be nonzero
    alg_bytes = {
        "warp_pca": (3 + 3 * K + 2) * es * live,
        # reads mean, U, f0; writes f and the K Jacobian volumes
        "warp_jac": (3 + 3 * K + 1 + 1 + K) * es * live,
        "drr_forward_eval": (K + 1) * es * N + 32 * M + 2 * es * M,
        "grad_w": (3 + 3 * K + 2) * es * N,
        "jacobian": (3 + 3 * K + 1 + K) * es * N,
        "drr_forward": es * N + 32 * M + 2 * es * M,
        "drr_adjoint": es * N + 32 * M + 2 * es * M,
        "drr_adjoint_chain": (3 + 3 * K + 1) * es * reach + 32 * M + 2 * es * M,
        "drr_forward_dot": K * es * N + 32 * M + 2 * es * M,
    }
    # per-class figures: from the timed steps where that class carried events,
    # else from the warmup steps ("events" says which)
    kernel_stats = {}
    for k in B.KERNEL_CLASSES:
        if kn.get(k):
            a, n_k, tot, src = avg[k], kn[k], kms[k], "timed"
        elif wn.get(k):
            a, n_k, tot, src = wms[k] / wn[k], wn[k], wms[k], "warmup"
        else:
            continue
        d = {"avg_ms": a, "launches": n_k, "total_ms": tot, "events": src}
        if k in alg_bytes:
            d["alg_GBs"] = alg_bytes[k] / (a * 1e-3) / 1e9
        if k in SAMPLE_KERNELS:
            nvol = {"drr_forward_dot": K, "drr_forward_eval": K + 1}.get(k, 1)
            d["Gsamples_s"] = S / (a * 1e-3) / 1e9
            d["effective_GBs"] = 8 * es * nvol * S / (a * 1e-3) / 1e9
        kernel_stats[k] = d
    measured = [k for k in kms if kn.get(k)]
    dominant = max(measured, key=lambda k: kms[k]) if measured else None

    roofline = None
    wl = "clinical" if args.workload == "clinical" else args.workload
    traffic = measured_traffic(dominant, wl) if dominant else None
    if dominant in alg_bytes and avg.get(dominant):
        if dominant in HBM_KERNELS:
            ach = alg_bytes[dominant] / (avg[dominant] * 1e-3) / 1e9
            roofline = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "kernel": dominant}
        else:
            # gather / VALU bound: algorithmic flops per projection sample (plus
            # the chain per voxel for the fused back-projection)
            work = flops_per_sample(dominant, K) * S
            if dominant == "drr_adjoint_chain":
                work += chain_flops_per_voxel(K) * reach
            ach = work / (avg[dominant] * 1e-3) / 1e12
            roofline = {"bound": "alu", "achieved": ach, "peak": VALU_F32_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": ach / VALU_F32_PEAK_TFLOPS, "traffic": traffic,
                        "kernel": dominant}

    # the other solver configurations (gradient route 0: projected Jacobian
    # volumes; 1: back-projection + chain; 2: fused evaluation; CG plain or
    # preconditioned by the Gauss-Newton matrix), same solve otherwise;
    # reported beside the contract line, not as `value`
    alt = {}
    for label, gm, pc in SOLVER_VARIANTS:
        if label == timed:
            continue
        alt_t = []
        opts_alt = B.default_opts(**{**base, "grad_mode": gm, "precond": pc})
        step(opts_alt)
        for _ in range(max(5, args.steps // 5)):
            t0 = time.perf_counter()
            w_alt, rep_alt = step(opts_alt)
            alt_t.append(time.perf_counter() - t0)
        alt_ms = np.array(alt_t) * 1e3
        alt[label] = {"grad_mode": gm, "precond": pc, "steps": len(alt_t),
                        "p50_ms": float(np.percentile(alt_ms, 50)),
                        "p99_ms": float(np.percentile(alt_ms, 99)),
                        "solves_s": float(1e3 / np.mean(alt_ms)), "n_fevals": rep_alt["n_fevals"],
                        "n_grads": rep_alt["n_grads"],
                        "w_rel_diff_vs_timed": float(np.linalg.norm(w_alt - w) /
                                                     np.linalg.norm(w))}
        log(f"solver {label}: p50 {alt[label]['p50_ms']:.3f} ms")

    # the quasi-Newton solver on the same problem (same line search, same
    # stops), beside the configured CG: latency and agreement of the minimisers
    qn = None
    if args.method == "cg":
        opts_qn = B.default_opts(**{**base, "method": 2, "precond": 0})
        step(opts_qn)
        qn_t = []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            w_qn, rep_qn = step(opts_qn)
            qn_t.append(time.perf_counter() - t0)
        qn_ms = np.array(qn_t) * 1e3
        qn = {"method": "bfgs", "steps": len(qn_t), "p50_ms": float(np.percentile(qn_ms, 50)),
              "p99_ms": float(np.percentile(qn_ms, 99)), "solves_s": float(1e3 / np.mean(qn_ms)),
              "iters": rep_qn["iters"], "n_fevals": rep_qn["n_fevals"],
              "n_grads": rep_qn["n_grads"], "status": rep_qn["status"],
              "grad_mode": args.grad_mode,
              "w_rel_diff_vs_timed": float(np.linalg.norm(w_qn - w) / np.linalg.norm(w)),
              "J_rel_diff_vs_timed": float((rep_qn["J"] - rep["J"]) / rep["J"])}
        log(f"quasi-Newton: p50 {qn['p50_ms']:.3f} ms, {qn['n_fevals']} evaluations")

    # accuracy of the timed solve against the FP64 oracle's minimiser
    gold = oracle_minimiser(case)
    acc = {}
    if gold is not None:
        w_ref = np.array(gold["w"])
        acc = {"w_rel_err_vs_oracle_minimiser": float(np.linalg.norm(w - w_ref) /
                                                      np.linalg.norm(w_ref)),
               "tumour_err_mm_vs_oracle": float(np.linalg.norm(np.array(rep["tumour_mm"]) -
                                                               np.array(gold["tumour_mm"])))}
    log(f"accuracy: {acc}")
    # the same solve without the polish step: it stops where FP32 values of J
    # stop resolving decreases
    opts_np = B.default_opts(**{**base, "polish": 0})
    step(opts_np)
    np_t = []
    for _ in range(max(5, args.steps // 5)):
        t0 = time.perf_counter()
        w_np, rep_np = step(opts_np)
        np_t.append((time.perf_counter() - t0) * 1e3)
    unpolished = {"steps": len(np_t), "p50_ms": float(np.percentile(np_t, 50)),
                  "solves_s": float(1e3 / np.mean(np_t)), "n_fevals": rep_np["n_fevals"],
                  "n_grads": rep_np["n_grads"]}
    if gold is not None:
        unpolished["w_rel_err_vs_oracle_minimiser"] = float(
            np.linalg.norm(w_np - np.array(gold["w"])) / np.linalg.norm(gold["w"]))
    log(f"unpolished: {unpolished}")

    # the same solve at seeded random gantry angles, each with its own
    # measured projection (same recipe: P f(w*) + 1% noise)
    rand = random_angles(case, dev, dt, args, base) if args.angles > 0 else None
    log(f"random angles: {rand}")

    tiny = tiny_latency(args) if args.tiny_steps > 0 and args.workload == "clinical" else None
    log(f"tiny: {tiny}")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host cores")
        cpu = cpu_baseline(case, S)

    drr = kernel_stats.get("drr_forward") or drr_alone(case, dev, S)
    if "drr_forward" not in kernel_stats:
        kernel_stats["drr_forward_alone"] = drr
    fused = kernel_stats.get("drr_forward_eval", {})
    # the back-projection alone (in the solve it runs fused with the chain)
    adj = adjoint_alone(case, dev, S)
    kernel_stats["drr_adjoint_alone"] = adj
    if case.dtype == "f32":
        kernel_stats["drr_adjoint32_alone"] = adjoint_alone(case, dev, S, acc32=True)
    out = {
        "metric": METRIC,
        "value": args.steps / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": float(total / args.steps * 1e3),
        "p50_ms": float(np.percentile(ms, 50)),
        "p99_ms": float(np.percentile(ms, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": case.dtype,
        "data": "synthetic",
        "config": {"workload": case.name, "volume": list(case.vol.n),
                   "spacing_mm": list(case.vol.spacing),
                   "detector": [case.proj.nu, case.proj.nv], "pitch_mm": case.proj.pitch_u,
                   "step_mm": case.proj.step, "K": K, "method": args.method, "max_iter": 30,
                   "samples_per_drr": S, "angle_rad": case.proj.angle,
                   "live_voxels": live, "reached_voxels": reach},
        "solve": {"iters": rep["iters"], "n_fevals": rep["n_fevals"], "n_grads": rep["n_grads"],
                  "status": rep["status"], "polish": 1, "w_rel_err_vs_planted": werr,
                  "tumour_mm": rep["tumour_mm"], **acc},
        "unpolished": unpolished,
        "host": host,
        "tiny": tiny,
        "drr_gsamples_s": drr.get("Gsamples_s"),
        "adjoint_gsamples_s": adj.get("Gsamples_s"),
        # the timed solve's projection of f with its K Jacobian volumes
        "fused_evaluation_gsamples_s": fused.get("Gsamples_s"),
        # 8 corner values of sizeof(T) per sample at the kernel's rate: a
        # nominal gather rate, not HBM traffic (most gathers hit LDS or L2)
        "drr_nominal_gather_GBs": drr.get("effective_GBs"),
        "adjoint_nominal_gather_GBs": adj.get("effective_GBs"),
        # HBM bytes the profiler measured per launch over the launch time
        "hbm_measured_frac": {k: measured_hbm_frac(k, wl, kernel_stats[k]["avg_ms"])
                              for k in kernel_stats if k in KERNEL_SOURCES},
        "kernels": kernel_stats,
        "timed_region_events": [k for i, k in enumerate(B.KERNEL_CLASSES) if mask >> i & 1],
        "solver": {"method": args.method, "grad_mode": args.grad_mode,
                   "precond": base["precond"], "label": timed},
        "other_solvers": alt,
        "quasi_newton": qn,
        "random_angles": rand,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "paper_context": "0.1-0.3 s per projection on a Tesla C1060 (different sizes; context only)",
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
