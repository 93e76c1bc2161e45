"""Serving at the mixed-size workload's own sizes: two requests of a
512x512x256 FP32 model with K = 5 modes and a 1024x768 detector at 0.4 mm,
and two of a 128x128x96 FP32 model with K = 3 and a 512x384 detector at
0.4 mm, in flight together in one server.  Every result must equal, bit for
bit, solve_projection's for the same request alone.

The small model is the seeded synthetic case of the serving benchmark.  The
large one is drawn here on the GPU (the same kinds of fields: an ellipsoid
phantom with textured lungs and a tumour, smooth Gaussian-bump modes), which
takes well under a second against about two minutes for the host recipe;
the comparison is between two GPU paths, so the inputs only need the right
sizes and shapes.  Both served gradient routes are checked: back-projection
with the chain fused, and the fused evaluation."""
import dataclasses
import math

import numpy as np
import pytest

from paper_1102_1712_amd import binding as B
from paper_1102_1712_amd import synth

from gpu_common import say, torch_or_skip

pytestmark = pytest.mark.gpu


def _gpu_model(torch, n, spacing, K, seed):
    """Phantom, mean field and K unit-RMS smooth modes as float32 device
    tensors, from seeded bump parameters."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    rng = np.random.default_rng(seed)
    n1, n2, n3 = n
    ax = [(torch.arange(m, device="cuda", dtype=torch.float64) - (m - 1) / 2.0) * s
          for m, s in zip(n, spacing)]
    E = np.array([m * s for m, s in zip(n, spacing)])
    X, Y, Z = ax[0][None, None, :], ax[1][None, :, None], ax[2][:, None, None]

    def ellipsoid(c, semi):
        return ((X - c[0]) / semi[0]) ** 2 + ((Y - c[1]) / semi[1]) ** 2 + \
               ((Z - c[2]) / semi[2]) ** 2 <= 1.0

    body = ellipsoid((0, 0, 0), 0.45 * E * np.array([1.0, 0.35 / 0.45, 0.48 / 0.45]))
    f0 = torch.where(body, 0.02, 0.0).to(torch.float64)
    for sgn in (1.0, -1.0):
        lung = ellipsoid((sgn * 0.2 * E[0], 0, 0), E * np.array([0.15, 0.22, 0.30])) & body
        f0 = torch.where(lung, 0.005, f0)
    f0 = torch.where(ellipsoid((-0.2 * E[0], 0.05 * E[1], 0.1 * E[2]), (5, 5, 5)), 0.02, f0)
    tex = torch.randn(f0.shape, generator=g, device="cuda", dtype=torch.float64) * 0.001
    f0 = torch.where(body, torch.clamp(f0 + tex, min=0.0), 0.0)

    def field():
        out = torch.zeros((3, n3, n2, n1), device="cuda", dtype=torch.float64)
        for _ in range(8):
            c = rng.uniform(-0.4, 0.4, 3) * E
            sig = rng.uniform(20.0, 50.0)
            d = rng.normal(size=3)
            d *= rng.uniform(0.0, 10.0) / np.linalg.norm(d)
            G = torch.exp(-(X - c[0]) ** 2 / (2 * sig * sig)) * \
                torch.exp(-(Y - c[1]) ** 2 / (2 * sig * sig)) * \
                torch.exp(-(Z - c[2]) ** 2 / (2 * sig * sig))
            for comp in range(3):
                out[comp] += float(d[comp]) * G
        return out / torch.sqrt(torch.mean(out * out) * 3.0)

    U = torch.stack([field() for _ in range(K)]).to(torch.float32).contiguous()
    mean = (0.5 * field()).to(torch.float32).contiguous()
    w_star = rng.normal(size=K) * 0.5
    return f0.to(torch.float32).contiguous(), mean, U, w_star


def _measured(torch, vol, proj, f0, mean, U, w, seed):
    rays = B.ray_table(vol, proj, torch.float32)
    p = B.drr_forward(vol, proj, rays, B.warp_pca(vol, f0, mean, U, w))
    rms = torch.sqrt(torch.mean(p.double() ** 2))
    noise = torch.randn(p.shape, generator=torch.Generator(device="cuda").manual_seed(seed),
                        device="cuda", dtype=torch.float64)
    return (p.double() + 0.01 * rms * noise).float().contiguous()


@pytest.mark.parametrize("grad_mode", [1, 2])
def test_mixed_full_size_served_equals_alone(grad_mode):
    torch = torch_or_skip()
    say("building the 512x512x256 K=5 model on the GPU")
    large_vol = synth.centred_volume((512, 512, 256), (0.75, 0.75, 1.25))
    lf0, lmean, lU, lw = _gpu_model(torch, large_vol.n, large_vol.spacing, 5, 41)
    large_proj = synth.Projection(angle=0.9, sad=1000.0, sid=1500.0, nu=1024, nv=768,
                                  pitch_u=0.4, pitch_v=0.4, step=0.375)
    say("building the 128x128x96 K=3 model")
    small = synth.serve_small()
    sf0, smean, sU = (torch.from_numpy(a).cuda() for a in small.arrays(np.float32))
    models = [(large_vol, lf0, lmean, lU, 5, lw), (small.vol, sf0, smean, sU, 3, small.w_star)]
    reqs = []
    for m, (vol, f0, mean, U, K, w) in enumerate(models):
        base = large_proj if m == 0 else small.proj
        for j in range(2):
            pj = dataclasses.replace(base, angle=base.angle + 1.3 * j + 0.4 * m)
            y = _measured(torch, vol, pj, f0, mean, U, w * (1.0 + 0.2 * j), 100 + 10 * m + j)
            reqs.append((m, pj, y))
    opts = B.default_opts(xtol=1e-7, grad_mode=grad_mode)
    srv0 = B.Server(B.Server.reserved_bytes(4) + (1 << 20), max_active=4)
    for vol, f0, mean, U, K, _ in models:
        srv0.add_model(vol, f0, mean, U)
    need = sum(srv0.request_bytes(m, pj, opts) for m, pj, _ in reqs)
    srv0.close()
    srv = B.Server(B.Server.reserved_bytes(4) + need + (4 << 20), max_active=4)
    for vol, f0, mean, U, K, _ in models:
        srv.add_model(vol, f0, mean, U)
    rids = [srv.submit(m, pj, y, np.zeros(models[m][4]), opts) for m, pj, y in reqs]
    s = srv.stats()
    say("submitted", s)
    results, steps = {}, 0
    while len(results) < len(rids):
        srv.step()
        steps += 1
        if steps == 1:
            assert srv.stats()["active"] == 4          # all four in flight together
        assert steps < 4000
        for rid in rids:
            if rid not in results:
                done, st, w, rep = srv.poll(rid)
                if done:
                    results[rid] = (st, w, rep)
    say("served in", steps, "steps")
    for rid, (m, pj, y) in zip(rids, reqs):
        st, w, rep = results[rid]
        vol, f0, mean, U, K, _ = models[m]
        w1, rep1 = B.solve_projection(vol, pj, f0, mean, U, y, np.zeros(K), opts)
        say("model", m, "w", w, rep["n_fevals"], rep["n_grads"])
        assert st == 0 and rep["status"] in ("converged", "max_iter")
        assert np.array_equal(w, w1), (m, w, w1)
        for key in ("status", "iters", "n_fevals", "n_grads", "J", "a", "b", "gnorm"):
            assert rep[key] == rep1[key], key
        assert math.isfinite(rep["J"])
    srv.close()
