"""Serving: concurrent solves of different volume sizes, K and dtype batched
into shared launches.  Every result must equal, bit for bit, the result of
solve_projection for the same request alone; admission is by arena
footprint; a failing request does not disturb the others."""
import numpy as np
import pytest

from paper_1102_1712_amd import binding as B
from paper_1102_1712_amd import serve as SV
from paper_1102_1712_amd import synth

from gpu_common import Dev, measured, say, to_dev, torch_or_skip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_or_skip()


def _models():
    """Three resident models: FP32 K=3, FP32 K=5 (another size), FP64 K=3."""
    a = synth.small(dtype="f32", seed=21)
    b = synth.make_case("serve-test-48x44x36-K5-f32", (48, 44, 36), (4.5, 5.0, 6.0), (56, 44),
                        (6.5, 7.5), 2.25, 5, "f32", 22)
    c = synth.small(dtype="f64", seed=23)
    return [a, b, c]


def _requests(cases, devs, n_per):
    """(model, projection, measurement) at several angles per model."""
    reqs = []
    for m, (c, d) in enumerate(zip(cases, devs)):
        for j in range(n_per):
            cj = synth.with_angle(c, c.proj.angle + 0.7 * j)
            y = to_dev(measured(cj), d.dt)
            reqs.append((m, cj.proj, y))
    return reqs


def _alone(c, d, proj, y, w0, opts):
    return B.solve_projection(c.vol, proj, d.f0, d.mean, d.U, y, w0, opts)


def _opts(c):
    xtol = 1e-7 if c.dtype == "f32" else 1e-10
    return B.default_opts(xtol=xtol, locate=1, c0_mm=tuple(c.tumour_c0))


@pytest.mark.parametrize("share,route", [(0.25, 1), (0.0, 1), (4.0, 1), (0.25, 2), (4.0, 2),
                                         (0.25, "mixed")])
def test_batched_results_equal_alone(torch, share, route):
    """Every request's result equals its solve alone, bit for bit, whatever
    the passes it ran in (one per step, or extra passes for cheap ones) and
    whichever gradient route it takes (back-projection, or the fused
    evaluation; "mixed": both kinds in flight together)."""
    cases = _models()
    devs = [Dev(c) for c in cases]
    reqs = _requests(cases, devs, 3)
    # one request of model 0 runs the Appendix algorithm, one without the
    # fit, two with the quasi-Newton solver, two with the polish step (which
    # evaluates into the second projection slot); two measure 100 y + 50, so
    # the FP32 one's first objective (moments about the fit (1, 0)) cancels
    # and is summed again by the two-pass residual
    reqs = [(m, pj, y * 100.0 + 50.0 if i in (0, 7) else y) for i, (m, pj, y) in enumerate(reqs)]
    opts = []
    for i, (m, pj, y) in enumerate(reqs):
        o = _opts(cases[m])
        if i == 1:
            o = B.paper_opts(locate=1, c0_mm=tuple(cases[m].tumour_c0))
        if i == 4:
            o.fit_intensity = 0
        if i in (2, 6):
            o.method = 2
        if i in (5, 6):
            o.polish = 1
        o.grad_mode = (1 + i % 2) if route == "mixed" else route
        if o.grad_mode == 2 and o.method == 1 and i % 3 == 0:
            o.precond = 1   # CG preconditioned by the Gauss-Newton matrix
        opts.append(o)
    srv = B.Server(256 << 20, max_active=16)
    srv.set_substep_share(share)
    mids = [srv.add_model(c.vol, d.f0, d.mean, d.U) for c, d in zip(cases, devs)]
    assert mids == [0, 1, 2]
    say("serving", len(reqs), "requests of 3 models")
    rids = [srv.submit(m, pj, y, np.zeros(cases[m].K), o) for (m, pj, y), o in zip(reqs, opts)]
    steps = 0
    results = {}
    while len(results) < len(rids):
        srv.step()
        steps += 1
        assert steps < 2000
        for rid in rids:
            if rid in results:
                continue
            done, st, w, rep = srv.poll(rid)
            if done:
                results[rid] = (st, w, rep)
    say("steps", steps)
    for rid, (m, pj, y), o in zip(rids, reqs, opts):
        st, w, rep = results[rid]
        assert st == 0
        c, d = cases[m], devs[m]
        w1, rep1 = _alone(c, d, pj, y, np.zeros(c.K), o)
        assert np.array_equal(w, w1), (m, w, w1)
        for key in ("status", "iters", "n_fevals", "n_grads", "J", "a", "b", "gnorm", "tumour_mm"):
            assert rep[key] == rep1[key], key
        # CG and BFGS requests by the back-projection route take gradients
        # launched behind their evaluations, as a solve alone does (the
        # Appendix algorithm never; the fused evaluation needs none)
        if o.method in (1, 2) and o.grad_mode == 1:
            assert rep["n_grads"] - 2 <= rep["spec_grads"] <= rep["n_grads"], (rep["spec_grads"], rep["n_grads"])
            assert rep["spec_grads"] == rep1["spec_grads"]
        else:
            assert rep["spec_grads"] == 0
    srv.close()


def test_admission_by_footprint_and_arrivals(torch):
    """An arena that holds two requests: the rest wait, and requests
    submitted while others run are admitted as space frees up."""
    c = synth.small(dtype="f32", seed=24)
    d = Dev(c)
    srv0 = B.Server(B.Server.reserved_bytes(4) + (1 << 20), max_active=4)
    mid = srv0.add_model(c.vol, d.f0, d.mean, d.U)
    need = srv0.request_bytes(mid, c.proj)
    srv0.close()
    srv = B.Server(B.Server.reserved_bytes(4) + 2 * need + 4096, max_active=4)
    mid = srv.add_model(c.vol, d.f0, d.mean, d.U)
    reqs = []
    for j in range(6):
        cj = synth.with_angle(c, c.proj.angle + 0.5 * j)
        reqs.append((cj.proj, to_dev(measured(cj), d.dt)))
    opts = B.default_opts(xtol=1e-7)
    rids = [srv.submit(mid, pj, y, np.zeros(c.K), opts) for pj, y in reqs[:4]]
    srv.step()
    s = srv.stats()
    say("after one step", s)
    assert s["active"] == 2 and s["pending"] == 2
    assert s["arena_used"] <= srv.arena.numel()
    for _ in range(3):
        srv.step()
    rids += [srv.submit(mid, pj, y, np.zeros(c.K), opts) for pj, y in reqs[4:]]
    results = {}
    steps = 0
    while len(results) < len(rids):
        srv.step()
        steps += 1
        assert steps < 2000
        for rid in rids:
            if rid not in results:
                done, st, w, rep = srv.poll(rid)
                if done:
                    results[rid] = (st, w)
    for rid, (pj, y) in zip(rids, reqs):
        st, w = results[rid]
        w1, _ = _alone(c, d, pj, y, np.zeros(c.K), opts)
        assert st == 0 and np.array_equal(w, w1)
    srv.close()


def test_failing_request_is_isolated(torch):
    c = synth.small(dtype="f32", seed=25)
    d = Dev(c)
    srv = B.Server(64 << 20, max_active=8)
    mid = srv.add_model(c.vol, d.f0, d.mean, d.U)
    y = to_dev(measured(c), d.dt)
    flat = torch.full_like(y, 3.0)                      # Y^T Y singular
    opts = B.default_opts(xtol=1e-7)
    good = srv.submit(mid, c.proj, y, np.zeros(c.K), opts)
    bad = srv.submit(mid, c.proj, flat, np.zeros(c.K), opts)
    res = {}
    for _ in range(2000):
        srv.step()
        for rid in (good, bad):
            if rid not in res:
                done, st, w, rep = srv.poll(rid)
                if done:
                    res[rid] = (st, w)
        if len(res) == 2:
            break
    assert res[bad][0] == -3                           # PCAS_ESINGULAR
    w1, _ = _alone(c, d, c.proj, y, np.zeros(c.K), opts)
    assert res[good][0] == 0 and np.array_equal(res[good][1], w1)
    with pytest.raises(B.PcasError):
        srv.submit(mid, c.proj, y, np.zeros(c.K), B.default_opts(grad_mode=0))
    srv.close()


def test_poisson_stream_driver(torch):
    """The request loop with Poisson arrivals and warm starts: every request
    completes and matches its own solve from the same starting point."""
    cases = _models()[:2]
    devs = [Dev(c) for c in cases]
    srv = B.Server(256 << 20, max_active=6)
    for c, d in zip(cases, devs):
        srv.add_model(c.vol, d.f0, d.mean, d.U)
    times = SV.poisson_times(200.0, 10, seed=3)
    arrivals = []
    for j, t in enumerate(times):
        m = j % 2
        cj = synth.with_angle(cases[m], cases[m].proj.angle + 0.3 * j)
        arrivals.append(SV.Arrival(t=float(t), model=m, proj=cj.proj,
                                   y=to_dev(measured(cj), devs[m].dt)))
    opts = {m: B.default_opts(xtol=1e-7) for m in range(2)}
    done = SV.run(srv, arrivals, opts, {m: cases[m].K for m in range(2)}, warm=False)
    say(SV.summary(done))
    assert len(done) == 10 and all(d.status == 0 for d in done)
    for dn in done:
        a = arrivals[dn.index]
        c, d = cases[a.model], devs[a.model]
        w1, _ = _alone(c, d, a.proj, a.y, np.zeros(c.K), opts[a.model])
        assert np.array_equal(dn.w, w1)
    srv.close()
