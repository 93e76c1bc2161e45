"""Solve parity: solve_projection through the C ABI against the oracle on
the same inputs and the same w0.  The library's CG and BFGS take steps of
their own (a model first trial, an extrapolated trial, a noise-band stop and
a polish step), so converged minimisers are compared with the oracle's
reference minimiser (oracle.minimise: plain CG, then Newton's method on the
gradient): 1e-4 relative in w, 0.05 mm in the tumour position.  The
Appendix algorithm, fully specified by the paper, is compared step for
step."""
import numpy as np
import pytest

import oracle as O
from paper_1102_1712_amd import binding as B
from paper_1102_1712_amd import synth

from gpu_common import Dev, measured, say, to_dev, to_np, torch_or_skip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_or_skip()


def _gpu_solve(d, y, opts):
    c = d.case
    return B.solve_projection(c.vol, c.proj, d.f0, d.mean, d.U, to_dev(y, d.dt), np.zeros(c.K), opts)


def _oracle_problem(c, y, fit=True):
    return O.Problem(c.vol, c.proj, c.f0, c.mean, c.U, y, fit_intensity=fit)


_MINIMISERS = {}


def _minimiser(c, y, fit=True):
    """oracle.minimise from w0 = 0, once per (case, fit) in this module."""
    key = (c.name, fit, y.tobytes()[:64], float(y.sum()))
    if key not in _MINIMISERS:
        _MINIMISERS[key] = O.minimise(_oracle_problem(c, y, fit), np.zeros(c.K))
    return _MINIMISERS[key]


@pytest.mark.parametrize("grad_mode", [1, 2])
def test_tiny_cg_matches_oracle(torch, grad_mode):
    """64^3 FP64, 128x128 detector, 1% noise, CG from w0 = 0 (the tiny
    workload), by the back-projection route and by the fused evaluation."""
    c = synth.tiny()
    d = Dev(c)
    y = measured(c)
    say("tiny CG solve, grad_mode", grad_mode)
    opts = B.default_opts(locate=1, c0_mm=tuple(c.tumour_c0), grad_mode=grad_mode)
    w, rep = _gpu_solve(d, y, opts)
    w_o, info = _minimiser(c, y)
    say("gpu", w, rep)
    say("oracle", w_o, info["J"], info["newton_steps"])
    # a stationary point: the gradient test, or a stop where FP64 values of J
    # no longer resolve a decrease, then the polish step
    assert rep["status"] in ("converged", "line_search")
    assert rep["gnorm"] <= 1e-6 * rep["gnorm0"]
    assert np.linalg.norm(w - w_o) <= 1e-4 * np.linalg.norm(w_o)
    assert abs(rep["J"] - info["J"]) <= 1e-8 * info["J"]
    loc_o, _ = O.locate(c.vol, c.mean, c.U, w_o, c.tumour_c0)
    assert np.linalg.norm(np.array(rep["tumour_mm"]) - loc_o) <= 0.05
    assert rep["locate_iters"] > 0


def test_tiny_paper_mode_matches_oracle(torch):
    """The Appendix algorithm (10 iterations, Armijo on the normalised
    gradient) in FP64: same accepted steps as the oracle."""
    c = synth.tiny()
    d = Dev(c)
    y = measured(c)
    say("tiny paper-mode solve")
    w, rep = _gpu_solve(d, y, B.paper_opts())
    w_o, rep_o = O.solve_paper(_oracle_problem(c, y), np.zeros(c.K))
    say("gpu", w, rep)
    say("oracle", w_o, rep_o.iters, rep_o.J)
    assert rep["iters"] == rep_o.iters
    assert np.linalg.norm(w - w_o) <= 1e-8 * np.linalg.norm(w_o)
    assert abs(rep["J"] - rep_o.J) <= 1e-9 * rep_o.J


@pytest.mark.parametrize("method", [1, 2])
def test_recovery32_noise_free(torch, method):
    """Noise-free 32^3 FP64: the GPU solve recovers the planted w."""
    c = synth.recovery32()
    d = Dev(c)
    y = measured(c)
    say("recovery32 solve method", method)
    w, rep = _gpu_solve(d, y, B.default_opts(method=method))
    say("gpu", w, rep)
    assert np.linalg.norm(w - c.w_star) <= 1e-8 * np.linalg.norm(c.w_star)


def test_tiny_bfgs_matches_oracle(torch):
    """The tiny workload with the quasi-Newton solver: the oracle's minimiser,
    in fewer evaluations than CG."""
    c = synth.tiny()
    d = Dev(c)
    y = measured(c)
    say("tiny BFGS solve")
    w, rep = _gpu_solve(d, y, B.default_opts(method=2))
    w_o, info = _minimiser(c, y)
    _, rep_cg = _gpu_solve(d, y, B.default_opts())
    say("gpu", w, rep)
    say("oracle", w_o, info["J"])
    assert rep["status"] in ("converged", "line_search")
    assert rep["gnorm"] <= 1e-6 * rep["gnorm0"]
    assert np.linalg.norm(w - w_o) <= 1e-4 * np.linalg.norm(w_o)
    assert abs(rep["J"] - info["J"]) <= 1e-8 * info["J"]
    assert rep["n_fevals"] < rep_cg["n_fevals"]


@pytest.mark.parametrize("method,extrap", [(1, 10.0), (1, 0.0), (2, 10.0)])
def test_reported_point_is_consistent(torch, method, extrap):
    """The returned J, (a, b) and ||g|| are those of the returned w: the
    gradient of every accepted point was taken from the projection slot that
    holds that point (an extrapolated trial writes the second slot)."""
    c = synth.small(dtype="f64", seed=21)
    d = Dev(c)
    y = measured(c)
    say("consistency method", method, "extrap", extrap)
    w, rep = _gpu_solve(d, y, B.default_opts(method=method, ls_extrap=extrap, max_iter=6))
    J, a, b, g = B.objective_gradient(c.vol, c.proj, d.f0, d.mean, d.U, to_dev(y, d.dt), w)
    say("gpu", rep, "J", J, "g", g)
    assert rep["J"] == J and rep["a"] == a and rep["b"] == b
    assert abs(rep["gnorm"] - np.linalg.norm(g)) <= 1e-13 * np.linalg.norm(g)


@pytest.mark.parametrize("method", [1, 2])
def test_polish_reported_point_is_consistent(torch, method):
    """FP32 with the polish step (which evaluates into the second projection
    slot): the returned J, (a, b) and ||g|| are those of the returned w.  An
    FP32 objective is summed from moments about a reference fit (the last
    fit found in a solve, (1, 0) in a single evaluation), so the two agree to
    rounding rather than bit for bit."""
    c = synth.small(dtype="f32", seed=6)
    d = Dev(c)
    y = measured(c)
    say("polish consistency method", method)
    w, rep = _gpu_solve(d, y, B.default_opts(method=method, polish=1, xtol=1e-7))
    J, a, b, g = B.objective_gradient(c.vol, c.proj, d.f0, d.mean, d.U, to_dev(y, d.dt), w)
    say("gpu", rep, "J", J, "g", g)
    assert abs(rep["J"] - J) <= 1e-12 * J
    assert abs(rep["a"] - a) <= 1e-13 * abs(a) and abs(rep["b"] - b) <= 1e-13 * max(1.0, abs(b))
    assert abs(rep["gnorm"] - np.linalg.norm(g)) <= 1e-12 * np.linalg.norm(g)


@pytest.mark.parametrize("grad_mode", [1, 2])
@pytest.mark.parametrize("method", [1, 2])
@pytest.mark.parametrize("fit", [True, False])
def test_small_f32_solve_matches_oracle(torch, fit, method, grad_mode):
    """Ragged anisotropic FP32 case with the default options (the polish step
    on): converged w within 1e-4 of the FP64 oracle's minimiser.
    (Comparisons of FP32 values of J stop at J's rounding noise, about 3e-7 J
    on this 1920-pixel detector; the polish step goes on from there with the
    gradient.)"""
    c = synth.small(dtype="f32", seed=6)
    d = Dev(c)
    y = measured(c)
    say("small f32 solve fit=", fit, "method", method, "grad_mode", grad_mode)
    opts = B.default_opts(fit_intensity=int(fit), xtol=1e-7, method=method, grad_mode=grad_mode)
    assert opts.polish == 1
    w, rep = _gpu_solve(d, y, opts)
    w_o, info = _minimiser(c, y, fit)
    say("gpu", w, rep)
    say("oracle", w_o, info["J"])
    assert np.linalg.norm(w - w_o) <= 1e-4 * np.linalg.norm(w_o)


@pytest.mark.parametrize("method", [1, 2])
@pytest.mark.parametrize("fit", [True, False])
def test_small_f32_default_stops_at_noise_band(torch, fit, method):
    """With the polish step off an FP32 solve ends where FP32 values of J can
    no longer show a decrease: the FP64 objective at the returned w exceeds
    its minimum by no more than twice the band 6 u sqrt(sum p^2 / (M J)) J
    (u = 2^-24), at any size, and the solve says it converged."""
    c = synth.small(dtype="f32", seed=6)
    d = Dev(c)
    y = measured(c)
    say("small f32 default solve fit=", fit, "method", method)
    opts = B.default_opts(fit_intensity=int(fit), xtol=1e-7, method=method, polish=0)
    w, rep = _gpu_solve(d, y, opts)
    prob = _oracle_problem(c, y, fit)
    w_o, info = _minimiser(c, y, fit)
    J64, a, b, r = prob.objective(w)
    p = r + a * y + b
    band = 6.0 * 2.0 ** -24 * np.sqrt(float(np.sum(p * p)) / (p.size * J64))
    say("gpu", w, rep["status"], "excess", (J64 - info["J"]) / info["J"], "band", band)
    assert rep["status"] == "converged"
    assert J64 - info["J"] <= 2.0 * band * info["J"]
    assert np.linalg.norm(w - w_o) <= 1e-3 * np.linalg.norm(w_o)


def test_k1_solve(torch):
    """K = 1 (the physical-phantom setting of the paper)."""
    c = synth.small(dtype="f64", seed=16, K=1)
    d = Dev(c)
    y = measured(c)
    say("K=1 solve")
    w, rep = _gpu_solve(d, y, B.default_opts())
    w_o, _ = _minimiser(c, y)
    assert abs(w[0] - w_o[0]) <= 1e-4 * max(abs(w_o[0]), 1.0)


def test_solve_errors_from_data(torch):
    c = synth.small(dtype="f64", seed=5)
    d = Dev(c)
    say("solve error paths")
    y_const = np.full((c.proj.nv, c.proj.nu), 3.0)
    with pytest.raises(B.PcasError) as e:
        _gpu_solve(d, y_const, B.default_opts())
    assert e.value.code == -3
    y_nan = measured(c)
    y_nan[3, 4] = np.nan
    with pytest.raises(B.PcasError) as e:
        _gpu_solve(d, y_nan, B.default_opts())
    assert e.value.code == -4
    # zero iterations: returns w0 and J0
    w, rep = _gpu_solve(d, measured(c), B.default_opts(max_iter=0))
    assert np.all(w == 0) and rep["iters"] == 0 and rep["status"] == "max_iter"


@pytest.mark.parametrize("case", ["tiny", "small32"])
def test_preconditioned_cg_matches_oracle(torch, case):
    """CG preconditioned by the fused evaluation's Gauss-Newton matrix
    (opts.precond): the oracle's minimiser within 1e-4 (FP64 tiny: 1e-6),
    in fewer evaluations than plain CG."""
    c = synth.tiny() if case == "tiny" else synth.small(dtype="f32", seed=6)
    d = Dev(c)
    y = measured(c)
    xtol = 1e-10 if c.dtype == "f64" else 1e-7
    say("preconditioned CG", case)
    w, rep = _gpu_solve(d, y, B.default_opts(grad_mode=2, precond=1, xtol=xtol))
    w1, rep1 = _gpu_solve(d, y, B.default_opts(grad_mode=2, xtol=xtol))
    w_o, info = _minimiser(c, y)
    err = np.linalg.norm(w - w_o) / np.linalg.norm(w_o)
    say("gpu", w, rep["n_fevals"], "plain CG", rep1["n_fevals"], "err", err)
    assert rep["status"] in ("converged", "line_search")
    assert err <= (1e-6 if c.dtype == "f64" else 1e-4)
    assert rep["n_fevals"] < rep1["n_fevals"]


def test_precond_option_is_checked(torch):
    c = synth.small(dtype="f32", seed=6)
    d = Dev(c)
    y = measured(c)
    for kw in (dict(precond=1), dict(precond=1, grad_mode=2, method=2), dict(precond=2, grad_mode=2)):
        with pytest.raises(B.PcasError):
            _gpu_solve(d, y, B.default_opts(**kw))


def test_solves_on_short_lived_threads(torch):
    """Each host thread keeps its own read-back mailbox and timing events and
    gives them back when it exits: solves on a run of threads that start and
    end one after another, with every kernel class timed, return what the
    same solve returns on this thread, bit for bit."""
    import threading
    c = synth.small(dtype="f32", seed=6)
    d = Dev(c)
    y = measured(c)
    opts = B.default_opts(grad_mode=2, precond=1, xtol=1e-7, profile=B.PROFILE_ALL)
    w0, rep0 = _gpu_solve(d, y, opts)
    out = []
    for i in range(6):
        say("solve on thread", i)
        t = threading.Thread(target=lambda: out.append(_gpu_solve(d, y, opts)))
        t.start()
        t.join()
    assert len(out) == 6
    for w, rep in out:
        assert np.array_equal(w, w0)
        assert rep["n_fevals"] == rep0["n_fevals"] and rep["J"] == rep0["J"]
        assert sum(rep["kernel_launches"].values()) > 0
