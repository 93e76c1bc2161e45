"""Speculative gradients (opts.speculate): a solve that starts the gradient
behind each evaluation, gated on the GPU by its own acceptance rule, must
return exactly what the same solve without speculation returns -- the same
w, J, fit, gradient norm and step counts, bit for bit -- and must actually
take most of its gradients from speculative launches."""
import numpy as np
import pytest

from paper_1102_1712_amd import binding as B
from paper_1102_1712_amd import synth

from gpu_common import Dev, measured, say, to_dev, torch_or_skip

pytestmark = pytest.mark.gpu

_KEYS = ("status", "iters", "n_fevals", "n_grads", "J0", "J", "a", "b", "gnorm0", "gnorm")


@pytest.fixture(scope="module")
def small32():
    torch_or_skip()
    c = synth.small(dtype="f32", seed=6)
    return c, Dev(c), measured(c)


def _solve(c, d, y, **kw):
    return B.solve_projection(c.vol, c.proj, d.f0, d.mean, d.U, to_dev(y, d.dt), np.zeros(c.K),
                              B.default_opts(**kw))


def _same(a, b):
    (w0, r0), (w1, r1) = a, b
    assert np.array_equal(w0, w1), (w0, w1)
    for k in _KEYS:
        assert r0[k] == r1[k], (k, r0[k], r1[k])


@pytest.mark.parametrize("method,extrap,polish,fit", [
    (1, 10.0, 1, 1), (1, 0.0, 1, 1), (1, 10.0, 0, 1), (1, 10.0, 1, 0),
    (2, 10.0, 1, 1), (2, 0.0, 0, 1), (2, 10.0, 1, 0)])
def test_speculation_changes_nothing(small32, method, extrap, polish, fit):
    c, d, y = small32
    kw = dict(method=method, ls_extrap=extrap, polish=polish, fit_intensity=fit, xtol=1e-7)
    say("speculation on/off, small f32", kw)
    off = _solve(c, d, y, speculate=0, **kw)
    on = _solve(c, d, y, speculate=1, **kw)
    say("off", off[1]["n_fevals"], off[1]["n_grads"], "on spec_grads", on[1]["spec_grads"])
    _same(off, on)
    assert off[1]["spec_grads"] == 0
    n = on[1]["n_grads"]
    # every gradient but those after an extrapolated trial that was not kept
    # comes from a speculative launch
    assert 0 < on[1]["spec_grads"] <= n
    assert on[1]["spec_grads"] >= n - 2


def test_speculation_with_profiling(small32):
    """Timing every class leaves the result alone; the adjoint class counts
    the launches that did the work, the skipped class those whose gate was
    shut (rejected or extrapolated trials)."""
    c, d, y = small32
    say("speculation with profiling")
    base = _solve(c, d, y, speculate=1, xtol=1e-7)
    w, rep = _solve(c, d, y, speculate=1, xtol=1e-7, profile=B.PROFILE_ALL)
    _same(base, (w, rep))
    L = rep["kernel_launches"]
    say("launches", L, "spec_grads", rep["spec_grads"])
    assert L["drr_adjoint_chain"] >= rep["n_grads"]
    assert L["drr_adjoint_chain"] + L["spec_skipped"] >= rep["spec_grads"]
    # a skipped launch exits at once
    if L["spec_skipped"]:
        skip = rep["kernel_ms"]["spec_skipped"] / L["spec_skipped"]
        full = rep["kernel_ms"]["drr_adjoint_chain"] / L["drr_adjoint_chain"]
        assert skip < 0.5 * full


def test_f64_speculates_and_jacobian_mode_does_not():
    """FP64 evaluations gate on J, a, b of the two-pass residual: the same
    results with and without speculation.  The projected-Jacobian gradient
    (grad_mode 0) never speculates."""
    torch_or_skip()
    c = synth.small(dtype="f64", seed=21)
    d = Dev(c)
    y = measured(c)
    for method in (1, 2):
        say("f64 solve with and without speculation, method", method)
        off = _solve(c, d, y, speculate=0, max_iter=6, method=method)
        on = _solve(c, d, y, speculate=1, max_iter=6, method=method)
        _same(off, on)
        assert off[1]["spec_grads"] == 0
        assert on[1]["n_grads"] - 2 <= on[1]["spec_grads"] <= on[1]["n_grads"]
    c32 = synth.small(dtype="f32", seed=6)
    d32 = Dev(c32)
    y32 = measured(c32)
    say("grad_mode 0 with speculate=1")
    w, rep = _solve(c32, d32, y32, speculate=1, grad_mode=0, xtol=1e-7)
    assert rep["spec_grads"] == 0


def test_speculate_option_is_checked(small32):
    c, d, y = small32
    with pytest.raises(B.PcasError):
        _solve(c, d, y, speculate=2)
