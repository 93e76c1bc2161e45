"""Solve parity at the benchmark's full size: the clinical workload
(256x256x128 FP32, K = 3, 512x384 detector, 1% noise) solved through the C
ABI, in the configuration bench.py times, against the FP64 oracle's
minimiser stored by tests/golden/make_clinical_minimiser.py (re-checked on
the CPU by test_clinical_golden_is_stationary).  Bars: w within 1e-4
relative, tumour position within 0.05 mm."""
import json
import os

import numpy as np
import pytest

from paper_1102_1712_amd import binding as B
from paper_1102_1712_amd import synth

from gpu_common import Dev, measured, say, to_dev, torch_or_skip

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "clinical_minimiser.json")


@pytest.fixture(scope="module")
def clinical():
    torch_or_skip()
    say("building the clinical workload")
    c = synth.clinical()
    d = Dev(c)
    y = to_dev(measured(c), d.dt)
    return c, d, y, json.load(open(GOLDEN))


def _solve(c, d, y, fit, method, polish=None, grad_mode=None):
    """The benchmark's options (the library defaults, xtol 1e-7, localisation
    on), with the method, fit and, when given, the polish step and the
    gradient route overridden."""
    kw = dict(xtol=1e-7, method=method, fit_intensity=int(fit), locate=1,
              c0_mm=tuple(c.tumour_c0))
    if grad_mode is not None:
        kw["grad_mode"] = grad_mode
    if polish is not None:
        kw["polish"] = polish
    opts = B.default_opts(**kw)
    return B.solve_projection(c.vol, c.proj, d.f0, d.mean, d.U, y, np.zeros(c.K), opts)


@pytest.mark.parametrize("grad_mode", [1, 2])
@pytest.mark.parametrize("method", [1, 2])
@pytest.mark.parametrize("fit", [True, False])
def test_clinical_timed_solve_matches_oracle_minimiser(clinical, fit, method, grad_mode):
    """The configuration bench.py times (default options, which include the
    polish step), by the back-projection route and by the fused evaluation:
    w within 1e-4 of the FP64 minimiser, tumour position within 0.05 mm."""
    c, d, y, gold = clinical
    ref = gold["fit" if fit else "nofit"]
    assert gold["workload"] == c.name and gold["angle"] == c.proj.angle
    say("clinical default solve fit", fit, "method", method, "grad_mode", grad_mode)
    w, rep = _solve(c, d, y, fit, method, grad_mode=grad_mode)
    w_ref = np.array(ref["w"])
    err = np.linalg.norm(w - w_ref) / np.linalg.norm(w_ref)
    say("gpu", w, rep["status"], rep["n_fevals"], rep["n_grads"], "err", err)
    assert rep["status"] == "converged"
    assert err <= 1e-4
    assert np.linalg.norm(np.array(rep["tumour_mm"]) - np.array(ref["tumour_mm"])) <= 0.05


@pytest.mark.parametrize("method", [1, 2])
@pytest.mark.parametrize("fit", [True, False])
def test_clinical_unpolished_solve_stops_at_band(clinical, oracle_lib, fit, method):
    """With the polish step off: the solve ends converged where
    FP32 values of J no longer resolve a decrease: the FP64 objective at the
    returned w exceeds the oracle's minimum by at most twice the noise band
    6 u sqrt(sum p^2 / (M J)) J (u = 2^-24); tumour within 0.05 mm."""
    import oracle as O
    c, d, y, gold = clinical
    ref = gold["fit" if fit else "nofit"]
    say("clinical unpolished solve fit", fit, "method", method)
    w, rep = _solve(c, d, y, fit, method, 0)
    prob = O.Problem(c.vol, c.proj, c.f0, c.mean, c.U, measured(c), fit_intensity=fit)
    J64, a, b, r = prob.objective(w)
    p = r + a * prob.y + b
    band = 6.0 * 2.0 ** -24 * np.sqrt(float(np.sum(p * p)) / (p.size * J64))
    say("gpu", w, rep["status"], "excess", (J64 - ref["J"]) / ref["J"], "band", band)
    assert rep["status"] == "converged"
    assert J64 - ref["J"] <= 2.0 * band * ref["J"]
    assert np.linalg.norm(np.array(rep["tumour_mm"]) - np.array(ref["tumour_mm"])) <= 0.05


@pytest.mark.parametrize("method", [1, 2])
def test_clinical_speculation_is_bit_identical(clinical, method):
    """The timed configuration with and without speculative gradients:
    identical results, and all but at most two gradients from speculative
    launches."""
    c, d, y, _ = clinical
    say("clinical speculation on/off, method", method)
    kw = dict(xtol=1e-7, method=method, locate=1, c0_mm=tuple(c.tumour_c0), grad_mode=1)
    w0, r0 = B.solve_projection(c.vol, c.proj, d.f0, d.mean, d.U, y, np.zeros(c.K),
                                B.default_opts(speculate=0, **kw))
    w1, r1 = B.solve_projection(c.vol, c.proj, d.f0, d.mean, d.U, y, np.zeros(c.K),
                                B.default_opts(**kw))
    say("n_grads", r1["n_grads"], "spec_grads", r1["spec_grads"])
    assert np.array_equal(w0, w1)
    for k in ("status", "iters", "n_fevals", "n_grads", "J", "a", "b", "gnorm", "tumour_mm"):
        assert r0[k] == r1[k], k
    assert r0["spec_grads"] == 0 and r1["spec_grads"] >= r1["n_grads"] - 2


@pytest.mark.parametrize("fit", [True, False])
def test_clinical_preconditioned_cg_matches_oracle_minimiser(clinical, fit):
    """CG preconditioned by the Gauss-Newton matrix (grad_mode 2, precond 1)
    at the benchmark's options: w within 1e-4 of the FP64 minimiser, tumour
    within 0.05 mm."""
    c, d, y, gold = clinical
    ref = gold["fit" if fit else "nofit"]
    kw = dict(xtol=1e-7, method=1, fit_intensity=int(fit), locate=1, c0_mm=tuple(c.tumour_c0),
              grad_mode=2, precond=1)
    w, rep = B.solve_projection(c.vol, c.proj, d.f0, d.mean, d.U, y, np.zeros(c.K),
                                B.default_opts(**kw))
    w_ref = np.array(ref["w"])
    err = np.linalg.norm(w - w_ref) / np.linalg.norm(w_ref)
    say("clinical preconditioned CG fit", fit, w, rep["status"], rep["n_fevals"], "err", err)
    assert rep["status"] == "converged"
    assert err <= 1e-4
    assert np.linalg.norm(np.array(rep["tumour_mm"]) - np.array(ref["tumour_mm"])) <= 0.05
