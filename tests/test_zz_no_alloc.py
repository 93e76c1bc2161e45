"""grad_w_noalloc (the entry point for callers that cannot allocate)
against grad_w, through the C ABI: two calls in a row on the same GPU, the
second on a smaller volume (the static scratch keeps the first call's
partials and counter), each bit for bit equal to grad_w's result, in FP64
and FP32."""
import numpy as np
import pytest

from paper_1102_1712_amd import binding as B
from paper_1102_1712_amd import synth

from gpu_common import Dev, say, to_dev, torch_or_skip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_or_skip()


def _case_pair(dtype):
    big = synth.small(dtype=dtype, seed=5)
    little = synth.small(n=(20, 18, 14), spacing=(9.0, 10.0, 12.0), det=(24, 20),
                         pitch=(14.0, 16.0), step=4.5, dtype=dtype, seed=8)
    return big, little


def test_scratch_size_is_modest(torch):
    n = B.lib().grad_w_noalloc_scratch_bytes()
    assert 0 < n <= 256 * 1024


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_grad_w_twice(torch, dtype):
    rng = np.random.default_rng(31)
    for case in _case_pair(dtype):
        d = Dev(case)
        w = case.w_star * 0.7
        bp = to_dev(rng.normal(size=case.vol.shape_zyx), d.dt)
        say("grad_w_noalloc", dtype, case.vol.n)
        ref = B.grad_w(case.vol, d.f0, d.mean, d.U, w, bp)
        out = torch.full((case.K,), np.nan, dtype=torch.float64, device="cuda")
        B.grad_w_noalloc(case.vol, d.f0, d.mean, d.U, w, bp, out)
        torch.cuda.synchronize()
        say("ref", ref.cpu().numpy(), "noalloc", out.cpu().numpy())
        assert torch.equal(out, ref)


def test_noalloc_rejects_bad_arguments(torch):
    case = synth.small(dtype="f64", seed=5)
    d = Dev(case)
    out = torch.empty(case.K, dtype=torch.float64, device="cuda")
    bp = torch.zeros(case.vol.shape_zyx, dtype=torch.float64, device="cuda")
    with pytest.raises(B.PcasError) as e:
        B.grad_w_noalloc(case.vol, d.f0, d.mean, d.U, np.full(case.K, np.nan), bp, out)
    assert e.value.code == -4
