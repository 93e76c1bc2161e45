"""Host logic of the streaming solve (no GPU): Eq. 3 prediction pinned to
the paper's fitted coefficients, and the least-squares predictor fit."""
import json
import os

import numpy as np
import pytest

from paper_1102_1712_amd import stream as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def test_predict_eq4_coefficients():
    """Eq. 4: with c_1 = (1.90, -0.98), a history w(t-1) = 1, w(t-2) = 0
    predicts 1.90 for the first coefficient, and (0, 1) predicts -0.98."""
    g = json.load(open(GOLDEN))
    c = np.array(g["eq4_digital_c"])
    assert np.allclose(S.predict(np.array([[0.0] * 3, [1.0] * 3]), c), [1.90, 1.51, 0.97])
    assert np.allclose(S.predict(np.array([[1.0] * 3, [0.0] * 3]), c), [-0.98, -0.84, -0.84])
    c5 = np.array(g["eq5_physical_c"])
    assert np.allclose(S.predict(np.array([[2.0], [3.0]]), c5), [1.96 * 3.0 - 0.99 * 2.0])


def test_fit_recovers_ar2_coefficients():
    """A noise-free AR(2) sequence per coefficient is reproduced exactly."""
    true = np.array([[1.90, -0.98], [1.51, -0.84]])
    T = 60
    w = np.zeros((T, 2))
    w[0], w[1] = [0.3, -0.2], [0.5, 0.1]
    for t in range(2, T):
        w[t] = true[:, 0] * w[t - 1] + true[:, 1] * w[t - 2]
    c = S.fit_predictor(w, L=2)
    np.testing.assert_allclose(c, true, rtol=1e-9, atol=1e-9)


def test_sinusoid_prediction_is_exact():
    """A sampled sinusoid obeys w(t) = 2 cos(omega) w(t-1) - w(t-2): the
    fitted predictor finds (2 cos(omega), -1)."""
    om = 2 * np.pi / 60.0
    t = np.arange(120)
    w = np.sin(om * t)[:, None]
    c = S.fit_predictor(w, L=2)
    np.testing.assert_allclose(c[0], [2 * np.cos(om), -1.0], atol=1e-10)


def test_breathing_trace_properties():
    s = S.breathing_trace(600, 15.0, seed=3)
    assert s.shape == (600,)
    assert s.min() >= 0.0
    # amplitude 5-20 mm plus a 2 mm/min drift over 40 s
    assert 4.0 < s.max() < 22.0
    w = S.planted_trajectory(s, 3, seed=4, scale=0.1)
    assert w.shape == (600, 3) and np.all(np.isfinite(w))


def test_localisation_errors():
    a = np.zeros((4, 3))
    b = np.array([[1.0, 0, 0], [0, 2.0, 0], [0, 0, 0], [3.0, 4.0, 0]])
    e = S.localisation_errors(a, b)
    assert np.isclose(e["e_mean_mm"], (1 + 2 + 0 + 5) / 4)
    assert np.isclose(e["e_max_mm"], 5.0)


def test_predictor_error_paths():
    """The library's Eq. 3 entry points refuse what they cannot do: a
    history shorter than L, a constant training sequence (the lagged values
    are linearly dependent for L = 2) and non-finite values."""
    from paper_1102_1712_amd import binding as B
    c = np.array([[1.9, -0.98]])
    with pytest.raises(B.PcasError) as e:
        S.predict(np.array([[1.0]]), c)
    assert e.value.code == -1
    with pytest.raises(B.PcasError) as e:
        S.fit_predictor(np.full((20, 1), 3.0), L=2)
    assert e.value.code == -3
    with pytest.raises(B.PcasError) as e:
        S.predict(np.array([[1.0], [np.nan]]), c)
    assert e.value.code == -4
