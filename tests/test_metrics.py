"""Host-side norms and time-to-error interpolation."""
import numpy as np
import pytest

from paper_2406_15632_amd import metrics as M


def test_norms():
    A = np.array([[1.0, 2.0], [3.0, 4.0]])
    B = np.array([[1.0, 2.0], [3.0, 2.0]])
    assert M.image_norm(A, B) == pytest.approx(2.0 / ((2 + 4 + 6 + 6) / 2))
    assert M.integral_norm(A, B) == pytest.approx((10 - 8) / 8)
    assert M.rms_error(A, B) == pytest.approx(2.0 / np.sqrt(1 + 4 + 9 + 4))
    assert M.rms_error(B, B) == 0.0


def test_time_to_error_power_law():
    # e = a t^-0.5 exactly: interpolation in log-log space is exact
    t = np.array([1.0, 4.0, 16.0, 64.0])
    e = 0.1 * t ** -0.5
    assert M.time_to_error(t, e, 0.025) == pytest.approx(16.0)
    assert M.time_to_error(t, e, 0.03) == pytest.approx((0.1 / 0.03) ** 2)
    assert M.time_to_error(t, e, 1e-6) is None
    assert M.time_to_error(t, e, 1.0) == 1.0


def test_central_mask():
    m = M.central_mask(8, 1.0, 0.3)
    assert not m[3, 3] and not m[4, 4] and m[0, 0]
    assert m.sum() == 64 - 4


def test_power_fit_recovers_exact_power_laws():
    t = np.array([1e-3, 4e-3, 2e-2, 0.1, 0.7])
    a, b = M.power_fit(t, 0.3 * t ** -0.7)
    assert a == pytest.approx(0.3, rel=1e-12) and b == pytest.approx(0.7, rel=1e-12)
    a, b = M.power_fit(t, 2.0 * t ** -0.5, b=0.5)
    assert a == pytest.approx(2.0, rel=1e-12) and b == 0.5
    # with b fixed, a is the geometric mean of e t^b
    e = np.array([1.0, 3.0, 2.0, 0.5, 0.1])
    a, _ = M.power_fit(t, e, b=0.5)
    assert a == pytest.approx(float(np.exp(np.mean(np.log(e * t ** 0.5)))), rel=1e-12)
    assert M.power_fit([1.0], [0.1]) is None
    assert M.power_fit([1.0, 2.0], [0.0, -1.0]) is None

