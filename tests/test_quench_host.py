"""Host logic of the quench driver: the caloric-curve slope estimator."""
from math import erf

import numpy as np
import pytest

from paper_1105_5613_amd.quench import caloric_slope


def test_slope_of_a_line_is_constant():
    T = np.linspace(0.3, 2.0, 40)
    tc, sl, _, smax, scold = caloric_slope(T, 3.0 + 1.5 * T, window=7)
    assert np.allclose(sl, 1.5) and smax == pytest.approx(1.5) and scold == pytest.approx(1.5)
    assert len(tc) == len(T) - 6 and np.all(np.diff(tc) > 0)


def test_peak_of_the_slope_is_found_from_unsorted_samples():
    # U = T + integral of exp(-(t - 0.6)^2 / w): dU/dT = 1 + exp(-(T - 0.6)^2 / w), peak at 0.6
    w = 0.02
    T = np.random.default_rng(1).permutation(np.linspace(0.3, 2.0, 200))
    U = T + np.sqrt(np.pi * w) / 2 * np.array([erf((t - 0.6) / np.sqrt(w)) for t in T])
    _, _, tg, smax, scold = caloric_slope(T, U, window=5)
    assert tg == pytest.approx(0.6, abs=0.02)
    assert smax == pytest.approx(2.0, rel=0.02)
    assert scold < smax


def test_needs_points():
    with pytest.raises(ValueError):
        caloric_slope([1.0, 2.0, 3.0], [1.0, 2.0, 3.0])
