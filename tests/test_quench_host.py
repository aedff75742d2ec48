"""Host logic of the quench driver: the caloric-curve breakpoint fit."""
import numpy as np
import pytest

from paper_1105_5613_amd.quench import caloric_break


def test_break_of_exact_two_line_curve():
    T = np.linspace(0.3, 2.0, 35)
    U = np.where(T < 0.62, -7.0 + 1.5 * (T - 0.62), -7.0 + 3.2 * (T - 0.62))
    tb, lo, hi = caloric_break(T, U)
    assert tb == pytest.approx(0.62, abs=0.004)
    assert lo == pytest.approx(1.5, rel=1e-2) and hi == pytest.approx(3.2, rel=1e-2)


def test_break_with_noise_and_unsorted_input():
    rng = np.random.default_rng(3)
    T = rng.permutation(np.linspace(0.3, 2.0, 60))
    U = np.where(T < 1.1, 2.0 * (T - 1.1), 4.0 * (T - 1.1)) + rng.normal(0, 0.002, T.size)
    tb, lo, hi = caloric_break(T, U)
    assert abs(tb - 1.1) < 0.03
    assert lo < hi


def test_break_needs_points():
    with pytest.raises(ValueError):
        caloric_break([1.0, 2.0, 3.0], [1.0, 2.0, 3.0])
