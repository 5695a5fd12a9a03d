"""Pins of the oracle's Iter-AUC and Time-AUC (Sec. 3, "Evaluation metrics")."""
import numpy as np
import pytest

import oracle as O


def test_geometric_history_closed_forms():
    # r_i = 10^-i, rtol = 1e-8, 10 iterations: sum_{i=0}^{10} (8 - i) = 88 - 55
    r = 10.0 ** -np.arange(11)
    assert O.iter_auc(r, 1e-8) == pytest.approx(33.0, abs=1e-12)
    # uniform steps of 0.5 s: 0.5 * sum_{i=1}^{10} (8 - i) = 0.5 * (80 - 55)
    t = 0.5 * np.arange(11)
    assert O.time_auc(r, t, 1e-8) == pytest.approx(12.5, abs=1e-12)


def test_history_at_rtol_is_zero_and_rtol_shift():
    r = np.full(7, 1e-6)
    assert O.iter_auc(r, 1e-6) == pytest.approx(0.0, abs=1e-13)
    h = np.array([1.0, 0.3, 0.02, 4e-4, 5e-7])
    # changing rtol by a factor 10 moves every one of the iters + 1 terms by 1
    assert O.iter_auc(h, 1e-9) - O.iter_auc(h, 1e-8) == pytest.approx(len(h), abs=1e-12)
    t = np.array([0.0, 0.1, 0.3, 0.35, 1.0])
    assert O.time_auc(h, t, 1e-9) - O.time_auc(h, t, 1e-8) == pytest.approx(1.0, abs=1e-12)


def test_time_auc_is_a_right_endpoint_sum():
    """Piecewise-constant r(t) equal to r_i on (t_{i-1}, t_i]: the integral of Sec. 3 exactly."""
    h = np.array([1.0, 0.1, 0.05, 1e-3])
    t = np.array([0.0, 2.0, 2.5, 4.0])
    integrand = lambda s: np.log10(h[np.searchsorted(t, s)]) + 8.0  # noqa: E731
    grid = np.linspace(0.0, 4.0, 400001)[1:]
    approx = np.sum(integrand(grid)) * (grid[1] - grid[0])
    assert O.time_auc(h, t, 1e-8) == pytest.approx(approx, rel=1e-4)
    # t_0 does not enter except through t_1 - t_0
    assert O.time_auc(h, t + 3.0, 1e-8) == pytest.approx(O.time_auc(h, t, 1e-8), abs=1e-12)


def test_zero_residual_and_single_entry():
    tiny = np.finfo(np.float64).tiny
    assert O.iter_auc([1.0, 0.0], 1e-8) == pytest.approx(8.0 + np.log10(tiny) + 8.0)
    assert O.iter_auc([0.01], 1e-8) == pytest.approx(6.0)
    assert O.time_auc([0.01], [0.0], 1e-8) == 0.0
