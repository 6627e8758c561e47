"""The sub-threshold LER fit p^(d_circ/2) exp(c0 + c1 p + c2 p^2) (Sec. 6.1).

Pins: exact recovery of known coefficients from points on the curve; the same
optimum as a general nonlinear least-squares solver (scipy's curve_fit on the
log model, a different algorithm); points without failures are dropped; too
few points is an error.
"""
import numpy as np
import pytest
from scipy.optimize import curve_fit

from paper_2607_27644_amd import stats


def test_exact_recovery():
    p = np.array([2e-3, 4e-3, 6e-3, 8e-3, 1e-2])
    for c, d in [((2.0, -300.0, 1e4), 8), ((11.6, -662.0, 39590.0), 10), ((-1.0, 50.0, 0.0), 14)]:
        y = stats.ler_model(p, c, d)
        got = stats.fit_ler(p, y, d, failures=[5, 10, 20, 40, 80])
        np.testing.assert_allclose(got, c, rtol=1e-7, atol=1e-6)


def test_matches_nonlinear_least_squares():
    rng = np.random.default_rng(3)
    p = np.linspace(3e-3, 1.2e-2, 7)
    c_true, d = (4.0, -200.0, 8000.0), 10
    y = stats.ler_model(p, c_true, d) * np.exp(rng.normal(0.0, 0.2, p.size))
    f = rng.integers(5, 200, p.size).astype(np.float64)
    c = stats.fit_ler(p, y, d, failures=f)

    def logmodel(pp, c0, c1, c2):
        return 0.5 * d * np.log(pp) + c0 + c1 * pp + c2 * pp * pp

    ref, _ = curve_fit(logmodel, p, np.log(y), p0=(0.0, 0.0, 0.0), sigma=1.0 / np.sqrt(f), absolute_sigma=False)
    np.testing.assert_allclose(c, ref, rtol=1e-5, atol=1e-4)
    # the weighted fit is not the unweighted one when the counts differ
    cu = stats.fit_ler(p, y, d)
    assert not np.allclose(c, cu)


def test_zero_failure_points_dropped_and_minimum():
    p = np.array([1e-3, 2e-3, 4e-3, 6e-3, 8e-3])
    c, d = (3.0, -100.0, 5000.0), 8
    y = stats.ler_model(p, c, d)
    y[0] = 0.0
    np.testing.assert_allclose(stats.fit_ler(p, y, d), c, rtol=1e-7, atol=1e-6)
    with pytest.raises(ValueError):
        stats.fit_ler(p[:3], np.array([0.0, 1e-6, 2e-6]), d)
    with pytest.raises(ValueError):
        stats.fit_ler(p, y, d, failures=[0, 0, 0, 1, 1])
