"""Pins of the autocorrelation analysis (Sec. III.A, III.C) on series with
known answers: a four-point series worked by hand, an AR(1) process (C(dt) =
phi^dt exactly, so tau = -1/ln phi), the interpolation of the 1/e crossing,
and the order parameter of hand-made counts."""
import math

import numpy as np
import pytest

from paper_2505_05919_amd import autocorr


def test_four_point_series_by_hand():
    # M = 1, 2, 3, 4: <M> = 5/2, <M^2> = 15/2, variance 5/4;
    # lag 1: <M(t+1) M(t)> over (2, 6, 12) = 20/3, C = (20/3 - 25/4) / (5/4) = 1/3
    # lag 2: over (3, 8) = 11/2, C = (11/2 - 25/4) / (5/4) = -3/5
    C = autocorr.c_m([1.0, 2.0, 3.0, 4.0], 2)
    assert C[0] == pytest.approx(1.0, abs=1e-15)
    assert C[1] == pytest.approx(1.0 / 3.0, abs=1e-15)
    assert C[2] == pytest.approx(-0.6, abs=1e-15)


def test_ar1_closed_form():
    phi, T = 0.9, 400_000
    rng = np.random.default_rng(11)
    e = rng.standard_normal(T)
    x = np.empty(T)
    x[0] = e[0] / math.sqrt(1 - phi * phi)
    for t in range(1, T):
        x[t] = phi * x[t - 1] + e[t]
    x += 5.0                                          # C_M is shift invariant
    C = autocorr.c_m(x, 30)
    for dt in (1, 2, 5, 10):
        # standard error of an AR(1) autocorrelation estimate ~ sqrt((1+phi^2)/(1-phi^2)/T)
        assert abs(C[dt] - phi ** dt) < 5 * math.sqrt((1 + phi * phi) / (1 - phi * phi) / T), dt
    tau = autocorr.tau_1e(C)
    assert tau == pytest.approx(-1.0 / math.log(phi), rel=0.03)


def test_tau_interpolation():
    # a piecewise-linear C crossing 1/e between lags 3 and 4 at exactly 3.25
    t = math.exp(-1.0)
    c3 = t + 0.25 * 0.2
    C = [1.0, 0.8, 0.6, c3, c3 - 0.2, 0.1]
    assert autocorr.tau_1e(C) == pytest.approx(3.25, abs=1e-12)
    assert math.isnan(autocorr.tau_1e([1.0, 0.9, 0.8]))
    assert autocorr.tau_1e([1.0, t]) == pytest.approx(1.0, abs=1e-12)


def test_order_parameter_and_errors():
    counts = np.array([[10, 2, 3, 1, 0, 0], [4, 4, 4, 4, 0, 0]])
    assert np.allclose(autocorr.order_parameter(counts, 16), [10 / 16, 4 / 16])
    with pytest.raises(ValueError):
        autocorr.c_m([1.0, 1.0, 1.0], 1)
    with pytest.raises(ValueError):
        autocorr.c_m([1.0, 2.0], 2)


def test_nearly_constant_series_is_not_resolvable():
    """M(t) that only jitters at the last digits (as under cluster shifts of
    an ordered lattice, which permute the state counts) gives C_M(1) > 1,
    impossible for a stationary series: tau is then reported undefined."""
    import numpy as np
    from paper_2505_05919_amd import autocorr
    rng = np.random.default_rng(3)
    x = 0.99 + 1e-7 * rng.standard_normal(4000)
    x[0] = x[-1] = 0.99 + 3e-7                      # the end terms of the lagged mean dominate the variance
    C = autocorr.c_m(x, 10)
    assert not autocorr.resolvable(C)
    y = np.sin(np.arange(4000) / 50.0) + 0.1 * rng.standard_normal(4000)
    assert autocorr.resolvable(autocorr.c_m(y, 10))
