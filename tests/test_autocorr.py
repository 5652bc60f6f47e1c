"""Pins of the autocorrelation analysis (Sec. III.A, III.C) on series with
known answers: a four-point series worked by hand, an AR(1) process (C(dt) =
phi^dt exactly, so tau = -1/ln phi), the interpolation of the 1/e crossing,
and the order parameter of hand-made counts."""
import math

import numpy as np
import pytest

from paper_2505_05919_amd import autocorr


def test_four_point_series_by_hand():
    # M = 1, 2, 3, 4: <M> = 5/2, d = (-3/2, -1/2, 1/2, 3/2), <d^2> = 5/4;
    # lag 1: <d(t+1) d(t)> over (3/4, -1/4, 3/4) = 5/12, C = (5/12) / (5/4) = 1/3
    # lag 2: over (-3/4, -3/4) = -3/4, C = (-3/4) / (5/4) = -3/5
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


def test_uneven_series_by_hand():
    # M = 1, 1, 2, 4: <M> = 2, d = M - <M> = (-1, -1, 0, 2), <d^2> = 6/4;
    # lag 1: <d(t+1) d(t)> over (1, 0, 0) = 1/3, C = (1/3) / (3/2) = 2/9.
    # (The uncentred <M(t+1) M(t)> - <M>^2 = 11/3 - 4 gives -2/9 here.)
    # lag 3: d(3) d(0) = -2, C = -2 / (3/2) = -4/3
    C = autocorr.c_m([1.0, 1.0, 2.0, 4.0], 3)
    assert C[1] == pytest.approx(2.0 / 9.0, abs=1e-15)
    assert C[3] == pytest.approx(-4.0 / 3.0, abs=1e-15)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_independent_series_with_large_mean(seed):
    """An independent series with the statistics of M under cluster shifts of
    an ordered lattice (mean 0.99, spread 2.4e-4, 4000 steps) has C_M(dt) = 0
    for dt > 0; the estimate must scatter by about 1/sqrt(T), not by the
    ratio of <M>^2 to the variance."""
    rng = np.random.default_rng(seed)
    x = 0.9898 + 2.4e-4 * rng.standard_normal(4000)
    C = autocorr.c_m(x, 20)
    assert np.all(np.abs(C[1:]) < 5.0 / math.sqrt(4000))
    assert autocorr.tau_1e(C) < 1.0


def test_ar1_with_large_offset_and_tiny_variance():
    phi, T = 0.8, 200_000
    rng = np.random.default_rng(12)
    e = rng.standard_normal(T)
    x = np.empty(T)
    x[0] = e[0] / math.sqrt(1 - phi * phi)
    for t in range(1, T):
        x[t] = phi * x[t - 1] + e[t]
    x = 0.99 + 2e-4 * x
    C = autocorr.c_m(x, 10)
    for dt in (1, 2, 5):
        assert abs(C[dt] - phi ** dt) < 5 * math.sqrt((1 + phi * phi) / (1 - phi * phi) / T), dt
    assert autocorr.tau_1e(C) == pytest.approx(-1.0 / math.log(phi), rel=0.03)
