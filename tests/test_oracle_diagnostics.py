"""Pins of the oracle's chain diagnostics (oracle/diagnostics.py)."""
import numpy as np
import pytest

from oracle import diagnostics


def _ar1(phi, t, seed=0):
    rng = np.random.default_rng(seed)
    e = rng.standard_normal(t)
    x = np.empty(t)
    x[0] = e[0] / np.sqrt(1 - phi * phi)
    for i in range(1, t):
        x[i] = phi * x[i - 1] + e[i]
    return 3.0 + 0.5 * x


def test_lag_sums_match_fft_autocovariance():
    x = _ar1(0.6, 3000, seed=1)
    c = diagnostics.acf(x, 40)
    dev = x - x.mean()
    f = np.fft.rfft(dev, n=2 * len(x))
    acov = np.fft.irfft(f * np.conj(f))[: 41]            # sum_i dev_i dev_{i+n}
    ref = acov / (len(x) - np.arange(41)) / np.mean(dev ** 2)
    assert np.allclose(c, ref, rtol=1e-11, atol=1e-13)
    assert c[0] == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("phi,nc", [(0.7, 7), (0.5, 4), (0.3, 2)])   # crossings >= 6 sigma from 0.1
def test_ar1_correlation_and_length(phi, nc):
    x = _ar1(phi, 400_000, seed=2)
    c = diagnostics.acf(x, 60)
    n = np.arange(61)
    # sampling error of C_n for an AR(1) series is about sqrt((1+phi^2)/(1-phi^2) / T)
    tol = 5.0 * np.sqrt((1 + phi * phi) / (1 - phi * phi) / len(x))
    assert np.all(np.abs(c - phi ** n) < tol)
    assert diagnostics.correlation_length(c) == nc
    assert int(np.ceil(np.log(0.1) / np.log(phi))) == nc


def test_correlation_length_edge_cases():
    assert diagnostics.correlation_length(np.array([1.0, 0.5, 0.2])) == -1
    assert diagnostics.correlation_length(np.array([1.0, 0.09])) == 1
    assert diagnostics.correlation_length(np.array([1.0, 0.1, 0.05])) == 2   # strictly below
    with pytest.raises(ValueError):
        diagnostics.acf(np.arange(5.0), 5)


def test_moments_population_form():
    rng = np.random.default_rng(3)
    s = rng.standard_normal((7, 4, 4, 4))
    mean, var = diagnostics.moments(s)
    assert np.allclose(mean, s.sum(0) / 7)
    assert np.allclose(var, np.var(s, axis=0, ddof=0))
