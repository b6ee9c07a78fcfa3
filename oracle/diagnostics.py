"""Chain diagnostics, plainly, in FP64 (test infrastructure only).

* Autocorrelation of a recorded chain of power-spectrum amplitudes (Sec. 5.1,
  Eq. CORR_COEFF): with mean <P> and variance Var(P) over the T recorded
  samples,
      C_n = < (P^i - <P>)(P^{i+n} - <P>) > / Var(P),
  the average running over the T - n pairs (i, i + n) in the chain.
* Correlation length: the smallest lag n_c with C_n < 0.1 (the ten-percent
  rule the paper applies), or -1 if C stays at or above 0.1 up to max_lag.
* Posterior moments of the signal: mean and variance (population form, 1/K)
  over the K recorded samples of s.

Pins (tests/test_oracle_diagnostics.py): the lag sums equal the
autocovariance obtained through a zero-padded FFT (Wiener-Khinchin, a
library routine); C_0 = 1; an AR(1) series with coefficient phi gives
C_n ~ phi^n within its sampling error, and the matching n_c.
"""
from __future__ import annotations

import numpy as np


def acf(x, max_lag: int) -> np.ndarray:
    """C_n for n = 0 .. max_lag of the 1-D series x (Eq. CORR_COEFF)."""
    x = np.asarray(x, dtype=np.float64)
    t = x.shape[0]
    if max_lag >= t:
        raise ValueError("max_lag must be smaller than the series length")
    mu = x.mean()
    var = np.mean((x - mu) ** 2)
    dev = x - mu
    out = np.empty(max_lag + 1)
    for n in range(max_lag + 1):
        out[n] = np.mean(dev[: t - n] * dev[n:]) / var
    return out


def correlation_length(c: np.ndarray, threshold: float = 0.1) -> int:
    below = np.flatnonzero(np.asarray(c) < threshold)
    return int(below[0]) if below.size else -1


def acf_bins(trace, max_lag: int):
    """Per-bin C_n and n_c of a trace [T][n_bins]."""
    trace = np.asarray(trace, dtype=np.float64)
    c = np.stack([acf(trace[:, b], max_lag) for b in range(trace.shape[1])], axis=1)
    nc = np.array([correlation_length(c[:, b]) for b in range(trace.shape[1])])
    return c, nc


def moments(samples):
    """Mean and population variance over a stack of recorded samples."""
    s = np.asarray(samples, dtype=np.float64)
    mean = s.mean(axis=0)
    return mean, np.mean((s - mean) ** 2, axis=0)
