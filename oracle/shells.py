"""|k|-shell binning of the power spectrum (test infrastructure only).

The paper notes that homogeneity and isotropy let the signal covariance be
averaged over spherical shells in Fourier space (Sec. "Sampling the signal
covariance", last paragraph) but leaves the details to earlier work.  The
reading taken here:

* n_bins equal-width bins in |k| on (0, sqrt(3) k_Ny], k_Ny = pi N / L; the
  k = 0 mode belongs to no bin (its power is zero, the field has zero mean);
* with k = k_f sqrt(q), k_f = 2 pi / L and q = m_x^2 + m_y^2 + m_z^2 (integer
  wavenumbers m in (-N/2, N/2]), bin b holds the q >= 1 with
  3 b^2 N^2 / (4 n_bins^2) <= q < 3 (b+1)^2 N^2 / (4 n_bins^2); the corner
  q = 3 N^2 / 4 joins the last bin.  The edges are compared in exact integer
  arithmetic: many edges fall exactly on a populated shell;
* n_b counts real degrees of freedom, i.e. full-grid modes in the bin.

Pins: brute-force enumeration of the full grid with exact rational edges, and
sum_b n_b = M - 1 (tests/test_oracle_shells.py).
"""
from __future__ import annotations

import numpy as np


def thresholds(n: int, n_bins: int) -> np.ndarray:
    """Smallest q of each bin: Q_0 = 1, Q_b = ceil(3 b^2 n^2 / (4 n_bins^2))."""
    q = [1]
    den = 4 * n_bins * n_bins
    for b in range(1, n_bins):
        q.append(-((-3 * b * b * n * n) // den))   # exact ceiling division
    return np.asarray(q, dtype=np.int64)


def integer_wavenumbers(n: int) -> np.ndarray:
    """m(i) = i for i <= n/2, i - n otherwise."""
    i = np.arange(n)
    return np.where(i <= n // 2, i, i - n).astype(np.int64)


def half_grid_q(n: int) -> np.ndarray:
    """q = m_x^2 + m_y^2 + m_z^2 on the half grid (ix, iy, iz), iz <= n/2."""
    m = integer_wavenumbers(n)
    mz = np.arange(n // 2 + 1, dtype=np.int64)
    return m[:, None, None] ** 2 + m[None, :, None] ** 2 + mz[None, None, :] ** 2


def bin_of_q(q: np.ndarray, n: int, n_bins: int) -> np.ndarray:
    """Bin index of each q (-1 for q = 0)."""
    q = np.asarray(q, dtype=np.int64)
    b = np.searchsorted(thresholds(n, n_bins)[1:], q, side="right")
    return np.where(q >= 1, b, -1).astype(np.int64)


def half_grid_weight(n: int) -> np.ndarray:
    """Full-grid modes each half-grid mode stands for: 1 on iz in {0, n/2}, else 2."""
    w = np.full(n // 2 + 1, 2.0)
    w[0] = 1.0
    w[n // 2] = 1.0
    return w


def mode_counts(n: int, n_bins: int) -> np.ndarray:
    """n_b: number of full-grid modes (real degrees of freedom) in each bin."""
    b = bin_of_q(half_grid_q(n), n, n_bins)
    w = np.broadcast_to(half_grid_weight(n)[None, None, :], b.shape)
    sel = b >= 0
    return np.bincount(b[sel], weights=w[sel], minlength=n_bins).astype(np.int64)
