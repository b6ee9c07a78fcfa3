"""Dense closed-form Wiener posterior on tiny grids (test infrastructure only).

For fixed P the target of the sampler is the Wiener posterior (paper Eq.
target_wiener_post): Gaussian with mean m = S R^T (R S R^T + N)^-1 d and
covariance C = S - S R^T (R S R^T + N)^-1 R S, with R diagonal (the per-voxel
response; 1 unless given) restricted to the observed voxels (finite N,
R != 0).  S is circulant on the periodic grid, S_xy = c(x - y) with
c = inverse DFT (with 1/M) of the per-voxel power P_grid(k), P(0) = 0.

This builds the M x M matrices explicitly and factorises them by Cholesky, so
it is meant for M <= 4096 (16^3).  It is the textbook formula written out and
is what pins the sampler, not a copy of it: it never touches the messenger
field.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import shells


def full_grid_power(n: int, n_bins: int, p_grid) -> np.ndarray:
    """P_grid on the full DFT grid from per-bin values (0 at k = 0)."""
    m = shells.integer_wavenumbers(n)
    q = m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2
    b = shells.bin_of_q(q, n, n_bins)
    p = np.asarray(p_grid, dtype=np.float64)
    return np.where(b >= 0, p[np.maximum(b, 0)], 0.0)


def signal_covariance(n: int, power_full: np.ndarray) -> np.ndarray:
    """Dense circulant S (M x M) with S[x, y] = c(x - y mod n)."""
    c = np.fft.ifftn(power_full).real
    idx = np.indices((n, n, n)).reshape(3, -1).T          # (M, 3)
    diff = (idx[:, None, :] - idx[None, :, :]) % n        # (M, M, 3)
    return c[diff[..., 0], diff[..., 1], diff[..., 2]]


def posterior(n: int, n_bins: int, p_grid, data, noise_var, response=None):
    """Wiener-filter mean and covariance (both flattened in C order)."""
    s_mat = signal_covariance(n, full_grid_power(n, n_bins, p_grid))
    d = np.asarray(data, dtype=np.float64).ravel()
    nv = np.asarray(noise_var, dtype=np.float64).ravel()
    r = np.ones_like(nv) if response is None else np.asarray(response, dtype=np.float64).ravel()
    o = np.isfinite(nv) & (r != 0.0)
    s_xo_r = s_mat[:, o] * r[o][None, :]                     # S R^T, observed columns
    a = r[o][:, None] * s_xo_r[o, :] + np.diag(nv[o])        # R S R^T + N
    cho = scipy.linalg.cho_factor(a, lower=True)
    mean = s_xo_r @ scipy.linalg.cho_solve(cho, d[o])
    cov = s_mat - s_xo_r @ scipy.linalg.cho_solve(cho, s_xo_r.T)
    return mean, cov


def draw(mean, cov, rng: np.random.Generator, jitter: float = 1e-12):
    """One exact draw from N(mean, cov) by Cholesky (cov is PSD with a zero
    k = 0 direction, hence the relative jitter)."""
    scale = np.trace(cov) / cov.shape[0]
    lo = np.linalg.cholesky(cov + jitter * scale * np.eye(cov.shape[0]))
    return mean + lo @ rng.standard_normal(cov.shape[0])
