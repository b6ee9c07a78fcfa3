"""Log-determinant term of the Gaussian likelihood's power-spectrum gradient,
plainly, in FP64 (test infrastructure only).

With the data model of Sec. 2, d = R s + eps on the observed voxels o, and a
Gaussian signal of covariance S(P), the data are Gaussian with covariance
A = (R S R + N)_oo, so

    ln L(P) = -1/2 d^T A^-1 d - 1/2 ln det A + const,
    d ln L / d P_b = 1/2 x^T R S_b R x - 1/2 T_b,   x = A^-1 d,
    T_b = tr(A^-1 R S_b R),   S_b = d S / d P_b.

The quadratic term is the chi2 of the messenger Wiener filter and its adjoint
(oracle/adjoint.py).  T_b is estimated by Hutchinson's identity
E[z^T M z] = tr(M) for E[z z^T] = 1, applied with probes of covariance N:

    z = sgn(R) sqrt(N) xi on observed voxels (xi = +-1), so E[z z^T] = N,
    u = A^-1 z = N^-1 (z - R s_WF(z)),   s_WF(z) the Wiener filter of data z,
    E[(R u)^T S_b (R z / N)] = tr(A^-1 R S_b R N^-1 N) = T_b.

For a real field y and x, y^T S_b x = (1/M) sum over the full-grid modes k of
bin b of Re(conj(y^_k) x^_k) with unnormalised DFTs (S = F^-1 diag(P) F in
grid units).  The filter s_WF(z) is K noise-free messenger sweeps on data z,
as in oracle/adjoint.py, so one probe costs K sweeps.

The probe signs come from Philox4x32-10 (oracle/philox.py): voxel v (C order
index) of probe j uses counter (v div 4, j, 4, chain), word v mod 4, and
xi = -1 when that word's top bit is set.

Pins (tests/test_oracle_logdet.py): a single probe equals the dense
z^T A^-1 R S_b R N^-1 z once the filter has converged; the probe average
matches the dense trace within its Monte Carlo error; the dense trace equals
central differences of the dense ln det A (Cholesky); the signs are balanced
and independent across probes.
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.linalg

from . import adjoint, philox, sampler, shells, wiener

PHASE_PROBE = 4


def probe_signs(n: int, seed: int, chain: int, probe: int) -> np.ndarray:
    """xi = +-1 for every voxel of an (n, n, n) grid."""
    v = np.arange(n ** 3, dtype=np.uint64)
    k0, k1 = philox.key_words(seed)
    words = philox.philox4x32_10(v >> np.uint64(2), probe, PHASE_PROBE, chain, k0, k1)
    w = np.choose((v & np.uint64(3)).astype(np.int64), words)
    return np.where(w >> np.uint32(31), -1.0, 1.0).reshape((n,) * 3)


def probe_vector(prob: sampler.Problem, probe: int) -> np.ndarray:
    """z = sgn(R) sqrt(N) xi on observed voxels, 0 elsewhere."""
    o = prob.observed
    xi = probe_signs(prob.n, prob.seed, prob.chain, probe)
    nv = np.where(o, prob.noise_var, 0.0)
    return np.where(o, np.sign(prob.r) * np.sqrt(nv) * xi, 0.0)


def bin_cross(prob: sampler.Problem, y, x) -> np.ndarray:
    """(1/M) sum over the full-grid modes of each bin of Re(conj(y^) x^)."""
    n = prob.n
    b = shells.bin_of_q(shells.half_grid_q(n), n, prob.n_bins)
    w = np.broadcast_to(shells.half_grid_weight(n)[None, None, :], b.shape)
    yh, xh = scipy.fft.rfftn(y), scipy.fft.rfftn(x)
    prod = (yh.real * xh.real + yh.imag * xh.imag) * w / prob.m
    sel = b >= 0
    return np.bincount(b[sel], weights=prod[sel], minlength=prob.n_bins)


def trace_probe(prob: sampler.Problem, p_grid, n_iter: int, probe: int) -> np.ndarray:
    """One Hutchinson sample of T_b (grid units, per unit of P_b / V_cell)."""
    o = prob.observed
    z = probe_vector(prob, probe)
    s_k, _ = adjoint.wf_forward(adjoint.with_data(prob, z), p_grid, n_iter)
    nv = np.where(o, prob.noise_var, np.inf)
    u = np.where(o, (z - prob.r * s_k) / nv, 0.0)
    return bin_cross(prob, prob.r * u, np.where(o, prob.r * z / nv, 0.0))


def trace_estimate(prob: sampler.Problem, p_grid, n_iter: int, probes) -> np.ndarray:
    return np.mean([trace_probe(prob, p_grid, n_iter, j) for j in probes], axis=0)


# ---------------------------------------------------------------- dense forms
def _dense(prob: sampler.Problem, p_grid):
    o = prob.observed.ravel()
    r = prob.r.ravel()[o]
    s = wiener.signal_covariance(prob.n, wiener.full_grid_power(prob.n, prob.n_bins, p_grid))
    a = r[:, None] * s[np.ix_(o, o)] * r[None, :] + np.diag(prob.noise_var.ravel()[o])
    return o, r, a


def bin_covariance(prob: sampler.Problem, b: int) -> np.ndarray:
    """S_b = d S / d P_b (grid units), dense M x M."""
    ind = np.zeros(prob.n_bins)
    ind[b] = 1.0
    return wiener.signal_covariance(prob.n, wiener.full_grid_power(prob.n, prob.n_bins, ind))


def dense_logdet(prob: sampler.Problem, p_grid) -> float:
    _, _, a = _dense(prob, p_grid)
    lo = scipy.linalg.cholesky(a, lower=True)
    return float(2.0 * np.sum(np.log(np.diag(lo))))


def dense_trace(prob: sampler.Problem, p_grid) -> np.ndarray:
    """T_b = tr(A^-1 R S_b R) for every bin."""
    o, r, a = _dense(prob, p_grid)
    cho = scipy.linalg.cho_factor(a, lower=True)
    out = np.zeros(prob.n_bins)
    for b in range(prob.n_bins):
        sb = r[:, None] * bin_covariance(prob, b)[np.ix_(o, o)] * r[None, :]
        out[b] = float(np.trace(scipy.linalg.cho_solve(cho, sb)))
    return out


def dense_probe(prob: sampler.Problem, p_grid, probe: int) -> np.ndarray:
    """z^T A^-1 R S_b R N^-1 z for the probe's z, for every bin."""
    o, r, a = _dense(prob, p_grid)
    z = probe_vector(prob, probe).ravel()[o]
    x = scipy.linalg.solve(a, z, assume_a="pos")
    y = z / prob.noise_var.ravel()[o]
    return np.array([float((r * x) @ bin_covariance(prob, b)[np.ix_(o, o)] @ (r * y))
                     for b in range(prob.n_bins)])
