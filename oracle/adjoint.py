"""Deterministic messenger Wiener-filter iteration, its chi^2 loss and the
loss's gradient, plainly, in FP64 (test infrastructure only).

With every unit normal set to zero and P fixed, a sweep of the messenger
sampler (Sec. 3.1: the means mu^t of the messenger conditional and mu^s of
the signal conditional) is the map

    s_{k+1} = C u_k,   u_k = mu^t(s_k) = A s_k + b,

where A = diag(N~/(T R^2 + N~)) = diag(1 - tau R_i^2/N_i) on observed voxels
(1 where unobserved), b = tau R d / N (0 where unobserved) and
C = F^-1 diag(f) F with
f = S^/(S^ + T^) = P/(P + tau) per |k| bin and f = 0 at k = 0.  Its fixed
point is the Wiener filter S R (R S R + N)^-1 d.  Starting from s_0 = 0, K
iterations give s_K and the loss

    chi2_K = sum_{i observed} d_i (d_i - R_i s_K,i) / N_i,

which tends to d_o^T (R S R + N)_oo^-1 d_o as K grows: N_oo^-1 (d - R s_WF)_o
equals (R S R + N)_oo^-1 d_o.

The gradient follows the chain rule backwards through the stored iterates
(reverse mode, no checkpointing).  Let g_k = d chi2 / d s_k; then
g_K = -R d/N on observed voxels, and for k = K-1 .. 0:
  r_k = C^T g_{k+1} = C g_{k+1}    (C is symmetric: f is real and even),
  d chi2 / d f_b += (1/M) sum over the full-grid modes j of bin b of
                    Re(conj(g^_{k+1,j}) u^_{k,j}),
  d chi2 / d b   += r_k,
  g_k = A r_k.
Then d chi2 / d d = (2 d - R s_K)/N + (tau R/N) sum_k r_k on observed voxels
(b = tau R d/N) and d chi2 / d P_b = d chi2 / d f_b * tau / (P_b + tau)^2 in
grid units.

Pins (tests/test_oracle_adjoint.py): central finite differences of
wf_forward; in the converged limit, the dense closed forms of
d_o^T (R S R + N)_oo^-1 d_o and of its gradients, 2 (R S R + N)_oo^-1 d_o and
-x^T (R dS/dP_b R)_oo x with x = (R S R + N)_oo^-1 d_o; with R given, the
same for a non-trivial response.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.fft

from . import sampler, shells


def with_data(prob: sampler.Problem, data) -> sampler.Problem:
    """The same noise model (N, mask, tau) with new data."""
    return dataclasses.replace(prob, data=np.asarray(data, dtype=np.float64))


def chi2(prob: sampler.Problem, s) -> float:
    o = prob.observed
    d = prob.data[o]
    return float(np.sum(d * (d - prob.r[o] * s[o]) / prob.noise_var[o]))


def wf_forward(prob: sampler.Problem, p_grid, n_iter: int, keep: bool = False):
    """K noise-free sweeps from s_0 = 0 at fixed P (grid units).

    Returns (s_K, chi2_K) and, with keep=True, the list of s_0 .. s_{K-1}."""
    st = sampler.State(s=np.zeros((prob.n,) * 3), p_grid=np.asarray(p_grid, dtype=np.float64))
    kept = []
    for _ in range(n_iter):
        if keep:
            kept.append(st.s)
        st = sampler.sweep(prob, st, sample_pk=False, noise=False)
    out = (st.s, chi2(prob, st.s))
    return out + (kept,) if keep else out


def filter_per_mode(prob: sampler.Problem, p_grid) -> np.ndarray:
    """f = P/(P + tau) on the half grid, 0 at k = 0."""
    n = prob.n
    b = shells.bin_of_q(shells.half_grid_q(n), n, prob.n_bins)
    p = np.asarray(p_grid, dtype=np.float64)
    pm = np.where(b >= 0, p[np.maximum(b, 0)], 0.0)
    return pm / (pm + prob.tau)


def wf_gradient(prob: sampler.Problem, p_grid, n_iter: int):
    """(chi2_K, d chi2/d P_b in grid units, d chi2/d d) by reverse mode."""
    n, m, tau = prob.n, prob.m, prob.tau
    o = prob.observed
    rr = prob.r
    nv = np.where(o, prob.noise_var, np.inf)
    a_diag = np.where(o, 1.0 - tau * rr * rr / nv, 1.0)
    s_k, loss, iterates = wf_forward(prob, p_grid, n_iter, keep=True)
    f = filter_per_mode(prob, p_grid)
    b = shells.bin_of_q(shells.half_grid_q(n), n, prob.n_bins)
    w = np.broadcast_to(shells.half_grid_weight(n)[None, None, :], b.shape)
    sel = b >= 0

    g = np.where(o, -rr * prob.data / nv, 0.0)
    grad_f = np.zeros(prob.n_bins)
    sum_r = np.zeros((n, n, n))
    for k in range(n_iter - 1, -1, -1):
        u_k, _ = sampler.messenger_moments(iterates[k], prob)
        g_hat = scipy.fft.rfftn(g)
        u_hat = scipy.fft.rfftn(u_k)
        prod = (g_hat.real * u_hat.real + g_hat.imag * u_hat.imag) * w / m
        grad_f += np.bincount(b[sel], weights=prod[sel], minlength=prob.n_bins)
        r = scipy.fft.irfftn(f * g_hat, s=(n, n, n))
        sum_r += r
        g = a_diag * r
    p = np.asarray(p_grid, dtype=np.float64)
    grad_p = grad_f * tau / (p + tau) ** 2
    grad_d = np.where(o, (2.0 * prob.data - rr * s_k) / nv + tau * rr / nv * sum_r, 0.0)
    return loss, grad_p, grad_d
