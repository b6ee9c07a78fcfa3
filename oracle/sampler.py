"""One Gibbs sweep of the messenger-field sampler, plainly, in FP64 (test
infrastructure only).

Model (paper Sec. "The augmented Wiener posterior"): data d = R s + eps with
diagonal noise covariance N, Gaussian signal prior with covariance S that is
diagonal in Fourier space, and a messenger field t with covariance T = tau 1.
Marginalising t recovers the Wiener posterior when the augmented noise is
N~ = N - R^T T R, which requires 0 < tau <= [(R^-1)^T N R^-1]_i = N_i / R_i^2
on every observed voxel; tau is taken as the smallest observed N_i / R_i^2.
R is diagonal: a per-voxel response R_i, 1 unless given.  A voxel is
observed when R_i != 0 and N_i is finite; elsewhere the paper's R^2 = 0
branch applies (N_i = +inf is the same thing).

One sweep of chain c, sweep index n (paper Algs. 1 and 2, eqs. for mu^t,
sigma^t, mu^s, sigma^s and the inverse-gamma conditional):
  1. messenger, voxel by voxel:  t_i ~ N(mu^t_i, (sigma^t_i)^2) with
     mu^t = T/(T R^2 + N~) R d + N~/(T R^2 + N~) s,
     (sigma^t)^2 = T N~ / (T R^2 + N~)   where R^2 > 0, else mu^t = s and
     (sigma^t)^2 = T;
  2. t^ = unnormalised forward DFT of t (the transform's normalisation makes
     T^ = M tau and S^_k = M P(k)/V_cell, the paper's remark after the
     messenger conditional);
  3. signal, mode by mode:  s^_k ~ N(mu^s_k, (sigma^s_k)^2) with
     mu^s = S^/(S^+T^) t^ and (sigma^s)^2 = S^ T^/(S^+T^).  The field is real,
     so s^_{-k} = conj(s^_k): a complex mode splits its variance equally over
     real and imaginary parts, self-conjugate modes are real with the full
     variance, and of each conjugate pair on the iz in {0, N/2} planes only
     the member with the smaller ix*N + iy is drawn;
  4. shell power sigma_b = sum over full-grid modes of bin b of |s^_k|^2;
  5. P(k) per bin from its conditional under Jeffreys' prior 1/P:
     P_b ~ InvGamma(n_b / 2, sigma_b / (2 M)) in grid units (variance per
     voxel), drawn as P_b = sigma_b / (2 M g) with g ~ Gamma(n_b / 2, 1); for a
     single mode this is the paper's chi-square construction
     S^ = |s^|^2 / G^2.  Optionally the prior is the conjugate
     InvGamma(a0, b0) (density ~ P^-(a0+1) exp(-b0/P), Jeffreys' at
     a0 = b0 = 0): the conditional becomes InvGamma(n_b/2 + a0,
     sigma_b/(2M) + b0), drawn as P_b = (sigma_b + 2 M b0) / (2 M g) with
     g ~ Gamma(n_b/2 + a0, 1).  Jeffreys' prior leaves the joint posterior
     improper as P_b -> 0 wherever the noise is finite; b0 > 0 removes that;
  6. s = inverse DFT of s^ (with the 1/M factor).
The redundant forward transform of s in Alg. 1 is skipped: s^ is redrawn in
full in step 3.  The draws come from the Philox contract in oracle.philox.

Pins (tests/test_oracle_sampler.py): the noise-free iteration converges to
the dense Wiener filter; fixed-P chains reproduce the dense posterior mean and
variance; with uniform noise and no mask one sweep is the textbook per-mode
Wiener posterior; P draws follow scipy.stats.invgamma; Parseval and exact
Hermitian symmetry hold every sweep; joint (s, P) moments agree with an
exact-block sampler that draws s | P by dense Cholesky.
"""
from __future__ import annotations

import dataclasses
import os
from typing import Optional

import numpy as np
import scipy.fft

from . import philox, shells


def _workers() -> int:
    return int(os.environ.get("ORACLE_FFT_WORKERS", "1"))


@dataclasses.dataclass
class Problem:
    n: int
    box: float
    n_bins: int
    data: np.ndarray        # (n, n, n) float64, ignored where unobserved
    noise_var: np.ndarray   # (n, n, n) float64, +inf where unobserved
    tau: float
    seed: int
    chain: int = 0
    response: Optional[np.ndarray] = None   # (n, n, n) float64 R_i; None: R_i = 1
    prior_shape: float = 0.0   # a0 of the InvGamma(a0, b0) prior on P_b (0, 0: Jeffreys)
    prior_scale: float = 0.0   # b0, physical units (volume)

    @property
    def m(self) -> int:
        return self.n ** 3

    @property
    def cell_volume(self) -> float:
        return (self.box / self.n) ** 3

    @property
    def prior_scale_grid(self) -> float:
        """b0 in grid units (variance per voxel), like P_grid."""
        return self.prior_scale / self.cell_volume

    @property
    def observed(self) -> np.ndarray:
        if self.response is None:
            return np.isfinite(self.noise_var)
        return np.isfinite(self.noise_var) & (self.response != 0.0)

    @property
    def r(self) -> np.ndarray:
        """R_i on observed voxels, 0 elsewhere."""
        one = np.ones_like(self.noise_var) if self.response is None else self.response
        return np.where(self.observed, one, 0.0)


def make_problem(data, noise_var, n_bins: int, box: float, seed: int, chain: int = 0,
                 tau: Optional[float] = None, response=None, prior=(0.0, 0.0)) -> Problem:
    """tau defaults to the smallest observed N_i / R_i^2; a given tau must not
    exceed it (the augmented noise N - R T R must stay positive).  prior =
    (a0, b0) of the InvGamma prior on every P_b, b0 in physical units; (0, 0)
    is Jeffreys' prior."""
    a0, b0 = (float(v) for v in prior)
    if not (np.isfinite(a0) and np.isfinite(b0) and a0 >= 0.0 and b0 >= 0.0):
        raise ValueError("prior (a0, b0) must be finite and >= 0")
    data = np.asarray(data, dtype=np.float64)
    noise_var = np.asarray(noise_var, dtype=np.float64)
    if response is not None:
        response = np.asarray(response, dtype=np.float64)
        if not np.all(np.isfinite(response)):
            raise ValueError("response not finite")
    n = data.shape[0]
    prob = Problem(n=n, box=float(box), n_bins=int(n_bins), data=data, noise_var=noise_var,
                   tau=0.0, seed=int(seed), chain=int(chain), response=response,
                   prior_shape=a0, prior_scale=b0)
    obs = prob.observed
    if not obs.any():
        raise ValueError("no observed voxel")
    tau_max = float(np.min(noise_var[obs] / prob.r[obs] ** 2))
    if tau is None or tau <= 0:
        tau = tau_max
    elif tau > tau_max:
        raise ValueError("tau exceeds the smallest observed N_i / R_i^2")
    return dataclasses.replace(prob, tau=float(tau))


# ---------------------------------------------------------------- draws
def messenger_normals(n: int, seed: int, chain: int, sweep: int) -> np.ndarray:
    """G(0,1) for every voxel (ix, iy, iz).  One Philox call per voxel quad
    iz in {c, c + N/4, c + N/2, c + 3N/4} of a z pencil, counter
    ((ix N + iy) N/4 + c, sweep, 0, chain); the quad takes the call's four
    normals in order (cos and sin of the first word pair, then of the second)."""
    q4 = n // 4
    ix = np.arange(n, dtype=np.uint64)[:, None, None]
    iy = np.arange(n, dtype=np.uint64)[None, :, None]
    c = np.arange(q4, dtype=np.uint64)[None, None, :]
    w0 = (ix * np.uint64(n) + iy) * np.uint64(q4) + c
    lanes = philox.normals4(w0, sweep, philox.PHASE_MESSENGER, chain, seed)
    return np.concatenate(lanes, axis=2)          # iz = j * N/4 + c


def signal_normals(n: int, seed: int, chain: int, sweep: int):
    """(G_re, G_im) for every half-grid mode (ix, iy, iz), iz <= n/2.  One Philox
    call per mode pair (ix, ix + N/2), ix < N/2, counter ((iz N + iy) N/2 + ix,
    sweep, 1, chain); ix < N/2 takes the first word pair, ix + N/2 the second."""
    h = n // 2
    p = np.arange(h, dtype=np.uint64)[:, None, None]
    iy = np.arange(n, dtype=np.uint64)[None, :, None]
    iz = np.arange(h + 1, dtype=np.uint64)[None, None, :]
    w0 = (iz * np.uint64(n) + iy) * np.uint64(h) + p
    ga, gb, gc, gd = philox.normals4(w0, sweep, philox.PHASE_SIGNAL, chain, seed)
    return np.concatenate([ga, gc], axis=0), np.concatenate([gb, gd], axis=0)


# ---------------------------------------------------------------- steps
def messenger_moments(s: np.ndarray, prob: Problem):
    """Conditional mean and variance of t given s, d (T = tau).  N~ = N - T R^2
    is >= 0 by the choice of tau and exactly 0 where N / R^2 is smallest;
    rounding of T R^2 there can leave -1 ulp, which is set back to 0."""
    T = prob.tau
    R = prob.r
    n_tilde = np.where(prob.observed, np.maximum(prob.noise_var - T * R * R, 0.0), 1.0)
    den = T * R * R + n_tilde
    d = np.where(prob.observed, prob.data, 0.0)
    mu = np.where(R * R > 0, T / den * R * d + n_tilde / den * s, s)
    var = np.where(R * R > 0, T * n_tilde / den, T)
    return mu, var


def messenger_step(s, prob: Problem, sweep: int, noise: bool = True):
    mu, var = messenger_moments(s, prob)
    if not noise:
        return mu
    return mu + np.sqrt(var) * messenger_normals(prob.n, prob.seed, prob.chain, sweep)


def _self_conjugate(n: int) -> np.ndarray:
    e = np.zeros(n, dtype=bool)
    e[0] = True
    e[n // 2] = True
    ez = np.zeros(n // 2 + 1, dtype=bool)
    ez[0] = True
    ez[n // 2] = True
    return e[:, None, None] & e[None, :, None] & ez[None, None, :]


def signal_moments(t_hat, p_grid, prob: Problem):
    """Per-mode conditional mean and variance of s^ given t^ and P."""
    n, m = prob.n, prob.m
    b = shells.bin_of_q(shells.half_grid_q(n), n, prob.n_bins)
    s_cov = np.where(b >= 0, m * np.asarray(p_grid, dtype=np.float64)[np.maximum(b, 0)], 0.0)
    t_cov = m * prob.tau
    mu = s_cov / (s_cov + t_cov) * t_hat
    var = s_cov * t_cov / (s_cov + t_cov)
    return mu, var


def hermitian_mirror(s_hat: np.ndarray) -> np.ndarray:
    """On the iz in {0, N/2} planes copy conj(s^) of the member of each conjugate
    pair with the smaller ix*N + iy onto the other member."""
    n = s_hat.shape[0]
    i = np.arange(n)
    lin = i[:, None] * n + i[None, :]
    j = (-i) % n
    lin_partner = j[:, None] * n + j[None, :]
    take = lin_partner < lin
    for iz in (0, n // 2):
        plane = s_hat[:, :, iz]
        partner = plane[j][:, j]
        plane[take] = np.conj(partner[take])
    return s_hat


def signal_step(t_hat, p_grid, prob: Problem, sweep: int, noise: bool = True):
    mu, var = signal_moments(t_hat, p_grid, prob)
    if not noise:
        s_hat = mu.copy()
        sc = _self_conjugate(prob.n)
        s_hat[sc] = mu[sc].real
        return hermitian_mirror(s_hat)
    g_re, g_im = signal_normals(prob.n, prob.seed, prob.chain, sweep)
    s_hat = mu + np.sqrt(0.5 * var) * (g_re + 1j * g_im)
    sc = _self_conjugate(prob.n)
    s_hat[sc] = mu[sc].real + np.sqrt(var[sc]) * g_re[sc]
    return hermitian_mirror(s_hat)


def shell_power(s_hat, prob: Problem) -> np.ndarray:
    """sigma_b = sum over the full-grid modes of bin b of |s^_k|^2."""
    n = prob.n
    b = shells.bin_of_q(shells.half_grid_q(n), n, prob.n_bins)
    w = np.broadcast_to(shells.half_grid_weight(n)[None, None, :], b.shape)
    p2 = (s_hat.real ** 2 + s_hat.imag ** 2) * w
    sel = b >= 0
    return np.bincount(b[sel], weights=p2[sel], minlength=prob.n_bins)


def power_step(sigma, p_grid, prob: Problem, sweep: int) -> np.ndarray:
    """Draw P_b (grid units) from InvGamma(n_b/2 + a0, sigma_b/(2M) + b0), the
    conditional under the InvGamma(a0, b0) prior (Jeffreys' at a0 = b0 = 0);
    empty bins keep P."""
    counts = shells.mode_counts(prob.n, prob.n_bins)
    out = np.array(p_grid, dtype=np.float64, copy=True)
    b0 = prob.prior_scale_grid
    for b in range(prob.n_bins):
        if counts[b] > 0:
            g = philox.gamma_mt(0.5 * counts[b] + prob.prior_shape, prob.seed, prob.chain,
                                sweep, b)
            out[b] = (sigma[b] + 2.0 * prob.m * b0) / (2.0 * prob.m * g)
    return out


@dataclasses.dataclass
class State:
    s: np.ndarray           # real-space signal, (n, n, n) float64
    p_grid: np.ndarray      # P per bin in grid units (P_phys / V_cell)
    sweep: int = 0          # index of the next sweep


def sweep(prob: Problem, state: State, sample_pk: bool = True, noise: bool = True,
          diagnostics: Optional[dict] = None) -> State:
    """One Gibbs sweep t -> s -> P; returns the new state.

    noise=False runs the deterministic messenger iteration (every G = 0, P
    fixed), whose fixed point is the Wiener-filter mean."""
    n = prob.n
    t = messenger_step(state.s, prob, state.sweep, noise=noise)
    t_hat = scipy.fft.rfftn(t, workers=_workers())
    s_hat = signal_step(t_hat, state.p_grid, prob, state.sweep, noise=noise)
    p_new = state.p_grid
    sigma = None
    if sample_pk and noise:
        sigma = shell_power(s_hat, prob)
        p_new = power_step(sigma, state.p_grid, prob, state.sweep)
    s_new = scipy.fft.irfftn(s_hat, s=(n, n, n), workers=_workers())
    if diagnostics is not None:
        diagnostics["t"] = t
        diagnostics["s_hat"] = s_hat
        diagnostics["sigma"] = shell_power(s_hat, prob) if sigma is None else sigma
    return State(s=s_new, p_grid=np.asarray(p_new, dtype=np.float64), sweep=state.sweep + 1)


def run_chain(prob: Problem, state: State, n_sweeps: int, sample_pk: bool = True,
              noise: bool = True) -> State:
    for _ in range(n_sweeps):
        state = sweep(prob, state, sample_pk=sample_pk, noise=noise)
    return state
