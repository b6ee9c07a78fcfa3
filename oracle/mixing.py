"""The mixing sampler (Sec. 3.3, Alg. 3) in its shell form, plainly, in FP64
(test infrastructure only).

Conditional on the messenger field, the paper samples the signal and its
covariance jointly in the coordinates s^ = sqrt(S^) x^, which moves S^ from
the signal prior into the messenger likelihood.  Here S^ is shared by the
modes of a |k| shell, S^_b = M P_b, with Jeffreys' prior 1/P_b.

Readings (the printed formulas disagree with the stated densities):
* x^ | S^, t^ is Gaussian with variance T^/(S^ + T^) and mean
  sqrt(S^) t^ / (S^ + T^), completing the square in the transformed density
  (the printed mean carries an extra factor T^).  Drawing x^ is the ordinary
  signal draw s^ | S^, t^ divided by sqrt(S^).
* Under Jeffreys' prior the transformed joint density is
  prod_b S^_b^-1 prod_k exp(-|x^_k|^2/2) exp(-|sqrt(S^_b) x^_k - t^_k|^2 / (2 T^)),
  so U = sqrt(S^_b) given x^, t^ has density proportional to
      U^-1 exp(-(U - R_b/X_b)^2 X_b / (2 T^)),
  X_b = sum |x^_k|^2 and R_b = sum Re(conj(x^_k) t^_k) over the full-grid
  modes of bin b.  With the paper's independence proposal, a normal with
  mean R_b/X_b and variance T^/X_b truncated to U' > 0, the acceptance
  probability is min(1, U/U'), not the printed min(1, (U'/U)^2), which
  corresponds to a U^2 prefactor.  For one mode per bin the proposal is the
  paper's, t^/x^ and T^/x^2.
* The truncated normal is drawn exactly.  Write a = -mean/sd for the
  standardised lower bound.  For a <= 0.5, propose z from N(0, 1) until
  z > a.  Otherwise use Robert's exponential proposal (Statistics and
  Computing 5, 1995): z = a - ln(U1)/r with r = (a + sqrt(a^2 + 4))/2,
  accepted when U2 <= exp(-(z - r)^2/2).

Random numbers: attempt j of bin b reads the Philox words of counter
(b * 2^16 + j, sweep, PHASE_MIX, chain).  z is the cosine normal of (x0, x1),
or U1 = U23(x0) and U2 = U23(x1) in the exponential regime.  The
acceptance uniform is U23(x3) of attempt 0.  After MIX_ATTEMPTS attempts
without a proposal the move is rejected.

One mixing sweep:
  t ~ messenger conditional;  t^ = DFT(t);  s^ ~ signal conditional at P;
  per bin: the MH move of S^_b;  s^_k *= sqrt(S^'_b / S^_b);  s = DFT^-1 s^.

With the optional conjugate prior InvGamma(a0, b0) on P_b (density
~ P^-(a0+1) exp(-b0/P)) in place of Jeffreys', the prior of U = sqrt(S^)
becomes ~ U^-(2 a0 + 1) exp(-M b0 / U^2) (b0 in grid units), and the
acceptance probability min(1, (U/U')^(2 a0 + 1) exp(M b0 (1/U^2 - 1/U'^2))).
At a0 = b0 = 0 this is Jeffreys' min(1, U/U'), which is evaluated as that
ratio itself.

Pins (tests/test_oracle_mixing.py): iterating the (x^, S^) update at fixed
t^ leaves the exact conditional marginal of P invariant,
p(P | t^) ~ prior(P) prod_k N(t^_k; 0, M (P + tau)), checked by quadrature
on a small grid, with Jeffreys' prior and with a proper InvGamma prior; the
printed (U'/U)^2 acceptance fails the same check.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from . import philox, sampler, shells

PHASE_MIX = 3
MIX_ATTEMPTS = 64
TN_SPLIT = 0.5


def shell_sums(x_hat, t_hat, prob: sampler.Problem):
    """X_b = sum |x^|^2 and R_b = sum Re(conj(x^) t^) over full-grid modes."""
    n = prob.n
    b = shells.bin_of_q(shells.half_grid_q(n), n, prob.n_bins)
    w = np.broadcast_to(shells.half_grid_weight(n)[None, None, :], b.shape)
    sel = b >= 0
    xx = (x_hat.real ** 2 + x_hat.imag ** 2) * w
    xt = (x_hat.real * t_hat.real + x_hat.imag * t_hat.imag) * w
    return (np.bincount(b[sel], weights=xx[sel], minlength=prob.n_bins),
            np.bincount(b[sel], weights=xt[sel], minlength=prob.n_bins))


def truncated_normal(mean: float, sd: float, seed: int, chain: int, sweep: int, b: int):
    """(U' drawn from N(mean, sd^2) truncated to U' > 0, or None; the MH uniform)."""
    k0, k1 = philox.key_words(seed)
    a = -mean / sd
    u_mh = None
    for j in range(MIX_ATTEMPTS):
        x0, x1, x2, x3 = philox.philox4x32_10(b * 65536 + j, sweep, PHASE_MIX, chain, k0, k1)
        if j == 0:
            u_mh = float(philox.u23(x3))
        if a <= TN_SPLIT:
            z = float(philox.box_muller(x0, x1)[0])
            if z > a:
                return mean + sd * z, u_mh
        else:
            r = 0.5 * (a + np.sqrt(a * a + 4.0))
            z = a - np.log(float(philox.u23(x0))) / r
            if float(philox.u23(x1)) <= np.exp(-0.5 * (z - r) ** 2):
                return mean + sd * z, u_mh
    return None, u_mh


def accept(u_mh: float, u: float, u_new: float, prob: sampler.Problem) -> bool:
    """Metropolis-Hastings acceptance of U -> U' for the independence
    proposal, under the problem's prior on P (grid units, S^ = M P = U^2)."""
    a0, b0 = prob.prior_shape, prob.prior_scale_grid
    if a0 == 0.0 and b0 == 0.0:
        return u_mh <= u / u_new
    log_ratio = (2.0 * a0 + 1.0) * np.log(u / u_new) + prob.m * b0 * (1.0 / (u * u)
                                                                      - 1.0 / (u_new * u_new))
    return np.log(u_mh) <= log_ratio


def mix_power_step(s_hat, t_hat, p_grid, prob: sampler.Problem, sweep: int):
    """The MH move of every S^_b given t^ and the drawn s^ (at the current P).

    Returns the new P (grid units) and the per-bin factor sqrt(S^'/S^) that
    turns s^ = sqrt(S^) x^ into sqrt(S^') x^."""
    m = prob.m
    t_cov = m * prob.tau                                   # T^
    p = np.asarray(p_grid, dtype=np.float64)
    b_of = shells.bin_of_q(shells.half_grid_q(prob.n), prob.n, prob.n_bins)
    root_s = np.sqrt(m * p)                                # sqrt(S^_b)
    x_hat = np.where(b_of >= 0, s_hat / root_s[np.maximum(b_of, 0)], 0.0)
    xx, xt = shell_sums(x_hat, t_hat, prob)
    p_new = p.copy()
    ratio = np.ones(prob.n_bins)
    for b in range(prob.n_bins):
        if xx[b] <= 0.0:
            continue
        u_new, u_mh = truncated_normal(xt[b] / xx[b], np.sqrt(t_cov / xx[b]), prob.seed,
                                       prob.chain, sweep, b)
        if u_new is not None and accept(u_mh, root_s[b], u_new, prob):
            p_new[b] = u_new * u_new / m
            ratio[b] = u_new / root_s[b]
    return p_new, ratio


def mixing_sweep(prob: sampler.Problem, state: sampler.State) -> sampler.State:
    n = prob.n
    t = sampler.messenger_step(state.s, prob, state.sweep)
    t_hat = scipy.fft.rfftn(t, workers=sampler._workers())
    s_hat = sampler.signal_step(t_hat, state.p_grid, prob, state.sweep)
    p_new, ratio = mix_power_step(s_hat, t_hat, state.p_grid, prob, state.sweep)
    b_of = shells.bin_of_q(shells.half_grid_q(n), n, prob.n_bins)
    s_hat = s_hat * np.where(b_of >= 0, ratio[np.maximum(b_of, 0)], 1.0)
    s_new = scipy.fft.irfftn(s_hat, s=(n, n, n), workers=sampler._workers())
    return sampler.State(s=s_new, p_grid=p_new, sweep=state.sweep + 1)
