"""Pins of the oracle's mixing sampler (oracle/mixing.py).

At fixed t^ the (x^, S^) update must leave the exact conditional of P
invariant: with Jeffreys' prior and the signal marginalised,
    p(P_b | t^) ~ P_b^-1 prod_{k in b} N(t^_k; 0, M (P_b + tau))
over the full-grid modes of bin b.  Its moments are computed by quadrature
and compared with long runs of the update.  With finite noise this density is
improper (its mass in ln P does not vanish as P -> 0); the bins used here hold
enough modes that the likelihood at P = 0 is below e^-40 of its peak, so the
region is never reached and the target is proper for all practical purposes.
The truncated-normal sampler is checked against scipy.stats.truncnorm.
"""
import numpy as np
import pytest
import scipy.integrate
import scipy.stats

from oracle import mixing, sampler, shells
from paper_1402_1763_amd import workloads


def _log_post(p, sum_t2, n_modes, m, tau, a0=0.0, b0=0.0):
    """ln of prior(P) prod_k N(t^_k; 0, M (P + tau)) up to a constant, with the
    InvGamma(a0, b0) prior P^-(a0+1) exp(-b0/P) (grid units; Jeffreys' at 0, 0)."""
    v = m * (p + tau)
    return -(a0 + 1.0) * np.log(p) - b0 / p - 0.5 * n_modes * np.log(v) - 0.5 * sum_t2 / v


def _quadrature_moments(sum_t2, n_modes, m, tau, a0=0.0, b0=0.0):
    """E[ln P] and Var[ln P] under p(P | t^), integrating over y = ln P."""
    y = np.linspace(-12, 12, 200001)
    p = np.exp(y)
    lp = _log_post(p, sum_t2, n_modes, m, tau, a0, b0) + y          # density in y
    w = np.exp(lp - lp.max())
    z = scipy.integrate.trapezoid(w, y)
    mean = scipy.integrate.trapezoid(w * y, y) / z
    var = scipy.integrate.trapezoid(w * (y - mean) ** 2, y) / z
    return mean, var


def _fixed_t_problem(n=8, n_bins=3, seed=3, prior=(0.0, 0.0)):
    w = workloads.small_workload(n, n_bins, mask="none", seed=seed, sigma2=1.0, box=15.625 * n)
    pb = workloads.make_problem(w)
    prob = sampler.make_problem(pb["data"], np.full((n,) * 3, 1.0), n_bins, w.box, seed=9,
                                prior=prior)
    rng = np.random.default_rng(seed)
    t = rng.standard_normal((n,) * 3) * 1.7          # a messenger field of variance ~ P + tau
    return prob, np.fft.rfftn(t)


def _run(prob, t_hat, p0, iters, accept_rule=None):
    p = np.array(p0, dtype=np.float64)
    logs = np.empty((iters, prob.n_bins))
    for it in range(iters):
        s_hat = sampler.signal_step(t_hat, p, prob, it)
        if accept_rule is None:
            p, _ = mixing.mix_power_step(s_hat, t_hat, p, prob, it)
        else:
            p = accept_rule(s_hat, t_hat, p, prob, it)
        logs[it] = np.log(p)
    return logs


def _rule(kind):
    """Negative controls: the printed acceptance min(1, (U'/U)^2), or
    accepting every proposal (a flat prior in U)."""
    def step(s_hat, t_hat, p, prob, sweep):
        m = prob.m
        b_of = shells.bin_of_q(shells.half_grid_q(prob.n), prob.n, prob.n_bins)
        root_s = np.sqrt(m * p)
        x_hat = np.where(b_of >= 0, s_hat / root_s[np.maximum(b_of, 0)], 0.0)
        xx, xt = mixing.shell_sums(x_hat, t_hat, prob)
        out = p.copy()
        for b in range(prob.n_bins):
            u_new, u_mh = mixing.truncated_normal(xt[b] / xx[b], np.sqrt(m * prob.tau / xx[b]),
                                                  prob.seed, prob.chain, sweep, b)
            ok = u_mh <= (u_new / root_s[b]) ** 2 if kind == "squared" else True
            if u_new is not None and ok:
                out[b] = u_new * u_new / m
        return out
    return step


def _check(logs, prob, t_hat):
    n = prob.n
    b_of = shells.bin_of_q(shells.half_grid_q(n), n, prob.n_bins)
    w = np.broadcast_to(shells.half_grid_weight(n)[None, None, :], b_of.shape)
    counts = shells.mode_counts(n, prob.n_bins)
    burn = 200
    z_scores = []
    for b in range(prob.n_bins):
        sel = b_of == b
        sum_t2 = float(np.sum((np.abs(t_hat) ** 2 * w)[sel]))
        mean, var = _quadrature_moments(sum_t2, counts[b], prob.m, prob.tau, prob.prior_shape,
                                        prob.prior_scale / prob.cell_volume)
        x = logs[burn:, b]
        batches = x[: len(x) // 50 * 50].reshape(50, -1).mean(axis=1)
        se = batches.std(ddof=1) / np.sqrt(50)
        z_scores.append((x.mean() - mean) / se)
        assert x.var() == pytest.approx(var, rel=0.15)
    return np.array(z_scores)


ITERS = 20000    # the correct rule stays within |z| < 1 here; the controls reach 6 to 25


# a proper InvGamma prior strong enough to move the conditional: b0 of 1.2
# in grid units against sum |t^|^2 / (M n_b) of about 3
PROPER_PRIOR = (2.0, 1.2 * 15.625 ** 3)


@pytest.mark.parametrize("prior", [(0.0, 0.0), PROPER_PRIOR])
def test_mixing_update_leaves_the_exact_conditional_invariant(prior):
    prob, t_hat = _fixed_t_problem(prior=prior)
    logs = _run(prob, t_hat, [1.0] * prob.n_bins, ITERS)
    z = _check(logs, prob, t_hat)
    print("z-scores", z)
    assert np.all(np.abs(z) < 4.0)


def test_jeffreys_rule_fails_under_a_proper_prior():
    """The prior enters the acceptance: Jeffreys' rule U/U' run on a problem
    with the proper prior misses that prior's conditional."""
    prob, t_hat = _fixed_t_problem(prior=PROPER_PRIOR)
    jeffreys = _fixed_t_problem()[0]

    def step(s_hat, t_hat, p, prob_, sweep):
        return mixing.mix_power_step(s_hat, t_hat, p, jeffreys, sweep)[0]
    logs = _run(prob, t_hat, [1.0] * prob.n_bins, ITERS, accept_rule=step)
    with pytest.raises(AssertionError):
        z = _check(logs, prob, t_hat)
        assert np.all(np.abs(z) < 4.0)


@pytest.mark.parametrize("kind", ["squared", "always"])
def test_other_acceptance_rules_fail_the_same_check(kind):
    prob, t_hat = _fixed_t_problem()
    logs = _run(prob, t_hat, [1.0] * prob.n_bins, ITERS, accept_rule=_rule(kind))
    with pytest.raises(AssertionError):
        z = _check(logs, prob, t_hat)
        assert np.all(np.abs(z) < 4.0)


@pytest.mark.parametrize("mean,sd", [(1.0, 1.0), (-0.6, 1.0), (-2.5, 0.8), (-7.0, 1.5)])
def test_truncated_normal_matches_scipy(mean, sd):
    draws = []
    for sweep in range(4000):
        u, _ = mixing.truncated_normal(mean, sd, seed=5, chain=0, sweep=sweep, b=1)
        assert u is not None and u > 0.0
        draws.append(u)
    ref = scipy.stats.truncnorm(-mean / sd, np.inf, loc=mean, scale=sd)
    assert scipy.stats.kstest(draws, ref.cdf).pvalue > 1e-3
