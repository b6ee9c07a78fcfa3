"""Pins of the oracle with a general diagonal response R (data model
d = R s + eps of Sec. 2, messenger conditional of Sec. 3.1 with its R_i
terms, tau bound [(R^-1)^T N R^-1]_i).

* noise-free iteration   -> dense Wiener mean S R (R S R + N)^-1 d
* messenger step         -> its two limits (N~ = 0 gives t = d / R exactly;
                            R = 0 gives t ~ N(s, tau))
* fixed-P chain          -> dense posterior mean and variance with R (MC error)
* rescaling              -> (d, N, R) and (d / R, N / R^2, 1) give the same chain
* Wiener-filter adjoint  -> central differences, and the dense closed forms of
                            d^T (R S R + N)^-1 d and of its gradients
"""
import numpy as np
import pytest

from oracle import adjoint, sampler, shells, wiener
from paper_1402_1763_amd import workloads


def _problem(n, n_bins, seed=7, zero_frac=0.1, mask="random", **kw):
    """A small problem with a response R in [0.3, 1.7], R = 0 on a random
    zero_frac of the voxels, and data R d0 with d0 the workload's data."""
    w = workloads.small_workload(n, n_bins, mask=mask, precision="fp64", seed=seed, **kw)
    pb = workloads.make_problem(w)
    rng = np.random.default_rng(seed + 100)
    r = rng.uniform(0.3, 1.7, (n,) * 3)
    r[rng.random((n,) * 3) < zero_frac] = 0.0
    data = np.where(np.isfinite(pb["noise_var"]), r * pb["data"], 0.0)
    prob = sampler.make_problem(data, pb["noise_var"], n_bins, w.box, seed=1234 + seed, response=r)
    return w, prob


def _batch_z(samples, target, n_batches):
    nb = len(samples) // n_batches
    means = samples[: nb * n_batches].reshape(n_batches, nb, -1).mean(axis=1)
    se = means.std(axis=0, ddof=1) / np.sqrt(n_batches)
    return (means.mean(axis=0) - target) / se


def test_tau_is_smallest_noise_over_response_squared():
    _, prob = _problem(8, 4)
    o = prob.observed
    assert np.all(prob.response[~o & np.isfinite(prob.noise_var)] == 0.0)
    assert prob.tau == np.min(prob.noise_var[o] / prob.response[o] ** 2)
    with pytest.raises(ValueError):
        sampler.make_problem(prob.data, prob.noise_var, 4, 500.0, 1, tau=1.01 * prob.tau,
                             response=prob.response)


def test_noise_free_iteration_reaches_wiener_mean_with_response():
    _, prob = _problem(8, 4)
    p_grid = np.array([40.0, 12.0, 5.0, 2.0]) * prob.tau
    mean, _ = wiener.posterior(8, 4, p_grid, prob.data, prob.noise_var, response=prob.response)
    st = sampler.run_chain(prob, sampler.State(s=np.zeros((8,) * 3), p_grid=p_grid), 3000,
                           noise=False)
    err = np.abs(st.s.ravel() - mean).max() / np.sqrt(np.mean(mean ** 2))
    assert err < 1e-10


def test_messenger_step_limits_with_response():
    _, prob = _problem(8, 4)
    s = np.random.default_rng(0).standard_normal((8,) * 3)
    mu, var = sampler.messenger_moments(s, prob)
    o, r = prob.observed, prob.response
    i = np.unravel_index(np.argmin(np.where(o, prob.noise_var / np.where(o, r, 1.0) ** 2, np.inf)),
                         s.shape)
    assert var[i] == 0.0
    assert mu[i] == pytest.approx(prob.data[i] / r[i], rel=1e-14)
    zero = (r == 0.0)
    assert zero.any()
    assert np.all(mu[zero] == s[zero]) and np.all(var[zero] == prob.tau)
    # observed: t interpolates d / R and s with weight tau R^2 / N
    wgt = prob.tau * r[o] ** 2 / prob.noise_var[o]
    assert np.allclose(mu[o], wgt * prob.data[o] / r[o] + (1 - wgt) * s[o], rtol=0, atol=1e-12)
    assert np.allclose(var[o], prob.tau * (1 - wgt), rtol=1e-12, atol=0)


def test_augmented_noise_stays_non_negative_at_the_tau_voxel():
    """With tau = N / R^2 of the minimising voxel, N - tau R^2 is 0 in exact
    arithmetic but rounds to -1 ulp for this (N, R) pair: the messenger
    variance there must come out 0, not negative."""
    n = 8
    nv = np.full((n,) * 3, 2.0)
    r = np.ones((n,) * 3)
    nv[3, 4, 5], r[3, 4, 5] = 0.5002257126660961, 1.6887569038041037
    tau = nv[3, 4, 5] / r[3, 4, 5] ** 2
    assert nv[3, 4, 5] - tau * r[3, 4, 5] * r[3, 4, 5] < 0.0   # the rounding case
    d = np.random.default_rng(1).standard_normal((n,) * 3)
    prob = sampler.make_problem(d, nv, 4, 500.0, 1, response=r)
    assert prob.tau == tau
    mu, var = sampler.messenger_moments(np.zeros((n,) * 3), prob)
    assert np.all(var >= 0.0) and var[3, 4, 5] == 0.0
    assert mu[3, 4, 5] == pytest.approx(d[3, 4, 5] / r[3, 4, 5], rel=1e-15)
    st = sampler.run_chain(prob, sampler.State(s=np.zeros((n,) * 3), p_grid=np.ones(4)), 2)
    assert np.all(np.isfinite(st.s)) and np.all(np.isfinite(st.p_grid))


@pytest.mark.slow
def test_fixed_power_chain_matches_dense_posterior_with_response():
    n, nbins = 8, 4
    _, prob = _problem(n, nbins, seed=21)
    p_grid = np.array([4.0, 3.0, 2.0, 1.0]) * prob.tau
    mean, cov = wiener.posterior(n, nbins, p_grid, prob.data, prob.noise_var,
                                 response=prob.response)
    st = sampler.State(s=mean.reshape((n,) * 3).copy(), p_grid=p_grid)
    samples = []
    for _ in range(6000):
        st = sampler.sweep(prob, st, sample_pk=False)
        samples.append(st.s.ravel())
    samples = np.array(samples)
    z = _batch_z(samples, mean, 60)
    assert 0.75 < np.mean(z ** 2) < 1.35
    assert np.max(np.abs(z)) < 4.8
    zv = _batch_z((samples - mean) ** 2, np.diag(cov), 60)
    assert 0.6 < np.mean(zv ** 2) < 1.6
    assert np.max(np.abs(zv)) < 5.0


def test_rescaled_problem_gives_the_same_chain():
    """d = R s + eps with noise N is the same likelihood for s as
    d / R = s + eps / R with noise N / R^2 on every observed voxel: the
    messenger coefficients, tau and hence every draw coincide."""
    n, nbins = 16, 6
    w, prob = _problem(n, nbins, seed=31)
    o = prob.observed
    r = prob.response
    d2 = np.where(o, prob.data / np.where(o, r, 1.0), 0.0)
    nv2 = np.where(o, prob.noise_var / np.where(o, r, 1.0) ** 2, np.inf)
    prob2 = sampler.make_problem(d2, nv2, nbins, w.box, seed=prob.seed)
    assert prob2.tau == pytest.approx(prob.tau, rel=1e-15)
    p0 = workloads.power_spectrum(workloads.bin_centres(w), w) / w.cell_volume
    a = sampler.run_chain(prob, sampler.State(s=np.zeros((n,) * 3), p_grid=p0), 6)
    b = sampler.run_chain(prob2, sampler.State(s=np.zeros((n,) * 3), p_grid=p0), 6)
    assert np.abs(a.s - b.s).max() < 1e-11 * np.sqrt(np.mean(a.s ** 2))
    assert np.max(np.abs(a.p_grid / b.p_grid - 1.0)) < 1e-11
    # the same identity fails when R enters the messenger with the wrong power
    wrong = sampler.make_problem(prob.data, prob.noise_var, nbins, w.box, seed=prob.seed,
                                 response=np.sqrt(np.abs(r)))
    c = sampler.run_chain(wrong, sampler.State(s=np.zeros((n,) * 3), p_grid=p0), 6)
    assert np.abs(a.s - c.s).max() > 1e-3 * np.sqrt(np.mean(a.s ** 2))


def _p_grid(prob, scale):
    return prob.tau * scale / (1.0 + np.arange(prob.n_bins)) ** 1.5


def test_adjoint_with_response_matches_central_differences():
    _, prob = _problem(8, 6, seed=5)
    p = _p_grid(prob, 8.0)
    k = 25
    loss, gp, gd = adjoint.wf_gradient(prob, p, k)
    counts = shells.mode_counts(prob.n, prob.n_bins)
    for b in range(prob.n_bins):
        if counts[b] == 0:
            continue
        h = 1e-3 * p[b]
        up, dn = p.copy(), p.copy()
        up[b] += h
        dn[b] -= h
        fd = (adjoint.wf_forward(prob, up, k)[1] - adjoint.wf_forward(prob, dn, k)[1]) / (2 * h)
        assert gp[b] == pytest.approx(fd, rel=2e-6, abs=1e-9 * np.abs(gp).max())
    rng = np.random.default_rng(0)
    obs = np.flatnonzero(prob.observed.ravel())
    for i in list(rng.choice(obs, 8, replace=False)) + list(np.flatnonzero(~prob.observed.ravel())[:2]):
        h = 1e-3 * np.sqrt(np.mean(prob.data[prob.observed] ** 2))
        up, dn = prob.data.copy().ravel(), prob.data.copy().ravel()
        up[i] += h
        dn[i] -= h
        fu = adjoint.wf_forward(adjoint.with_data(prob, up.reshape(prob.data.shape)), p, k)[1]
        fl = adjoint.wf_forward(adjoint.with_data(prob, dn.reshape(prob.data.shape)), p, k)[1]
        assert gd.ravel()[i] == pytest.approx((fu - fl) / (2 * h), rel=1e-7,
                                             abs=1e-9 * np.abs(gd).max())


def test_converged_adjoint_with_response_matches_dense_closed_form():
    _, prob = _problem(8, 5, seed=9)
    p = _p_grid(prob, 1.0)
    loss, gp, gd = adjoint.wf_gradient(prob, p, 150)
    o = prob.observed.ravel()
    r = prob.response.ravel()[o]
    s_full = wiener.signal_covariance(prob.n, wiener.full_grid_power(prob.n, prob.n_bins, p))
    a = r[:, None] * s_full[np.ix_(o, o)] * r[None, :] + np.diag(prob.noise_var.ravel()[o])
    d = prob.data.ravel()[o]
    x = np.linalg.solve(a, d)
    assert loss == pytest.approx(float(d @ x), rel=1e-10)
    assert np.allclose(gd.ravel()[o], 2.0 * x, rtol=0, atol=1e-9 * np.abs(x).max())
    assert np.all(gd.ravel()[~o] == 0.0)
    for b in range(prob.n_bins):
        ind = np.zeros(prob.n_bins)
        ind[b] = 1.0
        sb = wiener.signal_covariance(prob.n, wiener.full_grid_power(prob.n, prob.n_bins, ind))
        ref = -float((r * x) @ sb[np.ix_(o, o)] @ (r * x))
        assert gp[b] == pytest.approx(ref, rel=1e-8, abs=1e-10 * np.abs(gp).max())
