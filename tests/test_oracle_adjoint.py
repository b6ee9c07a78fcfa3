"""Pins of the oracle's Wiener-filter adjoint (oracle/adjoint.py).

The reverse-mode gradient is checked against two things it does not use:
central finite differences of the forward iteration, and, once the iteration
has converged, the dense closed forms of chi2 = d_o^T (S_oo + N_oo)^-1 d_o and
of its gradients with respect to d and to P_b.
"""
import numpy as np
import pytest

from oracle import adjoint, sampler, shells, wiener
from paper_1402_1763_amd import workloads


def _problem(n=8, n_bins=6, mask="random", seed=5):
    w = workloads.small_workload(n, n_bins, mask=mask, seed=seed, mask_frac=0.25)
    pb = workloads.make_problem(w)
    prob = sampler.make_problem(pb["data"], pb["noise_var"], n_bins, w.box, seed=1)
    return prob


def _p_grid(prob, scale):
    """Per-bin P (grid units) of a falling spectrum, scale * tau at the first bin."""
    return prob.tau * scale / (1.0 + np.arange(prob.n_bins)) ** 1.5


def test_gradient_matches_central_differences():
    prob = _problem()
    p = _p_grid(prob, 8.0)
    k = 25
    loss, gp, gd = adjoint.wf_gradient(prob, p, k)
    _, loss2 = adjoint.wf_forward(prob, p, k)
    assert loss == pytest.approx(loss2, rel=1e-14)
    counts = shells.mode_counts(prob.n, prob.n_bins)
    for b in range(prob.n_bins):
        if counts[b] == 0:
            assert gp[b] == 0.0
            continue
        h = 1e-3 * p[b]
        up, dn = p.copy(), p.copy()
        up[b] += h
        dn[b] -= h
        fd = (adjoint.wf_forward(prob, up, k)[1] - adjoint.wf_forward(prob, dn, k)[1]) / (2 * h)
        assert gp[b] == pytest.approx(fd, rel=2e-6, abs=1e-9 * np.abs(gp).max())
    rng = np.random.default_rng(0)
    obs = np.flatnonzero(prob.observed.ravel())
    masked = np.flatnonzero(~prob.observed.ravel())
    for i in list(rng.choice(obs, 8, replace=False)) + list(masked[:2]):
        h = 1e-3 * np.sqrt(np.mean(prob.data[prob.observed] ** 2))
        up, dn = prob.data.copy().ravel(), prob.data.copy().ravel()
        up[i] += h
        dn[i] -= h
        fu = adjoint.wf_forward(adjoint.with_data(prob, up.reshape(prob.data.shape)), p, k)[1]
        fl = adjoint.wf_forward(adjoint.with_data(prob, dn.reshape(prob.data.shape)), p, k)[1]
        fd = (fu - fl) / (2 * h)
        # chi2_K is quadratic in d: the central difference is exact up to rounding
        assert gd.ravel()[i] == pytest.approx(fd, rel=1e-7, abs=1e-9 * np.abs(gd).max())


@pytest.mark.parametrize("mask", ["random", "none"])
def test_converged_gradient_matches_dense_closed_form(mask):
    prob = _problem(n=8, n_bins=5, mask=mask, seed=9)
    p = _p_grid(prob, 1.0)     # f <= 1/2: the iteration contracts fast
    loss, gp, gd = adjoint.wf_gradient(prob, p, 120)
    o = prob.observed.ravel()
    s_full = wiener.signal_covariance(prob.n, wiener.full_grid_power(prob.n, prob.n_bins, p))
    a = s_full[np.ix_(o, o)] + np.diag(prob.noise_var.ravel()[o])
    d = prob.data.ravel()[o]
    x = np.linalg.solve(a, d)
    assert loss == pytest.approx(float(d @ x), rel=1e-10)
    assert np.allclose(gd.ravel()[o], 2.0 * x, rtol=0, atol=1e-9 * np.abs(x).max())
    assert np.all(gd.ravel()[~o] == 0.0)
    for b in range(prob.n_bins):
        ind = np.zeros(prob.n_bins)
        ind[b] = 1.0
        sb = wiener.signal_covariance(prob.n, wiener.full_grid_power(prob.n, prob.n_bins, ind))
        ref = -float(x @ sb[np.ix_(o, o)] @ x)
        assert gp[b] == pytest.approx(ref, rel=1e-8, abs=1e-10 * np.abs(gp).max())


def test_forward_converges_to_wiener_mean():
    prob = _problem(n=8, n_bins=5, seed=3)
    p = _p_grid(prob, 1.0)
    s_k, _ = adjoint.wf_forward(prob, p, 120)
    mean, _ = wiener.posterior(prob.n, prob.n_bins, p, prob.data, prob.noise_var)
    assert np.abs(s_k.ravel() - mean).max() < 1e-10 * np.abs(mean).max()
