"""Pins of the oracle's log-determinant trace estimator (oracle/logdet.py)
against dense linear algebra that does not go through the messenger field.

* one probe, converged filter -> dense z^T A^-1 R S_b R N^-1 z
* probe average              -> dense tr(A^-1 R S_b R) within Monte Carlo error
* dense trace                -> central differences of the dense ln det A
* probe signs                -> +-1, balanced, independent across probes and chains
* -1/2 (d chi2/d P + T)      -> a score: zero mean over data drawn at the true P,
                                negative at twice the true P
"""
import numpy as np
import pytest

from oracle import logdet, sampler
from paper_1402_1763_amd import workloads


def _problem(n=8, n_bins=5, seed=9, response=False, mask="random"):
    w = workloads.small_workload(n, n_bins, mask=mask, seed=seed, mask_frac=0.25)
    pb = workloads.make_problem(w)
    r = None
    data = pb["data"]
    if response:
        rng = np.random.default_rng(seed + 7)
        r = rng.uniform(0.3, 1.7, (n,) * 3) * np.where(rng.random((n,) * 3) < 0.2, -1.0, 1.0)
        r[rng.random((n,) * 3) < 0.1] = 0.0
        data = r * pb["data"]
    return sampler.make_problem(data, pb["noise_var"], n_bins, w.box, seed=seed + 100, response=r)


def _p_grid(prob, scale):
    return prob.tau * scale / (1.0 + np.arange(prob.n_bins)) ** 1.5


@pytest.mark.parametrize("response", [False, True])
def test_single_probe_matches_dense_form(response):
    prob = _problem(response=response)
    p = _p_grid(prob, 1.0)     # f <= 1/2: the filter converges fast
    for j in (0, 3):
        est = logdet.trace_probe(prob, p, 150, j)
        ref = logdet.dense_probe(prob, p, j)
        assert np.allclose(est, ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max()), (est, ref)


def test_probe_average_matches_dense_trace():
    prob = _problem(n=8, n_bins=4, seed=13, response=True)
    p = _p_grid(prob, 1.0)
    samples = np.array([logdet.trace_probe(prob, p, 60, j) for j in range(240)])
    ref = logdet.dense_trace(prob, p)
    se = samples.std(axis=0, ddof=1) / np.sqrt(len(samples))
    z = (samples.mean(axis=0) - ref) / se
    assert np.all(np.abs(z) < 4.0), z
    assert np.all(np.abs(samples.mean(axis=0) - ref) < 0.1 * np.abs(ref))
    # the estimator is noisy per probe but not degenerate
    assert np.all(samples.std(axis=0) > 0.05 * np.abs(ref))


@pytest.mark.parametrize("response", [False, True])
def test_dense_trace_is_the_logdet_derivative(response):
    prob = _problem(n=8, n_bins=5, seed=17, response=response)
    p = _p_grid(prob, 3.0)
    tr = logdet.dense_trace(prob, p)
    for b in range(prob.n_bins):
        h = 1e-4 * p[b]
        up, dn = p.copy(), p.copy()
        up[b] += h
        dn[b] -= h
        fd = (logdet.dense_logdet(prob, up) - logdet.dense_logdet(prob, dn)) / (2 * h)
        assert tr[b] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(tr).max())


def test_probe_signs_are_balanced_and_independent():
    n = 32
    m = n ** 3
    a = logdet.probe_signs(n, 5, 0, 0)
    b = logdet.probe_signs(n, 5, 0, 1)
    c = logdet.probe_signs(n, 5, 1, 0)
    for x in (a, b, c):
        assert set(np.unique(x)) == {-1.0, 1.0}
        assert abs(x.mean()) < 4.0 / np.sqrt(m)
    for x, y in ((a, b), (a, c)):
        assert abs(np.mean(x * y)) < 4.0 / np.sqrt(m)
    # neighbouring voxels (same Philox call, different words) are independent too
    flat = a.ravel()
    assert abs(np.mean(flat[0::4] * flat[1::4])) < 4.0 / np.sqrt(m / 4)


def _score_data(n, p_grid, mask, seed):
    """d = s + eps with s Gaussian of bin-constant power p_grid (grid units)
    and unit white noise on the observed voxels."""
    from oracle import shells
    rng = np.random.default_rng(seed)
    b = shells.bin_of_q(shells.half_grid_q(n), n, len(p_grid))
    pm = np.where(b >= 0, np.asarray(p_grid)[np.maximum(b, 0)], 0.0)
    s = np.fft.irfftn(np.fft.rfftn(rng.standard_normal((n,) * 3)) * np.sqrt(pm), s=(n,) * 3,
                      axes=(0, 1, 2))
    return np.where(mask, 0.0, s + rng.standard_normal((n,) * 3))


@pytest.mark.slow
def test_likelihood_gradient_is_a_score():
    """-1/2 (d chi2/d P + T) is the gradient of ln L: over data drawn at the
    true P its mean is zero, and at twice the true P it points down."""
    from oracle import adjoint
    n, k, probes, reals = 16, 120, 16, 8
    p_true = np.array([6.0, 4.0, 2.5, 1.5])
    mask = np.random.default_rng(0).random((n,) * 3) < 0.25
    nv = np.where(mask, np.inf, 1.0)
    z = {}
    for scale in (1.0, 2.0):
        g = []
        for r in range(reals):
            prob = sampler.make_problem(_score_data(n, p_true, mask, 100 + r), nv, 4, 250.0, seed=5)
            _, gp, _ = adjoint.wf_gradient(prob, scale * p_true, k)
            g.append(-0.5 * (gp + logdet.trace_estimate(prob, scale * p_true, k, range(probes))))
        g = np.array(g)
        z[scale] = g.mean(axis=0) / (g.std(axis=0, ddof=1) / np.sqrt(reals))
    assert np.all(np.abs(z[1.0]) < 4.0), z
    assert np.all(z[2.0] < -5.0), z
