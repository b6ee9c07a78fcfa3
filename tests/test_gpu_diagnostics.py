"""GPU tests of the chain diagnostics: recorded P traces and Welford posterior
moments against the oracle chain, and the autocorrelation kernel against the
oracle's Eq. CORR_COEFF."""
import numpy as np
import pytest

from oracle import diagnostics, sampler
from paper_1402_1763_amd import binding, workloads
from tests.gpu_util import TOL, gpu_sampler, oracle_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()
    torch.cuda.set_device(0)


def _oracle_samples(w, pb, n_sweeps, keep):
    prob = oracle_problem(w, pb)
    st = sampler.State(s=np.zeros((w.n,) * 3), p_grid=pb["pk_init"] / w.cell_volume)
    out = {}
    for n in range(n_sweeps + 1):
        if n in keep:
            out[n] = (st.s.copy(), st.p_grid * w.cell_volume)
        if n < n_sweeps:
            st = sampler.sweep(prob, st)
    return out


@pytest.mark.parametrize("precision,n", [("fp64", 32), ("fp32", 48)])
def test_trace_and_moments_match_oracle(precision, n):
    import torch
    w = workloads.small_workload(n, 8, precision=precision, seed=61, rng_seed=62)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    start, thin, sweeps = 2, 3, 14
    smp.set_diagnostics(start=start, thin=thin, trace_cap=10, moments=True)
    smp.sweep(sweeps)
    keep = list(range(start, sweeps, thin))
    assert smp.recorded() == len(keep) == 4
    trace = smp.trace().cpu().numpy()
    mean, var = (t.cpu().numpy() for t in smp.moments())
    torch.cuda.synchronize()
    ref = _oracle_samples(w, pb, sweeps, keep)
    p_ref = np.stack([ref[k][1] for k in keep])
    m_ref, v_ref = diagnostics.moments([ref[k][0] for k in keep])
    e_p = float(np.max(np.abs(trace - p_ref) / p_ref))
    rms = np.sqrt(np.mean(m_ref ** 2))
    e_m = float(np.abs(mean - m_ref).max() / rms)
    e_v = float(np.abs(var - v_ref).max() / np.mean(v_ref))
    print(f"diag n={n} {precision}: err trace={e_p:.2e} mean={e_m:.2e} var={e_v:.2e}", flush=True)
    tol = TOL[precision]
    assert e_p < tol and e_m < tol and e_v < tol


def test_acf_kernel_matches_oracle():
    import torch
    rng = np.random.default_rng(4)
    t, nb = 3000, 5
    x = np.empty((t, nb))
    x[0] = rng.standard_normal(nb)
    phi = np.array([0.0, 0.3, 0.6, 0.9, 0.97])
    for i in range(1, t):
        x[i] = phi * x[i - 1] + rng.standard_normal(nb)
    x = 10.0 + x
    c, nc = binding.acf(torch.from_numpy(x).cuda(), 120)
    c_ref, nc_ref = diagnostics.acf_bins(x, 120)
    err = float(np.abs(c.cpu().numpy() - c_ref).max())
    print(f"acf err={err:.2e} nc={nc.cpu().numpy()} ref={nc_ref}", flush=True)
    assert err < 1e-12
    assert np.array_equal(nc.cpu().numpy(), nc_ref)


def test_graph_replays_record_too():
    w = workloads.small_workload(32, 8, precision="fp32", seed=71, rng_seed=72)
    pb = workloads.make_problem(w)
    a, b = gpu_sampler(w, pb), gpu_sampler(w, pb)
    for smp in (a, b):
        smp.set_diagnostics(start=0, thin=2, trace_cap=8, moments=True)
    a.sweep(9)
    g = binding.SweepGraph([b])
    g.launch(9)
    g.close()
    assert a.recorded() == b.recorded() == 5
    assert np.array_equal(a.trace().cpu().numpy(), b.trace().cpu().numpy())
    ma, va = a.moments()
    mb, vb = b.moments()
    assert np.array_equal(ma.cpu().numpy(), mb.cpu().numpy())
    assert np.array_equal(va.cpu().numpy(), vb.cpu().numpy())


def test_diagnostic_errors():
    w = workloads.small_workload(16, 4, precision="fp32")
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    with pytest.raises(binding.MFError):
        smp.moments()                    # no buffer set
    smp.set_diagnostics(start=5, thin=1, moments=True)
    smp.sweep(3)
    with pytest.raises(binding.MFError) as e:
        smp.moments()                    # nothing recorded yet
    assert e.value.status == binding.MF_E_STATE
    with pytest.raises(binding.MFError):
        smp.set_diagnostics(start=0, thin=0, trace_cap=2)


def test_gpu_fixed_power_moments_match_the_dense_posterior():
    """End-to-end statistics on the GPU: 8 chains at fixed P on an 8^3 grid,
    Welford moments over 20,000 sweeps each, against the dense Cholesky
    posterior mean and variance (the Wiener posterior the sampler targets)."""
    from oracle import wiener
    w = workloads.small_workload(8, 4, mask="random", precision="fp64", seed=141, rng_seed=142,
                                 mask_frac=0.3)
    pb = workloads.make_problem(w)
    p_grid = workloads.power_spectrum(workloads.bin_centres(w), w) / w.cell_volume
    chains = 8
    smp = binding.Sampler([pb["data"]] * chains, [pb["noise_var"]] * chains,
                          [p_grid * w.cell_volume] * chains, w.n_bins, w.box, seed=143,
                          precision="fp64", sample_pk=False)
    smp.set_diagnostics(start=200, thin=1, moments=True)
    smp.sweep(20_200)
    means = np.stack([smp.moments(c)[0].cpu().numpy().ravel() for c in range(chains)])
    vars_ = np.stack([smp.moments(c)[1].cpu().numpy().ravel() for c in range(chains)])
    mean_ref, cov_ref = wiener.posterior(8, w.n_bins, p_grid, pb["data"], pb["noise_var"])
    var_ref = np.diag(cov_ref)
    se = means.std(axis=0, ddof=1) / np.sqrt(chains)
    z = (means.mean(axis=0) - mean_ref) / se
    ratio = vars_.mean(axis=0) / var_ref
    print(f"posterior moments: mean z^2 {np.mean(z ** 2):.3f} (t_7: 1.4), "
          f"variance ratio {ratio.mean():.4f} +- {ratio.std():.4f}", flush=True)
    assert abs(np.mean(z)) < 0.3 and 0.7 < np.mean(z ** 2) < 2.3
    assert abs(ratio.mean() - 1.0) < 0.02
