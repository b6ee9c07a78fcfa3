"""GPU parity: the HIP sweep against the FP64 oracle on identical seeded
problems, through the C ABI.  Tolerances: 1e-10 in FP64 mode and 1e-4 in
FP32 mode after 10 sweeps (s metric relative to rms(s), P per bin)."""
import numpy as np
import pytest

from paper_1402_1763_amd import binding, workloads
from tests.gpu_util import TOL, errors, gpu_sampler, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()
    torch.cuda.set_device(0)


def _case(n, nbins, precision, mask, sweeps, sample_pk=True, seed=7, **kw):
    print(f"case n={n} bins={nbins} {precision} mask={mask} sweeps={sweeps} "
          f"sample_pk={sample_pk} seed={seed}", flush=True)
    w = workloads.small_workload(n, nbins, mask=mask, precision=precision, seed=seed,
                                 rng_seed=100 + seed, **kw)
    pb = workloads.make_problem(w)
    g = gpu_sampler(w, pb, sample_pk=sample_pk)
    g.sweep(sweeps)
    s_gpu, p_gpu, done = g.state()
    g.close()
    s_ref, p_ref = run_oracle(w, pb, sweeps, sample_pk=sample_pk)
    err_s, err_p = errors(s_gpu, p_gpu, s_ref, p_ref)
    print(f"  err_s={err_s:.3e} err_P={err_p:.3e}", flush=True)
    assert done == sweeps
    assert np.all(np.isfinite(s_gpu))
    return err_s, err_p


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_state_roundtrip(precision):
    n = 32
    w = workloads.small_workload(n, 8, precision=precision)
    pb = workloads.make_problem(w)
    s0 = np.random.default_rng(1).standard_normal((n,) * 3)
    g = gpu_sampler(w, pb, s_init=s0)
    s, p, done = g.state()
    g.close()
    tol = 1e-13 if precision == "fp64" else 2e-6
    assert np.abs(s - s0).max() < tol * np.abs(s0).max()
    assert np.allclose(p, pb["pk_init"], rtol=1e-14)
    assert done == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_z_and_y_transforms(precision):
    n = 16
    w = workloads.small_workload(n, 4, precision=precision)
    pb = workloads.make_problem(w)
    s0 = np.random.default_rng(2).standard_normal((n,) * 3)
    g = gpu_sampler(w, pb, s_init=s0)
    spec = binding.mf_debug_spectrum(g.handle, 0, n)
    ref = np.fft.rfft(s0, axis=2).transpose(2, 0, 1) / n      # [kz][ix][iy]
    tol = 1e-12 if precision == "fp64" else 1e-5
    scale = np.abs(ref).max()
    assert np.abs(spec - ref).max() < tol * scale
    binding.mf_debug_run_kernel(g.handle, 1, 0)                 # forward y-DFT
    spec_y = binding.mf_debug_spectrum(g.handle, 0, n)
    ref_y = np.fft.fft(ref, axis=2)
    assert np.abs(spec_y - ref_y).max() < tol * np.abs(ref_y).max()
    binding.mf_debug_run_kernel(g.handle, 3, 0)                 # inverse y-DFT
    spec_b = binding.mf_debug_spectrum(g.handle, 0, n)
    assert np.abs(spec_b / n - ref).max() < tol * scale
    g.close()


@pytest.mark.parametrize("n,nbins,mask", [(32, 16, "random"), (16, 8, "none"), (8, 4, "random"),
                                           (64, 16, "survey")])
def test_parity_fp64(n, nbins, mask):
    kw = {"box": 62.5 * n} if mask == "survey" else {}
    err_s, err_p = _case(n, nbins, "fp64", mask, 10, **kw)
    assert err_s < TOL["fp64"] and err_p < TOL["fp64"]


@pytest.mark.parametrize("n,nbins,mask", [(32, 16, "random"), (64, 16, "survey"),
                                           (128, 32, "survey"), (16, 5, "none")])
def test_parity_fp32(n, nbins, mask):
    kw = {"box": 1000.0 * n / 128, "nbar": 3e-4} if mask == "survey" else {}
    err_s, err_p = _case(n, nbins, "fp32", mask, 10, **kw)
    assert err_s < TOL["fp32"] and err_p < TOL["fp32"]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_parity_fixed_power(precision):
    err_s, err_p = _case(32, 8, precision, "random", 10, sample_pk=False)
    assert err_s < TOL[precision] and err_p == 0.0


def test_small_grid_many_bins():
    # 8^3 with as many bins as shells allow, including empty bins
    err_s, err_p = _case(8, 12, "fp64", "random", 6)
    assert err_s < TOL["fp64"] and err_p < TOL["fp64"]


def test_deterministic_repeat():
    w = workloads.small_workload(64, 16, mask="random", precision="fp32", seed=9)
    pb = workloads.make_problem(w)
    outs = []
    for _ in range(2):
        g = gpu_sampler(w, pb)
        g.sweep(5)
        outs.append(g.state())
        g.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("n,precision", [(48, "fp64"), (80, "fp64"), (96, "fp64"),
                                         (48, "fp32"), (80, "fp32"), (96, "fp32")])
def test_parity_mixed_radix_sizes(n, precision):
    """Grid sides with radix-3 and radix-5 factors (48 = 3 * 16, 80 = 5 * 16,
    96 = 6 * 16): random masks with 10-40% unobserved voxels."""
    err_s, err_p = _case(n, 16, precision, "random", 10, seed=n, mask_frac=0.1 + 0.3 * (n % 7) / 7)
    assert err_s < TOL[precision] and err_p < TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_single_bin(precision):
    w = workloads.small_workload(32, 1, mask="random", precision=precision, seed=131, rng_seed=132)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    smp.sweep(5)
    s_gpu, p_gpu, _ = smp.state()
    s_ref, p_ref = run_oracle(w, pb, 5)
    err_s, err_p = errors(s_gpu, p_gpu, s_ref, p_ref)
    print(f"single bin {precision}: err_s={err_s:.3e} err_P={err_p:.3e}", flush=True)
    assert err_s < TOL[precision] and err_p < TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_user_tau_below_the_smallest_noise(precision):
    w = workloads.small_workload(32, 8, mask="random", precision=precision, seed=133, rng_seed=134)
    pb = workloads.make_problem(w)
    tau = 0.3 * float(np.min(pb["noise_var"][np.isfinite(pb["noise_var"])]))
    smp = gpu_sampler(w, pb, tau=tau)
    assert smp.tau() == pytest.approx(tau, rel=1e-15)
    smp.sweep(5)
    s_gpu, p_gpu, _ = smp.state()
    s_ref, p_ref = run_oracle(w, pb, 5, tau=tau)
    err_s, err_p = errors(s_gpu, p_gpu, s_ref, p_ref)
    print(f"user tau {precision}: err_s={err_s:.3e} err_P={err_p:.3e}", flush=True)
    assert err_s < TOL[precision] and err_p < TOL[precision]
