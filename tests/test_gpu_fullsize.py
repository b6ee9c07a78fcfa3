"""GPU parity on the canonical workloads, including the benchmarked 256^3
FP32 problem in the launch configuration bench.py times.

The oracle runs every sweep in FP64 on the host (scipy.fft with all host
cores), so the 256^3 case costs tens of seconds of CPU while the GPU idles.
"""
import os

import numpy as np
import pytest

from paper_1402_1763_amd import binding, workloads
from tests.gpu_util import TOL, errors, oracle_problem, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()
    torch.cuda.set_device(0)
    os.environ.setdefault("ORACLE_FFT_WORKERS", str(min(16, len(os.sched_getaffinity(0)))))


def _sampler(w, pb):
    return binding.Sampler(pb["data"], pb["noise_var"], pb["pk_init"], w.n_bins, w.box,
                           seed=w.rng_seed, precision=w.precision)


@pytest.mark.parametrize("name", ["gibbs-32^3-fp64", "gibbs-128^3-fp32-survey"])
def test_canonical_ten_sweeps(name):
    w = workloads.WORKLOADS[name]
    pb = workloads.make_problem(w)
    print(f"workload {name}: 10 sweeps", flush=True)
    g = _sampler(w, pb)
    g.sweep(10)
    s_gpu, p_gpu, done = g.state()
    g.close()
    s_ref, p_ref = run_oracle(w, pb, 10)
    err_s, err_p = errors(s_gpu, p_gpu, s_ref, p_ref)
    print(f"  err_s={err_s:.3e} err_P={err_p:.3e}", flush=True)
    assert done == 10
    assert err_s < TOL[w.precision] and err_p < TOL[w.precision]


@pytest.mark.timeout(600)
def test_benchmark_problem_ten_sweeps():
    """256^3, 64 bins, survey mask: 10 sweeps of the HIP path against 10 FP64
    oracle sweeps from the same initial state (s = 0, P = 0.1 x truth)."""
    w = workloads.SURVEY_256_MIXED
    pb = workloads.make_problem(w)
    print("256^3 benchmark problem: GPU 10 sweeps", flush=True)
    g = _sampler(w, pb)
    g.sweep(10)
    s_gpu, p_gpu, done = g.state()
    g.close()
    from oracle import sampler
    prob = oracle_problem(w, pb)
    st = sampler.State(s=np.zeros((w.n,) * 3), p_grid=pb["pk_init"] / w.cell_volume)
    for i in range(10):
        st = sampler.sweep(prob, st)
        print(f"  oracle sweep {i} done", flush=True)
    err_s, err_p = errors(s_gpu, p_gpu, st.s, st.p_grid * w.cell_volume)
    print(f"  err_s={err_s:.3e} err_P={err_p:.3e}", flush=True)
    assert done == 10
    assert err_s < TOL["fp32"] and err_p < TOL["fp32"]


@pytest.mark.timeout(300)
def test_benchmark_problem_sweep_from_gpu_state():
    """After 30 GPU sweeps, one more GPU sweep against one oracle sweep started
    from the GPU's own state (s read back, P read back, same sweep index)."""
    w = workloads.SURVEY_256_MIXED
    pb = workloads.make_problem(w)
    g = _sampler(w, pb)
    g.sweep(30)
    s30, p30, n30 = g.state()
    g.sweep(1)
    s31, p31, n31 = g.state()
    g.close()
    assert (n30, n31) == (30, 31)
    s_ref, p_ref = run_oracle(w, pb, 1, s0=s30, p0=p30, first_sweep=30)
    err_s, err_p = errors(s31, p31, s_ref, p_ref)
    print(f"  sweep 31 from GPU state: err_s={err_s:.3e} err_P={err_p:.3e}", flush=True)
    assert err_s < TOL["fp32"] and err_p < TOL["fp32"]
    assert np.all(np.isfinite(p31)) and np.all(p31 > 0)


@pytest.mark.timeout(600)
def test_largest_grid_one_sweep():
    """512^3 (three-stage transforms, whole-transform x-pass): one sweep from a
    random initial field against one oracle sweep."""
    w = workloads.Workload("test-512^3", n=512, box=4000.0, n_bins=32, mask="random",
                           mask_frac=0.2, precision="fp32", seed=5, rng_seed=9)
    pb = workloads.make_problem(w)
    s0 = np.random.default_rng(6).standard_normal((w.n,) * 3) * 3.0
    print("512^3: GPU sweep", flush=True)
    g = binding.Sampler(pb["data"], pb["noise_var"], pb["pk_init"], w.n_bins, w.box,
                        seed=w.rng_seed, precision=w.precision, s_init=s0)
    g.sweep(1)
    s_gpu, p_gpu, done = g.state()
    g.close()
    print("512^3: oracle sweep", flush=True)
    s_ref, p_ref = run_oracle(w, pb, 1, s0=s0)
    err_s, err_p = errors(s_gpu, p_gpu, s_ref, p_ref)
    print(f"  err_s={err_s:.3e} err_P={err_p:.3e}", flush=True)
    assert done == 1 and err_s < TOL["fp32"] and err_p < TOL["fp32"]
