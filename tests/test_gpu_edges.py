"""GPU edge cases: zero sweeps, and the largest bin count (1024 bins, most of
them empty at small |k|) on the 256^3 grid, where the FP64 shell histograms
need the most LDS (one copy per wave instead of 8, 33 KB per x-pass
workgroup for an FP32 Gibbs sweep and 66 KB for an FP64 mixing sweep);
the sweep-index bound; mixing sweeps with P held fixed; diagnostics under a
live graph."""
import numpy as np
import pytest

from oracle import mixing, sampler, shells
from paper_1402_1763_amd import binding, workloads
from tests.gpu_util import TOL, errors, gpu_sampler, oracle_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()
    torch.cuda.set_device(0)


def test_zero_sweeps_leave_the_state_alone():
    w = workloads.small_workload(32, 8, precision="fp64", seed=81, rng_seed=82)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    s0 = np.random.default_rng(3).standard_normal((32,) * 3)
    smp.set_state(0, s0, pb["pk_init"], 0)
    smp.sweep(0)
    smp.mixing_sweep(0)
    s, pk, n_done = smp.state()
    smp.close()
    assert n_done == 0
    assert np.abs(s - s0).max() < 1e-12 * np.abs(s0).max()     # up to the z-transform round trip
    assert np.allclose(pk, pb["pk_init"], rtol=1e-15, atol=0)


def _max_bins_problem(precision):
    n, nb = 256, 1024
    w = workloads.small_workload(n, nb, precision=precision, seed=91, rng_seed=92, box=2000.0)
    pb = workloads.make_problem(w)
    counts = shells.mode_counts(n, nb)
    assert (counts == 0).sum() > 0 and counts.sum() == n ** 3 - 1
    return w, pb, counts


def test_maximum_bins_gibbs_fp32():
    w, pb, counts = _max_bins_problem("fp32")
    print(f"1024 bins at 256^3 FP32: {(counts == 0).sum()} empty bins", flush=True)
    smp = gpu_sampler(w, pb)
    smp.sweep(2)
    s_gpu, p_gpu, _ = smp.state()
    smp.close()
    prob = oracle_problem(w, pb)
    st = sampler.run_chain(prob, sampler.State(s=np.zeros((256,) * 3),
                                               p_grid=pb["pk_init"] / w.cell_volume), 2)
    p_ref = st.p_grid * w.cell_volume
    err_s, err_p = errors(s_gpu, p_gpu, st.s, p_ref)
    print(f"  err_s={err_s:.2e} err_P={err_p:.2e}", flush=True)
    assert err_s < TOL["fp32"] and err_p < TOL["fp32"]
    # empty bins keep P (stored in grid units, P / V_cell, so up to rounding)
    assert np.allclose(p_gpu[counts == 0], pb["pk_init"][counts == 0], rtol=1e-14, atol=0)


def test_maximum_bins_mixing_fp64():
    w, pb, counts = _max_bins_problem("fp64")
    smp = gpu_sampler(w, pb)
    smp.sweep(1)
    smp.mixing_sweep(1)
    s_gpu, p_gpu, _ = smp.state()
    smp.close()
    prob = oracle_problem(w, pb)
    st = sampler.run_chain(prob, sampler.State(s=np.zeros((256,) * 3),
                                               p_grid=pb["pk_init"] / w.cell_volume), 1)
    st = mixing.mixing_sweep(prob, st)
    err_s, err_p = errors(s_gpu, p_gpu, st.s, st.p_grid * w.cell_volume)
    print(f"1024 bins at 256^3 FP64 mixing: err_s={err_s:.2e} err_P={err_p:.2e}", flush=True)
    assert err_s < TOL["fp64"] and err_p < TOL["fp64"]


def _status(exc_info):
    return exc_info.value.status


def test_sweep_index_stays_below_two_to_the_32():
    """The sweep index is Philox counter word 1: states at or beyond 2^32 are
    refused (set, checkpoint load, and sweeps that would reach it), and the
    last sweeps below it draw the oracle's numbers for those indices."""
    w = workloads.small_workload(32, 8, precision="fp64", seed=83, rng_seed=84)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    s0 = np.random.default_rng(5).standard_normal((32,) * 3)
    top = 2 ** 32 - 1
    with pytest.raises(binding.MFError) as e:
        smp.set_state(0, s0, pb["pk_init"], top + 1)
    assert _status(e) == binding.MF_E_INVALID_ARG
    assert smp.state(want_s=False)[2] == 0          # nothing changed
    smp.set_state(0, s0, pb["pk_init"], top - 2)
    smp.sweep(2)
    s_gpu, p_gpu, done = smp.state()
    assert done == top
    with pytest.raises(binding.MFError) as e:
        smp.sweep(1)
    assert _status(e) == binding.MF_E_INVALID_ARG
    with pytest.raises(binding.MFError) as e:
        smp.mixing_sweep(1)
    assert _status(e) == binding.MF_E_INVALID_ARG
    # a checkpoint at the last index reloads; one patched to 2^32 does not
    blob = smp.save_checkpoint(0)
    smp.load_checkpoint(blob, 0)
    bad = bytearray(blob)
    bad[24:32] = (top + 1).to_bytes(8, "little")     # header: magic, 4 int32, sweep
    with pytest.raises(binding.MFError) as e:
        smp.load_checkpoint(bytes(bad), 0)
    assert _status(e) == binding.MF_E_INVALID_ARG
    smp.close()
    from tests.gpu_util import run_oracle
    s_ref, p_ref = run_oracle(w, pb, 2, s0=s0, first_sweep=top - 2)
    err_s, err_p = errors(s_gpu, p_gpu, s_ref, p_ref)
    print(f"sweeps 2^32-3, 2^32-2: err_s={err_s:.2e} err_P={err_p:.2e}", flush=True)
    assert err_s < TOL["fp64"] and err_p < TOL["fp64"]


def test_mixing_sweep_refused_when_p_is_fixed():
    w = workloads.small_workload(32, 8, precision="fp32", seed=85, rng_seed=86)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb, sample_pk=False)
    with pytest.raises(binding.MFError) as e:
        smp.mixing_sweep(1)
    assert _status(e) == binding.MF_E_INVALID_ARG
    smp.sweep(1)
    _, pk, done = smp.state(want_s=False)
    smp.close()
    assert done == 1 and np.array_equal(pk, pb["pk_init"])


def test_diagnostics_cannot_change_under_a_live_graph():
    """A graph replays the recording buffers it captured, so changing them
    while it exists is refused and the old buffers stay in use."""
    import torch
    w = workloads.small_workload(32, 8, precision="fp32", seed=87, rng_seed=88)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    smp.set_diagnostics(start=0, thin=1, trace_cap=8)
    first = smp.trace_buf
    g = binding.SweepGraph([smp])
    with pytest.raises(binding.MFError) as e:
        smp.set_diagnostics(start=0, thin=1, trace_cap=16)
    assert _status(e) == binding.MF_E_STATE
    assert smp.trace_buf is first
    g.launch(3)
    torch.cuda.synchronize()
    assert smp.recorded() == 3
    assert bool(torch.all(smp.trace(0)[:3] > 0))
    g.close()
    smp.set_diagnostics(start=3, thin=1, trace_cap=16)    # allowed once the graph is gone
    smp.sweep(2)
    assert smp.recorded() == 2
    smp.close()
