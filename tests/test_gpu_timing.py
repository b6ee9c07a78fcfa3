"""GPU tests of the per-kernel timing entry points: mf_gibbs_sweep_timed and
mf_gibbs_sweep_timed_cold advance the chain exactly as plain sweeps do, the
eviction streams touch nothing but their own buffer, and their argument
checks."""
import ctypes

import numpy as np
import pytest

from paper_1402_1763_amd import binding, workloads
from tests.gpu_util import gpu_sampler

pytestmark = pytest.mark.gpu

EVICT_BYTES = 64 << 20   # the smallest eviction buffer the library takes


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()
    torch.cuda.set_device(0)


def _pair(seed):
    w = workloads.small_workload(64, 8, precision="fp32", seed=seed, rng_seed=seed + 1)
    pb = workloads.make_problem(w)
    return gpu_sampler(w, pb), gpu_sampler(w, pb)


def _same_chain(a, b):
    sa, pa, na = a.state()
    sb, pb_, nb = b.state()
    return np.array_equal(sa, sb) and np.array_equal(pa, pb_) and na == nb


def test_timed_sweeps_advance_the_chain_as_plain_sweeps():
    smp, ref = _pair(301)
    ms = smp.sweep_timed(9)
    ref.sweep(9)
    assert _same_chain(smp, ref)
    assert ms.shape == (binding.MF_NUM_KERNELS,)
    assert np.all(np.isfinite(ms)) and np.all(ms > 0)
    # fewer sweeps than kernels: the kernels never bracketed read NaN
    ms2 = smp.sweep_timed(2)
    ref.sweep(2)
    assert _same_chain(smp, ref)
    assert np.all(np.isfinite(ms2[:2])) and np.all(np.isnan(ms2[2:]))
    smp.close()
    ref.close()


@pytest.mark.parametrize("mode", binding.Sampler.EVICT_MODES)
def test_cold_timed_sweeps_leave_the_chain_and_touch_only_their_buffer(mode):
    import torch
    smp, ref = _pair(311)
    # the eviction buffer sits between two guard tensors that must not change
    guard0 = torch.full((1 << 16,), 7, dtype=torch.int32, device="cuda")
    evict = torch.zeros(EVICT_BYTES, dtype=torch.uint8, device="cuda")
    guard1 = torch.full((1 << 16,), 9, dtype=torch.int32, device="cuda")
    ms = smp.sweep_timed_cold(8, evict, mode)
    ref.sweep(8)
    torch.cuda.synchronize()
    assert _same_chain(smp, ref)
    assert np.all(np.isfinite(ms)) and np.all(ms > 0)
    assert bool((guard0 == 7).all()) and bool((guard1 == 9).all())
    smp.close()
    ref.close()


def test_cold_timing_argument_checks():
    import torch
    smp, _ = _pair(321)
    lib = binding.load()
    out = np.zeros(binding.MF_NUM_KERNELS, dtype=np.float64)
    evict = torch.zeros(EVICT_BYTES + 64, dtype=torch.uint8, device="cuda")
    base = evict.data_ptr()

    def call(ptr, nbytes, mode, n=4):
        return lib.mf_gibbs_sweep_timed_cold(
            ctypes.c_void_p(smp.handle), n, ctypes.c_void_p(smp.stream.cuda_stream),
            binding._dptr(out), binding.MF_NUM_KERNELS,
            ctypes.c_void_p(ptr), ctypes.c_size_t(nbytes), mode)

    sweep0 = smp.state(want_s=False)[2]
    assert call(0, EVICT_BYTES, 1) == binding.MF_E_INVALID_ARG              # NULL
    assert call(base + 8, EVICT_BYTES, 1) == binding.MF_E_INVALID_ARG       # not 16-byte aligned
    assert call(base, EVICT_BYTES - 32, 1) == binding.MF_E_INVALID_ARG      # below 64 MiB
    assert call(base, EVICT_BYTES + 16, 1) == binding.MF_E_INVALID_ARG      # not a multiple of 32
    assert call(base, EVICT_BYTES, 3) == binding.MF_E_INVALID_ARG           # no such mode
    assert call(base, EVICT_BYTES, -1) == binding.MF_E_INVALID_ARG
    assert call(base, EVICT_BYTES, 1, n=0) == binding.MF_E_INVALID_ARG      # no sweep
    assert smp.state(want_s=False)[2] == sweep0                            # nothing ran
    assert call(base, EVICT_BYTES, 1) == binding.MF_OK
    assert smp.state(want_s=False)[2] == sweep0 + 4
    with pytest.raises(binding.MFError):
        smp.sweep_timed(0)
    smp.close()
