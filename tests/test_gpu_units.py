"""GPU unit test of the device random numbers: with every voxel unobserved
except one, the messenger draw is t = s + sqrt(tau) G, so one z-pass from
s = 0 exposes the device's Philox4x32-10 + Box-Muller normals of the
messenger phase through the working spectrum.  They must equal the oracle's
(oracle.sampler.messenger_normals) to rounding, for every voxel and for two
chains and sweep indices."""
import numpy as np
import pytest

from oracle import sampler
from paper_1402_1763_amd import binding

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()
    torch.cuda.set_device(0)


@pytest.mark.parametrize("precision,n", [("fp64", 32), ("fp64", 48), ("fp32", 64)])
def test_messenger_normals_match_oracle(precision, n):
    import torch
    seed, chain_id, sweeps = 0x1234_5678_9ABC, 5, (0, 7, 1 << 20)
    nv = np.full((n,) * 3, np.inf)
    nv[0, 0, 0] = 1.0                 # tau = 1; at this voxel t = d = 0 exactly
    data = np.zeros((n,) * 3)
    smp = binding.Sampler([data, data], [nv, nv], [np.ones(4), np.ones(4)], 4, 15.625 * n,
                          seed=seed, chain_id=chain_id, precision=precision)
    tol = 1e-13 if precision == "fp64" else 2e-6
    for sweep in sweeps:
        for c in range(2):
            smp.set_state(c, np.zeros((n,) * 3), None, 0)
        binding.mf_debug_run_kernel(smp.handle, 0, sweep)        # the z-pass only
        torch.cuda.synchronize()
        for c in range(2):
            spec = binding.mf_debug_spectrum(smp.handle, c, n)    # DFT_z(t), [kz][ix][iy]
            t = np.fft.irfft(spec.transpose(1, 2, 0), n=n, axis=2)
            g = sampler.messenger_normals(n, seed, chain_id + c, sweep)
            g[0, 0, 0] = 0.0
            err = float(np.abs(t - g).max())
            print(f"{precision} n={n} sweep={sweep} chain={c}: max |t - G| = {err:.2e}", flush=True)
            assert err < tol * np.abs(g).max()
    smp.close()
