"""GPU parity of the optional conjugate prior on P(k): InvGamma(a0, b0) in
place of Jeffreys' 1/P (Sec. 3.2), in the Gibbs P step and in the mixing
sweep's Metropolis-Hastings move, against the oracle on the same seeded
problem."""
import numpy as np
import pytest

from oracle import mixing, sampler
from paper_1402_1763_amd import binding, workloads
from tests.gpu_util import TOL, errors, gpu_sampler

pytestmark = pytest.mark.gpu

# a0 and b0 (physical units): b0 / V_cell is about P_grid of the middle bins,
# so the prior moves the draws well beyond rounding
PRIOR = (1.5, 4.0e5)


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()
    torch.cuda.set_device(0)


def _oracle(w, pb, pattern, prior):
    prob = sampler.make_problem(pb["data"], pb["noise_var"], w.n_bins, w.box, w.rng_seed,
                                prior=prior)
    st = sampler.State(s=np.zeros((w.n,) * 3), p_grid=pb["pk_init"] / w.cell_volume)
    for kind in pattern:
        st = sampler.sweep(prob, st) if kind == "G" else mixing.mixing_sweep(prob, st)
    return st.s, st.p_grid * w.cell_volume


def _gpu(w, pb, pattern, prior):
    smp = gpu_sampler(w, pb, pk_prior=prior)
    for kind in pattern:
        (smp.sweep if kind == "G" else smp.mixing_sweep)(1)
    s, p, done = smp.state()
    smp.close()
    assert done == len(pattern)
    return s, p


@pytest.mark.parametrize("precision,pattern", [("fp64", "G" * 10), ("fp32", "G" * 10),
                                               ("fp64", "GGMMGM"), ("fp32", "GGMMGM")])
def test_prior_chain_matches_oracle(precision, pattern):
    w = workloads.small_workload(32, 8, mask="random", precision=precision, seed=61, rng_seed=62)
    pb = workloads.make_problem(w)
    print(f"InvGamma{PRIOR} prior, {precision}, sweeps {pattern}", flush=True)
    s_gpu, p_gpu = _gpu(w, pb, pattern, PRIOR)
    s_ref, p_ref = _oracle(w, pb, pattern, PRIOR)
    err_s, err_p = errors(s_gpu, p_gpu, s_ref, p_ref)
    print(f"  err_s={err_s:.3e} err_P={err_p:.3e}", flush=True)
    assert err_s < TOL[precision] and err_p < TOL[precision]
    # the prior acts: the same chain under Jeffreys' prior ends elsewhere
    _, p_jeff = _gpu(w, pb, pattern, (0.0, 0.0))
    assert np.max(np.abs(p_jeff - p_gpu) / p_gpu) > 1e-2

