"""GPU tests of the mixing sweep (Sec. 3.3, Alg. 3, shell form) against the
oracle (oracle/mixing.py), interleaved with Gibbs sweeps."""
import numpy as np
import pytest

from oracle import mixing, sampler
from paper_1402_1763_amd import binding, workloads
from tests.gpu_util import TOL, errors, gpu_sampler, oracle_problem

pytestmark = pytest.mark.gpu

PATTERN = "GMMGMM"      # G: Gibbs sweep, M: mixing sweep


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()
    torch.cuda.set_device(0)


def _oracle(w, pb, pattern):
    prob = oracle_problem(w, pb)
    st = sampler.State(s=np.zeros((w.n,) * 3), p_grid=pb["pk_init"] / w.cell_volume)
    accepted = 0
    for kind in pattern:
        if kind == "G":
            st = sampler.sweep(prob, st)
        else:
            p_old = st.p_grid
            st = mixing.mixing_sweep(prob, st)
            accepted += int(np.sum(st.p_grid != p_old))
    return st.s, st.p_grid * w.cell_volume, accepted


@pytest.mark.parametrize("precision,n,mask", [("fp64", 32, "random"), ("fp32", 32, "random"),
                                              ("fp32", 48, "none"), ("fp64", 64, "survey")])
def test_mixing_sweeps_match_oracle(precision, n, mask):
    w = workloads.small_workload(n, 8, mask=mask, precision=precision, seed=81, rng_seed=82)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    print(f"mixing n={n} {precision} {mask} pattern {PATTERN}", flush=True)
    for kind in PATTERN:
        if kind == "G":
            smp.sweep(1)
        else:
            smp.mixing_sweep(1)
    s_gpu, p_gpu, done = smp.state()
    s_ref, p_ref, accepted = _oracle(w, pb, PATTERN)
    err_s, err_p = errors(s_gpu, p_gpu, s_ref, p_ref)
    print(f"  err_s={err_s:.3e} err_P={err_p:.3e}  (oracle accepted {accepted} of "
          f"{PATTERN.count('M') * w.n_bins} moves)", flush=True)
    assert done == len(PATTERN)
    assert accepted > 0
    assert err_s < TOL[precision] and err_p < TOL[precision]


def test_long_mixing_run_with_rejections_matches_oracle():
    pattern = "G" * 4 + "M" * 20
    w = workloads.small_workload(32, 6, mask="random", precision="fp64", seed=85, rng_seed=86,
                                 mask_frac=0.3)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    for kind in pattern:
        (smp.sweep if kind == "G" else smp.mixing_sweep)(1)
    s_gpu, p_gpu, _ = smp.state()
    s_ref, p_ref, accepted = _oracle(w, pb, pattern)
    moves = pattern.count("M") * w.n_bins
    err_s, err_p = errors(s_gpu, p_gpu, s_ref, p_ref)
    print(f"long mixing: err_s={err_s:.3e} err_P={err_p:.3e} accepted {accepted}/{moves}", flush=True)
    assert 0 < accepted < moves
    assert err_s < TOL["fp64"] and err_p < TOL["fp64"]


def test_mixing_records_traces_and_rejects_small_grids():
    w = workloads.small_workload(32, 8, precision="fp32", seed=83, rng_seed=84)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    smp.set_diagnostics(start=0, thin=1, trace_cap=6, moments=True)
    smp.mixing_sweep(3)
    smp.sweep(2)
    assert smp.recorded() == 5
    tr = smp.trace().cpu().numpy()
    assert np.allclose(tr[0], pb["pk_init"], rtol=1e-12)
    assert np.all(np.isfinite(tr)) and np.all(tr > 0)
    w16 = workloads.small_workload(16, 4, precision="fp32")
    pb16 = workloads.make_problem(w16)
    with pytest.raises(binding.MFError) as e:
        gpu_sampler(w16, pb16).mixing_sweep(1)
    assert e.value.status == binding.MF_E_UNSUPPORTED_SIZE
