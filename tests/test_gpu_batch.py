"""GPU tests of independent chains: several chains in one problem (one launch
per pass, grid over chains), several problems of different sizes in one HIP
graph, and bitwise resume from checkpoints."""
import numpy as np
import pytest

from paper_1402_1763_amd import binding, workloads
from tests.gpu_util import TOL, errors, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()
    torch.cuda.set_device(0)


@pytest.mark.parametrize("precision,n,tuning", [
    ("fp64", 32, None), ("fp32", 64, None),
    # every chain of a multi-chain launch under the variants the autotuner
    # may pick: the lane-pair x tile, G/2 y groups, reversed radix order
    ("fp32", 96, ("split", 2, 1, 1)), ("fp64", 48, ("split", 2, 0, 1)),
    ("fp32", 80, ("whole", 0, 0, 0))])
def test_chains_in_one_problem_match_oracle(precision, n, tuning):
    ws, pbs = [], []
    for c in range(3):
        w = workloads.small_workload(n, 8, mask="random", precision=precision, seed=40 + c,
                                     rng_seed=77, mask_frac=0.1 + 0.1 * c, sigma2=0.5 + c)
        ws.append(w)
        pbs.append(workloads.make_problem(w))
    print(f"3 chains n={n} {precision} tuning={tuning}", flush=True)
    smp = binding.Sampler([pb["data"] for pb in pbs], [pb["noise_var"] for pb in pbs],
                          [pb["pk_init"] for pb in pbs], 8, ws[0].box, seed=77,
                          precision=precision, chain_id=5)
    if tuning is not None:
        smp.set_tuning(*tuning)
    smp.sweep(6)
    for c in range(3):
        s_gpu, p_gpu, done = smp.state(c)
        s_ref, p_ref = run_oracle(ws[c], pbs[c], 6, chain=5 + c)
        err_s, err_p = errors(s_gpu, p_gpu, s_ref, p_ref)
        print(f"  chain {c}: err_s={err_s:.3e} err_P={err_p:.3e}", flush=True)
        assert done == 6 and err_s < TOL[precision] and err_p < TOL[precision]
    smp.close()


def _pair():
    out = []
    for n, prec, nb in ((32, "fp64", 8), (64, "fp32", 16), (16, "fp32", 4)):
        w = workloads.small_workload(n, nb, mask="random", precision=prec, seed=n)
        out.append((w, workloads.make_problem(w)))
    return out


def _make(w, pb):
    return binding.Sampler(pb["data"], pb["noise_var"], pb["pk_init"], w.n_bins, w.box,
                           seed=w.rng_seed, precision=w.precision)


def test_graph_replays_match_eager_sweeps():
    import torch
    probs = _pair()
    graphed = [_make(w, pb) for w, pb in probs]
    eager = [_make(w, pb) for w, pb in probs]
    g = binding.SweepGraph(graphed)
    for rep in range(4):
        print(f"replay {rep}", flush=True)
        g.launch(2 if rep % 2 else 1)
        for smp in eager:                      # eager work between replays
            smp.sweep(2 if rep % 2 else 1)
        torch.cuda.synchronize()
        for a, b in zip(graphed, eager):
            sa, pa, na = a.state()
            sb, pbk, nb = b.state()
            assert na == nb
            assert np.array_equal(sa, sb) and np.array_equal(pa, pbk)
    g.close()
    for smp in graphed + eager:
        smp.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_checkpoint_resume_is_bitwise(precision):
    w = workloads.small_workload(32, 8, mask="random", precision=precision, seed=3)
    pb = workloads.make_problem(w)
    ref = _make(w, pb)
    ref.sweep(12)
    s_ref, p_ref, n_ref = ref.state()
    ref.close()
    a = _make(w, pb)
    a.sweep(5)
    ck = a.save_checkpoint()
    a.close()
    b = _make(w, pb)                          # fresh problem, different state
    b.sweep(1)
    b.load_checkpoint(ck)
    b.sweep(7)
    s_b, p_b, n_b = b.state()
    b.close()
    assert n_b == n_ref == 12
    assert np.array_equal(s_b, s_ref) and np.array_equal(p_b, p_ref)


def test_state_set_resume_close():
    """Resume through the physical-unit state interface: same chain to rounding."""
    w = workloads.small_workload(32, 8, mask="random", precision="fp64", seed=4)
    pb = workloads.make_problem(w)
    ref = _make(w, pb)
    ref.sweep(8)
    s_ref, p_ref, _ = ref.state()
    a = _make(w, pb)
    a.sweep(4)
    s4, p4, n4 = a.state()
    b = _make(w, pb)
    b.set_state(0, s4, p4, n4)
    b.sweep(4)
    s_b, p_b, n_b = b.state()
    err_s, err_p = errors(s_b, p_b, s_ref, p_ref)
    assert n_b == 8 and err_s < 1e-10 and err_p < 1e-10
    for smp in (ref, a, b):
        smp.close()


def test_mixed_size_graph_matches_oracle():
    """Chains of sides 48, 64, 80, 96 (two each) swept by one graph; one chain
    of every size checked against the oracle after 5 replays."""
    groups = []
    for n in (48, 64, 80, 96):
        ws = [workloads.batched_chain(n, c) for c in range(2)]
        pbs = [workloads.make_problem(w) for w in ws]
        smp = binding.Sampler([pb["data"] for pb in pbs], [pb["noise_var"] for pb in pbs],
                              [pb["pk_init"] for pb in pbs], 16, ws[0].box, seed=ws[0].rng_seed,
                              precision="fp32")
        groups.append((ws, pbs, smp))
    g = binding.SweepGraph([grp[2] for grp in groups])
    g.launch(5)
    for ws, pbs, smp in groups:
        c = 1
        s_gpu, p_gpu, done = smp.state(c)
        s_ref, p_ref = run_oracle(ws[c], pbs[c], 5, chain=c)
        err_s, err_p = errors(s_gpu, p_gpu, s_ref, p_ref)
        print(f"  n={ws[c].n} chain {c}: err_s={err_s:.3e} err_P={err_p:.3e}", flush=True)
        assert done == 5 and err_s < TOL["fp32"] and err_p < TOL["fp32"]
    g.close()
    for grp in groups:
        grp[2].close()
