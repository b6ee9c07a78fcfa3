"""GPU tests of the log-determinant trace estimator (mf_wiener_logdet_trace)
against the oracle (oracle/logdet.py): the same probes (Philox phase 4 signs)
give the same per-bin estimates, probe by probe and averaged, for one chain
and for several chains with responses in one launch; and, with the chi2
adjoint, the assembled likelihood gradient behaves as a score (zero mean over
data drawn at the true P)."""
import numpy as np
import pytest

from oracle import logdet, sampler
from paper_1402_1763_amd import binding, workloads
from tests.gpu_util import TOL, oracle_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()
    torch.cuda.set_device(0)


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("precision,n", [("fp64", 32), ("fp32", 32), ("fp64", 48)])
def test_probes_match_oracle(precision, n):
    import torch
    k = 10
    w = workloads.small_workload(n, 8, precision=precision, seed=101, rng_seed=102)
    pb = workloads.make_problem(w)
    smp = binding.Sampler(pb["data"], pb["noise_var"], pb["pk_init"], w.n_bins, w.box,
                          seed=w.rng_seed, precision=precision, sample_pk=False)
    pk = 0.5 * workloads.power_spectrum(workloads.bin_centres(w), w)
    wf = binding.WienerFilter(smp, k, k)
    pk_t = torch.from_numpy(pk).cuda()
    one = [wf.logdet_trace(pk_t, 1, probe0=j).cpu().numpy() for j in (0, 1)]
    mean3 = wf.logdet_trace(pk_t, 3, probe0=4).cpu().numpy()
    smp.close()
    prob = oracle_problem(w, pb)
    p_grid = pk / w.cell_volume
    ref = [logdet.trace_probe(prob, p_grid, k, j) / w.cell_volume for j in (0, 1)]
    ref3 = np.mean([logdet.trace_probe(prob, p_grid, k, j) for j in (4, 5, 6)], axis=0) / w.cell_volume
    errs = [_rel(a, b) for a, b in zip(one + [mean3], ref + [ref3])]
    print(f"logdet n={n} {precision}: per-probe err {errs[0]:.2e} {errs[1]:.2e}, mean of 3 "
          f"{errs[2]:.2e}", flush=True)
    assert max(errs) < TOL[precision]


def test_all_chains_with_responses_in_one_launch():
    import torch
    n, k, chains = 32, 8, 2
    w = workloads.small_workload(n, 6, precision="fp64", seed=111, rng_seed=112)
    pb = workloads.make_problem(w)
    rng = np.random.default_rng(5)
    rs = []
    for _ in range(chains):
        r = rng.uniform(0.3, 1.7, (n,) * 3) * np.where(rng.random((n,) * 3) < 0.2, -1.0, 1.0)
        r[rng.random((n,) * 3) < 0.1] = 0.0
        rs.append(r)
    ds = [np.where(np.isfinite(pb["noise_var"]), r * pb["data"], 0.0) for r in rs]
    smp = binding.Sampler(ds, [pb["noise_var"]] * chains, [pb["pk_init"]] * chains, w.n_bins,
                          w.box, seed=w.rng_seed, precision="fp64", sample_pk=False, response=rs)
    pk = 0.5 * workloads.power_spectrum(workloads.bin_centres(w), w)
    wf = binding.WienerFilter(smp, k, k, chain=None)
    tr = wf.logdet_trace(torch.from_numpy(np.stack([pk] * chains)).cuda(), 2, probe0=7).cpu().numpy()
    single = binding.WienerFilter(smp, k, k, chain=1).logdet_trace(torch.from_numpy(pk).cuda(), 2,
                                                                  probe0=7).cpu().numpy()
    smp.close()
    assert np.array_equal(tr[1], single)
    for c in range(chains):
        prob = sampler.make_problem(ds[c], pb["noise_var"], w.n_bins, w.box, w.rng_seed, chain=c,
                                    response=rs[c])
        ref = logdet.trace_estimate(prob, pk / w.cell_volume, k, (7, 8)) / w.cell_volume
        err = _rel(tr[c], ref)
        print(f"logdet chain {c} with response: err {err:.2e}", flush=True)
        assert err < TOL["fp64"]


def test_errors():
    import torch
    w = workloads.small_workload(32, 4, precision="fp32", seed=121)
    pb = workloads.make_problem(w)
    smp = binding.Sampler(pb["data"], pb["noise_var"], pb["pk_init"], w.n_bins, w.box,
                          seed=w.rng_seed, precision="fp32")
    wf = binding.WienerFilter(smp, 4, 4)
    pk = torch.from_numpy(pb["pk_init"]).cuda()
    with pytest.raises(binding.MFError) as e:
        wf.logdet_trace(pk, 0)
    assert e.value.status == binding.MF_E_INVALID_ARG
    lib = binding.load()
    import ctypes
    status = lib.mf_wiener_logdet_trace(ctypes.c_void_p(smp.handle), 0, ctypes.c_void_p(pk.data_ptr()),
                                        4, 1, 0, ctypes.c_void_p(wf._ld_ws.data_ptr() // 256 * 256 + 256),
                                        1024, ctypes.c_void_p(pk.data_ptr()), None)
    assert status == binding.MF_E_WORKSPACE
    with pytest.raises(binding.MFError) as e:
        binding.WienerFilter(smp, 4, 4, chain=3)
    assert e.value.status == binding.MF_E_STATE
    smp.close()


def test_likelihood_gradient_is_a_score_on_the_gpu():
    """-1/2 (d chi2/d P + T) from mf_wiener_backward and mf_wiener_logdet_trace
    behaves as the gradient of ln L: eight data sets drawn at the true P (one
    chain each, one launch) give a mean within noise of zero, and at twice the
    true P a clearly negative one."""
    import torch
    from tests.test_oracle_logdet import _score_data
    n, nb, k, probes, reals = 32, 6, 200, 32, 8
    box = 32 * 15.625
    vcell = (box / n) ** 3
    p_true = np.array([6.0, 5.0, 4.0, 3.0, 2.0, 1.5])          # grid units, tau = 1
    mask = np.random.default_rng(1).random((n,) * 3) < 0.25
    nv = np.where(mask, np.inf, 1.0)
    ds = [_score_data(n, p_true, mask, 200 + r) for r in range(reals)]
    smp = binding.Sampler(ds, [nv] * reals, [p_true * vcell] * reals, nb, box, seed=9,
                          precision="fp64", sample_pk=False)
    wf = binding.WienerFilter(smp, k, 20, chain=None)
    d_t = torch.from_numpy(np.stack(ds)).cuda()
    z = {}
    for scale in (1.0, 2.0):
        pk = torch.from_numpy(np.stack([scale * p_true * vcell] * reals)).cuda()
        wf.forward(d_t, pk)
        _, grad_pk = wf.backward(d_t)
        t = wf.logdet_trace(pk, probes)
        g = (-0.5 * (grad_pk + t)).cpu().numpy()
        z[scale] = g.mean(axis=0) / (g.std(axis=0, ddof=1) / np.sqrt(reals))
        print(f"score at {scale} x P_true: z = {np.round(z[scale], 2)}", flush=True)
    smp.close()
    assert np.all(np.abs(z[1.0]) < 4.0)
    assert np.all(z[2.0] < -5.0)
