"""GPU parity with a general per-voxel response R (data model d = R s + eps of
Sec. 2): Gibbs and mixing sweeps and the Wiener filter with its gradient,
against the oracle run with the same R."""
import numpy as np
import pytest

from oracle import adjoint, mixing, sampler
from paper_1402_1763_amd import binding, workloads
from tests.gpu_util import TOL, errors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()
    torch.cuda.set_device(0)


def _response_problem(n, n_bins, precision, seed, mask="random", chains=1):
    """Chains of one workload with responses R in [0.3, 1.7] (R = 0 on 10% of
    the voxels) and data R d0 on observed voxels."""
    w = workloads.small_workload(n, n_bins, mask=mask, precision=precision, seed=seed,
                                 rng_seed=seed + 1)
    pb = workloads.make_problem(w)
    rng = np.random.default_rng(seed + 2)
    rs, ds = [], []
    for _ in range(chains):
        r = rng.uniform(0.3, 1.7, (n,) * 3)
        r[rng.random((n,) * 3) < 0.1] = 0.0
        rs.append(r)
        ds.append(np.where(np.isfinite(pb["noise_var"]), r * pb["data"], 0.0))
    return w, pb, rs, ds


def _oracle(w, pb, d, r, chain=0):
    return sampler.make_problem(d, pb["noise_var"], w.n_bins, w.box, w.rng_seed, chain=chain,
                                response=r)


@pytest.mark.parametrize("precision,n,mask", [("fp64", 32, "random"), ("fp32", 48, "random"),
                                              ("fp32", 64, "survey")])
def test_gibbs_sweeps_with_response_match_oracle(precision, n, mask):
    sweeps = 10
    w, pb, rs, ds = _response_problem(n, 8, precision, 41, mask=mask)
    print(f"response gibbs n={n} {precision} {mask}", flush=True)
    smp = binding.Sampler(ds[0], pb["noise_var"], pb["pk_init"], w.n_bins, w.box,
                          seed=w.rng_seed, precision=precision, response=rs[0])
    prob = _oracle(w, pb, ds[0], rs[0])
    assert smp.tau() == pytest.approx(prob.tau, rel=1e-15)
    smp.sweep(sweeps)
    s_gpu, p_gpu, _ = smp.state()
    smp.close()
    st = sampler.run_chain(prob, sampler.State(s=np.zeros((n,) * 3),
                                               p_grid=pb["pk_init"] / w.cell_volume), sweeps)
    err_s, err_p = errors(s_gpu, p_gpu, st.s, st.p_grid * w.cell_volume)
    print(f"  err_s={err_s:.2e} err_P={err_p:.2e}", flush=True)
    assert err_s < TOL[precision] and err_p < TOL[precision]


def test_mixing_sweeps_with_response_match_oracle():
    w, pb, rs, ds = _response_problem(32, 8, "fp64", 43)
    smp = binding.Sampler(ds[0], pb["noise_var"], pb["pk_init"], w.n_bins, w.box,
                          seed=w.rng_seed, precision="fp64", response=rs[0])
    smp.sweep(3)
    smp.mixing_sweep(2)
    s_gpu, p_gpu, _ = smp.state()
    smp.close()
    prob = _oracle(w, pb, ds[0], rs[0])
    st = sampler.run_chain(prob, sampler.State(s=np.zeros((32,) * 3),
                                               p_grid=pb["pk_init"] / w.cell_volume), 3)
    st = mixing.mixing_sweep(prob, mixing.mixing_sweep(prob, st))
    err_s, err_p = errors(s_gpu, p_gpu, st.s, st.p_grid * w.cell_volume)
    print(f"response mixing err_s={err_s:.2e} err_P={err_p:.2e}", flush=True)
    assert err_s < TOL["fp64"] and err_p < TOL["fp64"]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_wiener_gradient_with_response_matches_oracle(precision):
    """Two chains with different responses in one launch (chain = -1)."""
    import torch
    k, every, n = 12, 5, 32
    w, pb, rs, ds = _response_problem(n, 8, precision, 45, chains=2)
    smp = binding.Sampler(ds, [pb["noise_var"]] * 2, [pb["pk_init"]] * 2, w.n_bins, w.box,
                          seed=w.rng_seed, precision=precision, sample_pk=False, response=rs)
    pk = 0.5 * workloads.power_spectrum(workloads.bin_centres(w), w)
    wf = binding.WienerFilter(smp, k, every, chain=None)
    d_t = torch.from_numpy(np.stack(ds)).cuda()
    pk_t = torch.from_numpy(np.stack([pk, pk])).cuda()
    chi2, s_k = wf.forward(d_t, pk_t, want_s=True)
    grad_d, grad_pk = wf.backward(d_t)
    torch.cuda.synchronize()
    tol = TOL[precision]
    for c in range(2):
        prob = _oracle(w, pb, ds[c], rs[c], chain=c)
        s_ref, _ = adjoint.wf_forward(prob, pk / w.cell_volume, k)
        loss, gp, gd = adjoint.wf_gradient(prob, pk / w.cell_volume, k)
        gp = gp / w.cell_volume
        e_s = float(np.abs(s_k[c].cpu().numpy() - s_ref).max() / np.sqrt(np.mean(s_ref ** 2)))
        e_c = abs(float(chi2[c]) - loss) / abs(loss)
        e_gd = float(np.abs(grad_d[c].cpu().numpy() - gd).max() / np.abs(gd).max())
        e_gp = float(np.abs(grad_pk[c].cpu().numpy() - gp).max() / np.abs(gp).max())
        print(f"response wiener {precision} chain {c}: s={e_s:.2e} chi2={e_c:.2e} "
              f"grad_d={e_gd:.2e} grad_P={e_gp:.2e}", flush=True)
        assert e_s < tol and e_c < tol and e_gd < tol and e_gp < tol
        assert np.all(grad_d[c].cpu().numpy()[~prob.observed] == 0.0)
    smp.close()


def test_response_in_fp32_mixing_and_in_a_graph():
    """FP32 mixing sweeps with a response against the oracle (the MH decisions
    are taken in FP64 from FP32 fields, so this also checks none flips here),
    and graph replays of a response problem against eager sweeps, bitwise."""
    w, pb, rs, ds = _response_problem(48, 8, "fp32", 47)
    smp = binding.Sampler(ds[0], pb["noise_var"], pb["pk_init"], w.n_bins, w.box,
                          seed=w.rng_seed, precision="fp32", response=rs[0])
    smp.sweep(3)
    smp.mixing_sweep(2)
    s_gpu, p_gpu, _ = smp.state()
    smp.close()
    prob = _oracle(w, pb, ds[0], rs[0])
    st = sampler.run_chain(prob, sampler.State(s=np.zeros((48,) * 3),
                                               p_grid=pb["pk_init"] / w.cell_volume), 3)
    st = mixing.mixing_sweep(prob, mixing.mixing_sweep(prob, st))
    err_s, err_p = errors(s_gpu, p_gpu, st.s, st.p_grid * w.cell_volume)
    print(f"response mixing fp32 err_s={err_s:.2e} err_P={err_p:.2e}", flush=True)
    assert err_s < TOL["fp32"] and err_p < TOL["fp32"]

    a = binding.Sampler(ds[0], pb["noise_var"], pb["pk_init"], w.n_bins, w.box,
                        seed=w.rng_seed, precision="fp32", response=rs[0])
    b = binding.Sampler(ds[0], pb["noise_var"], pb["pk_init"], w.n_bins, w.box,
                        seed=w.rng_seed, precision="fp32", response=rs[0])
    a.sweep(5)
    g = binding.SweepGraph([b])
    g.launch(5)
    g.close()
    sa, pa, na = a.state()
    sb, pb_, nb_ = b.state()
    a.close()
    b.close()
    assert na == nb_ == 5 and np.array_equal(sa, sb) and np.array_equal(pa, pb_)
