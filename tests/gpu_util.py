"""Shared helpers of the GPU tests: run the HIP path and the oracle on the
same seeded problem and measure the parity metrics.

Metrics: s by max_i |s_gpu - s_ref| / rms(s_ref) (a relative error per voxel
is ill-defined at zero crossings), P by max_b |P_gpu - P_ref| / P_ref.
"""
import numpy as np

from oracle import sampler
from paper_1402_1763_amd import binding, workloads


def oracle_problem(w, pb, chain=0, tau=None):
    return sampler.make_problem(pb["data"], pb["noise_var"], w.n_bins, w.box, w.rng_seed,
                                chain=chain, tau=tau)


def run_oracle(w, pb, n_sweeps, sample_pk=True, s0=None, p0=None, first_sweep=0, chain=0,
               tau=None):
    prob = oracle_problem(w, pb, chain=chain, tau=tau)
    st = sampler.State(s=np.zeros((w.n,) * 3) if s0 is None else np.array(s0, dtype=np.float64),
                       p_grid=(pb["pk_init"] if p0 is None else p0) / w.cell_volume,
                       sweep=first_sweep)
    st = sampler.run_chain(prob, st, n_sweeps, sample_pk=sample_pk)
    return st.s, st.p_grid * w.cell_volume


def errors(s_gpu, p_gpu, s_ref, p_ref):
    err_s = float(np.abs(s_gpu - s_ref).max() / np.sqrt(np.mean(s_ref ** 2)))
    ok = p_ref > 0
    err_p = float(np.max(np.abs(p_gpu[ok] - p_ref[ok]) / p_ref[ok])) if ok.any() else 0.0
    return err_s, err_p


def gpu_sampler(w, pb, sample_pk=True, **kw):
    return binding.Sampler(pb["data"], pb["noise_var"], pb["pk_init"], w.n_bins, w.box,
                           seed=w.rng_seed, precision=w.precision, sample_pk=sample_pk, **kw)


TOL = {"fp64": 1e-10, "fp32": 1e-4}
