"""Write the stored oracle results behind tests/test_gpu_long_horizon.py.

The oracle (FP64, the Philox contract) runs the configurations' full chain
lengths from the initial state s = 0, P = 0.1 x truth: the 128^3 survey for
1000 sweeps and the 256^3 survey for 500 sweeps.  At a few sweep counts it
records P_b of every bin, rms(s) over the whole grid and s at a fixed seeded
sample of voxels, so that the GPU test can compare its chain element by
element on the sample without rerunning the oracle (about 9 and 45 minutes
of host time on 8 cores).  Only oracle/ and the input generator are called.

Usage: python tests/golden/make_long_horizon.py [workload ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import sampler  # noqa: E402
from paper_1402_1763_amd import workloads  # noqa: E402

RUNS = {"gibbs-128^3-fp32-survey": (10, 100, 1000),
        "gibbs-256^3-fp32-survey": (10, 100, 500)}
N_SAMPLE = 2048
SAMPLE_SEED = 4242


def path_of(name: str) -> str:
    return os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        f"long_horizon_{name.split('-')[1].split('^')[0]}.json")


def run(name: str) -> None:
    w = workloads.WORKLOADS[name]
    marks = RUNS[name]
    pb = workloads.make_problem(w)
    prob = sampler.make_problem(pb["data"], pb["noise_var"], w.n_bins, w.box, w.rng_seed)
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(w.m, size=N_SAMPLE, replace=False))
    st = sampler.State(s=np.zeros((w.n,) * 3), p_grid=pb["pk_init"] / w.cell_volume)
    out = {"workload": name, "n": w.n, "n_bins": w.n_bins, "sample_seed": SAMPLE_SEED,
           "voxels": [int(i) for i in idx], "checkpoints": []}
    t0 = time.time()
    for k in range(1, marks[-1] + 1):
        st = sampler.sweep(prob, st)
        if k in marks:
            s = st.s.reshape(-1)
            out["checkpoints"].append({
                "sweeps": k,
                "pk": [float(v) for v in st.p_grid * w.cell_volume],
                "rms_s": float(np.sqrt(np.mean(s ** 2))),
                "s": [float(v) for v in s[idx]]})
            print(f"{name}: {k} sweeps, {time.time() - t0:.0f} s", flush=True)
    with open(path_of(name), "w") as f:
        json.dump(out, f)
        f.write("\n")


if __name__ == "__main__":
    os.environ.setdefault("ORACLE_FFT_WORKERS", str(len(os.sched_getaffinity(0))))
    for name in sys.argv[1:] or list(RUNS):
        run(name)
