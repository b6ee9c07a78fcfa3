"""Benchmark: Gibbs sweeps/s of the messenger-field sampler at 256^3, FP32
fields and FFTs with FP64 shell sums and inverse-gamma draws, on one GPU.

A step is one full Gibbs sweep (messenger draw, forward FFT, signal draw,
shell power, P(k) draw, inverse FFT) of one chain over the synthetic
survey-like problem (sphere of radius 0.45 L minus a 30-degree wedge, noise
1/(nbar sel(r) V_cell)).  Inputs are resident in HBM before timing starts.

Timing: after set-up (the x-path autotuner and a burn-in of the chain, which
also brings the GPU from its idle clock to its steady one) and --warmup
sweeps, --segments segments of --steps sweeps each are timed with events, a
device synchronisation on both sides of each; the median segment gives
`value`.  Per-kernel times for the roofline come from the library's
event-timed sweeps (one kernel per sweep between fenceless events), once in
sequence and once with the 256 MB last-level cache evicted before the kernel.

Prints one JSON line.  --gpus N > 1 is refused: the sampler runs one chain
per GPU, and the benchmark measures one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def source_digest() -> str:
    """Digest of the kernel sources; stored beside profiled counters so that
    traffic figures are only reported for the code they were measured on."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1402_1763_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def x_columns(n: int) -> int:
    """iy columns per x-pass workgroup, as the library picks them: for
    32 <= n <= 256 the largest divisor of n with (n / 16) * columns <= 256,
    else min(n, 4096 / n)."""
    if 32 <= n <= 256:
        return max(d for d in range(1, 256 // (n // 16) + 1) if n % d == 0)
    return min(n, 4096 // n)


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch measured by rocprofv3 counters, if recorded for
    the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    entry = rec.get(workload, {}).get(kernel)
    if not entry or entry.get("source_digest") != source_digest():
        return None
    return entry.get("hbm_bytes_per_launch")


def cpu_baseline(w, pb, max_seconds: float = 30.0):
    """The FP64 oracle timed on the host cores over a bounded sample."""
    ncores = len(os.sched_getaffinity(0))
    os.environ["ORACLE_FFT_WORKERS"] = str(ncores)
    from oracle import sampler
    prob = sampler.make_problem(pb["data"], pb["noise_var"], w.n_bins, w.box, w.rng_seed)
    st = sampler.State(s=np.zeros((w.n,) * 3), p_grid=pb["pk_init"] / w.cell_volume)
    t0 = time.perf_counter()
    st = sampler.sweep(prob, st)                      # warm-up sweep
    warm = time.perf_counter() - t0
    n_timed = max(1, min(3, int(max_seconds / max(warm, 1e-3)) - 1))
    t0 = time.perf_counter()
    for _ in range(n_timed):
        st = sampler.sweep(prob, st)
    dt = time.perf_counter() - t0
    # the same sweep with every draw replaced by its mean (no Philox, no P
    # draw): what the oracle spends outside its random numbers
    t0 = time.perf_counter()
    sampler.sweep(prob, st, noise=False)
    dt_det = time.perf_counter() - t0
    return {"value": n_timed / dt, "unit": "sweeps/s", "cores": ncores, "kind": "oracle",
            "no_rng_value": 1.0 / dt_det,
            "sample": f"{n_timed} FP64 oracle sweeps of the same {w.n}^3 problem after one "
                      f"warm-up sweep (numpy Philox single-threaded, scipy.fft with "
                      f"{ncores} workers); no_rng_value: one sweep with every draw "
                      f"replaced by its mean"}


def _r5(v):
    return None if v != v else round(float(v), 5)


def bench_batched(args):
    """Independent chains of sides 64 (32 chains), 48, 80 and 96 (8 chains each),
    FP32, 16 bins: one HIP graph replay sweeps all 56 chains once."""
    import torch

    from paper_1402_1763_amd import binding, workloads
    torch.cuda.set_device(0)
    samplers, chain_voxels, sweep_bytes = [], 0, 0
    for n, chains in workloads.BATCHED_SIZES:
        ws = [workloads.batched_chain(n, c) for c in range(chains)]
        pbs = [workloads.make_problem(w) for w in ws]
        samplers.append(binding.Sampler([pb["data"] for pb in pbs], [pb["noise_var"] for pb in pbs],
                                        [pb["pk_init"] for pb in pbs], 16, ws[0].box,
                                        seed=ws[0].rng_seed, chain_id=1000 * n, precision="fp32"))
        chain_voxels += chains * n ** 3
        sweep_bytes += sum(samplers[-1].sweep_bytes().values())
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def graph_ms(warm):
        g = binding.SweepGraph(samplers)
        g.launch(warm)
        torch.cuda.synchronize()
        start.record(stream)
        g.launch(args.steps)
        stop.record(stream)
        torch.cuda.synchronize()
        g.close()
        return start.elapsed_time(stop) / args.steps

    # the library's default tiles, for comparison on the same device, after
    # a burn-in that brings the device to its steady clock
    for smp in samplers:
        smp.sweep(args.warmup)
    ms_defaults = graph_ms(max(args.warmup, 1000))
    tuned = {}
    for (n, _), smp in zip(workloads.BATCHED_SIZES, samplers):
        res = smp.autotune(trials=10)                         # before the graph is captured
        tuned[f"{n}^3"] = {k: res[k] for k in ("path", "x_tile", "y_group", "y_radix",
                                                "x_cols", "x_k1", "x_hist", "y_units")}
        tuned[f"{n}^3"]["ms"] = {"path": {k: _r5(v) for k, v in res["ms"].items()},
                                 "x_tile": [_r5(v) for v in res["ms_x_tile"]],
                                 "y_group": [_r5(v) for v in res["ms_y_group"]],
                                 "y_radix": [_r5(v) for v in res["ms_y_radix"]]}
    ms = graph_ms(max(args.warmup, 1000))
    start.record(stream)
    for _ in range(args.steps):
        for smp in samplers:
            smp.sweep(1)
    stop.record(stream)
    torch.cuda.synchronize()
    ms_eager = start.elapsed_time(stop) / args.steps
    for smp in samplers:
        _, pk, _ = smp.state(want_s=False)
        assert np.all(np.isfinite(pk))
    # the plain way: every chain its own single-chain problem, swept in turn
    singles = []
    for n, chains in workloads.BATCHED_SIZES:
        for c in range(chains):
            wc = workloads.batched_chain(n, c)
            pc = workloads.make_problem(wc)
            singles.append(binding.Sampler(pc["data"], pc["noise_var"], pc["pk_init"], 16, wc.box,
                                           seed=wc.rng_seed, chain_id=1000 * n + c,
                                           precision="fp32"))
    plain_steps = max(1, args.steps // 10)
    for smp in singles:
        smp.sweep(2)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(plain_steps):
        for smp in singles:
            smp.sweep(1)
    stop.record(stream)
    torch.cuda.synchronize()
    ms_plain = start.elapsed_time(stop) / plain_steps
    for smp in singles:
        smp.close()
    chains = sum(c for _, c in workloads.BATCHED_SIZES)
    out = {
        "metric": "batched Gibbs sweeps/s (56 independent chains of sides 48-96, one graph replay each)",
        "value": round(1000.0 / ms, 2), "unit": "batch sweeps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "gibbs-batched-mixed",
                   "chains": {f"{n}^3": c for n, c in workloads.BATCHED_SIZES},
                   "tuning": tuned,
                   "default_tiles_ms_per_step": round(ms_defaults, 5),
                   "tuned_speedup_vs_default_tiles": round(ms_defaults / ms, 4),
                   "chain_sweeps_per_s": round(chains * 1000.0 / ms, 1),
                   "voxel_sweeps_per_s": round(chain_voxels * 1000.0 / ms, 1),
                   "sweep_bytes_algorithmic": sweep_bytes,
                   "sweep_hbm_frac": round(sweep_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "eager_ms_per_step": round(ms_eager, 5),
                   "graph_speedup_vs_eager": round(ms_eager / ms, 3),
                   "plain_single_chain_ms_per_step": round(ms_plain, 5),
                   "speedup_vs_plain_single_chain_sweeps": round(ms_plain / ms, 3)},
    }
    print(json.dumps(out), flush=True)


def hbm_reference(gib: float = 2.0, reps: int = 5) -> dict:
    """What plain streaming reaches on this GPU, as context for the roofline
    (whose peak stays the published 8 TB/s): the library's copy and read-only
    kernels over buffers far larger than the 256 MB last-level cache, each
    mode at several grid sizes (best kept), and torch's copy for comparison;
    event-timed."""
    import torch

    from paper_1402_1763_amd import binding
    n = int(gib * 2 ** 28)
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    sums = torch.empty(65536, dtype=torch.int32, device="cuda")
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def rate(fn, nbytes):
        fn()
        torch.cuda.synchronize()
        start.record()
        for _ in range(reps):
            fn()
        stop.record()
        torch.cuda.synchronize()
        return nbytes * reps / (start.elapsed_time(stop) * 1e-3) / 1e9

    out = {}
    for mode in binding.STREAM_MODES:
        target, nbytes = (dst, 8 * n) if mode.startswith("copy") else (sums, 4 * n)
        best = max((rate(lambda: binding.stream_reference(src, target, mode, blocks), nbytes), blocks)
                   for blocks in (1024, 2048, 4096, 8192, 16384))
        out[f"{mode}_gbs"] = round(best[0], 1)
        out[f"{mode}_blocks"] = best[1]
    out["torch_copy_gbs"] = round(rate(lambda: dst.copy_(src), 8 * n), 1)
    out["buffer_gib"] = gib
    del src, dst, sums
    torch.cuda.empty_cache()
    return out


def fp64_sweep_rate(w, pb, steps: int) -> float:
    """Plain FP64 sweeps/s of the same problem on the same GPU (after a
    warm-up and the path autotuner)."""
    import torch

    from paper_1402_1763_amd import binding
    smp = binding.Sampler(pb["data"], pb["noise_var"], pb["pk_init"], w.n_bins, w.box,
                          seed=w.rng_seed, precision="fp64")
    smp.autotune(trials=5)
    smp.sweep(5)
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    smp.sweep(steps)
    stop.record(stream)
    torch.cuda.synchronize()
    smp.close()
    return round(1000.0 * steps / start.elapsed_time(stop), 2)


def plain_sweep_ms(w, pb, steps: int, precision: str = "fp32") -> float:
    """ms per plain Gibbs sweep of one problem on this GPU."""
    import torch

    from paper_1402_1763_amd import binding
    smp = binding.Sampler(pb["data"], pb["noise_var"], pb["pk_init"], w.n_bins, w.box,
                          seed=w.rng_seed, precision=precision)
    smp.sweep(5)
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    smp.sweep(steps)
    stop.record(stream)
    torch.cuda.synchronize()
    smp.close()
    return start.elapsed_time(stop) / steps


# Prior on P(k) of the chain-efficiency runs besides Jeffreys': InvGamma with
# a0 = 0 and b0 = 50 h^-3 Mpc^3, a log-uniform prior cut off below about
# b0, well under the truth of every bin of the 128^3 survey (about 90 at the
# highest k); it makes the joint posterior proper as P -> 0.
EFFICIENCY_PRIOR = (0.0, 50.0)


def bench_chain_efficiency(args):
    """Statistical efficiency on the 128^3 survey problem (Sec. 5.1): after a
    burn-in, record every 10th of `steps` sweeps of P(k) and compute the
    autocorrelation and the ten-percent correlation length n_c of every bin,
    for Gibbs sweeps, mixing sweeps (Alg. 3) and the two alternating, under
    Jeffreys' prior and under the proper InvGamma prior EFFICIENCY_PRIOR."""
    import torch

    from paper_1402_1763_amd import binding, workloads
    torch.cuda.set_device(0)
    w = workloads.SURVEY_128_FP32
    pb = workloads.make_problem(w)
    thin, burn = 10, args.warmup
    cap = args.steps // thin
    truth = workloads.power_spectrum(workloads.bin_centres(w), w)
    runs = {}
    for prior_name, prior in (("jeffreys", (0.0, 0.0)), ("invgamma", EFFICIENCY_PRIOR)):
        out_runs = {}
        for kind in ("gibbs", "mixing", "alternating"):
            smp = binding.Sampler(pb["data"], pb["noise_var"], pb["pk_init"], w.n_bins, w.box,
                                  seed=w.rng_seed, precision="fp32", pk_prior=prior)

            def alternate(n, smp=smp):
                for i in range(n):
                    (smp.sweep if i % 2 == 0 else smp.mixing_sweep)(1)

            step = {"gibbs": smp.sweep, "mixing": smp.mixing_sweep, "alternating": alternate}[kind]
            step(burn)
            smp.set_diagnostics(start=burn, thin=thin, trace_cap=cap)
            stream = torch.cuda.current_stream()
            start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            start.record(stream)
            step(args.steps)
            stop.record(stream)
            torch.cuda.synchronize()
            ms = start.elapsed_time(stop) / args.steps
            trace = smp.trace()
            max_lag = min(cap - 1, 400)
            _, nc = binding.acf(trace, max_lag)
            mean_pk = trace.mean(dim=0).cpu().numpy()
            ncv = nc.cpu().numpy()
            out_runs[kind] = {"sweeps_per_s": round(1000.0 / ms, 1),
                              "n_c_recorded": [int(v) for v in ncv],
                              "bins_with_n_c_le_50": int(np.sum((ncv >= 0) & (ncv <= 50))),
                              "posterior_mean_over_truth": [round(float(v), 3)
                                                            for v in mean_pk / truth]}
            smp.close()
        runs[prior_name] = out_runs
    jeff = runs["jeffreys"]
    best = max(jeff, key=lambda k: jeff[k]["bins_with_n_c_le_50"])
    out = {
        "metric": "share of P(k) bins with correlation length n_c <= 50 recorded samples "
                  "(ten-percent rule, every 10th sweep) at 128^3 FP32",
        "value": round(jeff[best]["bins_with_n_c_le_50"] / w.n_bins, 4),
        "unit": "fraction of bins", "n_gpus": 1, "steps": args.steps, "warmup": burn,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "chain-efficiency-128^3-fp32-survey", "thin": thin,
                   "recorded": cap, "bins": w.n_bins, "max_lag": min(cap - 1, 400),
                   "best_sampler": best, **jeff,
                   "invgamma_prior": {"a0": EFFICIENCY_PRIOR[0], "b0": EFFICIENCY_PRIOR[1],
                                      **runs["invgamma"]}},
    }
    print(json.dumps(out), flush=True)


def bench_mixing(args):
    """Mixing sweeps (Sec. 3.3, shell form) on the 256^3 survey problem."""
    import torch

    from paper_1402_1763_amd import binding, workloads
    torch.cuda.set_device(0)
    w = workloads.SURVEY_256_MIXED
    pb = workloads.make_problem(w)
    smp = binding.Sampler(pb["data"], pb["noise_var"], pb["pk_init"], w.n_bins, w.box,
                          seed=w.rng_seed, precision=w.precision)
    stream = torch.cuda.current_stream()
    smp.mixing_sweep(args.warmup)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    smp.mixing_sweep(args.steps)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    _, pk, _ = smp.state(want_s=False)
    assert np.all(np.isfinite(pk))
    n = w.n
    n_wg_x = (n // 2 + 1) * (n // x_columns(n))
    spec = 8 * (n // 2 + 1) * n * n
    nbytes = (sum(smp.sweep_bytes().values())
              + 2 * spec + 2 * n_wg_x * w.n_bins * 8)        # rescaling pass, cross sums
    out = {
        "metric": "mixing sweeps/s at 256^3 FP32 (Alg. 3, shell form)",
        "value": round(1000.0 / ms, 2), "unit": "sweeps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "mixing-256^3-fp32-survey", "n": n, "n_bins": w.n_bins,
                   "sweep_bytes_algorithmic": nbytes,
                   "sweep_hbm_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
    }
    print(json.dumps(out), flush=True)


def wiener_grad_bytes(n: int, real_bytes: int, n_bins: int, n_iter: int, every: int,
                      coef_frac: float = 1.0) -> int:
    """Algorithmic HBM bytes of one chi2 forward + backward run of the
    messenger Wiener filter (K iterations, checkpoint every E): K plain
    iterations, K recomputed ones that store t^, K adjoint iterations that
    read it back and accumulate the adjoint field, plus set-up and read-out.
    coef_frac: share of the coefficients the z-pass reads (tiles with an
    observed voxel)."""
    m = n ** 3
    spec = 2 * real_bytes * (n // 2 + 1) * n * n  # half-complex field
    coef = 2 * real_bytes * m                      # (alpha, beta) per voxel
    zcoef = int(coef * coef_frac)
    field = real_bytes * m                         # one real field
    n_wg_x = (n // 2 + 1) * (n // x_columns(n))
    partials = 2 * n_wg_x * n_bins * 8
    n_ckpt = -(-n_iter // every)
    plain = 8 * spec + zcoef                       # z, y, x, y passes
    store = plain + spec                           # + t^ written
    adjoint = plain + spec + 2 * field + partials  # + t^ read, adjoint field summed
    forward_extra = (coef + 8 * m + coef           # data -> (alpha, beta)
                     + spec + 2 * spec * n_ckpt    # zero start, checkpoint copies
                     + spec + field                # s_K read-out
                     + coef + 8 * m + field)       # chi2
    backward_extra = (field + spec + 2 * spec * n_ckpt   # zeroing, checkpoint restores
                      + spec + field                     # s_K read-out
                      + spec + 2 * field                 # last adjoint field summed
                      + coef + 8 * m + 2 * field + 8 * m)  # d chi2 / d d
    return n_iter * (plain + store + adjoint) + forward_extra + backward_extra


def bench_wiener(args, chains: int = 1):
    """chi2 of the messenger Wiener filter and its gradient with respect to P
    and d: 128^3 survey problem, 32 bins, 50 iterations, checkpoint every 10;
    with chains > 1, that many data sets (seeds) of the same survey in one
    launch per pass."""
    import torch

    from paper_1402_1763_amd import binding, workloads
    torch.cuda.set_device(0)
    w = workloads.SURVEY_128_FP32
    n_iter, every = 50, 10
    pbs = [workloads.make_problem(w, seed=w.seed + 17 * c) for c in range(chains)]
    pb = pbs[0]
    smp = binding.Sampler([q["data"] for q in pbs], [q["noise_var"] for q in pbs],
                          [q["pk_init"] for q in pbs], w.n_bins, w.box,
                          seed=w.rng_seed, precision="fp32", sample_pk=False)
    pk1 = workloads.power_spectrum(workloads.bin_centres(w), w)
    if chains == 1:
        pk = torch.from_numpy(pk1).cuda()
        d = torch.from_numpy(pb["data"]).cuda()
        wf = binding.WienerFilter(smp, n_iter, every)
    else:
        pk = torch.from_numpy(np.stack([pk1] * chains)).cuda()
        d = torch.from_numpy(np.stack([q["data"] for q in pbs])).cuda()
        wf = binding.WienerFilter(smp, n_iter, every, chain=None)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        wf.forward(d, pk)
        wf.backward(d)
    torch.cuda.synchronize()
    start, mid, stop = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    fwd_ms = 0.0
    start.record(stream)
    for _ in range(args.steps):
        chi2, _ = wf.forward(d, pk)
        gd, gp = wf.backward(d)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    start.record(stream)
    wf.forward(d, pk)
    mid.record(stream)
    wf.backward(d)
    stop.record(stream)
    torch.cuda.synchronize()
    fwd_ms, bwd_ms = start.elapsed_time(mid), mid.elapsed_time(stop)
    assert bool(torch.isfinite(chi2).all()) and bool(torch.isfinite(gp).all())
    # the log-determinant term's trace estimator: 4 probes of n_iter iterations
    wf.logdet_trace(pk, 1)
    start.record(stream)
    tr = wf.logdet_trace(pk, 4)
    stop.record(stream)
    torch.cuda.synchronize()
    logdet_probe_ms = start.elapsed_time(stop) / 4
    assert bool(torch.isfinite(tr).all())
    gibbs_ms = plain_sweep_ms(w, pb, 200)
    spec = 8 * (w.n // 2 + 1) * w.n ** 2
    coef_frac = (smp.sweep_bytes()["zpass"] - 2 * spec * chains) / (8 * w.m * chains)
    nbytes = chains * wiener_grad_bytes(w.n, 4, w.n_bins, n_iter, every, coef_frac)
    out = {
        "metric": "messenger Wiener-filter chi2 + gradient evaluations/s (128^3, 50 iterations, "
                  "checkpoint every 10)" + (f", {chains} data sets per launch" if chains > 1 else ""),
        "value": round(chains * 1000.0 / ms, 2), "unit": "evaluations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": w.n, "n_bins": w.n_bins, "chains": chains,
                   "iterations": n_iter, "ckpt_every": every,
                   "forward_ms": round(fwd_ms, 4), "backward_ms": round(bwd_ms, 4),
                   "logdet_trace_ms_per_probe": round(logdet_probe_ms, 4),
                   "iterations_per_s": round(3 * n_iter * chains * 1000.0 / ms, 1),
                   "plain_gibbs_sweep_ms": round(gibbs_ms, 5),
                   "iteration_cost_vs_gibbs_sweep": round(ms / (3 * n_iter * chains) / gibbs_ms, 3),
                   "bytes_algorithmic": nbytes,
                   "hbm_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
    }
    if not args.no_cpu_baseline and chains == 1:
        out["cpu_baseline"] = wiener_cpu_baseline(w, pb, n_iter)
    print(json.dumps(out), flush=True)


def wiener_cpu_baseline(w, pb, n_iter: int) -> dict:
    """The oracle's reverse-mode gradient on the same problem, 5 iterations,
    scaled to 50."""
    ncores = len(os.sched_getaffinity(0))
    os.environ["ORACLE_FFT_WORKERS"] = str(ncores)
    from oracle import adjoint, sampler
    prob = sampler.make_problem(pb["data"], pb["noise_var"], w.n_bins, w.box, w.rng_seed)
    p_grid = workloads_power(w) / w.cell_volume
    k = 5
    t0 = time.perf_counter()
    adjoint.wf_gradient(prob, p_grid, k)
    dt = (time.perf_counter() - t0) * n_iter / k
    return {"value": round(1.0 / dt, 5), "unit": "evaluations/s", "cores": ncores,
            "kind": "oracle",
            "sample": f"oracle chi2 + reverse-mode gradient, {k} iterations of the same 128^3 "
                      f"problem, time scaled by {n_iter}/{k} (FP64, scipy.fft with {ncores} workers)"}


def workloads_power(w):
    from paper_1402_1763_amd import workloads
    return workloads.power_spectrum(workloads.bin_centres(w), w)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--burn-in", type=int, default=2000,
                    help="untimed sweeps of set-up before the warm-up (the chain's burn-in)")
    ap.add_argument("--segments", type=int, default=5,
                    help="timed segments of --steps sweeps each; the median is reported")
    ap.add_argument("--workload", default="gibbs-256^3-fp32-survey")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default path and tiles (for profiler runs)")
    ap.add_argument("--no-fp64-compare", action="store_true",
                    help="skip timing the same problem's FP64 sweep")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB ten times (calibrates "
                         "the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        src = torch.ones(args.calibrate_copy * 2 ** 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written":
                          dst.numel() * 4, "launches": 10}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: the sampler runs on one GPU "
              "(independent chains shard one per GPU; no multi-GPU figure is measured)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1402_1763_amd import binding, workloads

    if args.workload == "gibbs-batched-mixed":
        return bench_batched(args)
    if args.workload == "wiener-grad-128^3-fp32-survey":
        return bench_wiener(args)
    if args.workload == "wiener-grad-128^3-x8-fp32-survey":
        return bench_wiener(args, chains=8)
    if args.workload == "mixing-256^3-fp32-survey":
        return bench_mixing(args)
    if args.workload == "chain-efficiency-128^3-fp32-survey":
        return bench_chain_efficiency(args)
    w = workloads.WORKLOADS[args.workload]
    pb = workloads.make_problem(w)
    torch.cuda.set_device(0)
    smp = binding.Sampler(pb["data"], pb["noise_var"], pb["pk_init"], w.n_bins, w.box,
                          seed=w.rng_seed, precision=w.precision)
    stream = torch.cuda.current_stream()
    # set-up: picks the path and tiles, chain unchanged (profiling runs keep the
    # defaults to stay short)
    tune = smp.autotune(trials=30) if not args.no_autotune else dict(
        smp.tuning(), ms={"split": float("nan"), "whole": float("nan")},
        ms_x_tile=[float("nan")] * 3, ms_y_group=[float("nan")] * 3,
        ms_y_radix=[float("nan")] * 2)
    # set-up: the chain's burn-in, which also takes the GPU from its idle clock
    # (about 180 MHz) to its steady one before anything is timed
    smp.sweep(args.burn_in)
    smp.sweep(args.warmup)
    torch.cuda.synchronize()

    # `segments` timed segments of `steps` sweeps each, every one bracketed by
    # a device synchronisation on both sides; the median segment is the figure
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    seg_ms, wall_s = [], []
    for _ in range(args.segments):
        torch.cuda.synchronize()
        t_wall = time.perf_counter()
        start.record(stream)
        smp.sweep(args.steps)
        stop.record(stream)
        torch.cuda.synchronize()
        wall_s.append(time.perf_counter() - t_wall)
        seg_ms.append(start.elapsed_time(stop))
    ms_per_step = float(np.median(seg_ms)) / args.steps
    # context: one long segment right after (how far short segments sit from
    # a long chain's steady rate)
    long_sweeps = 1000
    torch.cuda.synchronize()
    start.record(stream)
    smp.sweep(long_sweeps)
    stop.record(stream)
    torch.cuda.synchronize()
    long_ms_per_step = start.elapsed_time(stop) / long_sweeps

    _, pk, n_done = smp.state(want_s=False)
    assert np.all(np.isfinite(pk))
    assert n_done == args.burn_in + args.warmup + args.segments * args.steps + long_sweeps

    real_bytes = 8 if w.precision == "fp64" else 4
    n = w.n
    alg = smp.sweep_bytes()
    sweep_bytes = sum(alg.values())

    roofline = None
    kernel_ms = None
    if not args.no_kernel_timing:
        kms = smp.sweep_timed(400)
        kernel_ms = dict(zip(binding.KERNEL_NAMES, [float(x) for x in kms]))
        # the same kernels started with the 256 MB last-level cache evicted
        # (a 1 GiB copy before each timed kernel): their inputs come from DRAM
        evict = torch.empty(2 ** 30, dtype=torch.uint8, device="cuda")
        cold_modes = {mode: dict(zip(binding.KERNEL_NAMES,
                                     [float(x) for x in smp.sweep_timed_cold(400, evict, mode)]))
                      for mode in binding.Sampler.EVICT_MODES}
        del evict
        cold_ms = cold_modes["read"]
        dom = max(kernel_ms, key=kernel_ms.get)
        achieved = alg[dom] / (kernel_ms[dom] * 1e-3) / 1e9
        traffic = load_traffic(dom, w.name)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic, "kernel": dom,
                    "algorithmic_bytes_per_launch": alg[dom],
                    "algorithmic_bytes": alg,
                    "kernel_ms": {k: round(v, 5) for k, v in kernel_ms.items()},
                    # every pass priced the same way (the dominant one is the
                    # longest; the z- and x-passes are within a few percent)
                    "per_kernel_frac": {k: round(alg[k] / (v * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                        for k, v in kernel_ms.items()},
                    # last-level cache evicted before each kernel: every byte it
                    # reads comes from DRAM
                    "kernel_ms_llc_evicted": {k: round(v, 5) for k, v in cold_ms.items()},
                    "per_kernel_frac_llc_evicted": {
                        k: round(alg[k] / (v * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                        for k, v in cold_ms.items()},
                    "llc_time_saving": {k: round(1.0 - kernel_ms[k] / cold_ms[k], 4)
                                        for k in kernel_ms},
                    "kernel_ms_llc_evicted_by_mode": {
                        m: {k: round(v, 5) for k, v in d.items()} for m, d in cold_modes.items()}}
    smp.close()
    fp64 = None if args.no_fp64_compare else fp64_sweep_rate(w, pb, min(args.steps, 100))
    stream_ref = hbm_reference()

    out = {
        "metric": "Gibbs sweeps/s at 256^3 FP32 (and % HBM roofline) vs plain FP64 sweep",
        "value": round(1000.0 / ms_per_step, 2),
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "box": w.box, "n_bins": w.n_bins,
                   "precision": "FP32 fields/FFTs/draws, FP64 shell sums and P draws",
                   "mask": "sphere r<0.45L minus seeded 30deg wedge",
                   "chains": 1,
                   "x_path": tune["path"],
                   "tuning": {k: tune[k] for k in ("x_tile", "y_group", "y_radix", "x_cols",
                                                   "x_k1", "x_hist", "y_units")},
                   "autotune_ms_per_sweep": {k: _r5(v) for k, v in tune["ms"].items()},
                   "autotune_ms_x_tile": [_r5(v) for v in tune["ms_x_tile"]],
                   "autotune_ms_y_group": [_r5(v) for v in tune["ms_y_group"]],
                   "autotune_ms_y_radix": [_r5(v) for v in tune["ms_y_radix"]],
                   "sweep_bytes_algorithmic": sweep_bytes,
                   "sweep_hbm_frac": round(sweep_bytes / (ms_per_step * 1e-3) / 1e9
                                           / HBM_PEAK_GBS, 4),
                   # the same rate priced at a five-pass schedule's 48.25 B/voxel
                   "sweep_hbm_frac_5pass_bytes": round(48.25 * w.m * real_bytes / 4
                                                       / (ms_per_step * 1e-3) / 1e9
                                                       / HBM_PEAK_GBS, 4),
                   "burn_in_sweeps": args.burn_in,
                   "timed_segments": args.segments,
                   "segment_ms_per_step": [round(v / args.steps, 5) for v in seg_ms],
                   "wall_s_timed_segments": [round(v, 4) for v in wall_s],
                   "long_segment_sweeps": long_sweeps,
                   "long_segment_sweeps_per_s": round(1000.0 / long_ms_per_step, 2),
                   "fp64_sweeps_per_s": fp64,
                   "hbm_reference": stream_ref,
                   "speedup_vs_fp64_sweep": (round(1000.0 / ms_per_step / fp64, 3)
                                             if fp64 else None)},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, pb)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
