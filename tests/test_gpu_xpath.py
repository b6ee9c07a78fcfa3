"""GPU tests of the two x-transform paths (split and whole pencils), of the
split path's tile variants, and of the autotuner that chooses among them."""
import numpy as np
import pytest

from oracle import mixing, sampler
from paper_1402_1763_amd import binding, workloads
from tests.gpu_util import TOL, errors, gpu_sampler, oracle_problem, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()
    torch.cuda.set_device(0)


@pytest.mark.parametrize("precision,n", [("fp64", 32), ("fp32", 48), ("fp64", 64), ("fp32", 80),
                                         ("fp32", 96), ("fp64", 128)])
def test_whole_path_matches_oracle(precision, n):
    w = workloads.small_workload(n, 8, precision=precision, seed=91, rng_seed=92)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    smp.set_x_path("whole")
    assert smp.x_path() == "whole"
    print(f"whole path n={n} {precision}", flush=True)
    smp.sweep(4)
    s_gpu, p_gpu, _ = smp.state()
    s_ref, p_ref = run_oracle(w, pb, 4)
    err_s, err_p = errors(s_gpu, p_gpu, s_ref, p_ref)
    print(f"  err_s={err_s:.3e} err_P={err_p:.3e}", flush=True)
    assert err_s < TOL[precision] and err_p < TOL[precision]


@pytest.mark.timeout(600)
def test_every_path_and_tile_at_256_matches_oracle():
    """The benchmarked 256^3 survey problem, 2 sweeps, on the whole-pencil path
    and on the split path with each x-tile variant and the reversed radix
    order, against the oracle (FP32, and FP64 for the lane-pair tile and the
    reversed order)."""
    w = workloads.SURVEY_256_MIXED
    pb = workloads.make_problem(w)
    print("256^3: oracle 2 sweeps", flush=True)
    s_ref, p_ref = run_oracle(w, pb, 2)
    for path, x_tile, y_radix in (("whole", 0, 0), ("split", 0, 0), ("split", 1, 0),
                                  ("split", 2, 0), ("split", 0, 1)):
        smp = gpu_sampler(w, pb)
        smp.set_tuning(path, x_tile, 0, y_radix)
        smp.sweep(2)
        s_gpu, p_gpu, _ = smp.state()
        geo = smp.tuning()
        smp.close()
        err_s, err_p = errors(s_gpu, p_gpu, s_ref, p_ref)
        print(f"  {path} x_tile={x_tile} ({geo['x_cols']} x {geo['x_k1']}, {geo['x_hist']} "
              f"histograms per wave) y_radix={y_radix}: err_s={err_s:.3e} "
              f"err_P={err_p:.3e}", flush=True)
        assert err_s < TOL["fp32"] and err_p < TOL["fp32"]
    # the same chain in FP64 mode (the oracle draws the same numbers) under the
    # lane-pair tile and the reversed radix order
    for x_tile, y_radix in ((2, 0), (0, 1)):
        smp = binding.Sampler(pb["data"], pb["noise_var"], pb["pk_init"], w.n_bins, w.box,
                              seed=w.rng_seed, precision="fp64")
        smp.set_tuning("split", x_tile, 0, y_radix)
        smp.sweep(2)
        s_gpu, p_gpu, _ = smp.state()
        smp.close()
        err_s, err_p = errors(s_gpu, p_gpu, s_ref, p_ref)
        print(f"  fp64 split x_tile={x_tile} y_radix={y_radix}: err_s={err_s:.3e} "
              f"err_P={err_p:.3e}", flush=True)
        assert err_s < TOL["fp64"] and err_p < TOL["fp64"]


@pytest.mark.parametrize("precision,n", [("fp32", 64), ("fp64", 96), ("fp32", 80), ("fp64", 128)])
@pytest.mark.parametrize("x_tile,y_group", [(1, 0), (2, 0), (0, 1), (0, 2)])
def test_tile_variants_match_oracle(precision, n, x_tile, y_group):
    """Each tile variant the autotuner may pick, x tiles and y groups, against
    the oracle over 3 sweeps."""
    w = workloads.small_workload(n, 8, precision=precision, seed=97, rng_seed=98)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    smp.set_tuning("split", x_tile, y_group)
    geo = smp.tuning()
    smp.sweep(3)
    s_gpu, p_gpu, _ = smp.state()
    smp.close()
    s_ref, p_ref = run_oracle(w, pb, 3)
    err_s, err_p = errors(s_gpu, p_gpu, s_ref, p_ref)
    print(f"n={n} {precision} x_tile={x_tile} ({geo['x_cols']} x {geo['x_k1']}, "
          f"{geo['x_hist']} histograms) "
          f"y_group={y_group} ({geo['y_units']} units): err_s={err_s:.3e} err_P={err_p:.3e}",
          flush=True)
    assert err_s < TOL[precision] and err_p < TOL[precision]


@pytest.mark.parametrize("precision,n", [("fp64", 32), ("fp32", 48), ("fp64", 80), ("fp32", 96),
                                         ("fp32", 128), ("fp64", 96)])
@pytest.mark.parametrize("y_group", [0, 1])
def test_reversed_y_radix_order_matches_oracle(precision, n, y_group):
    """The y transform's radix stages in reversed order (e.g. 4 x 4 x 6 at
    96), against the oracle over 3 sweeps."""
    w = workloads.small_workload(n, 8, precision=precision, seed=89, rng_seed=90)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    smp.set_tuning("split", 0, y_group, 1)
    assert smp.tuning()["y_radix"] == 1
    smp.sweep(3)
    s_gpu, p_gpu, _ = smp.state()
    smp.close()
    s_ref, p_ref = run_oracle(w, pb, 3)
    err_s, err_p = errors(s_gpu, p_gpu, s_ref, p_ref)
    print(f"n={n} {precision} y radix reversed, y_group={y_group}: err_s={err_s:.3e} "
          f"err_P={err_p:.3e}", flush=True)
    assert err_s < TOL[precision] and err_p < TOL[precision]


@pytest.mark.parametrize("n,expect", [
    # x tile -> (iy columns, k1 values, histograms per wave); y group -> units
    (256, {0: (128, 2, 8), 1: (128, 2, 2), 2: (128, 1, 8), "y": (1, 1, 1)}),
    (128, {0: (128, 2, 8), 1: (128, 2, 2), 2: (128, 1, 8), "y": (4, 2, 1)}),
    (96, {0: (32, 6, 8), 1: (32, 6, 2), 2: (96, 1, 8), "y": (4, 2, 1)}),
    (64, {0: (64, 4, 8), 1: (64, 4, 2), 2: (64, 2, 8), "y": (16, 8, 4)}),
])
def test_tuning_reports_the_documented_geometry(n, expect):
    """mf_get_tuning's geometry of every variant: the rule tile (128 columns x
    256/128 k1 values from 128 up), its 2-histogram twin, the lane-pair tile
    (two lanes per column) and the y groups G, G/2, G/4."""
    w = workloads.small_workload(n, 8, precision="fp32", seed=85, rng_seed=86)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    for x_tile in range(3):
        smp.set_tuning("split", x_tile, 0)
        t = smp.tuning()
        assert (t["x_cols"], t["x_k1"], t["x_hist"]) == expect[x_tile], (x_tile, t)
    for y_group in range(3):
        smp.set_tuning("split", 0, y_group)
        assert smp.tuning()["y_units"] == expect["y"][y_group], (y_group, smp.tuning())
    smp.set_tuning("whole", 0, 0)
    t = smp.tuning()
    assert (t["x_cols"], t["x_k1"], t["x_hist"], t["y_units"], t["y_radix"]) == (0, 0, 0, 0, 0)
    smp.close()


def test_tuning_errors():
    w = workloads.small_workload(32, 4, precision="fp32", seed=99, rng_seed=100)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    for bad in ((3, 0, 0), (0, -1, 0), (0, 0, 2), (0, 0, -1)):
        with pytest.raises(binding.MFError) as e:
            smp.set_tuning("split", *bad)
        assert e.value.status == binding.MF_E_INVALID_ARG
    t = smp.tuning()
    assert (t["x_tile"], t["y_group"], t["y_radix"]) == (0, 0, 0)   # the defaults
    smp.close()
    # 8 histograms per wave (x tiles 0 and 2) hold at most 255 bins
    w = workloads.small_workload(32, 300, precision="fp32", seed=99, rng_seed=100)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    assert smp.tuning()["x_tile"] == 1          # the default above 255 bins
    for x_tile in (0, 2):
        with pytest.raises(binding.MFError) as e:
            smp.set_tuning("split", x_tile, 0)
        assert e.value.status == binding.MF_E_INVALID_ARG
    res = smp.autotune(trials=1)
    assert np.isnan(res["ms_x_tile"][0]) and np.isnan(res["ms_x_tile"][2])
    assert res["path"] == "whole" or res["x_tile"] == 1
    smp.close()


def test_switching_paths_mid_chain_matches_oracle():
    w = workloads.small_workload(64, 8, precision="fp64", seed=93, rng_seed=94)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    for path in ("split", "whole", "split", "whole"):
        smp.set_x_path(path)
        smp.sweep(1)
    smp.mixing_sweep(1)          # always on the split path
    s_gpu, p_gpu, _ = smp.state()
    prob = oracle_problem(w, pb)
    st = sampler.State(s=np.zeros((w.n,) * 3), p_grid=pb["pk_init"] / w.cell_volume)
    st = sampler.run_chain(prob, st, 4)
    st = mixing.mixing_sweep(prob, st)
    err_s, err_p = errors(s_gpu, p_gpu, st.s, st.p_grid * w.cell_volume)
    assert err_s < TOL["fp64"] and err_p < TOL["fp64"]


def test_autotune_keeps_the_chain_and_picks_a_path():
    w = workloads.small_workload(64, 8, precision="fp32", seed=95, rng_seed=96)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    smp.set_diagnostics(start=0, thin=1, trace_cap=16, moments=True)
    smp.sweep(3)
    s0, p0, n0 = smp.state()
    rec0 = smp.recorded()
    res = smp.autotune(trials=3)
    print("autotune", res, flush=True)
    assert res["path"] in ("split", "whole") and smp.x_path() == res["path"]
    assert all(np.isfinite(v) and v > 0 for v in res["ms"].values())
    assert all(np.isfinite(v) and v > 0 for v in res["ms_x_tile"])
    assert smp.tuning() == {k: v for k, v in res.items() if not k.startswith("ms")}
    s1, p1, n1 = smp.state()
    assert np.array_equal(s0, s1) and np.array_equal(p0, p1) and n0 == n1
    assert smp.recorded() == rec0
    smp.sweep(2)
    # the tuned chain equals an untuned one that ran its first three sweeps on
    # the default path and the last two on the chosen one
    ref2 = gpu_sampler(w, pb)
    ref2.sweep(3)
    ref2.set_tuning(res["path"], res["x_tile"], res["y_group"], res["y_radix"])
    ref2.sweep(2)
    assert np.array_equal(smp.state()[0], ref2.state()[0])
    # 8 x 8 at 64 reads the same both ways: the radix order is not timed
    assert all(np.isnan(v) for v in res["ms_y_radix"])


def test_autotune_times_the_radix_order_where_it_differs():
    w = workloads.small_workload(48, 8, precision="fp32", seed=87, rng_seed=88)
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    res = smp.autotune(trials=2)
    print("autotune 48^3", res, flush=True)
    assert all(np.isfinite(v) and v > 0 for v in res["ms_y_radix"])
    assert res["path"] == "whole" or res["y_radix"] in (0, 1)
    assert smp.tuning() == {k: v for k, v in res.items() if not k.startswith("ms")}
    smp.close()


def test_graph_keeps_the_tiles_it_captured():
    """A graph replays the path, tile variants and radix order chosen when it
    was created: retuning the problem afterwards changes its eager sweeps
    only."""
    w = workloads.small_workload(48, 8, precision="fp32", seed=97, rng_seed=98)
    pb = workloads.make_problem(w)
    smp, ref = gpu_sampler(w, pb), gpu_sampler(w, pb)
    smp.set_tuning("split", 2, 1, 1)
    ref.set_tuning("split", 2, 1, 1)
    g = binding.SweepGraph([smp])
    smp.set_tuning("whole", 0, 0)
    g.launch(3)
    ref.sweep(3)
    assert np.array_equal(smp.state()[0], ref.state()[0])
    assert np.array_equal(smp.state()[1], ref.state()[1])
    smp.sweep(2)                       # eager sweeps take the new choice
    ref.set_tuning("whole", 0, 0)
    ref.sweep(2)
    assert np.array_equal(smp.state()[0], ref.state()[0])
    g.close()
    smp.close()
    ref.close()


def test_path_errors_and_small_grids():
    w = workloads.small_workload(16, 4, precision="fp32")
    pb = workloads.make_problem(w)
    smp = gpu_sampler(w, pb)
    assert smp.x_path() == "whole"
    with pytest.raises(binding.MFError) as e:
        smp.set_x_path("split")
    assert e.value.status == binding.MF_E_UNSUPPORTED_SIZE
    res = smp.autotune(trials=1)
    assert res["path"] == "whole" and np.isnan(res["ms"]["split"])
