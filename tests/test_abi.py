"""C-ABI checks that need no GPU: the library loads, exports every function
include/mf.h declares (and the binding declares the same set), and host-side
validation rejects bad descriptors and inputs with the documented status
before touching a device."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_1402_1763_amd import binding, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "mf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mf_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return binding.load()


def test_exports_every_declared_function(lib):
    names = header_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(binding.SIGNATURES), set(names) ^ set(binding.SIGNATURES)


def test_supported_sizes(lib):
    assert [n for n in range(4, 1100) if binding.mf_supported_n(n)] == [8, 16, 32, 48, 64, 80, 96, 128, 256, 512]


def test_workspace_bytes_and_descriptor_errors(lib):
    d = binding.make_desc(256, 64, 2000.0, 1, "fp32")
    ws = binding.mf_workspace_bytes(d)
    m = 256 ** 3
    # FP32: coefficients 8 B, 1 - alpha 4 B and staging 4 B per voxel, the half
    # spectrum, and two sets of shell partials [bin][x-pass workgroup] sized for
    # the x tile with the most workgroups (the lane-pair tile: 32 per kz plane)
    spectrum = 8 * (256 // 2 + 1) * 256 * 256
    partials = 2 * 64 * (256 // 2 + 1) * 32 * 8
    expected = 16 * m + spectrum + partials
    assert expected < ws < expected + (1 << 20)    # plus small tables and alignment
    d64 = binding.make_desc(256, 64, 2000.0, 1, "fp64")
    assert binding.mf_workspace_bytes(d64) > 1.9 * ws
    bad = [binding.make_desc(40, 16, 500.0, 1), binding.make_desc(32, 0, 500.0, 1),
           binding.make_desc(32, 16, -1.0, 1), binding.make_desc(32, 16, 500.0, 1, n_chains=0)]
    codes = []
    for desc in bad:
        with pytest.raises(binding.MFError) as e:
            binding.mf_workspace_bytes(desc)
        codes.append(e.value.status)
    assert codes == [binding.MF_E_UNSUPPORTED_SIZE, binding.MF_E_INVALID_ARG,
                     binding.MF_E_INVALID_ARG, binding.MF_E_INVALID_ARG]
    d.precision = 7
    with pytest.raises(binding.MFError):
        binding.mf_workspace_bytes(d)


def test_pk_prior_must_be_finite_and_non_negative(lib):
    """The InvGamma(a0, b0) prior on P: (0, 0) is Jeffreys' prior; negative
    or non-finite values are refused when the descriptor is checked."""
    ok = binding.make_desc(32, 16, 500.0, 1, pk_prior=(1.5, 4.0e5))
    assert binding.mf_workspace_bytes(ok) == binding.mf_workspace_bytes(
        binding.make_desc(32, 16, 500.0, 1))
    for bad in ((-1.0, 0.0), (0.0, -2.0), (float("nan"), 0.0), (0.0, float("inf"))):
        with pytest.raises(binding.MFError) as e:
            binding.mf_workspace_bytes(binding.make_desc(32, 16, 500.0, 1, pk_prior=bad))
        assert e.value.status == binding.MF_E_INVALID_ARG


def _init(desc, data, noise, pk, ws_ptr=256, ws_bytes=1 << 40):
    return binding.mf_init_problem(desc, [data], [noise], [pk], None, ws_ptr, ws_bytes, stream=0)


def test_init_validation_happens_on_the_host(lib):
    w = workloads.small_workload(8, 4)
    pb = workloads.make_problem(w)
    desc = binding.make_desc(8, 4, w.box, 1, "fp64")
    # tau above the smallest observed noise variance violates N - T > 0
    tmin = pb["noise_var"][np.isfinite(pb["noise_var"])].min()
    desc.tau = tmin * 1.01
    with pytest.raises(binding.MFError) as e:
        _init(desc, pb["data"], pb["noise_var"], pb["pk_init"])
    assert e.value.status == binding.MF_E_TAU
    desc.tau = 0.0
    noise = pb["noise_var"].copy()
    noise[1, 2, 3] = np.nan
    with pytest.raises(binding.MFError) as e:
        _init(desc, pb["data"], noise, pb["pk_init"])
    assert e.value.status == binding.MF_E_NONFINITE
    noise = pb["noise_var"].copy()
    noise[0, 0, 0] = -1.0
    with pytest.raises(binding.MFError) as e:
        _init(desc, pb["data"], noise, pb["pk_init"])
    assert e.value.status == binding.MF_E_NONFINITE
    data = pb["data"].copy()
    obs = np.argwhere(np.isfinite(pb["noise_var"]))[0]
    data[tuple(obs)] = np.inf
    with pytest.raises(binding.MFError) as e:
        _init(desc, data, pb["noise_var"], pb["pk_init"])
    assert e.value.status == binding.MF_E_NONFINITE
    with pytest.raises(binding.MFError) as e:
        _init(desc, pb["data"], np.full_like(noise, np.inf), pb["pk_init"])
    assert e.value.status == binding.MF_E_INVALID_ARG        # nothing observed
    pk = pb["pk_init"].copy()
    pk[2] = -1.0
    with pytest.raises(binding.MFError) as e:
        _init(desc, pb["data"], pb["noise_var"], pk)
    assert e.value.status == binding.MF_E_NONFINITE
    with pytest.raises(binding.MFError) as e:
        _init(desc, pb["data"], pb["noise_var"], pb["pk_init"], ws_ptr=0)
    assert e.value.status == binding.MF_E_WORKSPACE
    with pytest.raises(binding.MFError) as e:
        _init(desc, pb["data"], pb["noise_var"], pb["pk_init"], ws_ptr=256 + 8)
    assert e.value.status == binding.MF_E_WORKSPACE
    with pytest.raises(binding.MFError) as e:
        _init(desc, pb["data"], pb["noise_var"], pb["pk_init"], ws_bytes=1024)
    assert e.value.status == binding.MF_E_WORKSPACE
    assert "workspace" in binding.mf_last_error()


def test_response_validation_happens_on_the_host(lib):
    w = workloads.small_workload(8, 4)
    pb = workloads.make_problem(w)
    m = 8 ** 3
    plain = binding.make_desc(8, 4, w.box, 1, "fp64")
    with_r = binding.make_desc(8, 4, w.box, 1, "fp64", has_response=True)
    # the 1 / R array (FP64 per voxel) only with a response
    assert binding.mf_workspace_bytes(with_r) >= binding.mf_workspace_bytes(plain) + 8 * m
    resp = np.full((8,) * 3, 0.5)

    def init(desc, response):
        return binding.mf_init_problem(desc, [pb["data"]], [pb["noise_var"]], [pb["pk_init"]],
                                       None, 256, 1 << 40, stream=0, response=response)
    for desc, response in ((plain, [resp]), (with_r, None)):
        with pytest.raises(binding.MFError) as e:
            init(desc, response)
        assert e.value.status == binding.MF_E_INVALID_ARG
    bad = resp.copy()
    bad[3, 3, 3] = np.nan
    with pytest.raises(binding.MFError) as e:
        init(with_r, [bad])
    assert e.value.status == binding.MF_E_NONFINITE
    # the tau bound is min N / R^2 = 4 min N here
    tmin = pb["noise_var"][np.isfinite(pb["noise_var"])].min()
    with_r.tau = 4.0 * tmin * 1.01
    with pytest.raises(binding.MFError) as e:
        init(with_r, [resp])
    assert e.value.status == binding.MF_E_TAU
    assert "N / R^2" in binding.mf_last_error()
    with_r.tau = 0.0
    with pytest.raises(binding.MFError) as e:
        init(with_r, [np.zeros((8,) * 3)])
    assert e.value.status == binding.MF_E_INVALID_ARG        # R = 0 everywhere: nothing observed
    with_r.has_response = 2
    with pytest.raises(binding.MFError):
        binding.mf_workspace_bytes(with_r)


def test_null_handles_are_rejected(lib):
    assert lib.mf_gibbs_sweep(None, 1, None) == binding.MF_E_INVALID_ARG
    assert lib.mf_get_chain_state(None, 0, None, None, None, None) == binding.MF_E_INVALID_ARG
    assert lib.mf_graph_launch(None, 1, None) == binding.MF_E_INVALID_ARG
    assert lib.mf_wiener_logdet_trace(None, 0, None, 1, 1, 0, None, 0, None, None) == binding.MF_E_INVALID_ARG
    assert lib.mf_wiener_logdet_workspace_bytes(None, 0, None) == binding.MF_E_INVALID_ARG
    lib.mf_destroy_problem(None)
    lib.mf_graph_destroy(None)


def test_init_without_a_device_fails_after_the_host_set_up(lib):
    """With valid inputs the host set-up (validation, tau, bin thresholds, mode
    counts, twiddles) runs, then the first device call fails: MF_E_DEVICE and
    no handle.  Only where no GPU is visible."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible; the fake workspace pointer must not reach it")
    for n, nb, prec in ((8, 4, "fp64"), (48, 16, "fp32")):
        w = workloads.small_workload(n, nb)
        pb = workloads.make_problem(w)
        desc = binding.make_desc(n, nb, w.box, 1, prec, pk_prior=(0.5, 10.0))
        with pytest.raises(binding.MFError) as e:
            _init(desc, pb["data"], pb["noise_var"], pb["pk_init"])
        assert e.value.status == binding.MF_E_DEVICE
