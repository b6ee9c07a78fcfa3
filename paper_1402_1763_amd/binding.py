"""ctypes binding of libmfgibbs.so (the C ABI in include/mf.h).

Argument marshalling only: every step of a sweep runs in the library's HIP
kernels.  PyTorch provides the device workspace and the stream.  The module
raises ImportError-like errors when the library has not been built; there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# MFGIBBS_LIB selects another build of the same library (e.g. tuned variants).
LIB_PATH = os.environ.get("MFGIBBS_LIB") or os.path.join(HERE, "libmfgibbs.so")

MF_OK = 0
MF_E_INVALID_ARG = -1
MF_E_UNSUPPORTED_SIZE = -2
MF_E_TAU = -3
MF_E_NONFINITE = -4
MF_E_DEVICE = -5
MF_E_WORKSPACE = -6
MF_E_STATE = -7
MF_PREC_FP64 = 0
MF_PREC_FP32 = 1
MF_NUM_KERNELS = 4
KERNEL_NAMES = ("zpass", "yfwd", "xpass", "yinv_pk")

# Symbols declared in include/mf.h, with their ctypes signatures.
_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_double_pp = ctypes.POINTER(_c_double_p)


class mf_chain_desc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("n_bins", ctypes.c_int32),
        ("box", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("chain_id", ctypes.c_uint32),
        ("precision", ctypes.c_int32),
        ("sample_pk", ctypes.c_int32),
        ("n_chains", ctypes.c_int32),
        ("has_response", ctypes.c_int32),
        ("pk_prior_shape", ctypes.c_double),
        ("pk_prior_scale", ctypes.c_double),
    ]


class mf_tuning(ctypes.Structure):
    _fields_ = [
        ("x_path", ctypes.c_int32),
        ("x_tile", ctypes.c_int32),
        ("y_group", ctypes.c_int32),
        ("x_cols", ctypes.c_int32),
        ("x_k1", ctypes.c_int32),
        ("y_units", ctypes.c_int32),
        ("x_hist", ctypes.c_int32),
        ("y_radix", ctypes.c_int32),
    ]


MF_TUNE_SLOTS = 10

SIGNATURES = {
    "mf_supported_n": (ctypes.c_int32, [ctypes.c_int32]),
    "mf_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(mf_chain_desc),
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "mf_init_problem": (ctypes.c_int, [ctypes.POINTER(mf_chain_desc), _c_double_pp, _c_double_pp,
                                       _c_double_pp, _c_double_pp, _c_double_pp, ctypes.c_void_p,
                                       ctypes.c_size_t, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_void_p)]),
    "mf_gibbs_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "mf_mixing_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "mf_gibbs_sweep_timed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            _c_double_p, ctypes.c_int32]),
    "mf_gibbs_sweep_timed_cold": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                                 ctypes.c_void_p, _c_double_p, ctypes.c_int32,
                                                 ctypes.c_void_p, ctypes.c_size_t,
                                                 ctypes.c_int32]),
    "mf_get_chain_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _c_double_p,
                                          _c_double_p, ctypes.POINTER(ctypes.c_uint64),
                                          ctypes.c_void_p]),
    "mf_set_chain_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _c_double_p,
                                          _c_double_p, ctypes.c_uint64, ctypes.c_void_p]),
    "mf_get_tau": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _c_double_p]),
    "mf_sweep_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "mf_set_x_path": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "mf_get_x_path": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "mf_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, _c_double_p,
                                   ctypes.POINTER(mf_tuning)]),
    "mf_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(mf_tuning)]),
    "mf_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(mf_tuning)]),
    "mf_debug_run_kernel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64,
                                           ctypes.c_void_p]),
    "mf_debug_spectrum": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _c_double_p,
                                         ctypes.c_int32, ctypes.c_void_p]),
    "mf_checkpoint_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "mf_save_checkpoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_void_p]),
    "mf_load_checkpoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_void_p]),
    "mf_graph_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "mf_graph_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "mf_graph_destroy": (None, [ctypes.c_void_p]),
    "mf_wiener_workspace_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                                 ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "mf_wiener_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "mf_wiener_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "mf_wiener_logdet_workspace_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                                        ctypes.POINTER(ctypes.c_size_t)]),
    "mf_wiener_logdet_trace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                              ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32,
                                              ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                              ctypes.c_void_p]),
    "mf_wiener_logdet_trace_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                                      ctypes.c_void_p, ctypes.c_int32,
                                                      ctypes.c_int32, ctypes.c_uint32,
                                                      ctypes.c_void_p, ctypes.c_void_p]),
    "mf_stream_reference": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                           ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]),
    "mf_diagnostics_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_size_t),
                                            ctypes.POINTER(ctypes.c_size_t)]),
    "mf_set_diagnostics": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_void_p]),
    "mf_recorded_samples": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "mf_get_moments": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "mf_acf": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mf_destroy_problem": (None, [ctypes.c_void_p]),
    "mf_last_error": (ctypes.c_char_p, []),
}

_lib = None


class MFError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"mf status {status}: {message}")
        self.status = status


def load() -> ctypes.CDLL:
    """Load the built library; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                               "(the sampler has no non-HIP implementation)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, argtypes) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = argtypes
        _lib = lib
    return _lib


def _check(status: int):
    if status != MF_OK:
        raise MFError(status, load().mf_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_c_double_p)


def _ptr_array(arrays):
    arr = (_c_double_p * len(arrays))()
    for i, a in enumerate(arrays):
        arr[i] = _dptr(a) if a is not None else _c_double_p()
    return arr


def make_desc(n: int, n_bins: int, box: float, seed: int, precision: str = "fp32",
              tau: float = 0.0, chain_id: int = 0, sample_pk: bool = True,
              n_chains: int = 1, has_response: bool = False,
              pk_prior=(0.0, 0.0)) -> mf_chain_desc:
    prec = {"fp64": MF_PREC_FP64, "fp32": MF_PREC_FP32}[precision]
    return mf_chain_desc(n=n, n_bins=n_bins, box=box, tau=tau, seed=seed, chain_id=chain_id,
                         precision=prec, sample_pk=1 if sample_pk else 0, n_chains=n_chains,
                         has_response=1 if has_response else 0,
                         pk_prior_shape=float(pk_prior[0]), pk_prior_scale=float(pk_prior[1]))


def mf_supported_n(n: int) -> bool:
    return bool(load().mf_supported_n(n))


def mf_workspace_bytes(desc: mf_chain_desc) -> int:
    out = ctypes.c_size_t(0)
    _check(load().mf_workspace_bytes(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(stream)


def mf_init_problem(desc: mf_chain_desc, data: Sequence, noise_var: Sequence, pk_init: Sequence,
                    s_init: Optional[Sequence], workspace_ptr: int, workspace_bytes: int,
                    stream=None, response: Optional[Sequence] = None) -> int:
    data = [_f64(a) for a in data]
    noise_var = [_f64(a) for a in noise_var]
    pk_init = [_f64(a) for a in pk_init]
    s_list = None if s_init is None else [None if a is None else _f64(a) for a in s_init]
    r_list = None if response is None else [_f64(a) for a in response]
    handle = ctypes.c_void_p()
    _check(load().mf_init_problem(
        ctypes.byref(desc), _ptr_array(data), _ptr_array(noise_var),
        _ptr_array(r_list) if r_list is not None else None, _ptr_array(pk_init),
        _ptr_array(s_list) if s_list is not None else None, ctypes.c_void_p(workspace_ptr),
        workspace_bytes, ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(handle)))
    return handle.value


def mf_gibbs_sweep(handle: int, n_sweeps: int, stream=None):
    _check(load().mf_gibbs_sweep(ctypes.c_void_p(handle), n_sweeps,
                                 ctypes.c_void_p(_stream_ptr(stream))))


def mf_gibbs_sweep_timed(handle: int, n_sweeps: int, stream=None) -> np.ndarray:
    out = np.zeros(MF_NUM_KERNELS, dtype=np.float64)
    _check(load().mf_gibbs_sweep_timed(ctypes.c_void_p(handle), n_sweeps,
                                       ctypes.c_void_p(_stream_ptr(stream)), _dptr(out),
                                       MF_NUM_KERNELS))
    return out


def mf_get_chain_state(handle: int, chain: int, n: int, n_bins: int, stream=None,
                       want_s: bool = True):
    s = np.empty((n, n, n), dtype=np.float64) if want_s else None
    pk = np.empty(n_bins, dtype=np.float64)
    sweep = ctypes.c_uint64(0)
    _check(load().mf_get_chain_state(ctypes.c_void_p(handle), chain,
                                     _dptr(s) if s is not None else None, _dptr(pk),
                                     ctypes.byref(sweep), ctypes.c_void_p(_stream_ptr(stream))))
    return s, pk, sweep.value


def mf_set_chain_state(handle: int, chain: int, s, pk, sweep: int, stream=None):
    s = None if s is None else _f64(s)
    pk = None if pk is None else _f64(pk)
    _check(load().mf_set_chain_state(ctypes.c_void_p(handle), chain,
                                     _dptr(s) if s is not None else None,
                                     _dptr(pk) if pk is not None else None, sweep,
                                     ctypes.c_void_p(_stream_ptr(stream))))


def mf_get_tau(handle: int, chain: int = 0) -> float:
    out = ctypes.c_double(0.0)
    _check(load().mf_get_tau(ctypes.c_void_p(handle), chain, ctypes.byref(out)))
    return out.value


def mf_debug_run_kernel(handle: int, kernel: int, sweep: int, stream=None):
    _check(load().mf_debug_run_kernel(ctypes.c_void_p(handle), kernel, sweep,
                                      ctypes.c_void_p(_stream_ptr(stream))))


def mf_debug_spectrum(handle: int, chain: int, n: int, buf: Optional[np.ndarray] = None,
                      stream=None) -> np.ndarray:
    """Read (buf None) or write (buf given) the half-complex working buffer,
    shaped (N/2+1, N, N) complex [kz][ix][iy]."""
    shape = (n // 2 + 1, n, n)
    if buf is None:
        out = np.empty(shape + (2,), dtype=np.float64)
        _check(load().mf_debug_spectrum(ctypes.c_void_p(handle), chain, _dptr(out), 0,
                                        ctypes.c_void_p(_stream_ptr(stream))))
        return out[..., 0] + 1j * out[..., 1]
    arr = np.ascontiguousarray(np.stack([buf.real, buf.imag], axis=-1), dtype=np.float64)
    _check(load().mf_debug_spectrum(ctypes.c_void_p(handle), chain, _dptr(arr), 1,
                                    ctypes.c_void_p(_stream_ptr(stream))))
    return buf


def mf_checkpoint_bytes(handle: int) -> int:
    out = ctypes.c_size_t(0)
    _check(load().mf_checkpoint_bytes(ctypes.c_void_p(handle), ctypes.byref(out)))
    return out.value


def mf_save_checkpoint(handle: int, chain: int, stream=None) -> bytes:
    n = mf_checkpoint_bytes(handle)
    buf = ctypes.create_string_buffer(n)
    _check(load().mf_save_checkpoint(ctypes.c_void_p(handle), chain, buf, n,
                                     ctypes.c_void_p(_stream_ptr(stream))))
    return buf.raw


def mf_load_checkpoint(handle: int, chain: int, data: bytes, stream=None):
    buf = ctypes.create_string_buffer(data, len(data))
    _check(load().mf_load_checkpoint(ctypes.c_void_p(handle), chain, buf, len(data),
                                     ctypes.c_void_p(_stream_ptr(stream))))


def mf_graph_create(handles: Sequence[int], stream=None) -> int:
    arr = (ctypes.c_void_p * len(handles))(*handles)
    out = ctypes.c_void_p()
    _check(load().mf_graph_create(arr, len(handles), ctypes.c_void_p(_stream_ptr(stream)),
                                  ctypes.byref(out)))
    return out.value


def mf_graph_launch(graph: int, n_sweeps: int, stream=None):
    _check(load().mf_graph_launch(ctypes.c_void_p(graph), n_sweeps,
                                  ctypes.c_void_p(_stream_ptr(stream))))


def mf_graph_destroy(graph: int):
    if graph:
        load().mf_graph_destroy(ctypes.c_void_p(graph))


def mf_wiener_workspace_bytes(handle: int, chain: int, n_iter: int, ckpt_every: int) -> int:
    out = ctypes.c_size_t(0)
    _check(load().mf_wiener_workspace_bytes(ctypes.c_void_p(handle), chain, n_iter, ckpt_every,
                                            ctypes.byref(out)))
    return out.value


def mf_wiener_forward(handle: int, chain: int, d_ptr: int, pk_ptr: int, n_iter: int,
                      ckpt_every: int, ws_ptr: int, ws_bytes: int, chi2_ptr: int,
                      s_ptr: Optional[int], stream=None):
    _check(load().mf_wiener_forward(ctypes.c_void_p(handle), chain, ctypes.c_void_p(d_ptr),
                                    ctypes.c_void_p(pk_ptr), n_iter, ckpt_every,
                                    ctypes.c_void_p(ws_ptr), ws_bytes, ctypes.c_void_p(chi2_ptr),
                                    ctypes.c_void_p(s_ptr or None),
                                    ctypes.c_void_p(_stream_ptr(stream))))


def mf_wiener_backward(handle: int, chain: int, d_ptr: int, ws_ptr: int, ws_bytes: int,
                       grad_d_ptr: int, grad_pk_ptr: int, stream=None):
    _check(load().mf_wiener_backward(ctypes.c_void_p(handle), chain, ctypes.c_void_p(d_ptr),
                                     ctypes.c_void_p(ws_ptr), ws_bytes,
                                     ctypes.c_void_p(grad_d_ptr), ctypes.c_void_p(grad_pk_ptr),
                                     ctypes.c_void_p(_stream_ptr(stream))))


def mf_destroy_problem(handle: int):
    if handle:
        load().mf_destroy_problem(ctypes.c_void_p(handle))


def mf_last_error() -> str:
    return load().mf_last_error().decode()


class Sampler:
    """A problem on cuda:0 with a torch-owned workspace.

    data, noise_var: (N, N, N) float64 arrays (or lists of them, one per
    chain); noise_var = +inf marks unobserved voxels.  response: None (R = 1)
    or the per-voxel response R of the data model d = R s + eps, in the same
    form (R = 0 also marks unobserved voxels).  pk_init: initial P per bin in
    physical units.  pk_prior: (a0, b0) of the InvGamma prior on P, b0 in
    physical units; (0, 0) is Jeffreys' prior."""

    def __init__(self, data, noise_var, pk_init, n_bins: int, box: float, seed: int,
                 precision: str = "fp32", tau: float = 0.0, chain_id: int = 0,
                 sample_pk: bool = True, s_init=None, device: str = "cuda", response=None,
                 pk_prior=(0.0, 0.0)):
        import torch
        multi = isinstance(data, (list, tuple))
        data_l = list(data) if multi else [data]
        noise_l = list(noise_var) if multi else [noise_var]
        pk_l = list(pk_init) if multi else [pk_init]
        s_l = None if s_init is None else (list(s_init) if multi else [s_init])
        r_l = None if response is None else (list(response) if multi else [response])
        self.n = int(np.shape(data_l[0])[0])
        self.n_bins = n_bins
        self.n_chains = len(data_l)
        self.desc = make_desc(self.n, n_bins, box, seed, precision, tau, chain_id, sample_pk,
                              self.n_chains, has_response=response is not None,
                              pk_prior=pk_prior)
        self.workspace_bytes = mf_workspace_bytes(self.desc)
        self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        self._ptr = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream()
        self.handle = mf_init_problem(self.desc, data_l, noise_l, pk_l, s_l, self._ptr,
                                      self.workspace_bytes, self.stream.cuda_stream, r_l)

    def sweep(self, n_sweeps: int = 1):
        mf_gibbs_sweep(self.handle, n_sweeps, self.stream.cuda_stream)

    def mixing_sweep(self, n_sweeps: int = 1):
        """Mixing sweeps (joint (s^, P) update given the messenger field)."""
        _check(load().mf_mixing_sweep(ctypes.c_void_p(self.handle), n_sweeps,
                                      ctypes.c_void_p(self.stream.cuda_stream)))

    def sweep_timed(self, n_sweeps: int) -> np.ndarray:
        return mf_gibbs_sweep_timed(self.handle, n_sweeps, self.stream.cuda_stream)

    EVICT_MODES = ("copy", "read", "copy_read")

    def sweep_timed_cold(self, n_sweeps: int, evict, mode: str = "read") -> np.ndarray:
        """Per-kernel mean ms, every timed kernel started after `evict` (a cuda
        tensor far larger than the last-level cache) was streamed through
        (copied, read, or both)."""
        out = np.zeros(MF_NUM_KERNELS, dtype=np.float64)
        nbytes = evict.numel() * evict.element_size() // 32 * 32
        _check(load().mf_gibbs_sweep_timed_cold(ctypes.c_void_p(self.handle), n_sweeps,
                                                ctypes.c_void_p(self.stream.cuda_stream),
                                                _dptr(out), MF_NUM_KERNELS,
                                                ctypes.c_void_p(evict.data_ptr()), nbytes,
                                                self.EVICT_MODES.index(mode)))
        return out

    def state(self, chain: int = 0, want_s: bool = True):
        return mf_get_chain_state(self.handle, chain, self.n, self.n_bins,
                                  self.stream.cuda_stream, want_s)

    def set_state(self, chain: int, s, pk, sweep: int):
        mf_set_chain_state(self.handle, chain, s, pk, sweep, self.stream.cuda_stream)

    X_PATHS = ("split", "whole")

    def set_x_path(self, path: str):
        _check(load().mf_set_x_path(ctypes.c_void_p(self.handle), self.X_PATHS.index(path)))

    def x_path(self) -> str:
        out = ctypes.c_int32(0)
        _check(load().mf_get_x_path(ctypes.c_void_p(self.handle), ctypes.byref(out)))
        return self.X_PATHS[out.value]

    def tuning(self) -> dict:
        """The path, the split-path tile variants and the geometry they stand for."""
        t = mf_tuning()
        _check(load().mf_get_tuning(ctypes.c_void_p(self.handle), ctypes.byref(t)))
        return {"path": self.X_PATHS[t.x_path], "x_tile": t.x_tile, "y_group": t.y_group,
                "y_radix": t.y_radix, "x_cols": t.x_cols, "x_k1": t.x_k1,
                "y_units": t.y_units, "x_hist": t.x_hist}

    def set_tuning(self, path: str = "split", x_tile: int = 0, y_group: int = 0,
                   y_radix: int = 0):
        t = mf_tuning(x_path=self.X_PATHS.index(path), x_tile=x_tile, y_group=y_group,
                      y_radix=y_radix)
        _check(load().mf_set_tuning(ctypes.c_void_p(self.handle), ctypes.byref(t)))

    def autotune(self, trials: int = 20) -> dict:
        """Search the x path and the split path's tile variants and keep the
        fastest; returns the pick (as tuning()) with the timings:
        "ms" {"split", "whole"}, "ms_x_tile" [3], "ms_y_group" [3],
        "ms_y_radix" [2] (NaN where a candidate is not available or equals
        another).  State unchanged."""
        ms = (ctypes.c_double * MF_TUNE_SLOTS)()
        t = mf_tuning()
        _check(load().mf_autotune(ctypes.c_void_p(self.handle), trials,
                                  ctypes.c_void_p(self.stream.cuda_stream), ms, ctypes.byref(t)))
        out = self.tuning()
        out["ms"] = {"split": ms[0], "whole": ms[1]}
        out["ms_x_tile"] = [ms[2], ms[3], ms[4]]
        out["ms_y_group"] = [ms[5], ms[6], ms[7]]
        out["ms_y_radix"] = [ms[8], ms[9]]
        return out

    def sweep_bytes(self) -> dict:
        """Algorithmic HBM bytes of one sweep per kernel (all chains)."""
        out = (ctypes.c_size_t * MF_NUM_KERNELS)()
        _check(load().mf_sweep_bytes(ctypes.c_void_p(self.handle), out))
        return dict(zip(KERNEL_NAMES, (int(v) for v in out)))

    def tau(self, chain: int = 0) -> float:
        return mf_get_tau(self.handle, chain)

    def save_checkpoint(self, chain: int = 0) -> bytes:
        return mf_save_checkpoint(self.handle, chain, self.stream.cuda_stream)

    def load_checkpoint(self, data: bytes, chain: int = 0):
        mf_load_checkpoint(self.handle, chain, data, self.stream.cuda_stream)

    def set_diagnostics(self, start: int = 0, thin: int = 1, trace_cap: int = 0,
                        moments: bool = False):
        """Record samples start, start + thin, ...: P traces (trace_cap
        samples per chain) and/or Welford moments of s, in torch-owned device
        buffers."""
        import torch
        tb, mb = ctypes.c_size_t(0), ctypes.c_size_t(0)
        _check(load().mf_diagnostics_bytes(ctypes.c_void_p(self.handle), trace_cap,
                                           ctypes.byref(tb), ctypes.byref(mb)))
        dev = self.workspace.device
        trace_buf = (torch.zeros(self.n_chains, trace_cap, self.n_bins, dtype=torch.float64,
                                 device=dev) if trace_cap > 0 else None)
        moment_buf = (torch.empty(mb.value // 8, dtype=torch.float64, device=dev)
                      if moments else None)
        _check(load().mf_set_diagnostics(
            ctypes.c_void_p(self.handle), start, thin,
            ctypes.c_void_p(trace_buf.data_ptr() if trace_buf is not None else None),
            trace_cap,
            ctypes.c_void_p(moment_buf.data_ptr() if moment_buf is not None else None),
            ctypes.c_void_p(self.stream.cuda_stream)))
        # only now may the previous buffers go: the library refuses the call
        # (and keeps recording into them) while a graph holds their addresses
        self.trace_buf, self.moment_buf = trace_buf, moment_buf

    def recorded(self) -> int:
        out = ctypes.c_uint64(0)
        _check(load().mf_recorded_samples(ctypes.c_void_p(self.handle), ctypes.byref(out)))
        return out.value

    def trace(self, chain: int = 0):
        """Recorded P_b samples of a chain, a (count, n_bins) float64 cuda tensor."""
        k = min(self.recorded(), self.trace_buf.shape[1])
        return self.trace_buf[chain, :k]

    def moments(self, chain: int = 0):
        """(mean, variance) of the recorded s samples as (N, N, N) float64 cuda tensors."""
        import torch
        n = self.n
        mean = torch.empty((n, n, n), dtype=torch.float64, device=self.workspace.device)
        var = torch.empty_like(mean)
        _check(load().mf_get_moments(ctypes.c_void_p(self.handle), chain,
                                     ctypes.c_void_p(mean.data_ptr()),
                                     ctypes.c_void_p(var.data_ptr()),
                                     ctypes.c_void_p(self.stream.cuda_stream)))
        return mean, var

    def close(self):
        if getattr(self, "handle", None):
            mf_destroy_problem(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SweepGraph:
    """One HIP graph that sweeps several samplers (independent chains of any
    sizes) once per replay."""

    def __init__(self, samplers: Sequence["Sampler"]):
        import torch
        self.samplers = list(samplers)
        self.stream = torch.cuda.current_stream()
        self.handle = mf_graph_create([smp.handle for smp in self.samplers],
                                      self.stream.cuda_stream)

    def launch(self, n_sweeps: int = 1):
        mf_graph_launch(self.handle, n_sweeps, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "handle", None):
            mf_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class WienerFilter:
    """The deterministic messenger Wiener filter of a Sampler's chain (its
    noise model: N, mask, tau), n_iter iterations from s = 0 with a
    checkpoint every ckpt_every, and its adjoint.  chain=None runs every chain
    of the sampler in the same launches.  d and pk are float64 cuda tensors:
    (N, N, N) and (n_bins,) for one chain, with a leading chain axis for all
    chains; P in physical units."""

    def __init__(self, sampler: "Sampler", n_iter: int, ckpt_every: int, chain: Optional[int] = 0):
        import torch
        self.sampler, self.n_iter, self.ckpt_every = sampler, n_iter, ckpt_every
        self.chain = -1 if chain is None else chain
        self.n_chains = sampler.n_chains if chain is None else 1
        self.ws_bytes = mf_wiener_workspace_bytes(sampler.handle, self.chain, n_iter, ckpt_every)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8,
                                     device=sampler.workspace.device)
        self._ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.generation = 0      # increments with every forward run

    def _lead(self):
        return () if self.chain >= 0 else (self.n_chains,)

    def _check_inputs(self, d, pk):
        import torch
        n, nb = self.sampler.n, self.sampler.n_bins
        for name, t, shape in (("d", d, self._lead() + (n, n, n)), ("pk", pk, self._lead() + (nb,))):
            if (t.dtype != torch.float64 or not t.is_cuda or tuple(t.shape) != shape
                    or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float64 cuda tensor of shape {shape}")

    def forward(self, d, pk, want_s: bool = False):
        """chi2_K (a 0-dim tensor, or one per chain), and s_K when want_s."""
        import torch
        self._check_inputs(d, pk)
        chi2 = torch.empty(self._lead(), dtype=torch.float64, device=d.device)
        s = torch.empty_like(d) if want_s else None
        mf_wiener_forward(self.sampler.handle, self.chain, d.data_ptr(), pk.data_ptr(),
                          self.n_iter, self.ckpt_every, self._ptr, self.ws_bytes,
                          chi2.data_ptr(), s.data_ptr() if want_s else None,
                          self.sampler.stream.cuda_stream)
        self.generation += 1
        return chi2, s

    def logdet_trace(self, pk, n_probes: int, probe0: int = 0):
        """Hutchinson estimate of T_b = tr(A^-1 R (dS/dP_b) R), A = R S R + N
        on the observed voxels, the log-determinant term of the likelihood's
        P-gradient: d ln L/d P_b = -1/2 d chi2/d P_b - 1/2 T_b.  Mean over
        probes probe0 .. probe0 + n_probes - 1, each filtered by n_iter
        messenger iterations; per unit of physical P_b."""
        import torch
        n, nb = self.sampler.n, self.sampler.n_bins
        if (pk.dtype != torch.float64 or not pk.is_cuda or tuple(pk.shape) != self._lead() + (nb,)
                or not pk.is_contiguous()):
            raise ValueError(f"pk must be a contiguous float64 cuda tensor of shape {self._lead() + (nb,)}")
        out = ctypes.c_size_t(0)
        _check(load().mf_wiener_logdet_workspace_bytes(ctypes.c_void_p(self.sampler.handle),
                                                       self.chain, ctypes.byref(out)))
        if getattr(self, "_ld_bytes", 0) < out.value:
            self._ld_ws = torch.empty(out.value + 256, dtype=torch.uint8, device=pk.device)
            self._ld_bytes = out.value
        ptr = (self._ld_ws.data_ptr() + 255) // 256 * 256
        trace = torch.empty(self._lead() + (nb,), dtype=torch.float64, device=pk.device)
        _check(load().mf_wiener_logdet_trace(
            ctypes.c_void_p(self.sampler.handle), self.chain, ctypes.c_void_p(pk.data_ptr()),
            self.n_iter, n_probes, probe0, ctypes.c_void_p(ptr), self._ld_bytes,
            ctypes.c_void_p(trace.data_ptr()), ctypes.c_void_p(self.sampler.stream.cuda_stream)))
        return trace

    def backward(self, d):
        """(d chi2/d d, d chi2/d pk) of the last forward run (same d)."""
        import torch
        grad_d = torch.empty_like(d)
        grad_pk = torch.empty(self._lead() + (self.sampler.n_bins,), dtype=torch.float64,
                              device=d.device)
        mf_wiener_backward(self.sampler.handle, self.chain, d.data_ptr(), self._ptr,
                           self.ws_bytes, grad_d.data_ptr(), grad_pk.data_ptr(),
                           self.sampler.stream.cuda_stream)
        return grad_d, grad_pk


STREAM_MODES = ("copy", "copy_nt", "read", "read_nt")


def stream_reference(src, dst, mode: str, blocks: int, stream=None):
    """One launch of the streaming reference kernel over src (a cuda tensor)
    into dst (same size for the copies; >= 4 * blocks bytes for the reads)."""
    _check(load().mf_stream_reference(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                      src.numel() * src.element_size(), STREAM_MODES.index(mode),
                                      blocks, ctypes.c_void_p(_stream_ptr(stream))))


def acf(trace, max_lag: int, stream=None):
    """Autocorrelation C_n (n <= max_lag) and correlation length of every
    column of a (T, n_bins) float64 cuda tensor (Eq. CORR_COEFF, ten-percent
    rule); returns (acf (max_lag + 1, n_bins), nc (n_bins,) int32)."""
    import torch
    trace = trace.contiguous()
    t, nb = trace.shape
    out = torch.empty((max_lag + 1, nb), dtype=torch.float64, device=trace.device)
    nc = torch.empty(nb, dtype=torch.int32, device=trace.device)
    _check(load().mf_acf(ctypes.c_void_p(trace.data_ptr()), t, nb, max_lag,
                         ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(nc.data_ptr()),
                         ctypes.c_void_p(_stream_ptr(stream))))
    return out, nc
