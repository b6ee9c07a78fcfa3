"""MI355X-native messenger-field Gibbs sampler (Jasche & Lavaux 2014).

The sampler itself is the HIP library libmfgibbs.so (C ABI in include/mf.h).
``binding`` is its ctypes binding: ``Sampler`` (Gibbs and mixing sweeps,
state, checkpoints, diagnostics, the x-transform autotuner),
``SweepGraph`` (several problems per HIP graph replay), ``WienerFilter``
(messenger Wiener filter and its adjoint) and ``acf``.  ``autograd`` wraps
the Wiener filter's chi2 as a torch function, and ``workloads`` builds
seeded synthetic inputs.
"""
from . import binding, workloads  # noqa: F401
from .binding import Sampler, SweepGraph, WienerFilter, acf  # noqa: F401
