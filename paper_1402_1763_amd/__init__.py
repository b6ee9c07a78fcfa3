"""MI355X-native messenger-field Gibbs sampler (Jasche & Lavaux 2014).

The sampler itself is the HIP library libmfgibbs.so (C ABI in include/mf.h);
``binding`` is its ctypes binding and ``workloads`` builds seeded synthetic
inputs.
"""
from . import binding, workloads  # noqa: F401
from .binding import Sampler  # noqa: F401
