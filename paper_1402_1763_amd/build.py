"""Build the HIP library libmfgibbs.so in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmfgibbs.so")
SOURCES = [os.path.join(HERE, "csrc", "mf_api.hip")]
HEADERS = [os.path.join(HERE, "csrc", f) for f in ("fft.hpp", "philox.hpp", "sweep_kernels.hpp")]

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed-FP32 VALU forms are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def build(verbose: bool = False, extra_flags=None) -> str:
    """Compile the library (always recompiles) and return its path."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIP_FLAGS, *(extra_flags or []), "-I", os.path.join(ROOT, "include"),
           *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libmfgibbs.so")
    os.replace(tmp, LIB)
    return LIB


# Host half under AddressSanitizer and UndefinedBehaviorSanitizer, for the
# CPU tests of the C ABI's host code (argument and descriptor validation,
# set-up tables, error clean-up).  Every sanitizer flag is host-only; the
# device code is compiled unoptimised (the sanitized library never launches
# it) to keep the compilation short.  Load it with the sanitizer runtime preloaded
# (host_sanitizer_runtime()) and MFGIBBS_LIB pointing at it.
SANITIZE_FLAGS = [
    "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared", "-shared-libsan",
    "-Xarch_host", "-O1", "-Xarch_host", "-g",
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-omit-frame-pointer",
    "-Xarch_device", "-O0",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build_host_sanitized(out: str, verbose: bool = False) -> str:
    """Compile the library with sanitized host code to `out`."""
    cmd = [hipcc(), *SANITIZE_FLAGS, "-I", os.path.join(ROOT, "include"), *SOURCES, "-o", out]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building the sanitized host library")
    return out


def host_sanitizer_runtime() -> str:
    """The compiler's shared AddressSanitizer runtime (with UBSan's handlers)."""
    import glob
    hits = sorted(glob.glob(os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(hipcc()))),
                                         "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise RuntimeError("libclang_rt.asan-x86_64.so not found beside hipcc")
    return hits[-1]


if __name__ == "__main__":
    print(build(verbose=True))
