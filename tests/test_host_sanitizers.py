"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
on the CPU: the library is rebuilt with host-only sanitizer flags
(paper_1402_1763_amd/build.py, build_host_sanitized) and tests/test_abi.py
runs against it in a child process with the sanitizer runtime preloaded.  Any
report (heap or stack overflow, use after free, undefined behaviour) aborts
the child and fails this test."""
import os
import subprocess
import sys

import pytest

from paper_1402_1763_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_abi_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    lib = build.build_host_sanitized(str(tmp_path / "libmfgibbs_hostsan.so"))
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": build.host_sanitizer_runtime(),
        "MFGIBBS_LIB": lib,
        # Python itself is not instrumented and keeps memory until exit
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "HIP_VISIBLE_DEVICES": "",   # host paths only, also on a machine with a GPU
    })
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_abi.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    print(out[-3000:])
    assert res.returncode == 0, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out
