"""The C-ABI checks again, against the build whose host code carries AddressSanitizer.

The plan's descriptor validation, error reporting and argument checks are host code; the
sanitizer build (libsbp_asan.so, made by the build step) instruments exactly that code.  The
ABI tests run in a child process with the sanitizer runtime preloaded and must pass with no
sanitizer report.  CPU only: every call they make returns before any HIP work."""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2510_10070_amd", "libsbp_asan.so")


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm*/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.mark.skipif(not os.path.exists(LIB), reason="sanitizer build not present (run the build step)")
@pytest.mark.skipif(_asan_runtime() is None, reason="AddressSanitizer runtime not found")
def test_abi_checks_clean_under_address_sanitizer():
    env = dict(os.environ, LD_PRELOAD=_asan_runtime(), SBP_LIBRARY_VARIANT="asan",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
