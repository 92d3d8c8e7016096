"""The C-ABI argument checks under AddressSanitizer and UndefinedBehaviorSanitizer
on the host code: tests/test_abi.py run against librve_asan.so (built by
`python -m paper_1903_12227_amd.build --sanitize`, which instruments the host
code only) in a child process with the ASan runtime preloaded. Skipped when
that build is absent or older than the sources (it takes minutes to build),
or when the runtime cannot be found.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1903_12227_amd")
LIB = os.path.join(PKG, "librve_asan.so")


def _asan_runtime():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    clang = os.path.join(rocm, "llvm", "bin", "clang++")
    if os.path.exists(clang):
        out = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
        path = out.stdout.strip()
        if out.returncode == 0 and os.path.isabs(path) and os.path.exists(path):
            return path
    return None


def test_abi_checks_pass_under_host_sanitizers():
    if not os.path.exists(LIB):
        pytest.skip("librve_asan.so not built")
    sources = glob.glob(os.path.join(PKG, "csrc", "*"))
    if any(os.path.getmtime(s) > os.path.getmtime(LIB) for s in sources):
        pytest.skip("librve_asan.so is older than the sources")
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("ASan runtime not found")
    env = dict(os.environ, RVE_LIBRARY=LIB, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_abi.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, (res.stdout[-3000:], res.stderr[-3000:])
    assert "AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, res.stderr[-3000:]
