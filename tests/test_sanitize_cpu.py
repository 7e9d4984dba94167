"""The library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer: CSR validation, the layout builder (reverse
Cuthill-McKee, window sorts, row groups, slot assignment, the CSR -> slot
map), the assembly planners and the entry points' argument checks.  The
library is rebuilt with sanitized host code (device code unchanged) and the
host-only test modules run against it in a child process that preloads the
sanitizer runtime; any report ends that process with a non-zero status."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_TESTS = ["tests/test_abi_cpu.py", "tests/test_asm_host.py"]


def test_host_code_under_asan_and_ubsan():
    from paper_1501_00324_amd import _build
    rt = _build.sanitizer_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime in this toolchain")
    if _build.needs_build_sanitized():
        _build.build_sanitized()
    env = dict(os.environ)
    env["FESPMV_LIB"] = _build.LIB_SAN
    pre = env.get("LD_PRELOAD", "")
    env["LD_PRELOAD"] = rt + (":" + pre if pre else "")
    # Python itself is not instrumented and keeps memory to exit: no leak
    # report; every other finding stops the child with a marked status
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:exitcode=86"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=87"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q",
                        "-m", "not gpu", "-p", "no:cacheprovider",
                        *HOST_TESTS], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=1500)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in r.stderr, out
    assert "runtime error" not in r.stderr, out
    assert " passed" in r.stdout, out
