"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

libp3m is rebuilt with ASan + UBSan on the host side only
(build.build_host_sanitized: -Xarch_host -fsanitize=...; the device code is
compiled as usual and never runs here), and the host tests of the ABI
(argument validation, plan geometry and error paths, stencil and segment
rows, split tables, the cosmology helpers, the allocation-free entry point's
checks) run against it in a child process with the ASan runtime preloaded.
Any ASan or UBSan report fails the test; leak reports fail it when a leaked
block was allocated from libp3m (the interpreter's and torch's own leaks at
exit are not this library's).
"""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_TESTS = ["tests/test_abi_host.py", "tests/test_cosmology.py"]


@pytest.fixture(scope="module")
def sanitized():
    if not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")):
        pytest.skip("hipcc not available")
    from paper_1510_07621_amd import build
    return build.build_host_sanitized(), build.asan_runtime()


def _leaks_from_libp3m(text):
    """Leak reports (one block per 'leak of' header) whose stack names libp3m."""
    blocks = re.split(r"\n(?=(?:Direct|Indirect) leak of)", text)
    return [b for b in blocks if re.match(r"(?:Direct|Indirect) leak of", b)
            and ("libp3m" in b or "p3m::" in b or " p3m_" in b)]


def test_host_abi_under_asan_and_ubsan(sanitized):
    lib, runtime = sanitized
    env = dict(os.environ)
    env.update(P3M_LIBRARY=lib, LD_PRELOAD=runtime,
               ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:detect_odr_violation=0",
               LSAN_OPTIONS="exitcode=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *HOST_TESTS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out, out[-6000:]
    assert "runtime error:" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert re.search(r"\d+ passed", out), out[-3000:]
    leaks = _leaks_from_libp3m(out)
    assert not leaks, "\n".join(leaks)[:6000]


def test_the_sanitized_library_is_instrumented(sanitized):
    """The build carries the ASan and UBSan hooks (so the run above is not a
    plain build by mistake)."""
    lib, _ = sanitized
    with open(lib, "rb") as f:
        data = f.read()
    assert b"__asan_report_load" in data
    assert b"__ubsan_handle" in data
