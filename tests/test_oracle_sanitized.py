"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code): every C entry point runs on a small scene in a child
process with the sanitizer runtimes preloaded, and must finish without a
report.  Skipped when gcc has no sanitizer runtime."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    try:
        p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    except OSError:
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.timeout(600)
def test_oracle_under_asan_ubsan():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    env = dict(os.environ, LS2_ORACLE_SANITIZE="1", LD_PRELOAD=asan + ":" + ubsan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    # the sanitized library is built by the child (oracle.build on first use)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitized_workload.py")], env=env,
                       capture_output=True, text=True, timeout=580)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "sanitized workload ok" in r.stdout


@pytest.mark.timeout(900)
def test_library_validation_under_asan_ubsan():
    """The library's host code (argument and camera validation, workspace
    sizing, status strings) built with ASan + UBSan (device code unchanged):
    the C-ABI checks of test_abi_cpu.py run against it in a child process."""
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    import importlib.util
    spec = importlib.util.spec_from_file_location("_ls2_build_san", os.path.join(ROOT, "paper_2507_07136_amd",
                                                                                 "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    b.build(sanitize=True)
    env = dict(os.environ, LS2_LIB_SANITIZED="1", LD_PRELOAD=asan + ":" + ubsan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi_cpu.py"), "-q",
                        "-p", "no:cacheprovider"], env=env, capture_output=True, text=True, timeout=880, cwd=ROOT)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
