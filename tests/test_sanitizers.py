"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

  - the oracle: every entry point once on small media (tests/sanitize/oracle_driver.c),
    built here with gcc -fsanitize=address,undefined (no recovery: the first error aborts);
  - the C ABI: the driver tests/sanitize/abi_driver.cpp linked with the library's sources
    whose host code carries the same sanitizers (built by the package build next to the
    library).  Without a GPU it runs the calls that need none and checks that creating a
    handle fails cleanly; the GPU test runs every kind of entry point on a small medium.
"""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_SOURCES = ["velocity.c", "fmm.c", "dijkstra.c", "rays.c", "adjoint.c", "nested.c"]
DRIVER = os.path.join(ROOT, "tests", "sanitize", "abi_driver_asan")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_driver")
        cmd = ["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-O1", "-g", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off", "-o", exe,
               os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c")] + \
              [os.path.join(ROOT, "oracle", s) for s in ORACLE_SOURCES] + ["-lm"]
        subprocess.check_call(cmd)
        r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "every entry point ran clean" in r.stdout


def _run_driver():
    if not os.path.exists(DRIVER):
        pytest.skip("the sanitized C-ABI driver is built by paper_2302_10988_amd/build.py")
    r = subprocess.run([DRIVER], capture_output=True, text=True, env=ENV, timeout=600)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    return r.stdout


def test_c_abi_host_code_under_sanitizers_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("covered by the GPU test")
    assert "host-only entry points ran clean" in _run_driver()


@pytest.mark.gpu
def test_c_abi_host_code_under_sanitizers_on_gpu():
    print("sanitized C-ABI driver on the GPU", flush=True)
    assert "every entry point ran clean" in _run_driver()
