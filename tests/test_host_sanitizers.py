"""The library's host code (plan construction, bins, triplets, tile maps,
workspace layout, batching, argument checks) under AddressSanitizer and
UndefinedBehaviorSanitizer: a sanitizer build of the host C++ sources runs
the host-side ABI tests in a child process with the sanitizer runtimes
preloaded; any sanitizer report fails the test.  CPU only (no GPU calls)."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    r = subprocess.run(["g++", f"-print-file-name={name}"], stdout=subprocess.PIPE, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_abi_under_address_and_ub_sanitizers():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("g++ sanitizer runtimes not available")
    sys.path.insert(0, ROOT)
    from paper_2404_07249_amd import build_asan

    lib = build_asan.build()
    env = dict(os.environ, LD_PRELOAD=f"{asan} {ubsan}", PB3_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=900)
    out = r.stdout
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
