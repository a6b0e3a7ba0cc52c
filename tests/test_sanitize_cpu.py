"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The library's host code (plan set-up, argument validation, the solver's host
loop) is rebuilt with both sanitizers on the host side only, linked with the
unchanged device objects, and the host checks of test_abi_cpu.py run against
it in a child process with the clang AddressSanitizer runtime preloaded.  The
FFT engine self-test (index arithmetic, slot and mirror maps, sweeps) runs as a
g++ build with both sanitizers.  Any report fails the test: the builds stop at
the first error (-fno-sanitize-recover=all).
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORTS = ("AddressSanitizer", "runtime error:", "LeakSanitizer", "UndefinedBehaviorSanitizer")


@pytest.fixture(scope="module")
def sanitized():
    from paper_2102_11576_amd.build import asan_runtime, build_sanitized
    try:
        rt = asan_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    lib, exe = build_sanitized()
    return lib, exe, rt


def _clean(out):
    return not any(k in out for k in REPORTS)


def test_fft_selftest_under_sanitizers(sanitized):
    _, exe, _ = sanitized
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and r.stdout.strip().endswith("OK") and _clean(out), out[-4000:]


def test_host_validation_under_sanitizers(sanitized):
    lib, _, rt = sanitized
    env = dict(os.environ)
    pre = env.get("LD_PRELOAD", "")
    env["LD_PRELOAD"] = rt + (":" + pre if pre else "")  # the runtime must come first
    env["RSFDE_LIBRARY"] = lib
    # leaks: the Python interpreter and torch keep allocations until exit;
    # alloc/dealloc pairs in uninstrumented libraries are not ours to check
    env["ASAN_OPTIONS"] = "detect_leaks=0:alloc_dealloc_mismatch=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_abi_cpu.py"), "-k", "not selftest"]
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and _clean(out), out[-6000:]
    assert " passed" in r.stdout and "skipped" not in r.stdout, r.stdout[-2000:]
