"""tests/test_abi.py against the host-sanitized build of the library
(libkpm_asan.so: AddressSanitizer + UndefinedBehaviorSanitizer on the C ABI,
planner and launch layer), in a child process with the sanitizer runtime
preloaded.  Any invalid host memory access or undefined behaviour in the
argument checks, workspace queries, planner or relabelling search aborts the
child.  The sanitized library is built here when missing or older than any
of the library's sources (about 40 s)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_suite_under_address_and_ub_sanitizers():
    from paper_2104_13218_amd import build
    srcs = [os.path.join(build.CSRC, f) for f in os.listdir(build.CSRC)]
    srcs.append(os.path.join(ROOT, "include", "kpm.h"))
    stale = not os.path.exists(build.LIB_ASAN) or max(os.path.getmtime(f) for f in srcs) > os.path.getmtime(
        build.LIB_ASAN)
    if stale:
        try:
            build.build(sanitize=True)
        except RuntimeError as e:
            pytest.skip(f"sanitized build unavailable: {e}")
    env = dict(os.environ)
    env["KPM_LIBRARY"] = build.LIB_ASAN
    env["LD_PRELOAD"] = build.sanitizer_runtime()
    # leaks of the interpreter and the HIP runtime are not this library's
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "passed" in out and "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
