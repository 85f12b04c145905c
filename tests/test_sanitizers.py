"""Sanitizer runs on the CPU.

The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (g++)
runs its own pins, and the library built with both sanitizers on its host
code (hipcc; the device code objects are not sanitized) runs the host-side
library tests: argument validation, the phase and CCZ decompositions, the
gate-list numbering.  Each run is a child process with the matching ASan
runtime preloaded and every report fatal, so a finding fails the test with
the report in its message.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow


def _run_child(extra_env, test_files):
    env = dict(os.environ)
    env.update(extra_env)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    cmd = [sys.executable, "-m", "pytest", *test_files, "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, (r.stdout[-4000:] + "\n" + r.stderr[-4000:])
    assert " passed" in r.stdout


def test_oracle_under_asan_and_ubsan():
    from oracle import build_oracle

    lib = build_oracle.build_sanitized()
    _run_child({"CHSIM_ORACLE_LIB": lib, "LD_PRELOAD": build_oracle.asan_runtime()},
               ["tests/test_oracle_pins.py", "tests/test_oracle_mlp.py"])


def test_library_host_code_under_asan_and_ubsan():
    from paper_1808_00128_amd import build

    try:
        lib = build.build_host_sanitized()
        rt = build.asan_runtime()
    except (OSError, RuntimeError) as exc:  # no hipcc or no clang runtime on this machine
        pytest.skip(f"sanitizer build unavailable: {exc}")
    _run_child({"CHSIM_LIB": lib, "LD_PRELOAD": rt}, ["tests/test_library_cpu.py"])
