"""The plan, backward-schedule and persistent-segment table tests, run against a
build of the library whose host code carries AddressSanitizer and
UndefinedBehaviorSanitizer (plan construction, descriptor and chain tables,
the C ABI's argument checks).  Any report aborts the child run."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_plan_tests_clean_under_host_sanitizers():
    from paper_2107_09793_amd import build
    lib = build.build_host_sanitized()
    env = dict(os.environ)
    env.update(LD_PRELOAD=build.sanitizer_runtime(), TNMI_LIB_PATH=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "tests/test_plan.py", "tests/test_persist_tables.py",
                        "tests/test_backward_plan.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in tail, tail
