"""The host orchestration under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/hostsim builds the library's host code (api.hip, serinv.hip: argument
checks, chunking, workspace carving, plans, the point queue, the partitioned
solver's layout) with the sanitizers on the host side, links it with the CPU
double of the kernels, and the host-simulation tests run against it in a child
process that preloads the sanitizer runtime.  Any out-of-bounds access, use
after free or undefined behaviour in that code ends the child with a report."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.slow
def test_host_orchestration_under_asan_and_ubsan():
    sys.path.insert(0, os.path.join(HERE, "hostsim"))
    import build as hb
    hb.build(sanitize=True)
    env = dict(os.environ)
    env["NEGF_HOSTSIM_SANITIZED"] = "1"
    env["LD_PRELOAD"] = hb.asan_runtime()
    # leaks of the Python interpreter itself are not ours; the library's calls are checked for
    # invalid accesses and undefined behaviour
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_hostsim.py"), os.path.join(HERE, "test_hostsim_serinv.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout, tail
