"""The host orchestration called from several threads at once, under
ThreadSanitizer.

The library states that calls on distinct workspaces and streams may run
concurrently.  tests/hostsim builds its host code (api.hip, serinv.hip) with
ThreadSanitizer on the host side, linked with the CPU double of the kernels; a
child process that preloads the sanitizer runtime runs tests/hostsim/
threads_driver.py: four threads repeat negf_rgf_lesser_greater on their own
problems (ballistic, scattering, energy-dependent self-energies, chunked) while
a fifth creates, executes and destroys plans.  A data race in the library's
host code ends the child with a report; every result must also equal the same
call made alone."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.slow
def test_concurrent_calls_have_no_data_race():
    sys.path.insert(0, os.path.join(HERE, "hostsim"))
    import build as hb
    lib = hb.build(sanitize="thread")
    env = dict(os.environ)
    env["LD_PRELOAD"] = hb.runtime("tsan")
    env["TSAN_OPTIONS"] = "halt_on_error=1:exitcode=66:report_signal_unsafe=0"
    r = subprocess.run([sys.executable, os.path.join(HERE, "hostsim", "threads_driver.py"), lib], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-6000:]
    assert r.returncode == 0, tail
    assert "every result equals the call made alone" in r.stdout, tail
