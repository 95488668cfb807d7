import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_sessionfinish(session, exitstatus):
    """Write the per-point parity records of this run (if any) as JSON lines."""
    import json
    try:
        from helpers import RECORDS
    except Exception:
        return
    if not RECORDS:
        return
    out = os.path.join(ROOT, "gpurun_out", "parity")
    os.makedirs(out, exist_ok=True)
    with open(os.path.join(out, "records.jsonl"), "w") as fh:
        for r in RECORDS:
            fh.write(json.dumps(r) + "\n")
