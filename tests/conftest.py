import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle test taking more than a few seconds")


def pytest_sessionfinish(session, exitstatus):
    """Write the measured GPU-vs-oracle errors (tests/gpu_common.py) to $PARITY_REPORT, if set."""
    path = os.environ.get("PARITY_REPORT")
    if not path:
        return
    try:
        from gpu_common import ERRORS
    except ImportError:
        return
    import json
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        for e in ERRORS:
            f.write(json.dumps(e) + "\n")
