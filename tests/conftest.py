import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU oracle test")
    config.addinivalue_line("markers", "oracle_refs(*names): oracle references (tests/oracle_jobs.py) "
                                       "the test needs; computed in background threads from the "
                                       "start of the session")


@pytest.hookimpl(trylast=True)
def pytest_collection_modifyitems(session, config, items):
    names = []
    for item in items:
        for m in item.iter_markers("oracle_refs"):
            names.extend(n for n in m.args if n not in names)
    if not names:
        return
    try:
        import torch
        if torch.cuda.device_count() == 0:   # counts devices without initialising them
            return
    except Exception:
        return
    import oracle_jobs
    oracle_jobs.start(names)
