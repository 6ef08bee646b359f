import gc
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: full-size CPU checks")


def pytest_sessionfinish(session, exitstatus):
    # pytest keeps the last failure in sys.last_traceback; its frames hold
    # device tensors and library handles.  Release them now, while torch and
    # the HIP runtime are alive, instead of at interpreter finalisation.
    for name in ("last_type", "last_value", "last_traceback", "last_exc"):
        if hasattr(sys, name):
            setattr(sys, name, None)
    gc.collect()
    if "paper_1610_03154_amd" in sys.modules:
        sys.modules["paper_1610_03154_amd"]._close_all()
    if "torch" in sys.modules:
        torch = sys.modules["torch"]
        if torch.cuda.is_available() and torch.cuda.is_initialized():
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
