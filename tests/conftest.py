import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


def pytest_sessionfinish(session, exitstatus):
    session.config._fde_exitstatus = int(exitstatus)


@pytest.hookimpl(trylast=True)
def pytest_unconfigure(config):
    """After the report is printed, end the process with pytest's status when the GPU was used:
    native HIP/torch teardown at interpreter exit can crash after every test has finished,
    which would replace the real status with a signal."""
    if "torch" in sys.modules and "paper_1808_02937_amd" in sys.modules:
        try:
            import torch
            if torch.cuda.is_available() and torch.cuda.is_initialized():
                torch.cuda.synchronize()
                sys.stdout.flush()
                sys.stderr.flush()
                os._exit(getattr(config, "_fde_exitstatus", 0))
        except Exception:
            pass
