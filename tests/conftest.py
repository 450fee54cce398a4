import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@pytest.hookimpl(trylast=True)
def pytest_sessionfinish(session, exitstatus):
    """End the process with pytest's status once results are reported when the GPU was used:
    native HIP/torch teardown at interpreter exit can crash after every test has finished,
    which would replace the real status with a signal."""
    import sys
    if "torch" in sys.modules and "paper_1808_02937_amd" in sys.modules:
        try:
            import torch
            if torch.cuda.is_available() and torch.cuda.is_initialized():
                torch.cuda.synchronize()
                sys.stdout.flush()
                sys.stderr.flush()
                import os
                os._exit(int(exitstatus))
        except Exception:
            pass
