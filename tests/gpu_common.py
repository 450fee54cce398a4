"""Shared helpers for the GPU parity tests (no oracle arithmetic here)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1808_02937_amd as fde  # raises if the HIP library is missing
    return fde


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()
