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


EPS32 = 2.0 ** -24
EPS64 = 2.0 ** -53


def kappa1(A):
    """1-norm condition number estimate of a dense FP64 matrix: LAPACK getrf, then gecon's
    estimate of ||A^{-1}||_1 (Hager-Higham, exact within a small factor)."""
    import numpy as np
    from scipy.linalg import lapack
    A = np.asarray(A, dtype=np.float64)
    anorm = np.abs(A).sum(axis=0).max()
    lu, piv, info = lapack.dgetrf(A)
    assert info == 0, info
    rcond, info = lapack.dgecon(lu, anorm, norm="1")
    assert info == 0 and rcond > 0.0, (info, rcond)
    return 1.0 / rcond


def lu_residual(F, Ah):
    """||L U - A~||_F / ||A~||_F from packed factors F (L unit lower below the diagonal, U on and
    above it) and A~ in the same order (torch FP64 on F's device)."""
    import torch
    F = torch.as_tensor(F).to(torch.float64)
    Ah_t = torch.as_tensor(Ah, device=F.device).to(torch.float64)
    L = torch.tril(F, -1) + torch.eye(F.shape[0], dtype=F.dtype, device=F.device)
    U = torch.triu(F)
    return float(torch.linalg.norm(L @ U - Ah_t) / torch.linalg.norm(Ah_t))
