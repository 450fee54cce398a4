"""The C-ABI library loads and exports every symbol include/fde.h declares (no GPU)."""
import os
import re
import subprocess

import numpy as np
import pytest
from scipy.special import roots_jacobi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1808_02937_amd", "libfde.so")


def header_symbols():
    src = open(os.path.join(ROOT, "include", "fde.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fde_[a-z0-9_]+)\s*\(", src)) - {"fde_fn"})


def test_library_exists():
    assert os.path.exists(LIB), "run __graft_entry__.build() first"


def test_every_declared_symbol_is_exported():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (fde_[a-z0-9_]+)", out))
    missing = [s for s in header_symbols() if s not in exported]
    assert not missing, missing


def test_binding_declares_every_symbol():
    from paper_1808_02937_amd import _abi
    assert sorted(_abi.SIGNATURES) == header_symbols()
    _abi.load()


def test_library_is_built_for_gfx950():
    data = open(LIB, "rb").read()
    assert b"gfx950" in data
    for other in (b"gfx942", b"gfx90a", b"gfx1100"):
        assert other not in data


@pytest.mark.parametrize("n,a,b", [(1, 0.0, 0.0), (5, 0.0, 0.0), (17, 0.0, 0.0), (64, 0.0, 0.0),
                                   (9, 0.0, 0.5), (9, 0.0, -0.5), (12, 0.0, -0.9), (8, 0.0, 0.1),
                                   (33, 0.0, 0.95), (7, 0.3, 0.8)])
def test_own_gauss_jacobi_matches_scipy(n, a, b):
    import paper_1808_02937_amd as fde
    x, w = fde.gauss_jacobi(n, a, b)
    xr, wr = roots_jacobi(n, a, b)
    assert np.abs(x - xr).max() < 1e-14
    assert np.abs((w - wr) / wr).max() < 3e-12   # scipy itself is only ~1e-14 accurate at n=64
    if a == 0.0:
        # exact moments int (1+x)^b x^k from the binomial sum (160 digits: it cancels)
        import math
        import mpmath
        with mpmath.workdps(160):
            for k in range(0, 2 * n, max(1, n // 3)):
                bm = mpmath.mpf(b)
                ex = sum(math.comb(k, j) * (-1) ** (k - j) * mpmath.power(2, bm + j + 1) / (bm + j + 1)
                         for j in range(k + 1))
                assert abs(np.sum(w * x ** k) - float(ex)) <= 1e-13 * max(1.0, abs(float(ex)))


def test_quadrature_rejects_bad_arguments():
    import paper_1808_02937_amd as fde
    from paper_1808_02937_amd._abi import FDEError
    with pytest.raises(FDEError):
        fde.gauss_jacobi(4, -1.0, 0.0)
    with pytest.raises(FDEError):
        fde.gauss_jacobi(0, 0.0, 0.0)
