"""The allocation-free stiffness apply (fde_stiffness_apply_noalloc) against fde_stiffness_apply:
same kernels, so the same bits; two calls in a row, the second on a smaller input; no device
memory taken from the context; inputs too large for the fixed workspace rejected."""
import numpy as np
import pytest
import torch

import fde_inputs as fi
from tests.gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu

CASES = [
    # nodes, P, alpha, theta, rho, nrhs: the block-Toeplitz apply, then a smaller dense one
    (fi.uniform_mesh(1024), 8, 1.5, 0.5, 1.0, 4),
    (fi.two_sided_graded_mesh(64, 10, 0.5), 6, 1.7, 0.4, 0.0, 1),
]


def test_noalloc_apply_equals_apply():
    fde = need_gpu()
    from paper_1808_02937_amd._abi import FDE_EINVAL, FDEError
    ctx = fde.Context(0)
    gen = torch.Generator(device="cuda").manual_seed(5)
    ops = []
    for nodes, P, al, th, rho, nrhs in CASES:
        op = fde.Operator(ctx, nodes, P, al, th, rho)
        ops.append(op)
        say(f"noalloc apply: N={len(nodes) - 1} P={P} nrhs={nrhs} toeplitz={op.toeplitz}")
        X = torch.randn(nrhs, op.Nd, dtype=torch.float64, device="cuda", generator=gen)
        Y = torch.full_like(X, float("nan"))
        torch.cuda.synchronize()
        before = ctx.bytes_in_use()
        op.apply_noalloc(X, Y)
        torch.cuda.synchronize()
        assert ctx.bytes_in_use() == before
        Yref = op.apply(X)
        torch.cuda.synchronize()
        assert torch.equal(Y, Yref), float((Y - Yref).abs().max())
    # more columns than the fixed workspace holds
    big = ops[0]
    Xb = torch.zeros(200, big.Nd, dtype=torch.float64, device="cuda")
    with pytest.raises(FDEError) as ei:
        big.apply_noalloc(Xb, torch.empty_like(Xb))
    assert ei.value.code == FDE_EINVAL
    for op in ops:
        op.close()
    ctx.close()
