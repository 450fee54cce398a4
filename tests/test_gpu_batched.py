"""GPU: a batch of uneven instances (mesh class, N, P, alpha, theta all drawn per instance)
factored in one level-scheduled H-LU and solved in one lock-step FGMRES."""
import numpy as np
import pytest
import torch

import fde_inputs as fi
from tests.gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    fde = need_gpu()
    return fde.Context(0)


def test_uneven_batch_matches_alone(ctx):
    import paper_1808_02937_amd as fde
    insts = fi.config_batched(count=12, N_range=(64, 200), P_range=(2, 8))
    say("uneven batch: " + ", ".join(f"{i.mesh_kind}/N{len(i.nodes) - 1}/P{i.P}" for i in insts))
    ops = [fde.Operator(ctx, i.nodes, i.P, i.alpha, i.theta, i.rho) for i in insts]
    Gs = [op.load_vector(i.rhs[0]) for op, i in zip(ops, insts)]
    hms = [fde.HMatrix(op, R=i.R, leaf_elems=i.leaf) for op, i in zip(ops, insts)]
    lus = fde.factor_batched(hms, tol=1e-3, precision="fp32")
    Xs, infos = fde.solve_batched(ctx, ops, Gs, lus, rtol=1e-10)
    for op, G, X, inf, lu, hm in zip(ops, Gs, Xs, infos, lus, hms):
        assert inf[0]["status"] == 0 and inf[0]["relres"] <= 1e-10
        r = torch.linalg.norm(G - op.apply(X)) / torch.linalg.norm(G)
        assert float(r) <= 1.5e-10
        # alone: its own factorisation (the batch's factors are bit-identical) and its own solve
        alone = fde.HLU(hm, tol=1e-3, precision="fp32")
        assert torch.equal(alone.dense()[0], lu.dense()[0])
        Xa, _ = fde.solve(op, G, alone, rtol=1e-10)
        assert float(torch.linalg.norm(Xa - X) / torch.linalg.norm(Xa)) <= 1e-7
