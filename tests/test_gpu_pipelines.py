"""GPU: several contexts driven side by side, each on its own stream and host thread (how the
benchmark keeps batches in flight, and how its serving stream runs several servers). Every context's
results equal those of the same work run alone, bit for bit: contexts share no device state, and the
library's process-wide tables are locked."""
import threading

import numpy as np
import pytest
import torch

import fde_inputs as fi
from tests.gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu

PROBS = [
    (fi.uniform_mesh(96), 6, 1.5, 0.5, 1.0),
    (fi.two_sided_graded_mesh(64, 8, 0.5), 5, 1.7, 0.4, 0.0),
    (fi.geometric_mesh(48, 1.05), 4, 1.3, 0.8, 0.5),
]


def batch(fde, ctx, seed):
    """Operators, H-matrices, one batched FP32 H-LU and one batched FGMRES over the three problems."""
    ops = [fde.Operator(ctx, *p) for p in PROBS]
    rng = np.random.default_rng(seed)
    Gs = [torch.tensor(rng.standard_normal((2, o.Nd)), device="cuda") for o in ops]
    hms = [fde.HMatrix(o, R=6, lam=1.0, leaf_elems=4) for o in ops]
    lus = fde.factor_batched(hms, tol=1e-3, precision="fp32")
    Xs, infos = fde.solve_batched(ctx, ops, Gs, lus, rtol=1e-12)
    ctx.synchronize()
    out = [X.clone() for X in Xs]
    for o in lus + hms + ops:
        o.close()
    return out, infos


def test_contexts_side_by_side_equal_alone():
    fde = need_gpu()
    say("three contexts on three streams and threads vs alone")
    n = 3
    ctxs = [fde.Context(0, stream=torch.cuda.Stream(), apply_streams=0) for _ in range(n)]
    alone = []
    for i, c in enumerate(ctxs):
        with torch.cuda.stream(c._stream):
            alone.append(batch(fde, c, 100 + i)[0])
    res, errors = [None] * n, []

    def work(i):
        try:
            with torch.cuda.stream(ctxs[i]._stream):
                for _ in range(3):   # several rounds, so the threads overlap
                    res[i] = batch(fde, ctxs[i], 100 + i)
        except BaseException as e:
            errors.append(e)
    th = [threading.Thread(target=work, args=(i,)) for i in range(n)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors[0]
    for i in range(n):
        Xs, infos = res[i]
        assert all(x["status"] == 0 and x["relres"] <= 1e-12 for inf in infos for x in inf)
        for a, b in zip(alone[i], Xs):
            assert torch.equal(a, b)
    # and the same work with the applies forked onto side streams gives the same bits
    c3 = fde.Context(0, stream=torch.cuda.Stream())
    with torch.cuda.stream(c3._stream):
        side = batch(fde, c3, 100)[0]
    for a, b in zip(alone[0], side):
        assert torch.equal(a, b)
    for c in ctxs + [c3]:
        c.close()
