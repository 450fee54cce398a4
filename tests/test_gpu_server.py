"""GPU: the solver cache and batched serving (fde_server_*)."""
import numpy as np
import pytest
import torch

import fde_inputs as fi
from oracle.sem import SEM
from tests.gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu

PROBS = [
    (fi.uniform_mesh(32), 4, 1.5, 0.5, 1.0),
    (fi.graded_mesh(24, 2.0, 0.0, 1.0), 3, 1.3, 0.8, 0.0),
    (fi.geometric_mesh(40, 1.05), 5, 1.7, 0.3, 0.5),
    (fi.two_sided_graded_mesh(48, 6, 0.5), 4, 1.9, 0.6, 0.0),
]


@pytest.fixture(scope="module")
def ctx():
    fde = need_gpu()
    return fde.Context(0)


def rhs(prob, nrhs, seed):
    nodes, P = prob[0], prob[1]
    Nd = (len(nodes) - 1) * P - 1
    return torch.tensor(np.random.default_rng(seed).standard_normal((nrhs, Nd)), device="cuda")


def true_relres(prob, G, X):
    nodes, P, al, th, rho = prob
    A = SEM(nodes, P, al, th, rho).system_matrix()
    g, x = G.cpu().numpy(), X.cpu().numpy()
    return max(np.linalg.norm(g[j] - A @ x[j]) / np.linalg.norm(g[j]) for j in range(g.shape[0]))


def test_server_solves_and_caches(ctx):
    import paper_1808_02937_amd as fde
    say("server solves and caches")
    srv = fde.Server(ctx, R=6, leaf_elems=4, rtol=1e-12)
    Gs = [rhs(p, 1 + i % 3, 40 + i) for i, p in enumerate(PROBS)]
    Xs, infos, cached = srv.solve(PROBS, Gs)
    assert cached == [False] * len(PROBS)
    for p, G, X, inf in zip(PROBS, Gs, Xs, infos):
        assert all(s == 0 for (_, _, s) in inf), inf
        assert true_relres(p, G, X) <= 5e-12
    # the same problems again (one of them twice in the batch): all cached, same answers
    probs2 = PROBS + [PROBS[1]]
    Gs2 = Gs + [Gs[1]]
    Xs2, infos2, cached2 = srv.solve(probs2, Gs2)
    assert cached2 == [True] * len(probs2)
    for X, X2 in zip(Xs, Xs2):
        assert torch.allclose(X, X2, rtol=0, atol=1e-10 * float(X.abs().max()))
    st = srv.stats()
    assert st["entries"] == len(PROBS) and st["misses"] == len(PROBS) and st["hits"] == len(probs2)
    assert st["evictions"] == 0 and st["bytes"] > 0


def test_server_budget_evicts_least_recent(ctx):
    import paper_1808_02937_amd as fde
    say("server budget evictions")
    probe = fde.Server(ctx, R=6, leaf_elems=4)
    probe.solve([PROBS[0]], [rhs(PROBS[0], 1, 1)])
    one = probe.stats()["bytes"]
    probe.close()
    srv = fde.Server(ctx, R=6, leaf_elems=4, budget_bytes=int(12 * one))
    keys = [(fi.uniform_mesh(32 + 2 * k), 4, 1.5, 0.5, 1.0) for k in range(12)]
    for k, p in enumerate(keys):
        _, inf, cached = srv.solve([p], [rhs(p, 1, 100 + k)])
        assert inf[0][0][2] == 0 and not cached[0]
    st = srv.stats()
    assert st["evictions"] > 0
    assert st["bytes"] <= 12 * one
    # the most recent problem is still cached, the first one was evicted
    _, _, c_last = srv.solve([keys[-1]], [rhs(keys[-1], 1, 7)])
    _, _, c_first = srv.solve([keys[0]], [rhs(keys[0], 1, 8)])
    assert c_last == [True] and c_first == [False]


def test_server_rejects_what_cannot_fit(ctx):
    import paper_1808_02937_amd as fde
    from paper_1808_02937_amd._abi import FDE_ENOMEM
    say("server rejects an oversized problem")
    small = PROBS[0]
    big = (fi.graded_mesh(512, 2.0, 0.0, 1.0), 8, 1.5, 0.5, 0.0)   # dense path: 67 MB of moments
    srv = fde.Server(ctx, R=6, leaf_elems=4, budget_bytes=40 << 20)
    Gs = [rhs(small, 2, 3), rhs(big, 1, 4)]
    Xs, infos, cached = srv.solve([small, big], Gs)
    assert all(s == 0 for (_, _, s) in infos[0])
    assert infos[1][0][2] == FDE_ENOMEM
    assert true_relres(small, Gs[0], Xs[0]) <= 1e-9
    assert srv.stats()["entries"] == 1
