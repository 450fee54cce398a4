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


def _collect(srv, tickets):
    out = {}
    for t in tickets:
        done, inf, cached = srv.poll(t)
        assert done, t
        out[t] = (inf, cached)
    return out


def test_continuous_serving_same_result_alone_and_in_the_mix(ctx):
    """Requests join a server while others are in flight (iteration-level continuous batching); a
    request's solution is bit for bit the one it gets alone."""
    import paper_1808_02937_amd as fde
    say("continuous serving: alone vs in a mix")
    pa = PROBS[2]
    GA = rhs(pa, 3, 77)
    alone = fde.Server(ctx, R=6, leaf_elems=4, rtol=1e-12)
    tA, XA = alone.submit(pa, GA)
    alone.drain()
    infA = _collect(alone, [tA])[tA][0]
    alone.close()
    mix = fde.Server(ctx, R=6, leaf_elems=4, rtol=1e-12)
    GB, GC, GD = rhs(PROBS[0], 5, 78), rhs(PROBS[1], 2, 79), rhs(PROBS[3], 4, 80)
    res = {}

    def finished(tickets):   # polls (a done ticket is collected once) and says which are done
        for t in tickets:
            if t not in res:
                done, inf, cached = mix.poll(t)
                if done:
                    res[t] = (inf, cached)
        return [t in res for t in tickets]

    tB, XB = mix.submit(PROBS[0], GB)
    tC, XC = mix.submit(PROBS[1], GC)
    mix.step()
    tA2, XA2 = mix.submit(pa, GA)
    mix.step()   # A is admitted while B (and perhaps C) are on the device
    assert not all(finished([tB, tC])), "A should join while another request is in flight"
    tD, XD = mix.submit(PROBS[3], GD)
    mix.step()
    assert not finished([tA2])[0], "D should join while A is in flight"
    mix.drain()
    finished([tA2, tB, tC, tD])
    say(f"  alone iters {[i[0] for i in infA]}, in the mix {[i[0] for i in res[tA2][0]]}")
    assert torch.equal(XA, XA2)
    assert [i[0] for i in infA] == [i[0] for i in res[tA2][0]]
    for t, p, G, X in ((tB, PROBS[0], GB, XB), (tC, PROBS[1], GC, XC), (tD, PROBS[3], GD, XD)):
        assert all(s == 0 for (_, _, s) in res[t][0]), res[t]
        assert true_relres(p, G, X) <= 5e-12
    # the same problem again later: its factors are cached
    tE, XE = mix.submit(PROBS[0], GB)
    mix.drain()
    infE, cachedE = _collect(mix, [tE])[tE]
    assert cachedE and torch.equal(XE, XB)
    mix.close()


def test_continuous_serving_waits_for_memory(ctx):
    """With room for one problem, a second problem waits in the queue until the first request is
    done and its factors can be evicted; factors in use are never evicted."""
    import paper_1808_02937_amd as fde
    say("continuous serving: admission by memory")
    probe = fde.Server(ctx, R=6, leaf_elems=4)
    probe.solve([PROBS[0]], [rhs(PROBS[0], 1, 1)])
    one = probe.stats()["bytes"]
    probe.close()
    p0, p1 = PROBS[0], (fi.uniform_mesh(30), 4, 1.5, 0.5, 1.0)
    srv = fde.Server(ctx, R=6, leaf_elems=4, rtol=1e-12, budget_bytes=int(1.6 * one))
    G0, G1 = rhs(p0, 2, 5), rhs(p1, 2, 6)
    t0, X0 = srv.submit(p0, G0)
    t1, X1 = srv.submit(p1, G1)
    assert srv.step() == 2
    assert srv.stats()["entries"] == 1          # p1 waits: p0's factors are in use
    srv.drain()
    res = _collect(srv, [t0, t1])
    st = srv.stats()
    assert st["evictions"] == 1 and st["entries"] == 1 and st["bytes"] <= 1.6 * one
    for p, G, X, t in ((p0, G0, X0, t0), (p1, G1, X1, t1)):
        assert all(s == 0 for (_, _, s) in res[t][0])
        assert true_relres(p, G, X) <= 5e-12
    srv.close()


def test_continuous_serving_large_operator_bf16(ctx):
    """A request whose right-hand sides are too long for LDS (uniform N = 4096, P = 8: the H-solve
    keeps them in global memory) served with BF16 low-rank factors, alone and beside a small one in
    the same launches (which then take the global-memory variant too): the same bits either way,
    and the true residual of the large request at the requested 1e-10."""
    import paper_1808_02937_amd as fde
    say("continuous serving: N = 4096 with BF16 U, V, alone and in a mix")
    big = (fi.uniform_mesh(4096), 8, 1.35, 0.45, 1.0)
    small = PROBS[0]
    GL, GS = rhs(big, 2, 91), rhs(small, 3, 92)
    out = {}
    for name, reqs in (("big", [(big, GL)]), ("small", [(small, GS)]), ("mix", [(big, GL), (small, GS)])):
        srv = fde.Server(ctx, R=8, leaf_elems=8, tol=1e-3, precision="bf16uv", rtol=1e-10)
        subs = [srv.submit(p, G) for p, G in reqs]
        srv.drain()
        res = _collect(srv, [t for t, _ in subs])
        for (t, _), (p, _) in zip(subs, reqs):
            assert all(s == 0 and r <= 1e-10 for (_, r, s) in res[t][0]), res[t]
        out[name] = [X for _, X in subs]
        srv.close()
    assert torch.equal(out["mix"][0], out["big"][0])
    assert torch.equal(out["mix"][1], out["small"][0])
    op = fde.Operator(ctx, *big)
    R = GL - op.apply(out["big"][0])
    true = float((torch.linalg.norm(R, dim=1) / torch.linalg.norm(GL, dim=1)).max())
    say(f"  large request: recomputed true residual {true:.1e}")
    assert true <= 2e-10
    op.close()
