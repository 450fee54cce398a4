"""Section 5, Example 1 on the GPU: the paper's left-preconditioned BiCGSTAB (eq. (precondsys)) on
the device, with the FP64 H-LU of A~ (tol 1e-3, lambda = 1, leaf 2 elements) as preconditioner,
graded mesh x_i = 10 (i/N)^5, theta = 1, rho = 0, alpha = 1.6, tolerance 1e-13.

Iteration counts are compared with the oracle's BiCGSTAB on the same problem and with Tables 1
and 2 (tests/golden, read as two per BiCGSTAB step); the solution with the dense LU solution."""
import os

import numpy as np
import pytest
import torch

import fde_inputs as fi
from oracle.hmatrix import HLU as OHLU
from oracle.hmatrix import HMatrix as OHMatrix
from oracle.krylov import bicgstab, dense_solve
from oracle.sem import SEM
from tests.gpu_common import kappa1, need_gpu, say

pytestmark = pytest.mark.gpu

ALPHA = 1.6
RANKS = (2, 3, 5, 7)
# The iteration stops on the preconditioned residual (1e-13); the true residual |G - A X| / |G| then
# sits within kappa(A~) times that, 1e-13 to 2e-11 measured for N = 100 .. 2000 (kappa_1(A) ~ 1e8 at
# N = 100); the larger problems are held to the benchmark's 1e-10.
TRUE_RES = 1e-10


def golden():
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_table2_bicgstab_iterations.txt")
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            tab, key, *counts = line.split()
            out[(tab, int(key))] = [int(c) for c in counts]
    return out


@pytest.fixture(scope="module")
def ctx():
    fde = need_gpu()
    c = fde.Context(0)
    yield c
    c.close()


def device_counts(ctx, N, P, precision="fp64"):
    """(paper-style counts for R = 2, 3, 5, 7, true residuals, solutions) on the device."""
    import paper_1808_02937_amd as fde
    m = fi.example1(ALPHA)
    nodes = fi.graded_mesh(N, 5.0, 0.0, 10.0)
    op = fde.Operator(ctx, nodes, P, ALPHA, 1.0, 0.0)
    ft = m.f_terms
    G = op.load_vector_powers(ft.coef, ft.expo, ft.side)
    counts, rels, xs = [], [], []
    for R in RANKS:
        hm = fde.HMatrix(op, R=R, lam=1.0, leaf_elems=2)
        lu = fde.HLU(hm, tol=1e-3, precision=precision)
        X, info = fde.solve(op, G, lu, rtol=1e-13, maxit=200, method="bicgstab")
        counts.append(2 * info[0]["iters"])
        rels.append(info[0]["relres"])
        xs.append(X.cpu().numpy())
        hm.close()
    G = G.cpu().numpy()
    op.close()
    return counts, rels, xs, G


def test_example1_n100_counts_match_oracle_and_table1(ctx):
    say("example 1, N=100, P=3: device BiCGSTAB vs oracle and Table 1")
    counts, rels, xs, Gd = device_counts(ctx, 100, 3)
    m = fi.example1(ALPHA)
    sem = SEM(fi.graded_mesh(100, 5.0, 0.0, 10.0), 3, ALPHA, 1.0, 0.0)
    A = sem.system_matrix()
    G = sem.load_vector(m.f_terms)
    Xs, _ = dense_solve(A, G)
    kap = kappa1(A)
    ocounts = []
    for R in RANKS:
        F = OHLU(OHMatrix(sem, R, 1.0, 2), tol=1e-3)
        _, info = bicgstab(lambda v: A @ v, G, F.solve, tol=1e-13, side="left")
        ocounts.append(2 * info["iters"])
    say(f"  device {counts}  oracle {ocounts}  table 1 {golden()[('table1', 100)]}; true residuals "
        + " ".join(f"{r:.1e}" for r in rels) + f"; kappa_1(A) {kap:.2e}")
    assert counts == ocounts == golden()[("table1", 100)]
    assert np.abs(Gd - G).max() <= 1e-12 * np.abs(G).max()
    for X, r in zip(xs, rels):
        assert r <= 1e-11, r
        err = np.linalg.norm(X - Xs) / np.linalg.norm(Xs)
        assert err <= max(1e-10, 10 * kap * 1e-13), err


def test_example1_n400_counts_match_oracle(ctx):
    """N = 400: the device takes the oracle's number of steps (same readings: leaf 2, lambda 1)."""
    say("example 1, N=400, P=3: device vs oracle")
    counts, rels, _, _ = device_counts(ctx, 400, 3)
    m = fi.example1(ALPHA)
    sem = SEM(fi.graded_mesh(400, 5.0, 0.0, 10.0), 3, ALPHA, 1.0, 0.0)
    A = sem.system_matrix()
    G = sem.load_vector(m.f_terms)
    ocounts = []
    for R in RANKS:
        F = OHLU(OHMatrix(sem, R, 1.0, 2), tol=1e-3)
        _, info = bicgstab(lambda v: A @ v, G, F.solve, tol=1e-13, side="left")
        ocounts.append(2 * info["iters"])
    say(f"  device {counts}  oracle {ocounts}  table 1 {golden()[('table1', 400)]}")
    assert counts == ocounts
    assert max(rels) <= TRUE_RES, rels


def test_example1_table1_trends():
    """Table 1 (h-refinement, P = 3): with the leaf size fixed at two elements the counts grow with N
    faster than the printed ones for R <= 3 (the paper does not state its leaf size; at leaf 8 the
    oracle takes 8 8 4 4 at N = 400 and 10 10 6 4 at N = 800). What the table shows holds: R = 5
    and 7 need fewer steps than R = 2 and 3, counts do not fall with N, they stay within twice the
    printed count, and every solve reaches a true residual of 1e-10."""
    fde = need_gpu()
    ctx = fde.Context(0)
    prev = None
    for N in (400, 800, 1500, 2000):
        counts, rels, _, _ = device_counts(ctx, N, 3)
        ref = golden()[("table1", N)]
        say(f"example 1, N={N}, P=3: device {counts}  table 1 {ref}; true residuals "
            + " ".join(f"{r:.1e}" for r in rels))
        assert max(counts[2:]) <= min(counts[:2]), counts   # R = 5, 7 need fewer steps than R = 2, 3
        assert all(b - 2 <= a <= 2 * b for a, b in zip(counts, ref)), (counts, ref)
        assert max(rels) <= TRUE_RES, rels
        if prev is not None:
            assert all(a >= b for a, b in zip(counts, prev)), (counts, prev)
        prev = counts
    ctx.close()


@pytest.mark.parametrize("P", (3, 5, 9, 13, 19))
def test_example1_table2_within_one_step(ctx, P):
    """Table 2 (p-refinement, N = 300): within one BiCGSTAB step (two in the paper's count) of the
    printed number, and the same for every P, as the paper finds."""
    say(f"example 1, N=300, P={P}")
    counts, rels, _, _ = device_counts(ctx, 300, P)
    ref = golden()[("table2", P)]
    say(f"  device {counts}  table 2 {ref}; true residuals " + " ".join(f"{r:.1e}" for r in rels))
    assert all(abs(a - b) <= 2 for a, b in zip(counts, ref)), (counts, ref)
    assert max(rels) <= TRUE_RES, rels
    _TABLE2.setdefault("counts", counts)
    assert counts == _TABLE2["counts"], (counts, _TABLE2["counts"])


_TABLE2 = {}


def test_bicgstab_without_preconditioner_reaches_the_dense_solution(ctx):
    import paper_1808_02937_amd as fde
    say("bicgstab, no preconditioner")
    inst = fi.config_small()
    op = fde.Operator(ctx, inst.nodes, inst.P, inst.alpha, inst.theta, inst.rho)
    G = op.load_vector(inst.solution.f)
    X, info = fde.solve(op, G, None, rtol=1e-13, maxit=500, method="bicgstab")
    sem = SEM(inst.nodes, inst.P, inst.alpha, inst.theta, inst.rho)
    Xs, _ = dense_solve(sem.system_matrix(), sem.load_vector(inst.solution.f_terms))
    err = np.linalg.norm(X.cpu().numpy() - Xs) / np.linalg.norm(Xs)
    say(f"  iters {info[0]['iters']} relres {info[0]['relres']:.1e} err {err:.1e}")
    assert info[0]["status"] == 0 and info[0]["relres"] <= 1e-12 and err <= 1e-10
    op.close()


def test_bicgstab_batched_equals_alone(ctx):
    """Systems of different operators iterate in lock step; each gets the bits it gets alone."""
    import paper_1808_02937_amd as fde
    say("bicgstab batched vs alone")
    ops, lus, Gs = [], [], []
    for N, P in ((60, 3), (40, 5)):
        m = fi.example1(ALPHA)
        op = fde.Operator(ctx, fi.graded_mesh(N, 5.0, 0.0, 10.0), P, ALPHA, 1.0, 0.0)
        ft = m.f_terms
        Gs.append(op.load_vector_powers(ft.coef, ft.expo, ft.side))
        lus.append(fde.HLU(fde.HMatrix(op, R=5, lam=1.0, leaf_elems=2), tol=1e-3, precision="fp64"))
        ops.append(op)
    Xb, infob = fde.solve_batched(ctx, ops, Gs, lus, rtol=1e-13, maxit=200, method="bicgstab")
    for op, G, lu, X, ib in zip(ops, Gs, lus, Xb, infob):
        Xa, ia = fde.solve(op, G, lu, rtol=1e-13, maxit=200, method="bicgstab")
        assert ia[0]["iters"] == ib[0]["iters"]
        assert torch.equal(Xa, X)
    for op in ops:
        op.close()
