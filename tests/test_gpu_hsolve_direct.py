"""The H-matrix approximation system A~ X = G solved directly by the FP64 H-LU at Tol_HLU = 1e-13
(Section 5: the second of its three systems), on the GPU.

- At that tolerance the H-LU is an exact factorisation of A~ up to rounding, so X equals the
  dense solution of A~ X = G (checked against a LAPACK solve of the oracle's A~).
- As N grows, the solution of the approximate system stops converging to u and then degrades,
  because the H-matrix error of A~ accumulates, while the H-LU-preconditioned solve of A X = G
  keeps the SEM accuracy (Example 1, left of the h-refinement figure)."""
import numpy as np
import pytest
import torch

import fde_inputs as fi
from oracle.hmatrix import HMatrix as OHMatrix
from oracle.hmatrix import to_dense
from oracle.sem import SEM
from tests.gpu_common import EPS64, kappa1, need_gpu, say

pytestmark = pytest.mark.gpu

ALPHA = 1.6


@pytest.fixture(scope="module")
def ctx():
    fde = need_gpu()
    c = fde.Context(0)
    yield c
    c.close()


def example1_operator(ctx, N, P=3):
    import paper_1808_02937_amd as fde
    m = fi.example1(ALPHA)
    nodes = fi.graded_mesh(N, 5.0, 0.0, 10.0)
    op = fde.Operator(ctx, nodes, P, ALPHA, 1.0, 0.0)
    ft = m.f_terms
    return m, nodes, op, op.load_vector_powers(ft.coef, ft.expo, ft.side)


@pytest.mark.parametrize("R", (2, 7))
def test_direct_hsolve_is_the_dense_solution_of_the_approximate_system(ctx, R):
    import paper_1808_02937_amd as fde
    say(f"direct H-solve, N=100, R={R}")
    m, nodes, op, G = example1_operator(ctx, 100)
    hm = fde.HMatrix(op, R=R, lam=1.0, leaf_elems=2)
    lu = fde.HLU(hm, tol=1e-13, rank_cap=16, precision="fp64", pivot_floor=0.0)
    X = lu.solve(G).cpu().numpy()
    sem = SEM(nodes, 3, ALPHA, 1.0, 0.0)
    oh = OHMatrix(sem, R, 1.0, 2)
    At = np.empty((sem.Nd, sem.Nd))
    At[np.ix_(oh.h2p, oh.h2p)] = to_dense(oh.root)
    Gn = G.cpu().numpy()
    Xd = np.linalg.solve(At, Gn)
    kap = kappa1(At)
    err = np.linalg.norm(X - Xd) / np.linalg.norm(Xd)
    say(f"  |X - A~^-1 G| / |A~^-1 G| = {err:.2e} (kappa_1(A~) {kap:.2e}); ranks <= {lu.max_rank()}")
    assert err <= 10 * kap * EPS64, err
    op.close()


def test_direct_hsolve_loses_accuracy_with_n_while_the_preconditioned_solve_does_not(ctx):
    import paper_1808_02937_amd as fde
    Ns = (25, 50, 100, 200, 400, 800, 1600)
    rows = {}
    for N in Ns:
        m, nodes, op, G = example1_operator(ctx, N)
        sem = SEM(nodes, 3, ALPHA, 1.0, 0.0)
        k = min(40, N)
        t = np.concatenate([np.linspace(0.0, 10.0, 4001), nodes[:k] + 0.5 * np.diff(nodes[:k + 1])])
        u = m.u(t)

        def linf(X):
            return float(np.abs(sem.evaluate(X.cpu().numpy().ravel(), t) - u).max())

        errs = {}
        for R in (2, 5):
            hm = fde.HMatrix(op, R=R, lam=1.0, leaf_elems=2)
            direct = fde.HLU(hm, tol=1e-13, rank_cap=16, precision="fp64", pivot_floor=0.0)
            errs[("direct", R)] = linf(direct.solve(G))
            prec = fde.HLU(hm, tol=1e-3, precision="fp64")
            X, info = fde.solve(op, G, prec, rtol=1e-13, maxit=300, method="bicgstab")
            errs[("prec", R)] = linf(X)
            hm.close()
        rows[N] = errs
        say(f"N={N:5d}  L-inf error: preconditioned R=2 {errs[('prec', 2)]:.2e} R=5 {errs[('prec', 5)]:.2e} | "
            f"direct H-LU R=2 {errs[('direct', 2)]:.2e} R=5 {errs[('direct', 5)]:.2e}")
        op.close()
    prec2 = [rows[N][("prec", 2)] for N in Ns]
    # the preconditioned solve converges under h-refinement, whatever the rank
    assert all(b < a for a, b in zip(prec2, prec2[1:])), prec2
    for N in Ns:
        assert rows[N][("prec", 5)] == pytest.approx(rows[N][("prec", 2)], rel=1e-3, abs=1e-12)
    # the approximate system: at R = 2 its error stops falling and grows again as N grows, far above
    # the preconditioned one at the largest N; R = 5 stays close to the SEM error for longer
    d2 = [rows[N][("direct", 2)] for N in Ns]
    best = int(np.argmin(d2))
    assert best < len(Ns) - 1 and d2[-1] > 2 * d2[best], d2
    assert d2[-1] > 10 * prec2[-1], (d2[-1], prec2[-1])
    d5 = [rows[N][("direct", 5)] for N in Ns]
    assert all(a <= b for a, b in zip(d5, d2)), (d5, d2)
