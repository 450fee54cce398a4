"""GPU parity with a polynomial degree per element (the space S_N^P with degrees P_i, Section 2.2).

The device builds such an operator at the largest degree and decouples the unknowns the degrees
leave out. Compared here with the oracle's variable-degree SEM, element by element: the dense
operator, its apply (dense and block-Toeplitz paths), the load vector with lifting, the H-matrix
(against the oracle's H-matrix of the largest degree restricted to the space's unknowns: every
block of the approximation is built from per-basis-function quantities, so restricting rows and
columns is the construction on the smaller space), the FP64 H-solve at Tol_HLU = 1e-13 against a
dense solve of that A~, and the H-LU-preconditioned FGMRES against the dense solve of A X = G and
a polynomial of the space."""
import numpy as np
import pytest
import torch

import fde_inputs as fi
from oracle.hmatrix import HMatrix as OHMatrix
from oracle.hmatrix import to_dense
from oracle.sem import SEM
from oracle.sem_hp import SEMhp
from tests.gpu_common import EPS64, kappa1, need_gpu, say

pytestmark = pytest.mark.gpu

# name: (nodes, degrees, alpha, theta, rho); leaves of 4 elements, R = 6
CASES = {
    "graded": (fi.graded_mesh(24, 3.0, 0.0, 1.0), np.random.default_rng(1).integers(1, 9, size=24), 1.6, 1.0, 0.0),
    "two_sided": (fi.two_sided_graded_mesh(40, 6, 0.5), np.random.default_rng(2).integers(2, 10, size=40),
                  1.35, 0.4, 2.0),
    "uniform": (fi.uniform_mesh(32), np.random.default_rng(3).integers(3, 8, size=32), 1.8, 0.7, 0.5),
}
R, LEAF = 6, 4


@pytest.fixture(scope="module")
def ctx():
    fde = need_gpu()
    c = fde.Context(0)
    yield c
    c.close()


def build(ctx, name):
    import paper_1808_02937_amd as fde
    nodes, Ps, al, th, rho = CASES[name]
    op = fde.Operator(ctx, nodes, Ps, al, th, rho)
    sem = SEMhp(nodes, Ps, al, th, rho)
    assert op.Nd == sem.Nd == int(np.sum(Ps)) - 1
    return op, sem


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("name", list(CASES))
def test_hp_operator_and_apply_match_oracle(ctx, name):
    say(f"hp operator {name}")
    op, sem = build(ctx, name)
    A = sem.system_matrix()
    Ad = op.dense().cpu().numpy()
    r_dense = rel(Ad, A)
    X = np.random.default_rng(7).standard_normal((3, sem.Nd))
    Y = op.apply(torch.tensor(X, device="cuda")).cpu().numpy()
    Yo = (A @ X.T).T
    r_apply = float(np.linalg.norm(Y - Yo) / np.linalg.norm(Yo))
    say(f"  Nd {sem.Nd} (largest degree {op.P}, toeplitz {op.toeplitz}): dense {r_dense:.2e}, apply {r_apply:.2e}")
    assert r_dense <= 1e-13
    assert r_apply <= 1e-12
    op.close()


@pytest.mark.parametrize("name", list(CASES))
def test_hp_load_vector_matches_oracle(ctx, name):
    say(f"hp load vector {name}")
    op, sem = build(ctx, name)
    al, th, rho = CASES[name][2:]
    # theta = 1: u(b) = 1.2, the lifting of c2; otherwise u vanishes at both ends (a nonzero end
    # value puts a non-integrable power of the distance to that end into a two-sided f)
    coef = [0.0, 0.5, 1.0, -0.3] if th == 1.0 else [0.0, 0.7, 1.0, -2.5, 0.8]
    m = fi.manufactured_from_poly(coef, al, th, rho)
    ft = m.f_terms
    G = op.load_vector_powers(ft.coef, ft.expo, ft.side, m.c1, m.c2).cpu().numpy()
    Go = sem.load_vector(ft, m.c1, m.c2)
    # the power terms of f cancel (a polynomial re-expanded in powers of b - x): FP64 evaluation
    # errs by about eps times the terms' magnitudes, added to the quadrature bound (as for one degree)
    G_abs = sem.load_vector(fi.PowerSum(np.abs(ft.coef), ft.expo, ft.side))
    bound = 1e-12 * np.abs(Go).max() + 64 * np.finfo(float).eps * np.abs(G_abs).max()
    err = float(np.abs(G - Go).max())
    say(f"  max |G - G_o| = {err:.2e} (bound {bound:.2e})")
    assert err <= bound
    op.close()


@pytest.mark.parametrize("name", list(CASES))
def test_hp_hmatrix_and_direct_hsolve(ctx, name):
    import paper_1808_02937_amd as fde
    say(f"hp H-matrix {name}")
    op, sem = build(ctx, name)
    nodes, Ps, al, th, rho = CASES[name]
    Pmax = int(np.max(Ps))
    oh = OHMatrix(SEM(nodes, Pmax, al, th, rho), R, 1.0, LEAF)
    n = len(oh.h2p)
    assert n == len(nodes[1:]) * Pmax - 1
    full = np.empty((n, n))
    full[np.ix_(oh.h2p, oh.h2p)] = to_dense(oh.root)
    emb = sem.embed(Pmax)
    Ah = full[np.ix_(emb, emb)]
    hm = fde.HMatrix(op, R=R, lam=1.0, leaf_elems=LEAF)
    At = hm.dense().cpu().numpy()
    r_h = rel(At, Ah)
    # at Tol_HLU = 1e-13 the FP64 H-LU factors A~ exactly up to rounding
    lu = fde.HLU(hm, tol=1e-13, rank_cap=16, precision="fp64", pivot_floor=0.0)
    g = np.random.default_rng(8).standard_normal((2, sem.Nd))
    x = lu.solve(torch.tensor(g, device="cuda")).cpu().numpy()
    xd = np.linalg.solve(Ah, g.T).T
    err = float(np.linalg.norm(x - xd) / np.linalg.norm(xd))
    kap = kappa1(Ah)
    say(f"  |A~ - A~_o| {r_h:.2e}; direct H-solve {err:.2e} (kappa_1(A~) {kap:.2e})")
    assert r_h <= 1e-13
    assert err <= 10 * kap * EPS64
    lu.close()
    op.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name", list(CASES))
def test_hp_preconditioned_solve_matches_dense(ctx, name, precision):
    import paper_1808_02937_amd as fde
    say(f"hp solve {name} {precision}")
    op, sem = build(ctx, name)
    A = sem.system_matrix()
    Gs = np.random.default_rng(9).standard_normal((3, sem.Nd))
    Xs = np.linalg.solve(A, Gs.T).T
    hm = fde.HMatrix(op, R=R, lam=1.0, leaf_elems=LEAF)
    lu = fde.HLU(hm, tol=1e-3, precision=precision)
    X, info = fde.solve(op, torch.tensor(Gs, device="cuda"), lu, rtol=1e-13, maxit=300)
    x = X.cpu().numpy()
    err = float(np.linalg.norm(x - Xs) / np.linalg.norm(Xs))
    its = [i["iters"] for i in info]
    say(f"  iterations {its}, |X - X_dense| / |X_dense| = {err:.2e}")
    assert all(i["status"] == 0 and i["relres"] <= 1e-13 for i in info)
    assert max(its) <= 12
    assert err <= 1e-11
    lu.close()
    op.close()


def test_hp_polynomial_of_the_space_is_reproduced(ctx):
    """u of degree 4 and every P_i >= 4: the solve returns u's coefficients (Theorem 1)."""
    import paper_1808_02937_amd as fde
    nodes = fi.two_sided_graded_mesh(30, 5, 0.5)
    Ps = np.random.default_rng(10).integers(4, 11, size=30)
    al, th, rho = 1.55, 0.3, 1.0
    m = fi.manufactured_from_poly([0.0, 0.7, 1.0, -2.5, 0.8], al, th, rho)
    op = fde.Operator(ctx, nodes, Ps, al, th, rho)
    sem = SEMhp(nodes, Ps, al, th, rho)
    Xu = sem.interpolate_coefficients(m.u)
    ft = m.f_terms
    G = op.load_vector_powers(ft.coef, ft.expo, ft.side)
    lu = fde.HLU(fde.HMatrix(op, R=8, lam=1.0, leaf_elems=4), tol=1e-3, precision="fp32")
    X, info = fde.solve(op, G, lu, rtol=1e-13)
    err = float(np.linalg.norm(X.cpu().numpy() - Xu) / np.linalg.norm(Xu))
    say(f"hp polynomial of the space: {info[0]['iters']} iterations, |X - X_u| / |X_u| = {err:.2e}")
    assert err <= 1e-10
    lu.close()
    op.close()


def test_hp_one_degree_equals_the_uniform_operator(ctx):
    """Every P_i = P: the same numbers as the one-degree operator, bit for bit."""
    import paper_1808_02937_amd as fde
    nodes = fi.graded_mesh(20, 2.0, 0.0, 1.0)
    P, al, th, rho = 5, 1.5, 0.6, 0.0
    a = fde.Operator(ctx, nodes, [P] * 20, al, th, rho)
    b = fde.Operator(ctx, nodes, P, al, th, rho)
    assert a.Nd == b.Nd
    X = torch.tensor(np.random.default_rng(11).standard_normal((2, b.Nd)), device="cuda")
    assert torch.equal(a.apply(X), b.apply(X))
    la = fde.HLU(fde.HMatrix(a, R=6, lam=1.0, leaf_elems=4), tol=1e-3, precision="fp32")
    lb = fde.HLU(fde.HMatrix(b, R=6, lam=1.0, leaf_elems=4), tol=1e-3, precision="fp32")
    Xa, _ = fde.solve(a, X, la, rtol=1e-12)
    Xb, _ = fde.solve(b, X, lb, rtol=1e-12)
    assert torch.equal(Xa, Xb)
    for o in (la, lb, a, b):
        o.close()


def test_hp_unsupported_calls_are_refused(ctx):
    import paper_1808_02937_amd as fde
    from paper_1808_02937_amd._abi import FDE_EUNSUPPORTED, FDEError
    op = fde.Operator(ctx, fi.uniform_mesh(8), [2, 3, 4, 5, 2, 3, 4, 5], 1.5, 0.5, 0.0)
    X = torch.zeros(1, op.Nd, dtype=torch.float64, device="cuda")
    with pytest.raises(FDEError) as ei:
        op.apply_noalloc(X, torch.empty_like(X))
    assert ei.value.code == FDE_EUNSUPPORTED
    with pytest.raises(FDEError):
        fde.Operator(ctx, fi.uniform_mesh(4), [1, 1, 1, 1], 1.5, 0.5, 0.0)   # no degree >= 2
    op.close()
