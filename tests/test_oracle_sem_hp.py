"""Pins of the oracle's SEM with a polynomial degree per element (Section 2.2, S_N^P with P_i)."""
import numpy as np
import pytest

import fde_inputs as fi
from oracle.sem import SEM
from oracle.sem_hp import SEMhp

MESHES = {
    "uniform": fi.uniform_mesh(9),
    "graded": fi.graded_mesh(9, 3.0, 0.0, 1.0),
    "two_sided": fi.two_sided_graded_mesh(12, 3, 0.5),
}


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("mesh", list(MESHES))
def test_one_degree_reproduces_the_uniform_oracle(mesh):
    x = MESHES[mesh]
    P = 5
    hp = SEMhp(x, [P] * (len(x) - 1), 1.45, 0.3, 1.7)
    u = SEM(x, P, 1.45, 0.3, 1.7)
    assert hp.Nd == u.Nd
    assert rel(hp.system_matrix(), u.system_matrix()) <= 1e-14
    assert rel(hp.system_matrix(True), u.system_matrix(True)) <= 1e-14
    m = fi.manufactured_from_poly([0.0, 0.5, 1.0, -0.3], 1.45, 0.3, 1.7)
    assert rel(hp.load_vector(m.f_terms, m.c1, m.c2), u.load_vector(m.f_terms, m.c1, m.c2)) <= 1e-13


@pytest.mark.parametrize("mesh", list(MESHES))
def test_raising_degrees_nests_the_systems(mesh):
    """psi_p does not depend on P_i, so S_N^P with degrees Ps is a subspace of the one with
    degrees Ps' >= Ps, spanned by a subset of the same basis functions: the smaller system is the
    principal submatrix of the larger one (and its load vector the matching entries)."""
    x = MESHES[mesh]
    N = len(x) - 1
    rng = np.random.default_rng(5)
    Ps = rng.integers(1, 7, size=N)
    Ps[rng.integers(0, N)] = 1            # an element without bubbles
    Pmax = 8
    hp = SEMhp(x, Ps, 1.7, 0.6, 0.4)
    big = SEM(x, Pmax, 1.7, 0.6, 0.4)
    emb = hp.embed(Pmax)
    A = hp.system_matrix()
    assert rel(A, big.system_matrix()[np.ix_(emb, emb)]) <= 1e-13
    m = fi.manufactured_from_poly([0.0, 1.0, -1.0, 0.4], 1.7, 0.6, 0.4)
    G = hp.load_vector(m.f_terms, m.c1, m.c2)
    assert rel(G, big.load_vector(m.f_terms, m.c1, m.c2)[emb]) <= 1e-12
    # and between two hp spaces
    Ps2 = Ps + rng.integers(0, 3, size=N)
    hp2 = SEMhp(x, Ps2, 1.7, 0.6, 0.4)
    idx = np.zeros(hp.Nd, dtype=int)
    for e in range(N):
        for p in range(1, int(Ps[e])):
            idx[hp.idx_bubble(e, p)] = hp2.idx_bubble(e, p)
    for j in range(1, N):
        idx[hp.idx_hat(j)] = hp2.idx_hat(j)
    assert rel(A, hp2.system_matrix()[np.ix_(idx, idx)]) <= 1e-13
    assert hp.Nd == int(Ps.sum()) - 1


@pytest.mark.parametrize("theta,rho", [(0.5, 0.0), (1.0, 0.0), (0.2, 3.0)])
@pytest.mark.parametrize("mesh", list(MESHES))
def test_polynomial_in_the_space_is_reproduced(theta, rho, mesh):
    """u of degree 4 lies in S_N^P when every P_i >= 4: Galerkin + coercivity give A X_u = G
    exactly (Theorem 1, eq. (SEM)), with G from the closed-form right-hand side."""
    x = MESHES[mesh]
    N = len(x) - 1
    Ps = np.random.default_rng(6).integers(4, 9, size=N)
    m = fi.manufactured_from_poly([0.0, 0.7, 1.0, -2.5, 0.8], 1.55, theta, rho)
    hp = SEMhp(x, Ps, 1.55, theta, rho)
    A = hp.system_matrix()
    G = hp.load_vector(m.f_terms)
    X = hp.interpolate_coefficients(m.u)
    assert np.linalg.norm(A @ X - G) <= 1e-12 * np.linalg.norm(G)
    # the solution's higher modes vanish
    Xs = np.linalg.solve(A, G)
    assert np.linalg.norm(Xs - X) <= 1e-10 * np.linalg.norm(X)


def test_lifting_with_variable_degrees():
    m = fi.manufactured_from_poly([0.0, 0.5, 1.0, -0.3], 1.4, 1.0, 1.5)
    x = fi.graded_mesh(10, 2.0, 0.0, 1.0)
    Ps = [3, 4, 3, 5, 6, 3, 4, 3, 3, 7]
    hp = SEMhp(x, Ps, 1.4, 1.0, 1.5)
    G = hp.load_vector(m.f_terms, m.c1, m.c2)
    X = hp.interpolate_coefficients(m.u)
    assert np.linalg.norm(hp.system_matrix() @ X - G) <= 1e-13 * np.linalg.norm(G)


def test_transpose_identity_and_positivity():
    x = MESHES["two_sided"]
    Ps = [2, 3, 5, 1, 4, 6, 2, 3, 7, 2, 3, 4]
    A1 = SEMhp(x, Ps, 1.3, 0.2, 0.5).system_matrix()
    A2 = SEMhp(x, Ps, 1.3, 0.8, 0.5).system_matrix()
    assert np.abs(A1 - A2.T).max() <= 1e-13 * np.abs(A1).max()
    for th in (0.0, 0.37, 1.0):
        A = SEMhp(x, Ps, 1.3, th, 0.0).system_matrix()
        assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0.0
