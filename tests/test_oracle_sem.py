"""Pins for the oracle's SEM assembly (no GPU)."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import eval_jacobi, eval_legendre, gamma

import fde_inputs as fi
from oracle.sem import SEM


def brute_moment(sem, e, f, m, n):
    """gamma0 int_{I_e} int_{I_f} (t-s)_+^{1-alpha} L_m L_n by adaptive quadrature."""
    x, h, al = sem.x, sem.h, sem.alpha
    Lm = lambda t: eval_legendre(m, 2 * (t - x[e]) / h[e] - 1)
    Ln = lambda s: eval_legendre(n, 2 * (s - x[f]) / h[f] - 1)
    if e == f:
        inner = lambda t: integrate.quad(Ln, x[f], t, weight="alg", wvar=(0.0, 1.0 - al),
                                         epsabs=1e-15, epsrel=1e-13, limit=200)[0] if t > x[f] else 0.0
    else:
        hi = x[f + 1]
        if f == e - 1:
            inner = lambda t: integrate.quad(lambda s: Ln(s) * (t - s) ** (1 - al), x[f], hi,
                                             points=[hi], epsabs=1e-15, epsrel=1e-13, limit=200)[0]
        else:
            inner = lambda t: integrate.quad(lambda s: Ln(s) * (t - s) ** (1 - al), x[f], hi,
                                             epsabs=1e-15, epsrel=1e-13, limit=200)[0]
    val = integrate.quad(lambda t: Lm(t) * inner(t), x[e], x[e + 1], epsabs=1e-15, epsrel=1e-13,
                         limit=200)[0]
    return sem.gamma0 * val


def test_same_element_moment_closed_form():
    """gamma0 int_{-1}^{xi}(xi-eta)^{1-alpha} L_n = -1I^{mu} L_n
       = Gamma(n+1)/Gamma(n+1+mu) (1+xi)^mu P_n^{(-mu,mu)}(xi), mu = 2 - alpha."""
    for al in (1.15, 1.5, 1.85):
        P = 6
        sem = SEM(fi.uniform_mesh(1, -1.0, 1.0), P, al, 1.0, 0.0)
        K = sem.moment_same(2.0)
        mu = 2.0 - al
        for m in range(P):
            for n in range(P):
                g = lambda xi: (eval_legendre(m, xi) * gamma(n + 1) / gamma(n + 1 + mu)
                                * eval_jacobi(n, -mu, mu, xi))
                ref = integrate.quad(g, -1, 1, weight="alg", wvar=(mu, 0.0), epsabs=1e-15,
                                     epsrel=1e-14)[0]
                assert abs(K[m, n] - ref) <= 1e-13 * max(1.0, abs(ref)), (al, m, n)


@pytest.mark.parametrize("mesh", [
    fi.uniform_mesh(5),
    np.array([0.0, 0.001, 0.031, 0.3, 0.4, 1.0]),          # ratios up to 30 and 1/6
])
def test_moments_against_brute_force(mesh):
    sem = SEM(mesh, 3, 1.6, 1.0, 0.0)
    for (e, f) in [(0, 0), (2, 2), (1, 0), (2, 1), (4, 3), (2, 0), (3, 0), (4, 1), (5 - 1, 0)]:
        if e >= sem.N:
            continue
        K = sem.pair_moment(e, f)
        for (m, n) in [(0, 0), (1, 2), (2, 1), (2, 2)]:
            ref = brute_moment(sem, e, f, m, n)
            assert abs(K[m, n] - ref) <= 1e-11 * np.abs(K).max(), (e, f, m, n, K[m, n], ref)


def test_separated_uniform_L0_closed_form():
    """int int_{[-1,1]^2} (x - t + 2k)^{1-alpha} = [(2k+2)^{3-a} - 2(2k)^{3-a} + (2k-2)^{3-a}]/((2-a)(3-a))."""
    al = 1.45
    sem = SEM(fi.uniform_mesh(1, -1.0, 1.0), 4, al, 1.0, 0.0)
    for k in range(2, 9):
        K = sem.moment_separated(2.0, 2.0, 2.0 * (k - 1))
        ref = ((2 * k + 2) ** (3 - al) - 2 * (2 * k) ** (3 - al) + (2 * k - 2) ** (3 - al)) / ((2 - al) * (3 - al))
        assert abs(K[0, 0] / sem.gamma0 - ref) < 1e-13 * abs(ref)


def test_appendix_corrected_hat_generators():
    """Appendix A: b0 = gamma0 2^{3-a}/(4(2-a)(3-a)) (the printed value lacks 1/(2-a)),
    e0 = -gamma0 2^{3-a}/(4(3-a)); here from the same-element moment with half-hat slopes 1/2."""
    for al in (1.2, 1.7):
        sem = SEM(fi.uniform_mesh(1, -1.0, 1.0), 3, al, 1.0, 0.0)
        K = sem.moment_same(2.0)
        g0 = 1 / math.gamma(2 - al)
        b0 = 0.25 * K[0, 0]
        assert abs(b0 - g0 * 2 ** (3 - al) / (4 * (2 - al) * (3 - al))) < 1e-14
        # half hat (1-x)/2: derivative-outside form carries the boundary term (1+x)^{1-alpha}
        e0 = 0.25 * K[0, 0] - 0.5 * g0 * 2 ** (2 - al) / (2 - al)
        assert abs(e0 - (-g0 * 2 ** (3 - al) / (4 * (3 - al)))) < 1e-14


@pytest.mark.parametrize("theta,rho", [(0.5, 0.0), (1.0, 0.0), (0.0, 3.0), (0.3, 2.0)])
@pytest.mark.parametrize("mesh_kind", ["uniform", "graded", "two_sided"])
def test_manufactured_solution_in_space(theta, rho, mesh_kind):
    """u in S_N^P: Galerkin + coercivity give A X_u = G exactly (Theorem 1, eq. (SEM))."""
    m = fi.manufactured_from_poly([0.0, 0.7, 1.0, -2.5, 0.8], 1.55, theta, rho)
    mesh = {"uniform": fi.uniform_mesh(9), "graded": fi.graded_mesh(9, 3.0, 0.0, 1.0),
            "two_sided": fi.two_sided_graded_mesh(14, 3, 0.5)}[mesh_kind]
    sem = SEM(mesh, 4, 1.55, theta, rho)
    A = sem.system_matrix()
    G = sem.load_vector(m.f_terms)
    X = sem.interpolate_coefficients(m.u)
    assert np.linalg.norm(A @ X - G) <= 1e-12 * np.linalg.norm(G)


def test_config_small_reproduces_solution():
    inst = fi.config_small()
    sem = SEM(inst.nodes, inst.P, inst.alpha, inst.theta, inst.rho)
    A = sem.system_matrix()
    G = sem.load_vector(inst.solution.f_terms)
    Xs = np.linalg.solve(A, G)
    X = sem.interpolate_coefficients(inst.solution.u)
    assert np.linalg.norm(Xs - X) <= 1e-13 * np.linalg.norm(X)


def test_lifting_nonzero_boundary_value():
    """theta = 1, c1 = 0, c2 != 0 (lifting with the boundary hat varphi_N)."""
    m = fi.manufactured_from_poly([0.0, 0.5, 1.0, -0.3], 1.4, 1.0, 1.5)
    assert m.c1 == 0.0 and abs(m.c2 - 1.2) < 1e-14
    sem = SEM(fi.graded_mesh(10, 2.0, 0.0, 1.0), 3, 1.4, 1.0, 1.5)
    A = sem.system_matrix()
    G = sem.load_vector(m.f_terms, m.c1, m.c2)
    X = sem.interpolate_coefficients(m.u)
    assert np.linalg.norm(A @ X - G) <= 1e-13 * np.linalg.norm(G)


def test_transpose_symmetry_and_coercivity():
    mesh = fi.two_sided_graded_mesh(12, 3, 0.5)
    A1 = SEM(mesh, 4, 1.3, 0.2, 0.5).system_matrix()
    A2 = SEM(mesh, 4, 1.3, 0.8, 0.5).system_matrix()
    assert np.abs(A1 - A2.T).max() <= 1e-13 * np.abs(A1).max()
    Ah = SEM(mesh, 4, 1.3, 0.5, 0.0).system_matrix()
    assert np.abs(Ah - Ah.T).max() <= 1e-13 * np.abs(Ah).max()
    for th in (0.0, 0.37, 1.0):
        A = SEM(mesh, 4, 1.3, th, 0.0).system_matrix()
        assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0.0


def test_alpha_one_limit():
    """alpha = 1: kernel 1, gamma0 = 1, S_l(i,j) = (varphi_i', varphi_j); S = 0 at theta = 1/2."""
    mesh = np.array([0.0, 0.2, 0.25, 0.6, 1.0])
    sem = SEM(mesh, 3, 1.5, 1.0, 0.0)
    sem.alpha, sem.gamma0 = 1.0, 1.0
    Sl = sem.stiffness_lower()
    # (phi_i', phi_j) by Gauss-Legendre, independent of the moment code
    from oracle.sem import psi_table
    from oracle.quadrature import gauss_legendre
    xq, wq = gauss_legendre(8)
    Nd = sem.Nd
    ref = np.zeros((Nd, Nd))
    for e in range(sem.N):
        B = np.vstack([(1 - xq) / 2, (1 + xq) / 2, psi_table(3, xq)])
        dB = np.vstack([-0.5 * np.ones_like(xq), 0.5 * np.ones_like(xq),
                        -(2 * np.arange(1, 3)[:, None] + 1) * np.vstack([xq, 1.5 * xq ** 2 - 0.5])])
        dofs = sem.local_dofs(e)
        loc = (dB * wq) @ B.T          # int phi_a' phi_b dxi (derivative in xi)
        for a_, ia in enumerate(dofs):
            for b_, ib in enumerate(dofs):
                if ia >= 0 and ib >= 0:
                    ref[ia, ib] += loc[a_, b_]
    assert np.abs(Sl - ref).max() < 1e-13
    assert np.abs(Sl + Sl.T).max() < 1e-13


def test_alpha_two_trend():
    """alpha -> 2-: S approaches the classical stiffness (varphi_i', varphi_j')."""
    mesh = fi.uniform_mesh(6)
    errs = []
    for al in (1.9, 1.99, 1.999):
        sem = SEM(mesh, 3, al, 0.5, 0.0)
        A = sem.system_matrix()
        sem2 = SEM(mesh, 3, 1.5, 0.5, 0.0)
        D = sem2.derivative_map().toarray()
        P = 3
        Kc = np.zeros((sem.N * P, sem.N * P))
        for e in range(sem.N):
            Kc[e * P:(e + 1) * P, e * P:(e + 1) * P] = np.diag(sem.h[e] / (2 * np.arange(P) + 1))
        Lap = D.T @ Kc @ D
        errs.append(np.abs(A - Lap).max() / np.abs(Lap).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 5e-3


def test_rhs_formula_against_brute_force_fractional_derivative():
    """f of fde_inputs equals -D^2(theta aI^{2-a} u + (1-theta) xI_b^{2-a} u) + rho u."""
    al, th, rho = 1.6, 0.3, 0.7
    m = fi.manufactured_from_poly([0.0, 1.0, -1.0, 0.4], al, th, rho)
    beta = 2 - al
    def I_left(x):
        return integrate.quad(lambda s: m.u(np.array([s]))[0], 0, x, weight="alg",
                              wvar=(0.0, beta - 1), epsabs=1e-14, epsrel=1e-13)[0] / gamma(beta)
    def I_right(x):
        return integrate.quad(lambda s: m.u(np.array([s]))[0], x, 1, weight="alg",
                              wvar=(beta - 1, 0.0), epsabs=1e-14, epsrel=1e-13)[0] / gamma(beta)
    d = 1e-3
    for x in (0.3, 0.55, 0.8):
        def F(y):
            return th * I_left(y) + (1 - th) * I_right(y)
        d2 = (-F(x + 2 * d) + 16 * F(x + d) - 30 * F(x) + 16 * F(x - d) - F(x - 2 * d)) / (12 * d * d)
        ref = -d2 + rho * m.u(np.array([x]))[0]
        assert abs(m.f(np.array([x]))[0] - ref) < 1e-6 * max(1, abs(ref))
