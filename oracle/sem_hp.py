"""Spectral element discretisation with a polynomial degree per element, plain FP64 (oracle).
TEST INFRASTRUCTURE ONLY.

Section 2.2 defines the space S_N^P with degree P_i on element i: the hats varphi_j
(j = 1..N-1) plus the bubbles phi_i^p, p = 1..P_i - 1, on each element, so
Nd = sum_i P_i - 1, with the unknowns ordered X = [bubbles of element 1 (P_1 - 1 of them);
...; bubbles of element N; hats] (the vector X below eq. (lsys)). The entries are the same
bilinear forms as with one degree: S_l = D^T K D, where the pair of elements (e, f) contributes
the P_e x P_f block of kernel moments
    K^{ef}_{mn} = gamma0 int_{I_e} int_{I_f} (t-s)_+^{1-alpha} L_m(xi_e(t)) L_n(xi_f(s)) ds dt,
m < P_e, n < P_f (the derivative of a degree-P_e function on e is a Legendre series up to
L_{P_e - 1}). The oracle takes each block from the one-degree oracle run at degree
max(P_e, P_f), whose quadrature is exact or converged for every moment of that degree, and keeps
its leading P_e x P_f part; everything else (the derivative map, the mass matrix, the load vector
and the lifting) is written here per element with its own degree.

Pins (tests/test_oracle_sem_hp.py): one degree everywhere reproduces the one-degree oracle;
raising degrees nests the systems (the old matrix is the principal submatrix of the new one on
the shared basis functions, because psi_p does not depend on P_i); a polynomial of degree
<= min P_i is reproduced exactly from its closed-form right-hand side; the transpose identity
A(theta) = A(1 - theta)^T and positivity of the symmetric part.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .quadrature import gauss_jacobi, gauss_legendre, gauss_legendre_on, graded_panels
from .sem import SEM, psi_table


class SEMhp:
    """The SEM system of eq. (lsys) on a mesh x_0 < ... < x_N with degree Ps[i] on element i."""

    def __init__(self, nodes, Ps, alpha: float, theta: float, rho: float):
        self.x = np.asarray(nodes, dtype=np.float64)
        self.N = len(self.x) - 1
        self.h = np.diff(self.x)
        self.Ps = np.asarray(Ps, dtype=np.int64)
        self.alpha = float(alpha)
        self.theta = float(theta)
        self.rho = float(rho)
        self.gamma0 = 1.0 / math.gamma(2.0 - self.alpha)
        assert self.N >= 1 and len(self.Ps) == self.N and np.all(self.Ps >= 1) and np.all(self.h > 0)
        assert 1.0 < self.alpha < 2.0 and 0.0 <= self.theta <= 1.0
        self.nb = self.Ps - 1                                      # bubbles per element
        self.boff = np.concatenate([[0], np.cumsum(self.nb)])       # first bubble of each element
        self.loff = np.concatenate([[0], np.cumsum(self.Ps)])       # first Legendre row of each element
        self.Nd = int(self.Ps.sum()) - 1
        self._sems = {}
        self._K = None

    # ---- unknown order ----
    def idx_bubble(self, e: int, p: int) -> int:
        """Element e (0-based), mode p (1..P_e - 1)."""
        assert 1 <= p < self.Ps[e]
        return int(self.boff[e]) + p - 1

    def idx_hat(self, j: int) -> int:
        """Interior node j (1..N-1)."""
        return int(self.boff[-1]) + j - 1

    # ---- D: unknowns -> per-element Legendre coefficients of the derivative ----
    def derivative_map(self, with_boundary: bool = False) -> sp.csr_matrix:
        """Sparse (sum P_i) x Nd map (x (Nd+2) with the boundary hats varphi_0, varphi_N).

        On element e, (phi_e^p)' = -(2p+1) (2/h_e) L_p(xi_e); a hat has slope +-1/h_e, a
        multiple of L_0 (Section 2.2)."""
        N, h, lo = self.N, self.h, self.loff
        rows, cols, vals = [], [], []
        for e in range(N):
            for p in range(1, int(self.Ps[e])):
                rows.append(lo[e] + p); cols.append(self.idx_bubble(e, p)); vals.append(-(2 * p + 1) * 2.0 / h[e])
        for j in range(1, N):
            rows.append(lo[j - 1]); cols.append(self.idx_hat(j)); vals.append(1.0 / h[j - 1])
            rows.append(lo[j]); cols.append(self.idx_hat(j)); vals.append(-1.0 / h[j])
        ncol = self.Nd
        if with_boundary:
            rows.append(lo[0]); cols.append(self.Nd); vals.append(-1.0 / h[0])
            rows.append(lo[N - 1]); cols.append(self.Nd + 1); vals.append(1.0 / h[N - 1])
            ncol += 2
        return sp.csr_matrix((vals, (rows, cols)), shape=(int(lo[-1]), ncol))

    # ---- element-pair moments ----
    def _sem(self, P: int) -> SEM:
        P = max(int(P), 2)
        if P not in self._sems:
            self._sems[P] = SEM(self.x, P, self.alpha, self.theta, self.rho)
        return self._sems[P]

    def pair_moment(self, e: int, f: int) -> np.ndarray:
        """K^{ef} (P_e x P_f), f <= e."""
        Pe, Pf = int(self.Ps[e]), int(self.Ps[f])
        return self._sem(max(Pe, Pf)).pair_moment(e, f)[:Pe, :Pf]

    def element_operator(self) -> np.ndarray:
        """Dense block-lower K (sum P_i squared) with blocks K^{ef}, f <= e."""
        if self._K is None:
            lo = self.loff
            K = np.zeros((lo[-1], lo[-1]))
            for e in range(self.N):
                for f in range(e + 1):
                    K[lo[e]:lo[e + 1], lo[f]:lo[f + 1]] = self.pair_moment(e, f)
            self._K = K
        return self._K

    # ---- matrices of eq. (lsys) ----
    def local_mass(self, P: int) -> np.ndarray:
        """int_{-1}^{1} of products of [phi_L, phi_R, psi_1..psi_{P-1}] (reference element)."""
        xq, wq = gauss_legendre(P + 2)
        B = np.vstack([(1.0 - xq) / 2.0, (1.0 + xq) / 2.0, psi_table(P, xq)])
        return (B * wq) @ B.T

    def local_dofs(self, e: int, with_boundary: bool = False):
        """Global indices of [left hat, right hat, bubbles] on element e (-1 if absent)."""
        N = self.N

        def hat(j):
            if 1 <= j <= N - 1:
                return self.idx_hat(j)
            if with_boundary and j == 0:
                return self.Nd
            if with_boundary and j == N:
                return self.Nd + 1
            return -1
        return [hat(e), hat(e + 1)] + [self.idx_bubble(e, p) for p in range(1, int(self.Ps[e]))]

    def mass(self, with_boundary: bool = False) -> np.ndarray:
        n = self.Nd + (2 if with_boundary else 0)
        M = np.zeros((n, n))
        for e in range(self.N):
            Ml = self.local_mass(int(self.Ps[e]))
            d = self.local_dofs(e, with_boundary)
            for a_, ia in enumerate(d):
                for b_, ib in enumerate(d):
                    if ia >= 0 and ib >= 0:
                        M[ia, ib] += 0.5 * self.h[e] * Ml[a_, b_]
        return M

    def system_matrix(self, with_boundary: bool = False) -> np.ndarray:
        """A = rho M + theta S_l + (1-theta) S_l^T (rows: the Nd test functions)."""
        K = self.element_operator()
        D = self.derivative_map(with_boundary).toarray()
        Dr = D[:, :self.Nd]
        S = Dr.T @ (self.theta * K + (1.0 - self.theta) * K.T) @ D
        return self.rho * self.mass(with_boundary)[:self.Nd, :] + S

    # ---- load vector with lifting of c1, c2 ----
    def load_vector(self, f_terms, c1: float = 0.0, c2: float = 0.0) -> np.ndarray:
        """G_i = (f, varphi_i or phi_e^p) for f = sum_j c_j d_j(x)^{p_j} (signed powers).

        Each element uses its own degree: Gauss-Jacobi with weight (1+xi)^{p+1} on the element
        touching the singular end, graded Gauss-Legendre elsewhere; then the lifting
        G -= c1 a(varphi_0, .) + c2 a(varphi_N, .)."""
        N = self.N
        a, b = self.x[0], self.x[-1]
        G = np.zeros(self.Nd)
        for c, p, side in zip(f_terms.coef, f_terms.expo, f_terms.side):
            for e in range(N):
                P = int(self.Ps[e])
                he = self.h[e]
                touching = (side == 0 and e == 0) or (side == 1 and e == N - 1)
                if touching:
                    if side == 0:
                        xq, wq = gauss_jacobi(P + 2, 0.0, p + 1.0)
                        fac = 1.0 + xq
                    else:
                        xq, wq = gauss_jacobi(P + 2, p + 1.0, 0.0)
                        fac = 1.0 - xq
                    Bq = np.vstack([(1.0 - xq) / 2.0, (1.0 + xq) / 2.0, psi_table(P, xq)]) / fac
                    vals = c * (0.5 * he) ** (p + 1.0) * (Bq @ wq)
                else:
                    gap = (self.x[e] - a) if side == 0 else (b - self.x[e + 1])
                    vals = np.zeros(P + 1)
                    for lo, hi in graded_panels(he, gap):
                        uq, wq = gauss_legendre_on(P + 24, lo, hi)
                        xi = 2.0 * uq / he - 1.0 if side == 0 else 1.0 - 2.0 * uq / he
                        Bq = np.vstack([(1.0 - xi) / 2.0, (1.0 + xi) / 2.0, psi_table(P, xi)])
                        vals += Bq @ (wq * c * (gap + uq) ** p)
                for k, i in enumerate(self.local_dofs(e)):
                    if i >= 0:
                        G[i] += vals[k]
        if c1 != 0.0 or c2 != 0.0:
            Ab = self.system_matrix(with_boundary=True)
            G -= c1 * Ab[:, self.Nd] + c2 * Ab[:, self.Nd + 1]
        return G

    # ---- coefficients of a function of S_N^P ----
    def interpolate_coefficients(self, u) -> np.ndarray:
        """X of a function u of the space (exact when u is a polynomial of degree <= P_e on each
        element e): nodal values for the hats, a least-squares fit of u minus the hat
        interpolant by psi_1..psi_{P_e - 1} at Gauss points for the bubbles."""
        X = np.zeros(self.Nd)
        ux = u(self.x)
        for j in range(1, self.N):
            X[self.idx_hat(j)] = ux[j]
        for e in range(self.N):
            P = int(self.Ps[e])
            if P < 2:
                continue
            xq, _ = gauss_legendre(P + 4)
            Psi = psi_table(P, xq).T
            t = self.x[e] + 0.5 * (1.0 + xq) * self.h[e]
            lin = ux[e] * (1.0 - xq) / 2.0 + ux[e + 1] * (1.0 + xq) / 2.0
            coef, *_ = np.linalg.lstsq(Psi, u(t) - lin, rcond=None)
            X[self.boff[e]:self.boff[e + 1]] = coef
        return X

    def embed(self, Pmax: int) -> np.ndarray:
        """Index of each unknown of this space among the unknowns of the one-degree space of
        degree Pmax >= max P_i on the same mesh (the basis functions are shared)."""
        assert Pmax >= self.Ps.max()
        out = np.zeros(self.Nd, dtype=np.int64)
        for e in range(self.N):
            for p in range(1, int(self.Ps[e])):
                out[self.idx_bubble(e, p)] = e * (Pmax - 1) + p - 1
        for j in range(1, self.N):
            out[self.idx_hat(j)] = self.N * (Pmax - 1) + j - 1
        return out
