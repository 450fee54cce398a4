"""Spectral element discretisation, plain FP64 (oracle). TEST INFRASTRUCTURE ONLY.

Follows Section 2.2 of the paper:
  * nodal hat functions varphi_j (j = 1..N-1) and modal bubbles
    phi_i^p = psi_p(xi_i(x)), psi_p = L_{p-1} - L_{p+1}, p = 1..P-1 (eq. (RefBasis),
    eq. (LocalBasis));
  * unknown order X = [bubbles of element 1; ...; bubbles of element N; hats]
    (the vector X below eq. (lsys));
  * A = rho M + S, S = theta S_l + (1 - theta) S_l^T (eq. (lsys)).

The stiffness entries are written through the kernel form of the weak form
(Section 2.1, eq. (WeakForm)): for u, v vanishing at a and b,
    (aD^{alpha/2} u, xD_b^{alpha/2} v) = gamma0 int int_{s<t} v'(t) (t-s)^{1-alpha} u'(s) ds dt,
gamma0 = 1/Gamma(2-alpha), which is the entry formula of Section 3.2
(the B~ formula with the kernel in place of its expansion). Every basis derivative is a
Legendre series on each element, because psi_p' = -(2p+1) L_p, so
    S_l = D^T K D,
    K^{ef}_{mn} = gamma0 int_{I_e} int_{I_f} (t-s)_+^{1-alpha} L_m(xi_e(t)) L_n(xi_f(s)) ds dt,
with D the (sparse) map from unknowns to per-element Legendre derivative
coefficients. The paper does not give the singular quadrature (it cites
Mao & Shen, Lemma 4); the rules below are the reading documented with the oracle:
  same element  -- Duffy map, tensor Gauss-Jacobi: exact for polynomials;
  adjacent      -- Duffy split of the square, Gauss-Jacobi radially,
                   graded Gauss-Legendre panels on the smooth angular factor;
  separated     -- tensor Gauss-Legendre on panels graded toward the gap.
Pins: tests/test_oracle_sem.py (brute-force adaptive quadrature, the
fractional-integral closed form of Legendre polynomials, manufactured
solutions, transpose/symmetry/positivity identities, the alpha -> 1 limit and
the corrected Appendix A generators).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .quadrature import (gauss_jacobi, gauss_legendre, gauss_legendre_on, graded_panels,
                         jacobi_unit_weight)


def legendre_table(n: int, x: np.ndarray) -> np.ndarray:
    """L_0..L_{n-1} at x by the three-term recurrence of Section 2.2. Shape (n, len(x))."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((max(n, 2),) + x.shape)
    out[0] = 1.0
    out[1] = x
    for p in range(1, n - 1):
        out[p + 1] = ((2 * p + 1) * x * out[p] - p * out[p - 1]) / (p + 1)
    return out[:n]


def psi_table(P: int, x: np.ndarray) -> np.ndarray:
    """psi_p = L_{p-1} - L_{p+1}, p = 1..P-1 (eq. (RefBasis)). Shape (P-1, len(x))."""
    L = legendre_table(P + 1, x)
    return np.array([L[p - 1] - L[p + 1] for p in range(1, P)]).reshape((P - 1,) + np.shape(x))


class SEM:
    """The SEM system of eq. (lsys) on a mesh x_0 < ... < x_N with uniform degree P."""

    def __init__(self, nodes, P: int, alpha: float, theta: float, rho: float):
        self.x = np.asarray(nodes, dtype=np.float64)
        self.N = len(self.x) - 1
        self.h = np.diff(self.x)
        self.P = int(P)
        self.alpha = float(alpha)
        self.theta = float(theta)
        self.rho = float(rho)
        self.gamma0 = 1.0 / math.gamma(2.0 - self.alpha)
        self.Nd = self.N * self.P - 1
        assert self.P >= 2 and self.N >= 1 and np.all(self.h > 0)
        assert 1.0 < self.alpha < 2.0 and 0.0 <= self.theta <= 1.0
        self._K = None

    # ---- unknown order (paper order: bubbles element-major, then hats) ----
    def idx_bubble(self, e: int, p: int) -> int:
        """Element e (0-based), mode p (1..P-1)."""
        return e * (self.P - 1) + (p - 1)

    def idx_hat(self, j: int) -> int:
        """Interior node j (1..N-1)."""
        return self.N * (self.P - 1) + (j - 1)

    # ---- D: unknowns -> per-element Legendre coefficients of the derivative ----
    def derivative_map(self, with_boundary: bool = False) -> sp.csr_matrix:
        """Sparse (N*P) x Nd map (x (Nd+2) with the boundary hats varphi_0, varphi_N appended).

        On element e, (phi_e^p)' = -(2p+1) (2/h_e) L_p(xi_e) and a hat has slope
        +-1/h_e, a multiple of L_0 (Section 2.2).
        """
        key = "_D1" if with_boundary else "_D0"
        if getattr(self, key, None) is not None:
            return getattr(self, key)
        N, P, h = self.N, self.P, self.h
        rows, cols, vals = [], [], []
        for e in range(N):
            for p in range(1, P):
                rows.append(e * P + p); cols.append(self.idx_bubble(e, p))
                vals.append(-(2 * p + 1) * 2.0 / h[e])
        for j in range(1, N):
            rows.append((j - 1) * P); cols.append(self.idx_hat(j)); vals.append(1.0 / h[j - 1])
            rows.append(j * P); cols.append(self.idx_hat(j)); vals.append(-1.0 / h[j])
        ncol = self.Nd
        if with_boundary:
            rows.append(0); cols.append(self.Nd); vals.append(-1.0 / h[0])
            rows.append((N - 1) * P); cols.append(self.Nd + 1); vals.append(1.0 / h[N - 1])
            ncol += 2
        D = sp.csr_matrix((vals, (rows, cols)), shape=(N * P, ncol))
        setattr(self, key, D)
        return D

    # ---- element-pair moments K^{ef} ----
    def pair_moment(self, e: int, f: int) -> np.ndarray:
        """K^{ef} (P x P), f <= e, rows m <-> L_m on the test element e."""
        assert f <= e
        if e == f:
            return self.moment_same(self.h[e])
        if f == e - 1:
            return self.moment_adjacent(self.h[e], self.h[f])
        gap = self.x[e] - self.x[f + 1]
        return self.moment_separated(self.h[e], self.h[f], gap)

    def moment_same(self, he: float) -> np.ndarray:
        """Same element: t = s + (1+xi) w, Duffy; exact tensor Gauss-Jacobi."""
        P, al = self.P, self.alpha
        xo, wo = gauss_jacobi(P + 2, 0.0, 2.0 - al)           # (1+xi)^{2-alpha}
        wi_nodes, wi = jacobi_unit_weight(P + 2, 1.0 - al)    # w^{1-alpha} on [0,1]
        Lo = legendre_table(P, xo)                              # (P, no)
        eta = xo[:, None] - (1.0 + xo[:, None]) * wi_nodes[None, :]   # (no, ni)
        Li = legendre_table(P, eta)                             # (P, no, ni)
        inner = np.einsum("nij,j->ni", Li, wi)                  # (P, no)
        J = np.einsum("mi,i,ni->mn", Lo, wo, inner)
        return self.gamma0 * (0.5 * he) ** (3.0 - al) * J

    def moment_adjacent(self, he: float, hf: float) -> np.ndarray:
        """f = e-1. u = t - x_shared in [0,he], v = x_shared - s in [0,hf], kernel (u+v)^{1-alpha}.

        Square split along its diagonal; each triangle mapped to a square (Duffy).
        """
        P, al = self.P, self.alpha
        r, wr = jacobi_unit_weight(P + 2, 2.0 - al)            # radial weight r^{2-alpha}
        nq = P + 24
        out = np.zeros((P, P))
        # triangle b <= a: b = a w; factor (he + hf w)^{1-alpha}
        for lo, hi in graded_panels(1.0, he / hf):
            w, ww = gauss_legendre_on(nq, lo, hi)
            La = legendre_table(P, 2.0 * r - 1.0)                               # (P, nr)
            Lb = legendre_table(P, 1.0 - 2.0 * r[:, None] * w[None, :])         # (P, nr, nw)
            kern = (he + hf * w) ** (1.0 - al)
            out += np.einsum("mi,i,nij,j->mn", La, wr, Lb, ww * kern)
        # triangle a <= b: a = b w; factor (he w + hf)^{1-alpha}
        for lo, hi in graded_panels(1.0, hf / he):
            w, ww = gauss_legendre_on(nq, lo, hi)
            Lb = legendre_table(P, 1.0 - 2.0 * r)                               # (P, nr)
            La = legendre_table(P, 2.0 * r[:, None] * w[None, :] - 1.0)         # (P, nr, nw)
            kern = (he * w + hf) ** (1.0 - al)
            out += np.einsum("mij,i,ni,j->mn", La, wr, Lb, ww * kern)
        return self.gamma0 * he * hf * out

    def moment_separated(self, he: float, hf: float, gap: float) -> np.ndarray:
        """f <= e-2: t - s >= gap > 0; tensor Gauss-Legendre on panels graded toward the gap."""
        P, al = self.P, self.alpha
        nq = P + 20
        out = np.zeros((P, P))
        for tlo, thi in graded_panels(he, gap):        # u = t - x_e
            u, wu = gauss_legendre_on(nq, tlo, thi)
            Lt = legendre_table(P, 2.0 * u / he - 1.0)
            for slo, shi in graded_panels(hf, gap):    # v = x_{f+1} - s
                v, wv = gauss_legendre_on(nq, slo, shi)
                Ls = legendre_table(P, 1.0 - 2.0 * v / hf)
                kern = (gap + u[:, None] + v[None, :]) ** (1.0 - al)
                out += np.einsum("mi,i,ij,j,nj->mn", Lt, wu, kern, wv, Ls)
        return self.gamma0 * out

    def element_operator(self) -> np.ndarray:
        """Dense block-lower K (N*P x N*P) with blocks K^{ef}, f <= e."""
        if self._K is None:
            N, P = self.N, self.P
            K = np.zeros((N * P, N * P))
            for e in range(N):
                for f in range(e + 1):
                    K[e * P:(e + 1) * P, f * P:(f + 1) * P] = self.pair_moment(e, f)
            self._K = K
        return self._K

    # ---- matrices of eq. (lsys) ----
    def stiffness_lower(self, with_boundary: bool = False) -> np.ndarray:
        """S_l = D^T K D (Nd x Nd), or its (Nd+2)-column extension with boundary hats."""
        D = self.derivative_map(with_boundary)
        K = self.element_operator()
        Dd = D.toarray()
        return Dd.T @ K @ Dd

    def local_mass(self) -> np.ndarray:
        """int_{-1}^{1} of products of [phi_L, phi_R, psi_1..psi_{P-1}] (reference element)."""
        P = self.P
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
        return [hat(e), hat(e + 1)] + [self.idx_bubble(e, p) for p in range(1, self.P)]

    def mass_sparse(self, with_boundary: bool = False) -> sp.csr_matrix:
        n = self.Nd + (2 if with_boundary else 0)
        Ml = self.local_mass()
        rows, cols, vals = [], [], []
        for e in range(self.N):
            d = self.local_dofs(e, with_boundary)
            for a_, ia in enumerate(d):
                if ia < 0:
                    continue
                for b_, ib in enumerate(d):
                    if ib >= 0 and Ml[a_, b_] != 0.0:
                        rows.append(ia); cols.append(ib); vals.append(0.5 * self.h[e] * Ml[a_, b_])
        return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))

    def mass(self, with_boundary: bool = False) -> np.ndarray:
        return self.mass_sparse(with_boundary).toarray()

    def block(self, rows, cols) -> np.ndarray:
        """A[rows, cols] (paper order) from the element-pair moments it needs only."""
        rows = np.asarray(rows); cols = np.asarray(cols)
        D = self.derivative_map()
        Dr = D[:, rows].tocsc(); Dc = D[:, cols].tocsc()
        er = np.unique(Dr.nonzero()[0] // self.P)
        ec = np.unique(Dc.nonzero()[0] // self.P)
        P = self.P
        def sl(ei, ej, Da, Db):
            # S_l(a-set, b-set) = Da^T K[ei x ej] Db over pairs with f <= e
            Kb = np.zeros((len(ei) * P, len(ej) * P))
            for a_, e in enumerate(ei):
                for b_, f in enumerate(ej):
                    if f <= e:
                        Kb[a_ * P:(a_ + 1) * P, b_ * P:(b_ + 1) * P] = self._moment_cached(e, f)
            ri = (ei[:, None] * P + np.arange(P)[None, :]).ravel()
            rj = (ej[:, None] * P + np.arange(P)[None, :]).ravel()
            return Da[ri, :].toarray().T @ Kb @ Db[rj, :].toarray()
        S = self.theta * sl(er, ec, Dr, Dc) + (1.0 - self.theta) * sl(ec, er, Dc, Dr).T
        M = self.mass_sparse()[rows, :][:, cols].toarray()
        return self.rho * M + S

    def _moment_cached(self, e, f):
        if not hasattr(self, "_mcache"):
            self._mcache = {}
        key = (e, f)
        if key not in self._mcache:
            self._mcache[key] = self.pair_moment(e, f)
        return self._mcache[key]

    def system_matrix(self, with_boundary: bool = False) -> np.ndarray:
        """A = rho M + theta S_l + (1-theta) S_l^T (rows: test functions, Nd of them)."""
        if not with_boundary:
            Sl = self.stiffness_lower()
            return self.rho * self.mass() + self.theta * Sl + (1.0 - self.theta) * Sl.T
        D = self.derivative_map(True).toarray()
        K = self.element_operator()
        Dr = D[:, :self.Nd]
        S = Dr.T @ (self.theta * K + (1.0 - self.theta) * K.T) @ D
        return self.rho * self.mass(True)[:self.Nd, :] + S

    # ---- load vector (below eq. (lsys)) with lifting of c1, c2 ----
    def load_vector(self, f_terms, c1: float = 0.0, c2: float = 0.0) -> np.ndarray:
        """G_i = (f, varphi_i or phi_e^p) for f = sum_j c_j d_j(x)^{p_j} (signed powers).

        f_terms is a PowerSum (coef, expo, side). On the element touching the
        singular end the rule is Gauss-Jacobi with weight (1+xi)^{p+1}
        (test functions vanish there), elsewhere graded Gauss-Legendre.
        Then G -= c1 a(varphi_0, .) + c2 a(varphi_N, .)  (lifting).
        """
        N, P = self.N, self.P
        a, b = self.x[0], self.x[-1]
        G = np.zeros(self.Nd)
        for c, p, side in zip(f_terms.coef, f_terms.expo, f_terms.side):
            for e in range(N):
                dofs = self.local_dofs(e)
                he = self.h[e]
                touching = (side == 0 and e == 0) or (side == 1 and e == N - 1)
                if touching:
                    if side == 0:
                        xq, wq = gauss_jacobi(P + 2, 0.0, p + 1.0)
                        fac = (1.0 + xq)
                    else:
                        xq, wq = gauss_jacobi(P + 2, p + 1.0, 0.0)
                        fac = (1.0 - xq)
                    Bq = np.vstack([(1.0 - xq) / 2.0, (1.0 + xq) / 2.0, psi_table(P, xq)]) / fac
                    vals = c * (0.5 * he) ** (p + 1.0) * (Bq @ wq)
                else:
                    gap = (self.x[e] - a) if side == 0 else (b - self.x[e + 1])
                    vals = np.zeros(P + 1)
                    for lo, hi in graded_panels(he, gap):
                        uq, wq = gauss_legendre_on(P + 24, lo, hi)
                        if side == 0:
                            xi = 2.0 * uq / he - 1.0
                            d = gap + uq
                        else:
                            xi = 1.0 - 2.0 * uq / he
                            d = gap + uq
                        Bq = np.vstack([(1.0 - xi) / 2.0, (1.0 + xi) / 2.0, psi_table(P, xi)])
                        vals += Bq @ (wq * c * d ** p)
                for k, i in enumerate(dofs):
                    if i >= 0:
                        G[i] += vals[k]
        if c1 != 0.0 or c2 != 0.0:
            Ab = self.system_matrix(with_boundary=True)
            G -= c1 * Ab[:, self.Nd] + c2 * Ab[:, self.Nd + 1]
        return G

    # ---- coefficients of a function of S_N^P ----
    def interpolate_coefficients(self, u) -> np.ndarray:
        """X of a function u in S_N^P (exact when u is a polynomial of degree <= P per element).

        Hat values are nodal values; bubble coefficients come from the Legendre
        expansion of u - (hat interpolant) on each element, using
        (1 - xi^2) L_p'(xi)-type identities through a small least-squares fit at
        Gauss points (exact for members of the space).
        """
        N, P = self.N, self.P
        X = np.zeros(self.Nd)
        ux = u(self.x)
        for j in range(1, N):
            X[self.idx_hat(j)] = ux[j]
        xq, _ = gauss_legendre(P + 4)
        Psi = psi_table(P, xq).T                                 # (nq, P-1)
        for e in range(N):
            t = self.x[e] + 0.5 * (1.0 + xq) * self.h[e]
            lin = ux[e] * (1.0 - xq) / 2.0 + ux[e + 1] * (1.0 + xq) / 2.0
            coef, *_ = np.linalg.lstsq(Psi, u(t) - lin, rcond=None)
            for p in range(1, P):
                X[self.idx_bubble(e, p)] = coef[p - 1]
        return X

    def evaluate(self, X: np.ndarray, t: np.ndarray, c1: float = 0.0, c2: float = 0.0) -> np.ndarray:
        """u_N^P(t) for coefficients X (paper order) and boundary values c1, c2."""
        t = np.asarray(t, dtype=np.float64)
        e = np.clip(np.searchsorted(self.x, t, side="right") - 1, 0, self.N - 1)
        xi = 2.0 * (t - self.x[e]) / self.h[e] - 1.0
        hat = np.concatenate([[c1], X[self.N * (self.P - 1):], [c2]])
        val = hat[e] * (1.0 - xi) / 2.0 + hat[e + 1] * (1.0 + xi) / 2.0
        Ps = psi_table(self.P, xi)
        for p in range(1, self.P):
            val += X[e * (self.P - 1) + p - 1] * Ps[p - 1]
        return val
