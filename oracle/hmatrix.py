"""H-matrix approximation, H-LU and H-solves, plain FP64 (oracle). TEST INFRASTRUCTURE ONLY.

Section 3 (H-matrix representation) and Section 4.1 (H-LU):
  * degenerate kernel by the truncated Taylor series of (t-s)^{1-alpha}
    (eq. (eqdegen), Lemma with eq. (eqn:Lexpan)); expansion in s about the
    centre s0 of the column cluster, or in t about t0, whichever cluster has
    the smaller radius (Remark after the Lemma);
  * admissibility max(diam) <= lambda dist (eq. (admis)) applied to the union
    of basis supports of each index cluster (Section 3.2);
  * low-rank blocks Q W^T with Q = gamma0 int h_nu phi', W = int g_nu phi'
    (the B~, C~, E~, F~ formulas of Section 3.2), dense blocks holding the exact
    entries of A (text after eq. (approxmat));
  * H-LU  A~ ~= L_H U_H, L_H unit lower, with truncation to a tolerance
    (Section 4.1, the H-LU of Borm, Grasedyck and Hackbusch, Section 5.2.3),
    and the forward/backward H-substitutions.

Readings of points the paper leaves open (each one is listed with the oracle's
documentation):
  * H approximates S = theta S_l + (1-theta) S_l^T, and A~ = rho M + H. For an
    admissible pair with the row cluster right of the column cluster the block
    is theta Q W^T; the mirrored block is (1-theta) W Q^T; S_l vanishes on the
    upper admissible blocks, so both are exact uses of the expansion.
  * Unknowns are reordered element by element (bubbles of element e, then the
    hat at its right node) so each cluster of elements owns a contiguous range.
  * Cluster tree: bisection of element ranges to a common depth
    ceil(log2(N / leaf)); block tree over pairs of same-level clusters;
    admissible -> low rank, leaf pair -> dense, otherwise 2 x 2 children.
  * Truncation after every low-rank sum: QR of both factors, SVD of the small
    core, keep sigma_k > tol * sigma_1, at most `kmax` terms.
  * No pivoting (coercivity, Theorem 1, makes the leading blocks of A nonsingular).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla

from .quadrature import gauss_legendre_on
from .sem import SEM, legendre_table


# --------------------------------------------------------------------------
# Ordering and trees
# --------------------------------------------------------------------------

def h_order(sem: SEM) -> np.ndarray:
    """h2p[k] = paper index of the k-th unknown in element-interleaved order."""
    N, P = sem.N, sem.P
    out = []
    for e in range(N):
        for p in range(1, P):
            out.append(sem.idx_bubble(e, p))
        if e < N - 1:
            out.append(sem.idx_hat(e + 1))
    return np.array(out, dtype=np.int64)


@dataclass
class Cluster:
    e0: int
    e1: int          # elements [e0, e1)
    d0: int
    d1: int          # unknowns [d0, d1) in element-interleaved order
    lo: float
    hi: float        # union of the supports of its basis functions
    level: int
    children: List["Cluster"] = field(default_factory=list)

    @property
    def is_leaf(self):
        return not self.children


def cluster_tree(sem: SEM, leaf_elems: int) -> Cluster:
    N, P, x = sem.N, sem.P, sem.x
    depth = 0 if N <= leaf_elems else math.ceil(math.log2(N / leaf_elems))

    def make(e0, e1, level):
        d1 = min(e1 * P, N * P - 1)
        c = Cluster(e0, e1, e0 * P, d1, x[e0], x[min(e1 + 1, N)], level)
        if level < depth:
            mid = e0 + (e1 - e0) // 2
            c.children = [make(e0, mid, level + 1), make(mid, e1, level + 1)]
        return c
    return make(0, N, 0)


def admissible(tau: Cluster, sigma: Cluster, lam: float) -> bool:
    dist = max(0.0, sigma.lo - tau.hi, tau.lo - sigma.hi)
    diam = max(tau.hi - tau.lo, sigma.hi - sigma.lo)
    return dist > 0.0 and diam <= lam * dist


@dataclass
class Block:
    kind: str                    # 'D' dense, 'R' low rank, 'H' hierarchical
    tau: Cluster
    sigma: Cluster
    D: Optional[np.ndarray] = None
    U: Optional[np.ndarray] = None
    V: Optional[np.ndarray] = None
    ch: Optional[list] = None

    @property
    def shape(self):
        return (self.tau.d1 - self.tau.d0, self.sigma.d1 - self.sigma.d0)

    @property
    def rank(self):
        return 0 if self.U is None else self.U.shape[1]


def block_tree(tau: Cluster, sigma: Cluster, lam: float) -> Block:
    if admissible(tau, sigma, lam):
        return Block("R", tau, sigma)
    if tau.is_leaf or sigma.is_leaf:
        return Block("D", tau, sigma)
    ch = [[block_tree(t, s, lam) for s in sigma.children] for t in tau.children]
    return Block("H", tau, sigma, ch=ch)


def leaves(b: Block):
    if b.kind == "H":
        for row in b.ch:
            for c in row:
                yield from leaves(c)
    else:
        yield b


# --------------------------------------------------------------------------
# Low-rank factors from the Taylor expansion
# --------------------------------------------------------------------------

def taylor_coefficients(alpha: float, R: int) -> np.ndarray:
    """c_nu = prod_{l=1}^{nu} (alpha + l - 2) / nu!  (Lemma, h_nu of eq. (eqn:Lexpan))."""
    c = np.ones(R)
    for nu in range(1, R):
        c[nu] = c[nu - 1] * (alpha + nu - 2.0) / nu
    return c


def _cluster_factor(sem: SEM, cl: Cluster, h2p: np.ndarray, F, R: int) -> np.ndarray:
    """Matrix [int F_nu(x) phi_i'(x) dx]_{i in cl, nu < R}, rows in cluster order."""
    P = sem.P
    D = sem.derivative_map().tocsc()
    e_last = min(cl.e1, sem.N - 1)
    out = np.zeros((cl.d1 - cl.d0, R))
    cols = h2p[cl.d0:cl.d1]
    Dc = D[:, cols]
    for e in range(cl.e0, e_last + 1):
        xq, wq = gauss_legendre_on(P + 20, sem.x[e], sem.x[e + 1])
        Lq = legendre_table(P, 2.0 * (xq - sem.x[e]) / sem.h[e] - 1.0)     # (P, nq)
        mom = (Lq * wq) @ F(xq).T                                           # (P, R)
        out += Dc[e * P:(e + 1) * P, :].toarray().T @ mom
    return out


def lowrank_factors(sem: SEM, T: Cluster, S: Cluster, h2p, R: int):
    """(Qt, Ws) with S_l(T, S) ~= Qt Ws^T, T right of S (t > s)."""
    al, g0 = sem.alpha, sem.gamma0
    c = taylor_coefficients(al, R)
    nu = np.arange(R)[:, None]
    rT = 0.5 * (T.hi - T.lo)
    rS = 0.5 * (S.hi - S.lo)
    if rS <= rT:
        s0 = 0.5 * (S.lo + S.hi)
        Fh = lambda t: g0 * (c * rS ** np.arange(R))[:, None] * (t[None, :] - s0) ** (1.0 - al - nu)
        Fg = lambda s: ((s[None, :] - s0) / rS) ** nu
        return _cluster_factor(sem, T, h2p, Fh, R), _cluster_factor(sem, S, h2p, Fg, R)
    t0 = 0.5 * (T.lo + T.hi)
    sgn = (-1.0) ** np.arange(R)
    Fg = lambda t: ((t[None, :] - t0) / rT) ** nu
    Fh = lambda s: g0 * (sgn * c * rT ** np.arange(R))[:, None] * (t0 - s[None, :]) ** (1.0 - al - nu)
    return _cluster_factor(sem, T, h2p, Fg, R), _cluster_factor(sem, S, h2p, Fh, R)


class HMatrix:
    """A~ = rho M + H in element-interleaved order (eq. (approxsys))."""

    def __init__(self, sem: SEM, R: int, lam: float = 1.0, leaf_elems: int = 8, A: np.ndarray = None):
        """A (optional): the dense system matrix in paper order, to take the dense blocks from."""
        self.sem = sem
        self.R = R
        self.lam = lam
        self.h2p = h_order(sem)
        self.root_cluster = cluster_tree(sem, leaf_elems)
        self.root = block_tree(self.root_cluster, self.root_cluster, lam)
        th = sem.theta
        for b in leaves(self.root):
            rows = self.h2p[b.tau.d0:b.tau.d1]
            cols = self.h2p[b.sigma.d0:b.sigma.d1]
            if b.kind == "D":
                b.D = sem.block(rows, cols) if A is None else A[np.ix_(rows, cols)].copy()
            elif b.tau.lo >= b.sigma.hi:           # lower: theta * Q W^T
                Qt, Ws = lowrank_factors(sem, b.tau, b.sigma, self.h2p, R)
                b.U, b.V = (th * Qt, Ws) if th != 0.0 else (Qt[:, :0], Ws[:, :0])
            else:                                   # upper: (1-theta) W Q^T
                Qt, Ws = lowrank_factors(sem, b.sigma, b.tau, self.h2p, R)
                b.U, b.V = ((1.0 - th) * Ws, Qt) if th != 1.0 else (Ws[:, :0], Qt[:, :0])

    def counts(self):
        nd = sum(1 for b in leaves(self.root) if b.kind == "D")
        nr = sum(1 for b in leaves(self.root) if b.kind == "R")
        return nd, nr


def to_dense(b: Block) -> np.ndarray:
    if b.kind == "D":
        return b.D.copy()
    if b.kind == "R":
        return b.U @ b.V.T
    return np.block([[to_dense(c) for c in row] for row in b.ch])


def copy_block(b: Block) -> Block:
    nb = Block(b.kind, b.tau, b.sigma)
    if b.kind == "D":
        nb.D = b.D.copy()
    elif b.kind == "R":
        nb.U, nb.V = b.U.copy(), b.V.copy()
    else:
        nb.ch = [[copy_block(c) for c in row] for row in b.ch]
    return nb


# --------------------------------------------------------------------------
# H-arithmetic
# --------------------------------------------------------------------------

class HLUBreakdown(RuntimeError):
    pass


class HArith:
    """Recursive H-LU of Section 4.1 with truncation tolerance `tol` and rank cap `kmax`."""

    def __init__(self, tol: float, kmax: int, pivot_floor: float = 0.0):
        self.tol = tol
        self.kmax = kmax
        self.pivot_floor = pivot_floor
        # floating-point operations of the factorisation, counted per primitive at its actual
        # dimensions and ranks (the algorithmic work of the H-LU, not a model of it)
        self.flops = 0.0

    # -- truncation (reading of the "prescribed tolerance" of Section 4.1) --
    def truncate(self, U: np.ndarray, V: np.ndarray):
        if U.shape[1] == 0:
            return U, V
        Qu, Ru = np.linalg.qr(U)
        Qv, Rv = np.linalg.qr(V)
        a, s, bt = np.linalg.svd(Ru @ Rv.T)
        if s.size == 0 or s[0] == 0.0:   # an empty block (no rows or no columns) or a zero sum
            k = 0
        else:
            k = int(np.count_nonzero(s > self.tol * s[0]))
        k = min(k, self.kmax)
        m, n, kk = U.shape[0], V.shape[0], U.shape[1]
        # Householder QR with the thin Q formed (2 x (2 m k^2 - 2 k^3 / 3)), the core product,
        # an SVD with both factors (22 k^3), the truncated products
        self.flops += 4.0 * (m + n) * kk * kk - 8.0 * kk ** 3 / 3.0 + 2.0 * kk ** 3 + 22.0 * kk ** 3 + \
            2.0 * (m + n) * kk * k
        return Qu @ (a[:, :k] * s[:k]), Qv @ bt[:k].T

    # -- products of a block with a dense slab --
    def matmul(self, A: Block, X: np.ndarray) -> np.ndarray:
        if A.kind == "D":
            self.flops += 2.0 * A.D.shape[0] * A.D.shape[1] * X.shape[1]
            return A.D @ X
        if A.kind == "R":
            self.flops += 2.0 * (A.U.shape[0] + A.V.shape[0]) * A.U.shape[1] * X.shape[1]
            return A.U @ (A.V.T @ X)
        n0 = A.ch[0][0].shape[1]
        X0, X1 = X[:n0], X[n0:]
        return np.vstack([self.matmul(A.ch[0][0], X0) + self.matmul(A.ch[0][1], X1),
                          self.matmul(A.ch[1][0], X0) + self.matmul(A.ch[1][1], X1)])

    def matmul_T(self, A: Block, X: np.ndarray) -> np.ndarray:
        if A.kind == "D":
            self.flops += 2.0 * A.D.shape[0] * A.D.shape[1] * X.shape[1]
            return A.D.T @ X
        if A.kind == "R":
            self.flops += 2.0 * (A.U.shape[0] + A.V.shape[0]) * A.U.shape[1] * X.shape[1]
            return A.V @ (A.U.T @ X)
        m0 = A.ch[0][0].shape[0]
        X0, X1 = X[:m0], X[m0:]
        return np.vstack([self.matmul_T(A.ch[0][0], X0) + self.matmul_T(A.ch[1][0], X1),
                          self.matmul_T(A.ch[0][1], X0) + self.matmul_T(A.ch[1][1], X1)])

    # -- C <- C - X Y^T --
    def lr_sub(self, C: Block, X: np.ndarray, Y: np.ndarray):
        if C.kind == "D":
            self.flops += 2.0 * X.shape[0] * Y.shape[0] * X.shape[1]
            C.D -= X @ Y.T
        elif C.kind == "R":
            C.U, C.V = self.truncate(np.hstack([C.U, -X]), np.hstack([C.V, Y]))
        else:
            m0 = C.ch[0][0].shape[0]
            n0 = C.ch[0][0].shape[1]
            for i, Xi in enumerate((X[:m0], X[m0:])):
                for j, Yj in enumerate((Y[:n0], Y[n0:])):
                    self.lr_sub(C.ch[i][j], Xi, Yj)

    # -- C <- C - A B --
    def gemm_sub(self, C: Block, A: Block, B: Block):
        if A.kind == "R":
            if A.rank:
                self.lr_sub(C, A.U, self.matmul_T(B, A.V))
        elif B.kind == "R":
            if B.rank:
                self.lr_sub(C, self.matmul(A, B.U), B.V)
        elif A.kind == "D" and B.kind == "D":
            if C.kind == "D":
                self.flops += 2.0 * A.D.shape[0] * B.D.shape[1] * A.D.shape[1]
                C.D -= A.D @ B.D
            elif C.kind == "R":
                self.lr_sub(C, A.D, B.D.T)
            else:
                raise NotImplementedError("dense product into a hierarchical block")
        elif A.kind == "H" and B.kind == "H" and C.kind == "H":
            for i in range(2):
                for j in range(2):
                    for l in range(2):
                        self.gemm_sub(C.ch[i][j], A.ch[i][l], B.ch[l][j])
        else:
            raise NotImplementedError(f"gemm_sub {C.kind} -= {A.kind} {B.kind}")

    # -- triangular solves with factored diagonal blocks --
    def solve_L(self, L: Block, X: np.ndarray):
        """X <- L^{-1} X (unit lower), in place."""
        if L.kind == "D":
            self.flops += float(L.D.shape[0]) ** 2 * X.shape[1]
            X[:] = sla.solve_triangular(L.D, X, lower=True, unit_diagonal=True)
            return
        n0 = L.ch[0][0].shape[0]
        self.solve_L(L.ch[0][0], X[:n0])
        X[n0:] -= self.matmul(L.ch[1][0], X[:n0])
        self.solve_L(L.ch[1][1], X[n0:])

    def solve_U(self, U: Block, X: np.ndarray):
        """X <- U^{-1} X (upper), in place."""
        if U.kind == "D":
            self.flops += float(U.D.shape[0]) ** 2 * X.shape[1]
            X[:] = sla.solve_triangular(U.D, X, lower=False)
            return
        n0 = U.ch[0][0].shape[0]
        self.solve_U(U.ch[1][1], X[n0:])
        X[:n0] -= self.matmul(U.ch[0][1], X[n0:])
        self.solve_U(U.ch[0][0], X[:n0])

    def solve_UT(self, U: Block, X: np.ndarray):
        """X <- U^{-T} X, in place."""
        if U.kind == "D":
            self.flops += float(U.D.shape[0]) ** 2 * X.shape[1]
            X[:] = sla.solve_triangular(U.D, X, lower=False, trans="T")
            return
        n0 = U.ch[0][0].shape[0]
        self.solve_UT(U.ch[0][0], X[:n0])
        X[n0:] -= self.matmul_T(U.ch[0][1], X[:n0])
        self.solve_UT(U.ch[1][1], X[n0:])

    def trsm_L(self, L: Block, B: Block):
        """B <- L^{-1} B."""
        if B.kind == "R":
            if B.rank:
                self.solve_L(L, B.U)
        elif B.kind == "D":
            self.solve_L(L, B.D)
        else:
            self.trsm_L(L.ch[0][0], B.ch[0][0])
            self.trsm_L(L.ch[0][0], B.ch[0][1])
            self.gemm_sub(B.ch[1][0], L.ch[1][0], B.ch[0][0])
            self.gemm_sub(B.ch[1][1], L.ch[1][0], B.ch[0][1])
            self.trsm_L(L.ch[1][1], B.ch[1][0])
            self.trsm_L(L.ch[1][1], B.ch[1][1])

    def trsm_U(self, U: Block, B: Block):
        """B <- B U^{-1}."""
        if B.kind == "R":
            if B.rank:
                self.solve_UT(U, B.V)
        elif B.kind == "D":
            Bt = B.D.T.copy()
            self.solve_UT(U, Bt)
            B.D[:] = Bt.T
        else:
            self.trsm_U(U.ch[0][0], B.ch[0][0])
            self.trsm_U(U.ch[0][0], B.ch[1][0])
            self.gemm_sub(B.ch[0][1], B.ch[0][0], U.ch[0][1])
            self.gemm_sub(B.ch[1][1], B.ch[1][0], U.ch[0][1])
            self.trsm_U(U.ch[1][1], B.ch[0][1])
            self.trsm_U(U.ch[1][1], B.ch[1][1])

    def getrf(self, A: np.ndarray):
        """Dense LU without pivoting, in place (unit L below, U on and above the diagonal)."""
        n = A.shape[0]
        self.flops += 2.0 * n ** 3 / 3.0
        scale = np.max(np.abs(A)) if A.size else 0.0
        for k in range(n):
            if abs(A[k, k]) <= self.pivot_floor * scale or A[k, k] == 0.0:
                raise HLUBreakdown(f"pivot {A[k, k]:.3e} at {k}")
            A[k + 1:, k] /= A[k, k]
            A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])

    def hlu(self, A: Block):
        """A~ = L_H U_H in place (Section 4.1)."""
        if A.kind == "D":
            self.getrf(A.D)
            return
        self.hlu(A.ch[0][0])
        self.trsm_L(A.ch[0][0], A.ch[0][1])
        self.trsm_U(A.ch[0][0], A.ch[1][0])
        self.gemm_sub(A.ch[1][1], A.ch[1][0], A.ch[0][1])
        self.hlu(A.ch[1][1])


class HLU:
    """Factors L_H U_H of A~ and the forward/backward H-substitutions (Section 4.1)."""

    def __init__(self, H: HMatrix, tol: float = 1e-3, kmax: Optional[int] = None,
                 pivot_floor: float = 1e-14):
        self.H = H
        self.ar = HArith(tol, H.R if kmax is None else kmax, pivot_floor)
        self.root = copy_block(H.root)
        self.ar.hlu(self.root)
        self.flops = self.ar.flops   # floating-point operations of the factorisation

    def solve(self, G: np.ndarray) -> np.ndarray:
        """X ~= A~^{-1} G, G and X in paper order (1-D or Nd x k)."""
        h2p = self.H.h2p
        Y = np.array(G, dtype=np.float64)[h2p].copy()
        squeeze = Y.ndim == 1
        if squeeze:
            Y = Y[:, None]
        self.ar.solve_L(self.root, Y)
        self.ar.solve_U(self.root, Y)
        X = np.empty_like(Y)
        X[h2p] = Y
        return X[:, 0] if squeeze else X

    def dense_factors(self):
        """(L_H, U_H) as dense matrices in element-interleaved order."""
        F = to_dense(self.root)
        return np.tril(F, -1) + np.eye(F.shape[0]), np.triu(F)

    def ranks(self):
        return [b.rank for b in leaves(self.root) if b.kind == "R"]
