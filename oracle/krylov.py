"""Dense LU and preconditioned Krylov solvers, plain FP64 (oracle). TEST INFRASTRUCTURE ONLY.

Section 4.2: the H-LU factors of A~ precondition the original system A X = G
(eq. (precondsys)); the paper uses BiCGSTAB with tolerance 1e-13 (Section 5).
The dense LU solve is the plain definition of X* = A^{-1} G (eq. (lsys)).

Readings: the preconditioner is applied on the right inside FGMRES(m)
(flexible, since a mixed-precision preconditioner is not exactly linear), and
convergence is judged on the true residual ||G - A X|| / ||G||. BiCGSTAB is
provided in both left-preconditioned form (the paper's eq. (precondsys), whose
iteration counts Tables 1-2 report) and right-preconditioned form.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def dense_solve(A: np.ndarray, G: np.ndarray):
    """(X*, kappa_1 estimate): LAPACK getrf/getrs with partial pivoting, gecon."""
    lu, piv = sla.lu_factor(A)
    X = sla.lu_solve((lu, piv), G)
    anorm = np.linalg.norm(A, 1)
    rcond = sla.lapack.dgecon(lu, anorm, norm="1")[0]
    return X, (1.0 / rcond if rcond > 0 else np.inf)


def fgmres(apply_A, G: np.ndarray, precond=None, restart: int = 30, tol: float = 1e-10,
           maxit: int = 1000, x0=None):
    """Right-preconditioned flexible GMRES(m) for one right-hand side.

    Returns (X, info) with info = dict(iters, relres, history, converged).
    """
    M = precond if precond is not None else (lambda v: v.copy())
    n = G.shape[0]
    gnorm = np.linalg.norm(G)
    X = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    hist = []
    if gnorm == 0.0:
        return np.zeros(n), dict(iters=0, relres=0.0, history=[0.0], converged=True)
    iters = 0
    r = G - apply_A(X)
    rel = np.linalg.norm(r) / gnorm
    hist.append(rel)
    while rel > tol and iters < maxit:
        beta = np.linalg.norm(r)
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        Hm = np.zeros((restart + 1, restart))
        cs = np.zeros(restart); sn = np.zeros(restart)
        g = np.zeros(restart + 1); g[0] = beta
        V[0] = r / beta
        j_end = 0
        for j in range(restart):
            Z[j] = M(V[j])
            w = apply_A(Z[j])
            for i in range(j + 1):                     # modified Gram-Schmidt
                Hm[i, j] = V[i] @ w
                w = w - Hm[i, j] * V[i]
            Hm[j + 1, j] = np.linalg.norm(w)
            if Hm[j + 1, j] > 0:
                V[j + 1] = w / Hm[j + 1, j]
            for i in range(j):                         # apply previous rotations
                t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                Hm[i + 1, j] = -sn[i] * Hm[i, j] + cs[i] * Hm[i + 1, j]
                Hm[i, j] = t
            den = np.hypot(Hm[j, j], Hm[j + 1, j])
            cs[j], sn[j] = Hm[j, j] / den, Hm[j + 1, j] / den
            Hm[j, j] = den; Hm[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]; g[j] = cs[j] * g[j]
            iters += 1
            j_end = j + 1
            hist.append(abs(g[j + 1]) / gnorm)
            if abs(g[j + 1]) / gnorm <= tol or iters >= maxit:
                break
        y = sla.solve_triangular(Hm[:j_end, :j_end], g[:j_end], lower=False)
        X = X + Z[:j_end].T @ y
        r = G - apply_A(X)
        rel = np.linalg.norm(r) / gnorm
        hist[-1] = rel
    return X, dict(iters=iters, relres=rel, history=hist, converged=rel <= tol)


def bicgstab(apply_A, G: np.ndarray, precond=None, tol: float = 1e-13, maxit: int = 500,
             side: str = "left"):
    """Preconditioned BiCGSTAB (van der Vorst).

    side='left' iterates on M^{-1} A X = M^{-1} G and tests the preconditioned
    residual (eq. (precondsys)); side='right' iterates on A M^{-1} y = G and
    tests the true residual. Returns (X, info) with iters = full BiCGSTAB steps
    and half_steps = matrix-vector products with A.
    """
    M = precond if precond is not None else (lambda v: v.copy())
    n = G.shape[0]
    X = np.zeros(n)
    if side == "left":
        op = lambda v: M(apply_A(v))
        b = M(G)
    else:
        op = lambda v: apply_A(M(v))
        b = G.copy()
    bnorm = np.linalg.norm(b)
    r = b.copy()
    rhat = r.copy()
    rho_old = alpha = omega = 1.0
    v = np.zeros(n); p = np.zeros(n)
    y = np.zeros(n)
    hist = [1.0]
    half = 0
    it = 0
    rel = 1.0
    while it < maxit:
        rho = rhat @ r
        if rho == 0.0:
            break
        beta = (rho / rho_old) * (alpha / omega) if it > 0 else 0.0
        p = r + beta * (p - omega * v) if it > 0 else r.copy()
        v = op(p); half += 1
        alpha = rho / (rhat @ v)
        s = r - alpha * v
        y = y + alpha * p
        if np.linalg.norm(s) / bnorm <= tol:
            r = s; it += 1
            rel = np.linalg.norm(r) / bnorm; hist.append(rel)
            break
        t = op(s); half += 1
        omega = (t @ s) / (t @ t)
        y = y + omega * s
        r = s - omega * t
        rho_old = rho
        it += 1
        rel = np.linalg.norm(r) / bnorm
        hist.append(rel)
        if rel <= tol:
            break
    X = y if side == "left" else M(y)
    true_rel = np.linalg.norm(G - apply_A(X)) / np.linalg.norm(G)
    return X, dict(iters=it, half_steps=half, relres=rel, true_relres=true_rel,
                   history=hist, converged=rel <= tol)
