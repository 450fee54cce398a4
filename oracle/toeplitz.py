"""Block-Toeplitz stiffness apply by FFT on uniform and geometric meshes (oracle).

TEST INFRASTRUCTURE ONLY. Section 4.3 and Appendix A: on a mesh with a
constant ratio r = h_{e+1}/h_e, the element-pair moments satisfy
    K^{ef} = (h_e/2)^{2-alpha} (h_f/2) Khat_{e-f},
because (t - s)/(h_e/2) depends on e - f only (eq. (eq420) with the reading
that fixes the ratio convention of its generator). The lower block-Toeplitz
product is a causal convolution and its transpose a correlation; both are
evaluated with a zero-padded FFT of length >= 2N (circulant embedding,
Section 4.3). Pinned by tests/test_oracle_toeplitz.py: equal to the dense
product.
"""
from __future__ import annotations

import numpy as np

from .sem import SEM


def mesh_ratio(sem: SEM, rtol: float = 1e-12):
    """r if h_{e+1}/h_e is constant (uniform: 1.0), else None."""
    h = sem.h
    if len(h) == 1:
        return 1.0
    q = h[1:] / h[:-1]
    r = q.mean()
    return float(r) if np.all(np.abs(q - r) <= rtol * max(1.0, r)) else None


def generators(sem: SEM, r: float) -> np.ndarray:
    """Khat_k, k = 0..N-1 (N x P x P), for ratio r, at h_e = 2."""
    N = sem.N
    out = np.zeros((N, sem.P, sem.P))
    out[0] = sem.moment_same(2.0)
    if N > 1:
        out[1] = sem.moment_adjacent(2.0, 2.0 / r) / (1.0 / r)
    for k in range(2, N):
        hf = 2.0 * r ** (-k)
        gap = 2.0 * sum(r ** (-j) for j in range(1, k))
        out[k] = sem.moment_separated(2.0, hf, gap) / (0.5 * hf)
    return out


def apply(sem: SEM, X: np.ndarray, Khat: np.ndarray = None) -> np.ndarray:
    """A X for X of shape (Nd,) or (Nd, k), by FFT."""
    r = mesh_ratio(sem)
    assert r is not None, "mesh is not uniform or geometric"
    if Khat is None:
        Khat = generators(sem, r)
    N, P = sem.N, sem.P
    X2 = X[:, None] if X.ndim == 1 else X
    D = sem.derivative_map()
    c = (D @ X2).reshape(N, P, -1)                          # element coefficients
    sig = (0.5 * sem.h) ** (2.0 - sem.alpha)
    omg = 0.5 * sem.h
    L = 1
    while L < 2 * N:
        L *= 2
    Kw = np.fft.rfft(Khat, n=L, axis=0)                      # (L/2+1, P, P)
    Zc = np.fft.rfft(omg[:, None, None] * c, n=L, axis=0)    # causal part input
    Zr = np.fft.rfft(sig[:, None, None] * c, n=L, axis=0)    # transposed part input
    Yc = np.fft.irfft(np.einsum("wmn,wnk->wmk", Kw, Zc), n=L, axis=0)[:N]
    Yr = np.fft.irfft(np.einsum("wnm,wnk->wmk", np.conj(Kw), Zr), n=L, axis=0)[:N]
    ye = sem.theta * sig[:, None, None] * Yc + (1.0 - sem.theta) * omg[:, None, None] * Yr
    Y = D.T @ ye.reshape(N * P, -1) + sem.rho * (sem.mass_sparse() @ X2)
    return Y[:, 0] if X.ndim == 1 else Y


def dense_matrix(sem: SEM, Khat: np.ndarray = None) -> np.ndarray:
    """A (Nd x Nd, paper order) from the generators: the block-Toeplitz K, then D^T K D + rho M."""
    r = mesh_ratio(sem)
    assert r is not None, "mesh is not uniform or geometric"
    if Khat is None:
        Khat = generators(sem, r)
    N, P = sem.N, sem.P
    sig = (0.5 * sem.h) ** (2.0 - sem.alpha)
    omg = 0.5 * sem.h
    K = np.zeros((N * P, N * P))
    for e in range(N):
        for f in range(e + 1):
            K[e * P:(e + 1) * P, f * P:(f + 1) * P] = sig[e] * omg[f] * Khat[e - f]
    D = sem.derivative_map()
    KD = np.asarray(D.T @ (sem.theta * K + (1.0 - sem.theta) * K.T))
    S = np.asarray((D.T @ KD.T).T)
    return S + sem.rho * sem.mass_sparse().toarray()
