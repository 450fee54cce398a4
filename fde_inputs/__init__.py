"""Seeded synthetic inputs for the fractional diffusion solver.

This module is shared by the tests, the benchmark and the CPU oracle. It holds
problem *data* only -- meshes, manufactured solutions and the right-hand sides
they imply -- and none of the discretisation, H-matrix or solver arithmetic.

Problem (Section 1, eq. (Model)): on (a, b), 1 < alpha < 2, 0 <= theta <= 1,

    -D^2 ( theta aI^{2-alpha} u + (1-theta) xI_b^{2-alpha} u ) + rho u = f,
    u(a) = c1, u(b) = c2.

A manufactured solution is a generalised polynomial
    u(x) = sum_k a_k (x-a)^{mu_k}   (left form, used by the theta part)
         = sum_k b_k (b-x)^{nu_k}   (right form, used by the 1-theta part).
The Riemann-Liouville integral of a power is a power,
    aI^beta (x-a)^mu = Gamma(mu+1)/Gamma(mu+1+beta) (x-a)^(mu+beta),
and its mirror image for xI_b, so f is again a sum of signed powers:
    f = -theta   sum a_k Gamma(mu_k+1)/Gamma(mu_k+1-alpha) (x-a)^(mu_k-alpha)
        -(1-theta) sum b_k Gamma(nu_k+1)/Gamma(nu_k+1-alpha) (b-x)^(nu_k-alpha)
        + rho u.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

SEED_BASE = 1808029370


def rng(config_index: int, stream: int = 0) -> np.random.Generator:
    """The seeded generator for workload `config_index` (PCG64)."""
    return np.random.Generator(np.random.PCG64([SEED_BASE + config_index, stream]))


# ----------------------------------------------------------------------------
# Meshes (Section 2.2, eq. (Partition); mesh families of Sections 4.3 and 5)
# ----------------------------------------------------------------------------

def uniform_mesh(N: int, a: float = 0.0, b: float = 1.0) -> np.ndarray:
    x = a + (b - a) * np.arange(N + 1, dtype=np.float64) / N
    x[0], x[-1] = a, b
    return x


def geometric_mesh(N: int, r: float, a: float = 0.0, b: float = 1.0) -> np.ndarray:
    """Constant ratio h_{i+1}/h_i = r (Section 4.3)."""
    if abs(r - 1.0) < 1e-15:
        return uniform_mesh(N, a, b)
    h = r ** np.arange(N, dtype=np.float64)
    h *= (b - a) / h.sum()
    x = np.concatenate([[a], a + np.cumsum(h)])
    x[-1] = b
    return x


def graded_mesh(N: int, power: float = 5.0, a: float = 0.0, b: float = 10.0) -> np.ndarray:
    """x_i = a + (b-a) (i/N)^power (Section 5, Example 1 mesh)."""
    x = a + (b - a) * (np.arange(N + 1, dtype=np.float64) / N) ** power
    x[0], x[-1] = a, b
    return x


def two_sided_graded_mesh(N: int, layers: int = 20, q: float = 0.5,
                          a: float = 0.0, b: float = 1.0) -> np.ndarray:
    """Geometric layers toward both ends, uniform interior.

    L = min(layers, N // 4) elements of sizes h_int q^L, ..., h_int q^1 next to
    each endpoint (smallest at the endpoint) and N - 2L elements of size h_int,
    normalised to (a, b).
    """
    L = min(layers, N // 4)
    n_int = N - 2 * L
    left = q ** np.arange(L, 0, -1, dtype=np.float64)          # q^L .. q^1
    h = np.concatenate([left, np.ones(n_int), left[::-1]])
    h *= (b - a) / h.sum()
    x = np.concatenate([[a], a + np.cumsum(h)])
    x[-1] = b
    return x


# ----------------------------------------------------------------------------
# Manufactured solutions and their right-hand sides
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class PowerSum:
    """sum_k coef_k * (side distance)^(expo_k); side 'a' -> (x-a), 'b' -> (b-x)."""
    coef: np.ndarray
    expo: np.ndarray
    side: np.ndarray  # 0 for (x-a), 1 for (b-x)

    def __call__(self, x, a: float, b: float, da=None, db=None) -> np.ndarray:
        """Value at x; da = x - a and db = b - x may be given exactly (near the ends)."""
        x = np.asarray(x, dtype=np.float64)
        da = (x - a) if da is None else np.asarray(da, dtype=np.float64)
        db = (b - x) if db is None else np.asarray(db, dtype=np.float64)
        out = np.zeros_like(x)
        for c, e, s in zip(self.coef, self.expo, self.side):
            d = da if s == 0 else db
            with np.errstate(divide="ignore", invalid="ignore"):
                t = np.where(d > 0, c * np.power(np.maximum(d, 0.0), e), 0.0 if e > 0 else (c if e == 0 else np.inf))
            out = out + t
        return out


def _binomial_reexpand(a_coef: np.ndarray, L: float) -> np.ndarray:
    """Coefficients of sum_k a_k y^k in powers of z = L - y."""
    n = len(a_coef)
    out = np.zeros(n)
    for k in range(n):
        for j in range(k + 1):
            # y^k = (L - z)^k = sum_j C(k,j) L^(k-j) (-z)^j
            out[j] += a_coef[k] * math.comb(k, j) * L ** (k - j) * (-1) ** j
    return out


@dataclasses.dataclass
class Manufactured:
    """A solution u, its boundary values and the right-hand side f it implies."""
    a: float
    b: float
    alpha: float
    theta: float
    rho: float
    u_left: PowerSum          # u in powers of (x-a)
    u_right: PowerSum | None  # u in powers of (b-x); None if theta must be 1
    f_terms: PowerSum         # f as a sum of signed powers

    @property
    def c1(self) -> float:
        return float(self.u(np.array([self.a]))[0])

    @property
    def c2(self) -> float:
        return float(self.u(np.array([self.b]))[0])

    def u(self, x) -> np.ndarray:
        return self.u_left(x, self.a, self.b)

    def f(self, x, da=None, db=None) -> np.ndarray:
        """f at x; pass da = x - a, db = b - x when known without cancellation."""
        return self.f_terms(x, self.a, self.b, da, db)


def _rl_terms(coef, expo, side, alpha, weight):
    c, e, s = [], [], []
    for ck, mk in zip(coef, expo):
        if ck == 0.0:
            continue
        # -D^2 I^{2-alpha} d^mu = -Gamma(mu+1)/Gamma(mu+1-alpha) d^(mu-alpha)
        g = math.gamma(mk + 1.0) / math.gamma(mk + 1.0 - alpha)
        c.append(-weight * ck * g)
        e.append(mk - alpha)
        s.append(side)
    return c, e, s


def manufactured_from_poly(a_coef, alpha, theta, rho, a=0.0, b=1.0) -> Manufactured:
    """u(x) = sum_k a_coef[k] (x-a)^k, a polynomial."""
    a_coef = np.asarray(a_coef, dtype=np.float64)
    ks = np.arange(len(a_coef), dtype=np.float64)
    b_coef = _binomial_reexpand(a_coef, b - a)
    u_left = PowerSum(a_coef.copy(), ks.copy(), np.zeros(len(ks), dtype=int))
    u_right = PowerSum(b_coef, ks.copy(), np.ones(len(ks), dtype=int))
    c, e, s = _rl_terms(a_coef, ks, 0, alpha, theta)
    c2, e2, s2 = _rl_terms(b_coef, ks, 1, alpha, 1.0 - theta)
    c += c2; e += e2; s += s2
    if rho != 0.0:
        for ck, mk in zip(a_coef, ks):
            if ck != 0.0:
                c.append(rho * ck); e.append(mk); s.append(0)
    f = PowerSum(np.array(c), np.array(e), np.array(s, dtype=int))
    return Manufactured(a, b, alpha, theta, rho, u_left, u_right, f)


def manufactured_left_powers(coef, expo, alpha, rho, a=0.0, b=1.0) -> Manufactured:
    """u(x) = sum_k coef_k (x-a)^{expo_k} with theta = 1 (one-sided problem)."""
    coef = np.asarray(coef, dtype=np.float64)
    expo = np.asarray(expo, dtype=np.float64)
    u_left = PowerSum(coef, expo, np.zeros(len(coef), dtype=int))
    c, e, s = _rl_terms(coef, expo, 0, alpha, 1.0)
    if rho != 0.0:
        for ck, mk in zip(coef, expo):
            c.append(rho * ck); e.append(mk); s.append(0)
    f = PowerSum(np.array(c), np.array(e), np.array(s, dtype=int))
    return Manufactured(a, b, alpha, 1.0, rho, u_left, None, f)


def example1(alpha: float = 1.6, rho: float = 0.0, gamma_: float = 0.8,
             a: float = 0.0, b: float = 10.0) -> Manufactured:
    """Section 5, Example 1: u = (x-a) - (b-a)^{1-gamma} (x-a)^gamma, theta = 1."""
    return manufactured_left_powers([1.0, -(b - a) ** (1.0 - gamma_)], [1.0, gamma_],
                                    alpha, rho, a, b)


def shifted_legendre_monomials(n: int) -> np.ndarray:
    """Monomial coefficients of the shifted Legendre polynomial P*_n on [0,1]."""
    return np.array([(-1) ** (n + k) * math.comb(n, k) * math.comb(n + k, k)
                     for k in range(n + 1)], dtype=np.float64)


def random_smooth_solution(gen: np.random.Generator, modes: int, alpha, theta, rho,
                           a=0.0, b=1.0) -> Manufactured:
    """u = sum_{m=1}^{modes} c_m y(1-y) P*_{m-1}(y), y = (x-a)/(b-a), c_m ~ N(0,1)/m.

    u vanishes at both ends; f has the endpoint singularities (x-a)^{k-alpha}.
    """
    L = b - a
    poly = np.zeros(modes + 2)
    c = gen.standard_normal(modes) / np.arange(1, modes + 1)
    for m in range(1, modes + 1):
        pm = shifted_legendre_monomials(m - 1)
        # y(1-y) P*_{m-1}(y) = (y - y^2) * sum pm_k y^k
        for k, pk in enumerate(pm):
            poly[k + 1] += c[m - 1] * pk
            poly[k + 2] -= c[m - 1] * pk
    a_coef = poly / L ** np.arange(len(poly))   # in powers of (x-a)
    return manufactured_from_poly(a_coef, alpha, theta, rho, a, b)


def random_polynomial_rhs(gen: np.random.Generator, degree: int, count: int,
                          a=0.0, b=1.0) -> List[np.ndarray]:
    """`count` right-hand sides f_j = sum_{k<=degree} c_jk P*_k(y), c_jk ~ N(0,1).

    Returned as monomial coefficients in powers of (x-a) (smooth f).
    """
    L = b - a
    out = []
    for _ in range(count):
        cf = gen.standard_normal(degree + 1)
        poly = np.zeros(degree + 1)
        for k in range(degree + 1):
            pk = shifted_legendre_monomials(k)
            poly[:k + 1] += cf[k] * pk
        out.append(poly / L ** np.arange(degree + 1))
    return out


def poly_function(coef: np.ndarray, a: float):
    """Callable x -> sum_k coef_k (x-a)^k (Horner); accepts (x, da, db) too."""
    def f(x, da=None, db=None):
        x = (np.asarray(x, dtype=np.float64) - a) if da is None else np.asarray(da, dtype=np.float64)
        y = np.zeros_like(x)
        for ck in coef[::-1]:
            y = y * x + ck
        return y
    return f


# ----------------------------------------------------------------------------
# Workload descriptions
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Instance:
    nodes: np.ndarray
    P: int
    alpha: float
    theta: float
    rho: float
    rhs: List  # callables f(x)
    mesh_kind: str
    R: int = 8
    leaf: int = 8
    c1: float = 0.0
    c2: float = 0.0
    solution: Manufactured | None = None


def config_small() -> Instance:
    """Uniform N=16, P=4, alpha=1.5, theta=0.5, rho=0, u = x^2 (1-x)^2, R=4."""
    m = manufactured_from_poly([0.0, 0.0, 1.0, -2.0, 1.0], 1.5, 0.5, 0.0)
    return Instance(uniform_mesh(16), 4, 1.5, 0.5, 0.0, [m.f], "uniform", R=4, leaf=2,
                    solution=m)


def config_uniform_grid(alpha: float, theta: float, N: int = 1024, P: int = 8,
                        modes: int = 8, R: int = 8, leaf: int = 8) -> Instance:
    """Uniform (0,1), rho = 1, one smooth random solution of `modes` modes."""
    gen = rng(1, stream=int(round(alpha * 100)) * 1000 + int(round(theta * 100)))
    m = random_smooth_solution(gen, modes, alpha, theta, 1.0)
    return Instance(uniform_mesh(N), P, alpha, theta, 1.0, [m.f], "uniform", R=R, leaf=leaf,
                    solution=m)


UNIFORM_GRID_ALPHAS = (1.2, 1.5, 1.8)
UNIFORM_GRID_THETAS = (0.3, 0.5, 0.8)


def config_graded_multi_rhs(N: int = 256, P: int = 16, nrhs: int = 64, degree: int = 20,
                            R: int = 8, leaf: int = 4) -> Instance:
    """Two-sided graded mesh (20 layers, q=0.5), alpha=1.7, theta=0.4, rho=0, many RHS."""
    gen = rng(2)
    polys = random_polynomial_rhs(gen, degree, nrhs)
    return Instance(two_sided_graded_mesh(N), P, 1.7, 0.4, 0.0,
                    [poly_function(p, 0.0) for p in polys], "graded", R=R, leaf=leaf)


def config_batched(count: int = 256, seed_stream: int = 0, N_range=(64, 2048),
                   P_range=(2, 12)) -> List[Instance]:
    """Uneven instances: N ~ U{64..2048}, P ~ U{2..12}, alpha ~ U(1.1,1.9), theta ~ U(0,1)."""
    gen = rng(3, seed_stream)
    out = []
    for _ in range(count):
        N = int(gen.integers(N_range[0], N_range[1] + 1))
        P = int(gen.integers(P_range[0], P_range[1] + 1))
        alpha = float(gen.uniform(1.1, 1.9))
        theta = float(gen.uniform(0.0, 1.0))
        graded = bool(gen.integers(0, 2))
        nodes = two_sided_graded_mesh(N) if graded else uniform_mesh(N)
        poly = random_polynomial_rhs(gen, 20, 1)[0]
        out.append(Instance(nodes, P, alpha, theta, 0.0, [poly_function(poly, 0.0)],
                            "graded" if graded else "uniform", R=8, leaf=8))
    return out
