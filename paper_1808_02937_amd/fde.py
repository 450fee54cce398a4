"""Python binding of the C ABI (include/fde.h): argument marshalling only.

Device arrays are torch tensors on the context's device. A block of nrhs
vectors is a contiguous tensor of shape (nrhs, Nd): row r is column r of the
column-major Nd x nrhs array the library sees, with leading dimension Nd.
"""
from __future__ import annotations

import ctypes as C
import weakref
from typing import Callable, Optional, Sequence

import numpy as np
import torch

from . import _abi as A
from ._abi import check, load


def _dptr(t: torch.Tensor) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _np_dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class _Handle:
    """Owns one library handle; closing it first closes every handle created from it
    (so a garbage-collection cycle can never free a parent before its children)."""

    _destroy = None

    def _init_handle(self, h, parent=None):
        self.h = h
        self._children = weakref.WeakSet()
        if parent is not None:
            parent._children.add(self)

    def close(self):
        for c in list(getattr(self, "_children", ())):
            c.close()
        if getattr(self, "h", None):
            if not A.shutting_down():
                getattr(load(), self._destroy)(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _as_block(t: torch.Tensor, Nd: int, device) -> torch.Tensor:
    if t.dim() == 1:
        t = t.unsqueeze(0)
    if t.dtype != torch.float64 or t.device != device or not t.is_contiguous() or t.shape[-1] != Nd:
        raise ValueError(f"expected a contiguous float64 tensor of shape (nrhs, {Nd}) on {device}")
    return t


def gauss_jacobi(n: int, a: float, b: float):
    """The library's own Gauss rule for the weight (1-x)^a (1+x)^b (host)."""
    x = np.zeros(n)
    w = np.zeros(n)
    check(load().fde_gauss_jacobi(n, a, b, _np_dptr(x), _np_dptr(w)))
    return x, w


def plan_hlu(nodes, P: int, R: int = 8, lam: float = 1.0, leaf_elems: int = 8, rank_cap: int = 0,
             check_schedule: bool = False) -> dict:
    """Host-only plan of an H-LU (op and level counts, device bytes per factorisation);
    check_schedule also verifies the level schedule element by element (slow)."""
    x = np.ascontiguousarray(nodes, dtype=np.float64)
    info = A.PlanInfo()
    hp = A.HParams(R, lam, leaf_elems)
    check(load().fde_hlu_plan(_np_dptr(x), len(x) - 1, P, C.byref(hp), rank_cap, int(check_schedule),
                              C.byref(info)))
    return {name: getattr(info, name) for name, _ in A.PlanInfo._fields_}


class Context(_Handle):
    """Device, HIP stream (torch's current stream by default) and HBM budget."""

    _destroy = "fde_ctx_destroy"

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None, budget_bytes: int = 0,
                 apply_streams: int = 3):
        """apply_streams: side streams for the per-operator applies of a batched Krylov step (0 keeps
        everything on `stream`, e.g. for several contexts driven side by side)."""
        lib = load()
        self.device = torch.device("cuda", device)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._stream = s
        h = C.c_void_p()
        check(lib.fde_ctx_create(device, C.c_void_p(s.cuda_stream), budget_bytes, C.byref(h)))
        self._init_handle(h)
        A.register_root(self)
        if apply_streams != 3:
            check(lib.fde_ctx_set_apply_streams(h, int(apply_streams)))

    def set_stream(self, stream: torch.cuda.Stream):
        self._stream = stream
        check(load().fde_ctx_set_stream(self.h, C.c_void_p(stream.cuda_stream)))

    def bytes_in_use(self) -> int:
        return int(load().fde_ctx_bytes_in_use(self.h))

    def synchronize(self):
        self._stream.synchronize()


_MODES = {"auto": A.FDE_APPLY_AUTO, "dense": A.FDE_APPLY_DENSE, "toeplitz": A.FDE_APPLY_TOEPLITZ}


class Operator(_Handle):
    """A = rho M + theta S_l + (1-theta) S_l^T on a mesh (Section 2.2)."""

    _destroy = "fde_op_destroy"

    def __init__(self, ctx: Context, nodes, P, alpha: float, theta: float, rho: float,
                 apply: str = "auto"):
        """P: the degree of every element, or a sequence of N degrees (one per element)."""
        self.ctx = ctx
        x = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64))
        self.N = len(x) - 1
        self.alpha, self.theta, self.rho = float(alpha), float(theta), float(rho)
        h = C.c_void_p()
        if np.ndim(P) == 0:
            self.P, self.degrees = int(P), None
            check(load().fde_op_create(ctx.h, _np_dptr(x), self.N, self.P, self.alpha, self.theta, self.rho,
                                       _MODES[apply], C.byref(h)))
        else:
            self.degrees = np.ascontiguousarray(P, dtype=np.int32)
            self.P = int(self.degrees.max())   # the operator's moments are of this degree
            check(load().fde_op_create_hp(ctx.h, _np_dptr(x), self.N, self.degrees.ctypes.data_as(A.ip),
                                          self.alpha, self.theta, self.rho, _MODES[apply], C.byref(h)))
        self._init_handle(h, ctx)
        self.Nd = int(load().fde_op_ndof(h))
        self.toeplitz = bool(load().fde_op_is_toeplitz(h))

    def pair_moments(self, e: Sequence[int], f: Sequence[int]) -> np.ndarray:
        e = np.ascontiguousarray(e, dtype=np.int32)
        f = np.ascontiguousarray(f, dtype=np.int32)
        out = np.zeros((len(e), self.P, self.P))
        check(load().fde_op_pair_moments(self.h, len(e), e.ctypes.data_as(A.ip), f.ctypes.data_as(A.ip),
                                         _np_dptr(out)))
        return out

    def dense(self) -> torch.Tensor:
        """A (Nd x Nd) on the device."""
        At = torch.empty((self.Nd, self.Nd), dtype=torch.float64, device=self.ctx.device)  # At[j, i] = A[i, j]
        check(load().fde_op_dense(self.h, _dptr(At), self.Nd))
        return At.t()

    def load_nodes(self):
        """(x, x - a, b - x) of the load-vector quadrature nodes."""
        n = C.c_int()
        check(load().fde_load_nodes(self.h, C.byref(n), None, None, None))
        x, da, db = np.zeros(n.value), np.zeros(n.value), np.zeros(n.value)
        check(load().fde_load_nodes(self.h, C.byref(n), _np_dptr(x), _np_dptr(da), _np_dptr(db)))
        return x, da, db

    def load_vector(self, f, c1: float = 0.0, c2: float = 0.0) -> torch.Tensor:
        """G = (f, phi) with lifting of c1, c2.

        f: values at the nodes of load_nodes(), or a vectorised callable f(x) or
        f(x, da, db) (the latter receives the exact distances to a and b)."""
        if callable(f):
            x, da, db = self.load_nodes()
            try:
                vals = f(x, da, db)
            except TypeError:
                vals = f(x)
            fv = np.ascontiguousarray(np.asarray(vals, dtype=np.float64))
        else:
            fv = np.ascontiguousarray(np.asarray(f, dtype=np.float64))
        G = torch.empty(self.Nd, dtype=torch.float64, device=self.ctx.device)
        check(load().fde_load_vector(self.h, _np_dptr(fv), float(c1), float(c2), _dptr(G)))
        return G

    def load_vector_powers(self, coef, expo, side, c1: float = 0.0, c2: float = 0.0) -> torch.Tensor:
        """G for f = sum_k coef_k d_k^expo_k (d = x - a for side 0, b - x for side 1), f on the device."""
        c = np.ascontiguousarray(coef, dtype=np.float64)
        e = np.ascontiguousarray(expo, dtype=np.float64)
        sd = np.ascontiguousarray(side, dtype=np.int32)
        if not (len(c) == len(e) == len(sd)):
            raise ValueError("coef, expo and side must have the same length")
        G = torch.empty(self.Nd, dtype=torch.float64, device=self.ctx.device)
        check(load().fde_load_vector_powers(self.h, len(c), _np_dptr(c), _np_dptr(e), sd.ctypes.data_as(A.ip),
                                            float(c1), float(c2), _dptr(G)))
        return G

    def apply(self, X: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        X2 = _as_block(X, self.Nd, self.ctx.device)
        Y = torch.empty_like(X2) if out is None else _as_block(out, self.Nd, self.ctx.device)
        check(load().fde_stiffness_apply(self.h, X2.shape[0], _dptr(X2), X2.stride(0), _dptr(Y), Y.stride(0)))
        return Y.view_as(X) if out is None else out

    def apply_timed(self, X: torch.Tensor, out: torch.Tensor) -> float:
        """Y = A X into `out`, waited for; returns the HIP-event milliseconds of the kernels that
        read the operator (dense: the moment stream; Toeplitz: the symbol product)."""
        X2 = _as_block(X, self.Nd, self.ctx.device)
        Y = _as_block(out, self.Nd, self.ctx.device)
        ms = C.c_double()
        check(load().fde_stiffness_apply_timed(self.h, X2.shape[0], _dptr(X2), X2.stride(0), _dptr(Y), Y.stride(0),
                                               C.byref(ms)))
        return ms.value

    def apply_noalloc(self, X: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """Y = A X into `out` with the library's fixed per-GPU workspace (no device allocation)."""
        X2 = _as_block(X, self.Nd, self.ctx.device)
        Y = _as_block(out, self.Nd, self.ctx.device)
        check(load().fde_stiffness_apply_noalloc(self.h, X2.shape[0], _dptr(X2), X2.stride(0), _dptr(Y),
                                                 Y.stride(0)))
        return out


class HMatrix(_Handle):
    """A~ = rho M + H (Section 3)."""

    _destroy = "fde_hmat_destroy"

    def __init__(self, op: Operator, R: int = 8, lam: float = 1.0, leaf_elems: int = 8):
        self.op = op
        p = A.HParams(int(R), float(lam), int(leaf_elems))
        h = C.c_void_p()
        check(load().fde_build_hmatrix(op.h, C.byref(p), C.byref(h)))
        self._init_handle(h, op)

    def counts(self):
        nd, nr = C.c_int(), C.c_int()
        check(load().fde_hmat_counts(self.h, C.byref(nd), C.byref(nr)))
        return nd.value, nr.value

    def dense(self) -> torch.Tensor:
        Nd = self.op.Nd
        At = torch.empty((Nd, Nd), dtype=torch.float64, device=self.op.ctx.device)
        check(load().fde_hmat_to_dense(self.h, _dptr(At), Nd))
        return At.t()


class HLU(_Handle):
    """H-LU factors L_H U_H of A~ (Section 4.1)."""

    _destroy = "fde_hlu_destroy"

    def __init__(self, hm: HMatrix, tol: float = 1e-3, rank_cap: int = 0, precision: str = "fp32",
                 pivot_floor: float = 1e-14):
        self.hm = hm
        self.Nd = hm.op.Nd
        self.device = hm.op.ctx.device
        prec = {"fp64": A.FDE_FP64, "fp32": A.FDE_FP32, "bf16uv": A.FDE_FP32_BF16UV}[precision]
        p = A.HLUParams(float(tol), int(rank_cap), prec, float(pivot_floor))
        h = C.c_void_p()
        check(load().fde_hlu_factor(hm.h, C.byref(p), C.byref(h)))
        self._init_handle(h, hm)

    def solve(self, B: torch.Tensor) -> torch.Tensor:
        B2 = _as_block(B, self.Nd, self.device)
        X = torch.empty_like(B2)
        check(load().fde_hlu_solve(self.h, B2.shape[0], _dptr(B2), B2.stride(0), _dptr(X), X.stride(0)))
        return X.view_as(B)

    def solve_variant(self, nrhs: int = 1) -> dict:
        """Which H-solve a solve of nrhs columns runs: "lds", "global_rhs" or "ops" (op-list
        interpreter), its columns per workgroup and LDS bytes."""
        v, w, b = C.c_int(0), C.c_int(0), C.c_longlong(0)
        check(load().fde_hlu_solve_variant(self.h, nrhs, C.byref(v), C.byref(w), C.byref(b)))
        return {"variant": {0: "ops", 1: "lds", 2: "global_rhs"}[v.value], "cols": w.value, "lds_bytes": b.value}

    def dense(self):
        """(packed L\\U in the internal order as an Nd x Nd tensor, h2p order)."""
        Nd = self.Nd
        Ft = torch.empty((Nd, Nd), dtype=torch.float64, device=self.device)
        h2p = np.zeros(Nd, dtype=np.int32)
        check(load().fde_hlu_to_dense(self.h, _dptr(Ft), Nd, h2p.ctypes.data_as(A.ip)))
        return Ft.t(), h2p

    def stats(self):
        """(factor flops, factorisation launch ms, H-solve flops so far)."""
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        check(load().fde_hlu_stats(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def max_rank(self) -> int:
        r = C.c_int()
        check(load().fde_hlu_max_rank(self.h, C.byref(r)))
        return r.value


def factor_batched(hms: Sequence[HMatrix], tol: float = 1e-3, rank_cap: int = 0, precision: str = "fp32",
                   pivot_floor: float = 1e-14):
    """H-LU of several H-matrices together: each kernel launch runs one level of every factorisation."""
    n = len(hms)
    prec = {"fp64": A.FDE_FP64, "fp32": A.FDE_FP32, "bf16uv": A.FDE_FP32_BF16UV}[precision]
    p = A.HLUParams(float(tol), int(rank_cap), prec, float(pivot_floor))
    arr = (C.c_void_p * n)(*[hm.h.value for hm in hms])
    out = (C.c_void_p * n)()
    check(load().fde_hlu_factor_batched(n, arr, C.byref(p), out))
    res = []
    for hm, h in zip(hms, out):
        obj = HLU.__new__(HLU)
        obj.hm = hm
        obj.Nd = hm.op.Nd
        obj.device = hm.op.ctx.device
        obj._init_handle(C.c_void_p(h), hm)
        res.append(obj)
    return res


_METHODS = {"fgmres": A.FDE_FGMRES, "bicgstab": A.FDE_BICGSTAB}
_SIGMA = {"A": A.FDE_SIGMA_A, "Ainv": A.FDE_SIGMA_AINV, "Atilde_inv": A.FDE_SIGMA_ATILDE_INV,
          "precond": A.FDE_SIGMA_PRECOND}


def sigma_estimate(op: "Operator", kind: str, lu: Optional["HLU"] = None, steps: int = 64, seed: int = 1808029370):
    """(largest, smallest) singular value of the Arnoldi Hessenberg matrix of B after `steps` steps:
    B = A ("A"), A^{-1} ("Ainv"), the H-LU solve ("Atilde_inv"), or the preconditioned operator
    ("precond")."""
    smax, smin = C.c_double(), C.c_double()
    check(load().fde_sigma_estimate(op.h, lu.h if lu is not None else None, _SIGMA[kind], int(steps), int(seed),
                                    C.byref(smax), C.byref(smin)))
    return smax.value, smin.value


def _solve_params(rtol, restart, maxit, method="fgmres"):
    return A.SolveParams(_METHODS[method], int(restart), int(maxit), float(rtol))


def solve(op: Operator, G: torch.Tensor, prec: Optional[HLU] = None, rtol: float = 1e-10,
          restart: int = 30, maxit: int = 500, raise_on_noconv: bool = True, method: str = "fgmres"):
    """X with ||G - A X|| <= rtol ||G|| per column (right-preconditioned FGMRES), or the paper's
    left-preconditioned BiCGSTAB (method="bicgstab": preconditioned residual <= rtol). Returns
    (X, infos)."""
    G2 = _as_block(G, op.Nd, op.ctx.device)
    X = torch.empty_like(G2)
    nrhs = G2.shape[0]
    info = (A.SolveInfo * nrhs)()
    p = _solve_params(rtol, restart, maxit, method)
    rc = load().fde_solve(op.h, prec.h if prec is not None else None, nrhs, _dptr(G2), G2.stride(0),
                          _dptr(X), X.stride(0), C.byref(p), info)
    if rc != A.FDE_ENOCONV or raise_on_noconv:
        check(rc)
    infos = [dict(iters=i.iters, relres=i.relres, status=i.status) for i in info]
    return X.view_as(G), infos


def solve_batched(ctx: Context, ops: Sequence[Operator], Gs: Sequence[torch.Tensor],
                  precs: Optional[Sequence[Optional[HLU]]] = None, rtol: float = 1e-10,
                  restart: int = 30, maxit: int = 500, raise_on_noconv: bool = True,
                  outs: Optional[Sequence[torch.Tensor]] = None, method: str = "fgmres"):
    """Solve several independent systems in lock-step launches. Returns (Xs, infos per system)."""
    n = len(ops)
    precs = precs if precs is not None else [None] * n
    G2 = [_as_block(G, op.Nd, ctx.device) for G, op in zip(Gs, ops)]
    Xs = [torch.empty_like(g) for g in G2] if outs is None else [_as_block(x, op.Nd, ctx.device)
                                                                 for x, op in zip(outs, ops)]
    nr = (C.c_int * n)(*[g.shape[0] for g in G2])
    ldg = (C.c_int * n)(*[g.stride(0) for g in G2])
    ldx = (C.c_int * n)(*[x.stride(0) for x in Xs])
    op_h = (C.c_void_p * n)(*[o.h.value for o in ops])
    pr_h = (C.c_void_p * n)(*[(p.h.value if p is not None else None) for p in precs])
    g_p = (C.c_void_p * n)(*[g.data_ptr() for g in G2])
    x_p = (C.c_void_p * n)(*[x.data_ptr() for x in Xs])
    tot = sum(g.shape[0] for g in G2)
    info = (A.SolveInfo * tot)()
    p = _solve_params(rtol, restart, maxit, method)
    rc = load().fde_solve_batched(ctx.h, n, op_h, pr_h, nr, g_p, ldg, x_p, ldx, C.byref(p), info)
    if rc != A.FDE_ENOCONV or raise_on_noconv:
        check(rc)
    out, k = [], 0
    for g in G2:
        out.append([dict(iters=info[k + j].iters, relres=info[k + j].relres, status=info[k + j].status)
                    for j in range(g.shape[0])])
        k += g.shape[0]
    return [x.view_as(g0) for x, g0 in zip(Xs, Gs)], out


class Server(_Handle):
    """Solver cache and batched serving over one context (fde_server_*)."""

    _destroy = "fde_server_destroy"

    def __init__(self, ctx: Context, R: int = 8, lam: float = 1.0, leaf_elems: int = 8, tol: float = 1e-3,
                 rank_cap: int = 0, precision: str = "fp32", pivot_floor: float = 1e-14, rtol: float = 1e-10,
                 restart: int = 30, maxit: int = 500, budget_bytes: int = 0):
        lib = load()
        self.ctx = ctx
        hp = A.HParams(int(R), float(lam), int(leaf_elems))
        prec = {"fp64": A.FDE_FP64, "fp32": A.FDE_FP32, "bf16uv": A.FDE_FP32_BF16UV}[precision]
        lp = A.HLUParams(float(tol), int(rank_cap), prec, float(pivot_floor))
        sp = _solve_params(rtol, restart, maxit)
        h = C.c_void_p()
        check(lib.fde_server_create(ctx.h, C.byref(hp), C.byref(lp), C.byref(sp), int(budget_bytes), C.byref(h)))
        self._init_handle(h, ctx)

    def solve(self, problems, Gs):
        """problems: list of (nodes, P, alpha, theta, rho); Gs: list of (nrhs, Nd) float64 device tensors.
        Returns (Xs, infos per request, cached flags)."""
        n = len(problems)
        keep = []
        probs = (A.Problem * n)()
        for i, (nodes, P, alpha, theta, rho) in enumerate(problems):
            x = np.ascontiguousarray(nodes, dtype=np.float64)
            keep.append(x)
            probs[i] = A.Problem(_np_dptr(x), len(x) - 1, int(P), float(alpha), float(theta), float(rho))
        blocks = [_as_block(G, int(len(keep[i]) - 1) * int(problems[i][1]) - 1, self.ctx.device) for i, G in enumerate(Gs)]
        Xs = [torch.empty_like(B) for B in blocks]
        nr = (C.c_int * n)(*[B.shape[0] for B in blocks])
        ld = (C.c_int * n)(*[B.shape[1] for B in blocks])
        Gp = (C.c_void_p * n)(*[B.data_ptr() for B in blocks])
        Xp = (C.c_void_p * n)(*[X.data_ptr() for X in Xs])
        ns = sum(B.shape[0] for B in blocks)
        info = (A.SolveInfo * max(ns, 1))()
        cached = (C.c_int * n)()
        rc = load().fde_server_solve(self.h, n, probs, nr, Gp, ld, Xp, ld, info, cached)
        if rc not in (A.FDE_OK, A.FDE_ENOCONV, A.FDE_ENOMEM):
            check(rc)
        out, k = [], 0
        for B in blocks:
            out.append([(info[k + j].iters, info[k + j].relres, info[k + j].status) for j in range(B.shape[0])])
            k += B.shape[0]
        return Xs, out, [bool(c) for c in cached]

    # -- continuous serving --
    def submit(self, problem, G: torch.Tensor, X: Optional[torch.Tensor] = None):
        """Queue one request (problem = (nodes, P, alpha, theta, rho); G: (nrhs, Nd) float64 on the
        device). Returns (ticket, X); X is written when the request is done."""
        nodes, P, alpha, theta, rho = problem
        x = np.ascontiguousarray(nodes, dtype=np.float64)
        Nd = (len(x) - 1) * int(P) - 1
        B = _as_block(G, Nd, self.ctx.device)
        Xo = torch.empty_like(B) if X is None else _as_block(X, Nd, self.ctx.device)
        prob = A.Problem(_np_dptr(x), len(x) - 1, int(P), float(alpha), float(theta), float(rho))
        t = C.c_longlong()
        check(load().fde_server_submit(self.h, C.byref(prob), B.shape[0], _dptr(B), B.stride(0), _dptr(Xo),
                                       Xo.stride(0), C.byref(t)))
        self._live = getattr(self, "_live", {})
        self._live[t.value] = (B, Xo)   # keep the device arrays alive until the ticket is collected
        return t.value, Xo

    def step(self) -> int:
        """Admit what fits, advance every request in flight by one Krylov step; returns the number of
        requests still queued or running."""
        n = C.c_int()
        check(load().fde_server_step(self.h, C.byref(n)))
        return n.value

    def poll(self, ticket: int):
        """(done, infos, cached) for a ticket; once done the ticket is forgotten. A failed request
        raises FDEError with its status."""
        B, Xo = self._live[ticket]
        done = C.c_int()
        cached = C.c_int()
        info = (A.SolveInfo * max(B.shape[0], 1))()
        rc = load().fde_server_poll(self.h, ticket, C.byref(done), info, C.byref(cached))
        if rc == A.FDE_OK and not done.value:
            return False, None, None
        del self._live[ticket]
        check(rc)
        return True, [(info[j].iters, info[j].relres, info[j].status) for j in range(B.shape[0])], bool(cached.value)

    def drain(self, max_steps: int = 100000):
        """Step until nothing is queued or running."""
        for _ in range(max_steps):
            if self.step() == 0:
                return
        raise RuntimeError("server: requests still in flight after max_steps steps")

    def stats(self) -> dict:
        e = C.c_int()
        b = C.c_size_t()
        hi, mi, ev = C.c_longlong(), C.c_longlong(), C.c_longlong()
        check(load().fde_server_stats(self.h, C.byref(e), C.byref(b), C.byref(hi), C.byref(mi), C.byref(ev)))
        return {"entries": e.value, "bytes": b.value, "hits": hi.value, "misses": mi.value, "evictions": ev.value}
