"""ctypes declarations of the C ABI in include/fde.h (argument marshalling only)."""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfde.so")

FDE_OK = 0
FDE_EINVAL = -1
FDE_ENOMEM = -2
FDE_EBREAKDOWN = -3
FDE_ENOCONV = -4
FDE_EDEVICE = -5
FDE_EUNSUPPORTED = -6
FDE_FP64 = 0
FDE_FP32 = 1
FDE_FP32_BF16UV = 2
FDE_FGMRES = 0
FDE_BICGSTAB = 1
FDE_SIGMA_A = 0
FDE_SIGMA_AINV = 1
FDE_SIGMA_ATILDE_INV = 2
FDE_SIGMA_PRECOND = 3
FDE_APPLY_AUTO = 0
FDE_APPLY_DENSE = 1
FDE_APPLY_TOEPLITZ = 2

vp = C.c_void_p
i32 = C.c_int
f64 = C.c_double
dp = C.POINTER(C.c_double)
ip = C.POINTER(C.c_int)
sz = C.c_size_t


class HParams(C.Structure):
    _fields_ = [("R", i32), ("lam", f64), ("leaf_elems", i32)]


class HLUParams(C.Structure):
    _fields_ = [("tol", f64), ("rank_cap", i32), ("precision", i32), ("pivot_floor", f64)]


class SolveParams(C.Structure):
    _fields_ = [("method", i32), ("restart", i32), ("maxit", i32), ("rtol", f64)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", i32), ("relres", f64), ("status", i32)]


ll = C.c_longlong


class PlanInfo(C.Structure):
    _fields_ = [("ops", ll), ("levels", i32), ("max_width", i32), ("solve_ops", ll), ("arena_elems", ll),
                ("work_elems", ll), ("scratch_elems", ll), ("scratch_f64", ll), ("bytes_fp32", ll),
                ("bytes_fp64", ll), ("lr_blocks", i32), ("hsolve_steps", i32), ("hsolve_tslots", i32),
                ("hsolve_lds_fp32", ll), ("hsolve_lds_fp32_global_rhs", ll)]


class Problem(C.Structure):
    _fields_ = [("nodes", dp), ("N", i32), ("P", i32), ("alpha", f64), ("theta", f64), ("rho", f64)]


FN = C.CFUNCTYPE(C.c_double, C.c_double, C.c_void_p)

# name -> (restype, argtypes); every symbol declared in include/fde.h
SIGNATURES = {
    "fde_ctx_create": (i32, [i32, vp, sz, C.POINTER(vp)]),
    "fde_ctx_destroy": (None, [vp]),
    "fde_ctx_set_stream": (i32, [vp, vp]),
    "fde_ctx_set_apply_streams": (i32, [vp, i32]),
    "fde_ctx_bytes_in_use": (sz, [vp]),
    "fde_op_create": (i32, [vp, dp, i32, i32, f64, f64, f64, i32, C.POINTER(vp)]),
    "fde_op_create_hp": (i32, [vp, dp, i32, ip, f64, f64, f64, i32, C.POINTER(vp)]),
    "fde_op_destroy": (None, [vp]),
    "fde_op_ndof": (i32, [vp]),
    "fde_op_is_toeplitz": (i32, [vp]),
    "fde_op_pair_moments": (i32, [vp, i32, ip, ip, dp]),
    "fde_op_dense": (i32, [vp, vp, i32]),
    "fde_load_nodes": (i32, [vp, ip, dp, dp, dp]),
    "fde_load_vector": (i32, [vp, dp, f64, f64, vp]),
    "fde_load_vector_fn": (i32, [vp, FN, vp, f64, f64, vp]),
    "fde_load_vector_powers": (i32, [vp, i32, dp, dp, ip, f64, f64, vp]),
    "fde_stiffness_apply": (i32, [vp, i32, vp, i32, vp, i32]),
    "fde_stiffness_apply_noalloc": (i32, [vp, i32, vp, i32, vp, i32]),
    "fde_stiffness_apply_timed": (i32, [vp, i32, vp, i32, vp, i32, dp]),
    "fde_build_hmatrix": (i32, [vp, C.POINTER(HParams), C.POINTER(vp)]),
    "fde_hmat_destroy": (None, [vp]),
    "fde_hmat_counts": (i32, [vp, ip, ip]),
    "fde_hmat_to_dense": (i32, [vp, vp, i32]),
    "fde_hlu_factor": (i32, [vp, C.POINTER(HLUParams), C.POINTER(vp)]),
    "fde_hlu_factor_batched": (i32, [i32, C.POINTER(vp), C.POINTER(HLUParams), C.POINTER(vp)]),
    "fde_hlu_plan": (i32, [dp, i32, i32, C.POINTER(HParams), i32, i32, C.POINTER(PlanInfo)]),
    "fde_hlu_destroy": (None, [vp]),
    "fde_hlu_to_dense": (i32, [vp, vp, i32, ip]),
    "fde_hlu_max_rank": (i32, [vp, ip]),
    "fde_hlu_stats": (i32, [vp, dp, dp, dp]),
    "fde_hlu_solve": (i32, [vp, i32, vp, i32, vp, i32]),
    "fde_hlu_solve_variant": (i32, [vp, i32, ip, ip, C.POINTER(C.c_longlong)]),
    "fde_solve": (i32, [vp, vp, i32, vp, i32, vp, i32, C.POINTER(SolveParams), C.POINTER(SolveInfo)]),
    "fde_solve_batched": (i32, [vp, i32, C.POINTER(vp), C.POINTER(vp), ip, C.POINTER(vp), ip,
                                C.POINTER(vp), ip, C.POINTER(SolveParams), C.POINTER(SolveInfo)]),
    "fde_server_create": (i32, [vp, C.POINTER(HParams), C.POINTER(HLUParams), C.POINTER(SolveParams), sz,
                                C.POINTER(vp)]),
    "fde_server_destroy": (None, [vp]),
    "fde_server_solve": (i32, [vp, i32, C.POINTER(Problem), ip, C.POINTER(vp), ip, C.POINTER(vp), ip,
                               C.POINTER(SolveInfo), ip]),
    "fde_server_submit": (i32, [vp, C.POINTER(Problem), i32, vp, i32, vp, i32, C.POINTER(C.c_longlong)]),
    "fde_server_step": (i32, [vp, ip]),
    "fde_server_poll": (i32, [vp, C.c_longlong, ip, C.POINTER(SolveInfo), ip]),
    "fde_server_stats": (i32, [vp, ip, C.POINTER(sz), C.POINTER(C.c_longlong), C.POINTER(C.c_longlong),
                               C.POINTER(C.c_longlong)]),
    "fde_sigma_estimate": (i32, [vp, vp, i32, i32, C.c_ulonglong, dp, dp]),
    "fde_gauss_jacobi": (i32, [i32, f64, f64, dp, dp]),
    "fde_last_error": (C.c_char_p, []),
    "fde_version": (C.c_char_p, []),
}

_lib = None
_shutting_down = False
# root handles (contexts) still open; closing one closes every handle made from it
_roots = weakref.WeakSet()


def register_root(obj):
    _roots.add(obj)


def _shutdown():
    """At interpreter exit, while the HIP runtime is still whole: close every open context (its
    streams, events, pinned staging ring and cached device blocks go back to the runtime), then
    stop finalisers from calling into the library. Nothing of the library is left for the
    runtime's own teardown."""
    global _shutting_down
    for r in list(_roots):
        try:
            r.close()
        except Exception:
            pass
    _shutting_down = True


atexit.register(_shutdown)


def shutting_down() -> bool:
    return _shutting_down


def load():
    """Load libfde.so (built in-tree by __graft_entry__.build()); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(hipcc --offload-arch=gfx950); there is no fallback path")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


class FDEError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def check(rc):
    if rc != FDE_OK:
        msg = load().fde_last_error()
        raise FDEError(rc, msg.decode() if msg else "")
    return rc
