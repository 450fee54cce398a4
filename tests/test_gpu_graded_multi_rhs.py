"""GPU parity at the graded multi-right-hand-side shapes: two-sided graded N = 256, P = 16
(Nd = 4095), alpha = 1.7, theta = 0.4, R = 8, leaf 4 (64-row leaves), 64 right-hand sides -- the
structure the benchmark factors and solves in that workload (dense moment stream and FP64 matrix-core
apply, leaf-step H-solves of one column per workgroup, batched FGMRES over the 64 columns). The
H-matrix and the FP32 / FP64 H-solves are compared element by element with the oracle's; the FGMRES
solution is checked on rows of A X = G that the oracle computes one by one."""
import numpy as np
import pytest
import torch

import fde_inputs as fi
from oracle.hmatrix import HLU as OHLU
from oracle.hmatrix import HMatrix as OHMatrix
from oracle.hmatrix import to_dense
from oracle.sem import SEM
from tests.gpu_common import EPS32, EPS64, kappa1, need_gpu, say

pytestmark = pytest.mark.gpu

# H-solve bounds as at the other shapes: 10 kappa_1(A~) eps (kappa_1(A~) = 1.6e9 here), capped at
# about ten times the errors measured on the MI355X at this shape (FP32 1.5e-4, FP64 9.0e-13)
FP32_CAP = 2e-3
FP64_CAP = 1e-11


@pytest.fixture(scope="module")
def case():
    fde = need_gpu()
    inst = fi.config_graded_multi_rhs()
    say("graded multi-RHS shape: oracle H-matrix and H-LU (N=256, P=16)")
    sem = SEM(inst.nodes, inst.P, inst.alpha, inst.theta, inst.rho)
    oh = OHMatrix(sem, inst.R, 1.0, inst.leaf)
    ofac = OHLU(oh, tol=1e-3)
    Ah = to_dense(oh.root)
    kap = kappa1(Ah)
    ctx = fde.Context(0)
    op = fde.Operator(ctx, inst.nodes, inst.P, inst.alpha, inst.theta, inst.rho)
    hm = fde.HMatrix(op, R=inst.R, lam=1.0, leaf_elems=inst.leaf)
    say(f"  Nd {sem.Nd}, kappa_1(A~) = {kap:.3e}")
    yield dict(fde=fde, inst=inst, sem=sem, oh=oh, ofac=ofac, Ah=Ah, kappa=kap, ctx=ctx, op=op, hm=hm)
    op.close()
    ctx.close()


def test_graded_hmatrix_matches_oracle(case):
    say("graded multi-RHS shape: H-matrix")
    c = case
    assert c["hm"].counts() == c["oh"].counts()
    At = c["hm"].dense().cpu().numpy()
    ref = np.empty_like(At)
    h2p = c["oh"].h2p
    ref[np.ix_(h2p, h2p)] = c["Ah"]
    rel = np.abs(At - ref).max() / np.abs(ref).max()
    say(f"  max |A~_gpu - A~| / max |A~| = {rel:.2e}")
    assert rel <= 1e-13, rel


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graded_hsolve_64_rhs_matches_oracle(case, precision):
    c = case
    fde = c["fde"]
    say(f"graded multi-RHS shape: {precision} H-solve of 64 columns")
    lu = fde.HLU(c["hm"], tol=1e-3, precision=precision)
    assert lu.solve_variant(64)["variant"] == "lds"
    g = np.random.default_rng(41).standard_normal((64, c["sem"].Nd))
    x = lu.solve(torch.tensor(g, device="cuda")).cpu().numpy()
    xo = c["ofac"].solve(g.T).T
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    eps, cap = (EPS64, FP64_CAP) if precision == "fp64" else (EPS32, FP32_CAP)
    bound = min(cap, 10 * c["kappa"] * eps)
    say(f"  |X - X_o| / |X_o| = {err:.2e} (bound {bound:.2e})")
    assert err <= bound, err
    lu.close()


def test_graded_fgmres_64_rhs_sampled_rows(case):
    """FGMRES over the 64 polynomial right-hand sides with the FP32 H-LU: the library's residual
    reaches 1e-10; on 24 sampled rows the oracle's own A[i, :] X agrees with the device's apply to
    the FP64 rounding of the products (relative to |A| |X|) and with G to the requested residual."""
    c = case
    fde = c["fde"]
    say("graded multi-RHS shape: FGMRES, 64 columns")
    op = c["op"]
    G = torch.stack([op.load_vector(f) for f in c["inst"].rhs])
    lu = fde.HLU(c["hm"], tol=1e-3, precision="fp32")
    X, infos = fde.solve(op, G, lu, rtol=1e-10)
    assert all(i["status"] == 0 and i["relres"] <= 1e-10 for i in infos)
    its = [i["iters"] for i in infos]
    rows = np.sort(np.random.default_rng(42).choice(c["sem"].Nd, size=24, replace=False))
    A_rows = c["sem"].block(rows, np.arange(c["sem"].Nd))          # oracle rows of A
    x = X.cpu().numpy()
    AX_o = (A_rows @ x.T).T                                          # (64, 24)
    AX_d = op.apply(X).cpu().numpy()[:, rows]
    # relative to |A| |X| (the products cancel: A X = G is far smaller than |A| |X| here)
    rel = np.abs(AX_d - AX_o).max() / (np.abs(A_rows) @ np.abs(x).T).max()
    g = G.cpu().numpy()[:, rows]
    res = np.abs(g - AX_o).max() / np.abs(G.cpu().numpy()).max()
    say(f"  iterations {min(its)}..{max(its)}; sampled rows: |AX_gpu - AX_oracle| / |A||X| {rel:.2e}, "
        f"|G - AX_oracle| / max|G| {res:.2e}")
    assert rel <= 1e-12, rel
    assert res <= 1e-9, res
    lu.close()
