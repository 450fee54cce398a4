"""GPU parity: element-pair moments, dense A, stiffness apply and load vector vs the oracle."""
import numpy as np
import pytest
import torch

import fde_inputs as fi
from oracle import toeplitz
from oracle.sem import SEM
from tests.gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu

MESHES = {
    "uniform9": lambda: fi.uniform_mesh(9),
    "graded5": lambda: fi.graded_mesh(12, 5.0, 0.0, 10.0),
    "two_sided": lambda: fi.two_sided_graded_mesh(21, 4, 0.5),
    "extreme": lambda: np.array([0.0, 1e-4, 3.1e-3, 0.3, 0.4, 0.401, 1.0]),
    "geometric": lambda: fi.geometric_mesh(11, 1.15),
}


@pytest.fixture(scope="module")
def ctx():
    fde = need_gpu()
    return fde.Context(0)


@pytest.mark.parametrize("mesh", list(MESHES))
@pytest.mark.parametrize("P,alpha", [(2, 1.3), (4, 1.5), (7, 1.85), (16, 1.1)])
def test_pair_moments_match_oracle(ctx, mesh, P, alpha):
    import paper_1808_02937_amd as fde
    nodes = MESHES[mesh]()
    say(f"moments {mesh} P={P} alpha={alpha}")
    op = fde.Operator(ctx, nodes, P, alpha, 0.5, 0.0, apply="dense")
    sem = SEM(nodes, P, alpha, 0.5, 0.0)
    N = sem.N
    pairs = [(e, f) for e in range(N) for f in range(e + 1)]
    e = [p[0] for p in pairs]; f = [p[1] for p in pairs]
    got = op.pair_moments(e, f)
    for k, (ee, ff) in enumerate(pairs):
        ref = sem.pair_moment(ee, ff)
        err = np.abs(got[k] - ref).max() / np.abs(ref).max()
        assert err < 1e-13, (ee, ff, err)


@pytest.mark.parametrize("mesh", list(MESHES))
@pytest.mark.parametrize("theta,rho", [(0.5, 0.0), (1.0, 2.5), (0.2, 0.7)])
def test_dense_matrix_and_apply_match_oracle(ctx, mesh, theta, rho):
    import paper_1808_02937_amd as fde
    nodes = MESHES[mesh]()
    P, alpha = 5, 1.62
    say(f"dense/apply {mesh} theta={theta} rho={rho}")
    sem = SEM(nodes, P, alpha, theta, rho)
    A = sem.system_matrix()
    X = np.random.default_rng(7).standard_normal((3, sem.Nd))
    Xt = torch.tensor(X, device="cuda")
    for mode in ("dense", "auto"):
        op = fde.Operator(ctx, nodes, P, alpha, theta, rho, apply=mode)
        Ad = op.dense().cpu().numpy()
        assert np.abs(Ad - A).max() <= 1e-13 * np.abs(A).max(), mode
        Y = op.apply(Xt).cpu().numpy()
        ref = (A @ X.T).T
        assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max(), (mode, op.toeplitz)
        y1 = op.apply(Xt[1]).cpu().numpy()
        assert np.abs(y1 - ref[1]).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("N,P", [(1, 3), (2, 2), (33, 3), (100, 8), (257, 4)])
def test_apply_ragged_sizes_uniform_and_dense(ctx, N, P):
    import paper_1808_02937_amd as fde
    say(f"ragged N={N} P={P}")
    nodes = fi.uniform_mesh(N)
    sem = SEM(nodes, P, 1.45, 0.35, 0.3)
    X = np.random.default_rng(N).standard_normal((2, sem.Nd))
    Xt = torch.tensor(X, device="cuda")
    ref = toeplitz.apply(sem, X.T).T if N > 1 else (sem.system_matrix() @ X.T).T
    for mode in ("dense", "toeplitz"):
        op = fde.Operator(ctx, nodes, P, 1.45, 0.35, 0.3, apply=mode)
        Y = op.apply(Xt).cpu().numpy()
        assert np.abs(Y - ref).max() <= 2e-13 * np.abs(ref).max(), mode


@pytest.mark.parametrize("N,P,nrhs", [(40, 8, 8), (37, 5, 13), (33, 16, 64), (29, 6, 70), (50, 3, 9)])
def test_multi_rhs_dense_apply_matches_oracle(ctx, N, P, nrhs):
    """Eight or more right-hand sides take the matrix-core apply (chunks of 64; 70 = 64 + 6, the
    6 on the matrix cores too): every column equals the oracle's dense product and the one-column
    apply of the same column."""
    import paper_1808_02937_amd as fde
    say(f"multi-rhs dense apply N={N} P={P} nrhs={nrhs}")
    nodes = fi.two_sided_graded_mesh(N, min(6, N // 4), 0.5)
    sem = SEM(nodes, P, 1.7, 0.4, 0.2)
    A = sem.system_matrix()
    X = np.random.default_rng(1000 + nrhs).standard_normal((nrhs, sem.Nd))
    ref = (A @ X.T).T
    op = fde.Operator(ctx, nodes, P, 1.7, 0.4, 0.2)
    assert not op.toeplitz
    Xt = torch.tensor(X, device="cuda")
    Y = op.apply(Xt).cpu().numpy()
    assert np.abs(Y - ref).max() <= 2e-13 * np.abs(ref).max()
    for j in (0, nrhs // 2, nrhs - 1):
        y1 = op.apply(Xt[j].contiguous()).cpu().numpy()
        assert np.abs(Y[j] - y1).max() <= 1e-13 * np.abs(y1).max()
    op.close()


@pytest.mark.parametrize("case", ["small", "graded_theta1_lift", "random_modes"])
def test_load_vector_matches_oracle(ctx, case):
    import paper_1808_02937_amd as fde
    say(f"load vector {case}")
    if case == "small":
        inst = fi.config_small()
        m, nodes, P = inst.solution, inst.nodes, inst.P
    elif case == "graded_theta1_lift":
        m = fi.manufactured_from_poly([0.0, 0.5, 1.0, -0.3], 1.4, 1.0, 1.5)
        nodes, P = fi.graded_mesh(10, 2.0, 0.0, 1.0), 3
    else:
        m = fi.random_smooth_solution(fi.rng(1, 5), 8, 1.8, 0.3, 1.0)
        nodes, P = fi.uniform_mesh(64), 8
    sem = SEM(nodes, P, m.alpha, m.theta, m.rho)
    G = sem.load_vector(m.f_terms, m.c1, m.c2)
    # f is a sum of power terms that can cancel heavily (a polynomial re-expanded in powers of
    # b - x): evaluating it in FP64 carries an error of order eps times the term magnitudes, so
    # the bound adds 64 eps times the load vector of the term magnitudes to the quadrature bound
    ft = m.f_terms
    G_abs = sem.load_vector(fi.PowerSum(np.abs(ft.coef), ft.expo, ft.side))
    bound = 1e-12 * np.abs(G).max() + 64 * np.finfo(float).eps * np.abs(G_abs).max()
    op = fde.Operator(ctx, nodes, P, m.alpha, m.theta, m.rho)
    Gg = op.load_vector(m.f, m.c1, m.c2).cpu().numpy()
    assert np.abs(Gg - G).max() <= bound, (np.abs(Gg - G).max(), bound)
    # the same right-hand side evaluated on the device from its power terms
    Gp = op.load_vector_powers(ft.coef, ft.expo, ft.side, m.c1, m.c2).cpu().numpy()
    assert np.abs(Gp - G).max() <= bound, (np.abs(Gp - G).max(), bound)


def test_full_size_uniform_config_samples(ctx):
    """N=1024, P=8 uniform (the benchmark operator): sampled moments and the full apply."""
    import paper_1808_02937_amd as fde
    say("full size uniform N=1024 P=8")
    nodes = fi.uniform_mesh(1024)
    for alpha, theta in [(1.2, 0.3), (1.8, 0.8)]:
        sem = SEM(nodes, 8, alpha, theta, 1.0)
        op = fde.Operator(ctx, nodes, 8, alpha, theta, 1.0)
        assert op.toeplitz
        X = np.random.default_rng(3).standard_normal((2, sem.Nd))
        ref = toeplitz.apply(sem, X.T).T
        Y = op.apply(torch.tensor(X, device="cuda")).cpu().numpy()
        assert np.abs(Y - ref).max() <= 1e-12 * np.abs(ref).max()
        opd = fde.Operator(ctx, nodes, 8, alpha, theta, 1.0, apply="dense")
        pairs = [(0, 0), (1, 0), (5, 3), (1023, 0), (1023, 1022), (700, 11), (512, 510)]
        got = opd.pair_moments([p[0] for p in pairs], [p[1] for p in pairs])
        for k, (e, f) in enumerate(pairs):
            ref_m = sem.pair_moment(e, f)
            assert np.abs(got[k] - ref_m).max() <= 1e-13 * np.abs(ref_m).max(), (e, f)
        Yd = opd.apply(torch.tensor(X, device="cuda")).cpu().numpy()
        assert np.abs(Yd - ref).max() <= 1e-12 * np.abs(ref).max()


def test_bad_arguments_are_rejected(ctx):
    import paper_1808_02937_amd as fde
    from paper_1808_02937_amd._abi import FDEError, FDE_EINVAL
    for kw in [dict(alpha=1.0), dict(alpha=2.0), dict(theta=-0.1), dict(theta=1.5), dict(P=1), dict(rho=-1.0)]:
        args = dict(nodes=fi.uniform_mesh(4), P=3, alpha=1.5, theta=0.5, rho=0.0)
        args.update(kw)
        with pytest.raises(FDEError) as ei:
            fde.Operator(ctx, args["nodes"], args["P"], args["alpha"], args["theta"], args["rho"])
        assert ei.value.code == FDE_EINVAL
    with pytest.raises(FDEError):
        fde.Operator(ctx, np.array([0.0, 0.5, 0.4, 1.0]), 3, 1.5, 0.5, 0.0)
    with pytest.raises(FDEError):
        fde.Operator(ctx, fi.graded_mesh(8, 2.0, 0, 1), 3, 1.5, 0.5, 0.0, apply="toeplitz")


def test_budget_is_enforced():
    fde = need_gpu()
    from paper_1808_02937_amd._abi import FDEError, FDE_ENOMEM
    c = fde.Context(0, budget_bytes=1 << 20)
    with pytest.raises(FDEError) as ei:
        fde.Operator(c, fi.two_sided_graded_mesh(256, 20, 0.5), 16, 1.7, 0.4, 0.0)
    assert ei.value.code == FDE_ENOMEM
    assert c.bytes_in_use() < (1 << 20)
