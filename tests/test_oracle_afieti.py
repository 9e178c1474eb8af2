"""Pins of the oracle's tearing, coarse space, FD, Schur complement,
preconditioner and MINRES (Sections 4, 5.2, 5.2.1, Remark 1) against dense
linear algebra, brute force on tiny inputs and invariants."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle.afieti import AFIETI, minres, Breakdown, SingularCoarse
from oracle.direct import solve_conforming


@pytest.fixture(scope="module")
def sys2():
    return AFIETI(W.make_c1(n_el=3, p=2))


@pytest.fixture(scope="module")
def sys3():
    return AFIETI(W.make_c2(n_el=2, p=2))


def _kron_list(mats):
    T = np.ones((1, 1))
    for Mm in reversed(mats):
        T = np.kron(T, Mm)
    return T


def _Ahat_dense(s, k, l, interior=False):
    kap = s.kappa(k, l)
    A = 0
    for m in range(s.dim):
        mats = []
        for mm in range(s.dim):
            X = s.fd[k][mm]["K"] if mm == m else s.fd[k][mm]["M"]
            mats.append(X[1:-1, 1:-1] if interior else X)
        A = A + kap[m] * _kron_list(mats)
    return A


@pytest.mark.parametrize("name", ["sys2", "sys3"])
def test_B_rank_and_continuity(name, request):
    s = request.getfixturevalue(name)
    B = s.B.toarray()
    assert np.linalg.matrix_rank(B) == s.n_c  # ker B^T = 0
    # a continuous field vanishing on Gamma_D: u(x) = x_D * a (D = Dirichlet dir)
    ddir = 0 if s.dim == 2 else 2
    a = np.arange(1, s.dim + 1, dtype=float)
    parts = []
    for pa in s.patches:
        X = pa.ctrl.reshape(-1, s.dim)
        parts.append(np.outer(a, X[:, ddir]).reshape(-1))
    u = np.concatenate(parts)
    assert np.abs(B @ u).max() < 1e-13
    # a field that jumps across an interface is detected
    u2 = u.copy()
    u2[s.offsets[1]:s.offsets[2]] += 1.0
    assert np.abs(B @ u2).max() > 0.5


@pytest.mark.parametrize("name", ["sys2", "sys3"])
def test_BBt_block_diagonal_by_node(name, request):
    s = request.getfixturevalue(name)
    BBt = s.BBt.toarray()
    # rows of one node and component are contiguous; no coupling between nodes
    owner = np.zeros(s.n_c, dtype=int)
    r = 0
    for c in range(s.dim):
        for ci, (cp, isd) in enumerate(zip(s.classes, s.dirichlet_class)):
            nr = len(cp) if isd else len(cp) - 1
            owner[r:r + nr] = c * len(s.classes) + ci
            r += nr
    off = owner[:, None] != owner[None, :]
    assert np.all(BBt[off] == 0)


@pytest.mark.parametrize("name", ["sys2", "sys3"])
def test_coarse_space_and_projectors(name, request):
    s = request.getfixturevalue(name)
    rng = np.random.default_rng(0)
    G = s.G
    assert np.linalg.matrix_rank(G) == G.shape[1]
    y = rng.standard_normal(s.n_c)
    py = s.P_chi(y)
    assert np.allclose(s.P_chi(py), py, atol=1e-12)
    z = rng.standard_normal(s.n_c)
    assert s.P_chi(y) @ z == pytest.approx(y @ s.P_chi(z), rel=1e-12)
    assert np.abs(G.T @ py).max() < 1e-11
    f = s.load()
    lam0 = s.lambda0(f)
    assert np.allclose(G.T @ lam0, s.R.T @ f, atol=1e-12)
    x = rng.standard_normal(s.n_dof)
    pu = s.P_u(x)
    assert np.abs(s.R.T @ pu).max() < 1e-11
    assert np.allclose(s.apply_A(pu), s.apply_A(x), atol=1e-10)


@pytest.mark.parametrize("name", ["sys2", "sys3"])
def test_eigendecomposition_identities(name, request):
    s = request.getfixturevalue(name)
    for per in s.fd:
        for e in per:
            U, D = e["U"], e["D"]
            assert np.allclose(U.T @ e["M"] @ U, np.eye(len(D)), atol=1e-11)
            assert np.allclose(U.T @ e["K"] @ U, np.diag(D), atol=1e-9 * D.max())
            assert np.sum(np.abs(D) < 1e-9 * D.max()) == 1  # K is singular
            assert np.all(D > -1e-9 * D.max())
            assert np.all(e["Di"] > 0)


@pytest.mark.parametrize("name", ["sys2", "sys3"])
def test_fd_equals_dense_solve(name, request):
    s = request.getfixturevalue(name)
    rng = np.random.default_rng(1)
    for k in range(len(s.patches)):
        pa = s.patches[k]
        Mh = _kron_list([s.fd[k][m]["M"] for m in range(s.dim)])
        h = pa.diameter() ** (s.dim - 2)
        for l in range(s.dim):
            P = h * (_Ahat_dense(s, k, l) + Mh)
            r = rng.standard_normal(pa.shape)
            x = s.fd_solve(k, l, r)
            assert np.allclose(P @ x.reshape(-1), r.reshape(-1), atol=1e-10)
            Pi = _Ahat_dense(s, k, l, interior=True)
            ri = rng.standard_normal(tuple(n - 2 for n in pa.shape))
            xi = s.fd_solve_interior(k, l, ri)
            assert np.allclose(Pi @ xi.reshape(-1), ri.reshape(-1), atol=1e-10)


@pytest.mark.parametrize("name", ["sys2", "sys3"])
def test_Ahat_apply_matches_dense(name, request):
    s = request.getfixturevalue(name)
    rng = np.random.default_rng(2)
    pa = s.patches[0]
    for l in range(s.dim):
        x = rng.standard_normal(pa.shape)
        assert np.allclose(s.apply_Ahat(0, l, x).reshape(-1),
                           _Ahat_dense(s, 0, l) @ x.reshape(-1), atol=1e-11)


@pytest.mark.parametrize("name", ["sys2", "sys3"])
def test_Shat_equals_dense_schur(name, request):
    s = request.getfixturevalue(name)
    rng = np.random.default_rng(3)
    k = len(s.patches) - 1
    pa = s.patches[k]
    gm = pa.gamma_mask().reshape(-1)
    for l in range(s.dim):
        A = _Ahat_dense(s, k, l)
        G, I = np.nonzero(gm)[0], np.nonzero(~gm)[0]
        S = A[np.ix_(G, G)] - A[np.ix_(G, I)] @ np.linalg.solve(A[np.ix_(I, I)], A[np.ix_(I, G)])
        th = rng.standard_normal(pa.shape)
        y = s.apply_Shat(k, l, th).reshape(-1)
        assert np.allclose(y[G], S @ th.reshape(-1)[G], atol=1e-9 * np.abs(S).max())
        assert np.all(y[I] == 0)
        # kills constants on Gamma; symmetric positive semidefinite
        assert np.abs(S @ np.ones(len(G))).max() < 1e-9 * np.abs(S).max()
        assert np.allclose(S, S.T, atol=1e-10 * np.abs(S).max())
        assert np.linalg.eigvalsh(S).min() > -1e-9 * np.abs(S).max()


def test_PS_matches_dense_formula(sys3):
    s = sys3
    # dense W B Sblock B^T W built from explicit Schur complements
    n = s.n_dof
    Sfull = np.zeros((n, n))
    for k, pa in enumerate(s.patches):
        gm = pa.gamma_mask().reshape(-1)
        G, I = np.nonzero(gm)[0], np.nonzero(~gm)[0]
        h = pa.diameter() ** (s.dim - 2)
        for l in range(s.dim):
            A = _Ahat_dense(s, k, l)
            S = A[np.ix_(G, G)] - A[np.ix_(G, I)] @ np.linalg.solve(A[np.ix_(I, I)], A[np.ix_(I, G)])
            base = s.offsets[k] + l * pa.n_nodes
            Sfull[np.ix_(base + G, base + G)] = h * S
    B = s.B.toarray()
    Winv = np.linalg.inv(B @ B.T)
    Pd = Winv @ B @ Sfull @ B.T @ Winv
    y = np.random.default_rng(4).standard_normal(s.n_c)
    assert np.allclose(s.apply_PS(y), Pd @ y, atol=1e-9 * np.abs(Pd).max())
    assert np.allclose(s.apply_PS(y, "plain"), B @ Sfull @ B.T @ y, atol=1e-9 * np.abs(Sfull).max())


def test_minres_minimises_preconditioned_residual():
    # symmetric indefinite A, SPD P: x_j minimises ||b - A x||_P over K_j(PA, Pb)
    rng = np.random.default_rng(5)
    n = 12
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    A = Q @ np.diag(np.concatenate([rng.uniform(1, 3, 7), -rng.uniform(1, 3, 5)])) @ Q.T
    L = rng.standard_normal((n, n))
    P = L @ L.T + n * np.eye(n)
    b = rng.standard_normal(n)
    Pb = P @ b
    K = [Pb]
    for j in range(1, 7):
        x, its, hist = minres(lambda v: A @ v, lambda v: P @ v, b, 0.0, j)
        assert its == j
        V = np.array(K).T  # Krylov basis of dimension j
        # min over y of (b - A V y)^T P (b - A V y)
        C = sla.cholesky(P, lower=False)
        y = np.linalg.lstsq(C @ A @ V, C @ b, rcond=None)[0]
        xb = V @ y
        assert np.allclose(x, xb, atol=1e-9)
        r = b - A @ x
        assert hist[-1] == pytest.approx(np.sqrt(r @ P @ r) / np.sqrt(b @ P @ b), rel=1e-8)
        K.append(P @ A @ K[-1])
    x, its, hist = minres(lambda v: A @ v, lambda v: P @ v, b, 1e-13, 100)
    assert np.allclose(A @ x, b, atol=1e-10)
    assert its <= n + 3  # n steps in exact arithmetic; rounding may add a few
    assert all(hist[i + 1] <= hist[i] + 1e-15 for i in range(len(hist) - 1))


def test_minres_detects_indefinite_preconditioner():
    n = 6
    A = np.diag(np.arange(1.0, n + 1))
    P = np.diag([1, 1, 1, -1, -1, -1.0])
    with pytest.raises(Breakdown):
        minres(lambda v: A @ v, lambda v: P @ v, np.array([2, 2, 2, 1, 1, 1.0]), 1e-12, 50)


@pytest.mark.parametrize("mk", [lambda: W.make_c1(n_el=3, p=2),
                                lambda: W.make_c1(n_el=2, p=3, seed=4),
                                lambda: W.make_c2(n_el=2, p=2),
                                lambda: W.make_c3(n_el=2, p=2, grid=(2, 1, 2), seed=2)])
def test_solution_equals_conforming_galerkin(mk):
    s = AFIETI(mk())
    res = s.solve(tol=1e-12)
    uref = solve_conforming(s)
    assert np.linalg.norm(res["u"] - uref) <= 1e-10 * np.linalg.norm(uref)
    f = res["f"]
    r1 = s.apply_A(res["u"]) + s.B.T @ res["lam"] - f
    assert np.linalg.norm(r1) <= 1e-9 * np.linalg.norm(f)
    assert np.abs(s.B @ res["u"]).max() <= 1e-10 * np.abs(res["u"]).max()


def test_lambda_independent_of_lambda0(sys2):
    s = sys2
    base = s.solve(tol=1e-13)
    orig = s.lambda0
    extra = s.P_chi(np.random.default_rng(6).standard_normal(s.n_c))
    s.lambda0 = lambda f: orig(f) + extra
    try:
        other = s.solve(tol=1e-13)
    finally:
        s.lambda0 = orig
    assert np.allclose(other["u"], base["u"], atol=1e-10 * np.abs(base["u"]).max())
    assert np.allclose(other["lam"], base["lam"], atol=1e-8 * np.abs(base["lam"]).max())


def test_no_dirichlet_is_singular_coarse():
    prob = W.make_c1(n_el=2, p=2)
    for pd in prob["patches"]:
        pd["bc"] = [0] * 4
    with pytest.raises(SingularCoarse):
        AFIETI(prob)


def test_preconditioner_spd_on_subspace(sys2):
    s = sys2
    rng = np.random.default_rng(8)
    n = s.n_dof + s.n_c
    for _ in range(5):
        x = rng.standard_normal(n)
        x[:s.n_dof] = s.P_u(x[:s.n_dof])
        x[s.n_dof:] = s.P_chi(x[s.n_dof:])
        y = rng.standard_normal(n)
        y[:s.n_dof] = s.P_u(y[:s.n_dof])
        y[s.n_dof:] = s.P_chi(y[s.n_dof:])
        assert x @ s.apply_prec(x) > 0
        assert x @ s.apply_prec(y) == pytest.approx(y @ s.apply_prec(x), rel=1e-10)
