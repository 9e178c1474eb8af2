"""Pins of the geometry-inclusion local solvers of the oracle (Section
5.2.3, eq. geo_A, geo_S, tildeshur, inexact_S_non_r): the separable fit
against a brute-force least-squares solve, exactness on axis-aligned
boxes, the fast-diagonalization inverse against a dense solve of the
assembled Kronecker system, the diagonals against assembled matrices, the
Schur complement against its dense definition, and the whole solve against
the direct conforming solve."""
import numpy as np
import pytest

import workloads as W
from oracle.afieti import AFIETI
from oracle.direct import solve_conforming
from oracle import geo as G


def _kron(mats):
    out = np.ones((1, 1))
    for Ml in reversed(mats):
        out = np.kron(out, Ml)
    return out


def _dense_At(g, l, with_mass):
    b = g.blocks[l]
    d = g.pa.dim
    A = sum(_kron([b["K"][n] if n == m else b["M"][n] for n in range(d)]) for m in range(d))
    return A + g.h2 * _kron(b["M"]) if with_mass else A


def _perturbed(seed=3):
    prob = W.make_c2(n_el=2, p=2, seed=seed, delta=0.12)
    return AFIETI(prob, geometry=True)


def test_fit_equals_weighted_least_squares():
    """The closed-form fit minimises the weighted log-space residual: its
    fitted products equal those of a dense weighted least-squares solve
    (any minimiser: the gauge does not change the products)."""
    s = _perturbed()
    for pa in s.patches[:3]:
        d = pa.dim
        nq = [len(x) for x in pa.qx]
        Wg = G._grid_weights(pa).reshape(-1)
        for l in range(d):
            C, det = G.coefficient(pa, l)
            ys = [np.log(det).reshape(-1)] + [np.log(C[..., i, i]).reshape(-1) for i in range(d)]
            # unknowns: log nu_m (nq_m each) then log beta_m (nq_m each)
            off = np.concatenate([[0], np.cumsum(nq + nq)])
            idx = np.stack(np.meshgrid(*[np.arange(n) for n in reversed(nq)], indexing="ij"), -1)
            idx = idx.reshape(-1, d)[:, ::-1]               # idx[:, m] = q_m
            rows, rhs = [], []
            for i in range(d + 1):
                A = np.zeros((len(Wg), off[-1]))
                for m in range(d):
                    if i == 1 + m:
                        A[np.arange(len(Wg)), off[m] + idx[:, m]] = 1.0
                    else:
                        A[np.arange(len(Wg)), off[d + m] + idx[:, m]] = 1.0
                rows.append(A * np.sqrt(Wg)[:, None])
                rhs.append(ys[i] * np.sqrt(Wg))
            x = np.linalg.lstsq(np.vstack(rows), np.concatenate(rhs), rcond=None)[0]
            nu_ls = [np.exp(x[off[m]:off[m + 1]]) for m in range(d)]
            be_ls = [np.exp(x[off[d + m]:off[d + m + 1]]) for m in range(d)]
            nu, be = G.separable_fit(pa, l)
            for i in range(d):
                P1 = G._outer_prod([nu[m] if m == i else be[m] for m in range(d)])
                P2 = G._outer_prod([nu_ls[m] if m == i else be_ls[m] for m in range(d)])
                assert np.abs(P1 - P2).max() <= 1e-12 * np.abs(P2).max()
            assert np.allclose(G._outer_prod(be), G._outer_prod(be_ls), rtol=1e-12)
            # and the residual is not zero on a perturbed patch (the fit is a fit)
            Cf = G._outer_prod([nu[m] if m == 0 else be[m] for m in range(d)])
            assert np.abs(np.log(Cf) - np.log(C[..., 0, 0])).max() > 1e-6


@pytest.mark.parametrize("sides", [(1.0, 1.0, 1.0), (0.5, 2.0, 1.5)])
def test_exact_on_axis_aligned_boxes(sides):
    """On a box [0,a]x[0,b]x[0,c] C_l is diagonal and constant, the fit is
    exact, D_A = D_S = 1, and the FD block is the exact inverse of
    A_ll + H^-2 M (A from the assembled physical stiffness)."""
    a, b, c = sides
    corners = np.array([[x * a, y * b, z * c] for z in (0, 1) for y in (0, 1) for x in (0, 1)], dtype=float)
    pd = dict(p=2, reg=1, n_el=[2, 3, 2], corners=corners, lam=0.7, mu=1.3, bc=[0, 0, 0, 0, 1, 0])
    prob = dict(dim=3, patches=[pd], load=[(0, 1.0, [1, 1, 1], [0.0, 0.0, 0.0])], tol=1e-8)
    s = AFIETI(prob, geometry=True)
    g, pa = s.geo.patches[0], s.patches[0]
    A = pa.stiffness_matrix().toarray()
    Mm = pa.mass_matrix_scalar().toarray()
    nn = pa.n_nodes
    for l in range(3):
        blk = g.blocks[l]
        assert np.allclose(blk["DA"], 1.0, rtol=1e-12) and np.allclose(blk["DS"], 1.0, rtol=1e-12)
        All = A[l * nn:(l + 1) * nn, l * nn:(l + 1) * nn] + g.h2 * Mm
        r = W.random_vector(nn, l).reshape(pa.shape)
        z = g.PA_inv(l, r)
        ref = np.linalg.solve(All, r.reshape(-1)).reshape(pa.shape)
        assert np.abs(z - ref).max() <= 1e-12 * np.abs(ref).max()


def test_fd_equals_dense_kronecker_solve():
    s = _perturbed()
    for g in s.geo.patches[:2]:
        for l in range(3):
            blk = g.blocks[l]
            A = _dense_At(g, l, True)
            r = W.random_vector(A.shape[0], 5 + l)
            dA = blk["DA"].reshape(-1)
            ref = np.linalg.solve(np.sqrt(dA)[:, None] * A * np.sqrt(dA)[None, :], r)
            z = g.PA_inv(l, r.reshape(g.pa.shape)).reshape(-1)
            assert np.abs(z - ref).max() <= 1e-11 * np.abs(ref).max()
            assert blk["DA"].min() > 0 and blk["DS"].min() > 0


def test_diagonals_match_assembled_matrices():
    s = _perturbed()
    for g, pa in zip(s.geo.patches[:2], s.patches[:2]):
        A = pa.stiffness_matrix().diagonal()
        Md = pa.mass_matrix_scalar().diagonal()
        nn = pa.n_nodes
        assert np.abs(G.mass_diagonal(pa).reshape(-1) - Md).max() <= 1e-14 * Md.max()
        for l in range(3):
            ref = A[l * nn:(l + 1) * nn]
            assert np.abs(g.blocks[l]["A_diag"].reshape(-1) - ref).max() <= 1e-13 * ref.max()
            At = np.diag(_dense_At(g, l, False))
            assert np.abs(g.blocks[l]["At_diag"].reshape(-1) - At).max() <= 1e-13 * At.max()


def test_schur_complement_equals_dense():
    s = _perturbed()
    g = s.geo.patches[1]
    pa = g.pa
    gm = pa.gamma_mask().reshape(-1)
    Gi, Ii = np.nonzero(gm)[0], np.nonzero(~gm)[0]
    for l in range(3):
        A = _dense_At(g, l, False)
        S = A[np.ix_(Gi, Gi)] - A[np.ix_(Gi, Ii)] @ np.linalg.solve(A[np.ix_(Ii, Ii)], A[np.ix_(Ii, Gi)])
        th = W.random_vector(pa.n_nodes, 9 + l)
        y = g.apply_St(l, th.reshape(pa.shape)).reshape(-1)
        ref = S @ th[Gi]
        assert np.abs(y[Gi] - ref).max() <= 1e-11 * np.abs(ref).max()
        assert np.all(y[Ii] == 0)
        # the scaled block is symmetric
        x1, x2 = W.random_vector(pa.n_nodes, 1), W.random_vector(pa.n_nodes, 2)
        a = g.S_block(l, x1.reshape(pa.shape)).reshape(-1)[Gi] @ x2[Gi]
        b = g.S_block(l, x2.reshape(pa.shape)).reshape(-1)[Gi] @ x1[Gi]
        assert abs(a - b) <= 1e-12 * abs(a)


def test_preconditioner_symmetric_positive_definite():
    prob = W.make_c1(n_el=3, p=2, seed=2)
    s = AFIETI(prob, geometry=True)
    n = s.n_dof + s.n_c
    X = np.array([s.apply_prec(e) for e in np.eye(n)]).T
    assert np.abs(X - X.T).max() <= 1e-12 * np.abs(X).max()
    # positive definite on the ranges of P_u and P_chi
    Pu = np.array([s.P_u(e) for e in np.eye(s.n_dof)]).T
    Pc = np.array([s.P_chi(e) for e in np.eye(s.n_c)]).T
    Zu = sla_orth(Pu)
    Zc = sla_orth(Pc)
    ew = np.linalg.eigvalsh(Zu.T @ X[:s.n_dof, :s.n_dof] @ Zu)
    ec = np.linalg.eigvalsh(Zc.T @ X[s.n_dof:, s.n_dof:] @ Zc)
    assert ew.min() > 0 and ec.min() > 0


def sla_orth(P):
    import scipy.linalg as sla
    return sla.orth(P)


@pytest.mark.parametrize("mk", [lambda: W.make_c1(n_el=4, p=3, seed=1),
                                lambda: W.make_c3(n_el=2, p=2, grid=(2, 2, 1), seed=5)])
def test_geometry_solve_reproduces_direct(mk):
    prob = mk()
    s = AFIETI(prob, geometry=True)
    res = s.solve(tol=1e-12)
    ud = solve_conforming(s)
    assert np.abs(res["u"] - ud).max() <= 1e-9 * np.abs(ud).max()
