"""Pins of the oracle's exact local solvers (Section 5.1, eq. exact_AP,
exact_SP; Remark 1, eq. S_non_r): dense inverses and Schur complements on
small patches, the Schur complement annihilates rigid-mode traces, the
solve equals the direct conforming solve, and the inexact solvers need
more iterations than the exact ones (the paper's comparison)."""
import numpy as np
import pytest

import workloads as W
from oracle.afieti import AFIETI
from oracle.direct import solve_conforming


def test_pa_inverse_and_schur_equal_dense():
    prob = W.make_c2(n_el=2, p=2, seed=4, delta=0.1)
    s = AFIETI(prob, exact=True)
    for k in (0, 5):
        e, pa = s.geo.patches[k], s.patches[k]
        A = s.A[k].toarray()
        Ms = pa.mass_matrix_scalar().toarray()
        M = np.kron(np.eye(3), Ms)
        r = W.random_vector(pa.n_dof, k)
        ref = np.linalg.solve(A + pa.diameter() ** -2 * M, r)
        assert np.abs(e.PA_inv(r) - ref).max() <= 1e-11 * np.abs(ref).max()
        G, I = e.G, e.I
        S = A[np.ix_(G, G)] - A[np.ix_(G, I)] @ np.linalg.solve(A[np.ix_(I, I)], A[np.ix_(I, G)])
        th = W.random_vector(pa.n_dof, 10 + k)
        y = e.S(th)
        assert np.abs(y[G] - S @ th[G]).max() <= 1e-11 * np.abs(S @ th[G]).max()
        assert np.all(y[I] == 0)
        # rigid modes: A R = 0, so their traces are in the kernel of S
        for mode in pa.rigid_modes():
            t = e.S(mode)
            assert np.abs(t).max() <= 1e-10 * np.abs(A).max() * np.abs(mode).max()


@pytest.mark.parametrize("mk", [lambda: W.make_c1(n_el=4, p=2, seed=1),
                                lambda: W.make_c3(n_el=2, p=3, grid=(2, 2, 1), seed=5)])
def test_exact_solve_reproduces_direct(mk):
    prob = mk()
    s = AFIETI(prob, exact=True)
    res = s.solve(tol=1e-12)
    ud = solve_conforming(s)
    assert np.abs(res["u"] - ud).max() <= 1e-9 * np.abs(ud).max()


@pytest.mark.parametrize("mk", [lambda: W.make_c1(n_el=8, p=2, seed=1),
                                lambda: W.make_c3(n_el=3, p=2, grid=(2, 2, 2), seed=3)])
def test_inexact_needs_more_iterations_than_exact(mk):
    """The exact local solvers are the ideal choice (Section 5.1): the
    inexact ones, parametric or with geometry inclusion, take more MINRES
    iterations (the paper reports 1.6 to 2.3 times as many)."""
    prob = mk()
    its = {name: AFIETI(prob, **kw).solve(tol=1e-8)["iters"]
           for name, kw in (("exact", dict(exact=True)), ("fd", {}), ("geo", dict(geometry=True)))}
    print(its)
    assert its["exact"] < its["geo"] <= its["fd"] * 1.05
    assert its["fd"] <= 4 * its["exact"]
