"""Non-conforming nested interfaces in the oracle (Section 2.2; the
non-conforming test of Section 6): knot insertion, the gluing rows of B and
the AF-IETI solve on the paper's three-cube box with 4, 8 and 16 elements
per direction.

Pins (none re-types the construction):
  * T for p = 1 and one inserted midpoint, by hand;
  * T is a partition of unity with nonnegative entries, and each coarse
    B-spline equals its T-combination of fine B-splines at random points;
  * the saddle-form direct solve equals the conforming direct solve on a
    conforming problem;
  * a linear displacement (Dirichlet data on the whole boundary, no body
    force) is reproduced exactly by the glued non-conforming space;
  * the glued solution takes one value on both sides of an interface at
    random interface points;
  * the error against the smooth exact solution falls under refinement;
  * the iterative AF-IETI solve reaches the direct solution."""
import numpy as np
import pytest

import workloads as W
from oracle import bspline
from oracle.afieti import AFIETI
from oracle.direct import solve_conforming, solve_kkt
from oracle.nonconforming import is_nested, knot_insertion


def test_knot_insertion_p1_by_hand():
    T = knot_insertion([0, 0, 1, 1], [0, 0, 0.5, 1, 1], 1)
    assert np.allclose(T, [[1, 0], [0.5, 0.5], [0, 1]], atol=1e-15)


@pytest.mark.parametrize("p,coarse_el,fine", [(2, 3, None), (3, 4, None), (3, 2, [0.1, 0.25, 0.5, 0.7, 0.9])])
def test_knot_insertion_properties(p, coarse_el, fine):
    cknots = bspline.open_uniform_knots(coarse_el, p, p - 1)
    if fine is None:
        fknots = bspline.open_uniform_knots(2 * coarse_el, p, p - 1)
    else:
        inner = sorted(set(np.round(cknots[p + 1:-p - 1], 15)) | set(fine))
        fknots = np.concatenate([[0.0] * (p + 1), inner, [1.0] * (p + 1)])
    assert is_nested(cknots, fknots) and not is_nested(fknots, cknots)
    T = knot_insertion(cknots, fknots, p)
    assert np.allclose(T.sum(axis=1), 1.0, atol=1e-14)
    assert T.min() >= -1e-14
    x = np.random.default_rng(p).uniform(0, 1, 200)
    Bc, Bf = bspline.basis(cknots, p, x), bspline.basis(fknots, p, x)
    assert np.abs(Bf @ T - Bc).max() <= 1e-13


def test_kkt_equals_conforming_solve():
    o = AFIETI(W.make_c1(n_el=4, p=2, seed=3))
    a, b = solve_conforming(o), solve_kkt(o)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def _field(pa, coef, eta):
    """Spline field of one patch (coefficients (dim, n_d..n_1)) at
    parametric points eta (n, dim)."""
    Bs = [bspline.basis(pa.knots[l], pa.p, eta[:, l]) for l in range(pa.dim)]
    out = []
    for c in range(pa.dim):
        C = coef[c]
        if pa.dim == 2:
            out.append(np.einsum("ji,nj,ni->n", C, Bs[1], Bs[0]))
        else:
            out.append(np.einsum("kji,nk,nj,ni->n", C, Bs[2], Bs[1], Bs[0]))
    return np.stack(out, axis=1)


@pytest.mark.parametrize("dim,n_els,p", [(2, (1, 2, 4), 2), (3, (1, 2, 4), 2), (2, (2, 4, 8), 3)])
def test_linear_field_reproduced(dim, n_els, p):
    prob = W.make_nonconforming(p=p, n_els=n_els, dim=dim)
    A = np.random.default_rng(7).normal(size=(dim, dim))
    b = np.arange(1, dim + 1) * 0.1
    prob["dirichlet"] = lambda x: x @ A.T + b
    prob["body_force"] = None
    o = AFIETI(prob)
    assert len(o.nonconforming) == 2
    u = o.split(solve_kkt(o))
    for pa, uk in zip(o.patches, u):
        X = pa.ctrl.reshape(-1, dim)
        ref = X @ A.T + b
        got = uk.reshape(dim, -1).T
        assert np.abs(got - ref).max() <= 1e-11


@pytest.mark.parametrize("dim", [2, 3])
def test_glued_solution_continuous(dim):
    prob = W.make_nonconforming(p=2, n_els=(1, 2, 4) if dim == 3 else (2, 4, 8), dim=dim)
    o = AFIETI(prob)
    u = o.split(solve_kkt(o))
    rng = np.random.default_rng(1)
    for k in range(2):  # interfaces y = 1 and y = 2
        eta = rng.uniform(0, 1, (50, dim))
        lo, hi = eta.copy(), eta.copy()
        lo[:, 1], hi[:, 1] = 1.0, 0.0
        a = _field(o.patches[k], u[k], lo)
        b = _field(o.patches[k + 1], u[k + 1], hi)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def _error(prob, o, u):
    rng = np.random.default_rng(2)
    err = 0.0
    for k, (pa, uk) in enumerate(zip(o.patches, o.split(u))):
        eta = rng.uniform(0, 1, (200, o.dim))
        x = eta.copy()
        x[:, 1] += k
        err = max(err, np.abs(_field(pa, uk, eta) - prob["exact"](x)).max())
    return err


def test_refinement_reduces_error():
    errs = []
    for n_els in [(2, 4, 8), (4, 8, 16), (8, 16, 32)]:
        prob = W.make_nonconforming(p=2, n_els=n_els, dim=2)
        o = AFIETI(prob)
        errs.append(_error(prob, o, solve_kkt(o)))
    print(f"  max errors {errs}")
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3


@pytest.mark.parametrize("dim,n_els,p", [(2, (2, 4, 8), 2), (3, (1, 2, 4), 2)])
def test_afieti_reaches_direct_solution(dim, n_els, p):
    prob = W.make_nonconforming(p=p, n_els=n_els, dim=dim)
    o = AFIETI(prob)
    ref = solve_kkt(o)
    r = o.solve(tol=1e-10, maxit=2000)
    rg = AFIETI(prob, geometry=True).solve(tol=1e-10, maxit=2000)
    rx = AFIETI(prob, exact=True).solve(tol=1e-10, maxit=2000)
    e = [np.linalg.norm(x["u"] - ref) / np.linalg.norm(ref) for x in (r, rg, rx)]
    print(f"  iterations: FD {r['iters']}, geometry inclusion {rg['iters']}, exact {rx['iters']}; errors {e}")
    assert max(e) <= 1e-7
    assert rx["iters"] < r["iters"]
