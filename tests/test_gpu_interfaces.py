"""Explicit interface lists on the GPU (Section 2.2): cracked patch grids
(coinciding faces that are not listed stay apart) and a patch glued to a
rotated neighbour, through the C ABI against the oracle — jump operator,
preconditioner and the solves, under the same rules as the other parity
tests; the cracked solve also agrees with the oracle's direct conforming
solve of the cracked body."""
import numpy as np
import pytest

import workloads as W
from oracle.afieti import AFIETI
from oracle.direct import solve_conforming
from minres_band import iterate_bound, same_iterations

pytestmark = pytest.mark.gpu

CASES = {
    "cracked2d": lambda: W.make_cracked(2, n_el=6, p=2),
    "cracked3d": lambda: W.make_cracked(3, n_el=3, p=2),
}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("name", list(CASES))
def test_operators(name):
    torch = _torch()
    from paper_2001_09626_amd import Solver
    print(f"\n[{name}]", flush=True)
    prob = CASES[name]()
    o = AFIETI(prob)
    s = Solver(prob, tol=1e-8)
    x = W.random_vector(o.n_dof, 1)
    eb = _rel(_host(s.apply("B", torch.from_numpy(x).cuda())), o.B @ x)
    r = W.random_vector(o.n_dof + o.n_c, 2)
    ep = _rel(_host(s.apply("prec", torch.from_numpy(r).cuda())), o.apply_prec(r))
    ea = _rel(_host(s.apply("saddle", torch.from_numpy(r).cuda())), o.apply_op(r))
    print(f"  B {eb:.2e}, prec {ep:.2e}, saddle {ea:.2e}", flush=True)
    assert eb == 0 and ep <= 1e-11 and ea <= 1e-12
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_solve(name):
    _torch()
    from paper_2001_09626_amd import Solver
    prob = CASES[name]()
    o = AFIETI(prob)
    ref = o.solve(tol=1e-8, maxit=5000)
    alt = AFIETI(prob, eig_driver="gv").solve(tol=1e-8, maxit=5000)
    exact = solve_conforming(o)
    s = Solver(prob, tol=1e-8)
    u, _, st = s.solve()
    u = _host(u)
    nu = np.linalg.norm(exact)
    diff = np.linalg.norm(u - ref["u"]) / nu
    own = np.linalg.norm(ref["u"] - exact) / nu
    pair = np.linalg.norm(alt["u"] - ref["u"]) / nu
    print(f"  {name}: iterations gpu {st['iterations']} oracle {ref['iters']} (other driver {alt['iters']}); "
          f"|u-u_or| {diff:.2e}, own {own:.2e}, pair {pair:.2e}", flush=True)
    assert st["converged"] and same_iterations(st["iterations"], ref, 1e-8, alt=alt)
    assert diff <= iterate_bound(own, pair)
    s.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_rotated_neighbour(dim):
    _torch()
    from paper_2001_09626_amd import Solver
    prob, pair, orient = W.make_rotated_pair(dim)
    listed = dict(prob, interfaces=[pair + (orient,)])
    o = AFIETI(prob)
    exact = solve_conforming(o)
    a = Solver(prob, tol=1e-12)
    b = Solver(listed, tol=1e-12)
    ua, _, sa = a.solve()
    ub, _, sb = b.solve()
    ua, ub = _host(ua), _host(ub)
    e = _rel(ub, exact)
    print(f"  dim {dim}: matched {sa['iterations']} it, listed {sb['iterations']} it, "
          f"|u-u_direct| {e:.2e}", flush=True)
    assert np.array_equal(ua, ub) and e <= 1e-9
    a.close()
    b.close()
