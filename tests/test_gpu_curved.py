"""Explicit control nets on the GPU: a curved domain (a quarter of a thick
cylinder in B-spline patches) through the C ABI against the oracle —
stiffness (assembled: the matrix-free kernel needs the corners' multilinear
map), preconditioners with parametric FD and with geometry inclusion, and
the solves; and a net that reproduces a multilinear map gives the solution
of the corners' description.  Same rules as the other parity tests."""
import copy

import numpy as np
import pytest

import workloads as W
from oracle.afieti import AFIETI
from minres_band import iterate_bound, same_iterations

pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def curved():
    _torch()
    print("\n[curved: quarter thick cylinder, 2x2x2 patches, 3^3 elements, p=2]", flush=True)
    return W.make_curved(n_el=3, p=2)


@pytest.mark.parametrize("precond", ["fd", "geo"])
def test_operators(curved, precond):
    torch = _torch()
    from paper_2001_09626_amd import Solver
    o = AFIETI(curved, geometry=precond == "geo")
    s = Solver(curved, tol=1e-8, precond=precond)
    assert s.stiffness_bytes > 0  # assembled
    x = W.random_vector(o.n_dof, 1)
    e = _rel(_host(s.apply("stiffness", torch.from_numpy(x).cuda())), o.apply_A(x))
    r = W.random_vector(o.n_dof + o.n_c, 2)
    ep = _rel(_host(s.apply("prec", torch.from_numpy(r).cuda())), o.apply_prec(r))
    el = _rel(_host(s.apply("load")), o.load())
    print(f"  {precond}: stiffness {e:.2e}, prec {ep:.2e}, load {el:.2e}", flush=True)
    assert e <= 1e-12 and ep <= 1e-11 and el <= 1e-12
    s.close()


@pytest.mark.parametrize("precond", ["fd", "geo"])
def test_solve(curved, precond):
    _torch()
    from paper_2001_09626_amd import Solver
    kw = dict(geometry=precond == "geo")
    o = AFIETI(curved, **kw)
    ref = o.solve(tol=1e-8, maxit=5000)
    alt = AFIETI(curved, eig_driver="gv", **kw).solve(tol=1e-8, maxit=5000)
    tight = o.solve(tol=1e-13, maxit=5000)
    s = Solver(curved, tol=1e-8, precond=precond)
    u, _, st = s.solve()
    u = _host(u)
    nu = np.linalg.norm(tight["u"])
    diff = np.linalg.norm(u - ref["u"]) / nu
    own = np.linalg.norm(ref["u"] - tight["u"]) / nu
    pair = np.linalg.norm(alt["u"] - ref["u"]) / nu
    print(f"  {precond}: iterations gpu {st['iterations']} oracle {ref['iters']} (other driver {alt['iters']}); "
          f"|u-u_or| {diff:.2e}, own {own:.2e}, pair {pair:.2e}", flush=True)
    assert st["converged"] and same_iterations(st["iterations"], ref, 1e-8, alt=alt)
    assert diff <= iterate_bound(own, pair)
    s.close()


def test_net_of_multilinear_map_equals_corners():
    torch = _torch()
    from paper_2001_09626_amd import Solver
    prob = W.make_c2(n_el=3, p=2, seed=4)
    net = copy.deepcopy(prob)
    for pa, pd in zip(AFIETI(prob).patches, net["patches"]):
        pd["ctrl"] = pa.ctrl.copy()
        del pd["corners"]
    a = Solver(prob, tol=1e-12)
    b = Solver(net, tol=1e-12)
    ua, _, sa = a.solve()
    ub, _, sb = b.solve()
    e = _rel(_host(ub), _host(ua))
    print(f"  corners {sa['iterations']} it, net {sb['iterations']} it, rel diff {e:.2e}", flush=True)
    assert e <= 1e-10
    a.close()
    b.close()
    del torch
