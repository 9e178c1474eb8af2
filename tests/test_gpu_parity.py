"""GPU parity: every operator of the hot path, called through the C ABI on
the device, against the CPU oracle on the same seeded inputs, element by
element.  FP64 operators to 1e-12 relative to the largest entry (sums of at
most a few thousand products in a different order).

Solves: at tolerance 1e-8 the GPU and the oracle take the same number of
MINRES iterations (or stop apart where the oracle's own stopping estimate
sits within 10 % of the tolerance, tests/minres_band.py) and their iterates
differ by less than the rounding sensitivity of the iteration allows: a
tenth of the iterate's own distance to the converged solution, or four
times the distance between two oracle runs that differ only in LAPACK's
eigensolver driver, whichever is larger (tests/minres_band.py); at
tolerance 1e-12 the two solutions agree to 1e-10 relative (measured: at
most 2e-13) with iteration counts under the band rule."""
import numpy as np
import pytest

import workloads as W
from oracle.afieti import AFIETI
from minres_band import iterate_bound, same_iterations

pytestmark = pytest.mark.gpu

CASES = {
    "c1_small": lambda: W.make_c1(n_el=5, p=2, seed=3),
    "c1_p3": lambda: W.make_c1(n_el=3, p=3, seed=1),
    "c2_small": lambda: W.make_c2(n_el=4, p=3, seed=2),
    "c3_ragged": lambda: W.make_c3(n_el=3, p=2, grid=(2, 3, 2), seed=4),
}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module", params=list(CASES))
def pair(request):
    torch = _torch()
    from paper_2001_09626_amd import Solver
    print(f"\n[case {request.param}]", flush=True)
    prob = CASES[request.param]()
    o = AFIETI(prob)
    s = Solver(prob, tol=1e-8)
    yield request.param, prob, o, s, torch
    s.close()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _close(a, b, rtol):
    scale = max(np.abs(b).max(), 1e-300)
    err = np.abs(a - b).max() / scale
    print(f"  max rel err {err:.3e} (bound {rtol:.1e})", flush=True)
    assert err <= rtol, f"max rel err {err:.3e} > {rtol:.1e}"


def _per_tensor(o, x, fn):
    out = []
    for k, xk in enumerate(o.split(x)):
        out.append(np.array([fn(k, l, xk[l]) for l in range(o.dim)]))
    return o.join(out)


def test_fd_apply(pair):
    name, prob, o, s, torch = pair
    r = W.random_vector(o.n_dof, 10)
    z = _host(s.apply_fd(_dev(torch, r)))
    _close(z, o.apply_PA_inv(r), 1e-12)


def test_stiffness(pair):
    name, prob, o, s, torch = pair
    x = W.random_vector(o.n_dof, 11)
    _close(_host(s.apply("stiffness", _dev(torch, x))), o.apply_A(x), 1e-12)


def test_load(pair):
    name, prob, o, s, torch = pair
    _close(_host(s.apply("load")), o.load(), 1e-12)


def test_jump(pair):
    name, prob, o, s, torch = pair
    x = W.random_vector(o.n_dof, 12)
    y = W.random_vector(o.n_c, 13)
    _close(_host(s.apply("B", _dev(torch, x))), o.B @ x, 1e-15)
    _close(_host(s.apply("Bt", _dev(torch, y))), o.B.T @ y, 1e-15)


def test_projections(pair):
    name, prob, o, s, torch = pair
    x = W.random_vector(o.n_dof, 14)
    y = W.random_vector(o.n_c, 15)
    _close(_host(s.apply("P_u", _dev(torch, x))), o.P_u(x), 1e-12)
    _close(_host(s.apply("P_chi", _dev(torch, y))), o.P_chi(y), 1e-12)


def test_ahat_and_interior_fd(pair):
    name, prob, o, s, torch = pair
    x = W.random_vector(o.n_dof, 16)
    _close(_host(s.apply("Ahat", _dev(torch, x))), _per_tensor(o, x, o.apply_Ahat), 1e-12)
    ref = []
    for k, xk in enumerate(o.split(x)):
        inner = tuple(slice(1, -1) for _ in range(o.dim))
        blk = np.zeros_like(xk)
        for l in range(o.dim):
            blk[l][inner] = o.fd_solve_interior(k, l, xk[l][inner])
        ref.append(blk)
    _close(_host(s.apply("fd_interior", _dev(torch, x))), o.join(ref), 1e-12)


def test_schur(pair):
    name, prob, o, s, torch = pair
    x = W.random_vector(o.n_dof, 17)
    ref = _per_tensor(o, x, lambda k, l, t: o.patches[k].diameter() ** (o.dim - 2) * o.apply_Shat(k, l, t))
    _close(_host(s.apply("Shat", _dev(torch, x))), ref, 1e-11)
    y = W.random_vector(o.n_c, 18)
    _close(_host(s.apply("P_S", _dev(torch, y))), o.apply_PS(y), 1e-11)


def test_preconditioner_and_operator(pair):
    name, prob, o, s, torch = pair
    r = W.random_vector(o.n_dof + o.n_c, 19)
    _close(_host(s.apply("prec", _dev(torch, r))), o.apply_prec(r), 1e-11)
    _close(_host(s.apply("saddle", _dev(torch, r))), o.apply_op(r), 1e-12)


def test_solve_matches_oracle(pair):
    name, prob, o, s, torch = pair
    ref = o.solve()
    tight = o.solve(tol=1e-13)
    alt = AFIETI(prob, eig_driver="gv").solve()
    u, lam, st = s.solve()
    u, lam = _host(u), _host(lam)
    nu = np.linalg.norm(ref["u"])
    diff = np.linalg.norm(u - ref["u"]) / nu
    own = np.linalg.norm(ref["u"] - tight["u"]) / nu
    pair = np.linalg.norm(alt["u"] - ref["u"]) / nu
    dl = np.linalg.norm(lam - ref["lam"]) / np.linalg.norm(ref["lam"])
    print(f"  iterations gpu {st['iterations']} oracle {ref['iters']}; |u-u_or| {diff:.2e}, "
          f"|u_or-u*| {own:.2e}, oracle pair {pair:.2e}, |lam-lam_or| {dl:.2e}", flush=True)
    assert st["converged"]
    assert same_iterations(st["iterations"], ref, 1e-8, alt=alt)
    assert diff <= iterate_bound(own, pair) and diff <= 1e-8
    assert dl <= 1e-7


def test_solve_tight_matches_oracle_1e10(pair):
    name, prob, o, s, torch = pair
    from paper_2001_09626_amd import Solver
    st_ = Solver(prob, tol=1e-12)
    ref = o.solve(tol=1e-12)
    alt = AFIETI(prob, eig_driver="gv").solve(tol=1e-12)
    ext = o.solve(tol=1e-14, maxit=len(ref["history"]) + 20)
    alt_ext = AFIETI(prob, eig_driver="gv").solve(tol=1e-14, maxit=len(ref["history"]) + 20)
    u, lam, st = st_.solve()
    u, lam = _host(u), _host(lam)
    diff = np.linalg.norm(u - ref["u"]) / np.linalg.norm(ref["u"])
    dl = np.linalg.norm(lam - ref["lam"]) / np.linalg.norm(ref["lam"])
    print(f"  tol 1e-12: iterations gpu {st['iterations']} oracle {ref['iters']}; rel diff u {diff:.2e} "
          f"lam {dl:.2e}", flush=True)
    assert same_iterations(st["iterations"], ref, 1e-12, alt=alt, ext=ext, alt_ext=alt_ext)
    assert diff <= 1e-10 and dl <= 1e-9
    st_.close()


def test_fp32_fd_solve_close_to_fp64_oracle(pair):
    name, prob, o, s, torch = pair
    from paper_2001_09626_amd import Solver
    s32 = Solver(prob, tol=1e-8, fd_precision="fp32")
    ref = o.solve()
    tight = o.solve(tol=1e-13)
    u, lam, st = s32.solve()
    u = _host(u)
    nu = np.linalg.norm(tight["u"])
    e32 = np.linalg.norm(u - tight["u"]) / nu
    e64 = np.linalg.norm(ref["u"] - tight["u"]) / nu
    print(f"  FP32-FD: {st['iterations']} it (FP64 oracle {ref['iters']}); error vs converged "
          f"{e32:.2e} (FP64-FD iterate {e64:.2e})", flush=True)
    assert st["converged"]
    assert abs(st["iterations"] - ref["iters"]) <= max(3, ref["iters"] // 20)
    assert e32 <= 3 * e64 + 1e-12
    s32.close()


def test_solve_bitwise_repeatable(pair):
    name, prob, o, s, torch = pair
    u1, l1, st1 = s.solve()
    u2, l2, st2 = s.solve()
    assert torch.equal(u1, u2) and torch.equal(l1, l2)
    assert st1["iterations"] == st2["iterations"]


def test_solve_with_rhs(pair):
    name, prob, o, s, torch = pair
    f = W.random_vector(o.n_dof, 20)
    ref = o.solve(rhs=f)
    alt = AFIETI(prob, eig_driver="gv").solve(rhs=f)
    tight = o.solve(rhs=f, tol=1e-13)
    u, lam, st = s.solve(rhs=_dev(torch, f))
    nu = np.linalg.norm(ref["u"])
    diff = np.linalg.norm(_host(u) - ref["u"]) / nu
    own = np.linalg.norm(ref["u"] - tight["u"]) / nu
    print(f"  rhs: iterations {st['iterations']} / {ref['iters']}; diff {diff:.2e} own {own:.2e}")
    pair = np.linalg.norm(alt["u"] - ref["u"]) / nu
    assert same_iterations(st["iterations"], ref, 1e-8, alt=alt)
    assert diff <= iterate_bound(own, pair)


@pytest.mark.parametrize("case", ["c1_small", "c2_small"])
def test_plain_ps_variant_matches_oracle(case):
    """The plain inexact P_S (no (B B^T)^{-1} scaling) as a switch: P_S and the
    preconditioner against the oracle's "plain" variant, and the solve."""
    torch = _torch()
    from paper_2001_09626_amd import Solver
    prob = CASES[case]()
    o = AFIETI(prob)
    s = Solver(prob, tol=1e-8, ps_variant="plain")
    y = W.random_vector(o.n_c, 31)
    _close(_host(s.apply("P_S", _dev(torch, y))), o.apply_PS(y, "plain"), 1e-11)
    r = W.random_vector(o.n_dof + o.n_c, 32)
    _close(_host(s.apply("prec", _dev(torch, r))), o.apply_prec(r, "plain"), 1e-11)
    ref = o.solve(variant="plain")
    alt = AFIETI(prob, eig_driver="gv").solve(variant="plain")
    u, lam, st = s.solve()
    diff = np.linalg.norm(_host(u) - ref["u"]) / np.linalg.norm(ref["u"])
    print(f"  plain P_S: {st['iterations']} it (oracle {ref['iters']}), rel diff u {diff:.2e}", flush=True)
    assert st["converged"] and same_iterations(st["iterations"], ref, 1e-8, alt=alt)
    assert diff <= 1e-8
    s.close()
