"""GPU parity at the benchmark's full size (3D unit cube, 2x2x2 patches,
p=3 C^2, 32^3 elements per patch, 1,029,000 DOF), in the launch
configuration bench.py times.  The oracle computes the FD apply, the
preconditioner and the jump operators in full, the stiffness product on
sampled patches, and checks the solve through the saddle equations it must
satisfy."""
import numpy as np
import pytest

import workloads as W
from oracle.afieti import AFIETI

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_09626_amd import Solver
    prob = W.make_c2(seed=0)
    print("\n[full-size c2: setup]", flush=True)
    s64 = Solver(prob, tol=1e-8, fd_precision="fp64")
    s32 = Solver(prob, tol=1e-8, fd_precision="fp32")
    o = AFIETI(prob)
    yield prob, o, s64, s32, torch
    s64.close()
    s32.close()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_fd_full(full):
    prob, o, s64, s32, torch = full
    r = W.random_vector(o.n_dof, 21)
    ref = o.apply_PA_inv(r)
    e64 = _rel(_host(s64.apply_fd(_dev(torch, r))), ref)
    e32 = _rel(_host(s32.apply_fd(_dev(torch, r))), ref)
    print(f"  FD fp64 {e64:.2e}  fp32 {e32:.2e}", flush=True)
    assert e64 <= 1e-12
    # FP32 mode products: two passes of n = 35 term sums per mode, 3 modes,
    # unit round-off 6e-8 -> a few 1e-6 relative to the largest entry
    assert e32 <= 2e-5


def test_preconditioner_full(full):
    prob, o, s64, s32, torch = full
    r = W.random_vector(o.n_dof + o.n_c, 22)
    e = _rel(_host(s64.apply("prec", _dev(torch, r))), o.apply_prec(r))
    print(f"  prec {e:.2e}", flush=True)
    assert e <= 1e-11


def test_jump_and_projection_full(full):
    prob, o, s64, s32, torch = full
    x = W.random_vector(o.n_dof, 23)
    y = W.random_vector(o.n_c, 24)
    assert _rel(_host(s64.apply("B", _dev(torch, x))), o.B @ x) <= 1e-15
    assert _rel(_host(s64.apply("Bt", _dev(torch, y))), o.B.T @ y) <= 1e-15
    assert _rel(_host(s64.apply("P_chi", _dev(torch, y))), o.P_chi(y)) <= 1e-12
    assert _rel(_host(s64.apply("P_u", _dev(torch, x))), o.P_u(x)) <= 1e-12


def test_stiffness_sampled_patches(full):
    prob, o, s64, s32, torch = full
    x = W.random_vector(o.n_dof, 25)
    y = _host(s64.apply("stiffness", _dev(torch, x)))
    xs, ys = o.split(x), o.split(y)
    for k in (0, 7):
        ref = o.patches[k].stiffness_apply(xs[k])
        e = _rel(ys[k], ref)
        print(f"  stiffness patch {k}: {e:.2e}", flush=True)
        assert e <= 1e-12


def test_load_full(full):
    prob, o, s64, s32, torch = full
    assert _rel(_host(s64.apply("load")), o.load()) <= 1e-12


def test_solve_saddle_equations_full(full):
    prob, o, s64, s32, torch = full
    f = o.load()
    for name, s in (("fp64", s64), ("fp32", s32)):
        u, lam, st = s.solve()
        u, lam = _host(u), _host(lam)
        Bu = np.abs(o.B @ u).max() / np.abs(u).max()
        # first block row through the GPU stiffness (parity of which is
        # checked above) and the oracle's B^T
        Au = _host(s.apply("stiffness", _dev(torch, u)))
        r1 = np.linalg.norm(Au + o.B.T @ lam - f) / np.linalg.norm(f)
        print(f"  {name}-FD: {st['iterations']} it, |eta|/gamma1 {st['rel_residual']:.2e}, "
              f"|Bu|/|u| {Bu:.1e}, |Au+B^T lam-f|/|f| {r1:.2e}, {st['ms']:.0f} ms", flush=True)
        assert st["converged"] and st["rel_residual"] <= 1e-8
        # B u = P_chi B w is the second block of the MINRES residual: of the order of the tolerance
        assert Bu <= 1e-7
        assert r1 <= 1e-5
