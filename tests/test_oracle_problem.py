"""Pins of the oracle's general problem statement (Sections 2.1 and 3):
explicit knot vectors, a body force given as a function, tractions on the
faces marked 2 (Gamma_N) and non-homogeneous Dirichlet data.  Fields in the
spline space are reproduced exactly by both the direct conforming solve and
AF-IETI; the weak-scaling workload's forcing is -div sigma of its exact
solution."""
import copy

import numpy as np
import pytest

import workloads as W
from oracle.afieti import AFIETI
from oracle.direct import solve_conforming
from oracle.patch import apply_1d


def _outer_faces(pa):
    out = []
    for f in range(2 * pa.dim):
        fd, side = f // 2, f % 2
        idx = [c for c in range(2 ** pa.dim) if ((c >> fd) & 1) == side]
        if np.allclose(pa.corners[idx, fd], float(side)):
            out.append(f)
    return out


def _stress_fn(grad_fn, lam, mu):
    def sig(x):
        g = grad_fn(x)
        div = np.trace(g, axis1=1, axis2=2)
        return mu * (g + np.swapaxes(g, 1, 2)) + lam * div[:, None, None] * np.eye(g.shape[1])
    return sig


def _minus_div(sig, x, h=1e-3):
    """-div sigma by central differences (exact up to rounding for sigma
    linear in x; O(h^2) otherwise)."""
    f = np.zeros(x.shape)
    for a in range(x.shape[1]):
        e = np.zeros(x.shape[1])
        e[a] = h
        f -= (sig(x + e)[:, :, a] - sig(x - e)[:, :, a]) / (2 * h)
    return f


def _with_boundary_data(prob, u_fn, grad_fn):
    """Dirichlet data u_fn on the Dirichlet faces, traction sigma(u) n on the
    other outer faces (marked 2), body force -div sigma(u), no load modes;
    every patch takes the first patch's material, so that u_fn is the
    solution (with jumps in lambda, mu the interface tractions of a smooth
    field would not balance)."""
    prob = copy.deepcopy(prob)
    pd0 = prob["patches"][0]
    for pd in prob["patches"]:
        pd["lam"], pd["mu"] = pd0["lam"], pd0["mu"]
    sig = _stress_fn(grad_fn, pd0["lam"], pd0["mu"])
    s = AFIETI(prob)
    for pa, pd in zip(s.patches, prob["patches"]):
        for f in _outer_faces(pa):
            if pd["bc"][f] != 1:
                pd["bc"][f] = 2
    prob["load"] = []
    prob["dirichlet"] = u_fn
    prob["traction"] = lambda x, n: np.einsum("nij,nj->ni", sig(x), n)
    prob["body_force"] = lambda x: _minus_div(sig, x)
    return prob


def _at_gauss_points(s, u):
    """(field values, exact points) of a patch-stacked vector at every Gauss point."""
    vals, pts = [], []
    for pa, uk in zip(s.patches, s.split(u)):
        xq = pa.geometry()[0]
        vals.append(np.stack([apply_1d(uk[c], pa.V) for c in range(s.dim)], axis=-1).reshape(-1, s.dim))
        pts.append(xq.reshape(-1, s.dim))
    return np.concatenate(vals), np.concatenate(pts)


@pytest.mark.parametrize("mk", [lambda: W.make_c2(n_el=2, p=2, seed=5), lambda: W.make_c1(n_el=3, p=2, seed=9)])
def test_nonhomogeneous_dirichlet_linear_field(mk):
    """u*(x) = a + G x with u* as Dirichlet data on the Dirichlet faces and
    sigma(u*) n on the other outer faces, f = 0 (its divergence): u* lies in
    the spline space on the perturbed multilinear patches, its coefficients
    are its values at the control points, and both solves reproduce it."""
    prob = mk()
    d = prob["dim"]
    rng = np.random.default_rng(3)
    a, G = rng.standard_normal(d), rng.standard_normal((d, d))
    prob = _with_boundary_data(prob, lambda x: a + x @ G.T, lambda x: np.broadcast_to(G, (len(x), d, d)))
    prob["body_force"] = None
    s = AFIETI(prob)
    ustar = s.join([np.moveaxis(a + pa.ctrl @ G.T, -1, 0) for pa in s.patches])
    assert np.any(s.c != 0)
    res = s.solve(tol=1e-13)
    assert np.abs(res["u"] - ustar).max() <= 1e-9 * np.abs(ustar).max()
    ud = solve_conforming(s)
    assert np.abs(ud - ustar).max() <= 1e-10 * np.abs(ustar).max()


def test_quadratic_field_with_body_force():
    """On affine cube patches (p = 2) u*(x) = a + G x + z (H x) is in the
    spline space and linear on the Dirichlet face z = 0 (so the Greville
    interpolation of its data is exact); f = -div sigma(u*) is constant and
    the tractions are linear: the solution equals u* at every Gauss point."""
    prob = W.make_c2(n_el=2, p=2, seed=0, delta=0.0)
    rng = np.random.default_rng(4)
    a, G, H = rng.standard_normal(3), rng.standard_normal((3, 3)), rng.standard_normal((3, 3))

    def u_fn(x):
        return a + x @ G.T + x[:, 2:3] * (x @ H.T)

    def grad_fn(x):
        g = G + x[:, 2, None, None] * H
        g = np.array(g)
        g[:, :, 2] += x @ H.T
        return g

    prob = _with_boundary_data(prob, u_fn, grad_fn)
    s = AFIETI(prob)
    for u in (s.solve(tol=1e-13)["u"], solve_conforming(s)):
        uq, xq = _at_gauss_points(s, u)
        ref = u_fn(xq)
        assert np.abs(uq - ref).max() <= 1e-9 * np.abs(ref).max()


def test_constant_body_force_total_is_force_times_volume():
    prob = W.make_c2(n_el=3, p=2, seed=1)
    b = np.array([0.3, -1.2, 2.0])
    prob["load"] = []
    prob["body_force"] = lambda x: np.broadcast_to(b, x.shape)
    s = AFIETI(prob)
    F = s.load()
    tot = sum(Fk.reshape(3, -1).sum(axis=1) for Fk in s.split(F))
    assert np.allclose(tot, b * 1.0, rtol=1e-13)


def test_body_force_function_equals_trig_mode():
    prob = W.make_c2(n_el=2, p=3, seed=2)
    comp, amp, k, ph = prob["load"][1]
    mode_only = AFIETI(prob).load()
    prob2 = copy.deepcopy(prob)
    prob2["load"] = [m for j, m in enumerate(prob["load"]) if j != 1]

    def fn(x):
        f = np.zeros(x.shape)
        f[:, comp] = amp * np.prod(np.sin(np.pi * np.asarray(k) * x + np.asarray(ph)), axis=1)
        return f

    prob2["body_force"] = fn
    assert np.abs(AFIETI(prob2).load() - mode_only).max() <= 1e-14 * np.abs(mode_only).max()


def test_explicit_uniform_knots_equal_default():
    prob = W.make_c2(n_el=3, p=2, seed=2)
    from oracle import bspline
    prob2 = copy.deepcopy(prob)
    for pd in prob2["patches"]:
        pd["knots"] = [bspline.open_uniform_knots(3, 2, 1)] * 3
    a, b = AFIETI(prob), AFIETI(prob2)
    x = W.random_vector(a.n_dof, 1)
    assert np.array_equal(a.apply_A(x), b.apply_A(x))
    assert np.array_equal(a.load(), b.load())


def test_graded_knots_linear_field():
    """Non-uniform (graded) open knot vectors, equal across the interfaces:
    the linear-field test still holds exactly."""
    prob = W.make_c2(n_el=2, p=2, seed=6)
    kv = np.array([0, 0, 0, 0.15, 0.4, 1, 1, 1.0])
    for pd in prob["patches"]:
        pd["knots"] = [kv, kv, kv]
    d = 3
    rng = np.random.default_rng(5)
    a, G = rng.standard_normal(d), rng.standard_normal((d, d))
    prob = _with_boundary_data(prob, lambda x: a + x @ G.T, lambda x: np.broadcast_to(G, (len(x), d, d)))
    prob["body_force"] = None
    s = AFIETI(prob)
    assert s.patches[0].n == [5, 5, 5]
    ustar = s.join([np.moveaxis(a + pa.ctrl @ G.T, -1, 0) for pa in s.patches])
    res = s.solve(tol=1e-13)
    assert np.abs(res["u"] - ustar).max() <= 1e-9 * np.abs(ustar).max()


def test_weak_scaling_forcing_and_traction():
    """The weak-scaling workload's body force is -div sigma(u*) (central
    differences of its stress), its stress is mu (grad + grad^T) + lam div I
    of its exact solution (central differences of u*)."""
    prob = W.make_weak_scaling(k=2, n_el=2)
    lam, mu = W.STEEL_LAM, W.STEEL_MU
    x = np.random.default_rng(7).uniform(0.1, 0.9, (40, 3))
    sig = lambda y: W.weak_scaling_stress(y, lam, mu)  # noqa: E731
    assert np.allclose(prob["body_force"](x), _minus_div(sig, x, 1e-4), rtol=1e-6, atol=1e-7)
    h = 1e-5
    g = np.zeros((40, 3, 3))
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        g[:, :, a] = (W.weak_scaling_solution(x + e) - W.weak_scaling_solution(x - e)) / (2 * h)
    div = np.trace(g, axis1=1, axis2=2)
    ref = mu * (g + np.swapaxes(g, 1, 2)) + lam * div[:, None, None] * np.eye(3)
    assert np.allclose(sig(x), ref, rtol=1e-8, atol=1e-9)
    n = np.tile([-1.0, 0, 0], (40, 1))
    assert np.allclose(prob["traction"](x, n), -sig(x)[:, :, 0])


def test_weak_scaling_solution_converges_to_exact():
    """The discrete solution of the weak-scaling workload approaches u* as
    the elements refine.  The Dirichlet data enter through their values at
    the control points, a second-order approximation, so a halving of h cuts
    the error at the Gauss points by more than 2x (4x asymptotically)."""
    errs = []
    for n_el in (2, 4):
        s = AFIETI(W.make_weak_scaling(k=2, n_el=n_el))
        uq, xq = _at_gauss_points(s, s.solve(tol=1e-12)["u"])
        errs.append(np.abs(uq - W.weak_scaling_solution(xq)).max())
    assert errs[1] < errs[0] / 2 and errs[1] < 1e-2


def _as_explicit_net(prob):
    """The same problem with every patch given by its control net (the
    multilinear net of its corners) instead of its corners."""
    prob = copy.deepcopy(prob)
    s = AFIETI(prob)
    for pa, pd in zip(s.patches, prob["patches"]):
        pd["ctrl"] = pa.ctrl.copy()
        del pd["corners"]
    return prob


def test_explicit_net_of_the_multilinear_map_changes_nothing():
    """A patch given by the control net of its corners' multilinear map is
    the same patch: identical stiffness, load, diameter and solution."""
    prob = W.make_c2(n_el=2, p=2, seed=3)
    a, b = AFIETI(prob), AFIETI(_as_explicit_net(prob))
    assert all(pb.general and not pa.general for pa, pb in zip(a.patches, b.patches))
    x = W.random_vector(a.n_dof, 2)
    assert np.array_equal(a.apply_A(x), b.apply_A(x))
    assert np.array_equal(a.load(), b.load())
    assert [pa.diameter() for pa in a.patches] == pytest.approx([pb.diameter() for pb in b.patches], rel=1e-15)
    assert np.abs(a.solve(tol=1e-10)["u"] - b.solve(tol=1e-10)["u"]).max() <= 1e-14 * np.abs(a.solve(tol=1e-10)["u"]).max()


def test_curved_patches():
    """Explicit control nets of a curved domain (quarter of a thick
    cylinder): rigid modes are in the kernel of every patch stiffness
    (their strain vanishes pointwise, whatever the geometry), the
    volume is within 2 % of the cylinder sector's (the nets approximate
    the curved faces: measured 1.0 % below), the AF-IETI
    solution equals the direct conforming solve, and geometry inclusion
    needs far fewer iterations than the parametric FD (the preconditioner
    the paper proposes for curved patches)."""
    prob = W.make_curved(n_el=3, p=2)
    s = AFIETI(prob)
    for k, pa in enumerate(s.patches):
        A = s.A[k]
        assert np.abs(A @ pa.rigid_modes().T).max() <= 1e-13 * np.abs(A).max()
    vol = sum(pa.geometry()[1].sum() for pa in s.patches)
    assert vol == pytest.approx(0.25 * np.pi * (2.0 ** 2 - 1.0), rel=2e-2)
    res = s.solve(tol=1e-12)
    ud = solve_conforming(s)
    assert np.abs(res["u"] - ud).max() <= 1e-9 * np.abs(ud).max()
    its_fd = s.solve(tol=1e-8)["iters"]
    its_geo = AFIETI(prob, geometry=True).solve(tol=1e-8)["iters"]
    assert its_geo < its_fd / 2
