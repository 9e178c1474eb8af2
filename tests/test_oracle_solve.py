"""Whole-solve pins of the oracle: a manufactured displacement in the spline
space (patch test on perturbed multi-patch geometry) is reproduced, and the
adjoint gradient agrees with central finite differences."""
import copy

import numpy as np
import pytest

import workloads as W
from oracle.afieti import AFIETI
from oracle.adjoint import gradients, mass_loss


def _outer_faces(pa):
    """(face, ...) of the unit box boundary: every corner of the face sits on
    the plane x_fd = side."""
    out = []
    for f in range(2 * pa.dim):
        fd, side = f // 2, f % 2
        idx = [c for c in range(2 ** pa.dim) if ((c >> fd) & 1) == side]
        if np.allclose(pa.corners[idx, fd], float(side)):
            out.append(f)
    return out


@pytest.mark.parametrize("mk,ddir", [(lambda: W.make_c1(n_el=3, p=2, seed=9), 0),
                                     (lambda: W.make_c1(n_el=2, p=3, seed=1), 0),
                                     (lambda: W.make_c2(n_el=2, p=2, seed=5), 2)])
def test_patch_test_linear_field(mk, ddir):
    """u*(x) = x_D a, zero on the Dirichlet plane x_D = 0; f = 0; traction
    sigma(u*) n on the other outer faces.  u* lies in the spline space and the
    quadrature is exact for it, so the discrete solution equals u*."""
    prob = mk()
    s = AFIETI(prob)
    d = s.dim
    a = np.array([0.3, -0.7, 0.5][:d])
    grad = np.outer(a, np.eye(d)[ddir])
    sig = s.patches[0].mu * (grad + grad.T) + s.patches[0].lam * np.trace(grad) * np.eye(d)
    parts_f, parts_u = [], []
    for pa in s.patches:
        assert pa.mu == s.patches[0].mu and pa.lam == s.patches[0].lam
        F = np.zeros((d,) + pa.shape)
        for f in _outer_faces(pa):
            if pa.bc[f] == 1:
                continue
            F = F + pa.traction(f, lambda x, n: np.einsum("ij,...j->...i", sig, n))
        parts_f.append(F.reshape(-1))
        X = pa.ctrl.reshape(-1, d)
        parts_u.append(np.outer(a, X[:, ddir]).reshape(-1))
    rhs = np.concatenate(parts_f)
    ustar = np.concatenate(parts_u)
    res = s.solve(rhs=rhs, tol=1e-13)
    assert np.abs(res["u"] - ustar).max() < 1e-9 * np.abs(ustar).max()


def _loss_and_grad(prob, u_t):
    s = AFIETI(prob)
    u = s.solve(tol=1e-13)["u"]
    J, dJdu = mass_loss(s, u, u_t)
    return s, u, J, dJdu


def test_adjoint_gradient_central_differences():
    base = W.make_c1(n_el=2, p=2, seed=3)
    rng = np.random.default_rng(0)
    for pd in base["patches"]:
        pd["lam"] = float(np.exp(rng.normal(0, 0.5)))
        pd["mu"] = float(np.exp(rng.normal(0, 0.5)))
    target = W.redraw_parameters(base, seed=11)
    st = AFIETI(target)
    u_t = st.solve(tol=1e-13)["u"]
    s, u, J, dJdu = _loss_and_grad(base, u_t)
    g = gradients(s, u, dJdu, tol=1e-13)
    h = 1e-6

    def J_of(mod):
        prob = copy.deepcopy(base)
        mod(prob)
        return _loss_and_grad(prob, u_t)[2]

    for k in [0, 3]:
        for key, ref in (("mu", g["dmu"][k]), ("lam", g["dlam"][k])):
            def plus(pr, k=k, key=key, sgn=1):
                pr["patches"][k][key] += sgn * h
            fd = (J_of(plus) - J_of(lambda pr: plus(pr, sgn=-1))) / (2 * h)
            assert ref == pytest.approx(fd, rel=1e-6, abs=1e-10)
    for j in range(len(base["load"])):
        def amp(pr, j=j, sgn=1):
            c, a, k, ph = pr["load"][j]
            pr["load"][j] = (c, a + sgn * h, k, ph)
        fd = (J_of(amp) - J_of(lambda pr: amp(pr, sgn=-1))) / (2 * h)
        assert g["damp"][j] == pytest.approx(fd, rel=1e-6, abs=1e-10)
