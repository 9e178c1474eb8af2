"""GPU parity of the adjoint path: the physical mass operator, the adjoint
solve (the saddle operator is symmetric, so psi solves the forward system
with right-hand side dJ/du), the per-patch strain-energy contractions and
the load-mode products, against the oracle's adjoint gradient; parameter
updates; the torch.autograd.Function; central finite differences."""
import numpy as np
import pytest

import workloads as W
from oracle.afieti import AFIETI
from oracle.adjoint import gradients, mass_loss

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _small_c5(seed=0):
    return W.make_c5(seed=seed, n_el=2, p=2, n_modes=6)


@pytest.mark.parametrize("mk", [lambda: W.make_c1(n_el=4, p=2), _small_c5])
def test_mass_operator(mk):
    torch = _torch()
    from paper_2001_09626_amd import Solver
    prob = mk()
    o = AFIETI(prob)
    s = Solver(prob)
    x = W.random_vector(o.n_dof, 30)
    ref = o.join([pa.mass_apply(xk) for pa, xk in zip(o.patches, o.split(x))])
    y = _host(s.apply("mass", _dev(torch, x)))
    err = np.abs(y - ref).max() / np.abs(ref).max()
    print(f"  mass: {err:.2e}")
    assert err <= 1e-13


@pytest.mark.parametrize("mk", [lambda: W.make_c1(n_el=3, p=2, seed=2), _small_c5])
def test_adjoint_matches_oracle_gradient(mk):
    torch = _torch()
    from paper_2001_09626_amd import Solver
    prob = mk()
    target = W.redraw_parameters(prob, seed=7)
    o = AFIETI(prob)
    ot = AFIETI(target)
    u_t = ot.solve(tol=1e-13)["u"]
    u = o.solve(tol=1e-13)["u"]
    J, dJdu = mass_loss(o, u, u_t)
    g = gradients(o, u, dJdu, tol=1e-13)
    s = Solver(prob, tol=1e-13)
    ud, _, _ = s.solve(want_lambda=False)
    Me = s.apply("mass", ud - _dev(torch, u_t))
    psi, dlam, dmu, damp, its = s.solve_adjoint(Me, ud)
    e_psi = np.linalg.norm(_host(psi) - g["psi"]) / np.linalg.norm(g["psi"])
    e_l = np.abs(dlam - g["dlam"]).max() / np.abs(g["dlam"]).max()
    e_m = np.abs(dmu - g["dmu"]).max() / np.abs(g["dmu"]).max()
    e_a = np.abs(damp - g["damp"]).max() / np.abs(g["damp"]).max()
    print(f"  psi {e_psi:.2e}  dlam {e_l:.2e}  dmu {e_m:.2e}  damp {e_a:.2e}  ({its} it)")
    assert e_psi <= 1e-9 and e_l <= 1e-8 and e_m <= 1e-8 and e_a <= 1e-8


def test_set_parameters_matches_oracle():
    torch = _torch()
    from paper_2001_09626_amd import Solver
    prob = _small_c5(seed=1)
    s = Solver(prob, tol=1e-12)
    new = W.redraw_parameters(prob, seed=3)
    s.set_parameters(np.array([[p["lam"], p["mu"]] for p in new["patches"]]),
                     np.array([m[1] for m in new["load"]]))
    u, lam, st = s.solve()
    ref = AFIETI(new).solve(tol=1e-12)
    e = np.linalg.norm(_host(u) - ref["u"]) / np.linalg.norm(ref["u"])
    print(f"  after set_parameters: {st['iterations']} it (oracle {ref['iters']}), rel diff {e:.2e}")
    assert e <= 1e-10
    r = W.random_vector(s.n_dof, 5)
    z = _host(s.apply_fd(_dev(torch, r)))
    zr = AFIETI(new).apply_PA_inv(r)
    assert np.abs(z - zr).max() <= 1e-12 * np.abs(zr).max()


def test_autograd_function():
    torch = _torch()
    from paper_2001_09626_amd import Solver, AfietiSolve, mass_norm_loss
    prob = _small_c5(seed=2)
    target = W.redraw_parameters(prob, seed=9)
    u_t = AFIETI(target).solve(tol=1e-13)["u"]
    s = Solver(prob, tol=1e-13)
    lame = torch.tensor([[p["lam"], p["mu"]] for p in prob["patches"]], dtype=torch.float64, requires_grad=True)
    amps = torch.tensor([m[1] for m in prob["load"]], dtype=torch.float64, requires_grad=True)
    u = AfietiSolve(lame, amps, s)
    J = mass_norm_loss(u - _dev(torch, u_t), s)
    J.backward()
    o = AFIETI(prob)
    uo = o.solve(tol=1e-13)["u"]
    Jo, dJdu = mass_loss(o, uo, u_t)
    g = gradients(o, uo, dJdu, tol=1e-13)
    gl = lame.grad.numpy()
    assert float(J.detach()) == pytest.approx(Jo, rel=1e-9)
    assert np.abs(gl[:, 0] - g["dlam"]).max() <= 1e-8 * np.abs(g["dlam"]).max()
    assert np.abs(gl[:, 1] - g["dmu"]).max() <= 1e-8 * np.abs(g["dmu"]).max()
    assert np.abs(amps.grad.numpy() - g["damp"]).max() <= 1e-8 * np.abs(g["damp"]).max()


def test_autograd_with_geometry_inclusion():
    """The gradients do not depend on the preconditioner: with the
    geometry-inclusion local solvers (rebuilt by every parameter update)
    the autograd function gives the oracle's gradients, also after the
    parameters moved."""
    torch = _torch()
    from paper_2001_09626_amd import Solver, AfietiSolve, mass_norm_loss
    prob = _small_c5(seed=6)
    target = W.redraw_parameters(prob, seed=8)
    u_t = AFIETI(target).solve(tol=1e-13)["u"]
    s = Solver(prob, tol=1e-13, precond="geo")
    for step, pr in enumerate((prob, W.redraw_parameters(prob, seed=12))):
        lame = torch.tensor([[p["lam"], p["mu"]] for p in pr["patches"]], dtype=torch.float64, requires_grad=True)
        amps = torch.tensor([m[1] for m in pr["load"]], dtype=torch.float64, requires_grad=True)
        J = mass_norm_loss(AfietiSolve(lame, amps, s) - _dev(torch, u_t), s)
        J.backward()
        o = AFIETI(pr)
        uo = o.solve(tol=1e-13)["u"]
        Jo, dJdu = mass_loss(o, uo, u_t)
        g = gradients(o, uo, dJdu, tol=1e-13)
        gl = lame.grad.numpy()
        e = max(np.abs(gl[:, 0] - g["dlam"]).max() / np.abs(g["dlam"]).max(),
                np.abs(gl[:, 1] - g["dmu"]).max() / np.abs(g["dmu"]).max(),
                np.abs(amps.grad.numpy() - g["damp"]).max() / np.abs(g["damp"]).max())
        print(f"  step {step}: J {float(J.detach()):.6e} (oracle {Jo:.6e}), gradient rel err {e:.2e}")
        assert float(J.detach()) == pytest.approx(Jo, rel=1e-9)
        assert e <= 1e-8
    s.close()


def test_autograd_with_device_parameters():
    """Parameters living on the GPU get their gradients on the GPU, with
    the same values as for CPU parameters."""
    torch = _torch()
    from paper_2001_09626_amd import Solver, AfietiSolve, mass_norm_loss
    prob = _small_c5(seed=4)
    target = W.redraw_parameters(prob, seed=5)
    u_t = _dev(torch, AFIETI(target).solve(tol=1e-13)["u"])
    s = Solver(prob, tol=1e-13)
    grads = []
    for dev in ("cpu", "cuda"):
        lame = torch.tensor([[p["lam"], p["mu"]] for p in prob["patches"]], dtype=torch.float64,
                            device=dev, requires_grad=True)
        amps = torch.tensor([m[1] for m in prob["load"]], dtype=torch.float64, device=dev, requires_grad=True)
        J = mass_norm_loss(AfietiSolve(lame, amps, s) - u_t, s)
        J.backward()
        assert lame.grad.device.type == dev and amps.grad.device.type == dev
        grads.append((lame.grad.cpu(), amps.grad.cpu()))
    assert torch.equal(grads[0][0], grads[1][0]) and torch.equal(grads[0][1], grads[1][1])
    s.close()


def test_central_differences_full_c5():
    """Full adjoint workload (3x3x3 patches, 32^3 elements, p=3): adjoint
    gradient against central differences with step 1e-6 (relative for the
    Lame parameters, absolute for the load amplitudes) for every Lame
    parameter and eight load amplitudes.  Per family (lambda, mu, load
    amplitudes) the two gradient vectors agree to 1e-6 relative, and every
    entry to 1e-6 of itself up to the rounding floor of the difference
    quotient.  The forward solves run to tol 1e-13; what remains is the
    rounding of J itself (a sum over 3.5 M products after the solves, with
    error of order log2(N) eps |J| = 22 eps |J|), which the step h turns into
    an absolute floor of 50 eps |J| / h in each quotient (measured: at most
    11 eps |J| / h); it exceeds 1e-6 relative only for entries below
    about 5e-5 of the largest."""
    torch = _torch()
    from paper_2001_09626_amd import Solver
    prob = W.make_c5(seed=0)
    target = W.redraw_parameters(prob, seed=1)
    print("\n[c5 full: setup]", flush=True)
    st_ = Solver(target, tol=1e-13)
    u_t, _, _ = st_.solve(want_lambda=False)
    st_.close()
    s = Solver(prob, tol=1e-13)
    lame0 = s.lame.copy()
    amps0 = s.amps.copy()

    def J_of(lame, amps):
        s.set_parameters(lame, amps)
        u, _, st = s.solve(want_lambda=False)
        e = u - u_t
        return 0.5 * float(torch.dot(e, s.apply("mass", e))), u, st

    J0, u0, st0 = J_of(lame0, amps0)
    Me = s.apply("mass", u0 - u_t)
    _, dlam, dmu, damp, its = s.solve_adjoint(Me, u0)
    print(f"  J={J0:.9e}  forward {st0['iterations']} it ({st0['ms']:.0f} ms), adjoint {its} it", flush=True)
    checks = [(kind, k) for k in range(len(prob["patches"])) for kind in ("lam", "mu")]
    checks += [("amp", j) for j in range(0, 64, 8)]
    fam = {"lam": [], "mu": [], "amp": []}
    for kind, idx in checks:
        lp, lm = lame0.copy(), lame0.copy()
        ap, am = amps0.copy(), amps0.copy()
        if kind == "amp":
            h = 1e-6
            ap[idx] += h
            am[idx] -= h
            ref = damp[idx]
        else:
            col = 0 if kind == "lam" else 1
            h = 1e-6 * lame0[idx, col]
            lp[idx, col] += h
            lm[idx, col] -= h
            ref = (dlam if kind == "lam" else dmu)[idx]
        fd = (J_of(lp, ap)[0] - J_of(lm, am)[0]) / (2 * h)
        fam[kind].append((ref, fd, h))
        print(f"  d J / d {kind}[{idx}]: adjoint {ref:.9e}  central diff {fd:.9e}  "
              f"abs {abs(ref - fd):.2e} rel {abs(ref - fd) / abs(fd):.2e}", flush=True)
    eps = np.finfo(np.float64).eps
    for kind, vals in fam.items():
        g = np.array(vals)
        err = np.abs(g[:, 0] - g[:, 1])
        vec = np.linalg.norm(g[:, 0] - g[:, 1]) / np.linalg.norm(g[:, 1])
        floor = 50 * eps * abs(J0) / g[:, 2]
        excess = (err / (1e-6 * np.abs(g[:, 1]) + floor)).max()
        print(f"  {kind}: |g_adj - g_fd| / |g_fd| = {vec:.2e}; max error / (1e-6 |fd| + 50 eps |J| / h) "
              f"= {excess:.2f}; largest error {err.max():.2e}", flush=True)
        assert vec <= 1e-6
        assert excess <= 1.0
    s.set_parameters(lame0, amps0)
