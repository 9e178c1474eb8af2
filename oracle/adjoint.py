"""Gradients of a scalar J(u) of the AF-IETI displacement by one adjoint
solve.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Not in the paper; it follows from the symmetric saddle system of Section 4.
With [A B^T; B 0][u; lambda] = [f; 0] and A = sum_k (mu_k A_mu^(k) +
lam_k A_lam^(k)), f = sum_j a_j F_j, the adjoint [A B^T; B 0][psi; zeta] =
[dJ/du; 0] is the same saddle operator, so psi comes from the same AF-IETI
solve with right-hand side dJ/du, and
  dJ/dmu_k  = -psi^(k)T A_mu^(k) u^(k),
  dJ/dlam_k = -psi^(k)T A_lam^(k) u^(k),
  dJ/da_j   =  psi^T F_j.

Pinned by central finite differences of J through full solves
(tests/test_oracle_solve.py, test_adjoint_gradient_central_differences).
"""
from __future__ import annotations

import numpy as np


def gradients(sysm, u, dJdu, tol=1e-12):
    """Returns dict(psi, dmu[N_p], dlam[N_p], damp[n_modes])."""
    # the adjoint constraints are homogeneous: the Dirichlet data do not
    # depend on the parameters
    res = sysm.solve(rhs=dJdu, tol=tol, lift=False)
    psi = res["u"]
    dmu, dlam = [], []
    for k, pa in enumerate(sysm.patches):
        s = slice(sysm.offsets[k], sysm.offsets[k + 1])
        uk = u[s].reshape((sysm.dim,) + pa.shape)
        pk = psi[s].reshape(-1)
        a_mu = pa.stiffness_apply(uk, lam=0.0, mu=1.0).reshape(-1)
        a_lam = pa.stiffness_apply(uk, lam=1.0, mu=0.0).reshape(-1)
        dmu.append(-pk @ a_mu)
        dlam.append(-pk @ a_lam)
    Fj = [sysm.join([pa.mode_loads(sysm.load_modes)[j] for pa in sysm.patches])
          for j in range(len(sysm.load_modes))]
    damp = np.array([psi @ F for F in Fj])
    return dict(psi=psi, dmu=np.array(dmu), dlam=np.array(dlam), damp=damp,
                iters=res["iters"])


def mass_loss(sysm, u, u_target):
    """J = 1/2 (u - u_t)^T M (u - u_t) with the physical mass (Section 4) and
    dJ/du = M (u - u_t)."""
    e = u - u_target
    Me = sysm.join([pa.mass_apply(ek) for pa, ek in zip(sysm.patches, sysm.split(e))])
    return 0.5 * float(e @ Me), Me
