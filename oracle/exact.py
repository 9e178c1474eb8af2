"""Exact local solvers (paper Section 5.1: eq. exact_AP, eq. exact_SP;
Remark 1, eq. S_non_r), the comparison baseline of the paper's tables.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

  * P_A^ex = A + D_H M: per patch k the physical stiffness A^(k) plus
    (H^(k))^-2 times the physical mass of every component, inverted by a
    sparse LU factorisation;
  * S = blockdiag_k S^(k), S^(k) the Schur complement of A^(k) on the patch
    boundary Gamma (all components): S^(k) theta = A_GG theta - A_GI
    A_II^{-1} A_IG theta, the interior block by a sparse LU factorisation
    ("Dirichlet problems");
  * P_S^{ex-nr} = (B B^T)^{-1} B S B^T (B B^T)^{-1} (Remark 1; B touches
    only Gamma, so B_Gamma B_Gamma^T = B B^T), or P_S^ex = B S B^T
    (``variant="plain"``).
Pins (tests/test_oracle_exact.py): dense inverses and Schur complements on
small patches, S^(k) annihilates the traces of the rigid modes, and the
AF-IETI solve with these solvers equals the direct conforming solve.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class ExactPatch:
    """Factorisations of one patch."""

    def __init__(self, pa, A):
        self.pa = pa
        d, nn = pa.dim, pa.n_nodes
        Ms = pa.mass_matrix_scalar()
        M = sp.block_diag([Ms] * d, format="csc")
        self.PA = spla.splu((A + pa.diameter() ** -2 * M).tocsc())
        gam = np.tile(pa.gamma_mask().reshape(-1), d)
        self.G = np.nonzero(gam)[0]
        self.I = np.nonzero(~gam)[0]
        A = A.tocsr()
        self.A_GG = A[self.G][:, self.G]
        self.A_GI = A[self.G][:, self.I]
        self.A_IG = A[self.I][:, self.G]
        self.II = spla.splu(A[self.I][:, self.I].tocsc())
        self.n = d * nn

    def PA_inv(self, r):
        return self.PA.solve(r)

    def S(self, theta_full):
        """S^(k) theta on Gamma; interior of theta ignored, of the result zero."""
        th = theta_full[self.G]
        out = np.zeros(self.n)
        out[self.G] = self.A_GG @ th - self.A_GI @ self.II.solve(self.A_IG @ th)
        return out


class ExactPreconditioner:
    """P_A^ex and P_S^{ex-nr} (or P_S^ex) of an ``AFIETI`` system."""

    def __init__(self, sysm):
        self.sysm = sysm
        mats = sysm.A if sysm.A is not None else [pa.stiffness_matrix() for pa in sysm.patches]
        self.patches = [ExactPatch(pa, A) for pa, A in zip(sysm.patches, mats)]

    def apply_PA_inv(self, r):
        s = self.sysm
        return np.concatenate([e.PA_inv(r[s.offsets[k]:s.offsets[k + 1]]) for k, e in enumerate(self.patches)])

    def apply_PS(self, y, variant="nr"):
        s = self.sysm
        z = s._BBt_lu.solve(y) if variant == "nr" else y
        v = s.B.T @ z
        t = np.concatenate([e.S(v[s.offsets[k]:s.offsets[k + 1]]) for k, e in enumerate(self.patches)])
        t = s.B @ t
        return s._BBt_lu.solve(t) if variant == "nr" else t
