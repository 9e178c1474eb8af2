"""Direct solve of the conforming Galerkin problem of Section 3 (the result
AF-IETI must reproduce, Section 4: ker A and ker B meet only in zero, so the
recovered u is the conforming discrete solution).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Z maps the conforming unknowns (one per geometric node and component, nodes
on the Dirichlet boundary removed) to their patch copies; A_c = Z^T A Z,
f_c = Z^T f, u = Z A_c^{-1} f_c.

Pinned by: the patch test and polynomial reproduction (tests/test_oracle_solve.py);
``solve_kkt`` (any gluing matrix, e.g. non-conforming interfaces) by the
same patch test and by agreement with ``solve_conforming`` on conforming
problems (tests/test_oracle_nonconforming.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def conforming_map(sysm) -> sp.csr_matrix:
    """Boolean Z (N_dof x N_conf) from the node classes of an ``AFIETI``."""
    dim = sysm.dim
    shared = {}
    for ci, cp in enumerate(sysm.classes):
        for (k, i) in cp:
            shared[(k, i)] = ci
    rows, cols = [], []
    col = 0
    node_col = {}
    for k, pa in enumerate(sysm.patches):
        for i in range(pa.n_nodes):
            key = ("c", shared[(k, i)]) if (k, i) in shared else ("p", k, i)
            if key[0] == "c" and sysm.dirichlet_class[key[1]]:
                continue
            if key not in node_col:
                node_col[key] = col
                col += 1
    for k, pa in enumerate(sysm.patches):
        for i in range(pa.n_nodes):
            key = ("c", shared[(k, i)]) if (k, i) in shared else ("p", k, i)
            if key not in node_col:
                continue
            for c in range(dim):
                rows.append(sysm.dof(k, c, i))
                cols.append(node_col[key] * dim + c)
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)),
                         shape=(sysm.n_dof, col * dim))


def solve_conforming(sysm, f=None):
    """u = Z (Z^T A Z)^{-1} Z^T (f - A u_D) + u_D with the assembled patch
    matrices: the conforming unknowns away from the Dirichlet boundary, the
    Dirichlet copies fixed at their data u_D (zero for homogeneous data)."""
    if not sysm.assembled:
        raise ValueError("direct solve needs assembled patch matrices")
    f = sysm.load() if f is None else f
    Z = conforming_map(sysm)
    A = sp.block_diag(sysm.A, format="csr")
    Ac = (Z.T @ A @ Z).tocsc()
    uc = spla.spsolve(Ac, Z.T @ (f - A @ sysm.u_dir))
    return Z @ uc + sysm.u_dir


def solve_kkt(sysm, f=None):
    """The constrained Galerkin problem in saddle form, [A B^T; B 0]
    [u; lam] = [f; c], solved directly with the assembled patch matrices:
    the definition of the discrete solution for any gluing B (conforming
    classes and non-conforming interface rows alike; ker A and ker B meet
    only in zero, Section 4)."""
    if not sysm.assembled:
        raise ValueError("direct solve needs assembled patch matrices")
    f = sysm.load() if f is None else f
    A = sp.block_diag(sysm.A, format="csr")
    K = sp.bmat([[A, sysm.B.T], [sysm.B, None]], format="csc")
    rhs = np.concatenate([f, sysm.c])
    sol = spla.spsolve(K, rhs)
    return sol[:sysm.n_dof]
