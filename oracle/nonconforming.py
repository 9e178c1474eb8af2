"""Non-conforming nested interfaces (Section 2.2, and the non-conforming test
of Section 6): on an interface where the knot vectors of one patch refine
those of its neighbour, the splines of the coarser side are linear
combinations of the finer side's (knot insertion), and the gluing matrix B
ties every interface coefficient of the finer side to the coarse trace
written in the fine basis.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

  * knot insertion matrix T (n_f x n_c) of a nested pair of open knot vectors
    of one degree, b^c_j = sum_i T_ij b^f_i.  The definition written out: the
    two bases at the fine Greville abscissae (a unisolvent set for the fine
    space, Schoenberg-Whitney), T = V_f^{-1} V_c;
  * interfaces: two faces whose corners coincide; with equal knot vectors
    along the face they are conforming (glued node by node, elsewhere), with
    nested ones the finer side is glued to the coarser;
  * rows of B for a non-conforming interface: for every coefficient i of the
    finer face and every component c, e_{f,c,i} - sum_j (T_b (x) T_a)_{ij}
    e_{c,c,j} (u_f equals the coarse trace at the level of coefficients).
Readings and restrictions (NotImplementedError otherwise): the finer face's
coefficients on the Dirichlet boundary are glued to the coarse trace too
(they take no Dirichlet row of their own): with the Dirichlet data read at
the control points, independent values on the two sides of the interface's
boundary edges would make the trace jump there for nonlinear data; the two
faces' parametric directions are aligned (the corner order agrees), the
degrees are equal, and no finer-face coefficient is shared with a third
patch (the faces' edges lie on the outer boundary, as in the paper's
three-patch test).
Pins (tests/test_oracle_nonconforming.py): T for p = 1 by hand, partition of
unity and nonnegativity, coarse splines equal their T-combinations of fine
splines at random points, the glued solution is continuous across the
interface at random points, a linear field is reproduced exactly, and the
error against a smooth exact solution falls under refinement.
"""
from __future__ import annotations

import numpy as np

from . import bspline


def is_nested(coarse, fine, tol=1e-12) -> bool:
    """Every knot of the coarse vector appears in the fine one at least as
    often (same endpoints)."""
    f = list(np.asarray(fine, dtype=float))
    for t in np.asarray(coarse, dtype=float):
        hit = next((i for i, s in enumerate(f) if abs(s - t) <= tol), None)
        if hit is None:
            return False
        f.pop(hit)
    return True


def knot_insertion(coarse, fine, p: int) -> np.ndarray:
    """T with b^c_j = sum_i T_ij b^f_i, from the two bases at the fine
    Greville abscissae."""
    g = bspline.greville(np.asarray(fine, dtype=float), p)
    Vf = bspline.basis(fine, p, g)
    Vc = bspline.basis(coarse, p, g)
    return np.linalg.solve(Vf, Vc)


def _face_corners(pa, face):
    """The 2^(d-1) corners of a face, tangential directions ascending with
    the lowest fastest."""
    dim = pa.dim
    fd, side = face // 2, face % 2
    out = []
    for s in range(2 ** (dim - 1)):
        bits, t = 0, 0
        for l in range(dim):
            if l == fd:
                b = side
            else:
                b = (s >> t) & 1
                t += 1
            bits |= b << l
        out.append(pa.corners[bits])
    return np.array(out)


def find_interfaces(sysm, listed=None):
    """Non-conforming interfaces of an ``AFIETI`` system: list of dicts with
    the finer (``slave``) and coarser (``master``) patch and face, the face
    nodes of each (face order: tangential directions ascending, the lowest
    fastest) and T of the face.  ``listed``: only these (patch_a, face_a,
    patch_b, face_b, orient) pairs are candidates, else every pair of faces."""
    pats = sysm.patches
    dim = sysm.dim
    if listed is not None:
        pairs = [(e[0], e[1], e[2], e[3]) for e in listed]
    else:
        pairs = [(ka, fa, kb, fb) for ka in range(len(pats)) for kb in range(ka + 1, len(pats))
                 for fa in range(2 * dim) for fb in range(2 * dim)]
    out = []
    for ka, fa, kb, fb in pairs:
        A, B = pats[ka], pats[kb]
        ca, cb = _face_corners(A, fa), _face_corners(B, fb)
        d = np.linalg.norm(ca[:, None, :] - cb[None, :, :], axis=2)
        if not np.all(d.min(axis=1) <= 1e-9):
            continue
        na, nb = len(A.face_nodes(fa)), len(B.face_nodes(fb))
        if na == nb:
            continue  # conforming: glued node by node
        aligned = fa // 2 == fb // 2 and np.all(np.diag(d) <= 1e-9)
        if not aligned or A.p != B.p:
            raise NotImplementedError("non-conforming interface with rotated parametrisation or unequal degrees")
        tang = [l for l in range(dim) if l != fa // 2]
        (sk, sf, S), (mk, mf, M) = ((ka, fa, A), (kb, fb, B)) if na > nb else ((kb, fb, B), (ka, fa, A))
        Ts = []
        for l in tang:
            if not is_nested(M.knots[l], S.knots[l]):
                raise ValueError("interface knot vectors are neither equal nor nested")
            Ts.append(knot_insertion(M.knots[l], S.knots[l], S.p))
        T = Ts[0] if dim == 2 else np.kron(Ts[1], Ts[0])
        out.append(dict(slave=sk, sface=sf, master=mk, mface=mf,
                        snodes=S.face_nodes(sf), mnodes=M.face_nodes(mf), T=T))
    return out
