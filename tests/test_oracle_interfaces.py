"""Explicit interface lists in the oracle (Section 2.2: the interfaces are
the faces two patches share; a list names them, so that coinciding faces
not listed stay apart, e.g. a crack).

Pins (independent of the listing code):
  * the full list of a patch grid gives the same geometric nodes and the
    same jump matrix B as matching every coinciding control point;
  * a patch that no listed interface touches is a separate body: the
    conforming solution on it equals that of a problem made of it alone,
    and the rest equals the problem without it;
  * a crack makes the body more compliant: the compliance f^T u of the
    conforming solution (twice the negative minimum of the potential
    energy, over a larger space once the crack is open) grows, the
    displacement jumps across the crack and stays continuous across the
    listed faces;
  * listed faces that do not coincide are rejected."""
import copy

import numpy as np
import pytest

import workloads as W
from oracle.afieti import AFIETI
from oracle.direct import solve_conforming


def _full(prob, grid):
    p = copy.deepcopy(prob)
    p["interfaces"] = W.grid_interfaces(grid)
    return p


@pytest.mark.parametrize("mk,grid", [
    (lambda: W.make_c1(n_el=4, p=2, seed=2), (2, 2)),
    (lambda: W.make_c2(n_el=2, p=2, seed=1), (2, 2, 2)),
])
def test_full_list_equals_matching(mk, grid):
    prob = mk()
    a = AFIETI(prob)
    b = AFIETI(_full(prob, grid))
    assert a.classes == b.classes
    assert a.n_c == b.n_c
    assert abs(a.B - b.B).max() == 0


def _row_of_three():
    rng = np.random.default_rng(5)
    verts = W._grid_vertices((3, 1), rng, 0.0)
    pats = W._patches_from_grid((3, 1), verts, 2, 1, [4, 4], np.full(3, 1.3), np.full(3, 0.7), [(1, 0)])
    load = [(0, 1.0, [1, 2], [0.3, 0.1]), (1, -0.5, [2, 1], [0.0, 1.1])]
    return dict(dim=2, patches=pats, load=load, tol=1e-10)


def test_unlisted_patch_is_a_separate_body():
    prob = _row_of_three()
    prob["interfaces"] = [(0, 1, 1, 0, 0)]
    s = AFIETI(prob)
    u = s.split(solve_conforming(s))
    left = dict(prob, patches=prob["patches"][:2])
    left.pop("interfaces")
    right = dict(prob, patches=prob["patches"][2:])
    right.pop("interfaces")
    sl, sr = AFIETI(left), AFIETI(right)
    ul, ur = sl.split(solve_conforming(sl)), sr.split(solve_conforming(sr))
    scale = max(np.abs(x).max() for x in u)
    for a, b in zip(u, ul + ur):
        print(f"  patch difference {np.abs(a - b).max() / scale:.2e}")
        assert np.abs(a - b).max() <= 1e-12 * scale
    # and the glued problem differs on the third patch
    glued = AFIETI(dict(prob, interfaces=None))
    ug = glued.split(solve_conforming(glued))
    assert np.abs(ug[2] - u[2]).max() > 1e-3 * scale


def _jump(sysm, u, ka, fa, kb, fb):
    """Largest difference of the solution between coinciding control points
    of face fa of patch ka and face fb of patch kb, nodes on other faces of
    patch ka excluded (those may be glued through other patches)."""
    pa, pb = sysm.patches[ka], sysm.patches[kb]
    ia, ib = pa.face_nodes(fa), pb.face_nodes(fb)
    Xa, Xb = pa.ctrl.reshape(-1, sysm.dim)[ia], pb.ctrl.reshape(-1, sysm.dim)[ib]
    others = set()
    for f in range(2 * sysm.dim):
        if f != fa:
            others |= set(pa.face_nodes(f).tolist())
    us = sysm.split(u)
    worst = 0.0
    for i, x in zip(ia, Xa):
        if int(i) in others:
            continue
        j = ib[np.argmin(np.linalg.norm(Xb - x, axis=1))]
        for c in range(sysm.dim):
            worst = max(worst, abs(us[ka][c].reshape(-1)[i] - us[kb][c].reshape(-1)[j]))
    return worst


@pytest.mark.parametrize("dim", [2, 3])
def test_crack_opens_and_softens(dim):
    prob = W.make_cracked(dim=dim, n_el=4 if dim == 2 else 2, p=2)
    grid = (2,) * dim
    cr = AFIETI(prob)
    gl = AFIETI(_full(prob, grid))
    uc, ug = solve_conforming(cr), solve_conforming(gl)
    f = cr.load()
    assert np.allclose(f, gl.load(), rtol=0, atol=0)
    comp_c, comp_g = f @ uc, f @ ug
    print(f"  compliance cracked {comp_c:.6e} glued {comp_g:.6e}")
    assert comp_c > comp_g * (1 + 1e-6)
    scale = np.abs(uc).max()
    # across the crack (patch 0 face 1 | patch 1 face 0) the solution jumps
    assert _jump(cr, uc, 0, 1, 1, 0) > 1e-3 * scale
    assert _jump(gl, ug, 0, 1, 1, 0) <= 1e-13 * scale
    # across a listed face (patch 2 face 1 | patch 3 face 0) it is continuous
    assert _jump(cr, uc, 2, 1, 3, 0) <= 1e-13 * scale


def test_listed_faces_must_coincide():
    prob = W.make_c1(n_el=3, p=2)
    prob["interfaces"] = [(0, 0, 1, 0, 0)]  # x = 0 of patch 0 against x = 1/2 of patch 1
    with pytest.raises(ValueError):
        AFIETI(prob)
