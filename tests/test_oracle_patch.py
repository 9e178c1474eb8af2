"""Pins of the oracle's patch geometry and physical operators (Sections 2.2,
3, 4, 5.2) against closed forms and invariants."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle.patch import Patch, multilinear, apply_1d
from oracle import bspline


def _patch3(p=2, n_el=(3, 2, 4), seed=3, delta=0.08, lam=0.7, mu=1.3, corners=None):
    rng = np.random.default_rng(seed)
    if corners is None:
        corners = np.array([[(c >> l) & 1 for l in range(3)] for c in range(8)], float)
        corners = corners * np.array([1.0, 0.8, 1.2]) + rng.uniform(-delta, delta, (8, 3))
    return Patch(dict(corners=corners, p=p, reg=p - 1, n_el=list(n_el), lam=lam, mu=mu,
                      bc=[0] * 6), 3)


def _patch2(p=2, n_el=(4, 3), seed=4, delta=0.1, lam=1.1, mu=0.6):
    rng = np.random.default_rng(seed)
    corners = np.array([[(c >> l) & 1 for l in range(2)] for c in range(4)], float)
    corners = corners + rng.uniform(-delta, delta, (4, 2))
    return Patch(dict(corners=corners, p=p, reg=p - 1, n_el=list(n_el), lam=lam, mu=mu,
                      bc=[0] * 4), 2)


@pytest.mark.parametrize("mk", [_patch2, _patch3])
def test_control_net_reproduces_multilinear_map(mk):
    pa = mk()
    rng = np.random.default_rng(0)
    eta = rng.uniform(0, 1, (50, pa.dim))
    X = pa.ctrl.reshape(-1, pa.dim)
    B = np.ones((50, 1))
    for l in reversed(range(pa.dim)):
        v = bspline.basis(pa.knots[l], pa.p, eta[:, l])
        B = (B[:, :, None] * v[:, None, :]).reshape(50, -1)
    assert np.allclose(B @ X, multilinear(pa.corners, eta), atol=1e-14)


def test_volume_of_unit_cube_split():
    prob = W.make_c2(n_el=3, p=2)
    vol = sum(Patch(pd, 3).geometry()[1].sum() for pd in prob["patches"])
    assert vol == pytest.approx(1.0, abs=1e-13)
    prob = W.make_c1(n_el=3)
    vol = sum(Patch(pd, 2).geometry()[1].sum() for pd in prob["patches"])
    assert vol == pytest.approx(1.0, abs=1e-13)


@pytest.mark.parametrize("mk", [_patch2, _patch3])
def test_stiffness_symmetric_and_kills_rigid_modes(mk):
    pa = mk()
    A = pa.stiffness_matrix()
    assert abs(A - A.T).max() < 1e-13 * abs(A).max()
    R = pa.rigid_modes()
    assert np.abs(A @ R.T).max() < 1e-12 * abs(A).max()
    # positive semidefinite with a kernel of exactly the rigid modes
    ev = np.linalg.eigvalsh(A.toarray())
    nr = R.shape[0]
    assert np.all(ev[:nr] < 1e-10 * ev[-1]) and ev[nr] > 1e-8 * ev[-1]


@pytest.mark.parametrize("mk", [_patch2, _patch3])
def test_assembled_equals_quadrature_apply(mk):
    pa = mk()
    A = pa.stiffness_matrix()
    u = np.random.default_rng(5).standard_normal((pa.dim,) + pa.shape)
    y = pa.stiffness_apply(u)
    assert np.allclose(A @ u.reshape(-1), y.reshape(-1), atol=1e-12 * np.abs(y).max())


@pytest.mark.parametrize("mk", [_patch2, _patch3])
def test_strain_energy_of_linear_field(mk):
    # u(x) = G x: eps = sym(G), energy = (2 mu eps:eps + lam tr(eps)^2) vol
    pa = mk()
    A = pa.stiffness_matrix()
    rng = np.random.default_rng(7)
    G = rng.standard_normal((pa.dim, pa.dim))
    X = pa.ctrl.reshape(-1, pa.dim)
    u = (X @ G.T).T.reshape(-1)  # component-blocked coefficients
    eps = 0.5 * (G + G.T)
    vol = pa.geometry()[1].sum()
    exact = (2 * pa.mu * np.sum(eps * eps) + pa.lam * np.trace(eps) ** 2) * vol
    assert u @ (A @ u) == pytest.approx(exact, rel=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_axis_aligned_block_is_kronecker_form(dim):
    # cube of side s: A_ll = s^{d-2} (sum_m kappa_lm M x..K_m..x M) (Section 5.2)
    s = 0.7
    corners = np.array([[(c >> l) & 1 for l in range(dim)] for c in range(2 ** dim)], float) * s
    pd = dict(corners=corners, p=2, reg=1, n_el=[3] * dim, lam=0.9, mu=1.7, bc=[0] * 2 * dim)
    pa = Patch(pd, dim)
    A = pa.stiffness_matrix().toarray()
    nn = pa.n_nodes
    K, M = bspline.matrices_1d(pa.knots[0], pa.p)
    for l in range(dim):
        Ahat = 0
        for m in range(dim):
            kap = 2 * pa.mu + pa.lam if m == l else pa.mu
            mats = [K if mm == m else M for mm in range(dim)]
            T = np.ones((1, 1))
            for Mm in reversed(mats):
                T = np.kron(T, Mm)
            Ahat = Ahat + kap * T
        blk = A[l * nn:(l + 1) * nn, l * nn:(l + 1) * nn]
        assert np.allclose(blk, s ** (dim - 2) * Ahat, atol=1e-12 * np.abs(blk).max())


def test_mass_of_constants_is_volume():
    pa = _patch3()
    M = pa.mass_matrix_scalar()
    one = np.ones(pa.n_nodes)
    assert one @ (M @ one) == pytest.approx(pa.geometry()[1].sum(), rel=1e-13)
    u = np.random.default_rng(2).standard_normal((3,) + pa.shape)
    y = pa.mass_apply(u)
    for c in range(3):
        assert np.allclose(M @ u[c].reshape(-1), y[c].reshape(-1), atol=1e-14)


def test_body_force_of_constant_load():
    # f = e_c * 1 (sin(pi/2) = 1 with k=0 is not allowed; use phase pi/2, k=0)
    pa = _patch3()
    modes = [(1, 2.5, [0, 0, 0], [np.pi / 2] * 3)]
    F = pa.body_force(modes)
    assert F[0].sum() == pytest.approx(0.0)
    assert F[1].sum() == pytest.approx(2.5 * pa.geometry()[1].sum(), rel=1e-13)


def test_traction_divergence_theorem():
    # sum over faces of int sigma n . v = int sigma : grad v for constant sigma
    pa = _patch3()
    rng = np.random.default_rng(11)
    S = rng.standard_normal((3, 3))
    S = S + S.T
    tot = 0
    for f in range(6):
        tot = tot + pa.traction(f, lambda x, n: np.einsum("ij,...j->...i", S, n))
    # int S : grad B_i e_c = (A-like) flux with constant stress: compute via quadrature
    _, wdet, Jinv = pa.geometry()
    flux = np.einsum("cx,...ax->ca...", S, Jinv) * wdet
    ref = np.zeros((3,) + pa.shape)
    for c in range(3):
        for a in range(3):
            mats = [(pa.D[l] if l == a else pa.V[l]).T for l in range(3)]
            ref[c] += apply_1d(flux[c, a], mats)
    assert np.allclose(tot, ref, atol=1e-12)


def _box_patch(corners, dim):
    return Patch(dict(corners=np.asarray(corners, float), p=2, reg=1, n_el=[2] * dim, lam=1.0, mu=1.0,
                      bc=[0] * 2 * dim), dim)


def test_diameter_of_axis_aligned_boxes():
    """H^(k) (Section 2.2, the patch diameter that scales P_A and P_S): an
    a x b x c box has diameter sqrt(a^2 + b^2 + c^2), an a x b rectangle
    sqrt(a^2 + b^2), wherever the box sits."""
    a, b, c = 0.3, 1.7, 0.55
    unit = np.array([[(k >> l) & 1 for l in range(3)] for k in range(8)], float)
    pa = _box_patch(unit * [a, b, c] + [2.0, -1.0, 0.25], 3)
    assert pa.diameter() == pytest.approx(np.sqrt(a * a + b * b + c * c), rel=1e-15)
    unit2 = np.array([[(k >> l) & 1 for l in range(2)] for k in range(4)], float)
    pa2 = _box_patch(unit2 * [a, b] + [0.1, 0.2], 2)
    assert pa2.diameter() == pytest.approx(np.hypot(a, b), rel=1e-15)


def test_diameter_of_rotated_sheared_parallelepiped():
    """Parallelepiped spanned by e1 = (1, 0, 0), e2 = (0.4, 1, 0) and
    e3 = (0, 0, 0.6), then rotated by 30 degrees about z and 20 degrees about
    x (distances do not change, its bounding box does).  By hand, in the
    unrotated frame: the four long diagonals are 0-(1.4, 1, 0.6) and
    (0, 0, 0.6)-(1.4, 1, 0), of length sqrt(3.32), and (1, 0, 0)-(0.4, 1, 0.6),
    (0.4, 1, 0)-(1, 0, 0.6), of length sqrt(1.72); the face diagonals are
    at most sqrt(2.96).  So H = sqrt(3.32), while the rotated bounding box
    has a longer diagonal."""
    e = np.array([[1.0, 0, 0], [0.4, 1.0, 0], [0, 0, 0.6]])
    cz, sz = np.cos(np.pi / 6), np.sin(np.pi / 6)
    cx, sx = np.cos(np.pi / 9), np.sin(np.pi / 9)
    R = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]]) @ np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    corners = np.array([R @ sum(((k >> l) & 1) * e[l] for l in range(3)) for k in range(8)])
    pa = _box_patch(corners, 3)
    assert pa.diameter() == pytest.approx(np.sqrt(3.32), rel=1e-14)
    bbox = np.linalg.norm(corners.max(axis=0) - corners.min(axis=0))
    assert bbox > np.sqrt(3.32) * 1.05


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_diameter_is_sup_distance_of_mapped_points(seed):
    """For a perturbed trilinear patch, the diameter of the set F(0,1)^3:
    the largest distance between points of a dense sample of the mapped
    parametric cube (the corners excluded) approaches H from below, and no
    pair of points of the patch lies farther apart than H."""
    pa = _patch3(seed=seed, delta=0.15)
    t = np.linspace(0.0, 1.0, 9)
    g = np.stack(np.meshgrid(t, t, t, indexing="ij"), axis=-1).reshape(-1, 3)
    on_bnd = np.any((g == 0.0) | (g == 1.0), axis=1)
    is_corner = np.all((g == 0.0) | (g == 1.0), axis=1)
    X = multilinear(pa.corners, g[on_bnd & ~is_corner])
    Y = multilinear(pa.corners, g[~on_bnd])
    Xc = multilinear(pa.corners, g[is_corner])
    H = pa.diameter()
    d_inner = max(np.linalg.norm(X[:, None] - X[None], axis=-1).max(),
                  np.linalg.norm(Y[:, None] - Xc[None], axis=-1).max())
    assert d_inner <= H * (1 + 1e-14)
    d_all = np.linalg.norm(Xc[:, None] - Xc[None], axis=-1).max()
    assert d_all == pytest.approx(H, rel=1e-15)
    # points next to the farthest corners come within the sample spacing
    assert d_inner >= H - 2 * np.sqrt(3) * 0.125 * 1.5
