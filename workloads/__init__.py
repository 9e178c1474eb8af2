"""Seeded synthetic problem instances for multi-patch isogeometric elasticity.

This module only draws random numbers and lays out problem descriptions
(patch corner coordinates, spline degree and continuity, element counts,
Lame parameters, Dirichlet faces and load modes).  It contains none of the
solver's arithmetic: both the CPU oracle and the GPU library read the plain
dictionaries produced here, and each evaluates them with its own code.

Problem dictionary layout
-------------------------
``dim``          2 or 3.
``patches``      list of patch dicts, colexicographic over the patch grid:
    ``corners``  (2**dim, dim) float64 corner coordinates; corner index
                 a1 + 2*a2 + 4*a3 with a_l in {0, 1} (colexicographic, the
                 first parametric direction runs fastest).  The patch map is
                 the multilinear interpolant of its corners.
    ``p``        spline degree (same in every direction).
    ``reg``      continuity C^reg across interior knots (reg = p - 1 gives
                 knots of multiplicity one).
    ``n_el``     elements per parametric direction (uniform open knots).
    ``lam``, ``mu``  Lame parameters of the patch.
    ``bc``       2*dim face flags, order (dir1 min, dir1 max, dir2 min, ...):
                 0 = natural (traction-free or interface), 1 = Dirichlet
                 (u = 0, or the problem's ``dirichlet`` data), 2 = traction
                 (the problem's ``traction``).
    ``knots``    optional: explicit open knot vectors per direction.
``load``         list of separable trigonometric body-force modes
                 (component, amplitude, k[dim], phase[dim]) meaning
                 f_component(x) += amplitude * prod_d sin(pi*k_d*x_d + phase_d).
``tol``          MINRES tolerance on the preconditioned residual ratio.
``body_force``, ``traction``, ``dirichlet``  optional callables on arrays of
                 points (n, dim): f(x), g(x, normal), g_D(x), each -> (n, dim).
``interfaces``   optional list of (patch_a, face_a, patch_b, face_b, orient):
                 only these face pairs are glued (orient -1: from the
                 corners); absent, every pair of coinciding faces is.

Material constants: E = 1, nu = 0.3 gives lambda = 0.3/0.52, mu = 1/2.6
(the paper's "steel" values, Section 6).
"""
from __future__ import annotations

import copy
import math

import numpy as np

STEEL_LAM = 0.3 / 0.52
STEEL_MU = 1.0 / 2.6

FACE_FREE = 0
FACE_DIRICHLET = 1
FACE_TRACTION = 2


def _grid_vertices(grid, rng, delta):
    """Vertex lattice of the unit square/cube split into ``grid`` patches.

    Vertices strictly inside the domain are moved by U(-delta, delta)^dim;
    boundary vertices stay, so the outer boundary is the unit box.
    Returns an array of shape grid+1 (reversed, colex) + (dim,).
    """
    dim = len(grid)
    axes = [np.linspace(0.0, 1.0, g + 1) for g in grid]
    shape = tuple(g + 1 for g in grid)
    verts = np.zeros(shape + (dim,))
    for idx in np.ndindex(*shape):
        interior = all(0 < idx[d] < grid[d] for d in range(dim))
        pos = np.array([axes[d][idx[d]] for d in range(dim)])
        if interior and delta > 0:
            pos = pos + rng.uniform(-delta, delta, size=dim)
        verts[idx] = pos
    return verts


def _patches_from_grid(grid, verts, p, reg, n_el, lam, mu, dirichlet_planes):
    """Build patch dicts, colexicographic over the patch grid.

    ``dirichlet_planes``: list of (direction, side) of the unit box that carry
    u = 0 (side 0 = coordinate 0, side 1 = coordinate 1).
    """
    dim = len(grid)
    patches = []
    pid = 0
    for pidx in np.ndindex(*tuple(reversed(grid))):
        pidx = tuple(reversed(pidx))  # pidx[0] runs fastest
        corners = np.zeros((2 ** dim, dim))
        for c in range(2 ** dim):
            a = [(c >> d) & 1 for d in range(dim)]
            corners[c] = verts[tuple(pidx[d] + a[d] for d in range(dim))]
        bc = [FACE_FREE] * (2 * dim)
        for (d, side) in dirichlet_planes:
            if side == 0 and pidx[d] == 0:
                bc[2 * d] = FACE_DIRICHLET
            if side == 1 and pidx[d] == grid[d] - 1:
                bc[2 * d + 1] = FACE_DIRICHLET
        patches.append(dict(corners=corners, p=int(p), reg=int(reg),
                            n_el=[int(n) for n in n_el],
                            lam=float(lam[pid]), mu=float(mu[pid]), bc=bc))
        pid += 1
    return patches


def _random_modes(rng, n_modes, dim):
    modes = []
    for _ in range(n_modes):
        comp = int(rng.integers(0, dim))
        amp = float(rng.normal())
        k = [int(v) for v in rng.integers(1, 4, size=dim)]
        ph = [float(v) for v in rng.uniform(0.0, 2.0 * math.pi, size=dim)]
        modes.append((comp, amp, k, ph))
    return modes


def _lognormal(rng, n):
    return np.exp(rng.normal(0.0, 0.5, size=n))


def make_c1(seed=0, n_el=16, p=2, grid=(2, 2), delta=0.1):
    """2D: unit square in 2x2 bilinear patches, interior vertex moved by
    U(-0.1, 0.1)^2, p=2 C^1, 16x16 elements per patch, lambda = mu = 1,
    f = (sin(pi x) sin(pi y), cos(pi x) sin(pi y)), u = 0 on x = 0."""
    rng = np.random.default_rng(seed)
    verts = _grid_vertices(grid, rng, delta)
    n_p = int(np.prod(grid))
    patches = _patches_from_grid(grid, verts, p, p - 1, [n_el] * 2,
                                 np.ones(n_p), np.ones(n_p), [(0, 0)])
    half_pi = 0.5 * math.pi
    load = [(0, 1.0, [1, 1], [0.0, 0.0]),
            (1, 1.0, [1, 1], [half_pi, 0.0])]
    return dict(name="c1", dim=2, patches=patches, load=load, tol=1e-8)


def make_c2(seed=0, n_el=32, p=3, grid=(2, 2, 2), delta=0.05):
    """3D: unit cube in 2x2x2 trilinear patches, the interior vertex moved by
    U(-0.05, 0.05)^3, p=3 C^2, 32^3 elements per patch, E=1 nu=0.3,
    f = (sin sin sin, cos sin sin, sin cos sin)(pi x, pi y, pi z),
    u = 0 on z = 0."""
    rng = np.random.default_rng(seed)
    verts = _grid_vertices(grid, rng, delta)
    n_p = int(np.prod(grid))
    patches = _patches_from_grid(grid, verts, p, p - 1, [n_el] * 3,
                                 np.full(n_p, STEEL_LAM), np.full(n_p, STEEL_MU),
                                 [(2, 0)])
    hp = 0.5 * math.pi
    load = [(0, 1.0, [1, 1, 1], [0.0, 0.0, 0.0]),
            (1, 1.0, [1, 1, 1], [hp, 0.0, 0.0]),
            (2, 1.0, [1, 1, 1], [0.0, hp, 0.0])]
    return dict(name="c2", dim=3, patches=patches, load=load, tol=1e-8)


def make_c3(seed=0, p=3, n_el=24, grid=(4, 4, 4), rel_delta=0.1, n_modes=8):
    """3D: unit cube in 4x4x4 patches, interior vertices moved by
    U(-0.1 h_patch, 0.1 h_patch)^3, p in {2..5} at C^{p-1}, 24^3 elements,
    per-patch lambda, mu ~ lognormal(0, 0.5), 8 seeded trig load modes,
    u = 0 on z = 0."""
    rng = np.random.default_rng(seed)
    delta = rel_delta / max(grid)
    verts = _grid_vertices(grid, rng, delta)
    n_p = int(np.prod(grid))
    lam = _lognormal(rng, n_p)
    mu = _lognormal(rng, n_p)
    patches = _patches_from_grid(grid, verts, p, p - 1, [n_el] * 3, lam, mu,
                                 [(2, 0)])
    return dict(name="c3", dim=3, patches=patches,
                load=_random_modes(rng, n_modes, 3), tol=1e-8)


def make_c4(seed=0, n_problems=32, el_range=(8, 40), p_choices=(2, 3, 4),
            rel_delta=0.1, n_modes=8):
    """Ragged batch: each problem has a patch grid uniform in {1,2,3}^3,
    elements per direction uniform in [8, 40] (shared by the problem's
    patches), p uniform in {2,3,4} at C^{p-1}, perturbed interior vertices,
    lognormal Lame parameters, 8 seeded trig modes, u = 0 on z = 0."""
    rng = np.random.default_rng(seed)
    probs = []
    for j in range(n_problems):
        grid = tuple(int(g) for g in rng.integers(1, 4, size=3))
        n_el = [int(v) for v in rng.integers(el_range[0], el_range[1] + 1, size=3)]
        p = int(rng.choice(p_choices))
        delta = rel_delta / max(grid)
        verts = _grid_vertices(grid, rng, delta)
        n_p = int(np.prod(grid))
        lam = _lognormal(rng, n_p)
        mu = _lognormal(rng, n_p)
        patches = _patches_from_grid(grid, verts, p, p - 1, n_el, lam, mu, [(2, 0)])
        probs.append(dict(name=f"c4_{j}", dim=3, patches=patches,
                          load=_random_modes(rng, n_modes, 3), tol=1e-8))
    return probs


def make_c5(seed=0, n_el=32, p=3, grid=(3, 3, 3), rel_delta=0.1, n_modes=64):
    """Adjoint workload: 3x3x3 patches, 32^3 elements, p=3 C^2, lognormal
    per-patch Lame parameters, 64 seeded trig load modes whose amplitudes are
    the load coefficients, u = 0 on z = 0."""
    rng = np.random.default_rng(seed)
    delta = rel_delta / max(grid)
    verts = _grid_vertices(grid, rng, delta)
    n_p = int(np.prod(grid))
    lam = _lognormal(rng, n_p)
    mu = _lognormal(rng, n_p)
    patches = _patches_from_grid(grid, verts, p, p - 1, [n_el] * 3, lam, mu,
                                 [(2, 0)])
    return dict(name="c5", dim=3, patches=patches,
                load=_random_modes(rng, n_modes, 3), tol=1e-8)


def make_curved(seed=0, n_el=4, p=3, grid=(2, 2, 2), n_modes=8, r_in=1.0, r_out=2.0, height=1.0):
    """3D curved domain with explicit control nets: a quarter of a thick
    cylinder, r in [r_in, r_out], theta in [0, pi/2], z in [0, height], in
    grid[0] x grid[1] x grid[2] patches of (r, theta, z); p C^{p-1}, n_el^3
    elements per patch.  The control points of a patch are the cylinder map
    of an equispaced grid of its (r, theta, z) box (n_el + p points per
    direction, shared by neighbouring patches on their common faces), so the
    patches are B-spline approximations of the curved sectors.  Steel,
    ``n_modes`` seeded trig load modes, u = 0 on z = 0."""
    rng = np.random.default_rng(seed)
    n = n_el + p
    edges = [np.linspace(r_in, r_out, grid[0] + 1), np.linspace(0.0, 0.5 * math.pi, grid[1] + 1),
             np.linspace(0.0, height, grid[2] + 1)]
    patches = []
    for pidx in np.ndindex(*tuple(reversed(grid))):
        pidx = tuple(reversed(pidx))
        ax = [np.linspace(edges[d][pidx[d]], edges[d][pidx[d] + 1], n) for d in range(3)]
        Z, T, R = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")     # (n3, n2, n1)
        ctrl = np.stack([R * np.cos(T), R * np.sin(T), Z], axis=-1)
        bc = [FACE_FREE] * 6
        if pidx[2] == 0:
            bc[4] = FACE_DIRICHLET
        patches.append(dict(ctrl=ctrl, p=int(p), reg=int(p - 1), n_el=[int(n_el)] * 3,
                            lam=STEEL_LAM, mu=STEEL_MU, bc=bc))
    return dict(name="curved", dim=3, patches=patches, load=_random_modes(rng, n_modes, 3), tol=1e-8)


def grid_interfaces(grid):
    """Explicit interface list of a patch grid (colexicographic patches, all
    parametrised alike): for every pair of neighbours along direction d the
    row (patch_a, face 2d + 1, patch_b, face 2d, orient 0)."""
    dim = len(grid)
    out = []
    for pidx in np.ndindex(*tuple(reversed(grid))):
        pidx = tuple(reversed(pidx))
        ka = sum(pidx[d] * int(np.prod(grid[:d])) for d in range(dim))
        for d in range(dim):
            if pidx[d] + 1 < grid[d]:
                out.append((ka, 2 * d + 1, ka + int(np.prod(grid[:d])), 2 * d, 0))
    return out


def make_cracked(dim=2, seed=0, n_el=8, p=2, n_modes=4):
    """A patch grid with a crack: 2D, the unit square in 2x2 patches with the
    interface between patches 0 and 1 left open (a slit from (1/2, 0) to the
    centre); 3D, the unit cube in 2x2x2 patches with the interfaces of patch
    0 to patches 1 and 2 left open (two crack faces meeting along the edge
    x = y = 1/2, z < 1/2).  Interior vertex moved by U(-0.05, 0.05)^dim, p
    C^{p-1}, n_el elements per direction, steel, seeded trig loads, u = 0 on
    the far side (y = 1 in 2D, z = 1 in 3D); the crack faces are free."""
    rng = np.random.default_rng(seed)
    grid = (2,) * dim
    verts = _grid_vertices(grid, rng, 0.05)
    n_p = 2 ** dim
    patches = _patches_from_grid(grid, verts, p, p - 1, [n_el] * dim,
                                 np.full(n_p, STEEL_LAM), np.full(n_p, STEEL_MU), [(dim - 1, 1)])
    itf = grid_interfaces(grid)
    cut = {(0, 1)} if dim == 2 else {(0, 1), (0, 2)}
    itf = [e for e in itf if (e[0], e[2]) not in cut]
    return dict(name=f"cracked{dim}d", dim=dim, patches=patches, interfaces=itf,
                load=_random_modes(rng, n_modes, dim), tol=1e-8)


def make_rotated_pair(dim):
    """Two unit patches sharing the plane x = 1, the second parametrised in a
    rotated way: 2D (eta1, eta2) -> (2 - eta1, 1 - eta2), shared faces 1 and
    1, the common edge running against the first patch's direction (orient
    2); 3D (eta1, eta2, eta3) -> (1 + eta1, 1 - eta3, eta2), shared faces 1
    and 0, the first patch's y running along the second's eta3 reversed and
    its z along eta2 (orient swap 1 + 2 flip_0 = 3).  p = 2 C^1, 2 elements
    per direction, lambda = mu = 1, u = 0 on x = 0, trig loads.  Returns
    (problem, (patch_a, face_a, patch_b, face_b), orient)."""
    pats = []
    for k in range(2):
        cs = np.zeros((2 ** dim, dim))
        for c in range(2 ** dim):
            a = [(c >> d) & 1 for d in range(dim)]
            if k == 0:
                cs[c] = a
            elif dim == 2:
                cs[c] = [2 - a[0], 1 - a[1]]
            else:
                cs[c] = [1 + a[0], 1 - a[2], a[1]]
        bc = [FACE_FREE] * (2 * dim)
        if k == 0:
            bc[0] = FACE_DIRICHLET
        pats.append(dict(corners=cs, p=2, reg=1, n_el=[2] * dim, lam=1.0, mu=1.0, bc=bc))
    load = [(c, 1.0, [1] * dim, [0.1 * c] * dim) for c in range(dim)]
    face_b = 1 if dim == 2 else 0
    return dict(dim=dim, patches=pats, load=load, tol=1e-8), (0, 1, 1, face_b), (2 if dim == 2 else 3)


def make_nonconforming(p=3, n_els=(4, 8, 16), dim=3):
    """The paper's non-conforming test (Section 6, Table 1): the box
    (0,1) x (0,3) x (0,1) in three unit cubes stacked along y with n_els[k]
    elements per direction in cube k (4, 8, 16: each interface nested, the
    finer side refining the coarser by two), p C^{p-1}, E = 1, nu = 0.3, the
    exact solution u* = (cos x, z sin y, (x y z)^2): Dirichlet data u* on the
    whole outer boundary, body force -div sigma(u*).  ``dim`` = 2: the
    rectangle (0,1) x (0,3) in three unit squares, u* = (cos x, sin y)."""
    lam, mu = STEEL_LAM, STEEL_MU
    patches = []
    for k, ne in enumerate(n_els):
        cs = np.zeros((2 ** dim, dim))
        for c in range(2 ** dim):
            a = [(c >> d) & 1 for d in range(dim)]
            cs[c] = a
            cs[c, 1] += k
        bc = [FACE_DIRICHLET] * (2 * dim)
        if k > 0:
            bc[2] = FACE_FREE
        if k < len(n_els) - 1:
            bc[3] = FACE_FREE
        patches.append(dict(corners=cs, p=int(p), reg=int(p - 1), n_el=[int(ne)] * dim,
                            lam=lam, mu=mu, bc=bc))
    if dim == 3:
        sol = weak_scaling_solution
        force = lambda x: weak_scaling_force(x, lam, mu)  # noqa: E731
    else:
        sol = lambda x: np.stack([np.cos(x[:, 0]), np.sin(x[:, 1])], axis=1)  # noqa: E731
        # -div sigma for u = (cos x, sin y): sigma = diag(mu 2 u1' + lam div, mu 2 u2' + lam div)
        force = lambda x: np.stack([(2 * mu + lam) * np.cos(x[:, 0]),  # noqa: E731
                                    (2 * mu + lam) * np.sin(x[:, 1])], axis=1)
    return dict(name=f"nonconforming_p{p}", dim=dim, patches=patches, load=[], tol=1e-8,
                body_force=force, dirichlet=sol, exact=sol)


def make_weak_scaling(k=2, n_el=8, p=3):
    """Weak-scaling workload of the paper's third test (Section 6): the unit
    cube split into k^3 equal cubes, p = 3 C^2, n_el^3 elements per patch,
    E = 1, nu = 0.3, exact solution u* = (cos x, z sin y, (x y z)^2):
    traction sigma(u*) n on x = 0 and x = 1, Dirichlet data u* on the other
    four faces, body force f = -div sigma(u*).  Every entry is a closed-form
    function of the point (problem data), evaluated on arrays of points."""
    grid = (k, k, k)
    verts = _grid_vertices(grid, np.random.default_rng(0), 0.0)
    n_p = k ** 3
    lam, mu = STEEL_LAM, STEEL_MU
    patches = _patches_from_grid(grid, verts, p, p - 1, [n_el] * 3, np.full(n_p, lam), np.full(n_p, mu),
                                 [(1, 0), (1, 1), (2, 0), (2, 1)])
    for pd in patches:
        for f in (0, 1):
            if pd["bc"][f] == FACE_FREE and np.allclose(pd["corners"][[c for c in range(8) if (c & 1) == f], 0], f):
                pd["bc"][f] = FACE_TRACTION
    return dict(name=f"weak_{k}", dim=3, patches=patches, load=[], tol=1e-8,
                body_force=lambda x: weak_scaling_force(x, lam, mu),
                traction=lambda x, n: np.einsum("nij,nj->ni", weak_scaling_stress(x, lam, mu), n),
                dirichlet=weak_scaling_solution, exact=weak_scaling_solution)


def weak_scaling_solution(x):
    """u*(x) = (cos x, z sin y, (x y z)^2) at points x (n, 3)."""
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    return np.stack([np.cos(X), Z * np.sin(Y), (X * Y * Z) ** 2], axis=1)


def weak_scaling_stress(x, lam, mu):
    """sigma(u*) = mu (grad u* + grad u*^T) + lam (div u*) I at points x."""
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    g = np.zeros((len(x), 3, 3))  # g[n, c, a] = d u*_c / d x_a
    g[:, 0, 0] = -np.sin(X)
    g[:, 1, 1] = Z * np.cos(Y)
    g[:, 1, 2] = np.sin(Y)
    g[:, 2, 0] = 2 * X * Y ** 2 * Z ** 2
    g[:, 2, 1] = 2 * X ** 2 * Y * Z ** 2
    g[:, 2, 2] = 2 * X ** 2 * Y ** 2 * Z
    div = g[:, 0, 0] + g[:, 1, 1] + g[:, 2, 2]
    return mu * (g + np.swapaxes(g, 1, 2)) + lam * div[:, None, None] * np.eye(3)


def weak_scaling_force(x, lam, mu):
    """f = -div sigma(u*) = -mu lap u* - (mu + lam) grad div u* at points x."""
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    lap = np.stack([-np.cos(X), -Z * np.sin(Y), 2 * (Y ** 2 * Z ** 2 + X ** 2 * Z ** 2 + X ** 2 * Y ** 2)], axis=1)
    gdiv = np.stack([-np.cos(X) + 4 * X * Y ** 2 * Z, -Z * np.sin(Y) + 4 * X ** 2 * Y * Z,
                     np.cos(Y) + 2 * X ** 2 * Y ** 2], axis=1)
    return -mu * lap - (mu + lam) * gdiv


def redraw_parameters(prob, seed):
    """Second parameter draw (Lame per patch and load amplitudes) on the same
    geometry and discretisation; used for the adjoint target field."""
    rng = np.random.default_rng(seed)
    out = copy.deepcopy(prob)
    n_p = len(out["patches"])
    lam = _lognormal(rng, n_p)
    mu = _lognormal(rng, n_p)
    for k, pa in enumerate(out["patches"]):
        pa["lam"] = float(lam[k])
        pa["mu"] = float(mu[k])
    out["load"] = [(c, float(rng.normal()), k, ph) for (c, _a, k, ph) in out["load"]]
    return out


def with_overrides(prob, **kw):
    out = copy.deepcopy(prob)
    out.update(kw)
    return out


def random_vector(n, seed):
    """Seeded N(0,1) vector, shared input for both implementations."""
    return np.random.default_rng(seed).standard_normal(n)


CONFIGS = {
    "c1": make_c1,
    "c2": make_c2,
    "c3": make_c3,
    "c5": make_c5,
}
