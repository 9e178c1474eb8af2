"""One isogeometric patch: spline space, geometry map, and the physical
operators of compressible linear elasticity on it (paper Sections 2.2, 3, 4).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Conventions
  * A scalar spline field on a patch is an array of shape (n_d, ..., n_1):
    flattening it in C order gives the colexicographic numbering of
    Section 2.2 (the first parametric index runs fastest).
  * A vector field has a leading component axis: (dim, n_d, ..., n_1).
    Flattening gives the component-blocked patch vector of Section 4.
  * Quadrature: p+1 Gauss points per element and direction (the paper does
    not fix the rule; both implementations use this one).

Pins (tests/test_oracle_patch.py): the control net reproduces the
multilinear map, total volume of the unit box, symmetry, A R = 0 for the
rigid modes, strain energy of linear fields in closed form, the assembled
matrix equals the quadrature apply, the axis-aligned (l,l) block equals the
Kronecker form of Section 5.2 scaled by the side length, mass of constants.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from . import bspline


def apply_1d(T: np.ndarray, mats, lead: int = 0) -> np.ndarray:
    """Contract a tensor with one matrix per parametric direction.

    ``T`` has ``lead`` leading axes followed by (n_d, ..., n_1); ``mats[l]``
    (shape (r_l, n_l)) acts on direction l+1.  This is the Kronecker product
    (mats[d-1] x ... x mats[0]) applied to the colexicographic vector.
    """
    dim = len(mats)
    out = T
    for l, Ml in enumerate(mats):
        axis = lead + dim - 1 - l
        out = np.moveaxis(np.tensordot(Ml, out, axes=([1], [axis])), 0, axis)
    return out


def multilinear(corners: np.ndarray, eta: np.ndarray) -> np.ndarray:
    """Multilinear interpolant of the 2^d corners (corner index a1 + 2 a2 + 4 a3)
    at parametric points eta (..., d)."""
    dim = corners.shape[1]
    out = np.zeros(eta.shape[:-1] + (dim,))
    for c in range(2 ** dim):
        wgt = np.ones(eta.shape[:-1])
        for l in range(dim):
            a = (c >> l) & 1
            wgt = wgt * (eta[..., l] if a else 1.0 - eta[..., l])
        out += wgt[..., None] * corners[c]
    return out


class Patch:
    """Spline patch built from a ``workloads`` patch dictionary."""

    def __init__(self, pd: dict, dim: int):
        self.dim = dim
        self.p = int(pd["p"])
        self.reg = int(pd["reg"])
        self.n_el = list(pd["n_el"])
        self.lam = float(pd["lam"])
        self.mu = float(pd["mu"])
        self.bc = list(pd["bc"])
        if pd.get("knots") is not None:
            # explicit open knot vectors (Section 2.1); elements = non-empty spans
            self.knots = [np.asarray(pd["knots"][l], dtype=float) for l in range(dim)]
            self.n_el = [len(np.unique(k)) - 1 for k in self.knots]
        else:
            self.knots = [bspline.open_uniform_knots(self.n_el[l], self.p, self.reg)
                          for l in range(dim)]
        self.n = [bspline.n_functions(k, self.p) for k in self.knots]
        self.shape = tuple(reversed(self.n))  # (n_d, ..., n_1)
        self.n_nodes = int(np.prod(self.n))
        self.n_dof = dim * self.n_nodes
        if pd.get("ctrl") is not None:
            # explicit control net: the spline map sum_i X_i B_i (Section 2.2);
            # the corners are its corner control points
            self.ctrl = np.asarray(pd["ctrl"], dtype=float).reshape(self.shape + (dim,))
            idx = [tuple((n - 1) * ((c >> (dim - 1 - a)) & 1) for a, n in enumerate(self.shape))
                   for c in range(2 ** dim)]
            self.corners = np.array([self.ctrl[i] for i in idx])
            self.general = True
        else:
            # control points: images of the Greville points under the corner map
            self.corners = np.asarray(pd["corners"], dtype=float)
            g = [bspline.greville(k, self.p) for k in self.knots]
            grid = np.stack(np.meshgrid(*reversed(g), indexing="ij"), axis=-1)[..., ::-1]
            self.ctrl = multilinear(self.corners, grid)  # (n_d..n_1, dim)
            self.general = False
        # quadrature tables per direction
        self.qx, self.qw, self.V, self.D = [], [], [], []
        for l in range(dim):
            x, w, _ = bspline.quadrature(self.knots[l], self.p + 1)
            v, d = bspline.basis(self.knots[l], self.p, x, deriv=True)
            self.qx.append(x)
            self.qw.append(w)
            self.V.append(v)
            self.D.append(d)
        self._geom = None

    # ---------------------------------------------------------------- geometry
    def diameter(self) -> float:
        """H^(k): reading of "diameter" as the largest distance between two
        corners (exact for multilinear patches, the hull of their corners);
        for an explicit control net the largest distance between two control
        points (the patch lies in their hull; equal to the corner reading for
        a multilinear net)."""
        c = self.ctrl.reshape(-1, self.dim) if self.general else self.corners
        from scipy.spatial.distance import pdist
        return float(pdist(c).max())

    def geometry(self):
        """Physical points, weight w|det J| and J^{-1} at the tensor Gauss
        points, from the spline map F = sum_i X_i B_i (isoparametric)."""
        if self._geom is not None:
            return self._geom
        dim = self.dim
        X = np.moveaxis(self.ctrl, -1, 0)  # (dim, n_d..n_1)
        Fq = apply_1d(X, self.V, lead=1)
        J = np.zeros(Fq.shape[1:] + (dim, dim))  # J[..., x, a] = dF_x/deta_a
        for a in range(dim):
            mats = [self.D[l] if l == a else self.V[l] for l in range(dim)]
            J[..., :, a] = np.moveaxis(apply_1d(X, mats, lead=1), 0, -1)
        det = np.linalg.det(J)
        if np.any(det <= 0):
            raise ValueError("geometry map is not orientation preserving")
        Jinv = np.linalg.inv(J)  # Jinv[..., a, x]
        w = np.ones(Fq.shape[1:])
        for l in range(dim):
            shp = [1] * dim
            shp[dim - 1 - l] = -1
            w = w * self.qw[l].reshape(shp)
        self._geom = (np.moveaxis(Fq, 0, -1), w * det, Jinv)
        return self._geom

    # ------------------------------------------------------- physical operators
    def _ref_grads(self, u):
        """Parametric gradients of each component at the Gauss points:
        out[c, b] = d/deta_b of u_c."""
        dim = self.dim
        out = []
        for c in range(dim):
            row = []
            for b in range(dim):
                mats = [self.D[l] if l == b else self.V[l] for l in range(dim)]
                row.append(apply_1d(u[c], mats))
            out.append(row)
        return np.array(out)

    def stiffness_apply(self, u: np.ndarray, lam=None, mu=None) -> np.ndarray:
        """y = A^(k) u by quadrature of the bilinear form of Section 3:
        a(u, v) = int sigma(u) : grad v,  sigma = mu (grad u + grad u^T) +
        lam (div u) I  (equal to 2 mu eps(u):eps(v) + lam div u div v).
        ``u`` has shape (dim, n_d..n_1)."""
        lam = self.lam if lam is None else lam
        mu = self.mu if mu is None else mu
        dim = self.dim
        _, wdet, Jinv = self.geometry()
        gref = self._ref_grads(u)  # (c, b, q...)
        grad = np.einsum("cb...,...bx->...cx", gref, Jinv)  # grad[q, c, x]
        div = np.trace(grad, axis1=-2, axis2=-1)
        sig = mu * (grad + np.swapaxes(grad, -1, -2))
        sig = sig + lam * div[..., None, None] * np.eye(dim)
        flux = np.einsum("...cx,...ax->ca...", sig, Jinv) * wdet  # flux[c, a, q]
        y = np.zeros((dim,) + self.shape)
        for c in range(dim):
            for a in range(dim):
                mats = [(self.D[l] if l == a else self.V[l]).T for l in range(dim)]
                y[c] += apply_1d(flux[c, a], mats)
        return y

    def _kron(self, mats):
        out = sp.csr_matrix(np.ones((1, 1)))
        for Ml in reversed(mats):  # direction d first (slowest)
            out = sp.kron(out, sp.csr_matrix(Ml), format="csr")
        return out

    def _element_tables(self):
        """Per element: global node and Gauss-point indices of its (p+1)^d
        local functions / points, and the local parametric gradient tables
        g_a[e, Q, I] = d/deta_a of local basis I at local point Q."""
        dim, P = self.dim, self.p + 1
        lb, lq = [], []
        for l in range(dim):
            bl, ql = [], []
            for e in range(self.n_el[l]):
                q = np.arange(e * P, (e + 1) * P)
                nz = np.nonzero(np.any(self.V[l][q] != 0, axis=0))[0]
                assert len(nz) == P
                bl.append(nz)
                ql.append(q)
            lb.append(np.array(bl))
            lq.append(np.array(ql))
        els = np.array(list(itertools.product(*[range(n) for n in reversed(self.n_el)])))[:, ::-1]
        loc = np.array(list(itertools.product(range(P), repeat=dim)))[:, ::-1]
        nq = [len(x) for x in self.qx]
        node = np.zeros((len(els), len(loc)), dtype=np.int64)
        qpt = np.zeros((len(els), len(loc)), dtype=np.int64)
        sn, sq = 1, 1
        for l in range(dim):
            node += lb[l][els[:, l]][:, loc[:, l]] * sn
            qpt += lq[l][els[:, l]][:, loc[:, l]] * sq
            sn *= self.n[l]
            sq *= nq[l]
        grads = []
        for a in range(dim):
            g = 1.0
            for l in range(dim):
                T = self.D[l] if l == a else self.V[l]
                t = T[lq[l][:, :, None], lb[l][:, None, :]]  # (n_el, P, P)
                g = g * t[els[:, l]][:, loc[:, l]][:, :, loc[:, l]]
            grads.append(g)
        return node, qpt, grads

    def stiffness_matrix(self, lam=None, mu=None) -> sp.csr_matrix:
        """Assembled A^(k) (component blocks of Section 4), element by element:
        A[(c,i),(c',j)] = sum_e sum_q w|J| [mu d_cc' g_i.g_j + mu g_i[c'] g_j[c]
                                            + lam g_i[c] g_j[c']],
        with physical gradients g = J^{-T} (parametric gradient).  Local
        element matrices are summed into the global sparse matrix."""
        lam = self.lam if lam is None else lam
        mu = self.mu if mu is None else mu
        dim = self.dim
        _, wdet, Jinv = self.geometry()
        node, qpt, grads = self._element_tables()
        W = wdet.reshape(-1)[qpt]                       # (E, Q)
        Ji = Jinv.reshape(-1, dim, dim)[qpt]            # (E, Q, a, x)
        rows, cols, vals = [], [], []
        nn = self.n_nodes
        for c in range(dim):
            for cp in range(dim):
                K = 0.0
                for b in range(dim):
                    T = 0.0
                    for a in range(dim):
                        coef = mu * (c == cp) * np.einsum("eqx,eqx->eq", Ji[:, :, a, :], Ji[:, :, b, :])
                        coef = coef + mu * Ji[:, :, a, cp] * Ji[:, :, b, c]
                        coef = coef + lam * Ji[:, :, a, c] * Ji[:, :, b, cp]
                        T = T + grads[a] * (W * coef)[:, :, None]
                    K = K + np.matmul(np.ascontiguousarray(np.swapaxes(T, 1, 2)), grads[b])
                rows.append(np.broadcast_to(c * nn + node[:, :, None], K.shape).reshape(-1))
                cols.append(np.broadcast_to(cp * nn + node[:, None, :], K.shape).reshape(-1))
                vals.append(K.reshape(-1))
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.n_dof, self.n_dof))
        return A.tocsr()

    def mass_matrix_scalar(self) -> sp.csr_matrix:
        """Physical mass of one component: M[i,j] = int B_i B_j dx (Section 4)."""
        _, wdet, _ = self.geometry()
        E0 = self._kron(self.V)
        return (E0.T @ sp.diags(wdet.reshape(-1)) @ E0).tocsr()

    def mass_apply(self, u: np.ndarray) -> np.ndarray:
        """Block-diagonal physical mass applied to a vector field (dim, ...)."""
        _, wdet, _ = self.geometry()
        VT = [v.T for v in self.V]
        return np.array([apply_1d(wdet * apply_1d(u[c], self.V), VT)
                         for c in range(self.dim)])

    # ----------------------------------------------------------------- loads
    def body_force(self, modes, amps=None) -> np.ndarray:
        """f^(k)_(c,i) = int f_c B_i dx for f_c(x) = sum_j a_j prod_d
        sin(pi k_jd x_d + phi_jd) over the modes of component c."""
        xq, wdet, _ = self.geometry()
        VT = [v.T for v in self.V]
        out = np.zeros((self.dim,) + self.shape)
        for j, (comp, amp, k, ph) in enumerate(modes):
            a = amp if amps is None else amps[j]
            val = np.ones(wdet.shape)
            for d in range(self.dim):
                val = val * np.sin(np.pi * k[d] * xq[..., d] + ph[d])
            out[comp] += a * apply_1d(wdet * val, VT)
        return out

    def body_force_field(self, fn) -> np.ndarray:
        """f^(k)_(c,i) = int f_c B_i dx for a body force given as a function
        f(x) of an array of points (n, dim) -> (n, dim) (Section 3, the load
        term), by the Gauss rule of the patch."""
        xq, wdet, _ = self.geometry()
        dim = self.dim
        f = np.asarray(fn(xq.reshape(-1, dim)), dtype=float).reshape(xq.shape)
        VT = [v.T for v in self.V]
        return np.array([apply_1d(wdet * f[..., c], VT) for c in range(dim)])

    def mode_loads(self, modes) -> np.ndarray:
        """Load vector of each mode with unit amplitude: (n_modes, dim, ...)."""
        return np.array([self.body_force([(c, 1.0, k, ph)]) for (c, _a, k, ph) in modes])

    def traction(self, face: int, gfun) -> np.ndarray:
        """int_face g . v ds for the face ``face`` (2*dir + side), g = gfun(x, n)
        for arrays of points and outward unit normals (n, dim) -> (n, dim)."""
        dim = self.dim
        fd, side = face // 2, face % 2
        X = np.moveaxis(self.ctrl, -1, 0)
        # 1D tables: along fd evaluate at the end point; elsewhere Gauss points
        mats_v, mats_d, wts = [], [], []
        for l in range(dim):
            if l == fd:
                v, d = bspline.basis(self.knots[l], self.p, [float(side)], deriv=True)
                mats_v.append(v)
                mats_d.append(d)
                wts.append(np.ones(1))
            else:
                mats_v.append(self.V[l])
                mats_d.append(self.D[l])
                wts.append(self.qw[l])
        xq = np.moveaxis(apply_1d(X, mats_v, lead=1), 0, -1)
        J = np.zeros(xq.shape[:-1] + (dim, dim))
        for a in range(dim):
            m = [mats_d[l] if l == a else mats_v[l] for l in range(dim)]
            J[..., :, a] = np.moveaxis(apply_1d(X, m, lead=1), 0, -1)
        tang = [J[..., :, a] for a in range(dim) if a != fd]
        if dim == 2:
            t = tang[0]
            nvec = np.stack([t[..., 1], -t[..., 0]], axis=-1)
        else:
            nvec = np.cross(tang[0], tang[1])
        area = np.linalg.norm(nvec, axis=-1)
        nvec = nvec / area[..., None]
        # orient outward: compare with the parametric normal pushed forward
        Jinv_t = np.linalg.inv(J)  # rows = gradients of eta_a
        grad_eta = Jinv_t[..., fd, :]
        sgn = np.sign(np.sum(grad_eta * nvec, axis=-1)) * (1 if side == 1 else -1)
        nvec = nvec * sgn[..., None]
        w = np.ones(area.shape)
        for l in range(dim):
            shp = [1] * dim
            shp[dim - 1 - l] = -1
            w = w * wts[l].reshape(shp)
        g = np.asarray(gfun(xq.reshape(-1, dim), nvec.reshape(-1, dim)), dtype=float)
        g = g.reshape(xq.shape) * (w * area)[..., None]
        VT = [m.T for m in mats_v]
        return np.array([apply_1d(g[..., c], VT) for c in range(dim)])

    # ----------------------------------------------------------- rigid modes
    def rigid_modes(self) -> np.ndarray:
        """Raw rigid-body modes as coefficient vectors (Section 4): d
        translations, then the infinitesimal rotations built from the
        control-point coordinates.  3D: (0,x3,-x2), (x3,0,-x1), (x2,-x1,0);
        2D (not printed in the paper): (x2, -x1).  Shape (n_modes, n_dof)."""
        dim = self.dim
        X = [self.ctrl[..., l] for l in range(dim)]
        z = np.zeros(self.shape)
        o = np.ones(self.shape)
        modes = []
        for c in range(dim):
            modes.append([o if cc == c else z for cc in range(dim)])
        if dim == 3:
            x1, x2, x3 = X
            modes.append([z, x3, -x2])
            modes.append([x3, z, -x1])
            modes.append([x2, -x1, z])
        else:
            x1, x2 = X
            modes.append([x2, -x1])
        return np.array([np.concatenate([m.reshape(-1) for m in md]) for md in modes])

    # ------------------------------------------------------------ index sets
    def face_nodes(self, face: int) -> np.ndarray:
        """Colexicographic node indices with index 1 (side 0) or m (side 1)
        in direction face//2."""
        fd, side = face // 2, face % 2
        idx = np.arange(self.n_nodes).reshape(self.shape)
        axis = self.dim - 1 - fd
        sl = [slice(None)] * self.dim
        sl[axis] = 0 if side == 0 else self.n[fd] - 1
        return idx[tuple(sl)].reshape(-1)

    def gamma_mask(self) -> np.ndarray:
        """Nodes of the local interface Gamma (Section 4): some index equals
        1 or m_l (open knots make exactly these functions nonzero on the
        patch boundary)."""
        m = np.zeros(self.shape, dtype=bool)
        for l in range(self.dim):
            axis = self.dim - 1 - l
            sl = [slice(None)] * self.dim
            sl[axis] = 0
            m[tuple(sl)] = True
            sl[axis] = self.n[l] - 1
            m[tuple(sl)] = True
        return m


def all_offsets(dim, p):
    return list(itertools.product(range(-p, p + 1), repeat=dim))
