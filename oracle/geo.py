"""Inexact local solvers with geometry inclusion (paper Section 5.2.3:
eq. geo_A, eq. geo_S, eq. tildeshur; Remark 1, eq. inexact_S_non_r), the
variant behind the paper's numerical results (Section 6).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

What is computed, per patch k and displacement component l:
  * the coefficient matrix of the (l,l) block of the stiffness pulled back
    to the parameter domain,
        C_l = [mu J^{-1} J^{-T} + (mu + lam) J^{-1} e_l e_l^T J^{-T}] |det J|,
    at the tensor Gauss points of the patch;
  * a separable approximation of its diagonal,
        [C_l]_ii(eta) ~ nu_{l,i}(eta_i) prod_{m != i} beta_{l,m}(eta_m);
  * the univariate weighted matrices K~_{l,m} = int nu_{l,m} b_i' b_j' and
    M~_{l,m} = int beta_{l,m} b_i b_j, A~_l = sum_m (M~_{l,d} x .. K~_{l,m}
    .. x M~_{l,1}) and M~_l = M~_{l,d} x .. x M~_{l,1};
  * D_{A,l} = diag(A_ll + H^-2 M) / diag(A~_l + H^-2 M~_l) and
    D_{S,l} = diag(A_ll) / diag(A~_l), with A_ll the (l,l) block of the
    physical stiffness and M the physical mass;
  * P~_A^{-1} per block: D_{A,l}^{-1/2} (A~_l + H^-2 M~_l)^{-1} D_{A,l}^{-1/2},
    the middle factor by fast diagonalization with the pencils
    (K~_{l,m}, M~_{l,m}) (d^2 pencils per patch, eigenvalues
    H^-2 + sum_m D_{l,m});
  * S~^(k) per block: D_{S,l}^{1/2} S~_l D_{S,l}^{1/2}, S~_l the Schur
    complement of A~_l on Gamma (harmonic extension with the interior
    pencils), and P~_S = (B B^T)^{-1} B sum_k S~^(k) B^T (B B^T)^{-1}.
    The H scaling is that of the exact local solvers: H^-2 on the mass in
    P~_A, none in P~_S.

Reading of the separable approximation (the paper cites an algorithm that
it does not print): a least-squares fit in log space over the patch's
tensor Gauss points, weighted by the product Gauss weights, of the d
equations log [C_l]_ii = log nu_{l,i} + sum_{m != i} log beta_{l,m}
together with log |det J| = sum_m log beta_{l,m}, all with equal weight.
The last equation ties prod_m beta_{l,m} to the physical mass weight; the
fit is then determined up to constant factors s_m (prod s_m = 1) on
beta_{l,m} with nu_{l,m} scaled by s_m, which leave A~_l and M~_l unchanged.
With product weights the fit separates (ANOVA decomposition): writing
y_0 = log |det J| and y_i = log [C_l]_ii, ybar_i for the weighted mean and
y_i^(m) for the weighted mean over every direction but m minus ybar_i,
    log nu_{l,m}   = y_m^(m) + ybar_m - (d-1) ybar_0 / d,
    log beta_{l,m} = (1/d) sum_{i in {0} u {1..d} \\ {m}} y_i^(m) + ybar_0 / d.
It is exact whenever log [C_l]_ii and log |det J| are sums of univariate
functions consistent with one set of beta's, e.g. on axis-aligned boxes.
Pins (tests/test_oracle_geo.py): the closed form equals a brute-force
weighted least-squares solve on small grids, exactness on axis-aligned
boxes (where P~_A is the exact (A_ll + H^-2 M)^{-1}), FD equals a dense
solve of the assembled Kronecker system, the diagonals equal those of the
assembled matrices, S~_l equals the dense Schur complement.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .patch import apply_1d


def _grid_weights(pa):
    """Product Gauss weights W(q) on the patch's tensor grid (sum 1)."""
    W = 1.0
    for l in range(pa.dim):
        shp = [1] * pa.dim
        shp[pa.dim - 1 - l] = -1
        W = W * pa.qw[l].reshape(shp)
    return W


def jacobian(pa):
    """J[q..., x, a] = dF_x / deta_a at the tensor Gauss points."""
    dim = pa.dim
    X = np.moveaxis(pa.ctrl, -1, 0)
    J = None
    for a in range(dim):
        mats = [pa.D[l] if l == a else pa.V[l] for l in range(dim)]
        col = np.moveaxis(apply_1d(X, mats, lead=1), 0, -1)
        if J is None:
            J = np.zeros(col.shape + (dim,))
        J[..., :, a] = col
    return J


def coefficient(pa, l):
    """C_l at the Gauss points: array (q..., d, d)."""
    J = jacobian(pa)
    Ji = np.linalg.inv(J)                    # Ji[..., a, x] = (J^{-1})_{a x}
    det = np.abs(np.linalg.det(J))
    JJ = np.einsum("...ax,...bx->...ab", Ji, Ji)
    el = np.einsum("...a,...b->...ab", Ji[..., :, l], Ji[..., :, l])
    return (pa.mu * JJ + (pa.mu + pa.lam) * el) * det[..., None, None], det


def _marginal(y, W, pa, m):
    """Weighted mean of y over every direction but m (function of eta_m)."""
    dim = pa.dim
    axes = tuple(a for a in range(dim) if a != dim - 1 - m)
    w_m = pa.qw[m].reshape([-1 if a == dim - 1 - m else 1 for a in range(dim)])
    return (y * W).sum(axis=axes).reshape(-1) / w_m.reshape(-1)


def separable_fit(pa, l):
    """(nu[m], beta[m]) at the 1D Gauss points of each direction m (the
    closed form of the module docstring)."""
    dim = pa.dim
    C, det = coefficient(pa, l)
    W = _grid_weights(pa)
    ys = [np.log(det)] + [np.log(C[..., i, i]) for i in range(dim)]
    ybar = [float((y * W).sum()) for y in ys]
    nu, beta = [], []
    for m in range(dim):
        main = [_marginal(y, W, pa, m) - yb for y, yb in zip(ys, ybar)]
        a = main[1 + m] + ybar[1 + m] - (dim - 1) * ybar[0] / dim
        others = [main[0]] + [main[1 + i] for i in range(dim) if i != m]
        b = sum(others) / dim + ybar[0] / dim
        nu.append(np.exp(a))
        beta.append(np.exp(b))
    return nu, beta


def weighted_1d(pa, m, nu, beta):
    """K~ = int nu b' b', M~ = int beta b b on [0, 1] by the Gauss rule."""
    V, D, w = pa.V[m], pa.D[m], pa.qw[m]
    K = D.T @ ((w * nu)[:, None] * D)
    M = V.T @ ((w * beta)[:, None] * V)
    return K, M


def _outer_sum(vecs):
    dim = len(vecs)
    T = 0.0
    for m, v in enumerate(vecs):
        shp = [1] * dim
        shp[dim - 1 - m] = -1
        T = T + v.reshape(shp)
    return T


def _outer_prod(vecs):
    dim = len(vecs)
    T = 1.0
    for m, v in enumerate(vecs):
        shp = [1] * dim
        shp[dim - 1 - m] = -1
        T = T * v.reshape(shp)
    return T


def stiffness_diagonal(pa, l, C=None):
    """diag of the (l,l) block of the physical stiffness:
    sum_{a,b} int [C_l]_ab dB_i/deta_a dB_i/deta_b, by sum factorisation
    with the squared / mixed univariate tables."""
    dim = pa.dim
    if C is None:
        C, _ = coefficient(pa, l)
    W = _grid_weights(pa)
    out = 0.0
    for a in range(dim):
        for b in range(dim):
            mats = []
            for m in range(dim):
                Fa = pa.D[m] if m == a else pa.V[m]
                Fb = pa.D[m] if m == b else pa.V[m]
                mats.append((Fa * Fb).T)
            out = out + apply_1d(W * C[..., a, b], mats)
    return out


def mass_diagonal(pa):
    """diag of the physical scalar mass: int B_i^2 |det J|."""
    _, det = coefficient(pa, 0)
    W = _grid_weights(pa)
    return apply_1d(W * det, [(v * v).T for v in pa.V])


class GeoPatch:
    """Geometry-inclusion data of one patch (all components)."""

    def __init__(self, pa, eig_driver=None):
        self.pa = pa
        dim = pa.dim
        H = pa.diameter()
        self.h2 = H ** -2
        Md = mass_diagonal(pa)
        self.blocks = []
        for l in range(dim):
            C, _ = coefficient(pa, l)
            nu, beta = separable_fit(pa, l)
            K, M = zip(*[weighted_1d(pa, m, nu[m], beta[m]) for m in range(dim)])
            fd = []
            for m in range(dim):
                D, U = sla.eigh(K[m], M[m], driver=eig_driver)
                Di, Ui = sla.eigh(K[m][1:-1, 1:-1], M[m][1:-1, 1:-1], driver=eig_driver)
                fd.append(dict(D=D, U=U, Di=Di, Ui=Ui))
            kd = [np.diag(K[m]) for m in range(dim)]
            md = [np.diag(M[m]) for m in range(dim)]
            At_diag = 0.0
            for m in range(dim):
                At_diag = At_diag + _outer_prod([kd[n] if n == m else md[n] for n in range(dim)])
            Mt_diag = _outer_prod(md)
            A_diag = stiffness_diagonal(pa, l, C)
            self.blocks.append(dict(
                nu=nu, beta=beta, K=list(K), M=list(M), fd=fd,
                DA=(A_diag + self.h2 * Md) / (At_diag + self.h2 * Mt_diag),
                DS=A_diag / At_diag,
                A_diag=A_diag, At_diag=At_diag))

    def fd_solve(self, l, r):
        """(A~_l + H^-2 M~_l)^{-1} r by fast diagonalization (Algorithm 1
        with the weighted pencils): eigenvalues H^-2 + sum_m D_{l,m}."""
        fd = self.blocks[l]["fd"]
        U = [f["U"] for f in fd]
        rt = apply_1d(r, [u.T for u in U])
        lam = self.h2 + _outer_sum([f["D"] for f in fd])
        return apply_1d(rt / lam, U)

    def fd_solve_interior(self, l, r):
        """((A~_l)_II)^{-1} r: eigenvalues sum_m D~_{l,m} of the interior pencils."""
        fd = self.blocks[l]["fd"]
        U = [f["Ui"] for f in fd]
        rt = apply_1d(r, [u.T for u in U])
        return apply_1d(rt / _outer_sum([f["Di"] for f in fd]), U)

    def PA_inv(self, l, r):
        """Block l of (P~_A^{inex,(k)})^{-1}: D_A^{-1/2} (A~_l + H^-2 M~_l)^{-1} D_A^{-1/2}."""
        s = self.blocks[l]["DA"] ** -0.5
        return s * self.fd_solve(l, s * r)

    def apply_At(self, l, x):
        """A~_l x = sum_m (M~_{l,d} x .. K~_{l,m} .. x M~_{l,1}) x."""
        b = self.blocks[l]
        y = 0.0
        for m in range(self.pa.dim):
            y = y + apply_1d(x, [b["K"][n] if n == m else b["M"][n] for n in range(self.pa.dim)])
        return y

    def apply_St(self, l, theta_full):
        """S~_l theta by harmonic extension with A~_l; interior of theta
        ignored, of the result zero."""
        gm = self.pa.gamma_mask()
        inner = tuple(slice(1, -1) for _ in range(self.pa.dim))
        v = np.where(gm, theta_full, 0.0)
        t = self.apply_At(l, v)
        v[inner] = -self.fd_solve_interior(l, t[inner])
        return np.where(gm, self.apply_At(l, v), 0.0)

    def S_block(self, l, theta_full):
        """Block l of S~^(k) (eq. tildeshur): D_S^{1/2} S~_l D_S^{1/2}."""
        s = np.sqrt(self.blocks[l]["DS"])
        return s * self.apply_St(l, s * theta_full)


class GeoPreconditioner:
    """P~_A^inex (eq. geo_A) and P~_S^{inex-nr} (eq. inexact_S_non_r) of an
    ``AFIETI`` system."""

    def __init__(self, sysm):
        self.sysm = sysm
        self.patches = [GeoPatch(pa, sysm.eig_driver) for pa in sysm.patches]

    def apply_PA_inv(self, r):
        s = self.sysm
        return s.join([np.array([g.PA_inv(l, rk[l]) for l in range(s.dim)])
                       for g, rk in zip(self.patches, s.split(r))])

    def apply_PS(self, y, variant="nr"):
        """(B B^T)^{-1} B S~ B^T (B B^T)^{-1} y; ``variant="plain"`` drops
        (B B^T)^{-1} (eq. geo_S)."""
        s = self.sysm
        z = s._BBt_lu.solve(y) if variant == "nr" else y
        v = s.B.T @ z
        out = [np.array([g.S_block(l, vk[l]) for l in range(s.dim)])
               for g, vk in zip(self.patches, s.split(v))]
        t = s.B @ s.join(out)
        return s._BBt_lu.solve(t) if variant == "nr" else t
