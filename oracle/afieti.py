"""All-Floating IETI with inexact Fast-Diagonalization local solvers
(paper Sections 4, 5.2, 5.2.1 and Remark 1), written out plainly in FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Readings of points the paper leaves open:
  * Jump matrix B: the paper only requires Bv = 0 <=> continuity and
    homogeneous Dirichlet data, with no redundant rows.  Reading: a "star"
    to the lowest patch index.  For every geometric node with copies
    k_1 < ... < k_r and every component: a node on the Dirichlet boundary
    gets the r rows e_{k_j}; any other node gets the r-1 rows
    e_{k_1} - e_{k_j}.  Rows are ordered by (component, node, j); nodes are
    ordered by (lowest patch, local colexicographic index in that patch).
  * Rigid modes in 2D: two translations and (x2, -x1).
  * lambda_0: any solution of G^T lambda_0 = R^T f is allowed; reading: the
    minimal-norm one, G (G^T G)^{-1} R^T f.
  * H^(k): largest distance between two patch corners (for an explicit
    control net: between two control points).
  * P_S^{inex-nr}: Remark 1 with S replaced by S-hat and the per-patch factor
    (H^(k))^{d-2} of the inexact P_S kept; B_Gamma B_Gamma^T = B B^T because
    B only touches interface unknowns.
  * The per-patch operators in the inexact P_S are summed (each block of the
    printed block-diagonal display is N_c x N_c).
  * MINRES: the preconditioned Lanczos/Givens form (Paige-Saunders), x0 = 0,
    stopped when the preconditioned residual norm |eta| drops below
    tol * gamma_1 (the residual norm is not stated in the paper).
  * Non-homogeneous Dirichlet data (the paper only says the right-hand side
    changes): the spline coefficients of the data are its values at the
    control points (Schoenberg's variation-diminishing approximation; on
    the multilinear patches here a control point is the image of its
    Greville point), so the constraint row of a Dirichlet copy reads
    u_i = g_D(X_i)[c] and B u = c.  This is exact for g_D linear and of
    second order in h otherwise.  The solve lifts them: u_D = B^T (B B^T)^{-1} c satisfies
    B u_D = c, the projected system of Section 4 is solved for u - u_D with
    right-hand side f - A u_D and homogeneous constraints, and u_D is added
    back.
  * Loads: the trigonometric modes, a body force given as a function of
    the point, and a traction g(x, n) on the faces marked 2 (Gamma_N), as in
    the linear form of Section 3.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.spatial import cKDTree

from .patch import Patch, apply_1d


class SingularCoarse(Exception):
    """G^T G is not positive definite (not enough constraints)."""


class Breakdown(Exception):
    """MINRES met gamma^2 <= 0: the preconditioner is not positive definite."""


class AFIETI:
    """The AF-IETI system of one problem (``workloads`` dictionary)."""

    def __init__(self, prob: dict, assembled: bool | None = None, geometry: bool = False,
                 eig_driver: str | None = None, exact: bool = False):
        self.dim = int(prob["dim"])
        self.patches = [Patch(pd, self.dim) for pd in prob["patches"]]
        self.load_modes = prob["load"]
        self.body_force = prob.get("body_force")
        self.traction = prob.get("traction")
        self.dirichlet = prob.get("dirichlet")
        # explicit interface list (patch_a, face_a, patch_b, face_b, orient),
        # or None: every coinciding pair of boundary control points is glued
        itf = prob.get("interfaces")
        self.interfaces = None if itf is None or len(itf) == 0 else [tuple(int(v) for v in e) for e in itf]
        self.tol = float(prob.get("tol", 1e-8))
        # LAPACK driver of the generalised eigensolves (scipy.linalg.eigh's
        # default when None); another driver perturbs U and D at rounding
        # level, which the tests use to measure the solve's own sensitivity
        self.eig_driver = eig_driver
        sizes = [pa.n_dof for pa in self.patches]
        self.offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        self.n_dof = int(self.offsets[-1])
        if assembled is None:
            assembled = self.n_dof <= 60000
        self.assembled = assembled
        self.A = [pa.stiffness_matrix() for pa in self.patches] if assembled else None
        self._build_numbering()
        self._build_B()
        self._build_dirichlet_data()
        self._build_coarse()
        self._build_fd()
        # other local solvers replace the preconditioner's blocks: geometry
        # inclusion (Section 5.2.3) or the exact ones (Section 5.1)
        self.geo = None
        if geometry and exact:
            raise ValueError("choose one of geometry inclusion and exact local solvers")
        if geometry:
            from .geo import GeoPreconditioner
            self.geo = GeoPreconditioner(self)
        if exact:
            from .exact import ExactPreconditioner
            self.geo = ExactPreconditioner(self)

    # ------------------------------------------------------------ DOF helpers
    def split(self, x):
        """Patch-stacked vector -> list of (dim, n_d..n_1) arrays."""
        out = []
        for k, pa in enumerate(self.patches):
            out.append(x[self.offsets[k]:self.offsets[k + 1]].reshape((self.dim,) + pa.shape))
        return out

    def join(self, parts):
        return np.concatenate([np.asarray(p).reshape(-1) for p in parts])

    def dof(self, k, c, i):
        return int(self.offsets[k] + c * self.patches[k].n_nodes + i)

    # ------------------------------------------------------------- numbering
    def _build_numbering(self):
        """Geometric nodes: copies of a control point shared by patches that
        meet conformingly (Section 2.2).  Two boundary copies are the same
        node when their control points coincide (equal knots and a common
        face map); with an explicit interface list, only copies on the two
        faces of a listed pair are identified (directly, or through other
        listed pairs)."""
        # non-conforming (nested) interfaces: the finer side's face
        # coefficients are glued to the coarse trace by rows of their own
        # (_build_B), not identified with other copies; on the Dirichlet
        # boundary too, so that the trace is continuous there as well
        from .nonconforming import find_interfaces
        self.nonconforming = find_interfaces(self, self.interfaces)
        glued = set()
        for nc in self.nonconforming:
            for i in nc["snodes"]:
                glued.add((nc["slave"], int(i)))
        recs = []  # (patch, local node, coords)
        for k, pa in enumerate(self.patches):
            gm = pa.gamma_mask().reshape(-1)
            nodes = np.nonzero(gm)[0]
            X = pa.ctrl.reshape(-1, self.dim)[nodes]
            for i, x in zip(nodes, X):
                if (k, int(i)) not in glued:
                    recs.append((k, int(i), x))
        pts = np.array([r[2] for r in recs])
        if glued:
            tree = cKDTree(pts)
            masters = {nc["slave"]: set() for nc in self.nonconforming}
            for nc in self.nonconforming:
                masters[nc["slave"]].add(nc["master"])
            for (k, i) in glued:
                x = self.patches[k].ctrl.reshape(-1, self.dim)[i]
                for j in tree.query_ball_point(x, 1e-9):
                    if recs[j][0] != k and recs[j][0] not in masters[k]:
                        raise NotImplementedError("a non-conforming face coefficient is shared with a third patch")
        parent = list(range(len(recs)))

        def find(a):
            while parent[a] != a:
                parent[a] = parent[parent[a]]
                a = parent[a]
            return a

        def unite(a, b):
            ra, rb = find(a), find(b)
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)

        if self.interfaces is None:
            # every pair of coinciding boundary control points
            for a, b in cKDTree(pts).query_pairs(r=1e-9):
                unite(a, b)
        else:
            # only across the listed face pairs: each control point of one
            # face coincides with one of the other face (conforming faces)
            rec_of = {(k, i): j for j, (k, i, _) in enumerate(recs)}
            ncpairs = {(nc["slave"], nc["sface"]) for nc in self.nonconforming}
            for ka, fa, kb, fb, _orient in self.interfaces:
                if (ka, fa) in ncpairs or (kb, fb) in ncpairs:
                    continue
                ia = self.patches[ka].face_nodes(fa)
                ib = self.patches[kb].face_nodes(fb)
                ja = [rec_of[(ka, int(i))] for i in ia]
                jb = [rec_of[(kb, int(i))] for i in ib]
                dist, near = cKDTree(pts[jb]).query(pts[ja])
                if len(ia) != len(ib) or np.max(dist) > 1e-9 or len(set(near.tolist())) != len(ib):
                    raise ValueError("listed interface faces do not coincide")
                for x, y in zip(ja, near):
                    unite(x, jb[y])
        groups = {}
        for idx in range(len(recs)):
            groups.setdefault(find(idx), []).append(idx)
        classes = []
        for members in groups.values():
            copies = sorted((recs[m][0], recs[m][1]) for m in members)
            ks = [c[0] for c in copies]
            if len(set(ks)) != len(ks):
                raise ValueError("two control points of one patch coincide")
            classes.append(copies)
        classes.sort(key=lambda cp: cp[0])
        self.classes = classes

    def _on_dirichlet(self, k, i):
        pa = self.patches[k]
        for f in range(2 * self.dim):
            if pa.bc[f] == 1 and i in self._face_sets(k)[f]:
                return True
        return False

    def _face_sets(self, k):
        if not hasattr(self, "_fs"):
            self._fs = {}
        if k not in self._fs:
            pa = self.patches[k]
            self._fs[k] = [set(pa.face_nodes(f).tolist()) for f in range(2 * self.dim)]
        return self._fs[k]

    def _build_B(self):
        """Jump/constraint matrix B (Section 4), star pattern (module doc)."""
        rows, cols, vals = [], [], []
        self.dirichlet_class = [any(self._on_dirichlet(k, i) for (k, i) in cp)
                                for cp in self.classes]
        r = 0
        dir_rows = []  # (row, patch, node, component) of the Dirichlet rows
        for c in range(self.dim):
            for cp, isd in zip(self.classes, self.dirichlet_class):
                if isd:
                    for (k, i) in cp:
                        rows.append(r)
                        cols.append(self.dof(k, c, i))
                        vals.append(1.0)
                        dir_rows.append((r, k, i, c))
                        r += 1
                else:
                    k1, i1 = cp[0]
                    for (k, i) in cp[1:]:
                        rows += [r, r]
                        cols += [self.dof(k1, c, i1), self.dof(k, c, i)]
                        vals += [1.0, -1.0]
                        r += 1
            # non-conforming interfaces: u_f(i) - sum_j T_ij u_c(j) = 0 for
            # every coefficient of the finer face
            for nc in self.nonconforming:
                ks, km = nc["slave"], nc["master"]
                for a, i in enumerate(nc["snodes"]):
                    rows.append(r)
                    cols.append(self.dof(ks, c, int(i)))
                    vals.append(1.0)
                    for b in np.nonzero(np.abs(nc["T"][a]) > 0)[0]:
                        rows.append(r)
                        cols.append(self.dof(km, c, int(nc["mnodes"][b])))
                        vals.append(-float(nc["T"][a, b]))
                    r += 1
        self.n_c = r
        self._dir_rows = dir_rows
        self.B = sp.csr_matrix((vals, (rows, cols)), shape=(r, self.n_dof))
        self.BBt = (self.B @ self.B.T).tocsc()
        self._BBt_lu = spla.splu(self.BBt)

    def _build_dirichlet_data(self):
        """c: right-hand side of B u = c, g_D(X_i)[c] on the Dirichlet row of
        copy (k, i) and component c, zero elsewhere; u_D = B^T (B B^T)^{-1} c."""
        self.c = np.zeros(self.n_c)
        if self.dirichlet is not None and self._dir_rows:
            X = np.array([self.patches[k].ctrl.reshape(-1, self.dim)[i] for (_r, k, i, _c) in self._dir_rows])
            g = np.asarray(self.dirichlet(X), dtype=float).reshape(len(X), self.dim)
            for j, (r, _k, _i, c) in enumerate(self._dir_rows):
                self.c[r] = g[j, c]
        self.u_dir = self.B.T @ self._BBt_lu.solve(self.c)

    # ----------------------------------------------------------- coarse space
    def _build_coarse(self):
        """R (raw rigid modes, block diagonal), G = B R, C = G^T G (Section 4)."""
        blocks = [pa.rigid_modes().T for pa in self.patches]
        self.n_modes = blocks[0].shape[1]
        self.R = sp.block_diag([sp.csr_matrix(b) for b in blocks], format="csr")
        self.G = (self.B @ self.R).toarray()
        C = self.G.T @ self.G
        try:
            self.C_chol = sla.cho_factor(C)
        except np.linalg.LinAlgError as e:
            raise SingularCoarse(str(e))
        if np.min(np.linalg.eigvalsh(C)) <= 1e-12 * np.max(np.linalg.eigvalsh(C)):
            raise SingularCoarse("G^T G is singular")
        self.RtR = [sla.cho_factor(b.T @ b) for b in blocks]
        self.Rblocks = blocks

    def P_chi(self, y):
        """Orthogonal projector onto ker G^T: y - G (G^T G)^{-1} G^T y."""
        return y - self.G @ sla.cho_solve(self.C_chol, self.G.T @ y)

    def P_u(self, x):
        """Orthogonal projector onto range A: x - R (R^T R)^{-1} R^T x."""
        out = x.copy()
        for k in range(len(self.patches)):
            s = slice(self.offsets[k], self.offsets[k + 1])
            Rk = self.Rblocks[k]
            out[s] = x[s] - Rk @ sla.cho_solve(self.RtR[k], Rk.T @ x[s])
        return out

    def lambda0(self, f):
        """Minimal-norm solution of G^T lambda_0 = R^T f."""
        return self.G @ sla.cho_solve(self.C_chol, self.R.T @ f)

    # ----------------------------------------------------------- operators
    def apply_A(self, w):
        if self.assembled:
            return np.concatenate([self.A[k] @ w[self.offsets[k]:self.offsets[k + 1]]
                                   for k in range(len(self.patches))])
        return self.join([pa.stiffness_apply(wk)
                          for pa, wk in zip(self.patches, self.split(w))])

    def load(self, amps=None):
        """Assembled load: the trigonometric modes, the body-force function
        and the tractions on the faces marked 2 (Section 3)."""
        parts = []
        for pa in self.patches:
            F = pa.body_force(self.load_modes, amps)
            if self.body_force is not None:
                F = F + pa.body_force_field(self.body_force)
            for f in range(2 * self.dim):
                if pa.bc[f] == 2:
                    F = F + pa.traction(f, self.traction)
            parts.append(F)
        return self.join(parts)

    def apply_op(self, x):
        """Projected saddle operator of Section 4: [A w + B^T P_chi chi;
        P_chi B w]."""
        w, chi = x[:self.n_dof], x[self.n_dof:]
        return np.concatenate([self.apply_A(w) + self.B.T @ self.P_chi(chi),
                               self.P_chi(self.B @ w)])

    # -------------------------------------------------------------- FD data
    def _build_fd(self):
        """Generalised eigendecompositions of the univariate pencils (K, M)
        and of their interior blocks (Section 5.2.1): U^T M U = I,
        U^T K U = D."""
        self.fd = []
        from .bspline import matrices_1d
        for pa in self.patches:
            per_dir = []
            for l in range(self.dim):
                K, M = matrices_1d(pa.knots[l], pa.p)
                D, U = sla.eigh(K, M, driver=self.eig_driver)
                Di, Ui = sla.eigh(K[1:-1, 1:-1], M[1:-1, 1:-1], driver=self.eig_driver)
                per_dir.append(dict(K=K, M=M, D=D, U=U, Di=Di, Ui=Ui))
            self.fd.append(per_dir)

    def kappa(self, k, l):
        """Coefficients of the Kronecker terms of A-hat_l (Section 5.2):
        2 mu + lambda in direction l, mu in the others."""
        pa = self.patches[k]
        return [2 * pa.mu + pa.lam if m == l else pa.mu for m in range(self.dim)]

    def _outer_sum(self, vecs):
        """T[a_d..a_1] = sum_m vecs[m][a_m] (Kronecker sum of diagonals)."""
        dim = len(vecs)
        T = 0.0
        for m, v in enumerate(vecs):
            shp = [1] * dim
            shp[dim - 1 - m] = -1
            T = T + v.reshape(shp)
        return T

    def Lambda(self, k, l):
        """Eigenvalues of (H^(k))^{d-2} (A-hat_l + M-hat_l) (Section 5.2.1):
        H^{d-2} [1 + sum_m kappa_{l,m} D_m]."""
        pa = self.patches[k]
        kap = self.kappa(k, l)
        S = self._outer_sum([kap[m] * self.fd[k][m]["D"] for m in range(self.dim)])
        return pa.diameter() ** (self.dim - 2) * (1.0 + S)

    def Lambda_interior(self, k, l):
        """Eigenvalues of (A-hat_l)_II: sum_m kappa_{l,m} D-tilde_m."""
        kap = self.kappa(k, l)
        return self._outer_sum([kap[m] * self.fd[k][m]["Di"] for m in range(self.dim)])

    def fd_solve(self, k, l, r):
        """Algorithm 1 (FD): r~ = (U_d x..x U_1)^T r; q~ = Lambda_l^{-1} r~;
        s = (U_d x..x U_1) q~.  Returns (H^{d-2}(A-hat_l + M-hat_l))^{-1} r."""
        U = [self.fd[k][m]["U"] for m in range(self.dim)]
        rt = apply_1d(r, [u.T for u in U])
        return apply_1d(rt / self.Lambda(k, l), U)

    def fd_solve_interior(self, k, l, r):
        """Algorithm 1 with the interior factors: ((A-hat_l)_II)^{-1} r."""
        U = [self.fd[k][m]["Ui"] for m in range(self.dim)]
        rt = apply_1d(r, [u.T for u in U])
        return apply_1d(rt / self.Lambda_interior(k, l), U)

    def apply_PA_inv(self, r):
        """(P_A^inex)^{-1} r, block diagonal over patches and components."""
        out = []
        for k, rk in enumerate(self.split(r)):
            out.append(np.array([self.fd_solve(k, l, rk[l]) for l in range(self.dim)]))
        return self.join(out)

    def apply_Ahat(self, k, l, x):
        """A-hat_l x = sum_m kappa_{l,m} (M_d x..K_m..x M_1) x (Section 5.2;
        general-d reading of the printed d = 3 forms)."""
        kap = self.kappa(k, l)
        y = 0.0
        for m in range(self.dim):
            mats = [self.fd[k][mm]["K"] if mm == m else self.fd[k][mm]["M"]
                    for mm in range(self.dim)]
            y = y + kap[m] * apply_1d(x, mats)
        return y

    def apply_Shat(self, k, l, theta_full):
        """S-hat_l theta: Schur complement of A-hat_l on Gamma (Section 5.2),
        by discrete harmonic extension.  ``theta_full`` is a full patch tensor
        whose interior entries are ignored; the result is zero in the interior."""
        pa = self.patches[k]
        gm = pa.gamma_mask()
        inner = tuple(slice(1, -1) for _ in range(self.dim))
        v = np.where(gm, theta_full, 0.0)
        t = self.apply_Ahat(k, l, v)
        v[inner] = -self.fd_solve_interior(k, l, t[inner])
        y = self.apply_Ahat(k, l, v)
        return np.where(gm, y, 0.0)

    def apply_PS(self, y, variant="nr"):
        """P_S^{inex-nr} y = W B [sum_k H_k^{d-2} S-hat^(k)] B^T W y with
        W = (B B^T)^{-1} (Remark 1); ``variant="plain"`` drops W."""
        z = self._BBt_lu.solve(y) if variant == "nr" else y
        v = self.B.T @ z
        out = []
        for k, vk in enumerate(self.split(v)):
            h = self.patches[k].diameter() ** (self.dim - 2)
            out.append(np.array([h * self.apply_Shat(k, l, vk[l]) for l in range(self.dim)]))
        t = self.B @ self.join(out)
        return self._BBt_lu.solve(t) if variant == "nr" else t

    def apply_prec(self, r, variant="nr"):
        """Block preconditioner of Section 4: [P_u P_A^{-1} P_u r_w;
        P_chi P_S P_chi r_chi], with P~_A and P~_S of Section 5.2.3 when
        the system was built with ``geometry=True``, P_A^ex and P_S^{ex-nr}
        of Section 5.1 with ``exact=True``."""
        rw, rc = r[:self.n_dof], r[self.n_dof:]
        if self.geo is not None:
            zw = self.P_u(self.geo.apply_PA_inv(self.P_u(rw)))
            zc = self.P_chi(self.geo.apply_PS(self.P_chi(rc), variant))
        else:
            zw = self.P_u(self.apply_PA_inv(self.P_u(rw)))
            zc = self.P_chi(self.apply_PS(self.P_chi(rc), variant))
        return np.concatenate([zw, zc])

    # --------------------------------------------------------------- solve
    def solve(self, rhs=None, tol=None, maxit=2000, variant="nr", lift=True):
        """AF-IETI: MINRES on the preconditioned projected system, then the
        recovery of (u, lambda) of Section 4.  With Dirichlet data (and
        ``lift``) the system is solved for u - u_D (module docstring).
        Returns a dict."""
        f = self.load() if rhs is None else np.asarray(rhs, dtype=float)
        tol = self.tol if tol is None else tol
        if lift and np.any(self.c != 0):
            res = self.solve(rhs=f - self.apply_A(self.u_dir), tol=tol, maxit=maxit, variant=variant, lift=False)
            res["u"] = res["u"] + self.u_dir
            res["f"] = f
            return res
        lam0 = self.lambda0(f)
        b = np.concatenate([f - self.B.T @ lam0, np.zeros(self.n_c)])
        x, its, hist = minres(self.apply_op, lambda r: self.apply_prec(r, variant),
                              b, tol, maxit)
        w, chi = x[:self.n_dof], x[self.n_dof:]
        u = w - self.R @ sla.cho_solve(self.C_chol, self.G.T @ (self.B @ w))
        lam = lam0 + chi
        return dict(u=u, lam=lam, w=w, chi=chi, iters=its, history=hist,
                    f=f, lam0=lam0, b=b)


def minres(apply_A, apply_P, b, tol, maxit):
    """Preconditioned MINRES (Paige & Saunders), x0 = 0.

    Lanczos in the P^{-1} inner product with unnormalised v_j, z_j = P v_j,
    gamma_j = sqrt(<z_j, v_j>), followed by Givens rotations on the
    tridiagonal matrix.  |eta| after step j is the P-norm of the residual.
    Stops when |eta| <= tol * gamma_1.  Returns (x, iterations, history of
    |eta| / gamma_1).
    """
    n = len(b)
    x = np.zeros(n)
    v_old = np.zeros(n)
    v = b.copy()
    z = apply_P(v)
    g2 = float(z @ v)
    if g2 < 0:
        raise Breakdown("gamma_1^2 < 0")
    gamma = np.sqrt(g2)
    if gamma == 0:
        return x, 0, [0.0]
    gamma1 = gamma
    gamma_old = 1.0
    eta = gamma
    s_old = s = 0.0
    c_old = c = 1.0
    d_old = np.zeros(n)
    d = np.zeros(n)
    hist = [1.0]
    its = 0
    for j in range(1, maxit + 1):
        z = z / gamma
        q = apply_A(z)
        delta = float(q @ z)
        v_new = q - (delta / gamma) * v - (gamma / gamma_old) * v_old
        z_new = apply_P(v_new)
        g2 = float(z_new @ v_new)
        if g2 < 0:
            raise Breakdown(f"gamma^2 = {g2} < 0 at iteration {j}")
        gamma_new = np.sqrt(g2)
        a0 = c * delta - c_old * s * gamma
        a1 = np.sqrt(a0 * a0 + gamma_new * gamma_new)
        a2 = s * delta + c_old * c * gamma
        a3 = s_old * gamma
        c_new = a0 / a1
        s_new = gamma_new / a1
        d_new = (z - a3 * d_old - a2 * d) / a1
        x = x + c_new * eta * d_new
        eta = -s_new * eta
        its = j
        hist.append(abs(eta) / gamma1)
        # shift
        v_old, v = v, v_new
        z = z_new
        gamma_old, gamma = gamma, gamma_new
        c_old, c = c, c_new
        s_old, s = s, s_new
        d_old, d = d, d_new
        if abs(eta) <= tol * gamma1:
            break
    return x, its, hist
