// Host setup of the inexact AF-IETI solver (FP64, CPU).
//
// Spline data (Section 2.1), univariate pencils and their generalised
// eigendecompositions (Section 5.2.1, Algorithm 1 step 1), node matching
// across conforming interfaces (Section 2.2), the jump matrix B and the
// rigid-mode coarse space G = B R with its Cholesky factor (Section 4).
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "rigid.h"

namespace afieti {

namespace {

[[noreturn]] void fail(int code, const std::string& msg) { throw SetupError{code, msg}; }

inline int64_t node_index(const int* n, int i1, int i2, int i3) {
    return (int64_t)i1 + (int64_t)n[0] * ((int64_t)i2 + (int64_t)n[1] * i3);
}

// Dense Cholesky in place (lower, row major).  Returns false if a pivot is
// not positive or falls below rel_tol times the largest diagonal entry.
bool cholesky(int n, std::vector<double>& A, double rel_tol) {
    double dmax = 0;
    for (int i = 0; i < n; ++i) dmax = std::max(dmax, std::fabs(A[i * n + i]));
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
        if (!(s > rel_tol * dmax)) return false;
        double d = std::sqrt(s);
        A[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = t / d;
        }
        for (int i = 0; i < j; ++i) A[i * n + j] = 0.0;
    }
    return true;
}

// Inverse of an SPD matrix from its Cholesky factor L (lower, row major).
std::vector<double> chol_inverse(int n, const std::vector<double>& L) {
    std::vector<double> inv(n * n, 0.0), col(n);
    for (int e = 0; e < n; ++e) {
        // L y = e_e
        for (int i = 0; i < n; ++i) {
            double s = (i == e) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) s -= L[i * n + k] * col[k];
            col[i] = s / L[i * n + i];
        }
        // L^T x = y
        for (int i = n - 1; i >= 0; --i) {
            double s = col[i];
            for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * col[k];
            col[i] = s / L[i * n + i];
        }
        for (int i = 0; i < n; ++i) inv[i * n + e] = col[i];
    }
    // symmetrise (removes rounding asymmetry)
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double a = 0.5 * (inv[i * n + j] + inv[j * n + i]);
            inv[i * n + j] = inv[j * n + i] = a;
        }
    return inv;
}

double multilinear_coord(int dim, const double* corners, const double* eta, int x) {
    double s = 0;
    for (int c = 0; c < (1 << dim); ++c) {
        double w = 1;
        for (int l = 0; l < dim; ++l) w *= ((c >> l) & 1) ? eta[l] : 1.0 - eta[l];
        s += w * corners[3 * c + x];
    }
    return s;
}

// det of the Jacobian of the multilinear corner map at eta
double multilinear_det(int dim, const double* corners, const double* eta) {
    double J[3][3] = {{0}};
    for (int c = 0; c < (1 << dim); ++c) {
        for (int a = 0; a < dim; ++a) {
            double w = 1;
            for (int l = 0; l < dim; ++l) {
                int bit = (c >> l) & 1;
                if (l == a) w *= bit ? 1.0 : -1.0;
                else w *= bit ? eta[l] : 1.0 - eta[l];
            }
            for (int x = 0; x < dim; ++x) J[x][a] += w * corners[3 * c + x];
        }
    }
    if (dim == 2) return J[0][0] * J[1][1] - J[0][1] * J[1][0];
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

struct UnionFind {
    std::vector<int64_t> parent;
    explicit UnionFind(int64_t n) : parent(n) { std::iota(parent.begin(), parent.end(), 0); }
    int64_t find(int64_t a) {
        while (parent[a] != a) {
            parent[a] = parent[parent[a]];
            a = parent[a];
        }
        return a;
    }
    void unite(int64_t a, int64_t b) {
        a = find(a);
        b = find(b);
        if (a != b) parent[std::max(a, b)] = std::min(a, b);
    }
};

void build_dir(Dir1D& d, int n_el, int p, int reg) {
    d.p = p;
    d.n_el = n_el;
    d.knots = open_uniform_knots(n_el, p, reg);
    d.n = (int)d.knots.size() - p - 1;
    const int P = p + 1;
    std::vector<double> gx(P), gw(P);
    gauss_legendre(P, gx.data(), gw.data());
    std::vector<double> brk;
    for (double t : d.knots)
        if (brk.empty() || t > brk.back()) brk.push_back(t);
    if ((int)brk.size() - 1 != n_el) fail(AFIETI_EINVAL, "knot spans do not match n_el");
    d.nq = n_el * P;
    d.qx.resize(d.nq);
    d.qw.resize(d.nq);
    d.qfirst.resize(d.nq);
    d.qval.assign((size_t)d.nq * P, 0.0);
    d.qder.assign((size_t)d.nq * P, 0.0);
    d.el_first.assign(d.n, 1 << 30);
    d.el_last.assign(d.n, -1);
    for (int e = 0; e < n_el; ++e) {
        double a = brk[e], b = brk[e + 1];
        for (int q = 0; q < P; ++q) {
            int g = e * P + q;
            d.qx[g] = a + (b - a) * gx[q];
            d.qw[g] = (b - a) * gw[q];
            int first;
            bspline_eval(d.knots, p, d.qx[g], first, &d.qval[(size_t)g * P], &d.qder[(size_t)g * P]);
            d.qfirst[g] = first;
            for (int t = 0; t < P; ++t) {
                d.el_first[first + t] = std::min(d.el_first[first + t], e);
                d.el_last[first + t] = std::max(d.el_last[first + t], e);
            }
        }
    }
    // K[i][j] = int b_i' b_j',  M[i][j] = int b_i b_j  (exact: degree <= 2p)
    d.K.assign((size_t)d.n * d.n, 0.0);
    d.M.assign((size_t)d.n * d.n, 0.0);
    for (int g = 0; g < d.nq; ++g) {
        int f = d.qfirst[g];
        for (int s = 0; s < P; ++s)
            for (int t = 0; t < P; ++t) {
                d.K[(size_t)(f + s) * d.n + f + t] += d.qw[g] * d.qder[g * P + s] * d.qder[g * P + t];
                d.M[(size_t)(f + s) * d.n + f + t] += d.qw[g] * d.qval[g * P + s] * d.qval[g * P + t];
            }
    }
    d.U.resize((size_t)d.n * d.n);
    d.D.resize(d.n);
    if (sym_gen_eig(d.n, d.K.data(), d.M.data(), d.U.data(), d.D.data()) != 0)
        fail(AFIETI_ESINGULAR, "univariate mass matrix not positive definite");
    int ni = d.n - 2;
    std::vector<double> Ki((size_t)ni * ni), Mi((size_t)ni * ni);
    for (int i = 0; i < ni; ++i)
        for (int j = 0; j < ni; ++j) {
            Ki[(size_t)i * ni + j] = d.K[(size_t)(i + 1) * d.n + j + 1];
            Mi[(size_t)i * ni + j] = d.M[(size_t)(i + 1) * d.n + j + 1];
        }
    d.Ui.resize((size_t)ni * ni);
    d.Di.resize(ni);
    if (sym_gen_eig(ni, Ki.data(), Mi.data(), d.Ui.data(), d.Di.data()) != 0)
        fail(AFIETI_ESINGULAR, "interior univariate mass matrix not positive definite");
}

void dummy_dir(Dir1D& d) {
    d.n = 1;
    d.p = 0;
    d.U = {1.0};
    d.D = {0.0};
    d.Ui = {1.0};
    d.Di = {0.0};
    d.K = {0.0};
    d.M = {1.0};
}

bool on_face(const PatchPlan& pp, int64_t node, int face) {
    int fd = face / 2, side = face % 2;
    int64_t i1 = node % pp.n[0];
    int64_t i2 = (node / pp.n[0]) % pp.n[1];
    int64_t i3 = node / ((int64_t)pp.n[0] * pp.n[1]);
    int64_t idx[3] = {i1, i2, i3};
    return idx[fd] == (side ? pp.n[fd] - 1 : 0);
}

bool is_gamma(const PatchPlan& pp, int64_t node) {
    for (int f = 0; f < 2 * pp.dim; ++f)
        if (on_face(pp, node, f)) return true;
    return false;
}

}  // namespace

// ------------------------------------------------------------------ spline
std::vector<double> open_uniform_knots(int n_el, int p, int reg) {
    if (p < 1 || reg < 0 || reg >= p || n_el < 1) fail(AFIETI_EINVAL, "need p >= 1, 0 <= reg < p, n_el >= 1");
    std::vector<double> t(p + 1, 0.0);
    for (int e = 1; e < n_el; ++e)
        for (int r = 0; r < p - reg; ++r) t.push_back((double)e / n_el);
    for (int r = 0; r <= p; ++r) t.push_back(1.0);
    return t;
}

// Nonzero B-splines of degree p and their first derivatives at x (Section
// 2.1).  The span s with knots[s] <= x < knots[s+1] is located (x = 1 uses
// the last non-empty span); the p+1 functions s-p..s follow from the
// triangular form of the Cox-de Boor recursion, and the derivatives from
// the degree p-1 values.  first = s - p.
void bspline_eval(const std::vector<double>& t, int p, double x, int& first, double* val, double* der) {
    const int m = (int)t.size() - p - 1;
    int s = p;
    if (x >= t[m]) {
        s = m - 1;
        while (s > p && t[s] == t[s + 1]) --s;
    } else {
        int lo = p, hi = m;  // t[lo] <= x < t[hi]
        while (hi - lo > 1) {
            int mid = (lo + hi) / 2;
            if (x < t[mid]) hi = mid;
            else lo = mid;
        }
        s = lo;
    }
    first = s - p;
    std::vector<double> N(p + 1, 0.0), Nm(p + 1, 0.0), left(p + 1), right(p + 1);
    N[0] = 1.0;
    for (int j = 1; j <= p; ++j) {
        if (j == p) Nm = N;  // degree p-1 values, functions s-p+1..s
        left[j] = x - t[s + 1 - j];
        right[j] = t[s + j] - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            double den = right[r + 1] + left[j - r];
            double tmp = den != 0.0 ? N[r] / den : 0.0;
            N[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        N[j] = saved;
    }
    for (int k = 0; k <= p; ++k) val[k] = N[k];
    if (p == 0) {
        der[0] = 0.0;
        return;
    }
    for (int k = 0; k <= p; ++k) {
        int i = first + k;  // basis index
        double a = 0.0, b = 0.0;
        if (k >= 1) {  // b_{i,p-1} is Nm[k-1]
            double den = t[i + p] - t[i];
            if (den != 0.0) a = Nm[k - 1] / den;
        }
        if (k <= p - 1) {  // b_{i+1,p-1} is Nm[k]
            double den = t[i + p + 1] - t[i + 1];
            if (den != 0.0) b = Nm[k] / den;
        }
        der[k] = p * (a - b);
    }
}

// Legendre P_n(z) and P_{n-1}(z) by the three-term recurrence.
static void legendre(int n, double z, double& pn, double& pnm1) {
    pnm1 = 1.0;
    pn = z;
    for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * pn - (k - 1.0) * pnm1) / k;
        pnm1 = pn;
        pn = pk;
    }
}

// Gauss-Legendre rule with n points on [0, 1]: roots of P_n by Newton's
// method, weights 2 / ((1 - z^2) P_n'(z)^2) on [-1, 1], then mapped.
void gauss_legendre(int n, double* x, double* w) {
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double pn, pnm1, dp;
        for (int it = 0; it < 100; ++it) {
            legendre(n, z, pn, pnm1);
            dp = n * (z * pn - pnm1) / (z * z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        legendre(n, z, pn, pnm1);
        dp = n * (z * pn - pnm1) / (z * z - 1.0);
        double wi = 2.0 / ((1.0 - z * z) * dp * dp);
        x[n - 1 - i] = 0.5 * (z + 1.0);  // ascending on [0, 1]
        w[n - 1 - i] = 0.5 * wi;
    }
}

// Generalised symmetric-definite eigenproblem K u = d M u (n small):
// M = L L^T (Cholesky), C = L^{-1} K L^{-T}, cyclic Jacobi rotations
// C = V diag(d) V^T, U = L^{-T} V.  Then U^T M U = I and U^T K U = diag(d).
// Eigenvalues ascending.  Returns nonzero if M is not positive definite.
int sym_gen_eig(int n, const double* K, const double* M, double* U, double* D) {
    std::vector<double> L(M, M + (size_t)n * n);
    if (!cholesky(n, L, 1e-300)) return 1;
    // C = L^{-1} K L^{-T}: first X = L^{-1} K, then C = L^{-1} X^T
    std::vector<double> X((size_t)n * n), C((size_t)n * n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double s = K[(size_t)i * n + j];
            for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * X[(size_t)k * n + j];
            X[(size_t)i * n + j] = s / L[(size_t)i * n + i];
        }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double s = X[(size_t)j * n + i];
            for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * C[(size_t)k * n + j];
            C[(size_t)i * n + j] = s / L[(size_t)i * n + i];
        }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double a = 0.5 * (C[(size_t)i * n + j] + C[(size_t)j * n + i]);
            C[(size_t)i * n + j] = C[(size_t)j * n + i] = a;
        }
    std::vector<double> V((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0, tot = 0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double c2 = C[(size_t)i * n + j] * C[(size_t)i * n + j];
                tot += c2;
                if (i != j) off += c2;
            }
        if (off <= 1e-32 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = C[(size_t)p * n + q];
                if (apq == 0.0) continue;
                double app = C[(size_t)p * n + p], aqq = C[(size_t)q * n + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // columns p, q
                    double ckp = C[(size_t)k * n + p], ckq = C[(size_t)k * n + q];
                    C[(size_t)k * n + p] = c * ckp - s * ckq;
                    C[(size_t)k * n + q] = s * ckp + c * ckq;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q
                    double cpk = C[(size_t)p * n + k], cqk = C[(size_t)q * n + k];
                    C[(size_t)p * n + k] = c * cpk - s * cqk;
                    C[(size_t)q * n + k] = s * cpk + c * cqk;
                }
                for (int k = 0; k < n; ++k) {
                    double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return C[(size_t)a * n + a] < C[(size_t)b * n + b]; });
    // U = L^{-T} V (columns in ascending eigenvalue order)
    for (int jj = 0; jj < n; ++jj) {
        int j = ord[jj];
        D[jj] = C[(size_t)j * n + j];
        for (int i = n - 1; i >= 0; --i) {
            double s = V[(size_t)i * n + j];
            for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * U[(size_t)k * n + jj];
            U[(size_t)i * n + jj] = s / L[(size_t)i * n + i];
        }
    }
    return 0;
}

double rigid_mode(int dim, int m, int c, const double* X) { return rigid_mode_value(dim, m, c, X); }

// -------------------------------------------------------------------- plan
Plan build_plan(const afieti_problem* probs, int n_problems) {
    if (!probs || n_problems < 1) fail(AFIETI_EINVAL, "no problems");
    Plan plan;
    int64_t dof = 0, crow = 0;
    for (int pi = 0; pi < n_problems; ++pi) {
        const afieti_problem& pr = probs[pi];
        if ((pr.dim != 2 && pr.dim != 3) || pr.n_patches < 1 || !pr.patches)
            fail(AFIETI_EINVAL, "problem needs dim 2 or 3 and at least one patch");
        if (pr.n_load_modes < 0 || (pr.n_load_modes > 0 && !pr.load_modes))
            fail(AFIETI_EINVAL, "bad load modes");
        const int dim = pr.dim;
        ProblemPlan pp;
        pp.dim = dim;
        pp.patch0 = (int)plan.patches.size();
        pp.n_patches = pr.n_patches;
        pp.dof_off = dof;
        pp.n_modes = rigid_mode_count(dim);
        for (int j = 0; j < pr.n_load_modes; ++j) {
            const afieti_load_mode& lm = pr.load_modes[j];
            if (lm.comp < 0 || lm.comp >= dim || !std::isfinite(lm.amp))
                fail(AFIETI_EINVAL, "bad load mode");
            pp.load.push_back(lm);
        }
        // ---- patches: spline data, geometry, eigendecompositions
        for (int k = 0; k < pr.n_patches; ++k) {
            const afieti_patch& in = pr.patches[k];
            PatchPlan P;
            P.prob = pi;
            P.dim = dim;
            P.p = in.p;
            P.reg = in.reg;
            if (in.p < 1 || in.p > 8 || in.reg < 0 || in.reg >= in.p)
                fail(AFIETI_EINVAL, "degree must be 1..8 and 0 <= reg < p");
            if (!(in.lambda > 0) || !(in.mu > 0) || !std::isfinite(in.lambda) || !std::isfinite(in.mu))
                fail(AFIETI_EINVAL, "Lame parameters must be positive");
            P.lam = in.lambda;
            P.mu = in.mu;
            for (int c = 0; c < 24; ++c) {
                if (!std::isfinite(in.corners[c])) fail(AFIETI_EINVAL, "non-finite corner");
                P.corners[c] = in.corners[c];
            }
            if (dim == 2)
                for (int c = 0; c < 4; ++c) P.corners[3 * c + 2] = 0.0;
            for (int f = 0; f < 6; ++f) P.bc[f] = f < 2 * dim ? in.face_bc[f] : 0;
            for (int l = 0; l < 3; ++l) {
                if (l < dim) {
                    if (in.n_el[l] < 1) fail(AFIETI_EINVAL, "n_el must be >= 1");
                    build_dir(P.dir[l], in.n_el[l], in.p, in.reg);
                    if (P.dir[l].n < 3) fail(AFIETI_EINVAL, "need at least 3 basis functions per direction");
                    if (P.dir[l].n > 48) fail(AFIETI_EUNSUPPORTED, "at most 48 basis functions per direction");
                } else {
                    dummy_dir(P.dir[l]);
                }
                P.n[l] = P.dir[l].n;
            }
            P.nodes = (int64_t)P.n[0] * P.n[1] * P.n[2];
            P.dof_off = dof;
            dof += dim * P.nodes;
            // diameter: largest corner distance
            double H = 0;
            for (int a = 0; a < (1 << dim); ++a)
                for (int b = 0; b < (1 << dim); ++b) {
                    double s = 0;
                    for (int x = 0; x < dim; ++x) {
                        double dd = P.corners[3 * a + x] - P.corners[3 * b + x];
                        s += dd * dd;
                    }
                    H = std::max(H, std::sqrt(s));
                }
            P.H = H;
            P.hscale = dim == 3 ? H : 1.0;
            // det J > 0 at every Gauss point of the multilinear map
            for (int64_t q3 = 0; q3 < (dim == 3 ? P.dir[2].nq : 1); ++q3)
                for (int q2 = 0; q2 < P.dir[1].nq; ++q2)
                    for (int q1 = 0; q1 < P.dir[0].nq; ++q1) {
                        double eta[3] = {P.dir[0].qx[q1], P.dir[1].qx[q2], dim == 3 ? P.dir[2].qx[q3] : 0.0};
                        if (!(multilinear_det(dim, P.corners, eta) > 0))
                            fail(AFIETI_EGEOM, "patch map is not orientation preserving");
                    }
            // control points at the Greville abscissae
            std::vector<double> g[3];
            for (int l = 0; l < 3; ++l) {
                g[l].assign(P.n[l], 0.0);
                if (l < dim)
                    for (int i = 0; i < P.n[l]; ++i) {
                        double s = 0;
                        for (int r = 1; r <= P.p; ++r) s += P.dir[l].knots[i + r];
                        g[l][i] = s / P.p;
                    }
            }
            P.ctrl.assign((size_t)P.nodes * 3, 0.0);
            for (int i3 = 0; i3 < P.n[2]; ++i3)
                for (int i2 = 0; i2 < P.n[1]; ++i2)
                    for (int i1 = 0; i1 < P.n[0]; ++i1) {
                        double eta[3] = {g[0][i1], g[1][i2], g[2][i3]};
                        int64_t nd = node_index(P.n, i1, i2, i3);
                        for (int x = 0; x < dim; ++x) P.ctrl[nd * 3 + x] = multilinear_coord(dim, P.corners, eta, x);
                    }
            plan.patches.push_back(std::move(P));
        }
        pp.n_dof = dof - pp.dof_off;

        // ---- node matching across faces (union-find over patch nodes)
        std::vector<int64_t> node_off(pr.n_patches + 1, 0);
        for (int k = 0; k < pr.n_patches; ++k) node_off[k + 1] = node_off[k] + plan.patches[pp.patch0 + k].nodes;
        UnionFind uf(node_off.back());
        double scale = 0;
        for (int k = 0; k < pr.n_patches; ++k) scale = std::max(scale, plan.patches[pp.patch0 + k].H);
        const double tol = 1e-10 * std::max(scale, 1e-300);
        const int nfc = 1 << (dim - 1);  // corners per face
        auto face_corner = [&](const PatchPlan& P, int face, int s, double* X) {
            int fd = face / 2, side = face % 2;
            int bits = 0, t = 0;
            for (int l = 0; l < dim; ++l) {
                int bit;
                if (l == fd) bit = side;
                else bit = (s >> (t++)) & 1;
                bits |= bit << l;
            }
            for (int x = 0; x < 3; ++x) X[x] = P.corners[3 * bits + x];
        };
        for (int ka = 0; ka < pr.n_patches; ++ka)
            for (int kb = ka + 1; kb < pr.n_patches; ++kb) {
                const PatchPlan& A = plan.patches[pp.patch0 + ka];
                const PatchPlan& B = plan.patches[pp.patch0 + kb];
                for (int fa = 0; fa < 2 * dim; ++fa)
                    for (int fb = 0; fb < 2 * dim; ++fb) {
                        int map[4];
                        bool ok = true;
                        for (int s = 0; s < nfc && ok; ++s) {
                            double Xa[3], Xb[3];
                            face_corner(A, fa, s, Xa);
                            map[s] = -1;
                            for (int t = 0; t < nfc; ++t) {
                                face_corner(B, fb, t, Xb);
                                double d2 = 0;
                                for (int x = 0; x < 3; ++x) d2 += (Xa[x] - Xb[x]) * (Xa[x] - Xb[x]);
                                if (std::sqrt(d2) <= tol) map[s] = t;
                            }
                            if (map[s] < 0) ok = false;
                        }
                        if (!ok) continue;
                        // tangential directions of each face, ascending
                        int ta[2], tb[2], na = 0, nb = 0;
                        for (int l = 0; l < dim; ++l) {
                            if (l != fa / 2) ta[na++] = l;
                            if (l != fb / 2) tb[nb++] = l;
                        }
                        // where does tangential direction j of A go in B, flipped?
                        int to[2], flip[2];
                        for (int j = 0; j < dim - 1; ++j) {
                            int u0 = map[0], u1 = map[1 << j];
                            int diff = u0 ^ u1;
                            if (diff != 1 && diff != 2) fail(AFIETI_EGEOM, "degenerate face correspondence");
                            int jb = diff == 1 ? 0 : 1;
                            to[j] = tb[jb];
                            flip[j] = (u0 >> jb) & 1;
                            if (A.n[ta[j]] != B.n[to[j]] || A.p != B.p || A.reg != B.reg ||
                                A.dir[ta[j]].n_el != B.dir[to[j]].n_el)
                                fail(AFIETI_EGEOM, "non-conforming interface");
                        }
                        // unite the face nodes
                        int na1 = A.n[ta[0]], na2 = dim == 3 ? A.n[ta[1]] : 1;
                        for (int s2 = 0; s2 < na2; ++s2)
                            for (int s1 = 0; s1 < na1; ++s1) {
                                int ia[3] = {0, 0, 0}, ib[3] = {0, 0, 0};
                                ia[fa / 2] = (fa % 2) ? A.n[fa / 2] - 1 : 0;
                                ia[ta[0]] = s1;
                                if (dim == 3) ia[ta[1]] = s2;
                                ib[fb / 2] = (fb % 2) ? B.n[fb / 2] - 1 : 0;
                                ib[to[0]] = flip[0] ? B.n[to[0]] - 1 - s1 : s1;
                                if (dim == 3) ib[to[1]] = flip[1] ? B.n[to[1]] - 1 - s2 : s2;
                                uf.unite(node_off[ka] + node_index(A.n, ia[0], ia[1], ia[2]),
                                         node_off[kb] + node_index(B.n, ib[0], ib[1], ib[2]));
                            }
                    }
            }
        // ---- classes in (lowest patch, local index) order
        struct Copy { int k; int64_t node; };
        std::vector<std::vector<Copy>> classes;
        std::vector<int64_t> class_of(node_off.back(), -1);
        for (int k = 0; k < pr.n_patches; ++k) {
            const PatchPlan& P = plan.patches[pp.patch0 + k];
            for (int64_t nd = 0; nd < P.nodes; ++nd) {
                if (!is_gamma(P, nd)) continue;
                int64_t root = uf.find(node_off[k] + nd);
                if (class_of[root] < 0) {
                    class_of[root] = (int64_t)classes.size();
                    classes.emplace_back();
                }
                classes[class_of[root]].push_back({k, nd});
            }
        }
        std::vector<char> dirichlet(classes.size(), 0);
        for (size_t ci = 0; ci < classes.size(); ++ci) {
            auto& cp = classes[ci];
            std::sort(cp.begin(), cp.end(), [](const Copy& a, const Copy& b) { return a.k < b.k; });
            for (size_t j = 1; j < cp.size(); ++j)
                if (cp[j].k == cp[j - 1].k) fail(AFIETI_EGEOM, "a patch touches itself");
            for (auto& c : cp) {
                const PatchPlan& P = plan.patches[pp.patch0 + c.k];
                for (int f = 0; f < 2 * dim; ++f)
                    if (P.bc[f] == AFIETI_FACE_DIRICHLET && on_face(P, c.node, f)) dirichlet[ci] = 1;
            }
        }
        // ---- rows of B
        pp.c_off = crow;
        auto gdof = [&](const Copy& c, int comp) {
            const PatchPlan& P = plan.patches[pp.patch0 + c.k];
            return P.dof_off + comp * P.nodes + c.node;
        };
        for (int comp = 0; comp < dim; ++comp)
            for (size_t ci = 0; ci < classes.size(); ++ci) {
                const auto& cp = classes[ci];
                int r = (int)cp.size();
                if (dirichlet[ci]) {
                    int start = (int)plan.c_plus.size();
                    for (int j = 0; j < r; ++j) {
                        plan.c_plus.push_back(gdof(cp[j], comp));
                        plan.c_minus.push_back(-1);
                        plan.c_patch_plus.push_back(pp.patch0 + cp[j].k);
                        plan.c_patch_minus.push_back(-1);
                        plan.c_blk_start.push_back(start);
                        plan.c_blk_size.push_back(r);
                        plan.c_blk_dir.push_back(1);
                    }
                } else if (r >= 2) {
                    int start = (int)plan.c_plus.size();
                    for (int j = 1; j < r; ++j) {
                        plan.c_plus.push_back(gdof(cp[0], comp));
                        plan.c_minus.push_back(gdof(cp[j], comp));
                        plan.c_patch_plus.push_back(pp.patch0 + cp[0].k);
                        plan.c_patch_minus.push_back(pp.patch0 + cp[j].k);
                        plan.c_blk_start.push_back(start);
                        plan.c_blk_size.push_back(r - 1);
                        plan.c_blk_dir.push_back(0);
                    }
                }
            }
        crow = (int64_t)plan.c_plus.size();
        pp.n_c = crow - pp.c_off;
        if (pp.n_c == 0) fail(AFIETI_ESINGULAR, "no constraints: the problem has no Dirichlet boundary");
        plan.probs.push_back(std::move(pp));
    }
    plan.n_dof = dof;
    plan.n_c = crow;
    if (plan.n_dof > (int64_t)INT32_MAX || plan.n_c > (int64_t)INT32_MAX)
        fail(AFIETI_EUNSUPPORTED, "more than 2^31 unknowns");

    // ---- B^T by DOF (CSR), rows ascending within a DOF
    std::vector<int64_t> cnt(plan.n_dof + 1, 0);
    for (int64_t r = 0; r < plan.n_c; ++r) {
        cnt[plan.c_plus[r] + 1]++;
        if (plan.c_minus[r] >= 0) cnt[plan.c_minus[r] + 1]++;
    }
    for (int64_t i = 0; i < plan.n_dof; ++i) cnt[i + 1] += cnt[i];
    plan.bt_ptr = cnt;
    plan.bt_row.assign(cnt.back(), 0);
    plan.bt_sign.assign(cnt.back(), 0.0);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t r = 0; r < plan.n_c; ++r) {  // ascending r: rows sorted per DOF
        int64_t a = fill[plan.c_plus[r]]++;
        plan.bt_row[a] = (int)r;
        plan.bt_sign[a] = 1.0;
        if (plan.c_minus[r] >= 0) {
            int64_t b = fill[plan.c_minus[r]]++;
            plan.bt_row[b] = (int)r;
            plan.bt_sign[b] = -1.0;
        }
    }
    // ---- rigid modes: G rows, R^T R per patch, G^T G per problem
    plan.g_plus.assign(plan.n_c * 6, 0.0);
    plan.g_minus.assign(plan.n_c * 6, 0.0);
    auto dof_mode = [&](int64_t gd, int k, int m) {
        const PatchPlan& P = plan.patches[k];
        int64_t loc = gd - P.dof_off;
        int comp = (int)(loc / P.nodes);
        int64_t nd = loc % P.nodes;
        return rigid_mode_value(P.dim, m, comp, &P.ctrl[nd * 3]);
    };
    for (int64_t r = 0; r < plan.n_c; ++r) {
        int kp = plan.c_patch_plus[r];
        int nm = rigid_mode_count(plan.patches[kp].dim);
        for (int m = 0; m < nm; ++m) {
            plan.g_plus[r * 6 + m] = dof_mode(plan.c_plus[r], kp, m);
            if (plan.c_minus[r] >= 0) plan.g_minus[r * 6 + m] = dof_mode(plan.c_minus[r], plan.c_patch_minus[r], m);
        }
    }
    plan.RtR_inv.assign(plan.patches.size() * 36, 0.0);
    for (size_t k = 0; k < plan.patches.size(); ++k) {
        const PatchPlan& P = plan.patches[k];
        int nm = rigid_mode_count(P.dim);
        std::vector<double> A(nm * nm, 0.0);
        for (int comp = 0; comp < P.dim; ++comp)
            for (int64_t nd = 0; nd < P.nodes; ++nd) {
                double v[6];
                for (int m = 0; m < nm; ++m) v[m] = rigid_mode_value(P.dim, m, comp, &P.ctrl[nd * 3]);
                for (int a = 0; a < nm; ++a)
                    for (int b = 0; b < nm; ++b) A[a * nm + b] += v[a] * v[b];
            }
        if (!cholesky(nm, A, 1e-14)) fail(AFIETI_EGEOM, "rigid modes are linearly dependent");
        std::vector<double> inv = chol_inverse(nm, A);
        for (int a = 0; a < nm; ++a)
            for (int b = 0; b < nm; ++b) plan.RtR_inv[k * 36 + a * 6 + b] = inv[a * nm + b];
    }
    for (auto& pp : plan.probs) {
        int nm = pp.n_modes;
        int nc = nm * pp.n_patches;
        std::vector<double> C((size_t)nc * nc, 0.0);
        for (int64_t r = pp.c_off; r < pp.c_off + pp.n_c; ++r) {
            int ia = (plan.c_patch_plus[r] - pp.patch0) * nm;
            int ib = plan.c_minus[r] >= 0 ? (plan.c_patch_minus[r] - pp.patch0) * nm : -1;
            const double* gp = &plan.g_plus[r * 6];
            const double* gm = &plan.g_minus[r * 6];
            for (int a = 0; a < nm; ++a)
                for (int b = 0; b < nm; ++b) {
                    C[(size_t)(ia + a) * nc + ia + b] += gp[a] * gp[b];
                    if (ib >= 0) {
                        C[(size_t)(ib + a) * nc + ib + b] += gm[a] * gm[b];
                        C[(size_t)(ia + a) * nc + ib + b] -= gp[a] * gm[b];
                        C[(size_t)(ib + a) * nc + ia + b] -= gm[a] * gp[b];
                    }
                }
        }
        pp.CtC = C;
        if (!cholesky(nc, C, 1e-12)) fail(AFIETI_ESINGULAR, "G^T G is singular: not enough Dirichlet constraints");
        pp.Cinv = chol_inverse(nc, C);
    }
    return plan;
}

}  // namespace afieti
