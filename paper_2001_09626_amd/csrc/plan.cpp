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
#include <map>
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

// Jacobian J[x][a] = dF_x / deta_a of the multilinear corner map at eta
void multilinear_jac(int dim, const double* corners, const double* eta, double (&J)[3][3]) {
    for (auto& row : J)
        for (double& v : row) v = 0.0;
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
}

double det_of(int dim, const double (&J)[3][3]) {
    if (dim == 2) return J[0][0] * J[1][1] - J[0][1] * J[1][0];
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// det of the Jacobian of the multilinear corner map at eta
double multilinear_det(int dim, const double* corners, const double* eta) {
    double J[3][3];
    multilinear_jac(dim, corners, eta, J);
    return det_of(dim, J);
}

// A non-conforming interface: face `sface` of patch `slave` refines face
// `mface` of patch `master` (parametric directions aligned); T[j] (ns[j] x
// nm[j], row major) takes the coarse B-splines along tangential direction
// tang[j] to the fine ones.
struct NcIface {
    int slave = 0, sface = 0, master = 0, mface = 0;
    int tang[2] = {0, -1};
    int ns[2] = {1, 1}, nm[2] = {1, 1};
    std::vector<double> T[2];
    // node of the slave (fine) or master face at face position (i1, i2)
    int64_t face_node(const PatchPlan& P, int i1, int i2, bool is_slave = false) const {
        const int f = is_slave ? sface : mface;
        int idx[3] = {0, 0, 0};
        idx[f / 2] = (f % 2) ? P.n[f / 2] - 1 : 0;
        idx[tang[0]] = i1;
        if (tang[1] >= 0) idx[tang[1]] = i2;
        return idx[0] + (int64_t)P.n[0] * (idx[1] + (int64_t)P.n[1] * idx[2]);
    }
};

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

// univariate spline data of one direction from its open knot vector
void build_dir(Dir1D& d, const std::vector<double>& knots, int p) {
    d.p = p;
    d.knots = knots;
    d.n = (int)d.knots.size() - p - 1;
    const int P = p + 1;
    std::vector<double> gx(P), gw(P);
    gauss_legendre(P, gx.data(), gw.data());
    std::vector<double> brk;
    for (double t : d.knots)
        if (brk.empty() || t > brk.back()) brk.push_back(t);
    const int n_el = (int)brk.size() - 1;
    d.n_el = n_el;
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

// The Gauss rule and nonzero basis values of one direction as the load
// integrals read them; a direction the patch does not have (2D) is one
// point of weight 1 where its single function is 1.
struct QuadDir {
    int nq, P;
    const double *qx, *qw, *qval;
    const int* qfirst;
    double one_x = 0.0, one_w = 1.0, one_v = 1.0;
    int one_f = 0;
    explicit QuadDir(const Dir1D& d) {
        if (d.nq > 0) {
            nq = d.nq;
            P = d.p + 1;
            qx = d.qx.data();
            qw = d.qw.data();
            qval = d.qval.data();
            qfirst = d.qfirst.data();
        } else {
            nq = 1;
            P = 1;
            qx = &one_x;
            qw = &one_w;
            qval = &one_v;
            qfirst = &one_f;
        }
    }
};

// load of the body-force callback on one patch (Section 3: int f . v dx by
// the Gauss rule of the stiffness): f at every Gauss point, weighted by
// w |det J|, contracted with the basis direction by direction; added to
// F[c * nodes + node]
void add_body_force(const PatchPlan& P, afieti_field_fn fn, void* ctx, double* F) {
    const int dim = P.dim;
    QuadDir Q0(P.dir[0]), Q1(P.dir[1]), Q2(P.dir[2]);
    const int64_t nq = (int64_t)Q0.nq * Q1.nq * Q2.nq;
    std::vector<double> x((size_t)nq * dim), f((size_t)nq * dim, 0.0), W(nq);
    for (int q3 = 0; q3 < Q2.nq; ++q3)
        for (int q2 = 0; q2 < Q1.nq; ++q2)
            for (int q1 = 0; q1 < Q0.nq; ++q1) {
                const int64_t q = q1 + (int64_t)Q0.nq * (q2 + (int64_t)Q1.nq * q3);
                const double eta[3] = {Q0.qx[q1], Q1.qx[q2], Q2.qx[q3]};
                double X[3], J[3][3];
                patch_map(P, eta, X, J);
                for (int c = 0; c < dim; ++c) x[q * dim + c] = X[c];
                W[q] = Q0.qw[q1] * Q1.qw[q2] * Q2.qw[q3] * std::fabs(det_of(dim, J));
            }
    fn(nq, x.data(), f.data(), ctx);
    for (double v : f)
        if (!std::isfinite(v)) fail(AFIETI_EINVAL, "non-finite body force");
    // contract direction 1, then 2, then 3
    const int n1 = P.n[0], n2 = P.n[1], n3 = P.n[2];
    std::vector<double> A1((size_t)dim * Q2.nq * Q1.nq * n1, 0.0), A2((size_t)dim * Q2.nq * n2 * n1, 0.0);
    for (int c = 0; c < dim; ++c)
        for (int q3 = 0; q3 < Q2.nq; ++q3)
            for (int q2 = 0; q2 < Q1.nq; ++q2) {
                double* a = &A1[(((size_t)c * Q2.nq + q3) * Q1.nq + q2) * n1];
                for (int q1 = 0; q1 < Q0.nq; ++q1) {
                    const int64_t q = q1 + (int64_t)Q0.nq * (q2 + (int64_t)Q1.nq * q3);
                    const double v = W[q] * f[q * dim + c];
                    for (int t = 0; t < Q0.P; ++t) a[Q0.qfirst[q1] + t] += Q0.qval[(size_t)q1 * Q0.P + t] * v;
                }
            }
    for (int c = 0; c < dim; ++c)
        for (int q3 = 0; q3 < Q2.nq; ++q3)
            for (int q2 = 0; q2 < Q1.nq; ++q2) {
                const double* a = &A1[(((size_t)c * Q2.nq + q3) * Q1.nq + q2) * n1];
                for (int t = 0; t < Q1.P; ++t) {
                    const double b = Q1.qval[(size_t)q2 * Q1.P + t];
                    double* o = &A2[(((size_t)c * Q2.nq + q3) * n2 + Q1.qfirst[q2] + t) * n1];
                    for (int i1 = 0; i1 < n1; ++i1) o[i1] += b * a[i1];
                }
            }
    for (int c = 0; c < dim; ++c)
        for (int q3 = 0; q3 < Q2.nq; ++q3)
            for (int t = 0; t < Q2.P; ++t) {
                const double b = Q2.qval[(size_t)q3 * Q2.P + t];
                const int i3 = Q2.qfirst[q3] + t;
                for (int i2 = 0; i2 < n2; ++i2) {
                    const double* a = &A2[(((size_t)c * Q2.nq + q3) * n2 + i2) * n1];
                    double* o = &F[(size_t)c * P.nodes + ((size_t)i3 * n2 + i2) * n1];
                    for (int i1 = 0; i1 < n1; ++i1) o[i1] += b * a[i1];
                }
            }
}

// load of the traction callback on face `face` of a patch (Section 3: the
// boundary term int_{Gamma_N} g . v ds) by the Gauss rule of the face's
// directions; the face basis functions are the products of the tangential
// ones (the normal direction's end function is 1 on the face)
void add_traction(const PatchPlan& P, int face, afieti_traction_fn fn, void* ctx, double* F) {
    const int dim = P.dim, fd = face / 2, side = face % 2;
    int tan[2] = {0, 0}, nt = 0;
    for (int l = 0; l < dim; ++l)
        if (l != fd) tan[nt++] = l;
    QuadDir Qa(P.dir[tan[0]]), Qb(dim == 3 ? P.dir[tan[1]] : P.dir[2]);
    const int64_t nq = (int64_t)Qa.nq * Qb.nq;
    std::vector<double> x((size_t)nq * dim), nrm((size_t)nq * dim), g((size_t)nq * dim, 0.0), wa(nq);
    for (int qb = 0; qb < Qb.nq; ++qb)
        for (int qa = 0; qa < Qa.nq; ++qa) {
            const int64_t q = qa + (int64_t)Qa.nq * qb;
            double eta[3] = {0, 0, 0};
            eta[fd] = side ? 1.0 : 0.0;
            eta[tan[0]] = Qa.qx[qa];
            if (dim == 3) eta[tan[1]] = Qb.qx[qb];
            double J[3][3], X[3];
            patch_map(P, eta, X, J);
            double n[3] = {0, 0, 0};
            if (dim == 3) {
                const int a = tan[0], b = tan[1];
                n[0] = J[1][a] * J[2][b] - J[2][a] * J[1][b];
                n[1] = J[2][a] * J[0][b] - J[0][a] * J[2][b];
                n[2] = J[0][a] * J[1][b] - J[1][a] * J[0][b];
            } else {
                n[0] = J[1][tan[0]];
                n[1] = -J[0][tan[0]];
            }
            double area = 0;
            for (int c = 0; c < dim; ++c) area += n[c] * n[c];
            area = std::sqrt(area);
            // outward: along the gradient of eta_fd on the max side, against
            // it on the min side (the gradient is row fd of J^{-1}, i.e. the
            // cofactors of column fd of J up to the sign of det J)
            double grad[3] = {0, 0, 0};
            if (dim == 3) {
                const int a = (fd + 1) % 3, b = (fd + 2) % 3;
                grad[0] = J[1][a] * J[2][b] - J[2][a] * J[1][b];
                grad[1] = J[2][a] * J[0][b] - J[0][a] * J[2][b];
                grad[2] = J[0][a] * J[1][b] - J[1][a] * J[0][b];
            } else {
                const int a = 1 - fd;
                grad[0] = (fd == 0 ? 1.0 : -1.0) * J[1][a];
                grad[1] = (fd == 0 ? -1.0 : 1.0) * J[0][a];
            }
            const double det = det_of(dim, J);
            double dot = 0;
            for (int c = 0; c < dim; ++c) dot += grad[c] * n[c];
            const double sgn = ((dot * det) >= 0 ? 1.0 : -1.0) * (side ? 1.0 : -1.0);
            for (int c = 0; c < dim; ++c) {
                x[q * dim + c] = X[c];
                nrm[q * dim + c] = sgn * n[c] / area;
            }
            wa[q] = Qa.qw[qa] * Qb.qw[qb] * area;
        }
    fn(nq, x.data(), nrm.data(), g.data(), ctx);
    for (double v : g)
        if (!std::isfinite(v)) fail(AFIETI_EINVAL, "non-finite traction");
    for (int qb = 0; qb < Qb.nq; ++qb)
        for (int qa = 0; qa < Qa.nq; ++qa) {
            const int64_t q = qa + (int64_t)Qa.nq * qb;
            for (int tb = 0; tb < Qb.P; ++tb)
                for (int ta = 0; ta < Qa.P; ++ta) {
                    int idx[3] = {0, 0, 0};
                    idx[fd] = side ? P.n[fd] - 1 : 0;
                    idx[tan[0]] = Qa.qfirst[qa] + ta;
                    if (dim == 3) idx[tan[1]] = Qb.qfirst[qb] + tb;
                    const double b = Qa.qval[(size_t)qa * Qa.P + ta] * Qb.qval[(size_t)qb * Qb.P + tb] * wa[q];
                    const int64_t node = node_index(P.n, idx[0], idx[1], idx[2]);
                    for (int c = 0; c < dim; ++c) F[(size_t)c * P.nodes + node] += b * g[q * dim + c];
                }
        }
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
// Knot insertion (Boehm): the coefficients of the coarse B-splines in the
// basis of a refined knot vector, T[i * n_c + j] with b^c_j = sum_i T_ij
// b^f_i; the knots of `fine` missing from `coarse` are inserted one at a
// time, each insertion mixing p consecutive coefficients with the weights
// (t - u_i) / (u_{i+p} - u_i).  Empty if `fine` does not contain `coarse`.
std::vector<double> knot_insertion_matrix(const std::vector<double>& coarse, const std::vector<double>& fine, int p) {
    std::vector<double> ins;
    size_t a = 0;
    for (double t : fine) {
        if (a < coarse.size() && std::fabs(coarse[a] - t) <= 1e-12) ++a;
        else ins.push_back(t);
    }
    if (a != coarse.size()) return {};
    std::vector<double> U = coarse;
    const int nc = (int)coarse.size() - p - 1;
    int n = nc;
    std::vector<double> P((size_t)n * nc, 0.0);  // rows: current basis, columns: coarse functions
    for (int j = 0; j < nc; ++j) P[(size_t)j * nc + j] = 1.0;
    for (double t : ins) {
        int k = p;
        while (k + 1 < (int)U.size() - p - 1 && U[k + 1] <= t) ++k;
        std::vector<double> Q((size_t)(n + 1) * nc, 0.0);
        for (int i = 0; i <= n; ++i) {
            double* q = &Q[(size_t)i * nc];
            if (i <= k - p) {
                for (int j = 0; j < nc; ++j) q[j] = P[(size_t)i * nc + j];
            } else if (i <= k) {
                const double al = (t - U[i]) / (U[i + p] - U[i]);
                for (int j = 0; j < nc; ++j) q[j] = al * P[(size_t)i * nc + j] + (1.0 - al) * P[(size_t)(i - 1) * nc + j];
            } else {
                for (int j = 0; j < nc; ++j) q[j] = P[(size_t)(i - 1) * nc + j];
            }
        }
        U.insert(U.begin() + k + 1, t);
        P.swap(Q);
        ++n;
    }
    return P;
}

int check_open_knots(const std::vector<double>& t, int p) {
    const int m = (int)t.size();
    if (m < 2 * (p + 1)) fail(AFIETI_EINVAL, "knot vector too short for its degree");
    for (int i = 0; i <= p; ++i)
        if (t[i] != 0.0 || t[m - 1 - i] != 1.0) fail(AFIETI_EINVAL, "knot vector must be open on [0, 1]");
    int mult = 0, worst = 0;
    for (int i = p + 1; i < m - p - 1; ++i) {
        if (!std::isfinite(t[i]) || t[i] < t[i - 1] || !(t[i] > 0.0) || !(t[i] < 1.0))
            fail(AFIETI_EINVAL, "interior knots must be non-decreasing inside (0, 1)");
        mult = (i > p + 1 && t[i] == t[i - 1]) ? mult + 1 : 1;
        worst = std::max(worst, mult);
    }
    if (worst > p) fail(AFIETI_EINVAL, "interior knot multiplicity above the degree (discontinuous splines)");
    return p - std::max(worst, 1);
}

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
// A pair (p, q) is rotated while |c_pq| exceeds a few units of round-off of
// sqrt(|c_pp c_qq|), not of the whole matrix, and the sweeps go on until
// one rotates nothing: the eigenvectors of the small eigenvalues (which
// dominate the fast-diagonalization inverse) are then limited by the
// rounding of C itself, not by an off-diagonal remainder of the size of
// round-off times the largest eigenvalue.
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
    constexpr double kRel = 1e-17;
    for (int sweep = 0; sweep < 100; ++sweep) {
        int rotated = 0;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = C[(size_t)p * n + q];
                double app = C[(size_t)p * n + p], aqq = C[(size_t)q * n + q];
                if (std::fabs(apq) <= kRel * std::sqrt(std::fabs(app * aqq))) continue;
                ++rotated;
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
                // the rotated pair, exactly: zero coupling, diagonal moved by t c_pq
                C[(size_t)p * n + q] = C[(size_t)q * n + p] = 0.0;
                C[(size_t)p * n + p] = app - t * apq;
                C[(size_t)q * n + q] = aqq + t * apq;
                for (int k = 0; k < n; ++k) {
                    double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
        if (!rotated) break;
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

void multilinear_jacobian(int dim, const double* corners, const double* eta, double (&J)[3][3]) {
    multilinear_jac(dim, corners, eta, J);
}

void patch_map(const PatchPlan& P, const double* eta, double* x, double (&J)[3][3]) {
    const int dim = P.dim;
    if (!P.general) {
        multilinear_jac(dim, P.corners, eta, J);
        if (x)
            for (int c = 0; c < 3; ++c) x[c] = c < dim ? multilinear_coord(dim, P.corners, eta, c) : 0.0;
        return;
    }
    // spline map: x = sum_i X_i B_i(eta), dx/deta_a with the derivative in a
    double val[3][9] = {}, der[3][9] = {};
    int first[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
    for (int l = 0; l < 3; ++l) {
        if (l < dim) {
            bspline_eval(P.dir[l].knots, P.p, eta[l], first[l], val[l], der[l]);
            cnt[l] = P.p + 1;
        } else {
            val[l][0] = 1.0;
        }
    }
    for (auto& r : J)
        for (double& v : r) v = 0.0;
    double xx[3] = {0, 0, 0};
    for (int t3 = 0; t3 < cnt[2]; ++t3)
        for (int t2 = 0; t2 < cnt[1]; ++t2)
            for (int t1 = 0; t1 < cnt[0]; ++t1) {
                const int64_t nd = node_index(P.n, first[0] + t1, first[1] + t2, first[2] + t3);
                const double* X = &P.ctrl[nd * 3];
                const double b = val[0][t1] * val[1][t2] * val[2][t3];
                const double g[3] = {der[0][t1] * val[1][t2] * val[2][t3], val[0][t1] * der[1][t2] * val[2][t3],
                                     val[0][t1] * val[1][t2] * der[2][t3]};
                for (int c = 0; c < dim; ++c) {
                    xx[c] += b * X[c];
                    for (int a = 0; a < dim; ++a) J[c][a] += g[a] * X[c];
                }
            }
    if (x)
        for (int c = 0; c < 3; ++c) x[c] = xx[c];
}

// Rows of B for the non-conforming interfaces of a problem and component
// (Section 2.2): for every node i of the finer face, e_{f,i} - sum_j T_ij
// e_{c,j} (the coarse trace in the fine basis), and the dense blocks of
// B B^T they form with the Dirichlet rows of the coarse nodes they touch
// (inverted here).  Rows of this component start at comp_start.
void add_gluing_rows(Plan& plan, const ProblemPlan& pp, const std::vector<NcIface>& ncs, int comp, int64_t comp_start) {
    std::map<int64_t, int64_t> dir_row;  // DOF -> its Dirichlet row (this component)
    for (int64_t r = comp_start; r < (int64_t)plan.c_plus.size(); ++r) {
        if (plan.c_minus[r] == -1) dir_row[plan.c_plus[r]] = r;
    }
    std::map<int64_t, char> in_star;
    for (int64_t r = comp_start; r < (int64_t)plan.c_plus.size(); ++r)
        if (plan.c_minus[r] >= 0) in_star[plan.c_plus[r]] = in_star[plan.c_minus[r]] = 1;
    for (const NcIface& nc : ncs) {
        const PatchPlan& Ps = plan.patches[pp.patch0 + nc.slave];
        const PatchPlan& Pm = plan.patches[pp.patch0 + nc.master];
        std::vector<int64_t> rows;
        std::map<int64_t, int64_t> touched;  // Dirichlet rows coupled to the gluing rows
        for (int s2 = 0; s2 < nc.ns[1]; ++s2)
            for (int s1 = 0; s1 < nc.ns[0]; ++s1) {
                const int64_t r = (int64_t)plan.c_plus.size();
                rows.push_back(r);
                plan.c_plus.push_back(Ps.dof_off + comp * Ps.nodes + nc.face_node(Ps, s1, s2, true));
                plan.c_minus.push_back(-2 - (int64_t)(plan.glue_ptr.size() - 1));
                for (int t2 = 0; t2 < nc.nm[1]; ++t2)
                    for (int t1 = 0; t1 < nc.nm[0]; ++t1) {
                        const double w = nc.T[0][(size_t)s1 * nc.nm[0] + t1] * nc.T[1][(size_t)s2 * nc.nm[1] + t2];
                        if (w == 0.0) continue;
                        const int64_t d = Pm.dof_off + comp * Pm.nodes + nc.face_node(Pm, t1, t2);
                        if (in_star.count(d))
                            throw SetupError{AFIETI_EUNSUPPORTED,
                                             "a coarse node of a non-conforming interface shared with a third patch"};
                        auto it = dir_row.find(d);
                        if (it != dir_row.end()) touched[it->second] = 1;
                        plan.glue_col.push_back(d);
                        plan.glue_val.push_back(w);
                    }
                plan.glue_ptr.push_back((int64_t)plan.glue_col.size());
                plan.c_patch_plus.push_back(pp.patch0 + nc.slave);
                plan.c_patch_minus.push_back(pp.patch0 + nc.master);
                plan.c_blk_start.push_back(0);
                plan.c_blk_size.push_back(0);
                plan.c_blk_dir.push_back(2);
            }
        for (const auto& kv : touched) {
            if (plan.c_blk_dir[kv.first] == 2)
                throw SetupError{AFIETI_EUNSUPPORTED, "a Dirichlet node coupled to two non-conforming interfaces"};
            rows.push_back(kv.first);
        }
        // B B^T on the block: rows as sparse vectors over DOFs
        const int n = (int)rows.size();
        std::map<int64_t, std::vector<std::pair<int, double>>> by_dof;
        for (int a = 0; a < n; ++a) {
            const int64_t r = rows[a];
            by_dof[plan.c_plus[r]].push_back({a, 1.0});
            if (plan.c_minus[r] <= -2) {
                const int64_t g = -2 - plan.c_minus[r];
                for (int64_t e = plan.glue_ptr[g]; e < plan.glue_ptr[g + 1]; ++e)
                    by_dof[plan.glue_col[e]].push_back({a, -plan.glue_val[e]});
            }
        }
        std::vector<double> M((size_t)n * n, 0.0);
        for (const auto& kv : by_dof)
            for (const auto& x : kv.second)
                for (const auto& y : kv.second) M[(size_t)x.first * n + y.first] += x.second * y.second;
        if (!cholesky(n, M, 1e-14)) throw SetupError{AFIETI_ESINGULAR, "B B^T of a non-conforming interface is singular"};
        const std::vector<double> inv = chol_inverse(n, M);
        const int blk = (int)plan.dblk_ptr.size() - 1;
        for (int a = 0; a < n; ++a) {
            plan.c_blk_dir[rows[a]] = 2;
            plan.c_blk_start[rows[a]] = blk;
            plan.c_blk_size[rows[a]] = a;
            plan.dblk_rows.push_back((int)rows[a]);
        }
        plan.dblk_ptr.push_back((int64_t)plan.dblk_rows.size());
        plan.dblk_mat.insert(plan.dblk_mat.end(), inv.begin(), inv.end());
        plan.dblk_moff.push_back((int64_t)plan.dblk_mat.size());
    }
}

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
        if (pr.n_interfaces < 0 || (pr.n_interfaces > 0 && !pr.interfaces))
            fail(AFIETI_EINVAL, "bad interface list");
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
            P.general = in.ctrl != nullptr;
            for (int c = 0; c < 24 && !P.general; ++c) {
                if (!std::isfinite(in.corners[c])) fail(AFIETI_EINVAL, "non-finite corner");
                P.corners[c] = in.corners[c];
            }
            if (dim == 2)
                for (int c = 0; c < 4; ++c) P.corners[3 * c + 2] = 0.0;
            for (int f = 0; f < 6; ++f) {
                P.bc[f] = f < 2 * dim ? in.face_bc[f] : 0;
                if (P.bc[f] < AFIETI_FACE_FREE || P.bc[f] > AFIETI_FACE_TRACTION) fail(AFIETI_EINVAL, "bad face condition");
                if (P.bc[f] == AFIETI_FACE_TRACTION && !pr.traction)
                    fail(AFIETI_EINVAL, "a traction face needs the problem's traction callback");
            }
            int reg_min = in.p;
            for (int l = 0; l < 3; ++l) {
                if (l < dim) {
                    std::vector<double> kv;
                    if (in.knots[l]) {
                        kv.assign(in.knots[l], in.knots[l] + std::max(in.n_knots[l], 0));
                        reg_min = std::min(reg_min, check_open_knots(kv, in.p));
                    } else {
                        if (in.n_el[l] < 1) fail(AFIETI_EINVAL, "n_el must be >= 1");
                        kv = open_uniform_knots(in.n_el[l], in.p, in.reg);
                        reg_min = std::min(reg_min, in.n_el[l] > 1 ? in.reg : in.p - 1);
                    }
                    build_dir(P.dir[l], kv, in.p);
                    if (P.dir[l].n < 3) fail(AFIETI_EINVAL, "need at least 3 basis functions per direction");
                    if (P.dir[l].n > 48) fail(AFIETI_EUNSUPPORTED, "at most 48 basis functions per direction");
                } else {
                    dummy_dir(P.dir[l]);
                }
                P.n[l] = P.dir[l].n;
            }
            // smallest continuity across the patch's interior knots
            P.reg = std::min(reg_min, in.p - 1);
            P.nodes = (int64_t)P.n[0] * P.n[1] * P.n[2];
            P.dof_off = dof;
            dof += dim * P.nodes;
            if (P.general) {
                // explicit control net: the spline map sum_i X_i B_i; the
                // corners are the corner control points; the diameter is the
                // largest distance between two control points (the patch
                // lies in their convex hull; for a multilinear net this is
                // the largest corner distance)
                P.ctrl.assign((size_t)P.nodes * 3, 0.0);
                for (int64_t nd = 0; nd < P.nodes; ++nd)
                    for (int x = 0; x < dim; ++x) {
                        const double v = in.ctrl[nd * 3 + x];
                        if (!std::isfinite(v)) fail(AFIETI_EINVAL, "non-finite control point");
                        P.ctrl[nd * 3 + x] = v;
                    }
                for (int c = 0; c < (1 << dim); ++c) {
                    const int64_t nd = node_index(P.n, (c & 1) ? P.n[0] - 1 : 0, (c & 2) ? P.n[1] - 1 : 0,
                                                  (c & 4) ? P.n[2] - 1 : 0);
                    for (int x = 0; x < 3; ++x) P.corners[3 * c + x] = P.ctrl[nd * 3 + x];
                }
                double H2 = 0;
                for (int64_t a = 0; a < P.nodes; ++a)
                    for (int64_t b = a + 1; b < P.nodes; ++b) {
                        double s2 = 0;
                        for (int x = 0; x < dim; ++x) {
                            const double dd = P.ctrl[a * 3 + x] - P.ctrl[b * 3 + x];
                            s2 += dd * dd;
                        }
                        H2 = std::max(H2, s2);
                    }
                P.H = std::sqrt(H2);
                P.hscale = dim == 3 ? P.H : 1.0;
                // det J > 0 at every Gauss point of the spline map
                for (int64_t q3 = 0; q3 < (dim == 3 ? P.dir[2].nq : 1); ++q3)
                    for (int q2 = 0; q2 < P.dir[1].nq; ++q2)
                        for (int q1 = 0; q1 < P.dir[0].nq; ++q1) {
                            const double eta[3] = {P.dir[0].qx[q1], P.dir[1].qx[q2], dim == 3 ? P.dir[2].qx[q3] : 0.0};
                            double J[3][3];
                            patch_map(P, eta, nullptr, J);
                            if (!(det_of(dim, J) > 0)) fail(AFIETI_EGEOM, "patch map is not orientation preserving");
                        }
            } else {
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
                // det J > 0 at every Gauss point of the multilinear map.  The
                // first column of J does not depend on eta_1 and the others are
                // linear in it, so along a line of Gauss points det J is a
                // quadratic in eta_1, fixed by its values at 0, 1/2 and 1.
                for (int64_t q3 = 0; q3 < (dim == 3 ? P.dir[2].nq : 1); ++q3)
                    for (int q2 = 0; q2 < P.dir[1].nq; ++q2) {
                        double eta[3] = {0.0, P.dir[1].qx[q2], dim == 3 ? P.dir[2].qx[q3] : 0.0};
                        const double d0 = multilinear_det(dim, P.corners, eta);
                        eta[0] = 0.5;
                        const double dh = multilinear_det(dim, P.corners, eta);
                        eta[0] = 1.0;
                        const double d1 = multilinear_det(dim, P.corners, eta);
                        const double c1 = -3.0 * d0 + 4.0 * dh - d1, c2 = 2.0 * d0 - 4.0 * dh + 2.0 * d1;
                        for (int q1 = 0; q1 < P.dir[0].nq; ++q1) {
                            const double t = P.dir[0].qx[q1];
                            if (!(d0 + t * (c1 + t * c2) > 0))
                                fail(AFIETI_EGEOM, "patch map is not orientation preserving");
                        }
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
            }
            plan.patches.push_back(std::move(P));
        }
        pp.n_dof = dof - pp.dof_off;
        // ---- loads of the callbacks (body force, tractions)
        bool any_traction = false;
        for (int k = 0; k < pr.n_patches; ++k)
            for (int f = 0; f < 2 * dim; ++f) any_traction |= plan.patches[pp.patch0 + k].bc[f] == AFIETI_FACE_TRACTION;
        if (pr.body_force || any_traction) {
            pp.fixed_load.assign(pp.n_dof, 0.0);
            for (int k = 0; k < pr.n_patches; ++k) {
                const PatchPlan& P = plan.patches[pp.patch0 + k];
                double* F = pp.fixed_load.data() + (P.dof_off - pp.dof_off);
                if (pr.body_force) add_body_force(P, pr.body_force, pr.ctx, F);
                for (int f = 0; f < 2 * dim; ++f)
                    if (P.bc[f] == AFIETI_FACE_TRACTION) add_traction(P, f, pr.traction, pr.ctx, F);
            }
        }

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
        // glue face fa of patch ka to face fb of patch kb if their corners
        // coincide (returns false otherwise); `orient` >= 0 must equal the
        // orientation the corners give (swap + 2 flip_0 + 4 flip_1)
        std::vector<NcIface> ncs;  // non-conforming interfaces of the problem
        auto glue = [&](int ka, int fa, int kb, int fb, int orient) -> bool {
            const PatchPlan& A = plan.patches[pp.patch0 + ka];
            const PatchPlan& B = plan.patches[pp.patch0 + kb];
            int map[4];
            for (int s = 0; s < nfc; ++s) {
                double Xa[3], Xb[3];
                face_corner(A, fa, s, Xa);
                map[s] = -1;
                for (int t = 0; t < nfc; ++t) {
                    face_corner(B, fb, t, Xb);
                    double d2 = 0;
                    for (int x = 0; x < 3; ++x) d2 += (Xa[x] - Xb[x]) * (Xa[x] - Xb[x]);
                    if (std::sqrt(d2) <= tol) map[s] = t;
                }
                if (map[s] < 0) return false;
            }
            // tangential directions of each face, ascending
            int ta[2], tb[2], na = 0, nb = 0;
            for (int l = 0; l < dim; ++l) {
                if (l != fa / 2) ta[na++] = l;
                if (l != fb / 2) tb[nb++] = l;
            }
            // where does tangential direction j of A go in B, flipped?
            int to[2], flip[2] = {0, 0}, swap = 0;
            bool a_finer = false, b_finer = false;  // knot vectors along the face nested
            for (int j = 0; j < dim - 1; ++j) {
                int u0 = map[0], u1 = map[1 << j];
                int diff = u0 ^ u1;
                if (diff != 1 && diff != 2) fail(AFIETI_EGEOM, "degenerate face correspondence");
                int jb = diff == 1 ? 0 : 1;
                to[j] = tb[jb];
                flip[j] = (u0 >> jb) & 1;
                if (j == 0) swap = jb;
                // equal knot vectors along the face (reversed where flipped),
                // or nested ones (a non-conforming interface, Section 2.2)
                const std::vector<double>& ka_ = A.dir[ta[j]].knots;
                const std::vector<double>& kb_ = B.dir[to[j]].knots;
                bool same = A.p == B.p && ka_.size() == kb_.size();
                for (size_t i = 0; same && i < ka_.size(); ++i)
                    same = std::fabs(ka_[i] - (flip[j] ? 1.0 - kb_[kb_.size() - 1 - i] : kb_[i])) <= 1e-12;
                if (!same) {
                    std::vector<double> kbo(kb_.size());
                    for (size_t i = 0; i < kb_.size(); ++i) kbo[i] = flip[j] ? 1.0 - kb_[kb_.size() - 1 - i] : kb_[i];
                    if (A.p == B.p && !knot_insertion_matrix(ka_, kbo, A.p).empty()) b_finer = true;
                    else if (A.p == B.p && !knot_insertion_matrix(kbo, ka_, A.p).empty()) a_finer = true;
                    else fail(AFIETI_EGEOM, "non-conforming interface");
                }
            }
            if (orient >= 0 && orient != swap + 2 * flip[0] + 4 * flip[1])
                fail(AFIETI_EGEOM, "interface orientation does not match the corners");
            if (A.bc[fa] == AFIETI_FACE_TRACTION || B.bc[fb] == AFIETI_FACE_TRACTION)
                fail(AFIETI_EGEOM, "a traction face is an interface");
            if (a_finer || b_finer) {
                // non-conforming: the finer face is glued to the coarse trace
                // (rows of their own below); parametric directions aligned
                if (a_finer && b_finer) fail(AFIETI_EGEOM, "non-conforming interface refined on both sides");
                if (fa / 2 != fb / 2 || swap || flip[0] || flip[1])
                    fail(AFIETI_EUNSUPPORTED, "non-conforming interface with differently oriented parametrisations");
                NcIface nc;
                nc.slave = a_finer ? ka : kb;
                nc.sface = a_finer ? fa : fb;
                nc.master = a_finer ? kb : ka;
                nc.mface = a_finer ? fb : fa;
                const PatchPlan& Ps = a_finer ? A : B;
                const PatchPlan& Pm = a_finer ? B : A;
                for (int j = 0; j < dim - 1; ++j) {
                    nc.ns[j] = Ps.n[ta[j]];
                    nc.nm[j] = Pm.n[ta[j]];
                    nc.T[j] = knot_insertion_matrix(Pm.dir[ta[j]].knots, Ps.dir[ta[j]].knots, Ps.p);
                }
                if (dim == 2) nc.ns[1] = nc.nm[1] = 1, nc.T[1] = {1.0};
                nc.tang[0] = ta[0];
                nc.tang[1] = dim == 3 ? ta[1] : -1;
                if (Ps.general || Pm.general) {  // the finer face net is the coarse one refined
                    for (int s2 = 0; s2 < nc.ns[1]; ++s2)
                        for (int s1 = 0; s1 < nc.ns[0]; ++s1) {
                            double X[3] = {0, 0, 0};
                            for (int t2 = 0; t2 < nc.nm[1]; ++t2)
                                for (int t1 = 0; t1 < nc.nm[0]; ++t1) {
                                    const double w = nc.T[0][(size_t)s1 * nc.nm[0] + t1] * nc.T[1][(size_t)s2 * nc.nm[1] + t2];
                                    if (w == 0.0) continue;
                                    const int64_t nd = nc.face_node(Pm, t1, t2);
                                    for (int x = 0; x < 3; ++x) X[x] += w * Pm.ctrl[nd * 3 + x];
                                }
                            const int64_t nd = nc.face_node(Ps, s1, s2, true);
                            double d2 = 0;
                            for (int x = 0; x < 3; ++x) d2 += (X[x] - Ps.ctrl[nd * 3 + x]) * (X[x] - Ps.ctrl[nd * 3 + x]);
                            if (std::sqrt(d2) > tol) fail(AFIETI_EGEOM, "interface control points differ");
                        }
                }
                ncs.push_back(std::move(nc));
                return true;
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
                    const int64_t na_ = node_index(A.n, ia[0], ia[1], ia[2]);
                    const int64_t nb_ = node_index(B.n, ib[0], ib[1], ib[2]);
                    if (A.general || B.general) {  // the two faces' nets must coincide
                        double d2 = 0;
                        for (int x = 0; x < 3; ++x) {
                            const double dd = A.ctrl[na_ * 3 + x] - B.ctrl[nb_ * 3 + x];
                            d2 += dd * dd;
                        }
                        if (std::sqrt(d2) > tol) fail(AFIETI_EGEOM, "interface control points differ");
                    }
                    uf.unite(node_off[ka] + na_, node_off[kb] + nb_);
                }
            return true;
        };
        if (pr.n_interfaces == 0) {
            // every pair of faces whose corners coincide
            for (int ka = 0; ka < pr.n_patches; ++ka)
                for (int kb = ka + 1; kb < pr.n_patches; ++kb)
                    for (int fa = 0; fa < 2 * dim; ++fa)
                        for (int fb = 0; fb < 2 * dim; ++fb) glue(ka, fa, kb, fb, -1);
        } else {
            // only the listed pairs (coinciding faces not listed stay apart)
            std::vector<char> used((size_t)pr.n_patches * 2 * dim, 0);
            for (int i = 0; i < pr.n_interfaces; ++i) {
                const int* e = pr.interfaces + 5 * i;
                const int ka = e[0], fa = e[1], kb = e[2], fb = e[3], orient = e[4];
                if (ka < 0 || ka >= pr.n_patches || kb < 0 || kb >= pr.n_patches || ka == kb || fa < 0 ||
                    fa >= 2 * dim || fb < 0 || fb >= 2 * dim || orient < -1 || orient > (dim == 3 ? 7 : 2) ||
                    (dim == 2 && orient >= 0 && (orient & 5)))
                    fail(AFIETI_EINVAL, "bad interface entry");
                char& ua = used[(size_t)ka * 2 * dim + fa];
                char& ub = used[(size_t)kb * 2 * dim + fb];
                if (ua || ub) fail(AFIETI_EINVAL, "a face is listed in two interfaces");
                ua = ub = 1;
                if (!glue(ka, fa, kb, fb, orient)) fail(AFIETI_EGEOM, "listed interface faces do not coincide");
            }
        }
        // ---- the finer faces of non-conforming interfaces: their nodes are
        // glued to the coarse trace by rows of their own, not identified with
        // other copies (a node shared with a third patch is not supported)
        std::vector<char> glued(node_off.back(), 0);
        for (const NcIface& nc : ncs) {
            const PatchPlan& Ps = plan.patches[pp.patch0 + nc.slave];
            for (int s2 = 0; s2 < nc.ns[1]; ++s2)
                for (int s1 = 0; s1 < nc.ns[0]; ++s1) {
                    const int64_t g = node_off[nc.slave] + nc.face_node(Ps, s1, s2, true);
                    if (glued[g]) fail(AFIETI_EUNSUPPORTED, "a face node in two non-conforming interfaces");
                    glued[g] = 1;
                }
        }
        {
            std::vector<int64_t> size(node_off.back(), 0);
            for (int64_t g = 0; g < node_off.back(); ++g) size[uf.find(g)]++;
            for (int64_t g = 0; g < node_off.back(); ++g)
                if (glued[g] && size[uf.find(g)] > 1)
                    fail(AFIETI_EUNSUPPORTED, "a non-conforming face node shared with a third patch");
        }
        // ---- classes in (lowest patch, local index) order
        struct Copy { int k; int64_t node; };
        std::vector<std::vector<Copy>> classes;
        std::vector<int64_t> class_of(node_off.back(), -1);
        for (int k = 0; k < pr.n_patches; ++k) {
            const PatchPlan& P = plan.patches[pp.patch0 + k];
            for (int64_t nd = 0; nd < P.nodes; ++nd) {
                if (!is_gamma(P, nd) || glued[node_off[k] + nd]) continue;
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
        for (int comp = 0; comp < dim; ++comp) {
            const int64_t comp_start = (int64_t)plan.c_plus.size();
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
            if (!ncs.empty()) add_gluing_rows(plan, pp, ncs, comp, comp_start);
        }
        crow = (int64_t)plan.c_plus.size();
        pp.n_c = crow - pp.c_off;
        if (pp.n_c == 0) fail(AFIETI_ESINGULAR, "no constraints: the problem has no Dirichlet boundary");
        // ---- Dirichlet data: g_D at the control point of every Dirichlet
        // copy, one call for the problem; rows of the Dirichlet nodes read
        // B u = g_D
        if (pr.dirichlet) {
            std::vector<int64_t> rows;
            std::vector<double> pts;
            for (int64_t r = pp.c_off; r < crow; ++r) {
                if (plan.c_minus[r] != -1) continue;
                const PatchPlan& P = plan.patches[plan.c_patch_plus[r]];
                const int64_t loc = plan.c_plus[r] - P.dof_off;
                const int64_t nd = loc % P.nodes;
                rows.push_back(r);
                for (int x = 0; x < dim; ++x) pts.push_back(P.ctrl[nd * 3 + x]);
            }
            std::vector<double> val(pts.size(), 0.0);
            if (!rows.empty()) pr.dirichlet((int64_t)rows.size(), pts.data(), val.data(), pr.ctx);
            if (plan.c_rhs.empty()) plan.c_rhs.assign(crow, 0.0);
            plan.c_rhs.resize(crow, 0.0);
            for (size_t i = 0; i < rows.size(); ++i) {
                const int64_t r = rows[i];
                const PatchPlan& P = plan.patches[plan.c_patch_plus[r]];
                const int comp = (int)((plan.c_plus[r] - P.dof_off) / P.nodes);
                const double v = val[i * dim + comp];
                if (!std::isfinite(v)) fail(AFIETI_EINVAL, "non-finite Dirichlet data");
                plan.c_rhs[r] = v;
            }
        } else if (!plan.c_rhs.empty()) {
            plan.c_rhs.resize(crow, 0.0);
        }
        plan.probs.push_back(std::move(pp));
    }
    plan.n_dof = dof;
    plan.n_c = crow;
    if (!plan.c_rhs.empty()) plan.c_rhs.resize(crow, 0.0);
    if (plan.n_dof > (int64_t)INT32_MAX || plan.n_c > (int64_t)INT32_MAX)
        fail(AFIETI_EUNSUPPORTED, "more than 2^31 unknowns");

    // ---- B^T by DOF (CSR), rows ascending within a DOF
    std::vector<int64_t> cnt(plan.n_dof + 1, 0);
    for (int64_t r = 0; r < plan.n_c; ++r) {
        cnt[plan.c_plus[r] + 1]++;
        if (plan.c_minus[r] >= 0) cnt[plan.c_minus[r] + 1]++;
        if (plan.c_minus[r] <= -2) {
            const int64_t g = -2 - plan.c_minus[r];
            for (int64_t e = plan.glue_ptr[g]; e < plan.glue_ptr[g + 1]; ++e) cnt[plan.glue_col[e] + 1]++;
        }
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
        if (plan.c_minus[r] <= -2) {
            const int64_t g = -2 - plan.c_minus[r];
            for (int64_t e = plan.glue_ptr[g]; e < plan.glue_ptr[g + 1]; ++e) {
                int64_t b = fill[plan.glue_col[e]]++;
                plan.bt_row[b] = (int)r;
                plan.bt_sign[b] = -plan.glue_val[e];
            }
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
            if (plan.c_minus[r] <= -2) {  // the coarse trace's modes: sum_j T_ij R(j)
                const int64_t g = -2 - plan.c_minus[r];
                double v = 0.0;
                for (int64_t e = plan.glue_ptr[g]; e < plan.glue_ptr[g + 1]; ++e)
                    v += plan.glue_val[e] * dof_mode(plan.glue_col[e], plan.c_patch_minus[r], m);
                plan.g_minus[r * 6 + m] = v;
            }
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
            int ib = plan.c_patch_minus[r] >= 0 ? (plan.c_patch_minus[r] - pp.patch0) * nm : -1;
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
