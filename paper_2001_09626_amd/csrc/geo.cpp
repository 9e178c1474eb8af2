// Inexact local solvers with geometry inclusion (Section 5.2.3), host part:
// per patch k and displacement component l,
//   * the coefficient matrix of the (l,l) stiffness block pulled back to the
//     parameter domain, C_l = [mu J^-1 J^-T + (mu + lam) J^-1 e_l e_l^T J^-T]
//     |det J|, at the tensor Gauss points;
//   * the separable approximation [C_l]_ii ~ nu_{l,i}(eta_i) prod_{m != i}
//     beta_{l,m}(eta_m): a least-squares fit in log space over the Gauss
//     points, weighted by the product Gauss weights, of the d diagonal
//     entries together with log |det J| = sum_m log beta_{l,m} (the mass
//     weight, which fixes the factors up to constants that leave the
//     Kronecker operators unchanged).  With product weights the fit
//     separates into weighted means: y_0 = log |det J|, y_i = log [C_l]_ii,
//     ybar_i their weighted means and y_i^(m)(eta_m) the weighted means
//     over every direction but m minus ybar_i:
//       log nu_{l,m}   = y_m^(m) + ybar_m - (d-1) ybar_0 / d,
//       log beta_{l,m} = (1/d) sum_{i in {0} u {1..d}, i != m} y_i^(m) + ybar_0 / d;
//   * the weighted univariate pencils K~_{l,m} = int nu b' b',
//     M~_{l,m} = int beta b b and their generalised eigendecompositions
//     (full and interior);
//   * the scalings D_A = diag(A_ll + H^-2 M) / diag(A~_l + H^-2 M~_l) and
//     D_S = diag(A_ll) / diag(A~_l), the diagonals of the physical stiffness
//     block and mass by sum factorisation over the Gauss grid.
// Patches are processed on several host threads.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <vector>

#include "plan.h"

namespace afieti {

namespace {

// The Gauss rule of one direction (a direction the patch does not have is
// one point of weight 1 where its single function is 1, with derivative 0).
struct Line {
    int nq = 1, P = 1, n = 1;
    std::vector<double> x, w, val, der;  // val/der: [q][t], basis first[q] + t
    std::vector<int> first;
    explicit Line(const Dir1D& d, bool active) {
        if (active) {
            nq = d.nq;
            P = d.p + 1;
            n = d.n;
            x = d.qx;
            w = d.qw;
            val = d.qval;
            der = d.qder;
            first = d.qfirst;
        } else {
            x = {0.0};
            w = {1.0};
            val = {1.0};
            der = {0.0};
            first = {0};
        }
    }
};

void invert3(const double (&J)[3][3], int dim, double (&Ji)[3][3], double& det) {
    for (auto& r : Ji)
        for (double& v : r) v = 0.0;
    if (dim == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        Ji[0][0] = J[1][1] / det;
        Ji[0][1] = -J[0][1] / det;
        Ji[1][0] = -J[1][0] / det;
        Ji[1][1] = J[0][0] / det;
        return;
    }
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    Ji[0][0] = c00 / det;
    Ji[1][0] = c01 / det;
    Ji[2][0] = c02 / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
}

// C_l at one point (Ji[a][x] = (J^-1)_{a x}, adet = |det J|), symmetric d x d
void coefficient(const double (&Ji)[3][3], double adet, int dim, double lam, double mu, int l, double (&C)[3][3]) {
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) {
            double g = 0;
            for (int x = 0; x < dim; ++x) g += Ji[a][x] * Ji[b][x];
            C[a][b] = (mu * g + (mu + lam) * Ji[a][l] * Ji[b][l]) * adet;
        }
}

// y_i^(m) accumulators: sums over the grid of W_{-m} y at each 1D point of m
struct Marginals {
    // [set i = 0..d][direction m][q_m]
    std::vector<double> v[4][3];
    double mean[4] = {0, 0, 0, 0};
};

// diag of sum_q F(q) prod_m T_m(i_m, q_m) by sum factorisation: the field is
// delivered one q1-line at a time (accumulate), then contracted along q2, q3
struct DiagContraction {
    int n[3], nq[3];
    std::vector<double> g1;  // [q3][q2][i1]
    void init(const int* n_, const int* nq_) {
        for (int m = 0; m < 3; ++m) {
            n[m] = n_[m];
            nq[m] = nq_[m];
        }
        g1.assign((size_t)nq[2] * nq[1] * n[0], 0.0);
    }
    // add the contraction of one q1-line F[q1] with T1 (table [q][t], first)
    void line(int q2, int q3, const double* F, const Line& L1, const double* T1) {
        double* out = &g1[((size_t)q3 * nq[1] + q2) * n[0]];
        for (int q = 0; q < L1.nq; ++q)
            for (int t = 0; t < L1.P; ++t) out[L1.first[q] + t] += T1[(size_t)q * L1.P + t] * F[q];
    }
    // finish along q2 (T2) and q3 (T3): result [i3][i2][i1]
    std::vector<double> finish(const Line& L2, const double* T2, const Line& L3, const double* T3) const {
        std::vector<double> g2((size_t)nq[2] * n[1] * n[0], 0.0);
        for (int q3 = 0; q3 < nq[2]; ++q3)
            for (int q = 0; q < L2.nq; ++q)
                for (int t = 0; t < L2.P; ++t) {
                    const double c = T2[(size_t)q * L2.P + t];
                    const double* src = &g1[((size_t)q3 * nq[1] + q) * n[0]];
                    double* dst = &g2[((size_t)q3 * n[1] + L2.first[q] + t) * n[0]];
                    for (int i1 = 0; i1 < n[0]; ++i1) dst[i1] += c * src[i1];
                }
        std::vector<double> g3((size_t)n[2] * n[1] * n[0], 0.0);
        const size_t sl = (size_t)n[1] * n[0];
        for (int q = 0; q < L3.nq; ++q)
            for (int t = 0; t < L3.P; ++t) {
                const double c = T3[(size_t)q * L3.P + t];
                const double* src = &g2[(size_t)q * sl];
                double* dst = &g3[(size_t)(L3.first[q] + t) * sl];
                for (size_t e = 0; e < sl; ++e) dst[e] += c * src[e];
            }
        return g3;
    }
};

// T_m for the pair (a, b) of parametric derivatives: f_a f_b, f = der on the
// differentiated direction, val elsewhere
std::vector<double> pair_table(const Line& L, int m, int a, int b) {
    std::vector<double> T(L.val.size());
    for (size_t e = 0; e < T.size(); ++e) {
        const double fa = m == a ? L.der[e] : L.val[e];
        const double fb = m == b ? L.der[e] : L.val[e];
        T[e] = fa * fb;
    }
    return T;
}

void build_patch(PatchPlan& P) {
    const int dim = P.dim;
    const Line L[3] = {Line(P.dir[0], true), Line(P.dir[1], true), Line(P.dir[2], dim == 3)};
    const int nq[3] = {L[0].nq, L[1].nq, L[2].nq};
    const int nb[3] = {P.n[0], P.n[1], P.n[2]};
    const double h2 = 1.0 / (P.H * P.H);
    // pairs (a <= b) of parametric directions; the diagonal sums 2 C_ab for a < b
    std::vector<std::pair<int, int>> pairs;
    for (int a = 0; a < dim; ++a)
        for (int b = a; b < dim; ++b) pairs.push_back({a, b});
    const int npair = (int)pairs.size();
    // one contraction per (component, pair), plus the mass
    std::vector<DiagContraction> dc((size_t)dim * npair + 1);
    for (auto& c : dc) c.init(nb, nq);
    std::vector<std::vector<double>> T1(npair);
    for (int j = 0; j < npair; ++j) T1[j] = pair_table(L[0], 0, pairs[j].first, pairs[j].second);
    const std::vector<double> T1m = pair_table(L[0], 0, -1, -1);
    Marginals mg[3];
    for (int l = 0; l < dim; ++l)
        for (int i = 0; i <= dim; ++i)
            for (int m = 0; m < dim; ++m) mg[l].v[i][m].assign(nq[m], 0.0);
    std::vector<double> F((size_t)nq[0]);
    std::vector<double> Cl((size_t)nq[0] * dim * 9), adet(nq[0]);
    for (int q3 = 0; q3 < nq[2]; ++q3)
        for (int q2 = 0; q2 < nq[1]; ++q2) {
            const double w23 = L[1].w[q2] * L[2].w[q3];
            for (int q1 = 0; q1 < nq[0]; ++q1) {
                const double eta[3] = {L[0].x[q1], L[1].x[q2], dim == 3 ? L[2].x[q3] : 0.0};
                double J[3][3], Ji[3][3], det;
                patch_map(P, eta, nullptr, J);
                invert3(J, dim, Ji, det);
                adet[q1] = std::fabs(det);
                for (int l = 0; l < dim; ++l) {
                    double C[3][3];
                    coefficient(Ji, adet[q1], dim, P.lam, P.mu, l, C);
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) Cl[((size_t)q1 * dim + l) * 9 + a * 3 + b] = C[a][b];
                }
            }
            // marginal sums of the logs (set 0: |det J|, set 1 + i: [C_l]_ii)
            for (int l = 0; l < dim; ++l)
                for (int q1 = 0; q1 < nq[0]; ++q1) {
                    const double W = L[0].w[q1] * w23;
                    const int qm[3] = {q1, q2, q3};
                    for (int i = 0; i <= dim; ++i) {
                        const double y =
                            std::log(i == 0 ? adet[q1] : Cl[((size_t)q1 * dim + l) * 9 + (i - 1) * 4]);
                        mg[l].mean[i] += W * y;
                        for (int m = 0; m < dim; ++m) mg[l].v[i][m][qm[m]] += W / L[m].w[qm[m]] * y;
                    }
                }
            // diagonal contractions along q1
            for (int l = 0; l < dim; ++l)
                for (int j = 0; j < npair; ++j) {
                    const int a = pairs[j].first, b = pairs[j].second;
                    for (int q1 = 0; q1 < nq[0]; ++q1)
                        F[q1] = L[0].w[q1] * w23 * (a == b ? 1.0 : 2.0) * Cl[((size_t)q1 * dim + l) * 9 + a * 3 + b];
                    dc[(size_t)l * npair + j].line(q2, q3, F.data(), L[0], T1[j].data());
                }
            for (int q1 = 0; q1 < nq[0]; ++q1) F[q1] = L[0].w[q1] * w23 * adet[q1];
            dc.back().line(q2, q3, F.data(), L[0], T1m.data());
        }
    // mass diagonal
    const std::vector<double> T2m = pair_table(L[1], 1, -1, -1), T3m = pair_table(L[2], 2, -1, -1);
    const std::vector<double> mdiag = dc.back().finish(L[1], T2m.data(), L[2], T3m.data());
    for (int l = 0; l < dim; ++l) {
        // stiffness diagonal of the (l,l) block
        std::vector<double> adiag((size_t)P.nodes, 0.0);
        for (int j = 0; j < npair; ++j) {
            const int a = pairs[j].first, b = pairs[j].second;
            const std::vector<double> T2 = pair_table(L[1], 1, a, b), T3 = pair_table(L[2], 2, a, b);
            const std::vector<double> g = dc[(size_t)l * npair + j].finish(L[1], T2.data(), L[2], T3.data());
            for (int64_t e = 0; e < P.nodes; ++e) adiag[e] += g[e];
        }
        // the separable fit
        const Marginals& M = mg[l];
        std::vector<double> nu[3], beta[3];
        for (int m = 0; m < dim; ++m) {
            nu[m].resize(nq[m]);
            beta[m].resize(nq[m]);
            for (int q = 0; q < nq[m]; ++q) {
                const double a = M.v[1 + m][m][q] - (dim - 1) * M.mean[0] / dim;
                double b = M.v[0][m][q] - M.mean[0];
                for (int i = 0; i < dim; ++i)
                    if (i != m) b += M.v[1 + i][m][q] - M.mean[1 + i];
                nu[m][q] = std::exp(a);
                beta[m][q] = std::exp(b / dim + M.mean[0] / dim);
            }
        }
        // weighted univariate pencils and their eigendecompositions
        for (int m = 0; m < 3; ++m) {
            GeoPencil& g = P.gp[l][m];
            const int n = nb[m];
            if (m >= dim) {
                g.K = {0.0};
                g.M = {1.0};
                g.U = {1.0};
                g.D = {0.0};
                g.Ui = {1.0};
                g.Di = {0.0};
                continue;
            }
            const Line& Lm = L[m];
            g.K.assign((size_t)n * n, 0.0);
            g.M.assign((size_t)n * n, 0.0);
            for (int q = 0; q < Lm.nq; ++q) {
                const int f = Lm.first[q];
                for (int s = 0; s < Lm.P; ++s)
                    for (int t = 0; t < Lm.P; ++t) {
                        g.K[(size_t)(f + s) * n + f + t] +=
                            Lm.w[q] * nu[m][q] * Lm.der[(size_t)q * Lm.P + s] * Lm.der[(size_t)q * Lm.P + t];
                        g.M[(size_t)(f + s) * n + f + t] +=
                            Lm.w[q] * beta[m][q] * Lm.val[(size_t)q * Lm.P + s] * Lm.val[(size_t)q * Lm.P + t];
                    }
            }
            g.U.resize((size_t)n * n);
            g.D.resize(n);
            if (sym_gen_eig(n, g.K.data(), g.M.data(), g.U.data(), g.D.data()) != 0)
                throw SetupError{AFIETI_ESINGULAR, "weighted univariate mass matrix not positive definite"};
            const int ni = n - 2;
            std::vector<double> Ki((size_t)ni * ni), Mi((size_t)ni * ni);
            for (int i = 0; i < ni; ++i)
                for (int j = 0; j < ni; ++j) {
                    Ki[(size_t)i * ni + j] = g.K[(size_t)(i + 1) * n + j + 1];
                    Mi[(size_t)i * ni + j] = g.M[(size_t)(i + 1) * n + j + 1];
                }
            g.Ui.resize((size_t)ni * ni);
            g.Di.resize(ni);
            if (sym_gen_eig(ni, Ki.data(), Mi.data(), g.Ui.data(), g.Di.data()) != 0)
                throw SetupError{AFIETI_ESINGULAR, "weighted interior univariate mass matrix not positive definite"};
        }
        // the scalings
        double* da = &P.geo_da[(size_t)l * P.nodes];
        double* ds = &P.geo_ds[(size_t)l * P.nodes];
        for (int i3 = 0; i3 < nb[2]; ++i3)
            for (int i2 = 0; i2 < nb[1]; ++i2)
                for (int i1 = 0; i1 < nb[0]; ++i1) {
                    const int idx[3] = {i1, i2, i3};
                    double kd[3], md[3];
                    for (int m = 0; m < 3; ++m) {
                        const GeoPencil& g = P.gp[l][m];
                        const int n = m < dim ? nb[m] : 1;
                        kd[m] = g.K[(size_t)idx[m] * n + idx[m]];
                        md[m] = g.M[(size_t)idx[m] * n + idx[m]];
                    }
                    double at = 0.0;
                    for (int m = 0; m < dim; ++m) {
                        double t = kd[m];
                        for (int o = 0; o < dim; ++o)
                            if (o != m) t *= md[o];
                        at += t;
                    }
                    double mt = 1.0;
                    for (int m = 0; m < dim; ++m) mt *= md[m];
                    const int64_t e = i1 + (int64_t)nb[0] * (i2 + (int64_t)nb[1] * i3);
                    da[e] = 1.0 / std::sqrt((adiag[e] + h2 * mdiag[e]) / (at + h2 * mt));
                    ds[e] = std::sqrt(adiag[e] / at);
                }
    }
}

}  // namespace

void build_geometry_inclusion(Plan& plan, int n_threads) {
    const int np = (int)plan.patches.size();
    for (auto& P : plan.patches) {
        P.geo_da.assign((size_t)P.dim * P.nodes, 0.0);
        P.geo_ds.assign((size_t)P.dim * P.nodes, 0.0);
    }
    std::atomic<int> next{0};
    std::vector<std::thread> pool;
    std::vector<SetupError> first_err(std::max(1, n_threads));
    std::vector<int> has_err(std::max(1, n_threads), 0);
    const int nt = std::max(1, std::min(n_threads, np));
    for (int t = 0; t < nt; ++t)
        pool.emplace_back([&, t] {
            for (int k = next++; k < np; k = next++) {
                try {
                    build_patch(plan.patches[k]);
                } catch (const SetupError& e) {
                    if (!has_err[t]) first_err[t] = e;
                    has_err[t] = 1;
                }
            }
        });
    for (auto& th : pool) th.join();
    for (int t = 0; t < nt; ++t)
        if (has_err[t]) throw first_err[t];
}

}  // namespace afieti
