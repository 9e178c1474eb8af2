// Host-side setup of the inexact AF-IETI solver: everything that is built
// once per problem in FP64 on the CPU (spline data, univariate pencils and
// their eigendecompositions, node matching, the jump matrix B, rigid modes,
// the coarse factorisation and the index tables the device kernels read).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "afieti.h"

namespace afieti {

struct SetupError {
    int code;
    std::string msg;
};

// Univariate spline data of one parametric direction of one patch.
struct Dir1D {
    int n = 1;                    // number of B-splines m_l
    int n_el = 0;                 // elements (non-empty spans)
    int p = 0;
    std::vector<double> knots;
    // composite Gauss rule, p+1 points per element
    int nq = 0;
    std::vector<double> qx, qw;
    std::vector<int> qfirst;      // first nonzero basis index at each point
    std::vector<double> qval, qder;  // [q][t], t = 0..p (basis qfirst+t)
    std::vector<int> el_first, el_last;  // elements in the support of basis i
    // univariate matrices (dense n x n, row major)
    std::vector<double> K, M;
    // generalised eigendecompositions: U^T M U = I, U^T K U = diag(D)
    std::vector<double> U, D;     // full pencil, U[i*n + a]
    std::vector<double> Ui, Di;   // interior pencil (n-2)
};

// Weighted univariate pencil of one (displacement component, direction) of a
// patch for the geometry-inclusion local solvers (Section 5.2.3).
struct GeoPencil {
    std::vector<double> K, M;     // K~ = int nu b' b', M~ = int beta b b (n x n)
    std::vector<double> U, D;     // U^T M~ U = I, U^T K~ U = diag(D)
    std::vector<double> Ui, Di;   // interior pencil (n-2)
};

struct PatchPlan {
    int prob = 0;                 // problem index
    int dim = 3;
    int p = 1, reg = 0;
    Dir1D dir[3];                 // 2D: dir[2] is a dummy of size 1
    int n[3] = {1, 1, 1};         // basis counts, n[2] = 1 in 2D
    int64_t nodes = 0;            // n1*n2*n3
    int64_t dof_off = 0;          // global DOF offset of the patch
    double lam = 1, mu = 1, H = 1, hscale = 1;  // hscale = H^{d-2}
    double corners[24] = {0};
    int bc[6] = {0};
    std::vector<double> ctrl;     // [node][3] control points (z = 0 in 2D)
    bool general = false;         // explicit control net (else the corners' multilinear map)
    // geometry inclusion (filled by build_geometry_inclusion)
    GeoPencil gp[3][3];           // [component][direction]
    std::vector<double> geo_da;   // [component][node]: D_A^{-1/2}
    std::vector<double> geo_ds;   // [component][node]: D_S^{1/2}
};

struct ProblemPlan {
    int dim = 3;
    int patch0 = 0, n_patches = 0;
    int64_t dof_off = 0, n_dof = 0;
    int64_t c_off = 0, n_c = 0;
    int n_modes = 6;              // rigid modes per patch (3 in 2D)
    std::vector<double> Cinv;     // (G^T G)^{-1}, dense (n_modes*N_p)^2
    std::vector<double> CtC;      // G^T G (for export)
    std::vector<afieti_load_mode> load;
    // load of the body-force and traction callbacks (n_dof of the problem,
    // patch-stacked), empty without callbacks
    std::vector<double> fixed_load;
};

struct Plan {
    std::vector<PatchPlan> patches;
    std::vector<ProblemPlan> probs;
    int64_t n_dof = 0, n_c = 0;
    // constraints (global rows): B row r = e_{plus[r]} - e_{minus[r]}
    // (minus = -1 for a Dirichlet row, whose entry is +1 on plus; minus =
    // -2 - g for the gluing row g of a non-conforming interface, B row
    // e_{plus} - sum_e glue_val[e] e_{glue_col[e]} over e in
    // [glue_ptr[g], glue_ptr[g + 1]))
    std::vector<int64_t> c_plus, c_minus;
    std::vector<int64_t> glue_ptr{0}, glue_col;
    std::vector<double> glue_val;
    // block of B B^T holding each row: dir 0 star block (start, size), 1
    // identity (a Dirichlet row alone), 2 dense block (start = block index,
    // size = the row's position in it)
    std::vector<int> c_blk_start, c_blk_size, c_blk_dir;
    // dense blocks of B B^T (non-conforming interfaces with the Dirichlet
    // rows they couple to): rows dblk_rows[dblk_ptr[b] ..], inverse
    // dblk_mat[dblk_moff[b] ..] row major
    std::vector<int64_t> dblk_ptr{0}, dblk_moff{0};
    std::vector<int> dblk_rows;
    std::vector<double> dblk_mat;
    // B^T by DOF: CSR over all DOFs, entries (row, sign)
    std::vector<int64_t> bt_ptr;
    std::vector<int> bt_row;
    std::vector<double> bt_sign;
    // rigid-mode values of G rows: G[r][m] for plus and minus copies
    std::vector<double> g_plus, g_minus;  // [r][6]
    std::vector<int> c_patch_plus, c_patch_minus;  // patch of each copy (-1)
    // (R^(k)T R^(k))^{-1} per patch, [k][6][6]
    std::vector<double> RtR_inv;
    // right-hand side of the constraints B u = c: the Dirichlet data of the
    // Dirichlet rows (zero on interface rows); empty when all data are zero
    std::vector<double> c_rhs;
};

// Build the host plan.  Throws SetupError.
Plan build_plan(const afieti_problem* probs, int n_problems);

// Geometry-inclusion data of every patch (separable fit, weighted pencils,
// scalings; Section 5.2.3), on up to n_threads host threads.  Depends on
// the patches' Lame parameters.  Throws SetupError.
void build_geometry_inclusion(Plan& plan, int n_threads);

// Helpers exposed for testing.
std::vector<double> open_uniform_knots(int n_el, int p, int reg);
// checks an explicit open knot vector of degree p on [0, 1]; returns the
// smallest continuity p - (largest interior multiplicity)
int check_open_knots(const std::vector<double>& t, int p);
// coarse B-splines in the basis of a refined knot vector (knot insertion):
// T[i * n_c + j], b^c_j = sum_i T_ij b^f_i; empty unless fine contains coarse
std::vector<double> knot_insertion_matrix(const std::vector<double>& coarse, const std::vector<double>& fine, int p);
void bspline_eval(const std::vector<double>& knots, int p, double x, int& first,
                  double* val, double* der);
void gauss_legendre(int n, double* x, double* w);
int sym_gen_eig(int n, const double* K, const double* M, double* U, double* D);
// J[x][a] = dF_x / deta_a of the multilinear map of the 2^dim corners
void multilinear_jacobian(int dim, const double* corners, const double* eta, double (&J)[3][3]);
// point x (may be NULL) and Jacobian J[x][a] = dF_x / deta_a of a patch's
// geometry map at eta: the corners' multilinear map, or the spline map of
// an explicit control net
void patch_map(const PatchPlan& P, const double* eta, double* x, double (&J)[3][3]);
double rigid_mode(int dim, int m, int c, const double* X);

}  // namespace afieti
