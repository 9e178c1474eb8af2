// Device-side descriptors shared by the HIP kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace afieti {

constexpr int kMaxN = 48;        // largest univariate basis size on the device path
constexpr int kBlock = 256;      // threads per block for the streaming kernels
constexpr int kChunk = 1024;     // elements per reduction chunk (DOF and Krylov vectors)
constexpr int kGamChunk = 256;   // Gamma DOFs per reduction chunk

// One patch as the kernels see it.
struct DevPatch {
    int64_t dof_off;             // global DOF offset
    int64_t nodes;               // n1 * n2 * n3
    int64_t ctrl_off;            // offset (in doubles) into the control-point array
    int64_t stencil_off;         // offset (in doubles) into the stencil values
    int64_t geo_off;             // offset (in doubles) into the Gauss-point geometry
    int n[3];                    // basis counts (n[2] = 1 in 2D)
    int nq[3];                   // Gauss points per direction (nq[2] = 1 in 2D)
    int q_off[3];                // offsets into the univariate quadrature tables
    int band_off[3][3];          // [component][direction]: offsets into the banded univariate
                                 // K, M tables of the operator A-hat_l (or A~_l)
    double kap[3][3];            // [component][direction]: its Kronecker coefficients
    int el_off[3];               // offsets into the per-basis element ranges
    int dim, p, prob, nmodes;
    double lam, mu, hscale;
    double corners[24];          // multilinear patch map (corner a1 + 2 a2 + 4 a3)
    double jcoef[36];            // dF_x/deta_a = c0 + c1 eta_b + c2 eta_c + c3 eta_b eta_c, [a][x][4]
    int nb[3];                   // matrix-free bricks per direction
    int mf;                      // 1: stiffness applied matrix-free
    int64_t ybuf_off;            // offset (in doubles) of its bricks' partial results
    int64_t tab_off[3];          // offsets (in doubles) of its per-brick univariate tables
};

// One tensor of an FD solve (a patch/component pair, or its interior).
struct FdTensor {
    int64_t in_off, out_off;     // first entry in the FP64 input / output vector
    int64_t tmp_off;             // first entry in the intermediate buffer
    int n1, n2, n3;              // tensor sizes
    int s2, s3;                  // strides of directions 2 and 3 in the vectors
    int u_off[3];                // U_m (n_m x n_m, U[i*n + a]) in the eigenvector table
    int d_off[3];                // D_m in the eigenvalue table
    double kappa[3];             // Kronecker coefficients kappa_{l,m}
    double scale;                // (H^(k))^{d-2} for P_A, 1 for the interior solve
    double mass;                 // 1 for P_A (mass term), 0 for the interior solve
    double alpha;                // output = alpha * solution
    int prob;                    // problem index (for the stop mask)
    int pad;
};

// The d component tensors of one patch in one FD operator (or their
// interiors): they share the univariate eigenvectors U_m, so the matrix-core
// FD kernels process them together.  Component c of the group starts at
// in_off + c cstride (out_off + c cstride) in the FP64 vectors and at
// tmp_off + c n1 n2 n3 in the intermediate buffer.
struct FdGroup {
    int64_t in_off, out_off;     // component 0 in the FP64 input / output vector
    int64_t cstride;             // offset between components in the vectors
    int64_t tmp_off;             // component 0 in the intermediate buffer
    int n1, n2, n3, nc;          // tensor sizes, number of components
    int s2, s3;                  // strides of directions 2 and 3 in the vectors
    int u_off[3];                // U_m (n_m x n_m, U[i*n + a]) in the eigenvector table
    int d_off[3];                // D_m in the eigenvalue table
    double kappa[3][3];          // Kronecker coefficients kappa_{c,m} per component
    double scale;                // (H^(k))^{d-2} for P_A, 1 for the interior solve
    double mass;                 // 1 for P_A (mass term), 0 for the interior solve
    double alpha;                // output = alpha * solution
    int prob;                    // problem index (for the stop mask)
    int pad;
};

struct Chunk {                   // contiguous range inside one segment
    int64_t begin, end;
    int seg;                     // patch or problem index
    int pad;
};

// MINRES scalars of one problem (preconditioned Lanczos + Givens).
struct MinresState {
    double gamma, gamma_old, gamma1, eta;
    double c, c_old, s, s_old;
    double delta;
    double cv_q, cv_v, cv_vold;  // v_new = cv_q q + cv_v v + cv_vold v_old
    double cd_z, cd_dold, cd_d;  // d_new = cd_z z + cd_dold d_old + cd_d d
    double cx;                   // x += cx d_new
    double rel;                  // |eta| / gamma1
    double tol;
    int its, maxit;
    int stop;                    // 1 converged, 2 breakdown, 3 maxit
    int upd;                     // 1 while the d/x update of this iteration is pending
    int skip;                    // stop as it was before the preconditioner of this
                                 // iteration forked (written by k_minres_dv on the
                                 // main stream): the masked kernels read this copy,
                                 // never stop, which the Givens step of the side
                                 // branch may write meanwhile
};

}  // namespace afieti
