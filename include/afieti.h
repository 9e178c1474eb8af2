/*
 * afieti.h -- C ABI of the MI355X (gfx950) inexact All-Floating IETI solver
 * for multi-patch isogeometric compressible linear elasticity with Fast
 * Diagonalization local solvers (Bosy, Montardini, Sangalli, Tani,
 * arXiv 2001.09626).
 *
 * Problem statement (paper Sections 2.2 and 3): patches Omega^(k) given by a
 * multilinear map of their corners (the spline map F^(k) with control
 * points at the Greville images), splines of degree p on open knot vectors
 * (uniform with continuity C^reg, or given explicitly), Lame parameters per
 * patch, a body force f (trigonometric modes and/or a callback), a traction
 * g on faces marked AFIETI_FACE_TRACTION (Gamma_N), Dirichlet data u = g_D
 * on faces marked AFIETI_FACE_DIRICHLET (homogeneous, or from a callback),
 * natural conditions elsewhere.  Interfaces (Section 2.2) are the pairs of
 * patch faces whose corners coincide, or the pairs listed explicitly.  With
 * equal knot vectors along the face an interface is conforming (its nodes
 * are matched one to one); with nested knot vectors (one side refines the
 * other) it is non-conforming, and every node of the finer face is glued to
 * the coarse trace written in the fine basis by knot insertion.  A
 * non-conforming interface needs aligned parametrisations of its two faces
 * and finer-face nodes that no third patch shares (AFIETI_EUNSUPPORTED
 * otherwise); unequal degrees, knot vectors along a face that are neither
 * equal nor nested, or a face refined on each side in another direction
 * give AFIETI_EGEOM.
 *
 * Vector layouts (all double precision, device memory, caller owned):
 *   DOF vector   patch-stacked (Section 4): for each problem, for each
 *                patch k, for each component c, the colexicographic nodes
 *                (first parametric index fastest).  Problems are stacked in
 *                the order given to afieti_setup.  Length info.n_dof.
 *   multipliers  one entry per row of the jump matrix B, problems stacked.
 *                Length info.n_c.
 *
 * Rows of B ("star" pattern to the lowest patch index): for each problem,
 * component c, geometric node (ordered by lowest patch, then its local
 * index) with copies k_1 < ... < k_r: a node on the Dirichlet boundary has
 * the r rows e_{k_j}; any other node the r-1 rows e_{k_1} - e_{k_j}.  Then,
 * per component, for each non-conforming interface and each node i of its
 * finer face, the row e_{f,i} - sum_j T_ij e_{c,j} (T the face's
 * knot-insertion matrix, j over the coarse face's nodes); the finer face's
 * nodes take no other row.
 *
 * Streams: every `stream` argument is a hipStream_t (NULL = default
 * stream).  Work is enqueued on it; calls that report a scalar result to
 * the host (afieti_solve, afieti_solve_adjoint) synchronise it.
 *
 * Errors: every int-returning call returns AFIETI_OK (0) on success, a
 * positive AFIETI_NOT_CONVERGED when MINRES stopped at maxit (outputs hold
 * the last iterate), or a negative code; afieti_last_error() gives text.
 * A handle is not thread safe; distinct handles are independent.
 */
#ifndef AFIETI_H
#define AFIETI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AFIETI_OK 0
#define AFIETI_NOT_CONVERGED 1
#define AFIETI_EINVAL (-1)       /* bad sizes, degree, NULL pointer, NaN     */
#define AFIETI_EGEOM (-2)        /* det J <= 0 or faces that do not match    */
#define AFIETI_ESINGULAR (-3)    /* G^T G or B B^T not positive definite     */
#define AFIETI_EBREAKDOWN (-4)   /* MINRES gamma^2 < 0: preconditioner not SPD */
#define AFIETI_ENOMEM (-5)
#define AFIETI_EHIP (-6)         /* a HIP runtime call failed                */
#define AFIETI_EUNSUPPORTED (-7)   /* valid input the library does not build:
                                    rotated non-conforming interfaces, FD
                                    tiles beyond the device limit, ...       */

#define AFIETI_FACE_FREE 0       /* natural condition or interface (auto)    */
#define AFIETI_FACE_DIRICHLET 1  /* Dirichlet u = g_D (g_D = 0 without the
                                    problem's dirichlet callback)            */
#define AFIETI_FACE_TRACTION 2   /* boundary face with the problem's traction
                                    callback (Gamma_N); not an interface      */

/* precision of the FD mode products (Section 5.2.1, Algorithm 1); the
 * Krylov vectors, residuals and projections are always FP64.  FP64, FP32
 * and BF16 run on the matrix cores (FP32 accumulation for BF16);
 * FP64_VALU and FP32_VALU are the vector-ALU paths. */
#define AFIETI_FD_FP64 0
#define AFIETI_FD_FP32 1
#define AFIETI_FD_BF16 2
#define AFIETI_FD_FP32_VALU 3
#define AFIETI_FD_FP64_VALU 4

/* choice of P_S: non-redundant inexact (Remark 1, default) or plain
 * inexact (Section 5.2, eq. inexact_SP) */
#define AFIETI_PS_NR 0
#define AFIETI_PS_PLAIN 1

/* the inexact local solvers: FD of the parametric operators (Section 5.2,
 * eq. inexact_AP / inexact_SP with Algorithm 1, default), or with geometry
 * inclusion (Section 5.2.3, eq. geo_A / geo_S / tildeshur): per patch and
 * displacement component a separable fit of the diagonal of the
 * pulled-back coefficient matrix (a least-squares fit in log space over the
 * Gauss points, weighted by the product Gauss weights, of the diagonal
 * entries together with |det J| as the product of the mass factors),
 * weighted univariate pencils (d^2 per patch), and the diagonal scalings
 * D_A, D_S.  With it P_A carries H^-2 on the mass and P_S no H factor. */
#define AFIETI_PRECOND_FD 0
#define AFIETI_PRECOND_GEO 1

/* how the patch stiffness A^(k) is applied: AUTO = matrix-free where
 * possible (3D, C^{p-1}, p <= 6; sum-factorised Gauss quadrature of the
 * bilinear form of Section 3), assembled stencil elsewhere; ASSEMBLED =
 * always the assembled FP64 stencil; MATRIX_FREE = always matrix-free
 * (EUNSUPPORTED where not possible).  Both apply the same quadrature. */
#define AFIETI_STIFFNESS_AUTO 0
#define AFIETI_STIFFNESS_ASSEMBLED 1
#define AFIETI_STIFFNESS_MATRIX_FREE 2

/* One patch (Section 2.2).  Corner index a1 + 2 a2 + 4 a3 (a_l in {0,1}),
 * coordinates corners[3*index + x] (2D: only the first 4 corners and x < 2
 * are read).  face_bc order: (dir1 min, dir1 max, dir2 min, dir2 max, dir3
 * min, dir3 max).  Knot vectors (Section 2.1): with knots[l] == NULL,
 * direction l has the uniform open vector of n_el[l] elements and interior
 * multiplicity p - reg; otherwise knots[l] (host, n_knots[l] entries, read
 * during afieti_setup) is an open vector on [0, 1]: p + 1 zeros, p + 1
 * ones, non-decreasing, interior knots of multiplicity at most p (so the
 * splines are continuous); n_el[l] and reg are then ignored for l. */
typedef struct {
    int p;             /* degree, 1..8                                     */
    int reg;           /* continuity C^reg, 0 <= reg < p (uniform knots)   */
    int n_el[3];       /* elements per parametric direction (>= 1)         */
    double corners[24];
    double lambda, mu; /* Lame parameters (> 0)                            */
    int face_bc[6];    /* AFIETI_FACE_*                                    */
    const double* knots[3];  /* explicit open knot vectors, or NULL         */
    int n_knots[3];
    const double* ctrl;      /* explicit control net (host, read during
                                afieti_setup), or NULL for the multilinear
                                map of the corners: ctrl[3*node + x],
                                node = i1 + n1 (i2 + n2 i3) colexicographic
                                over the n1 x n2 (x n3) B-splines (z read
                                as 0 in 2D); the geometry is then the spline
                                map sum_i ctrl_i B_i (Section 2.2), corners
                                is ignored (the corner control points take
                                its place), and the stiffness is assembled  */
} afieti_patch;

/* body force f_comp(x) += amp * prod_d sin(pi k[d] x_d + phase[d]) */
typedef struct {
    int comp;
    double amp;
    int k[3];
    double phase[3];
} afieti_load_mode;

/* Host callbacks of a problem, each called during afieti_setup with n
 * points at a time (x: [n][dim] physical coordinates, row major), filling
 * [n][dim] outputs; they may be NULL.
 *   body_force  f(x): added to the load modes, integrated by the Gauss rule
 *               of the stiffness (p+1 points per element and direction).
 *   traction    g(x, normal): on the faces marked AFIETI_FACE_TRACTION,
 *               normal the outward unit normal, integrated by the face
 *               Gauss rule (Section 3, the boundary term of the load).
 *   dirichlet   g_D(x): at the control point of every basis function on a
 *               face marked AFIETI_FACE_DIRICHLET; the constraint rows of
 *               those functions read B u = g_D(control point): the
 *               data's values at the control points serve as its spline
 *               coefficients (exact for linear data, second order in h
 *               otherwise). */
typedef void (*afieti_field_fn)(int64_t n, const double* x, double* out, void* ctx);
typedef void (*afieti_traction_fn)(int64_t n, const double* x, const double* normal, double* out, void* ctx);

typedef struct {
    int dim;                          /* 2 or 3                          */
    int n_patches;
    const afieti_patch* patches;
    int n_load_modes;
    const afieti_load_mode* load_modes;
    afieti_field_fn body_force;       /* may be NULL                     */
    afieti_traction_fn traction;      /* may be NULL                     */
    afieti_field_fn dirichlet;        /* may be NULL (homogeneous)       */
    void* ctx;                        /* passed to the callbacks         */
    /* Interfaces: n_interfaces = 0 glues every pair of faces whose corners
     * coincide.  Otherwise only the listed pairs are glued (coinciding
     * faces not listed stay apart: a crack), interfaces[5 i .. 5 i + 4] =
     * (patch_a, face_a, patch_b, face_b, orient), host memory read during
     * afieti_setup; faces numbered as face_bc.  orient = -1 takes the
     * orientation from the corners; otherwise it must equal
     * swap + 2 flip_0 + 4 flip_1, where t_0 < t_1 are the parametric
     * directions along face_a and u_0 < u_1 those along face_b: swap = 1
     * when t_0 runs along u_1, flip_j = 1 when t_j runs against the
     * direction it lies along (in 2D orient is 0 or 2).  Errors:
     * AFIETI_EINVAL for indices out of range, a patch paired with itself
     * or a face listed twice; AFIETI_EGEOM for listed faces whose corners
     * (or, with explicit control nets, face nets) do not coincide, knot
     * vectors that differ along the face, an orient that the corners
     * contradict, or a traction face. */
    int n_interfaces;
    const int* interfaces;
} afieti_problem;

typedef struct {
    double tol;          /* MINRES: stop when |eta| <= tol * gamma_1 (1e-8) */
    int maxit;           /* default 5000                                   */
    int fd_precision;    /* AFIETI_FD_*                                    */
    int ps_variant;      /* AFIETI_PS_*                                    */
    int check_every;     /* iterations between host convergence checks (8) */
    int host_only;       /* 1: build the host plan only, no device work    */
    int use_graph;       /* 1: replay MINRES iterations as a captured HIP
                            graph (6 iterations per launch) on a stream the
                            handle owns; the graph exists in two schedules
                            (pipelined, classic) with identical results,
                            the first solve of a handle times both (with a
                            host synchronisation per launch while it does)
                            and later solves use the faster;
                            0: enqueue kernels one by one                  */
    int stiffness;       /* AFIETI_STIFFNESS_*                             */
    int fd_tune;         /* launch shape of the matrix-core FD kernels
                            (FP64, FP32, BF16): -1 = autotune at setup
                            (every shape timed on the handle's tensors, the
                            choice kept per tensor shapes for the process),
                            0..3 = fixed: layout (0 the d components of a
                            patch together, 1 one per workgroup) * 2 +
                            (0: 64, 1: 128 columns per block of the mode-3
                            pass).  All shapes give bitwise identical
                            results.                                       */
    double ps_weight;    /* weight w of the multiplier block of the
                            preconditioner, [P_u P_A^-1 P_u ; w P_chi P_S
                            P_chi] (1).  Any w > 0 keeps it positive
                            definite (w = 1 is the method as stated);
                            w <= 0 makes it indefinite, and MINRES stops
                            with AFIETI_EBREAKDOWN at the first iteration
                            whose <z, v> is negative.                      */
    int precond;         /* AFIETI_PRECOND_* (FD)                          */
    /* device memory of the handle (NULL: hipMalloc / hipFree): dev_alloc
     * (bytes, ctx) returns memory on the device current at afieti_setup,
     * or NULL on failure (the call then fails with AFIETI_ENOMEM); every
     * block is returned through dev_free(ptr, bytes, ctx) by
     * afieti_destroy, after the device has finished all work (e.g. a
     * framework's caching allocator).  Blocks stay in use until then; a
     * solve_adjoint with load vectors may allocate more.                   */
    void* (*dev_alloc)(size_t bytes, void* ctx);
    void (*dev_free)(void* ptr, size_t bytes, void* ctx);
    void* alloc_ctx;
} afieti_options;

typedef struct {
    int64_t n_dof, n_c;       /* totals over all problems                  */
    int n_problems, n_patches_total;
    int64_t stiffness_bytes;  /* device memory of the assembled stencils   */
    int64_t device_bytes;     /* all device memory held by the handle      */
} afieti_info;

typedef struct {
    int iterations;           /* max over problems                         */
    int converged;            /* 1 if every problem converged              */
    double rel_residual;      /* max over problems of |eta| / gamma_1      */
    double ms_solve;          /* wall time of the solve on the stream      */
} afieti_stats;

typedef struct afieti_handle afieti_handle;

/* Options with the defaults listed above. */
void afieti_default_options(afieti_options* opt);

/*
 * Set up n_problems independent problems (Sections 2.2, 4, 5.2.1): knots,
 * Gauss rules, univariate K and M and their generalised eigendecompositions
 * (Algorithm 1, step 1), node matching, B, rigid modes R, G = B R and the
 * Cholesky factor of G^T G, then (unless host_only) device assembly of the
 * patch stiffness stencils and load vectors.  Inputs are host memory, read
 * during the call only.  On success *out owns all device memory.
 */
int afieti_setup(const afieti_problem* probs, int n_problems,
                 const afieti_options* opt, void* stream, afieti_handle** out);

int afieti_get_info(const afieti_handle* h, afieti_info* info);

/* Per-problem results of the last solve (host arrays of n_problems entries,
 * each may be NULL): MINRES iterations, |eta| / gamma_1, and status
 * (1 converged, 2 breakdown, 3 maxit reached). */
int afieti_get_problem_stats(const afieti_handle* h, int* iterations, double* rel_residual, int* status);

/* Per problem: n_dof, n_c and the DOF offset of every patch; arrays sized by
 * the caller (dof_off: n_patches_total + 1 entries, c_off: n_problems + 1). */
int afieti_get_offsets(const afieti_handle* h, int64_t* dof_off, int64_t* c_off);

/*
 * z = (P_A^inex)^{-1} r for all problems, patches and components
 * (Section 5.2, eq. inexact_AP; applied by Algorithm 1): per patch k and
 * component l, (H^(k))^{d-2} (A-hat_l + M-hat_l) z = r.  With
 * AFIETI_PRECOND_GEO it is P~_A (Section 5.2.3, eq. geo_A):
 * D_A^{1/2} (A~_l + (H^(k))^-2 M~_l) D_A^{1/2} z = r.  r, z: device DOF
 * vectors (may not alias).  Precision of the mode products as configured.
 */
int afieti_apply_fd(afieti_handle* h, const double* r, double* z, void* stream);

/*
 * The same z = (P_A^inex)^{-1} r as afieti_apply_fd (same kernels, bitwise
 * equal results), for callers that cannot allocate during the call: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  The FD intermediate tensor lives in a fixed device array of
 * AFIETI_NOALLOC_SCRATCH_BYTES (8 MiB) per GPU, held until the process ends,
 * instead of handle memory; the call allocates nothing (no hipMalloc, no
 * hipFree, no allocating library routine).  The handle's device must be
 * current.  Returns AFIETI_EUNSUPPORTED when the handle's intermediate
 * (one FP64 entry per DOF for the FP64 precisions, one FP32 entry for the
 * others) exceeds the array.  Every call on one GPU shares the array: calls
 * that overlap in time on one GPU (other streams, threads or handles) race
 * on it.  Nothing of a previous call's contents is read.
 */
#define AFIETI_NOALLOC_SCRATCH_BYTES (8 << 20)
int afieti_apply_fd_noalloc(afieti_handle* h, const double* r, double* z, void* stream);

/*
 * AF-IETI solve (Section 4): MINRES on the preconditioned projected saddle
 * system, then u = (I - R (G^T G)^{-1} G^T B) w and lambda = lambda_0 + chi.
 * With Dirichlet data (B u = c, c the g_D values of the Dirichlet rows) the
 * solve runs on u_0 = u - u_D, u_D = B^T (B B^T)^{-1} c, with right-hand
 * side rhs - A u_D and homogeneous constraints, and returns u_0 + u_D.
 * rhs: device DOF vector, or NULL for the assembled load (modes, body
 * force, tractions).  u: device DOF vector (out); lambda: device multiplier
 * vector or NULL.  st may be NULL.
 */
int afieti_solve(afieti_handle* h, const double* rhs, double* u, double* lambda,
                 afieti_stats* st, void* stream);

/*
 * Adjoint gradients of a scalar J(u) (follows from the symmetric saddle
 * system of Section 4): psi solves the same system with right-hand side
 * dJdu (device DOF vector) and homogeneous constraints (the Dirichlet data
 * do not depend on the parameters); u is the forward solution (device DOF
 * vector).  psi (out, device, may be NULL); dJ_dlame (out, host, 2 per
 * patch in problem-stacked patch order: dJ/dlambda_k, dJ/dmu_k);
 * dJ_damp (out, host, one per load mode of each problem, stacked);
 * load_vectors (device, n_load_vectors x n_dof, row major, may be NULL):
 * loads F_j of the caller, with dJ_dload[j] = psi^T F_j (host, out) the
 * derivative of J with respect to the coefficient c_j of a load sum_j c_j F_j.
 */
int afieti_solve_adjoint(afieti_handle* h, const double* dJdu, const double* u,
                         double* psi, double* dJ_dlame, double* dJ_damp,
                         int n_load_vectors, const double* load_vectors, double* dJ_dload,
                         afieti_stats* st, void* stream);

/*
 * Change the per-patch Lame parameters and/or the load amplitudes of an
 * existing handle (both optional, host arrays): lame = [lambda_k, mu_k] per
 * patch in problem-stacked order; amps = one amplitude per load mode of each
 * problem, stacked.  New Lame values re-assemble the stiffness stencils and
 * update the FD eigenvalue scaling (the eigenvectors depend on the knots
 * only, Section 5.2.1); new amplitudes recombine the stored unit-mode loads.
 */
int afieti_set_parameters(afieti_handle* h, const double* lame, const double* amps, void* stream);

/* Individual operators of the hot path, for checking and measurement.
 * x and y are device vectors of the sizes listed; they may not alias. */
#define AFIETI_OP_STIFFNESS 0   /* y = A x              (DOF -> DOF) eq. block_A     */
#define AFIETI_OP_B 1           /* y = B x              (DOF -> mult) Section 4      */
#define AFIETI_OP_BT 2          /* y = B^T x            (mult -> DOF)                */
#define AFIETI_OP_P_U 3         /* y = P_u x            (DOF -> DOF) eq. all_precond.*/
#define AFIETI_OP_P_CHI 4       /* y = P_chi x          (mult -> mult) eq. proj_chi  */
#define AFIETI_OP_SHAT 5        /* y = blockdiag_k H^{d-2} S-hat^(k) x on Gamma
                                   (DOF -> DOF, interior of x ignored, of y zero)     */
#define AFIETI_OP_PS 6          /* y = P_S x            (mult -> mult) Remark 1      */
#define AFIETI_OP_PREC 7        /* y = B^{-1} x, block preconditioner (DOF+mult)     */
#define AFIETI_OP_SADDLE 8      /* y = projected saddle operator (DOF+mult)          */
#define AFIETI_OP_FD_INTERIOR 9 /* y_I = ((A-hat_l)_II)^{-1} x_I per patch/component,
                                   boundary of y zero (DOF -> DOF) eq. fac_schur      */
#define AFIETI_OP_AHAT 10       /* y = A-hat x per patch/component (DOF -> DOF)      */
#define AFIETI_OP_MASS 11       /* y = M x, physical mass (DOF -> DOF) eq. le_local_MS */
#define AFIETI_OP_LOAD 12       /* y = assembled load: modes, body force, tractions
                                   (x ignored, DOF)                                  */
#define AFIETI_OP_DIRICHLET_LIFT 13 /* y = u_D = B^T (B B^T)^{-1} c, the Dirichlet
                                   data as a DOF vector (x ignored)                  */
int afieti_apply(afieti_handle* h, int op, const double* x, double* y, void* stream);

/* Host copies of setup data, for checking (valid also with host_only):
 *  what = 0: B as triples, buf = [row, dof_plus, dof_minus] x n_c int64:
 *            dof_minus -1 for a Dirichlet row (entry +1 on dof_plus), -2 - g
 *            for the gluing row g of a non-conforming interface (entries
 *            listed by what = 9)
 *  what = 1: eigenvalues D of every patch and direction, concatenated (double)
 *  what = 2: diameters H^(k) (double, one per patch)
 *  what = 3: G^T G of problem 0, row major (double)
 *  what = 4: the load terms assembled on the host, body force and
 *            tractions of every problem, DOF-ordered (double, n_dof)
 *  what = 5: c, the right-hand side of B u = c: Dirichlet data on the
 *            Dirichlet rows, zero elsewhere (double, n_c)
 *  what = 6: eigenvectors U of every patch and direction, in the order of
 *            what = 1, each n x n row major (column j: eigenvalue j)
 *  what = 7: with AFIETI_PRECOND_GEO: D_A^{-1/2} per DOF (n_dof), then
 *            D_S^{1/2} per DOF (n_dof), DOF-ordered
 *  what = 8: with AFIETI_PRECOND_GEO: eigenvalues of the weighted pencils
 *            per patch, component and direction, concatenated
 *  what = 9: the weighted entries of the gluing rows of non-conforming
 *            interfaces (Section 2.2): [row, dof, value] per entry (double),
 *            in row order; the row has +1 on its dof_plus and these
 *            values (minus the coarse trace's knot-insertion weights)     */
int afieti_export(const afieti_handle* h, int what, void* buf, int64_t buf_bytes);
int64_t afieti_export_size(const afieti_handle* h, int what);

void afieti_destroy(afieti_handle* h);
const char* afieti_strerror(int code);
const char* afieti_last_error(const afieti_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* AFIETI_H */
