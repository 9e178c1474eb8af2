// Launch wrappers of the HIP kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace afieti {

// ---- Fast Diagonalization (Algorithm 1) on the vector ALU: three passes
// over the tensors.  Kernels of problems whose MINRES has stopped
// (mask[prob].skip != 0) return at once; mask may be NULL.  prec 0: FP64;
// 1: FP32.  d_cols: 32-column blocks of the mode-3 pass.  scale (may be
// NULL): a per-DOF factor applied to the input as it is read and to the
// output as it is written, out = s .* FD(s .* in) (the diagonal scaling of
// geometry inclusion).
void launch_fd(int prec, const FdTensor* d_tensors, int n_tensors,
               const int2* d_slabs, int n_slabs, const int2* d_cols, int n_colblocks,
               const void* u_table, const double* d_table,
               const double* in, double* out, void* tmp, const MinresState* mask, const double* scale,
               hipStream_t s);

// ---- Fast Diagonalization on the matrix cores (fd.hip): the d component
// tensors of a patch (a group) share U_m and are transformed together (or
// one per group, the per-component layout).  Device lists: slabs (group,
// i3), column blocks (group, block) of 64 and of 128 columns.
struct FdGroupSet {
    const FdGroup* groups = nullptr;
    const int2* slabs = nullptr;
    const int2* cols64 = nullptr;
    const int2* cols128 = nullptr;
    int n_groups = 0, n_slabs = 0, n_cols64 = 0, n_cols128 = 0;
    int max_n1 = 1, max_n2 = 1, max_n3 = 1, max_nc = 1;
};
// launch shapes the autotuner picks from (bitwise identical results): per
// layout, variant 0 or 1 = 64 or 128 columns per mode-3 block
constexpr int kFdVariants = 2;
int fd_variant_ncb(int variant);
// compile-time depth extent (28, 36 or 48) the kernels use for a set
int fd_depth_extent(const FdGroupSet& set);
// LDS bytes of the larger pass of a set for a variant
int64_t fd_lds_bytes(int mode, int variant, const FdGroupSet& set);
// mode 0: FP32 operands, 1: BF16 operands (FP32 accumulation), 2: FP64.
// tmp holds one FP32 (FP64 for mode 2) entry per tensor element.
// scale as for launch_fd.
void launch_fd_groups(int mode, int variant, const FdGroupSet& set, const void* ut, const double* dt,
                      const double* in, double* out, void* tmp, const MinresState* mask, const double* scale,
                      hipStream_t s);

// ---- fixed scratch for callers that cannot allocate
// Bytes of the file-scope device array that afieti_apply_fd_noalloc uses for
// the FD intermediate tensor (one copy per GPU, held until the process ends).
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
// Resolve the array's device address on the current device (once per
// device; later calls return the stored address).  Returns nullptr and sets
// *err when the runtime call fails.
void* noalloc_scratch_acquire(hipError_t* err);
// The address resolved for `device` by an earlier acquire, or nullptr.
void* noalloc_scratch_ptr(int device);

// ---- setup kernels
void launch_geometry(const DevPatch* dp, int k, const DevPatch& hp, const double* ctrl,
                     const double* qval, const double* qder, const int* qfirst, const double* qw,
                     double* geo, hipStream_t s);
void launch_assemble(const DevPatch* dp, int k, const DevPatch& hp, const double* geo,
                     const double* qval, const double* qder, const int* qfirst,
                     const int* el_first, const int* el_last, double* stencil,
                     double lam_w, double mu_w, hipStream_t s);
// f[dof - f_base] = body-force load of patch k for the given modes
void launch_load(const DevPatch* dp, int k, const DevPatch& hp, const double* geo,
                 const double* qval, const int* qfirst, const int* el_first, const int* el_last,
                 const double* modes, int n_modes, double* f, int64_t f_base, hipStream_t s);
// y = M x on patch k (physical mass, both passes); qbuf holds dim values per Gauss point
void launch_mass(const DevPatch* dp, int k, const DevPatch& hp, const double* geo, const double* qval,
                 const int* qfirst, const int* el_first, const int* el_last, const double* x, double* qbuf,
                 double* y, hipStream_t s);
// per-block partial (e_mu, e_lam) of patch k; returns the number of blocks
int launch_energy(const DevPatch* dp, int k, const DevPatch& hp, const double* geo, const double* qval,
                  const double* qder, const int* qfirst, const double* u, const double* psi, double* part,
                  hipStream_t s);
// part[mode][chunk] partial dot products of F[mode] (length n) with psi[off:]; returns chunks
int launch_mdot(const double* F, int64_t n, int n_modes, int64_t off, const double* psi, double* part,
                hipStream_t s);

// ---- operators
// y = A x (+ B^T t if t != nullptr) for every row of every patch
void launch_stiffness_dp(int dim, int p, const DevPatch* dp, const int4* d_rowblocks, int n_rowblocks,
                         const double* stencil, const double* x, double* y,
                         const int64_t* bt_ptr, const int* bt_row, const double* bt_sign,
                         const double* t, const MinresState* mask, hipStream_t s);
// zero the interior nodes of every patch and component
void launch_mask_interior(const DevPatch* dp, const int4* d_rowblocks, int n_rowblocks, double* y, hipStream_t s);
// Matrix-free y = A x (+ B^T t) for the 3D C^{p-1} patches of degree p, in
// two launches: launch_mf_bricks does the sum-factorised quadrature of every
// brick (bricks: (patch, b1, b2, b3) in patch order) into ybuf,
// launch_mf_gather sums the brick contributions per node over the row
// blocks rb and adds B^T t.  tab: the per-brick univariate tables
// (mf_table_doubles(p) doubles per direction and brick, from
// DevPatch::tab_off[d]): V[q][t], D[q][t], W[q], E[q].
void launch_mf_bricks(int p, const DevPatch* dp, const int4* bricks, int n_bricks, const double* tab,
                      const double* x, double* ybuf, const MinresState* mask, hipStream_t s);
void launch_mf_gather(int p, const DevPatch* dp, const int4* rb, int nrb, const double* ybuf, double* y,
                      const int64_t* bt_ptr, const int* bt_row, const double* bt_sign, const double* t,
                      const MinresState* mask, hipStream_t s);
// elements per brick direction of the matrix-free kernel for degree p
int mf_brick_elems(int p);
// doubles per (direction, brick) table of the matrix-free kernel for degree p
int mf_table_doubles(int p);
// Rows of B that glue a non-conforming interface: a row r with
// minus[r] <= -2 reads x[plus] - sum_e val[e] x[col[e]] over e in
// [ptr[g], ptr[g + 1]), g = -2 - minus[r] (empty when there are none).
struct GlueRows {
    const int64_t* ptr = nullptr;
    const int64_t* col = nullptr;
    const double* val = nullptr;
};
// Dense blocks of B B^T (rows whose block kind is 2): block b holds the rows
// rows[ptr[b] .. ptr[b + 1]) and its inverse at mat + moff[b], row major;
// blk[j] is the block of the j-th listed
// row, total the number of listed rows and tmp (total doubles) the row
// values between the two kernels of an application.
struct DenseBlocks {
    int n = 0, total = 0;
    const int64_t* ptr = nullptr;
    const int* rows = nullptr;
    const int* blk = nullptr;
    const int64_t* moff = nullptr;
    const double* mat = nullptr;
    double* tmp = nullptr;
};
// y[r] = alpha (x[plus] - x[minus]) (Dirichlet rows: alpha x[plus]; gluing
// rows as GlueRows); with in_scale (may be NULL) x is read as in_scale .* x
void launch_B(const int64_t* plus, const int64_t* minus, const GlueRows& glue, int64_t n_c, double alpha,
              const double* x, double* y, hipStream_t s, const double* in_scale = nullptr);
// y[i] = sum sign * x[row] for every DOF; with out_scale (may be NULL)
// y[i] = out_scale[i] * (that sum)
void launch_Bt(const int64_t* bt_ptr, const int* bt_row, const double* bt_sign, int64_t n_dof,
               const double* x, double* y, hipStream_t s, const double* out_scale = nullptr);
// z = (B B^T)^{-1} y (node blocks, and the dense blocks of the
// non-conforming interfaces)
void launch_W(const int* blk_start, const int* blk_size, const int* blk_dir, const DenseBlocks& dense, int64_t n_c,
              const double* y, double* z, hipStream_t s);
// y = scale_k * A-hat x per patch and component for the patches of degree p
// (banded Kronecker form, sum-factorised, one workgroup per slab).  slabs:
// (patch, component, i3); max_n12: largest n1 n2 of those patches (LDS size);
// bnd_in != 0 promises that x is zero away from the patch boundary;
// bnd_out != 0 asks only for the patch-boundary entries of y (the others are
// left as they were).
void launch_ahat(int p, const DevPatch* dp, const int4* slabs, int n_slabs, int max_n12, int max_n1n2,
                 const double* kb,
                 const double* mb, const double* x, double* y, int use_h, int bnd_in, int bnd_out,
                 const MinresState* mask, hipStream_t s);
// z = (B B^T)^{-1} (B x), and z = (B B^T)^{-1} (y - G zc), with the B and the
// G rows computed inside the block solve
void launch_BW(const int* blk_start, const int* blk_size, const int* blk_dir, const DenseBlocks& dense, int64_t n_c,
               const int64_t* plus, const int64_t* minus, const GlueRows& glue, const double* x, double* z,
               hipStream_t s, const double* in_scale = nullptr);
void launch_GW(const int* blk_start, const int* blk_size, const int* blk_dir, const DenseBlocks& dense, int64_t n_c,
               const int* patch_plus, const int* patch_minus, const double* g_plus, const double* g_minus,
               const double* zc, const double* y, double* z, hipStream_t s);
// partial sums of R^T x over patch DOF chunks (nm values per chunk)
void launch_rigid_partial(const DevPatch* dp, const Chunk* chunks, int n_chunks,
                          const double* ctrl, const double* x, double* partials, hipStream_t s);
// partial sums of G^T y = R^T (B^T y) over chunks of the per-patch lists of
// multiplier copies (row, signed rigid-mode values [mode][copy], n_mc copies)
void launch_gamma_partial(const Chunk* chunks, int n_chunks, const int* mc_row, const double* mc_val,
                          int64_t n_mc, const double* y, double* partials, hipStream_t s);
// per problem: g = sum partials; zc = Cinv g (coefficients per patch)
void launch_coarse_finalize(const int* prob_patch0, const int* prob_npatch, const int* prob_nmodes,
                            const int64_t* prob_cinv_off, int n_probs, const int* patch_chunk_ptr,
                            const double* partials, const double* Cinv, double* zc, int max_nc,
                            hipStream_t s);
// coef[k] = RtR_inv[k] * sum(partials of patch k)
void launch_rigid_finalize(const int* patch_chunk_ptr, int n_patches, const double* partials,
                           const double* RtR_inv, double* coef, hipStream_t s);
// y = x - R coef (all DOFs)
void launch_rigid_update(const DevPatch* dp, const Chunk* chunks, int n_chunks, const double* ctrl,
                         const double* coef, const double* x, double* y, hipStream_t s);
// y[r] = beta x[r] + alpha (G zc)[r]
void launch_G_apply(const int* patch_plus, const int* patch_minus, const double* g_plus,
                    const double* g_minus, int64_t n_c, const double* zc, double alpha,
                    double beta, const double* x, double* y, hipStream_t s);

// ---- vector kernels
void launch_copy(const double* x, double* y, int64_t n, hipStream_t s);
// y = a .* x (elementwise; y may be x)
void launch_mul(const double* a, const double* x, double* y, int64_t n, hipStream_t s);
void launch_fill(double* y, double v, int64_t n, hipStream_t s);
void launch_axpby(double a, const double* x, double b, const double* y, double* z, int64_t n, hipStream_t s);
// per-chunk partial dot products <x, y>
void launch_dot_partial(const Chunk* chunks, int n_chunks, const double* x, const double* y,
                        double* partials, hipStream_t s);
// MINRES scalar steps (one thread per problem)
void launch_minres_givens(MinresState* st, const int* prob_chunk_ptr, int n_probs,
                          const double* partials, hipStream_t s);
void launch_minres_init(MinresState* st, const int* prob_chunk_ptr, int n_probs,
                        const double* partials, double tol, int maxit, hipStream_t s);
// delta_j from the chunk partials of <A z_j, z_j> (cptr: per-problem chunk
// ranges), then v_new = cv_q q + cv_v v + cv_vold v_old, in one launch
// (skipped for stopped problems)
void launch_minres_dv(MinresState* st, const Chunk* chunks, int n_chunks, const int* cptr, const double* part,
                      const double* q, const double* v, const double* v_old, double* v_new, hipStream_t s);
// d_new = cd_z z + cd_dold d_old + cd_d d; x += cx d_new   (only when upd)
void launch_minres_dx(const MinresState* st, const Chunk* chunks, int n_chunks, const double* z,
                      const double* d_old, const double* d, double* d_new, double* x, hipStream_t s);

}  // namespace afieti
