// HIP kernels of the inexact AF-IETI hot path for gfx950 (wave64).
//
//  * FD (Algorithm 1 of Section 5.2.1) on the vector ALU (FP64, FP32): mode
//    products with the univariate generalised eigenvectors in three passes
//    (modes 1+2 per slab, mode 3 with the eigenvalue divide fused, modes 2+1
//    per slab), tiles in LDS; the matrix-core variants are in fd.hip.
//  * stiffness stencil assembly (Gauss quadrature of the bilinear form of
//    Section 3) and the matrix-vector product with the assembled stencil,
//    with B^T t fused into its epilogue (first block row of the projected
//    saddle operator, Section 4).
//  * jump operator B, B^T, the node-block inverse of B B^T (Remark 1),
//    banded Kronecker application of A-hat (Section 5.2), rigid-mode
//    reductions and updates for P_u, P_chi, lambda_0 and the recovery.
//  * deterministic two-stage reductions and the MINRES vector updates.
//
// Every reduction sums in a fixed order (thread strides, then a fixed
// shuffle tree, then chunks in index order): repeated runs are bitwise
// identical.  No atomics.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "device.h"
#include "kernels.h"
#include "rigid.h"

namespace afieti {

namespace {

constexpr int kQStride = 9;  // row stride of the univariate quadrature tables (p <= 8)

inline unsigned blocks_for(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

// Stencil storage: row (c, i) couples to (c', i + o_s) for the S offsets
// o_s in [-p, p]^d (s colexicographic, o1 fastest); values are stored as
// one array over the nodes per (c, c', s):
//   index = ((c d + c') S + s) nodes + node,
// so a wave streams 64 consecutive values of one (c, c', s) per load.

// ------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum NV values over a block of kBlock threads; result valid in thread 0.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* lds /* NV * 4 */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        double s = wave_sum(v[m]);
        if (lane == 0) lds[m * 4 + wave] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int m = 0; m < NV; ++m) v[m] = ((lds[m * 4 + 0] + lds[m * 4 + 1]) + lds[m * 4 + 2]) + lds[m * 4 + 3];
    }
}

// dst[e] = load(e) for e < n (n <= IT kBlock): every global load of a thread
// is issued before its LDS stores, so their latencies overlap
template <int IT, int BS = kBlock, typename T, typename F>
__device__ inline void batched_copy(T* dst, int n, F load) {
    T v[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int e = threadIdx.x + it * BS;
        v[it] = e < n ? load(e) : (T)0;
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int e = threadIdx.x + it * BS;
        if (e < n) dst[e] = v[it];
    }
}


// =============================================================== FD kernels
// threads of the FD kernels (vector ALU and matrix cores): eight wavefronts
// per slab or column block; four workgroups of the matrix-core kernels, two
// of the FP64 vector-ALU kernels fit in the LDS of a CU
constexpr int kFdBlock = 512;
constexpr int kFdSlabIt = (kMaxN * kMaxN + kFdBlock - 1) / kFdBlock;  // loads per thread of an n x n slab

// Pass 1: per (tensor, slab i3): Y[a2][a1] = sum_{i2,i1} U2[i2][a2] X[i2][i1] U1[i1][a1]
template <typename T>
__global__ void __launch_bounds__(kFdBlock) k_fd_fwd12(const FdTensor* __restrict__ tens, const int2* __restrict__ slabs,
                                                     const T* __restrict__ ut, const double* __restrict__ in,
                                                     T* __restrict__ tmp, const MinresState* __restrict__ mask,
                                                     const double* __restrict__ scale) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 it = slabs[blockIdx.x];
    const FdTensor t = tens[it.x];
    if (mask && mask[t.prob].skip) return;
    const int i3 = it.y, n1 = t.n1, n2 = t.n2, n12 = n1 * n2;
    T* X = reinterpret_cast<T*>(smem);
    T* Y = X + kMaxN * kMaxN;
    T* U = Y + kMaxN * kMaxN;
    const double* src = in + t.in_off + (int64_t)i3 * t.s3;
    const double* ssrc = scale ? scale + t.in_off + (int64_t)i3 * t.s3 : nullptr;
    batched_copy<kFdSlabIt, kFdBlock>(X, n12, [&](int e) {
        const int i2 = e / n1, i1 = e - i2 * n1;
        const int64_t o = (int64_t)i2 * t.s2 + i1;
        return (T)(ssrc ? src[o] * ssrc[o] : src[o]);
    });
    batched_copy<kFdSlabIt, kFdBlock>(U, n1 * n1, [&](int e) { return ut[t.u_off[0] + e]; });
    __syncthreads();
    for (int e = threadIdx.x; e < n12; e += kFdBlock) {  // Y[i2][a1]
        int i2 = e / n1, a1 = e - i2 * n1;
        T acc = 0;
        for (int i1 = 0; i1 < n1; ++i1) acc += X[i2 * n1 + i1] * U[i1 * n1 + a1];
        Y[e] = acc;
    }
    __syncthreads();
    batched_copy<kFdSlabIt, kFdBlock>(U, n2 * n2, [&](int e) { return ut[t.u_off[1] + e]; });
    __syncthreads();
    T* dst = tmp + t.tmp_off + (int64_t)i3 * n12;
    for (int e = threadIdx.x; e < n12; e += kFdBlock) {  // Z[a2][a1]
        int a2 = e / n1, a1 = e - a2 * n1;
        T acc = 0;
        for (int i2 = 0; i2 < n2; ++i2) acc += U[i2 * n2 + a2] * Y[i2 * n1 + a1];
        dst[e] = acc;
    }
}

// Pass 2: per (tensor, block of 32 columns (a1,a2)): mode-3 product with U3^T,
// divide by the Kronecker-sum eigenvalues Lambda, mode-3 product with U3.
template <typename T>
__global__ void __launch_bounds__(kFdBlock) k_fd_mid3(const FdTensor* __restrict__ tens, const int2* __restrict__ cols,
                                                    const T* __restrict__ ut, const double* __restrict__ dt,
                                                    T* __restrict__ tmp, const MinresState* __restrict__ mask) {
    constexpr int NC = 32;
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 it = cols[blockIdx.x];
    const FdTensor t = tens[it.x];
    if (mask && mask[t.prob].skip) return;
    const int n1 = t.n1, n3 = t.n3, n12 = t.n1 * t.n2;
    const int col0 = it.y * NC;
    T* Z = reinterpret_cast<T*>(smem);
    T* Zt = Z + kMaxN * NC;
    T* U = Zt + kMaxN * NC;
    T* base = tmp + t.tmp_off;
    batched_copy<(kMaxN * NC + kFdBlock - 1) / kFdBlock, kFdBlock>(Z, n3 * NC, [&](int e) {
        const int i3 = e / NC, col = col0 + e - i3 * NC;
        return col < n12 ? base[(int64_t)i3 * n12 + col] : (T)0;
    });
    batched_copy<kFdSlabIt, kFdBlock>(U, n3 * n3, [&](int e) { return ut[t.u_off[2] + e]; });
    __syncthreads();
    const int c = threadIdx.x % NC, g = threadIdx.x / NC;  // 8 groups over a3
    const int col = col0 + c;
    const int a2 = col / n1, a1 = col - a2 * n1;
    double lam12 = 0;
    if (col < n12) lam12 = t.mass + t.kappa[0] * dt[t.d_off[0] + a1] + t.kappa[1] * dt[t.d_off[1] + a2];
    for (int a3 = g; a3 < n3; a3 += kFdBlock / NC) {
        T acc = 0;
        for (int i3 = 0; i3 < n3; ++i3) acc += U[i3 * n3 + a3] * Z[i3 * NC + c];
        double lam = t.scale * (lam12 + t.kappa[2] * dt[t.d_off[2] + a3]);
        Zt[a3 * NC + c] = (col < n12) ? (T)((double)acc / lam) : (T)0;
    }
    __syncthreads();
    for (int i3 = g; i3 < n3; i3 += kFdBlock / NC) {
        T acc = 0;
        for (int a3 = 0; a3 < n3; ++a3) acc += U[i3 * n3 + a3] * Zt[a3 * NC + c];
        if (col < n12) base[(int64_t)i3 * n12 + col] = acc;
    }
}

// Pass 3: per (tensor, slab i3): X[i2][i1] = alpha sum_{a2,a1} U2[i2][a2] Z[a2][a1] U1[i1][a1]
template <typename T>
__global__ void __launch_bounds__(kFdBlock) k_fd_bwd12(const FdTensor* __restrict__ tens, const int2* __restrict__ slabs,
                                                     const T* __restrict__ ut, const T* __restrict__ tmp,
                                                     double* __restrict__ out, const MinresState* __restrict__ mask,
                                                     const double* __restrict__ scale) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 it = slabs[blockIdx.x];
    const FdTensor t = tens[it.x];
    if (mask && mask[t.prob].skip) return;
    const int i3 = it.y, n1 = t.n1, n2 = t.n2, n12 = n1 * n2;
    T* Z = reinterpret_cast<T*>(smem);
    T* Y = Z + kMaxN * kMaxN;
    T* U = Y + kMaxN * kMaxN;
    const T* src = tmp + t.tmp_off + (int64_t)i3 * n12;
    batched_copy<kFdSlabIt, kFdBlock>(Z, n12, [&](int e) { return src[e]; });
    batched_copy<kFdSlabIt, kFdBlock>(U, n1 * n1, [&](int e) { return ut[t.u_off[0] + e]; });
    __syncthreads();
    for (int e = threadIdx.x; e < n12; e += kFdBlock) {  // Y[a2][i1] = sum_a1 Z[a2][a1] U1[i1][a1]
        int a2 = e / n1, i1 = e - a2 * n1;
        T acc = 0;
        for (int a1 = 0; a1 < n1; ++a1) acc += Z[a2 * n1 + a1] * U[i1 * n1 + a1];
        Y[e] = acc;
    }
    __syncthreads();
    batched_copy<kFdSlabIt, kFdBlock>(U, n2 * n2, [&](int e) { return ut[t.u_off[1] + e]; });
    __syncthreads();
    double* dst = out + t.out_off + (int64_t)i3 * t.s3;
    const double* sdst = scale ? scale + t.out_off + (int64_t)i3 * t.s3 : nullptr;
    for (int e = threadIdx.x; e < n12; e += kFdBlock) {  // X[i2][i1] = sum_a2 U2[i2][a2] Y[a2][i1]
        int i2 = e / n1, i1 = e - i2 * n1;
        T acc = 0;
        for (int a2 = 0; a2 < n2; ++a2) acc += U[i2 * n2 + a2] * Y[a2 * n1 + i1];
        const int64_t o = (int64_t)i2 * t.s2 + i1;
        const double v = t.alpha * (double)acc;
        dst[o] = sdst ? v * sdst[o] : v;
    }
}

// ============================================================ setup kernels
// Geometry at the Gauss points of patch k from the spline map with the
// control net: per point [w |det J|, J^{-1} (3x3, row a = d eta_a / dx),
// x (3)], 13 doubles.
template <int DIM>
__global__ void k_geometry(const DevPatch* __restrict__ dps, int k, const double* __restrict__ ctrl,
                           const double* __restrict__ qval, const double* __restrict__ qder,
                           const int* __restrict__ qfirst, const double* __restrict__ qw,
                           double* __restrict__ geo) {
    const DevPatch pa = dps[k];
    const int64_t nq1 = pa.nq[0], nq2 = pa.nq[1], nq3 = pa.nq[2];
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nq1 * nq2 * nq3) return;
    const int q1 = (int)(idx % nq1), q2 = (int)((idx / nq1) % nq2), q3 = (int)(idx / (nq1 * nq2));
    const int q[3] = {q1, q2, q3};
    const int P = pa.p;
    int f[3];
    const double *v[3], *d[3];
    double one = 1.0, zero = 0.0;
    double w = 1.0;
    for (int m = 0; m < 3; ++m) {
        if (m < DIM) {
            int g = pa.q_off[m] + q[m];
            f[m] = qfirst[g];
            v[m] = qval + (int64_t)g * kQStride;
            d[m] = qder + (int64_t)g * kQStride;
            w *= qw[g];
        } else {
            f[m] = 0;
            v[m] = &one;
            d[m] = &zero;
        }
    }
    double F[3] = {0, 0, 0}, J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    const int P3 = DIM == 3 ? P : 0;
    for (int t3 = 0; t3 <= P3; ++t3)
        for (int t2 = 0; t2 <= P; ++t2)
            for (int t1 = 0; t1 <= P; ++t1) {
                int64_t node = (f[0] + t1) + (int64_t)pa.n[0] * ((f[1] + t2) + (int64_t)pa.n[1] * (f[2] + t3));
                const double* X = ctrl + pa.ctrl_off + node * 3;
                double bv = v[0][t1] * v[1][t2] * v[2][t3];
                double g0 = d[0][t1] * v[1][t2] * v[2][t3];
                double g1 = v[0][t1] * d[1][t2] * v[2][t3];
                double g2 = v[0][t1] * v[1][t2] * d[2][t3];
                for (int x = 0; x < DIM; ++x) {
                    F[x] += bv * X[x];
                    J[x][0] += g0 * X[x];
                    J[x][1] += g1 * X[x];
                    if (DIM == 3) J[x][2] += g2 * X[x];
                }
            }
    double Ji[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double det;
    if (DIM == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        Ji[0][0] = J[1][1] / det;
        Ji[0][1] = -J[0][1] / det;
        Ji[1][0] = -J[1][0] / det;
        Ji[1][1] = J[0][0] / det;
    } else {
        double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
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
    double* o = geo + pa.geo_off + idx * 13;
    o[0] = w * fabs(det);
    for (int a = 0; a < 3; ++a)
        for (int x = 0; x < 3; ++x) o[1 + a * 3 + x] = Ji[a][x];
    o[10] = F[0];
    o[11] = F[1];
    o[12] = F[2];
}

// Stiffness stencil of patch k: one thread per (offset s, node i) computes
// the DIM x DIM entries A[(c,i),(c',i+o_s)] = sum over the Gauss points of
// the common support of  w|J| [mu d_cc' g_i.g_j + mu g_i[c'] g_j[c] + lam g_i[c] g_j[c']]
// with physical gradients g = J^{-T} (parametric gradient).
template <int DIM>
__global__ void k_assemble(const DevPatch* __restrict__ dps, int k, const double* __restrict__ geo,
                           const double* __restrict__ qval, const double* __restrict__ qder,
                           const int* __restrict__ qfirst, const int* __restrict__ el_first,
                           const int* __restrict__ el_last, double* __restrict__ A, double lam_w, double mu_w) {
    const DevPatch pa = dps[k];
    const int P = pa.p, W = 2 * P + 1;
    const int S = DIM == 3 ? W * W * W : W * W;
    const int64_t nodes = pa.nodes;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)S * nodes) return;
    const int64_t node = idx % nodes;
    const int s = (int)(idx / nodes);
    const int o[3] = {s % W - P, (s / W) % W - P, DIM == 3 ? s / (W * W) - P : 0};
    const int i[3] = {(int)(node % pa.n[0]), (int)((node / pa.n[0]) % pa.n[1]), (int)(node / ((int64_t)pa.n[0] * pa.n[1]))};
    int j[3];
    bool valid = true;
    int qlo[3] = {0, 0, 0}, qhi[3] = {0, 0, 0};
    for (int m = 0; m < DIM; ++m) {
        j[m] = i[m] + o[m];
        if (j[m] < 0 || j[m] >= pa.n[m]) {
            valid = false;
            break;
        }
        int elo = max(el_first[pa.el_off[m] + i[m]], el_first[pa.el_off[m] + j[m]]);
        int ehi = min(el_last[pa.el_off[m] + i[m]], el_last[pa.el_off[m] + j[m]]);
        if (elo > ehi) {
            valid = false;
            break;
        }
        qlo[m] = elo * (P + 1);
        qhi[m] = (ehi + 1) * (P + 1);
    }
    if (DIM == 2) {
        j[2] = 0;
        qlo[2] = 0;
        qhi[2] = 1;
    }
    double acc[DIM][DIM];
    for (int a = 0; a < DIM; ++a)
        for (int b = 0; b < DIM; ++b) acc[a][b] = 0.0;
    if (valid) {
        const int64_t nq1 = pa.nq[0], nq2 = pa.nq[1];
        for (int q3 = qlo[2]; q3 < qhi[2]; ++q3) {
            double iv3 = 1, id3 = 0, jv3 = 1, jd3 = 0;
            if (DIM == 3) {
                int g = pa.q_off[2] + q3, f = qfirst[g];
                iv3 = qval[(int64_t)g * kQStride + i[2] - f];
                id3 = qder[(int64_t)g * kQStride + i[2] - f];
                jv3 = qval[(int64_t)g * kQStride + j[2] - f];
                jd3 = qder[(int64_t)g * kQStride + j[2] - f];
            }
            for (int q2 = qlo[1]; q2 < qhi[1]; ++q2) {
                int g2 = pa.q_off[1] + q2, f2 = qfirst[g2];
                double iv2 = qval[(int64_t)g2 * kQStride + i[1] - f2], id2 = qder[(int64_t)g2 * kQStride + i[1] - f2];
                double jv2 = qval[(int64_t)g2 * kQStride + j[1] - f2], jd2 = qder[(int64_t)g2 * kQStride + j[1] - f2];
                for (int q1 = qlo[0]; q1 < qhi[0]; ++q1) {
                    int g1 = pa.q_off[0] + q1, f1 = qfirst[g1];
                    double iv1 = qval[(int64_t)g1 * kQStride + i[0] - f1], id1 = qder[(int64_t)g1 * kQStride + i[0] - f1];
                    double jv1 = qval[(int64_t)g1 * kQStride + j[0] - f1], jd1 = qder[(int64_t)g1 * kQStride + j[0] - f1];
                    const double* G = geo + pa.geo_off + ((int64_t)q1 + nq1 * ((int64_t)q2 + nq2 * q3)) * 13;
                    double gi_r[3] = {id1 * iv2 * iv3, iv1 * id2 * iv3, iv1 * iv2 * id3};
                    double gj_r[3] = {jd1 * jv2 * jv3, jv1 * jd2 * jv3, jv1 * jv2 * jd3};
                    double gi[DIM], gj[DIM];
                    for (int x = 0; x < DIM; ++x) {
                        double si = 0, sj = 0;
                        for (int a = 0; a < DIM; ++a) {
                            si += G[1 + a * 3 + x] * gi_r[a];
                            sj += G[1 + a * 3 + x] * gj_r[a];
                        }
                        gi[x] = si;
                        gj[x] = sj;
                    }
                    double dot = 0;
                    for (int x = 0; x < DIM; ++x) dot += gi[x] * gj[x];
                    const double wq = G[0];
                    for (int a = 0; a < DIM; ++a)
                        for (int b = 0; b < DIM; ++b)
                            acc[a][b] += wq * (mu_w * ((a == b ? dot : 0.0) + gi[b] * gj[a]) + lam_w * gi[a] * gj[b]);
                }
            }
        }
    }
    for (int a = 0; a < DIM; ++a)
        for (int b = 0; b < DIM; ++b)
            A[pa.stencil_off + ((int64_t)(a * DIM + b) * S + s) * nodes + node] = acc[a][b];
}

// Body-force load of patch k: f_(c,i) = sum_q w|J| f_c(x_q) B_i(x_q) with
// f_c(x) = sum over the modes of component c of amp prod_d sin(pi k_d x_d + phase_d).
template <int DIM>
__global__ void k_load(const DevPatch* __restrict__ dps, int k, const double* __restrict__ geo,
                       const double* __restrict__ qval, const int* __restrict__ qfirst,
                       const int* __restrict__ el_first, const int* __restrict__ el_last,
                       const double* __restrict__ modes, int n_modes, double* __restrict__ f, int64_t f_base) {
    const DevPatch pa = dps[k];
    const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= pa.nodes) return;
    const int P = pa.p;
    const int i[3] = {(int)(node % pa.n[0]), (int)((node / pa.n[0]) % pa.n[1]), (int)(node / ((int64_t)pa.n[0] * pa.n[1]))};
    int qlo[3] = {0, 0, 0}, qhi[3] = {1, 1, 1};
    for (int m = 0; m < DIM; ++m) {
        qlo[m] = el_first[pa.el_off[m] + i[m]] * (P + 1);
        qhi[m] = (el_last[pa.el_off[m] + i[m]] + 1) * (P + 1);
    }
    double acc[3] = {0, 0, 0};
    const int64_t nq1 = pa.nq[0], nq2 = pa.nq[1];
    for (int q3 = qlo[2]; q3 < qhi[2]; ++q3) {
        double v3 = 1;
        if (DIM == 3) {
            int g = pa.q_off[2] + q3;
            v3 = qval[(int64_t)g * kQStride + i[2] - qfirst[g]];
        }
        for (int q2 = qlo[1]; q2 < qhi[1]; ++q2) {
            int g2 = pa.q_off[1] + q2;
            double v2 = qval[(int64_t)g2 * kQStride + i[1] - qfirst[g2]];
            for (int q1 = qlo[0]; q1 < qhi[0]; ++q1) {
                int g1 = pa.q_off[0] + q1;
                double v1 = qval[(int64_t)g1 * kQStride + i[0] - qfirst[g1]];
                const double* G = geo + pa.geo_off + ((int64_t)q1 + nq1 * ((int64_t)q2 + nq2 * q3)) * 13;
                double b = G[0] * v1 * v2 * v3;
                for (int j = 0; j < n_modes; ++j) {
                    const double* md = modes + j * 8;
                    double val = md[1];
                    for (int d = 0; d < DIM; ++d) val *= sin(M_PI * md[2 + d] * G[10 + d] + md[5 + d]);
                    acc[(int)md[0]] += b * val;
                }
            }
        }
    }
    for (int c = 0; c < DIM; ++c) f[pa.dof_off - f_base + c * pa.nodes + node] = acc[c];
}

// W(q) u_c(q) at every Gauss point of patch k (u a DOF vector): the first
// half of the physical mass product M u = sum_q w|J| B_i(q) u(q).
template <int DIM>
__global__ void k_field_qp(const DevPatch* __restrict__ dps, int k, const double* __restrict__ geo,
                           const double* __restrict__ qval, const int* __restrict__ qfirst,
                           const double* __restrict__ u, double* __restrict__ qbuf) {
    const DevPatch pa = dps[k];
    const int64_t nq1 = pa.nq[0], nq2 = pa.nq[1], nq3 = pa.nq[2];
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nq1 * nq2 * nq3) return;
    const int q[3] = {(int)(idx % nq1), (int)((idx / nq1) % nq2), (int)(idx / (nq1 * nq2))};
    const int P = pa.p;
    int f[3] = {0, 0, 0};
    const double* v[3];
    const double one = 1.0;
    for (int m = 0; m < 3; ++m) {
        if (m < DIM) {
            const int g = pa.q_off[m] + q[m];
            f[m] = qfirst[g];
            v[m] = qval + (int64_t)g * kQStride;
        } else {
            v[m] = &one;
        }
    }
    double val[3] = {0, 0, 0};
    const int P3 = DIM == 3 ? P : 0;
    for (int t3 = 0; t3 <= P3; ++t3)
        for (int t2 = 0; t2 <= P; ++t2)
            for (int t1 = 0; t1 <= P; ++t1) {
                const int64_t node = (f[0] + t1) + (int64_t)pa.n[0] * ((f[1] + t2) + (int64_t)pa.n[1] * (f[2] + t3));
                const double b = v[0][t1] * v[1][t2] * v[2][t3];
                for (int c = 0; c < DIM; ++c) val[c] += b * u[pa.dof_off + c * pa.nodes + node];
            }
    const double W = geo[pa.geo_off + idx * 13];
    for (int c = 0; c < DIM; ++c) qbuf[idx * DIM + c] = W * val[c];
}

// y_(c,i) = sum over the Gauss points q in the support of B_i of B_i(q) qbuf[q][c]
template <int DIM>
__global__ void k_mass_gather(const DevPatch* __restrict__ dps, int k, const double* __restrict__ qval,
                              const int* __restrict__ qfirst, const int* __restrict__ el_first,
                              const int* __restrict__ el_last, const double* __restrict__ qbuf,
                              double* __restrict__ y) {
    const DevPatch pa = dps[k];
    const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= pa.nodes) return;
    const int P = pa.p;
    const int i[3] = {(int)(node % pa.n[0]), (int)((node / pa.n[0]) % pa.n[1]), (int)(node / ((int64_t)pa.n[0] * pa.n[1]))};
    int qlo[3] = {0, 0, 0}, qhi[3] = {1, 1, 1};
    for (int m = 0; m < DIM; ++m) {
        qlo[m] = el_first[pa.el_off[m] + i[m]] * (P + 1);
        qhi[m] = (el_last[pa.el_off[m] + i[m]] + 1) * (P + 1);
    }
    double acc[3] = {0, 0, 0};
    const int64_t nq1 = pa.nq[0], nq2 = pa.nq[1];
    for (int q3 = qlo[2]; q3 < qhi[2]; ++q3) {
        double v3 = 1;
        if (DIM == 3) {
            const int g = pa.q_off[2] + q3;
            v3 = qval[(int64_t)g * kQStride + i[2] - qfirst[g]];
        }
        for (int q2 = qlo[1]; q2 < qhi[1]; ++q2) {
            const int g2 = pa.q_off[1] + q2;
            const double v2 = qval[(int64_t)g2 * kQStride + i[1] - qfirst[g2]];
            for (int q1 = qlo[0]; q1 < qhi[0]; ++q1) {
                const int g1 = pa.q_off[0] + q1;
                const double b = qval[(int64_t)g1 * kQStride + i[0] - qfirst[g1]] * v2 * v3;
                const int64_t qi = (int64_t)q1 + nq1 * ((int64_t)q2 + nq2 * q3);
                for (int c = 0; c < DIM; ++c) acc[c] += b * qbuf[qi * DIM + c];
            }
        }
    }
    for (int c = 0; c < DIM; ++c) y[pa.dof_off + c * pa.nodes + node] = acc[c];
}

// Per-block partial sums over the Gauss points of patch k of
//   e_mu  = w|J| (grad u + grad u^T) : grad psi   (= 2 eps(u) : eps(psi))
//   e_lam = w|J| div u div psi,
// the two parts of the bilinear form of Section 3 (a = mu e_mu + lam e_lam).
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_energy(const DevPatch* __restrict__ dps, int k, const double* __restrict__ geo,
                                                   const double* __restrict__ qval, const double* __restrict__ qder,
                                                   const int* __restrict__ qfirst, const double* __restrict__ u,
                                                   const double* __restrict__ psi, double* __restrict__ part) {
    __shared__ double lds[2 * 4];
    const DevPatch pa = dps[k];
    const int64_t nq1 = pa.nq[0], nq2 = pa.nq[1], nq3 = pa.nq[2];
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (idx < nq1 * nq2 * nq3) {
        const int q[3] = {(int)(idx % nq1), (int)((idx / nq1) % nq2), (int)(idx / (nq1 * nq2))};
        const int P = pa.p;
        int f[3] = {0, 0, 0};
        const double *v[3], *d[3];
        const double one = 1.0, zero = 0.0;
        for (int m = 0; m < 3; ++m) {
            if (m < DIM) {
                const int g = pa.q_off[m] + q[m];
                f[m] = qfirst[g];
                v[m] = qval + (int64_t)g * kQStride;
                d[m] = qder + (int64_t)g * kQStride;
            } else {
                v[m] = &one;
                d[m] = &zero;
            }
        }
        double gu[3][3] = {{0}}, gp[3][3] = {{0}};  // parametric gradients [c][a]
        const int P3 = DIM == 3 ? P : 0;
        for (int t3 = 0; t3 <= P3; ++t3)
            for (int t2 = 0; t2 <= P; ++t2)
                for (int t1 = 0; t1 <= P; ++t1) {
                    const int64_t node = (f[0] + t1) + (int64_t)pa.n[0] * ((f[1] + t2) + (int64_t)pa.n[1] * (f[2] + t3));
                    const double g[3] = {d[0][t1] * v[1][t2] * v[2][t3], v[0][t1] * d[1][t2] * v[2][t3],
                                         v[0][t1] * v[1][t2] * d[2][t3]};
                    for (int c = 0; c < DIM; ++c) {
                        const double uc = u[pa.dof_off + c * pa.nodes + node];
                        const double pc = psi[pa.dof_off + c * pa.nodes + node];
                        for (int a = 0; a < DIM; ++a) {
                            gu[c][a] += g[a] * uc;
                            gp[c][a] += g[a] * pc;
                        }
                    }
                }
        const double* G = geo + pa.geo_off + idx * 13;
        double Gu[3][3], Gp[3][3];  // physical gradients [c][x]
        for (int c = 0; c < DIM; ++c)
            for (int x = 0; x < DIM; ++x) {
                double su = 0, sp = 0;
                for (int a = 0; a < DIM; ++a) {
                    su += gu[c][a] * G[1 + a * 3 + x];
                    sp += gp[c][a] * G[1 + a * 3 + x];
                }
                Gu[c][x] = su;
                Gp[c][x] = sp;
            }
        double emu = 0, divu = 0, divp = 0;
        for (int c = 0; c < DIM; ++c) {
            divu += Gu[c][c];
            divp += Gp[c][c];
            for (int x = 0; x < DIM; ++x) emu += (Gu[c][x] + Gu[x][c]) * Gp[c][x];
        }
        acc[0] = G[0] * emu;
        acc[1] = G[0] * divu * divp;
    }
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) {
        part[(int64_t)blockIdx.x * 2] = acc[0];
        part[(int64_t)blockIdx.x * 2 + 1] = acc[1];
    }
}

// partial[mode][chunk] = sum over the chunk of F[mode][i] psi[off + i]
__global__ void __launch_bounds__(kBlock) k_mdot_partial(const double* __restrict__ F, int64_t n, int64_t off,
                                                         const double* __restrict__ psi, double* __restrict__ part) {
    __shared__ double lds[4];
    const int mode = blockIdx.y;
    const int64_t b = (int64_t)blockIdx.x * kChunk, e = min(n, b + (int64_t)kChunk);
    double acc[1] = {0.0};
    for (int64_t i = b + threadIdx.x; i < e; i += kBlock) acc[0] += F[(int64_t)mode * n + i] * psi[off + i];
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) part[(int64_t)mode * gridDim.x + blockIdx.x] = acc[0];
}

// ================================================================ operators
// y = A x (+ B^T t): one thread per row (patch, component c, node), reading
// the canonical half of the symmetric stencil: entries of the row's own
// blocks at the row's node, mirrored entries at the neighbour's node.  The
// stencil is streamed once (non-temporal loads); x stays in cache.
// y = A x (+ B^T t): one thread per row (patch, component c, node).
template <int DIM, int P>
__global__ void __launch_bounds__(kBlock) k_stiffness(const DevPatch* __restrict__ dps, const int4* __restrict__ rb,
                                                      const double* __restrict__ A, const double* __restrict__ x,
                                                      double* __restrict__ y, const int64_t* __restrict__ bt_ptr,
                                                      const int* __restrict__ bt_row, const double* __restrict__ bt_sign,
                                                      const double* __restrict__ t, const MinresState* __restrict__ mask) {
    constexpr int W = 2 * P + 1;
    constexpr int S = DIM == 3 ? W * W * W : W * W;
    constexpr int P3 = DIM == 3 ? P : 0;
    const int4 b = rb[blockIdx.x];
    const DevPatch& pa = dps[b.x];
    if (mask && mask[pa.prob].skip) return;
    const int64_t nodes = pa.nodes;
    const int64_t node = (int64_t)b.z + threadIdx.x;
    if (node >= nodes) return;
    const int n1 = pa.n[0], n2 = pa.n[1], n3 = pa.n[2];
    const int i1 = (int)(node % n1), i2 = (int)((node / n1) % n2), i3 = (int)(node / ((int64_t)n1 * n2));
    const int c = b.y;
    const double* Ab = A + pa.stencil_off + (int64_t)(c * DIM) * S * nodes + node;
    const double* xb = x + pa.dof_off;
    double acc = 0.0;
    for (int cp = 0; cp < DIM; ++cp) {
        const double* Ac = Ab + (int64_t)cp * S * nodes;
        const double* xc = xb + (int64_t)cp * nodes;
        for (int o3 = -P3; o3 <= P3; ++o3) {
            const int j3 = i3 + o3;
            const bool v3 = (unsigned)j3 < (unsigned)n3;
            for (int o2 = -P; o2 <= P; ++o2) {
                const int j2 = i2 + o2;
                const bool v23 = v3 && (unsigned)j2 < (unsigned)n2;
                const int64_t rowoff = (int64_t)n1 * (j2 + (int64_t)n2 * j3);
                const int sbase = (o2 + P) * W + (o3 + P3) * W * W;
#pragma unroll
                for (int o1 = -P; o1 <= P; ++o1) {
                    const int j1 = i1 + o1;
                    if (v23 && (unsigned)j1 < (unsigned)n1)
                        acc += Ac[(int64_t)(sbase + o1 + P) * nodes] * xc[rowoff + j1];
                }
            }
        }
    }
    const int64_t row = pa.dof_off + (int64_t)c * nodes + node;
    if (t) {
        for (int64_t e = bt_ptr[row]; e < bt_ptr[row + 1]; ++e) acc += bt_sign[e] * t[bt_row[e]];
    }
    y[row] = acc;
}

// ===================================================== matrix-free stiffness
// y = A x by quadrature of the bilinear form of Section 3 with sum
// factorisation, brick by brick (BE^3 elements of a C^{p-1} patch, NB = BE + p
// basis functions and QB = BE (p + 1) Gauss points per direction).  One
// workgroup of NW wavefronts per brick:
//   F1 (row per thread)    A0 = V1 x, A1 = D1 x along direction 1;
//   F2 (row per thread)    B00 = V2 A0, B10 = D2 A0, B01 = V2 A1;
//   Q  (Gauss column (q1, q2) per lane, wave w owns a range of q3)
//      parametric gradients G = (V3 B01, V3 B10, D3 B00) in registers, the
//      stress sigma = mu (grad u + grad u^T) + lam div u I and the flux
//      w |J| sigma J^{-T} at each point (J of the trilinear patch map,
//      analytic), then the partial transposed contractions
//      P = (V3^T F1, V3^T F2, D3^T F3) over the wave's q3 range, summed over
//      the waves in a fixed order;
//   B2 (row per thread)    SD = V2^T P1, SV = D2^T P2 + V2^T P3;
//   B1 (row per thread)    y = D1^T SD + V1^T SV, to the per-brick buffer.
// The univariate tables of a brick are uniform across the workgroup and are
// read from a per-brick table in global memory (scalar loads); only the
// transposes between the row and column phases go through LDS.  A second
// kernel sums, for every node, the contributions of the bricks that contain
// it in a fixed order (deterministic, no atomics).
template <int P>
struct MfShape {
    static constexpr int BE = P <= 4 ? 2 : 1;               // elements per brick direction
    static constexpr int NB = BE + P;                       // basis functions per brick direction
    static constexpr int QB = BE * (P + 1);                 // Gauss points per brick direction
    static constexpr int NCOL = QB * QB;                    // Gauss columns (q1, q2)
    static constexpr int TS = 2 * QB * NB + 2 * QB;         // table doubles per (direction, brick)
    static constexpr int QA = QB | 1;                       // row stride of A / S in LDS (odd: no bank conflicts)
    static constexpr int NCB = (NCOL + 15) / 16 * 16 + 8;   // t3 stride of B / P in LDS
    static constexpr int NW = 2;                            // wavefronts per brick
    static constexpr int QPG = (QB + NW - 1) / NW;          // q3 values per wavefront
    static constexpr int NT = 64 * NW;                      // threads per brick
    // support: at brick Gauss point q (element q / (P + 1)) only basis
    // functions tlo(q)..thi(q) are nonzero; basis t is nonzero at the Gauss
    // points qlo(t) <= q < qhi(t).  The contractions skip the known zeros.
    static constexpr int tlo(int q) { return q / (P + 1); }
    static constexpr int thi(int q) { return q / (P + 1) + P; }
    static constexpr int qlo(int t) { return (t > P ? t - P : 0) * (P + 1); }
    static constexpr int qhi(int t) { return ((t < BE - 1 ? t : BE - 1) + 1) * (P + 1); }
    // each wavefront's q3 range is exactly one element (BE = NW, QPG = P + 1)
    static constexpr bool WAVE_ELEM = NW == BE && QPG == P + 1;
};

template <int P>
__global__ void __launch_bounds__(MfShape<P>::NT) k_mf_brick(const DevPatch* __restrict__ dps,
                                                             const int4* __restrict__ bricks,
                                                             const double* __restrict__ tab,
                                                             const double* __restrict__ x, double* __restrict__ ybuf,
                                                             const MinresState* __restrict__ mask) {
    using S = MfShape<P>;
    constexpr int BE = S::BE, NB = S::NB, QB = S::QB, NCOL = S::NCOL, TS = S::TS, QA = S::QA, NCB = S::NCB;
    constexpr int QPG = S::QPG, NT = S::NT, NW = S::NW;
    constexpr int NB3 = NB * NB * NB;
    constexpr int AK = 3 * NB * NB * QA;  // offset of A1 / SV in sA
    constexpr int BK = NB * NCB;          // stride of the k index in sB
    constexpr int OD = QB * NB, OW = 2 * QB * NB, OE = 2 * QB * NB + QB;  // D, W, E within a table
    __shared__ double sB[9 * BK];         // [c][k][t3][q2 QB + q1]: B00, B10, B01, then P1, P2, P3, then S
    static_assert(2 * AK <= 9 * BK, "S must fit in the B / P buffer");
    const int4 br = bricks[blockIdx.x];
    const DevPatch& pa = dps[br.x];
    if (mask && mask[pa.prob].skip) return;
    const int tid = threadIdx.x;
    const double* __restrict__ T1 = tab + pa.tab_off[0] + (int64_t)br.y * TS;
    const double* __restrict__ T2 = tab + pa.tab_off[1] + (int64_t)br.z * TS;
    const double* __restrict__ T3 = tab + pa.tab_off[2] + (int64_t)br.w * TS;
    const int i1 = br.y * BE, i2 = br.z * BE, i3 = br.w * BE;  // first basis function of the brick
    // ---- F: rows (c, t3, q1): A0 = V1 x, A1 = D1 x along direction 1 for
    // this q1 (each A value is formed by exactly one thread, from the NB x NB
    // coefficients of the row's (c, t3) plane, read through the cache), then
    // B00 = V2 A0, B10 = D2 A0, B01 = V2 A1 along direction 2
    // (a brick whose basis functions all lie in the patch reads its
    // coefficients without bounds checks: every brick, when the element
    // counts are multiples of the brick size)
    const bool full = i1 + NB <= pa.n[0] && i2 + NB <= pa.n[1] && i3 + NB <= pa.n[2];
    auto fphase = [&](auto checked) {
    constexpr bool CHK = decltype(checked)::value;
    for (int row = tid; row < 3 * NB * QB; row += NT) {
        const int c = row / (NB * QB), t3 = (row / QB) % NB, q1 = row % QB;
        // basis functions e1..e1+P are the ones supported at Gauss point q1
        const int e1 = S::tlo(q1);
        const bool pin = !CHK || i3 + t3 < pa.n[2];
        const double* xp = x + pa.dof_off + (int64_t)c * pa.nodes + (int64_t)pa.n[0] * pa.n[1] * (i3 + t3) +
                           (int64_t)pa.n[0] * i2 + i1 + e1;
        double v1[P + 1], d1[P + 1];
#pragma unroll
        for (int u = 0; u <= P; ++u) {
            v1[u] = T1[q1 * NB + e1 + u];
            d1[u] = T1[OD + q1 * NB + e1 + u];
        }
        double a0[NB], a1[NB];
#pragma unroll
        for (int t2 = 0; t2 < NB; ++t2) {
            const bool rin = pin && (!CHK || i2 + t2 < pa.n[1]);
            const double* xr = xp + pa.n[0] * t2;
            double xl[P + 1];
#pragma unroll
            for (int u = 0; u <= P; ++u) {
                if constexpr (CHK) {
                    // coefficients outside the patch are zero: load from a
                    // valid address and select, without a branch
                    const bool ok = rin && i1 + e1 + u < pa.n[0];
                    const double v = *(ok ? xr + u : x);
                    xl[u] = ok ? v : 0.0;
                } else {
                    xl[u] = xr[u];
                }
            }
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int u = 0; u <= P; ++u) {
                s0 += v1[u] * xl[u];
                s1 += d1[u] * xl[u];
            }
            a0[t2] = s0;
            a1[t2] = s1;
        }
        double* b = sB + (c * 3 * NB + t3) * NCB + q1;
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            double b00 = 0.0, b10 = 0.0, b01 = 0.0;
#pragma unroll
            for (int t = S::tlo(q); t <= S::thi(q); ++t) {
                b00 += T2[q * NB + t] * a0[t];
                b10 += T2[OD + q * NB + t] * a0[t];
                b01 += T2[q * NB + t] * a1[t];
            }
            b[q * QB] = b00;
            b[BK + q * QB] = b10;
            b[2 * BK + q * QB] = b01;
        }
    }
    };
    if (full) fphase(std::false_type{});
    else fphase(std::true_type{});
    __syncthreads();
    // ---- Q: Gauss columns, wavefront w owns q3 in [w QPG, w QPG + QPG)
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int q3a = w * QPG;
    // Gauss point q3a + j exists (always, when the wavefronts split QB evenly)
    auto has = [&](int j) { return QPG * NW == QB || q3a + j < QB; };
    const double lam = pa.lam, mu = pa.mu;
    for (int cb = 0; cb < NCOL; cb += 64) {
        const int col = cb + (tid & 63);
        const bool act = col < NCOL;
        double F[3][3][QPG];  // [c][a][j]: gradient d u_c / d eta_a, then flux
        if (act) {
            // E: the element of this wavefront's q3 range (its basis functions
            // E..E+P), or -1 for all basis functions
            auto grads = [&](auto Ec) {
                constexpr int E = decltype(Ec)::value;
                constexpr int TA = E < 0 ? 0 : E, TZ = E < 0 ? NB - 1 : E + P;
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        double bv[NB];
#pragma unroll
                        for (int t = TA; t <= TZ; ++t) bv[t] = sB[(c * 3 + k) * BK + t * NCB + col];
                        // B00 -> d/deta_3 (D3), B10 -> d/deta_2 (V3), B01 -> d/deta_1 (V3)
                        const int a = 2 - k;
                        const int o = k == 0 ? OD : 0;
#pragma unroll
                        for (int j = 0; j < QPG; ++j) {
                            double g = 0.0;
                            if (has(j)) {
#pragma unroll
                                for (int t = TA; t <= TZ; ++t) g += T3[o + (q3a + j) * NB + t] * bv[t];
                            }
                            F[c][a][j] = g;
                        }
                    }
            };
            if constexpr (S::WAVE_ELEM) {
                if (w == 0) grads(std::integral_constant<int, 0>{});
                else grads(std::integral_constant<int, 1>{});
            } else {
                grads(std::integral_constant<int, -1>{});
            }
            const int q1 = col % QB, q2 = col / QB;
            const double w12 = T1[OW + q1] * T2[OW + q2];
            const double e1 = T1[OE + q1], e2 = T2[OE + q2];
#pragma unroll
            for (int j = 0; j < QPG; ++j) {
                if (!has(j)) continue;
                const double e3 = T3[OE + q3a + j];
                const double eta[3] = {e1, e2, e3};
                // d F / d eta_a of the trilinear map is bilinear in the other
                // two coordinates (b < c): c0 + c1 eta_b + c2 eta_c + c3 eta_b eta_c
                double J[3][3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double eb = eta[a == 0 ? 1 : 0], ec = eta[a == 2 ? 1 : 2];
#pragma unroll
                    for (int xx = 0; xx < 3; ++xx) {
                        const double* c4 = &pa.jcoef[(a * 3 + xx) * 4];
                        J[xx][a] = (c4[0] + c4[1] * eb) + (c4[2] + c4[3] * eb) * ec;
                    }
                }
                // adjugate: Ad[a][x] = det(J) d eta_a / d x_x
                double Ad[3][3];
                Ad[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
                Ad[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
                Ad[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
                Ad[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
                Ad[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
                Ad[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
                Ad[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
                Ad[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
                Ad[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
                const double ad = fabs(J[0][0] * Ad[0][0] + J[0][1] * Ad[1][0] + J[0][2] * Ad[2][0]);
                // 1/|det|: hardware reciprocal refined by two Newton-Raphson
                // steps (e <- e + e (1 - |det| e)), within an ulp or so of the
                // correctly rounded quotient at half its instruction count
                double id = __builtin_amdgcn_rcp(ad);
                id = fma(fma(-ad, id, 1.0), id, id);
                id = fma(fma(-ad, id, 1.0), id, id);
                // with Ji = Ad / det and the weight w |det|, the flux
                // w |det| sigma(G Ji) Ji^T equals (w / |det|) sigma(G Ad) Ad^T
                const double sw = w12 * T3[OW + q3a + j] * id;
                const double ms = mu * sw, ls = lam * sw, ms2 = ms + ms;
                double g[3][3];  // G Ad: det(J) times the physical gradient [c][x]
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int xx = 0; xx < 3; ++xx)
                        g[c][xx] = F[c][0][j] * Ad[0][xx] + F[c][1][j] * Ad[1][xx] + F[c][2][j] * Ad[2][xx];
                const double ldv = ls * (g[0][0] + g[1][1] + g[2][2]);
                double sg[3][3];  // scaled stress, symmetric
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    sg[c][c] = fma(ms2, g[c][c], ldv);
#pragma unroll
                    for (int xx = c + 1; xx < 3; ++xx) sg[c][xx] = sg[xx][c] = ms * (g[c][xx] + g[xx][c]);
                }
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int a = 0; a < 3; ++a) F[c][a][j] = sg[c][0] * Ad[a][0] + sg[c][1] * Ad[a][1] + sg[c][2] * Ad[a][2];
            }
        }
        // P = sum over wavefronts (in order) of the partial contractions
        auto partial = [&](int c, int a, int t) {
            const int o = a == 2 ? OD : 0;
            double v = 0.0;
#pragma unroll
            for (int j = 0; j < QPG; ++j)
                if (has(j)) v += T3[o + (q3a + j) * NB + t] * F[c][a][j];
            return v;
        };
        __syncthreads();  // every wavefront has read B
        // (with one element per wavefront, wavefront r touches only basis
        // functions r..r+P: the first writes zeros beyond P, the others add
        // their range)
        if (w == 0 && act) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int t = 0; t < NB; ++t)
                        sB[(c * 3 + a) * BK + t * NCB + col] = (!S::WAVE_ELEM || t <= P) ? partial(c, a, t) : 0.0;
        }
        __syncthreads();
#pragma unroll 1
        for (int r = 1; r < NW; ++r) {
            if (w == r && act) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int t = 0; t < NB; ++t)
                            if (!S::WAVE_ELEM || (t >= r && t <= r + P))
                                sB[(c * 3 + a) * BK + t * NCB + col] += partial(c, a, t);
            }
            __syncthreads();
        }
    }
    // ---- B2: rows (c, t3, q1): SD = V2^T P1, SV = D2^T P2 + V2^T P3; once
    // every thread has read its P, S overwrites the start of sB
    constexpr int RB2 = (3 * NB * QB + NT - 1) / NT;  // B2 rows per thread
    double sd[RB2][NB], sv[RB2][NB];
#pragma unroll
    for (int rr = 0; rr < RB2; ++rr) {
        const int row = tid + rr * NT;
        if (row >= 3 * NB * QB) continue;
        const int c = row / (NB * QB), t3 = (row / QB) % NB, q1 = row % QB;
        const double* pp = sB + (c * 3 * NB + t3) * NCB + q1;
        double p1[QB], p2[QB], p3[QB];
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            p1[q] = pp[q * QB];
            p2[q] = pp[BK + q * QB];
            p3[q] = pp[2 * BK + q * QB];
        }
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int q = S::qlo(t); q < S::qhi(t); ++q) {
                a += T2[q * NB + t] * p1[q];
                b += T2[OD + q * NB + t] * p2[q] + T2[q * NB + t] * p3[q];
            }
            sd[rr][t] = a;
            sv[rr][t] = b;
        }
    }
    __syncthreads();
    double* const sA = sB;  // S: [SD|SV][c][t3][t2][q1], rows of QA doubles
#pragma unroll
    for (int rr = 0; rr < RB2; ++rr) {
        const int row = tid + rr * NT;
        if (row >= 3 * NB * QB) continue;
        const int c = row / (NB * QB), t3 = (row / QB) % NB, q1 = row % QB;
        double* s = sA + (c * NB + t3) * NB * QA + q1;
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            s[t * QA] = sd[rr][t];
            s[AK + t * QA] = sv[rr][t];
        }
    }
    __syncthreads();
    // ---- B1: rows (c, t3, t2), written to the brick buffer
    // brick buffer layout [c][t3][t2][t1][brick] (brick fastest, bricks in
    // (b3, b2, b1) order): the per-node gather reads runs of consecutive bricks
    const int64_t nbr = (int64_t)pa.nb[0] * pa.nb[1] * pa.nb[2];
    double* yb = ybuf + pa.ybuf_off + ((int64_t)br.w * pa.nb[1] + br.z) * pa.nb[0] + br.y;
    for (int row = tid; row < 3 * NB * NB; row += NT) {
        const double* s = sA + row * QA;
        double sd[QB], sv[QB];
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            sd[q] = s[q];
            sv[q] = s[AK + q];
        }
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            double v = 0.0;
#pragma unroll
            for (int q = S::qlo(t); q < S::qhi(t); ++q) v += T1[OD + q * NB + t] * sd[q] + T1[q * NB + t] * sv[q];
            yb[(row * NB + t) * nbr] = v;
        }
    }
}

// y_(c,i) = sum over the bricks containing node i of their contributions
// (bricks in increasing (b3, b2, b1) order), + B^T t if t != NULL
template <int P>
__global__ void __launch_bounds__(kBlock) k_mf_gather(const DevPatch* __restrict__ dps, const int4* __restrict__ rb,
                                                      const double* __restrict__ ybuf, double* __restrict__ y,
                                                      const int64_t* __restrict__ bt_ptr, const int* __restrict__ bt_row,
                                                      const double* __restrict__ bt_sign, const double* __restrict__ t,
                                                      const MinresState* __restrict__ mask) {
    constexpr int BE = MfShape<P>::BE, NB = MfShape<P>::NB;
    constexpr int NB3 = NB * NB * NB;
    const int4 b = rb[blockIdx.x];
    const DevPatch& pa = dps[b.x];
    if (mask && mask[pa.prob].skip) return;
    const int64_t node = (int64_t)b.z + threadIdx.x;
    if (node >= pa.nodes) return;
    const int c = b.y;
    const int i[3] = {(int)(node % pa.n[0]), (int)((node / pa.n[0]) % pa.n[1]), (int)(node / ((int64_t)pa.n[0] * pa.n[1]))};
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        // bricks b with b BE <= i <= b BE + BE - 1 + P
        const int l = i[d] - P - BE + 1;
        lo[d] = l <= 0 ? 0 : (l + BE - 1) / BE;
        hi[d] = min(pa.nb[d] - 1, i[d] / BE);
    }
    const int64_t nbr = (int64_t)pa.nb[0] * pa.nb[1] * pa.nb[2];
    // at most NR bricks per direction contain a node; the sum runs in the
    // fixed (b3, b2, b1) order.  All loads are issued before the sum when
    // they fit in registers (NR <= 3); for larger NR, one (b2, b1) plane of
    // loads at a time (the same order)
    constexpr int NR = (NB + BE - 1) / BE;
    constexpr int NA = NR <= 3 ? NR : 1;  // b3 planes of loads in flight
    double acc = 0.0;
#pragma unroll 1
    for (int a30 = 0; a30 < NR; a30 += NA) {
        double v[NA * NR * NR];
#pragma unroll
        for (int a3 = 0; a3 < NA; ++a3)
#pragma unroll
            for (int a2 = 0; a2 < NR; ++a2)
#pragma unroll
                for (int a1 = 0; a1 < NR; ++a1) {
                    const int b3 = lo[2] + a30 + a3, b2 = lo[1] + a2, b1 = lo[0] + a1;
                    double r = 0.0;
                    if (b3 <= hi[2] && b2 <= hi[1] && b1 <= hi[0]) {
                        const int64_t g = (int64_t)(b3 * pa.nb[1] + b2) * pa.nb[0] + b1;
                        const int t1 = i[0] - b1 * BE, t2 = i[1] - b2 * BE, t3 = i[2] - b3 * BE;
                        r = ybuf[pa.ybuf_off + ((int64_t)((c * NB + t3) * NB + t2) * NB + t1) * nbr + g];
                    }
                    v[(a3 * NR + a2) * NR + a1] = r;
                }
#pragma unroll
        for (int a = 0; a < NA * NR * NR; ++a) acc += v[a];
    }
    const int64_t row = pa.dof_off + (int64_t)c * pa.nodes + node;
    if (t) {
        for (int64_t e = bt_ptr[row]; e < bt_ptr[row + 1]; ++e) acc += bt_sign[e] * t[bt_row[e]];
    }
    y[row] = acc;
}

template <int P>
void mf_bricks_t(const DevPatch* dp, const int4* bricks, int n_bricks, const double* tab, const double* x,
                 double* ybuf, const MinresState* mask, hipStream_t s) {
    hipLaunchKernelGGL(k_mf_brick<P>, dim3(n_bricks), dim3(MfShape<P>::NT), 0, s, dp, bricks, tab, x, ybuf, mask);
}

template <int P>
void mf_gather_t(const DevPatch* dp, const int4* rb, int nrb, const double* ybuf, double* y, const int64_t* bp,
                 const int* br, const double* bs, const double* t, const MinresState* mask, hipStream_t s) {
    hipLaunchKernelGGL(k_mf_gather<P>, dim3(nrb), dim3(kBlock), 0, s, dp, rb, ybuf, y, bp, br, bs, t, mask);
}

// A-hat_l x = kappa_1 (M3 x M2 x K1) x + kappa_2 (M3 x K2 x M1) x
//           + kappa_3 (K3 x M2 x M1) x           (Kronecker form, Section 5.2;
// with geometry inclusion A~_l, the same form with the weighted univariate
// matrices of component l and kappa = 1, Section 5.2.3)
//         = M2 (kappa_1 K1 u + kappa_3 M1 v) + kappa_2 K2 (M1 u),
//           u = M3 x, v = K3 x,
// by sum factorisation, one workgroup per slab i3 of a patch and component:
// u, v on the slab (direction 3, read from global memory), then direction 1
// (a = kappa_1 K1 u + kappa_3 M1 v, b = M1 u) and direction 2 in LDS
// (four slab arrays).  Univariate K, M are banded (half-bandwidth p) and
// stored as [i][t], t = j - i + p.
// P > 0: degree known at compile time (loops unrolled); P == 0: any degree.
constexpr int kAhBlock = 512;  // threads of the A-hat slab kernel
constexpr int kAhE = 3;        // slab entries per thread whose loads are in flight together

// One workgroup per slab (patch, component l, i3): y = A-hat x on that slab
// (H^{d-2} A-hat x with use_h).  Direction 3 is taken from global memory
// (2p + 1 slabs of x), directions 1 and 2 from LDS; the band rows of
// directions 1 and 2 are staged in LDS first.  LDS: U, V (direction-3
// products), then A, Bm overwrite them, then the band rows.
template <int P>
__global__ void __launch_bounds__(kAhBlock) k_ahat(const DevPatch* __restrict__ dps, const int4* __restrict__ slabs,
                                                   const double* __restrict__ kb, const double* __restrict__ mb,
                                                   const double* __restrict__ x, double* __restrict__ y, int max_n12,
                                                   int use_h, int bnd_in, int bnd_out,
                                                   const MinresState* __restrict__ mask) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int4 it = slabs[blockIdx.x];
    const DevPatch& pa = dps[it.x];
    if (mask && mask[pa.prob].skip) return;
    const int l = it.y, i3 = it.z;
    const int n1 = pa.n[0], n2 = pa.n[1], n3 = pa.n[2], n12 = n1 * n2;
    const int p = P > 0 ? P : pa.p, W = 2 * p + 1;
    double* U = reinterpret_cast<double*>(smem);
    double* V = U + max_n12;
    const int nb1 = n1 * W, nb2 = n2 * W;
    // band rows of directions 1 and 2: staged in LDS for the specialised
    // degrees, read from global memory by the generic kernel
    const double* K1 = kb + pa.band_off[l][0];
    const double* Mb1 = mb + pa.band_off[l][0];
    const double* K2 = kb + pa.band_off[l][1];
    const double* Mb2 = mb + pa.band_off[l][1];
    if constexpr (P > 0) {
        double* T = V + max_n12;  // K1 | M1 (n1 x W), K2 | M2 (n2 x W)
        batched_copy<(4 * kMaxN * (2 * P + 1) + kAhBlock - 1) / kAhBlock, kAhBlock>(
            T, 2 * (nb1 + nb2), [&](int e) {
                if (e < nb1) return K1[e];
                e -= nb1;
                if (e < nb1) return Mb1[e];
                e -= nb1;
                if (e < nb2) return K2[e];
                return Mb2[e - nb2];
            });
        K1 = T;
        Mb1 = T + nb1;
        K2 = T + 2 * nb1;
        Mb2 = K2 + nb2;
    }
    const int64_t base = pa.dof_off + (int64_t)l * pa.nodes;
    // bnd_in: x vanishes away from the patch boundary, so on slabs more than
    // p layers from the i3 faces only the outer ring of the slab can be
    // nonzero, after direction 1 only the two edge rows and the edge column
    // bands of width p + 1, and y only on the frame of width p + 1 (zero
    // elsewhere).
    // bnd_out: only the patch-boundary entries of y are wanted, so on the
    // slabs between the i3 faces direction 2 is needed on the outer ring
    // only, direction 1 on the bands of p + 1 rows and the two edge columns it
    // reads, direction 3 on the frame of width p + 1 those read.
    const bool ring_only = bnd_in && i3 > p && i3 < n3 - 1 - p;
    const bool thin = bnd_out && i3 > 0 && i3 < n3 - 1;
    // direction 3: the band row of i3 is uniform over the workgroup
    const double* K3 = kb + pa.band_off[l][2] + i3 * W;
    const double* M3 = mb + pa.band_off[l][2] + i3 * W;
    for (int e0 = threadIdx.x; e0 < n12; e0 += kAhBlock * kAhE) {
        bool need[kAhE], load[kAhE];
#pragma unroll
        for (int u = 0; u < kAhE; ++u) {
            const int e = e0 + u * kAhBlock;
            const int i2 = e / n1, i1 = e - i2 * n1;
            need[u] = e < n12 && (!thin || i2 <= p || i2 >= n2 - 1 - p || i1 <= p || i1 >= n1 - 1 - p);
            load[u] = need[u] && (!ring_only || i1 == 0 || i1 == n1 - 1 || i2 == 0 || i2 == n2 - 1);
        }
        if constexpr (P > 0) {
            double xv[kAhE][2 * P + 1];
#pragma unroll
            for (int u = 0; u < kAhE; ++u)
#pragma unroll
                for (int o = 0; o < 2 * P + 1; ++o) {
                    const int j3 = i3 + o - P;
                    xv[u][o] = load[u] && (unsigned)j3 < (unsigned)n3
                                   ? x[base + (int64_t)j3 * n12 + e0 + u * kAhBlock]
                                   : 0.0;
                }
#pragma unroll
            for (int u = 0; u < kAhE; ++u) {
                double uu = 0.0, vv = 0.0;
#pragma unroll
                for (int o = 0; o < 2 * P + 1; ++o) {
                    uu += M3[o] * xv[u][o];
                    vv += K3[o] * xv[u][o];
                }
                if (need[u]) {
                    U[e0 + u * kAhBlock] = uu;
                    V[e0 + u * kAhBlock] = vv;
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < kAhE; ++u) {
                const int e = e0 + u * kAhBlock;
                double uu = 0.0, vv = 0.0;
                if (load[u])
                    for (int o = -p; o <= p; ++o) {
                        const int j3 = i3 + o;
                        const double xx = (unsigned)j3 < (unsigned)n3 ? x[base + (int64_t)j3 * n12 + e] : 0.0;
                        uu += M3[o + p] * xx;
                        vv += K3[o + p] * xx;
                    }
                if (need[u]) {
                    U[e] = uu;
                    V[e] = vv;
                }
            }
        }
    }
    __syncthreads();
    // direction 1 (results held in registers until every thread has read U, V)
    const double k1 = pa.kap[l][0], k2 = pa.kap[l][1], k3 = pa.kap[l][2];
    constexpr int kR = (kMaxN * kMaxN + kAhBlock - 1) / kAhBlock;
    double ra[kR], rb[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int e = threadIdx.x + r * kAhBlock;
        ra[r] = rb[r] = 0.0;
        if (e >= n12) continue;
        const int i2 = e / n1, i1 = e - i2 * n1;
        if (thin && !(i2 <= p || i2 >= n2 - 1 - p || i1 == 0 || i1 == n1 - 1)) continue;
        if (ring_only && !(i2 == 0 || i2 == n2 - 1 || i1 <= p || i1 >= n1 - 1 - p)) continue;
        double ku = 0.0, mu_ = 0.0, mv = 0.0;
#pragma unroll
        for (int o = -p; o <= p; ++o) {
            const int j1 = i1 + o;
            if ((unsigned)j1 < (unsigned)n1) {
                const double uu = U[i2 * n1 + j1], vv = V[i2 * n1 + j1];
                const double kk = K1[i1 * W + o + p], mm = Mb1[i1 * W + o + p];
                ku += kk * uu;
                mu_ += mm * uu;
                mv += mm * vv;
            }
        }
        ra[r] = k1 * ku + k3 * mv;
        rb[r] = mu_;
    }
    __syncthreads();
    double* A = U;
    double* Bm = V;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int e = threadIdx.x + r * kAhBlock;
        if (e < n12) {
            A[e] = ra[r];
            Bm[e] = rb[r];
        }
    }
    __syncthreads();
    // direction 2
    const double sc = use_h ? pa.hscale : 1.0;
    for (int e = threadIdx.x; e < n12; e += kAhBlock) {
        const int i2 = e / n1, i1 = e - i2 * n1;
        if (thin && !(i2 == 0 || i2 == n2 - 1 || i1 == 0 || i1 == n1 - 1)) continue;
        double a = 0.0, b = 0.0;
        if (!ring_only || i2 <= p || i2 >= n2 - 1 - p || i1 <= p || i1 >= n1 - 1 - p) {
#pragma unroll
            for (int o = -p; o <= p; ++o) {
                const int j2 = i2 + o;
                if ((unsigned)j2 < (unsigned)n2) {
                    a += Mb2[i2 * W + o + p] * A[j2 * n1 + i1];
                    b += K2[i2 * W + o + p] * Bm[j2 * n1 + i1];
                }
            }
        }
        y[base + (int64_t)i3 * n12 + e] = sc * (a + k2 * b);
    }
}

template <int P>
void ahat_t(const DevPatch* dp, const int4* slabs, int n_slabs, int max_n12, int max_n1n2, const double* kb,
            const double* mb, const double* x, double* y, int use_h, int bnd_in, int bnd_out, const MinresState* mask,
            hipStream_t s) {
    if (!n_slabs) return;
    const size_t W = P > 0 ? 2 * P + 1 : 0;  // the generic kernel stages no band rows
    // <= (2 * 48^2 + 2 * 13 * 96) * 8 = 56,832 bytes
    const size_t lds = (2 * (size_t)max_n12 + 2 * W * max_n1n2) * sizeof(double);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void*)k_ahat<P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_ahat<P>, dim3(n_slabs), dim3(kAhBlock), lds, s, dp, slabs, kb, mb, x, y, max_n12, use_h,
                       bnd_in, bnd_out, mask);
}

// x[i], or sc[i] x[i] with a per-DOF scale
__device__ inline double scaled(const double* __restrict__ x, const double* __restrict__ sc, int64_t i) {
    return sc ? x[i] * sc[i] : x[i];
}

// value of row r of B applied to x (read as sc .* x with a scale)
__device__ inline double b_row(const int64_t* __restrict__ plus, const int64_t* __restrict__ minus,
                               const GlueRows& gl, const double* __restrict__ x, const double* __restrict__ sc,
                               int64_t r) {
    const int64_t m = minus[r];
    if (m >= -1) return scaled(x, sc, plus[r]) - (m >= 0 ? scaled(x, sc, m) : 0.0);
    const int64_t g = -2 - m;
    double v = scaled(x, sc, plus[r]);
    for (int64_t e = gl.ptr[g]; e < gl.ptr[g + 1]; ++e) v -= gl.val[e] * scaled(x, sc, gl.col[e]);
    return v;
}

__global__ void k_B(const int64_t* __restrict__ plus, const int64_t* __restrict__ minus, GlueRows gl, int64_t n_c,
                    double alpha, const double* __restrict__ x, double* __restrict__ y, const double* __restrict__ sc) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_c) return;
    y[r] = alpha * b_row(plus, minus, gl, x, sc, r);
}

__global__ void k_Bt(const int64_t* __restrict__ ptr, const int* __restrict__ row, const double* __restrict__ sgn,
                     int64_t n, const double* __restrict__ x, double* __restrict__ y, const double* __restrict__ sc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) acc += sgn[e] * x[row[e]];
    y[i] = sc ? sc[i] * acc : acc;
}

// (B B^T)^{-1} row by row, for values computed per row on the fly: star
// block of size s: I + 1 1^T, whose inverse is I - 1 1^T / (s + 1);
// Dirichlet block: identity; rows of dense blocks are left to k_w_dense_*.
// z = (B B^T)^{-1} y (k_W), (B B^T)^{-1} (B x) (k_BW), (B B^T)^{-1} (y - G zc)
// (k_GW); the arithmetic of every row value equals k_B / k_G_apply.
template <typename RowValue>
__device__ inline void w_row(const int* __restrict__ bs, const int* __restrict__ bn, const int* __restrict__ bd,
                             int64_t r, double* __restrict__ z, const RowValue& val) {
    const int kind = bd[r];
    if (kind == 1) {
        z[r] = val(r);
        return;
    }
    if (kind == 2) return;
    const int s0 = bs[r], sz = bn[r];
    double sum = 0.0;
    for (int j = 0; j < sz; ++j) sum += val(s0 + j);
    z[r] = val(r) - sum / (sz + 1);
}

struct PlainVal {
    const double* y;
    __device__ double operator()(int64_t q) const { return y[q]; }
};

struct BVal {
    const int64_t* plus;
    const int64_t* minus;
    GlueRows gl;
    const double* x;
    const double* sc;
    __device__ double operator()(int64_t q) const { return 1.0 * b_row(plus, minus, gl, x, sc, q); }
};

struct GVal {
    const int* pp;
    const int* pm;
    const double* gp;
    const double* gm;
    const double* zc;
    const double* y;
    __device__ double operator()(int64_t q) const {
        const int a = pp[q], b = pm[q];
        double s = 0.0;
        for (int m = 0; m < 6; ++m) s += gp[q * 6 + m] * zc[a * 6 + m];
        if (b >= 0)
            for (int m = 0; m < 6; ++m) s -= gm[q * 6 + m] * zc[b * 6 + m];
        return 1.0 * y[q] + -1.0 * s;
    }
};

__global__ void k_W(const int* __restrict__ bs, const int* __restrict__ bn, const int* __restrict__ bd, int64_t n_c,
                    double* __restrict__ z, PlainVal val) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n_c) w_row(bs, bn, bd, r, z, val);
}

__global__ void k_BW(const int* __restrict__ bs, const int* __restrict__ bn, const int* __restrict__ bd, int64_t n_c,
                     double* __restrict__ z, BVal val) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n_c) w_row(bs, bn, bd, r, z, val);
}

__global__ void k_GW(const int* __restrict__ bs, const int* __restrict__ bn, const int* __restrict__ bd, int64_t n_c,
                     double* __restrict__ z, GVal val) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n_c) w_row(bs, bn, bd, r, z, val);
}

// dense blocks: the row values of every listed row (k_w_dense_val), then
// z_a = sum_c Minv[a][c] v_c per row, summed in a fixed order (k_w_dense_mv)
template <typename RowValue>
__global__ void __launch_bounds__(kBlock) k_w_dense_val(DenseBlocks db, RowValue val) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j < db.total) db.tmp[j] = val(db.rows[j]);
}

__global__ void __launch_bounds__(kBlock) k_w_dense_mv(DenseBlocks db, double* __restrict__ z) {
    // one wavefront per row: lane l sums the columns c = l (mod 64), then a
    // fixed butterfly adds the lanes' sums
    const int j = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (j >= db.total) return;
    const int b = db.blk[j];
    const int64_t b0 = db.ptr[b];
    const int n = (int)(db.ptr[b + 1] - b0), a = (int)(j - b0);
    const double* M = db.mat + db.moff[b] + (int64_t)a * n;
    const double* v = db.tmp + b0;
    double acc = 0.0;
    for (int c = lane; c < n; c += 64) acc += M[c] * v[c];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) z[db.rows[j]] = acc;
}

// f(integral_constant<int, dim>) for the dimension of a patch (uniform per
// workgroup): with the dimension and the mode index known at compile time the
// mode values reduce to selects (no branches per DOF and mode)
template <typename F>
__device__ inline void with_dim(int dim, F f) {
    if (dim == 3)
        f(std::integral_constant<int, 3>{});
    else
        f(std::integral_constant<int, 2>{});
}

// a chunk of patch DOFs as one thread sees it: kChunk / kBlock entries, with
// every load issued before any use
struct RigidRows {
    static_assert(kChunk % kBlock == 0, "whole rounds of a DOF chunk per thread");
    static constexpr int kIt = kChunk / kBlock;
    bool ok[kIt];
    int comp[kIt];
    double X[kIt][3];
    __device__ RigidRows(const DevPatch& pa, const Chunk& c, const double* __restrict__ ctrl) {
        const int nodes = (int)pa.nodes;
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int64_t i = c.begin + threadIdx.x + it * kBlock;
            ok[it] = i < c.end;
            const int loc = ok[it] ? (int)(i - pa.dof_off) : 0;
            comp[it] = loc / nodes;
            const double* P = ctrl + pa.ctrl_off + (int64_t)(loc - comp[it] * nodes) * 3;
#pragma unroll
            for (int a = 0; a < 3; ++a) X[it][a] = ok[it] ? P[a] : 0.0;
        }
    }
};

// partial sums of R^T x over chunks of one patch's DOFs
__global__ void __launch_bounds__(kBlock) k_rigid_partial(const DevPatch* __restrict__ dps, const Chunk* __restrict__ ch,
                                                          const double* __restrict__ ctrl, const double* __restrict__ x,
                                                          double* __restrict__ part) {
    __shared__ double lds[6 * 4];
    const Chunk c = ch[blockIdx.x];
    const DevPatch& pa = dps[c.seg];
    double v[RigidRows::kIt];
#pragma unroll
    for (int it = 0; it < RigidRows::kIt; ++it) {
        const int64_t i = c.begin + threadIdx.x + it * kBlock;
        v[it] = i < c.end ? x[i] : 0.0;
    }
    const RigidRows r(pa, c, ctrl);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    with_dim(pa.dim, [&](auto D) {
        constexpr int DIM = decltype(D)::value, NM = DIM == 3 ? 6 : 3;
#pragma unroll
        for (int it = 0; it < RigidRows::kIt; ++it)
#pragma unroll
            for (int m = 0; m < NM; ++m) acc[m] += rigid_mode_value(DIM, m, r.comp[it], r.X[it]) * v[it];
    });
    block_sum<6>(acc, lds);
    if (threadIdx.x == 0)
        for (int m = 0; m < 6; ++m) part[(int64_t)blockIdx.x * 6 + m] = acc[m];
}

// partial sums of G^T y over chunks of one patch's multiplier copies: copy e
// of row r adds y_r times its signed rigid-mode values (one copy per thread)
__global__ void __launch_bounds__(kBlock) k_gamma_partial(const Chunk* __restrict__ ch, const int* __restrict__ row,
                                                          const double* __restrict__ val, int64_t n_mc,
                                                          const double* __restrict__ y, double* __restrict__ part) {
    static_assert(kGamChunk == kBlock, "one multiplier copy per thread");
    __shared__ double lds[6 * 4];
    const Chunk c = ch[blockIdx.x];
    const int64_t e = c.begin + threadIdx.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    if (e < c.end) {
        const double v = y[row[e]];
#pragma unroll
        for (int m = 0; m < 6; ++m) acc[m] = val[m * n_mc + e] * v;
    }
    block_sum<6>(acc, lds);
    if (threadIdx.x == 0)
        for (int m = 0; m < 6; ++m) part[(int64_t)blockIdx.x * 6 + m] = acc[m];
}

// one block per patch: coef = (R^T R)^{-1} sum(partials)
__global__ void __launch_bounds__(kBlock) k_rigid_finalize(const int* __restrict__ cptr, const double* __restrict__ part,
                                                           const double* __restrict__ rtr, double* __restrict__ coef) {
    __shared__ double lds[6 * 4];
    const int k = blockIdx.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int c = cptr[k] + threadIdx.x; c < cptr[k + 1]; c += kBlock)
        for (int m = 0; m < 6; ++m) acc[m] += part[(int64_t)c * 6 + m];
    block_sum<6>(acc, lds);
    if (threadIdx.x == 0)
        for (int a = 0; a < 6; ++a) {
            double s = 0.0;
            for (int b = 0; b < 6; ++b) s += rtr[k * 36 + a * 6 + b] * acc[b];
            coef[k * 6 + a] = s;
        }
}

// one block per problem: g = sum of the partials per patch and mode (one
// wave per entry, lanes strided over the chunks, fixed shuffle tree),
// zc = (G^T G)^{-1} g, scattered to zc[patch * 6 + mode]; the slots of the
// modes a 2D patch does not have are set to zero (G_apply reads all six)
constexpr int kFinBlock = 1024;  // threads of the coarse finalisation (16 wavefronts)
constexpr int kFinSub = 16;      // lanes per row of the (G^T G)^{-1} product
constexpr int kFinRows = kFinBlock / kFinSub;  // product rows per pass

__global__ void __launch_bounds__(kFinBlock) k_coarse_finalize(const int* __restrict__ p0, const int* __restrict__ np,
                                                               const int* __restrict__ nmod,
                                                               const int64_t* __restrict__ coff,
                                                               const int* __restrict__ cptr,
                                                               const double* __restrict__ part,
                                                               const double* __restrict__ cinv,
                                                               double* __restrict__ zc) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* g = reinterpret_cast<double*>(smem);
    constexpr int NWV = kFinBlock / 64, U = 4;
    const int pr = blockIdx.x;
    const int nm = nmod[pr], npch = np[pr], patch0 = p0[pr];
    const int nc = nm * npch;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // U entries per wavefront at a time, so that their loads overlap
    for (int e0 = wave; e0 < nc; e0 += U * NWV) {
        double s[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * NWV;
            s[u] = 0.0;
            if (e < nc) {
                const int k = patch0 + e / nm, m = e % nm;
                for (int c = cptr[k] + lane; c < cptr[k + 1]; c += 64) s[u] += part[(int64_t)c * 6 + m];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double t = wave_sum(s[u]);
            if (lane == 0 && e0 + u * NWV < nc) g[e0 + u * NWV] = t;
        }
    }
    __syncthreads();
    // zc = C g: kFinSub lanes per row, partial sums over j = sub (mod kFinSub),
    // then a fixed butterfly over the kFinSub lanes
    const double* C = cinv + coff[pr];
    const int sub = threadIdx.x % kFinSub;
    for (int base = 0; base < nc; base += kFinRows) {
        const int e = base + threadIdx.x / kFinSub;
        double s = 0.0;
        if (e < nc)
            for (int j = sub; j < nc; j += kFinSub) s += C[(int64_t)e * nc + j] * g[j];
#pragma unroll
        for (int o = kFinSub / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (sub == 0 && e < nc) zc[(patch0 + e / nm) * 6 + e % nm] = s;
    }
    for (int e = threadIdx.x; e < npch * (6 - nm); e += kFinBlock)
        zc[(patch0 + e / (6 - nm)) * 6 + nm + e % (6 - nm)] = 0.0;
}

// The same on a grid (problem, row block), for coarse matrices of more than
// kFinRows rows: every block forms all of g (cheap) and kFinRows rows of the
// product, so that a large coarse matrix (64 patches: 384 x 384) is read by
// many CUs at once.  Loads are issued in batches before their sums; every
// sum keeps its order, so the result equals the one-block kernel's.
__global__ void __launch_bounds__(kFinBlock) k_coarse_finalize_rows(const int* __restrict__ p0, const int* __restrict__ np,
                                                                    const int* __restrict__ nmod,
                                                                    const int64_t* __restrict__ coff,
                                                                    const int* __restrict__ cptr,
                                                                    const double* __restrict__ part,
                                                                    const double* __restrict__ cinv,
                                                                    double* __restrict__ zc) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* g = reinterpret_cast<double*>(smem);
    constexpr int NWV = kFinBlock / 64, U = 8, KU = 8;
    const int pr = blockIdx.x;
    const int nm = nmod[pr], npch = np[pr], patch0 = p0[pr];
    const int nc = nm * npch;
    const int rbase = blockIdx.y * kFinRows;
    if (rbase >= nc) return;  // (uniform over the block)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // U entries per wavefront at a time; each lane's first chunk of every
    // entry is loaded before any sum
    for (int e0 = wave; e0 < nc; e0 += U * NWV) {
        double s[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * NWV;
            s[u] = 0.0;
            if (e < nc) {
                const int k = patch0 + e / nm, m = e % nm;
                const int c = cptr[k] + lane;
                if (c < cptr[k + 1]) s[u] = 0.0 + part[(int64_t)c * 6 + m];  // (as a sum from zero)
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * NWV;
            if (e < nc) {  // more than 64 chunks in a patch: the rest, in order
                const int k = patch0 + e / nm, m = e % nm;
                for (int c = cptr[k] + lane + 64; c < cptr[k + 1]; c += 64) s[u] += part[(int64_t)c * 6 + m];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double t = wave_sum(s[u]);
            if (lane == 0 && e0 + u * NWV < nc) g[e0 + u * NWV] = t;
        }
    }
    __syncthreads();
    // zc = C g: kFinSub lanes per row, partial sums over j = sub (mod kFinSub)
    // in ascending j, then a fixed butterfly over the kFinSub lanes
    const int sub = threadIdx.x % kFinSub;
    const int e = rbase + threadIdx.x / kFinSub;
    double acc = 0.0;
    if (e < nc) {
        const double* Ce = cinv + coff[pr] + (int64_t)e * nc;
        for (int j = sub; j < nc; j += KU * kFinSub) {
            double cv[KU];
#pragma unroll
            for (int u = 0; u < KU; ++u) cv[u] = j + u * kFinSub < nc ? Ce[j + u * kFinSub] : 0.0;
#pragma unroll
            for (int u = 0; u < KU; ++u)
                if (j + u * kFinSub < nc) acc += cv[u] * g[j + u * kFinSub];
        }
    }
#pragma unroll
    for (int o = kFinSub / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (sub == 0 && e < nc) zc[(patch0 + e / nm) * 6 + e % nm] = acc;
    if (blockIdx.y == 0)
        for (int t = threadIdx.x; t < npch * (6 - nm); t += kFinBlock)
            zc[(patch0 + t / (6 - nm)) * 6 + nm + t % (6 - nm)] = 0.0;
}

// y = x - R coef over chunks of patch DOFs
__global__ void __launch_bounds__(kBlock) k_rigid_update(const DevPatch* __restrict__ dps, const Chunk* __restrict__ ch,
                                                         const double* __restrict__ ctrl, const double* __restrict__ coef,
                                                         const double* __restrict__ x, double* __restrict__ y) {
    const Chunk c = ch[blockIdx.x];
    const DevPatch& pa = dps[c.seg];
    double v[RigidRows::kIt];
#pragma unroll
    for (int it = 0; it < RigidRows::kIt; ++it) {
        const int64_t i = c.begin + threadIdx.x + it * kBlock;
        v[it] = i < c.end ? x[i] : 0.0;
    }
    const RigidRows r(pa, c, ctrl);
    double cf[6];
    for (int m = 0; m < 6; ++m) cf[m] = coef[c.seg * 6 + m];
    with_dim(pa.dim, [&](auto D) {
        constexpr int DIM = decltype(D)::value, NM = DIM == 3 ? 6 : 3;
#pragma unroll
        for (int it = 0; it < RigidRows::kIt; ++it) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < NM; ++m) s += rigid_mode_value(DIM, m, r.comp[it], r.X[it]) * cf[m];
            if (r.ok[it]) y[c.begin + threadIdx.x + it * kBlock] = v[it] - s;
        }
    });
}

// y[r] = beta x[r] + alpha (G zc)[r],  G row = R(plus copy) - R(minus copy)
__global__ void k_G_apply(const int* __restrict__ pp, const int* __restrict__ pm, const double* __restrict__ gp,
                          const double* __restrict__ gm, int64_t n_c, const double* __restrict__ zc, double alpha,
                          double beta, const double* __restrict__ x, double* __restrict__ y) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_c) return;
    const int a = pp[r], b = pm[r];
    double s = 0.0;
    for (int m = 0; m < 6; ++m) s += gp[r * 6 + m] * zc[a * 6 + m];
    if (b >= 0)
        for (int m = 0; m < 6; ++m) s -= gm[r * 6 + m] * zc[b * 6 + m];
    y[r] = (x ? beta * x[r] : 0.0) + alpha * s;
}

// ============================================================ vector kernels
__global__ void k_copy(const double* __restrict__ x, double* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i];
}
__global__ void k_mul(const double* __restrict__ a, const double* x, double* y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a[i] * x[i];
}
__global__ void k_fill(double* __restrict__ y, double v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = v;
}
__global__ void k_axpby(double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                        double* __restrict__ z, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = a * x[i] + b * y[i];
}

__global__ void __launch_bounds__(kBlock) k_dot_partial(const Chunk* __restrict__ ch, const double* __restrict__ x,
                                                        const double* __restrict__ y, double* __restrict__ part) {
    __shared__ double lds[4];
    const Chunk c = ch[blockIdx.x];
    double acc[1] = {0.0};
    for (int64_t i = c.begin + threadIdx.x; i < c.end; i += kBlock) acc[0] += x[i] * y[i];
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// sum of the chunk partials of problem blockIdx.x, in a fixed order; valid in thread 0
__device__ inline double block_chunk_sum(const int* cptr, const double* part, double* lds) {
    const int pr = blockIdx.x;
    double acc[1] = {0.0};
    for (int c = cptr[pr] + threadIdx.x; c < cptr[pr + 1]; c += kBlock) acc[0] += part[c];
    block_sum<1>(acc, lds);
    return acc[0];
}

__global__ void __launch_bounds__(kBlock) k_minres_init(MinresState* st, const int* cptr, const double* part,
                                                        double tol, int maxit) {
    __shared__ double lds[4];
    const double g2 = block_chunk_sum(cptr, part, lds);
    if (threadIdx.x != 0) return;
    MinresState s = {};
    s.tol = tol;
    s.maxit = maxit;
    s.gamma_old = 1.0;
    s.c = s.c_old = 1.0;
    s.s = s.s_old = 0.0;
    if (g2 < 0.0) {
        s.stop = 2;
    } else {
        s.gamma = sqrt(g2);
        s.gamma1 = s.gamma;
        s.eta = s.gamma;
        s.rel = s.gamma > 0 ? 1.0 : 0.0;
        s.stop = s.gamma > 0 ? 0 : 1;
    }
    s.skip = s.stop;
    st[blockIdx.x] = s;
}

// gamma_{j+1}, the Givens rotation and the d/x-update weights
__global__ void __launch_bounds__(kBlock) k_minres_givens(MinresState* st, const int* cptr, const double* part) {
    __shared__ double lds[4];
    const double g2 = block_chunk_sum(cptr, part, lds);
    if (threadIdx.x != 0) return;
    MinresState& s = st[blockIdx.x];
    if (s.stop) return;
    if (g2 < 0.0) {
        s.stop = 2;
        return;
    }
    const double gnew = sqrt(g2);
    const double a0 = s.c * s.delta - s.c_old * s.s * s.gamma;
    const double a1 = sqrt(a0 * a0 + gnew * gnew);
    const double a2 = s.s * s.delta + s.c_old * s.c * s.gamma;
    const double a3 = s.s_old * s.gamma;
    const double cn = a0 / a1, sn = gnew / a1;
    s.cd_z = 1.0 / (s.gamma * a1);
    s.cd_dold = -a3 / a1;
    s.cd_d = -a2 / a1;
    s.cx = cn * s.eta;
    s.eta = -sn * s.eta;
    s.its += 1;
    s.rel = fabs(s.eta) / s.gamma1;
    s.gamma_old = s.gamma;
    s.gamma = gnew;
    s.c_old = s.c;
    s.c = cn;
    s.s_old = s.s;
    s.s = sn;
    s.upd = 1;
    if (s.rel <= s.tol) s.stop = 1;
    else if (s.its >= s.maxit) s.stop = 3;
}

// delta_j = <A z_j, z_j> with z_j = zraw / gamma_j, the v-update weights and
// v_{j+1} in one launch: every block sums the chunk partials of its problem
// in the same fixed order (so all blocks hold the same delta), and the first
// block of the problem records delta and the weights in the state
__global__ void __launch_bounds__(kBlock) k_minres_dv(MinresState* __restrict__ st, const Chunk* __restrict__ ch,
                                                      const int* __restrict__ cptr, const double* __restrict__ part,
                                                      const double* __restrict__ q, const double* __restrict__ v,
                                                      const double* __restrict__ vo, double* __restrict__ vn) {
    __shared__ double lds[4];
    __shared__ double sum_s;
    const Chunk c = ch[blockIdx.x];
    const int pr = c.seg;
    MinresState& s = st[pr];
    const bool first = (int)blockIdx.x == cptr[pr];
    if (first && threadIdx.x == 0) {
        s.upd = 0;
        s.skip = s.stop;
    }
    if (s.stop) return;
    {
        double acc[1] = {0.0};
        for (int j = cptr[pr] + threadIdx.x; j < cptr[pr + 1]; j += kBlock) acc[0] += part[j];
        block_sum<1>(acc, lds);
        if (threadIdx.x == 0) sum_s = acc[0];
        __syncthreads();
    }
    const double g = s.gamma;
    const double delta = sum_s / (g * g);
    const double a = 1.0 / g, b = -delta / g, d = -g / s.gamma_old;
    if (first && threadIdx.x == 0) {
        s.delta = delta;
        s.cv_q = a;
        s.cv_v = b;
        s.cv_vold = d;
    }
    for (int64_t i = c.begin + threadIdx.x; i < c.end; i += kBlock) vn[i] = a * q[i] + b * v[i] + d * vo[i];
}

__global__ void __launch_bounds__(kBlock) k_minres_dx(const MinresState* __restrict__ st, const Chunk* __restrict__ ch,
                                                      const double* __restrict__ z, const double* __restrict__ dold,
                                                      const double* __restrict__ d, double* __restrict__ dn,
                                                      double* __restrict__ x) {
    const Chunk c = ch[blockIdx.x];
    const MinresState& s = st[c.seg];
    if (!s.upd) return;
    const double a = s.cd_z, b = s.cd_dold, e = s.cd_d, cx = s.cx;
    for (int64_t i = c.begin + threadIdx.x; i < c.end; i += kBlock) {
        const double v = a * z[i] + b * dold[i] + e * d[i];
        dn[i] = v;
        x[i] += cx * v;
    }
}

// zero the interior nodes (all indices strictly inside) of every patch/component
__global__ void __launch_bounds__(kBlock) k_mask_interior(const DevPatch* __restrict__ dps, const int4* __restrict__ rb,
                                                          double* __restrict__ y) {
    const int4 b = rb[blockIdx.x];
    const DevPatch& pa = dps[b.x];
    const int64_t node = (int64_t)b.z + threadIdx.x;
    if (node >= pa.nodes) return;
    const int n1 = pa.n[0], n2 = pa.n[1], n3 = pa.n[2];
    const int i1 = (int)(node % n1), i2 = (int)((node / n1) % n2), i3 = (int)(node / ((int64_t)n1 * n2));
    bool inner = i1 > 0 && i1 < n1 - 1 && i2 > 0 && i2 < n2 - 1;
    if (pa.dim == 3) inner = inner && i3 > 0 && i3 < n3 - 1;
    if (inner) y[pa.dof_off + (int64_t)b.y * pa.nodes + node] = 0.0;
}

template <int DIM, int P>
void stiffness_t(const DevPatch* dp, const int4* rb, int nrb, const double* A, const double* x, double* y,
                 const int64_t* bp, const int* br, const double* bs, const double* t, const MinresState* mask,
                 hipStream_t s) {
    hipLaunchKernelGGL((k_stiffness<DIM, P>), dim3(nrb), dim3(kBlock), 0, s, dp, rb, A, x, y, bp, br, bs, t, mask);
}

}  // namespace

// ====================================================== fixed scratch array
// FD intermediate tensor of afieti_apply_fd_noalloc: a file-scope device
// array, so that the entry point calls no allocator.  In host code its name
// is only a stand-in for the symbol: every host use goes through the device
// address that hipGetSymbolAddress returns for the current device, kept per
// device (each GPU holds its own copy of the array).
__device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};
}  // namespace

void* noalloc_scratch_acquire(hipError_t* err) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && (dev < 0 || dev >= kMaxDevices)) e = hipErrorInvalidDevice;
    if (e != hipSuccess) {
        if (err) *err = e;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            if (err) *err = e;
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    if (err) *err = hipSuccess;
    return g_scratch_ptr[dev];
}

void* noalloc_scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

// ======================================================== launch wrappers
void launch_fd(int prec, const FdTensor* tens, int n_tensors, const int2* slabs, int n_slabs, const int2* cols,
               int n_colblocks, const void* ut, const double* dt, const double* in, double* out, void* tmp,
               const MinresState* mask, const double* scale, hipStream_t s) {
    (void)n_tensors;
    if (n_slabs == 0) return;
    if (prec == 0) {
        const size_t sh12 = 3 * kMaxN * kMaxN * sizeof(double);
        const size_t sh3 = (2 * kMaxN * 32 + kMaxN * kMaxN) * sizeof(double);
        hipLaunchKernelGGL(k_fd_fwd12<double>, dim3(n_slabs), dim3(kFdBlock), sh12, s, tens, slabs,
                           (const double*)ut, in, (double*)tmp, mask, scale);
        hipLaunchKernelGGL(k_fd_mid3<double>, dim3(n_colblocks), dim3(kFdBlock), sh3, s, tens, cols,
                           (const double*)ut, dt, (double*)tmp, mask);
        hipLaunchKernelGGL(k_fd_bwd12<double>, dim3(n_slabs), dim3(kFdBlock), sh12, s, tens, slabs,
                           (const double*)ut, (const double*)tmp, out, mask, scale);
    } else {
        const size_t sh12 = 3 * kMaxN * kMaxN * sizeof(float);
        const size_t sh3 = (2 * kMaxN * 32 + kMaxN * kMaxN) * sizeof(float);
        hipLaunchKernelGGL(k_fd_fwd12<float>, dim3(n_slabs), dim3(kFdBlock), sh12, s, tens, slabs,
                           (const float*)ut, in, (float*)tmp, mask, scale);
        hipLaunchKernelGGL(k_fd_mid3<float>, dim3(n_colblocks), dim3(kFdBlock), sh3, s, tens, cols,
                           (const float*)ut, dt, (float*)tmp, mask);
        hipLaunchKernelGGL(k_fd_bwd12<float>, dim3(n_slabs), dim3(kFdBlock), sh12, s, tens, slabs,
                           (const float*)ut, (const float*)tmp, out, mask, scale);
    }
}

void launch_geometry(const DevPatch* dp, int k, const DevPatch& hp, const double* ctrl, const double* qval,
                     const double* qder, const int* qfirst, const double* qw, double* geo, hipStream_t s) {
    const int64_t n = (int64_t)hp.nq[0] * hp.nq[1] * hp.nq[2];
    if (hp.dim == 3)
        hipLaunchKernelGGL(k_geometry<3>, dim3(blocks_for(n)), dim3(kBlock), 0, s, dp, k, ctrl, qval, qder, qfirst, qw, geo);
    else
        hipLaunchKernelGGL(k_geometry<2>, dim3(blocks_for(n)), dim3(kBlock), 0, s, dp, k, ctrl, qval, qder, qfirst, qw, geo);
}

void launch_assemble(const DevPatch* dp, int k, const DevPatch& hp, const double* geo, const double* qval,
                     const double* qder, const int* qfirst, const int* el_first, const int* el_last, double* stencil,
                     double lam_w, double mu_w, hipStream_t s) {
    const int W = 2 * hp.p + 1;
    const int64_t S = hp.dim == 3 ? W * W * W : W * W;
    const int64_t n = S * hp.nodes;
    if (hp.dim == 3)
        hipLaunchKernelGGL(k_assemble<3>, dim3(blocks_for(n)), dim3(kBlock), 0, s, dp, k, geo, qval, qder, qfirst,
                           el_first, el_last, stencil, lam_w, mu_w);
    else
        hipLaunchKernelGGL(k_assemble<2>, dim3(blocks_for(n)), dim3(kBlock), 0, s, dp, k, geo, qval, qder, qfirst,
                           el_first, el_last, stencil, lam_w, mu_w);
}

void launch_load(const DevPatch* dp, int k, const DevPatch& hp, const double* geo, const double* qval,
                 const int* qfirst, const int* el_first, const int* el_last, const double* modes, int n_modes,
                 double* f, int64_t f_base, hipStream_t s) {
    if (hp.dim == 3)
        hipLaunchKernelGGL(k_load<3>, dim3(blocks_for(hp.nodes)), dim3(kBlock), 0, s, dp, k, geo, qval, qfirst,
                           el_first, el_last, modes, n_modes, f, f_base);
    else
        hipLaunchKernelGGL(k_load<2>, dim3(blocks_for(hp.nodes)), dim3(kBlock), 0, s, dp, k, geo, qval, qfirst,
                           el_first, el_last, modes, n_modes, f, f_base);
}

void launch_mass(const DevPatch* dp, int k, const DevPatch& hp, const double* geo, const double* qval,
                 const int* qfirst, const int* el_first, const int* el_last, const double* x, double* qbuf,
                 double* y, hipStream_t s) {
    const int64_t nq = (int64_t)hp.nq[0] * hp.nq[1] * hp.nq[2];
    if (hp.dim == 3) {
        hipLaunchKernelGGL(k_field_qp<3>, dim3(blocks_for(nq)), dim3(kBlock), 0, s, dp, k, geo, qval, qfirst, x, qbuf);
        hipLaunchKernelGGL(k_mass_gather<3>, dim3(blocks_for(hp.nodes)), dim3(kBlock), 0, s, dp, k, qval, qfirst,
                           el_first, el_last, qbuf, y);
    } else {
        hipLaunchKernelGGL(k_field_qp<2>, dim3(blocks_for(nq)), dim3(kBlock), 0, s, dp, k, geo, qval, qfirst, x, qbuf);
        hipLaunchKernelGGL(k_mass_gather<2>, dim3(blocks_for(hp.nodes)), dim3(kBlock), 0, s, dp, k, qval, qfirst,
                           el_first, el_last, qbuf, y);
    }
}

int launch_energy(const DevPatch* dp, int k, const DevPatch& hp, const double* geo, const double* qval,
                  const double* qder, const int* qfirst, const double* u, const double* psi, double* part,
                  hipStream_t s) {
    const int64_t nq = (int64_t)hp.nq[0] * hp.nq[1] * hp.nq[2];
    const unsigned nb = blocks_for(nq);
    if (hp.dim == 3)
        hipLaunchKernelGGL(k_energy<3>, dim3(nb), dim3(kBlock), 0, s, dp, k, geo, qval, qder, qfirst, u, psi, part);
    else
        hipLaunchKernelGGL(k_energy<2>, dim3(nb), dim3(kBlock), 0, s, dp, k, geo, qval, qder, qfirst, u, psi, part);
    return (int)nb;
}

int launch_mdot(const double* F, int64_t n, int n_modes, int64_t off, const double* psi, double* part,
                hipStream_t s) {
    const unsigned nch = blocks_for(n, kChunk);
    if (n_modes > 0 && n > 0)
        hipLaunchKernelGGL(k_mdot_partial, dim3(nch, n_modes), dim3(kBlock), 0, s, F, n, off, psi, part);
    return (int)nch;
}

#define AFIETI_DISPATCH_P(DIM, FN, ...)            \
    switch (p) {                                   \
        case 1: FN<DIM, 1>(__VA_ARGS__); break;     \
        case 2: FN<DIM, 2>(__VA_ARGS__); break;     \
        case 3: FN<DIM, 3>(__VA_ARGS__); break;     \
        case 4: FN<DIM, 4>(__VA_ARGS__); break;     \
        case 5: FN<DIM, 5>(__VA_ARGS__); break;     \
        case 6: FN<DIM, 6>(__VA_ARGS__); break;     \
        case 7: FN<DIM, 7>(__VA_ARGS__); break;     \
        default: FN<DIM, 8>(__VA_ARGS__); break;    \
    }

void launch_stiffness_dp(int dim, int p, const DevPatch* dp, const int4* rb, int nrb, const double* A,
                         const double* x, double* y, const int64_t* bp, const int* br, const double* bs,
                         const double* t, const MinresState* mask, hipStream_t s) {
    if (nrb == 0) return;
    if (dim == 3) {
        AFIETI_DISPATCH_P(3, stiffness_t, dp, rb, nrb, A, x, y, bp, br, bs, t, mask, s)
    } else {
        AFIETI_DISPATCH_P(2, stiffness_t, dp, rb, nrb, A, x, y, bp, br, bs, t, mask, s)
    }
}

void launch_ahat(int p, const DevPatch* dp, const int4* slabs, int n_slabs, int max_n12, int max_n1n2, const double* kb,
                 const double* mb, const double* x, double* y, int use_h, int bnd_in, int bnd_out,
                 const MinresState* mask, hipStream_t s) {
    switch (p) {
        case 1: ahat_t<1>(dp, slabs, n_slabs, max_n12, max_n1n2, kb, mb, x, y, use_h, bnd_in, bnd_out, mask, s); break;
        case 2: ahat_t<2>(dp, slabs, n_slabs, max_n12, max_n1n2, kb, mb, x, y, use_h, bnd_in, bnd_out, mask, s); break;
        case 3: ahat_t<3>(dp, slabs, n_slabs, max_n12, max_n1n2, kb, mb, x, y, use_h, bnd_in, bnd_out, mask, s); break;
        case 4: ahat_t<4>(dp, slabs, n_slabs, max_n12, max_n1n2, kb, mb, x, y, use_h, bnd_in, bnd_out, mask, s); break;
        case 5: ahat_t<5>(dp, slabs, n_slabs, max_n12, max_n1n2, kb, mb, x, y, use_h, bnd_in, bnd_out, mask, s); break;
        case 6: ahat_t<6>(dp, slabs, n_slabs, max_n12, max_n1n2, kb, mb, x, y, use_h, bnd_in, bnd_out, mask, s); break;
        default: ahat_t<0>(dp, slabs, n_slabs, max_n12, max_n1n2, kb, mb, x, y, use_h, bnd_in, bnd_out, mask, s); break;
    }
}

void launch_mask_interior(const DevPatch* dp, const int4* rb, int nrb, double* y, hipStream_t s) {
    if (nrb) hipLaunchKernelGGL(k_mask_interior, dim3(nrb), dim3(kBlock), 0, s, dp, rb, y);
}

void launch_mf_bricks(int p, const DevPatch* dp, const int4* bricks, int n_bricks, const double* tab,
                      const double* x, double* ybuf, const MinresState* mask, hipStream_t s) {
    if (n_bricks == 0) return;
    switch (p) {
        case 1: mf_bricks_t<1>(dp, bricks, n_bricks, tab, x, ybuf, mask, s); break;
        case 2: mf_bricks_t<2>(dp, bricks, n_bricks, tab, x, ybuf, mask, s); break;
        case 3: mf_bricks_t<3>(dp, bricks, n_bricks, tab, x, ybuf, mask, s); break;
        case 4: mf_bricks_t<4>(dp, bricks, n_bricks, tab, x, ybuf, mask, s); break;
        case 5: mf_bricks_t<5>(dp, bricks, n_bricks, tab, x, ybuf, mask, s); break;
        default: mf_bricks_t<6>(dp, bricks, n_bricks, tab, x, ybuf, mask, s); break;
    }
}

void launch_mf_gather(int p, const DevPatch* dp, const int4* rb, int nrb, const double* ybuf, double* y,
                      const int64_t* bp, const int* br, const double* bs, const double* t, const MinresState* mask,
                      hipStream_t s) {
    if (nrb == 0) return;
    switch (p) {
        case 1: mf_gather_t<1>(dp, rb, nrb, ybuf, y, bp, br, bs, t, mask, s); break;
        case 2: mf_gather_t<2>(dp, rb, nrb, ybuf, y, bp, br, bs, t, mask, s); break;
        case 3: mf_gather_t<3>(dp, rb, nrb, ybuf, y, bp, br, bs, t, mask, s); break;
        case 4: mf_gather_t<4>(dp, rb, nrb, ybuf, y, bp, br, bs, t, mask, s); break;
        case 5: mf_gather_t<5>(dp, rb, nrb, ybuf, y, bp, br, bs, t, mask, s); break;
        default: mf_gather_t<6>(dp, rb, nrb, ybuf, y, bp, br, bs, t, mask, s); break;
    }
}

int mf_brick_elems(int p) { return p <= 4 ? 2 : 1; }

int mf_table_doubles(int p) {
    const int be = mf_brick_elems(p), nb = be + p, qb = be * (p + 1);
    return 2 * qb * nb + 2 * qb;
}

void launch_B(const int64_t* plus, const int64_t* minus, const GlueRows& glue, int64_t n_c, double alpha,
              const double* x, double* y, hipStream_t s, const double* in_scale) {
    if (n_c)
        hipLaunchKernelGGL(k_B, dim3(blocks_for(n_c)), dim3(kBlock), 0, s, plus, minus, glue, n_c, alpha, x, y,
                           in_scale);
}

void launch_Bt(const int64_t* bt_ptr, const int* bt_row, const double* bt_sign, int64_t n_dof, const double* x,
               double* y, hipStream_t s, const double* out_scale) {
    hipLaunchKernelGGL(k_Bt, dim3(blocks_for(n_dof)), dim3(kBlock), 0, s, bt_ptr, bt_row, bt_sign, n_dof, x, y,
                       out_scale);
}

template <typename RowValue>
void w_launch(void (*rows)(const int*, const int*, const int*, int64_t, double*, RowValue), const int* bs,
              const int* bn, const int* bd, const DenseBlocks& db, int64_t n_c, double* z, const RowValue& val,
              hipStream_t s) {
    if (!n_c) return;
    hipLaunchKernelGGL(rows, dim3(blocks_for(n_c)), dim3(kBlock), 0, s, bs, bn, bd, n_c, z, val);
    if (db.n) {
        hipLaunchKernelGGL(k_w_dense_val<RowValue>, dim3(blocks_for(db.total)), dim3(kBlock), 0, s, db, val);
        hipLaunchKernelGGL(k_w_dense_mv, dim3(blocks_for(db.total, kBlock / 64)), dim3(kBlock), 0, s, db, z);
    }
}

void launch_W(const int* bs, const int* bn, const int* bd, const DenseBlocks& db, int64_t n_c, const double* y,
              double* z, hipStream_t s) {
    w_launch(k_W, bs, bn, bd, db, n_c, z, PlainVal{y}, s);
}

void launch_BW(const int* bs, const int* bn, const int* bd, const DenseBlocks& db, int64_t n_c, const int64_t* plus,
               const int64_t* minus, const GlueRows& glue, const double* x, double* z, hipStream_t s,
               const double* in_scale) {
    w_launch(k_BW, bs, bn, bd, db, n_c, z, BVal{plus, minus, glue, x, in_scale}, s);
}

void launch_GW(const int* bs, const int* bn, const int* bd, const DenseBlocks& db, int64_t n_c, const int* pp,
               const int* pm, const double* gp, const double* gm, const double* zc, const double* y, double* z,
               hipStream_t s) {
    w_launch(k_GW, bs, bn, bd, db, n_c, z, GVal{pp, pm, gp, gm, zc, y}, s);
}

void launch_rigid_partial(const DevPatch* dp, const Chunk* chunks, int n_chunks, const double* ctrl, const double* x,
                          double* partials, hipStream_t s) {
    if (n_chunks) hipLaunchKernelGGL(k_rigid_partial, dim3(n_chunks), dim3(kBlock), 0, s, dp, chunks, ctrl, x, partials);
}

void launch_gamma_partial(const Chunk* chunks, int n_chunks, const int* mc_row, const double* mc_val, int64_t n_mc,
                          const double* y, double* partials, hipStream_t s) {
    if (n_chunks)
        hipLaunchKernelGGL(k_gamma_partial, dim3(n_chunks), dim3(kBlock), 0, s, chunks, mc_row, mc_val, n_mc, y,
                           partials);
}

void launch_coarse_finalize(const int* p0, const int* np, const int* nm, const int64_t* coff, int n_probs,
                            const int* cptr, const double* partials, const double* Cinv, double* zc, int max_nc,
                            hipStream_t s) {
    // (one block per problem while the coarse matrices fit one pass of rows)
    if (max_nc <= kFinRows)
        hipLaunchKernelGGL(k_coarse_finalize, dim3(n_probs), dim3(kFinBlock), max_nc * sizeof(double), s, p0, np,
                           nm, coff, cptr, partials, Cinv, zc);
    else
        hipLaunchKernelGGL(k_coarse_finalize_rows, dim3(n_probs, (max_nc + kFinRows - 1) / kFinRows),
                           dim3(kFinBlock), max_nc * sizeof(double), s, p0, np, nm, coff, cptr, partials, Cinv, zc);
}

void launch_rigid_finalize(const int* cptr, int n_patches, const double* partials, const double* RtR_inv,
                           double* coef, hipStream_t s) {
    hipLaunchKernelGGL(k_rigid_finalize, dim3(n_patches), dim3(kBlock), 0, s, cptr, partials, RtR_inv, coef);
}

void launch_rigid_update(const DevPatch* dp, const Chunk* chunks, int n_chunks, const double* ctrl, const double* coef,
                         const double* x, double* y, hipStream_t s) {
    if (n_chunks) hipLaunchKernelGGL(k_rigid_update, dim3(n_chunks), dim3(kBlock), 0, s, dp, chunks, ctrl, coef, x, y);
}

void launch_G_apply(const int* pp, const int* pm, const double* gp, const double* gm, int64_t n_c, const double* zc,
                    double alpha, double beta, const double* x, double* y, hipStream_t s) {
    if (n_c)
        hipLaunchKernelGGL(k_G_apply, dim3(blocks_for(n_c)), dim3(kBlock), 0, s, pp, pm, gp, gm, n_c, zc, alpha, beta, x, y);
}

void launch_copy(const double* x, double* y, int64_t n, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_copy, dim3(blocks_for(n)), dim3(kBlock), 0, s, x, y, n);
}
void launch_mul(const double* a, const double* x, double* y, int64_t n, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_mul, dim3(blocks_for(n)), dim3(kBlock), 0, s, a, x, y, n);
}
void launch_fill(double* y, double v, int64_t n, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(kBlock), 0, s, y, v, n);
}
void launch_axpby(double a, const double* x, double b, const double* y, double* z, int64_t n, hipStream_t s) {
    if (n) hipLaunchKernelGGL(k_axpby, dim3(blocks_for(n)), dim3(kBlock), 0, s, a, x, b, y, z, n);
}
void launch_dot_partial(const Chunk* chunks, int n_chunks, const double* x, const double* y, double* partials,
                        hipStream_t s) {
    if (n_chunks) hipLaunchKernelGGL(k_dot_partial, dim3(n_chunks), dim3(kBlock), 0, s, chunks, x, y, partials);
}
void launch_minres_init(MinresState* st, const int* cptr, int n, const double* part, double tol, int maxit,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_minres_init, dim3(n), dim3(kBlock), 0, s, st, cptr, part, tol, maxit);
}
void launch_minres_givens(MinresState* st, const int* cptr, int n, const double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_minres_givens, dim3(n), dim3(kBlock), 0, s, st, cptr, part);
}
void launch_minres_dv(MinresState* st, const Chunk* chunks, int n_chunks, const int* cptr, const double* part,
                      const double* q, const double* v, const double* v_old, double* v_new, hipStream_t s) {
    if (n_chunks)
        hipLaunchKernelGGL(k_minres_dv, dim3(n_chunks), dim3(kBlock), 0, s, st, chunks, cptr, part, q, v, v_old, v_new);
}

void launch_minres_dx(const MinresState* st, const Chunk* chunks, int n_chunks, const double* z, const double* d_old,
                      const double* d, double* d_new, double* x, hipStream_t s) {
    if (n_chunks) hipLaunchKernelGGL(k_minres_dx, dim3(n_chunks), dim3(kBlock), 0, s, st, chunks, z, d_old, d, d_new, x);
}

}  // namespace afieti
