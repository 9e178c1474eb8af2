// Fast Diagonalization (Section 5.2.1, Algorithm 1) on the matrix cores of
// gfx950: for each patch, the d component tensors r_c (sizes n1 x n2 x n3)
// are transformed together, since they share the univariate generalised
// eigenvectors U_1, U_2, U_3:
//   pass 1 (per slab i3):      Z = U_2^T (X U_1) for every component,
//   pass 2 (per column block): W = U_3 ((U_3^T Z) / Lambda),
//   pass 3 (per slab i3):      out = alpha U_2 (W U_1^T).
// Each slab product is a small GEMM whose long side stacks the components
// (rows (c, i2) in the first product, columns (c, a1) in the second), so
// only the short side is padded to the 16-wide tile of v_mfma_*_16x16x4.
// The depth is a compile-time extent KM (28, 36 or 48, the smallest that
// holds the set's largest n), zero past n, so that operand reads and the
// chain of matrix instructions are straight-line code.  A wavefront
// computes a strip of tiles that shares one operand (a row of tiles with
// one A, or a column with one B), which cuts the LDS reads per matrix
// instruction from 2 to 1 + 1/3.  The intermediate tensor between passes is
// FP32 (FP64 for the FP64 mode).
//
// Every output element is a sum over the depth in the same order in every
// launch shape (K steps ascending), so the shapes the autotuner picks from
// (components per workgroup, mode-3 column block) and the depth extent give
// bitwise identical results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "device.h"
#include "kernels.h"

namespace afieti {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kFdWaves = 8;  // wavefronts per workgroup
constexpr int kFdThreads = 64 * kFdWaves;

// MODE 0: FP32 operands (v_mfma_f32_16x16x4_f32), 1: BF16 operands
// (v_mfma_f32_16x16x32_bf16), 2: FP64 (v_mfma_f64_16x16x4_f64).  Lane l of a
// wave holds A(row l % 16, k-group l / 16), B(k-group l / 16, column l % 16);
// result row of accumulator q in lane group g: 4 g + q (FP32 accumulators)
// or g + 4 q (FP64 accumulators), column l % 16.
template <int MODE>
struct Mf {
    static constexpr int KSTEP = MODE == 1 ? 32 : 4;
    using T = typename std::conditional<MODE == 0, float, typename std::conditional<MODE == 1, __bf16, double>::type>::type;
    using Acc = typename std::conditional<MODE == 2, doublex4, floatx4>::type;
    using Tmp = typename std::conditional<MODE == 2, double, float>::type;  // between passes
    using U = typename std::conditional<MODE == 2, double, float>::type;    // eigenvector table
    __device__ static inline int row(int g, int q) { return MODE == 2 ? g + 4 * q : 4 * g + q; }
};

// Depth extent KM of a launch: K = KM rounded up to the instruction depth,
// KS instructions per tile, NTU tiles of 16 covering n <= KM, E the side of
// the staged eigenvector blocks (and the row extent of the arrays a
// product reads along its depth).
template <int MODE, int KM>
struct Dep {
    static constexpr int K = (KM + Mf<MODE>::KSTEP - 1) / Mf<MODE>::KSTEP * Mf<MODE>::KSTEP;
    static constexpr int KS = K / Mf<MODE>::KSTEP;
    static constexpr int NTU = (KM + 15) / 16;
    static constexpr int E = K > 16 * NTU ? K : 16 * NTU;
    static constexpr int LD = E + (MODE == 1 ? 8 : 1);  // odd (FP32/FP64): rows spread over the banks
};

__host__ __device__ inline int pad16(int n) { return (n + 15) & ~15; }

// LDS layouts (element offsets), identical on the host (sizing) and device.
struct Pass12Layout {  // passes 1 and 3
    int RP, LDA, LDU, LDY;
    int oU1, oY, oU2, total;
};
template <int MODE, int KM>
__host__ __device__ inline Pass12Layout pass12_layout(int n1, int n2, int nc) {
    using D = Dep<MODE, KM>;
    Pass12Layout L;
    L.RP = pad16(nc * n2);           // rows (c, i2) x depth
    L.LDA = D::LD;
    L.LDU = D::LD;
    L.LDY = pad16(nc * n1) + 4;      // depth rows x stacked columns
    L.oU1 = L.RP * L.LDA;
    L.oY = L.oU1 + D::E * L.LDU;
    L.oU2 = L.oY + D::E * L.LDY;
    L.total = L.oU2 + D::E * L.LDU;
    return L;
}
struct Pass3Layout {  // pass 2 (the mode-3 pass)
    int LDZ, LDU, oZt, oU, total;
};
template <int MODE, int KM>
__host__ __device__ inline Pass3Layout mid_layout(int ncb) {
    using D = Dep<MODE, KM>;
    Pass3Layout L;
    L.LDZ = ncb + 4;
    L.LDU = D::LD;
    L.oZt = D::E * L.LDZ;
    L.oU = L.oZt + D::E * L.LDZ;
    L.total = L.oU + D::E * L.LDU;
    return L;
}

template <typename T, typename S>
__device__ inline T cvt(S v) {
    if constexpr (std::is_same<T, __bf16>::value) return (T)(float)v;
    else return (T)v;
}

// Buffer resource over [base, base + bytes): raw buffer loads at an offset
// at or past the end return zero, so padded tiles are staged without
// branches (an invalid element gets the offset kOob).
constexpr uint32_t kOob = 0xffffffffu;
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* base, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename V>
__device__ inline V bload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    if constexpr (sizeof(V) == 8) return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    else return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// dst[i * ld + j] = load(roff(i) + coff(j)), the element at that byte
// offset of a buffer (V typed; a kOob row or column gives zero), for
// i < rows, j < cols.  Wavefront w stages rows w, w + NW, ... (the row part
// of the address is uniform over the wavefront); lane l takes columns l,
// l + 64, ... (cols <= 64 CPL), the column part computed once per lane.  A
// thread issues the loads of CH rows before it stores any of them.
template <int NW, int CPL, typename V, typename T, typename RowOff, typename ColOff, typename Load>
__device__ inline void stage_with(T* dst, int ld, int rows, int cols, RowOff roff, ColOff coff, Load load) {
    constexpr int CH = 8 / CPL;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    uint32_t co[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        const int j = lane + 64 * q;
        co[q] = j < cols ? coff(j) : kOob;
    }
    for (int i0 = wave; i0 < rows; i0 += NW * CH) {
        V v[CH][CPL];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int i = i0 + u * NW;
            const uint32_t ro = i < rows ? roff(i) : kOob;
#pragma unroll
            for (int q = 0; q < CPL; ++q) v[u][q] = load((ro == kOob || co[q] == kOob) ? kOob : ro + co[q]);
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int i = i0 + u * NW;
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                const int j = lane + 64 * q;
                if (i < rows && j < cols) dst[i * ld + j] = cvt<T>(v[u][q]);
            }
        }
    }
}

// the elements of buffer r
template <int NW, int CPL, typename V, typename T, typename RowOff, typename ColOff>
__device__ inline void stage(T* dst, int ld, int rows, int cols, __amdgpu_buffer_rsrc_t r, RowOff roff,
                             ColOff coff) {
    stage_with<NW, CPL, V>(dst, ld, rows, cols, roff, coff, [&](uint32_t o) { return bload<V>(r, o); });
}

// operand of step s: A(m0 + r, k) (Tr: stored [k][m]) or B(k, n0 + r) (Tr:
// stored [n][k]); FP32/FP64 one value per lane, BF16 eight (k-group g)
template <int MODE, bool Tr>
__device__ inline auto opnd_a(const typename Mf<MODE>::T* __restrict__ a, int lda, int m0, int s) {
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    if constexpr (MODE != 1) {
        const int k = 4 * s + g;
        return Tr ? a[k * lda + m0 + r] : a[(m0 + r) * lda + k];
    } else {
        bf16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 32 * s + 8 * g + e;
            v[e] = Tr ? a[k * lda + m0 + r] : a[(m0 + r) * lda + k];
        }
        return v;
    }
}
template <int MODE, bool Tr>
__device__ inline auto opnd_b(const typename Mf<MODE>::T* __restrict__ b, int ldb, int n0, int s) {
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    if constexpr (MODE != 1) {
        const int k = 4 * s + g;
        return Tr ? b[(n0 + r) * ldb + k] : b[k * ldb + n0 + r];
    } else {
        bf16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 32 * s + 8 * g + e;
            v[e] = Tr ? b[(n0 + r) * ldb + k] : b[k * ldb + n0 + r];
        }
        return v;
    }
}
template <int MODE, typename V>
__device__ inline typename Mf<MODE>::Acc mfma(V a, V b, typename Mf<MODE>::Acc c) {
    if constexpr (MODE == 0) return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    else if constexpr (MODE == 1) return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// A row strip: tiles (m0, 16 j) for j < NT sharing the A operand
template <int MODE, int KS, int NT, bool At, bool Bt>
__device__ inline void strip_row(const typename Mf<MODE>::T* __restrict__ a, int lda,
                                 const typename Mf<MODE>::T* __restrict__ b, int ldb, int m0,
                                 typename Mf<MODE>::Acc (&acc)[NT]) {
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = typename Mf<MODE>::Acc{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const auto av = opnd_a<MODE, At>(a, lda, m0, s);
        decltype(opnd_b<MODE, Bt>(b, ldb, 0, s)) bv[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) bv[j] = opnd_b<MODE, Bt>(b, ldb, 16 * j, s);
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[j] = mfma<MODE>(av, bv[j], acc[j]);
    }
}
// A column strip: tiles (16 i, n0) for i < NT sharing the B operand
template <int MODE, int KS, int NT, bool At, bool Bt>
__device__ inline void strip_col(const typename Mf<MODE>::T* __restrict__ a, int lda,
                                 const typename Mf<MODE>::T* __restrict__ b, int ldb, int n0,
                                 typename Mf<MODE>::Acc (&acc)[NT]) {
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[i] = typename Mf<MODE>::Acc{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const auto bv = opnd_b<MODE, Bt>(b, ldb, n0, s);
        decltype(opnd_a<MODE, At>(a, lda, 0, s)) av[NT];
#pragma unroll
        for (int i = 0; i < NT; ++i) av[i] = opnd_a<MODE, At>(a, lda, 16 * i, s);
#pragma unroll
        for (int i = 0; i < NT; ++i) acc[i] = mfma<MODE>(av[i], bv, acc[i]);
    }
}

// stage U (n x n, U[i * n + a]) into an E x E block (zero outside n x n)
template <int MODE, int KM>
__device__ inline void stage_u(typename Mf<MODE>::T* dst, const typename Mf<MODE>::U* __restrict__ u, int n) {
    using U = typename Mf<MODE>::U;
    using D = Dep<MODE, KM>;
    stage<kFdWaves, (D::E + 63) / 64, U>(dst, D::LD, D::E, D::E, rsrc(u, (int64_t)n * n * sizeof(U)),
                                         [&](int i) { return i < n ? (uint32_t)(i * n * sizeof(U)) : kOob; },
                                         [&](int a) { return a < n ? (uint32_t)(a * sizeof(U)) : kOob; });
}

// ---------------------------------------------------------------- pass 1
// per (group, slab i3): Y[(c, i2)][a1] = sum_i1 X[(c, i2)][i1] U1[i1][a1];
// Z[a2][(c, a1)] = sum_i2 U2[i2][a2] Y[i2][(c, a1)]  -> tmp
template <int MODE, int KM>
__global__ void __launch_bounds__(kFdThreads) k_fdg_fwd(const FdGroup* __restrict__ groups,
                                                        const int2* __restrict__ slabs,
                                                        const typename Mf<MODE>::U* __restrict__ ut,
                                                        const double* __restrict__ in,
                                                        typename Mf<MODE>::Tmp* __restrict__ tmp,
                                                        const MinresState* __restrict__ mask,
                                                        const double* __restrict__ scale) {
    using M = Mf<MODE>;
    using T = typename M::T;
    using D = Dep<MODE, KM>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 it = slabs[blockIdx.x];
    const FdGroup& G = groups[it.x];
    if (mask && mask[G.prob].skip) return;
    const int i3 = it.y, n1 = G.n1, n2 = G.n2, nc = G.nc;
    const Pass12Layout L = pass12_layout<MODE, KM>(n1, n2, nc);
    T* XA = reinterpret_cast<T*>(smem);
    T* U1 = XA + L.oU1;
    T* YB = XA + L.oY;
    T* U2 = XA + L.oU2;
    const int R = nc * n2, C = nc * n1;
    // the slab of every component: rows (c, i2), columns i1 (times the
    // per-DOF scale, at the same offsets of its vector, when given)
    const int64_t span = (int64_t)(nc - 1) * G.cstride + (int64_t)(n2 - 1) * G.s2 + n1;
    const int64_t first = G.in_off + (int64_t)i3 * G.s3;
    const auto roff = [&](int r) {
        const int c = r / n2, i2 = r - c * n2;
        return r < R ? (uint32_t)((c * G.cstride + (int64_t)i2 * G.s2) * 8) : kOob;
    };
    const auto coff = [&](int k) { return k < n1 ? (uint32_t)(k * 8) : kOob; };
    const __amdgpu_buffer_rsrc_t rx = rsrc(in + first, span * 8);
    if (scale) {
        const __amdgpu_buffer_rsrc_t rs = rsrc(scale + first, span * 8);
        stage_with<kFdWaves, (D::K + 63) / 64, double>(XA, L.LDA, L.RP, D::K, roff, coff, [&](uint32_t o) {
            return bload<double>(rx, o) * bload<double>(rs, o);
        });
    } else {
        stage<kFdWaves, (D::K + 63) / 64, double>(XA, L.LDA, L.RP, D::K, rx, roff, coff);
    }
    stage_u<MODE, KM>(U1, ut + G.u_off[0], n1);
    stage_u<MODE, KM>(U2, ut + G.u_off[1], n2);
    // depth rows of the second product past n2 and columns past C stay zero
    const int CP = pad16(C);
    for (int e = threadIdx.x; e < D::E * L.LDY; e += kFdThreads) YB[e] = (T)0.f;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    // Y = X U1: strips of one row tile (c, i2) across the a1 tiles
    for (int t = wave; t < L.RP / 16; t += kFdWaves) {
        typename M::Acc acc[D::NTU];
        strip_row<MODE, D::KS, D::NTU, false, false>(XA, L.LDA, U1, L.LDU, 16 * t, acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = 16 * t + M::row(g, q);
            const int c = row / n2, i2 = row - c * n2;
#pragma unroll
            for (int j = 0; j < D::NTU; ++j) {
                const int a1 = 16 * j + r;
                if (row < R && a1 < n1) YB[i2 * L.LDY + c * n1 + a1] = (T)acc[j][q];
            }
        }
    }
    __syncthreads();
    // Z = U2^T Y: strips of one stacked column tile (c, a1) across the a2 tiles
    {
        const int64_t n12 = (int64_t)n1 * n2, n123 = n12 * G.n3;
        typename M::Tmp* dst = tmp + G.tmp_off + (int64_t)i3 * n12;
        for (int t = wave; t < CP / 16; t += kFdWaves) {
            typename M::Acc acc[D::NTU];
            strip_col<MODE, D::KS, D::NTU, true, false>(U2, L.LDU, YB, L.LDY, 16 * t, acc);
            const int col = 16 * t + r;
            const int c = col / n1, a1 = col - c * n1;
#pragma unroll
            for (int i = 0; i < D::NTU; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int a2 = 16 * i + M::row(g, q);
                    if (a2 < n2 && col < C) dst[c * n123 + a2 * n1 + a1] = (typename M::Tmp)acc[i][q];
                }
        }
    }
}

// ---------------------------------------------------------------- pass 2
// per (group, block of NCB columns col = (c, a2, a1)): Zt = U3^T Zc, divide
// by the Kronecker-sum eigenvalues, W = U3 Zt written back in place
template <int MODE, int KM, int NCB>
__global__ void __launch_bounds__(kFdThreads) k_fdg_mid(const FdGroup* __restrict__ groups,
                                                        const int2* __restrict__ cols,
                                                        const typename Mf<MODE>::U* __restrict__ ut,
                                                        const double* __restrict__ dt,
                                                        typename Mf<MODE>::Tmp* __restrict__ tmp,
                                                        const MinresState* __restrict__ mask) {
    using M = Mf<MODE>;
    using T = typename M::T;
    using D = Dep<MODE, KM>;
    using Tp = typename M::Tmp;
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 it = cols[blockIdx.x];
    const FdGroup& G = groups[it.x];
    if (mask && mask[G.prob].skip) return;
    const int n1 = G.n1, n3 = G.n3;
    const int n12 = n1 * G.n2;
    const int64_t n123 = (int64_t)n12 * n3;
    const int ncol = G.nc * n12;
    const int col0 = it.y * NCB;
    const Pass3Layout L = mid_layout<MODE, KM>(NCB);
    T* Zc = reinterpret_cast<T*>(smem);
    T* Zt = Zc + L.oZt;
    T* U3 = Zc + L.oU;
    Tp* base = tmp + G.tmp_off;
    stage<kFdWaves, NCB / 64, Tp>(
        Zc, L.LDZ, D::E, NCB, rsrc(base, G.nc * n123 * (int64_t)sizeof(Tp)),
        [&](int i3) { return i3 < n3 ? (uint32_t)(i3 * n12 * sizeof(Tp)) : kOob; },
        [&](int j) {
            const int col = col0 + j;
            const int c = col / n12, jj = col - c * n12;
            return col < ncol ? (uint32_t)((c * n123 + jj) * sizeof(Tp)) : kOob;
        });
    stage_u<MODE, KM>(U3, ut + G.u_off[2], n3);
    // depth rows of Zt past the tiles stay zero
    for (int e = 16 * D::NTU * L.LDZ + threadIdx.x; e < D::E * L.LDZ; e += kFdThreads) Zt[e] = (T)0.f;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    constexpr int TN = NCB / 16;
    for (int t = wave; t < TN; t += kFdWaves) {
        typename M::Acc acc[D::NTU];
        strip_col<MODE, D::KS, D::NTU, true, false>(U3, L.LDU, Zc, L.LDZ, 16 * t, acc);
        const int col = col0 + 16 * t + r;
        const bool cin = col < ncol;
        const int c = col / n12, jj = col - c * n12, a2 = jj / n1, a1 = jj - a2 * n1;
        const int cc = cin ? c : 0;
        const double lam12 =
            cin ? G.mass + G.kappa[cc][0] * dt[G.d_off[0] + a1] + G.kappa[cc][1] * dt[G.d_off[1] + a2] : 0.0;
#pragma unroll
        for (int i = 0; i < D::NTU; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int a3 = 16 * i + M::row(g, q);
                double v = 0.0;
                if (cin && a3 < n3) v = (double)acc[i][q] / (G.scale * (lam12 + G.kappa[cc][2] * dt[G.d_off[2] + a3]));
                Zt[a3 * L.LDZ + 16 * t + r] = (T)v;
            }
    }
    __syncthreads();
    for (int t = wave; t < TN; t += kFdWaves) {
        typename M::Acc acc[D::NTU];
        strip_col<MODE, D::KS, D::NTU, false, false>(U3, L.LDU, Zt, L.LDZ, 16 * t, acc);
        const int col = col0 + 16 * t + r;
        if (col < ncol) {
            const int c = col / n12, jj = col - c * n12;
#pragma unroll
            for (int i = 0; i < D::NTU; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i3 = 16 * i + M::row(g, q);
                    if (i3 < n3) base[c * n123 + (int64_t)i3 * n12 + jj] = (Tp)acc[i][q];
                }
        }
    }
}

// ---------------------------------------------------------------- pass 3
// per (group, slab i3): Y[(c, a2)][i1] = sum_a1 W[(c, a2)][a1] U1[i1][a1];
// X[i2][(c, i1)] = sum_a2 U2[i2][a2] Y[a2][(c, i1)];  out = alpha X (times
// the per-DOF scale, when given)
template <int MODE, int KM>
__global__ void __launch_bounds__(kFdThreads) k_fdg_bwd(const FdGroup* __restrict__ groups,
                                                        const int2* __restrict__ slabs,
                                                        const typename Mf<MODE>::U* __restrict__ ut,
                                                        const typename Mf<MODE>::Tmp* __restrict__ tmp,
                                                        double* __restrict__ out,
                                                        const MinresState* __restrict__ mask,
                                                        const double* __restrict__ scale) {
    using M = Mf<MODE>;
    using T = typename M::T;
    using D = Dep<MODE, KM>;
    using Tp = typename M::Tmp;
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 it = slabs[blockIdx.x];
    const FdGroup& G = groups[it.x];
    if (mask && mask[G.prob].skip) return;
    const int i3 = it.y, n1 = G.n1, n2 = G.n2, nc = G.nc;
    const Pass12Layout L = pass12_layout<MODE, KM>(n1, n2, nc);
    T* ZA = reinterpret_cast<T*>(smem);
    T* U1 = ZA + L.oU1;
    T* YB = ZA + L.oY;
    T* U2 = ZA + L.oU2;
    const int R = nc * n2, C = nc * n1;
    const int64_t n12 = (int64_t)n1 * n2, n123 = n12 * G.n3;
    const Tp* src = tmp + G.tmp_off + (int64_t)i3 * n12;
    stage<kFdWaves, (D::K + 63) / 64, Tp>(
        ZA, L.LDA, L.RP, D::K, rsrc(src, ((nc - 1) * n123 + n12) * (int64_t)sizeof(Tp)),
        [&](int row) {
            const int c = row / n2, a2 = row - c * n2;
            return row < R ? (uint32_t)((c * n123 + a2 * n1) * sizeof(Tp)) : kOob;
        },
        [&](int a1) { return a1 < n1 ? (uint32_t)(a1 * sizeof(Tp)) : kOob; });
    stage_u<MODE, KM>(U1, ut + G.u_off[0], n1);
    stage_u<MODE, KM>(U2, ut + G.u_off[1], n2);
    const int CP = pad16(C);
    for (int e = threadIdx.x; e < D::E * L.LDY; e += kFdThreads) YB[e] = (T)0.f;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    // Y = W U1^T: strips of one row tile (c, a2) across the i1 tiles
    for (int t = wave; t < L.RP / 16; t += kFdWaves) {
        typename M::Acc acc[D::NTU];
        strip_row<MODE, D::KS, D::NTU, false, true>(ZA, L.LDA, U1, L.LDU, 16 * t, acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = 16 * t + M::row(g, q);
            const int c = row / n2, a2 = row - c * n2;
#pragma unroll
            for (int j = 0; j < D::NTU; ++j) {
                const int i1 = 16 * j + r;
                if (row < R && i1 < n1) YB[a2 * L.LDY + c * n1 + i1] = (T)acc[j][q];
            }
        }
    }
    __syncthreads();
    // X = U2 Y: strips of one stacked column tile (c, i1) across the i2 tiles
    {
        double* dst = out + G.out_off + (int64_t)i3 * G.s3;
        const double* sdst = scale ? scale + G.out_off + (int64_t)i3 * G.s3 : nullptr;
        for (int t = wave; t < CP / 16; t += kFdWaves) {
            typename M::Acc acc[D::NTU];
            strip_col<MODE, D::KS, D::NTU, false, false>(U2, L.LDU, YB, L.LDY, 16 * t, acc);
            const int col = 16 * t + r;
            const int c = col / n1, i1 = col - c * n1;
#pragma unroll
            for (int i = 0; i < D::NTU; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i2 = 16 * i + M::row(g, q);
                    if (i2 < n2 && col < C) {
                        const int64_t o = c * G.cstride + (int64_t)i2 * G.s2 + i1;
                        const double v = G.alpha * (double)acc[i][q];
                        dst[o] = sdst ? v * sdst[o] : v;
                    }
                }
        }
    }
}

template <int MODE, int KM>
int64_t lds_elems(int pass, int n1, int n2, int nc, int ncb) {
    return pass == 0 ? pass12_layout<MODE, KM>(n1, n2, nc).total : mid_layout<MODE, KM>(ncb).total;
}

template <int MODE, int KM, int NCB>
void fdg_run(const FdGroupSet& set, const void* ut, const double* dt, const double* in, double* out, void* tmp,
             const MinresState* mask, const double* scale, hipStream_t s) {
    using M = Mf<MODE>;
    const auto* u = static_cast<const typename M::U*>(ut);
    auto* tp = static_cast<typename M::Tmp*>(tmp);
    const size_t b12 = (size_t)lds_elems<MODE, KM>(0, set.max_n1, set.max_n2, set.max_nc, NCB) * sizeof(typename M::T);
    const size_t b3 = (size_t)lds_elems<MODE, KM>(1, set.max_n1, set.max_n2, set.max_nc, NCB) * sizeof(typename M::T);
    const int2* colblocks = NCB == 64 ? set.cols64 : set.cols128;
    const int n_colblocks = NCB == 64 ? set.n_cols64 : set.n_cols128;
    // launches with more than 64 KiB of LDS need the attribute
    if (b12 > 65536) {
        (void)hipFuncSetAttribute((const void*)k_fdg_fwd<MODE, KM>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b12);
        (void)hipFuncSetAttribute((const void*)k_fdg_bwd<MODE, KM>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b12);
    }
    if (b3 > 65536)
        (void)hipFuncSetAttribute((const void*)k_fdg_mid<MODE, KM, NCB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)b3);
    hipLaunchKernelGGL((k_fdg_fwd<MODE, KM>), dim3(set.n_slabs), dim3(kFdThreads), b12, s, set.groups, set.slabs, u, in,
                       tp, mask, scale);
    hipLaunchKernelGGL((k_fdg_mid<MODE, KM, NCB>), dim3(n_colblocks), dim3(kFdThreads), b3, s, set.groups, colblocks,
                       u, dt, tp, mask);
    hipLaunchKernelGGL((k_fdg_bwd<MODE, KM>), dim3(set.n_slabs), dim3(kFdThreads), b12, s, set.groups, set.slabs, u,
                       tp, out, mask, scale);
}

template <int MODE, int KM>
void fdg_ncb(int ncb, const FdGroupSet& set, const void* ut, const double* dt, const double* in, double* out,
             void* tmp, const MinresState* mask, const double* scale, hipStream_t s) {
    if (ncb == 64) fdg_run<MODE, KM, 64>(set, ut, dt, in, out, tmp, mask, scale, s);
    else fdg_run<MODE, KM, 128>(set, ut, dt, in, out, tmp, mask, scale, s);
}

template <int MODE>
void fdg_dispatch(int ncb, const FdGroupSet& set, const void* ut, const double* dt, const double* in, double* out,
                  void* tmp, const MinresState* mask, const double* scale, hipStream_t s) {
    switch (fd_depth_extent(set)) {
        case 28: fdg_ncb<MODE, 28>(ncb, set, ut, dt, in, out, tmp, mask, scale, s); break;
        case 36: fdg_ncb<MODE, 36>(ncb, set, ut, dt, in, out, tmp, mask, scale, s); break;
        default: fdg_ncb<MODE, 48>(ncb, set, ut, dt, in, out, tmp, mask, scale, s); break;
    }
}

template <int MODE>
int64_t lds_for(int km, int pass, int n1, int n2, int nc, int ncb) {
    switch (km) {
        case 28: return lds_elems<MODE, 28>(pass, n1, n2, nc, ncb);
        case 36: return lds_elems<MODE, 36>(pass, n1, n2, nc, ncb);
        default: return lds_elems<MODE, 48>(pass, n1, n2, nc, ncb);
    }
}

}  // namespace

int fd_depth_extent(const FdGroupSet& set) {
    const int n = std::max(set.max_n1, std::max(set.max_n2, set.max_n3));
    return n <= 28 ? 28 : (n <= 36 ? 36 : 48);
}

int fd_variant_ncb(int variant) { return variant & 1 ? 128 : 64; }

int64_t fd_lds_bytes(int mode, int variant, const FdGroupSet& set) {
    const int ncb = fd_variant_ncb(variant), km = fd_depth_extent(set);
    const int64_t es = mode == 0 ? 4 : (mode == 1 ? 2 : 8);
    int64_t a, b;
    if (mode == 0) {
        a = lds_for<0>(km, 0, set.max_n1, set.max_n2, set.max_nc, ncb);
        b = lds_for<0>(km, 1, set.max_n1, set.max_n2, set.max_nc, ncb);
    } else if (mode == 1) {
        a = lds_for<1>(km, 0, set.max_n1, set.max_n2, set.max_nc, ncb);
        b = lds_for<1>(km, 1, set.max_n1, set.max_n2, set.max_nc, ncb);
    } else {
        a = lds_for<2>(km, 0, set.max_n1, set.max_n2, set.max_nc, ncb);
        b = lds_for<2>(km, 1, set.max_n1, set.max_n2, set.max_nc, ncb);
    }
    return es * (a > b ? a : b);
}

void launch_fd_groups(int mode, int variant, const FdGroupSet& set, const void* ut, const double* dt,
                      const double* in, double* out, void* tmp, const MinresState* mask, const double* scale,
                      hipStream_t s) {
    if (set.n_slabs == 0) return;
    const int ncb = fd_variant_ncb(variant);
    if (mode == 0) fdg_dispatch<0>(ncb, set, ut, dt, in, out, tmp, mask, scale, s);
    else if (mode == 1) fdg_dispatch<1>(ncb, set, ut, dt, in, out, tmp, mask, scale, s);
    else fdg_dispatch<2>(ncb, set, ut, dt, in, out, tmp, mask, scale, s);
}

}  // namespace afieti
