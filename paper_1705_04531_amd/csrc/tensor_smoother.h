// Tensor-product (fast-diagonalisation) smoother kernels of the finest multigrid level.  Uses the
// FP64 MFMA block helpers and the mask helpers of kernels.h.
#pragma once

#include <type_traits>

#include "kernels.h"

namespace ieti {

// ---------------------------------------------------------------------------
// Tensor-product smoother of the finest level (2D): y = m U (Lambda_0 (+) Lambda_1 + c)^{-1} U^T m r per
// patch, U = U_1 (x) U_0 the generalised eigenvectors of the separable stiffness.  With the residual of a
// patch as the M1 x M0 matrix R[i1][i0] (i0 fastest, as stored):
//   forward:   Z = (U_1^T R U_0) ./ (lambda_1[b] + lambda_0[a] + c)     (P1 x P0, into scratch)
//   backward:  x[i1][i0] (+)= tau (U_1 Z U_0^T)[i1][i0] on unmasked coefficients
// Both kernels take one work-group per (pair of 16-column blocks, patch), the work-groups of a patch on
// one XCD (fd_block) so that they share its L2: the forward one forms the column blocks W = R U_0[:, blk]
// and then U_1^T W, the backward one T = Z U_0[blk, :]^T and then U_1 T.  The operands are staged in LDS
// (U_1 in the first matrix's space once the first product is done); each wave runs the block products of
// one 16-row block for both columns on the matrix cores in the multigrid precision: FP64
// (v_mfma_f64_16x16x4f64) or, with FP32 V-cycles, FP32 (v_mfma_f32_16x16x4f32) with FP32 operands, LDS
// and scratch; the eigenvalue scaling is done in FP64.  Patches without smoother data (P0 = 0) and
// inactive patches return.

constexpr int FD_THREADS = 512;

struct FdInfo {
    int64_t u0, u1, u2;    // offsets of U_d (P_d x P_d, row-major) in the U array (u2: 3D only)
    int64_t l0, l1, l2;    // offsets of lambda_d in the eigenvalue array
    int64_t zoff;          // scratch of the patch (P1 x P0, 3D: P2 x P1 x P0)
    int32_t P0, P1, P2;    // padded sizes (multiples of 16); P0 = 0: no tensor smoother on this patch; P2 = 0 in 2D
    double shift, tau;
};

struct FdArgs {
    const PatchLev* L;     // level-0 patch descriptors, index = patch
    const FdInfo* info;    // of the mode, index = patch
    const double* U;
    const double* lam;
    double* z;
    const int* active;
    int mode;
    int N;                 // patches
    int ncb;               // 2D: pairs of column blocks per patch in the grid (largest P0 / 32, rounded up)
    double* z2;            // 3D: second scratch buffer (same offsets as z)
    const float* U32;      // 2D, FP32 multigrid: U in FP32 (same offsets as U)
    float* z32;            // 2D, FP32 multigrid: the scratch in FP32 (same offsets as z)
};

// Block products of the 2D transforms in the multigrid's precision CT: FP64 on v_mfma_f64_16x16x4f64,
// FP32 on v_mfma_f32_16x16x4f32.  Both take A[l % 16][k0 + l / 16] and B[k0 + l / 16][l % 16] from lane l;
// element r of lane l is C[l / 16 + 4 r][l % 16] for FP64 and C[4 (l / 16) + r][l % 16] for FP32 (both
// checked on the device).
typedef float mf_f4 __attribute__((ext_vector_type(4)));
template <typename CT> struct FdMf;
template <> struct FdMf<double> {
    typedef mf_d4 acc;
    __device__ static acc mfma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int l, int r) { return (l >> 4) + 4 * r; }
};
template <> struct FdMf<float> {
    typedef mf_f4 acc;
    __device__ static acc mfma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};

// c += A B on 16 x 16 blocks (A[i][k] at A[i * lda + k], TA: at A[k * lda + i]; B[k][j] at B[k * ldb + j])
template <typename CT, bool TA>
__device__ __forceinline__ typename FdMf<CT>::acc fd_mfb(const CT* A, int lda, const CT* B, int ldb,
                                                         typename FdMf<CT>::acc c) {
    const int l = threadIdx.x & 63, i = l & 15, kq = l >> 4;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k = 4 * s + kq;
        c = FdMf<CT>::mfma(TA ? A[k * lda + i] : A[i * lda + k], B[k * ldb + i], c);
    }
    return c;
}

template <typename CT>
__device__ __forceinline__ void fd_mfs(CT* C, int ldc, typename FdMf<CT>::acc c) {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < 4; ++r) C[FdMf<CT>::row(l, r) * ldc + (l & 15)] = c[r];
}

// LDS words (of the multigrid precision) of either kernel for the largest padded sizes: the first
// operand (P1 x ld), the pair of products (P1 x 33) and the pair of U_0 blocks (P0 x 33)
__host__ __device__ inline size_t fd_lds_words(int p0max, int p1max) {
    const int ld = (p0max > p1max ? p0max : p1max) + 1;
    return (size_t)p1max * ld + (size_t)33 * (p1max + p0max);
}

// dst[i * ld + j] = get(i, j) for i < rows, j < cols (cols a multiple of 16): thread -> (row tid / 16 of a
// step of 32 rows, column lane tid % 16); up to 8 column blocks' loads issued before their stores
template <typename CT, typename G>
__device__ __forceinline__ void fd_stage(CT* dst, int ld, int rows, int cols, G get) {
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15, ncb = cols >> 4;
    for (int r0 = 0; r0 < rows; r0 += FD_THREADS / 16) {
        const int i = r0 + tr;
        if (i >= rows) break;
        for (int c0 = 0; c0 < ncb; c0 += 8) {
            double v[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) v[c] = c0 + c < ncb ? get(i, (c0 + c) * 16 + tc) : 0.0;
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (c0 + c < ncb) dst[i * ld + (c0 + c) * 16 + tc] = (CT)v[c];
        }
    }
}

// XCD-aware work-group -> (patch, pair of 16-column blocks): consecutive work-groups go to consecutive
// XCDs, so the work-groups of patch k are all placed on XCD k mod 8 and share its L2 for the patch's
// operands.  Grid: 8 * ceil(N / 8) * ncp one-dimensional (ncp pairs per patch); false for the unused tail.
__device__ __forceinline__ bool fd_block(int N, int ncp, int& k, int& cp) {
    const int L = blockIdx.x, x = L & 7, s = L >> 3;
    k = (s / ncp) * 8 + x;
    cp = s % ncp;
    return k < N;
}

// forward: column blocks 2 cp and 2 cp + 1 (if it exists) of Z; the shared R fragment feeds two
// accumulation chains
template <typename T>
__global__ __launch_bounds__(FD_THREADS) void k_fd_fwd(FdArgs a, const T* __restrict__ r) {
    int k, cp;
    if (!fd_block(a.N, a.ncb, k, cp)) return;
    const FdInfo f = a.info[k];
    if (f.P0 == 0 || (a.active && !a.active[k])) return;
    const int P0 = f.P0, P1 = f.P1, ncb = P0 / 16, cb = 2 * cp;
    if (cb >= ncb) return;
    const bool two = cb + 1 < ncb;
    const PatchLev& P = a.L[k];
    const int M0 = P.M[0], M1 = P.M[1], ld = (P0 > P1 ? P0 : P1) + 1;
    typedef T CT;
    typedef typename FdMf<CT>::acc acc;
    extern __shared__ double fd_sm[];
    CT* Rg = (CT*)fd_sm;                      // R (P1 x P0), then U_1 (P1 x P1); leading dimension ld
    CT* Wb = Rg + (size_t)P1 * ld;            // W (P1 x 32), ld 33
    CT* Ub = Wb + (size_t)P1 * 33;            // U_0[:, blocks cb, cb + 1] (P0 x 32), ld 33
    const CT* Ua = std::is_same<CT, float>::value ? (const CT*)(const void*)a.U32 : (const CT*)(const void*)a.U;
    const CT* U0 = Ua + f.u0;
    const CT* U1 = Ua + f.u1;
    const int mode = a.mode;
    fd_stage(Rg, ld, P1, P0, [&](int i1, int i0) -> double {
        return (i0 < M0 && i1 < M1 && !masked(P, mode, i0, i1, 0)) ? (double)r[P.voff + i0 + (int64_t)M0 * i1] : 0.0;
    });
    fd_stage(Ub, 33, P0, two ? 32 : 16, [&](int i, int j) -> double { return (double)U0[(int64_t)i * P0 + cb * 16 + j]; });
    __syncthreads();
    const int wv = threadIdx.x / WAVE, l = threadIdx.x & (WAVE - 1);
    for (int w = wv; w < P1 / 16; w += FD_THREADS / WAVE) {   // W[block w] = R[block w, :] U_0[:, pair]
        acc c0 = {0, 0, 0, 0}, c1 = c0;
        for (int kb = 0; kb < P0 / 16; ++kb) {
            c0 = fd_mfb<CT, false>(Rg + (size_t)w * 16 * ld + kb * 16, ld, Ub + kb * 16 * 33, 33, c0);
            if (two) c1 = fd_mfb<CT, false>(Rg + (size_t)w * 16 * ld + kb * 16, ld, Ub + kb * 16 * 33 + 16, 33, c1);
        }
        fd_mfs<CT>(Wb + w * 16 * 33, 33, c0);
        if (two) fd_mfs<CT>(Wb + w * 16 * 33 + 16, 33, c1);
    }
    __syncthreads();
    fd_stage(Rg, ld, P1, P1, [&](int i, int j) -> double { return (double)U1[(int64_t)i * P1 + j]; });
    __syncthreads();
    const double* l0 = a.lam + f.l0;
    const double* l1 = a.lam + f.l1;
    for (int w = wv; w < P1 / 16; w += FD_THREADS / WAVE) {   // Z[block w, pair] = U_1[:, block w]^T W, scaled
        acc c0 = {0, 0, 0, 0}, c1 = c0;
        for (int kb = 0; kb < P1 / 16; ++kb) {
            c0 = fd_mfb<CT, true>(Rg + (size_t)kb * 16 * ld + w * 16, ld, Wb + kb * 16 * 33, 33, c0);
            if (two) c1 = fd_mfb<CT, true>(Rg + (size_t)kb * 16 * ld + w * 16, ld, Wb + kb * 16 * 33 + 16, 33, c1);
        }
        CT* z = std::is_same<CT, float>::value ? (CT*)(void*)a.z32 : (CT*)(void*)a.z;
        const int a0 = cb * 16 + (l & 15), a1 = a0 + 16;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int bb = w * 16 + FdMf<CT>::row(l, rr);
            z[f.zoff + (int64_t)bb * P0 + a0] = (CT)((double)c0[rr] / (l1[bb] + l0[a0] + f.shift));
            if (two) z[f.zoff + (int64_t)bb * P0 + a1] = (CT)((double)c1[rr] / (l1[bb] + l0[a1] + f.shift));
        }
    }
}

// backward, column blocks 2 cp and 2 cp + 1 of x.  SET: x = tau y (masked coefficients 0); otherwise
// x += tau y
template <typename T, bool SET>
__global__ __launch_bounds__(FD_THREADS) void k_fd_bwd(FdArgs a, T* __restrict__ x) {
    int k, cp;
    if (!fd_block(a.N, a.ncb, k, cp)) return;
    const FdInfo f = a.info[k];
    if (f.P0 == 0 || (a.active && !a.active[k])) return;
    const PatchLev& P = a.L[k];
    const int M0 = P.M[0], M1 = P.M[1], P0 = f.P0, P1 = f.P1, ld = (P0 > P1 ? P0 : P1) + 1, jc = 2 * cp;
    if (jc * 16 >= M0) return;
    const bool two = (jc + 1) * 16 < M0;
    typedef T CT;
    typedef typename FdMf<CT>::acc acc;
    extern __shared__ double fd_sm[];
    CT* Zg = (CT*)fd_sm;                      // Z (P1 x P0), then U_1 (P1 x P1); leading dimension ld
    CT* Tb = Zg + (size_t)P1 * ld;            // T (P1 x 32), ld 33
    CT* Ub = Tb + (size_t)P1 * 33;            // U_0[blocks jc, jc + 1, :]^T (P0 x 32), ld 33
    const CT* Ua = std::is_same<CT, float>::value ? (const CT*)(const void*)a.U32 : (const CT*)(const void*)a.U;
    const CT* U0 = Ua + f.u0;
    const CT* U1 = Ua + f.u1;
    const CT* Z = (std::is_same<CT, float>::value ? (const CT*)(const void*)a.z32 : (const CT*)(const void*)a.z) + f.zoff;
    const int wv = threadIdx.x / WAVE, l = threadIdx.x & (WAVE - 1);
    fd_stage(Zg, ld, P1, P0, [&](int i, int j) -> double { return (double)Z[(int64_t)i * P0 + j]; });
    fd_stage(Ub, 33, P0, two ? 32 : 16, [&](int i, int j) -> double { return (double)U0[(int64_t)(jc * 16 + j) * P0 + i]; });
    __syncthreads();
    for (int w = wv; w < P1 / 16; w += FD_THREADS / WAVE) {   // T[block w] = Z[block w, :] U_0[pair, :]^T
        acc c0 = {0, 0, 0, 0}, c1 = c0;
        for (int kb = 0; kb < P0 / 16; ++kb) {
            c0 = fd_mfb<CT, false>(Zg + (size_t)w * 16 * ld + kb * 16, ld, Ub + kb * 16 * 33, 33, c0);
            if (two) c1 = fd_mfb<CT, false>(Zg + (size_t)w * 16 * ld + kb * 16, ld, Ub + kb * 16 * 33 + 16, 33, c1);
        }
        fd_mfs<CT>(Tb + w * 16 * 33, 33, c0);
        if (two) fd_mfs<CT>(Tb + w * 16 * 33 + 16, 33, c1);
    }
    __syncthreads();
    fd_stage(Zg, ld, P1, P1, [&](int i, int j) -> double { return (double)U1[(int64_t)i * P1 + j]; });
    __syncthreads();
    for (int w = wv; w < P1 / 16; w += FD_THREADS / WAVE) {   // Y[block w, pair] = U_1[block w, :] T
        acc c0 = {0, 0, 0, 0}, c1 = c0;
        for (int kb = 0; kb < P1 / 16; ++kb) {
            c0 = fd_mfb<CT, false>(Zg + (size_t)w * 16 * ld + kb * 16, ld, Tb + kb * 16 * 33, 33, c0);
            if (two) c1 = fd_mfb<CT, false>(Zg + (size_t)w * 16 * ld + kb * 16, ld, Tb + kb * 16 * 33 + 16, 33, c1);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (q == 1 && !two) break;
            const int i0 = (jc + q) * 16 + (l & 15);
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int i1 = w * 16 + FdMf<CT>::row(l, rr);
                if (i0 >= M0 || i1 >= M1) continue;
                const double v = q ? c1[rr] : c0[rr];
                const int64_t vi = P.voff + i0 + (int64_t)M0 * i1;
                const bool m = masked(P, a.mode, i0, i1, 0);
                if (SET) x[vi] = m ? T(0) : T(f.tau * v);
                else if (!m) x[vi] = T((double)x[vi] + f.tau * v);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// 3D: the transforms as three contractions along one axis each, on padded P2 x P1 x P0 arrays (index
// a + P0 (b + P1 c)) in the two scratch buffers:
//   forward   za = R x_0 U_0,  zb = za x_1 U_1,  za = (zb x_2 U_2) ./ (lambda_0 + lambda_1 + lambda_2 + c)
//   backward  zb = za x_2 U_2^T,  za = zb x_1 U_1^T,  x (+)= tau (za x_0 U_0^T) on unmasked coefficients
// (x_d U: contraction of the axis-d index i with U[i][.]).  One wave per 16 x 16 output tile, FD3_THREADS / 64
// tiles per work-group, the contraction (P_d <= 128) read straight from memory; every entry of the padded
// arrays is written (padding rows and columns come out zero), so no scratch needs clearing.

constexpr int FD3_THREADS = 256;

// tile t of patch k (grid: blockIdx.y = patch, FD3_THREADS / 64 tiles per work-group); false if t is past
// the patch's tiles
__device__ __forceinline__ bool fd3_tile(const FdArgs& a, int& k, FdInfo& f, int& t) {
    k = blockIdx.y;
    f = a.info[k];
    if (f.P0 == 0 || (a.active && !a.active[k])) return false;
    t = blockIdx.x * (FD3_THREADS / WAVE) + threadIdx.x / WAVE;
    return t < (f.P0 / 16) * (f.P1 / 16) * (f.P2 / 16) * 16;
}

// forward axis 0: za[o][a] = sum_i0 m r[o][i0] U_0[i0][a], o = i1 + P1 i2
template <typename T>
__global__ __launch_bounds__(FD3_THREADS) void k_fd3_ax0_fwd(FdArgs a, const T* __restrict__ r) {
    int k, t;
    FdInfo f;
    if (!fd3_tile(a, k, f, t)) return;
    const PatchLev& P = a.L[k];
    const int nco = f.P0 / 16, ro = t / nco, co = t % nco;
    const int l = threadIdx.x & (WAVE - 1), i = l & 15, kq = l >> 4;
    const int o = ro * 16 + i, i1 = o % f.P1, i2 = o / f.P1;
    const bool rowok = i1 < P.M[1] && i2 < P.M[2];
    const double* U0 = a.U + f.u0;
    mf_d4 c = {0.0, 0.0, 0.0, 0.0};
    for (int kb = 0; kb < f.P0 / 16; ++kb)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int i0 = kb * 16 + 4 * s + kq;
            double av = 0.0;
            if (rowok && i0 < P.M[0] && !masked(P, a.mode, i0, i1, i2))
                av = (double)r[P.voff + i0 + (int64_t)P.M[0] * (i1 + (int64_t)P.M[1] * i2)];
            c = __builtin_amdgcn_mfma_f64_16x16x4f64(av, U0[(int64_t)i0 * f.P0 + co * 16 + i], c, 0, 0, 0);
        }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int orow = ro * 16 + (l >> 4) + 4 * rr;
        a.z[f.zoff + (int64_t)orow * f.P0 + co * 16 + i] = c[rr];
    }
}

// axis AX (1 or 2) viewed as [outer][P_AX][inner]: FWD out[o][c][n] = sum_i U[i][c] in[o][i][n],
// otherwise sum_i U[c][i] in[o][i][n]; SCALE divides by lambda_0[a] + lambda_1[b] + lambda_2[c] + shift
template <int AX, bool FWD, bool SCALE>
__global__ __launch_bounds__(FD3_THREADS) void k_fd3_axn(FdArgs a, const double* __restrict__ in, double* __restrict__ out) {
    int k, t;
    FdInfo f;
    if (!fd3_tile(a, k, f, t)) return;
    const int Pax = AX == 1 ? f.P1 : f.P2;
    const int inner = AX == 1 ? f.P0 : f.P0 * f.P1;
    const int nci = inner / 16, ncr = Pax / 16;
    const int o = t / (ncr * nci), rem = t % (ncr * nci), cr = rem / nci, ci = rem % nci;
    const double* U = a.U + (AX == 1 ? f.u1 : f.u2);
    const double* B = in + f.zoff + (int64_t)o * Pax * inner + ci * 16;
    mf_d4 c = {0.0, 0.0, 0.0, 0.0};
    for (int kb = 0; kb < ncr; ++kb)
        c = FWD ? mf_block<true>(U + (int64_t)kb * 16 * Pax + cr * 16, Pax, B + (int64_t)kb * 16 * inner, inner, c, 1.0)
                : mf_block<false>(U + (int64_t)cr * 16 * Pax + kb * 16, Pax, B + (int64_t)kb * 16 * inner, inner, c, 1.0);
    const int l = threadIdx.x & (WAVE - 1);
    const int n = ci * 16 + (l & 15);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int row = cr * 16 + (l >> 4) + 4 * rr;
        double v = c[rr];
        if (SCALE) {
            const int ia = n % f.P0, ib = n / f.P0;
            v /= a.lam[f.l0 + ia] + a.lam[f.l1 + ib] + a.lam[f.l2 + row] + f.shift;
        }
        out[f.zoff + (int64_t)o * Pax * inner + (int64_t)row * inner + n] = v;
    }
}

// backward axis 0: y[o][i0] = sum_a za[o][a] U_0[i0][a]; SET: x = tau y (masked 0), else x += tau y
template <typename T, bool SET>
__global__ __launch_bounds__(FD3_THREADS) void k_fd3_ax0_bwd(FdArgs a, T* __restrict__ x) {
    int k, t;
    FdInfo f;
    if (!fd3_tile(a, k, f, t)) return;
    const PatchLev& P = a.L[k];
    const int nco = f.P0 / 16, ro = t / nco, co = t % nco;
    const double* U0 = a.U + f.u0;
    mf_d4 c = {0.0, 0.0, 0.0, 0.0};
    for (int kb = 0; kb < f.P0 / 16; ++kb)
        c = mf_block<false, true>(a.z + f.zoff + (int64_t)ro * 16 * f.P0 + kb * 16, f.P0,
                                  U0 + (int64_t)co * 16 * f.P0 + kb * 16, f.P0, c, 1.0);
    const int l = threadIdx.x & (WAVE - 1);
    const int i0 = co * 16 + (l & 15);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int o = ro * 16 + (l >> 4) + 4 * rr, i1 = o % f.P1, i2 = o / f.P1;
        if (i0 >= P.M[0] || i1 >= P.M[1] || i2 >= P.M[2]) continue;
        const int64_t vi = P.voff + i0 + (int64_t)P.M[0] * (i1 + (int64_t)P.M[1] * i2);
        const bool m = masked(P, a.mode, i0, i1, i2);
        if (SET) x[vi] = m ? T(0) : T(f.tau * c[rr]);
        else if (!m) x[vi] = T((double)x[vi] + f.tau * c[rr]);
    }
}

}  // namespace ieti
