// Tensor-product (fast-diagonalisation) smoother kernels of the finest multigrid level.  Uses the
// FP64 MFMA block helpers and the mask helpers of kernels.h.
#pragma once

#include <type_traits>

#include "kernels.h"

namespace ieti {

// ---------------------------------------------------------------------------
// Tensor-product smoother of the finest level (2D): y = m U (Lambda_0 (+) Lambda_1 + c)^{-1} U^T m r per
// patch, U = U_1 (x) U_0 the generalised eigenvectors of the separable stiffness.  With the residual of a
// patch as the M1 x M0 matrix R[i1][i0] (i0 fastest, as stored), zero-padded to P1 x P0:
//   W = (m R) U_0                                     (second scratch)
//   Z = (U_1^T W) ./ (lambda_1[b] + lambda_0[a] + c)   (scratch)
//   T = Z U_0^T                                       (second scratch)
//   x (+)= tau m (U_1 T)                              on the M1 x M0 coefficients
// Four batched block products, one wave per 16 x 16 output block of a patch's P1 x P0 array (grid:
// blockIdx.y = patch, FD2_THREADS / 64 blocks per work-group), on the matrix cores in the multigrid
// precision: FP64 (v_mfma_f64_16x16x4f64) or, with FP32 V-cycles, FP32 (v_mfma_f32_16x16x4f32) with FP32
// operands and scratch; the eigenvalue scaling is done in FP64.  The operands come straight from memory
// (mostly L2): no LDS, so a CU holds many work-groups that hide each other's load latency, and the blocks
// of all patches spread over the chip.  Patches without smoother data (P0 = 0) and inactive patches
// return.

constexpr int FD2_THREADS = 256;

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
    double* z2;            // second scratch buffer (same offsets as z)
    const float* U32;      // 2D, FP32 multigrid: U in FP32 (same offsets as U)
    float* z32;            // 2D, FP32 multigrid: the scratch in FP32 (same offsets as z)
    float* z232;           // 2D, FP32 multigrid: the second scratch in FP32
};

// Block products in the multigrid's precision CT: FP64 on v_mfma_f64_16x16x4f64, FP32 on
// v_mfma_f32_16x16x4f32.  Both take A[l % 16][k0 + l / 16] and B[k0 + l / 16][l % 16] from lane l;
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

// masked_bits without short-circuit evaluation (bitwise operations only), so that an operand getter that
// calls it compiles without branches and its loads can be issued together
__host__ __device__ __forceinline__ bool masked_nb(uint32_t mb, int dim, int M0, int M1, int M2, int i0, int i1,
                                                   int i2) {
    const uint32_t sides = mb & 0xFFu, corners = mb >> 8;
    const uint32_t d3 = dim == 3;
    const uint32_t lo0 = i0 == 0, hi0 = i0 == M0 - 1, lo1 = i1 == 0, hi1 = i1 == M1 - 1;
    const uint32_t lo2 = d3 & (uint32_t)(i2 == 0), hi2 = d3 & (uint32_t)(i2 == M2 - 1);
    const uint32_t side = (lo0 | (hi0 << 1) | (lo1 << 2) | (hi1 << 3) | (lo2 << 4) | (hi2 << 5)) & sides;
    const uint32_t corner = (lo0 | hi0) & (lo1 | hi1) & ((d3 ^ 1u) | lo2 | hi2);
    const uint32_t cb = hi0 | (hi1 << 1) | (hi2 << 2);
    return (side | (corner & (corners >> cb))) != 0u;   // corner is 0 or 1
}

// the output block of this wave: patch k (blockIdx.y), block row bi and column bj of its P1 x P0 array;
// false if the patch has no smoother data, is inactive, or the block is past its blocks
__device__ __forceinline__ bool fd2_tile(const FdArgs& a, int& k, FdInfo& f, int& bi, int& bj) {
    k = blockIdx.y;
    f = a.info[k];
    if (f.P0 == 0 || (a.active && !a.active[k])) return false;
    const int t = blockIdx.x * (FD2_THREADS / WAVE) + threadIdx.x / WAVE, nb0 = f.P0 / 16;
    if (t >= (f.P1 / 16) * nb0) return false;
    bi = t / nb0;
    bj = t % nb0;
    return true;
}

// c = sum over K blocks kb < nkb of A[block][kb] B[kb][block].  Within a 16-wide K block, lane group
// kq = l / 16 supplies k = 4 kq + s to the s-th of the four MFMAs, so that a lane's A values A[i][k0 .. k0+3]
// and B values B[k0 .. k0+3][j] (k0 = 16 kb + 4 kq) are four consecutive K indices: ga(i, k0, v) and
// gb(k0, j, v) fill v[0..3] (one 32-byte load where K is the contiguous index of the layout, four loads
// that are contiguous across the lanes otherwise).  Steps of FD2_KG K blocks: their operand loads are issued
// before their products (a step past nkb re-reads the last block and skips its products).
constexpr int FD2_KG = 4;   // 16-wide K blocks whose operands are loaded before their products (8: fewer waves fit, 16x16 workload 120.6 -> 134 ms)
template <typename CT, typename GA, typename GB>
__device__ __forceinline__ typename FdMf<CT>::acc fd2_product(int nkb, GA ga, GB gb) {
    typedef typename FdMf<CT>::acc acc;
    const int l = threadIdx.x & (WAVE - 1), i = l & 15, kq = l >> 4;
    acc c = {0, 0, 0, 0};
    for (int kb0 = 0; kb0 < nkb; kb0 += FD2_KG) {
        CT av[4 * FD2_KG], bv[4 * FD2_KG];
#pragma unroll
        for (int q = 0; q < FD2_KG; ++q) {
            const int k0 = min(kb0 + q, nkb - 1) * 16 + 4 * kq;
            ga(i, k0, av + 4 * q);
            gb(k0, i, bv + 4 * q);
        }
#pragma unroll
        for (int q = 0; q < FD2_KG; ++q)
            if (kb0 + q < nkb) {
#pragma unroll
                for (int s = 0; s < 4; ++s) c = FdMf<CT>::mfma(av[4 * q + s], bv[4 * q + s], c);
            }
    }
    return c;
}

// four consecutive values p[0..3] by one vector load (p 4-element aligned: offsets that are multiples of 4
// in arrays whose patch offsets are multiples of 256)
template <typename CT>
__device__ __forceinline__ void load4(const CT* p, CT* v) {
    typedef CT v4 __attribute__((ext_vector_type(4)));
    const v4 t = *(const v4*)p;
    v[0] = t[0];
    v[1] = t[1];
    v[2] = t[2];
    v[3] = t[3];
}

template <typename CT>
__device__ __forceinline__ const CT* fd_u(const FdArgs& a) {
    return std::is_same<CT, float>::value ? (const CT*)(const void*)a.U32 : (const CT*)(const void*)a.U;
}
template <typename CT>
__device__ __forceinline__ CT* fd_scr(const FdArgs& a, bool second) {
    if (std::is_same<CT, float>::value) return (CT*)(void*)(second ? a.z232 : a.z32);
    return (CT*)(void*)(second ? a.z2 : a.z);
}

// W = (m R) U_0 into the second scratch
template <typename T>
__global__ __launch_bounds__(FD2_THREADS) void k_fd2_w(FdArgs a, const T* __restrict__ r) {
    typedef T CT;
    int k, bi, bj;
    FdInfo f;
    if (!fd2_tile(a, k, f, bi, bj)) return;
    const PatchLev& P = a.L[k];
    const int M0 = P.M[0], M1 = P.M[1], P0 = f.P0, mode = a.mode;
    const CT* U0 = fd_u<CT>(a) + f.u0;
    const uint32_t mb = P.mbits[mode];
    auto ga = [&](int i, int k0, CT* v) {
        const int i1 = bi * 16 + i;
        const T* row = r + P.voff + (int64_t)M0 * min(i1, M1 - 1);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int kk = k0 + s;
            const CT x = (CT)row[min(kk, M0 - 1)];
            const bool keep = (kk < M0) & (i1 < M1) & !masked_nb(mb, 2, M0, M1, 1, kk, i1, 0);
            v[s] = keep ? x : CT(0);
        }
    };
    auto gb = [&](int k0, int j, CT* v) {
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = U0[(int64_t)(k0 + s) * P0 + bj * 16 + j];
    };
    const auto c = fd2_product<CT>(P0 / 16, ga, gb);
    CT* W = fd_scr<CT>(a, true) + f.zoff;
    const int l = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) W[(int64_t)(bi * 16 + FdMf<CT>::row(l, rr)) * P0 + bj * 16 + (l & 15)] = c[rr];
}

// Z = (U_1^T W) ./ (lambda_1[b] + lambda_0[a] + c) into the scratch
template <typename T>
__global__ __launch_bounds__(FD2_THREADS) void k_fd2_z(FdArgs a) {
    typedef T CT;
    int k, bi, bj;
    FdInfo f;
    if (!fd2_tile(a, k, f, bi, bj)) return;
    const int P0 = f.P0, P1 = f.P1;
    const CT* U1 = fd_u<CT>(a) + f.u1;
    const CT* W = fd_scr<CT>(a, true) + f.zoff;
    auto ga = [&](int i, int k0, CT* v) {
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = U1[(int64_t)(k0 + s) * P1 + bi * 16 + i];
    };
    auto gb = [&](int k0, int j, CT* v) {
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = W[(int64_t)(k0 + s) * P0 + bj * 16 + j];
    };
    const auto c = fd2_product<CT>(P1 / 16, ga, gb);
    CT* z = fd_scr<CT>(a, false) + f.zoff;
    const double* l0 = a.lam + f.l0;
    const double* l1 = a.lam + f.l1;
    const int l = threadIdx.x & (WAVE - 1), a0 = bj * 16 + (l & 15);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int bb = bi * 16 + FdMf<CT>::row(l, rr);
        z[(int64_t)bb * P0 + a0] = (CT)((double)c[rr] / (l1[bb] + l0[a0] + f.shift));
    }
}

// T = Z U_0^T into the second scratch (column blocks that reach past M0 are not needed)
template <typename T>
__global__ __launch_bounds__(FD2_THREADS) void k_fd2_t(FdArgs a) {
    typedef T CT;
    int k, bi, bj;
    FdInfo f;
    if (!fd2_tile(a, k, f, bi, bj)) return;
    if (bj * 16 >= a.L[k].M[0]) return;
    const int P0 = f.P0;
    const CT* U0 = fd_u<CT>(a) + f.u0;
    const CT* Z = fd_scr<CT>(a, false) + f.zoff;
    auto ga = [&](int i, int k0, CT* v) { load4(Z + (int64_t)(bi * 16 + i) * P0 + k0, v); };
    auto gb = [&](int k0, int j, CT* v) { load4(U0 + (int64_t)(bj * 16 + j) * P0 + k0, v); };
    const auto c = fd2_product<CT>(P0 / 16, ga, gb);
    CT* Tm = fd_scr<CT>(a, true) + f.zoff;
    const int l = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) Tm[(int64_t)(bi * 16 + FdMf<CT>::row(l, rr)) * P0 + bj * 16 + (l & 15)] = c[rr];
}

// x (+)= tau m (U_1 T) on the M1 x M0 coefficients.  SET: x = tau y (masked coefficients 0); otherwise
// x += tau y
template <typename T, bool SET>
__global__ __launch_bounds__(FD2_THREADS) void k_fd2_y(FdArgs a, T* __restrict__ x) {
    typedef T CT;
    int k, bi, bj;
    FdInfo f;
    if (!fd2_tile(a, k, f, bi, bj)) return;
    const PatchLev& P = a.L[k];
    const int M0 = P.M[0], M1 = P.M[1], P0 = f.P0, P1 = f.P1;
    if (bj * 16 >= M0 || bi * 16 >= M1) return;
    const CT* U1 = fd_u<CT>(a) + f.u1;
    const CT* Tm = fd_scr<CT>(a, true) + f.zoff;
    auto ga = [&](int i, int k0, CT* v) { load4(U1 + (int64_t)(bi * 16 + i) * P1 + k0, v); };
    auto gb = [&](int k0, int j, CT* v) {
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = Tm[(int64_t)(k0 + s) * P0 + bj * 16 + j];
    };
    const auto c = fd2_product<CT>(P1 / 16, ga, gb);
    const int l = threadIdx.x & (WAVE - 1), i0 = bj * 16 + (l & 15);
    double old[4] = {0.0, 0.0, 0.0, 0.0};
    if (!SET) {   // the four old values loaded together (clamped to valid coefficients)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int i1 = min(bi * 16 + FdMf<CT>::row(l, rr), M1 - 1);
            old[rr] = (double)x[P.voff + min(i0, M0 - 1) + (int64_t)M0 * i1];
        }
    }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int i1 = bi * 16 + FdMf<CT>::row(l, rr);
        if (i0 >= M0 || i1 >= M1) continue;
        const double v = c[rr];
        const int64_t vi = P.voff + i0 + (int64_t)M0 * i1;
        const bool m = masked(P, a.mode, i0, i1, 0);
        if (SET) x[vi] = m ? T(0) : T(f.tau * v);
        else if (!m) x[vi] = T(old[rr] + f.tau * v);
    }
}

// The same four products fused in pairs per column block: one work-group per (patch, 16-wide column block
// bj) computes the intermediate column block (W[:, bj] = m R U_0[:, bj], or T[:, bj] = Z U_0[bj, :]^T) into
// LDS, one 16 x 16 block per wave and pass, then the final column block from it (Z[:, bj] = U_1^T W[:, bj]
// scaled, or the update of x with U_1 T[:, bj]).  Each block's sums run in the K order of the unfused
// kernels, so the results are the same; the intermediates never go to memory and two launches are saved.
// Grid: (largest P0 / 16, N) work-groups of FD2C_THREADS, dynamic LDS of (largest P1) x FD2C_LD words; used while
// the largest P1 is at most FD2C_MAXP (the unfused kernels above otherwise).
constexpr int FD2C_LD = 17;     // LDS row length of an intermediate column block (P1 x 16, one word of padding)
constexpr int FD2C_MAXP = 256;
constexpr int FD2C_THREADS = 512;   // eight waves: one 16-row block each for patches up to 128 coefficients

__device__ __forceinline__ bool fd2_colblock(const FdArgs& a, int& k, FdInfo& f, int& bj) {
    k = blockIdx.y;
    f = a.info[k];
    if (f.P0 == 0 || (a.active && !a.active[k])) return false;
    bj = blockIdx.x;
    return bj < f.P0 / 16;
}

// forward: Z[:, bj] = (U_1^T (m R U_0)[:, bj]) ./ (lambda_1 + lambda_0 + c) into the scratch
template <typename T>
__global__ __launch_bounds__(FD2C_THREADS) void k_fd2_fwd(FdArgs a, const T* __restrict__ r) {
    typedef T CT;
    extern __shared__ double fd2c_sm[];
    CT* Wl = (CT*)fd2c_sm;
    int k, bj;
    FdInfo f;
    if (!fd2_colblock(a, k, f, bj)) return;
    const PatchLev& P = a.L[k];
    const int M0 = P.M[0], M1 = P.M[1], P0 = f.P0, P1 = f.P1, nb1 = P1 / 16, mode = a.mode;
    const CT* U0 = fd_u<CT>(a) + f.u0;
    const CT* U1 = fd_u<CT>(a) + f.u1;
    const uint32_t mb = P.mbits[mode];
    const int wv = threadIdx.x / WAVE, l = threadIdx.x & (WAVE - 1);
    for (int bi = wv; bi < nb1; bi += FD2C_THREADS / WAVE) {
        auto ga = [&](int i, int k0, CT* v) {
            const int i1 = bi * 16 + i;
            const T* row = r + P.voff + (int64_t)M0 * min(i1, M1 - 1);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int kk = k0 + s;
                const CT x = (CT)row[min(kk, M0 - 1)];
                const bool keep = (kk < M0) & (i1 < M1) & !masked_nb(mb, 2, M0, M1, 1, kk, i1, 0);
                v[s] = keep ? x : CT(0);
            }
        };
        auto gb = [&](int k0, int j, CT* v) {
#pragma unroll
            for (int s = 0; s < 4; ++s) v[s] = U0[(int64_t)(k0 + s) * P0 + bj * 16 + j];
        };
        const auto c = fd2_product<CT>(P0 / 16, ga, gb);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) Wl[(bi * 16 + FdMf<CT>::row(l, rr)) * FD2C_LD + (l & 15)] = c[rr];
    }
    __syncthreads();
    CT* z = fd_scr<CT>(a, false) + f.zoff;
    const double* l0 = a.lam + f.l0;
    const double* l1 = a.lam + f.l1;
    const int a0 = bj * 16 + (l & 15);
    for (int bi = wv; bi < nb1; bi += FD2C_THREADS / WAVE) {
        auto ga = [&](int i, int k0, CT* v) {
#pragma unroll
            for (int s = 0; s < 4; ++s) v[s] = U1[(int64_t)(k0 + s) * P1 + bi * 16 + i];
        };
        auto gb = [&](int k0, int j, CT* v) {
#pragma unroll
            for (int s = 0; s < 4; ++s) v[s] = Wl[(k0 + s) * FD2C_LD + j];
        };
        const auto c = fd2_product<CT>(nb1, ga, gb);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int bb = bi * 16 + FdMf<CT>::row(l, rr);
            z[(int64_t)bb * P0 + a0] = (CT)((double)c[rr] / (l1[bb] + l0[a0] + f.shift));
        }
    }
}

// backward: x[:, bj] (+)= tau m (U_1 (Z U_0^T)[:, bj]) on the M1 x M0 coefficients (SET: x = tau y, masked
// coefficients 0); column blocks past M0 are skipped
template <typename T, bool SET>
__global__ __launch_bounds__(FD2C_THREADS) void k_fd2_bwd(FdArgs a, T* __restrict__ x) {
    typedef T CT;
    extern __shared__ double fd2c_sm[];
    CT* Tl = (CT*)fd2c_sm;
    int k, bj;
    FdInfo f;
    if (!fd2_colblock(a, k, f, bj)) return;
    const PatchLev& P = a.L[k];
    const int M0 = P.M[0], M1 = P.M[1], P0 = f.P0, P1 = f.P1, nb1 = P1 / 16;
    if (bj * 16 >= M0) return;
    const CT* U0 = fd_u<CT>(a) + f.u0;
    const CT* U1 = fd_u<CT>(a) + f.u1;
    const CT* Z = fd_scr<CT>(a, false) + f.zoff;
    const int wv = threadIdx.x / WAVE, l = threadIdx.x & (WAVE - 1);
    for (int bi = wv; bi < nb1; bi += FD2C_THREADS / WAVE) {
        auto ga = [&](int i, int k0, CT* v) { load4(Z + (int64_t)(bi * 16 + i) * P0 + k0, v); };
        auto gb = [&](int k0, int j, CT* v) { load4(U0 + (int64_t)(bj * 16 + j) * P0 + k0, v); };
        const auto c = fd2_product<CT>(P0 / 16, ga, gb);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) Tl[(bi * 16 + FdMf<CT>::row(l, rr)) * FD2C_LD + (l & 15)] = c[rr];
    }
    __syncthreads();
    const int i0 = bj * 16 + (l & 15);
    for (int bi = wv; bi < nb1; bi += FD2C_THREADS / WAVE) {
        if (bi * 16 >= M1) break;
        auto ga = [&](int i, int k0, CT* v) { load4(U1 + (int64_t)(bi * 16 + i) * P1 + k0, v); };
        auto gb = [&](int k0, int j, CT* v) {
#pragma unroll
            for (int s = 0; s < 4; ++s) v[s] = Tl[(k0 + s) * FD2C_LD + j];
        };
        const auto c = fd2_product<CT>(nb1, ga, gb);
        double old[4] = {0.0, 0.0, 0.0, 0.0};
        if (!SET) {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int i1 = min(bi * 16 + FdMf<CT>::row(l, rr), M1 - 1);
                old[rr] = (double)x[P.voff + min(i0, M0 - 1) + (int64_t)M0 * i1];
            }
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int i1 = bi * 16 + FdMf<CT>::row(l, rr);
            if (i0 >= M0 || i1 >= M1) continue;
            const double v = c[rr];
            const int64_t vi = P.voff + i0 + (int64_t)M0 * i1;
            const bool m = masked(P, a.mode, i0, i1, 0);
            if (SET) x[vi] = m ? T(0) : T(f.tau * v);
            else if (!m) x[vi] = T(old[rr] + f.tau * v);
        }
    }
}

// ---------------------------------------------------------------------------
// 3D: the transforms as contractions along one axis each, on padded P2 x P1 x P0 arrays (index
// a + P0 (b + P1 c)) in the two scratch buffers:
//   forward   zb = (R x_0 U_0) x_1 U_1 (k_fd3_fwd01),  za = (zb x_2 U_2) ./ (lambda_0 + lambda_1 + lambda_2 + c)
//   backward  zb = za x_2 U_2^T,  x (+)= tau ((zb x_0 U_0^T) x_1 U_1^T) on unmasked coefficients (k_fd3_bwd10)
// (x_d U: contraction of the axis-d index i with U[i][.]).  Axis 2: one wave per 16 x 16 output tile,
// FD3_THREADS / 64 tiles per work-group, the contraction (P_d <= 128) read straight from memory; every entry
// of the padded arrays is written (padding rows and columns come out zero), so no scratch needs clearing.

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
    auto ga = [&](int i, int k0, double* v) {   // A[c][i] = U[i][c] (FWD) or U[c][i]
        if (FWD) {
#pragma unroll
            for (int s = 0; s < 4; ++s) v[s] = U[(int64_t)(k0 + s) * Pax + cr * 16 + i];
        } else {
            load4(U + (int64_t)(cr * 16 + i) * Pax + k0, v);
        }
    };
    auto gb = [&](int k0, int j, double* v) {
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = B[(int64_t)(k0 + s) * inner + j];
    };
    const mf_d4 c = fd2_product<double>(ncr, ga, gb);
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

// Axes 0 and 1 fused per (patch, plane c, 16-wide column block bj), the 2D pairing applied to one plane:
//   forward   zb[c][:, bj] = U_1^T (m R_c U_0)[:, bj]      (into the second scratch, unscaled; axis 2 follows)
//   backward  x_c[:, bj] (+)= tau m (U_1 (zb_c U_0^T)[:, bj])   (zb from the second scratch, after axis 2)
// The intermediate column block in LDS (P1 x FD2C_LD words), one 16 x 16 block per wave.  Grid:
// (largest P0 / 16 x largest P2, N) work-groups of FD3_THREADS; the backward pass multiplies in the order
// U_1 (zb U_0^T) rather than (U_1 zb) U_0^T of the separate contractions (equal up to rounding).
__device__ __forceinline__ bool fd3_plane_block(const FdArgs& a, int ncbmax, int& k, FdInfo& f, int& c, int& bj) {
    k = blockIdx.y;
    f = a.info[k];
    if (f.P0 == 0 || (a.active && !a.active[k])) return false;
    c = blockIdx.x / ncbmax;
    bj = blockIdx.x % ncbmax;
    return bj < f.P0 / 16 && c < f.P2;
}

template <typename T>
__global__ __launch_bounds__(FD3_THREADS) void k_fd3_fwd01(FdArgs a, const T* __restrict__ r, int ncbmax) {
    extern __shared__ double fd3c_sm[];
    double* Wl = fd3c_sm;
    int k, c, bj;
    FdInfo f;
    if (!fd3_plane_block(a, ncbmax, k, f, c, bj)) return;
    const PatchLev& P = a.L[k];
    const int M0 = P.M[0], M1 = P.M[1], M2 = P.M[2], P0 = f.P0, P1 = f.P1, nb1 = P1 / 16;
    const uint32_t mb = P.mbits[a.mode];
    const double* U0 = a.U + f.u0;
    const double* U1 = a.U + f.u1;
    const int wv = threadIdx.x / WAVE, l = threadIdx.x & (WAVE - 1);
    const bool planeok = c < M2;
    for (int bi = wv; bi < nb1; bi += FD3_THREADS / WAVE) {
        auto ga = [&](int i, int k0, double* v) {
            const int i1 = bi * 16 + i;
            const T* row = r + P.voff + (int64_t)M0 * (min(i1, M1 - 1) + (int64_t)M1 * min(c, M2 - 1));
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int i0 = k0 + s;
                const double x = (double)row[min(i0, M0 - 1)];
                v[s] = (planeok & (i1 < M1) & (i0 < M0) & !masked_nb(mb, 3, M0, M1, M2, i0, i1, c)) ? x : 0.0;
            }
        };
        auto gb = [&](int k0, int j, double* v) {
#pragma unroll
            for (int s = 0; s < 4; ++s) v[s] = U0[(int64_t)(k0 + s) * P0 + bj * 16 + j];
        };
        const mf_d4 cc = fd2_product<double>(P0 / 16, ga, gb);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) Wl[(bi * 16 + (l >> 4) + 4 * rr) * FD2C_LD + (l & 15)] = cc[rr];
    }
    __syncthreads();
    double* zb = a.z2 + f.zoff + (int64_t)c * P1 * P0;
    for (int bi = wv; bi < nb1; bi += FD3_THREADS / WAVE) {
        auto ga = [&](int i, int k0, double* v) {
#pragma unroll
            for (int s = 0; s < 4; ++s) v[s] = U1[(int64_t)(k0 + s) * P1 + bi * 16 + i];
        };
        auto gb = [&](int k0, int j, double* v) {
#pragma unroll
            for (int s = 0; s < 4; ++s) v[s] = Wl[(k0 + s) * FD2C_LD + j];
        };
        const mf_d4 cc = fd2_product<double>(nb1, ga, gb);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) zb[(int64_t)(bi * 16 + (l >> 4) + 4 * rr) * P0 + bj * 16 + (l & 15)] = cc[rr];
    }
}

template <typename T, bool SET>
__global__ __launch_bounds__(FD3_THREADS) void k_fd3_bwd10(FdArgs a, T* __restrict__ x, int ncbmax) {
    extern __shared__ double fd3c_sm[];
    double* Tl = fd3c_sm;
    int k, c, bj;
    FdInfo f;
    if (!fd3_plane_block(a, ncbmax, k, f, c, bj)) return;
    const PatchLev& P = a.L[k];
    const int M0 = P.M[0], M1 = P.M[1], M2 = P.M[2], P0 = f.P0, P1 = f.P1, nb1 = P1 / 16;
    if (bj * 16 >= M0 || c >= M2) return;
    const double* U0 = a.U + f.u0;
    const double* U1 = a.U + f.u1;
    const double* zb = a.z2 + f.zoff + (int64_t)c * P1 * P0;
    const int wv = threadIdx.x / WAVE, l = threadIdx.x & (WAVE - 1);
    for (int bi = wv; bi < nb1; bi += FD3_THREADS / WAVE) {
        auto ga = [&](int i, int k0, double* v) { load4(zb + (int64_t)(bi * 16 + i) * P0 + k0, v); };
        auto gb = [&](int k0, int j, double* v) { load4(U0 + (int64_t)(bj * 16 + j) * P0 + k0, v); };
        const mf_d4 cc = fd2_product<double>(P0 / 16, ga, gb);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) Tl[(bi * 16 + (l >> 4) + 4 * rr) * FD2C_LD + (l & 15)] = cc[rr];
    }
    __syncthreads();
    const int i0 = bj * 16 + (l & 15);
    for (int bi = wv; bi < nb1; bi += FD3_THREADS / WAVE) {
        if (bi * 16 >= M1) break;
        auto ga = [&](int i, int k0, double* v) { load4(U1 + (int64_t)(bi * 16 + i) * P1 + k0, v); };
        auto gb = [&](int k0, int j, double* v) {
#pragma unroll
            for (int s = 0; s < 4; ++s) v[s] = Tl[(k0 + s) * FD2C_LD + j];
        };
        const mf_d4 cc = fd2_product<double>(nb1, ga, gb);
        double old[4] = {0.0, 0.0, 0.0, 0.0};
        if (!SET) {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int i1 = min(bi * 16 + (l >> 4) + 4 * rr, M1 - 1);
                old[rr] = (double)x[P.voff + min(i0, M0 - 1) + (int64_t)M0 * (i1 + (int64_t)M1 * c)];
            }
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int i1 = bi * 16 + (l >> 4) + 4 * rr;
            if (i0 >= M0 || i1 >= M1) continue;
            const int64_t vi = P.voff + i0 + (int64_t)M0 * (i1 + (int64_t)M1 * c);
            const bool m = masked(P, a.mode, i0, i1, c);
            if (SET) x[vi] = m ? T(0) : T(f.tau * cc[rr]);
            else if (!m) x[vi] = T(old[rr] + f.tau * cc[rr]);
        }
    }
}

}  // namespace ieti
