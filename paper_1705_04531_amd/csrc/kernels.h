// gfx950 kernels of the IETI-DP solve.  Included once, by runtime.hip.
//
// Vectors of one multigrid level hold all patches of that level back to
// back; each patch block is preceded and followed by a zero guard as long as
// the largest linear stencil offset, so stencil reads never leave the
// allocation.  Stencil arrays use the same guarded layout per entry.  Every
// coefficient a mode masks holds 0 in every vector, so a stencil apply needs
// to mask its output only.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.h"

namespace ieti {

constexpr int WAVE = 64;

// ------------------------------------------------------------------ helpers

// Work-group -> tile map: the hardware hands consecutive work-groups to the
// eight XCDs in turn, so give XCD x the contiguous tile range x*per ..
// (x+1)*per-1: neighbouring tiles of a patch share that XCD's L2 for the
// stencil halo.  Launch 8*per work-groups.
__device__ __forceinline__ int tile_index(int ntiles) {
    const int per = (ntiles + 7) >> 3;
    const int b = blockIdx.x;
    const int t = (b & 7) * per + (b >> 3);
    return t < ntiles ? t : -1;
}

__device__ __forceinline__ bool masked_bits(uint32_t mb, int dim, int M0, int M1, int M2, int i0, int i1, int i2) {
    const uint32_t sides = mb & 0xFFu, corners = mb >> 8;
    const bool lo0 = i0 == 0, hi0 = i0 == M0 - 1, lo1 = i1 == 0, hi1 = i1 == M1 - 1;
    const bool lo2 = dim == 3 && i2 == 0, hi2 = dim == 3 && i2 == M2 - 1;
    bool m = (lo0 && (sides & 1u)) || (hi0 && (sides & 2u)) || (lo1 && (sides & 4u)) || (hi1 && (sides & 8u)) ||
             (lo2 && (sides & 16u)) || (hi2 && (sides & 32u));
    const bool corner = (lo0 || hi0) && (lo1 || hi1) && (dim == 2 || lo2 || hi2);
    const int cb = (hi0 ? 1 : 0) | (hi1 ? 2 : 0) | (hi2 ? 4 : 0);
    if (corner && ((corners >> cb) & 1u)) m = true;
    return m;
}

__device__ __forceinline__ bool masked(const PatchLev& P, int mode, int i0, int i1, int i2) {
    return masked_bits(P.mbits[mode], P.dim, P.M[0], P.M[1], P.M[2], i0, i1, i2);
}

__device__ __forceinline__ void unlin(const PatchLev& P, int64_t i, int& i0, int& i1, int& i2) {
    const int M0 = P.M[0], M01 = P.M[0] * P.M[1];
    const int ii = (int)i;
    i2 = ii / M01;
    const int r = ii - i2 * M01;
    i1 = r / M0;
    i0 = r - i1 * M0;
}

// sum of the per-tile partials v[S u + c], u = beg .. end-1, for c < NS, added in
// index order (as a plain loop would) with eight loads in flight
template <int NS>
__device__ __forceinline__ void ordered_sums(const double* __restrict__ v, int beg, int end, double (&s)[NS]) {
#pragma unroll
    for (int c = 0; c < NS; ++c) s[c] = 0.0;
    int u = beg;
    for (; u + 8 <= end; u += 8) {
        double t[8][NS];
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int c = 0; c < NS; ++c) t[j][c] = v[NS * (u + j) + c];
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int c = 0; c < NS; ++c) s[c] += t[j][c];
    }
    for (; u < end; ++u)
#pragma unroll
        for (int c = 0; c < NS; ++c) s[c] += v[NS * u + c];
}

// deterministic block sum of NV doubles (blockDim.x == TILE); result valid in thread 0
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
        for (int o = WAVE / 2; o > 0; o >>= 1) v[k] += __shfl_down(v[k], o, WAVE);
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[w * NV + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x / WAVE;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int j = 0; j < nw; ++j) s += lds[j * NV + k];
            v[k] = s;
        }
    }
    __syncthreads();
}

// dst[j] = src[j], j < n, by the whole work-group with U loads per thread in
// flight before the first store (a plain copy loop waits out one memory
// latency per element and thread).
template <int U, typename T>
__device__ __forceinline__ void group_copy(T* dst, const T* __restrict__ src, int n) {
    const int nt = blockDim.x;
    for (int base = threadIdx.x; base < n; base += U * nt) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = base + u * nt;
            if (j < n) v[u] = src[j];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = base + u * nt;
            if (j < n) dst[j] = v[u];
        }
    }
}

// As group_copy for ne rows of w elements, row e from src + e * sstride to
// dst + e * w.
template <int U, typename T>
__device__ __forceinline__ void group_copy_rows(T* dst, const T* __restrict__ src, int ne, int w, int64_t sstride) {
    const int nt = blockDim.x, n = ne * w;
    for (int base = threadIdx.x; base < n; base += U * nt) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = base + u * nt;
            if (j < n) {
                const int e = j / w;
                v[u] = src[(int64_t)e * sstride + (j - e * w)];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = base + u * nt;
            if (j < n) dst[j] = v[u];
        }
    }
}

// ------------------------------------------------------------------ degree classes
//
// Loops over stencil offsets and transfer bands are unrolled for the common
// degrees (one kernel instance per class, see degree_class) so that every
// load of a work-item is in flight at once and no instance carries the
// register needs of another.  P0 < 0 selects generic loops.

// sum_o K(i, i+o) x(i+o) over the full stencil from the half stencil at i
// (upper half) and at i-o (lower half, by symmetry); diag = K(i, i).
// P0 < 0: degrees p0..p2 at run time.
template <int P0, int P1, int P2, typename TC, typename TX>
__device__ __forceinline__ TC stencil_sum(const TC* __restrict__ c, const TX* __restrict__ xp, int cs, int M0,
                                          int M01, int p0, int p1, int p2, TC& diag) {
    TC acc = TC(0);
    if constexpr (P0 >= 0) {
        int s = 0;
#pragma unroll
        for (int o2 = 0; o2 <= P2; ++o2)
#pragma unroll
            for (int o1 = (o2 == 0 ? 0 : -P1); o1 <= P1; ++o1)
#pragma unroll
                for (int o0 = ((o2 == 0 && o1 == 0) ? 0 : -P0); o0 <= P0; ++o0) {
                    const int off = o0 + o1 * M0 + o2 * M01;
                    const TC cu = c[s * cs];
                    if (s == 0) {
                        diag = cu;
                        acc += cu * TC(xp[0]);
                    } else {
                        acc += cu * TC(xp[off]) + c[s * cs - off] * TC(xp[-off]);
                    }
                    ++s;
                }
    } else {
        int s = 0;
        for (int o2 = 0; o2 <= p2; ++o2)
            for (int o1 = (o2 == 0 ? 0 : -p1); o1 <= p1; ++o1) {
                const int o0s = (o2 == 0 && o1 == 0) ? 0 : -p0;
                const int base = o1 * M0 + o2 * M01;
                for (int o0 = o0s; o0 <= p0; ++o0, ++s) {
                    const int off = base + o0;
                    const TC cu = c[s * cs];
                    if (s == 0) {
                        diag = cu;
                        acc += cu * TC(xp[0]);
                    } else {
                        acc += cu * TC(xp[off]) + c[s * cs - off] * TC(xp[-off]);
                    }
                }
            }
    }
    return acc;
}

// As stencil_sum for 3D classes, one o2-plane of the stencil per loop trip
// (the plane's offsets unrolled): bounds the registers of a 125-point
// stencil while keeping a plane's loads in flight together.
template <int P0, int P1, int P2, typename TC, typename TX>
__device__ __forceinline__ TC stencil_sum_planes(const TC* __restrict__ c, const TX* __restrict__ xp, int cs, int M0,
                                                 int M01, TC& diag) {
    TC acc = TC(0);
    int s = 0;
#pragma unroll
    for (int o1 = 0; o1 <= P1; ++o1)
#pragma unroll
        for (int o0 = (o1 == 0 ? 0 : -P0); o0 <= P0; ++o0) {
            const int off = o0 + o1 * M0;
            const TC cu = c[s * cs];
            if (s == 0) {
                diag = cu;
                acc += cu * TC(xp[0]);
            } else {
                acc += cu * TC(xp[off]) + c[s * cs - off] * TC(xp[-off]);
            }
            ++s;
        }
    constexpr int PLANE = (2 * P1 + 1) * (2 * P0 + 1);
#pragma unroll 1
    for (int o2 = 1; o2 <= P2; ++o2) {
        const TC* cp = c + (s + (o2 - 1) * PLANE) * cs;
        const int zo = o2 * M01;
#pragma unroll
        for (int o1 = -P1; o1 <= P1; ++o1)
#pragma unroll
            for (int o0 = -P0; o0 <= P0; ++o0) {
                const int off = zo + o1 * M0 + o0;
                const int sj = (o1 + P1) * (2 * P0 + 1) + (o0 + P0);
                acc += cp[sj * cs] * TC(xp[off]) + cp[sj * cs - off] * TC(xp[-off]);
            }
    }
    return acc;
}

// As stencil_sum, but only the innermost offset loop is unrolled (fewer
// registers; used inside the coarse-level kernel).
template <int P0, typename TC, typename TX>
__device__ __forceinline__ TC stencil_sum_rows(const TC* __restrict__ c, const TX* __restrict__ xp, int cs, int M0,
                                               int M01, int p0, int p1, int p2, TC& diag) {
    TC acc = TC(0);
    int s = 0;
    for (int o2 = 0; o2 <= p2; ++o2)
        for (int o1 = (o2 == 0 ? 0 : -p1); o1 <= p1; ++o1) {
            const int base = o1 * M0 + o2 * M01;
            if (o2 == 0 && o1 == 0) {
                // row of the diagonal: offsets 0..p0
                const TC c0 = c[0];
                diag = c0;
                acc += c0 * TC(xp[0]);
                if constexpr (P0 >= 0) {
#pragma unroll
                    for (int o0 = 1; o0 <= P0; ++o0)
                        acc += c[o0 * cs] * TC(xp[o0]) + c[o0 * cs - o0] * TC(xp[-o0]);
                    s = P0 + 1;
                } else {
                    for (int o0 = 1; o0 <= p0; ++o0) acc += c[o0 * cs] * TC(xp[o0]) + c[o0 * cs - o0] * TC(xp[-o0]);
                    s = p0 + 1;
                }
            } else {
                if constexpr (P0 >= 0) {
#pragma unroll
                    for (int o0 = -P0; o0 <= P0; ++o0) {
                        const int off = base + o0;
                        const int sj = s + o0 + P0;
                        acc += c[sj * cs] * TC(xp[off]) + c[sj * cs - off] * TC(xp[-off]);
                    }
                    s += 2 * P0 + 1;
                } else {
                    for (int o0 = -p0; o0 <= p0; ++o0) {
                        const int off = base + o0;
                        const int sj = s + o0 + p0;
                        acc += c[sj * cs] * TC(xp[off]) + c[sj * cs - off] * TC(xp[-off]);
                    }
                    s += 2 * p0 + 1;
                }
            }
        }
    return acc;
}

// As stencil_sum_rows (same accumulation order) for compile-time degrees: after the diagonal row, the
// NR = P1 + P2 (2 P1 + 1) further stencil rows in trips of R rows (a loop that is not unrolled, its body
// unrolled), so that the loads of R rows are in flight together: a work-item waits on memory 1 + NR/R
// times instead of 1 + NR, with the registers of R rows.  Used where the coarse-level kernel reads the
// operator from memory.
template <int P0, int P1, int P2>
__host__ __device__ constexpr int chunk_rows() {
    // the largest divisor of NR with at most 40 coefficient loads per trip
    const int nr = P1 + P2 * (2 * P1 + 1);
    int best = 1;
    for (int r = 1; r <= nr; ++r)
        if (nr % r == 0 && 2 * (2 * P0 + 1) * r <= 40) best = r;
    return best;
}

template <int P0, int P1, int P2, typename TC, typename TX>
__device__ __forceinline__ TC stencil_sum_chunked(const TC* __restrict__ c, const TX* __restrict__ xp, int cs,
                                                  int M0, int M01, TC& diag) {
    constexpr int W = 2 * P0 + 1, NR = P1 + P2 * (2 * P1 + 1), R = chunk_rows<P0, P1, P2>();
    static_assert(NR % R == 0, "trips of whole row groups");
    TC acc = TC(0);
    const TC c0 = c[0];
    diag = c0;
    acc += c0 * TC(xp[0]);
#pragma unroll
    for (int o0 = 1; o0 <= P0; ++o0) acc += c[o0 * cs] * TC(xp[o0]) + c[o0 * cs - o0] * TC(xp[-o0]);
#pragma unroll 1
    for (int q0 = 0; q0 < NR; q0 += R) {
        // the trip's coefficients into registers first, then the products: written this way the loads are
        // issued together (interleaved with the products, the scheduler of a kernel near its register
        // budget waits on each pair)
        TC cu[R * W], cl[R * W];
        int offs[R];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            // row q after the diagonal one: (o1, o2) = (q + 1, 0) in the o2 = 0 plane, then the planes o2 >= 1
            // from o1 = -P1
            const int q = q0 + rr;
            const int t = q - P1;
            const int o2 = q < P1 ? 0 : 1 + t / (2 * P1 + 1);
            const int o1 = q < P1 ? q + 1 : t % (2 * P1 + 1) - P1;
            offs[rr] = o1 * M0 + o2 * M01;
            const int s = P0 + 1 + q * W;
#pragma unroll
            for (int o0 = -P0; o0 <= P0; ++o0) {
                const int sj = s + o0 + P0;
                cu[rr * W + o0 + P0] = c[sj * cs];
                cl[rr * W + o0 + P0] = c[sj * cs - offs[rr] - o0];
            }
        }
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int o0 = -P0; o0 <= P0; ++o0) {
                const int off = offs[rr] + o0;
                acc += cu[rr * W + o0 + P0] * TC(xp[off]) + cl[rr * W + o0 + P0] * TC(xp[-off]);
            }
    }
    return acc;
}

// Tensor transfer sum over a band: sum_{a} v0[a0] v1[a1] v2[a2] src[row(a1,a2) + lo0 + a0]
// with compile-time band widths W = p + 2 (W < 0: run time w0..w2).
template <int W0, int W1, int W2, typename T>
__device__ __forceinline__ double band_sum(const T* __restrict__ v0, const T* __restrict__ v1,
                                           const T* __restrict__ v2, const T* __restrict__ src, int M0, int M01,
                                           int w0, int w1, int w2, int dim) {
    double acc = 0.0;
    if constexpr (W0 > 0) {
#pragma unroll
        for (int a2 = 0; a2 < W2; ++a2) {
            const double f2 = W2 > 1 ? (double)v2[a2] : 1.0;
#pragma unroll
            for (int a1 = 0; a1 < W1; ++a1) {
                const double f12 = f2 * (double)v1[a1];
                const T* row = src + a1 * M0 + a2 * M01;
#pragma unroll
                for (int a0 = 0; a0 < W0; ++a0) acc += f12 * (double)v0[a0] * (double)row[a0];
            }
        }
    } else {
        for (int a2 = 0; a2 < w2; ++a2) {
            const double f2 = dim == 3 ? (double)v2[a2] : 1.0;
            for (int a1 = 0; a1 < w1; ++a1) {
                const double f12 = f2 * (double)v1[a1];
                const T* row = src + a1 * M0 + a2 * M01;
                for (int a0 = 0; a0 < w0; ++a0) acc += f12 * (double)v0[a0] * (double)row[a0];
            }
        }
    }
    return acc;
}

// ------------------------------------------------------------------ stencil apply

enum Epi : int {
    EPI_APPLY = 0,   // y = alpha * m (K x)
    EPI_RESID = 1,   // y = m (b - K x)
    EPI_CHEB = 2,    // r = b - K x; d = s1 d + s2 r / diag; y = x + d  (y, d written)
    EPI_DOTS = 3,    // y = m (K x); partial[tile] = (x . y, x . r64)
    EPI_CHEB0 = 4,   // the first two Chebyshev steps from x = 0: x1 = d1 = m s2_0 b / diag (not stored),
                     // then EPI_CHEB step 1 from x1 (finest-level staged instances only; x unused)
};

struct StencilArgs {
    const PatchLev* L;
    const Tile* tiles;
    int ntiles;
    int mode;
    const void* coef;
    const void* x;
    void* y;
    const void* b;         // EPI_RESID, EPI_CHEB
    void* d;               // EPI_CHEB
    const int* active;     // per patch, or null
    double alpha;          // EPI_APPLY
    int cheb_k;            // EPI_CHEB step
    const double* cheb;    // EPI_CHEB: (s1, s2) per (patch-level, mode, step)
    double* partial;       // EPI_DOTS: 2 per tile
    const double* r64;     // EPI_DOTS
    const double* dotq;    // EPI_CHEB: if set, dpart[tile] = sum of y . dotq over the tile
    double* dpart;
};

// One thread per output coefficient; reads K(i, i+o) at i and K(i-o, i) at
// i-o (symmetry) for the lower half of the stencil.  FINE marks launches on
// the finest level (the bandwidth-bound sweeps) so that profilers report
// them apart from the latency-bound coarse-level launches.
// Finest-level sweeps stage the tile's x window [start - reach, start + TILE
// + reach), reach = p2 M0 M1 + p1 M0 + p0 (the guard length), in LDS: each x
// value then passes the vector memory pipeline once per tile instead of once
// per stencil entry.  The window is clipped to the patch block and its
// guards, so the loads stay inside the vector.  Launches of these instances
// must supply (TILE + 2 reach) elements of dynamic LDS; the host uses the
// FINE = false instance where that is too large.  2D issues every
// coefficient load before the window barrier; 3D (125-point stencils) keeps
// the compiler's interleaving of loads and FMAs (registers).
template <int P0, int P2, bool FINE>
__host__ __device__ constexpr bool stencil_stages_x() {
    return FINE && P0 >= 0;
}

// The x window of a staged sweep: a copy of x, or for EPI_CHEB0 the first
// Chebyshev iterate x1 = m s2_0 b / diag computed from b and the stencil's
// diagonal (0 outside the patch).
template <int EPI, typename TC, typename TX, typename TY>
__device__ __forceinline__ void fill_window(TX* win, const StencilArgs& a, const PatchLev& P, const Tile& tl,
                                            int reach, int w_len) {
    if constexpr (EPI == EPI_CHEB0) {
        const TY* b = (const TY*)a.b;
        const TC* dg = (const TC*)a.coef + P.coff;
        const double s2 = a.cheb[2 * (((int64_t)tl.pl * 2 + a.mode) * KMAX) + 1];
        const int n = (int)P.n, M0 = P.M[0], M1 = P.M[1], M01 = M0 * M1;
        constexpr int U = 4;
        for (int base = threadIdx.x; base < w_len; base += U * TILE) {
            double bv[U], dv[U];
            bool on[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = base + u * TILE, g = tl.start - reach + j;
                on[u] = j < w_len && g >= 0 && g < n;
                if (on[u]) {
                    const int g2 = g / M01, r = g - g2 * M01, g1 = r / M0, g0 = r - g1 * M0;
                    on[u] = !masked_bits(P.mbits[a.mode], P.dim, M0, M1, P.M[2], g0, g1, g2);
                }
                bv[u] = on[u] ? (double)b[P.voff + g] : 0.0;
                dv[u] = on[u] ? (double)dg[g] : 1.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = base + u * TILE;
                if (j < w_len) win[j] = on[u] ? TX(s2 * bv[u] / dv[u]) : TX(0);
            }
        }
    } else {
        group_copy<4>(win, (const TX*)a.x + P.voff + tl.start - reach, w_len);
    }
}

template <int P0, int P1, int P2, typename TC, typename TX, typename TY, int EPI, bool FINE>
__device__ __forceinline__ void stencil_body(const StencilArgs& a, const Tile& tl, double* lds,
                                             unsigned char* st_lds_raw) {
    constexpr bool STAGE = stencil_stages_x<P0, P2, FINE>();
    const PatchLev& P = a.L[tl.pl];
    if (a.active && !a.active[P.patch]) return;
    const int n = (int)P.n;
    const int i = tl.start + (int)threadIdx.x;
    const TC* __restrict__ coef = (const TC*)a.coef;
    const TX* __restrict__ x = (const TX*)a.x;
    TY* __restrict__ y = (TY*)a.y;
    double dv0 = 0.0, dv1 = 0.0;
    const int M0 = P.M[0], M1 = P.M[1], M01 = M0 * M1;
    const bool live = i < n;
    bool m = true;
    if (live) {
        const int i2 = i / M01, r = i - i2 * M01, i1 = r / M0, i0 = r - i1 * M0;
        m = masked_bits(P.mbits[a.mode], P.dim, M0, M1, P.M[2], i0, i1, i2);
    }
    const int64_t vi = P.voff + i;
    TC acc = TC(0), diag = TC(1);
    TX xi = TX(0);
    if constexpr (STAGE && P2 > 0) {
        const int reach = P2 * M01 + P1 * M0 + P0;
        TX* win = (TX*)st_lds_raw;
        const int w_len = min(tl.start + TILE, n) + 2 * reach - tl.start;   // clipped to the patch and its guards
        fill_window<EPI, TC, TX, TY>(win, a, P, tl, reach, w_len);
        __syncthreads();
        const TX* xw = win + reach + (int)threadIdx.x;
        if (live) xi = xw[0];
        if (!m) acc = stencil_sum_planes<P0, P1, P2>(coef + P.coff + i, xw, (int)P.cstride, M0, M01, diag);
    } else if constexpr (STAGE) {
        // every coefficient load is issued before the window barrier
        constexpr int NH = (P0 + 1) + P1 * (2 * P0 + 1);
        TC cu[NH], cw[NH];
        const TC* c = coef + P.coff + i;
        const int cs = (int)P.cstride;
        if (!m) {
            int s = 0;
#pragma unroll
            for (int o1 = 0; o1 <= P1; ++o1)
#pragma unroll
                for (int o0 = (o1 == 0 ? 0 : -P0); o0 <= P0; ++o0) {
                    cu[s] = c[s * cs];
                    cw[s] = s == 0 ? TC(0) : c[s * cs - (o0 + o1 * M0)];
                    ++s;
                }
        }
        const int reach = P1 * M0 + P0;
        TX* win = (TX*)st_lds_raw;
        const int w_len = min(tl.start + TILE, n) + 2 * reach - tl.start;   // clipped to the patch and its guards
        fill_window<EPI, TC, TX, TY>(win, a, P, tl, reach, w_len);
        __syncthreads();
        const TX* xw = win + reach + (int)threadIdx.x;
        if (live) xi = xw[0];
        if (!m) {
            diag = cu[0];
            acc += cu[0] * TC(xi);
            int s = 1;
#pragma unroll
            for (int o1 = 0; o1 <= P1; ++o1)
#pragma unroll
                for (int o0 = (o1 == 0 ? 1 : -P0); o0 <= P0; ++o0) {
                    const int off = o0 + o1 * M0;
                    acc += cu[s] * TC(xw[off]) + cw[s] * TC(xw[-off]);
                    ++s;
                }
        }
    } else {
        if (live) xi = x[vi];
        if constexpr (P0 >= 0 && P2 > 0) {
            if (!m) acc = stencil_sum_planes<P0, P1, P2>(coef + P.coff + i, x + vi, (int)P.cstride, M0, M01, diag);
        } else {
            if (!m)
                acc = stencil_sum<P0, P1, P2>(coef + P.coff + i, x + vi, (int)P.cstride, M0, M01, P.p[0], P.p[1],
                                              P.p[2], diag);
        }
    }
    if (live) {
        if constexpr (EPI == EPI_APPLY) {
            y[vi] = m ? TY(0) : TY(a.alpha * (double)acc);
        } else if constexpr (EPI == EPI_RESID) {
            const TY* b = (const TY*)a.b;
            y[vi] = m ? TY(0) : TY(TC(b[vi]) - acc);
        } else if constexpr (EPI == EPI_CHEB || EPI == EPI_CHEB0) {
            const TY* b = (const TY*)a.b;
            TY* d = (TY*)a.d;
            if (m) {
                y[vi] = TY(0);
                d[vi] = TY(0);
            } else {
                const double* cc = a.cheb + 2 * (((int64_t)tl.pl * 2 + a.mode) * KMAX + a.cheb_k);
                const TC s1 = TC(cc[0]), s2 = TC(cc[1]);
                const TC rr = TC(b[vi]) - acc;
                // EPI_CHEB0: the previous direction d1 equals x1
                const TC dprev = EPI == EPI_CHEB0 ? TC(xi) : (a.cheb_k > 0 ? TC(d[vi]) : TC(0));
                const TC dn = (EPI == EPI_CHEB0 || a.cheb_k > 0 ? s1 * dprev : TC(0)) + s2 * rr / diag;
                d[vi] = TY(dn);
                const TY yn = TY(TC(xi) + dn);
                y[vi] = yn;
                if (a.dotq) dv0 = (double)yn * a.dotq[vi];
            }
        } else if constexpr (EPI == EPI_DOTS) {
            const double q = m ? 0.0 : (double)acc;
            y[vi] = TY(q);
            const double xv = (double)xi;
            dv0 = xv * q;
            dv1 = xv * a.r64[vi];
        }
    }
    if constexpr (EPI == EPI_DOTS) {
        double dv[2] = {dv0, dv1};
        block_sum<2>(dv, lds);
        if (threadIdx.x == 0) {
            a.partial[2 * tl.gid] = dv[0];
            a.partial[2 * tl.gid + 1] = dv[1];
        }
    }
    if constexpr (EPI == EPI_CHEB || EPI == EPI_CHEB0) {
        if (a.dotq) {
            double dv[1] = {dv0};
            block_sum<1>(dv, lds);
            if (threadIdx.x == 0) a.dpart[tl.gid] = dv[0];
        }
    }
}

template <int P0, int P1, int P2, typename TC, typename TX, typename TY, int EPI, bool FINE>
__global__ __launch_bounds__(TILE) void k_stencil(StencilArgs a) {
    __shared__ double lds[2 * TILE / WAVE];
    extern __shared__ unsigned char st_lds_raw[];
    const int t = tile_index(a.ntiles);
    if (t < 0) return;
    const Tile tl = a.tiles[t];
    stencil_body<P0, P1, P2, TC, TX, TY, EPI, FINE>(a, tl, lds, st_lds_raw);
}

// Finest-level sweep over the tiles of several 2D degree classes in one
// launch (levels that mix degrees): each work-group takes its tile's class
// instance (a uniform branch).  Registers are those of the largest class.
template <typename TC, typename TX, typename TY, int EPI>
__global__ __launch_bounds__(TILE) void k_stencil_2d(StencilArgs a) {
    __shared__ double lds[2 * TILE / WAVE];
    extern __shared__ unsigned char st_lds_raw[];
    const int t = tile_index(a.ntiles);
    if (t < 0) return;
    const Tile tl = a.tiles[t];
    switch (a.L[tl.pl].pclass) {
    case 0: stencil_body<2, 2, 0, TC, TX, TY, EPI, true>(a, tl, lds, st_lds_raw); break;
    case 1: stencil_body<3, 2, 0, TC, TX, TY, EPI, true>(a, tl, lds, st_lds_raw); break;
    case 2: stencil_body<4, 2, 0, TC, TX, TY, EPI, true>(a, tl, lds, st_lds_raw); break;
    case 3: stencil_body<2, 3, 0, TC, TX, TY, EPI, true>(a, tl, lds, st_lds_raw); break;
    case 4: stencil_body<3, 3, 0, TC, TX, TY, EPI, true>(a, tl, lds, st_lds_raw); break;
    case 5: stencil_body<4, 3, 0, TC, TX, TY, EPI, true>(a, tl, lds, st_lds_raw); break;
    case 6: stencil_body<2, 4, 0, TC, TX, TY, EPI, true>(a, tl, lds, st_lds_raw); break;
    case 7: stencil_body<3, 4, 0, TC, TX, TY, EPI, true>(a, tl, lds, st_lds_raw); break;
    case 8: stencil_body<4, 4, 0, TC, TX, TY, EPI, true>(a, tl, lds, st_lds_raw); break;
    default: break;
    }
}

// ------------------------------------------------------------------ smoother start, transfers, coarse solve

// First Chebyshev step from a zero guess: x = d = m b / (theta diag)
template <typename T>
__global__ __launch_bounds__(TILE) void k_cheb_zero(const PatchLev* L, const Tile* tiles, int ntiles, const T* coef,
                                                    const T* b, T* x, T* d, int mode, const double* cheb,
                                                    const int* active) {
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev& P = L[tl.pl];
    if (active && !active[P.patch]) return;
    const int i = tl.start + (int)threadIdx.x;
    if (i >= (int)P.n) return;
    int i0, i1, i2;
    unlin(P, i, i0, i1, i2);
    const int64_t vi = P.voff + i;
    if (masked(P, mode, i0, i1, i2)) {
        x[vi] = T(0);
        d[vi] = T(0);
        return;
    }
    const double s2 = cheb[2 * (((int64_t)tl.pl * 2 + mode) * KMAX) + 1];
    const double v = s2 * (double)b[vi] / (double)coef[P.coff + i];
    x[vi] = T(v);
    d[vi] = T(v);
}

// Width of a row of the nested prolongation (knot insertion at every element
// midpoint): a fine coefficient of degree p is a combination of at most
// (p + 1) / 2 + 1 consecutive coarse coefficients, while a coarse B-spline is
// a combination of p + 2 fine ones (a column of the prolongation: the
// restriction's width).
__host__ __device__ constexpr int prol_width(int p) { return (p + 1) / 2 + 1; }

template <int PA, int PB, bool PROL, typename T>
__device__ __forceinline__ double band_sum_2d(const T* v0, const T* v1, const T* src, int M0, int M01) {
    constexpr int W0 = PROL ? prol_width(PA) : PA + 2, W1 = PROL ? prol_width(PB) : PB + 2;
    return band_sum<W0, W1, 1>(v0, v1, v1, src, M0, M01, W0, W1, 1, 2);
}

// Transfer band sum for the degree class of F (PROL: a prolongation row, else
// a restriction column): P0 = -2 selects the 2D class of F at run time
// (launches over several classes), else as band_sum.
template <int P0, int P1, int P2, bool PROL, typename T>
__device__ __forceinline__ double band_sum_cls(const PatchLev& F, const T* v0, const T* v1, const T* v2, const T* src,
                                               int M0, int M01) {
    const bool three = F.dim == 3;
    auto w = [](int p) { return PROL ? prol_width(p) : p + 2; };
    if constexpr (P0 == -2) {
        switch (F.pclass) {
        case 0: return band_sum_2d<2, 2, PROL>(v0, v1, src, M0, M01);
        case 1: return band_sum_2d<3, 2, PROL>(v0, v1, src, M0, M01);
        case 2: return band_sum_2d<4, 2, PROL>(v0, v1, src, M0, M01);
        case 3: return band_sum_2d<2, 3, PROL>(v0, v1, src, M0, M01);
        case 4: return band_sum_2d<3, 3, PROL>(v0, v1, src, M0, M01);
        case 5: return band_sum_2d<4, 3, PROL>(v0, v1, src, M0, M01);
        case 6: return band_sum_2d<2, 4, PROL>(v0, v1, src, M0, M01);
        case 7: return band_sum_2d<3, 4, PROL>(v0, v1, src, M0, M01);
        case 8: return band_sum_2d<4, 4, PROL>(v0, v1, src, M0, M01);
        default:
            return band_sum<-1, -1, -1>(v0, v1, v2, src, M0, M01, w(F.p[0]), w(F.p[1]), three ? w(F.p[2]) : 1,
                                        F.dim);
        }
    } else {
        constexpr int W0 = P0 >= 0 ? (PROL ? prol_width(P0) : P0 + 2) : -1;
        constexpr int W1 = P0 >= 0 ? (PROL ? prol_width(P1) : P1 + 2) : -1;
        constexpr int W2 = P0 >= 0 ? (P2 > 0 ? (PROL ? prol_width(P2) : P2 + 2) : 1) : -1;
        return band_sum<W0, W1, W2>(v0, v1, v2, src, M0, M01, w(F.p[0]), w(F.p[1]), three ? w(F.p[2]) : 1, F.dim);
    }
}

// Restriction b_c = m_c P^T r_f, one thread per coarse coefficient (P0 = -2:
// tiles of several 2D classes).
template <int P0, int P1, int P2, typename T>
__global__ __launch_bounds__(TILE) void k_restrict(const PatchLev* Lf, const PatchLev* Lc, const Tile* tiles,
                                                   int ntiles, const int32_t* rlo, const T* rval, const T* rf, T* bc,
                                                   int mode, const int* active) {
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev& C = Lc[tl.pl];
    if (active && !active[C.patch]) return;
    const int I = tl.start + (int)threadIdx.x;
    if (I >= (int)C.n) return;
    const PatchLev& F = Lf[C.fine];
    int I0, I1, I2;
    unlin(C, I, I0, I1, I2);
    if (masked(C, mode, I0, I1, I2)) {
        bc[C.voff + I] = T(0);
        return;
    }
    const bool three = F.dim == 3;
    const int lo0 = rlo[F.roff[0] + I0], lo1 = rlo[F.roff[1] + I1], lo2 = three ? rlo[F.roff[2] + I2] : 0;
    const T* v0 = rval + (F.roff[0] + I0) * PW;
    const T* v1 = rval + (F.roff[1] + I1) * PW;
    const T* v2 = three ? rval + (F.roff[2] + I2) * PW : v1;
    const int M0 = F.M[0], M01 = F.M[0] * F.M[1];
    const T* src = rf + F.voff + lo0 + (int64_t)lo1 * M0 + (int64_t)lo2 * M01;
    bc[C.voff + I] = T(band_sum_cls<P0, P1, P2, false>(F, v0, v1, v2, src, M0, M01));
}

// Prolongation x_f += m_f P e_c, one thread per fine coefficient (P0 = -2:
// tiles of several 2D classes).
template <int P0, int P1, int P2, typename T>
__global__ __launch_bounds__(TILE) void k_prolong(const PatchLev* Lf, const PatchLev* Lc, const Tile* tiles,
                                                  int ntiles, const int32_t* plo, const T* pval, const T* ec, T* xf,
                                                  int mode, const int* active) {
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev& F = Lf[tl.pl];
    if (active && !active[F.patch]) return;
    const int i = tl.start + (int)threadIdx.x;
    if (i >= (int)F.n) return;
    int i0, i1, i2;
    unlin(F, i, i0, i1, i2);
    if (masked(F, mode, i0, i1, i2)) return;
    const PatchLev& C = Lc[F.coarse];
    const bool three = F.dim == 3;
    const int lo0 = plo[F.toff[0] + i0], lo1 = plo[F.toff[1] + i1], lo2 = three ? plo[F.toff[2] + i2] : 0;
    const T* v0 = pval + (F.toff[0] + i0) * PW;
    const T* v1 = pval + (F.toff[1] + i1) * PW;
    const T* v2 = three ? pval + (F.toff[2] + i2) * PW : v1;
    const int M0 = C.M[0], M01 = C.M[0] * C.M[1];
    const T* src = ec + C.voff + lo0 + (int64_t)lo1 * M0 + (int64_t)lo2 * M01;
    const double acc = band_sum_cls<P0, P1, P2, true>(F, v0, v1, v2, src, M0, M01);
    const int64_t vi = F.voff + i;
    xf[vi] = T((double)xf[vi] + acc);
}

// ---- transfers between non-nested levels (degree p finest, degree 1 coarse): the L2 projection of the
// parameter domain, P = D_f M_f^{-1} M_fc D_c, R = P^T (D the masks of the mode).  The mixed mass matrix
// M_fc is a tensor product of 1D bands (rows of the fine level: plo/pval; columns: rlo/rval, width PW);
// M_f^{-1} is applied by 1D banded Cholesky solves along every direction.

// t_f = D_f M_fc e_c (fine tiles)
template <typename T>
__global__ __launch_bounds__(TILE) void k_l2_prolong(const PatchLev* Lf, const PatchLev* Lc, const Tile* tiles,
                                                     int ntiles, const int32_t* plo, const T* pval, const T* ec,
                                                     T* t, int mode, const int* active) {
    const int tt = tile_index(ntiles);
    if (tt < 0) return;
    const Tile tl = tiles[tt];
    const PatchLev& F = Lf[tl.pl];
    if (active && !active[F.patch]) return;
    const int i = tl.start + (int)threadIdx.x;
    if (i >= (int)F.n) return;
    int i0, i1, i2;
    unlin(F, i, i0, i1, i2);
    const int64_t vi = F.voff + i;
    if (masked(F, mode, i0, i1, i2)) {
        t[vi] = T(0);
        return;
    }
    const PatchLev& C = Lc[F.coarse];
    const bool three = F.dim == 3;
    const int lo0 = plo[F.toff[0] + i0], lo1 = plo[F.toff[1] + i1], lo2 = three ? plo[F.toff[2] + i2] : 0;
    const T* v0 = pval + (F.toff[0] + i0) * PW;
    const T* v1 = pval + (F.toff[1] + i1) * PW;
    const T* v2 = three ? pval + (F.toff[2] + i2) * PW : nullptr;
    const int C0 = C.M[0], C1 = C.M[1], C2 = C.M[2];
    double acc = 0.0;
    for (int a2 = 0; a2 < (three ? PW : 1); ++a2) {
        const int j2 = lo2 + a2;
        if (j2 >= C2) break;
        const double w2 = three ? (double)v2[a2] : 1.0;
        for (int a1 = 0; a1 < PW && lo1 + a1 < C1; ++a1) {
            const double w12 = w2 * (double)v1[a1];
            const T* row = ec + C.voff + (int64_t)(j2 * C1 + lo1 + a1) * C0 + lo0;
            for (int a0 = 0; a0 < PW && lo0 + a0 < C0; ++a0) acc += w12 * (double)v0[a0] * (double)row[a0];
        }
    }
    t[vi] = T(acc);
}

// b_c = D_c M_cf t_f (coarse tiles)
template <typename T>
__global__ __launch_bounds__(TILE) void k_l2_restrict(const PatchLev* Lf, const PatchLev* Lc, const Tile* tiles,
                                                      int ntiles, const int32_t* rlo, const T* rval, const T* tf,
                                                      T* bc, int mode, const int* active) {
    const int tt = tile_index(ntiles);
    if (tt < 0) return;
    const Tile tl = tiles[tt];
    const PatchLev& C = Lc[tl.pl];
    if (active && !active[C.patch]) return;
    const int I = tl.start + (int)threadIdx.x;
    if (I >= (int)C.n) return;
    int I0, I1, I2;
    unlin(C, I, I0, I1, I2);
    if (masked(C, mode, I0, I1, I2)) {
        bc[C.voff + I] = T(0);
        return;
    }
    const PatchLev& F = Lf[C.fine];
    const bool three = F.dim == 3;
    const int lo0 = rlo[F.roff[0] + I0], lo1 = rlo[F.roff[1] + I1], lo2 = three ? rlo[F.roff[2] + I2] : 0;
    const T* v0 = rval + (F.roff[0] + I0) * PW;
    const T* v1 = rval + (F.roff[1] + I1) * PW;
    const T* v2 = three ? rval + (F.roff[2] + I2) * PW : nullptr;
    const int M0 = F.M[0], M1 = F.M[1], M2 = F.M[2];
    double acc = 0.0;
    for (int a2 = 0; a2 < (three ? PW : 1); ++a2) {
        const int j2 = lo2 + a2;
        if (j2 >= M2) break;
        const double w2 = three ? (double)v2[a2] : 1.0;
        for (int a1 = 0; a1 < PW && lo1 + a1 < M1; ++a1) {
            const double w12 = w2 * (double)v1[a1];
            const T* row = tf + F.voff + (int64_t)(j2 * M1 + lo1 + a1) * M0 + lo0;
            for (int a0 = 0; a0 < PW && lo0 + a0 < M0; ++a0) acc += w12 * (double)v0[a0] * (double)row[a0];
        }
    }
    bc[C.voff + I] = T(acc);
}

// out = (mask_out ? D_f : I) M_f^{-1} in on the patches of plist (one work-group each, the patch's array in
// LDS): a forward and a backward banded substitution along every line of every direction
template <typename T>
__global__ __launch_bounds__(TILE) void k_mass_solve(const PatchLev* L, const int32_t* plist, int nlist,
                                                     const double* mchol, const T* in, T* out, int mode,
                                                     int mask_out, const int* active) {
    extern __shared__ unsigned char ms_lds_raw[];
    T* a = (T*)ms_lds_raw;
    if ((int)blockIdx.x >= nlist) return;
    const PatchLev& P = L[plist[blockIdx.x]];
    if (active && !active[P.patch]) return;
    const int n = (int)P.n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) a[i] = in[P.voff + i];
    __syncthreads();
    const int M[3] = {P.M[0], P.M[1], P.M[2]};
    for (int d = 0; d < P.dim; ++d) {
        const int Md = M[d], pd = P.p[d], w = pd + 1;
        const int stride = d == 0 ? 1 : (d == 1 ? M[0] : M[0] * M[1]);
        const double* Lc = mchol + P.moff[d];
        const int nlines = n / Md;
        for (int ln = threadIdx.x; ln < nlines; ln += blockDim.x) {
            // line ln: the other coordinates; base index of its entry 0
            int base;
            if (d == 0) base = ln * M[0];
            else if (d == 1) base = (ln % M[0]) + (ln / M[0]) * M[0] * M[1];
            else base = ln;
            for (int i = 0; i < Md; ++i) {   // L y = a
                double v = (double)a[base + i * stride];
                for (int k = (i - pd > 0 ? i - pd : 0); k < i; ++k)
                    v -= Lc[(int64_t)i * w + (k - i + pd)] * (double)a[base + k * stride];
                a[base + i * stride] = T(v / Lc[(int64_t)i * w + pd]);
            }
            for (int i = Md - 1; i >= 0; --i) {   // L^T x = y
                double v = (double)a[base + i * stride];
                for (int k = i + 1; k <= (i + pd < Md - 1 ? i + pd : Md - 1); ++k)
                    v -= Lc[(int64_t)k * w + (i - k + pd)] * (double)a[base + k * stride];
                a[base + i * stride] = T(v / Lc[(int64_t)i * w + pd]);
            }
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        T v = a[i];
        if (mask_out) {
            int i0, i1, i2;
            unlin(P, i, i0, i1, i2);
            if (masked(P, mode, i0, i1, i2)) v = T(0);
        }
        out[P.voff + i] = v;
    }
}

// x += y on the tiles of active patches
template <typename T>
__global__ __launch_bounds__(TILE) void k_add_act(const PatchLev* L, const Tile* tiles, int ntiles, const T* y, T* x,
                                                  const int* active) {
    const int tt = tile_index(ntiles);
    if (tt < 0) return;
    const Tile tl = tiles[tt];
    const PatchLev& P = L[tl.pl];
    if (active && !active[P.patch]) return;
    const int i = tl.start + (int)threadIdx.x;
    if (i >= (int)P.n) return;
    x[P.voff + i] += y[P.voff + i];
}

// Partial dot product of row r of a dense matrix stored by columns (entry
// (r, j) at At[j * n + r]) with b over the columns j0 .. j1-1: U loads in
// flight, the last batch clamped to a valid column and its products skipped.
template <typename T, typename TB>
__device__ __forceinline__ double col_dot(const T* __restrict__ At, int n, const TB* b, int r, int j0, int j1) {
    constexpr int U = 32;
    double acc = 0.0;
    int j = j0;
    for (; j + U <= j1; j += U) {
        T a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = At[(int64_t)(j + u) * n + r];
#pragma unroll
        for (int u = 0; u < U; ++u) acc += (double)a[u] * (double)b[j + u];
    }
    if (j < j1) {
        T a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = At[(int64_t)min(j + u, j1 - 1) * n + r];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j + u < j1) acc += (double)a[u] * (double)b[j + u];
    }
    return acc;
}

// y = A b for a dense n x n matrix stored by columns, by the whole work-group
// (every thread calls it): whole passes of one row per thread, so that every
// column load is contiguous across the lanes and a wave streams whole columns;
// the rows left after the last whole pass (nt of them) are split into G column
// groups, G = min(blockDim / nt, n / 32 rounded up), one (row, group) per
// thread, whose partial sums go to part (at least blockDim doubles, shared) and
// are added in group order.  The split depends only on n and the group size,
// so every call with the same n rounds the same way.  Without part every row
// is one thread's.  (Splitting the columns of every row over four lanes of a
// wave reads shorter runs and measured slower when few groups stream.)
template <typename T, typename TB, typename TY>
__device__ __forceinline__ void col_gemv(const T* __restrict__ At, int n, const TB* b, TY* y, double* part) {
    const int B = blockDim.x, t = threadIdx.x;
    const int nfull = part ? n / B * B : n;
    for (int r = t; r < nfull; r += B) y[r] = TY(col_dot(At, n, b, r, 0, n));
    const int nt = n - nfull;
    if (nt == 0) return;
    const int G = max(1, min(B / nt, (n + 31) / 32));
    const int cw = (n + G - 1) / G;
    if (t < nt * G) {
        const int g = t / nt, r = nfull + (t - g * nt);
        part[t] = col_dot(At, n, b, r, g * cw, min(n, (g + 1) * cw));
    }
    __syncthreads();
    if (t < nt) {
        double acc = part[t];
        for (int g = 1; g < G; ++g) acc += part[g * nt + t];
        y[nfull + t] = TY(acc);
    }
}

// Coarsest level: x = A^{-1} b with the stored dense inverse (by columns);
// one work-group per patch.
template <typename T>
__global__ __launch_bounds__(TILE) void k_coarse(const PatchLev* L, const int32_t* list, int nlist, const T* inv,
                                                 const T* b, T* x, int mode, const int* active) {
    __shared__ double part[TILE];
    if ((int)blockIdx.x >= nlist) return;
    const PatchLev& P = L[list[blockIdx.x]];
    if (active && !active[P.patch]) return;
    const int n = (int)P.n;
    col_gemv(inv + P.invoff + (int64_t)mode * n * n, n, b + P.voff, x + P.voff, part);
}

// ------------------------------------------------------------------ elementwise helpers

template <typename T>
__global__ void k_fill(T* v, int64_t n, T val) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = val;
}

// y += x over the coefficients of a level (guards untouched)
template <typename T>
__global__ __launch_bounds__(TILE) void k_add(const PatchLev* L, const Tile* tiles, int ntiles, const T* x, T* y) {
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev& P = L[tl.pl];
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    if (i >= P.n) return;
    y[P.voff + i] = T((double)y[P.voff + i] + (double)x[P.voff + i]);
}

// y = m x (type conversion + masking)
template <typename TX, typename TY>
__global__ __launch_bounds__(TILE) void k_convert(const PatchLev* L, const Tile* tiles, int ntiles, const TX* x, TY* y,
                                                  int mode, double alpha) {
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev& P = L[tl.pl];
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    if (i >= P.n) return;
    int i0, i1, i2;
    unlin(P, i, i0, i1, i2);
    const int64_t vi = P.voff + i;
    y[vi] = masked(P, mode, i0, i1, i2) ? TY(0) : TY(alpha * (double)x[vi]);
}

// y = y + x (x converted to double), level 0
template <typename TX>
__global__ __launch_bounds__(TILE) void k_add_conv(const PatchLev* L, const Tile* tiles, int ntiles, const TX* x,
                                                   double* y) {
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev& P = L[tl.pl];
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    if (i >= P.n) return;
    y[P.voff + i] += (double)x[P.voff + i];
}

// z = a - b
__global__ __launch_bounds__(TILE) void k_sub(const PatchLev* L, const Tile* tiles, int ntiles, const double* a,
                                              const double* b, double* z) {
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev& P = L[tl.pl];
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    if (i >= P.n) return;
    z[P.voff + i] = a[P.voff + i] - b[P.voff + i];
}

// edge means of NPMAX level-0 vectors: A[k][j][e] = mean of Y_j over edge constraint e of patch k
__global__ __launch_bounds__(TILE) void k_edge_avg(int npatch, const int32_t* npk, const int64_t* edge_ptr,
                                                   const int64_t* edge_dev, const double* Y, int64_t stride,
                                                   double* A) {
    __shared__ double lds[TILE / WAVE];
    const int k = blockIdx.x;
    if (k >= npatch) return;
    const int nj = npk[k];
    for (int j = 0; j < nj; ++j)
        for (int e = 0; e < nj; ++e) {
            const int64_t b = edge_ptr[k * NPMAX + e], en = edge_ptr[k * NPMAX + e + 1];
            double v[1] = {0.0};
            for (int64_t r = b + threadIdx.x; r < en; r += blockDim.x) v[0] += Y[(int64_t)j * stride + edge_dev[r]];
            block_sum<1>(v, lds);
            if (threadIdx.x == 0) A[((int64_t)k * NPMAX + j) * NPMAX + e] = en > b ? v[0] / (double)(en - b) : 0.0;
        }
}

// psiG[s][j] = psi_j[slot_dev[s]]
__global__ void k_psi_slots(int64_t nslots, const int32_t* slot_patch, const int64_t* slot_dev, const int32_t* npk,
                            const double* psi, int64_t stride, double* psiG) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslots) return;
    const int k = slot_patch[s];
    for (int j = 0; j < NPMAX; ++j) psiG[s * NPMAX + j] = j < npk[k] ? psi[(int64_t)j * stride + slot_dev[s]] : 0.0;
}

// ------------------------------------------------------------------ flexible CG on all patches (level 0, FP64)

// x = 0, r = m b, rT = r, d = q = 0, partial = |r|^2
template <typename T>
__global__ __launch_bounds__(TILE) void k_fcg_init(const PatchLev* L, const Tile* tiles, int ntiles, const double* b,
                                                   double* x, double* r, T* rT, double* d, double* q, double* partial,
                                                   int mode) {
    __shared__ double lds[TILE / WAVE];
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev& P = L[tl.pl];
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    double v[1] = {0.0};
    if (i < P.n) {
        int i0, i1, i2;
        unlin(P, i, i0, i1, i2);
        const int64_t vi = P.voff + i;
        const double rv = masked(P, mode, i0, i1, i2) ? 0.0 : b[vi];
        x[vi] = 0.0;
        r[vi] = rv;
        rT[vi] = T(rv);
        d[vi] = 0.0;
        q[vi] = 0.0;
        v[0] = rv * rv;
    }
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) partial[tl.gid] = v[0];
}

// per-tile partial of z . q
template <typename T>
__global__ __launch_bounds__(TILE) void k_fcg_zq(const PatchLev* L, const Tile* tiles, int ntiles, const T* z,
                                                 const double* q, double* partial, const int* active) {
    __shared__ double lds[TILE / WAVE];
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev& P = L[tl.pl];
    if (!active[P.patch]) return;
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    double v[1] = {0.0};
    if (i < P.n) v[0] = (double)z[P.voff + i] * q[P.voff + i];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) partial[tl.gid] = v[0];
}

// d = m (z - beta d), beta = first ? 0 : sum over the patch's tiles of (z . q_prev) / dq
template <typename T>
__global__ __launch_bounds__(TILE) void k_fcg_dir(const PatchLev* L, const Tile* tiles, int ntiles, const T* z,
                                                  double* d, const double* pzq, const int32_t* tile_beg,
                                                  const int32_t* tile_end, const double* dq, int first, int mode,
                                                  const int* active) {
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev& P = L[tl.pl];
    const int k = P.patch;
    if (!active[k]) return;
    double bt = 0.0;
    if (!first) {
        double s[1];
        ordered_sums<1>(pzq, tile_beg[k], tile_end[k], s);
        bt = s[0] / dq[k];
    }
    const int i = tl.start + (int)threadIdx.x;
    if (i >= (int)P.n) return;
    int i0, i1, i2;
    unlin(P, i, i0, i1, i2);
    const int64_t vi = P.voff + i;
    d[vi] = masked(P, mode, i0, i1, i2) ? 0.0 : (double)z[vi] - bt * d[vi];
}

// alpha = sum(d.r) / sum(d.q) over the patch's tiles; x += alpha d, r -= alpha q,
// rT = r, prr = |r|^2 per tile.  The patch's first tile stores dq (for the next
// beta) and flags a breakdown (dq <= 0: alpha = 0).  (The convergence test
// stays a kernel of its own: folding it in through a per-patch arrival
// counter needs a device-scope release fence per work-group, which writes
// back the XCD's L2 and costs more than the launch.)
template <typename T>
__global__ __launch_bounds__(TILE) void k_fcg_update(const PatchLev* L, const Tile* tiles, int ntiles,
                                                     const double* d, const double* q, double* x, double* r, T* rT,
                                                     const double* pdots, const int32_t* tile_beg,
                                                     const int32_t* tile_end, double* dq, int* brk, double* prr,
                                                     const int* active) {
    __shared__ double lds[TILE / WAVE];
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev& P = L[tl.pl];
    const int k = P.patch;
    if (!active[k]) return;
    double sd[2];
    ordered_sums<2>(pdots, tile_beg[k], tile_end[k], sd);
    const double sdq = sd[0], sdr = sd[1];
    const bool ok = sdq > 0.0;
    const double al = ok ? sdr / sdq : 0.0;
    if (threadIdx.x == 0 && tl.gid == tile_beg[k]) {
        dq[k] = sdq;
        if (!ok) brk[k] = 1;
    }
    const int i = tl.start + (int)threadIdx.x;
    double v[1] = {0.0};
    if (i < (int)P.n) {
        const int64_t vi = P.voff + i;
        x[vi] += al * d[vi];
        const double rv = r[vi] - al * q[vi];
        r[vi] = rv;
        rT[vi] = T(rv);
        v[0] = rv * rv;
    }
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) prr[tl.gid] = v[0];
}

// Per-patch convergence, one work-group: init: bb = |r|^2, its = 0, active = bb > 0;
// check: its += 1, active = |r|^2 > tol^2 bb && its < maxit && no breakdown.
// nactive[0] = number of active patches afterwards.
__global__ __launch_bounds__(256) void k_fcg_check(int npatch, const int32_t* tile_beg, const int32_t* tile_end,
                                                   const double* prr, int init, double* bb, int* active, int* its,
                                                   int* brk, double tol2, int maxit, int* nactive) {
    // nactive[1]: sum over patches of iterations of finished solves, nactive[2]: max, nactive[3]: patch solves,
    // nactive[4]: solves retired above the tolerance (iteration limit or breakdown), nactive[5]: solves whose
    // residual is not finite (a NaN or Inf from the V-cycle or the data)
    __shared__ int cnt[256 / WAVE];
    int c = 0;
    for (int k = threadIdx.x; k < npatch; k += blockDim.x) {
        if (!init && !active[k]) continue;
        double ss[1];
        ordered_sums<1>(prr, tile_beg[k], tile_end[k], ss);
        const double s = ss[0];
        if (init) {
            bb[k] = s;
            its[k] = 0;
            brk[k] = 0;
            active[k] = s > 0.0 ? 1 : 0;
        } else {
            its[k] += 1;
            const bool finite = s - s == 0.0;
            const bool above = !finite || s > tol2 * bb[k];
            active[k] = (above && finite && its[k] < maxit && !brk[k]) ? 1 : 0;
            if (!active[k]) {
                atomicAdd(&nactive[1], its[k]);
                atomicMax(&nactive[2], its[k]);
                atomicAdd(&nactive[3], 1);
                if (!finite) atomicAdd(&nactive[5], 1);
                else if (above) atomicAdd(&nactive[4], 1);
            }
        }
        c += active[k];
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) c += __shfl_down(c, o, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) cnt[threadIdx.x / WAVE] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) tot += cnt[w];
        nactive[0] = tot;
    }
}

// ------------------------------------------------------------------ jump operators

// v[slot_dev[s]] = sum_e w_e lam[slot_lam[e]],  w_e = sgn_e (B) or sgn_e / mult (B_D)
__global__ void k_scatter(int64_t nslots, const int64_t* slot_dev, const int64_t* slot_ptr, const int64_t* slot_lam,
                          const double* slot_w, const double* lam, double* v) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslots) return;
    double acc = 0.0;
    for (int64_t e = slot_ptr[s]; e < slot_ptr[s + 1]; ++e) acc += slot_w[e] * lam[slot_lam[e]];
    v[slot_dev[s]] = acc;
}

// out[l] = w_l (v[plus_l] - v[minus_l]); with minus == null: out[l] = w_l v[plus_l]
__global__ void k_gather(int64_t nlam, const int64_t* plus, const int64_t* minus, const double* w, const double* v,
                         double* out) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlam) return;
    const double s = w ? w[l] : 1.0;
    out[l] = minus ? s * (v[plus[l]] - v[minus[l]]) : s * v[plus[l]];
}

// ------------------------------------------------------------------ primal space

// Per patch k (one work-group): c[k][j] = psi_j . g over the patch's rows,
// all j in one pass over g, and, for edge constraints, e[k][j] = mean of y
// over the edge.  Rows are either the patch's interface slots (compact psiG,
// slot-major with NPMAX stride; row_ptr/row_dev give the slots of each patch)
// or, with L0 != null, all coefficients of the patch (psi, j-major).
__global__ __launch_bounds__(TILE) void k_pri_dots(int npatch, const int32_t* npk, const int64_t* row_ptr,
                                                   const int64_t* row_dev, const PatchLev* L0, const double* psi,
                                                   int64_t psi_stride, const double* g, const double* y,
                                                   const int64_t* edge_ptr, const int64_t* edge_dev, double* c,
                                                   double* e) {
    __shared__ double lds[NPMAX * TILE / WAVE];
    const int k = blockIdx.x;
    if (k >= npatch) return;
    const int nj = npk[k];
    double v[NPMAX];
#pragma unroll
    for (int j = 0; j < NPMAX; ++j) v[j] = 0.0;
    if (L0) {
        const PatchLev& P = L0[k];
        for (int64_t r = threadIdx.x; r < P.n; r += blockDim.x) {
            const double gv = g[P.voff + r];
#pragma unroll
            for (int j = 0; j < NPMAX; ++j)
                if (j < nj) v[j] += psi[(int64_t)j * psi_stride + P.voff + r] * gv;
        }
    } else {
        for (int64_t r = row_ptr[k] + threadIdx.x; r < row_ptr[k + 1]; r += blockDim.x) {
            const double gv = g[row_dev[r]];
#pragma unroll
            for (int j = 0; j < NPMAX; ++j)
                if (j < nj) v[j] += psi[r * NPMAX + j] * gv;
        }
    }
    block_sum<NPMAX>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NPMAX; ++j)
            if (j < nj) c[k * NPMAX + j] = v[j];
    }
    if (!y) {
        if (threadIdx.x == 0)
            for (int j = 0; j < nj; ++j) e[k * NPMAX + j] = 0.0;
        return;
    }
#pragma unroll
    for (int j = 0; j < NPMAX; ++j) {
        v[j] = 0.0;
        if (j < nj) {
            const int64_t eb = edge_ptr[k * NPMAX + j], ee = edge_ptr[k * NPMAX + j + 1];
            for (int64_t r = eb + threadIdx.x; r < ee; r += blockDim.x) v[j] += y[edge_dev[r]];
        }
    }
    block_sum<NPMAX>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NPMAX; ++j)
            if (j < nj) {
                const int64_t cnt = edge_ptr[k * NPMAX + j + 1] - edge_ptr[k * NPMAX + j];
                e[k * NPMAX + j] = cnt > 0 ? v[j] / (double)cnt : 0.0;
            }
    }
}

// u_Pi = S_PiPi^{-1} g_Pi, 64 rows per work-group: every work-group first
// assembles g_Pi (sum of the patch contributions c) in LDS, then its four
// waves split the columns of the inverse (stored by columns: entry (r, K) at
// Sinv[K * npi + r]) and their partial sums are added in a fixed order.
__global__ __launch_bounds__(256) void k_pri_coarse(int64_t npi, const int64_t* pri_ptr, const int64_t* pri_patch,
                                                    const int64_t* pri_local, const double* c, const double* Sinv,
                                                    double* upi) {
    extern __shared__ double sg[];
    __shared__ double part[4][WAVE];
    for (int64_t J = threadIdx.x; J < npi; J += blockDim.x) {
        double s = 0.0;
        for (int64_t q = pri_ptr[J]; q < pri_ptr[J + 1]; ++q) s += c[pri_patch[q] * NPMAX + pri_local[q]];
        sg[J] = s;
    }
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int64_t r = (int64_t)blockIdx.x * WAVE + lane;
    double s = 0.0;
    if (r < npi) {   // the wave's terms in K order, their loads eight at a time (same sums as one at a time)
        int64_t K = w;
        for (; K + 28 < npi; K += 32) {
            double a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = Sinv[(K + 4 * u) * npi + r];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += a[u] * sg[K + 4 * u];
        }
        for (; K < npi; K += 4) s += Sinv[K * npi + r] * sg[K];
    }
    part[w][lane] = s;
    __syncthreads();
    if (w == 0 && r < npi) upi[r] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// coef[k][j] = uPi[R_kj] - e[k][j]
__global__ void k_pri_coef(int npatch, const int32_t* npk, const int64_t* Rk, const double* upi, const double* e,
                           double* coef) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)npatch * NPMAX) return;
    const int k = (int)(q / NPMAX), j = (int)(q % NPMAX);
    coef[q] = j < npk[k] ? upi[Rk[q]] - e[q] : 0.0;
}

// y[slot] += sum_j psiG[slot][j] coef[k][j]
__global__ void k_pri_apply_slots(int64_t nslots, const int32_t* slot_patch, const int64_t* slot_dev,
                                  const int32_t* npk, const double* psiG, const double* coef, double* y) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslots) return;
    const int k = slot_patch[s];
    double acc = 0.0;
    for (int j = 0; j < npk[k]; ++j) acc += psiG[s * NPMAX + j] * coef[k * NPMAX + j];
    y[slot_dev[s]] += acc;
}

// u = y + sum_j psi_j coef[k][j] over all coefficients (level 0)
__global__ __launch_bounds__(TILE) void k_pri_apply_full(const PatchLev* L, const Tile* tiles, int ntiles,
                                                         const int32_t* npk, const double* psi, int64_t psi_stride,
                                                         const double* coef, const double* y, double* u) {
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev& P = L[tl.pl];
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    if (i >= P.n) return;
    const int64_t vi = P.voff + i;
    const int k = P.patch;
    double acc = y[vi];
    for (int j = 0; j < npk[k]; ++j) acc += psi[(int64_t)j * psi_stride + vi] * coef[k * NPMAX + j];
    u[vi] = acc;
}

// ------------------------------------------------------------------ load vector, groups, output

// Load vector f_i = sum_q w_q f(x_q) N_i(x_q) by sum factorisation over the
// patch's tensor grid of Gauss points: pass d contracts direction d of the
// patch's array (directions below d already in coefficients, d and above in
// quadrature points; x0 fastest) with the 1D basis table,
//   out[.., i, ..] = sum over elements e in [i - p, i] and their Gauss points g of N_{i-e}(q) in[.., q, ..],
// q = e (p + 1) + g; pass 0 reads the weighted values w_q f(x_q), the last
// pass writes the coefficients.  One thread per output entry; grid (largest
// output of a patch / TILE, patches).
__global__ __launch_bounds__(TILE) void k_qcontract(const PatchLev* L, const PatchQ* PQ, int d, const double* basis,
                                                    const double* qpw, const double* in, double* out) {
    const int k = blockIdx.y;
    const PatchLev& P = L[k];
    const PatchQ Q = PQ[k];
    const int dim = P.dim;
    int si[3], so[3];
    for (int c = 0; c < 3; ++c) {
        si[c] = c < dim ? (c < d ? P.M[c] : Q.Q[c]) : 1;
        so[c] = c < dim ? (c <= d ? P.M[c] : Q.Q[c]) : 1;
    }
    const int64_t nout = (int64_t)so[0] * so[1] * so[2];
    const int64_t o = (int64_t)blockIdx.x * TILE + threadIdx.x;
    if (o >= nout) return;
    int a[3];
    a[0] = (int)(o % so[0]);
    a[1] = (int)((o / so[0]) % so[1]);
    a[2] = (int)(o / ((int64_t)so[0] * so[1]));
    const int p = P.p[d], np = p + 1, i = a[d];
    const int64_t stride = d == 0 ? 1 : d == 1 ? (int64_t)si[0] : (int64_t)si[0] * si[1];
    a[d] = 0;
    const int64_t base = a[0] + (int64_t)si[0] * (a[1] + (int64_t)si[1] * a[2]);
    const double* src = d == 0 ? in + Q.qoff : in + Q.toff[d - 1];
    const double* wq = d == 0 ? qpw + Q.qoff : nullptr;
    const double* bt = basis + Q.boff[d];
    const int elo = i - p > 0 ? i - p : 0, ehi = i < Q.nel[d] - 1 ? i : Q.nel[d] - 1;
    double acc = 0.0;
    for (int e = elo; e <= ehi; ++e)
        for (int g = 0; g < np; ++g) {
            const int q = e * np + g;
            const int64_t at = base + q * stride;
            const double v = d == 0 ? wq[at] * src[at] : src[at];
            acc += bt[(int64_t)q * np + (i - e)] * v;
        }
    double* dst = d == dim - 1 ? out + P.voff : out + Q.toff[d];
    dst[o] = acc;
}

// mean of every group of copies, written back to all copies
__global__ void k_group_mean(int64_t ngroups, const int64_t* gptr, const int64_t* gdev, double* v) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngroups) return;
    double s = 0.0;
    for (int64_t e = gptr[g]; e < gptr[g + 1]; ++e) s += v[gdev[e]];
    s /= (double)(gptr[g + 1] - gptr[g]);
    for (int64_t e = gptr[g]; e < gptr[g + 1]; ++e) v[gdev[e]] = s;
}

// assemble a torn vector in place: the first copy of every group receives the
// sum of all copies, the other copies are set to 0 (then |v| is the norm of
// the assembled vector)
__global__ void k_group_assemble(int64_t ngroups, const int64_t* gptr, const int64_t* gdev, double* v) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngroups) return;
    double s = 0.0;
    for (int64_t e = gptr[g]; e < gptr[g + 1]; ++e) s += v[gdev[e]];
    v[gdev[gptr[g]]] = s;
    for (int64_t e = gptr[g] + 1; e < gptr[g + 1]; ++e) v[gdev[e]] = 0.0;
}

// per-tile partial of m |v|^2 on level 0
__global__ __launch_bounds__(TILE) void k_sq(const PatchLev* L, const Tile* tiles, int ntiles, const double* v,
                                             int mode, double* partial) {
    __shared__ double lds[TILE / WAVE];
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev& P = L[tl.pl];
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    double acc[1] = {0.0};
    if (i < P.n) {
        int i0, i1, i2;
        unlin(P, i, i0, i1, i2);
        if (!masked(P, mode, i0, i1, i2)) acc[0] = v[P.voff + i] * v[P.voff + i];
    }
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) partial[tl.gid] = acc[0];
}

// out (torn layout) = v (guarded level-0 layout)
__global__ __launch_bounds__(TILE) void k_copy_out(const PatchLev* L, const Tile* tiles, int ntiles,
                                                   const int64_t* torn_off, const double* v, double* out) {
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev& P = L[tl.pl];
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    if (i >= P.n) return;
    out[torn_off[P.patch] + i] = v[P.voff + i];
}

// sum of n doubles in one work-group (fixed order), out[0] = sum
__global__ __launch_bounds__(1024) void k_sum(const double* v, int64_t n, double* out) {
    __shared__ double lds[1024 / WAVE];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += v[i];
    for (int o = WAVE / 2; o > 0; o >>= 1) acc += __shfl_down(acc, o, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) lds[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int j = 0; j < (int)(blockDim.x / WAVE); ++j) s += lds[j];
        out[0] = s;
    }
}

// ------------------------------------------------------------------ outer CG on lambda (one work-group)

__device__ double wg_dot(const double* a, const double* b, int64_t n, double* lds) {
    // a thread's terms in index order, their loads eight strides at a time (same sums as one at a time)
    double acc = 0.0;
    const int64_t st = blockDim.x;
    int64_t i = threadIdx.x;
    for (; i + 7 * st < n; i += 8 * st) {
        double av[8], bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            av[u] = a[i + u * st];
            bv[u] = b[i + u * st];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += av[u] * bv[u];
    }
    for (; i < n; i += st) acc += a[i] * b[i];
    for (int o = WAVE / 2; o > 0; o >>= 1) acc += __shfl_down(acc, o, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) lds[threadIdx.x / WAVE] = acc;
    __syncthreads();
    double s = 0.0;
    for (int j = 0; j < (int)(blockDim.x / WAVE); ++j) s += lds[j];
    __syncthreads();
    return s;
}

// Outer CG of ncomp independent problems at once (one for ieti_solve, several for a serving batch), with the
// scalars of problem c in sc + 16 c: [0] rz, [1] alpha, [2] beta, [3] |r|^2, [4] breakdown flag, [5] |d|^2
// (scale), [6] pq, [7] the new rz before it replaces [0].  Stages: 0 start (p = z, rz), 1 step (pq, alpha,
// lambda += alpha p, r -= alpha q, |r|^2, breakdown flag), 2 direction (rz' = r.z, beta = rz'/rz,
// p = z + beta p, rz = rz').
// The stages run over several work-groups per problem (the outer CG on ~10^5 multipliers would be one CU's
// stream in a single work-group).  Problem c's range is cut into nb_c = pcg_blocks(n_c) chunks (a function of its own size
// only, so that a problem gives the same result alone and in a serving batch); work-group b of problem c
// (grid PCG_NB x ncomp, blocks past nb_c return) takes chunk b.  Partial sums go to part[c PCG_NB + b] and
// are added in chunk order, every time in the same order.
//   k_pcg_part:  part = chunk sums of x.y   (stage 0: r.z, 1: p.q, 2: r.z)
//   k_pcg_apply: s = sum of part, then stage 0: p = z, sc[0] = s; stage 1: alpha = sc[0]/s, lambda += alpha p,
//                r -= alpha q, part2 = chunk sums of r.r, sc[1] alpha, sc[4] breakdown flag, sc[6] pq;
//                stage 2: beta = s/sc[0], p = z + beta p, sc[2] beta, sc[7] = s
//   k_pcg_fin:   stage 1: sc[3] = sum of part2; stage 2: sc[0] = sc[7]
// done[c] != 0: problem c has stopped; stages 0 and 2 zero its search direction (so that F p holds no load
// from it) and stage 1 leaves it alone.
constexpr int PCG_NB = 64, PCG_THREADS = 256;
__host__ __device__ inline int pcg_blocks(int64_t n) {
    const int64_t b = (n + 2047) / 2048;
    return (int)(b < 1 ? 1 : b > PCG_NB ? PCG_NB : b);
}

// chunk sum of x.y over [lo, hi) (terms of a thread in index order, loads four strides at a time), reduced over
// the work-group in a fixed order; valid in every thread
__device__ double chunk_dot(const double* x, const double* y, int64_t lo, int64_t hi, double* lds) {
    double acc = 0.0;
    const int64_t st = blockDim.x;
    int64_t i = lo + threadIdx.x;
    for (; i + 3 * st < hi; i += 4 * st) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = x[i + u * st];
            b[u] = y[i + u * st];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += a[u] * b[u];
    }
    for (; i < hi; i += st) acc += x[i] * y[i];
    for (int o = WAVE / 2; o > 0; o >>= 1) acc += __shfl_down(acc, o, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) lds[threadIdx.x / WAVE] = acc;
    __syncthreads();
    double s = 0.0;
    for (int j = 0; j < (int)(blockDim.x / WAVE); ++j) s += lds[j];
    __syncthreads();
    return s;
}

__device__ __forceinline__ bool pcg_chunk(const int64_t* beg, int c, int b, int64_t& lo, int64_t& hi) {
    const int64_t b0 = beg[c], n = beg[c + 1] - b0;
    const int nb = pcg_blocks(n);
    if (b >= nb) return false;
    const int64_t ch = (n + nb - 1) / nb;
    lo = b0 + b * ch;
    hi = lo + ch < b0 + n ? lo + ch : b0 + n;
    return true;
}

__global__ __launch_bounds__(PCG_THREADS) void k_pcg_part(int stage, const int64_t* beg, const int* done,
                                                          const double* r, const double* z, const double* p,
                                                          const double* q, double* part) {
    __shared__ double lds[PCG_THREADS / WAVE];
    const int c = blockIdx.y, b = blockIdx.x;
    int64_t lo, hi;
    if (!pcg_chunk(beg, c, b, lo, hi) || (done && done[c])) return;
    const double s = stage == 1 ? chunk_dot(p, q, lo, hi, lds) : chunk_dot(r, z, lo, hi, lds);
    if (threadIdx.x == 0) part[c * PCG_NB + b] = s;
}

__global__ __launch_bounds__(PCG_THREADS) void k_pcg_apply(int stage, const int64_t* beg, const int* done,
                                                           double* lam, double* r, const double* z, double* p,
                                                           const double* q, double* sc, const double* part,
                                                           double* part2) {
    __shared__ double lds[PCG_THREADS / WAVE];
    __shared__ double s_sum;
    const int c = blockIdx.y, b = blockIdx.x;
    int64_t lo, hi;
    if (!pcg_chunk(beg, c, b, lo, hi)) return;
    const int64_t st = blockDim.x;
    sc += 16 * c;
    if (done && done[c]) {
        if (stage != 1)
            for (int64_t i = lo + threadIdx.x; i < hi; i += st) p[i] = 0.0;
        return;
    }
    if (threadIdx.x == 0) {
        const int nb = pcg_blocks(beg[c + 1] - beg[c]);
        double t = 0.0;
        for (int j = 0; j < nb; ++j) t += part[c * PCG_NB + j];
        s_sum = t;
    }
    __syncthreads();
    const double s = s_sum;
    if (stage == 0) {
        for (int64_t i = lo + threadIdx.x; i < hi; i += st) p[i] = z[i];
        if (b == 0 && threadIdx.x == 0) sc[0] = s;
    } else if (stage == 1) {
        double alpha = sc[0] / s;
        const bool brk = !(s > 0.0);
        if (brk) alpha = 0.0;
        int64_t i = lo + threadIdx.x;
        for (; i + 3 * st < hi; i += 4 * st) {
            double lv[4], pv[4], rv[4], qv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                lv[u] = lam[i + u * st];
                pv[u] = p[i + u * st];
                rv[u] = r[i + u * st];
                qv[u] = q[i + u * st];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                lam[i + u * st] = lv[u] + alpha * pv[u];
                r[i + u * st] = rv[u] - alpha * qv[u];
            }
        }
        for (; i < hi; i += st) {
            lam[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        __syncthreads();
        const double rr = chunk_dot(r, r, lo, hi, lds);
        if (threadIdx.x == 0) {
            part2[c * PCG_NB + b] = rr;
            if (b == 0) {
                sc[1] = alpha;
                sc[4] = brk ? 1.0 : 0.0;
                sc[6] = s;
            }
        }
    } else {
        const double beta = s / sc[0];
        int64_t i = lo + threadIdx.x;
        for (; i + 3 * st < hi; i += 4 * st) {
            double zv[4], pv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                zv[u] = z[i + u * st];
                pv[u] = p[i + u * st];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) p[i + u * st] = zv[u] + beta * pv[u];
        }
        for (; i < hi; i += st) p[i] = z[i] + beta * p[i];
        if (b == 0 && threadIdx.x == 0) {
            sc[2] = beta;
            sc[7] = s;
        }
    }
}

__global__ void k_pcg_fin(int stage, const int64_t* beg, const int* done, double* sc, const double* part2, int nc) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc || (done && done[c])) return;
    if (stage == 1) {
        const int nb = pcg_blocks(beg[c + 1] - beg[c]);
        double t = 0.0;
        for (int j = 0; j < nb; ++j) t += part2[c * PCG_NB + j];
        sc[16 * c + 3] = t;
    } else {
        sc[16 * c + 0] = sc[16 * c + 7];
    }
}

// |a|^2 and |b|^2 (+ |c|^2) into out[0..2] (one work-group)
// |a|^2, |b|^2, |c|^2 of each problem's multiplier range (work-group per problem) into out + 16 c + {0, 1, 2}
__global__ __launch_bounds__(1024) void k_norms(const int64_t* beg, const double* a, const double* b, const double* c,
                                                double* out) {
    __shared__ double lds[1024 / WAVE];
    const int g = blockIdx.x;
    const int64_t o = beg[g], n = beg[g + 1] - o;
    const double na = wg_dot(a + o, a + o, n, lds);
    const double nb = b ? wg_dot(b + o, b + o, n, lds) : 0.0;
    const double nc = c ? wg_dot(c + o, c + o, n, lds) : 0.0;
    if (threadIdx.x == 0) {
        out[16 * g + 0] = na;
        out[16 * g + 1] = nb;
        out[16 * g + 2] = nc;
    }
}

// Per-problem sums of per-tile partials: work-group c adds the tiles of its patches [pbeg[c], pbeg[c+1]) in patch
// order (tiles of patch k: [tile_beg[k], tile_end[k])) into out[16 c]
__global__ __launch_bounds__(256) void k_sum_comp(const double* partial, const int32_t* tile_beg,
                                                  const int32_t* tile_end, const int64_t* pbeg, double* out) {
    __shared__ double lds[256 / WAVE];
    const int c = blockIdx.x;
    double acc[1] = {0.0};
    for (int64_t k = pbeg[c]; k < pbeg[c + 1]; ++k)
        for (int u = tile_beg[k] + (int)threadIdx.x; u < tile_end[k]; u += blockDim.x) acc[0] += partial[u];
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) out[16 * c] = acc[0];
}

// ------------------------------------------------------------------ setup helpers

// e = unit vector at the corner of local primal column j of every patch (level-0 FP64)
__global__ void k_unit(int npatch, const int64_t* unit_dev, int j, double* v) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npatch) return;
    const int64_t pos = unit_dev[k * NPMAX + j];
    if (pos >= 0) v[pos] = 1.0;
}

// v = 1/n_e on the coefficients of edge constraint j of every patch
// Floating patches (no Dirichlet and no primal-vertex coefficient, K singular on the constants): their local
// Neumann operator is K + gamma sum_e c_e c_e^T, c_e the average over the coefficients of edge constraint e,
// equal to K on {C w = 0}.  After the sweep q = K d with its per-tile dots (d . q): q += gamma sum_e c_e (c_e . d)
// on the edge coefficients and (d . q) += gamma sum_e (c_e . d)^2 on the patch's first tile.  One work-group per
// floating patch; its edges are disjoint, so the updates of q do not meet.
__global__ __launch_bounds__(TILE) void k_float_penalty(int nfloat, const int32_t* flist, const int32_t* npk,
                                                        const int64_t* edge_ptr, const int64_t* edge_dev,
                                                        const double* gam, const double* d, double* q, double* pdots,
                                                        const int32_t* tile_beg, const int* active) {
    __shared__ double lds[TILE / WAVE];
    __shared__ double mean_sh;
    if ((int)blockIdx.x >= nfloat) return;
    const int k = flist[blockIdx.x];
    if (active && !active[k]) return;
    const double g = gam[k];
    double acc = 0.0;
    for (int j = 0; j < npk[k]; ++j) {
        const int64_t b = edge_ptr[k * NPMAX + j], e = edge_ptr[k * NPMAX + j + 1];
        if (e <= b) continue;
        double v[1] = {0.0};
        for (int64_t r = b + threadIdx.x; r < e; r += blockDim.x) v[0] += d[edge_dev[r]];
        block_sum<1>(v, lds);
        if (threadIdx.x == 0) mean_sh = v[0] / (double)(e - b);
        __syncthreads();
        const double mean = mean_sh;
        __syncthreads();
        const double add = g * mean / (double)(e - b);
        for (int64_t r = b + threadIdx.x; r < e; r += blockDim.x) q[edge_dev[r]] += add;
        acc += g * mean * mean;
    }
    if (threadIdx.x == 0) pdots[2 * tile_beg[k]] += acc;
}

__global__ void k_edge_rhs(int npatch, const int64_t* edge_ptr, const int64_t* edge_dev, int j, double* v) {
    const int k = blockIdx.x;
    if (k >= npatch) return;
    const int64_t b = edge_ptr[k * NPMAX + j], e = edge_ptr[k * NPMAX + j + 1];
    for (int64_t r = b + threadIdx.x; r < e; r += blockDim.x) v[edge_dev[r]] = 1.0 / (double)(e - b);
}

// psi_j = unit_j + sum_j' Y_j' T[k][j'][j]   (T: NPMAX x NPMAX per patch)
__global__ __launch_bounds__(TILE) void k_combine(const PatchLev* L, const Tile* tiles, int ntiles, const int32_t* npk,
                                                  const int64_t* unit_dev, const double* Y, const double* T,
                                                  int64_t stride, double* psi) {
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev& P = L[tl.pl];
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    if (i >= P.n) return;
    const int64_t vi = P.voff + i;
    const int k = P.patch;
    const int nj = npk[k];
    for (int j = 0; j < nj; ++j) {
        double acc = unit_dev[k * NPMAX + j] == vi ? 1.0 : 0.0;
        for (int jp = 0; jp < nj; ++jp) acc += Y[(int64_t)jp * stride + vi] * T[((int64_t)k * NPMAX + jp) * NPMAX + j];
        psi[(int64_t)j * stride + vi] = acc;
    }
}

// S[k][i][j] = psi_i . t_j over all coefficients of patch k (t_j = K psi_j), one work-group per patch
__global__ __launch_bounds__(TILE) void k_patch_gram(int npatch, const PatchLev* L, const int32_t* npk,
                                                     const double* psi, const double* t, int64_t stride, int j,
                                                     double* S) {
    __shared__ double lds[TILE / WAVE];
    const int k = blockIdx.x;
    if (k >= npatch) return;
    const PatchLev& P = L[k];
    const int nj = npk[k];
    if (j >= nj) return;
    for (int i = 0; i < nj; ++i) {
        double v[1] = {0.0};
        for (int64_t r = threadIdx.x; r < P.n; r += blockDim.x)
            v[0] += psi[(int64_t)i * stride + P.voff + r] * t[(int64_t)j * stride + P.voff + r];
        block_sum<1>(v, lds);
        if (threadIdx.x == 0) S[((int64_t)k * NPMAX + i) * NPMAX + j] = v[0];
    }
}


// ------------------------------------------------------------------ coarse part of a V-cycle in one kernel
//
// One work-group per patch runs levels l0 .. L-1 of the V-cycle with all
// level vectors in LDS (rhs b, iterate x, its partner y, Chebyshev direction
// d per level; x and y carry zero guards for the stencil reads): Chebyshev
// pre-smoothing, residual, restriction, dense solve on the coarsest level,
// prolongation, Chebyshev post-smoothing.  It replaces about ten launches per
// coarse level, each of them too small to fill the chip.  With STAGE set,
// the half stencils of these levels (each entry with a front guard of the
// stencil reach, for the lower-half reads) and the coarsest inverse of the
// current mode are copied to LDS once per V-cycle, so that the sweeps read
// no operator data from memory: a work-group is bound by the vector memory
// throughput of its one CU otherwise.  STAGE is a template parameter so that
// each instance holds one copy of the sweep (register pressure).

constexpr int LMAX = 12;     // multigrid levels per patch
constexpr int VC_THREADS = 512;
// FP32 3D levels (family 1): 1024 threads per work-group (those instances
// fit in 128 registers), so that a level-1 sweep takes fewer rounds (4^3 cube
// p=2: 215 -> 200 ms per solve); the 2D family measured slower with 1024
// (16x16 mixed workload 183 -> 191 ms) and FP64 needs more registers: 512.
template <typename T, int FAM>
__host__ __device__ constexpr int vc_threads() { return sizeof(T) == 4 && FAM == 1 ? 2 * VC_THREADS : VC_THREADS; }

struct CoarseArgs {
    const PatchLev* L[LMAX];
    const void* coef[LMAX];
    const int32_t* plo[LMAX];
    const void* pval[LMAX];
    const int32_t* rlo[LMAX];
    const void* rval[LMAX];
    const void* inv[LMAX];
    const double* cheb[LMAX];
    const int32_t* chain;     // chain[k * LMAX + l]: index of patch k in level l (-1: no such level)
    const int32_t* plist;     // patches of this launch, one work-group each
    int nlist;
    int l0;                   // first level run by this kernel (>= 1)
    const void* b1;           // level-l0 right-hand side (global, level-l0 layout)
    void* x1;                 // level-l0 correction (global, level-l0 layout)
    int mode;
    int m;                    // Chebyshev degree per smoothing phase
    const int* active;
};

// LDS words the kernel needs for one patch chain: per level x, y (guarded),
// b, d; for the coarsest level the GEMV's partial sums (part_words, and one
// word for their alignment); staged, also nst * (n + guard) stencil words per
// smoothed level and n * n for the coarsest inverse.
__host__ __device__ inline int64_t vcoarse_level_words(int64_t n, int64_t guard, int nst, bool coarsest,
                                                       bool stage, int64_t part_words) {
    int64_t w = 2 * (n + 2 * guard) + 2 * n;
    if (coarsest) w += part_words + 1;
    if (stage) w += coarsest ? n * n : (int64_t)nst * (n + guard);
    return w;
}

// how vc_sweep sums a stencil: every load of a work-item in flight at once (2D
// classes up to degree 3 read from memory); one stencil row at a time (operator
// data in LDS, where the short latency needs no deep load queue and the full
// unroll would spill registers; run-time degrees); chunks of rows (3D classes
// and 2D classes with a degree 4 read from memory)
enum VcForm : int { VC_FULL = 0, VC_ROWS = 1, VC_CHUNK = 2 };

template <int P0, int P1, int P2, bool STAGE>
__host__ __device__ constexpr int vc_form() {
    return STAGE || P0 < 0 ? VC_ROWS : (P2 == 0 && P0 <= 3 && P1 <= 3 ? VC_FULL : VC_CHUNK);
}

// one Chebyshev step (or, with resid, the residual) on a level held in LDS;
// c points at entry 0 of dof 0 of the half stencil, entries cs apart.
template <int P0, int P1, int P2, typename T, int FORM>
__device__ __forceinline__ void vc_sweep(const PatchLev& P, const T* c, int cs, const T* xs, T* ys, const T* bs,
                                         T* ds, int mode, const double* cc, int k, bool resid) {
    const int n = (int)P.n, M0 = P.M[0], M1 = P.M[1], M01 = M0 * M1;
    const double s1 = cc[2 * k], s2 = cc[2 * k + 1];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int i2 = i / M01, r = i - i2 * M01, i1 = r / M0, i0 = r - i1 * M0;
        if (masked_bits(P.mbits[mode], P.dim, M0, M1, P.M[2], i0, i1, i2)) {
            ys[i] = T(0);
            if (!resid) ds[i] = T(0);
            continue;
        }
        T diag = T(1);
        // 2D from memory: every load of a coefficient in flight at once; else one stencil row at a time
        T acc;
        if constexpr (FORM == VC_FULL)
            acc = stencil_sum<P0, P1, P2>(c + i, xs + i, cs, M0, M01, P.p[0], P.p[1], P.p[2], diag);
        else if constexpr (FORM == VC_CHUNK)
            acc = stencil_sum_chunked<P0, P1, P2>(c + i, xs + i, cs, M0, M01, diag);
        else
            acc = stencil_sum_rows<P0>(c + i, xs + i, cs, M0, M01, P.p[0], P.p[1], P.p[2], diag);
        const T rr = bs[i] - acc;
        if (resid) {
            ys[i] = rr;
        } else {
            const T dn = (k > 0 ? T(s1) * ds[i] : T(0)) + T(s2) * rr / diag;
            ds[i] = dn;
            ys[i] = xs[i] + dn;
        }
    }
}

// work-group state of k_vcoarse
struct VcShared {
    int pl[LMAX];        // patch-level index per level
    int off[LMAX][5];    // LDS offsets of x, y (guarded, at entry 0), b, d, operator data
    int cur[LMAX];       // which of x (0) / y (1) holds the level's current iterate
    int nl, vec, part;   // levels, vector words, LDS offset of the coarsest GEMV's partial sums
};

// the cycle of patch k from level a.l0 on, for the degree class P0..P2
template <int P0, int P1, int P2, typename T, bool STAGE>
__device__ __forceinline__ void vcoarse_body(const CoarseArgs& a, int k, T* lds, VcShared& sh) {
    int* sh_pl = sh.pl;
    int (*sh_off)[5] = sh.off;
    int* sh_cur = sh.cur;
    int& sh_nl = sh.nl;
    int& sh_vec = sh.vec;
    const int l0 = a.l0;
    constexpr bool stage = STAGE;
    const int mode = a.mode;
    if (threadIdx.x == 0) {
        int nl = l0 + 1;
        while (nl < LMAX && a.chain[k * LMAX + nl] >= 0) ++nl;
        int off = 0;
        for (int l = l0; l < nl; ++l) {
            const int pl = a.chain[k * LMAX + l];
            sh_pl[l] = pl;
            const PatchLev& P = a.L[l][pl];
            const int n = (int)P.n;
            const int g = P.p[0] + P.p[1] * P.M[0] + P.p[2] * P.M[0] * P.M[1];
            sh_off[l][0] = off + g;
            off += n + 2 * g;
            sh_off[l][1] = off + g;
            off += n + 2 * g;
            sh_off[l][2] = off;
            off += n;
            sh_off[l][3] = off;
            off += n;
            if (l == nl - 1) {
                // partial sums of the coarsest GEMV: blockDim doubles, 8-byte aligned
                off += (int)((off * sizeof(T)) & 7) / (int)sizeof(T);
                sh.part = off;
                off += (int)(blockDim.x * sizeof(double) / sizeof(T));
            }
        }
        sh_vec = off;
        for (int l = l0; l < nl && stage; ++l) {
            const PatchLev& P = a.L[l][sh_pl[l]];
            const int n = (int)P.n;
            const int g = P.p[0] + P.p[1] * P.M[0] + P.p[2] * P.M[0] * P.M[1];
            if (l == nl - 1) {
                sh_off[l][4] = off;
                off += n * n;
            } else {
                sh_off[l][4] = off + g;
                off += (int)P.nst * (n + g);
            }
        }
        sh_nl = nl;
    }
    __syncthreads();
    const int nl = sh_nl;
    for (int i = threadIdx.x; i < sh_vec; i += blockDim.x) lds[i] = T(0);
    // the copies below write words that other waves zero above
    __syncthreads();
    {
        const PatchLev& P = a.L[l0][sh_pl[l0]];
        group_copy<4>(lds + sh_off[l0][2], (const T*)a.b1 + P.voff, (int)P.n);
    }
    if (stage) {
        for (int l = l0; l < nl; ++l) {
            const PatchLev& P = a.L[l][sh_pl[l]];
            const int n = (int)P.n;
            if (l == nl - 1) {
                group_copy<16>(lds + sh_off[l][4], (const T*)a.inv[l] + P.invoff + (int64_t)mode * n * n, n * n);
            } else {
                // entry e, dofs -g .. n-1 (the front guard holds zeros in memory too)
                const int g = P.p[0] + P.p[1] * P.M[0] + P.p[2] * P.M[0] * P.M[1];
                group_copy_rows<16>(lds + sh_off[l][4] - g, (const T*)a.coef[l] + P.coff - g, (int)P.nst, n + g,
                                    P.cstride);
            }
        }
    }
    __syncthreads();
    // ---- down
    for (int l = l0; l < nl; ++l) {
        const int pl = sh_pl[l];
        const PatchLev& P = a.L[l][pl];
        const int n = (int)P.n;
        const int g = P.p[0] + P.p[1] * P.M[0] + P.p[2] * P.M[0] * P.M[1];
        const T* cg = (const T*)a.coef[l] + P.coff;   // half stencil in memory
        const T* cl = lds + sh_off[l][4];              // staged copy (stage only)
        T* xl = lds + sh_off[l][0];
        T* yl = lds + sh_off[l][1];
        T* bl = lds + sh_off[l][2];
        T* dl = lds + sh_off[l][3];
        if (l == nl - 1) {
            double* part = (double*)(lds + sh.part);
            if constexpr (STAGE) col_gemv(cl, n, bl, xl, part);
            else col_gemv((const T*)a.inv[l] + P.invoff + (int64_t)mode * n * n, n, bl, xl, part);
            if (threadIdx.x == 0) sh_cur[l] = 0;
            __syncthreads();
            break;
        }
        const double* cc = a.cheb[l] + 2 * (((int64_t)pl * 2 + mode) * KMAX);
        {
            const int M0 = P.M[0], M1 = P.M[1], M01 = M0 * M1;
            const T s20 = T(cc[1]);
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const int i2 = i / M01, r = i - i2 * M01, i1 = r / M0, i0 = r - i1 * M0;
                T v = T(0);
                if (!masked_bits(P.mbits[mode], P.dim, M0, M1, P.M[2], i0, i1, i2))
                    v = s20 * bl[i] / (stage ? cl[i] : cg[i]);
                xl[i] = v;
                dl[i] = v;
            }
        }
        __syncthreads();
        T* X = xl;
        T* Y = yl;
        int c = 0;
        for (int step = 1; step <= a.m; ++step) {
            const bool resid = step == a.m;
            if (resid && threadIdx.x == 0) sh_cur[l] = c;
            if constexpr (STAGE) vc_sweep<P0, P1, P2, T, VC_ROWS>(P, cl, n + g, X, Y, bl, dl, mode, cc, resid ? 0 : step, resid);
            else vc_sweep<P0, P1, P2, T, vc_form<P0, P1, P2, false>()>(P, cg, (int)P.cstride, X, Y, bl, dl, mode, cc, resid ? 0 : step, resid);
            __syncthreads();
            if (!resid) {
                T* tmp = X; X = Y; Y = tmp;
                c ^= 1;
            }
        }
        {
            const PatchLev& C = a.L[l + 1][sh_pl[l + 1]];
            T* bc = lds + sh_off[l + 1][2];
            const int32_t* rlo = a.rlo[l];
            const T* rval = (const T*)a.rval[l];
            const bool three = P.dim == 3;
            const int M0 = P.M[0], M01 = P.M[0] * P.M[1];
            const int nc = (int)C.n, C0 = C.M[0], C1 = C.M[1], C01 = C0 * C1;
            for (int I = threadIdx.x; I < nc; I += blockDim.x) {
                const int I2 = I / C01, r = I - I2 * C01, I1 = r / C0, I0 = r - I1 * C0;
                T v = T(0);
                if (!masked_bits(C.mbits[mode], C.dim, C0, C1, C.M[2], I0, I1, I2)) {
                    const int lo0 = rlo[P.roff[0] + I0], lo1 = rlo[P.roff[1] + I1];
                    const int lo2 = three ? rlo[P.roff[2] + I2] : 0;
                    const T* v0 = rval + (P.roff[0] + I0) * PW;
                    const T* v1 = rval + (P.roff[1] + I1) * PW;
                    const T* v2 = three ? rval + (P.roff[2] + I2) * PW : v1;
                    constexpr int W0 = P0 >= 0 ? P0 + 2 : -1, W1 = P0 >= 0 ? P1 + 2 : -1;
                    constexpr int W2 = P0 >= 0 ? (P2 > 0 ? P2 + 2 : 1) : -1;
                    v = T(band_sum<W0, W1, W2>(v0, v1, v2, Y + lo0 + lo1 * M0 + lo2 * M01, M0, M01, P.p[0] + 2,
                                               P.p[1] + 2, three ? P.p[2] + 2 : 1, P.dim));
                }
                bc[I] = v;
            }
        }
        __syncthreads();
    }
    // ---- up
    for (int lu = nl - 2; lu >= l0; --lu) {
        const int pl = sh_pl[lu];
        const PatchLev& P = a.L[lu][pl];
        const int n = (int)P.n;
        const int g = P.p[0] + P.p[1] * P.M[0] + P.p[2] * P.M[0] * P.M[1];
        const T* cg = (const T*)a.coef[lu] + P.coff;
        const T* cl = lds + sh_off[lu][4];
        const double* cc = a.cheb[lu] + 2 * (((int64_t)pl * 2 + mode) * KMAX);
        const int cu = sh_cur[lu];
        T* X = lds + sh_off[lu][cu];
        T* Y = lds + sh_off[lu][1 - cu];
        T* bl = lds + sh_off[lu][2];
        T* dl = lds + sh_off[lu][3];
        const T* E = lds + sh_off[lu + 1][sh_cur[lu + 1]];
        {
            const PatchLev& C = a.L[lu + 1][sh_pl[lu + 1]];
            const int32_t* plo = a.plo[lu];
            const T* pval = (const T*)a.pval[lu];
            const bool three = P.dim == 3;
            const int M0 = P.M[0], M1 = P.M[1], M01 = M0 * M1;
            const int C0 = C.M[0], C01 = C.M[0] * C.M[1];
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const int i2 = i / M01, r = i - i2 * M01, i1 = r / M0, i0 = r - i1 * M0;
                if (masked_bits(P.mbits[mode], P.dim, M0, M1, P.M[2], i0, i1, i2)) continue;
                const int lo0 = plo[P.toff[0] + i0], lo1 = plo[P.toff[1] + i1];
                const int lo2 = three ? plo[P.toff[2] + i2] : 0;
                const T* v0 = pval + (P.toff[0] + i0) * PW;
                const T* v1 = pval + (P.toff[1] + i1) * PW;
                const T* v2 = three ? pval + (P.toff[2] + i2) * PW : v1;
                constexpr int W0 = P0 >= 0 ? prol_width(P0) : -1, W1 = P0 >= 0 ? prol_width(P1) : -1;
                constexpr int W2 = P0 >= 0 ? (P2 > 0 ? prol_width(P2) : 1) : -1;
                X[i] += T(band_sum<W0, W1, W2>(v0, v1, v2, E + lo0 + lo1 * C0 + lo2 * C01, C0, C01,
                                               prol_width(P.p[0]), prol_width(P.p[1]),
                                               three ? prol_width(P.p[2]) : 1, P.dim));
            }
        }
        __syncthreads();
        int c = cu;
        for (int step = 0; step < a.m; ++step) {
            if constexpr (STAGE) vc_sweep<P0, P1, P2, T, VC_ROWS>(P, cl, n + g, X, Y, bl, dl, mode, cc, step, false);
            else vc_sweep<P0, P1, P2, T, vc_form<P0, P1, P2, false>()>(P, cg, (int)P.cstride, X, Y, bl, dl, mode, cc, step, false);
            __syncthreads();
            T* tmp = X; X = Y; Y = tmp;
            c ^= 1;
        }
        if (threadIdx.x == 0) sh_cur[lu] = c;
        __syncthreads();
    }
    {
        const PatchLev& P = a.L[l0][sh_pl[l0]];
        group_copy<4>((T*)a.x1 + P.voff, lds + sh_off[l0][sh_cur[l0]], (int)P.n);
    }
}

// One launch for the patches of all degree classes of a family (FAM 0: the
// 2D classes 0..8; FAM 1: the 3D classes and the generic one): each
// work-group takes its patch's class instance (a uniform branch).  Two
// families because the compiler spills registers when all twelve instances
// share one kernel.
__host__ __device__ constexpr int vcoarse_family(int cls) { return cls <= 8 ? 0 : 1; }

template <typename T, bool STAGE, int FAM>
__global__ __launch_bounds__((vc_threads<T, FAM>())) void k_vcoarse(CoarseArgs a) {
    extern __shared__ __align__(16) unsigned char vc_lds_raw[];
    __shared__ VcShared sh;
    if ((int)blockIdx.x >= a.nlist) return;
    const int k = a.plist[blockIdx.x];
    if (a.active && !a.active[k]) return;
    const int cls = a.L[a.l0][a.chain[k * LMAX + a.l0]].pclass;
    T* lds = (T*)vc_lds_raw;
    if constexpr (FAM == 0) {
        switch (cls) {
        case 0: vcoarse_body<2, 2, 0, T, STAGE>(a, k, lds, sh); break;
        case 1: vcoarse_body<3, 2, 0, T, STAGE>(a, k, lds, sh); break;
        case 2: vcoarse_body<4, 2, 0, T, STAGE>(a, k, lds, sh); break;
        case 3: vcoarse_body<2, 3, 0, T, STAGE>(a, k, lds, sh); break;
        case 4: vcoarse_body<3, 3, 0, T, STAGE>(a, k, lds, sh); break;
        case 5: vcoarse_body<4, 3, 0, T, STAGE>(a, k, lds, sh); break;
        case 6: vcoarse_body<2, 4, 0, T, STAGE>(a, k, lds, sh); break;
        case 7: vcoarse_body<3, 4, 0, T, STAGE>(a, k, lds, sh); break;
        case 8: vcoarse_body<4, 4, 0, T, STAGE>(a, k, lds, sh); break;
        default: break;
        }
    } else {
        switch (cls) {
        case 9: vcoarse_body<2, 2, 2, T, STAGE>(a, k, lds, sh); break;
        case 10: vcoarse_body<3, 3, 3, T, STAGE>(a, k, lds, sh); break;
        default: vcoarse_body<-1, -1, -1, T, STAGE>(a, k, lds, sh); break;
        }
    }
}


// ------------------------------------------------------------------ exact local solves (banded Cholesky)
//
// x = (L L^T)^{-1} b for every patch, one work-group per patch, the patch's
// vector in LDS with zero guards of b entries on both sides.  Forward then
// backward substitution in blocks of BNB rows: the off-diagonal part of a
// block row is a GEMV with the already solved entries (8 threads per row,
// shuffle reduction), the diagonal block is applied through its stored
// inverse.  Layout of the factor data per block row:
//   [L_off (BNB x b) | U_off (BNB x b) | inv(L_diag) (BNB x BNB)].

constexpr int BNB = 64;
constexpr int BAND_THREADS = 512;

__device__ __forceinline__ double sum8(double v) {
    v += __shfl_xor(v, 1, WAVE);
    v += __shfl_xor(v, 2, WAVE);
    v += __shfl_xor(v, 4, WAVE);
    return v;
}

__global__ __launch_bounds__(BAND_THREADS) void k_band_solve(const PatchLev* L, const int64_t* band_off,
                                                           const int32_t* band_b, const double* band, int mode,
                                                           const double* rhs, double* x, const int* active) {
    extern __shared__ double bs_lds[];
    const int k = blockIdx.x;
    if (active && !active[k]) return;
    const PatchLev& P = L[k];
    const int n = (int)P.n;
    const int b = band_b[k];
    const int nblk = (n + BNB - 1) / BNB;
    const int64_t bsz = (int64_t)BNB * (2 * b + BNB);
    const double* F = band + band_off[2 * k + mode];
    double* xs = bs_lds + b;                    // xs[-b .. nblk*BNB + b)
    double* t = bs_lds + 2 * b + nblk * BNB;    // BNB scratch
    const int tot = 2 * b + nblk * BNB;
    for (int i = threadIdx.x; i < tot; i += blockDim.x) {
        const int j = i - b;
        bs_lds[i] = (j >= 0 && j < n) ? rhs[P.voff + j] : 0.0;
    }
    __syncthreads();
    const int ii = threadIdx.x >> 3, l8 = threadIdx.x & 7;
    // forward: L y = rhs
    for (int r = 0; r < nblk; ++r) {
        const double* blk = F + r * bsz;
        const double* row = blk + (int64_t)ii * b;
        const double* xw = xs + r * BNB - b;
        double acc = 0.0;
        for (int c = l8; c < b; c += 8) acc += row[c] * xw[c];
        acc = sum8(acc);
        if (l8 == 0) t[ii] = xs[r * BNB + ii] - acc;
        __syncthreads();
        const double* inv = blk + 2 * (int64_t)BNB * b + (int64_t)ii * BNB;
        double a2 = 0.0;
        for (int c = l8; c < BNB; c += 8) a2 += inv[c] * t[c];
        a2 = sum8(a2);
        if (l8 == 0) xs[r * BNB + ii] = a2;
        __syncthreads();
    }
    // backward: L^T x = y
    for (int r = nblk - 1; r >= 0; --r) {
        const double* blk = F + r * bsz;
        const double* row = blk + (int64_t)BNB * b + (int64_t)ii * b;
        const double* xw = xs + (r + 1) * BNB;
        double acc = 0.0;
        for (int c = l8; c < b; c += 8) acc += row[c] * xw[c];
        acc = sum8(acc);
        if (l8 == 0) t[ii] = xs[r * BNB + ii] - acc;
        __syncthreads();
        const double* inv = blk + 2 * (int64_t)BNB * b;
        double a2 = 0.0;
        for (int c = l8; c < BNB; c += 8) a2 += inv[(int64_t)c * BNB + ii] * t[c];
        a2 = sum8(a2);
        if (l8 == 0) xs[r * BNB + ii] = a2;
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) x[P.voff + i] = xs[i];
}

// The same solve with the factor rows of a block step in registers: 1024 threads, 16 per block row, J
// off-diagonal values per thread (band width b <= 16 J).  With DB (J = 16, b <= 256) the next block's
// share (J values and 4 of the inverse diagonal) is loaded while the current block is reduced and its
// diagonal block applied, so a step waits on LDS and barriers only; without DB (J = 32, b <= 512, for
// register room) all loads of a step are issued together at its start, one memory latency per step.
constexpr int BAND_PF_THREADS = 1024;

__device__ __forceinline__ double sum16(double v) {
    v += __shfl_xor(v, 1, WAVE);
    v += __shfl_xor(v, 2, WAVE);
    v += __shfl_xor(v, 4, WAVE);
    v += __shfl_xor(v, 8, WAVE);
    return v;
}

template <int J, bool DB>
__global__ __launch_bounds__(BAND_PF_THREADS) void k_band_solve_pf(const PatchLev* L, const int64_t* band_off,
                                                                 const int32_t* band_b, const double* band, int mode,
                                                                 const double* rhs, double* x, const int* active) {
    extern __shared__ double bs_lds[];
    const int k = blockIdx.x;
    if (active && !active[k]) return;
    const PatchLev& P = L[k];
    const int n = (int)P.n;
    const int b = band_b[k];
    const int nblk = (n + BNB - 1) / BNB;
    const int64_t bsz = (int64_t)BNB * (2 * b + BNB);
    const double* F = band + band_off[2 * k + mode];
    double* xs = bs_lds + b;                    // xs[-b .. nblk*BNB + b)
    double* t = bs_lds + 2 * b + nblk * BNB;    // BNB scratch
    const int tot = 2 * b + nblk * BNB;
    for (int i = threadIdx.x; i < tot; i += blockDim.x) {
        const int j = i - b;
        bs_lds[i] = (j >= 0 && j < n) ? rhs[P.voff + j] : 0.0;
    }
    __syncthreads();
    const int ii = threadIdx.x >> 4, l16 = threadIdx.x & 15;
    double rc[J], rn[DB ? J : 1], ic[4], in4[4];
    // block r's share of the forward (L_off row ii, inv(L_diag) row ii) or backward (U_off row ii,
    // inv(L_diag) column ii) factor data
    auto load = [&](int r, bool fwd, double* rv, double* iv) {
        const double* blk = F + (int64_t)r * bsz;
        const double* row = blk + (fwd ? 0 : (int64_t)BNB * b) + (int64_t)ii * b;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int c = l16 + 16 * j;
            rv[j] = c < b ? row[c] : 0.0;
        }
        const double* inv = blk + 2 * (int64_t)BNB * b;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            iv[j] = fwd ? inv[(int64_t)ii * BNB + l16 + 16 * j] : inv[(int64_t)(l16 + 16 * j) * BNB + ii];
    };
    auto step = [&](int r, const double* xw) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int c = l16 + 16 * j;
            if (c < b) acc += rc[j] * xw[c];
        }
        acc = sum16(acc);
        if (l16 == 0) t[ii] = xs[r * BNB + ii] - acc;
        __syncthreads();
        double a2 = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) a2 += ic[j] * t[l16 + 16 * j];
        a2 = sum16(a2);
        if (l16 == 0) xs[r * BNB + ii] = a2;
        __syncthreads();
    };
    // forward: L y = rhs
    if (DB && nblk > 0) load(0, true, rn, in4);
    for (int r = 0; r < nblk; ++r) {
        if (DB) {
#pragma unroll
            for (int j = 0; j < J; ++j) rc[j] = rn[DB ? j : 0];
#pragma unroll
            for (int j = 0; j < 4; ++j) ic[j] = in4[j];
            if (r + 1 < nblk) load(r + 1, true, rn, in4);
        } else {
            load(r, true, rc, ic);
        }
        step(r, xs + r * BNB - b);
    }
    // backward: L^T x = y
    if (DB && nblk > 0) load(nblk - 1, false, rn, in4);
    for (int r = nblk - 1; r >= 0; --r) {
        if (DB) {
#pragma unroll
            for (int j = 0; j < J; ++j) rc[j] = rn[DB ? j : 0];
#pragma unroll
            for (int j = 0; j < 4; ++j) ic[j] = in4[j];
            if (r > 0) load(r - 1, false, rn, in4);
        } else {
            load(r, false, rc, ic);
        }
        step(r, xs + (r + 1) * BNB);
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) x[P.voff + i] = xs[i];
}

// ------------------------------------------------------------------ exact local solves, 3D: factorised on the device
//
// The band of a 3D patch (b = p0 + p1 M0 + p2 M0 M1, ~1400 for 26^3 coefficients at p = 2) is too wide for
// the host factorisation and for the LDS-resident solve above.  Here the masked level-0 stiffness (masked
// rows and columns replaced by the identity) of each job (patch, mode) is held in block-band storage of
// BNB x BNB blocks: block row R keeps blocks C = R - W .. R (W = ceil(b / BNB)) at slots w = C - R + W, each
// row-major; blocks left of column 0 are zero and the padding rows past n carry the identity.  It is
// factorised in place, right-looking over block columns k (batched over all jobs, three launches per k):
//   L_kk = chol(A_kk) (its inverse kept for the solves), L_Rk = A_Rk L_kk^{-T} (R = k+1 .. k+W),
//   A_RC -= L_Rk L_Ck^T (k < C <= R <= k+W).
// The solve streams the factor from HBM, one work-group per patch, with a window of the last W+1 solved
// blocks in LDS.

struct BandJob {
    int64_t off;       // first double of the job's block band (nb x (W+1) blocks)
    int64_t doff;      // first double of the inverses of its diagonal blocks (nb blocks)
    int32_t patch, mode, nb, W;
    int32_t toff;      // offset of the patch's stencil slot table
};

// slot table of a patch: entry (d0+p0) + (2p0+1)((d1+p1) + (2p1+1)(d2+p2)) for the offset d = j - i gives
// s + 1 when K(i, j) = coef[s][i] (d in the upper half), -(s + 1) when K(i, j) = coef[s][j] (d in the lower
// half, -d in the upper), 0 for no entry
__global__ __launch_bounds__(256) void k_bb_assemble(const PatchLev* L, const BandJob* jobs, const int32_t* stab,
                                                     const double* coef, double* F) {
    const BandJob J = jobs[blockIdx.y];
    const int nblocks = J.nb * (J.W + 1);
    if ((int)blockIdx.x >= nblocks) return;
    const int R = blockIdx.x / (J.W + 1), w = blockIdx.x % (J.W + 1), C = R - J.W + w;
    const PatchLev& P = L[J.patch];
    const int n = (int)P.n;
    double* blk = F + J.off + (int64_t)blockIdx.x * BNB * BNB;
    const int M0 = P.M[0], M01 = P.M[0] * P.M[1];
    const int w0 = 2 * P.p[0] + 1, w1 = 2 * P.p[1] + 1;
    for (int e = threadIdx.x; e < BNB * BNB; e += blockDim.x) {
        const int ii = e / BNB, jj = e % BNB;
        const int i = R * BNB + ii, j = C * BNB + jj;
        double v = 0.0;
        if (C >= 0 && j <= i) {
            if (i >= n || j >= n) {
                v = i == j ? 1.0 : 0.0;
            } else {
                const int i2 = i / M01, ri = i - i2 * M01, i1 = ri / M0, i0 = ri - i1 * M0;
                const int j2 = j / M01, rj = j - j2 * M01, j1 = rj / M0, j0 = rj - j1 * M0;
                if (masked(P, J.mode, i0, i1, i2) || masked(P, J.mode, j0, j1, j2)) {
                    v = i == j ? 1.0 : 0.0;
                } else {
                    const int d0 = j0 - i0, d1 = j1 - i1, d2 = j2 - i2;
                    if (abs(d0) <= P.p[0] && abs(d1) <= P.p[1] && abs(d2) <= P.p[2]) {
                        const int t = stab[J.toff + (d0 + P.p[0]) + w0 * ((d1 + P.p[1]) + w1 * (d2 + P.p[2]))];
                        if (t > 0) v = coef[P.coff + (int64_t)(t - 1) * P.cstride + i];
                        else if (t < 0) v = coef[P.coff + (int64_t)(-t - 1) * P.cstride + j];
                    }
                }
            }
        }
        blk[e] = v;
    }
}

// L_kk = chol(A_kk) in place (upper triangle zeroed) and D_k = L_kk^{-1}; one work-group per job
__global__ __launch_bounds__(256) void k_bb_potrf(const BandJob* jobs, int k, double* F, double* D, int* err) {
    __shared__ double A[BNB][BNB + 1];
    const BandJob J = jobs[blockIdx.x];
    if (k >= J.nb) return;
    double* blk = F + J.off + ((int64_t)k * (J.W + 1) + J.W) * BNB * BNB;
    for (int e = threadIdx.x; e < BNB * BNB; e += blockDim.x) A[e / BNB][e % BNB] = blk[e];
    __syncthreads();
    for (int c = 0; c < BNB; ++c) {
        const double d = A[c][c];
        if (!(d > 0.0)) {
            if (threadIdx.x == 0) atomicExch(err, 1);
            return;   // uniform: every thread read the same d
        }
        const double sd = sqrt(d);
        __syncthreads();
        for (int r = c + 1 + threadIdx.x; r < BNB; r += blockDim.x) A[r][c] /= sd;
        if (threadIdx.x == 0) A[c][c] = sd;
        __syncthreads();
        // trailing update of the lower triangle
        for (int e = threadIdx.x; e < BNB * BNB; e += blockDim.x) {
            const int r = e / BNB, q = e % BNB;
            if (q > c && r >= q) A[r][q] -= A[r][c] * A[q][c];
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < BNB * BNB; e += blockDim.x) {
        const int r = e / BNB, q = e % BNB;
        blk[e] = q <= r ? A[r][q] : 0.0;
    }
    // D = L^{-1}: column q by forward substitution (one thread per column)
    double* Dk = D + J.doff + (int64_t)k * BNB * BNB;
    if (threadIdx.x < BNB) {
        const int q = threadIdx.x;
        double x[BNB];
        for (int r = 0; r < BNB; ++r) {
            double t = r == q ? 1.0 : 0.0;
            for (int u = q; u < r; ++u) t -= A[r][u] * x[u];
            x[r] = r < q ? 0.0 : t / A[r][r];
        }
        for (int r = 0; r < BNB; ++r) Dk[(int64_t)r * BNB + q] = x[r];
    }
}

// one 64 x 64 x 64 product on a work-group of 256 threads: C (-)= A B^T, operands in LDS (row-major, padded);
// thread (ty, tx) owns rows 4 ty .. 4 ty + 3 and columns tx + 16 c, c = 0..3
__device__ __forceinline__ void bb_gemm_nt(const double (*a)[BNB + 1], const double (*b)[BNB + 1], double (&acc)[4][4]) {
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    for (int t = 0; t < BNB; ++t) {
        double av[4], bv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) av[r] = a[4 * ty + r][t];
#pragma unroll
        for (int c = 0; c < 4; ++c) bv[c] = b[tx + 16 * c][t];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] += av[r] * bv[c];
    }
}

// L_Rk = A_Rk D_k^T for R = k + 1 + blockIdx.x (grid: W x jobs)
__global__ __launch_bounds__(256) void k_bb_trsm(const BandJob* jobs, int k, double* F, const double* D) {
    __shared__ double a[BNB][BNB + 1], dm[BNB][BNB + 1];
    const BandJob J = jobs[blockIdx.y];
    const int R = k + 1 + (int)blockIdx.x;
    if (k >= J.nb || (int)blockIdx.x >= J.W || R >= J.nb) return;
    double* blk = F + J.off + ((int64_t)R * (J.W + 1) + (k - R + J.W)) * BNB * BNB;
    const double* Dk = D + J.doff + (int64_t)k * BNB * BNB;
    for (int e = threadIdx.x; e < BNB * BNB; e += blockDim.x) {
        a[e / BNB][e % BNB] = blk[e];
        dm[e / BNB][e % BNB] = Dk[e];
    }
    __syncthreads();
    double acc[4][4] = {};
    bb_gemm_nt(a, dm, acc);
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) blk[(4 * ty + r) * BNB + tx + 16 * c] = acc[r][c];
}

// A_RC -= L_Rk L_Ck^T for k < C <= R <= k + W (grid: W (W + 1) / 2 x jobs; pair index -> (a, b), 1 <= b <= a)
__global__ __launch_bounds__(256) void k_bb_update(const BandJob* jobs, int k, double* F) {
    __shared__ double a[BNB][BNB + 1], b[BNB][BNB + 1];
    const BandJob J = jobs[blockIdx.y];
    if (k >= J.nb || (int)blockIdx.x >= J.W * (J.W + 1) / 2) return;
    int ia = 1, rem = (int)blockIdx.x;
    while (rem >= ia) {
        rem -= ia;
        ++ia;
    }
    const int ib = rem + 1;   // 1 <= ib <= ia
    const int R = k + ia, C = k + ib;
    if (R >= J.nb) return;
    const int64_t rowR = (int64_t)R * (J.W + 1), rowC = (int64_t)C * (J.W + 1);
    const double* Lr = F + J.off + (rowR + (k - R + J.W)) * BNB * BNB;
    const double* Lc = F + J.off + (rowC + (k - C + J.W)) * BNB * BNB;
    double* Ab = F + J.off + (rowR + (C - R + J.W)) * BNB * BNB;
    for (int e = threadIdx.x; e < BNB * BNB; e += blockDim.x) {
        a[e / BNB][e % BNB] = Lr[e];
        b[e / BNB][e % BNB] = Lc[e];
    }
    __syncthreads();
    double acc[4][4] = {};
    bb_gemm_nt(a, b, acc);
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) Ab[(4 * ty + r) * BNB + tx + 16 * c] -= acc[r][c];
}

// x = (L L^T)^{-1} rhs for the jobs of one mode, one work-group of 1024 threads per patch (job_of[patch], -1:
// none).  Forward: wave w owns rows 4w .. 4w+3 of a block row, its lanes the columns of each block;
// backward: lanes own the rows of block R, wave w the rows jj = w (mod 16) of each block L_CR.  The last W+1
// solved blocks stay in LDS (slot = block mod (W+1)); y goes to x between the two passes.
constexpr int BB_THREADS = 1024;
constexpr int BB_WMAX = 40;   // off-diagonal blocks per row the solve's LDS window holds (b <= 2560)
__global__ __launch_bounds__(BB_THREADS) void k_bb_solve(const PatchLev* L, const BandJob* jobs, const int32_t* job_of,
                                                         const double* F, const double* D, const double* rhs,
                                                         double* x, const int* active) {
    __shared__ double win[(BB_WMAX + 1) * BNB];
    __shared__ double part[BB_THREADS / WAVE][BNB];
    __shared__ double t[BNB];
    const int k = blockIdx.x;
    if (active && !active[k]) return;
    const int jid = job_of[k];
    if (jid < 0) return;
    const BandJob J = jobs[jid];
    const PatchLev& P = L[k];
    const int n = (int)P.n, W = J.W, nb = J.nb, WP = W + 1;
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const double* Fj = F + J.off;
    const double* Dj = D + J.doff;
    // forward: L y = rhs
    for (int R = 0; R < nb; ++R) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int C = (R - W > 0 ? R - W : 0); C < R; ++C) {
            const double yc = win[(C % WP) * BNB + lane];
            const double* blk = Fj + ((int64_t)R * WP + (C - R + W)) * BNB * BNB;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += blk[(4 * wv + q) * BNB + lane] * yc;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double v = acc[q];
            for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_down(v, o, WAVE);
            if (lane == 0) {
                const int i = R * BNB + 4 * wv + q;
                t[4 * wv + q] = (i < n ? rhs[P.voff + i] : 0.0) - v;
            }
        }
        __syncthreads();
        {   // y_R = D_R t: 16 threads per row
            const int ii = threadIdx.x >> 4, g = threadIdx.x & 15;
            const double* Dr = Dj + (int64_t)R * BNB * BNB + (int64_t)ii * BNB;
            double a2 = 0.0;
            for (int c = g; c < BNB; c += 16) a2 += Dr[c] * t[c];
            a2 = sum16(a2);
            if (g == 0) {
                win[(R % WP) * BNB + ii] = a2;
                const int i = R * BNB + ii;
                if (i < n) x[P.voff + i] = a2;
            }
        }
        __syncthreads();
    }
    // backward: L^T x = y (the window keeps the last forward blocks, which are the first backward ones' y;
    // it is refilled with x as blocks are solved)
    for (int R = nb - 1; R >= 0; --R) {
        double acc = 0.0;
        const int Cend = R + W < nb - 1 ? R + W : nb - 1;
        for (int C = R + 1; C <= Cend; ++C) {
            const double* blk = Fj + ((int64_t)C * WP + (R - C + W)) * BNB * BNB;
            const double* xc = win + (C % WP) * BNB;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int jj = wv + 16 * q;
                acc += blk[(int64_t)jj * BNB + lane] * xc[jj];
            }
        }
        part[wv][lane] = acc;
        __syncthreads();
        if (threadIdx.x < BNB) {
            const int ii = threadIdx.x;
            double sacc = 0.0;
            for (int w = 0; w < BB_THREADS / WAVE; ++w) sacc += part[w][ii];
            const int i = R * BNB + ii;
            t[ii] = (i < n ? x[P.voff + i] : 0.0) - sacc;
        }
        __syncthreads();
        {   // x_R = D_R^T t
            const int ii = threadIdx.x >> 4, g = threadIdx.x & 15;
            const double* Dr = Dj + (int64_t)R * BNB * BNB;
            double a2 = 0.0;
            for (int c = g; c < BNB; c += 16) a2 += Dr[(int64_t)c * BNB + ii] * t[c];
            a2 = sum16(a2);
            if (g == 0) {
                win[(R % WP) * BNB + ii] = a2;
                const int i = R * BNB + ii;
                if (i < n) x[P.voff + i] = a2;
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ dense SPD inverse on matrix cores
//
// S^{-1} of the assembled primal Schur complement (n x n, FP64) through the
// Cholesky factor: S = L L^T, X = L^{-1}, S^{-1} = X^T X.  Row-major N x N
// working matrices, N = n rounded up to 16 (identity padding); 16 x 16
// blocks; one wave per work-group; every block product on
// v_mfma_f64_16x16x4f64 (four k-steps per block).  Operand layout of that
// instruction on gfx950: lane l supplies A[l % 16][k0 + l / 16] and
// B[k0 + l / 16][l % 16]; result element r of lane l is C[l / 16 + 4 r][l % 16].
// blockIdx.y selects the matrix of a batch (stride N * N).

typedef double mf_d4 __attribute__((ext_vector_type(4)));
constexpr int MB = 16;

// c += A B for 16 x 16 blocks, A[i][k] at A[i * lda + k], B[k][j] at B[k * ldb + j];
// with TA, A is read transposed (A[i][k] at A[k * lda + i]), with TB, B (B[k][j] at
// B[j * ldb + k]); sign -1 subtracts.
template <bool TA, bool TB = false>
__device__ __forceinline__ mf_d4 mf_block(const double* __restrict__ A, int lda, const double* __restrict__ B, int ldb,
                                          mf_d4 c, double sign) {
    const int l = threadIdx.x & 63, i = l & 15, kq = l >> 4;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k = 4 * s + kq;
        const double a = sign * (TA ? A[k * lda + i] : A[i * lda + k]);
        const double b = TB ? B[i * ldb + k] : B[k * ldb + i];   // column j = l % 16 = i
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    return c;
}

__device__ __forceinline__ mf_d4 mf_load(const double* __restrict__ C, int ldc) {
    const int l = threadIdx.x & 63;
    mf_d4 c;
#pragma unroll
    for (int r = 0; r < 4; ++r) c[r] = C[((l >> 4) + 4 * r) * ldc + (l & 15)];
    return c;
}

__device__ __forceinline__ void mf_store(double* C, int ldc, mf_d4 c) {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < 4; ++r) C[((l >> 4) + 4 * r) * ldc + (l & 15)] = c[r];
}

// Cholesky of the 16 x 16 block D (in LDS, lower triangle used) in place and
// Dinv = its inverse (lower); one wave, lane r < 16 owns row r.  A non-positive
// pivot sets *err.
__device__ __forceinline__ void mf_diag_factor(double (*D)[MB + 1], double (*Dinv)[MB + 1], int* err) {
    const int l = threadIdx.x;
    for (int c = 0; c < MB; ++c) {
        if (l == c) {
            const double p = D[c][c];
            if (!(p > 0.0)) atomicOr(err, 1);
            D[c][c] = p > 0.0 ? sqrt(p) : 1.0;
        }
        __syncthreads();
        if (l > c && l < MB) D[l][c] /= D[c][c];
        __syncthreads();
        if (l > c && l < MB)
            for (int j = c + 1; j <= l; ++j) D[l][j] -= D[l][c] * D[j][c];
        __syncthreads();
    }
    if (l < MB) {   // column l of the inverse, forward substitution
        for (int i = 0; i < MB; ++i) {
            double s = i == l ? 1.0 : 0.0;
            for (int k = l; k < i; ++k) s -= D[i][k] * Dinv[k][l];
            Dinv[i][l] = i < l ? 0.0 : s / D[i][i];
        }
    }
    __syncthreads();
}

// Block step k: work-group b factors the diagonal block of A (every group, in
// LDS); group 0 stores L_kk, group b > 0 stores L[k + b][k] = A[k + b][k] L_kk^{-T}.
__global__ __launch_bounds__(64) void k_spd_panel(const double* A, double* L, int N, int k, int* err) {
    __shared__ double D[MB][MB + 1], Dinv[MB][MB + 1];
    const size_t off = (size_t)blockIdx.y * N * N;
    A += off;
    L += off;
    const int l = threadIdx.x;
    for (int e = l; e < MB * MB; e += 64) D[e / MB][e % MB] = A[(size_t)(k * MB + e / MB) * N + k * MB + e % MB];
    __syncthreads();
    mf_diag_factor(D, Dinv, err);
    const int ib = k + (int)blockIdx.x;
    if (blockIdx.x == 0) {
        for (int e = l; e < MB * MB; e += 64) {
            const int r = e / MB, c = e % MB;
            L[(size_t)(k * MB + r) * N + k * MB + c] = c <= r ? D[r][c] : 0.0;
        }
        return;
    }
    // C = A_blk Dinv^T: B[kk][j] = Dinv[j][kk]
    __shared__ double DinvT[MB][MB];
    for (int e = l; e < MB * MB; e += 64) DinvT[e / MB][e % MB] = Dinv[e % MB][e / MB];
    __syncthreads();
    mf_d4 c = {0.0, 0.0, 0.0, 0.0};
    c = mf_block<false>(A + (size_t)ib * MB * N + k * MB, N, &DinvT[0][0], MB, c, 1.0);
    mf_store(L + (size_t)ib * MB * N + k * MB, N, c);
}

// Trailing update of step k: A[ib][jb] -= L[ib][k] L[jb][k]^T for k < jb <= ib,
// one work-group per block pair (lower triangle, packed by rows).
__global__ __launch_bounds__(64) void k_spd_update(double* A, const double* L, int N, int k) {
    const size_t off = (size_t)blockIdx.y * N * N;
    A += off;
    L += off;
    const int q = (int)blockIdx.x;
    int p = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
    while ((p + 1) * (p + 2) / 2 <= q) ++p;
    while (p * (p + 1) / 2 > q) --p;
    const int ib = k + 1 + p, jb = k + 1 + (q - p * (p + 1) / 2);
    double* C = A + (size_t)ib * MB * N + jb * MB;
    mf_d4 c = mf_load(C, N);
    // B[kk][j] = L[jb][k][j][kk]: the transposed operand read as A^T of mf_block's B slot
    const double* Li = L + (size_t)ib * MB * N + k * MB;
    const double* Lj = L + (size_t)jb * MB * N + k * MB;
    const int l = threadIdx.x & 63, i = l & 15, kq = l >> 4;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int kk = 4 * s + kq;
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(-Li[i * N + kk], Lj[i * N + kk], c, 0, 0, 0);
    }
    mf_store(C, N, c);
}

// X_ii = L_ii^{-1} for every diagonal block i (one work-group each).
__global__ __launch_bounds__(64) void k_spd_diag_inv(const double* L, double* X, int N, int* err) {
    __shared__ double D[MB][MB + 1], Dinv[MB][MB + 1];
    const size_t off = (size_t)blockIdx.y * N * N;
    L += off;
    X += off;
    const int b = (int)blockIdx.x, l = threadIdx.x;
    for (int e = l; e < MB * MB; e += 64) {
        const int r = e / MB, c = e % MB;
        D[r][c] = c <= r ? L[(size_t)(b * MB + r) * N + b * MB + c] : 0.0;
    }
    __syncthreads();
    // D is already the factor: invert it (lane-per-column forward substitution)
    if (l < MB) {
        for (int i = 0; i < MB; ++i) {
            double s = i == l ? 1.0 : 0.0;
            for (int k = l; k < i; ++k) s -= D[i][k] * Dinv[k][l];
            if (i >= l && !(D[i][i] != 0.0)) atomicOr(err, 2);
            Dinv[i][l] = i < l ? 0.0 : s / D[i][i];
        }
    }
    __syncthreads();
    for (int e = l; e < MB * MB; e += 64) X[(size_t)(b * MB + e / MB) * N + b * MB + e % MB] = Dinv[e / MB][e % MB];
}

// Block column j of X = L^{-1} below the diagonal: X[i][j] = -X_ii sum_{j <= m < i} L[i][m] X[m][j],
// i = j + 1, j + 2, ... in order (one work-group per column; each block is written
// before the wave reads it back).
__global__ __launch_bounds__(64) void k_spd_tri_inv(const double* L, double* X, int N) {
    __shared__ double T[MB][MB];
    const size_t off = (size_t)blockIdx.y * N * N;
    L += off;
    X += off;
    const int j = (int)blockIdx.x, nb = N / MB, l = threadIdx.x;
    for (int i = j + 1; i < nb; ++i) {
        mf_d4 c = {0.0, 0.0, 0.0, 0.0};
        for (int m = j; m < i; ++m)
            c = mf_block<false>(L + (size_t)i * MB * N + m * MB, N, X + (size_t)m * MB * N + j * MB, N, c, 1.0);
        mf_store(&T[0][0], MB, c);
        __syncthreads();
        mf_d4 x = {0.0, 0.0, 0.0, 0.0};
        x = mf_block<false>(X + (size_t)i * MB * N + i * MB, N, &T[0][0], MB, x, -1.0);
        mf_store(X + (size_t)i * MB * N + j * MB, N, x);
        __threadfence_block();
        __syncthreads();
        (void)l;
    }
}

// S^{-1} = X^T X for the leading n x n, written by columns (entry (r, c) at out[c * n + r]);
// one work-group per block pair.
__global__ __launch_bounds__(64) void k_spd_xtx(const double* X, double* out, int N, int n) {
    const size_t off = (size_t)blockIdx.y * N * N;
    X += off;
    out += (size_t)blockIdx.y * n * n;
    const int nb = N / MB, ib = (int)blockIdx.x / nb, jb = (int)blockIdx.x % nb;
    mf_d4 c = {0.0, 0.0, 0.0, 0.0};
    for (int m = ib > jb ? ib : jb; m < nb; ++m)
        c = mf_block<true>(X + (size_t)m * MB * N + ib * MB, N, X + (size_t)m * MB * N + jb * MB, N, c, 1.0);
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = ib * MB + (l >> 4) + 4 * r, col = jb * MB + (l & 15);
        if (row < n && col < n) out[(size_t)col * n + row] = c[r];
    }
}

// ------------------------------------------------------------------ saddle-point iteration (MG-MG-S)
//
// Flat kernels over whole level-0 (guarded) or multiplier vectors: guards are
// zero in every operand, so they stay zero.

// partial[b] = sum over the block's slice of a . b (fixed order)
__global__ __launch_bounds__(TILE) void k_dot_flat(int64_t n, const double* a, const double* b, double* partial) {
    __shared__ double lds[TILE / WAVE];
    double v[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * TILE + threadIdx.x; i < n; i += (int64_t)gridDim.x * TILE) v[0] += a[i] * b[i];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

// y += sign * s[idx] * x
__global__ void k_axpy_dev(int64_t n, double* y, const double* x, const double* s, int idx, double sign) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += sign * s[idx] * x[i];
}

// p = z + s[idx] * p
__global__ void k_xpby_dev(int64_t n, double* p, const double* z, const double* s, int idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = z[i] + s[idx] * p[i];
}

// y = a * x (a host scalar)
__global__ void k_scale_flat(int64_t n, double* y, const double* x, double a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i];
}

// out = g - C_E^T c_E per patch: every edge constraint j of patch k (edge list
// [edge_ptr, edge_ptr + 1)) subtracts c[k][j] / |E_j| on its coefficients
// (edge lists of one patch are disjoint; vertex constraints have none).  out
// must already hold g.
__global__ __launch_bounds__(TILE) void k_edge_scatter_sub(int npatch, const int32_t* npk, const int64_t* edge_ptr,
                                                           const int64_t* edge_dev, const double* c, double* out) {
    const int k = blockIdx.x;
    if (k >= npatch) return;
    for (int j = 0; j < npk[k]; ++j) {
        const int64_t eb = edge_ptr[k * NPMAX + j], ee = edge_ptr[k * NPMAX + j + 1];
        if (ee <= eb) continue;
        const double v = c[k * NPMAX + j] / (double)(ee - eb);
        for (int64_t r = eb + threadIdx.x; r < ee; r += blockDim.x) out[edge_dev[r]] -= v;
    }
}

// Scalars of the Bramble-Pasciak iteration in sc (one thread):
//   stage 0 (start): rho = sc[0] + sc[1]; rho0 = rho
//   stage 1: gamma = sc[2] + sc[3]; alpha = rho / gamma (0 and a breakdown flag if gamma <= 0)
//   stage 2: rho' = sc[0] + sc[1]; beta = rho' / rho; rho = rho'
// layout: [0..3] dot sums, [4] rho, [5] rho0, [6] alpha, [7] beta, [8] breakdown
__global__ void k_bp_scalars(int stage, double* sc) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (stage == 0) {
        sc[4] = sc[0] + sc[1];
        sc[5] = sc[4];
        sc[8] = 0.0;
    } else if (stage == 1) {
        const double g = sc[2] + sc[3];
        if (g > 0.0 && sc[4] > 0.0) {
            sc[6] = sc[4] / g;
        } else {
            sc[6] = 0.0;
            sc[8] = 1.0;
        }
    } else {
        const double r = sc[0] + sc[1];
        sc[7] = sc[4] > 0.0 ? r / sc[4] : 0.0;
        sc[4] = r;
    }
}

}  // namespace ieti
