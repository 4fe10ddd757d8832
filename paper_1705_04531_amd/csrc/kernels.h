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

__device__ __forceinline__ bool masked(const PatchLev& P, int mode, int i0, int i1, int i2) {
    const uint32_t mb = P.mbits[mode];
    const uint32_t sides = mb & 0xFFu, corners = mb >> 8;
    const int ii[3] = {i0, i1, i2};
    bool m = false;
    int cb = 0, nend = 0;
    for (int d = 0; d < P.dim; ++d) {
        const bool lo = ii[d] == 0, hi = ii[d] == P.M[d] - 1;
        if (lo && ((sides >> (2 * d)) & 1u)) m = true;
        if (hi && ((sides >> (2 * d + 1)) & 1u)) m = true;
        if (lo || hi) {
            ++nend;
            if (hi) cb |= 1 << d;
        }
    }
    if (nend == P.dim && ((corners >> cb) & 1u)) m = true;
    return m;
}

__device__ __forceinline__ void unlin(const PatchLev& P, int64_t i, int& i0, int& i1, int& i2) {
    const int64_t M01 = (int64_t)P.M[0] * P.M[1];
    i2 = (int)(i / M01);
    const int64_t r = i - (int64_t)i2 * M01;
    i1 = (int)(r / P.M[0]);
    i0 = (int)(r - (int64_t)i1 * P.M[0]);
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

// Chebyshev step coefficients: d_k = s1 d_{k-1} + s2 D^{-1} r_k on [lo, hi] * lmax
__device__ __forceinline__ void cheb_coeffs(double lmax, double lo, double hi, int k, double& s1, double& s2) {
    const double a = lo * lmax, b = hi * lmax;
    const double theta = 0.5 * (a + b), delta = 0.5 * (b - a), sigma = theta / delta;
    if (k == 0) {
        s1 = 0.0;
        s2 = 1.0 / theta;
        return;
    }
    double rho_prev = 1.0 / sigma, rho = rho_prev;
    for (int j = 1; j <= k; ++j) {
        rho_prev = rho;
        rho = 1.0 / (2.0 * sigma - rho_prev);
    }
    s1 = rho * rho_prev;
    s2 = 2.0 * rho / delta;
}

// ------------------------------------------------------------------ stencil apply

enum Epi : int {
    EPI_APPLY = 0,   // y = alpha * m (K x)
    EPI_RESID = 1,   // y = m (b - K x)
    EPI_CHEB = 2,    // r = b - K x; d = s1 d + s2 r / diag; y = x + d  (y, d written)
    EPI_DOTS = 3,    // y = m (K x); partial[tile] = (x . y, x . r64)
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
    double cheb_hi;        // upper end of the smoothing interval (x lambda_max); lower end per patch
    double* partial;       // EPI_DOTS: 2 per tile
    const double* r64;     // EPI_DOTS
};

// One thread per output coefficient; reads K(i, i+o) at i and K(i-o, i) at
// i-o (symmetry) for the lower half of the stencil.  FINE marks launches on
// the finest level (the bandwidth-bound sweeps) so that profilers report
// them apart from the latency-bound coarse-level launches.
template <typename TC, typename TX, typename TY, int EPI, bool FINE>
__global__ __launch_bounds__(TILE) void k_stencil(StencilArgs a) {
    __shared__ double lds[2 * TILE / WAVE];
    const int t = tile_index(a.ntiles);
    if (t < 0) return;
    const Tile tl = a.tiles[t];
    const PatchLev P = a.L[tl.pl];
    if (a.active && !a.active[P.patch]) return;
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    const TC* __restrict__ coef = (const TC*)a.coef;
    const TX* __restrict__ x = (const TX*)a.x;
    TY* __restrict__ y = (TY*)a.y;
    double dv[2] = {0.0, 0.0};
    if (i < P.n) {
        int i0, i1, i2;
        unlin(P, i, i0, i1, i2);
        const bool m = masked(P, a.mode, i0, i1, i2);
        const int64_t vi = P.voff + i;
        TC acc = TC(0), diag = TC(1);
        if (!m) {
            const TC* c = coef + P.coff + i;
            const TX* xp = x + vi;
            const int64_t cs = P.cstride;
            const int64_t M0 = P.M[0], M01 = (int64_t)P.M[0] * P.M[1];
            const int p0 = P.p[0], p1 = P.p[1], p2 = P.p[2];
            int s = 0;
            for (int o2 = 0; o2 <= p2; ++o2)
                for (int o1 = (o2 == 0 ? 0 : -p1); o1 <= p1; ++o1) {
                    const int o0s = (o2 == 0 && o1 == 0) ? 0 : -p0;
                    const int64_t base = o1 * M0 + o2 * M01;
                    for (int o0 = o0s; o0 <= p0; ++o0, ++s) {
                        const int64_t off = base + o0;
                        const TC cu = c[s * cs];
                        acc += cu * TC(xp[off]);
                        if (s) acc += c[s * cs - off] * TC(xp[-off]);
                        else diag = cu;
                    }
                }
        }
        if constexpr (EPI == EPI_APPLY) {
            y[vi] = m ? TY(0) : TY(a.alpha * (double)acc);
        } else if constexpr (EPI == EPI_RESID) {
            const TY* b = (const TY*)a.b;
            y[vi] = m ? TY(0) : TY(TC(b[vi]) - acc);
        } else if constexpr (EPI == EPI_CHEB) {
            const TY* b = (const TY*)a.b;
            TY* d = (TY*)a.d;
            if (m) {
                y[vi] = TY(0);
                d[vi] = TY(0);
            } else {
                double s1, s2;
                cheb_coeffs(P.lmax[a.mode], P.clo, a.cheb_hi, a.cheb_k, s1, s2);
                const TC r = TC(b[vi]) - acc;
                const TC dn = (s1 != 0.0 ? TC(s1) * TC(d[vi]) : TC(0)) + TC(s2) * r / diag;
                d[vi] = TY(dn);
                y[vi] = TY(TC(x[vi]) + dn);
            }
        } else if constexpr (EPI == EPI_DOTS) {
            const double q = m ? 0.0 : (double)acc;
            y[vi] = TY(q);
            const double xv = (double)x[vi];
            dv[0] = xv * q;
            dv[1] = xv * a.r64[vi];
        }
    }
    if constexpr (EPI == EPI_DOTS) {
        block_sum<2>(dv, lds);
        if (threadIdx.x == 0) {
            a.partial[2 * t] = dv[0];
            a.partial[2 * t + 1] = dv[1];
        }
    }
}

// ------------------------------------------------------------------ smoother start, transfers, coarse solve

// First Chebyshev step from a zero guess: x = d = m b / (theta diag)
template <typename T>
__global__ __launch_bounds__(TILE) void k_cheb_zero(const PatchLev* L, const Tile* tiles, int ntiles, const T* coef,
                                                    const T* b, T* x, T* d, int mode, double hi,
                                                    const int* active) {
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev P = L[tl.pl];
    if (active && !active[P.patch]) return;
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    if (i >= P.n) return;
    int i0, i1, i2;
    unlin(P, i, i0, i1, i2);
    const int64_t vi = P.voff + i;
    if (masked(P, mode, i0, i1, i2)) {
        x[vi] = T(0);
        d[vi] = T(0);
        return;
    }
    const double lm = P.lmax[mode];
    const double theta = 0.5 * (P.clo + hi) * lm;
    const double v = (double)b[vi] / (theta * (double)coef[P.coff + i]);
    x[vi] = T(v);
    d[vi] = T(v);
}

// Restriction b_c = m_c P^T r_f, one thread per coarse coefficient.
template <typename T>
__global__ __launch_bounds__(TILE) void k_restrict(const PatchLev* Lf, const PatchLev* Lc, const Tile* tiles,
                                                   int ntiles, const int32_t* rlo, const T* rval, const T* rf, T* bc,
                                                   int mode, const int* active) {
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev C = Lc[tl.pl];
    if (active && !active[C.patch]) return;
    const int64_t I = (int64_t)tl.start + threadIdx.x;
    if (I >= C.n) return;
    const PatchLev F = Lf[C.fine];
    int I0, I1, I2;
    unlin(C, I, I0, I1, I2);
    if (masked(C, mode, I0, I1, I2)) {
        bc[C.voff + I] = T(0);
        return;
    }
    const int Ic[3] = {I0, I1, I2};
    int lo[3] = {0, 0, 0}, w[3] = {1, 1, 1};
    const T* v[3] = {nullptr, nullptr, nullptr};
    for (int d = 0; d < F.dim; ++d) {
        lo[d] = rlo[F.roff[d] + Ic[d]];
        v[d] = rval + (F.roff[d] + Ic[d]) * PW;
        w[d] = F.p[d] + 2;
    }
    const int64_t M0 = F.M[0], M01 = (int64_t)F.M[0] * F.M[1];
    double acc = 0.0;
    for (int a2 = 0; a2 < w[2]; ++a2) {
        const double v2 = F.dim == 3 ? (double)v[2][a2] : 1.0;
        if (v2 == 0.0) continue;
        for (int a1 = 0; a1 < w[1]; ++a1) {
            const double v12 = v2 * (double)v[1][a1];
            if (v12 == 0.0) continue;
            const int64_t row = F.voff + (lo[1] + a1) * M0 + (F.dim == 3 ? (lo[2] + a2) * M01 : 0) + lo[0];
            for (int a0 = 0; a0 < w[0]; ++a0) acc += v12 * (double)v[0][a0] * (double)rf[row + a0];
        }
    }
    bc[C.voff + I] = T(acc);
}

// Prolongation x_f += m_f P e_c, one thread per fine coefficient.
template <typename T>
__global__ __launch_bounds__(TILE) void k_prolong(const PatchLev* Lf, const PatchLev* Lc, const Tile* tiles,
                                                  int ntiles, const int32_t* plo, const T* pval, const T* ec, T* xf,
                                                  int mode, const int* active) {
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev F = Lf[tl.pl];
    if (active && !active[F.patch]) return;
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    if (i >= F.n) return;
    int i0, i1, i2;
    unlin(F, i, i0, i1, i2);
    if (masked(F, mode, i0, i1, i2)) return;
    const PatchLev C = Lc[F.coarse];
    const int ii[3] = {i0, i1, i2};
    int lo[3] = {0, 0, 0}, w[3] = {1, 1, 1};
    const T* v[3] = {nullptr, nullptr, nullptr};
    for (int d = 0; d < F.dim; ++d) {
        lo[d] = plo[F.toff[d] + ii[d]];
        v[d] = pval + (F.toff[d] + ii[d]) * PW;
        w[d] = F.p[d] + 2;
    }
    const int64_t M0 = C.M[0], M01 = (int64_t)C.M[0] * C.M[1];
    double acc = 0.0;
    for (int a2 = 0; a2 < w[2]; ++a2) {
        const double v2 = F.dim == 3 ? (double)v[2][a2] : 1.0;
        if (v2 == 0.0) continue;
        for (int a1 = 0; a1 < w[1]; ++a1) {
            const double v12 = v2 * (double)v[1][a1];
            if (v12 == 0.0) continue;
            const int64_t row = C.voff + (lo[1] + a1) * M0 + (F.dim == 3 ? (lo[2] + a2) * M01 : 0) + lo[0];
            for (int a0 = 0; a0 < w[0]; ++a0) acc += v12 * (double)v[0][a0] * (double)ec[row + a0];
        }
    }
    const int64_t vi = F.voff + i;
    xf[vi] = T((double)xf[vi] + acc);
}

// Coarsest level: x = A^{-1} b with the stored dense inverse; one work-group per patch.
template <typename T>
__global__ __launch_bounds__(TILE) void k_coarse(const PatchLev* L, const int32_t* list, int nlist, const T* inv,
                                                 const T* b, T* x, int mode, const int* active) {
    if ((int)blockIdx.x >= nlist) return;
    const PatchLev P = L[list[blockIdx.x]];
    if (active && !active[P.patch]) return;
    const int64_t n = P.n;
    const T* A = inv + P.invoff + (int64_t)mode * n * n;
    const T* bb = b + P.voff;
    for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
        double acc = 0.0;
        const T* row = A + r * n;
        for (int64_t j = 0; j < n; ++j) acc += (double)row[j] * (double)bb[j];
        x[P.voff + r] = T(acc);
    }
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
    const PatchLev P = L[tl.pl];
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
    const PatchLev P = L[tl.pl];
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
    const PatchLev P = L[tl.pl];
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
    const PatchLev P = L[tl.pl];
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
    const PatchLev P = L[tl.pl];
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
    if (threadIdx.x == 0) partial[t] = v[0];
}

// per-tile partial of z . q
template <typename T>
__global__ __launch_bounds__(TILE) void k_fcg_zq(const PatchLev* L, const Tile* tiles, int ntiles, const T* z,
                                                 const double* q, double* partial, const int* active) {
    __shared__ double lds[TILE / WAVE];
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev P = L[tl.pl];
    if (!active[P.patch]) return;
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    double v[1] = {0.0};
    if (i < P.n) v[0] = (double)z[P.voff + i] * q[P.voff + i];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) partial[t] = v[0];
}

// d = m (z - beta d)
template <typename T>
__global__ __launch_bounds__(TILE) void k_fcg_dir(const PatchLev* L, const Tile* tiles, int ntiles, const T* z,
                                                  double* d, const double* beta, int mode, const int* active) {
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev P = L[tl.pl];
    if (!active[P.patch]) return;
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    if (i >= P.n) return;
    int i0, i1, i2;
    unlin(P, i, i0, i1, i2);
    const int64_t vi = P.voff + i;
    const double bt = beta[P.patch];
    d[vi] = masked(P, mode, i0, i1, i2) ? 0.0 : (double)z[vi] - bt * d[vi];
}

// x += alpha d, r -= alpha q, rT = r, partial = |r|^2
template <typename T>
__global__ __launch_bounds__(TILE) void k_fcg_update(const PatchLev* L, const Tile* tiles, int ntiles,
                                                     const double* d, const double* q, double* x, double* r, T* rT,
                                                     const double* alpha, double* partial, const int* active) {
    __shared__ double lds[TILE / WAVE];
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev P = L[tl.pl];
    if (!active[P.patch]) return;
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    double v[1] = {0.0};
    if (i < P.n) {
        const int64_t vi = P.voff + i;
        const double al = alpha[P.patch];
        x[vi] += al * d[vi];
        const double rv = r[vi] - al * q[vi];
        r[vi] = rv;
        rT[vi] = T(rv);
        v[0] = rv * rv;
    }
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) partial[t] = v[0];
}

// Per-patch scalars from tile partials (one thread per patch, fixed summation order).
//  stage 0 (init):   bb = sum |r|^2; active = bb > 0; its = 0
//  stage 1 (beta):   beta = first ? 0 : sum(z.q) / dq
//  stage 2 (alpha):  dq = sum(d.q); alpha = sum(d.r) / dq   (dq <= 0 stops the patch)
//  stage 3 (check):  rr = sum |r|^2; its += 1; active = rr > tol^2 bb && its < maxit
__global__ void k_fcg_scalars(int npatch, const int32_t* tile_ptr, const double* partial, int stride, int stage,
                              double* bb, double* dq, double* beta, double* alpha, int* active, int* its,
                              double tol2, int maxit, int first, int* nactive) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npatch) return;
    if (stage != 0 && !active[k]) return;
    double s0 = 0.0, s1 = 0.0;
    for (int t = tile_ptr[k]; t < tile_ptr[k + 1]; ++t) {
        s0 += partial[(int64_t)stride * t];
        if (stride > 1) s1 += partial[(int64_t)stride * t + 1];
    }
    if (stage == 0) {
        bb[k] = s0;
        active[k] = s0 > 0.0 ? 1 : 0;
        its[k] = 0;
        if (active[k]) atomicAdd(nactive, 1);
    } else if (stage == 1) {
        beta[k] = first ? 0.0 : s0 / dq[k];
    } else if (stage == 2) {
        dq[k] = s0;
        if (!(s0 > 0.0)) {
            alpha[k] = 0.0;
            active[k] = 0;
        } else {
            alpha[k] = s1 / s0;
        }
    } else {
        its[k] += 1;
        const bool go = s0 > tol2 * bb[k] && its[k] < maxit;
        active[k] = go ? 1 : 0;
        if (go) atomicAdd(nactive, 1);
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

// Per patch k (one work-group): c[k][j] = psi_j . g over the patch's rows and,
// for edge constraints, e[k][j] = mean of y over the edge.  Rows are either
// the patch's interface slots (compact psiG, slot-major with NPMAX stride;
// row_ptr/row_dev give the slots of each patch) or, with L0 != null, all
// coefficients of the patch (full psi: NPMAX level-0 vectors).
__global__ __launch_bounds__(TILE) void k_pri_dots(int npatch, const int32_t* npk, const int64_t* row_ptr,
                                                   const int64_t* row_dev, const PatchLev* L0, const double* psi,
                                                   int64_t psi_stride, const double* g, const double* y,
                                                   const int64_t* edge_ptr, const int64_t* edge_dev, double* c,
                                                   double* e) {
    __shared__ double lds[TILE / WAVE];
    const int k = blockIdx.x;
    if (k >= npatch) return;
    const int nj = npk[k];
    for (int j = 0; j < nj; ++j) {
        double v[1] = {0.0};
        if (L0) {
            const PatchLev P = L0[k];
            for (int64_t r = threadIdx.x; r < P.n; r += blockDim.x)
                v[0] += psi[(int64_t)j * psi_stride + P.voff + r] * g[P.voff + r];
        } else {
            for (int64_t r = row_ptr[k] + threadIdx.x; r < row_ptr[k + 1]; r += blockDim.x)
                v[0] += psi[r * NPMAX + j] * g[row_dev[r]];
        }
        block_sum<1>(v, lds);
        if (threadIdx.x == 0) c[k * NPMAX + j] = v[0];
        const int64_t eb = edge_ptr[k * NPMAX + j], ee = edge_ptr[k * NPMAX + j + 1];
        if (y && ee > eb) {
            double w[1] = {0.0};
            for (int64_t r = eb + threadIdx.x; r < ee; r += blockDim.x) w[0] += y[edge_dev[r]];
            block_sum<1>(w, lds);
            if (threadIdx.x == 0) e[k * NPMAX + j] = w[0] / (double)(ee - eb);
        } else if (threadIdx.x == 0) {
            e[k * NPMAX + j] = 0.0;
        }
    }
}

// One work-group: gPi = sum of contributions, uPi = Sinv gPi, coef[k][j] = uPi[R_kj] - e[k][j]
__global__ __launch_bounds__(1024) void k_pri_coarse(int64_t npi, const int64_t* pri_ptr, const int64_t* pri_patch,
                                                     const int64_t* pri_local, const double* c, const double* Sinv,
                                                     double* gpi, double* upi, int npatch, const int32_t* npk,
                                                     const int64_t* Rk, const double* e, double* coef) {
    for (int64_t J = threadIdx.x; J < npi; J += blockDim.x) {
        double s = 0.0;
        for (int64_t q = pri_ptr[J]; q < pri_ptr[J + 1]; ++q) s += c[pri_patch[q] * NPMAX + pri_local[q]];
        gpi[J] = s;
    }
    __syncthreads();
    for (int64_t J = threadIdx.x; J < npi; J += blockDim.x) {
        double s = 0.0;
        for (int64_t K = 0; K < npi; ++K) s += Sinv[J * npi + K] * gpi[K];
        upi[J] = s;
    }
    __syncthreads();
    for (int64_t q = threadIdx.x; q < (int64_t)npatch * NPMAX; q += blockDim.x) {
        const int k = (int)(q / NPMAX), j = (int)(q % NPMAX);
        coef[q] = j < npk[k] ? upi[Rk[q]] - e[q] : 0.0;
    }
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
    const PatchLev P = L[tl.pl];
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    if (i >= P.n) return;
    const int64_t vi = P.voff + i;
    const int k = P.patch;
    double acc = y[vi];
    for (int j = 0; j < npk[k]; ++j) acc += psi[(int64_t)j * psi_stride + vi] * coef[k * NPMAX + j];
    u[vi] = acc;
}

// ------------------------------------------------------------------ load vector, groups, output

// f_i = sum_q w_q |det J_q| f(x_q) N_i(xi_q), one thread per coefficient (level 0)
__global__ __launch_bounds__(TILE) void k_loadvec(const PatchLev* L, const PatchQ* PQ, const Tile* tiles, int ntiles,
                                                  const double* basis, const double* qpw, const double* fq,
                                                  double* fvec) {
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev P = L[tl.pl];
    const PatchQ Q = PQ[P.patch];
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    if (i >= P.n) return;
    int ii[3];
    unlin(P, i, ii[0], ii[1], ii[2]);
    int elo[3] = {0, 0, 0}, ehi[3] = {0, 0, 0}, ng[3] = {1, 1, 1};
    for (int d = 0; d < P.dim; ++d) {
        elo[d] = ii[d] - P.p[d] > 0 ? ii[d] - P.p[d] : 0;
        ehi[d] = ii[d] < Q.nel[d] - 1 ? ii[d] : Q.nel[d] - 1;
        ng[d] = P.p[d] + 1;
    }
    double acc = 0.0;
    for (int e2 = elo[2]; e2 <= ehi[2]; ++e2)
        for (int g2 = 0; g2 < ng[2]; ++g2) {
            const int q2 = e2 * ng[2] + g2;
            const double b2 = P.dim == 3 ? basis[Q.boff[2] + (int64_t)q2 * ng[2] + (ii[2] - e2)] : 1.0;
            for (int e1 = elo[1]; e1 <= ehi[1]; ++e1)
                for (int g1 = 0; g1 < ng[1]; ++g1) {
                    const int q1 = e1 * ng[1] + g1;
                    const double b12 = b2 * basis[Q.boff[1] + (int64_t)q1 * ng[1] + (ii[1] - e1)];
                    const int64_t qrow = Q.qoff + ((int64_t)(P.dim == 3 ? q2 : 0) * Q.Q[1] + q1) * Q.Q[0];
                    for (int e0 = elo[0]; e0 <= ehi[0]; ++e0)
                        for (int g0 = 0; g0 < ng[0]; ++g0) {
                            const int q0 = e0 * ng[0] + g0;
                            const double b = b12 * basis[Q.boff[0] + (int64_t)q0 * ng[0] + (ii[0] - e0)];
                            acc += b * qpw[qrow + q0] * fq[qrow + q0];
                        }
                }
        }
    fvec[P.voff + i] = acc;
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
    const PatchLev P = L[tl.pl];
    const int64_t i = (int64_t)tl.start + threadIdx.x;
    double acc[1] = {0.0};
    if (i < P.n) {
        int i0, i1, i2;
        unlin(P, i, i0, i1, i2);
        if (!masked(P, mode, i0, i1, i2)) acc[0] = v[P.voff + i] * v[P.voff + i];
    }
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) partial[t] = acc[0];
}

// out (torn layout) = v (guarded level-0 layout)
__global__ __launch_bounds__(TILE) void k_copy_out(const PatchLev* L, const Tile* tiles, int ntiles,
                                                   const int64_t* torn_off, const double* v, double* out) {
    const int t = tile_index(ntiles);
    if (t < 0) return;
    const Tile tl = tiles[t];
    const PatchLev P = L[tl.pl];
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
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += a[i] * b[i];
    for (int o = WAVE / 2; o > 0; o >>= 1) acc += __shfl_down(acc, o, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) lds[threadIdx.x / WAVE] = acc;
    __syncthreads();
    double s = 0.0;
    for (int j = 0; j < (int)(blockDim.x / WAVE); ++j) s += lds[j];
    __syncthreads();
    return s;
}

// sc: [0] rz, [1] alpha, [2] beta, [3] |r|^2, [4] breakdown flag, [5] |d|^2 (scale), [6] pq
// stage 0: rz = r.z, p = z            (start)
// stage 1: pq = p.q; alpha = rz/pq; lam += alpha p; r -= alpha q; |r|^2
// stage 2: rz' = r.z; beta = rz'/rz; p = z + beta p; rz = rz'
__global__ __launch_bounds__(1024) void k_pcg(int stage, int64_t n, double* lam, double* r, const double* z,
                                              double* p, const double* q, double* sc) {
    __shared__ double lds[1024 / WAVE];
    if (stage == 0) {
        const double rz = wg_dot(r, z, n, lds);
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = z[i];
        if (threadIdx.x == 0) sc[0] = rz;
    } else if (stage == 1) {
        const double pq = wg_dot(p, q, n, lds);
        double alpha = sc[0] / pq;
        const bool brk = !(pq > 0.0);
        if (brk) alpha = 0.0;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            lam[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        __syncthreads();
        const double rr = wg_dot(r, r, n, lds);
        if (threadIdx.x == 0) {
            sc[1] = alpha;
            sc[3] = rr;
            sc[4] = brk ? 1.0 : 0.0;
            sc[6] = pq;
        }
    } else {
        const double rzn = wg_dot(r, z, n, lds);
        const double beta = rzn / sc[0];
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = z[i] + beta * p[i];
        if (threadIdx.x == 0) {
            sc[2] = beta;
            sc[0] = rzn;
        }
    }
}

// |a|^2 and |b|^2 (+ |c|^2) into out[0..2] (one work-group)
__global__ __launch_bounds__(1024) void k_norms(int64_t n, const double* a, const double* b, const double* c,
                                                double* out) {
    __shared__ double lds[1024 / WAVE];
    const double na = wg_dot(a, a, n, lds);
    const double nb = b ? wg_dot(b, b, n, lds) : 0.0;
    const double nc = c ? wg_dot(c, c, n, lds) : 0.0;
    if (threadIdx.x == 0) {
        out[0] = na;
        out[1] = nb;
        out[2] = nc;
    }
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
    const PatchLev P = L[tl.pl];
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
    const PatchLev P = L[k];
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

}  // namespace ieti
