// Device-side descriptors shared by the HIP kernels and the runtime.
#pragma once
#include <cstdint>

namespace ieti {

constexpr int TILE = 256;        // coefficients per work-group tile (one per thread)
constexpr int PW = 12;           // padded width of 1D transfer bands (nested: degree <= 10; L2 projection to degree 1: p <= 8)
constexpr int NPMAX = 20;        // local primal constraints per patch (8 vertices + 12 edges)

// Degree classes with their own unrolled kernels: 2D (p0, p1) in {2,3,4}^2 ->
// (p0-2) + 3 (p1-2); 3D p0=p1=p2 in {2,3} -> 9 + (p-2); anything else runs
// generic loops (class NCLASS).
constexpr int NCLASS = 11;
inline int degree_class(int dim, int p0, int p1, int p2) {
    if (dim == 2 && p0 >= 2 && p0 <= 4 && p1 >= 2 && p1 <= 4) return (p0 - 2) + 3 * (p1 - 2);
    if (dim == 3 && p0 == p1 && p1 == p2 && p0 >= 2 && p0 <= 3) return 9 + (p0 - 2);
    return NCLASS;
}

// Calls L(P0, P1, P2) with the compile-time degrees of class cls (-1: generic).
#define IETI_CLASS_SWITCH(cls, L)                \
    switch (cls) {                               \
    case 0: L(2, 2, 0); break;                   \
    case 1: L(3, 2, 0); break;                   \
    case 2: L(4, 2, 0); break;                   \
    case 3: L(2, 3, 0); break;                   \
    case 4: L(3, 3, 0); break;                   \
    case 5: L(4, 3, 0); break;                   \
    case 6: L(2, 4, 0); break;                   \
    case 7: L(3, 4, 0); break;                   \
    case 8: L(4, 4, 0); break;                   \
    case 9: L(2, 2, 2); break;                   \
    case 10: L(3, 3, 3); break;                  \
    default: L(-1, -1, -1); break;               \
    }

// One patch at one multigrid level.
struct PatchLev {
    int32_t M[3];          // basis functions per direction (1 in unused directions)
    int32_t p[3];          // degree per direction (0 in unused directions)
    int32_t dim, nst;
    int32_t pclass;        // compile-time degree class of the kernels, -1 = generic loops
    uint32_t mbits[3];     // per mode (N, D, K): side bits | corner bits << 8
    int32_t patch;         // patch id
    int32_t coarse;        // index of the same patch in the next coarser level, -1 if coarsest here
    int32_t fine;          // index of the same patch in the next finer level, -1 on level 0
    int64_t n;             // prod M
    int64_t voff;          // first coefficient in the level's vectors
    int64_t coff;          // first entry (s = 0) in the level's stencil array
    int64_t cstride;       // distance between consecutive stencil entries s, s+1
    double lmax[2];        // lambda_max(D^{-1}K), modes N and D
    double clo;            // lower end of the Chebyshev interval (x lambda_max)
    int64_t toff[3];       // prolongation table offsets per direction (fine = this level)
    int64_t roff[3];       // restriction table offsets per direction (coarse = next level)
    int64_t invoff;        // coarsest level: offset of the dense inverses (mode N, then mode D)
    int64_t moff[3];       // L2-projection transfer to the next level: offsets of the banded Cholesky factors
                           // of the 1D parametric mass matrices (M_d x (p_d + 1) each); moff[0] < 0: nested
};

// Level-0 quadrature layout of one patch (load vector).
struct PatchQ {
    int32_t nel[3];        // elements per direction
    int32_t Q[3];          // quadrature points per direction
    int64_t qoff;          // first quadrature point of the patch
    int64_t boff[3];       // 1D basis tables: Q[d] x (p+1) values per direction
    int64_t toff[2];       // load vector: the patch's intermediates after contracting direction 0 (and 1)
};

struct Tile {
    int32_t pl;            // index into the level's PatchLev array
    int32_t start;         // first coefficient of the tile
    int32_t gid;           // index of the tile in the level's list of all tiles (partial sums)
    int32_t pad;
};

constexpr int KMAX = 8;    // Chebyshev steps with precomputed coefficients

}  // namespace ieti
