// Host-side plan of an IETI-DP solve: topology, numbering, multigrid
// hierarchy and FP64 operator data.  Built once per ieti_setup; the device
// runtime uploads it.  Internal header (not part of the C ABI).
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ieti.h"

namespace ieti {

// Internal error carrying an ABI status code; caught at the ABI boundary.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// Masking modes of the patch stiffness (which coefficients are held at 0).
enum Mode : int {
    MODE_N = 0,   // local Neumann problem: boundary sides + primal (and boundary) vertices
    MODE_D = 1,   // local Dirichlet problem: every side of the patch
    MODE_K = 2,   // patch stiffness with only the boundary coefficients removed
};

// One multigrid level of one patch.
struct Level {
    int p[3] = {0, 0, 0};          // spline degree of the level's space per direction (0 in unused directions)
    int M[3] = {1, 1, 1};          // basis functions per direction (1 in unused directions)
    int nel[3] = {1, 1, 1};        // elements per direction
    int64_t n = 0;                 // prod M
    int64_t guard = 0;             // largest linear stencil offset p0 + p1 M0 + p2 M0 M1
    std::vector<double> knots[3];
    int nst = 0;                   // entries of the half stencil
    std::vector<int32_t> offs;     // 3 * nst offsets (o0, o1, o2); entry 0 is the diagonal
    std::vector<double> coef;      // nst * n, offset-major: K(i, i + o_s) at coef[s * n + i]
    double lmax[2] = {0, 0};       // lambda_max(D^{-1} K) for MODE_N, MODE_D
    // prolongation from the next coarser level into this one: dense Mf x Mc per direction.  Nested levels
    // (same degree): the canonical embedding.  Degree-1 coarse levels under a finest level of degree p
    // (options.coarse_degree = 1, Sec. 4): P holds the mixed parametric mass matrix M_fc (fine x coarse)
    // and mchol the banded Cholesky factor of the fine parametric mass matrix M_f (Mf x (p+1): row i holds
    // L(i, i-p .. i)), so that the transfer is the L2 projection M_f^{-1} M_fc and its transpose
    std::vector<double> P[3];
    int Mc[3] = {1, 1, 1};
    bool l2 = false;
    std::vector<double> mchol[3];
    // coarsest level only: dense inverses (n x n, masked rows/cols zero) for MODE_N, MODE_D
    std::vector<double> inv[2];
};

struct Patch {
    int dim = 2;
    int p[3] = {0, 0, 0};
    std::vector<double> knots[3];
    std::vector<double> ctrl;      // n * dim
    uint32_t bside = 0;            // bit 2d+e: side xi_d = e is on the boundary
    uint32_t pcorner = 0;          // bit c: corner c (c = e0 + 2 e1 + 4 e2) is a primal vertex
    uint32_t dcorner = 0;          // bit c: corner c is a boundary coefficient though on no boundary side
    bool affine = false;
    // no Dirichlet coefficient and no primal vertex: K is singular (the constants) and only the edge-average
    // constraints fix them.  The local Neumann solves then run on K + gamma C^T C (gamma = float_gamma), whose
    // restriction to {C w = 0} is K, and the multigrid levels >= 1 carry K + alpha M^ (M^ the mass matrix of the
    // parameter domain, alpha = FLOAT_ALPHA)
    bool floating = false;
    double float_gamma = 0.0;
    std::vector<Level> lv;         // lv[0] finest
    std::vector<double> qpw;       // w_q |det J_q| at the level-0 quadrature points
    std::vector<double> qpx;       // physical quadrature points, n_qp * dim
    std::vector<double> qpN[3];    // level-0 space basis at the quadrature points, Q_d x (p_d+1)
    std::vector<double> qpc[3];    // level 0: metric diagonal |det J| (J^{-1} J^{-T})_dd at the quadrature points
    // tensor-product smoother of the finest level, per mode (N, D): generalised eigenvectors U_d (P_d x P_d,
    // row-major, zero rows for coefficients the mode removes, zero padding) and eigenvalues (1e300 padding)
    struct Tensor {
        int Pd[3] = {0, 0, 0};
        std::vector<double> U[3], lam[3];
        double shift = 0.0, tau = 0.0;
    } ts[2];
    int64_t n_qp = 0;
    int64_t torn_off = 0;          // first coefficient in the torn layout
    // exact local solves: banded Cholesky factor L of the masked stiffness (modes N, D) in
    // 64-row blocks: per block row [L_off (64 x b) | U_off (64 x b) | inv(L_diag) (64 x 64)]
    int64_t band_b = 0, band_nblk = 0;
    std::vector<double> band[2];
    // local primal constraints: vertices (corner order) then edge averages (edge order)
    std::vector<int64_t> primal_global;
    std::vector<int> primal_corner;              // corner id, or -1 for an edge constraint
    std::vector<std::vector<int64_t>> primal_edge;  // local coefficients averaged by an edge constraint
};

struct Plan {
    int dim = 2;
    int N = 0;
    ieti_options opt{};
    std::string tune_cache;        // owned copy of opt.tune_cache (opt.tune_cache points into it)
    std::vector<Patch> patches;
    int64_t ndof_torn = 0, ndof_global = 0, n_qp = 0;
    int64_t n_lambda = 0, n_primal = 0, n_primal_vertices = 0;
    int max_levels = 0;
    // multipliers: torn positions of the +1 and -1 entries, multiplicity of the coefficient
    std::vector<int64_t> lam_plus, lam_minus;
    std::vector<int32_t> lam_mult;
    // B^T: interface slots (torn position) with their multipliers, CSR
    std::vector<int64_t> slot_pos, slot_ptr;
    std::vector<int64_t> slot_lam;
    std::vector<double> slot_sgn;                 // +1 / -1
    std::vector<int32_t> slot_mult;
    // groups of copies of shared non-boundary coefficients (torn positions), CSR
    std::vector<int64_t> grp_ptr, grp_pos;
    // global primal: contributors (patch, local constraint) per global primal, CSR
    std::vector<int64_t> pri_ptr, pri_patch, pri_local;
    // independent problems planned together (serving batches): patches, multipliers and quadrature points of
    // problem c are the ranges [beg[c], beg[c+1]); one problem unless planned with component ids
    int ncomp = 1;
    std::vector<int64_t> comp_patch_beg, comp_lam_beg, comp_qp_beg, comp_torn_beg;
};

constexpr int BAND_NB = 64;   // row block of the blocked banded triangular solves
constexpr double FLOAT_ALPHA = 1e-2;   // mass shift of the regularised multigrid of floating patches (Sec. 3.2)

// comp (may be NULL): non-decreasing problem id per patch; patches of different problems never share a vertex,
// side or multiplier, even where their geometry coincides
Plan* build_plan(const ieti_patch* patches, int n, const double* primal_vertices, int n_pv,
                 const ieti_options* opt, const int32_t* comp = nullptr);

// helpers shared with the runtime
void default_options(ieti_options* o);
int cheb_degree_for(const ieti_options& o, int dim, int pmax);
int cheb_degree_coarse_for(const ieti_options& o, int dim, int pmax);
double cheb_lower_for(const ieti_options& o, int dim, int pmax);
void set_last_error(const std::string& s);

}  // namespace ieti
