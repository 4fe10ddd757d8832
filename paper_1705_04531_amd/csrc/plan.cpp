// Host-side planning of an IETI-DP solve (no device calls).
//
//  * interfaces and the torn numbering (Sec. 2: patches, interface Gamma,
//    tearing of the interface unknowns);
//  * primal constraints -- vertex values and optional 3D edge averages
//    (the strongly enforced continuity conditions of Sec. 2 / Sec. 4) --
//    and the fully redundant Lagrange multipliers of the jump operator B;
//  * the multigrid hierarchy of every patch: nested h-levels obtained by
//    removing every second breakpoint, the canonical embedding between them
//    (knot insertion), Galerkin stiffness of each level on the fine geometry
//    (Sec. 4: nested grids, p fixed), dense inverses on the coarsest level;
//  * Chebyshev smoothing intervals (power iteration on D^{-1} K).
//
// Operator data are half stencils: for coefficient i and offset o with o in
// the "upper" half (last nonzero component positive, diagonal first),
// coef[s][i] = K(i, i + o_s); the lower half follows from symmetry.
#include "plan.h"

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <numeric>
#include <thread>

namespace ieti {

static thread_local std::string g_last_error;
void set_last_error(const std::string& s) { g_last_error = s; }
const char* last_error() { return g_last_error.c_str(); }

void default_options(ieti_options* o) {
    std::memset(o, 0, sizeof(*o));
    o->local_solver = IETI_LOCAL_MG;
    o->mg_precision = 64;
    o->primal = IETI_PRIMAL_VERTICES;
    o->cheb_degree = 0;
    o->cheb_degree_coarse = 0;
    o->cheb_lower = 0.0;
    o->prec_vcycles = 2;
    o->max_it = 300;
    o->inner_max_it = 400;
    o->tol = 1e-8;
    o->inner_tol = 1e-10;
    o->basis_tol = 1e-12;
    o->check_every = 4;
    o->use_graph = 0;
    o->coarse_level = 0;
    o->coarse_dofs = 512;
    o->autotune = 0;
    o->smoother = IETI_SMOOTHER_CHEBYSHEV;
    o->smoother_sigma = 0.3;
    o->device = -1;
    o->stream = nullptr;
    o->hbm_budget = 0;
    o->batch_dofs = 2000000;
    o->coarse_degree = 0;
}

// Smoother choice per dimension and spline degree (degree of the Chebyshev
// polynomial per smoothing phase, lower end of its interval as a fraction of
// lambda_max), from measured solve times on MI355X over a grid of both
// parameters: higher degrees pay off because a V-cycle's coarse part costs
// about as much as several finest-level sweeps; the coarse levels, whose
// sweeps are latency bound, take a lower degree.  In 3D (p <= 2) the weaker
// point-Jacobi smoothing of the 27-point couplings wants a higher degree and
// a wider interval than in 2D.
int cheb_degree_for(const ieti_options& o, int dim, int pmax) {
    if (o.cheb_degree > 0) return o.cheb_degree;
    if (pmax <= 2) return dim == 3 ? 4 : 3;
    if (pmax == 3) return 6;
    if (pmax == 4) return 7;
    return 8;
}
int cheb_degree_coarse_for(const ieti_options& o, int dim, int pmax) {
    (void)dim;
    (void)pmax;
    if (o.cheb_degree_coarse > 0) return o.cheb_degree_coarse;
    // under the finest-level tensor smoother one step per coarse phase is enough (measured: fewer stencil
    // reads in the per-patch coarse kernel outweigh the slightly higher inner iteration counts)
    return o.smoother == IETI_SMOOTHER_TENSOR ? 1 : 2;
}
double cheb_lower_for(const ieti_options& o, int dim, int pmax) {
    if (o.cheb_lower > 0) return o.cheb_lower;
    if (pmax <= 2) return dim == 3 ? 0.05 : 0.08;
    if (pmax == 3) return 0.03;
    if (pmax == 4) return 0.02;
    return 0.01;
}

// ----------------------------------------------------------------------------
// thread pool helper
static void parallel_for(int n, const std::function<void(int)>& fn) {
    int nt = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 16u);
    nt = std::min(nt, n);
    if (nt <= 1) {
        for (int i = 0; i < n; ++i) fn(i);
        return;
    }
    std::atomic<int> next(0);
    std::vector<std::thread> th;
    std::vector<std::string> errs(nt);
    std::vector<int> codes(nt, 0);
    for (int t = 0; t < nt; ++t) {
        th.emplace_back([&, t] {
            try {
                for (int i = next++; i < n; i = next++) fn(i);
            } catch (const Error& e) {
                codes[t] = e.code;
                errs[t] = e.what();
            } catch (const std::exception& e) {
                codes[t] = IETI_EINVAL;
                errs[t] = e.what();
            }
        });
    }
    for (auto& x : th) x.join();
    for (int t = 0; t < nt; ++t)
        if (codes[t]) throw Error(codes[t], errs[t]);
}

// ----------------------------------------------------------------------------
// B-splines

// Span k with t[k] <= x < t[k+1] among the non-empty spans p..m-1 (m basis functions).
static int find_span(const std::vector<double>& t, int p, double x) {
    int m = (int)t.size() - p - 1;
    if (x >= t[m]) return m - 1;
    if (x <= t[p]) return p;
    int lo = p, hi = m;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (x < t[mid]) hi = mid; else lo = mid;
    }
    return lo;
}

// Values and first derivatives of the p+1 basis functions k-p..k that are
// nonzero on span k, built degree by degree from the Cox-de Boor recursion.
static void basis_on_span(const std::vector<double>& t, int p, int k, double x, double* N, double* dN) {
    double prev[16], cur[16];
    prev[0] = 1.0;   // degree 0: function k
    for (int q = 1; q <= p; ++q) {
        // degree q: functions k-q .. k; prev holds degree q-1 functions k-q+1 .. k
        for (int r = 0; r <= q; ++r) {
            int i = k - q + r;
            double v = 0.0;
            if (r >= 1) v += (x - t[i]) / (t[i + q] - t[i]) * prev[r - 1];
            if (r <= q - 1) v += (t[i + q + 1] - x) / (t[i + q + 1] - t[i + 1]) * prev[r];
            cur[r] = v;
        }
        if (q == p && dN) {
            for (int r = 0; r <= p; ++r) {
                int i = k - p + r;
                double d = 0.0;
                if (r >= 1) d += p / (t[i + p] - t[i]) * prev[r - 1];
                if (r <= p - 1) d -= p / (t[i + p + 1] - t[i + 1]) * prev[r];
                dN[r] = d;
            }
        }
        for (int r = 0; r <= q; ++r) prev[r] = cur[r];
    }
    if (p == 0 && dN) dN[0] = 0.0;
    for (int r = 0; r <= p; ++r) N[r] = prev[r];
}

static std::vector<double> breakpoints(const std::vector<double>& t) {
    std::vector<double> b;
    for (double v : t)
        if (b.empty() || v > b.back()) b.push_back(v);
    return b;
}

// Gauss-Legendre nodes/weights on [0,1] by Newton's method on P_n.
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) { p1 = z; p0 = 1.0; }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[n - 1 - i] = 0.5 * (z + 1.0);
        w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);   // = 2/((1-z^2)P'^2) scaled by 1/2
    }
}

// Canonical embedding S_p(coarse) -> S_p(fine) by inserting the missing knots
// one at a time (Boehm): each insertion of x into span k maps coefficients by
// Q_i = a_i P_i + (1 - a_i) P_{i-1}, a_i = 1 (i <= k-p), (x - t_i)/(t_{i+p} - t_i)
// (k-p < i <= k), 0 (i > k).  Returns the dense Mf x Mc matrix (row-major).
static std::vector<double> prolongation(const std::vector<double>& coarse, const std::vector<double>& fine, int p,
                                        int& Mf, int& Mc) {
    Mc = (int)coarse.size() - p - 1;
    std::vector<double> t = coarse;
    int rows = Mc;
    std::vector<double> P((size_t)Mc * Mc, 0.0);
    for (int i = 0; i < Mc; ++i) P[(size_t)i * Mc + i] = 1.0;
    std::vector<double> bc = breakpoints(coarse), bf = breakpoints(fine);
    for (double x : bf) {
        if (std::binary_search(bc.begin(), bc.end(), x)) continue;
        int k = find_span(t, p, x);
        std::vector<double> Q((size_t)(rows + 1) * Mc, 0.0);
        for (int i = 0; i <= rows; ++i) {
            double a;
            if (i <= k - p) a = 1.0;
            else if (i > k) a = 0.0;
            else a = (x - t[i]) / (t[i + p] - t[i]);
            for (int c = 0; c < Mc; ++c) {
                double v = 0.0;
                if (a != 0.0 && i < rows) v += a * P[(size_t)i * Mc + c];
                if (a != 1.0 && i >= 1) v += (1.0 - a) * P[(size_t)(i - 1) * Mc + c];
                Q[(size_t)i * Mc + c] = v;
            }
        }
        t.insert(t.begin() + k + 1, x);
        P.swap(Q);
        ++rows;
    }
    Mf = rows;
    if ((int)fine.size() - p - 1 != Mf) throw Error(IETI_EINVAL, "knot insertion did not reach the fine knot vector");
    for (auto& v : P)
        if (std::fabs(v) < 1e-15) v = 0.0;
    return P;
}

// Mixed parametric mass matrix (Mf x Mc, dense row-major) of the spline spaces (tf, pf) and (tc, pc) on
// [0,1]: int N_i^f N_j^c, by Gauss quadrature on the union of both meshes' breakpoints with
// max(pf, pc) + 1 points per interval (exact for the degree pf + pc products).
static std::vector<double> mixed_mass(const std::vector<double>& tf, int pf, const std::vector<double>& tc, int pc) {
    const int Mf = (int)tf.size() - pf - 1, Mc = (int)tc.size() - pc - 1;
    std::vector<double> bf = breakpoints(tf), bcv = breakpoints(tc), b;
    b.insert(b.end(), bf.begin(), bf.end());
    b.insert(b.end(), bcv.begin(), bcv.end());
    std::sort(b.begin(), b.end());
    b.erase(std::unique(b.begin(), b.end(), [](double x, double y) { return std::fabs(x - y) < 1e-14; }), b.end());
    std::vector<double> gx, gw;
    gauss_legendre(std::max(pf, pc) + 1, gx, gw);
    std::vector<double> A((size_t)Mf * Mc, 0.0), Nf(pf + 1), dNf(pf + 1), Nc(pc + 1), dNc(pc + 1);
    for (size_t e = 0; e + 1 < b.size(); ++e) {
        const double a = b[e], c = b[e + 1], mid = 0.5 * (a + c);
        const int kf = find_span(tf, pf, mid), kc = find_span(tc, pc, mid);
        for (size_t g = 0; g < gx.size(); ++g) {
            const double x = a + (c - a) * gx[g], w = (c - a) * gw[g];
            basis_on_span(tf, pf, kf, x, Nf.data(), dNf.data());
            basis_on_span(tc, pc, kc, x, Nc.data(), dNc.data());
            for (int i = 0; i <= pf; ++i)
                for (int j = 0; j <= pc; ++j) A[(size_t)(kf - pf + i) * Mc + (kc - pc + j)] += w * Nf[i] * Nc[j];
        }
    }
    return A;
}

// Banded Cholesky factor of the parametric mass matrix of the spline space (t, p) on [0,1]: M x (p+1),
// row i holds L(i, i-p .. i) (entries before column 0 are zero).
static std::vector<double> band_mass_chol(const std::vector<double>& t, int p) {
    const std::vector<double> Mm = mixed_mass(t, p, t, p);
    const int M = (int)t.size() - p - 1, w = p + 1;
    std::vector<double> L((size_t)M * w, 0.0);
    auto at = [&](int i, int j) -> double& { return L[(size_t)i * w + (j - i + p)]; };   // j in [i-p, i]
    for (int j = 0; j < M; ++j) {
        double d = Mm[(size_t)j * M + j];
        for (int k = std::max(0, j - p); k < j; ++k) d -= at(j, k) * at(j, k);
        if (!(d > 0)) throw Error(IETI_EINVAL, "mass matrix is not positive definite");
        const double c = std::sqrt(d);
        at(j, j) = c;
        for (int i = j + 1; i <= std::min(M - 1, j + p); ++i) {
            double v = Mm[(size_t)i * M + j];
            for (int k = std::max(0, i - p); k < j; ++k) v -= at(i, k) * at(j, k);
            at(i, j) = v / c;
        }
    }
    return L;
}

// ----------------------------------------------------------------------------
// per-direction quadrature tables of one level

struct DirTable {
    int p = 0, nel = 0, Q = 0;          // Q = nel * (p + 1) points
    std::vector<double> xi, w;          // parameter points and weights
    std::vector<int> first;             // first nonzero space function of the element of each point
    std::vector<double> N, dN;          // (p+1) per point: space basis
    int pg = 0;
    std::vector<int> gfirst;            // first nonzero geometry function at each point
    std::vector<double> G, dG;          // (pg+1) per point: geometry basis
};

static DirTable make_dir(const std::vector<double>& tl, int p, const std::vector<double>& tg, int pg) {
    DirTable d;
    d.p = p;
    d.pg = pg;
    std::vector<double> b = breakpoints(tl);
    d.nel = (int)b.size() - 1;
    std::vector<double> gx, gw;
    gauss_legendre(p + 1, gx, gw);
    d.Q = d.nel * (p + 1);
    d.xi.resize(d.Q);
    d.w.resize(d.Q);
    d.first.resize(d.Q);
    d.N.resize((size_t)d.Q * (p + 1));
    d.dN.resize((size_t)d.Q * (p + 1));
    d.gfirst.resize(d.Q);
    d.G.resize((size_t)d.Q * (pg + 1));
    d.dG.resize((size_t)d.Q * (pg + 1));
    for (int e = 0; e < d.nel; ++e) {
        double a = b[e], c = b[e + 1];
        // span of element e in the space knots: last k with t[k] == a
        int k = find_span(tl, p, 0.5 * (a + c));
        for (int g = 0; g <= p; ++g) {
            int q = e * (p + 1) + g;
            double x = a + (c - a) * gx[g];
            d.xi[q] = x;
            d.w[q] = (c - a) * gw[g];
            d.first[q] = k - p;
            basis_on_span(tl, p, k, x, &d.N[(size_t)q * (p + 1)], &d.dN[(size_t)q * (p + 1)]);
            int kg = find_span(tg, pg, x);
            d.gfirst[q] = kg - pg;
            basis_on_span(tg, pg, kg, x, &d.G[(size_t)q * (pg + 1)], &d.dG[(size_t)q * (pg + 1)]);
        }
    }
    return d;
}

// 1D Galerkin matrices between the level's functions: A[u][v](i,j) = sum_q w X_u(i) X_v(j),
// X_0 = value, X_1 = derivative.  Dense M x M.
static void one_d_matrices(const DirTable& d, int M, std::vector<double> A[2][2]) {
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) A[u][v].assign((size_t)M * M, 0.0);
    int p = d.p;
    for (int q = 0; q < d.Q; ++q) {
        const double* N = &d.N[(size_t)q * (p + 1)];
        const double* dN = &d.dN[(size_t)q * (p + 1)];
        for (int a = 0; a <= p; ++a)
            for (int b = 0; b <= p; ++b) {
                int i = d.first[q] + a, j = d.first[q] + b;
                double X[2] = {N[a], dN[a]}, Y[2] = {N[b], dN[b]};
                for (int u = 0; u < 2; ++u)
                    for (int v = 0; v < 2; ++v) A[u][v][(size_t)i * M + j] += d.w[q] * X[u] * Y[v];
            }
    }
}

// half-stencil offsets: diagonal first; then o2 = 0, o1 = 0, o0 > 0; o2 = 0, o1 > 0; o2 > 0
static void half_offsets(int dim, const int* p, std::vector<int32_t>& offs) {
    offs.clear();
    int p2 = dim == 3 ? p[2] : 0;
    for (int o2 = 0; o2 <= p2; ++o2)
        for (int o1 = (o2 == 0 ? 0 : -p[1]); o1 <= p[1]; ++o1)
            for (int o0 = (o2 == 0 && o1 == 0 ? 0 : -p[0]); o0 <= p[0]; ++o0) {
                offs.push_back(o0);
                offs.push_back(o1);
                offs.push_back(o2);
            }
}

static inline int64_t lin(const int* M, int i0, int i1, int i2) { return i0 + (int64_t)M[0] * (i1 + (int64_t)M[1] * i2); }

// Assemble the half stencil of level `L` of patch `P` (space = L.knots, geometry = patch level 0).
// On level 0 also the quadrature weights w |det J| and the physical points.
static void assemble_level(Patch& P, Level& L, bool level0) {
    const int dim = P.dim;
    DirTable dt[3];
    for (int d = 0; d < dim; ++d) dt[d] = make_dir(L.knots[d], L.p[d], P.knots[d], P.p[d]);
    int Mg[3] = {1, 1, 1};
    for (int d = 0; d < dim; ++d) Mg[d] = (int)P.knots[d].size() - P.p[d] - 1;
    half_offsets(dim, L.p, L.offs);
    L.nst = (int)L.offs.size() / 3;
    L.coef.assign((size_t)L.nst * L.n, 0.0);
    // slot table: (o0+p0) + (2p0+1)((o1+p1) + (2p1+1)(o2+p2)) -> s
    int w0 = 2 * L.p[0] + 1, w1 = 2 * L.p[1] + 1, w2 = dim == 3 ? 2 * L.p[2] + 1 : 1;
    int p2 = dim == 3 ? L.p[2] : 0;
    std::vector<int> slot((size_t)w0 * w1 * w2, -1);
    for (int s = 0; s < L.nst; ++s) {
        int o0 = L.offs[3 * s], o1 = L.offs[3 * s + 1], o2 = L.offs[3 * s + 2];
        slot[(o0 + L.p[0]) + (size_t)w0 * ((o1 + L.p[1]) + (size_t)w1 * (o2 + p2))] = s;
    }
    const int Q0 = dt[0].Q, Q1 = dt[1].Q, Q2 = dim == 3 ? dt[2].Q : 1;
    if (level0) {
        for (int d = 0; d < dim; ++d) P.qpN[d] = dt[d].N;
        P.n_qp = (int64_t)Q0 * Q1 * Q2;
        P.qpw.assign(P.n_qp, 0.0);
        P.qpx.assign(P.n_qp * dim, 0.0);
        for (int d = 0; d < dim; ++d) P.qpc[d].assign(P.n_qp, 0.0);
    }
    if (P.affine) {
        // constant Jacobian A: columns = ctrl(corner e_d) - ctrl(corner 0)
        double A[3][3] = {{0}}, c0[3] = {0};
        for (int c = 0; c < dim; ++c) c0[c] = P.ctrl[c];
        for (int d = 0; d < dim; ++d) {
            int idx[3] = {0, 0, 0};
            idx[d] = Mg[d] - 1;
            int64_t k = lin(Mg, idx[0], idx[1], idx[2]);
            for (int c = 0; c < dim; ++c) A[c][d] = P.ctrl[k * dim + c] - c0[c];
        }
        double det, Ai[3][3];
        if (dim == 2) {
            det = A[0][0] * A[1][1] - A[0][1] * A[1][0];
            Ai[0][0] = A[1][1] / det; Ai[0][1] = -A[0][1] / det;
            Ai[1][0] = -A[1][0] / det; Ai[1][1] = A[0][0] / det;
        } else {
            det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                  A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    int i1 = (j + 1) % 3, i2 = (j + 2) % 3, j1 = (i + 1) % 3, j2 = (i + 2) % 3;
                    Ai[i][j] = (A[i1][j1] * A[i2][j2] - A[i1][j2] * A[i2][j1]) / det;
                }
        }
        if (!(det > 0)) throw Error(IETI_EGEOM, "geometry map is not orientation preserving");
        double Gh[3][3];
        for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b) {
                double s = 0;
                for (int c = 0; c < dim; ++c) s += Ai[a][c] * Ai[b][c];
                Gh[a][b] = det * s;
            }
        std::vector<double> A1[3][2][2];
        for (int d = 0; d < dim; ++d) one_d_matrices(dt[d], L.M[d], A1[d]);
        for (int i2 = 0; i2 < L.M[2]; ++i2)
            for (int i1 = 0; i1 < L.M[1]; ++i1)
                for (int i0 = 0; i0 < L.M[0]; ++i0) {
                    int64_t i = lin(L.M, i0, i1, i2);
                    int ii[3] = {i0, i1, i2};
                    for (int s = 0; s < L.nst; ++s) {
                        int o[3] = {L.offs[3 * s], L.offs[3 * s + 1], L.offs[3 * s + 2]};
                        int jj[3];
                        bool ok = true;
                        for (int d = 0; d < dim; ++d) {
                            jj[d] = ii[d] + o[d];
                            if (jj[d] < 0 || jj[d] >= L.M[d]) ok = false;
                        }
                        if (!ok) continue;
                        double v = 0.0;
                        for (int a = 0; a < dim; ++a)
                            for (int b = 0; b < dim; ++b) {
                                double prod = Gh[a][b];
                                for (int d = 0; d < dim; ++d)
                                    prod *= A1[d][d == a ? 1 : 0][d == b ? 1 : 0][(size_t)ii[d] * L.M[d] + jj[d]];
                                v += prod;
                            }
                        L.coef[(size_t)s * L.n + i] = v;
                    }
                }
        if (level0) {
            for (int q2 = 0; q2 < Q2; ++q2)
                for (int q1 = 0; q1 < Q1; ++q1)
                    for (int q0 = 0; q0 < Q0; ++q0) {
                        int64_t q = q0 + (int64_t)Q0 * (q1 + (int64_t)Q1 * q2);
                        double wq = dt[0].w[q0] * dt[1].w[q1] * (dim == 3 ? dt[2].w[q2] : 1.0);
                        P.qpw[q] = wq * det;
                        for (int d = 0; d < dim; ++d) P.qpc[d][q] = Gh[d][d];
                        double xi[3] = {dt[0].xi[q0], dt[1].xi[q1], dim == 3 ? dt[2].xi[q2] : 0.0};
                        for (int c = 0; c < dim; ++c) {
                            double x = c0[c];
                            for (int d = 0; d < dim; ++d) x += A[c][d] * xi[d];
                            P.qpx[q * dim + c] = x;
                        }
                    }
        }
        return;
    }

    // ---- curved patch: element-by-element with the metric at every quadrature point
    const int pl[3] = {L.p[0], L.p[1], dim == 3 ? L.p[2] : 0};
    const int nq1[3] = {pl[0] + 1, pl[1] + 1, pl[2] + 1};
    const int nloc = nq1[0] * nq1[1] * nq1[2];
    const int nqe = nloc;   // (p+1)^d points per element
    const int pg[3] = {P.p[0], P.p[1], dim == 3 ? P.p[2] : 0};
    std::vector<double> grad((size_t)nloc * nqe * 3), h((size_t)nloc * nqe * 3), Ke((size_t)nloc * nloc);
    const int ne[3] = {dt[0].nel, dt[1].nel, dim == 3 ? dt[2].nel : 1};
    for (int e2 = 0; e2 < ne[2]; ++e2)
        for (int e1 = 0; e1 < ne[1]; ++e1)
            for (int e0 = 0; e0 < ne[0]; ++e0) {
                int first[3];
                // qp loop
                for (int g2 = 0; g2 < nq1[2]; ++g2)
                    for (int g1 = 0; g1 < nq1[1]; ++g1)
                        for (int g0 = 0; g0 < nq1[0]; ++g0) {
                            int qd[3] = {e0 * nq1[0] + g0, e1 * nq1[1] + g1, e2 * nq1[2] + g2};
                            int ql = g0 + nq1[0] * (g1 + nq1[1] * g2);
                            for (int d = 0; d < dim; ++d) first[d] = dt[d].first[qd[d]];
                            if (dim == 2) first[2] = 0;
                            // geometry: x and J
                            double x[3] = {0, 0, 0}, J[3][3] = {{0}};
                            const double* Gv[3];
                            const double* Gd[3];
                            int gf[3] = {0, 0, 0};
                            for (int d = 0; d < dim; ++d) {
                                Gv[d] = &dt[d].G[(size_t)qd[d] * (pg[d] + 1)];
                                Gd[d] = &dt[d].dG[(size_t)qd[d] * (pg[d] + 1)];
                                gf[d] = dt[d].gfirst[qd[d]];
                            }
                            for (int a2 = 0; a2 <= pg[2]; ++a2)
                                for (int a1 = 0; a1 <= pg[1]; ++a1)
                                    for (int a0 = 0; a0 <= pg[0]; ++a0) {
                                        int64_t k = lin(Mg, gf[0] + a0, gf[1] + a1, dim == 3 ? gf[2] + a2 : 0);
                                        double v0 = Gv[0][a0], v1 = Gv[1][a1], v2 = dim == 3 ? Gv[2][a2] : 1.0;
                                        double d0 = Gd[0][a0], d1 = Gd[1][a1], d2 = dim == 3 ? Gd[2][a2] : 0.0;
                                        double bv = v0 * v1 * v2;
                                        double bd[3] = {d0 * v1 * v2, v0 * d1 * v2, v0 * v1 * d2};
                                        for (int c = 0; c < dim; ++c) {
                                            double cp = P.ctrl[k * dim + c];
                                            x[c] += cp * bv;
                                            for (int a = 0; a < dim; ++a) J[c][a] += cp * bd[a];
                                        }
                                    }
                            double det, Ji[3][3];
                            if (dim == 2) {
                                det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
                                Ji[0][0] = J[1][1] / det; Ji[0][1] = -J[0][1] / det;
                                Ji[1][0] = -J[1][0] / det; Ji[1][1] = J[0][0] / det;
                            } else {
                                det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                      J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                      J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                                for (int i = 0; i < 3; ++i)
                                    for (int j = 0; j < 3; ++j) {
                                        int i1 = (j + 1) % 3, i2 = (j + 2) % 3, j1 = (i + 1) % 3, j2 = (i + 2) % 3;
                                        Ji[i][j] = (J[i1][j1] * J[i2][j2] - J[i1][j2] * J[i2][j1]) / det;
                                    }
                            }
                            if (!(det > 0)) throw Error(IETI_EGEOM, "geometry map is not orientation preserving");
                            double wq = dt[0].w[qd[0]] * dt[1].w[qd[1]] * (dim == 3 ? dt[2].w[qd[2]] : 1.0);
                            double Gm[3][3];
                            for (int a = 0; a < dim; ++a)
                                for (int b = 0; b < dim; ++b) {
                                    double s = 0;
                                    for (int c = 0; c < dim; ++c) s += Ji[a][c] * Ji[b][c];
                                    Gm[a][b] = wq * det * s;
                                }
                            if (level0) {
                                int64_t q = qd[0] + (int64_t)Q0 * (qd[1] + (int64_t)Q1 * (dim == 3 ? qd[2] : 0));
                                P.qpw[q] = wq * det;
                                for (int c = 0; c < dim; ++c) P.qpx[q * dim + c] = x[c];
                                for (int d = 0; d < dim; ++d) P.qpc[d][q] = Gm[d][d] / wq;
                            }
                            // space basis gradients (parameter domain) and G * grad
                            const double* Nv[3];
                            const double* Nd[3];
                            for (int d = 0; d < dim; ++d) {
                                Nv[d] = &dt[d].N[(size_t)qd[d] * (pl[d] + 1)];
                                Nd[d] = &dt[d].dN[(size_t)qd[d] * (pl[d] + 1)];
                            }
                            for (int a2 = 0; a2 < nq1[2]; ++a2)
                                for (int a1 = 0; a1 < nq1[1]; ++a1)
                                    for (int a0 = 0; a0 < nq1[0]; ++a0) {
                                        int al = a0 + nq1[0] * (a1 + nq1[1] * a2);
                                        double v0 = Nv[0][a0], v1 = Nv[1][a1], v2 = dim == 3 ? Nv[2][a2] : 1.0;
                                        double d0 = Nd[0][a0], d1 = Nd[1][a1], d2 = dim == 3 ? Nd[2][a2] : 0.0;
                                        double gr[3] = {d0 * v1 * v2, v0 * d1 * v2, v0 * v1 * d2};
                                        double* gp = &grad[((size_t)al * nqe + ql) * 3];
                                        double* hp = &h[((size_t)al * nqe + ql) * 3];
                                        for (int c = 0; c < 3; ++c) gp[c] = c < dim ? gr[c] : 0.0;
                                        for (int a = 0; a < 3; ++a) {
                                            double s = 0;
                                            for (int b = 0; b < dim; ++b) s += (a < dim ? Gm[a][b] : 0.0) * gr[b];
                                            hp[a] = a < dim ? s : 0.0;
                                        }
                                    }
                        }
                // element matrix and scatter into the half stencil
                for (int d = 0; d < dim; ++d) first[d] = dt[d].first[e0 * 0 + (d == 0 ? e0 : d == 1 ? e1 : e2) * nq1[d]];
                if (dim == 2) first[2] = 0;
                for (int al = 0; al < nloc; ++al) {
                    int a0 = al % nq1[0], a1 = (al / nq1[0]) % nq1[1], a2 = al / (nq1[0] * nq1[1]);
                    const double* hp = &h[(size_t)al * nqe * 3];
                    for (int bl = 0; bl < nloc; ++bl) {
                        int b0 = bl % nq1[0], b1 = (bl / nq1[0]) % nq1[1], b2 = bl / (nq1[0] * nq1[1]);
                        int o0 = b0 - a0, o1 = b1 - a1, o2 = b2 - a2;
                        int s = slot[(o0 + L.p[0]) + (size_t)w0 * ((o1 + L.p[1]) + (size_t)w1 * (o2 + p2))];
                        if (s < 0) continue;
                        const double* gp = &grad[(size_t)bl * nqe * 3];
                        double v = 0.0;
                        for (int t = 0; t < nqe * 3; ++t) v += hp[t] * gp[t];
                        int64_t i = lin(L.M, first[0] + a0, first[1] + a1, first[2] + a2);
                        L.coef[(size_t)s * L.n + i] += v;
                    }
                }
            }
}

// coef += alpha M^ on level L, M^ the mass matrix of the level's spline space on the parameter domain
// (0,1)^d: the tensor product of the 1D parametric mass matrices (Gauss quadrature in parameter space).
static void add_param_mass(const Patch& P, Level& L, double alpha) {
    const int dim = P.dim;
    std::vector<double> A1[3][2][2];
    for (int d = 0; d < dim; ++d) one_d_matrices(make_dir(L.knots[d], L.p[d], P.knots[d], P.p[d]), L.M[d], A1[d]);
    for (int i2 = 0; i2 < L.M[2]; ++i2)
        for (int i1 = 0; i1 < L.M[1]; ++i1)
            for (int i0 = 0; i0 < L.M[0]; ++i0) {
                const int ii[3] = {i0, i1, i2};
                const int64_t i = lin(L.M, i0, i1, i2);
                for (int s = 0; s < L.nst; ++s) {
                    double v = alpha;
                    for (int d = 0; d < dim && v != 0.0; ++d) {
                        const int j = ii[d] + L.offs[3 * s + d];
                        v = (j < 0 || j >= L.M[d]) ? 0.0 : v * A1[d][0][0][(size_t)ii[d] * L.M[d] + j];
                    }
                    L.coef[(size_t)s * L.n + i] += v;
                }
            }
}

// y = m (K m x) with the half stencil, FP64, on the host.
// sum_k a[k] b[k] in four interleaved partial sums (independent multiply-add chains)
static inline double dot4(const double* a, const double* b, int64_t m) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t k = 0;
    for (; k + 4 <= m; k += 4) {
        s0 += a[k] * b[k];
        s1 += a[k + 1] * b[k + 1];
        s2 += a[k + 2] * b[k + 2];
        s3 += a[k + 3] * b[k + 3];
    }
    for (; k < m; ++k) s0 += a[k] * b[k];
    return (s0 + s1) + (s2 + s3);
}

static void host_apply(const Patch& P, const Level& L, const std::vector<uint8_t>& mask, const double* x, double* y) {
    std::fill(y, y + L.n, 0.0);
    for (int i2 = 0; i2 < L.M[2]; ++i2)
        for (int i1 = 0; i1 < L.M[1]; ++i1)
            for (int i0 = 0; i0 < L.M[0]; ++i0) {
                int64_t i = lin(L.M, i0, i1, i2);
                if (mask[i]) continue;
                for (int s = 0; s < L.nst; ++s) {
                    int j0 = i0 + L.offs[3 * s], j1 = i1 + L.offs[3 * s + 1], j2 = i2 + L.offs[3 * s + 2];
                    if (j0 < 0 || j0 >= L.M[0] || j1 < 0 || j1 >= L.M[1] || j2 < 0 || j2 >= L.M[2]) continue;
                    int64_t j = lin(L.M, j0, j1, j2);
                    if (mask[j]) continue;
                    double c = L.coef[(size_t)s * L.n + i];
                    y[i] += c * x[j];
                    if (s) y[j] += c * x[i];
                }
            }
}

// mask[i] = 1 where coefficient i is held at zero in the given mode
static std::vector<uint8_t> level_mask(const Patch& P, const Level& L, int mode) {
    uint32_t sides = mode == MODE_D ? (P.dim == 3 ? 0x3Fu : 0xFu) : P.bside;
    uint32_t corners = mode == MODE_N ? (P.pcorner | P.dcorner) : mode == MODE_K ? P.dcorner : 0u;
    std::vector<uint8_t> m(L.n, 0);
    for (int i2 = 0; i2 < L.M[2]; ++i2)
        for (int i1 = 0; i1 < L.M[1]; ++i1)
            for (int i0 = 0; i0 < L.M[0]; ++i0) {
                int ii[3] = {i0, i1, i2};
                bool msk = false;
                int cbits = 0, nend = 0;
                for (int d = 0; d < P.dim; ++d) {
                    bool lo = ii[d] == 0, hi = ii[d] == L.M[d] - 1;
                    if ((lo && (sides >> (2 * d) & 1)) || (hi && (sides >> (2 * d + 1) & 1))) msk = true;
                    if (lo || hi) { ++nend; if (hi) cbits |= 1 << d; }
                }
                if (nend == P.dim && (corners >> cbits & 1)) msk = true;
                m[lin(L.M, i0, i1, i2)] = msk;
            }
    return m;
}

// lambda_max of D^{-1} K (masked) by power iteration
static double power_lmax(const Patch& P, const Level& L, int mode) {
    auto mask = level_mask(P, L, mode);
    std::vector<double> x(L.n), y(L.n);
    uint64_t s = 0x9E3779B97F4A7C15ull;
    for (int64_t i = 0; i < L.n; ++i) {
        s ^= s << 13; s ^= s >> 7; s ^= s << 17;
        x[i] = mask[i] ? 0.0 : ((s >> 11) * (1.0 / 9007199254740992.0) - 0.5);
    }
    double lam = 0.0;
    for (int it = 0; it < 40; ++it) {
        host_apply(P, L, mask, x.data(), y.data());
        double nx = 0, ny = 0;
        for (int64_t i = 0; i < L.n; ++i) {
            if (mask[i]) { y[i] = 0; continue; }
            y[i] /= L.coef[i];
            nx += x[i] * x[i];
            ny += y[i] * y[i];
        }
        if (ny == 0 || nx == 0) return 1.0;
        lam = std::sqrt(ny / nx);
        double sc = 1.0 / std::sqrt(ny);
        for (int64_t i = 0; i < L.n; ++i) x[i] = y[i] * sc;
    }
    return lam;
}

// ----------------------------------------------------------------------------
// tensor-product smoother of the finest level (2D)

// Best rank-one approximation g ~ a b^T of a positive Q0 x Q1 array g[q0 + Q0 q1]: the leading singular
// pair by alternating power steps.
static void rank_one(const std::vector<double>& g, int Q0, int Q1, std::vector<double>& a, std::vector<double>& b) {
    a.assign(Q0, 0.0);
    b.assign(Q1, 1.0);
    std::vector<double> nb(Q1);
    for (int it = 0; it < 200; ++it) {
        double bb = 0.0;
        for (double v : b) bb += v * v;
        for (int i = 0; i < Q0; ++i) {
            double t = 0.0;
            for (int j = 0; j < Q1; ++j) t += g[i + (size_t)Q0 * j] * b[j];
            a[i] = t / bb;
        }
        double aa = 0.0;
        for (double v : a) aa += v * v;
        double diff = 0.0, mx = 0.0;
        for (int j = 0; j < Q1; ++j) {
            double t = 0.0;
            for (int i = 0; i < Q0; ++i) t += g[i + (size_t)Q0 * j] * a[i];
            nb[j] = t / aa;
            diff = std::max(diff, std::fabs(nb[j] - b[j]));
            mx = std::max(mx, std::fabs(nb[j]));
        }
        b.swap(nb);
        if (diff <= 1e-15 * mx) break;
    }
}

// Symmetric eigenproblem A = Z diag(w) Z^T (A row-major n x n, destroyed; Z row-major, eigenvectors by
// columns): Householder reduction to tridiagonal form, then implicit QL sweeps with the shift from the
// leading 2 x 2 block; both accumulate their orthogonal transformations into Z.  The QL sweep is the
// published implicit QL algorithm with Wilkinson-type shifts of Bowdler, Martin, Reinsch and Wilkinson
// (Numer. Math. 11, 1968; the EISPACK routine tql2), restated here step by step.
static void sym_eig(int n, std::vector<double>& A, std::vector<double>& w, std::vector<double>& Z) {
    Z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    std::vector<double> v(n, 0.0), pv(n, 0.0), qv(n, 0.0);
    for (int k = 0; k + 2 < n; ++k) {
        double alpha = 0.0;
        for (int i = k + 1; i < n; ++i) alpha += A[(size_t)i * n + k] * A[(size_t)i * n + k];
        alpha = std::sqrt(alpha);
        if (alpha == 0.0) continue;
        const double sg = A[(size_t)(k + 1) * n + k] >= 0.0 ? 1.0 : -1.0;
        for (int i = k + 1; i < n; ++i) v[i] = A[(size_t)i * n + k];
        v[k + 1] += sg * alpha;
        double vn = 0.0;
        for (int i = k + 1; i < n; ++i) vn += v[i] * v[i];
        vn = std::sqrt(vn);
        for (int i = k + 1; i < n; ++i) v[i] /= vn;
        // H = I - 2 v v^T maps column k below the diagonal to -sg alpha e_{k+1}
        for (int i = k + 1; i < n; ++i) A[(size_t)i * n + k] = A[(size_t)k * n + i] = 0.0;
        A[(size_t)(k + 1) * n + k] = A[(size_t)k * n + k + 1] = -sg * alpha;
        // trailing block: A <- H A H = A - v q^T - q v^T, q = 2 (A v - (v^T A v) v)
        double K = 0.0;
        for (int i = k + 1; i < n; ++i) {
            double t = 0.0;
            for (int j = k + 1; j < n; ++j) t += A[(size_t)i * n + j] * v[j];
            pv[i] = t;
            K += v[i] * t;
        }
        for (int i = k + 1; i < n; ++i) qv[i] = 2.0 * (pv[i] - K * v[i]);
        for (int i = k + 1; i < n; ++i)
            for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= v[i] * qv[j] + qv[i] * v[j];
        // Z <- Z H
        for (int r = 0; r < n; ++r) {
            double t = 0.0;
            for (int j = k + 1; j < n; ++j) t += Z[(size_t)r * n + j] * v[j];
            for (int j = k + 1; j < n; ++j) Z[(size_t)r * n + j] -= 2.0 * t * v[j];
        }
    }
    std::vector<double> d(n), e(n, 0.0);
    for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
    for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];   // e[i] couples d[i] and d[i+1]
    for (int l = 0; l < n; ++l) {
        for (int iter = 0;; ++iter) {
            int m = l;
            for (; m + 1 < n; ++m)
                if (std::fabs(e[m]) <= 1e-16 * (std::fabs(d[m]) + std::fabs(d[m + 1]))) break;
            if (m == l) break;
            if (iter > 100) throw Error(IETI_EINVAL, "tensor smoother: eigenvalue iteration did not converge");
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
            double sn = 1.0, cs = 1.0, pp = 0.0;
            bool split = false;
            for (int i = m - 1; i >= l; --i) {
                const double f = sn * e[i], b = cs * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {   // the rotation decouples the matrix: restart on the smaller block
                    d[i + 1] -= pp;
                    e[m] = 0.0;
                    split = true;
                    break;
                }
                sn = f / r;
                cs = g / r;
                g = d[i + 1] - pp;
                r = (d[i] - g) * sn + 2.0 * cs * b;
                pp = sn * r;
                d[i + 1] = g + pp;
                g = cs * r - b;
                for (int k = 0; k < n; ++k) {
                    const double z1 = Z[(size_t)k * n + i + 1], z0 = Z[(size_t)k * n + i];
                    Z[(size_t)k * n + i + 1] = sn * z0 + cs * z1;
                    Z[(size_t)k * n + i] = cs * z0 - sn * z1;
                }
            }
            if (split) continue;
            d[l] -= pp;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    w = d;
}

// Generalised eigenproblem A U = B U diag(lam), U^T B U = I (A symmetric, B SPD, n x n row-major):
// B = L L^T, C = L^{-1} A L^{-T} = Z diag(lam) Z^T, U = L^{-T} Z.
static void gen_eig(int n, const std::vector<double>& A, const std::vector<double>& B, std::vector<double>& U,
                    std::vector<double>& lam) {
    std::vector<double> L((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double dd = B[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) dd -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(dd > 0.0)) throw Error(IETI_EINVAL, "tensor smoother: 1D mass matrix not positive definite");
        const double ljj = std::sqrt(dd);
        L[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double t = B[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = t / ljj;
        }
    }
    // X = L^{-1} A (column by column), C = L^{-1} X^T
    std::vector<double> X((size_t)n * n), C((size_t)n * n);
    auto fwd = [&](const double* rhs, int stride, double* out) {   // out = L^{-1} rhs (rhs entries at stride)
        for (int i = 0; i < n; ++i) {
            double t = rhs[(size_t)i * stride];
            for (int k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * out[k];
            out[i] = t / L[(size_t)i * n + i];
        }
    };
    std::vector<double> col(n);
    for (int j = 0; j < n; ++j) {
        fwd(&A[j], n, col.data());
        for (int i = 0; i < n; ++i) X[(size_t)i * n + j] = col[i];
    }
    for (int j = 0; j < n; ++j) {
        fwd(&X[(size_t)j * n], 1, col.data());   // column j of X^T is row j of X
        for (int i = 0; i < n; ++i) C[(size_t)i * n + j] = col[i];
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) C[(size_t)i * n + j] = C[(size_t)j * n + i] = 0.5 * (C[(size_t)i * n + j] + C[(size_t)j * n + i]);
    std::vector<double> Z;
    sym_eig(n, C, lam, Z);
    // U = L^{-T} Z
    U.assign((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j)
        for (int i = n - 1; i >= 0; --i) {
            double t = Z[(size_t)i * n + j];
            for (int k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * U[(size_t)k * n + j];
            U[(size_t)i * n + j] = t / L[(size_t)i * n + i];
        }
}

// y = m U (Lambda_0 (+) Lambda_1 + c)^{-1} U^T m r on one patch (host, for the damping estimate)
static void tensor_apply_host(const Patch::Tensor& T, int M0, int M1, const std::vector<uint8_t>& mask,
                              const double* r, double* y) {
    const int P0 = T.Pd[0], P1 = T.Pd[1];
    std::vector<double> W((size_t)M1 * P0, 0.0), Z((size_t)P1 * P0, 0.0), V((size_t)M1 * P0, 0.0);
    for (int i1 = 0; i1 < M1; ++i1)
        for (int i0 = 0; i0 < M0; ++i0) {
            const size_t i = (size_t)i0 + (size_t)M0 * i1;
            if (mask[i]) continue;
            const double x = r[i];
            for (int a = 0; a < P0; ++a) W[(size_t)i1 * P0 + a] += x * T.U[0][(size_t)i0 * P0 + a];
        }
    for (int b = 0; b < P1; ++b)
        for (int a = 0; a < P0; ++a) {
            double t = 0.0;
            for (int i1 = 0; i1 < M1; ++i1) t += T.U[1][(size_t)i1 * P1 + b] * W[(size_t)i1 * P0 + a];
            Z[(size_t)b * P0 + a] = t / (T.lam[0][a] + T.lam[1][b] + T.shift);
        }
    for (int i1 = 0; i1 < M1; ++i1)
        for (int a = 0; a < P0; ++a) {
            double t = 0.0;
            for (int b = 0; b < P1; ++b) t += T.U[1][(size_t)i1 * P1 + b] * Z[(size_t)b * P0 + a];
            V[(size_t)i1 * P0 + a] = t;
        }
    for (int i1 = 0; i1 < M1; ++i1)
        for (int i0 = 0; i0 < M0; ++i0) {
            const size_t i = (size_t)i0 + (size_t)M0 * i1;
            double t = 0.0;
            if (!mask[i])
                for (int a = 0; a < P0; ++a) t += V[(size_t)i1 * P0 + a] * T.U[0][(size_t)i0 * P0 + a];
            y[i] = t;
        }
}

// Finest-level tensor smoother of a 2D patch for the Neumann (if mode_n) and Dirichlet modes: rank-one
// fits g_00 ~ a00 (x) b00 and g_11 ~ a11 (x) b11 of the metric diagonals on the quadrature grid (the mass
// weights b00 and a11 scaled to unit mean), 1D matrices A_0 = (a00 u', v'), B_0 = (a11 u, v),
// A_1 = (b11 u', v'), B_1 = (b00 u, v), so that K_sep = A_0 (x) B_1 + B_0 (x) A_1, and per mode the
// generalised eigenvectors on the coefficients the mode keeps (its masked sides removed per direction;
// masked corners stay in the tensor space and are cut by the mask).
static void tensor_setup(Patch& P, const ieti_options& opt, bool mode_n) {
    const Level& L0 = P.lv[0];
    DirTable dt[2];
    for (int d = 0; d < 2; ++d) dt[d] = make_dir(L0.knots[d], P.p[d], P.knots[d], P.p[d]);
    const int Q0 = dt[0].Q, Q1 = dt[1].Q;
    std::vector<double> a00, b00, a11, b11;
    rank_one(P.qpc[0], Q0, Q1, a00, b00);
    rank_one(P.qpc[1], Q0, Q1, a11, b11);
    double m1 = 0.0, m0 = 0.0;
    for (int q = 0; q < Q1; ++q) m1 += dt[1].w[q] * b00[q];
    for (int q = 0; q < Q0; ++q) m0 += dt[0].w[q] * a11[q];
    for (auto& v : b00) v /= m1;
    for (auto& v : a00) v *= m1;
    for (auto& v : a11) v /= m0;
    for (auto& v : b11) v *= m0;
    auto weighted = [](const DirTable& t, int M, const std::vector<double>& ws, const std::vector<double>& wm,
                       std::vector<double>& A, std::vector<double>& B) {
        A.assign((size_t)M * M, 0.0);
        B.assign((size_t)M * M, 0.0);
        const int p = t.p;
        for (int q = 0; q < t.Q; ++q)
            for (int a = 0; a <= p; ++a)
                for (int b = 0; b <= p; ++b) {
                    const int i = t.first[q] + a, j = t.first[q] + b;
                    const size_t o = (size_t)q * (p + 1);
                    A[(size_t)i * M + j] += t.w[q] * ws[q] * t.dN[o + a] * t.dN[o + b];
                    B[(size_t)i * M + j] += t.w[q] * wm[q] * t.N[o + a] * t.N[o + b];
                }
    };
    std::vector<double> A1d[2], B1d[2];
    weighted(dt[0], L0.M[0], a00, a11, A1d[0], B1d[0]);
    weighted(dt[1], L0.M[1], b11, b00, A1d[1], B1d[1]);
    const double shift = opt.smoother_sigma * 0.5 * ((double)L0.nel[0] * L0.nel[0] + (double)L0.nel[1] * L0.nel[1]);
    for (int mode = 0; mode < 2; ++mode) {
        if (mode == MODE_N && !mode_n) continue;
        Patch::Tensor& T = P.ts[mode];
        const uint32_t sides = mode == MODE_D ? 0xFu : P.bside;
        for (int d = 0; d < 2; ++d) {
            const int M = L0.M[d];
            std::vector<int> keep;
            for (int i = 0; i < M; ++i) {
                const bool cut = (i == 0 && (sides >> (2 * d) & 1u)) || (i == M - 1 && (sides >> (2 * d + 1) & 1u));
                if (!cut) keep.push_back(i);
            }
            const int nk = (int)keep.size();
            std::vector<double> Ak((size_t)nk * nk), Bk((size_t)nk * nk), Uk, lk;
            for (int i = 0; i < nk; ++i)
                for (int j = 0; j < nk; ++j) {
                    Ak[(size_t)i * nk + j] = A1d[d][(size_t)keep[i] * M + keep[j]];
                    Bk[(size_t)i * nk + j] = B1d[d][(size_t)keep[i] * M + keep[j]];
                }
            gen_eig(nk, Ak, Bk, Uk, lk);
            const int Pd = (M + 15) / 16 * 16;
            T.Pd[d] = Pd;
            T.U[d].assign((size_t)Pd * Pd, 0.0);
            T.lam[d].assign(Pd, 1e300);
            for (int i = 0; i < nk; ++i)
                for (int a = 0; a < nk; ++a) T.U[d][(size_t)keep[i] * Pd + a] = Uk[(size_t)i * nk + a];
            for (int a = 0; a < nk; ++a) T.lam[d][a] = lk[a];
        }
        T.shift = shift;
        // tau = 1 / lambda_max(m S^{-1} m K) by power steps
        auto mask = level_mask(P, L0, mode);
        std::vector<double> x(L0.n), y(L0.n), z(L0.n);
        uint64_t sd = 0xBF58476D1CE4E5B9ull;
        for (int64_t i = 0; i < L0.n; ++i) {
            sd ^= sd << 13; sd ^= sd >> 7; sd ^= sd << 17;
            x[i] = mask[i] ? 0.0 : ((sd >> 11) * (1.0 / 9007199254740992.0) - 0.5);
        }
        double lam = 1.0;
        for (int it = 0; it < 20; ++it) {
            host_apply(P, L0, mask, x.data(), y.data());
            tensor_apply_host(T, L0.M[0], L0.M[1], mask, y.data(), z.data());
            double nx = 0.0, nz = 0.0;
            for (int64_t i = 0; i < L0.n; ++i) {
                nx += x[i] * x[i];
                nz += z[i] * z[i];
            }
            if (!(nz > 0.0) || !(nx > 0.0)) break;
            lam = std::sqrt(nz / nx);
            const double sc = 1.0 / std::sqrt(nz);
            for (int64_t i = 0; i < L0.n; ++i) x[i] = z[i] * sc;
        }
        T.tau = 1.0 / lam;
    }
}

// Best rank-one approximation g ~ x0 (x) x1 (x) x2 of a positive Q0 x Q1 x Q2 array g[q0 + Q0 (q1 + Q1 q2)]
// by alternating power steps (higher-order power method).
static void rank_one3(const std::vector<double>& g, const int* Q, std::vector<double> (&x)[3]) {
    for (int d = 0; d < 3; ++d) x[d].assign(Q[d], 1.0);
    for (int it = 0; it < 200; ++it) {
        double change = 0.0;
        for (int d = 0; d < 3; ++d) {
            const int e = (d + 1) % 3, f = (d + 2) % 3;
            double ne = 0.0, nf = 0.0;
            for (double v : x[e]) ne += v * v;
            for (double v : x[f]) nf += v * v;
            std::vector<double> nx(Q[d], 0.0);
            for (int q2 = 0; q2 < Q[2]; ++q2)
                for (int q1 = 0; q1 < Q[1]; ++q1)
                    for (int q0 = 0; q0 < Q[0]; ++q0) {
                        const int qq[3] = {q0, q1, q2};
                        nx[qq[d]] += g[q0 + (size_t)Q[0] * (q1 + (size_t)Q[1] * q2)] * x[e][qq[e]] * x[f][qq[f]];
                    }
            double mx = 0.0;
            for (int i = 0; i < Q[d]; ++i) {
                nx[i] /= ne * nf;
                change = std::max(change, std::fabs(nx[i] - x[d][i]));
                mx = std::max(mx, std::fabs(nx[i]));
            }
            x[d].swap(nx);
            change /= mx;
        }
        if (change <= 1e-15) break;
    }
}

// y = m (U_2 (x) U_1 (x) U_0) (Lambda_0 (+) Lambda_1 (+) Lambda_2 + c)^{-1} (...)^T m r on one 3D patch (host)
static void tensor_apply_host3(const Patch::Tensor& T, const int* M, const std::vector<uint8_t>& mask, const double* r,
                               double* y) {
    const int P0 = T.Pd[0], P1 = T.Pd[1], P2 = T.Pd[2];
    // forward: contract i0, then i1, then i2
    std::vector<double> A((size_t)P0 * M[1] * M[2], 0.0), B((size_t)P0 * P1 * M[2], 0.0), Z((size_t)P0 * P1 * P2, 0.0);
    for (int i2 = 0; i2 < M[2]; ++i2)
        for (int i1 = 0; i1 < M[1]; ++i1)
            for (int i0 = 0; i0 < M[0]; ++i0) {
                const size_t i = i0 + (size_t)M[0] * (i1 + (size_t)M[1] * i2);
                if (mask[i]) continue;
                for (int a = 0; a < P0; ++a) A[a + (size_t)P0 * (i1 + (size_t)M[1] * i2)] += r[i] * T.U[0][(size_t)i0 * P0 + a];
            }
    for (int i2 = 0; i2 < M[2]; ++i2)
        for (int i1 = 0; i1 < M[1]; ++i1)
            for (int b = 0; b < P1; ++b) {
                const double u = T.U[1][(size_t)i1 * P1 + b];
                if (u == 0.0) continue;
                for (int a = 0; a < P0; ++a)
                    B[a + (size_t)P0 * (b + (size_t)P1 * i2)] += u * A[a + (size_t)P0 * (i1 + (size_t)M[1] * i2)];
            }
    for (int i2 = 0; i2 < M[2]; ++i2)
        for (int c = 0; c < P2; ++c) {
            const double u = T.U[2][(size_t)i2 * P2 + c];
            if (u == 0.0) continue;
            for (size_t n = 0; n < (size_t)P0 * P1; ++n) Z[n + (size_t)P0 * P1 * c] += u * B[n + (size_t)P0 * P1 * i2];
        }
    for (int c = 0; c < P2; ++c)
        for (int b = 0; b < P1; ++b)
            for (int a = 0; a < P0; ++a)
                Z[a + (size_t)P0 * (b + (size_t)P1 * c)] /= T.lam[0][a] + T.lam[1][b] + T.lam[2][c] + T.shift;
    // backward
    std::fill(B.begin(), B.end(), 0.0);
    std::fill(A.begin(), A.end(), 0.0);
    for (int i2 = 0; i2 < M[2]; ++i2)
        for (int c = 0; c < P2; ++c) {
            const double u = T.U[2][(size_t)i2 * P2 + c];
            if (u == 0.0) continue;
            for (size_t n = 0; n < (size_t)P0 * P1; ++n) B[n + (size_t)P0 * P1 * i2] += u * Z[n + (size_t)P0 * P1 * c];
        }
    for (int i2 = 0; i2 < M[2]; ++i2)
        for (int i1 = 0; i1 < M[1]; ++i1)
            for (int b = 0; b < P1; ++b) {
                const double u = T.U[1][(size_t)i1 * P1 + b];
                if (u == 0.0) continue;
                for (int a = 0; a < P0; ++a)
                    A[a + (size_t)P0 * (i1 + (size_t)M[1] * i2)] += u * B[a + (size_t)P0 * (b + (size_t)P1 * i2)];
            }
    for (int i2 = 0; i2 < M[2]; ++i2)
        for (int i1 = 0; i1 < M[1]; ++i1)
            for (int i0 = 0; i0 < M[0]; ++i0) {
                const size_t i = i0 + (size_t)M[0] * (i1 + (size_t)M[1] * i2);
                double t = 0.0;
                if (!mask[i])
                    for (int a = 0; a < P0; ++a) t += A[a + (size_t)P0 * (i1 + (size_t)M[1] * i2)] * T.U[0][(size_t)i0 * P0 + a];
                y[i] = t;
            }
}

// The 3D form of tensor_setup: each metric diagonal g_dd ~ f_d0 (x) f_d1 (x) f_d2 (rank one); the mass
// factors f_de (e != d) scaled to unit mean, their scales moved into the stiffness factor f_dd; the mass
// weight of direction e is the geometric mean of the two factors f_de (the Kronecker sum needs one mass
// matrix per direction), the stiffness weight of direction d is f_dd:
//   K_sep = A_0 (x) B_1 (x) B_2 + B_0 (x) A_1 (x) B_2 + B_0 (x) B_1 (x) A_2   (exact for tensor-product maps).
static void tensor_setup3(Patch& P, const ieti_options& opt, bool mode_n) {
    const Level& L0 = P.lv[0];
    DirTable dt[3];
    for (int d = 0; d < 3; ++d) dt[d] = make_dir(L0.knots[d], P.p[d], P.knots[d], P.p[d]);
    const int Q[3] = {dt[0].Q, dt[1].Q, dt[2].Q};
    std::vector<double> f[3][3];
    for (int d = 0; d < 3; ++d) {
        std::vector<double> x[3];
        rank_one3(P.qpc[d], Q, x);
        for (int e = 0; e < 3; ++e) {
            if (e == d) continue;
            double m = 0.0;
            for (int q = 0; q < Q[e]; ++q) m += dt[e].w[q] * x[e][q];
            for (auto& v : x[e]) v /= m;
            for (auto& v : x[d]) v *= m;
        }
        for (int e = 0; e < 3; ++e) f[d][e] = x[e];
    }
    std::vector<double> A1d[3], B1d[3];
    for (int e = 0; e < 3; ++e) {
        const int d1 = (e + 1) % 3, d2 = (e + 2) % 3;
        std::vector<double> wm(Q[e]);
        for (int q = 0; q < Q[e]; ++q) wm[q] = std::sqrt(f[d1][e][q] * f[d2][e][q]);
        const DirTable& t = dt[e];
        const int M = L0.M[e], p = t.p;
        A1d[e].assign((size_t)M * M, 0.0);
        B1d[e].assign((size_t)M * M, 0.0);
        for (int q = 0; q < t.Q; ++q)
            for (int a = 0; a <= p; ++a)
                for (int b = 0; b <= p; ++b) {
                    const int i = t.first[q] + a, j = t.first[q] + b;
                    const size_t o = (size_t)q * (p + 1);
                    A1d[e][(size_t)i * M + j] += t.w[q] * f[e][e][q] * t.dN[o + a] * t.dN[o + b];
                    B1d[e][(size_t)i * M + j] += t.w[q] * wm[q] * t.N[o + a] * t.N[o + b];
                }
    }
    double msq = 0.0;
    for (int d = 0; d < 3; ++d) msq += (double)L0.nel[d] * L0.nel[d];
    const double shift = opt.smoother_sigma * msq / 3.0;
    for (int mode = 0; mode < 2; ++mode) {
        if (mode == MODE_N && !mode_n) continue;
        Patch::Tensor& T = P.ts[mode];
        const uint32_t sides = mode == MODE_D ? 0x3Fu : P.bside;
        for (int d = 0; d < 3; ++d) {
            const int M = L0.M[d];
            std::vector<int> keep;
            for (int i = 0; i < M; ++i) {
                const bool cut = (i == 0 && (sides >> (2 * d) & 1u)) || (i == M - 1 && (sides >> (2 * d + 1) & 1u));
                if (!cut) keep.push_back(i);
            }
            const int nk = (int)keep.size();
            std::vector<double> Ak((size_t)nk * nk), Bk((size_t)nk * nk), Uk, lk;
            for (int i = 0; i < nk; ++i)
                for (int j = 0; j < nk; ++j) {
                    Ak[(size_t)i * nk + j] = A1d[d][(size_t)keep[i] * M + keep[j]];
                    Bk[(size_t)i * nk + j] = B1d[d][(size_t)keep[i] * M + keep[j]];
                }
            gen_eig(nk, Ak, Bk, Uk, lk);
            const int Pd = (M + 15) / 16 * 16;
            T.Pd[d] = Pd;
            T.U[d].assign((size_t)Pd * Pd, 0.0);
            T.lam[d].assign(Pd, 1e300);
            for (int i = 0; i < nk; ++i)
                for (int a = 0; a < nk; ++a) T.U[d][(size_t)keep[i] * Pd + a] = Uk[(size_t)i * nk + a];
            for (int a = 0; a < nk; ++a) T.lam[d][a] = lk[a];
        }
        T.shift = shift;
        auto mask = level_mask(P, L0, mode);
        std::vector<double> x(L0.n), y(L0.n), z(L0.n);
        uint64_t sd = 0xBF58476D1CE4E5B9ull;
        for (int64_t i = 0; i < L0.n; ++i) {
            sd ^= sd << 13; sd ^= sd >> 7; sd ^= sd << 17;
            x[i] = mask[i] ? 0.0 : ((sd >> 11) * (1.0 / 9007199254740992.0) - 0.5);
        }
        double lam = 1.0;
        for (int it = 0; it < 20; ++it) {
            host_apply(P, L0, mask, x.data(), y.data());
            tensor_apply_host3(T, L0.M, mask, y.data(), z.data());
            double nx = 0.0, nz = 0.0;
            for (int64_t i = 0; i < L0.n; ++i) {
                nx += x[i] * x[i];
                nz += z[i] * z[i];
            }
            if (!(nz > 0.0) || !(nx > 0.0)) break;
            lam = std::sqrt(nz / nx);
            const double sc = 1.0 / std::sqrt(nz);
            for (int64_t i = 0; i < L0.n; ++i) x[i] = z[i] * sc;
        }
        T.tau = 1.0 / lam;
    }
}

// dense inverse of the masked level matrix (masked rows/cols zero) by Cholesky
static std::vector<double> dense_inverse(const Patch& P, const Level& L, int mode) {
    auto mask = level_mask(P, L, mode);
    int64_t n = L.n;
    std::vector<double> A((size_t)n * n, 0.0);
    std::vector<double> e(n, 0.0), col(n);
    for (int64_t j = 0; j < n; ++j) {
        if (mask[j]) { A[(size_t)j * n + j] = 1.0; continue; }
        e[j] = 1.0;
        host_apply(P, L, mask, e.data(), col.data());
        e[j] = 0.0;
        for (int64_t i = 0; i < n; ++i) A[(size_t)i * n + j] = col[i];
    }
    // Cholesky A = C C^T (lower, row-major, in place): every dot product runs over two contiguous rows
    for (int64_t j = 0; j < n; ++j) {
        const double* Cj = &A[(size_t)j * n];
        const double s = A[(size_t)j * n + j] - dot4(Cj, Cj, j);
        if (!(s > 0)) throw Error(IETI_EINVAL, "coarsest-level matrix is not positive definite");
        const double c = std::sqrt(s);
        A[(size_t)j * n + j] = c;
        for (int64_t i = j + 1; i < n; ++i) A[(size_t)i * n + j] = (A[(size_t)i * n + j] - dot4(&A[(size_t)i * n], Cj, j)) / c;
    }
    // C^T by rows, so that the backward substitutions read contiguous rows too
    std::vector<double> CT((size_t)n * n, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = 0; k <= i; ++k) CT[(size_t)k * n + i] = A[(size_t)i * n + k];
    std::vector<double> inv((size_t)n * n, 0.0), z(n);
    for (int64_t j = 0; j < n; ++j) {
        if (mask[j]) continue;
        // C y = e_j: y[i] = 0 for i < j
        std::fill(z.begin(), z.end(), 0.0);
        for (int64_t i = j; i < n; ++i) {
            const double t = (i == j ? 1.0 : 0.0) - dot4(&A[(size_t)i * n + j], &z[j], i - j);
            z[i] = t / A[(size_t)i * n + i];
        }
        // C^T x = y
        for (int64_t i = n - 1; i >= 0; --i) {
            const double t = z[i] - dot4(&CT[(size_t)i * n + i + 1], &z[i + 1], n - 1 - i);
            z[i] = t / A[(size_t)i * n + i];
        }
        for (int64_t i = 0; i < n; ++i) inv[(size_t)i * n + j] = mask[i] ? 0.0 : z[i];
    }
    return inv;
}

// Banded Cholesky A = L L^T of the masked level-0 stiffness (masked rows and
// columns replaced by the identity), then the blocked layout of the GPU
// triangular solves: for every block row r of BAND_NB rows
//   L_off[ii][c] = L(i, r*nb - b + c)      (columns left of the block)
//   U_off[ii][c] = L((r+1)*nb + c, i)      (L^T right of the block)
//   Linv[ii][cc] = inv(L_rr)(ii, cc)       (diagonal block inverse)
// with i = r*nb + ii; entries outside the band or the matrix are 0.
static void band_factor(const Patch& P, const Level& L, int mode, int64_t b, std::vector<double>& out) {
    const int64_t n = L.n, w = b + 1;
    auto mask = level_mask(P, L, mode);
    std::vector<double> A((size_t)n * w, 0.0);   // A[i][j - i + b], j in [i-b, i]
    for (int i2 = 0; i2 < L.M[2]; ++i2)
        for (int i1 = 0; i1 < L.M[1]; ++i1)
            for (int i0 = 0; i0 < L.M[0]; ++i0) {
                const int64_t j = lin(L.M, i0, i1, i2);
                for (int s = 0; s < L.nst; ++s) {
                    const int k0 = i0 + L.offs[3 * s], k1 = i1 + L.offs[3 * s + 1], k2 = i2 + L.offs[3 * s + 2];
                    if (k0 < 0 || k0 >= L.M[0] || k1 < 0 || k1 >= L.M[1] || k2 < 0 || k2 >= L.M[2]) continue;
                    const int64_t i = lin(L.M, k0, k1, k2);   // i >= j (upper-half offset)
                    double v = L.coef[(size_t)s * L.n + j];
                    if (mask[i] || mask[j]) v = (i == j) ? 1.0 : 0.0;
                    A[(size_t)i * w + (j - i + b)] = v;
                }
            }
    // row-oriented Cholesky in band storage (L overwrites A)
    for (int64_t i = 0; i < n; ++i) {
        const int64_t j0 = std::max<int64_t>(0, i - b);
        for (int64_t j = j0; j <= i; ++j) {
            double s = A[(size_t)i * w + (j - i + b)];
            const int64_t k0 = std::max(j0, j - b);
            const double* Li = &A[(size_t)i * w + (k0 - i + b)];
            const double* Lj = &A[(size_t)j * w + (k0 - j + b)];
            s -= dot4(Li, Lj, j - k0);
            if (j == i) {
                if (!(s > 0)) throw Error(IETI_EINVAL, "local stiffness is not positive definite");
                A[(size_t)i * w + b] = std::sqrt(s);
            } else {
                A[(size_t)i * w + (j - i + b)] = s / A[(size_t)j * w + b];
            }
        }
    }
    auto Lat = [&](int64_t i, int64_t j) -> double {   // L(i, j), 0 outside the band / matrix
        if (i < 0 || j < 0 || i >= n || j >= n || j > i || i - j > b) return 0.0;
        return A[(size_t)i * w + (j - i + b)];
    };
    const int64_t nb = BAND_NB, nblk = (n + nb - 1) / nb, bs = nb * (2 * b + nb);
    out.assign((size_t)(nblk * bs), 0.0);
    std::vector<double> D((size_t)nb * nb), Di((size_t)nb * nb);
    for (int64_t r = 0; r < nblk; ++r) {
        double* blk = &out[(size_t)(r * bs)];
        for (int64_t ii = 0; ii < nb; ++ii) {
            const int64_t i = r * nb + ii;
            for (int64_t c = 0; c < b; ++c) {
                blk[ii * b + c] = Lat(i, r * nb - b + c);
                blk[nb * b + ii * b + c] = Lat((r + 1) * nb + c, i);
            }
        }
        // diagonal block (identity on padding rows) and its inverse (forward substitution)
        for (int64_t ii = 0; ii < nb; ++ii)
            for (int64_t cc = 0; cc < nb; ++cc) {
                const int64_t i = r * nb + ii, j = r * nb + cc;
                D[ii * nb + cc] = i >= n ? (ii == cc ? 1.0 : 0.0) : (j <= i ? Lat(i, j) : 0.0);
            }
        for (int64_t c = 0; c < nb; ++c)
            for (int64_t ii = 0; ii < nb; ++ii) {
                double s = ii == c ? 1.0 : 0.0;
                for (int64_t k = c; k < ii; ++k) s -= D[ii * nb + k] * Di[k * nb + c];
                Di[ii * nb + c] = ii < c ? 0.0 : s / D[ii * nb + ii];
            }
        std::copy(Di.begin(), Di.end(), blk + 2 * nb * b);
    }
}

// ----------------------------------------------------------------------------
// topology

struct UF {
    std::vector<int64_t> p;
    explicit UF(int64_t n) : p(n) { std::iota(p.begin(), p.end(), 0); }
    int64_t find(int64_t x) {
        while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
        return x;
    }
    void unite(int64_t a, int64_t b) {
        a = find(a); b = find(b);
        if (a != b) p[std::max(a, b)] = std::min(a, b);
    }
};

static void validate_patch(const ieti_patch& ip, int dim0, int k) {
    auto fail = [&](const std::string& m) { throw Error(IETI_EINVAL, "patch " + std::to_string(k) + ": " + m); };
    if (ip.dim != 2 && ip.dim != 3) fail("dim must be 2 or 3");
    if (ip.dim != dim0) fail("all patches must have the same dimension");
    if (!ip.ctrl) fail("null control points");
    for (int d = 0; d < ip.dim; ++d) {
        int p = ip.degree[d];
        if (p < 1 || p > 6) fail("degree must be in 1..6");
        if (!ip.knots[d]) fail("null knot vector");
        int nk = ip.n_knots[d];
        if (nk < 2 * (p + 1)) fail("knot vector too short");
        const double* t = ip.knots[d];
        for (int i = 0; i < nk; ++i)
            if (!std::isfinite(t[i])) fail("non-finite knot");
        for (int i = 0; i <= p; ++i)
            if (t[i] != 0.0 || t[nk - 1 - i] != 1.0) fail("knot vectors must be open on [0,1]");
        for (int i = p; i < nk - p - 1; ++i)
            if (!(t[i + 1] > t[i])) fail("interior knots must be simple and increasing");
    }
}

Plan* build_plan(const ieti_patch* in, int n, const double* pv, int n_pv, const ieti_options* optp,
                 const int32_t* comp) {
    if (!in || n <= 0) throw Error(IETI_EINVAL, "no patches");
    if (comp)
        for (int k = 1; k < n; ++k)
            if (comp[k] < comp[k - 1]) throw Error(IETI_EINVAL, "problem ids of the patches must not decrease");
    auto comp_of = [&](int k) { return comp ? comp[k] : 0; };
    ieti_options opt;
    if (optp) opt = *optp; else default_options(&opt);
    if (opt.mg_precision != 32 && opt.mg_precision != 64) throw Error(IETI_EINVAL, "mg_precision must be 32 or 64");
    if (opt.local_solver != IETI_LOCAL_MG && opt.local_solver != IETI_LOCAL_EXACT &&
        opt.local_solver != IETI_LOCAL_EXACT_MG && opt.local_solver != IETI_LOCAL_MG_SADDLE)
        throw Error(IETI_EINVAL, "unknown local solver");
    if (!(opt.tol > 0) || !(opt.inner_tol > 0) || !(opt.basis_tol > 0) || opt.max_it <= 0 || opt.inner_max_it <= 0)
        throw Error(IETI_EINVAL, "tolerances and iteration limits must be positive");
    if (opt.prec_vcycles < 1) throw Error(IETI_EINVAL, "prec_vcycles must be >= 1");
    if (opt.check_every < 1) opt.check_every = 1;
    if (opt.coarse_level < -1) throw Error(IETI_EINVAL, "coarse_level must be >= -1");
    if (opt.coarse_dofs < 0) throw Error(IETI_EINVAL, "coarse_dofs must be >= 0");
    if (opt.coarse_degree != 0 && opt.coarse_degree != 1) throw Error(IETI_EINVAL, "coarse_degree must be 0 or 1");
    if (opt.cheb_degree < 0 || opt.cheb_degree > 8 || opt.cheb_degree_coarse < 0 || opt.cheb_degree_coarse > 8)
        throw Error(IETI_EINVAL, "Chebyshev degrees must be in 0..8");
    if (opt.smoother != IETI_SMOOTHER_CHEBYSHEV && opt.smoother != IETI_SMOOTHER_TENSOR)
        throw Error(IETI_EINVAL, "unknown smoother");
    if (opt.smoother == IETI_SMOOTHER_TENSOR && !(opt.smoother_sigma > 0))
        throw Error(IETI_EINVAL, "smoother_sigma must be positive");
    const int dim = in[0].dim;
    for (int k = 0; k < n; ++k) validate_patch(in[k], dim, k);
    auto P = std::make_unique<Plan>();
    Plan& pl = *P;
    pl.dim = dim;
    pl.N = n;
    pl.opt = opt;
    if (opt.tune_cache) {
        pl.tune_cache = opt.tune_cache;
        pl.opt.tune_cache = pl.tune_cache.c_str();
    }
    pl.patches.resize(n);
    int64_t off = 0;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int k = 0; k < n; ++k) {
        Patch& pa = pl.patches[k];
        pa.dim = dim;
        int64_t nd = 1;
        int M[3] = {1, 1, 1};
        for (int d = 0; d < dim; ++d) {
            pa.p[d] = in[k].degree[d];
            pa.knots[d].assign(in[k].knots[d], in[k].knots[d] + in[k].n_knots[d]);
            M[d] = in[k].n_knots[d] - pa.p[d] - 1;
            nd *= M[d];
        }
        pa.ctrl.assign(in[k].ctrl, in[k].ctrl + nd * dim);
        for (double v : pa.ctrl)
            if (!std::isfinite(v)) throw Error(IETI_EINVAL, "non-finite control point");
        for (int64_t i = 0; i < nd; ++i)
            for (int c = 0; c < dim; ++c) {
                lo[c] = std::min(lo[c], pa.ctrl[i * dim + c]);
                hi[c] = std::max(hi[c], pa.ctrl[i * dim + c]);
            }
        Level L0;
        for (int d = 0; d < 3; ++d) {
            L0.M[d] = M[d];
            if (d < dim) {
                L0.p[d] = pa.p[d];
                L0.knots[d] = pa.knots[d];
                L0.nel[d] = (int)breakpoints(pa.knots[d]).size() - 1;
            }
        }
        L0.n = nd;
        pa.lv.push_back(L0);
        pa.torn_off = off;
        off += nd;
    }
    pl.ndof_torn = off;
    double diam = 0;
    for (int c = 0; c < dim; ++c) diam = std::max(diam, hi[c] - lo[c]);
    const double tol = 1e-9 * std::max(diam, 1e-300);

    // ---- corners -> vertices
    const int ncorner = 1 << dim;
    std::vector<std::array<double, 3>> vcoord;
    std::vector<int> vcomp;   // problem of each vertex
    std::vector<std::vector<int>> cvert(n, std::vector<int>(ncorner));
    auto corner_index = [&](const Patch& pa, int c) {
        int idx[3] = {0, 0, 0};
        for (int d = 0; d < dim; ++d) idx[d] = (c >> d & 1) ? pa.lv[0].M[d] - 1 : 0;
        return lin(pa.lv[0].M, idx[0], idx[1], idx[2]);
    };
    for (int k = 0; k < n; ++k)
        for (int c = 0; c < ncorner; ++c) {
            const Patch& pa = pl.patches[k];
            int64_t i = corner_index(pa, c);
            std::array<double, 3> x = {0, 0, 0};
            for (int d = 0; d < dim; ++d) x[d] = pa.ctrl[i * dim + d];
            int found = -1;
            for (size_t v = 0; v < vcoord.size() && found < 0; ++v) {
                if (vcomp[v] != comp_of(k)) continue;
                double dd = 0;
                for (int d = 0; d < dim; ++d) dd = std::max(dd, std::fabs(vcoord[v][d] - x[d]));
                if (dd <= tol) found = (int)v;
            }
            if (found < 0) {
                found = (int)vcoord.size();
                vcoord.push_back(x);
                vcomp.push_back(comp_of(k));
            }
            cvert[k][c] = found;
        }

    // ---- sides: match by their corner vertex sequences
    struct SideRef { int k, d, e; };
    std::map<std::vector<int>, std::vector<SideRef>> sides;
    for (int k = 0; k < n; ++k)
        for (int d = 0; d < dim; ++d)
            for (int e = 0; e < 2; ++e) {
                std::vector<int> seq;
                for (int c = 0; c < ncorner; ++c)
                    if ((c >> d & 1) == e) seq.push_back(cvert[k][c]);
                std::vector<int> key = seq;
                std::sort(key.begin(), key.end());
                sides[key].push_back({k, d, e});
            }
    UF uf(pl.ndof_torn);
    for (auto& kv : sides) {
        auto& v = kv.second;
        if (v.size() == 1) {
            pl.patches[v[0].k].bside |= 1u << (2 * v[0].d + v[0].e);
            continue;
        }
        if (v.size() > 2) throw Error(IETI_ENONCONFORMING, "more than two patches share a side");
        SideRef a = v[0], b = v[1];
        if (a.e == 1 && b.e == 0) {} else if (a.e == 0 && b.e == 1) std::swap(a, b);
        else throw Error(IETI_ENONCONFORMING, "interface orientation not supported");
        if (a.d != b.d) throw Error(IETI_ENONCONFORMING, "interface orientation not supported");
        // same orientation: corner sequences in the same order
        std::vector<int> sa, sb;
        for (int c = 0; c < ncorner; ++c) {
            if ((c >> a.d & 1) == 1) sa.push_back(cvert[a.k][c]);
            if ((c >> b.d & 1) == 0) sb.push_back(cvert[b.k][c]);
        }
        if (sa != sb) throw Error(IETI_ENONCONFORMING, "interface orientation not supported");
        const Patch& A = pl.patches[a.k];
        const Patch& B = pl.patches[b.k];
        for (int d = 0; d < dim; ++d) {
            if (d == a.d) continue;
            if (A.p[d] != B.p[d] || A.knots[d].size() != B.knots[d].size())
                throw Error(IETI_ENONCONFORMING, "spline spaces differ along an interface");
            for (size_t i = 0; i < A.knots[d].size(); ++i)
                if (std::fabs(A.knots[d][i] - B.knots[d][i]) > 1e-12)
                    throw Error(IETI_ENONCONFORMING, "knot vectors differ along an interface");
        }
        const int* MA = A.lv[0].M;
        const int* MB = B.lv[0].M;
        int t1 = a.d == 0 ? 1 : 0, t2 = a.d == 2 ? 1 : 2;
        int n1 = MA[t1], n2 = dim == 3 ? MA[t2] : 1;
        for (int j2 = 0; j2 < n2; ++j2)
            for (int j1 = 0; j1 < n1; ++j1) {
                int ia[3] = {0, 0, 0}, ib[3] = {0, 0, 0};
                ia[a.d] = MA[a.d] - 1;
                ib[a.d] = 0;
                ia[t1] = ib[t1] = j1;
                if (dim == 3) ia[t2] = ib[t2] = j2;
                int64_t la = lin(MA, ia[0], ia[1], ia[2]), lb = lin(MB, ib[0], ib[1], ib[2]);
                double dd = 0;
                for (int c = 0; c < dim; ++c) dd = std::max(dd, std::fabs(A.ctrl[la * dim + c] - B.ctrl[lb * dim + c]));
                if (dd > tol) throw Error(IETI_ENONCONFORMING, "patches do not meet along an interface");
                uf.unite(A.torn_off + la, B.torn_off + lb);
            }
    }

    // ---- groups of shared coefficients and boundary status
    auto on_bside = [&](const Patch& pa, int64_t i) {
        int M0 = pa.lv[0].M[0], M1 = pa.lv[0].M[1];
        int ii[3] = {(int)(i % M0), (int)((i / M0) % M1), (int)(i / ((int64_t)M0 * M1))};
        for (int d = 0; d < dim; ++d) {
            if (ii[d] == 0 && (pa.bside >> (2 * d) & 1)) return true;
            if (ii[d] == pa.lv[0].M[d] - 1 && (pa.bside >> (2 * d + 1) & 1)) return true;
        }
        return false;
    };
    std::vector<std::pair<int64_t, int64_t>> rp;   // (root, position) for shared coefficients
    auto pos_patch = [&](int64_t pos) {
        int lo_ = 0, hi_ = n - 1;
        while (lo_ < hi_) {
            int mid = (lo_ + hi_ + 1) / 2;
            if (pl.patches[mid].torn_off <= pos) lo_ = mid; else hi_ = mid - 1;
        }
        return lo_;
    };
    for (int64_t pos = 0; pos < pl.ndof_torn; ++pos) {
        int64_t r = uf.find(pos);
        if (r != pos) rp.push_back({r, pos});
    }
    // include roots of groups
    {
        std::vector<uint8_t> isroot(pl.ndof_torn, 0);
        for (auto& x : rp) isroot[x.first] = 1;
        for (int64_t pos = 0; pos < pl.ndof_torn; ++pos)
            if (isroot[pos]) rp.push_back({pos, pos});
    }
    std::sort(rp.begin(), rp.end());
    rp.erase(std::unique(rp.begin(), rp.end()), rp.end());
    struct Group { std::vector<int64_t> pos; bool dir = false; };
    std::vector<Group> groups;
    for (size_t i = 0; i < rp.size();) {
        size_t j = i;
        Group g;
        while (j < rp.size() && rp[j].first == rp[i].first) { g.pos.push_back(rp[j].second); ++j; }
        std::sort(g.pos.begin(), g.pos.end());
        for (int64_t pos : g.pos) {
            int k = pos_patch(pos);
            if (on_bside(pl.patches[k], pos - pl.patches[k].torn_off)) g.dir = true;
        }
        groups.push_back(std::move(g));
        i = j;
    }
    std::vector<int64_t> group_of(pl.ndof_torn, -1);
    for (size_t gi = 0; gi < groups.size(); ++gi)
        for (int64_t pos : groups[gi].pos) group_of[pos] = (int64_t)gi;

    // boundary coefficients at corners that lie on no boundary side of their patch
    for (int k = 0; k < n; ++k) {
        Patch& pa = pl.patches[k];
        for (int c = 0; c < ncorner; ++c) {
            int64_t li = corner_index(pa, c);
            int64_t g = group_of[pa.torn_off + li];
            if (g >= 0 && groups[g].dir && !on_bside(pa, li)) pa.dcorner |= 1u << c;
        }
    }

    // ---- primal vertices
    std::vector<uint8_t> gprimal(groups.size(), 0);
    std::vector<int64_t> vgroups;
    for (int k = 0; k < n; ++k) {
        const Patch& pa = pl.patches[k];
        for (int c = 0; c < ncorner; ++c) {
            int64_t g = group_of[pa.torn_off + corner_index(pa, c)];
            if (g < 0 || groups[g].dir || gprimal[g]) continue;
            bool take = (opt.primal & IETI_PRIMAL_VERTICES) != 0;
            if (pv && take) {
                take = false;
                int64_t li = corner_index(pa, c);
                for (int v = 0; v < n_pv && !take; ++v) {
                    double dd = 0;
                    for (int d = 0; d < dim; ++d) dd = std::max(dd, std::fabs(pv[v * dim + d] - pa.ctrl[li * dim + d]));
                    if (dd <= tol) take = true;
                }
            }
            if (take) { gprimal[g] = 1; vgroups.push_back(g); }
        }
    }
    std::sort(vgroups.begin(), vgroups.end());
    std::map<int64_t, int64_t> vindex;
    for (size_t i = 0; i < vgroups.size(); ++i) vindex[vgroups[i]] = (int64_t)i;
    pl.n_primal_vertices = (int64_t)vgroups.size();
    // ---- edge averages (3D)
    std::map<int64_t, int64_t> eindex;   // group of first interior edge coefficient -> global primal
    struct LocalEdge { int k; int e; std::vector<int64_t> loc; int64_t key; };
    std::vector<LocalEdge> ledges;
    if (opt.primal & IETI_PRIMAL_EDGES) {
        for (int k = 0; k < n; ++k) {
            const Patch& pa = pl.patches[k];
            const int* M = pa.lv[0].M;
            int eid = 0;
            if (dim == 2) {
                // the edges of a 2D decomposition are the patch sides (corners excluded)
                for (int fr = 0; fr < 2; ++fr)
                    for (int e = 0; e < 2; ++e, ++eid) {
                        LocalEdge le;
                        le.k = k;
                        le.e = eid;
                        for (int t = 1; t < M[fr] - 1; ++t) {
                            int ii[3] = {0, 0, 0};
                            ii[fr] = t;
                            ii[1 - fr] = e ? M[1 - fr] - 1 : 0;
                            le.loc.push_back(lin(M, ii[0], ii[1], 0));
                        }
                        if (le.loc.empty()) continue;
                        int64_t g = group_of[pa.torn_off + le.loc[0]];
                        if (g < 0 || groups[g].dir) continue;
                        le.key = g;
                        eindex[g] = 0;
                        ledges.push_back(le);
                    }
                continue;
            }
            for (int fr = 0; fr < 3; ++fr) {
                int oa = fr == 0 ? 1 : 0, ob = fr == 2 ? 1 : 2;
                for (int ea = 0; ea < 2; ++ea)
                    for (int eb = 0; eb < 2; ++eb, ++eid) {
                        LocalEdge le;
                        le.k = k;
                        le.e = eid;
                        for (int t = 1; t < M[fr] - 1; ++t) {
                            int ii[3];
                            ii[fr] = t;
                            ii[oa] = ea ? M[oa] - 1 : 0;
                            ii[ob] = eb ? M[ob] - 1 : 0;
                            le.loc.push_back(lin(M, ii[0], ii[1], ii[2]));
                        }
                        if (le.loc.empty()) continue;
                        int64_t g = group_of[pa.torn_off + le.loc[0]];
                        if (g < 0 || groups[g].dir) continue;
                        le.key = g;
                        eindex[g] = 0;
                        ledges.push_back(le);
                    }
            }
        }
        int64_t c = (int64_t)vgroups.size();
        for (auto& kv : eindex) kv.second = c++;
    }
    pl.n_primal = (int64_t)vgroups.size() + (int64_t)eindex.size();
    for (int k = 0; k < n; ++k) {
        Patch& pa = pl.patches[k];
        for (int c = 0; c < ncorner; ++c) {
            int64_t g = group_of[pa.torn_off + corner_index(pa, c)];
            if (g >= 0 && gprimal[g]) {
                pa.pcorner |= 1u << c;
                pa.primal_global.push_back(vindex[g]);
                pa.primal_corner.push_back(c);
                pa.primal_edge.emplace_back();
            }
        }
    }
    for (auto& le : ledges) {
        Patch& pa = pl.patches[le.k];
        pa.primal_global.push_back(eindex[le.key]);
        pa.primal_corner.push_back(-1);
        pa.primal_edge.push_back(le.loc);
    }
    // floating patches: no Dirichlet coefficient and no eliminated primal vertex, so K is singular on the
    // constants; edge-average constraints fix them (Sec. 3.2, eq. (6) with a semi-definite block).  The local
    // Neumann solves run on K + gamma sum_e c_e c_e^T (c_e the edge-average functional): on {C w = 0} this is
    // K, so the unconstrained solve followed by the energy-minimising projection gives the constrained
    // minimiser; gamma = alpha / n_e gives the constants the energy alpha 1^T M^ 1 = alpha they have in the
    // regularised multigrid operator K + alpha M^ of the coarser levels.
    for (int k = 0; k < n; ++k) {
        Patch& pa = pl.patches[k];
        if (pa.bside != 0 || pa.pcorner != 0 || pa.dcorner != 0) continue;
        int ne = 0;
        for (size_t j = 0; j < pa.primal_corner.size(); ++j)
            if (pa.primal_corner[j] < 0 && !pa.primal_edge[j].empty()) ++ne;
        if (ne == 0)
            throw Error(IETI_EINVAL, "patch " + std::to_string(k) +
                                         " has no boundary side, no primal vertex and no edge-average constraint");
        if (opt.local_solver != IETI_LOCAL_MG)
            throw Error(IETI_ENOTSUP, "patch " + std::to_string(k) +
                                          " floats (no Dirichlet or primal-vertex coefficient): only the MG-MG "
                                          "variant supports floating patches");
        pa.floating = true;
        pa.float_gamma = FLOAT_ALPHA / (double)ne;
    }
    {
        std::vector<std::vector<std::pair<int64_t, int64_t>>> contrib(pl.n_primal);
        for (int k = 0; k < n; ++k)
            for (size_t j = 0; j < pl.patches[k].primal_global.size(); ++j)
                contrib[pl.patches[k].primal_global[j]].push_back({k, (int64_t)j});
        pl.pri_ptr.push_back(0);
        for (auto& c : contrib) {
            for (auto& x : c) { pl.pri_patch.push_back(x.first); pl.pri_local.push_back(x.second); }
            pl.pri_ptr.push_back((int64_t)pl.pri_patch.size());
        }
    }

    // ---- consistency: boundary status must follow from side/corner masks
    for (size_t gi = 0; gi < groups.size(); ++gi)
        for (int64_t pos : groups[gi].pos) {
            int k = pos_patch(pos);
            const Patch& pa = pl.patches[k];
            int64_t li = pos - pa.torn_off;
            bool masked = on_bside(pa, li);
            if (!masked) {
                for (int c = 0; c < ncorner; ++c)
                    if ((pa.dcorner >> c & 1) && corner_index(pa, c) == li) masked = true;
            }
            if (masked != groups[gi].dir) throw Error(IETI_ENOTSUP, "boundary coefficient inside a patch side");
        }

    // ---- multipliers (fully redundant) and B^T slots
    std::map<int64_t, std::vector<std::pair<int64_t, double>>> slot_map;   // pos -> (lambda, sign)
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const Group& g = groups[gi];
        if (g.dir || gprimal[gi] || g.pos.size() < 2) continue;
        int m = (int)g.pos.size();
        for (int a = 0; a < m; ++a)
            for (int b = a + 1; b < m; ++b) {
                int64_t l = (int64_t)pl.lam_plus.size();
                pl.lam_plus.push_back(g.pos[a]);
                pl.lam_minus.push_back(g.pos[b]);
                pl.lam_mult.push_back(m);
                slot_map[g.pos[a]].push_back({l, 1.0});
                slot_map[g.pos[b]].push_back({l, -1.0});
            }
    }
    pl.n_lambda = (int64_t)pl.lam_plus.size();
    pl.slot_ptr.push_back(0);
    for (auto& kv : slot_map) {
        pl.slot_pos.push_back(kv.first);
        int m = (int)groups[group_of[kv.first]].pos.size();
        pl.slot_mult.push_back(m);
        for (auto& x : kv.second) { pl.slot_lam.push_back(x.first); pl.slot_sgn.push_back(x.second); }
        pl.slot_ptr.push_back((int64_t)pl.slot_lam.size());
    }
    pl.grp_ptr.push_back(0);
    int64_t nshared = 0;
    for (auto& g : groups) {
        if (g.dir || g.pos.size() < 2) continue;
        for (int64_t pos : g.pos) pl.grp_pos.push_back(pos);
        pl.grp_ptr.push_back((int64_t)pl.grp_pos.size());
        ++nshared;
    }
    // global dofs: shared non-boundary groups + coefficients held by one patch only and not on the boundary
    int64_t nsingle = 0;
    for (int k = 0; k < n; ++k) {
        const Patch& pa = pl.patches[k];
        for (int64_t i = 0; i < pa.lv[0].n; ++i)
            if (group_of[pa.torn_off + i] < 0 && !on_bside(pa, i)) ++nsingle;
    }
    pl.ndof_global = nshared + nsingle;

    // ---- affine detection, multigrid levels, assembly
    for (int k = 0; k < n; ++k) {
        Patch& pa = pl.patches[k];
        const int* M = pa.lv[0].M;
        double A[3][3] = {{0}}, c0[3] = {0};
        for (int c = 0; c < dim; ++c) c0[c] = pa.ctrl[c];
        for (int d = 0; d < dim; ++d) {
            int idx[3] = {0, 0, 0};
            idx[d] = M[d] - 1;
            int64_t i = lin(M, idx[0], idx[1], idx[2]);
            for (int c = 0; c < dim; ++c) A[c][d] = pa.ctrl[i * dim + c] - c0[c];
        }
        std::vector<double> gr[3];
        for (int d = 0; d < dim; ++d) {
            int p = pa.p[d];
            for (int i = 0; i < M[d]; ++i) {
                double s = 0;
                for (int j = 1; j <= p; ++j) s += pa.knots[d][i + j];
                gr[d].push_back(s / p);
            }
        }
        bool aff = true;
        for (int i2 = 0; i2 < M[2] && aff; ++i2)
            for (int i1 = 0; i1 < M[1] && aff; ++i1)
                for (int i0 = 0; i0 < M[0] && aff; ++i0) {
                    double xi[3] = {gr[0][i0], gr[1][i1], dim == 3 ? gr[2][i2] : 0.0};
                    int64_t i = lin(M, i0, i1, i2);
                    for (int c = 0; c < dim; ++c) {
                        double x = c0[c];
                        for (int d = 0; d < dim; ++d) x += A[c][d] * xi[d];
                        if (std::fabs(x - pa.ctrl[i * dim + c]) > 1e-13 * std::max(diam, 1.0)) aff = false;
                    }
                }
        pa.affine = aff;
        // levels: halve while every direction has an even number (>= 6) of elements
        // and the level is larger than coarse_dofs
        const bool mg = opt.local_solver != IETI_LOCAL_EXACT;              // some problems by multigrid
        while (mg) {
            const Level& f = pa.lv.back();
            bool ok = opt.coarse_dofs == 0 || f.n > opt.coarse_dofs;
            for (int d = 0; d < dim; ++d)
                if (f.nel[d] % 2 || f.nel[d] / 2 < 3) ok = false;
            if (!ok) break;
            Level c;
            for (int d = 0; d < dim; ++d) {
                // degree 1 on every coarse level with coarse_degree = 1 (Sec. 4), else the patch's degree
                const int pc = opt.coarse_degree == 1 ? 1 : pa.p[d];
                std::vector<double> b = breakpoints(f.knots[d]), bc;
                for (size_t i = 0; i < b.size(); i += 2) bc.push_back(b[i]);
                std::vector<double> t(pc + 1, bc.front());
                for (size_t i = 1; i + 1 < bc.size(); ++i) t.push_back(bc[i]);
                for (int i = 0; i <= pc; ++i) t.push_back(bc.back());
                c.p[d] = pc;
                c.knots[d] = t;
                c.nel[d] = (int)bc.size() - 1;
                c.M[d] = (int)t.size() - pc - 1;
            }
            c.n = (int64_t)c.M[0] * c.M[1] * c.M[2];
            pa.lv.push_back(c);
        }
        for (Level& L : pa.lv) {
            L.guard = L.p[0] + (int64_t)L.p[1] * L.M[0] + (dim == 3 ? (int64_t)L.p[2] * L.M[0] * L.M[1] : 0);
        }
        pl.max_levels = std::max(pl.max_levels, (int)pa.lv.size());
    }
    parallel_for(n, [&](int k) {
        const bool mg = opt.local_solver != IETI_LOCAL_EXACT;
        const bool neumann_mg = opt.local_solver == IETI_LOCAL_MG || opt.local_solver == IETI_LOCAL_MG_SADDLE;
        Patch& pa = pl.patches[k];
        for (size_t l = 0; l < pa.lv.size(); ++l) assemble_level(pa, pa.lv[l], l == 0);
        // floating patches: the coarser levels of the multigrid carry K + alpha M^ (definite), the finest
        // level keeps K (its stencil is also the exact operator of the local solves)
        if (pa.floating)
            for (size_t l = 1; l < pa.lv.size(); ++l) add_param_mass(pa, pa.lv[l], FLOAT_ALPHA);
        for (size_t l = 0; l + 1 < pa.lv.size(); ++l) {
            Level& f = pa.lv[l];
            const Level& c = pa.lv[l + 1];
            f.l2 = false;
            for (int d = 0; d < dim; ++d)
                if (f.p[d] != c.p[d]) f.l2 = true;
            for (int d = 0; d < dim; ++d) {
                if (f.l2) {   // non-nested spaces: L2 projection M_f^{-1} M_fc (parametric)
                    f.P[d] = mixed_mass(f.knots[d], f.p[d], c.knots[d], c.p[d]);
                    f.Mc[d] = c.M[d];
                    f.mchol[d] = band_mass_chol(f.knots[d], f.p[d]);
                    continue;
                }
                int Mf, Mc;
                f.P[d] = prolongation(c.knots[d], f.knots[d], c.p[d], Mf, Mc);
                f.Mc[d] = Mc;
            }
        }
        if (mg)
            for (size_t l = 0; l + 1 < pa.lv.size(); ++l) {
                if (neumann_mg) pa.lv[l].lmax[MODE_N] = power_lmax(pa, pa.lv[l], MODE_N);
                pa.lv[l].lmax[MODE_D] = power_lmax(pa, pa.lv[l], MODE_D);
            }
        if (mg && opt.smoother == IETI_SMOOTHER_TENSOR && pa.lv.size() > 1) {
            if (dim == 2) tensor_setup(pa, opt, neumann_mg);
            else tensor_setup3(pa, opt, neumann_mg);
        }
        Level& cl = pa.lv.back();
        if (mg) {
            if (neumann_mg && pa.floating && pa.lv.size() == 1) {   // a one-level floating patch: K + alpha M^
                Level reg = cl;
                add_param_mass(pa, reg, FLOAT_ALPHA);
                cl.inv[MODE_N] = dense_inverse(pa, reg, MODE_N);
            } else if (neumann_mg) {
                cl.inv[MODE_N] = dense_inverse(pa, cl, MODE_N);
            }
            cl.inv[MODE_D] = dense_inverse(pa, cl, MODE_D);
        }
        if (!neumann_mg) {
            const Level& L0 = pa.lv[0];
            pa.band_b = L0.guard;
            pa.band_nblk = (L0.n + BAND_NB - 1) / BAND_NB;
            if (dim == 2) {   // 3D bands are factorised on the device (the runtime's block-band path)
                band_factor(pa, L0, MODE_N, pa.band_b, pa.band[MODE_N]);
                if (!mg) band_factor(pa, L0, MODE_D, pa.band_b, pa.band[MODE_D]);
            }
        }
    });
    int64_t nq = 0;
    for (auto& pa : pl.patches) nq += pa.n_qp;
    pl.n_qp = nq;
    // ranges of the independent problems: patches, multipliers (groups, hence multipliers, follow the torn
    // order, and a group never spans two problems), quadrature points, torn coefficients
    pl.ncomp = 0;
    pl.comp_patch_beg.clear();
    for (int k = 0; k < n; ++k)
        if (k == 0 || comp_of(k) != comp_of(k - 1)) pl.comp_patch_beg.push_back(k);
    pl.ncomp = (int)pl.comp_patch_beg.size();
    pl.comp_patch_beg.push_back(n);
    pl.comp_lam_beg.assign(pl.ncomp + 1, 0);
    pl.comp_qp_beg.assign(pl.ncomp + 1, 0);
    pl.comp_torn_beg.assign(pl.ncomp + 1, 0);
    {
        std::vector<int> pcomp(n);
        for (int c = 0; c < pl.ncomp; ++c)
            for (int64_t k = pl.comp_patch_beg[c]; k < pl.comp_patch_beg[c + 1]; ++k) pcomp[k] = c;
        int last = 0;
        for (int64_t l = 0; l < pl.n_lambda; ++l) {
            const int c = pcomp[pos_patch(pl.lam_plus[l])];
            if (c < last) throw Error(IETI_EINVAL, "internal: multipliers not ordered by problem");
            last = c;
            pl.comp_lam_beg[c + 1] = l + 1;
        }
        for (int c = 0; c < pl.ncomp; ++c) pl.comp_lam_beg[c + 1] = std::max(pl.comp_lam_beg[c + 1], pl.comp_lam_beg[c]);
        for (int c = 0; c < pl.ncomp; ++c) {
            int64_t q = 0, t = 0;
            for (int64_t k = pl.comp_patch_beg[c]; k < pl.comp_patch_beg[c + 1]; ++k) {
                q += pl.patches[k].n_qp;
                t += pl.patches[k].lv[0].n;
            }
            pl.comp_qp_beg[c + 1] = pl.comp_qp_beg[c] + q;
            pl.comp_torn_beg[c + 1] = pl.comp_torn_beg[c] + t;
        }
    }
    return P.release();
}

}  // namespace ieti

// ----------------------------------------------------------------------------
// C ABI: host-only planning entry points

using namespace ieti;

extern "C" {

void ieti_default_options(ieti_options* opt) {
    if (opt) default_options(opt);
}

int ieti_plan_create(const ieti_patch* patches, int32_t n_patches, const double* primal_vertices,
                     int32_t n_primal_vertices, const ieti_options* opt, ieti_plan** out) {
    if (!out) return IETI_EINVAL;
    *out = nullptr;
    try {
        *out = reinterpret_cast<ieti_plan*>(build_plan(patches, n_patches, primal_vertices, n_primal_vertices, opt));
        return IETI_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return IETI_ENOMEM;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return IETI_EINVAL;
    }
}

void ieti_plan_destroy(ieti_plan* plan) { delete reinterpret_cast<Plan*>(plan); }

int ieti_plan_sizes(const ieti_plan* plan, int64_t* ndof_torn, int64_t* ndof_global, int64_t* n_lambda,
                    int64_t* n_primal, int64_t* n_qp, int32_t* max_levels) {
    if (!plan) return IETI_EINVAL;
    const Plan& p = *reinterpret_cast<const Plan*>(plan);
    if (ndof_torn) *ndof_torn = p.ndof_torn;
    if (ndof_global) *ndof_global = p.ndof_global;
    if (n_lambda) *n_lambda = p.n_lambda;
    if (n_primal) *n_primal = p.n_primal;
    if (n_qp) *n_qp = p.n_qp;
    if (max_levels) *max_levels = p.max_levels;
    return IETI_OK;
}

int ieti_plan_array(const ieti_plan* plan, int32_t which, int32_t patch, int32_t level, void* out, int64_t* count) {
    if (!plan || !count) return IETI_EINVAL;
    const Plan& p = *reinterpret_cast<const Plan*>(plan);
    auto emit = [&](const void* src, int64_t cnt, size_t elem) {
        if (out) std::memcpy(out, src, (size_t)cnt * elem);
        *count = cnt;
        return IETI_OK;
    };
    if (which == IETI_ARR_LAMBDA_MAP) {
        std::vector<int64_t> v(2 * p.n_lambda);
        for (int64_t l = 0; l < p.n_lambda; ++l) { v[2 * l] = p.lam_plus[l]; v[2 * l + 1] = p.lam_minus[l]; }
        return emit(v.data(), (int64_t)v.size(), sizeof(int64_t));
    }
    if (patch < 0 || patch >= p.N) return IETI_EINVAL;
    const Patch& pa = p.patches[patch];
    if (which == IETI_ARR_MASKS) {
        int32_t v[3] = {(int32_t)pa.bside, (int32_t)(pa.pcorner | pa.dcorner), (int32_t)pa.lv.size()};
        return emit(v, 3, sizeof(int32_t));
    }
    if (which == IETI_ARR_QP_WEIGHT) return emit(pa.qpw.data(), (int64_t)pa.qpw.size(), sizeof(double));
    if (which == IETI_ARR_PRIMAL_MAP) return emit(pa.primal_global.data(), (int64_t)pa.primal_global.size(), sizeof(int64_t));
    if (which == IETI_ARR_BAND) {
        if (level < 0 || level > 1 || pa.band[level].empty()) return IETI_EINVAL;
        return emit(pa.band[level].data(), (int64_t)pa.band[level].size(), sizeof(double));
    }
    if (which == IETI_ARR_TENSOR_U || which == IETI_ARR_TENSOR_LAMBDA || which == IETI_ARR_TENSOR_PARAMS) {
        const int mode = which == IETI_ARR_TENSOR_PARAMS ? level : level >> 8, d = level & 255;
        if (mode < 0 || mode > 1 || pa.ts[mode].U[0].empty()) return IETI_EINVAL;
        const Patch::Tensor& T = pa.ts[mode];
        if (which == IETI_ARR_TENSOR_PARAMS) {
            double v[5] = {(double)T.Pd[0], (double)T.Pd[1], T.shift, T.tau, (double)T.Pd[2]};
            return emit(v, 5, sizeof(double));
        }
        if (d < 0 || d >= p.dim) return IETI_EINVAL;
        if (which == IETI_ARR_TENSOR_U) return emit(T.U[d].data(), (int64_t)T.U[d].size(), sizeof(double));
        return emit(T.lam[d].data(), (int64_t)T.lam[d].size(), sizeof(double));
    }
    int lev = which == IETI_ARR_PROLONG ? (level & 255) : level;
    if (lev < 0 || lev >= (int)pa.lv.size()) return IETI_EINVAL;
    const Level& L = pa.lv[lev];
    switch (which) {
    case IETI_ARR_STENCIL: return emit(L.coef.data(), (int64_t)L.coef.size(), sizeof(double));
    case IETI_ARR_STENCIL_OFFS: return emit(L.offs.data(), (int64_t)L.offs.size(), sizeof(int32_t));
    case IETI_ARR_SHAPE: return emit(L.M, 3, sizeof(int32_t));
    case IETI_ARR_LMAX: return emit(L.lmax, 2, sizeof(double));
    case IETI_ARR_PROLONG: {
        int d = level >> 8;
        if (d < 0 || d >= p.dim || L.P[d].empty()) return IETI_EINVAL;
        return emit(L.P[d].data(), (int64_t)L.P[d].size(), sizeof(double));
    }
    default: return IETI_EINVAL;
    }
}

int ieti_quadrature_points(const ieti_patch* patches, int32_t n, double* x, int64_t* n_qp) {
    if (!patches || n <= 0) return IETI_EINVAL;
    try {
        const int dim = patches[0].dim;
        int64_t o = 0;
        for (int k = 0; k < n; ++k) {
            validate_patch(patches[k], dim, k);
            const ieti_patch& ip = patches[k];
            std::vector<double> t[3];
            int M[3] = {1, 1, 1};
            DirTable dt[3];
            for (int d = 0; d < dim; ++d) {
                t[d].assign(ip.knots[d], ip.knots[d] + ip.n_knots[d]);
                M[d] = ip.n_knots[d] - ip.degree[d] - 1;
                dt[d] = make_dir(t[d], ip.degree[d], t[d], ip.degree[d]);
            }
            const int Q0 = dt[0].Q, Q1 = dt[1].Q, Q2 = dim == 3 ? dt[2].Q : 1;
            const int pg2 = dim == 3 ? ip.degree[2] : 0;
            if (x) {
                for (int q2 = 0; q2 < Q2; ++q2)
                    for (int q1 = 0; q1 < Q1; ++q1)
                        for (int q0 = 0; q0 < Q0; ++q0) {
                            const int qd[3] = {q0, q1, q2};
                            double xx[3] = {0, 0, 0};
                            for (int a2 = 0; a2 <= pg2; ++a2)
                                for (int a1 = 0; a1 <= ip.degree[1]; ++a1)
                                    for (int a0 = 0; a0 <= ip.degree[0]; ++a0) {
                                        const int g0 = dt[0].gfirst[qd[0]] + a0, g1 = dt[1].gfirst[qd[1]] + a1;
                                        const int g2 = dim == 3 ? dt[2].gfirst[qd[2]] + a2 : 0;
                                        double bv = dt[0].G[(size_t)qd[0] * (ip.degree[0] + 1) + a0] *
                                                    dt[1].G[(size_t)qd[1] * (ip.degree[1] + 1) + a1];
                                        if (dim == 3) bv *= dt[2].G[(size_t)qd[2] * (ip.degree[2] + 1) + a2];
                                        const int64_t i = lin(M, g0, g1, g2);
                                        for (int c = 0; c < dim; ++c) xx[c] += ip.ctrl[i * dim + c] * bv;
                                    }
                            for (int c = 0; c < dim; ++c) x[o * dim + c] = xx[c];
                            ++o;
                        }
            } else {
                o += (int64_t)Q0 * Q1 * Q2;
            }
        }
        if (n_qp) *n_qp = o;
        return IETI_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return IETI_EINVAL;
    }
}

int ieti_plan_quadrature(const ieti_plan* plan, double* x) {
    if (!plan || !x) return IETI_EINVAL;
    const Plan& p = *reinterpret_cast<const Plan*>(plan);
    int64_t o = 0;
    for (const auto& pa : p.patches) {
        std::memcpy(x + o, pa.qpx.data(), pa.qpx.size() * sizeof(double));
        o += (int64_t)pa.qpx.size();
    }
    return IETI_OK;
}

}  // extern "C"
