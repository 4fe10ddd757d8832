// Device runtime of the IETI-DP solver: uploads a plan, builds the primal
// basis, and runs ieti_solve (right-hand side d, outer CG on F lambda = d
// with the scaled Dirichlet preconditioner, recovery of u).
//
//   F p   = B K~^{-1} B^T p                 (Sec. 2, eq. (4))
//   K~^{-1} g = [K_rr^{-1} g_r - Psi_E C_E K_rr^{-1} g_r] + Psi S_PiPi^{-1} Psi^T g
//         (local Neumann problem of eq. (7): unconstrained minimiser, then the
//          energy-minimising projection; primal part with the basis of eq. (6))
//   M^{-1} r = B_D S B_D^T r,  S v = K v - K_{.I} K_II^{-1} K_{I.} v  (Sec. 2, 3.1)
//
// K_rr is the patch stiffness with boundary coefficients and primal
// vertices removed, positive definite on every patch.  Inexact local solves:
// flexible CG (FP64) preconditioned by one multigrid V-cycle (FP32 or FP64),
// to a relative residual inner_tol (Sec. 3.2 / Sec. 4: MG-MG).  The
// Dirichlet problems in the preconditioner use prec_vcycles V-cycles.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "kernels.h"
#include "tensor_smoother.h"
#include "plan.h"

namespace ieti {
const char* last_error();
}

namespace ieti {

#define HIPCHECK(x)                                                                                    \
    do {                                                                                               \
        hipError_t e_ = (x);                                                                           \
        if (e_ != hipSuccess) throw Error(IETI_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

static inline int64_t align64(int64_t x) { return (x + 63) & ~int64_t(63); }
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
static inline unsigned tile_grid(int ntiles) { return (unsigned)(8 * ((ntiles + 7) / 8)); }

// one kernel instance per degree class (see degree_class)

// Launch groups over class-ordered tiles: {class, first tile, end tile}.  With
// multi set and at least two 2D classes present, the 2D classes 0..8 (whose
// tiles are contiguous) form one group, class MULTI_2D.
constexpr int MULTI_2D = -2;

static std::vector<std::array<int, 3>> launch_groups(const int* beg, const int* end, bool multi) {
    std::vector<std::array<int, 3>> g;
    int n2d = 0;
    for (int c = 0; c <= 8; ++c) n2d += end[c] > beg[c] ? 1 : 0;
    int c0 = 0;
    if (multi && n2d >= 2) {
        g.push_back({MULTI_2D, beg[0], end[8]});
        c0 = 9;
    }
    for (int c = c0; c <= NCLASS; ++c)
        if (end[c] > beg[c]) g.push_back({c, beg[c], end[c]});
    return g;
}

// With ev0/ev1 set, the launch records them at kernel start and end (profiling).
// dynamic LDS a launch may take without raising the kernel's limit
constexpr size_t STAGE_X_MAX_BYTES = 65536;

template <typename TC, typename TX, typename TY, int EPI, bool FINE>
static void launch_stencil(int cls, hipStream_t st, const StencilArgs& a, int reach, hipEvent_t ev0 = nullptr,
                           hipEvent_t ev1 = nullptr) {
    if (cls == MULTI_2D) {   // the finest level's 2D classes in one launch (always staged)
        const size_t lds = (size_t)(TILE + 2 * reach) * sizeof(TX);
        if (ev0)
            hipExtLaunchKernelGGL((k_stencil_2d<TC, TX, TY, EPI>), dim3(tile_grid(a.ntiles)), dim3(TILE), lds, st, ev0,
                                  ev1, 0, a);
        else
            hipLaunchKernelGGL((k_stencil_2d<TC, TX, TY, EPI>), dim3(tile_grid(a.ntiles)), dim3(TILE), lds, st, a);
        return;
    }
#define IETI_LS(A, B, C)                                                                                              \
    do {                                                                                                              \
        const size_t lds = stencil_stages_x<A, C, FINE>() ? (size_t)(TILE + 2 * reach) * sizeof(TX) : 0;          \
        if (ev0)                                                                                                      \
            hipExtLaunchKernelGGL((k_stencil<A, B, C, TC, TX, TY, EPI, FINE>), dim3(tile_grid(a.ntiles)), dim3(TILE), \
                                  lds, st, ev0, ev1, 0, a);                                                           \
        else                                                                                                          \
            hipLaunchKernelGGL((k_stencil<A, B, C, TC, TX, TY, EPI, FINE>), dim3(tile_grid(a.ntiles)), dim3(TILE),    \
                               lds, st, a);                                                                           \
    } while (0)
    IETI_CLASS_SWITCH(cls, IETI_LS)
#undef IETI_LS
}

template <typename T, bool STAGE, int FAM>
static void launch_vcoarse(hipStream_t st, const CoarseArgs& a, size_t lds_bytes, bool set_attr, hipEvent_t ev0,
                           hipEvent_t ev1) {
    if (set_attr)
        HIPCHECK(hipFuncSetAttribute((const void*)k_vcoarse<T, STAGE, FAM>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
    else if (ev0)
        hipExtLaunchKernelGGL((k_vcoarse<T, STAGE, FAM>), dim3(a.nlist), dim3((vc_threads<T, FAM>())), lds_bytes, st,
                              ev0, ev1, 0, a);
    else
        hipLaunchKernelGGL((k_vcoarse<T, STAGE, FAM>), dim3(a.nlist), dim3((vc_threads<T, FAM>())), lds_bytes, st, a);
}

template <typename T>
static void launch_vcoarse(int fam, bool stage, hipStream_t st, const CoarseArgs& a, size_t lds_bytes, bool set_attr,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
    if (fam == 0) {
        if (stage) launch_vcoarse<T, true, 0>(st, a, lds_bytes, set_attr, ev0, ev1);
        else launch_vcoarse<T, false, 0>(st, a, lds_bytes, set_attr, ev0, ev1);
    } else {
        if (stage) launch_vcoarse<T, true, 1>(st, a, lds_bytes, set_attr, ev0, ev1);
        else launch_vcoarse<T, false, 1>(st, a, lds_bytes, set_attr, ev0, ev1);
    }
}

template <typename T>
static void launch_restrict(int cls, hipStream_t st, const PatchLev* Lf, const PatchLev* Lc, const Tile* tiles,
                            int nt, const int32_t* rlo, const T* rval, const T* rf, T* bc, int mode, const int* act) {
    if (cls == MULTI_2D) {
        hipLaunchKernelGGL((k_restrict<-2, 0, 0, T>), dim3(tile_grid(nt)), dim3(TILE), 0, st, Lf, Lc, tiles, nt, rlo,
                           rval, rf, bc, mode, act);
        return;
    }
#define IETI_LR(A, B, C)                                                                                      \
    hipLaunchKernelGGL((k_restrict<A, B, C, T>), dim3(tile_grid(nt)), dim3(TILE), 0, st, Lf, Lc, tiles, nt, rlo, \
                       rval, rf, bc, mode, act)
    IETI_CLASS_SWITCH(cls, IETI_LR)
#undef IETI_LR
}

template <typename T>
static void launch_prolong(int cls, hipStream_t st, const PatchLev* Lf, const PatchLev* Lc, const Tile* tiles, int nt,
                           const int32_t* plo, const T* pval, const T* ec, T* xf, int mode, const int* act) {
    if (cls == MULTI_2D) {
        hipLaunchKernelGGL((k_prolong<-2, 0, 0, T>), dim3(tile_grid(nt)), dim3(TILE), 0, st, Lf, Lc, tiles, nt, plo,
                           pval, ec, xf, mode, act);
        return;
    }
#define IETI_LP(A, B, C)                                                                                     \
    hipLaunchKernelGGL((k_prolong<A, B, C, T>), dim3(tile_grid(nt)), dim3(TILE), 0, st, Lf, Lc, tiles, nt, plo, \
                       pval, ec, xf, mode, act)
    IETI_CLASS_SWITCH(cls, IETI_LP)
#undef IETI_LP
}

// ------------------------------------------------------------------ device memory arena

// Device memory of a server: the blocks of a finished request are cached and handed to later requests, so
// that a request costs no hipMalloc/hipFree once the pool has warmed up (hipFree waits for the whole device
// and stalls the other slots).  Blocks come in size classes of 1/8 of a power of two (at least 64 KiB; at
// most 12.5 % over the request) and are reused only for the same class.  When a new block would take the
// pool's bytes past the cap (the server's HBM budget; 0: none), or hipMalloc fails, the cached blocks are
// released first.  A block is returned only after the work that used it has finished (the server
// synchronizes the request's stream before it destroys the request's state).
struct DevicePool {
    std::mutex mu;
    std::multimap<size_t, void*> cached;
    std::unordered_map<void*, size_t> size_of;
    size_t total = 0, cap = 0;
    static size_t size_class(size_t b) {
        size_t c = std::max<size_t>(b, (size_t)64 << 10), pw = 1;
        while (pw * 2 <= c) pw *= 2;
        const size_t step = pw / 8;
        return (c + step - 1) / step * step;
    }
    void release_locked() {
        for (auto& kv : cached) {
            (void)hipFree(kv.second);
            total -= kv.first;
            size_of.erase(kv.second);
        }
        cached.clear();
    }
    void* get(size_t b) {
        const size_t c = size_class(b);
        {
            std::lock_guard<std::mutex> lk(mu);
            auto it = cached.find(c);
            if (it != cached.end()) {
                void* p = it->second;
                cached.erase(it);
                return p;
            }
            if (cap && total + c > cap) release_locked();
        }
        void* p = nullptr;
        if (hipMalloc(&p, c) != hipSuccess) {
            {
                std::lock_guard<std::mutex> lk(mu);
                release_locked();
            }
            if (hipMalloc(&p, c) != hipSuccess) return nullptr;
        }
        std::lock_guard<std::mutex> lk(mu);
        size_of[p] = c;
        total += c;
        return p;
    }
    void put(void* p) {
        std::lock_guard<std::mutex> lk(mu);
        cached.emplace(size_of.at(p), p);
    }
    // pinned host blocks (a request's scalars read back by the host), cached the same way (hipHostFree also
    // waits for the device)
    std::multimap<size_t, void*> cached_h;
    std::unordered_map<void*, size_t> size_h;
    void* get_host(size_t b) {
        const size_t c = std::max<size_t>(b, 4096);
        {
            std::lock_guard<std::mutex> lk(mu);
            auto it = cached_h.lower_bound(c);
            if (it != cached_h.end() && it->first <= 4 * c) {
                void* p = it->second;
                cached_h.erase(it);
                return p;
            }
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, c) != hipSuccess) return nullptr;
        std::lock_guard<std::mutex> lk(mu);
        size_h[p] = c;
        return p;
    }
    void put_host(void* p) {
        std::lock_guard<std::mutex> lk(mu);
        cached_h.emplace(size_h.at(p), p);
    }
    ~DevicePool() {
        for (auto& kv : size_of) (void)hipFree(kv.first);
        for (auto& kv : size_h) (void)hipHostFree(kv.first);
    }
};

// the pool of the server whose worker runs on this thread (null elsewhere: plain hipMalloc/hipFree)
static thread_local DevicePool* t_pool = nullptr;

static void* dev_alloc(size_t b) {
    void* p = nullptr;
    if (t_pool) return t_pool->get(b);
    return hipMalloc(&p, b) == hipSuccess ? p : nullptr;
}

struct Arena {
    std::vector<void*> ptrs;
    size_t bytes = 0;
    size_t budget = 0;
    DevicePool* pool = t_pool;
    ~Arena() {
        for (void* p : ptrs) {
            if (pool) pool->put(p);
            else (void)hipFree(p);
        }
    }
    template <typename T>
    T* alloc(int64_t n, hipStream_t st, bool zero = true) {
        if (n <= 0) n = 1;
        size_t b = (size_t)n * sizeof(T);
        if (budget && bytes + b > budget) throw Error(IETI_ENOMEM, "device memory budget exceeded");
        void* p = pool ? pool->get(b) : dev_alloc(b);
        if (!p) throw Error(IETI_ENOMEM, "hipMalloc failed");
        ptrs.push_back(p);
        bytes += b;
        if (zero) HIPCHECK(hipMemsetAsync(p, 0, b, st));
        return (T*)p;
    }
    // gives one block back before the arena ends, once the work queued on st has finished
    void release(void* p, size_t b, hipStream_t st) {
        auto it = std::find(ptrs.begin(), ptrs.end(), p);
        if (it == ptrs.end()) return;
        HIPCHECK(hipStreamSynchronize(st));
        ptrs.erase(it);
        bytes -= b;
        if (pool) pool->put(p);
        else (void)hipFree(p);
    }
    template <typename T>
    T* upload(const std::vector<T>& v, hipStream_t st) {
        T* p = alloc<T>((int64_t)v.size(), st, false);
        if (!v.empty()) HIPCHECK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
        return p;
    }
};

// ------------------------------------------------------------------ solver base

// Event-bracketed launches of the profiled kernel classes.
struct KProf {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    std::vector<std::pair<int, double>> pending;   // (class, bytes) of used pool entries
    int64_t launches[IETI_KPROF_COUNT] = {};
    double ms[IETI_KPROF_COUNT] = {};
    double bytes[IETI_KPROF_COUNT] = {};
    ~KProf() {
        for (auto& e : pool) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    }
    void reset() {
        for (int c = 0; c < IETI_KPROF_COUNT; ++c) launches[c] = 0, ms[c] = 0, bytes[c] = 0;
    }
    std::pair<hipEvent_t, hipEvent_t> next(int cls, double b) {
        size_t i = pending.size();
        if (i == pool.size()) {
            hipEvent_t a, c;
            HIPCHECK(hipEventCreate(&a));
            HIPCHECK(hipEventCreate(&c));
            pool.push_back({a, c});
        }
        pending.push_back({cls, b});
        return pool[i];
    }
    // after a stream synchronisation: fold the recorded pairs into the totals
    void collect() {
        for (size_t i = 0; i < pending.size(); ++i) {
            float t = 0.f;
            HIPCHECK(hipEventElapsedTime(&t, pool[i].first, pool[i].second));
            int c = pending[i].first;
            launches[c] += 1;
            ms[c] += t;
            bytes[c] += pending[i].second;
        }
        pending.clear();
    }
};

struct SolverBase {
    KProf prof;
    virtual ~SolverBase() = default;
    virtual void setup() = 0;
    virtual int solve(const double* f_qp, double* u, ieti_stats* st) = 0;
    // ieti_solve_noalloc: the same solve with its per-solve scratch in the static array `scratch`
    virtual int solve_noalloc(const double* f_qp, double* u, ieti_stats* st) = 0;
    double* noalloc_base = nullptr;   // device address of `scratch` on the handle's device
    // statistics and status of every problem of the last solve (several in a serving batch)
    std::vector<ieti_stats> comp_stats;
    std::vector<int> comp_rc;
    virtual void quadrature(double* x, bool on_device) = 0;
    std::unique_ptr<Plan> plan;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    Arena arena;
};

struct DevLevel {
    // per degree class: sum of n and of n * nst (half-stencil words) over the launch's patches
    double words_all[NCLASS + 1] = {0}, words_smooth[NCLASS + 1] = {0};
    double st_all[NCLASS + 1] = {0}, st_smooth[NCLASS + 1] = {0};
    // per degree class: largest linear stencil reach (the guard length; x window staged in LDS)
    int reach[NCLASS + 1] = {0};
    std::vector<PatchLev> hL;
    PatchLev* L = nullptr;
    int64_t len = 0, clen = 0;
    std::vector<Tile> h_all, h_smooth;
    Tile* tiles_all = nullptr;
    Tile* tiles_smooth = nullptr;
    int nt_all = 0, nt_smooth = 0;
    // tiles of each degree class are contiguous: [cls_beg[c], cls_end[c]) in tiles_all / tiles_smooth
    int cls_beg_all[NCLASS + 1] = {0}, cls_end_all[NCLASS + 1] = {0};
    int cls_beg_sm[NCLASS + 1] = {0}, cls_end_sm[NCLASS + 1] = {0};
    double* cheb = nullptr;                       // (s1, s2) per (patch-level, mode, step)
    std::vector<int32_t> h_coarse;
    int32_t* coarse_list = nullptr;
    int n_coarse = 0;
    int32_t* plo = nullptr;
    int32_t* rlo = nullptr;
    void* pval = nullptr;
    void* rval = nullptr;
    void* coefT = nullptr;
    void* inv = nullptr;
    void *vb = nullptr, *vx = nullptr, *vxa = nullptr, *vd = nullptr, *vr = nullptr;
};

template <typename T>
struct Solver : SolverBase {
    std::vector<DevLevel> lev;
    int N = 0, dim = 2, nlev = 0;
    int cheb_m = 2;     // Chebyshev degree per smoothing phase, finest level
    int cheb_mc = 2;    // coarse levels
    bool stage_all0 = false;   // every finest-level smoothing tile runs a staged (x window in LDS) instance
    bool stage_fine = true;    // finest-level tiles stage their x window in LDS where it fits (autotuned)
    double cheb_hi = 1.1;
    // tensor-product smoother of the finest level (options.smoother): per mode and patch the factors of
    // the fast diagonalisation, the forward transform's scratch, the largest padded sizes
    bool fd_on = false;
    FdInfo* fd_info[2] = {nullptr, nullptr};
    double *fd_U = nullptr, *fd_lam = nullptr, *fd_z = nullptr, *fd_z2 = nullptr;
    float *fd_U32 = nullptr, *fd_z32 = nullptr, *fd_z232 = nullptr;   // 2D with FP32 V-cycles: FP32 copies
    int fd_p0max = 0, fd_p1max = 0, fd_p2max = 0, fd_tiles2 = 0, fd_tiles3 = 0;
    // level 0 FP64
    double* coef64 = nullptr;
    int64_t len0 = 0;
    double *f64 = nullptr, *b64 = nullptr, *e64 = nullptr, *w64 = nullptr, *s64 = nullptr, *u64 = nullptr;
    double *fx = nullptr, *fr = nullptr, *fd = nullptr, *fq = nullptr;
    T *rT = nullptr, *zT = nullptr, *bT = nullptr, *xIT = nullptr, *x2T = nullptr, *r2T = nullptr;
    double* partial = nullptr;
    int32_t *tile_beg = nullptr, *tile_end = nullptr;
    double *bb = nullptr, *dq = nullptr, *beta = nullptr, *alpha = nullptr;
    int *active = nullptr, *its = nullptr, *nactive = nullptr, *brk = nullptr;
    int* h_nactive = nullptr;   // pinned
    // jump operators
    int64_t nslots = 0, nlam = 0;
    int64_t *slot_dev = nullptr, *slot_ptr = nullptr, *slot_lam = nullptr;
    double *slot_wB = nullptr, *slot_wBD = nullptr;
    int32_t* slot_patch = nullptr;
    int64_t* row_ptr = nullptr;
    int64_t *lam_plus = nullptr, *lam_minus = nullptr;
    double* lam_wBD = nullptr;
    // primal
    int64_t npi = 0;
    int npk_max = 0;
    int32_t* npk = nullptr;
    int64_t *Rk = nullptr, *unit_dev = nullptr, *edge_ptr = nullptr, *edge_dev = nullptr;
    int64_t *pri_ptr = nullptr, *pri_patch = nullptr, *pri_local = nullptr;
    double *psi = nullptr, *psiG = nullptr, *Sinv = nullptr, *upi = nullptr;
    double *cbuf = nullptr, *ebuf = nullptr, *coefbuf = nullptr;
    // groups and output
    int64_t ngroups = 0;
    int64_t *grp_ptr = nullptr, *grp_dev = nullptr;
    int64_t* torn_off = nullptr;
    // load vector
    PatchQ* PQ = nullptr;
    double *basis = nullptr, *qpw = nullptr;
    double* qtmp = nullptr;            // load vector: intermediates of the sum factorisation
    int64_t qtmp_len = 0;
    int64_t qc_grid[3] = {1, 1, 1};    // work-groups per patch of the contraction passes
    double* qpx = nullptr;
    // lambda space
    double *lam = nullptr, *lr = nullptr, *lz = nullptr, *lp = nullptr, *lq = nullptr, *ltmp = nullptr;
    double* sc = nullptr;
    double* pcgp = nullptr;   // the multi-work-group outer CG's partial sums: 2 PCG_NB per problem
    double* h_sc = nullptr;    // pinned
    // exact local solves (banded Cholesky factors, blocked triangular solves): Neumann problems
    // (exact), also the preconditioner's Dirichlet problems (prec_exact)
    bool exact = false, prec_exact = false;
    int64_t* band_off = nullptr;
    int32_t* band_b = nullptr;
    double* band = nullptr;
    size_t band_lds = 0;
    int band_bmax = 0;   // widest band of the exact local solves (the register-resident solve takes b <= 512)
    // fused coarse V-cycle: one work-group per patch for levels >= fuse_l0 (nlev: none)
    int fuse_l0 = 0;
    bool fuse_stage = false;
    int32_t* chain = nullptr;
    std::vector<int32_t> h_plist[2];   // patches of the fused kernel per class family, largest chain first
    int32_t* plist[2] = {nullptr, nullptr};
    size_t vc_lds[2] = {0, 0};
    double vc_bytes[2] = {0.0, 0.0};   // algorithmic bytes of one launch over all patches of a family
    // statistics of the current solve
    int64_t inner_calls = 0, inner_sum = 0;
    int inner_max = 0;
    std::vector<int> h_its;
    int hint_solve = 1, hint_basis = 1;   // inner iterations of the last batched solve per tolerance

    // independent problems (a serving batch; one for ieti_solve): multiplier and patch ranges, stop flags,
    // and the statistics and status of each problem from the last solve
    int ncomp = 1;
    std::vector<int64_t> h_comp_lam;
    int64_t *comp_lam = nullptr, *comp_patch = nullptr;
    int* done_dev = nullptr;
    int* h_done = nullptr;   // pinned
    std::vector<double> comp_gres;
    // degree-1 coarse levels (options.coarse_degree = 1): the finest level's L2-projection transfer
    bool l2_on = false;
    double* l2_mchol = nullptr;          // banded Cholesky factors of the 1D parametric mass matrices
    int32_t* l2_list = nullptr;          // level-0 patch-levels with a coarse level
    int l2_n = 0;
    size_t l2_lds = 0;
    T* l2_tmp = nullptr;                 // level-0 scratch vector
    // floating patches (K singular, edge constraints only): their list and the penalty gamma per patch
    int n_float = 0;
    int32_t* float_list = nullptr;
    double* float_gam = nullptr;

    // ---------------------------------------------------------------- launch helpers
    void sync() { HIPCHECK(hipStreamSynchronize(stream)); }
    void check_launch() { HIPCHECK(hipGetLastError()); }

    template <typename TC, typename TX, typename TY, int EPI>
    void stencil(int l, bool smooth_only, int mode, const void* coef, const void* x, void* y, const void* b, void* d,
                 const int* act, double alpha_, int cheb_k, double* part = nullptr, const double* r64 = nullptr,
                 const double* dotq = nullptr, double* dpart = nullptr) {
        DevLevel& D = lev[l];
        const int ntot = smooth_only ? D.nt_smooth : D.nt_all;
        if (ntot == 0) return;
        if (cheb_k >= KMAX) throw Error(IETI_ENOTSUP, "Chebyshev degree too high");
        StencilArgs a{};
        a.L = D.L;
        a.mode = mode;
        a.coef = coef;
        a.x = x;
        a.y = y;
        a.b = b;
        a.d = d;
        a.active = act;
        a.alpha = alpha_;
        a.cheb_k = cheb_k;
        a.cheb = D.cheb;
        a.partial = part;
        a.r64 = r64;
        a.dotq = dotq;
        a.dpart = dpart;
        int pcls = -1;
        if (prof.on && l == 0) {
            if (EPI == EPI_CHEB) pcls = IETI_KPROF_SMOOTH_FINE;
            else if (EPI == EPI_DOTS) pcls = IETI_KPROF_APPLY64;
            else if (EPI == EPI_RESID && smooth_only) pcls = IETI_KPROF_RESID_FINE;
        }
        const Tile* base = smooth_only ? D.tiles_smooth : D.tiles_all;
        const int* beg = smooth_only ? D.cls_beg_sm : D.cls_beg_all;
        const int* end = smooth_only ? D.cls_end_sm : D.cls_end_all;
        int reach2d = 0;
        for (int c = 0; c <= 8; ++c) reach2d = std::max(reach2d, D.reach[c]);
        const bool multi = l == 0 && stage_fine && (size_t)(TILE + 2 * reach2d) * sizeof(TX) <= STAGE_X_MAX_BYTES;
        for (const auto& g : launch_groups(beg, end, multi)) {
            const int c = g[0];
            a.tiles = base + g[1];
            a.ntiles = g[2] - g[1];
            std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
            if (pcls >= 0) {
                // algorithmic bytes: every vector the epilogue touches and the half stencil, once per coefficient
                double n = 0.0, nst = 0.0;
                for (int cc = c == MULTI_2D ? 0 : c; cc <= (c == MULTI_2D ? 8 : c); ++cc) {
                    n += smooth_only ? D.words_smooth[cc] : D.words_all[cc];
                    nst += smooth_only ? D.st_smooth[cc] : D.st_all[cc];
                }
                const double vec_words = EPI == EPI_CHEB ? (cheb_k > 0 ? 5.0 : 4.0) : 3.0;
                double bytes = nst * sizeof(TC) + n * (vec_words - 1.0) * sizeof(TY) + n * sizeof(TX);
                if (EPI == EPI_DOTS) bytes = nst * sizeof(TC) + n * (sizeof(TX) + sizeof(TY) + sizeof(double));
                ev = prof.next(pcls, bytes);
            }
            const int reach = c == MULTI_2D ? reach2d : D.reach[c];
            const bool window_fits = (size_t)(TILE + 2 * reach) * sizeof(TX) <= STAGE_X_MAX_BYTES;
            if constexpr (EPI == EPI_CHEB0) {   // staged finest-level instances only (vcycle checks stage_all0)
                launch_stencil<TC, TX, TY, EPI, true>(c, stream, a, reach, ev.first, ev.second);
            } else {
                if (l == 0 && window_fits && stage_fine)
                    launch_stencil<TC, TX, TY, EPI, true>(c, stream, a, reach, ev.first, ev.second);
                else
                    launch_stencil<TC, TX, TY, EPI, false>(c, stream, a, reach, ev.first, ev.second);
            }
            check_launch();
        }
    }
    template <typename V>
    void fill(V* p, int64_t n, V v) {
        hipLaunchKernelGGL(k_fill<V>, dim3(nblk(n, 256)), dim3(256), 0, stream, p, n, v);
        check_launch();
    }

    // ---------------------------------------------------------------- multigrid V-cycle
    // x0 = V(b0) on all patches (mode N or D); the result lands in x0.  Levels
    // below fuse_l0 run as batched launches over all patches; from fuse_l0 on,
    // one work-group per patch runs the rest of the cycle (k_vcoarse).
    // finest level, patches with tensor-smoother data: x = tau P r (set) or x += tau P r
    void fd_smooth(int mode, const int* act, const T* r, T* x, bool set) {
        if (dim == 3) {   // six axis contractions through the two scratch buffers
            FdArgs a{lev[0].L, fd_info[mode], fd_U, fd_lam, fd_z, act, mode, N, fd_z2, nullptr, nullptr, nullptr};
            const dim3 g((fd_tiles3 + FD3_THREADS / WAVE - 1) / (FD3_THREADS / WAVE), N), b(FD3_THREADS);
            // axes 0 and 1 fused per plane and column block (intermediate column in LDS), axis 2 on its own
            const int ncb = fd_p0max / 16;
            const dim3 gp(ncb * fd_p2max, N);
            const size_t lds = (size_t)fd_p1max * FD2C_LD * sizeof(double);
            hipLaunchKernelGGL(k_fd3_fwd01<T>, gp, b, lds, stream, a, r, ncb);
            check_launch();
            hipLaunchKernelGGL((k_fd3_axn<2, true, true>), g, b, 0, stream, a, (const double*)fd_z2, fd_z);
            check_launch();
            hipLaunchKernelGGL((k_fd3_axn<2, false, false>), g, b, 0, stream, a, (const double*)fd_z, fd_z2);
            check_launch();
            if (set) hipLaunchKernelGGL((k_fd3_bwd10<T, true>), gp, b, lds, stream, a, x, ncb);
            else hipLaunchKernelGGL((k_fd3_bwd10<T, false>), gp, b, lds, stream, a, x, ncb);
            check_launch();
            return;
        }
        // 2D: four block products (W, Z, T, then the update of x), the blocks of all patches in each grid
        FdArgs a{lev[0].L, fd_info[mode], fd_U, fd_lam, fd_z, act, mode, N, fd_z2, fd_U32, fd_z32, fd_z232};
        const dim3 g((fd_tiles2 + FD2_THREADS / WAVE - 1) / (FD2_THREADS / WAVE), N), b(FD2_THREADS);
        if (fd_p1max <= FD2C_MAXP) {   // the products fused in pairs per column block (intermediate in LDS)
            const dim3 gc(fd_p0max / 16, N), bc(FD2C_THREADS);
            const size_t lds = (size_t)fd_p1max * FD2C_LD * sizeof(T);
            hipLaunchKernelGGL(k_fd2_fwd<T>, gc, bc, lds, stream, a, r);
            check_launch();
            if (set)
                hipLaunchKernelGGL((k_fd2_bwd<T, true>), gc, bc, lds, stream, a, x);
            else
                hipLaunchKernelGGL((k_fd2_bwd<T, false>), gc, bc, lds, stream, a, x);
            check_launch();
            return;
        }
        hipLaunchKernelGGL(k_fd2_w<T>, g, b, 0, stream, a, r);
        check_launch();
        hipLaunchKernelGGL(k_fd2_z<T>, g, b, 0, stream, a);
        check_launch();
        hipLaunchKernelGGL(k_fd2_t<T>, g, b, 0, stream, a);
        check_launch();
        if (set)
            hipLaunchKernelGGL((k_fd2_y<T, true>), g, b, 0, stream, a, x);
        else
            hipLaunchKernelGGL((k_fd2_y<T, false>), g, b, 0, stream, a, x);
        check_launch();
    }
    void vcycle(int mode, const int* act, const T* b0, T* x0, const double* dotq = nullptr, double* dpart = nullptr) {
        std::vector<T*> cur(nlev, nullptr);
        int deepest = 0;
        for (int l = 0; l < nlev; ++l) {
            DevLevel& D = lev[l];
            if (l > 0 && l == fuse_l0) {
                vcoarse(l, mode, act);
                cur[l] = (T*)D.vxa;
                deepest = l;
                break;
            }
            const T* B = l == 0 ? b0 : (const T*)D.vb;
            T* S = l == 0 ? (T*)D.vxa : (T*)D.vx;       // start buffer
            T* F = l == 0 ? x0 : (T*)D.vxa;              // buffer holding the final result
            if (D.n_coarse) {
                hipLaunchKernelGGL(k_coarse<T>, dim3(D.n_coarse), dim3(TILE), 0, stream, D.L, D.coarse_list,
                                   D.n_coarse, (const T*)D.inv, B, F, mode, act);
                check_launch();
            }
            cur[l] = F;
            deepest = l;
            if (D.nt_smooth == 0) break;
            // pre-smoothing: Chebyshev from zero (on the finest level the zero start is fused into step 1),
            // or one tensor-smoother step from zero on the finest level
            T* X = S;
            T* XA = F;
            if (l == 0 && fd_on) {
                fd_smooth(mode, act, B, F, true);
                X = F;
            } else {
                const int m = l == 0 ? cheb_m : cheb_mc;
                int k1 = 1;
                if (l == 0 && m >= 2 && stage_all0 && stage_fine) {
                    stencil<T, T, T, EPI_CHEB0>(0, true, mode, D.coefT, nullptr, XA, B, D.vd, act, 0.0, 1);
                    std::swap(X, XA);
                    k1 = 2;
                } else {
                    hipLaunchKernelGGL(k_cheb_zero<T>, dim3(tile_grid(D.nt_smooth)), dim3(TILE), 0, stream, D.L,
                                       D.tiles_smooth, D.nt_smooth, (const T*)D.coefT, B, X, (T*)D.vd, mode, D.cheb,
                                       act);
                    check_launch();
                }
                for (int k = k1; k < m; ++k) {
                    stencil<T, T, T, EPI_CHEB>(l, true, mode, D.coefT, X, XA, B, D.vd, act, 0.0, k);
                    std::swap(X, XA);
                }
            }
            stencil<T, T, T, EPI_RESID>(l, true, mode, D.coefT, X, D.vr, B, nullptr, act, 0.0, 0);
            cur[l] = X;
            DevLevel& C = lev[l + 1];
            if (l == 0 && l2_on) {   // b_c = D_c M_cf M_f^{-1} r_f
                hipLaunchKernelGGL(k_mass_solve<T>, dim3(l2_n), dim3(TILE), l2_lds, stream, D.L, l2_list, l2_n,
                                   (const double*)l2_mchol, (const T*)D.vr, l2_tmp, mode, 0, act);
                check_launch();
                hipLaunchKernelGGL(k_l2_restrict<T>, dim3(tile_grid(C.nt_all)), dim3(TILE), 0, stream, D.L, C.L,
                                   C.tiles_all, C.nt_all, D.rlo, (const T*)D.rval, (const T*)l2_tmp, (T*)C.vb, mode,
                                   act);
                check_launch();
                continue;
            }
            for (const auto& g : launch_groups(C.cls_beg_all, C.cls_end_all, true)) {
                launch_restrict<T>(g[0], stream, D.L, C.L, C.tiles_all + g[1], g[2] - g[1], D.rlo, (const T*)D.rval,
                                   (const T*)D.vr, (T*)C.vb, mode, act);
                check_launch();
            }
        }
        for (int l = deepest - 1; l >= 0; --l) {
            DevLevel& D = lev[l];
            const T* B = l == 0 ? b0 : (const T*)D.vb;
            T* X = cur[l];
            T* A0 = l == 0 ? (T*)D.vxa : (T*)D.vx;   // the level's two x buffers
            T* A1 = l == 0 ? x0 : (T*)D.vxa;
            T* XA = (X == A0) ? A1 : A0;
            if (l == 0 && l2_on) {   // x_f += D_f M_f^{-1} M_fc e_c
                hipLaunchKernelGGL(k_l2_prolong<T>, dim3(tile_grid(D.nt_smooth)), dim3(TILE), 0, stream, D.L,
                                   lev[1].L, D.tiles_smooth, D.nt_smooth, D.plo, (const T*)D.pval,
                                   (const T*)cur[1], l2_tmp, mode, act);
                check_launch();
                hipLaunchKernelGGL(k_mass_solve<T>, dim3(l2_n), dim3(TILE), l2_lds, stream, D.L, l2_list, l2_n,
                                   (const double*)l2_mchol, (const T*)l2_tmp, l2_tmp, mode, 1, act);
                check_launch();
                hipLaunchKernelGGL(k_add_act<T>, dim3(tile_grid(D.nt_smooth)), dim3(TILE), 0, stream, D.L,
                                   D.tiles_smooth, D.nt_smooth, (const T*)l2_tmp, X, act);
                check_launch();
            } else {
                for (const auto& g : launch_groups(D.cls_beg_sm, D.cls_end_sm, true)) {
                    launch_prolong<T>(g[0], stream, D.L, lev[l + 1].L, D.tiles_smooth + g[1], g[2] - g[1], D.plo,
                                      (const T*)D.pval, (const T*)cur[l + 1], X, mode, act);
                    check_launch();
                }
            }
            if (l == 0 && fd_on) {   // one tensor-smoother step
                if (dotq) throw Error(IETI_ENOTSUP, "internal: fused dot with the tensor smoother");
                stencil<T, T, T, EPI_RESID>(0, true, mode, D.coefT, X, D.vr, B, nullptr, act, 0.0, 0);
                fd_smooth(mode, act, (const T*)D.vr, X, false);
            } else {
                const int m = l == 0 ? cheb_m : cheb_mc;
                for (int k = 0; k < m; ++k) {
                    const bool last0 = l == 0 && k == m - 1;
                    stencil<T, T, T, EPI_CHEB>(l, true, mode, D.coefT, X, XA, B, D.vd, act, 0.0, k, nullptr, nullptr,
                                               last0 ? dotq : nullptr, last0 ? dpart : nullptr);
                    std::swap(X, XA);
                }
            }
            cur[l] = X;
        }
        if (cur[0] != x0) throw Error(IETI_EDEVICE, "internal: V-cycle result buffer mismatch");
        if (dotq && deepest == 0) throw Error(IETI_ENOTSUP, "internal: fused dot needs a smoothed level 0");
    }

    // levels >= l0 of every patch that has level l0: lev[l0].vb -> lev[l0].vxa
    void vcoarse(int l0, int mode, const int* act) {
        CoarseArgs a{};
        for (int l = 0; l < nlev && l < LMAX; ++l) {
            a.L[l] = lev[l].L;
            a.coef[l] = lev[l].coefT;
            a.plo[l] = lev[l].plo;
            a.pval[l] = lev[l].pval;
            a.rlo[l] = lev[l].rlo;
            a.rval[l] = lev[l].rval;
            a.inv[l] = lev[l].inv;
            a.cheb[l] = lev[l].cheb;
        }
        a.chain = chain;
        a.l0 = l0;
        a.b1 = lev[l0].vb;
        a.x1 = lev[l0].vxa;
        a.mode = mode;
        a.m = cheb_mc;
        a.active = act;
        for (int fam = 0; fam < 2; ++fam) {
            if (h_plist[fam].empty()) continue;
            a.plist = plist[fam];
            a.nlist = (int)h_plist[fam].size();
            // kernel events on launches that run every patch (no activity mask: the preconditioner's cycles)
            std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
            if (prof.on && act == nullptr) ev = prof.next(IETI_KPROF_COARSE, vc_bytes[fam]);
            launch_vcoarse<T>(fam, fuse_stage, stream, a, vc_lds[fam], false, ev.first, ev.second);
            check_launch();
        }
    }

    // ---------------------------------------------------------------- batched flexible CG: fx = K_rr^{-1} b
    // b: level-0 FP64 (masked to mode N here).  All patches in every launch.
    void fcg(const double* b, double tol, int maxit) {
        DevLevel& D = lev[0];
        const int nt = D.nt_all;
        double* prr = partial + 3 * nt;     // nt (pzq, pdots: see fcg_iteration)
        hipLaunchKernelGGL(k_fcg_init<T>, dim3(tile_grid(nt)), dim3(TILE), 0, stream, D.L, D.tiles_all, nt, b, fx,
                           fr, rT, fd, fq, prr, (int)MODE_N);
        check_launch();
        hipLaunchKernelGGL(k_fcg_check, dim3(1), dim3(256), 0, stream, N, tile_beg, tile_end, prr, 1, bb, active, its,
                           brk, tol * tol, maxit, nactive);
        check_launch();
        // patches whose finest level is also their coarsest cannot fuse z . q into the smoother
        const bool fuse_zq = lev[0].n_coarse == 0 && !fd_on;
        // host checks: first near the iteration count the previous solve at this tolerance needed, then
        // every check_every iterations (a sync costs more than an extra iteration of finished patches)
        const int every = std::max(1, plan->opt.check_every);
        int& hint = tol < 1e-11 ? hint_basis : hint_solve;
        int next_check = std::max(1, hint - 1);
        int last_it = 0;
        // iterations after the first are the same launch sequence with the same arguments: with use_graph
        // they replay captured graphs per tolerance (not while kernel events are recorded): one of check_every
        // iterations for the stretches between two host checks, one of a single iteration for the rest
        FcgGraphs* gx = nullptr;
        if (plan->opt.use_graph && graphs_ok && !prof.on && !noalloc_call) {
            auto& g = fcg_graphs[std::make_pair(tol, maxit)];
            if (!g.one) g.one = capture_fcg_iterations(fuse_zq, tol, maxit, 1);
            if (!g.run && every > 1) g.run = capture_fcg_iterations(fuse_zq, tol, maxit, every);
            if (g.one) gx = &g;
        }
        for (int it = 0; it < maxit;) {
            if (it == next_check) {
                HIPCHECK(hipMemcpyAsync(h_nactive, nactive, sizeof(int), hipMemcpyDeviceToHost, stream));
                sync();
                if (*h_nactive == 0) break;
                next_check = it + every;
            }
            if (it > 0 && gx && gx->run && it + every <= next_check && it + every <= maxit) {
                HIPCHECK(hipGraphLaunch(gx->run, stream));
                it += every;
            } else if (it > 0 && gx) {
                HIPCHECK(hipGraphLaunch(gx->one, stream));
                ++it;
            } else {
                fcg_iteration(it, fuse_zq, tol, maxit);
                ++it;
            }
            last_it = it;
        }
        hint = last_it;
    }
    struct FcgGraphs {
        hipGraphExec_t one = nullptr, run = nullptr;
    };
    std::map<std::pair<double, int>, FcgGraphs> fcg_graphs;
    bool graphs_ok = true;   // cleared when the stream cannot be captured (e.g. the legacy null stream)

    hipGraphExec_t capture_fcg_iterations(bool fuse_zq, double tol, int maxit, int count) {
        if (stream == nullptr) {
            graphs_ok = false;
            return nullptr;
        }
        if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            graphs_ok = false;
            return nullptr;
        }
        hipGraph_t graph = nullptr;
        try {
            for (int c = 0; c < count; ++c) fcg_iteration(1, fuse_zq, tol, maxit);
        } catch (...) {
            (void)hipStreamEndCapture(stream, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        HIPCHECK(hipStreamEndCapture(stream, &graph));
        hipGraphExec_t ex = nullptr;
        const hipError_t e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHECK(e);
        return ex;
    }

    // one flexible-CG iteration on all active patches (it == 0: first direction)
    void fcg_iteration(int it, bool fuse_zq, double tol, int maxit) {
        DevLevel& D = lev[0];
        const int nt = D.nt_all;
        double* pzq = partial;              // nt
        double* pdots = partial + nt;       // 2 nt
        double* prr = partial + 3 * nt;     // nt
        if (fuse_zq && it > 0) {
            vcycle(MODE_N, active, rT, zT, fq, pzq);
        } else {
            vcycle(MODE_N, active, rT, zT);
            if (it > 0) {
                hipLaunchKernelGGL(k_fcg_zq<T>, dim3(tile_grid(nt)), dim3(TILE), 0, stream, D.L, D.tiles_all, nt, zT,
                                   fq, pzq, active);
                check_launch();
            }
        }
        hipLaunchKernelGGL(k_fcg_dir<T>, dim3(tile_grid(nt)), dim3(TILE), 0, stream, D.L, D.tiles_all, nt, zT, fd,
                           pzq, tile_beg, tile_end, dq, it == 0 ? 1 : 0, (int)MODE_N, active);
        check_launch();
        stencil<double, double, double, EPI_DOTS>(0, false, MODE_N, coef64, fd, fq, nullptr, nullptr, active, 0.0, 0,
                                                  pdots, fr);
        if (n_float > 0) {   // floating patches: + gamma C^T C d
            hipLaunchKernelGGL(k_float_penalty, dim3(n_float), dim3(TILE), 0, stream, n_float, float_list, npk,
                               edge_ptr, edge_dev, float_gam, (const double*)fd, fq, pdots, tile_beg, active);
            check_launch();
        }
        hipLaunchKernelGGL(k_fcg_update<T>, dim3(tile_grid(nt)), dim3(TILE), 0, stream, D.L, D.tiles_all, nt, fd, fq,
                           fx, fr, rT, pdots, tile_beg, tile_end, dq, brk, prr, active);
        check_launch();
        hipLaunchKernelGGL(k_fcg_check, dim3(1), dim3(256), 0, stream, N, tile_beg, tile_end, prr, 0, bb, active, its,
                           brk, tol * tol, maxit, nactive);
        check_launch();
    }

    // 3D exact local solves: block-band factors built on the device (k_bb_*)
    bool band3 = false;
    BandJob* bb_jobs = nullptr;
    int32_t* bb_job_of = nullptr;   // [mode][patch] -> job, -1: none
    double *bb_F = nullptr, *bb_D = nullptr;
    std::vector<BandJob> h_bb_jobs;
    void setup_band3() {
        const Plan& pl = *plan;
        hipStream_t st = stream;
        std::vector<int32_t> stab, job_of(2 * (size_t)N, -1);
        int64_t off = 0, doff = 0;
        int nbmax = 0, wmax = 0;
        for (int k = 0; k < N; ++k) {
            const Patch& pa = pl.patches[k];
            const Level& L0 = pa.lv[0];
            const int toff = (int)stab.size();
            const int w0 = 2 * pa.p[0] + 1, w1 = 2 * pa.p[1] + 1, w2 = 2 * pa.p[2] + 1;
            stab.resize(stab.size() + (size_t)w0 * w1 * w2, 0);
            auto at = [&](int o0, int o1, int o2) -> int32_t& {
                return stab[toff + (o0 + pa.p[0]) + (size_t)w0 * ((o1 + pa.p[1]) + (size_t)w1 * (o2 + pa.p[2]))];
            };
            for (int s = 0; s < L0.nst; ++s) {
                const int o0 = L0.offs[3 * s], o1 = L0.offs[3 * s + 1], o2 = L0.offs[3 * s + 2];
                at(o0, o1, o2) = s + 1;                // K(i, i + o) = coef[s][i]
                if (s > 0) at(-o0, -o1, -o2) = -(s + 1);   // K(i, i - o) = K(i - o, i) = coef[s][i - o]
            }
            const int nb = (int)((L0.n + BNB - 1) / BNB), W = (int)((L0.guard + BNB - 1) / BNB);
            nbmax = std::max(nbmax, nb);
            wmax = std::max(wmax, W);
            for (int m = 0; m < 2; ++m) {
                if (m == MODE_D && !prec_exact) continue;
                job_of[(size_t)m * N + k] = (int32_t)h_bb_jobs.size();
                h_bb_jobs.push_back(BandJob{off, doff, k, m, nb, W, toff});
                off += (int64_t)nb * (W + 1) * BNB * BNB;
                doff += (int64_t)nb * BNB * BNB;
            }
        }
        if (wmax > BB_WMAX) throw Error(IETI_ENOTSUP, "3D exact local solves: band wider than the solve's window");
        const int nj = (int)h_bb_jobs.size();
        bb_F = arena.alloc<double>(off, st, false);
        bb_D = arena.alloc<double>(doff, st, false);
        bb_jobs = arena.upload(h_bb_jobs, st);
        bb_job_of = arena.upload(job_of, st);
        int32_t* stab_d = arena.upload(stab, st);
        int* err = arena.alloc<int>(1, st);
        hipLaunchKernelGGL(k_bb_assemble, dim3(nbmax * (wmax + 1), nj), dim3(256), 0, st, lev[0].L, bb_jobs, stab_d,
                           (const double*)coef64, bb_F);
        check_launch();
        for (int k = 0; k < nbmax; ++k) {
            hipLaunchKernelGGL(k_bb_potrf, dim3(nj), dim3(256), 0, st, bb_jobs, k, bb_F, bb_D, err);
            check_launch();
            if (wmax > 0) {
                hipLaunchKernelGGL(k_bb_trsm, dim3(wmax, nj), dim3(256), 0, st, bb_jobs, k, bb_F, (const double*)bb_D);
                check_launch();
                hipLaunchKernelGGL(k_bb_update, dim3(wmax * (wmax + 1) / 2, nj), dim3(256), 0, st, bb_jobs, k, bb_F);
                check_launch();
            }
        }
        int herr = 0;
        HIPCHECK(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        if (herr) throw Error(IETI_EINVAL, "local stiffness matrix is not positive definite");
        band3 = true;
    }
    void band_solve(int mode, const double* rhs, double* x) {
        if (band3) {
            hipLaunchKernelGGL(k_bb_solve, dim3(N), dim3(BB_THREADS), 0, stream, lev[0].L, bb_jobs,
                               bb_job_of + (size_t)mode * N, (const double*)bb_F, (const double*)bb_D, rhs, x,
                               nullptr);
            check_launch();
            return;
        }
        if (band_bmax <= 256)
            hipLaunchKernelGGL((k_band_solve_pf<16, true>), dim3(N), dim3(BAND_PF_THREADS), band_lds, stream, lev[0].L,
                               band_off, band_b, band, mode, rhs, x, nullptr);
        else if (band_bmax <= 512)
            hipLaunchKernelGGL((k_band_solve_pf<32, false>), dim3(N), dim3(BAND_PF_THREADS), band_lds, stream,
                               lev[0].L, band_off, band_b, band, mode, rhs, x, nullptr);
        else
            hipLaunchKernelGGL(k_band_solve, dim3(N), dim3(BAND_THREADS), band_lds, stream, lev[0].L, band_off,
                               band_b, band, mode, rhs, x, nullptr);
        check_launch();
    }

    // fx = K_rr^{-1} b (b masked to mode N): exact or multigrid-preconditioned flexible CG
    void local_solve(const double* b, double tol) {
        if (exact) band_solve(MODE_N, b, fx);
        else fcg(b, tol, plan->opt.inner_max_it);
    }

    // ---------------------------------------------------------------- K~^{-1} g, primal part on the slots or on all rows
    // g: level-0 FP64 (local load-type vector); the FCG solves with m_N g.
    // full == false: only the interface slots of the result are corrected (F apply).
    void ktilde_inv(const double* g, bool full, double tol, double* out_full) {
        if (full) {
            DevLevel& D = lev[0];
            hipLaunchKernelGGL((k_convert<double, double>), dim3(tile_grid(D.nt_all)), dim3(TILE), 0, stream, D.L,
                               D.tiles_all, D.nt_all, g, e64, (int)MODE_N, 1.0);
            check_launch();
            local_solve(e64, tol);
        } else {
            local_solve(g, tol);
        }
        if (npi > 0) {
            hipLaunchKernelGGL(k_pri_dots, dim3(N), dim3(TILE), 0, stream, N, npk, row_ptr, slot_dev,
                               full ? lev[0].L : nullptr, full ? psi : psiG, len0, g, fx, edge_ptr, edge_dev, cbuf,
                               ebuf);
            check_launch();
            hipLaunchKernelGGL(k_pri_coarse, dim3(nblk(npi, WAVE)), dim3(256), npi * sizeof(double), stream, npi,
                               pri_ptr, pri_patch, pri_local, cbuf, Sinv, upi);
            check_launch();
            hipLaunchKernelGGL(k_pri_coef, dim3(nblk((int64_t)N * NPMAX, 256)), dim3(256), 0, stream, N, npk, Rk, upi,
                               ebuf, coefbuf);
            check_launch();
        }
        if (full) {
            DevLevel& D = lev[0];
            if (npi > 0) {
                hipLaunchKernelGGL(k_pri_apply_full, dim3(tile_grid(D.nt_all)), dim3(TILE), 0, stream, D.L,
                                   D.tiles_all, D.nt_all, npk, psi, len0, coefbuf, fx, out_full);
            } else {
                HIPCHECK(hipMemcpyAsync(out_full, fx, sizeof(double) * len0, hipMemcpyDeviceToDevice, stream));
            }
            check_launch();
        } else if (npi > 0) {
            hipLaunchKernelGGL(k_pri_apply_slots, dim3(nblk(nslots, 256)), dim3(256), 0, stream, nslots, slot_patch,
                               slot_dev, npk, psiG, coefbuf, fx);
            check_launch();
        }
    }

    void scatter(const double* lamv, bool scaled, double* v) {
        fill<double>(v, len0, 0.0);
        if (nslots == 0) return;
        hipLaunchKernelGGL(k_scatter, dim3(nblk(nslots, 256)), dim3(256), 0, stream, nslots, slot_dev, slot_ptr,
                           slot_lam, scaled ? slot_wBD : slot_wB, lamv, v);
        check_launch();
    }
    void gather(const double* v, bool scaled, double* out, bool plus_only = false, bool minus_only = false) {
        if (nlam == 0) return;
        const int64_t* pl = minus_only ? lam_minus : lam_plus;
        const int64_t* mi = (plus_only || minus_only) ? nullptr : lam_minus;
        hipLaunchKernelGGL(k_gather, dim3(nblk(nlam, 256)), dim3(256), 0, stream, nlam, pl, mi,
                           scaled ? lam_wBD : nullptr, v, out);
        check_launch();
    }

    // ---------------------------------------------------------------- algorithmic bytes of F and M^{-1}
    // Each array a kernel must stream counted once per launch (s: bytes of the multigrid word): a Chebyshev
    // step (5 + nst) n s (the step from zero 4 n s), a residual (3 + nst) n s, a restriction (n + n_c) s, a
    // prolongation (2 n + n_c) s; the fused coarse part its right-hand side and result once, the half
    // stencils of its smoothed levels and the coarsest inverse once; a coarsest solve outside it 2 n_c s +
    // n_c^2 s.  A tensor-smoother step on the finest level (padded sizes P_d, PP = prod P_d): forward
    // transform r (n s) and U_d in, the transformed array (PP) out; backward transform the array, U_d and the
    // eigenvalues in, x out (and in, when it adds); in 3D each of the six axis contractions streams the
    // padded array in and out with its U_d.  vcycle_bytes(k, mode): patch k, one V-cycle of that mode.
    double fd_step_bytes(int k, int mode, bool set) const {
        const Patch& pa = plan->patches[k];
        const Patch::Tensor& Tz = pa.ts[mode];
        if (Tz.U[0].empty()) return 0.0;
        const double s = sizeof(T), n = (double)pa.lv[0].n;
        const double P0 = Tz.Pd[0], P1 = Tz.Pd[1], P2 = dim == 3 ? Tz.Pd[2] : 1.0;
        const double PP = P0 * P1 * P2;
        const double su = (dim == 2 && std::is_same<T, float>::value) ? 4.0 : 8.0;   // U and array in FP32 (2D)
        const double U = P0 * P0 + P1 * P1 + (dim == 3 ? P2 * P2 : 0.0);
        const double lam = 8.0 * (P0 + P1 + (dim == 3 ? P2 : 0.0));
        const double xio = set ? n * s : 2.0 * n * s;
        // 2D: W = m R U_0, Z = U_1^T W (scaled), T = Z U_0^T, x (+)= U_1 T: each U twice, Z written once and
        // read once (W and T too where the products are not fused in pairs)
        if (dim == 2) return n * s + 2.0 * U * su + (fd_p1max <= FD2C_MAXP ? 2.0 : 6.0) * PP * su + lam + xio;
        // 3D: r -> zb (axes 0 and 1 fused), zb -> za (axis 2, scaled), za -> zb (axis 2), zb -> x (axes 1 and 0
        // fused): each U twice, the padded array written and read three times
        return n * s + 2.0 * U * 8.0 + 6.0 * PP * 8.0 + lam + xio;
    }
    double vcycle_bytes(int k, int mode) const {
        const Patch& pa = plan->patches[k];
        const int nl = (int)pa.lv.size();
        const double s = sizeof(T);
        double b = 0.0;
        for (int l = 0; l < nl; ++l) {
            const Level& L = pa.lv[l];
            const double n = (double)L.n, nst = L.nst;
            if (l >= fuse_l0) {   // the fused kernel from here on
                b += 2.0 * n * s;
                for (int q = l; q < nl; ++q) {
                    const Level& Q = pa.lv[q];
                    b += q == nl - 1 ? (double)Q.n * (double)Q.n * s : (double)Q.nst * (double)Q.n * s;
                }
                break;
            }
            if (l == nl - 1) {   // coarsest solve by the batched dense GEMV
                b += 2.0 * n * s + n * n * s;
                break;
            }
            const double nc = (double)pa.lv[l + 1].n;
            // transfers: nested (n + n_c) s down, (2 n + n_c) s up; L2 projection: the mass solve (n in, n out)
            // and the band (n + n_c) down, the band (n_c + n), the mass solve (2 n) and the add (3 n) up
            const double tdown = L.l2 ? (3.0 * n + nc) * s : (n + nc) * s;
            const double tup = L.l2 ? (6.0 * n + nc) * s : (2.0 * n + nc) * s;
            if (l == 0 && fd_on && !pa.ts[mode].U[0].empty()) {
                b += fd_step_bytes(k, mode, true) + (3.0 + nst) * n * s + tdown;   // step from zero, residual
                b += tup + (3.0 + nst) * n * s + fd_step_bytes(k, mode, false);
                continue;
            }
            const int m = l == 0 ? cheb_m : cheb_mc;
            b += 4.0 * n * s + (m - 1) * (5.0 + nst) * n * s;   // pre-smoothing from zero
            b += (3.0 + nst) * n * s + tdown;                     // residual, restriction
            b += tup + m * (5.0 + nst) * n * s;                   // prolongation, post-smoothing
        }
        return b;
    }
    // factor data one exact local solve streams: the host-built 2D layout once (its L and L^T halves are
    // separate copies), the 3D block band twice (forward by rows, backward by columns) with the diagonal
    // inverses
    double band_bytes(int k, int mode) const {
        const Patch& pa = plan->patches[k];
        if (!band3) return (double)pa.band[mode].size() * 8.0;
        const double nb = (double)((pa.lv[0].n + BNB - 1) / BNB), W = (double)((pa.lv[0].guard + BNB - 1) / BNB);
        return 2.0 * nb * (W + 1.0) * BNB * BNB * 8.0;
    }
    // one F apply with the inner iteration counts its_k of its local solves
    double fapply_bytes(const std::vector<int>& itk) const {
        const double s = sizeof(T);
        double b = 8.0 * (double)len0 + 24.0 * (double)nslots + 24.0 * (double)nlam;   // B^T p, B w
        for (int k = 0; k < N; ++k) {
            const Patch& pa = plan->patches[k];
            const double n = (double)pa.lv[0].n, nst = pa.lv[0].nst;
            if (exact) {
                b += band_bytes(k, MODE_N) + 16.0 * n;
                continue;
            }
            const double init = n * (40.0 + s);
            const double iter = vcycle_bytes(k, MODE_N) + n * (s + 8.0) + n * (s + 16.0) + n * (8.0 * nst + 24.0) +
                                n * (48.0 + s);
            b += init + (double)itk[k] * iter;
        }
        b += 16.0 * (double)nslots * (double)std::max(npk_max, 0);   // primal part on the slots
        return b;
    }
    double prec_bytes() const {
        const double s = sizeof(T);
        double b = 8.0 * (double)len0 + 24.0 * (double)nslots + 24.0 * (double)nlam;
        for (int k = 0; k < N; ++k) {
            const Patch& pa = plan->patches[k];
            const double n = (double)pa.lv[0].n, nst = pa.lv[0].nst;
            b += n * (8.0 + 8.0 * nst + s);                 // b_I = -K v
            if (prec_exact) {
                b += band_bytes(k, MODE_D) + 16.0 * n;
            } else {
                const int cyc = std::max(1, plan->opt.prec_vcycles);
                b += cyc * vcycle_bytes(k, MODE_D) + (cyc - 1) * ((3.0 + nst) * n * s + 3.0 * n * s);
            }
            b += n * (s + 16.0) + n * (8.0 * nst + 16.0);   // w = v + x_I, s = K w
        }
        return b;
    }

    // q = F p
    void applyF(const double* p, double* q) {
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        size_t slot = 0;
        if (prof.on) {
            ev = prof.next(IETI_KPROF_FAPPLY, 0.0);
            slot = prof.pending.size() - 1;   // the kernel classes inside add entries after this one
            HIPCHECK(hipEventRecord(ev.first, stream));
        }
        scatter(p, false, b64);
        ktilde_inv(b64, false, plan->opt.inner_tol, nullptr);
        gather(fx, false, q);
        if (prof.on) {
            HIPCHECK(hipEventRecord(ev.second, stream));
            std::vector<int> itk(N, 0);
            if (!exact) HIPCHECK(hipMemcpyAsync(itk.data(), its, N * sizeof(int), hipMemcpyDeviceToHost, stream));
            sync();
            prof.pending[slot].second = fapply_bytes(itk);
        }
    }

    // z = B_D S B_D^T r
    void applyPrec(const double* r, double* z) {
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        if (prof.on) {
            ev = prof.next(IETI_KPROF_PREC, prec_bytes());
            HIPCHECK(hipEventRecord(ev.first, stream));
        }
        applyPrecBody(r, z);
        if (prof.on) HIPCHECK(hipEventRecord(ev.second, stream));
    }
    void applyPrecBody(const double* r, double* z) {
        DevLevel& D = lev[0];
        scatter(r, true, w64);
        // b_I = -m_D (K v)
        stencil<double, double, T, EPI_APPLY>(0, false, MODE_D, coef64, w64, bT, nullptr, nullptr, nullptr, -1.0, 0);
        if (prec_exact) {
            if (!std::is_same<T, double>::value) throw Error(IETI_EDEVICE, "internal: exact solves need FP64");
            band_solve(MODE_D, (const double*)bT, (double*)xIT);
        } else {
            vcycle(MODE_D, nullptr, bT, xIT);
        }
        for (int c = 1; !prec_exact && c < plan->opt.prec_vcycles; ++c) {
            stencil<T, T, T, EPI_RESID>(0, false, MODE_D, D.coefT, xIT, r2T, bT, nullptr, nullptr, 0.0, 0);
            vcycle(MODE_D, nullptr, r2T, x2T);
            hipLaunchKernelGGL(k_add<T>, dim3(tile_grid(D.nt_all)), dim3(TILE), 0, stream, D.L, D.tiles_all, D.nt_all,
                               (const T*)x2T, xIT);
            check_launch();
        }
        // w = v + x_I;  s = K w (mode K); z = B_D s
        hipLaunchKernelGGL(k_add_conv<T>, dim3(tile_grid(D.nt_all)), dim3(TILE), 0, stream, D.L, D.tiles_all,
                           D.nt_all, (const T*)xIT, w64);
        check_launch();
        stencil<double, double, double, EPI_APPLY>(0, false, MODE_K, coef64, w64, s64, nullptr, nullptr, nullptr, 1.0,
                                                   0);
        gather(s64, true, z);
    }

    // ---------------------------------------------------------------- saddle-point iteration (MG-MG-S)
    // Vectors of W~ (primal continuity built in) are level-0 torn vectors u = w + Psi R u_Pi; their dual
    // (residuals) is any torn representative.  A = K~ acts as the patch stiffness (mode K), B~ as the jump.
    bool saddle = false;
    double bp_omega = 1.0;   // A0^{-1} = omega * (P_E V3 P_E^T + Psi R S^{-1} R^T Psi^T), A0 < A
    double *bx = nullptr, *br = nullptr, *bz = nullptr, *bhz = nullptr, *bp = nullptr, *bs = nullptr, *bt = nullptr,
           *bht = nullptr, *bg = nullptr, *bw = nullptr, *bg2 = nullptr;
    double *lxx = nullptr, *lrr = nullptr, *lzz = nullptr, *lhz = nullptr, *lpp = nullptr, *lss = nullptr,
           *ltt = nullptr, *lht = nullptr, *bsc = nullptr, *dpart = nullptr;
    int ndpart = 0;

    void flat_dot(int64_t n, const double* a, const double* b, double* out) {
        if (n <= 0) {
            fill<double>(out, 1, 0.0);
            return;
        }
        const int g = (int)std::min<int64_t>(ndpart, nblk(n, TILE));
        hipLaunchKernelGGL(k_dot_flat, dim3(g), dim3(TILE), 0, stream, n, a, b, dpart);
        check_launch();
        hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, stream, dpart, (int64_t)g, out);
        check_launch();
    }
    void axpy_dev(int64_t n, double* y, const double* x, int idx, double sign) {
        if (n <= 0) return;
        hipLaunchKernelGGL(k_axpy_dev, dim3(nblk(n, 256)), dim3(256), 0, stream, n, y, x, bsc, idx, sign);
        check_launch();
    }
    void xpby_dev(int64_t n, double* p, const double* z, int idx) {
        if (n <= 0) return;
        hipLaunchKernelGGL(k_xpby_dev, dim3(nblk(n, 256)), dim3(256), 0, stream, n, p, z, bsc, idx);
        check_launch();
    }
    void copy_dev(int64_t n, double* dst, const double* src) {
        if (n <= 0) return;
        HIPCHECK(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, stream));
    }
    void applyA(const double* v, double* out) {
        stencil<double, double, double, EPI_APPLY>(0, false, MODE_K, coef64, v, out, nullptr, nullptr, nullptr, 1.0,
                                                   0);
    }
    // out = omega [P_E V3 P_E^T g + Psi R S^{-1} sum_k R_k^T Psi_k^T g] (out must not alias g)
    void A0inv(const double* g, double* out, double omega) {
        DevLevel& D = lev[0];
        if (npi > 0) {
            hipLaunchKernelGGL(k_pri_dots, dim3(N), dim3(TILE), 0, stream, N, npk, row_ptr, slot_dev, lev[0].L, psi,
                               len0, g, nullptr, edge_ptr, edge_dev, cbuf, ebuf);
            check_launch();
        }
        // P_E^T g, masked to the K_rr space
        hipLaunchKernelGGL((k_convert<double, double>), dim3(tile_grid(D.nt_all)), dim3(TILE), 0, stream, D.L,
                           D.tiles_all, D.nt_all, g, bg, (int)MODE_N, 1.0);
        check_launch();
        if (npi > 0) {
            hipLaunchKernelGGL(k_edge_scatter_sub, dim3(N), dim3(TILE), 0, stream, N, npk, edge_ptr, edge_dev, cbuf,
                               bg);
            check_launch();
        }
        // three V-cycles as a stationary iteration from zero
        hipLaunchKernelGGL((k_convert<double, T>), dim3(tile_grid(D.nt_all)), dim3(TILE), 0, stream, D.L,
                           D.tiles_all, D.nt_all, bg, bT, (int)MODE_N, 1.0);
        check_launch();
        vcycle(MODE_N, nullptr, bT, xIT);
        for (int c = 1; c < 3; ++c) {
            stencil<T, T, T, EPI_RESID>(0, false, MODE_N, D.coefT, xIT, r2T, bT, nullptr, nullptr, 0.0, 0);
            vcycle(MODE_N, nullptr, r2T, x2T);
            hipLaunchKernelGGL(k_add<T>, dim3(tile_grid(D.nt_all)), dim3(TILE), 0, stream, D.L, D.tiles_all, D.nt_all,
                               (const T*)x2T, xIT);
            check_launch();
        }
        hipLaunchKernelGGL((k_convert<T, double>), dim3(tile_grid(D.nt_all)), dim3(TILE), 0, stream, D.L,
                           D.tiles_all, D.nt_all, (const T*)xIT, bw, (int)MODE_N, 1.0);
        check_launch();
        if (npi > 0) {
            // edge means of the V-cycle result (P_E) and the primal part
            hipLaunchKernelGGL(k_pri_dots, dim3(N), dim3(TILE), 0, stream, N, npk, row_ptr, slot_dev, lev[0].L, psi,
                               len0, g, bw, edge_ptr, edge_dev, cbuf, ebuf);
            check_launch();
            hipLaunchKernelGGL(k_pri_coarse, dim3(nblk(npi, WAVE)), dim3(256), npi * sizeof(double), stream, npi,
                               pri_ptr, pri_patch, pri_local, cbuf, Sinv, upi);
            check_launch();
            hipLaunchKernelGGL(k_pri_coef, dim3(nblk((int64_t)N * NPMAX, 256)), dim3(256), 0, stream, N, npk, Rk,
                               upi, ebuf, coefbuf);
            check_launch();
            hipLaunchKernelGGL(k_pri_apply_full, dim3(tile_grid(D.nt_all)), dim3(TILE), 0, stream, D.L, D.tiles_all,
                               D.nt_all, npk, psi, len0, coefbuf, bw, out);
            check_launch();
        } else {
            copy_dev(len0, out, bw);
        }
        hipLaunchKernelGGL(k_scale_flat, dim3(nblk(len0, 256)), dim3(256), 0, stream, len0, out, out, omega);
        check_launch();
    }
    // Smallest eigenvalue of a symmetric tridiagonal matrix (diagonal a, off-diagonal b) by bisection on
    // the Sturm count (the number of negative pivots of T - x I).
    static double tridiag_min_eig(const std::vector<double>& a, const std::vector<double>& b) {
        const size_t k = a.size();
        double lo = 1e300, hi = -1e300;
        for (size_t i = 0; i < k; ++i) {   // Gershgorin bounds
            const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
            lo = std::min(lo, a[i] - r);
            hi = std::max(hi, a[i] + r);
        }
        for (int step = 0; step < 200 && hi - lo > 1e-14 * std::max(1.0, std::fabs(hi)); ++step) {
            const double x = 0.5 * (lo + hi);
            int neg = 0;
            double d = 1.0;
            for (size_t i = 0; i < k; ++i) {
                d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
                if (d == 0.0) d = -1e-300;
                if (d < 0.0) ++neg;
            }
            if (neg >= 1) hi = x;
            else lo = x;
        }
        return 0.5 * (lo + hi);
    }
    // omega of the V-cycle block: A0 < A on W~ needs omega > 1 / lambda_min(T), T = A0^{-1} A at omega = 1.
    // lambda_min is the smallest Ritz value of the Lanczos matrix that k steps of CG on A x = b (b seeded,
    // preconditioner A0^{-1}) build from their step lengths alpha_j and ratios beta_j:
    //   T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},  T_j,j+1 = sqrt(beta_j)/alpha_j.
    // Ritz values approach the spectrum's edge from inside, so the factor 1.1 covers the remaining gap; a
    // too small omega that still slips through is caught by the iteration (a non-positive H-energy).
    void estimate_omega() {
        std::vector<double> h(len0);
        uint64_t x = 0xD1B54A32D192ED03ull;
        for (auto& v : h) {
            x ^= x << 13; x ^= x >> 7; x ^= x << 17;
            v = (double)(x >> 11) * (1.0 / 9007199254740992.0) - 0.5;
        }
        HIPCHECK(hipMemcpyAsync(br, h.data(), len0 * sizeof(double), hipMemcpyHostToDevice, stream));
        A0inv(br, bz, 1.0);
        copy_dev(len0, bp, bz);
        flat_dot(len0, br, bz, bsc + 10);
        double rz = 0.0;
        HIPCHECK(hipMemcpyAsync(&rz, bsc + 10, sizeof(double), hipMemcpyDeviceToHost, stream));
        sync();
        // stop well above the rounding floor of the CG residual: once it is reached the Lanczos vectors lose
        // orthogonality and the coefficients no longer describe T (an FP32 V-cycle is symmetric only to FP32)
        const double rz_floor = (std::is_same<T, float>::value ? 1e-8 : 1e-16) * rz;
        std::vector<double> al, be, ta, tb;
        double lmin = 1.0, lprev = 2.0;
        for (int k = 0; k < 40 && rz > 0.0; ++k) {
            applyA(bp, bs);
            flat_dot(len0, bp, bs, bsc + 10);
            double pap = 0.0;
            HIPCHECK(hipMemcpyAsync(&pap, bsc + 10, sizeof(double), hipMemcpyDeviceToHost, stream));
            sync();
            if (!(pap > 0.0)) break;
            const double alpha = rz / pap;
            ta.push_back(1.0 / alpha + (k > 0 ? be.back() / al.back() : 0.0));
            al.push_back(alpha);
            fill<double>(bsc + 11, 1, alpha);
            axpy_dev(len0, br, bs, 11, -1.0);
            A0inv(br, bz, 1.0);
            flat_dot(len0, br, bz, bsc + 10);
            double rz1 = 0.0;
            HIPCHECK(hipMemcpyAsync(&rz1, bsc + 10, sizeof(double), hipMemcpyDeviceToHost, stream));
            sync();
            lmin = tridiag_min_eig(ta, tb);
            if (!(rz1 > rz_floor) || (k >= 3 && std::fabs(lmin - lprev) <= 1e-3 * lmin)) break;
            const double beta = rz1 / rz;
            rz = rz1;
            be.push_back(beta);
            tb.push_back(std::sqrt(beta) / alpha);
            fill<double>(bsc + 11, 1, beta);
            xpby_dev(len0, bp, bz, 11);
            lprev = lmin;
        }
        if (!(lmin > 0.1)) throw Error(IETI_ENOCONV, "V-cycle preconditioner too weak for the saddle-point iteration");
        bp_omega = 1.1 / std::min(lmin, 1.0);
    }
    int solve_saddle(ieti_stats& st);
    void finish_solution(ieti_stats& st, double* u_out);

    // ---------------------------------------------------------------- setup
    // Chebyshev coefficients d_k = s1 d_{k-1} + s2 D^{-1} r_k on [lower_scale clo, hi] lambda_max,
    // per (patch-level, mode, step)
    static std::vector<double> cheb_table(const DevLevel& D, double hi, double lower_scale) {
        std::vector<double> ch(D.hL.size() * 2 * KMAX * 2, 0.0);
        for (size_t i = 0; i < D.hL.size(); ++i)
            for (int m = 0; m < 2; ++m) {
                const double lm = D.hL[i].lmax[m] > 0 ? D.hL[i].lmax[m] : 1.0;
                const double aa = std::min(D.hL[i].clo * lower_scale, 0.5) * lm, bb = hi * lm;
                const double theta = 0.5 * (aa + bb), delta = 0.5 * (bb - aa), sigma = theta / delta;
                double rho_prev = 1.0 / sigma, rho = rho_prev;
                for (int k = 0; k < KMAX; ++k) {
                    double s1 = 0.0, s2 = 1.0 / theta;
                    if (k > 0) {
                        rho_prev = rho;
                        rho = 1.0 / (2.0 * sigma - rho_prev);
                        s1 = rho * rho_prev;
                        s2 = 2.0 * rho / delta;
                    }
                    const size_t o = 2 * ((i * 2 + m) * KMAX + k);
                    ch[o] = s1;
                    ch[o + 1] = s2;
                }
            }
        return ch;
    }
    double cheb_lower_scale = 1.0;
    bool tune_cached = false;   // the autotuner's choice came from opt.tune_cache
    void set_smoother(int m, int mc, double lower_scale) {
        cheb_m = m;
        cheb_mc = mc;
        cheb_lower_scale = lower_scale;
        for (int l = 0; l < nlev; ++l) {
            const std::vector<double> ch = cheb_table(lev[l], cheb_hi, lower_scale);
            HIPCHECK(hipMemcpyAsync(lev[l].cheb, ch.data(), ch.size() * sizeof(double), hipMemcpyHostToDevice, stream));
        }
        sync();
    }
    // Smoother autotuner: candidates around the tuned table (finest degree +-1, coarse degree 2/3, interval
    // lower end x0.67/1/1.5) and the tile variant of the finest-level sweeps (x window staged in LDS or read
    // directly), ranked by complete solves of a smooth seeded load (a batched Neumann solve for the
    // saddle-point variant); the fastest is kept.  With opt.tune_cache the choice is looked up in /
    // appended to that file, keyed by tune_key().
    std::string tune_key() const {
        const Plan& pl = *plan;
        std::vector<std::string> shapes;
        for (const auto& pa : pl.patches) {
            std::string t;
            for (int d = 0; d < pl.dim; ++d)
                t += (d ? "," : "") + std::to_string(pa.p[d]) + "/" + std::to_string(pa.lv[0].nel[d]);
            shapes.push_back(t);
        }
        std::sort(shapes.begin(), shapes.end());
        shapes.erase(std::unique(shapes.begin(), shapes.end()), shapes.end());
        std::string k = "d" + std::to_string(pl.dim) + ";fp" + std::to_string(pl.opt.mg_precision) + ";ls" +
                        std::to_string(pl.opt.local_solver) + ";cd" + std::to_string(pl.opt.coarse_dofs) + ";";
        for (size_t i = 0; i < shapes.size(); ++i) k += (i ? " " : "") + shapes[i];
        return k;
    }
    // cache line: {"key": "<key>", "cheb_degree": m, "cheb_degree_coarse": mc, "cheb_lower": s, "stage": 0|1}
    bool tune_lookup(const std::string& key, int& m, int& mc, double& sc, int& stg) const {
        const char* path = plan->opt.tune_cache;
        if (!path) return false;
        FILE* fp = std::fopen(path, "r");
        if (!fp) return false;
        char line[4096];
        const std::string want = "{\"key\": \"" + key + "\", ";
        bool found = false;
        while (std::fgets(line, sizeof line, fp)) {
            if (std::strncmp(line, want.c_str(), want.size()) != 0) continue;
            int a = 0, b = 0, c = 0;
            double d = 0.0;
            if (std::sscanf(line + want.size(), "\"cheb_degree\": %d, \"cheb_degree_coarse\": %d, \"cheb_lower\": %lf, "
                            "\"stage\": %d}", &a, &b, &d, &c) == 4 && a >= 2 && a < KMAX && b >= 2 && b < KMAX && d > 0) {
                m = a; mc = b; sc = d; stg = c;
                found = true;   // the last entry for a key wins
            }
        }
        std::fclose(fp);
        return found;
    }
    void tune_store(const std::string& key, int m, int mc, double sc, int stg) const {
        const char* path = plan->opt.tune_cache;
        if (!path) return;
        FILE* fp = std::fopen(path, "a");
        if (!fp) return;   // the cache is an optimisation: an unwritable path is not an error
        std::fprintf(fp, "{\"key\": \"%s\", \"cheb_degree\": %d, \"cheb_degree_coarse\": %d, \"cheb_lower\": %.17g, "
                     "\"stage\": %d}\n", key.c_str(), m, mc, sc, stg);
        std::fclose(fp);
    }
    void autotune_smoother() {
        if (exact || nlev < 2 || fd_on) return;
        const std::string key = tune_key();
        int cm = 0, cmc = 0, cstg = 1;
        double csc = 1.0;
        if (tune_lookup(key, cm, cmc, csc, cstg)) {
            stage_fine = cstg != 0;
            set_smoother(cm, cmc, csc);
            tune_cached = true;
            return;
        }
        const Plan& pl = *plan;
        const int m0 = cheb_m;
        struct Cand {
            double ms;
            int m, mc, stg;
            double sc;
        };
        std::vector<Cand> cands;
        const double scales[3] = {0.67, 1.0, 1.5};
        for (int stg = 1; stg >= 0; --stg)
            for (int m = std::max(2, m0 - 1); m <= std::min(KMAX - 1, m0 + 1); ++m)
                for (int mc = 2; mc <= 3; ++mc)
                    for (double sc : scales) cands.push_back({1e300, m, mc, stg, sc});
        auto apply = [&](const Cand& c) {
            stage_fine = c.stg != 0;
            set_smoother(c.m, c.mc, c.sc);
        };
        if (!saddle) {
            // complete solves with a smooth seeded load f = sum_{k_d <= 3} c_k prod_d sin(k_d pi x_d),
            // c_k uniform in [-1, 1]: one per candidate, then two more for the best four
            const int nk = pl.dim == 2 ? 9 : 27;
            std::vector<double> coef(nk);
            uint64_t y = 0xC2B2AE3D27D4EB4Full;
            for (auto& v : coef) {
                y ^= y << 13; y ^= y >> 7; y ^= y << 17;
                v = 2.0 * (double)(y >> 11) * (1.0 / 9007199254740992.0) - 1.0;
            }
            std::vector<double> hf(pl.n_qp);
            int64_t q = 0;
            for (const auto& pa : pl.patches)
                for (int64_t j = 0; j < pa.n_qp; ++j, ++q) {
                    const double* x = &pa.qpx[(size_t)j * pl.dim];
                    double v = 0.0;
                    for (int t = 0; t < nk; ++t) {
                        double term = coef[t];
                        int r = t;
                        for (int d = 0; d < pl.dim; ++d) {
                            term *= std::sin((double)(r % 3 + 1) * M_PI * x[d]);
                            r /= 3;
                        }
                        v += term;
                    }
                    hf[q] = v;
                }
            double* fq = arena.upload(hf, stream);
            double* uq = arena.alloc<double>(pl.ndof_torn, stream);
            sync();
            auto timed = [&](const Cand& c) {
                apply(c);
                ieti_stats st{};
                solve(fq, uq, &st);
                return st.time_total_ms;
            };
            timed(cands.front());   // warm-up
            for (auto& c : cands) c.ms = timed(c);
            std::stable_sort(cands.begin(), cands.end(), [](const Cand& a, const Cand& b) { return a.ms < b.ms; });
            for (int i = 0; i < std::min<int>(4, (int)cands.size()); ++i)
                for (int rep = 0; rep < 2; ++rep) cands[i].ms = std::min(cands[i].ms, timed(cands[i]));
        } else {
            // saddle-point iteration (omega is estimated after this choice): one batched Neumann solve of a
            // seeded right-hand side per candidate, best of three
            std::vector<double> h(len0);
            uint64_t x = 0x9E3779B97F4A7C15ull;
            for (auto& v : h) {
                x ^= x << 13; x ^= x >> 7; x ^= x << 17;
                v = (double)(x >> 11) * (1.0 / 9007199254740992.0) - 0.5;
            }
            HIPCHECK(hipMemcpyAsync(e64, h.data(), len0 * sizeof(double), hipMemcpyHostToDevice, stream));
            sync();
            hipEvent_t e0, e1;
            HIPCHECK(hipEventCreate(&e0));
            HIPCHECK(hipEventCreate(&e1));
            for (auto& c : cands) {
                apply(c);
                for (int rep = 0; rep < 3; ++rep) {
                    HIPCHECK(hipEventRecord(e0, stream));
                    fcg(e64, pl.opt.inner_tol, pl.opt.inner_max_it);
                    HIPCHECK(hipEventRecord(e1, stream));
                    HIPCHECK(hipEventSynchronize(e1));
                    float t = 0.f;
                    HIPCHECK(hipEventElapsedTime(&t, e0, e1));
                    c.ms = std::min(c.ms, (double)t);
                }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
        }
        const Cand best = *std::min_element(cands.begin(), cands.end(),
                                            [](const Cand& a, const Cand& b) { return a.ms < b.ms; });
        apply(best);
        tune_store(key, best.m, best.mc, best.sc, best.stg);
    }
    // Sinv = S^{-1} (n x n SPD, host row-major) by k_spd_* on the device, stored by columns
    void spd_inverse(const std::vector<double>& S, int64_t n) {
        const int N = (int)((n + MB - 1) / MB) * MB, nb = N / MB;
        std::vector<double> Ah((size_t)N * N, 0.0);
        for (int64_t i = 0; i < N; ++i)
            for (int64_t j = 0; j < N; ++j)
                Ah[(size_t)i * N + j] = (i < n && j < n) ? S[(size_t)i * n + j] : (i == j ? 1.0 : 0.0);
        double* A = arena.upload(Ah, stream);
        double* L = arena.alloc<double>((int64_t)N * N, stream);
        double* X = arena.alloc<double>((int64_t)N * N, stream);
        int* err = arena.alloc<int>(1, stream);
        Sinv = arena.alloc<double>(n * n, stream, false);
        for (int k = 0; k < nb; ++k) {
            hipLaunchKernelGGL(k_spd_panel, dim3(nb - k, 1), dim3(64), 0, stream, A, L, N, k, err);
            check_launch();
            const int m = nb - k - 1;
            if (m > 0) {
                hipLaunchKernelGGL(k_spd_update, dim3(m * (m + 1) / 2, 1), dim3(64), 0, stream, A, L, N, k);
                check_launch();
            }
        }
        hipLaunchKernelGGL(k_spd_diag_inv, dim3(nb, 1), dim3(64), 0, stream, L, X, N, err);
        check_launch();
        hipLaunchKernelGGL(k_spd_tri_inv, dim3(nb, 1), dim3(64), 0, stream, L, X, N);
        check_launch();
        hipLaunchKernelGGL(k_spd_xtx, dim3(nb * nb, 1), dim3(64), 0, stream, X, Sinv, N, (int)n);
        check_launch();
        int herr = 0;
        HIPCHECK(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, stream));
        sync();
        if (herr) throw Error(IETI_EINVAL, "coarse matrix S_PiPi is not positive definite");
    }
    // ---------------------------------------------------------------- no-allocation solve
    // The per-solve scratch of the kernels -- partial sums of the reductions, the outer CG's scalars, the
    // local solves' per-patch scalars and counters, the saddle-point iteration's scalars and partials --
    // carved from one block (offsets in doubles, 256-byte aligned; int arrays take half a word per entry).
    bool noalloc_call = false;   // graphs and kernel events stay off (instantiation and event pools allocate)
    struct ScratchMap {
        int64_t partial, sc, pcgp, bb, dq, beta, alpha, active, its, brk, nactive, bsc, dpart, words;
    };
    ScratchMap scratch_map() const {
        ScratchMap m{};
        int64_t o = 0;
        auto take = [&](int64_t n) {
            const int64_t at = o;
            o += (std::max<int64_t>(n, 1) + 31) / 32 * 32;
            return at;
        };
        m.partial = take(4 * (int64_t)lev[0].nt_all + 4);
        m.sc = take(16 * (int64_t)ncomp);
        m.pcgp = take(2 * (int64_t)PCG_NB * ncomp);
        m.bb = take(N);
        m.dq = take(N);
        m.beta = take(N);
        m.alpha = take(N);
        m.active = take((N + 1) / 2);
        m.its = take((N + 1) / 2);
        m.brk = take((N + 1) / 2);
        m.nactive = take(4);
        m.bsc = saddle ? take(16) : -1;
        m.dpart = saddle ? take(ndpart) : -1;
        m.words = o;
        return m;
    }
    int solve_noalloc(const double* f_qp, double* u, ieti_stats* st) override {
        const ScratchMap m = scratch_map();
        if ((uint64_t)m.words * sizeof(double) > (uint64_t)IETI_NOALLOC_SCRATCH_BYTES)
            throw Error(IETI_ENOTSUP, "ieti_solve_noalloc: this handle needs " +
                                          std::to_string((uint64_t)m.words * sizeof(double)) +
                                          " bytes of scratch, above the static maximum of " +
                                          std::to_string((uint64_t)IETI_NOALLOC_SCRATCH_BYTES));
        if (!noalloc_base) throw Error(IETI_EDEVICE, "internal: address of the static scratch not resolved");
        double* base = noalloc_base;
        double* const keep_d[] = {partial, sc, bb, dq, beta, alpha, bsc, dpart, pcgp};
        int* const keep_i[] = {active, its, brk, nactive};
        const bool prof_on = prof.on;
        auto restore = [&] {
            partial = keep_d[0], sc = keep_d[1], bb = keep_d[2], dq = keep_d[3];
            beta = keep_d[4], alpha = keep_d[5], bsc = keep_d[6], dpart = keep_d[7], pcgp = keep_d[8];
            active = keep_i[0], its = keep_i[1], brk = keep_i[2], nactive = keep_i[3];
            prof.on = prof_on;
            noalloc_call = false;
        };
        partial = base + m.partial;
        sc = base + m.sc;
        pcgp = base + m.pcgp;
        bb = base + m.bb;
        dq = base + m.dq;
        beta = base + m.beta;
        alpha = base + m.alpha;
        active = (int*)(base + m.active);
        its = (int*)(base + m.its);
        brk = (int*)(base + m.brk);
        nactive = (int*)(base + m.nactive);
        if (saddle) {
            bsc = base + m.bsc;
            dpart = base + m.dpart;
        }
        prof.on = false;
        noalloc_call = true;
        int rc = IETI_OK;
        try {
            // the array keeps the previous call's contents (any handle on this device): start from zeros,
            // as the handle's own buffers did (a fill kernel, not a memset node)
            fill<double>(base, m.words, 0.0);
            rc = solve(f_qp, u, st);   // synchronises the stream before returning
        } catch (...) {
            restore();
            throw;
        }
        restore();
        return rc;
    }
    // one stage of the outer CG of every problem (k_pcg_part, k_pcg_apply, k_pcg_fin over PCG_NB work-groups per problem)
    void pcg_stage(int stage, double* lam, double* lr, const double* lz, double* lp, const double* lq) {
        const dim3 g(PCG_NB, ncomp);
        hipLaunchKernelGGL(k_pcg_part, g, dim3(PCG_THREADS), 0, stream, stage, comp_lam, done_dev, lr, lz, lp, lq,
                           pcgp);
        check_launch();
        hipLaunchKernelGGL(k_pcg_apply, g, dim3(PCG_THREADS), 0, stream, stage, comp_lam, done_dev, lam, lr, lz, lp,
                           lq, sc, pcgp, pcgp + (int64_t)PCG_NB * ncomp);
        check_launch();
        if (stage == 0) return;
        hipLaunchKernelGGL(k_pcg_fin, dim3(nblk(ncomp, 64)), dim3(64), 0, stream, stage, comp_lam, done_dev, sc,
                           pcgp + (int64_t)PCG_NB * ncomp, ncomp);
        check_launch();
    }
    void setup() override;
    int solve(const double* f_qp, double* u, ieti_stats* st) override;
    void quadrature(double* x, bool on_device) override {
        const Plan& pl = *plan;
        if (on_device) {
            HIPCHECK(hipMemcpyAsync(x, qpx, sizeof(double) * pl.n_qp * pl.dim, hipMemcpyDeviceToDevice, stream));
            sync();
        } else {
            int64_t o = 0;
            for (const auto& pa : pl.patches) {
                std::memcpy(x + o, pa.qpx.data(), pa.qpx.size() * sizeof(double));
                o += (int64_t)pa.qpx.size();
            }
        }
    }
    ~Solver() override {
        for (auto& g : fcg_graphs)
            for (hipGraphExec_t ex : {g.second.one, g.second.run})
                if (ex) (void)hipGraphExecDestroy(ex);
        for (void* p : {(void*)h_nactive, (void*)h_sc, (void*)h_done}) {
            if (!p) continue;
            if (arena.pool) arena.pool->put_host(p);
            else (void)hipHostFree(p);
        }
    }
};

template <typename T>
void Solver<T>::setup() {
    Plan& pl = *plan;
    N = pl.N;
    dim = pl.dim;
    nlev = pl.max_levels;
    hipStream_t st = stream;
    arena.budget = pl.opt.hbm_budget;
    int pmax = 0;
    for (auto& pa : pl.patches)
        for (int d = 0; d < dim; ++d) pmax = std::max(pmax, pa.p[d]);
    cheb_m = cheb_degree_for(pl.opt, dim, pmax);
    cheb_mc = cheb_degree_coarse_for(pl.opt, dim, pmax);
    if (cheb_m > KMAX || cheb_mc > KMAX) throw Error(IETI_ENOTSUP, "Chebyshev degree above 8");
    lev.resize(nlev);
    // ---- descriptors, layouts, tiles
    for (int l = 0; l < nlev; ++l) {
        DevLevel& D = lev[l];
        int64_t cur = 0, ccur = 0;
        for (int k = 0; k < N; ++k) {
            const Patch& pa = pl.patches[k];
            if ((int)pa.lv.size() <= l) continue;
            const Level& L = pa.lv[l];
            PatchLev P{};
            for (int d = 0; d < 3; ++d) {
                P.M[d] = L.M[d];
                P.p[d] = d < dim ? L.p[d] : 0;
            }
            P.dim = dim;
            P.nst = L.nst;
            P.pclass = degree_class(dim, P.p[0], P.p[1], P.p[2]);
            const uint32_t all = dim == 3 ? 0x3Fu : 0xFu;
            P.mbits[MODE_N] = pa.bside | ((pa.pcorner | pa.dcorner) << 8);
            P.mbits[MODE_D] = all;
            P.mbits[MODE_K] = pa.bside | (pa.dcorner << 8);
            P.patch = k;
            P.coarse = -1;
            P.fine = -1;
            P.moff[0] = P.moff[1] = P.moff[2] = -1;
            P.n = L.n;
            P.voff = align64(cur + L.guard);
            cur = P.voff + L.n + L.guard;
            P.cstride = align64(L.n + 2 * L.guard);
            P.coff = align64(ccur) + L.guard;
            ccur = align64(ccur) + (int64_t)L.nst * P.cstride;
            P.lmax[0] = L.lmax[0];
            P.lmax[1] = L.lmax[1];
            int pk = 0;
            for (int d = 0; d < dim; ++d) pk = std::max(pk, pa.p[d]);
            P.clo = cheb_lower_for(pl.opt, dim, pk);
            D.hL.push_back(P);
        }
        D.len = align64(cur) + 64;
        D.clen = align64(ccur) + 64;
    }
    // cross-level indices
    for (int l = 0; l + 1 < nlev; ++l) {
        DevLevel& F = lev[l];
        DevLevel& C = lev[l + 1];
        for (size_t c = 0; c < C.hL.size(); ++c)
            for (size_t f = 0; f < F.hL.size(); ++f)
                if (F.hL[f].patch == C.hL[c].patch) {
                    F.hL[f].coarse = (int)c;
                    C.hL[c].fine = (int)f;
                }
    }
    const double hi = cheb_hi;
    for (int l = 0; l < nlev; ++l) {
        DevLevel& D = lev[l];
        for (int c = 0; c <= NCLASS; ++c) {
            D.cls_beg_all[c] = (int)D.h_all.size();
            for (size_t i = 0; i < D.hL.size(); ++i) {
                const PatchLev& P = D.hL[i];
                if (P.pclass != c) continue;
                for (int64_t s = 0; s < P.n; s += TILE)
                    D.h_all.push_back({(int32_t)i, (int32_t)s, (int32_t)D.h_all.size(), 0});
            }
            D.cls_end_all[c] = (int)D.h_all.size();
        }
        for (int c = 0; c <= NCLASS; ++c) {
            D.cls_beg_sm[c] = (int)D.h_smooth.size();
            for (int t = D.cls_beg_all[c]; t < D.cls_end_all[c]; ++t)
                if (D.hL[D.h_all[t].pl].coarse >= 0) D.h_smooth.push_back(D.h_all[t]);
            D.cls_end_sm[c] = (int)D.h_smooth.size();
        }
        for (size_t i = 0; i < D.hL.size(); ++i)
            if (D.hL[i].coarse < 0) D.h_coarse.push_back((int32_t)i);
        D.nt_all = (int)D.h_all.size();
        D.nt_smooth = (int)D.h_smooth.size();
        D.n_coarse = (int)D.h_coarse.size();
        for (const PatchLev& P : D.hL) {
            const int c = P.pclass;
            D.reach[c] = std::max(D.reach[c], P.p[2] * P.M[0] * P.M[1] + P.p[1] * P.M[0] + P.p[0]);
            D.words_all[c] += (double)P.n;
            D.st_all[c] += (double)P.n * P.nst;
            if (P.coarse >= 0) {
                D.words_smooth[c] += (double)P.n;
                D.st_smooth[c] += (double)P.n * P.nst;
            }
        }
        D.cheb = arena.upload(cheb_table(D, hi, 1.0), st);
        if (l == 0) {
            stage_all0 = true;
            for (int c = 0; c <= NCLASS; ++c) {
                if (D.cls_end_sm[c] <= D.cls_beg_sm[c]) continue;
                if (c == NCLASS || (size_t)(TILE + 2 * D.reach[c]) * sizeof(T) > STAGE_X_MAX_BYTES) stage_all0 = false;
            }
        }
        HIPCHECK(hipStreamSynchronize(st));
    }
    // ---- L2-projection transfer of the finest level (degree-1 coarse levels): mass factors per direction
    {
        std::vector<double> mc;
        std::vector<int32_t> lst;
        DevLevel& D = lev[0];
        for (size_t i = 0; i < D.hL.size(); ++i) {
            PatchLev& P = D.hL[i];
            const Level& L = pl.patches[P.patch].lv[0];
            if (P.coarse < 0 || !L.l2) continue;
            for (int d = 0; d < dim; ++d) {
                P.moff[d] = (int64_t)mc.size();
                mc.insert(mc.end(), L.mchol[d].begin(), L.mchol[d].end());
            }
            lst.push_back((int32_t)i);
            l2_lds = std::max(l2_lds, (size_t)L.n * sizeof(T));
        }
        if (!lst.empty()) {
            int dev = 0, max_lds = 0;
            HIPCHECK(hipGetDevice(&dev));
            HIPCHECK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
            if (l2_lds > (size_t)max_lds)
                throw Error(IETI_ENOTSUP, "degree-1 coarse levels: a patch's finest level exceeds the LDS of the mass solve");
            HIPCHECK(hipFuncSetAttribute((const void*)k_mass_solve<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)l2_lds));
            l2_on = true;
            l2_n = (int)lst.size();
            l2_mchol = arena.upload(mc, st);
            l2_list = arena.upload(lst, st);
            HIPCHECK(hipStreamSynchronize(st));
        }
    }
    // ---- transfer tables, stencils, inverses
    for (int l = 0; l < nlev; ++l) {
        DevLevel& D = lev[l];
        std::vector<int32_t> plo, rlo;
        std::vector<T> pval, rval;
        std::vector<T> coefT(D.clen, T(0));
        std::vector<double> c64;
        if (l == 0) c64.assign(D.clen, 0.0);
        std::vector<T> inv;
        for (auto& P : D.hL) {
            const Patch& pa = pl.patches[P.patch];
            const Level& L = pa.lv[l];
            for (int s = 0; s < L.nst; ++s)
                for (int64_t i = 0; i < L.n; ++i) {
                    double v = L.coef[(size_t)s * L.n + i];
                    coefT[P.coff + s * P.cstride + i] = T(v);
                    if (l == 0) c64[P.coff + s * P.cstride + i] = v;
                }
            if (P.coarse >= 0) {
                for (int d = 0; d < dim; ++d) {
                    // nested levels: the embedding's columns hold p + 2 entries, its rows at most
                    // prol_width(p) (the kernels read that many); the L2 projection's mixed mass matrix M_fc
                    // (degree p onto degree 1) up to PW both ways
                    const int Mf = L.M[d], Mc = L.Mc[d], w = L.l2 ? PW : L.p[d] + 2;
                    const int wr = L.l2 ? PW : prol_width(L.p[d]);
                    if (w > PW) throw Error(IETI_ENOTSUP, "degree too high for the transfer tables");
                    const std::vector<double>& Pm = L.P[d];
                    P.toff[d] = (int64_t)plo.size();
                    for (int r = 0; r < Mf; ++r) {
                        int cmin = Mc, cmax = -1;
                        for (int c = 0; c < Mc; ++c)
                            if (Pm[(size_t)r * Mc + c] != 0.0) { cmin = std::min(cmin, c); cmax = std::max(cmax, c); }
                        if (cmax < 0) cmin = cmax = 0;
                        if (cmax - cmin + 1 > wr) throw Error(IETI_ENOTSUP, "prolongation row wider than the table");
                        int lo = std::max(0, std::min(cmin, Mc - wr));
                        plo.push_back(lo);
                        for (int a = 0; a < PW; ++a) {
                            int c = lo + a;
                            pval.push_back(a < wr && c < Mc ? T(Pm[(size_t)r * Mc + c]) : T(0));
                        }
                    }
                    P.roff[d] = (int64_t)rlo.size();
                    for (int c = 0; c < Mc; ++c) {
                        int rmin = Mf, rmax = -1;
                        for (int r = 0; r < Mf; ++r)
                            if (Pm[(size_t)r * Mc + c] != 0.0) { rmin = std::min(rmin, r); rmax = std::max(rmax, r); }
                        if (rmax < 0) rmin = rmax = 0;
                        if (rmax - rmin + 1 > w) throw Error(IETI_ENOTSUP, "restriction column wider than the table");
                        int lo = std::max(0, std::min(rmin, Mf - w));
                        rlo.push_back(lo);
                        for (int a = 0; a < PW; ++a) {
                            int r = lo + a;
                            rval.push_back(a < w && r < Mf ? T(Pm[(size_t)r * Mc + c]) : T(0));
                        }
                    }
                }
            } else if (pl.opt.local_solver != IETI_LOCAL_EXACT) {
                // stored by columns: entry (r, j) at j * n + r; a mode without multigrid (D-MG: Neumann) holds zeros
                P.invoff = (int64_t)inv.size();
                const int64_t n = L.n;
                for (int m = 0; m < 2; ++m)
                    for (int64_t j = 0; j < n; ++j)
                        for (int64_t r = 0; r < n; ++r)
                            inv.push_back(L.inv[m].empty() ? T(0) : T(L.inv[m][(size_t)(r * n + j)]));
            }
        }
        D.L = arena.upload(D.hL, st);
        D.tiles_all = arena.upload(D.h_all, st);
        D.tiles_smooth = arena.upload(D.h_smooth, st);
        D.coarse_list = arena.upload(D.h_coarse, st);
        D.plo = arena.upload(plo, st);
        D.rlo = arena.upload(rlo, st);
        D.pval = arena.upload(pval, st);
        D.rval = arena.upload(rval, st);
        D.coefT = arena.upload(coefT, st);
        D.inv = arena.upload(inv, st);
        if (l == 0) {
            if (std::is_same<T, double>::value) coef64 = (double*)D.coefT;
            else coef64 = arena.upload(c64, st);
        }
        D.vb = arena.alloc<T>(D.len, st);
        D.vx = arena.alloc<T>(D.len, st);
        D.vxa = arena.alloc<T>(D.len, st);
        D.vd = arena.alloc<T>(D.len, st);
        D.vr = arena.alloc<T>(D.len, st);
        HIPCHECK(hipStreamSynchronize(st));   // host vectors above go out of scope
    }
    // ---- fused coarse V-cycle
    // Start level with coarse_level = 0: level 1, with the operator data
    // staged in LDS when every chain fits, else read from memory (batched
    // launches of a coarse level cost more than the fused kernel's sweeps);
    // the lowest level from which the vectors fit if level 1 does not.
    fuse_l0 = nlev;
    if (nlev > 1 && nlev <= LMAX && pl.opt.local_solver != IETI_LOCAL_EXACT && pl.opt.coarse_level >= 0) {
        int dev = 0;
        HIPCHECK(hipGetDevice(&dev));
        int max_lds = 0;
        HIPCHECK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        const int64_t budget = (int64_t)max_lds - 1024;   // static shared memory of the kernel
        // the coarsest GEMV's partial sums: one double per thread of the wider family
        const int64_t part_words =
            (int64_t)std::max(vc_threads<T, 0>(), vc_threads<T, 1>()) * (int64_t)(sizeof(double) / sizeof(T));
        auto chain_bytes = [&](int k, int f, bool stage) -> int64_t {
            const Patch& pa = pl.patches[k];
            const int nl = (int)pa.lv.size();
            int64_t w = 0;
            for (int l = f; l < nl; ++l) {
                const Level& L = pa.lv[l];
                w += vcoarse_level_words(L.n, L.guard, L.nst, l == nl - 1, stage, part_words);
            }
            return w * (int64_t)sizeof(T);
        };
        auto feasible = [&](int f, bool stage) {
            for (int k = 0; k < N; ++k)
                if ((int)pl.patches[k].lv.size() > f && chain_bytes(k, f, stage) > budget) return false;
            return true;
        };
        int f = nlev;
        bool stage = false;
        if (pl.opt.coarse_level > 0) {
            f = std::min(pl.opt.coarse_level, nlev - 1);
            stage = feasible(f, true);
            if (!stage && !feasible(f, false)) f = nlev;
        } else if (feasible(1, true)) {
            f = 1;
            stage = true;
        } else {
            for (int g = 1; g < nlev && f == nlev; ++g)
                if (feasible(g, false)) f = g;
        }
        if (f < nlev) {
            fuse_l0 = f;
            fuse_stage = stage;
            std::vector<int32_t> ch((size_t)N * LMAX, -1);
            for (int l = 0; l < nlev; ++l)
                for (size_t i = 0; i < lev[l].hL.size(); ++i) ch[(size_t)lev[l].hL[i].patch * LMAX + l] = (int32_t)i;
            chain = arena.upload(ch, st);
            std::vector<std::pair<int64_t, int32_t>> order[2];
            for (int k = 0; k < N; ++k) {
                if ((int)pl.patches[k].lv.size() <= f) continue;
                const int64_t b = chain_bytes(k, f, stage);
                const int fam = vcoarse_family(lev[f].hL[ch[(size_t)k * LMAX + f]].pclass);
                order[fam].push_back({-b, k});
                vc_lds[fam] = std::max(vc_lds[fam], (size_t)b);
                // algorithmic bytes of the patch's fused part: its right-hand side in and correction out, every
                // smoothed level's half stencil and the coarsest inverse once
                const Patch& pa = pl.patches[k];
                const int nl = (int)pa.lv.size();
                double w = 2.0 * (double)pa.lv[f].n;
                for (int q = f; q < nl; ++q)
                    w += q == nl - 1 ? (double)pa.lv[q].n * (double)pa.lv[q].n : (double)pa.lv[q].nst * (double)pa.lv[q].n;
                vc_bytes[fam] += w * sizeof(T);
            }
            for (int fam = 0; fam < 2; ++fam) {
                std::sort(order[fam].begin(), order[fam].end());
                for (auto& o : order[fam]) h_plist[fam].push_back(o.second);
                if (h_plist[fam].empty()) continue;
                plist[fam] = arena.upload(h_plist[fam], st);
                CoarseArgs dummy{};
                launch_vcoarse<T>(fam, stage, st, dummy, vc_lds[fam], true);
            }
        }
        HIPCHECK(hipStreamSynchronize(st));
    }
    // ---- tensor-product smoother of the finest level
    if (pl.opt.smoother == IETI_SMOOTHER_TENSOR && pl.opt.local_solver != IETI_LOCAL_EXACT && nlev > 1) {
        std::vector<double> hu, hl;
        std::vector<FdInfo> info(2 * (size_t)N);
        int64_t zlen = 0;
        for (int k = 0; k < N; ++k) {
            const Patch& pa = pl.patches[k];
            if (lev[0].hL[k].patch != k) throw Error(IETI_EDEVICE, "internal: level-0 patch order");
            int64_t zk = 0;
            for (int m = 0; m < 2; ++m) {
                const Patch::Tensor& Tz = pa.ts[m];
                FdInfo& f = info[(size_t)m * N + k];
                f = FdInfo{};
                if (Tz.U[0].empty()) continue;
                f.P0 = Tz.Pd[0];
                f.P1 = Tz.Pd[1];
                f.P2 = dim == 3 ? Tz.Pd[2] : 0;
                f.u0 = (int64_t)hu.size();
                hu.insert(hu.end(), Tz.U[0].begin(), Tz.U[0].end());
                f.u1 = (int64_t)hu.size();
                hu.insert(hu.end(), Tz.U[1].begin(), Tz.U[1].end());
                f.l0 = (int64_t)hl.size();
                hl.insert(hl.end(), Tz.lam[0].begin(), Tz.lam[0].end());
                f.l1 = (int64_t)hl.size();
                hl.insert(hl.end(), Tz.lam[1].begin(), Tz.lam[1].end());
                if (dim == 3) {
                    f.u2 = (int64_t)hu.size();
                    hu.insert(hu.end(), Tz.U[2].begin(), Tz.U[2].end());
                    f.l2 = (int64_t)hl.size();
                    hl.insert(hl.end(), Tz.lam[2].begin(), Tz.lam[2].end());
                    fd_tiles3 = std::max(fd_tiles3, f.P0 * f.P1 * f.P2 / 256);
                } else {
                    fd_tiles2 = std::max(fd_tiles2, f.P0 * f.P1 / 256);
                }
                f.zoff = zlen;   // one scratch per patch: the two modes never run at the same time
                f.shift = Tz.shift;
                f.tau = Tz.tau;
                zk = std::max(zk, (int64_t)f.P0 * f.P1 * (dim == 3 ? f.P2 : 1));
                fd_p0max = std::max(fd_p0max, f.P0);
                fd_p1max = std::max(fd_p1max, f.P1);
                fd_p2max = std::max(fd_p2max, f.P2);
            }
            zlen += zk;
        }
        if (dim == 3 && (fd_p0max > 128 || fd_p1max > 128))
            throw Error(IETI_ENOTSUP, "tensor smoother: more than 128 coefficients per direction in 3D");
        if (fd_p0max > 0) {
            fd_on = true;
            fd_U = arena.upload(hu, st);
            fd_lam = arena.upload(hl, st);
            if (dim == 2 && std::is_same<T, float>::value) {   // the 2D transforms run in FP32
                std::vector<float> hu32(hu.begin(), hu.end());
                fd_U32 = arena.upload(hu32, st);
                fd_z32 = arena.alloc<float>(zlen, st);
                fd_z232 = arena.alloc<float>(zlen, st);
            } else {
                fd_z = arena.alloc<double>(zlen, st);
                fd_z2 = arena.alloc<double>(zlen, st);
            }
            std::vector<FdInfo> i0(info.begin(), info.begin() + N), i1(info.begin() + N, info.end());
            fd_info[0] = arena.upload(i0, st);
            fd_info[1] = arena.upload(i1, st);
            HIPCHECK(hipStreamSynchronize(st));
        }
    }
    // ---- exact local solves
    if (pl.opt.local_solver == IETI_LOCAL_EXACT || pl.opt.local_solver == IETI_LOCAL_EXACT_MG) {
        exact = true;
        prec_exact = pl.opt.local_solver == IETI_LOCAL_EXACT;
        if (dim == 3) {
            setup_band3();
        } else {
        int dev = 0, max_lds = 0;
        HIPCHECK(hipGetDevice(&dev));
        HIPCHECK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        std::vector<int64_t> offs(2 * (size_t)N);
        std::vector<int32_t> bw(N);
        int64_t tot = 0;
        for (int k = 0; k < N; ++k) {
            const Patch& pa = pl.patches[k];
            bw[k] = (int32_t)pa.band_b;
            band_bmax = std::max(band_bmax, (int)pa.band_b);
            for (int m = 0; m < 2; ++m) {
                offs[2 * k + m] = tot;
                tot += (int64_t)pa.band[m].size();
            }
            const size_t lds = sizeof(double) * (size_t)(2 * pa.band_b + pa.band_nblk * BNB + BNB);
            band_lds = std::max(band_lds, lds);
        }
        if ((int64_t)band_lds > max_lds) throw Error(IETI_ENOTSUP, "patch too large for exact local solves in LDS");
        band = arena.alloc<double>(tot, st, false);
        for (int k = 0; k < N; ++k)
            for (int m = 0; m < 2; ++m)
                HIPCHECK(hipMemcpyAsync(band + offs[2 * k + m], pl.patches[k].band[m].data(),
                                        pl.patches[k].band[m].size() * sizeof(double), hipMemcpyHostToDevice, st));
        band_off = arena.upload(offs, st);
        band_b = arena.upload(bw, st);
        HIPCHECK(hipFuncSetAttribute((const void*)k_band_solve, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)band_lds));
        HIPCHECK(hipFuncSetAttribute((const void*)k_band_solve_pf<16, true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)band_lds));
        HIPCHECK(hipFuncSetAttribute((const void*)k_band_solve_pf<32, false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)band_lds));
        HIPCHECK(hipStreamSynchronize(st));
        }
    }
    DevLevel& D0 = lev[0];
    len0 = D0.len;
    for (double** p : {&f64, &b64, &e64, &w64, &s64, &u64, &fx, &fr, &fd, &fq}) *p = arena.alloc<double>(len0, st);
    for (T** p : {&rT, &zT, &bT, &xIT, &x2T, &r2T}) *p = arena.alloc<T>(len0, st);
    if (l2_on) l2_tmp = arena.alloc<T>(len0, st);
    partial = arena.alloc<double>(4 * (int64_t)D0.nt_all + 4, st);
    if (pl.opt.local_solver == IETI_LOCAL_MG_SADDLE) {
        saddle = true;
        for (double** p : {&bx, &br, &bz, &bhz, &bp, &bs, &bt, &bht, &bg, &bw, &bg2}) *p = arena.alloc<double>(len0, st);
        const int64_t nlb = std::max<int64_t>(pl.n_lambda, 1);
        for (double** p : {&lxx, &lrr, &lzz, &lhz, &lpp, &lss, &ltt, &lht}) *p = arena.alloc<double>(nlb, st);
        bsc = arena.alloc<double>(16, st);
        ndpart = 1024;
        dpart = arena.alloc<double>(ndpart, st);
    }
    {
        std::vector<int32_t> tb(N, 0), te(N, 0);
        for (size_t t = 0; t < D0.h_all.size(); ++t) {
            const int k = D0.hL[D0.h_all[t].pl].patch;
            if (te[k] == 0) tb[k] = (int32_t)t;
            te[k] = (int32_t)t + 1;
        }
        tile_beg = arena.upload(tb, st);
        tile_end = arena.upload(te, st);
    }
    bb = arena.alloc<double>(N, st);
    dq = arena.alloc<double>(N, st);
    beta = arena.alloc<double>(N, st);
    alpha = arena.alloc<double>(N, st);
    active = arena.alloc<int>(N, st);
    its = arena.alloc<int>(N, st);
    brk = arena.alloc<int>(N, st);
    nactive = arena.alloc<int>(8, st);
    h_its.assign(N, 0);
    ncomp = std::max(1, pl.ncomp);
    if (ncomp > 1 && pl.opt.local_solver == IETI_LOCAL_MG_SADDLE)
        throw Error(IETI_ENOTSUP, "MG-MG-S solves one problem at a time");
    h_comp_lam = pl.comp_lam_beg;
    if ((int)h_comp_lam.size() != ncomp + 1) h_comp_lam = {0, pl.n_lambda};
    {
        std::vector<int64_t> cp = pl.comp_patch_beg;
        if ((int)cp.size() != ncomp + 1) cp = {0, (int64_t)N};
        comp_lam = arena.upload(h_comp_lam, st);
        comp_patch = arena.upload(cp, st);
    }
    done_dev = arena.alloc<int>(ncomp, st);
    auto pinned = [&](size_t b) -> void* {
        void* p = nullptr;
        if (arena.pool) p = arena.pool->get_host(b);
        else if (hipHostMalloc(&p, b) != hipSuccess) p = nullptr;
        if (!p) throw Error(IETI_ENOMEM, "hipHostMalloc failed");
        return p;
    };
    h_nactive = (int*)pinned(sizeof(int));
    h_sc = (double*)pinned(16 * (size_t)ncomp * sizeof(double));
    h_done = (int*)pinned((size_t)ncomp * sizeof(int));

    // ---- jump operators (device positions on level 0)
    auto devpos = [&](int64_t torn) {
        int lo = 0, hi = N - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) / 2;
            if (pl.patches[mid].torn_off <= torn) lo = mid; else hi = mid - 1;
        }
        return D0.hL[lo].voff + (torn - pl.patches[lo].torn_off);
    };
    auto patch_of = [&](int64_t torn) {
        int lo = 0, hi = N - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) / 2;
            if (pl.patches[mid].torn_off <= torn) lo = mid; else hi = mid - 1;
        }
        return lo;
    };
    nslots = (int64_t)pl.slot_pos.size();
    nlam = pl.n_lambda;
    {
        std::vector<int64_t> sd(nslots), rp(N + 1, 0);
        std::vector<int32_t> sp(nslots);
        std::vector<double> wb(pl.slot_lam.size()), wbd(pl.slot_lam.size());
        for (int64_t s = 0; s < nslots; ++s) {
            sd[s] = devpos(pl.slot_pos[s]);
            sp[s] = patch_of(pl.slot_pos[s]);
            rp[sp[s] + 1]++;
            for (int64_t e = pl.slot_ptr[s]; e < pl.slot_ptr[s + 1]; ++e) {
                wb[e] = pl.slot_sgn[e];
                wbd[e] = pl.slot_sgn[e] / (double)pl.slot_mult[s];
            }
        }
        for (int k = 0; k < N; ++k) rp[k + 1] += rp[k];
        slot_dev = arena.upload(sd, st);
        slot_patch = arena.upload(sp, st);
        row_ptr = arena.upload(rp, st);
        slot_ptr = arena.upload(pl.slot_ptr, st);
        slot_lam = arena.upload(pl.slot_lam, st);
        slot_wB = arena.upload(wb, st);
        slot_wBD = arena.upload(wbd, st);
        std::vector<int64_t> lp(nlam), lm(nlam);
        std::vector<double> lw(nlam);
        for (int64_t l = 0; l < nlam; ++l) {
            lp[l] = devpos(pl.lam_plus[l]);
            lm[l] = devpos(pl.lam_minus[l]);
            lw[l] = 1.0 / (double)pl.lam_mult[l];
        }
        lam_plus = arena.upload(lp, st);
        lam_minus = arena.upload(lm, st);
        lam_wBD = arena.upload(lw, st);
        std::vector<int64_t> gp = pl.grp_ptr, gd(pl.grp_pos.size());
        for (size_t i = 0; i < gd.size(); ++i) gd[i] = devpos(pl.grp_pos[i]);
        ngroups = (int64_t)gp.size() - 1;
        grp_ptr = arena.upload(gp, st);
        grp_dev = arena.upload(gd, st);
        std::vector<int64_t> to(N);
        for (int k = 0; k < N; ++k) to[k] = pl.patches[k].torn_off;
        torn_off = arena.upload(to, st);
        HIPCHECK(hipStreamSynchronize(st));
    }
    // ---- lambda space
    int64_t nl = std::max<int64_t>(nlam, 1);
    lam = arena.alloc<double>(nl, st);
    lr = arena.alloc<double>(nl, st);
    lz = arena.alloc<double>(nl, st);
    lp = arena.alloc<double>(nl, st);
    lq = arena.alloc<double>(nl, st);
    ltmp = arena.alloc<double>(nl, st);
    sc = arena.alloc<double>(16 * (int64_t)ncomp, st);
    pcgp = arena.alloc<double>(2 * (int64_t)PCG_NB * ncomp, st);
    // ---- load-vector tables
    {
        std::vector<PatchQ> pq(N);
        std::vector<double> bas, w, x;
        int64_t qo = 0;
        for (int k = 0; k < N; ++k) {
            const Patch& pa = pl.patches[k];
            PatchQ& Q = pq[k];
            for (int d = 0; d < 3; ++d) {
                Q.nel[d] = d < dim ? pa.lv[0].nel[d] : 1;
                Q.Q[d] = d < dim ? Q.nel[d] * (pa.p[d] + 1) : 1;
                Q.boff[d] = (int64_t)bas.size();
                if (d < dim) bas.insert(bas.end(), pa.qpN[d].begin(), pa.qpN[d].end());
            }
            Q.qoff = qo;
            qo += pa.n_qp;
            w.insert(w.end(), pa.qpw.begin(), pa.qpw.end());
            x.insert(x.end(), pa.qpx.begin(), pa.qpx.end());
            // sum factorisation of the load vector: direction 0 contracted (M0 Q1 Q2), then direction 1
            // (M0 M1 Q2, 3D); the last pass writes the coefficients
            const int64_t M0 = pa.lv[0].M[0], M1 = pa.lv[0].M[1];
            const int64_t t1 = M0 * Q.Q[1] * Q.Q[2], t2 = dim == 3 ? M0 * M1 * Q.Q[2] : 0;
            Q.toff[0] = qtmp_len;
            Q.toff[1] = qtmp_len + t1;
            qtmp_len += t1 + t2;
            qc_grid[0] = std::max(qc_grid[0], (t1 + TILE - 1) / TILE);
            qc_grid[1] = std::max(qc_grid[1], ((dim == 3 ? t2 : pa.lv[0].n) + TILE - 1) / TILE);
            qc_grid[2] = std::max(qc_grid[2], (pa.lv[0].n + TILE - 1) / TILE);
        }
        qtmp = arena.alloc<double>(qtmp_len, st);
        PQ = arena.upload(pq, st);
        basis = arena.upload(bas, st);
        qpw = arena.upload(w, st);
        qpx = arena.upload(x, st);
        HIPCHECK(hipStreamSynchronize(st));
    }
    // ---- primal space
    npi = pl.n_primal;
    // the coarse GEMV keeps g_Pi in LDS (64 KB)
    if (npi > 8192) throw Error(IETI_ENOTSUP, "more than 8192 primal unknowns (dense coarse problem)");
    {
        std::vector<int32_t> nk(N);
        std::vector<int64_t> R((size_t)N * NPMAX, 0), ud((size_t)N * NPMAX, -1), ep((size_t)N * NPMAX + 1, 0), ed;
        for (int k = 0; k < N; ++k) {
            const Patch& pa = pl.patches[k];
            nk[k] = (int32_t)pa.primal_global.size();
            if (nk[k] > NPMAX) throw Error(IETI_ENOTSUP, "too many primal constraints on a patch");
            npk_max = std::max(npk_max, nk[k]);
            for (int j = 0; j < NPMAX; ++j) {
                ep[(size_t)k * NPMAX + j] = (int64_t)ed.size();
                if (j < nk[k]) {
                    R[(size_t)k * NPMAX + j] = pa.primal_global[j];
                    if (pa.primal_corner[j] >= 0) {
                        int c = pa.primal_corner[j];
                        int idx[3] = {0, 0, 0};
                        for (int d = 0; d < dim; ++d) idx[d] = (c >> d & 1) ? pa.lv[0].M[d] - 1 : 0;
                        int64_t li = idx[0] + (int64_t)pa.lv[0].M[0] * (idx[1] + (int64_t)pa.lv[0].M[1] * idx[2]);
                        ud[(size_t)k * NPMAX + j] = D0.hL[k].voff + li;
                    } else {
                        for (int64_t li : pa.primal_edge[j]) ed.push_back(D0.hL[k].voff + li);
                    }
                }
            }
        }
        ep[(size_t)N * NPMAX] = (int64_t)ed.size();
        npk = arena.upload(nk, st);
        Rk = arena.upload(R, st);
        unit_dev = arena.upload(ud, st);
        edge_ptr = arena.upload(ep, st);
        edge_dev = arena.upload(ed, st);
        pri_ptr = arena.upload(pl.pri_ptr, st);
        pri_patch = arena.upload(pl.pri_patch, st);
        pri_local = arena.upload(pl.pri_local, st);
        std::vector<int32_t> fl;
        std::vector<double> fg(N, 0.0);
        for (int k = 0; k < N; ++k)
            if (pl.patches[k].floating) {
                fl.push_back(k);
                fg[k] = pl.patches[k].float_gamma;
            }
        n_float = (int)fl.size();
        if (n_float) {
            float_list = arena.upload(fl, st);
            float_gam = arena.upload(fg, st);
        }
        cbuf = arena.alloc<double>((int64_t)N * NPMAX, st);
        ebuf = arena.alloc<double>((int64_t)N * NPMAX, st);
        coefbuf = arena.alloc<double>((int64_t)N * NPMAX, st);
        upi = arena.alloc<double>(std::max<int64_t>(npi, 1), st);
        psiG = arena.alloc<double>(std::max<int64_t>(nslots, 1) * NPMAX, st);
        HIPCHECK(hipStreamSynchronize(st));
    }
    if (npi > 0) {
        const int nj = npk_max;
        psi = arena.alloc<double>((int64_t)nj * len0, st);
        // raw columns Y_j = K_rr^{-1} rhs_j (device scratch for setup, released below)
        double* Y = arena.alloc<double>((int64_t)nj * len0, st, false);
        HIPCHECK(hipMemsetAsync(Y, 0, sizeof(double) * (size_t)nj * len0, st));
        for (int j = 0; j < nj; ++j) {
            fill<double>(e64, len0, 0.0);
            hipLaunchKernelGGL(k_unit, dim3(nblk(N, 256)), dim3(256), 0, st, N, unit_dev, j, e64);
            check_launch();
            stencil<double, double, double, EPI_APPLY>(0, false, MODE_N, coef64, e64, b64, nullptr, nullptr, nullptr,
                                                       -1.0, 0);
            hipLaunchKernelGGL(k_edge_rhs, dim3(N), dim3(256), 0, st, N, edge_ptr, edge_dev, j, b64);
            check_launch();
            local_solve(b64, pl.opt.basis_tol);
            HIPCHECK(hipMemcpyAsync(Y + (size_t)j * len0, fx, sizeof(double) * len0, hipMemcpyDeviceToDevice, st));
        }
        // edge means of the raw columns -> combination coefficients (host, tiny dense algebra)
        double* A = arena.alloc<double>((int64_t)N * NPMAX * NPMAX, st);
        hipLaunchKernelGGL(k_edge_avg, dim3(N), dim3(TILE), 0, st, N, npk, edge_ptr, edge_dev, Y, len0, A);
        check_launch();
        std::vector<double> hA((size_t)N * NPMAX * NPMAX), hT((size_t)N * NPMAX * NPMAX, 0.0);
        HIPCHECK(hipMemcpyAsync(hA.data(), A, hA.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        sync();
        for (int k = 0; k < N; ++k) {
            const Patch& pa = pl.patches[k];
            const int nkj = (int)pa.primal_global.size();
            std::vector<int> V, E;
            for (int j = 0; j < nkj; ++j) (pa.primal_corner[j] >= 0 ? V : E).push_back(j);
            const int ne = (int)E.size();
            auto Aat = [&](int col, int e) { return hA[((size_t)k * NPMAX + col) * NPMAX + e]; };
            // H[e][e'] = mean over edge e of raw column e'
            std::vector<double> H((size_t)ne * ne), Hi((size_t)ne * ne, 0.0);
            for (int a = 0; a < ne; ++a)
                for (int b = 0; b < ne; ++b) H[(size_t)a * ne + b] = Aat(E[b], E[a]);
            // invert H by Gauss-Jordan with partial pivoting
            for (int a = 0; a < ne; ++a) Hi[(size_t)a * ne + a] = 1.0;
            for (int c = 0; c < ne; ++c) {
                int piv = c;
                for (int r = c + 1; r < ne; ++r)
                    if (std::fabs(H[(size_t)r * ne + c]) > std::fabs(H[(size_t)piv * ne + c])) piv = r;
                if (H[(size_t)piv * ne + c] == 0.0) throw Error(IETI_EINVAL, "singular edge-average system");
                for (int q = 0; q < ne; ++q) {
                    std::swap(H[(size_t)c * ne + q], H[(size_t)piv * ne + q]);
                    std::swap(Hi[(size_t)c * ne + q], Hi[(size_t)piv * ne + q]);
                }
                double dv = H[(size_t)c * ne + c];
                for (int q = 0; q < ne; ++q) {
                    H[(size_t)c * ne + q] /= dv;
                    Hi[(size_t)c * ne + q] /= dv;
                }
                for (int r = 0; r < ne; ++r)
                    if (r != c) {
                        double f = H[(size_t)r * ne + c];
                        if (f == 0.0) continue;
                        for (int q = 0; q < ne; ++q) {
                            H[(size_t)r * ne + q] -= f * H[(size_t)c * ne + q];
                            Hi[(size_t)r * ne + q] -= f * Hi[(size_t)c * ne + q];
                        }
                    }
            }
            auto Tset = [&](int jp, int j, double v) { hT[((size_t)k * NPMAX + jp) * NPMAX + j] = v; };
            // edge columns: psi_e = sum_e' Y_e' Hinv[e'][e]
            for (int a = 0; a < ne; ++a)
                for (int b = 0; b < ne; ++b) Tset(E[b], E[a], Hi[(size_t)b * ne + a]);
            // vertex columns: psi_v = e_v + Y_v - Psi_E (C_E Y_v)
            for (int v : V) {
                Tset(v, v, 1.0);
                for (int b = 0; b < ne; ++b) {
                    double s = 0.0;
                    for (int a = 0; a < ne; ++a) s += Hi[(size_t)b * ne + a] * Aat(v, E[a]);
                    Tset(E[b], v, -s);
                }
            }
        }
        double* Tm = arena.upload(hT, st);
        hipLaunchKernelGGL(k_combine, dim3(tile_grid(D0.nt_all)), dim3(TILE), 0, st, D0.L, D0.tiles_all, D0.nt_all,
                           npk, unit_dev, Y, Tm, len0, psi);
        check_launch();
        // local coarse matrices S_k = Psi^T K Psi  (K without the boundary), assembled on the host
        for (int j = 0; j < nj; ++j)
            stencil<double, double, double, EPI_APPLY>(0, false, MODE_K, coef64, psi + (size_t)j * len0,
                                                       Y + (size_t)j * len0, nullptr, nullptr, nullptr, 1.0, 0);
        double* Sk = arena.alloc<double>((int64_t)N * NPMAX * NPMAX, st);
        for (int j = 0; j < nj; ++j) {
            hipLaunchKernelGGL(k_patch_gram, dim3(N), dim3(TILE), 0, st, N, D0.L, npk, psi, Y, len0, j, Sk);
            check_launch();
        }
        std::vector<double> hS((size_t)N * NPMAX * NPMAX);
        HIPCHECK(hipMemcpyAsync(hS.data(), Sk, hS.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        sync();
        arena.release(Y, sizeof(double) * (size_t)nj * len0, st);
        std::vector<double> S((size_t)npi * npi, 0.0);
        for (int k = 0; k < N; ++k) {
            const Patch& pa = pl.patches[k];
            const int nkj = (int)pa.primal_global.size();
            for (int a = 0; a < nkj; ++a)
                for (int b = 0; b < nkj; ++b)
                    S[(size_t)pa.primal_global[a] * npi + pa.primal_global[b]] +=
                        0.5 * (hS[((size_t)k * NPMAX + a) * NPMAX + b] + hS[((size_t)k * NPMAX + b) * NPMAX + a]);
        }
        // S^{-1} on the matrix cores: blocked Cholesky, triangular inverse, X^T X (FP64 MFMA)
        spd_inverse(S, npi);
        hipLaunchKernelGGL(k_psi_slots, dim3(nblk(std::max<int64_t>(nslots, 1), 256)), dim3(256), 0, st, nslots,
                           slot_patch, slot_dev, npk, psi, len0, psiG);
        check_launch();
        sync();
    }
    sync();
    if (pl.opt.autotune) autotune_smoother();
    if (saddle) estimate_omega();
}

template <typename T>
int Solver<T>::solve(const double* f_qp, double* u_out, ieti_stats* stp) {
    const Plan& pl = *plan;
    using clk = std::chrono::steady_clock;
    auto ms = [](clk::time_point a, clk::time_point b) { return std::chrono::duration<double, std::milli>(b - a).count(); };
    inner_calls = inner_sum = 0;
    inner_max = 0;
    fill<int>(nactive, 8, 0);
    ieti_stats st{};
    st.ndof_torn = pl.ndof_torn;
    st.ndof_global = pl.ndof_global;
    st.n_lambda = pl.n_lambda;
    st.n_primal = pl.n_primal;
    st.cheb_degree = (exact && prec_exact) || fd_on ? 0 : cheb_m;
    st.cheb_degree_coarse = exact && prec_exact ? 0 : cheb_mc;
    st.cheb_lower = cheb_lower_scale;
    st.fine_tile_staged = stage_fine && !fd_on ? 1 : 0;
    st.tune_cached = tune_cached ? 1 : 0;
    DevLevel& D0 = lev[0];
    sync();
    auto t0 = clk::now();
    // ---- load vector and d = B K~^{-1} f
    for (int d = 0; d < dim; ++d) {
        const double* in = d == 0 ? f_qp : qtmp;
        double* out = d == dim - 1 ? f64 : qtmp;
        hipLaunchKernelGGL(k_qcontract, dim3((unsigned)qc_grid[d], N), dim3(TILE), 0, stream, D0.L, PQ, d, basis, qpw,
                           in, out);
        check_launch();
    }
    // reject non-finite data: |f|^2 must be finite
    hipLaunchKernelGGL(k_sq, dim3(tile_grid(D0.nt_all)), dim3(TILE), 0, stream, D0.L, D0.tiles_all, D0.nt_all, f64,
                       (int)MODE_K, partial);
    check_launch();
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, stream, partial, (int64_t)D0.nt_all, sc + 8);
    check_launch();
    if (saddle) {
        HIPCHECK(hipMemcpyAsync(h_sc, sc, 16 * sizeof(double), hipMemcpyDeviceToHost, stream));
        sync();
        if (!std::isfinite(h_sc[8])) throw Error(IETI_EINVAL, "right-hand side is not finite");
        auto t1s = clk::now();
        const int rc = solve_saddle(st);
        auto t2s = clk::now();
        st.time_rhs_ms = ms(t0, t1s);
        st.time_pcg_ms = ms(t1s, t2s);
        finish_solution(st, u_out);
        st.time_recovery_ms = ms(t2s, clk::now());
        st.time_total_ms = ms(t0, clk::now());
        if (prof.on) prof.collect();
        if (stp) *stp = st;
        return rc;
    }
    ktilde_inv(f64, true, pl.opt.inner_tol, u64);
    const int64_t nl = nlam;
    const int nc = ncomp;
    if (nl > 0) {
        gather(u64, false, lr);
        gather(u64, false, lz, true);
        gather(u64, false, ltmp, false, true);
        hipLaunchKernelGGL(k_norms, dim3(nc), dim3(1024), 0, stream, comp_lam, lr, lz, ltmp, sc + 10);
        check_launch();
    }
    HIPCHECK(hipMemcpyAsync(h_sc, sc, 16 * (size_t)nc * sizeof(double), hipMemcpyDeviceToHost, stream));
    sync();
    if (!std::isfinite(h_sc[8])) throw Error(IETI_EINVAL, "right-hand side is not finite");
    // ---- outer CG, one per problem (ieti_solve: one; a serving batch: one per request), batched launches
    std::vector<double> r0(nc, 0.0), rnorm(nc, 0.0);
    std::vector<int> its_c(nc, 0), conv(nc, 0), brk_c(nc, 0);
    for (int c = 0; c < nc; ++c) {
        const bool has = h_comp_lam[c + 1] > h_comp_lam[c];
        r0[c] = rnorm[c] = has ? std::sqrt(h_sc[16 * c + 10]) : 0.0;
        const double scale = has ? std::sqrt(h_sc[16 * c + 11] + h_sc[16 * c + 12]) : 0.0;
        const double zero_thr = (exact ? 1e-13 : 10.0 * pl.opt.inner_tol) * scale;
        h_done[c] = 0;
        if (!has) {   // no multipliers: the primal part alone solves it
            h_done[c] = 1;
            conv[c] = 1;
        } else if (!(r0[c] > zero_thr && r0[c] > 0.0)) {   // d vanished to rounding: lambda = 0 (reading R10)
            h_done[c] = 1;
            conv[c] = 1;
            brk_c[c] = 1;
        }
    }
    auto t1 = clk::now();
    fill<double>(lam, std::max<int64_t>(nl, 1), 0.0);
    int it = 0;
    auto active_left = [&] {
        for (int c = 0; c < nc; ++c)
            if (!h_done[c]) return true;
        return false;
    };
    if (nl > 0 && active_left()) {
        HIPCHECK(hipMemcpyAsync(done_dev, h_done, nc * sizeof(int), hipMemcpyHostToDevice, stream));
        applyPrec(lr, lz);
        pcg_stage(0, lam, lr, lz, lp, lq);
        while (it < pl.opt.max_it) {
            applyF(lp, lq);
            pcg_stage(1, lam, lr, lz, lp, lq);
            HIPCHECK(hipMemcpyAsync(h_sc, sc, 16 * (size_t)nc * sizeof(double), hipMemcpyDeviceToHost, stream));
            sync();
            ++it;
            for (int c = 0; c < nc; ++c) {
                if (h_done[c]) continue;
                ++its_c[c];
                const double rn = std::sqrt(h_sc[16 * c + 3]);
                rnorm[c] = rn;
                if (!(rn - rn == 0.0)) {   // NaN or Inf: stopped, not converged
                    h_done[c] = 1;
                } else if (rn <= pl.opt.tol * r0[c]) {
                    h_done[c] = 1;
                    conv[c] = 1;
                } else if (h_sc[16 * c + 4] != 0.0) {
                    // (p, F p) <= 0 with a residual above the tolerance: F is not positive on the search direction
                    // (inexact local solves that failed, or rounding); report it and stop unconverged
                    h_done[c] = 1;
                    brk_c[c] = 1;
                }
            }
            if (!active_left()) break;
            HIPCHECK(hipMemcpyAsync(done_dev, h_done, nc * sizeof(int), hipMemcpyHostToDevice, stream));
            applyPrec(lr, lz);
            pcg_stage(2, lam, lr, lz, lp, lq);
        }
    }
    sync();
    auto t2 = clk::now();
    // ---- recovery u = K~^{-1} (f - B^T lambda), averaged copies, global residual
    scatter(lam, false, b64);
    hipLaunchKernelGGL(k_sub, dim3(tile_grid(D0.nt_all)), dim3(TILE), 0, stream, D0.L, D0.tiles_all, D0.nt_all, f64,
                       b64, w64);
    check_launch();
    ktilde_inv(w64, true, pl.opt.inner_tol, u64);
    finish_solution(st, u_out);
    sync();
    auto t3 = clk::now();
    if (prof.on) prof.collect();
    st.time_rhs_ms = ms(t0, t1);
    st.time_pcg_ms = ms(t1, t2);
    st.time_recovery_ms = ms(t2, t3);
    st.time_total_ms = ms(t0, t3);
    {
        int h8[8];
        HIPCHECK(hipMemcpyAsync(h8, nactive, sizeof(h8), hipMemcpyDeviceToHost, stream));
        sync();
        inner_sum = h8[1];
        inner_max = h8[2];
        inner_calls = h8[3];
        st.inner_unconverged = h8[4];
        st.inner_nonfinite = h8[5];
    }
    st.inner_iterations_max = inner_max;
    st.inner_iterations_mean = inner_calls ? (double)inner_sum / (double)inner_calls : 0.0;
    // per-problem statistics (the batch's inner-iteration figures are shared)
    comp_stats.assign(nc, st);
    comp_rc.assign(nc, IETI_OK);
    for (int c = 0; c < nc; ++c) {
        ieti_stats& cs = comp_stats[c];
        cs.outer_iterations = its_c[c];
        cs.residual_initial = r0[c];
        cs.residual_final = rnorm[c];
        cs.breakdown = brk_c[c];
        cs.global_residual = comp_gres[c];
        cs.n_lambda = h_comp_lam[c + 1] - h_comp_lam[c];
        cs.ndof_torn = pl.comp_torn_beg[c + 1] - pl.comp_torn_beg[c];
        if (st.inner_nonfinite > 0 || !conv[c]) comp_rc[c] = IETI_ENOCONV;
    }
    st = comp_stats[0];
    if (nc > 1) {   // the whole batch: totals and the worst problem
        st.outer_iterations = it;
        st.n_lambda = nl;
        st.ndof_torn = pl.ndof_torn;
        st.breakdown = 0;
        for (int c = 0; c < nc; ++c) {
            st.residual_final = std::max(st.residual_final, comp_stats[c].residual_final);
            st.global_residual = std::max(st.global_residual, comp_stats[c].global_residual);
            st.breakdown |= comp_stats[c].breakdown;
        }
    }
    if (stp) *stp = st;
    int rc = IETI_OK;
    for (int c = 0; c < nc; ++c)
        if (comp_rc[c] != IETI_OK) rc = comp_rc[c];
    if (st.inner_nonfinite > 0) {
        set_last_error("a local solve produced a non-finite residual");
        return IETI_ENOCONV;
    }
    if (rc != IETI_OK)
        set_last_error(st.breakdown ? "outer CG breakdown above the tolerance" : "outer CG did not converge");
    return rc;
}

// Bramble-Pasciak CG on [A B^T; B 0] (u; lambda) = (f; 0) (the saddle-point system (2) in W~):
// preconditioner P^{-1}(q_u; q_l) = (A0^{-1} q_u; S^-1 (B A0^{-1} q_u - q_l)), S^-1 the scaled Dirichlet
// preconditioner; CG for P^{-1} [A B^T; B 0] in the inner product H = diag(A - A0, S).  For every vector
// v = P^{-1} q the iteration keeps q beside it, so that H v = (A v_u - q_u; B v_u - q_l) needs no A0.
// Iterates until sqrt(rho_k / rho_0) <= tol, rho = <z, z>_H.  The solution u lands in u64.
template <typename T>
int Solver<T>::solve_saddle(ieti_stats& st) {
    const Plan& pl = *plan;
    const int64_t nl = nlam, n = len0;
    DevLevel& D0 = lev[0];
    double w = bp_omega;
    auto sub = [&](double* a, const double* b) {   // a -= b on the coefficients
        hipLaunchKernelGGL(k_sub, dim3(tile_grid(D0.nt_all)), dim3(TILE), 0, stream, D0.L, D0.tiles_all, D0.nt_all,
                           a, b, a);
        check_launch();
    };
    // The recurrences' energy rho reaches a rounding floor (its H-product mixes A and A0 terms), and with
    // FP32 V-cycles the preconditioner is linear only to FP32 rounding, which a (non-flexible) CG cannot
    // absorb: each cycle reduces its own sqrt(rho) by restart_red (or stops when rho grows by 1e6 over
    // its minimum), then the iteration restarts from the true FP64 residual r (mixed-precision
    // refinement).  Convergence is decided there on eta = (z_u, r_u) + (z_l, S^ z_l), z = P^{-1} r, which
    // is positive for any omega.  A non-positive H-energy (rho at a restart, or a breakdown in a cycle's
    // first step) means A - A0 is not positive on W~: omega grows by 1.5 and the iteration starts over.
    const double restart_red = std::is_same<T, float>::value ? 1e-4 : 1e-7;
    fill<double>(bsc, 16, 0.0);
    fill<double>(bsc + 12, 1, 1.0);
    fill<double>(bx, n, 0.0);
    if (nl > 0) fill<double>(lxx, nl, 0.0);
    double hs[10];
    double eta0 = -1.0, eta = 0.0;
    int it = 0, raises = 0;
    bool conv = false, fresh = true;
    while (!conv && it < pl.opt.max_it) {
        // true residual r = (f - A x_u - B^T x_l, -B x_u)
        hipLaunchKernelGGL((k_convert<double, double>), dim3(tile_grid(D0.nt_all)), dim3(TILE), 0, stream, D0.L,
                           D0.tiles_all, D0.nt_all, f64, br, (int)MODE_K, 1.0);   // Dirichlet rows out
        check_launch();
        if (!fresh) {
            applyA(bx, bs);
            sub(br, bs);
            if (nl > 0) {
                scatter(lxx, false, bg2);
                sub(br, bg2);
                gather(bx, false, lrr);
                hipLaunchKernelGGL(k_scale_flat, dim3(nblk(nl, 256)), dim3(256), 0, stream, nl, lrr, lrr, -1.0);
                check_launch();
            }
        } else if (nl > 0) {
            fill<double>(lrr, nl, 0.0);
        }
        // z = P^{-1} r, Hz = (A z_u - r_u, B z_u - r_l)
        A0inv(br, bz, w);
        if (nl > 0) {
            gather(bz, false, lhz);
            axpy_dev(nl, lhz, lrr, 12, -1.0);
            applyPrec(lhz, lzz);
        }
        applyA(bz, bhz);
        sub(bhz, br);
        flat_dot(n, bz, bhz, bsc + 0);
        flat_dot(nl, lzz, lhz, bsc + 1);
        flat_dot(n, bz, br, bsc + 9);
        hipLaunchKernelGGL(k_bp_scalars, dim3(1), dim3(1), 0, stream, 0, bsc);
        check_launch();
        copy_dev(n, bp, bz);
        copy_dev(nl, lpp, lzz);
        HIPCHECK(hipMemcpyAsync(hs, bsc, 10 * sizeof(double), hipMemcpyDeviceToHost, stream));
        sync();
        const double rho_c = hs[5];   // H-energy at the start of this cycle
        eta = hs[9] + hs[1];
        if (eta0 < 0.0) {
            eta0 = eta;
            st.residual_initial = eta0 > 0.0 ? std::sqrt(eta0) : 0.0;
            if (!(eta0 > 0.0)) {   // f vanishes on W~: u = 0
                st.breakdown = 1;
                conv = true;
                break;
            }
        }
        if (std::sqrt(std::max(eta, 0.0) / eta0) <= pl.opt.tol) {
            conv = true;
            break;
        }
        auto raise_omega = [&]() {
            if (++raises > 8) throw Error(IETI_ENOCONV, "saddle-point iteration: no positive omega scaling found");
            w *= 1.5;
            bp_omega = w;
            fill<double>(bx, n, 0.0);
            if (nl > 0) fill<double>(lxx, nl, 0.0);
            eta0 = -1.0;
            fresh = true;
        };
        if (!(rho_c > 0.0)) {
            raise_omega();
            continue;
        }
        fresh = false;
        const double cycle_goal = std::max(pl.opt.tol * std::sqrt(eta0 / eta), restart_red);
        double rho_min = rho_c;
        bool restart_over = false;
        for (int cit = 0; it < pl.opt.max_it; ++cit) {
            // s = A~ p, t = P^{-1} s, Ht
            applyA(bp, bs);
            if (nl > 0) {
                scatter(lpp, false, bg2);
                hipLaunchKernelGGL(k_add<double>, dim3(tile_grid(D0.nt_all)), dim3(TILE), 0, stream, D0.L,
                                   D0.tiles_all, D0.nt_all, (const double*)bg2, bs);
                check_launch();
                gather(bp, false, lss);
            }
            A0inv(bs, bt, w);
            if (nl > 0) {
                gather(bt, false, lht);
                axpy_dev(nl, lht, lss, 12, -1.0);   // Ht_l = B t_u - s_l
                applyPrec(lht, ltt);
            }
            applyA(bt, bht);
            sub(bht, bs);
            flat_dot(n, bp, bht, bsc + 2);
            flat_dot(nl, lpp, lht, bsc + 3);
            hipLaunchKernelGGL(k_bp_scalars, dim3(1), dim3(1), 0, stream, 1, bsc);
            check_launch();
            axpy_dev(n, bx, bp, 6, 1.0);
            axpy_dev(n, bz, bt, 6, -1.0);
            axpy_dev(n, bhz, bht, 6, -1.0);
            if (nl > 0) {
                axpy_dev(nl, lxx, lpp, 6, 1.0);
                axpy_dev(nl, lzz, ltt, 6, -1.0);
                axpy_dev(nl, lhz, lht, 6, -1.0);
            }
            flat_dot(n, bz, bhz, bsc + 0);
            flat_dot(nl, lzz, lhz, bsc + 1);
            hipLaunchKernelGGL(k_bp_scalars, dim3(1), dim3(1), 0, stream, 2, bsc);
            check_launch();
            HIPCHECK(hipMemcpyAsync(hs, bsc, 10 * sizeof(double), hipMemcpyDeviceToHost, stream));
            sync();
            ++it;
            const double rho = hs[4];
            if (hs[8] != 0.0) {   // (p, H P^{-1} A~ p) <= 0 or rho <= 0: indefinite H, or rounding in a late step
                if (cit == 0) restart_over = true;
                break;
            }
            const double red = std::sqrt(std::max(rho, 0.0) / rho_c);
            rho_min = std::min(rho_min, rho);
            if (red <= cycle_goal || rho > 1e6 * rho_min) break;   // restart from the true residual
            xpby_dev(n, bp, bz, 7);
            xpby_dev(nl, lpp, lzz, 7);
        }
        if (restart_over) raise_omega();
    }
    copy_dev(n, u64, bx);
    st.outer_iterations = it;
    st.residual_final = std::sqrt(std::max(eta, 0.0));
    st.saddle_omega = bp_omega;
    return conv ? IETI_OK : IETI_ENOCONV;
}

// u64 (torn, level-0 layout) -> averaged interface copies, FP64 assembled residual, caller's torn output
template <typename T>
void Solver<T>::finish_solution(ieti_stats& st, double* u_out) {
    DevLevel& D0 = lev[0];
    if (ngroups > 0) {
        hipLaunchKernelGGL(k_group_mean, dim3(nblk(ngroups, 256)), dim3(256), 0, stream, ngroups, grp_ptr, grp_dev,
                           u64);
        check_launch();
    }
    stencil<double, double, double, EPI_RESID>(0, false, MODE_K, coef64, u64, s64, f64, nullptr, nullptr, 0.0, 0);
    // |r| and |f| of the assembled (conforming) vectors
    HIPCHECK(hipMemcpyAsync(e64, f64, sizeof(double) * len0, hipMemcpyDeviceToDevice, stream));
    std::vector<double> acc(2, 0.0);
    for (int which = 0; which < 2; ++which) {
        double* v = which == 0 ? s64 : e64;
        if (ngroups > 0) {
            hipLaunchKernelGGL(k_group_assemble, dim3(nblk(ngroups, 256)), dim3(256), 0, stream, ngroups, grp_ptr,
                               grp_dev, v);
            check_launch();
        }
        hipLaunchKernelGGL(k_sq, dim3(tile_grid(D0.nt_all)), dim3(TILE), 0, stream, D0.L, D0.tiles_all, D0.nt_all, v,
                           (int)MODE_K, partial);
        check_launch();
        if (ncomp == 1) {
            hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, stream, partial, (int64_t)D0.nt_all, sc + 12 + which);
        } else {   // per problem of a batch
            hipLaunchKernelGGL(k_sum_comp, dim3(ncomp), dim3(256), 0, stream, partial, tile_beg, tile_end, comp_patch,
                               sc + 12 + which);
        }
        check_launch();
    }
    HIPCHECK(hipMemcpyAsync(h_sc, sc, 16 * (size_t)ncomp * sizeof(double), hipMemcpyDeviceToHost, stream));
    sync();
    comp_gres.assign(ncomp, 0.0);
    for (int c = 0; c < ncomp; ++c) {
        acc[0] = h_sc[16 * c + 12];
        acc[1] = h_sc[16 * c + 13];
        comp_gres[c] = acc[1] > 0 ? std::sqrt(std::max(acc[0], 0.0) / acc[1]) : 0.0;
    }
    st.global_residual = comp_gres[0];
    hipLaunchKernelGGL(k_copy_out, dim3(tile_grid(D0.nt_all)), dim3(TILE), 0, stream, D0.L, D0.tiles_all, D0.nt_all,
                       torn_off, u64, u_out);
    check_launch();
    sync();
}

}  // namespace ieti

// ------------------------------------------------------------------ C ABI

using namespace ieti;

struct ieti_handle {
    std::unique_ptr<SolverBase> s;
};

template <typename F>
static int guarded(F&& f) {
    try {
        return f();
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

extern "C" {

}  // extern "C"

// Scratch of ieti_solve_noalloc: one copy per GPU, held until the process ends.  In host code `scratch`
// names a host-side stand-in, never the device memory: kernels and fills get the address that
// hipGetSymbolAddress returns for the current device (scratch_address).
static __device__ __align__(256) double scratch[IETI_NOALLOC_SCRATCH_BYTES / sizeof(double)];
static std::mutex g_scratch_mu;
static std::map<int, double*> g_scratch_addr;

// The device address of `scratch` on device `dev`, which must be current; resolved once per device.
static double* scratch_address(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it != g_scratch_addr.end()) return it->second;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
        throw Error(IETI_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_addr[dev] = (double*)p;
    return (double*)p;
}

// A handle around a plan: device state built on the plan's stream (or a new one).
static ieti_handle* make_handle(std::unique_ptr<Plan> plan) {
    if (plan->opt.device >= 0) HIPCHECK(hipSetDevice(plan->opt.device));
    std::unique_ptr<SolverBase> s;
    if (plan->opt.mg_precision == 32 && plan->opt.local_solver != IETI_LOCAL_EXACT) s.reset(new Solver<float>());
    else s.reset(new Solver<double>());
    s->plan = std::move(plan);
    if (s->plan->opt.stream) {
        s->stream = (hipStream_t)s->plan->opt.stream;
    } else {
        HIPCHECK(hipStreamCreate(&s->stream));
        s->own_stream = true;
    }
    s->setup();
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev));
    s->noalloc_base = scratch_address(dev);
    auto* h = new ieti_handle();
    h->s = std::move(s);
    return h;
}

// Device bytes a handle built from this plan will hold (upper estimate used for
// admission; mirrors the allocations of Solver::setup with a margin).
static size_t estimate_device_bytes(const Plan& pl) {
    const bool exact = pl.opt.local_solver == IETI_LOCAL_EXACT;
    const double T = (pl.opt.mg_precision == 32 && !exact) ? 4.0 : 8.0;
    double b = 0.0;
    int npk = 0;
    for (const Patch& pa : pl.patches) {
        npk = std::max(npk, (int)pa.primal_global.size());
        for (size_t l = 0; l < pa.lv.size(); ++l) {
            const Level& L = pa.lv[l];
            const double len = (double)(L.n + 2 * L.guard + 64);
            b += L.nst * len * T + 5.0 * len * T;                      // operator data, MG vectors
            if (l == 0) b += (T == 4.0 ? L.nst * len * 8.0 : 0.0) + 10.0 * len * 8.0 + 6.0 * len * T;
            if (!L.inv[0].empty()) b += 2.0 * L.n * L.n * T;
        }
        b += 2.0 * npk * (double)(pa.lv[0].n + 2 * pa.lv[0].guard + 64) * 8.0;   // Psi + setup scratch
        b += (double)(pa.band[0].size() + pa.band[1].size()) * 8.0;
        if (pl.dim == 3 && (pl.opt.local_solver == IETI_LOCAL_EXACT || pl.opt.local_solver == IETI_LOCAL_EXACT_MG)) {
            // device block band of the Neumann (and, for D-D, the Dirichlet) problem with the diagonal inverses
            const double nb = (double)((pa.lv[0].n + BNB - 1) / BNB);
            const double W = (double)((pa.lv[0].guard + BNB - 1) / BNB);
            const double modes = pl.opt.local_solver == IETI_LOCAL_EXACT ? 2.0 : 1.0;
            b += modes * nb * (W + 2.0) * BNB * BNB * 8.0;
        }
        b += (double)pa.n_qp * (16.0 + 8.0 * pa.dim);
        for (int m = 0; m < 2; ++m)   // tensor smoother: U_d, lambda_d, scratch (two buffers in 3D)
            if (!pa.ts[m].U[0].empty())
                b += 8.0 * (double)(pa.ts[m].U[0].size() + pa.ts[m].U[1].size() + pa.ts[m].U[2].size() +
                                    2.0 * pa.ts[m].Pd[0] * pa.ts[m].Pd[1] * std::max(1, pa.ts[m].Pd[2]));
    }
    const double npad = (double)((pl.n_primal + 15) / 16 * 16);
    b += (double)pl.n_lambda * 8.0 * 8.0 + (double)pl.n_primal * pl.n_primal * 8.0 + 3.0 * npad * npad * 8.0;
    return (size_t)(1.15 * b) + (16u << 20);
}

extern "C" {

int ieti_setup(const ieti_patch* patches, int32_t n_patches, const double* primal_vertices, int32_t n_primal_vertices,
               const ieti_options* opt, ieti_handle** out) {
    if (!out) return IETI_EINVAL;
    *out = nullptr;
    return guarded([&] {
        std::unique_ptr<Plan> plan(build_plan(patches, n_patches, primal_vertices, n_primal_vertices, opt));
        *out = make_handle(std::move(plan));
        return IETI_OK;
    });
}

int ieti_quadrature(const ieti_handle* h, double* x, int32_t on_device, int64_t* n_qp) {
    if (!h) return IETI_EINVAL;
    return guarded([&] {
        if (n_qp) *n_qp = h->s->plan->n_qp;
        if (x) h->s->quadrature(x, on_device != 0);
        return IETI_OK;
    });
}

int ieti_solve(ieti_handle* h, const double* f_qp, double* u, ieti_stats* stats) {
    if (!h || !f_qp || !u) return IETI_EINVAL;
    return guarded([&] { return h->s->solve(f_qp, u, stats); });
}

int ieti_solve_noalloc(ieti_handle* h, const double* f_qp, double* u, ieti_stats* stats) {
    if (!h || !f_qp || !u) return IETI_EINVAL;
    return guarded([&] { return h->s->solve_noalloc(f_qp, u, stats); });
}

int ieti_profile_enable(ieti_handle* h, int32_t enable) {
    if (!h) return IETI_EINVAL;
    return guarded([&] {
        HIPCHECK(hipStreamSynchronize(h->s->stream));
        h->s->prof.collect();
        h->s->prof.reset();
        h->s->prof.on = enable != 0;
        return IETI_OK;
    });
}

int ieti_profile_query(const ieti_handle* h, int32_t kernel, int64_t* launches, double* total_ms,
                       double* total_bytes) {
    if (!h || kernel < 0 || kernel >= IETI_KPROF_COUNT) return IETI_EINVAL;
    const KProf& p = h->s->prof;
    if (launches) *launches = p.launches[kernel];
    if (total_ms) *total_ms = p.ms[kernel];
    if (total_bytes) *total_bytes = p.bytes[kernel];
    return IETI_OK;
}

int ieti_sizes(const ieti_handle* h, int64_t* n_qp, int64_t* ndof_torn, int64_t* device_bytes) {
    if (!h) return IETI_EINVAL;
    if (n_qp) *n_qp = h->s->plan->n_qp;
    if (ndof_torn) *ndof_torn = h->s->plan->ndof_torn;
    if (device_bytes) *device_bytes = (int64_t)h->s->arena.bytes;
    return IETI_OK;
}

void ieti_destroy(ieti_handle* h) {
    if (!h) return;
    try {
        if (h->s) {
            (void)hipStreamSynchronize(h->s->stream);
            hipStream_t st = h->s->stream;
            bool own = h->s->own_stream;
            h->s.reset();
            if (own) (void)hipStreamDestroy(st);
        }
    } catch (...) {
    }
    delete h;
}

const char* ieti_strerror(int code) {
    switch (code) {
    case IETI_OK: return "ok";
    case IETI_EINVAL: return "invalid argument";
    case IETI_ENONCONFORMING: return "non-conforming interface";
    case IETI_EGEOM: return "invalid geometry";
    case IETI_ENOMEM: return "out of memory";
    case IETI_ENOCONV: return "no convergence";
    case IETI_EDEVICE: return "device error";
    case IETI_ENOTSUP: return "not supported";
    case IETI_PENDING: return "pending";
    default: return "unknown error";
    }
}

const char* ieti_last_error(void) { return ieti::last_error(); }

}  // extern "C"

// ------------------------------------------------------------------ serving

// One request: deep copies of its patches and f, the caller's output buffer.
struct SrvReq {
    int64_t ticket = 0;
    std::vector<std::vector<double>> knots, ctrl;
    std::vector<ieti_patch> patches;
    std::vector<double> f;
    double* u_out = nullptr;
    int dim = 2;
    int64_t ndof = 0;          // torn dofs
    int status = IETI_PENDING;
    ieti_stats st{};
    double t_submit = 0, t_admit = 0, t_done = 0;
};

struct ieti_server {
    DevicePool pool;          // device memory of the requests (declared first: released after the workers end)
    ieti_options opt{};
    std::string tune_cache;   // owned copy of opt.tune_cache
    int slots = 1;
    size_t budget = 0;      // 0: unlimited
    size_t in_use = 0;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_mem, cv_done;
    std::deque<SrvReq*> queue;
    std::map<int64_t, std::unique_ptr<SrvReq>> reqs;
    int64_t next = 1;
    bool stop = false;
    int running = 0;
    std::vector<std::thread> workers;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

// A worker owns one stream.  It takes a batch of waiting requests (the oldest one and, behind it, requests
// of the same dimension while the torn dofs stay within batch_dofs), plans them as one multi-problem solve,
// waits until the HBM budget admits the batch's estimated device footprint, builds the device state, solves
// (one outer CG per request, all launches over all their patches), copies every u to its caller and frees
// everything.  Batches of different workers overlap on the GPU.  If a batch of several requests cannot be
// planned (one invalid request), its requests are retried one by one so that only the invalid one fails.
static void server_solve(ieti_server* S, hipStream_t st, std::vector<SrvReq*>& batch) {
    size_t bytes = 0;
    bool admitted = false;
    double* fd = nullptr;
    double* ud = nullptr;
    ieti_handle* h = nullptr;
    std::vector<int> rcs(batch.size(), IETI_OK);
    std::vector<ieti_stats> sts(batch.size());
    try {
        ieti_options o = S->opt;
        o.stream = st;
        o.hbm_budget = 0;
        o.device = S->device;
        std::vector<ieti_patch> all;
        std::vector<int32_t> comp;
        for (size_t b = 0; b < batch.size(); ++b)
            for (const ieti_patch& p : batch[b]->patches) {
                all.push_back(p);
                comp.push_back((int32_t)b);
            }
        std::unique_ptr<Plan> plan(build_plan(all.data(), (int)all.size(), nullptr, 0, &o, comp.data()));
        if (plan->ncomp != (int)batch.size()) throw Error(IETI_EINVAL, "internal: batch problem count");
        for (size_t b = 0; b < batch.size(); ++b)
            if ((int64_t)batch[b]->f.size() != plan->comp_qp_beg[b + 1] - plan->comp_qp_beg[b])
                throw Error(IETI_EINVAL, "f has the wrong number of values");
        bytes = estimate_device_bytes(*plan) + (size_t)(plan->n_qp + plan->ndof_torn) * sizeof(double);
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->budget && bytes > S->budget) throw Error(IETI_ENOMEM, "request larger than the HBM budget");
            S->cv_mem.wait(lk, [&] { return !S->budget || S->in_use + bytes <= S->budget; });
            S->in_use += bytes;
            admitted = true;
            const double ta = S->now_ms();   // one admission for the whole batch
            for (SrvReq* r : batch) r->t_admit = ta;
        }
        const int64_t nq = plan->n_qp, nt = plan->ndof_torn;
        std::vector<int64_t> tb = plan->comp_torn_beg;
        h = make_handle(std::move(plan));
        fd = (double*)S->pool.get(sizeof(double) * nq);
        ud = (double*)S->pool.get(sizeof(double) * nt);
        if (!fd || !ud) throw Error(IETI_ENOMEM, "hipMalloc failed");
        int64_t qo = 0;
        for (SrvReq* r : batch) {
            HIPCHECK(hipMemcpyAsync(fd + qo, r->f.data(), sizeof(double) * r->f.size(), hipMemcpyHostToDevice, st));
            qo += (int64_t)r->f.size();
        }
        ieti_stats all_st{};
        const int rc_all = h->s->solve(fd, ud, &all_st);
        for (size_t b = 0; b < batch.size(); ++b) {
            HIPCHECK(hipMemcpyAsync(batch[b]->u_out, ud + tb[b], sizeof(double) * (size_t)(tb[b + 1] - tb[b]),
                                    hipMemcpyDeviceToHost, st));
            sts[b] = b < h->s->comp_stats.size() ? h->s->comp_stats[b] : all_st;
            rcs[b] = b < h->s->comp_rc.size() ? h->s->comp_rc[b] : rc_all;
            if (all_st.inner_nonfinite > 0) rcs[b] = IETI_ENOCONV;
        }
        HIPCHECK(hipStreamSynchronize(st));
    } catch (const Error& e) {
        for (auto& rc : rcs) rc = e.code;
        set_last_error(e.what());
    } catch (const std::exception& e) {
        for (auto& rc : rcs) rc = IETI_EINVAL;
        set_last_error(e.what());
    }
    (void)hipStreamSynchronize(st);   // nothing of this batch in flight before its memory goes back to the pool
    if (h) ieti_destroy(h);
    if (fd) S->pool.put(fd);
    if (ud) S->pool.put(ud);
    if (!admitted && batch.size() > 1 && rcs[0] != IETI_OK) {
        // the batch failed before it ran: retry its requests one by one
        for (SrvReq* r : batch) {
            std::vector<SrvReq*> one{r};
            server_solve(S, st, one);
        }
        return;
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (admitted) S->in_use -= bytes;
        const double t = S->now_ms();
        for (size_t b = 0; b < batch.size(); ++b) {
            batch[b]->st = sts[b];
            batch[b]->t_done = t;
            batch[b]->status = rcs[b];
            --S->running;
        }
    }
    S->cv_mem.notify_all();
    S->cv_done.notify_all();
}

static void server_worker(ieti_server* S) {
    (void)hipSetDevice(S->device);
    t_pool = &S->pool;
    hipStream_t st = nullptr;
    if (hipStreamCreate(&st) != hipSuccess) return;
    for (;;) {
        std::vector<SrvReq*> batch;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
            if (S->queue.empty()) break;
            int64_t dofs = 0;
            for (auto it = S->queue.begin(); it != S->queue.end();) {
                SrvReq* r = *it;
                if (!batch.empty() && (r->dim != batch[0]->dim || dofs + r->ndof > S->opt.batch_dofs)) {
                    if (dofs + r->ndof > S->opt.batch_dofs) break;   // keep arrival order within the size cap
                    ++it;
                    continue;
                }
                batch.push_back(r);
                dofs += r->ndof;
                it = S->queue.erase(it);
                if (S->opt.batch_dofs <= 0) break;
            }
            S->running += (int)batch.size();
        }
        server_solve(S, st, batch);
    }
    (void)hipStreamDestroy(st);
}

extern "C" {

int ieti_plan_device_bytes(const ieti_plan* plan, size_t* bytes) {
    if (!plan || !bytes) return IETI_EINVAL;
    const Plan& pl = *reinterpret_cast<const Plan*>(plan);
    *bytes = estimate_device_bytes(pl) + (size_t)(pl.n_qp + pl.ndof_torn) * sizeof(double);
    return IETI_OK;
}

int ieti_server_create(const ieti_options* opt, int32_t max_slots, ieti_server** out) {
    if (!out || max_slots < 1 || max_slots > 16) return IETI_EINVAL;
    *out = nullptr;
    return guarded([&] {
        auto* S = new ieti_server();
        if (opt) S->opt = *opt; else default_options(&S->opt);
        if (S->opt.tune_cache) {   // keep no caller pointer: the workers plan with the server's own copy
            S->tune_cache = S->opt.tune_cache;
            S->opt.tune_cache = S->tune_cache.c_str();
        }
        S->slots = max_slots;
        S->budget = S->opt.hbm_budget;
        S->pool.cap = S->budget;
        int dev = S->opt.device;
        if (dev < 0) HIPCHECK(hipGetDevice(&dev));
        S->device = dev;
        for (int i = 0; i < max_slots; ++i) S->workers.emplace_back(server_worker, S);
        *out = S;
        return IETI_OK;
    });
}

int ieti_server_submit(ieti_server* S, const ieti_patch* patches, int32_t n_patches, const double* f_qp,
                       int64_t n_qp, double* u, int64_t* ticket) {
    if (!S || !patches || n_patches <= 0 || !f_qp || n_qp <= 0 || !u || !ticket) return IETI_EINVAL;
    return guarded([&] {
        auto r = std::make_unique<SrvReq>();
        for (int k = 0; k < n_patches; ++k) {
            ieti_patch p = patches[k];
            if (p.dim != 2 && p.dim != 3) throw Error(IETI_EINVAL, "dim must be 2 or 3");
            int64_t nc = 1;
            for (int d = 0; d < p.dim; ++d) {
                if (!p.knots[d] || p.n_knots[d] <= 2 * p.degree[d] + 1) throw Error(IETI_EINVAL, "bad knot vector");
                r->knots.emplace_back(p.knots[d], p.knots[d] + p.n_knots[d]);
                nc *= p.n_knots[d] - p.degree[d] - 1;
            }
            r->ctrl.emplace_back(p.ctrl, p.ctrl + nc * p.dim);
            r->patches.push_back(p);
            r->dim = p.dim;
            r->ndof += nc;
        }
        size_t kk = 0;
        for (int k = 0; k < n_patches; ++k) {
            ieti_patch& p = r->patches[k];
            for (int d = 0; d < p.dim; ++d) p.knots[d] = r->knots[kk++].data();
            p.ctrl = r->ctrl[k].data();
        }
        r->f.assign(f_qp, f_qp + n_qp);
        r->u_out = u;
        std::lock_guard<std::mutex> lk(S->mu);
        r->ticket = S->next++;
        r->t_submit = S->now_ms();
        *ticket = r->ticket;
        S->queue.push_back(r.get());
        S->reqs[r->ticket] = std::move(r);
        S->cv_work.notify_one();
        return IETI_OK;
    });
}

int ieti_server_poll(ieti_server* S, int64_t ticket, int32_t wait, ieti_stats* st, double* times_ms) {
    if (!S) return IETI_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return IETI_EINVAL;
    SrvReq* r = it->second.get();
    if (wait) S->cv_done.wait(lk, [&] { return r->status != IETI_PENDING; });
    if (r->status == IETI_PENDING) return IETI_PENDING;
    if (st) *st = r->st;
    if (times_ms) {
        times_ms[0] = r->t_submit;
        times_ms[1] = r->t_admit;
        times_ms[2] = r->t_done;
    }
    const int rc = r->status;
    S->reqs.erase(it);
    return rc;
}

int ieti_server_load(ieti_server* S, int32_t* queued, int32_t* running, size_t* bytes_in_use) {
    if (!S) return IETI_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (queued) *queued = (int32_t)S->queue.size();
    if (running) *running = S->running;
    if (bytes_in_use) *bytes_in_use = S->in_use;
    return IETI_OK;
}

void ieti_server_destroy(ieti_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto& t : S->workers) t.join();
    delete S;
}

}  // extern "C"

