/*
 * ieti.h -- C ABI of the MI355X (gfx950) inexact IETI-DP Poisson solver.
 *
 * Problem (Sec. 1, eq. (1)): find u in H^1_0(Omega) with
 *     int grad u . grad v dx = int f v dx   for all v in H^1_0(Omega),
 * Omega a multipatch domain whose patches are tensor-product B-spline images
 * of (0,1)^d, d in {2,3} (Sec. 2).  The solver tears the patches apart,
 * keeps the primal unknowns (patch vertices, optionally 3D edge averages)
 * continuous through an energy-minimising primal subspace (Sec. 2, eq. (6))
 * and solves the dual problem F lambda = d (eq. (4)) by CG with the scaled
 * Dirichlet preconditioner.  Local solves are exact (banded Cholesky) or
 * inexact multigrid-preconditioned (Sec. 3.2, eq. (7); the MG-MG variant of
 * Sec. 3.3).
 *
 * Conventions
 *  - Every call returns 0 on success or a negative IETI_E* code; no call
 *    throws or exits.  ieti_strerror() names a code; ieti_last_error()
 *    returns a thread-local message for the last failure.
 *  - The caller owns every buffer it passes.  Setup copies what it needs;
 *    no caller pointer is kept after a call returns.
 *  - A handle owns all of its device memory and is not thread-safe: calls on
 *    one handle must not overlap.  Different handles are independent.
 *  - Coefficient ("torn") layout: patches in input order; inside patch k the
 *    prod_i M_i coefficients, M_i = n_knots[i] - degree[i] - 1, direction 0
 *    fastest.  Every copy of an interface coefficient holds the same value
 *    in a returned solution; boundary coefficients are 0.
 *  - Quadrature: (p_i+1) Gauss-Legendre points per element and direction.
 *    Point order: patch by patch; inside a patch a tensor grid, direction 0
 *    fastest; along direction i the points of element 0, then element 1, ...
 */
#ifndef IETI_H
#define IETI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define IETI_OK               0
#define IETI_EINVAL          -1  /* invalid argument (sizes, knots, degree, NaN/Inf in f, ...) */
#define IETI_ENONCONFORMING  -2  /* patches meet along a side with different spline spaces or orientation */
#define IETI_EGEOM           -3  /* geometry map not orientation preserving (det J <= 0 at a quadrature point) */
#define IETI_ENOMEM          -4  /* host or device allocation failed, or HBM budget exceeded */
#define IETI_ENOCONV         -5  /* outer CG did not reach tol in max_it iterations (u is still written) */
#define IETI_EDEVICE         -6  /* HIP runtime error */
#define IETI_ENOTSUP         -7  /* configuration outside what this build supports */
#define IETI_PENDING          1  /* serving: request not finished yet */

/* ---- options ---- */
#define IETI_LOCAL_MG     0   /* inexact local solves: flexible CG + multigrid V-cycle (MG-MG) */
#define IETI_LOCAL_EXACT  1   /* exact local solves: banded Cholesky (D-D) */
#define IETI_LOCAL_EXACT_MG 2 /* exact Neumann solves in F, d and the recovery; multigrid V-cycles for the
                                 Dirichlet problems of the preconditioner (D-MG, Sec. 3.3) */
#define IETI_LOCAL_MG_SADDLE 3 /* MG-MG-S (Sec. 3.3): Bramble-Pasciak CG on the saddle-point system (2) with
                                  three V-cycles (plus the exact primal coarse solve) as the preconditioner of
                                  K~ and the scaled Dirichlet preconditioner for the Schur complement; no
                                  inner solves. outer_iterations counts its iterations, the residuals are its
                                  preconditioned energy norms */

#define IETI_PRIMAL_VERTICES  1   /* primal unknowns at patch vertices (eliminated from the local problems) */
#define IETI_PRIMAL_EDGES     2   /* edge averages (3D: patch edges; 2D: patch sides); alone (without
                                     IETI_PRIMAL_VERTICES) the paper's 3D primal set of Sec. 4: vertex copies are
                                     then joined by multipliers, and a patch with no Dirichlet coefficient is
                                     "floating" -- K is singular there and only its edge averages fix the
                                     constants (Sec. 3.2, eq. (6) with a semi-definite block).  Floating patches
                                     are supported by IETI_LOCAL_MG: the local solves run on K + gamma C^T C
                                     (equal to K on {C w = 0}, gamma = 1e-2 / number of edge constraints) with
                                     multigrid levels >= 1 on K + 1e-2 M^ (M^ the mass matrix of the parameter
                                     domain); other local solvers return IETI_ENOTSUP for them */

/* Finest-level multigrid smoother (options.smoother).  TENSOR is the p-robust smoother of Sec. 4 (a
 * subspace-corrected mass smoother variant with a rank-one approximation of the geometry): per patch,
 * x += tau m (K_sep + c M_sep)^{-1} m r, where K_sep is the stiffness with each metric diagonal
 * |det J| (J^{-1} J^{-T})_dd replaced by its best rank-one (separable) approximation on the quadrature grid
 * (2D: A_0 (x) B_1 + B_0 (x) A_1; 3D: A_0 (x) B_1 (x) B_2 + B_0 (x) A_1 (x) B_2 + B_0 (x) B_1 (x) A_2, the
 * mass weight of a direction the geometric mean of its fitted factors), M_sep = B_0 (x) B_1 (x) B_2 the
 * matching weighted mass, c = sigma * mean_d(n_el,d^2), m the mask of the mode,
 * tau = 1 / lambda_max(m (K_sep + c M_sep)^{-1} m K).  The inverse is applied by fast diagonalisation
 * (generalised eigenvectors of (A_d, B_d) per direction), one pre- and one post-smoothing step per
 * V-cycle; 3D patches at most 128 coefficients per direction (IETI_ENOTSUP beyond), 2D no limit. */
#define IETI_SMOOTHER_CHEBYSHEV 0
#define IETI_SMOOTHER_TENSOR    1

typedef struct ieti_patch {
    int32_t dim;               /* 2 or 3 */
    int32_t degree[3];         /* spline degree per direction, 1..6 */
    int32_t n_knots[3];        /* length of each knot vector */
    const double* knots[3];    /* open knot vectors on [0,1]: p+1-fold end knots, simple interior knots (host) */
    const double* ctrl;        /* prod_i M_i control points x dim doubles, direction 0 fastest (host) */
} ieti_patch;

typedef struct ieti_options {
    int32_t local_solver;      /* IETI_LOCAL_MG (default), IETI_LOCAL_EXACT, IETI_LOCAL_EXACT_MG or
                                  IETI_LOCAL_MG_SADDLE */
    int32_t mg_precision;      /* 32 or 64: arithmetic of V-cycles and their operator data (default 64) */
    int32_t primal;            /* IETI_PRIMAL_VERTICES (default), IETI_PRIMAL_VERTICES|IETI_PRIMAL_EDGES or
                                  IETI_PRIMAL_EDGES */
    int32_t cheb_degree;       /* Chebyshev smoother degree per smoothing phase; 0 = tuned per dimension and spline degree */
    int32_t cheb_degree_coarse;/* the same on the coarser multigrid levels; 0 = the table: 2, or 1 under the tensor smoother */
    double  cheb_lower;        /* lower end of the smoothing interval as a fraction of lambda_max; 0 = tuned */
    int32_t prec_vcycles;      /* V-cycles for the Dirichlet problems in the preconditioner (default 2) */
    int32_t max_it;            /* outer CG iteration limit (default 300) */
    int32_t inner_max_it;      /* inner flexible-CG iteration limit (default 400) */
    double  tol;               /* outer: ||r_k||_2 <= tol ||r_0||_2 (default 1e-8) */
    double  inner_tol;         /* local Neumann solves in F, d and recovery (default 1e-10) */
    double  basis_tol;         /* local solves building the primal basis (default 1e-12) */
    int32_t check_every;       /* inner iterations between host convergence checks (default 4) */
    int32_t use_graph;         /* 1: the local solves' flexible-CG iterations replay captured HIP graphs (per
                                  tolerance: check_every iterations between two host convergence checks, one
                                  iteration for the rest); results bitwise equal to 0: the same launches one
                                  by one (the default) */
    int32_t device;            /* HIP device ordinal, -1 = current (default) */
    void*   stream;            /* hipStream_t for all work, NULL = the library's own stream */
    size_t  hbm_budget;        /* bytes of device memory the handle may use, 0 = unlimited */
    int32_t coarse_level;      /* first multigrid level run by the per-patch fused coarse kernel: 0 = chosen
                                  from the LDS size (default), -1 = none (every level by batched launches) */
    int32_t autotune;          /* 1: at setup, time one batched local solve per candidate (finest and coarse
                                  Chebyshev degrees, interval lower end, and the finest-level tile variant: x
                                  window staged in LDS or read directly) around the tuned table and keep the
                                  fastest; 0: the table (default) */
    int32_t coarse_dofs;       /* multigrid: a patch level with at most this many coefficients is not
                                  coarsened further (dense exact solve there); 0 = no such limit. Coarsening
                                  also stops where a direction's element count is odd or below 6 (default 512) */
    int32_t smoother;          /* finest-level smoother: IETI_SMOOTHER_CHEBYSHEV (default) or
                                  IETI_SMOOTHER_TENSOR (coarser levels keep Chebyshev) */
    double  smoother_sigma;    /* IETI_SMOOTHER_TENSOR: mass shift sigma of the tensor smoother, in units of the
                                  mean squared inverse element size of the patch (default 0.3) */
    const char* tune_cache;    /* autotune = 1: path of a JSON-lines file of earlier choices (one object per line:
                                  key, cheb_degree, cheb_degree_coarse, cheb_lower, stage), keyed by dimension,
                                  MG precision, local solver, coarse_dofs and the set of patch shapes (degree /
                                  elements per direction); a hit skips the timing, a miss appends the new choice.
                                  Read at setup only; NULL = no cache (default) */
    int64_t batch_dofs;        /* serving: a worker takes the oldest waiting request and, behind it, further
                                  waiting requests of the same dimension while their torn dofs together stay
                                  within batch_dofs, and solves them as one batch: one plan and one device state,
                                  every kernel launch over the patches of all of them, one outer CG per request
                                  (its own scalars, stopping test and statistics).  0 = one request per batch.
                                  Default 2,000,000 */
    int32_t coarse_degree;     /* multigrid: 0 = every level keeps the patch's spline degree (nested levels,
                                  canonical embedding; default); 1 = degree 1 on all levels but the finest
                                  (Sec. 4, the paper's choice for higher degrees): the finest-to-first-coarse
                                  transfers are the L2 projection of the parameter domain, M_f^{-1} M_fc, and its
                                  transpose (non-nested spaces); coarser transfers stay nested */
} ieti_options;

typedef struct ieti_stats {
    int32_t outer_iterations;
    int32_t inner_iterations_max;      /* max over patches and calls */
    double  inner_iterations_mean;     /* mean inner iterations per local solve (over patches and calls) */
    double  residual_initial;          /* ||d||_2 */
    double  residual_final;            /* ||r_k||_2 of the dual problem */
    double  global_residual;           /* ||f - K u|| / ||f|| on the conforming system, FP64 */
    double  time_rhs_ms;               /* load vector + d */
    double  time_pcg_ms;               /* outer CG loop */
    double  time_recovery_ms;          /* recovery of u + residual */
    double  time_total_ms;             /* whole ieti_solve */
    int64_t ndof_torn;                 /* sum of patch coefficient counts */
    int64_t ndof_global;               /* conforming dofs without the boundary */
    int64_t n_lambda;
    int64_t n_primal;
    int32_t breakdown;                 /* 1 if d vanished to rounding and lambda = 0 was returned (IETI_OK), or
                                          if the outer CG met (p, F p) <= 0 above the tolerance (IETI_ENOCONV) */
    int32_t cheb_degree;               /* smoother in use: Chebyshev degree on the finest level, */
    int32_t cheb_degree_coarse;        /* on the coarser levels, */
    double  cheb_lower;                /* and the interval's lower end over the tuned table's (1 = table) */
    double  saddle_omega;              /* MG-MG-S: the scaling omega of the V-cycle block in use (0 otherwise) */
    int32_t fine_tile_staged;          /* finest-level sweep tiles stage their x window in LDS (1) or not (0) */
    int32_t tune_cached;               /* 1 if the autotuner's choice came from options.tune_cache */
    int32_t inner_unconverged;         /* local flexible-CG solves that stopped above inner_tol (iteration
                                          limit or a vanished search direction); their result is still used */
    int32_t inner_nonfinite;           /* local solves with a NaN/Inf residual; the solve then returns
                                          IETI_ENOCONV */
} ieti_stats;

typedef struct ieti_handle ieti_handle;
typedef struct ieti_plan ieti_plan;

/* Fills *opt with the defaults listed above. */
void ieti_default_options(ieti_options* opt);

/*
 * Host-side planning only (no device call): validates the patches, finds the
 * interfaces (sides whose corner control points coincide; same orientation
 * required), numbers boundary, primal and dual coefficients, builds the jump
 * operators and the multigrid hierarchy and assembles all operator data in
 * FP64.  primal_vertices: n_primal_vertices points (dim doubles each, host)
 * selecting which interior patch vertices are primal; NULL = all of them
 * (none without IETI_PRIMAL_VERTICES).  A patch with no Dirichlet
 * coefficient must keep a primal vertex or an edge-average constraint.
 */
int ieti_plan_create(const ieti_patch* patches, int32_t n_patches,
                     const double* primal_vertices, int32_t n_primal_vertices,
                     const ieti_options* opt, ieti_plan** out);
void ieti_plan_destroy(ieti_plan* plan);

/* Sizes of a plan (host).  Any pointer may be NULL. */
int ieti_plan_sizes(const ieti_plan* plan, int64_t* ndof_torn, int64_t* ndof_global, int64_t* n_lambda,
                    int64_t* n_primal, int64_t* n_qp, int32_t* max_levels);

/*
 * Copies one internal host array of a plan into out (host) for inspection by
 * tests; *count receives the number of elements written (or needed when out
 * is NULL).  which: see IETI_ARR_* below; patch and level select the block.
 */
#define IETI_ARR_STENCIL      1  /* double: half stencil of K, nst x ndof (offset-major), level `level` */
#define IETI_ARR_STENCIL_OFFS 2  /* int32: the nst offsets (o0,o1,o2) of patch/level, 3 per entry */
#define IETI_ARR_PROLONG      3  /* double: dense M_fine x M_coarse 1D prolongation of direction `level>>8`, fine level `level&255` */
#define IETI_ARR_SHAPE        4  /* int32: M0, M1, M2 of patch/level */
#define IETI_ARR_MASKS        5  /* int32: [boundary side bits, primal corner bits, n_levels] of a patch */
#define IETI_ARR_LAMBDA_MAP   6  /* int64: per multiplier (pos_plus, pos_minus) in the torn layout */
#define IETI_ARR_QP_WEIGHT    7  /* double: w_q |det J_q| of patch at level 0 */
#define IETI_ARR_LMAX         8  /* double: [lambda_max Neumann, lambda_max Dirichlet] of D^{-1}K, patch/level */
#define IETI_ARR_PRIMAL_MAP   9  /* int64: per local primal constraint of `patch`: global primal index */
#define IETI_ARR_BAND        10  /* double: exact solves only: blocked band Cholesky data of `patch`, level = 0 (Neumann)
                                    or 1 (Dirichlet); per 64-row block [L_off 64 x b | U_off 64 x b | inv(L_diag) 64 x 64],
                                    b = p0 + p1 M0 (+ p2 M0 M1) */
#define IETI_ARR_TENSOR_U     11  /* double: tensor smoother only: generalised eigenvectors U_d of (A_d, B_d) of `patch`,
                                    level = 256 mode + d (mode 0 Neumann, 1 Dirichlet); P_d x P_d row-major, P_d = M_d
                                    rounded up to 16; row i = coefficient i (zero where the mode removes it), column a =
                                    eigenvector a (U_d^T B_d U_d = I on the kept coefficients; zero padding) */
#define IETI_ARR_TENSOR_LAMBDA 12 /* double: the P_d generalised eigenvalues of the same block (1e300 in the padding) */
#define IETI_ARR_TENSOR_PARAMS 13 /* double: [P_0, P_1, shift c, tau, P_2 (0 in 2D)] of `patch`, level = mode */
int ieti_plan_array(const ieti_plan* plan, int32_t which, int32_t patch, int32_t level, void* out,
                    int64_t* count);

/* Physical coordinates of all quadrature points (n_qp x dim doubles, host). */
int ieti_plan_quadrature(const ieti_plan* plan, double* x_qp_host);

/*
 * Setup (Sec. 1, eq. (1) and Sec. 2): the multipatch B-spline discretisation
 * of the model problem from the patches' degrees, knot vectors and control
 * points, the tearing into patch-local spaces with the primal unknowns at the
 * selected vertices (and edge averages), and the energy-minimising primal
 * basis of eq. (6).  Plans on the host (as ieti_plan_create) and builds the
 * device state: operator data in FP64 and the multigrid precision, the primal
 * basis by batched local solves to basis_tol, the coarse matrix S_PiPi and
 * its factorisation.
 *   patches: n_patches host descriptors (read during the call only);
 *   primal_vertices / n_primal_vertices: as for ieti_plan_create;
 *   opt: host options (NULL = defaults; copied, tune_cache string included);
 *   out: receives the handle (NULL on failure).
 * Errors: IETI_EINVAL (sizes, knots, degrees), IETI_ENONCONFORMING,
 * IETI_EGEOM, IETI_ENOMEM (allocation or hbm_budget), IETI_ENOTSUP, IETI_EDEVICE.
 */
int ieti_setup(const ieti_patch* patches, int32_t n_patches,
               const double* primal_vertices, int32_t n_primal_vertices,
               const ieti_options* opt, ieti_handle** out);

/* Physical quadrature points, n_qp x dim doubles; x_qp is a device pointer if on_device != 0. */
int ieti_quadrature(const ieti_handle* h, double* x_qp, int32_t on_device, int64_t* n_qp);

/*
 * Solve for one right-hand side: the dual problem F lambda = d of eq. (4) by
 * CG with the scaled Dirichlet preconditioner, with the local solves of the
 * variant chosen in the options (Sec. 3.3: exact, MG-MG, D-MG, MG-MG-S), then
 * the recovery of u from lambda (Sec. 2).  f_qp: f at the ieti_quadrature
 * points (n_qp doubles, device pointer, read only).  u: ndof_torn doubles
 * (device pointer, written), the torn layout described above.  stats may be
 * NULL (host).  Runs on the handle's stream and synchronises it before
 * returning.  Errors: IETI_EINVAL (NULL pointers, non-finite f),
 * IETI_ENOCONV (tol not reached in max_it iterations, an outer breakdown
 * above tol, or a non-finite local residual; u is still written),
 * IETI_EDEVICE.
 */
int ieti_solve(ieti_handle* h, const double* f_qp, double* u, ieti_stats* stats);

/*
 * For callers that cannot allocate (serving loops and harnesses that forbid
 * device allocation while they run): ieti_solve with the same arguments,
 * kernels and result (bitwise), but the per-solve scratch of its kernels --
 * the reductions' partial sums, the outer CG's scalars, the local solves'
 * per-patch scalars and counters -- lives in one static device array of
 * IETI_NOALLOC_SCRATCH_BYTES per GPU (held until the process ends) instead
 * of the handle's memory.  Allocates nothing (no device or pinned memory, no
 * graph instantiation, no kernel events: the handle's use_graph and
 * profiling are ignored for this call).  The array is cleared by a fill
 * kernel at the start of every call.  All handles on one GPU share that
 * GPU's array, so calls on the same GPU must not overlap (two threads or
 * streams calling it at once race on the array).  Errors as ieti_solve, and
 * IETI_ENOTSUP if the handle needs more scratch than the maximum (about
 * 32 bytes per stiffness tile of 256 coefficients plus 48 bytes per patch;
 * roughly 30M coefficients).
 */
#define IETI_NOALLOC_SCRATCH_BYTES (4u << 20)
int ieti_solve_noalloc(ieti_handle* h, const double* f_qp, double* u, ieti_stats* stats);

/* Number of quadrature points and torn dofs of a handle. */
int ieti_sizes(const ieti_handle* h, int64_t* n_qp, int64_t* ndof_torn, int64_t* device_bytes);

void ieti_destroy(ieti_handle* h);

/*
 * Kernel timing for roofline reports.  With profiling enabled, every launch
 * of the kernel classes below is bracketed by HIP events on the handle's
 * stream, and its algorithmic bytes (each array the kernel must stream
 * counted once: vectors and the half-stencil operator data) are added up.
 * Enabling resets the counters.  Query returns launches, summed kernel time
 * (ms) and summed algorithmic bytes of a class since the last reset.
 */
#define IETI_KPROF_SMOOTH_FINE  0   /* Chebyshev sweep (stencil + fused update) on the finest level */
#define IETI_KPROF_APPLY64      1   /* FP64 stiffness apply + fused dot products of the flexible CG */
#define IETI_KPROF_RESID_FINE   2   /* residual sweep on the finest level before restriction */
#define IETI_KPROF_FAPPLY       3   /* one whole F apply q = B K~^{-1} B^T p of the outer CG (every kernel of it,
                                       host convergence checks of the local solves included); bytes: the
                                       algorithmic bytes of all its kernels from the per-patch inner iteration
                                       counts (multigrid variants with the Chebyshev smoother, exact local solves) */
#define IETI_KPROF_PREC         4   /* one whole preconditioner apply z = B_D S B_D^T r, same accounting */
#define IETI_KPROF_COARSE       5   /* the fused per-patch coarse part of a V-cycle (levels >= 1), on the launches
                                       that run every patch (the preconditioner's cycles); bytes: each patch's
                                       right-hand side and correction, the half stencils of its smoothed coarse
                                       levels and its coarsest inverse, once */
#define IETI_KPROF_COUNT        6
int ieti_profile_enable(ieti_handle* h, int32_t enable);
int ieti_profile_query(const ieti_handle* h, int32_t kernel, int64_t* launches, double* total_ms,
                       double* total_bytes);

/*
 * Physical quadrature points of a set of patches without planning (host;
 * geometry evaluation only): the points at which a serving request's f must be
 * sampled.  x_host may be NULL to query *n_qp.
 */
int ieti_quadrature_points(const ieti_patch* patches, int32_t n_patches, double* x_host, int64_t* n_qp);

/*
 * Serving: a request loop for many independent solves.  max_slots worker
 * streams (1..16) each take a batch of waiting requests (the oldest one and
 * the ones queued behind it up to opt->batch_dofs torn dofs), plan them as one
 * multi-problem solve, wait until opt->hbm_budget (0 = unlimited) admits the
 * batch's estimated device footprint, set it up, solve -- the requests' outer
 * CG iterations run together, every launch covering all their patches, with
 * per-request scalars and stopping tests -- and copy each u back; batches of
 * different slots overlap on the device and a slot takes the next batch as
 * soon as it finishes.  Submit copies patches
 * and f (host, at ieti_quadrature_points order); u (host, ndof_torn doubles)
 * must stay valid until the request is polled done.  Poll returns
 * IETI_PENDING while running (or blocks with wait != 0), then the solve's
 * status once; times_ms (3 doubles, may be NULL) receives submit, admission
 * and completion times on the server clock.  Requests are independent: a
 * result does not depend on what else is in flight beyond rounding (the
 * primal coarse solve of a batch is one block-diagonal matrix; within the
 * stated tolerance) and the smoother degree, which the batch takes from its
 * highest spline degree unless options.cheb_degree fixes it.
 */
typedef struct ieti_server ieti_server;
/* Device bytes the server reserves for a request with this plan (host). */
int ieti_plan_device_bytes(const ieti_plan* plan, size_t* bytes);
int ieti_server_create(const ieti_options* opt, int32_t max_slots, ieti_server** out);
int ieti_server_submit(ieti_server* s, const ieti_patch* patches, int32_t n_patches, const double* f_qp,
                       int64_t n_qp, double* u, int64_t* ticket);
int ieti_server_poll(ieti_server* s, int64_t ticket, int32_t wait, ieti_stats* stats, double* times_ms);
int ieti_server_load(ieti_server* s, int32_t* queued, int32_t* running, size_t* bytes_in_use);
void ieti_server_destroy(ieti_server* s);

const char* ieti_strerror(int code);
const char* ieti_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IETI_H */
