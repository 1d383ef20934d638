/*
 * sem.h -- C ABI of the MI355X spectral-element Poisson library.
 *
 * Solves the spectral-element (SE) discretisation of -lap u = f (arXiv:2110.07663,
 * Sec. 2.1, eqs. 1-3: A u = B f with A = Q^T A_L Q, B = Q^T B_L Q) on a structured
 * mesh of hexahedra with isoparametric GLL nodes, preconditioned by a single-pass
 * p-multigrid V-cycle (Sec. 2.2.2, Algorithm 1) whose smoother is Chebyshev
 * acceleration (Sec. 2.2.3, Algorithm 2) of Jacobi or of overlapping Schwarz solved
 * by the fast diagonalisation method (Sec. 2.2.2, eqs. 4-9), inside flexible CG or
 * flexible GMRES (Sec. 2.2).
 *
 * Conventions shared by every call:
 *  - Status: every function returns sem_status (0 = OK, < 0 = error); nothing is
 *    thrown across the ABI.  sem_last_error() returns a thread-local message for the
 *    last non-OK status of the calling thread.
 *  - Memory: the library never allocates device memory.  The caller asks sem_plan
 *    for the workspace size and passes one device buffer of at least that many bytes
 *    to sem_setup; the context keeps pointers into it.  The caller owns the mesh
 *    arrays (host, read during setup only), the workspace and every vector.  The
 *    context object itself is host memory owned by the library, released by
 *    sem_destroy (which does not touch the workspace).
 *  - Streams: `stream` is a hipStream_t passed as void* (0 = the null stream).  All
 *    device work of a call is enqueued on it, in order.  Calls that return host
 *    scalars (setup, solve) synchronise the stream before returning.
 *  - Vectors: device "E-vectors" of one level, layout [E][N][N][N] with
 *    N = p+1, element e = (ez*ney + ey)*nex + ex and node (i,j,k) of an element at
 *    ((k*N + j)*N + i), i fastest.  Values on nodes shared by several elements are
 *    consistent copies; values on Dirichlet nodes are zero on output.  Precision is
 *    double (SEM_F64) or float (SEM_F32) as the call states.
 *  - Numbering: global node (gx, gy, gz) on the (nex*p+1) x (ney*p+1) x (nez*p+1)
 *    node grid with gx = ex*p + i (likewise y, z); gid = (gz*ny + gy)*nx + gx.
 *  - Calls on one context must not overlap (they share its workspace vectors).
 */
#ifndef SEM_H
#define SEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SEM_OK = 0,
  SEM_EINVAL = -1,       /* bad argument (shape, degree, schedule, null pointer)       */
  SEM_EWORKSPACE = -2,   /* workspace smaller than sem_plan's size                      */
  SEM_EHIP = -3,         /* a HIP runtime call failed (message names it)                */
  SEM_ENOCONV = -4,      /* solve stopped at maxit; x and info hold the last iterate     */
  SEM_ENAN = -5,         /* NaN/Inf met in a residual norm or an inner product          */
  SEM_EUNSUPPORTED = -6, /* valid request the library does not implement               */
  SEM_EGEOM = -7         /* non-positive Jacobian determinant (inverted element)        */
} sem_status;

typedef enum { SEM_F64 = 0, SEM_F32 = 1, SEM_BF16 = 2, SEM_F16 = 3 } sem_prec;

typedef enum {              /* surrogate smoother S inside Chebyshev (Sec. 2.2.3)       */
  SEM_SMOOTH_JACOBI = 0,    /* S = diag(A)^{-1}                                          */
  SEM_SMOOTH_RAS = 1,       /* restrictive additive Schwarz, FDM local solves            */
  SEM_SMOOTH_ASM = 2        /* additive Schwarz (eq. 4) with 1/#boxes post-weights       */
} sem_smoother;

typedef enum { SEM_KRYLOV_PCG = 0, SEM_KRYLOV_FCG = 1, SEM_KRYLOV_FGMRES = 2 } sem_krylov;
typedef enum { SEM_PRECOND_PMG = 0, SEM_PRECOND_JACOBI = 1 } sem_precond;

/* Mesh: structured nex x ney x nez hexahedra.  xyz (host, read only during setup)
 * holds the node coordinates of every element at the tensor GLL points of degree
 * p_geom, layout [E][(p_geom+1)^3][3], node (i,j,k) at (k*Ng + j)*Ng + i.  p_geom = 1
 * gives the 8 vertices (trilinear elements).  Coordinates of every multigrid level
 * are the degree-p_geom isoparametric interpolant (Sec. 2.1) at that level's nodes. */
typedef struct {
  int32_t nex, ney, nez;
  int32_t p_geom;
  const double *xyz;
} sem_mesh;

/* Solver options; sem_default_opts fills the paper's defaults:
 * pMG schedule (p, ..., 1) given in p_levels, Chebyshev order 2, bounds
 * (0.1, 1.1) * lambda~ from 10 Arnoldi steps (Sec. 2.2.3), FCG, coarse Jacobi-PCG
 * to 1e-10 relative residual. */
typedef struct {
  int32_t nlevels;            /* entries used in p_levels; p_levels[0] must equal p       */
  int32_t p_levels[8];        /* strictly decreasing degrees, e.g. {7, 3, 1}              */
  int32_t precond;            /* sem_precond                                              */
  int32_t smoother;           /* sem_smoother, used on every level except the coarsest    */
  int32_t cheb_order;         /* K of Algorithm 2 (K products with A per application);    */
                              /* 0: no acceleration (Sec. 2.2.2): the smoother S once,    */
                              /* x += S(b - Ax), in an additive V-cycle x = S b +         */
                              /* P V(P^T b) without post-smoothing                        */
  double lmin_fac, lmax_fac;  /* (lambda_min, lambda_max) = (lmin_fac, lmax_fac)*lambda~  */
  int32_t arnoldi_steps;      /* Arnoldi steps on S*A for lambda~ (<= 16)                 */
  uint64_t seed;              /* Arnoldi start vector: SplitMix64(seed XOR gid) in [-1,1) */
  double lambda_override[8];  /* > 0: use this lambda~ on level l instead of Arnoldi      */
  int32_t smoother_prec;      /* SEM_F64 or SEM_F32: precision of the V-cycle levels      */
  int32_t fdm_prec;           /* FDM contraction inputs: F64/F32 (= smoother_prec), or    */
                              /* SEM_BF16 / SEM_F16 on MFMA with FP32 accumulation        */
  int32_t krylov;             /* sem_krylov                                               */
  int32_t gmres_restart;      /* m of FGMRES(m), <= 64                                    */
  double coarse_tol;          /* relative residual of the coarse Jacobi-PCG; 0 = run      */
  int32_t coarse_maxit;       /*   exactly coarse_maxit iterations                        */
  int32_t ax_variant;         /* Ax kernel shape at p = 7: 0 generic slab kernel, 1 one   */
                              /* wavefront per element, 2 same with non-temporal streams, */
                              /* -1 library default                                       */
  int32_t batch_rhs;          /* right sides this context can take in sem_batch_solve     */
  int32_t coarse_solver;      /* p = 1 coarsest level: 0 Jacobi-PCG (coarse_tol,          */
                              /* coarse_maxit), 1 exact block-tridiagonal elimination     */
                              /* over z-planes (3 nz (nx ny)^2 doubles of workspace, and  */
                              /* as many floats under an FP32 smoother, whose sweeps read */
                              /* FP32 copies; falls back to the PCG if the level is       */
                              /* singular), -1 library default: 1 when the doubles take   */
                              /* <= 4 GiB                                                 */
  int32_t proj_max;           /* > 0: sem_solve starts from the A-conjugate projection of */
                              /* b onto up to proj_max prior solutions (successive right  */
                              /* sides, Sec. 3.2 / 4.2) and stops at ||r|| <= rtol ||b||; */
                              /* 0: off (the default).  At most 32.                       */
  int32_t geom_prec;          /* storage of the geometric factors G (Sec. 2.1) that the   */
                              /* FP32 smoother's A reads on its smoothed levels: SEM_F32  */
                              /* (the default) or SEM_F16 (12 instead of 24 bytes per     */
                              /* point: each element's six factors scaled by one power of */
                              /* two and rounded to FP16, the products still in FP32;     */
                              /* at most 2^-11 relative error per factor).  SEM_F16 needs */
                              /* smoother_prec = SEM_F32; the coarsest level keeps FP32.  */
} sem_opts;

typedef struct {
  int32_t iters;              /* outer Krylov iterations                                  */
  int32_t converged;          /* 1 if the true relative residual met rtol                 */
  double rel_res;             /* final ||r||/||r0|| of the recurrence                     */
  double true_rel_res;        /* ||b - A x||/||r0|| recomputed in FP64 at exit            */
  double r0_norm;             /* ||b - A x0||                                             */
  int32_t coarse_iters;       /* coarse PCG iterations of the last V-cycle                */
  double lambda_tilde[8];     /* lambda~ used on each level (0 on the coarsest)           */
} sem_solve_info;

typedef struct {
  int32_t p, N;               /* degree and points per direction (N = p + 1)              */
  int64_t E;                  /* elements                                                 */
  int64_t nlocal;             /* E * N^3, entries of one E-vector                         */
  int64_t nglobal;            /* unique nodes (nex*p+1)(ney*p+1)(nez*p+1)                 */
  int64_t nshared;            /* gather-scatter segments (shared or Dirichlet nodes)      */
  double lmin, lmax;          /* Chebyshev bounds of this level (0 on the coarsest)       */
  int64_t nmembers;           /* E-vector entries in those segments                       */
} sem_level_desc;

void sem_default_opts(sem_opts *opts);

/* Workspace bytes sem_setup needs for this problem.  bc[6] = Dirichlet (1) or
 * Neumann (0) flag of the faces x-, x+, y-, y+, z-, z+ (Sec. 2.1).  Fails with
 * SEM_EINVAL on an invalid schedule or mesh, SEM_EUNSUPPORTED for p > 15. */
sem_status sem_plan(const sem_mesh *mesh, int32_t p, const int8_t bc[6], const sem_opts *opts,
                    size_t *workspace_bytes);

typedef struct sem_ctx sem_ctx;

/* Builds every level: GLL basis, coordinates, geometric factors G and mass B_L
 * (Sec. 2.1), the sorted gather-scatter numbering, Jacobi diagonals, FDM data
 * (eqs. 5-9), transfer matrices, and the Chebyshev bounds by Arnoldi (Sec. 2.2.3).
 * `workspace` is a device buffer of workspace_bytes >= sem_plan's size, 256-byte
 * aligned.  Synchronises `stream`.  Returns SEM_EGEOM if an element is inverted. */
sem_status sem_setup(const sem_mesh *mesh, int32_t p, const int8_t bc[6], const sem_opts *opts,
                     void *workspace, size_t workspace_bytes, void *stream, sem_ctx **out);

/* Releases the host context (not the caller's workspace).  Accepts NULL. */
sem_status sem_destroy(sem_ctx *ctx);

const char *sem_last_error(void);

/* Shape of level `level` (0 = finest). */
sem_status sem_level_info(const sem_ctx *ctx, int32_t level, sem_level_desc *out);

/* GLL nodes of degree p (Sec. 2.1), computed on the device into nodes_dev[p+1]
 * and weights_dev[p+1] (device doubles; weights_dev may be NULL). */
sem_status sem_gll(int32_t p, double *nodes_dev, double *weights_dev, void *stream);

/* Node coordinates of a level: xyz_dev[3][nlocal] (device doubles). */
sem_status sem_coords(const sem_ctx *ctx, int32_t level, double *xyz_dev, void *stream);

/* Boolean gather u_L = Q u (Sec. 2.1): u_global_dev[nglobal] -> u_local_dev[nlocal]. */
sem_status sem_gather(const sem_ctx *ctx, int32_t level, const double *u_global_dev,
                      double *u_local_dev, void *stream);

/* Right side b = mask * QQ^T (B_L f) on the finest level (eq. 3); f is the source
 * sampled at the fine nodes (E-vector), b an E-vector; both FP64 device. */
sem_status sem_rhs(sem_ctx *ctx, const double *f_dev, double *b_dev, void *stream);

/* Au = mask * QQ^T A_L u on `level` (Sec. 2.1, A = Q^T A_L Q applied by sum
 * factorisation).  prec SEM_F64 (double E-vectors, FP64 G) or SEM_F32 (float
 * E-vectors, FP32 arithmetic; G stored in FP32, or in FP16 on the smoothed
 * levels of a context set up with geom_prec = SEM_F16).  u and Au must not
 * alias. */
sem_status sem_apply_A(sem_ctx *ctx, int32_t level, int32_t prec, const void *u, void *Au,
                       void *stream);

/* z = S r, the level's surrogate smoother (Jacobi diagonal inverse, or the Schwarz
 * sum of eq. 4 with RAS/ASM weights and FDM local solves of eq. 8), masked.
 * prec SEM_F64 or SEM_F32 (E-vectors of that type); for Schwarz, the FDM
 * contraction precision is the context's fdm_prec when prec is SEM_F32. */
sem_status sem_apply_S(sem_ctx *ctx, int32_t level, int32_t prec, const void *r, void *z,
                       void *stream);

/* x <- x + Cheb(b - A x) on `level` (Algorithm 2 with the level's bounds and
 * order; the result of the algorithm is read as a correction added to x). */
sem_status sem_smooth(sem_ctx *ctx, int32_t level, int32_t prec, const void *b, void *x,
                      void *stream);

/* Transfers between level l (fine) and l+1 (coarse) (Algorithm 1):
 * prolong: xf += P xc; restrict: rc = mask_c * P^T rf. */
sem_status sem_prolong(sem_ctx *ctx, int32_t level, int32_t prec, const void *xc, void *xf,
                       void *stream);
sem_status sem_restrict(sem_ctx *ctx, int32_t level, int32_t prec, const void *rf, void *rc,
                        void *stream);

/* z = M r: one V-cycle of Algorithm 1 from x = 0 on the finest level (levels in the
 * context's smoother precision, coarse solve in FP64), FP64 in and out.  With
 * precond = SEM_PRECOND_JACOBI, z = diag(A)^{-1} r. */
sem_status sem_vcycle(sem_ctx *ctx, const double *r, double *z, void *stream);

/* Solves A x = b to ||b - A x|| <= rtol ||b - A x0|| (2-norm over unique free
 * nodes) with the context's Krylov method, x_inout the initial guess and result.
 * Returns SEM_ENOCONV at maxit (x and info hold the last iterate), SEM_ENAN on a
 * NaN/Inf residual.  info may be NULL.
 * With opts.proj_max > 0 (successive right sides, Sec. 3.2 / 4.2): the input x
 * is ignored; the initial guess is x0 = sum_i (x_i, b) x_i over the context's
 * A-orthonormal basis of prior solutions, the test is ||b - A x|| <= rtol ||b||
 * (0 iterations when x0 already passes it; rel_res and true_rel_res are then
 * relative to ||b||), and afterwards the correction x - x0 is A-orthogonalised
 * against the basis (classical Gram-Schmidt, two passes, one extra product with
 * A) and appended; a full basis restarts from the latest solution alone. */
sem_status sem_solve(sem_ctx *ctx, const double *b, double *x_inout, double rtol, int32_t maxit,
                     sem_solve_info *info, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): sem_solve with the same arguments,
 * results and errors, except that the scratch of its reductions (block
 * partials, reduction results, the recurrence's device scalars, last-block
 * counters, and the finest level's element shares of (p, A p)) lives in a
 * 512 KiB array of device memory owned by the library (one per GPU, held
 * until the process ends) instead of the context's workspace.  The call
 * allocates nothing.  Limit: the finest level may have at most 56832
 * elements, else SEM_EINVAL.  Every call on one GPU shares that GPU's array,
 * so calls that overlap on one GPU (other streams or threads) race; calls in
 * turn are safe, the array keeps only scratch between them. */
sem_status sem_solve_static(sem_ctx *ctx, const double *b, double *x_inout, double rtol,
                            int32_t maxit, sem_solve_info *info, void *stream);

/* Empties the basis of prior solutions used by opts.proj_max. */
sem_status sem_projection_reset(sem_ctx *ctx);

/* Kernel timing of the finest level, for roofline reporting.  While enabled, the
 * library records a pair of HIP events on the call's stream around every launch
 * of the instrumented kernels below (finest level only; the last two classes
 * bracket whole phases), so durations are those of the kernels themselves.  The
 * events are recorded without a system-scope fence (timing only).  enable: 0
 * off, 1 every class, otherwise a mask whose bit k + 1 records class k (fewer
 * events, less disturbance of the timed work).  Enabling clears the counters;
 * a negative value is SEM_EINVAL.  sem_profile_read synchronises on the
 * recorded events and returns, per class, the summed duration in ms
 * (total_ms[SEM_PROF_COUNT]) and the launch count. */
typedef enum {
  SEM_PROF_AX64 = 0,   /* sum-factorised A_L, FP64 (outer Krylov operator)          */
  SEM_PROF_AX32 = 1,   /* sum-factorised A_L, FP32 (smoother operator)              */
  SEM_PROF_FDM = 2,    /* Schwarz FDM local solves (any precision)                  */
  SEM_PROF_GS64 = 3,   /* QQ^T gather-scatter + mask, FP64                          */
  SEM_PROF_GS32 = 4,   /* QQ^T gather-scatter + mask, FP32                          */
  SEM_PROF_COARSE = 5, /* whole coarse-grid solve of one V-cycle (all its launches)  */
  SEM_PROF_VCYCLE = 6, /* whole preconditioner application z = M r                   */
  SEM_PROF_COUNT = 7
} sem_prof_kernel;
sem_status sem_profile(sem_ctx *ctx, int32_t enable);
sem_status sem_profile_read(sem_ctx *ctx, double *total_ms, int64_t *launches);

/* Batched solves: nctx independent problems (contexts set up with batch_rhs >=
 * nrhs), nrhs right sides each, advanced together by flexible CG whose scalars
 * stay on the device.  One outer iteration of every unconverged (problem, right
 * side) pair is recorded as one HIP graph (a branch per problem, branches on
 * several streams) and replayed iters_per_launch times between host checks of
 * the convergence flags; the graph is recorded again when pairs finish.  The
 * coarse solve inside a recorded V-cycle runs a fixed iteration count (the count
 * the first, eager V-cycle of that problem needed, plus 4, at most coarse_maxit).
 * When the context's hierarchy ends in the assembled p = 1 level and nrhs > 1,
 * its work vectors hold batch_rhs right sides and the nrhs right sides of a
 * problem share every operator application, V-cycle and coarse sweep (one launch
 * per kernel for all of them; finished right sides are carried along, their CG
 * kernels do nothing); environment SEM_BATCH_JOINT=0 runs them one at a time.
 * Both give bit-identical iterates.
 * b[i*nrhs + k], x[i*nrhs + k]: device FP64 E-vectors of problem i, right side k
 * (x is the initial guess and the result).  infos (may be NULL) has nctx*nrhs
 * entries.  Returns SEM_ENOCONV if some pair misses rtol within maxit. */
sem_status sem_batch_solve(int32_t nctx, sem_ctx *const *ctx, int32_t nrhs, const double *const *b,
                           double *const *x, double rtol, int32_t maxit, int32_t iters_per_launch,
                           sem_solve_info *infos, void *stream);

/* Auto-tuner (Sec. 5: exhaustive search over a small parameter space on the first
 * solve, at the problem the user runs).  Every candidate option set is set up in
 * turn in the same workspace, solved `repeats` times from x = 0 on the caller's
 * right side b (an E-vector of the finest level, which all candidates share: same
 * mesh and p), and timed with HIP events; the fastest candidate that converges to
 * rtol within maxit wins (ties: lower Chebyshev order, then fewer levels).  b and x
 * are caller-owned device FP64 E-vectors; x is overwritten.  Candidates that are
 * rejected or do not converge are reported with their status and skipped. */
#define SEM_TUNE_MAX 96
typedef struct {
  int32_t ncand;
  sem_opts cand[SEM_TUNE_MAX];
  int32_t repeats;            /* timed solves per candidate (the median is kept)         */
  double rtol;
  int32_t maxit;
} sem_tune_request;

typedef struct {
  int32_t best;               /* index into cand[], -1 if none converged                */
  double ms[SEM_TUNE_MAX];    /* median solve time (setup excluded)                     */
  double setup_ms[SEM_TUNE_MAX];
  int32_t iters[SEM_TUNE_MAX];
  int32_t status[SEM_TUNE_MAX];
} sem_tune_result;

/* Fills req with the paper's pMG search space for degree p (Sec. 5 table: Cheby-ASM,
 * Cheby-RAS and Cheby-Jacobi with their schedules), crossed with Chebyshev orders
 * 1..3, smoother precisions (FP64; FP32; FP32 with FP16 MFMA FDM) and, at p = 7,
 * the two Ax kernel shapes.  Fields of `base` not searched are copied. */
sem_status sem_tune_space(int32_t p, const sem_opts *base, sem_tune_request *req);
sem_status sem_tune_plan(const sem_mesh *mesh, int32_t p, const int8_t bc[6],
                         const sem_tune_request *req, size_t *workspace_bytes);
sem_status sem_tune(const sem_mesh *mesh, int32_t p, const int8_t bc[6],
                    const sem_tune_request *req, const double *b, double *x, void *workspace,
                    size_t workspace_bytes, void *stream, sem_tune_result *out);

#ifdef __cplusplus
}
#endif
#endif
