/*
 * lsh.h -- C ABI of the MI355X (gfx950) HBS-preconditioned Lippmann-Schwinger
 * solver.
 *
 * Method: Gopal & Martinsson, "An accelerated, high-order accurate direct
 * solver for the Lippmann-Schwinger equation for acoustic scattering in the
 * plane" (arXiv 2007.12718).
 *
 * Problem (paper Sec. 1, eqs. (ansatz), (kernel), (ls); Sec. 2.2, eqs.
 * (corrected), (linsys), (Gmat)): on an n x n cell-centred grid of mesh h
 * (node (i1, i2) at (x0 + (i1 + 1/2) h, y0 + (i2 + 1/2) h)), find sigma with
 *     sigma_i + kappa^2 b_i sum_j K_ij sigma_j = -kappa^2 b_i u_inc_i,
 *     K_ij = h^2 [ (i/4) H0(kappa |x_i - x_j|) [i != j] + tau_{x_j - x_i} ],
 * tau the order-p corrected-trapezoidal weights (p = 4, 6, 8, 10; Fig. 2
 * stencils), and the scattered field u = K sigma.
 *
 * Pipeline: lsh_plan_create (tree, weights, kernel table, proxy-source row IDs
 * of the b-independent 4th-order G, Sec. 3.2) -> lsh_factor_create (Algorithm
 * 1 for a given b) -> lsh_solve (flexible GMRES on the order-p operator
 * applied by FFT, right-preconditioned with Algorithm 2; Sec. 5).
 *
 * Conventions for every call:
 *  - Field arrays are interleaved complex FP64 ("double2"), C order
 *    [nrhs][n][n] with x1 fastest; b is real FP64 [n][n].
 *  - Array pointers are DEVICE pointers owned by the caller unless the
 *    argument says "host".  The library reads inputs and writes outputs only
 *    on the given stream; it keeps no reference to caller arrays after a call
 *    returns, except for the workspaces of handles (below).
 *  - The library allocates no device memory.  Each plan, factor and solve
 *    works in a device workspace that the caller owns: query its size with
 *    the matching lsh_*_workspace call (host-only), allocate it (e.g. a
 *    torch tensor; 256-byte aligned, any contents), and pass the pointer and
 *    its size.  A plan or factor workspace belongs to its handle until the
 *    handle is destroyed (a handle is invalid once its workspace is freed);
 *    a solve workspace is in use until the call's work on the stream is
 *    done.  A workspace smaller than the query gives
 *    LSH_ERR_WORKSPACE_TOO_SMALL.  Plan sizes are upper bounds (the ranks
 *    are found while the plan is built; lsh_plan_workspace_used reports what
 *    was used); factor and solve sizes are exact for the given plan.
 *  - Handles are small host objects; destroy them with the matching
 *    *_destroy call (host only; the workspace stays the caller's).  A
 *    factor refers to its plan: destroy the factor first.
 *  - The stream is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls that must read back small device values synchronise the stream
 *    and say so.
 *  - Return value: LSH_OK (0), LSH_NOT_CONVERGED (1: outputs hold the best
 *    iterate), or a negative error code; lsh_last_error() gives the message
 *    of the calling thread's last failure.  No C++ exception crosses the
 *    ABI.  Handles are not thread-safe.
 */
#ifndef LSH_H
#define LSH_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LSH_OK = 0,
  LSH_NOT_CONVERGED = 1,
  LSH_ERR_INVALID_ARG = -1,
  LSH_ERR_INPUT_NONFINITE = -2,
  LSH_ERR_SINGULAR = -3,
  LSH_ERR_HIP = -4,
  LSH_ERR_NOMEM = -5,
  LSH_ERR_UNSUPPORTED = -6,
  LSH_ERR_WORKSPACE_TOO_SMALL = -7
};

/* factor flags: LSH_FACTOR_TRANSPOSE reserves room in the factor's workspace
 * for the transposed copies that M^T needs (lsh_apply_precond with
 * transpose = 1, lsh_solve_adjoint); without it those calls fail with
 * LSH_ERR_INVALID_ARG. */
#define LSH_FACTOR_TRANSPOSE 1

enum { LSH_FP64 = 0, LSH_FP32 = 1 };

#define LSH_MAX_LEVELS 32
#define LSH_MAX_ITERS 200

typedef struct lsh_plan_s* lsh_plan_t;
typedef struct lsh_factor_s* lsh_factor_t;

/* Problem and method description. */
typedef struct {
  int n;            /* grid side (n x n nodes); n / leaf must be a power of two */
  double h;         /* mesh width (unit square: 1/n) */
  double x0, y0;    /* lower-left corner of the grid square (unit square: -0.5) */
  double kappa;     /* wavenumber > 0 */
  int op_order;     /* 4, 6, 8 or 10: correction order of the GMRES operator */
  int leaf;         /* leaf box side in nodes (e.g. 8) */
  double tol;       /* compression tolerance eps (>= 0; 0 = exact full-rank HBS) */
  int proxy_width;  /* layers of proxy points around each box (1..3) */
  int hbs_prec;     /* LSH_FP64 or LSH_FP32: precision of factor and apply */
  int merge;        /* LSH_MERGE_*: form of the merge inverses X_tau (below) */
  int hbs_order;    /* correction order of the compressed matrix: 0 or 4 (the 4th-order
                       preconditioner, Sec. 5), or 6, 8, 10 (direct-solver mode, Sec. 6:
                       the HBS of that order's matrix, used with or without GMRES; its
                       correction stencil reaches 1, 2, 3 lattice steps and proxy_width
                       must be at least that) */
  int plan_cache;   /* 1: take each level's row IDs from the process-wide plan cache
                       when present and add the ones computed (lsh_plan_cache_*); 0: off */
  int full_levels;  /* boxes of levels 1 .. full_levels keep all their candidate nodes
                       (U_l = I, no row ID; their merges take the children's skeletons
                       whole): 0 compresses every box below the root (Sec. 3); 1 leaves
                       the root's two children uncompressed, where the row ID keeps most
                       candidates anyway and is the longest step of the plan */
} lsh_desc;

/* Merge inverses X_tau of Algorithm 1 (eq. (localsol)).  SCHUR inverts the
 * c x c Schur complement I - S_b G_ab^T S_a G_ab of every parent.  LOWRANK
 * takes a row ID G_ab ~= L R^T of the level's sibling block at the
 * compression tolerance (once per level, in the plan) and uses the Woodbury
 * form of the remark after Algorithm 2 (eq. (blockinv), with the scattering
 * matrices the printed formula leaves out): X_tau = I - P (I + Q P)^{-1} Q,
 * P = diag(S_a L, S_b R), Q = [[0, R^T], [L^T, 0]], whose inverse is of
 * order r (by the same Schur step).  AUTO (0, the default) uses LOWRANK on
 * the levels where r <= 0.6 c and SCHUR elsewhere (and everywhere at
 * tol = 0). */
enum { LSH_MERGE_AUTO = 0, LSH_MERGE_SCHUR = 1, LSH_MERGE_LOWRANK = 2 };

typedef struct {
  double tol;       /* stop when ||f - A x|| / ||f|| < tol (true residual re-checked) */
  int maxit;        /* at most LSH_MAX_ITERS */
  int precondition; /* 1: HBS preconditioner (default); 0: none */
} lsh_solve_opts;

typedef struct {
  int iterations;                       /* FGMRES iterations of the last rhs */
  double residual;                      /* Givens estimate at exit (last rhs) */
  double true_residual;                 /* max over rhs of ||f - A sigma|| / ||f|| */
  double history[LSH_MAX_ITERS + 1];    /* residual estimates of the last rhs */
  double ms_precond, ms_operator, ms_ortho;  /* time on the stream (hipEvents) in the
                                               preconditioner applies, the FFT operator
                                               applies and the Gram-Schmidt passes of the
                                               call (all right-hand sides) */
} lsh_info;

/* ---- plan: paper Sec. 3 (tree, proxy-source IDs; independent of b) ----
 * Builds the tree (Sec. 3.1-3.2), the correction weights (Sec. 2.2), the
 * kernel offset table, one row ID per level (eqs. (leafid), (proxy),
 * (parentid); translation invariance), the sibling blocks (eq. (sibint)) and
 * the spectrum of the order-p operator for the FFT matvec.
 * Synchronises the stream (ranks are read back level by level).
 * Row-ID method (for tol >= 1e-7; below, column-pivoted QR): environment
 * LSH_ROWID=block (default) pivots several rows per step, accepting a pivot
 * whose Schur diagonal is at least LSH_BP_ALPHA (default 0.65; 1 = greedy)
 * times the largest; LSH_ROWID=panel pivots greedily one row at a time.
 * Errors: LSH_ERR_INVALID_ARG for a bad descriptor or LSH_BP_ALPHA outside
 * (0, 1]; LSH_ERR_UNSUPPORTED for sizes beyond the kernels' limits;
 * LSH_ERR_WORKSPACE_TOO_SMALL.
 * ws: device workspace of at least lsh_plan_workspace bytes (ws_bytes its
 * size), the plan's memory until lsh_plan_destroy. */
int lsh_plan_workspace(const lsh_desc* desc, size_t* bytes /* host */);
int lsh_plan_create(const lsh_desc* desc, void* ws, size_t ws_bytes, void* stream, lsh_plan_t* plan);
int lsh_plan_destroy(lsh_plan_t plan);
/* host: bytes of the plan's workspace used at most so far, and its size */
int lsh_plan_workspace_used(lsh_plan_t plan, size_t* used, size_t* size);
/* host: number of levels L and the ranks k_l (l = 0..L; k_0 = 0) */
int lsh_plan_ranks(lsh_plan_t plan, int* L, int* ranks /* host, L+1 */);
/* host: level-l compression data for inspection.  m = candidate rows,
 * k = rank; copies (if non-NULL) J (host int[k], candidate indices in pivot
 * order), cand (host int[2m], box-local lattice coordinates) and U (device
 * double2[m*k], row-major, FP64).  Synchronises the stream. */
int lsh_plan_level(lsh_plan_t plan, int level, int* m, int* k, int* J, int* cand, void* U, void* stream);
/* host: sibling block G_ab of parent level l (device double2[c*c]) and the
 * leaf block (level = -1, device double2[mL*mL]); c via *rows. */
int lsh_plan_block(lsh_plan_t plan, int level, int* rows, void* out, void* stream);
/* device out[(D+1)^2]: offset table T[dy][dx] = h^2 (i/4) H0(kappa h |d|),
 * T[0][0] = h^2 tau_0 (4th order); D via *D. */
int lsh_plan_table(lsh_plan_t plan, int* D, void* out, void* stream);
/* host: low-rank form G_ab ~= L R^T of parent level l's sibling block:
 * *c its order, *r the rank (0: this level's merges use the Schur form);
 * copies (if non-NULL and r > 0) L (device double2[c*r], row-major, FP64;
 * L[J, :] = I) and R^T = G_ab[J, :] (device double2[r*c]).  Synchronises
 * the stream. */
int lsh_plan_lowrank(lsh_plan_t plan, int level, int* c, int* r, void* L, void* Rt, void* stream);

/* ---- plan cache: universal compression (Sec. 3.2 remark: the compression
 * of G depends only on box size and kappa h, so it can be stored and reused)
 * Plans created with desc.plan_cache = 1 look up every row ID (of a level's
 * proxy matrix and of a sibling block) by box size, kappa h, tol,
 * proxy_width, hbs_order and pivoting rule (LSH_ROWID, LSH_BP_ALPHA), and
 * store the ones they compute; a hit copies the pivots and U instead of
 * computing them, so later plans on other b, or on other grids with the same
 * kappa h, skip the row IDs.  Entries live in host memory (the only memory
 * the library owns) and are keyed by device.  Not safe against a concurrent
 * lsh_plan_cache_clear or _load. */
int lsh_plan_cache_info(int* entries, size_t* host_bytes);
int lsh_plan_cache_clear(void);
/* host: writes every entry to a file (binary: pivots, candidates, U) /
 * reads a file written by lsh_plan_cache_save into the cache of the current
 * device (replacing equal keys).  Errors: LSH_ERR_INVALID_ARG for a file
 * that cannot be opened or is not such a file. */
int lsh_plan_cache_save(const char* path);
int lsh_plan_cache_load(const char* path);

/* ---- factor: Algorithm 1 (leaf inverses, scattering matrices, merges) ----
 * b: device double[n*n].  flags: 0 or LSH_FACTOR_TRANSPOSE.  ws: device
 * workspace of at least lsh_factor_workspace(plan, flags) bytes, the
 * factor's memory until lsh_factor_destroy (it holds the factor, a copy of
 * b and the apply vectors).  Errors: LSH_ERR_INPUT_NONFINITE (non-finite b),
 * LSH_ERR_SINGULAR (zero pivot in a local inverse),
 * LSH_ERR_WORKSPACE_TOO_SMALL. */
int lsh_factor_workspace(lsh_plan_t plan, int flags, size_t* bytes /* host */);
int lsh_factor_create(lsh_plan_t plan, const double* b, int flags, void* ws, size_t ws_bytes, void* stream,
                      lsh_factor_t* factor);
int lsh_factor_workspace_used(lsh_factor_t factor, size_t* used, size_t* size);

/* Plan and factor in one call, pipelined by level: the factor of level l
 * (Algorithm 1) starts as soon as the row ID and sibling block of level l
 * exist (Sec. 3.2 builds them leaves-up, like Algorithm 1), so the
 * latency-bound pivot loops of the compression overlap the factor's matrix
 * products.  Same results as lsh_plan_create + lsh_factor_create; destroy
 * the factor, then the plan.  Synchronises the stream before returning.
 * The plan runs on library streams (the level row IDs, the sibling blocks,
 * and the parent-level Gram rows built during each row ID); the factor runs
 * on a library stream kept off LSH_PLAN_CUS compute units (default: an
 * eighth of them for FP32 factors, none for FP64; 0 = the caller's stream,
 * unmasked), so that the plan's latency-bound kernels find free units while
 * the factor's products fill the rest.  Up to five streams are busy at once:
 * give the process at least that many hardware queues (GPU_MAX_HW_QUEUES,
 * read when the HIP runtime starts), or two of them share a queue and
 * serialise.  The factor starts before the ranks are known, so both
 * workspaces are sized by the plan's rank bounds (lsh_build_workspace:
 * plan_bytes as lsh_plan_workspace, factor_bytes at least what
 * lsh_factor_workspace would give once the plan exists).
 * Errors: as lsh_plan_create and lsh_factor_create. */
int lsh_build_workspace(const lsh_desc* desc, int flags, size_t* plan_bytes, size_t* factor_bytes);
int lsh_build(const lsh_desc* desc, const double* b, int flags, void* plan_ws, size_t plan_ws_bytes,
              void* factor_ws, size_t factor_ws_bytes, void* stream, lsh_plan_t* plan, lsh_factor_t* factor);
int lsh_factor_destroy(lsh_factor_t factor);

/* Algorithm 1 for ninst independent problems at once (many uneven instances:
 * different grids, wavenumbers and ranks).  plans: host array of ninst plans;
 * b: host array of ninst device pointers (double[n_i*n_i]); factors: host
 * array receiving ninst handles, each usable like one from
 * lsh_factor_create (destroy each; a factor refers to its plan).  For FP32
 * plans the levels are aligned from the leaves (level L_i - d of every
 * instance at step d) and each product and inverse of a step is one grouped
 * launch over all instances' boxes; the results equal per-instance
 * lsh_factor_create bitwise.  FP64 plans are factored one by one.
 * Workspaces: ws[i] (device, ws_bytes[i] bytes; host arrays of ninst) is
 * instance i's factor workspace, as for lsh_factor_create; shared_ws
 * (shared_bytes) holds the grouped launches' tables, flags and inverse
 * workspace during the call.  lsh_batch_factor_workspace writes the
 * sizes (factor_bytes: host size_t[ninst]).
 * Synchronises the stream.  Errors: as lsh_factor_create (the message names
 * the instance); on error no handle is returned. */
int lsh_batch_factor_workspace(int ninst, const lsh_plan_t* plans, int flags, size_t* factor_bytes,
                               size_t* shared_bytes);
int lsh_batch_factor(int ninst, const lsh_plan_t* plans, const double* const* b, int flags, void* const* ws,
                     const size_t* ws_bytes, void* shared_ws, size_t shared_bytes, void* stream,
                     lsh_factor_t* factors);

/* y = M x: Algorithm 2 (M ~ (I + B G)^{-1}); transpose = 1 applies M^T
 * (needs LSH_FACTOR_TRANSPOSE; the first such call builds the transposed
 * copies in the factor's workspace and synchronises the stream).
 * x, y: device double2[nrhs*n*n]; x and y must not overlap.  Uses the
 * factor's apply vectors: calls on one factor must not overlap. */
int lsh_apply_precond(lsh_factor_t factor, int transpose, const void* x, void* y, int nrhs, void* stream);

/* y = A x = x + kappa^2 b (K * x), K of order op_order, by FFT (Sec. 5);
 * b == NULL gives y = K * x (the scattered field of density x). */
int lsh_apply_operator(lsh_plan_t plan, const double* b, const void* x, void* y, int nrhs, void* stream);

/* sigma (and u = K sigma if u != NULL) for each incident field:
 * right-preconditioned flexible GMRES (x0 = 0, CGS2, no restart).
 * nrhs >= 2: groups of up to 8 right-hand sides run in lockstep (one
 * preconditioner and one operator application per iteration for the whole
 * group; each right-hand side keeps its own Krylov basis and stopping
 * test, so it takes the iterations of its own one-column solve).
 * ws: device workspace of lsh_solve_workspace(factor, nrhs, opts->maxit)
 * bytes (the Krylov bases: about (2 maxit + 3) min(nrhs, 8) n^2 complex FP64
 * values).  Synchronises once per iteration (residual read-back).
 * Returns LSH_NOT_CONVERGED if some rhs did not reach opts->tol; sigma
 * then holds the last iterate and info->true_residual its residual. */
int lsh_solve_workspace(lsh_factor_t factor, int nrhs, int maxit, size_t* bytes /* host */);
int lsh_solve(lsh_factor_t factor, const void* u_inc, int nrhs, void* sigma, void* u, const lsh_solve_opts* opts,
              lsh_info* info, void* ws, size_t ws_bytes, void* stream);

/* lambda = A^{-H} g (the adjoint solve of a misfit gradient; not in the
 * paper, derived from eq. (linsys)).  Since K is complex symmetric,
 * A^H lambda = g  <=>  A^T conj(lambda) = conj(g) with A^T = I + K B; this is
 * solved by the same flexible GMRES on the transposed FFT operator,
 * right-preconditioned by M^T (Algorithm 2 transposed; the factor needs
 * LSH_FACTOR_TRANSPOSE).  ws as for lsh_solve (same size).  Synchronises
 * once per iteration. */
int lsh_solve_adjoint(lsh_factor_t factor, const void* g, int nrhs, void* lambda, const lsh_solve_opts* opts,
                      lsh_info* info, void* ws, size_t ws_bytes, void* stream);

/* u(x_r) = h^2 sum_j (i/4) H0(kappa |x_r - x_j|) sigma_j at off-grid points
 * (eq. (ansatz), trapezoidal sum).  xy: device double[2*npts];
 * u_pts: device double2[nrhs*npts]. */
int lsh_eval_points(lsh_plan_t plan, const void* sigma, const double* xy, int npts, void* u_pts, int nrhs,
                    void* stream);

/* out[m][j] = h^2 sum_r conj((i/4) H0(kappa |x_r - x_j|)) g[m][r]: the
 * adjoint of lsh_eval_points.  g: device double2[nrhs*npts]; out: device
 * double2[nrhs*n*n]. */
int lsh_eval_points_adjoint(lsh_plan_t plan, const void* g_pts, const double* xy, int npts, void* out, int nrhs,
                            void* stream);

/* grad[k] = -kappa^2 Re sum_m conj(lambda[m][k]) (u_inc[m][k] + u[m][k]):
 * the derivative of a real misfit L with respect to b (differentiating
 * eq. (linsys): d sigma = -kappa^2 A^{-1} (db * u_tot)), given
 * lambda = A^{-H} g with g the conjugate-Wirtinger gradient 2 dL/d conj(sigma),
 * the incident fields u_inc and the scattered fields u = K sigma (device
 * double2[nrhs*n*n]); grad: device double[n*n]. */
int lsh_grad_b(lsh_plan_t plan, const void* lambda, const void* u_inc, const void* u, int nrhs, double* grad,
               void* stream);

/* host: dimensionless corrections tau_d of the given order at kappa*h (the
 * matrix entry is h^2 (G + tau_d)); writes count entries (<= 25) of
 * offsets (host int[2*count]) and tau (host double[2*count], re/im). */
int lsh_correction_weights(int order, double kh, int* count, int* offsets, double* tau);

/* ---- tracing: per-kernel hipEvent timing (off by default) ----
 * lsh_profile_enable(1) clears the records and starts recording a start/stop
 * event pair around each instrumented launch (on the launch's stream),
 * tagged with the launch's algorithmic work (flops for cgemm_* / inverse_*,
 * bytes for the bandwidth-bound kernels).  lsh_profile_query synchronises
 * the device and returns, for one kernel name, the number of launches, the
 * summed event time (ms) and the summed work.  lsh_profile_names writes the
 * recorded names, ';'-separated, into buf (host char[cap]). */
int lsh_profile_enable(int on);
/* Restrict recording to names that start with prefix (NULL or "" = all). */
int lsh_profile_only(const char* prefix);
int lsh_profile_query(const char* name, int* launches, double* ms, double* work);
/* summed algorithmic bytes of one kernel name's records (for the GEMMs,
 * whose work is flops: each distinct operand once, the result once) */
int lsh_profile_bytes(const char* name, double* bytes);
int lsh_profile_names(char* buf, int cap);

const char* lsh_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LSH_H */
