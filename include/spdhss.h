/*
 * spdhss.h -- C ABI of the MI355X library that builds an SPD HSS
 * preconditioner from an H^2 representation of a dense SPD kernel matrix and
 * solves sigma*I + K(X, X) with preconditioned CG.
 *
 * The method is that of "Efficient construction of an HSS preconditioner for
 * symmetric positive definite H^2 matrices" (Xing, Huang, Chow):
 *   - the problem: SPD kernel systems sigma*I + K(X, X) on 3-D points, solved
 *     by PCG with an SPD HSS preconditioner (Section 6, kernel list and
 *     Section 6.2 diagonal shift);
 *   - H^2 representation and block types: Section 5.1 (eq. uniformbasis_h2),
 *     Section 5.2.2 (Type-1/2/3 blocks);
 *   - the construction: Algorithm 5.3 with Algorithms 5.1 and 5.2;
 *   - the HSS form and its nested factors: Sections 2 and 4 (eqs. nested,
 *     Aii0, Si0, Si, Cij, Mijk, Rik).
 *
 * Conventions shared by every entry point
 *   - Ownership: the caller owns every pointer argument.  The library copies
 *     what it keeps and never retains a caller pointer after returning.
 *     Handles are self-contained (an HSS handle does not borrow the H^2 handle,
 *     a ULV handle does not borrow the HSS handle).
 *   - Memory: unless stated otherwise, array arguments are DEVICE pointers on
 *     the current HIP device.  Vectors are column-major, N x nrhs with leading
 *     dimension ld >= N, rows in the ORIGINAL point order.
 *   - Streams: `stream` is a hipStream_t (NULL = default stream).  Work is
 *     ordered on it; functions that produce host-visible results (handles,
 *     iteration counts) synchronize it before returning.
 *   - Errors: every function returns an spd_status; nothing throws or aborts
 *     across the ABI.  On failure *out is set to NULL and spd_last_error()
 *     returns a thread-local message (for SPD_E_NOT_SPD it names the node and
 *     level whose factorization failed).
 *   - Threads: a handle keeps per-call workspace (product plans, staging
 *     vectors) and the stream of its last call, so one handle serves one call
 *     at a time; calls on distinct handles may run concurrently from
 *     different host threads (the device memory pool is locked).
 *   - Determinism: results are bitwise reproducible for identical inputs on
 *     the same device (no floating-point atomics).
 *   - Precision: all arithmetic is IEEE FP64.  The *_ex entry points can keep
 *     operators in FP32 (rounded once, widened to FP64 on every use).
 */
#ifndef SPDHSS_H
#define SPDHSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPD_PENDING = 1,          /* spd_server_wait without blocking: not finished yet */
  SPD_OK = 0,
  SPD_E_INVALID = -1,       /* bad argument (null pointer, size, option) */
  SPD_E_NOMEM = -2,         /* device allocation failed */
  SPD_E_NOT_SPD = -3,       /* a Cholesky factorization met a non-positive pivot */
  SPD_E_NOT_CONVERGED = -4, /* PCG reached maxit before rtol on some column */
  SPD_E_DEVICE = -5         /* a HIP runtime call failed */
} spd_status;

/* Kernel functions, length-scale form (r = |x - y|):
 *   GAUSSIAN     exp(-r^2 / ell^2)
 *   MATERN32     (1 + sqrt(3) r / ell) exp(-sqrt(3) r / ell)
 *   EXPONENTIAL  exp(-r / ell)
 *   IMQ          1 / sqrt(r^2 + ell^2)
 *   RPY          the Rotne-Prager-Yamakawa 3 x 3 tensor with particle radius
 *                a = ell (Section 6; self term I / a, and for r = x - y,
 *                rr = r r^T / |r|^2: 3/(4|r|)(I + rr) + 3a^2/(2|r|^3)(I/3 - rr)
 *                for |r| >= 2a, (1/a)(1 - 9|r|/(32a)) I + 3|r|/(32a^2) rr
 *                below).  The matrix has 3N rows, row 3p + c being component
 *                c of point p: every vector of the handle (b, x, y) has 3N
 *                rows, and N in the sizes and leading dimensions below means
 *                3N.  The proxy spheres of its ID hold twice proxy_per_shell
 *                points each (capped at proxy_per_shell_max), 3 columns a point.
 * The matrix is shift * I + K(X, X) (Section 6 kernels, Section 6.2 shift). */
typedef enum {
  SPD_K_GAUSSIAN = 0,
  SPD_K_MATERN32 = 1,
  SPD_K_EXPONENTIAL = 2,
  SPD_K_IMQ = 3,
  SPD_K_RPY = 4
} spd_kernel_kind;

typedef struct {
  int32_t kind;   /* spd_kernel_kind */
  double ell;     /* length scale (> 0) */
  double shift;   /* diagonal shift sigma (finite; the paper's are >= 0.  A
                   * negative one can make the leaf blocks indefinite, which
                   * spdhss_build reports as SPD_E_NOT_SPD) */
} spd_kernel;

/* Partition tree of the points (Section 2 assumes a perfect tree). */
typedef enum {
  SPD_TREE_KD = 0,  /* binary kd-tree: depth D is the smallest with
                       N <= leaf_size * 2^D; a node is split on the axis of its
                       largest extent into halves of floor(n/2) and the rest */
  SPD_TREE_BOX = 1  /* the 2^d-ary box-bisection tree of Section 6 (d = 3) as
                       a perfect binary tree with 3 levels per 2^d-ary level: a
                       node at depth t is bisected along axis t mod 3 (x, y, z)
                       at the midpoint of its points' extent, and D is the
                       smallest multiple of 3 with at most leaf_size points in
                       every node at depth D (at most 24).  Leaves are ragged.
                       A node with no extent along its axis cannot be bisected:
                       SPD_E_INVALID */
} spd_tree_kind;

/* H^2 construction options (Section 5.1; construction method: proxy-point
 * interpolative decomposition, this library's choice since the paper does not
 * describe one).
 *
 * Every node with a far field gets proxy_shells Fibonacci spheres centred at
 * its box, from the nearest far box to the farthest root-box corner.  Each
 * sphere has P_v = proxy_density * (rho_in / ell)^2 points (rho_in: radius of
 * the innermost sphere), rounded up to a multiple of 64 and clamped to
 * [proxy_per_shell, proxy_per_shell_max]; proxy_density = 0 keeps
 * P_v = proxy_per_shell.  The densities resolve the kernel's length scale on
 * the spheres of large boxes, without which the ID misses tol by orders of
 * magnitude at the upper levels.  When the M = proxy_shells * P_v proxy rows
 * exceed l = max(2c, c + 16) (c candidates), the proxy matrix is first
 * multiplied by an M x l standard normal sketch (entry (t, j): SplitMix64 on
 * the counter (t << 24) | j under sketch_seed, then Box-Muller), a randomized
 * interpolative decomposition.  c may not exceed 8000 (SPD_E_INVALID). */
typedef struct {
  int32_t leaf_size;            /* max points per leaf, in [1, 512] */
  double eta;                   /* admissibility: r_i + r_j <= eta * |c_i - c_j| */
  double tol;                   /* relative truncation of the ID (|R_tt| > tol |R_00|) */
  int32_t proxy_shells;         /* proxy spheres per node, in [1, 64] */
  int32_t proxy_per_shell;      /* minimum points per sphere (>= 4) */
  int32_t proxy_per_shell_max;  /* maximum points per sphere (>= proxy_per_shell;
                                   proxy_shells * maximum <= 65536) */
  double proxy_density;         /* >= 0, see above */
  uint64_t sketch_seed;         /* seed of the sketch's generator */
  int32_t tree;                 /* spd_tree_kind (0, the kd-tree, when left zero) */
} spd_h2_opts;

/* SPD HSS construction options (Algorithm 5.3, Algorithm 5.1). */
typedef struct {
  double tol;           /* relative CPQR threshold, 0 = fixed rank max_rank */
  int32_t max_rank;     /* rank cap r (>= 0; 0 gives block Jacobi) */
  int32_t oversample;   /* p; Omega has max_rank + oversample columns, at
                           most 256 (above 128 the compression runs in the
                           global-memory pivoted QR) */
  uint64_t seed;        /* seed of the internal Gaussian generator */
  const double* omega;  /* optional DEVICE N x (max_rank+oversample), column-
                           major, ld = N, ORIGINAL point order; NULL = internal
                           generator */
} spd_hss_opts;

typedef struct spd_h2* spd_h2_t;
typedef struct spd_hss* spd_hss_t;
typedef struct spd_ulv* spd_ulv_t;

/* Build the H^2 representation of shift*I + K(X, X).
 * points: DEVICE, n x 3 row-major (x0 y0 z0 x1 ...), original order; n >= 1.
 * Builds the partition tree, the near/coupling lists, the proxy-point ID bases and
 * stores the dense near blocks and the coupling blocks on the device. */
spd_status h2_build(const double* points, int64_t n, spd_kernel kernel,
                    const spd_h2_opts* opts, void* stream, spd_h2_t* out);

/* Algorithm 5.3: build the SPD HSS approximation of the H^2 matrix A.
 * Fails with SPD_E_NOT_SPD when a leaf block or an I + bold B_ii block is not
 * positive definite (which cannot happen when A is SPD, Section 3.2). */
spd_status spdhss_build(spd_h2_t A, const spd_hss_opts* opts, void* stream,
                        spd_hss_t* out);

/* Nested symmetric factorization of the HSS matrix for solves: keeps the leaf
 * Cholesky factors S_i, bases V_i, factors F_i of I + bold B_ii and V-bar_i,
 * and factors the root block I + bold B_root (eqs. Aii0, Si0, Si). */
spd_status ulv_factor(spd_hss_t M, void* stream, spd_ulv_t* out);

/* Precision of the solve operators of a factorization. */
typedef enum {
  SPD_SOLVE_F64 = 0, /* every operator and sum in FP64 */
  SPD_SOLVE_F32 = 1  /* the per-level solve operators stored in FP32 and read
                        as FP32; vectors and sums stay FP64 */
} spd_solve_precision;

/* ulv_factor with a choice of precision for the solve operators (the
 * preconditioner side of PCG, Section 6: the preconditioner only has to be
 * SPD and close to A, so its operators can be rounded to FP32; the H^2
 * operator, the residuals and the dot products of PCG stay FP64, so the
 * attainable residual is unchanged).  SPD_SOLVE_F32 halves the bytes of each
 * apply with at most 16 right-hand sides (more columns use the FP64
 * operators); ulv_apply then differs from the FP64 apply by about the FP32
 * rounding of the operators, and pcg_solve switches to the flexible
 * (Polak-Ribiere) beta, which tolerates that inexactness.
 * precision: spd_solve_precision; other values give SPD_E_INVALID.  The
 * FP32 copies are kept with the nested factors (shared with the HSS handle). */
spd_status ulv_factor_ex(spd_hss_t M, int32_t precision, void* stream, spd_ulv_t* out);

/* x = M^{-1} b for the factored HSS matrix; b, x: DEVICE N x nrhs, ld >= N,
 * original order.  b and x may alias. */
spd_status ulv_apply(spd_ulv_t F, const double* b, double* x, int32_t nrhs,
                     int64_t ld, void* stream);

/* ulv_apply for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and result as ulv_apply (the same recorded sweeps), but
 * every device buffer it needs (tree-order copies of b and x, the stacked
 * rank-space blocks, launch descriptors, partial sums) lives in one static
 * device array of SPD_NOALLOC_SCRATCH_BYTES per GPU, held until the process
 * ends; the call makes no hipMalloc/hipFree.  Vectors need
 * 16 * nrhs * (N + stack rows) bytes of it (spd_noalloc_bytes); larger
 * requests fail with SPD_E_INVALID, and descriptors beyond the rest with
 * SPD_E_NOMEM.  All calls on one GPU share that GPU's array: calls that
 * overlap on one GPU race (serialize them).  Returns after the stream has
 * completed the apply. */
#define SPD_NOALLOC_SCRATCH_BYTES (64ll << 20)
spd_status ulv_apply_noalloc(spd_ulv_t F, const double* b, double* x, int32_t nrhs, int64_t ld,
                             void* stream);
/* Bytes of the array that ulv_apply_noalloc's vectors take for nrhs columns
 * (-1 for a null handle or nrhs < 1). */
int64_t spd_noalloc_bytes(spd_ulv_t F, int32_t nrhs);

/* y = A x with the H^2 representation (upward, coupling, downward and
 * near-field passes); x, y: DEVICE N x nrhs, ld >= N, original order; must not
 * alias. */
spd_status h2_matvec(spd_h2_t A, const double* x, double* y, int32_t nrhs,
                     int64_t ld, void* stream);

/* h2_matvec with a choice of precision for the stored blocks.  SPD_SOLVE_F32
 * (at most 16 columns) streams FP32 copies of the near-field and coupling
 * blocks (made on first use and kept with the handle, about half the bytes of
 * the FP64 blocks the product reads) and accumulates in FP64; the
 * interpolation, vectors and sums stay FP64.  This is a different operator
 * from the FP64 one: each block entry is rounded to FP32 (relative 6e-8).
 * Argument errors as for h2_matvec; an unknown precision, or SPD_SOLVE_F32
 * with more than 16 columns, gives SPD_E_INVALID. */
spd_status h2_matvec_ex(spd_h2_t A, const double* x, double* y, int32_t nrhs,
                        int64_t ld, int32_t precision, void* stream);

/* Solve A x = b column by column with PCG preconditioned by M (M = NULL: plain
 * CG), x0 = 0, stopping column c when ||r_c|| <= rtol * ||b_c||.
 * b, x: DEVICE N x nrhs (ld >= N, original order).
 * iters, relres: HOST arrays of nrhs entries (may be NULL): iterations taken
 * and the true relative residual ||b - A x|| / ||b|| at exit.
 * A column whose recursively updated residual reaches rtol while its true
 * residual is still above rtol (they drift apart on ill-conditioned systems)
 * continues from the true residual, at most 4 times, within maxit (residual
 * replacement; the paper's PCG stops at the recursive residual), so that a
 * converged column meets rtol on its true residual.
 * Returns SPD_E_NOT_CONVERGED if some column did not reach rtol in maxit, or
 * its true residual stayed above rtol. */
spd_status pcg_solve(spd_h2_t A, spd_ulv_t M, const double* b, double* x,
                     int32_t nrhs, int64_t ld, double rtol, int32_t maxit,
                     void* stream, int32_t* iters, double* relres);

/* pcg_solve with a choice of precision for the product inside the iteration
 * (mixed-precision PCG, beyond the paper).  With SPD_SOLVE_F32 (at most 16
 * columns) every iteration applies the FP32-block product of h2_matvec_ex,
 * and the residual is kept honest with the FP64 product: whenever an active
 * column's recursively updated residual has halved since the last
 * replacement (checked every 8 iterations), r = b - A x is recomputed with the
 * FP64 product for every column (reliable updates), without restarting the
 * recurrence.  It pays when the FP32 rounding of the blocks is small against
 * the smallest eigenvalues (roughly cond(A) * 6e-8 << 1); otherwise the
 * iteration count grows.  The
 * stopping test, the reported true residuals and the final restarts use the
 * FP64 product, so the result meets rtol against the FP64 operator.
 * op_precision SPD_SOLVE_F64 is pcg_solve.  Errors as for pcg_solve; an
 * unknown precision, or SPD_SOLVE_F32 with more than 16 columns, gives
 * SPD_E_INVALID. */
spd_status pcg_solve_ex(spd_h2_t A, spd_ulv_t M, const double* b, double* x,
                        int32_t nrhs, int64_t ld, double rtol, int32_t maxit,
                        int32_t op_precision, void* stream, int32_t* iters,
                        double* relres);

/* ---- many independent instances ---------------------------------------
 * One solve request: points, kernel and options as for h2_build and
 * spdhss_build, then pcg_solve of b (nrhs columns) preconditioned by the
 * factored HSS matrix with the given solve precision.  All arrays are DEVICE
 * except iters/relres (HOST, nrhs entries each, may be NULL).  b and x are
 * N x nrhs with ld = N, original point order (3N rows, row 3p + c, for the
 * RPY tensor). */
typedef struct {
  const double* points;     /* DEVICE n x 3 row-major */
  int64_t n;
  spd_kernel kernel;
  spd_h2_opts h2;
  spd_hss_opts hss;         /* hss.omega may be NULL (internal generator) */
  int32_t solve_precision;  /* spd_solve_precision */
  const double* b;
  double* x;
  int32_t nrhs;
  double rtol;
  int32_t maxit;
  int32_t* iters;           /* HOST, may be NULL */
  double* relres;           /* HOST, may be NULL */
} spd_instance;

typedef struct {
  int32_t status;           /* spd_status of this instance */
  int32_t iters_max;        /* largest iteration count over its columns */
  double relres_max;        /* largest true relative residual over its columns */
  double seconds_h2;        /* wall time of h2_build on its worker */
  double seconds_build;     /* spdhss_build + ulv_factor */
  double seconds_solve;     /* pcg_solve */
} spd_instance_result;

/* Run count independent instances end to end (h2_build, spdhss_build,
 * ulv_factor_ex, pcg_solve, destroy) on `workers` host threads, each with its
 * own HIP stream on the calling thread's device, so that the GPU works on
 * several instances at once (the level-by-level rank read-backs of one
 * instance block only its worker).  Workers take the instances largest
 * first (by rows).  Every instance gives the same result as the same calls
 * made alone.  Returns SPD_E_INVALID for bad arguments
 * (count < 0, workers < 1, null pointers); otherwise SPD_OK, with each
 * instance's own status in results[i] (its message is not kept).  The
 * instances' device buffers must not overlap where they are written. */
spd_status spd_solve_batch(const spd_instance* instances, int32_t count, int32_t workers,
                           spd_instance_result* results);

/* ---- serving ------------------------------------------------------------
 * A request loop over a pool of workers (each with its own stream on the
 * creating thread's device).  Requests (spd_instance, as for spd_solve_batch)
 * are admitted first-come-first-served while the sum of the estimated device
 * footprints of the admitted requests stays within hbm_budget_bytes (a
 * request larger than the budget is admitted alone); requests that arrive
 * while others run are admitted as workers and memory free up, and their work
 * overlaps on the device.  A request's H^2, HSS and factor state stays on the
 * device from its build to the end of its solve.  Each result equals the same
 * request run alone.  The caller keeps the request's buffers (points, b, x,
 * omega, iters, relres) valid until spd_server_wait reports it finished. */
typedef struct spd_server* spd_server_t;

/* workers >= 1; hbm_budget_bytes > 0. */
spd_status spd_server_create(int32_t workers, int64_t hbm_budget_bytes, spd_server_t* out);

/* Queue a request; *ticket identifies it for spd_server_wait. */
spd_status spd_server_submit(spd_server_t S, const spd_instance* request, int64_t* ticket);

/* Queue a request whose matrix is named by key (nonzero).  Requests with the
 * same key must have the same points (contents), n, kernel, h2 and hss
 * options and solve precision; their right-hand sides, tolerances and
 * iteration limits may differ.  The first of them builds the H^2, HSS and
 * factor state and leaves it on the device; the later ones run only
 * pcg_solve on it (their results report seconds_h2 = seconds_build = 0) and
 * equal the same request run alone.  Requests with one key run one at a
 * time; one that waits for its state does not hold up the requests behind
 * it.  A resident state counts against hbm_budget_bytes with its footprint
 * estimate less the PCG vectors; idle states are released, least recently
 * used first, when a request cannot be admitted otherwise, and all of them at
 * spd_server_destroy.  A failed build leaves nothing resident.
 * SPD_E_INVALID for a zero key or null arguments. */
spd_status spd_server_submit_keyed(spd_server_t S, const spd_instance* request, uint64_t key,
                                   int64_t* ticket);

/* block != 0: wait until the request has finished.  Returns SPD_PENDING
 * (block == 0, not finished) or SPD_OK with *result filled and, if not NULL,
 * the seconds from submission to admission (*seconds_queued) and to
 * completion (*seconds_total); the ticket is then retired.  Unknown or
 * retired tickets give SPD_E_INVALID, and so does a blocking wait whose
 * ticket another thread collected meanwhile.  Thread-safe. */
spd_status spd_server_wait(spd_server_t S, int64_t ticket, int32_t block,
                           spd_instance_result* result, double* seconds_queued,
                           double* seconds_total);

/* Where a submitted, not yet collected request is: *phase = 0 queued,
 * 1 building its state, 2 solving, 3 finished.  SPD_E_INVALID for unknown or
 * collected tickets.  Thread-safe. */
spd_status spd_server_phase(spd_server_t S, int64_t ticket, int32_t* phase);

/* Estimated device bytes of a request (the admission estimate). */
int64_t spd_request_footprint(const spd_instance* request);

/* Finishes every submitted request, then stops the workers and frees S.  No
 * other call on S may run during it or follow it; results not yet collected
 * with spd_server_wait are discarded. */
void spd_server_destroy(spd_server_t S);

/* Device memory released by destroyed handles is kept in a process-wide cache
 * and reused by later handles (freeing device memory waits for the whole
 * device, which would stall concurrent instances).  This frees the cache;
 * memory held by live handles is not affected. */
void spd_release_cached_memory(void);

void h2_destroy(spd_h2_t A);
void spdhss_destroy(spd_hss_t M);
void ulv_destroy(spd_ulv_t F);

/* Thread-local message of the last failure on this thread ("" if none). */
const char* spd_last_error(void);

/* ---- introspection (tests, statistics).  Output buffers are HOST memory;
 * `bytes` is their capacity; SPD_E_INVALID if too small. ------------------- */
typedef enum {
  SPD_Q_N = 0,            /* int64[1]: number of points */
  SPD_Q_LEVELS = 1,       /* int64[1]: L */
  SPD_Q_PERM = 2,         /* int64[N]: tree position -> original index */
  SPD_Q_NODE_START = 3,   /* int64[nnodes+1]-style: start of every node, heap order */
  SPD_Q_H2_RANK = 4,      /* int32[nnodes]: skeleton size k_v */
  SPD_Q_SKELETON = 5,     /* int64[sum k_v]: skeleton original indices, node by node */
  SPD_Q_NEAR_PTR = 6,     /* int64[nnodes+1]: CSR of near lists */
  SPD_Q_NEAR_IDX = 7,     /* int32[..] */
  SPD_Q_COUP_PTR = 8,     /* int64[nnodes+1]: CSR of coupling lists */
  SPD_Q_COUP_IDX = 9,     /* int32[..] */
  SPD_Q_NNODES = 10,      /* int64[1] */
  SPD_Q_BYTES = 11,       /* int64[1]: device bytes held by the handle */
  SPD_Q_H2_TIMES = 12,    /* double[4]: seconds for tree+lists, bases, blocks, total */
  SPD_Q_PROXY_COUNT = 13, /* int32[nnodes]: points per proxy sphere (0: no ID ran) */
  SPD_Q_H2_STORAGE = 14   /* int64[3]: bytes of the near blocks, coupling blocks and
                             interpolation matrices (W_v, W_v^T, E_v, E_v^T) */
} spd_h2_query;

spd_status spd_h2_query_get(spd_h2_t A, int32_t what, void* host_out, int64_t bytes);

typedef enum {
  SPD_HQ_RANK = 0,       /* int32[nnodes]: HSS rank r_v (root: 0) */
  SPD_HQ_PIVOTS = 1,     /* int32[r_v] of node `node`: CPQR pivot columns */
  SPD_HQ_BASIS = 2,      /* double[rows x r_v]: V_v (leaf) or V-bar_v, col-major */
  SPD_HQ_TRANSFER = 3,   /* double[rho x r_v]: R_v = F_v V-bar_v (nonleaf) */
  SPD_HQ_PHIU = 4,       /* double[r_v x k_v]: Phi_v U_v^H2 */
  SPD_HQ_COUPLING = 5,   /* double[r_v x r_node2]: B_{v,node2} (a near or coupling pair) */
  SPD_HQ_FACTOR = 6,     /* double[n x n]: S_v (leaf) or F_v (nonleaf, root), lower */
  SPD_HQ_ROWS = 7,       /* int64[1]: row count of the node's basis (n_v or rho_v) */
  SPD_HQ_BYTES = 8,      /* int64[1]: device bytes held */
  SPD_HQ_TIMES = 9,      /* double[8]: seconds per phase of the build */
  SPD_HQ_FLOPS = 10      /* double[4]: algorithmic flops of the build phases */
} spd_hss_query;

spd_status spd_hss_query_get(spd_hss_t M, int32_t what, int32_t node,
                             int32_t node2, void* host_out, int64_t bytes);

/* Time the dominant kernel of h2_matvec, the leaf-level pass y_i = U_i y-hat_i
 * + sum_j A_ij x_j over all leaves, for nrhs columns: reps launches bracketed
 * by HIP events on `stream`.  *ms = average milliseconds per launch; *bytes =
 * algorithmic bytes per launch (every near block, leaf basis and skeleton
 * input once, x read once, y written once).  Works on the handle's internal
 * buffers; no caller data is touched. */
spd_status spd_h2_time_near(spd_h2_t A, int32_t nrhs, int32_t reps, void* stream, double* ms,
                            double* bytes);

/* Time each kernel launch of h2_matvec for nrhs columns separately, in the
 * order the product issues them: reps launches each, bracketed by HIP events
 * on `stream`.  ms[i], bytes[i], tags[i] (HOST arrays of cap entries; tags may
 * be NULL): average milliseconds, algorithmic bytes (every A operand once,
 * every distinct B operand once, C once; 0 for the partial-sum reductions
 * that follow a split product) and pass of launch i: 100 + l upward pass at
 * level l, 200 coupling pass, 300 + l downward pass at level l, 400 leaf pass
 * (near field and leaf bases).  *count = number of launches written. */
spd_status spd_h2_time_launches(spd_h2_t A, int32_t nrhs, int32_t reps, void* stream, double* ms,
                                double* bytes, int32_t* tags, int32_t cap, int32_t* count);

/* ---- kernel test hooks: run one batched device kernel on caller buffers.
 * All pointers are DEVICE pointers; shapes are uniform across the batch.
 * They exist so that each kernel can be compared on its own against the
 * CPU oracle; the solver never needs them. ---------------------------------- */
/* C_b = beta C_b + alpha op(A_b) op(B_b), batch stride = matrix size */
spd_status spd_test_gemm(const double* A, const double* B, double* C, int32_t batch,
                         int32_t m, int32_t n, int32_t k, int32_t transA,
                         int32_t transB, double alpha, double beta, void* stream);
/* Y = S X for the block-cyclic symmetric matrix S with nblk block rows of m
 * rows: row i holds nterm blocks A_it (m x m, column-major, ld m, stored at
 * A + (i*nterm + t)*m*m), S_ij = A_it and S_ji = A_it^T for j = (i+1+t) mod
 * nblk, zero elsewhere (nblk >= 2*nterm+1, so no pair repeats).  X and Y are
 * nblk*m x n (ld nblk*m), 1 <= n <= 16: the symmetric-pair product of the H^2
 * matvec on a synthetic layout.  With reps >= 1 the product launch is then
 * replayed reps times alone and *ms receives its average time. */
spd_status spd_test_symm(const double* A, const double* X, double* Y, int32_t nblk,
                         int32_t m, int32_t nterm, int32_t n, int32_t reps, void* stream,
                         double* ms);
/* in-place lower Cholesky of batch n x n matrices; fail[b] = 1 if not SPD */
spd_status spd_test_chol(double* A, int32_t batch, int32_t n, int32_t* fail, void* stream);
/* B_b <- op(L_b)^{-1} B_b (lower L; upper = 1 reads L as upper triangular) */
spd_status spd_test_trsm(const double* L, double* B, int32_t batch, int32_t n,
                         int32_t nrhs, int32_t trans, int32_t upper, void* stream);
/* column-pivoted QR of batch m x n matrices (A destroyed): Q (m x maxrank),
 * piv, rank, diag; which = 0 register kernel, 1 global-memory kernel */
spd_status spd_test_cpqr(double* A, double* Q, int32_t* piv, int32_t* rank,
                         double* diag, int32_t batch, int32_t m, int32_t n,
                         int32_t maxrank, double tol, int32_t which, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SPDHSS_H */
