/*
 * ddlr.h -- C ABI of the DDLR (domain-decomposition low-rank) preconditioner
 * library for AMD Instinct MI355X (gfx950).
 *
 * The method is that of Li & Saad, "Low-rank correction methods for algebraic
 * domain decomposition preconditioners": a symmetric sparse A is split along a
 * partition into p subdomains as A = A0 - E E^T (Sec. 3.1, eqs. splitA1 and
 * split), A0 = blockdiag(B_i + alpha^{-2} E_i E_i^T, C + alpha^2 I), and the
 * inverse is approximated through the Sherman-Morrison-Woodbury formula with a
 * rank-k correction computed by Lanczos (Sec. 3.2 DDLR-1, Sec. 3.3 DDLR-2,
 * Sec. 4.4 (sec:Lan) Lanczos).  The preconditioner is applied inside CG or GMRES
 * (Sec. 5).
 *
 * Conventions for every call:
 *   - All functions return ddlr_status; no exception or abort crosses the ABI.
 *     On failure ddlr_last_error() returns a message for the calling thread.
 *   - Host arrays are plain C arrays owned by the caller and only read (or
 *     written, for outputs) during the call.
 *   - Device vectors are hipMalloc'ed device pointers owned by the caller,
 *     column-major with leading dimension ld >= n, in the caller's own row
 *     order ("user order").  Work is queued on the given hipStream_t (passed
 *     as void*, NULL = the default stream); calls that return results to host
 *     memory synchronise that stream.
 *   - A ddlr_prec is used by one stream at a time; it owns all of its device
 *     memory (matrix, factors, U_k, workspaces) until ddlr_destroy.
 *   - Indices are 0-based.  Matrices are CSR with full symmetric storage and
 *     sorted column indices.
 */
#ifndef DDLR_H
#define DDLR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DDLR_OK = 0,
    DDLR_E_INVALID = -1,         /* bad argument, partition, size or handle state */
    DDLR_E_NOT_SYMMETRIC = -2,   /* A is not symmetric (pattern or values) */
    DDLR_E_BREAKDOWN = -3,       /* zero / non-positive pivot in a local factor */
    DDLR_E_NOT_SPD = -4,         /* preconditioner not SPD: CG refused, or G/H_k singular */
    DDLR_E_NO_CONVERGENCE = -5,  /* Krylov solve hit maxit; x and info are still written */
    DDLR_E_LANCZOS = -6,         /* Lanczos broke down before k+1 Ritz values */
    DDLR_E_OOM = -7,             /* device allocation failed */
    DDLR_E_BUDGET = -8,          /* serving: the HBM budget cannot hold the matrix */
    DDLR_E_DEVICE = -9           /* HIP error, or a host-only handle used for device work */
} ddlr_status;

typedef enum {
    DDLR_VARIANT_A0 = 0,  /* no low-rank part: M^{-1} = A0^{-1} (block-Jacobi-like) */
    DDLR_1 = 1,           /* one-sided, eq. (Mprec) with G_{k,theta}^{-1} of eq. (gkt) */
    DDLR_2 = 2            /* two-sided, eq. (Form2a): A0^{-1} + U_k H_k U_k^T */
} ddlr_variant;

typedef enum { DDLR_THETA_LAMBDA_K1 = 0, DDLR_THETA_ZERO = 1 } ddlr_theta;
typedef enum { DDLR_FACTOR_IC0 = 0, DDLR_FACTOR_ILDL0 = 1 } ddlr_factor;
typedef enum { DDLR_CORDER_MULTICOLOR = 0, DDLR_CORDER_NATURAL = 1 } ddlr_corder;
/* Solver of C_alpha inside every A0 solve (Sec. 4.3 (sec:csolve)): its incomplete LDL^T
 * like the B blocks, or the sparse approximate inverse X of Algorithm alg:mr
 * (self-preconditioned global MR with dropping, X_0 = diag(C_alpha)^{-1}),
 * applied as one sparse product.  X's dropping rule (the paper gives no
 * details or values): Z is symmetrised; in each column the diagonal stays,
 * off-diagonal entries below cinv_tol * ||z_:j||_2 are dropped and the
 * cinv_lfil largest of the rest kept (ties: lower row); an entry stays only if
 * it stays in its column and its row's column, so X is symmetric.  Sums follow
 * a fixed order (each product entry from 0.0 in ascending summation index;
 * traces and norms as running sums in row-major order), so the result is
 * reproducible bit for bit.  X counts as SPD when ||I - C_alpha X||_inf < 1
 * (largest absolute row sum; it bounds the spectral radius of I - C_alpha X). */
/* DDLR_CSOLVE_CHEB: the paper's other C_alpha solver, cheb_iters steps of
 * Chebyshev acceleration (Saad, Iterative Methods for Sparse Linear Systems,
 * Alg. 12.1) from 0, preconditioned by the block-Jacobi matrix
 * D_alpha = blockdiag(C_i) of each subdomain's interface couplings (factored
 * by incomplete LDL^T), on an interval from cheb_lanczos Lanczos steps on the
 * pencil (C_alpha, D_alpha) started from the vector of ones, each extreme Ritz
 * value widened by its residual bound (a non-positive lower end becomes half
 * the smallest Ritz value).  The polynomial solve is symmetric; it counts as
 * SPD when D_alpha's pivots and the smallest Ritz value are positive. */
typedef enum { DDLR_CSOLVE_FACTOR = 0, DDLR_CSOLVE_MR = 1, DDLR_CSOLVE_CHEB = 2 } ddlr_csolve;
/* How DDLR-2's U_k and V_k are computed (Sec. 4.4 (sec:Lan)): Lanczos on
 * E^T A0^{-2} E, then U_k = A0^{-1} E V_k (k more solves); or the Lanczos
 * (Golub-Kahan) bidiagonalisation of A0^{-1} E, which gives both at once:
 * B Q_m = P_m B_m, Z_k = leading right singular vectors of B_m,
 * V_k = Q_m Z_k, U_k = P_m B_m Z_k.  Both use full reorthogonalisation;
 * the bidiagonalisation keeps the n x m basis P_m during the build and its
 * run cannot be continued by ddlr_extend_lowrank. */
typedef enum { DDLR_BUILD_LANCZOS = 0, DDLR_BUILD_BIDIAG = 1 } ddlr_lowrank_build;

/* Reorthogonalisation of the Lanczos vectors (Sec. 4.4, sec:Lan).
 * FULL: every new vector is orthogonalised against all earlier ones
 * (classical Gram-Schmidt twice).  PARTIAL: the scheme the paper uses,
 * Simon's partial reorthogonalisation (Math. Comp. 42, 1984): a recurrence
 * estimates omega_i = q_i^T q_{j+1} from alpha and beta alone,
 *   beta_j omega'_i = beta_i omega_{i+1} + (alpha_i - alpha_j) omega_i
 *                     + beta_{i-1} omega_{i-1} - beta_{j-1} omega''_i + theta
 * (omega: estimates against q_j, omega'': against q_{j-1}; theta = 2 eps
 * ||T||, ||T|| the running max of |alpha_i| + beta_i + beta_{i-1}, with the
 * sign of the rest; omega'_j = eps sqrt(s), omega'_{j+1} = 1; eps = 2^-52);
 * when some |omega'_i| exceeds sqrt(eps), q_{j+1} and q_{j+2} are
 * orthogonalised against all earlier vectors (classical Gram-Schmidt twice)
 * and their estimates reset to eps.  The basis then stays orthogonal to
 * sqrt(eps), the Ritz values are those of full reorthogonalisation to
 * rounding level and the preconditioner agrees to about sqrt(eps). */
typedef enum { DDLR_REORTH_FULL = 0, DDLR_REORTH_PARTIAL = 1 } ddlr_reorth;
typedef enum { DDLR_FP64 = 0, DDLR_FP32 = 1, DDLR_FP32_UK_BF16 = 2 } ddlr_precision;

/* Symmetric matrix, host memory, full storage, sorted columns. */
typedef struct {
    int64_t n;
    const int64_t *row_ptr; /* n+1 */
    const int32_t *col_idx; /* row_ptr[n] */
    const double *val;      /* row_ptr[n] */
} ddlr_csr;

typedef struct {
    double alpha;          /* splitting scale of eq. (EF); default 1 */
    int32_t lanczos_steps; /* Lanczos steps m (k+1..1024); 0 -> 2k */
    int32_t theta;         /* ddlr_theta; default lambda_{k+1} (Sec. 5) */
    int32_t factor;        /* ddlr_factor: IC(0) (positive pivots) or ILDL(0) (nonzero pivots) */
    int32_t corder;        /* ddlr_corder: order of the interface block inside C_alpha's factor */
    int32_t precision;     /* ddlr_precision of the preconditioner; Krylov is always FP64 */
    int32_t device;        /* HIP device ordinal; -1 = host-only setup (ordering and factors only) */
    int32_t no_autotune;   /* 0: tune launch shapes on the first solve with a column count (default) */
    int32_t lanczos_check; /* 0: lanczos_steps fixed steps; > 0: the control of Sec. 5 -- eq. (converge) on the
                              sum of the k largest Ritz values, tested every lanczos_check steps (paper: 10) */
    int32_t lanczos_max;   /* with lanczos_check > 0: step limit; 0 -> 5k (Sec. 5); steps are at most 1024 */
    double lanczos_tol;    /* with lanczos_check > 0: tolerance of eq. (converge); 0 -> 1e-4 (Sec. 5) */
    uint64_t seed;                /* Lanczos start vector when lanczos_start is NULL */
    const double *lanczos_start;  /* host, length n, user order: its interface entries form q_1 */
    int32_t csolve;        /* ddlr_csolve; default DDLR_CSOLVE_FACTOR */
    int32_t cinv_iters;    /* DDLR_CSOLVE_MR: MR steps (>= 0); default 3 */
    double cinv_tol;       /* DDLR_CSOLVE_MR: drop tolerance relative to the column norm (>= 0); default 0.01 */
    int32_t cinv_lfil;     /* DDLR_CSOLVE_MR: kept off-diagonal entries per column (>= 0); default 20 */
    int32_t lowrank_build; /* ddlr_lowrank_build; DDLR_BUILD_BIDIAG needs DDLR_2 and lanczos_check = 0; default
                              DDLR_BUILD_LANCZOS */
    int32_t cheb_iters;    /* DDLR_CSOLVE_CHEB: Chebyshev steps per solve (1..64); default 5 (the paper's) */
    int32_t cheb_lanczos;  /* DDLR_CSOLVE_CHEB: Lanczos steps of the spectrum estimate (2..200); default 10 */
    int32_t lanczos_reorth; /* ddlr_reorth of the low-rank Lanczos run (DDLR_BUILD_LANCZOS only); default
                               DDLR_REORTH_FULL */
} ddlr_options;

typedef struct {
    int32_t method;  /* 0 = CG (Sec. 5, SPD matrix and preconditioner), 1 = GMRES(restart) */
    int32_t restart; /* GMRES restart length; default 40 */
    int32_t maxit;   /* default 500 */
    int32_t reserved;
    double rtol;     /* stop when ||r|| <= rtol ||b||; default 1e-6 */
} ddlr_solve_options;

typedef struct {
    int32_t iters;       /* iterations (GMRES: inner steps) */
    int32_t status;      /* DDLR_OK or DDLR_E_NO_CONVERGENCE for this right-hand side */
    double relres;       /* recursive residual / ||b|| (GMRES: the least-squares estimate) */
    double relres_true;  /* ||b - A x|| / ||b|| computed after the solve */
} ddlr_solve_info;

typedef struct {
    int64_t n, m, s;        /* order, interior unknowns, interface unknowns */
    int64_t nnz_a, nnz_l, nnz_e;
    int32_t p, k, variant, lanczos_steps;
    int32_t ncolours, levels_b_max, levels_c, spd;
    int32_t precision, on_device;
    double theta, c0;
    double fill_ratio;      /* stored preconditioner entries / nnz(A) */
    double setup_ms, lanczos_ms;
    int32_t csolve;         /* ddlr_csolve in use */
    int32_t cinv_iters;     /* MR steps taken (fewer than asked if C Z vanished) */
    int64_t nnz_cinv;       /* stored entries of X */
    double cinv_res;        /* ||I - C_alpha X||_F */
    double cinv_res_inf;    /* ||I - C_alpha X||_inf (the SPD certificate needs < 1) */
    double cheb_lo, cheb_hi;           /* DDLR_CSOLVE_CHEB: safeguarded interval of D_alpha^{-1} C_alpha */
    double cheb_ritz_lo, cheb_ritz_hi; /* its smallest and largest Ritz value */
    int32_t lanczos_reorth;            /* ddlr_reorth of the run */
    int32_t lanczos_reorth_steps;      /* steps whose new vector was reorthogonalised (FULL: every step) */
} ddlr_info;

typedef struct ddlr_prec ddlr_prec;

/* A context: the device that handles created in it run on and a budget of
 * device memory (HBM) that all of their allocations share.  The problem
 * statement (Sec. 2.1) places one linear system on one machine; a context is
 * that machine's share: device ordinal (-1: host-only handles, setup and
 * factors without device work) and budget in bytes (0 = unlimited).  Every
 * device allocation of a handle in the context -- matrix, factors, U_k,
 * Lanczos basis, solver workspaces grown later -- is counted while it lives;
 * one that would exceed the budget fails with DDLR_E_BUDGET (a failing setup
 * frees what it took, *out = NULL).  ddlr_ctx_destroy may be called while
 * handles of the context still exist: the context is freed when the last of
 * them is destroyed.  Errors: DDLR_E_INVALID (null out, device < -1),
 * DDLR_E_DEVICE (no such device). */
typedef struct ddlr_ctx ddlr_ctx;
ddlr_status ddlr_ctx_create(int32_t device, size_t hbm_budget_bytes, ddlr_ctx **out);
/* Bytes currently allocated by the context's handles, the most ever held at
 * once, and the budget (0 = unlimited).  Any output may be NULL. */
ddlr_status ddlr_ctx_usage(const ddlr_ctx *ctx, size_t *used, size_t *peak, size_t *budget);
void ddlr_ctx_destroy(ddlr_ctx *ctx);

/* Library version (major*100 + minor). */
int32_t ddlr_version(void);

/* Fills *opt with the defaults listed above. */
void ddlr_options_default(ddlr_options *opt);
void ddlr_solve_options_default(ddlr_solve_options *opt);

/*
 * Builds a DDLR preconditioner (Sec. 4.1, the four steps of the build):
 *  1. classifies unknowns as interior / interface by the edge separator of
 *     `part` (Sec. 2.1) and reorders to the form of eq. (Bmat);
 *  2./3. forms B_{i,alpha}, C_alpha and E (Sec. 3.1) and factors every block by
 *     incomplete LDL^T with the block's own pattern (Sec. 5);
 *  4. runs `lanczos_steps` Lanczos steps with full or partial
 *     reorthogonalisation (opt->lanczos_reorth) on
 *     E^T A0^{-1} E (DDLR-1) or E^T A0^{-2} E (DDLR-2) (Sec. 4.4 (sec:Lan)) and forms
 *     U_k with G_{k,theta}^{-1} (eq. gkt) or H_k (Lemma on H_k).
 * ctx: context (device and memory budget; its device replaces opt->device), or
 * NULL for opt->device and no budget.
 * A: host CSR (copied); part: host int32[n] with values in [0,p) (copied);
 * k: rank (ignored for DDLR_VARIANT_A0; 1 <= k < number of interface unknowns).
 * Errors: DDLR_E_INVALID, DDLR_E_NOT_SYMMETRIC, DDLR_E_BREAKDOWN (message names
 * the row), DDLR_E_LANCZOS, DDLR_E_NOT_SPD (theta >= 1 or I - U_k^T E V_k not
 * SPD), DDLR_E_OOM, DDLR_E_BUDGET (the context's budget), DDLR_E_DEVICE.  On
 * failure *out is NULL and nothing leaks.
 */
ddlr_status ddlr_setup(ddlr_ctx *ctx, const ddlr_csr *A, const int32_t *part, int32_t p, int32_t k,
                       int32_t variant, const ddlr_options *opt, ddlr_prec **out);

/* Saving and restoring a built preconditioner (the computed data that Sec.
 * 4.7, sec:improv, keeps and reuses).  ddlr_export_setup writes to `path`
 * everything the build computed from A and the partition: the ordering of
 * step 1 (perm, block offsets, interface colours), the local factors (strict
 * lower L in internal order as CSR, and D), the level of every row, the
 * approximate inverse X of C_alpha or the Chebyshev interval when those
 * solvers are used, and the low-rank part (U_k in user order with
 * lambda_1..lambda_k and theta, or H_k).  ddlr_import_setup rebuilds a handle
 * from A and such a file without classifying, factoring or running Lanczos;
 * the result applies the same operator as the exported handle.  A file written
 * by another program with the same layout (e.g. another implementation of
 * the same build) is accepted after these checks: perm is a permutation; the interiors
 * of different blocks are not coupled in A; L is strictly lower with sorted
 * columns inside its row's block; pivots are finite and nonzero; stored levels,
 * if present, equal the schedule recomputed from L.
 *
 * File layout (little-endian): the 8 bytes "DDLRSET1", int32 version (1),
 * int32 record count, then per record: 16-byte NUL-padded name, int32 type (1
 * int32, 2 int64, 3 float64), int32 0, int64 element count, the elements.
 * Records: "n_p" int64 {n, p}; "alpha" f64 {alpha}; "csolve_prec_nu" int32
 * {ddlr_csolve, ddlr_precision, Chebyshev steps}; "perm" int32[n] (internal
 * position -> user row: interiors of blocks 0..p-1, then the interface);
 * "boff" int64[p+2] (block starts, boff[p] = interior count, boff[p+1] = n);
 * "colour" int32[s]; "L.rowptr" int64[n+1], "L.col" int32, "L.val" f64 (strict
 * lower, internal order); "D" f64[n]; optional "level" int32[n]; with
 * DDLR_CSOLVE_MR "X.rowptr" int64[s+1], "X.col" int32, "X.val" f64 (interface
 * positions), "X.cert" f64 {||I - C_alpha X||_inf, SPD flag} and "X.res" f64
 * (||I - C_alpha X_j||_F for j = 0..steps, as ddlr_get_cinv returns); with
 * DDLR_CSOLVE_CHEB "cheb" f64 {lo, hi, smallest Ritz, largest Ritz}; with a
 * low-rank part "lowrank" int32 {variant, k}, "U" f64[n*k] (user order,
 * column-major) and "aux" f64 (DDLR-1: lambda_1..lambda_k, theta; DDLR-2:
 * H_k column-major), the layout of ddlr_get_lowrank.
 *
 * Export: any handle (host-only handles have no low-rank part).  Import: ctx
 * as in ddlr_setup (NULL: device 0, no budget); the precision is the stored
 * one; a host-only context ignores the low-rank records.  Errors:
 * DDLR_E_INVALID (IO error, bad file, data that fail the checks above, another
 * matrix order), DDLR_E_OOM, DDLR_E_BUDGET, DDLR_E_DEVICE.  On failure *out is
 * NULL and nothing leaks. */
ddlr_status ddlr_export_setup(const ddlr_prec *h, const char *path);
ddlr_status ddlr_import_setup(ddlr_ctx *ctx, const ddlr_csr *A, const char *path, ddlr_prec **out);

/* y = M^{-1} x for nrhs columns.  DDLR-1: eq. (Mprec) with G_{k,theta}^{-1}
 * of eq. (gkt), evaluated with two A0 solves as in Algorithm alg:prec1
 * (Sec. 4.2); DDLR-2: one A0 solve plus U_k H_k U_k^T x (eq. Form2a).
 * x, y: device, user order, x and y must not overlap. */
ddlr_status ddlr_apply(ddlr_prec *h, int32_t nrhs, const double *x, int64_t ldx, double *y, int64_t ldy,
                       void *stream);

/* y = A0^{-1} x with the local factors only (the A0 solves of Algorithm
 * alg:prec1: the p solves with B_{i,alpha} and the solve with C_alpha). */
ddlr_status ddlr_a0_solve(ddlr_prec *h, int32_t nrhs, const double *x, int64_t ldx, double *y, int64_t ldy,
                          void *stream);

/* y = A x (the operator of the Krylov solves), device, user order. */
ddlr_status ddlr_spmv(ddlr_prec *h, int32_t nrhs, const double *x, int64_t ldx, double *y, int64_t ldy,
                      void *stream);

/* Solves A x = b for nrhs right-hand sides with PCG or right-preconditioned
 * GMRES(restart), x0 = 0, stopping rule of Sec. 5 (residual reduced by rtol,
 * at most maxit iterations).  b, x: device, user order.  info: host array of
 * nrhs entries.  Returns DDLR_E_NOT_SPD for CG with a preconditioner that is
 * not certified SPD (largest Ritz value >= 1), DDLR_E_NO_CONVERGENCE if any
 * right-hand side did not converge (x and info written for all). Synchronises
 * the stream. */
ddlr_status ddlr_solve(ddlr_prec *h, int32_t nrhs, const double *b, int64_t ldb, double *x, int64_t ldx,
                       const ddlr_solve_options *opt, ddlr_solve_info *info, void *stream);

/* ddlr_apply for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, result and errors as ddlr_apply, and the same kernels, but every
 * temporary (gathered input and output, the A0-solve and interface vectors,
 * the low-rank reduction partials, the Chebyshev vectors) lives in one 64 MiB
 * device array owned by the library, one per GPU, held until the process
 * ends; the call allocates nothing and runs no autotuning (it uses the shapes
 * already tuned for the handle, else the defaults).  Columns go through in
 * chunks of at most 16 that fit the array.  Errors: DDLR_E_INVALID (besides
 * ddlr_apply's) when a single column needs more scratch than the array holds
 * (about 32 bytes per row plus 16 per interface row in FP64, 24 + 8 in FP32,
 * plus 8 KiB per rank, four more n-vectors with the Chebyshev solver); the
 * message gives both sizes.  The array is shared by every call on the same
 * GPU and keeps the last call's contents (every temporary is written before
 * it is read): calls that overlap in time on one GPU, from any handle or
 * stream, race and must be serialised by the caller. */
ddlr_status ddlr_apply_noalloc(ddlr_prec *h, int32_t nrhs, const double *x, int64_t ldx, double *y, int64_t ldy,
                               void *stream);

/* Sizes, counts and timings of a built preconditioner. */
ddlr_status ddlr_query(const ddlr_prec *h, ddlr_info *info);

/* Reordering of step 1: perm[i] = user row at internal position i (interiors
 * of subdomain 0..p-1, then the interface block in C_alpha's factor order);
 * iface[u] = 1 for interface rows (user order); colour[j] = colour of the j-th
 * interface position (0 with natural order).  Host arrays n, n, s. */
ddlr_status ddlr_get_ordering(const ddlr_prec *h, int32_t *perm, int32_t *iface, int32_t *colour);

/* Local factors in internal order: strict lower L as CSR (row_ptr n+1,
 * col/val nnz_l) and D (n).  Host arrays.  With DDLR_CSOLVE_MR the interface
 * rows of L are empty and D is 1 there; with DDLR_CSOLVE_CHEB they hold the
 * factor of D_alpha = blockdiag(C_i). */
ddlr_status ddlr_get_factor(const ddlr_prec *h, int64_t *row_ptr, int32_t *col, double *val, double *D);

/* The approximate inverse X ~ C_alpha^{-1} of Algorithm alg:mr (Sec. 4.3 (sec:csolve)),
 * DDLR_CSOLVE_MR only: s x s CSR in interface positions of the internal order
 * (row_ptr s+1, col/val nnz_cinv of ddlr_query) and, if res is non-NULL, the
 * residual norms ||I - C_alpha X_j||_F for j = 0..cinv_iters.  Host arrays
 * owned by the caller.  Errors: DDLR_E_INVALID (null argument, or C_alpha
 * factored).  Works on host-only handles. */
ddlr_status ddlr_get_cinv(const ddlr_prec *h, int64_t *row_ptr, int32_t *col, double *val, double *res);

/* A partition of the unknowns for matrices without a geometric split.  The
 * method takes the partition into p subdomains as an input produced by a
 * graph partitioner (Sec. 2.1); this helper is a deterministic recursive
 * bisection of the adjacency graph of A (pattern only): a vertex set with q
 * parts to form is cut after the first round(|set| floor(q/2) / q) vertices of
 * a breadth-first order of its induced subgraph, started from a
 * pseudo-peripheral vertex (George-Liu search from the lowest-numbered
 * vertex, neighbours in ascending order, unreached components appended from
 * their lowest vertex); the first piece gets the lower part ids.  part: host
 * array of n entries (0..p-1), written on success.  Errors: DDLR_E_INVALID for
 * bad arguments or if a part would be empty (fewer vertices than parts in a
 * piece). */
ddlr_status ddlr_partition_graph(const ddlr_csr *A, int32_t p, int32_t *part);

/* The geometric partition of the model problems (the configurations' box
 * splits; the paper partitions with an external tool, Sec. 2.1): a grid of
 * nx*ny*nz points numbered lexicographically (x fastest; nz = 1 for 2-D) is
 * cut into px*py*pz boxes, each axis into P runs of consecutive points whose
 * first (N mod P) runs are one point longer; the point (x, y, z) gets part
 * bx + px*(by + py*bz).  part: host array of nx*ny*nz entries.  Errors:
 * DDLR_E_INVALID (null part, a count < 1, more parts than points on an axis). */
ddlr_status ddlr_partition_box(int32_t nx, int32_t ny, int32_t nz, int32_t px, int32_t py, int32_t pz,
                               int32_t *part);

/* Level of each internal row in its block's forward triangular schedule. */
ddlr_status ddlr_get_levels(const ddlr_prec *h, int32_t *level);

/* Lanczos record: alpha_1..alpha_m, beta_1..beta_m and Ritz values (descending),
 * m = info.lanczos_steps.  Host arrays. */
ddlr_status ddlr_get_lanczos(const ddlr_prec *h, double *alpha, double *beta, double *ritz);

/* Per-step reorthogonalisation of the stored Lanczos run (Sec. 4.4,
 * sec:Lan, with DDLR_REORTH_PARTIAL): flags host int32[lanczos_steps],
 * flags[j] = 1 when the vector q_{j+1} made at step j was orthogonalised
 * against the earlier ones (with DDLR_REORTH_FULL every flag is 1).  Errors:
 * DDLR_E_INVALID for a null handle or a handle without a Lanczos run. */
ddlr_status ddlr_get_lanczos_reorth(const ddlr_prec *h, int32_t *flags);

/* Low-rank data in user order (host).  U: n x k column-major (DDLR-1: only the
 * interface rows are nonzero).  aux: DDLR-1 lambda_1..lambda_k then theta
 * (k+1 values); DDLR-2 H_k (k x k column-major). */
ddlr_status ddlr_get_lowrank(const ddlr_prec *h, double *U, double *aux);

/* Replaces the low-rank data (same layout as ddlr_get_lowrank), e.g. to
 * restore a saved preconditioner.  variant 1 or 2; 1 <= k. */
ddlr_status ddlr_set_lowrank(ddlr_prec *h, int32_t variant, int32_t k, const double *U, const double *aux);

/* Kernel timing with HIP events recorded on the launch stream around each
 * launch of a kernel class: 0 = the per-block triangular-solve kernel of the
 * A0 solve (all B_{i,alpha} blocks, and C_alpha when it is not level-split),
 * 1 = the per-level kernels of C_alpha, 2 = the SpMV with A, 3 = the low-rank
 * correction kernels.  on != 0 enables and resets the counters; 0 disables.
 * Synchronises the device. */
ddlr_status ddlr_profile(ddlr_prec *h, int32_t on);

/* Accumulated milliseconds and launches of kernel class `which` since
 * profiling was enabled, counting only launches that took at least min_us
 * microseconds (0: all; a launch after every column of a solve has converged
 * returns at once, and a threshold of a few microseconds leaves those out).
 * Synchronises the device. */
ddlr_status ddlr_profile_read(ddlr_prec *h, int32_t which, double min_us, double *total_ms, int64_t *launches);

/* Improving a given preconditioner (Sec. on improving a given
 * preconditioner): continues the Lanczos run of ddlr_setup (kept on the
 * device: s x (m+1) doubles) by `more_steps` steps -- or, with check > 0, until
 * eq. (converge) holds at a multiple of `check` (tolerance tol, 0 -> 1e-4)
 * within `more_steps` -- and rebuilds U_k and G_k^{-1} / H_k with rank k (any
 * k with k+1 <= total steps, larger or smaller than before).  The result is
 * the same as a setup whose Lanczos ran the combined number of steps.  After
 * a breakdown the run cannot grow and only the rank can change.  Errors:
 * DDLR_E_INVALID (no Lanczos run: variant 0 or data from ddlr_set_lowrank;
 * bad arguments), DDLR_E_LANCZOS (fewer than k+1 steps), DDLR_E_NOT_SPD as
 * for ddlr_setup; on error the previous low-rank part is gone and the handle
 * acts as the A0-only preconditioner until a successful call.  Synchronises
 * the device. */
ddlr_status ddlr_extend_lowrank(ddlr_prec *h, int32_t k, int32_t more_steps, int32_t check, double tol);

/* Launch-shape autotuner.  The block triangular solve of the A0 solve (the
 * local solves of Sec. 4.2, steps 1 and 5) can give a workgroup 1, 2, 4 or 8
 * right-hand sides of one block, sharing the block's factor entries between
 * them; with one right-hand side per workgroup, blocks whose levels are
 * narrow can use workgroups of 64 (one wave, no barriers) or 256 threads
 * instead of 512; the plain per-level kernel (CSR rows, no ring) is also a
 * candidate; and the interface block's level kernels can run beside it on a
 * side stream or in line.  The first solve, apply or A0 solve with a given column
 * count times the eligible shapes on the device (HIP events, a few
 * milliseconds) and keeps the fastest; every shape does the same arithmetic
 * in the same order, so results do not depend on the choice.  ddlr_tune runs
 * (retune != 0: re-runs) the tuner for nrhs in 1..16 on `stream` and reports
 * the choice and the measured times; it synchronises the stream.  Batches
 * (ddlr_batch_*) use fixed shapes (the smallest eligible workgroup, one
 * column).  Setting options.no_autotune keeps the defaults (one column per
 * workgroup of the smallest eligible size, overlap on) unless ddlr_tune is
 * called.  PCG (ddlr_solve, method 0) runs its iterations in chunks of 8,
 * replayed from a captured HIP graph or launched eagerly: graph replay saves
 * launch overhead, but forked branches of a replayed graph (the interface
 * levels beside the block solve) may run one after the other.  Unless the
 * environment forces one form (DDLR_CG_GRAPH=1 graphs, 0 eager), the first
 * solves with a column count time whole chunks on the host, three per
 * candidate: replayed and eager, each with the interface block's solve beside
 * and in line with the block solve (that overlap competes with other forked
 * work inside an iteration and a replayed graph may serialise it, so its
 * A0-only timing above does not decide it for PCG); the fastest (minimum over
 * its chunks) is kept, but replayed chunks with the interface solve in line
 * stay unless another candidate is more than 1 % faster.
 * cg_* below report that measurement.  For systems of at most 262,144 rows
 * with the interface block factored, DDLR-1 or A0 alone, FP64 or FP32 and
 * k <= 64, PCG may also run in the persistent form: one launch per solve, one
 * workgroup per right-hand side running every step of every iteration (the
 * A0 solve over the merged levels of all blocks, the solve vector in LDS when
 * it fits) until its residual test holds.  Its workgroup size (64 to 1024
 * threads) is tuned on its first launch (a few timed iterations each);
 * the first such solve of a column count runs persistent and records its time
 * per iteration, and once the chunked forms are measured the faster per
 * iteration is used.  DDLR_CG_PERSIST=1 / 0 forces it on / off. */
typedef struct {
    int32_t nrhs;            /* column count the shape is for */
    int32_t ring_cols;       /* right-hand sides per workgroup of the block triangular solve */
    int32_t overlap;         /* 1: interface levels on the side stream, 0: in line */
    int32_t ring_threads;    /* threads per workgroup of the block triangular solve (64, 256, 512), or -1:
                                the plain per-level kernel (CSR rows, no LDS ring) */
    float a0_us[4];          /* A0 solve time, 512 threads, 1, 2, 4, 8 columns per workgroup (0: not eligible);
                                one column runs the packed-record kernel when its data exist */
    float a0_no_overlap_us;  /* best shape with the interface levels in line (0: not measured) */
    float a0_thin_us[2];     /* one column per workgroup of 64 / 256 threads (0: not eligible) */
    float a0_plain_us;       /* the plain per-level kernel (0: not measured) */
    int32_t cg_graph;        /* PCG chunks of this column count: 1 replayed graphs, 0 eager launches,
                                -1 still being measured */
    float cg_eager_us;       /* fastest timed eager chunk of 8 PCG iterations with the interface solve beside
                                the block solve, or in the only form when nothing overlaps (0: none yet) */
    float cg_graph_us;       /* the same for replayed chunks */
    int32_t cg_overlap;      /* PCG: interface solve beside (1) or in line with (0) the block solve; -1: still
                                being measured, or nothing to overlap */
    float cg_eager_in_line_us; /* fastest eager chunk with the interface solve in line (0: not timed) */
    float cg_graph_in_line_us; /* fastest replayed chunk with the interface solve in line (0: not timed) */
    int32_t cg_persist;        /* PCG in the persistent form (one launch per solve, one workgroup per column):
                                  1 chosen, 0 not (not eligible, or slower per iteration), -1 not yet decided */
    float cg_persist_us;       /* measured time per iteration of the persistent form (0: not measured) */
    int32_t persist_threads;   /* workgroup size the persistent form uses (0: not tuned yet) */
    float persist_nt_us[5];    /* its tuning: time per iteration with 64, 128, 256, 512, 1024 threads */
} ddlr_tuning;
ddlr_status ddlr_tune(ddlr_prec *h, int32_t nrhs, int32_t retune, ddlr_tuning *out, void *stream);

/* Releases everything the handle owns.  NULL is ignored. */
void ddlr_destroy(ddlr_prec *h);

/*
 * Batches of independent systems.  The paper motivates reuse of a built
 * preconditioner for many solves (Sec. 6); a batch solves many different
 * systems at once: their device structures are concatenated so that every
 * kernel (SpMV, the A0 solve, E / E^T) covers all systems in one launch,
 * while dot products, CG scalars and the rank-k correction are per system.
 * The iteration loop is captured once into a HIP graph and replayed.
 *
 * ddlr_batch_create: members are built device handles (same device and
 * precision, variant DDLR_1 or DDLR_VARIANT_A0, FP64 or FP32); the batch copies
 * what it needs, so members may be destroyed afterwards.  nsys <= 1024.
 * Vectors of a batch are device arrays holding the systems' vectors one after
 * the other, each in its own user order; ddlr_batch_offsets gives the nsys+1
 * start offsets (host array).
 */
typedef struct ddlr_batch ddlr_batch;
ddlr_status ddlr_batch_create(int32_t nsys, ddlr_prec *const *members, ddlr_batch **out);
ddlr_status ddlr_batch_offsets(const ddlr_batch *b, int64_t *offsets);
/* y = M_q^{-1} x_q for every system q. */
/* The batch's solve form: persistent = 1 when ddlr_batch_solve runs the
 * persistent PCG (one workgroup per system, the whole solve in one launch,
 * captured once into a HIP graph and replayed; batches whose rank exceeds 64
 * or with DDLR_BATCH_PERSIST=0 replay captured chunks of 8 iterations
 * instead); threads = the workgroup size tuned on the first solve (0 before);
 * us_per_iter[5] = its tuning: microseconds per iteration of the launch with
 * 64, 128, 256, 512 and 1024 threads. */
ddlr_status ddlr_batch_tuning(const ddlr_batch *b, int32_t *persistent, int32_t *threads, float *us_per_iter);
/* Workgroups per system of the persistent form (members: host array of nsys
 * entries; 0 for every system when the batch replays chunks).  A batch whose
 * systems differ in size runs as long as its slowest system, so
 * ddlr_batch_create gives the systems estimated to be slowest several
 * workgroups (a group) when the lanes fit the resident workgroups of the
 * device: in the A0 solves the first min(G, p) members each sweep the merged
 * levels of their own subdomain blocks (the blocks of A0 are independent,
 * Sec. 3.1), the last of them also the interface block and the interface step
 * of the correction; the SpMV, dot products and vector updates split the rows
 * evenly over all G members; members meet at workgroup barriers in device
 * memory.  When the library chose the groups, its first persistent solves
 * (up to two, each of at least 20 iterations) measure every system's time
 * (ddlr_batch_times) and choose the groups again from those times; the tables
 * are rebuilt when that lowers the slowest system's time by a tenth, so a
 * later solve may differ from the first at rounding level.
 * DDLR_BATCH_GROUP=0 keeps one workgroup per system, =N asks for N (no
 * regrouping); DDLR_BATCH_REGROUP=0 keeps the first choice.
 * Errors: DDLR_E_INVALID (null argument). */
ddlr_status ddlr_batch_members(const ddlr_batch *b, int32_t *members);
/* Device time of each system in the last persistent ddlr_batch_solve (us: host
 * array of nsys entries, microseconds from the launch start of the system's
 * workgroups to the end of its slowest one, by the device wall clock; 0 for
 * every system before such a solve or with the chunked form).  The batch
 * takes as long as its largest entry.  Errors: DDLR_E_INVALID (null argument). */
ddlr_status ddlr_batch_times(const ddlr_batch *b, double *us);
ddlr_status ddlr_batch_apply(ddlr_batch *b, const double *x, double *y, void *stream);
/* PCG on every system (x0 = 0, stopping rule of Sec. 5); info: host array of
 * nsys entries.  Synchronises the stream.  DDLR_E_NO_CONVERGENCE if any system
 * hit maxit (x and info written for all). */
ddlr_status ddlr_batch_solve(ddlr_batch *b, const double *bvec, double *x, const ddlr_solve_options *opt,
                             ddlr_solve_info *info, void *stream);
void ddlr_batch_destroy(ddlr_batch *b);

/*
 * Serving: resident preconditioners, requests of 1..nrhs right-hand sides
 * arriving at any time, continuous batching.  Every added matrix keeps its
 * factors and U_k on the device and owns `slots_per_matrix` CG lanes (columns).
 * A worker thread admits queued right-hand sides into free lanes of their
 * matrix, runs a few CG iterations on every matrix with lanes (one stream per
 * matrix, so matrices overlap on the device; only the lanes up to the highest
 * occupied one are iterated), and retires finished lanes, computing the true
 * residual ||b - A x|| and copying x back.  Each lane's arithmetic is
 * independent of the other lanes and of its admission time, so a result is the
 * same alone and in a mix.  The device lock is taken per matrix while its work
 * is queued, so other calls on the device interleave with the worker.
 *
 * ddlr_server_create: device, HBM budget in bytes (0 = unlimited), lanes per
 *   matrix (1..16).
 * ddlr_server_add: the server uses `h` exclusively from now on (do not use it
 *   for other calls until the server is destroyed); DDLR_E_BUDGET if the
 *   resident bytes of all added matrices would exceed the budget.
 * ddlr_server_submit: b_host / x_host are host arrays of nrhs columns (user
 *   order, ld = n) that must stay valid until the request is done; x_host is
 *   written when the request completes.  CG only (method 0).
 * ddlr_server_poll / ddlr_server_wait: info is a host array of nrhs entries
 *   (relres_true = ||b - A x|| / ||b|| of the returned x).
 * ddlr_server_stats: counters, solves/s over the span from the first submit
 *   to the last completion, p50 / p99 request latency (submit to completion).
 * ddlr_server_reset_stats: starts a new measurement window: clears the
 *   latency record and the submitted / done / solves counters; requests in
 *   flight are counted in the new window when they complete.
 */
typedef struct ddlr_server ddlr_server;
typedef struct {
    int64_t requests_submitted, requests_done, solves_done, queued;
    double solves_per_s, p50_ms, p99_ms;
    size_t hbm_used, hbm_budget;
    int32_t matrices, reserved;
} ddlr_server_counters;
ddlr_status ddlr_server_create(int32_t device, size_t hbm_budget_bytes, int32_t slots_per_matrix, ddlr_server **out);
ddlr_status ddlr_server_add(ddlr_server *s, ddlr_prec *h, int32_t *matrix_id);
ddlr_status ddlr_server_submit(ddlr_server *s, int32_t matrix_id, int32_t nrhs, const double *b_host, double *x_host,
                               const ddlr_solve_options *opt, uint64_t *ticket);
ddlr_status ddlr_server_poll(ddlr_server *s, uint64_t ticket, int32_t *done, ddlr_solve_info *info);
ddlr_status ddlr_server_wait(ddlr_server *s, uint64_t ticket, ddlr_solve_info *info);
ddlr_status ddlr_server_stats(ddlr_server *s, ddlr_server_counters *stats);
ddlr_status ddlr_server_reset_stats(ddlr_server *s);
void ddlr_server_destroy(ddlr_server *s);

const char *ddlr_status_string(int32_t status);
const char *ddlr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DDLR_H */
