/*
 * sait.h -- C ABI of libsait, an MI355X (gfx950) implementation of the
 * sparse approximate inverse for triangular matrices (SAIT) of
 * Z. Lu, "A sparse approximate inverse for triangular matrices based on
 * Jacobi iteration", arXiv 2106.12836.
 *
 * The library takes a sparse matrix A, forms incomplete LU factors
 * A ~ L U (Sec. 3.1), builds M_L ~ L^-1 and M_U ~ U^-1 with the truncated
 * Jacobi series evaluated in Horner form with dropping (Sec. 2, Eq. M_m,
 * Eq. Recursive; Alg. 2 SAIT_Thr, Alg. 3 SAIT_Pat) and replaces the two
 * triangular solves U(Lx) = y of ILU preconditioning by two sparse
 * matrix-vector products x = M_U (M_L y) (Sec. 3.1) inside restarted
 * (flexible) GMRES.
 *
 * General rules for every entry point:
 *   - Sparse matrices are CSR: int32 row pointers (n+1 entries, starting
 *     at 0, non-decreasing), int32 column indices sorted and unique within
 *     each row, double values.
 *   - Pointers documented as "host" are read (or written) only during the
 *     call; the caller keeps ownership.  Pointers documented as "device"
 *     are caller-owned device memory on the device that was current when
 *     the handle was built; the library reads/writes them in stream order
 *     on `hip_stream` (a hipStream_t; NULL = the null stream).
 *   - Dense vectors / blocks of vectors are row-major n x nrhs with leading
 *     dimension ld >= nrhs (element (i,k) at i*ld + k); nrhs = 1 uses ld 1.
 *   - A negative return value is an error (nothing is leaked, output
 *     handles stay NULL); a positive value is a usable result with a
 *     caveat.  No entry point aborts or prints; sait_last_error() returns
 *     a thread-local description of the last non-OK status.
 *   - Entry points are thread-safe for distinct handles; calls that share
 *     a handle must not overlap.
 */
#ifndef SAIT_H
#define SAIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sait_handle_s *sait_handle;

/* Status codes. */
enum {
    SAIT_OK = 0,
    SAIT_NOT_CONVERGED = 1,   /* solve hit maxit; x holds the last iterate */
    SAIT_BREAKDOWN = 2,       /* LOBPCG: the trial basis became numerically dependent */
    SAIT_E_INVALID = -1,      /* bad argument, malformed CSR, unsupported shape */
    SAIT_E_ZERO_PIVOT = -2,   /* zero (or missing) diagonal in ILU or in a SAIT input */
    SAIT_E_NONFINITE = -3,    /* NaN/Inf in an input or produced by a factorisation */
    SAIT_E_NOMEM = -4,        /* device or host allocation failed */
    SAIT_E_DEVICE = -5        /* HIP runtime error */
};

/* Incomplete factorisation feeding SAIT (Sec. 3.1 takes L, U from ILU).
 * SAIT_PARILU is the fine-grained parallel ILU of Chow and Patel (cited in
 * the introduction for building ILU factors in parallel): the symbolic
 * pattern is formed on the host, the factors on the device by synchronous
 * sweeps u_ij = a_ij - sum_{k<i} l_ik u_kj, l_ij = (a_ij - sum_{k<j} l_ik u_kj)
 * / u_jj over the pattern; enough sweeps give the ILU factors of that
 * pattern exactly.  SAIT_PARIC is its symmetric (incomplete Cholesky) form
 * for a symmetric A: only u_ij (i <= j) are iterated, u_ij = a_ij -
 * sum_{k<i} (u_ki / u_kk) u_kj, and l_ji = u_ij / u_ii, so L and U stay
 * symmetric after every sweep (as PCG needs); the pattern must be
 * structurally symmetric (SAIT_E_INVALID otherwise) and the upper triangle
 * of A is read. */
enum { SAIT_ILU0 = 0, SAIT_ILUT = 1, SAIT_ILUK = 2, SAIT_PARILU = 3, SAIT_PARIC = 4 };

/* Storage precision of M_L, M_U values (accumulation is FP64 for SAIT_F64,
 * binary32 otherwise). */
enum { SAIT_F64 = 0, SAIT_F32 = 1, SAIT_BF16 = 2 };

/* Matrices a handle can export (sait_export). */
enum { SAIT_MAT_A = 0, SAIT_MAT_L = 1, SAIT_MAT_U = 2, SAIT_MAT_ML = 3, SAIT_MAT_MU = 4 };

/* Optional device allocator.  alloc returns device memory of at least
 * `bytes` bytes (or NULL: the call fails with SAIT_E_NOMEM); free releases
 * it.  NULL allocator => hipMalloc / hipFree. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *p, void *ctx);
    void *ctx;
} sait_allocator;

/* Build options (sait_default_build_opts fills the defaults in brackets). */
typedef struct {
    int ilu_kind;        /* SAIT_ILU0 [default], SAIT_ILUT, SAIT_ILUK (levels of fill, Sec. 4), SAIT_PARILU
                            (fine-grained parallel ILU on the device, on the level-ilu_level pattern) or
                            SAIT_PARIC (its symmetric form) */
    double ilut_tau;     /* ILUT drop tolerance, relative to ||a_i,*||_2 [1e-3] */
    int ilut_fill;       /* ILUT: keep at most this many off-diagonals per row in each of L, U [10] */
    int m;               /* number of Horner passes M <- T~ M + I (Alg. 1-3) [3]; for U see upper_side */
    double tau;          /* SAIT_Thr drop tolerance: keep |M_ij| > tau, 0 <= tau < 1 (Alg. 2) [1e-2] */
    int max_nnz_row;     /* optional cap: keep the diagonal and the max_nnz_row-1 largest |M_ij| per row; 0 = off [0] */
    int pattern_p;       /* < 0: threshold dropping (SAIT_Thr) [-1];  >= 0: SAIT_Pat(p, m) (Alg. 3) */
    int precision;       /* SAIT_F64 [default], SAIT_F32 or SAIT_BF16 storage of M_L, M_U */
    int build_transpose; /* also build A^T, M_L^T, M_U^T for transpose solves / gradients [0] */
    int ilu_level;       /* SAIT_ILUK, SAIT_PARILU, SAIT_PARIC: keep fill of level <= ilu_level (1: level-1 ILU) [1] */
    int upper_side;      /* side of T~ in the passes that build M_U: SAIT_SIDE_RIGHT [default] or SAIT_SIDE_LEFT */
    int parilu_sweeps;   /* SAIT_PARILU, SAIT_PARIC: synchronous sweeps from l_ij = a_ij / a_jj, u_ij = a_ij [3] */
} sait_build_opts;

/* Side of T~ in a Horner pass.  SAIT_SIDE_LEFT: M <- drop(T~ M + I), Alg. 1
 * as printed (always used for M_L).  SAIT_SIDE_RIGHT: M <- drop(M T~ + I).
 * Without dropping both give the same truncated series (the polynomial in
 * T~ commutes with T~); with dropping they differ.  Right-multiplying for
 * the upper factor of a symmetric A (U = D L^T) gives M_U = M_L^T D^-1 and
 * a symmetric positive definite M_U M_L, which the PCG experiments of
 * Sec. 4 need; it reproduces their level-1 ILU iteration counts. */
enum { SAIT_SIDE_LEFT = 0, SAIT_SIDE_RIGHT = 1 };

/* Solve options. */
typedef struct {
    int restart;         /* GMRES restart length k >= 1 [30] */
    int maxit;           /* maximum total inner iterations [10000] */
    double rtol;         /* stop when ||b - A x||_2 <= rtol ||b||_2 (true residual for GMRES,
                            the recursively updated residual for PCG) [1e-8] */
    int flexible;        /* 0: right-preconditioned GMRES; 1: FGMRES (stores M v_j) [0] */
    int method;          /* SAIT_METHOD_GMRES [default] or SAIT_METHOD_PCG */
} sait_solve_opts;

/* Krylov methods of sait_solve.  PCG (Sec. 4 of the paper: the solver of
 * its experiments) is the textbook preconditioned conjugate gradient method
 * for symmetric positive definite A; the SAIT preconditioner M_U M_L is not
 * symmetric (its factors are built by the same left-multiplied recursion),
 * as in the paper's runs.  PCG is single system, one right-hand side, not
 * transposed. */
enum { SAIT_METHOD_GMRES = 0, SAIT_METHOD_PCG = 1 };

/* Preconditioners sait_apply / sait_solve use (sait_set_preconditioner):
 * SAIT: z = M_U (M_L r) [default];
 * JACOBI: s Jacobi sweeps from zero on L, then on U -- the paper's
 *   comparison (Sec. 4), equal to the SAIT series with no dropping and
 *   m = s - 1 (Sec. 2) evaluated without forming it;
 * EXACT: the forward and backward substitutions with L and U
 *   (level-scheduled);
 * NONE: z = r. */
enum { SAIT_PREC_SAIT = 0, SAIT_PREC_JACOBI = 1, SAIT_PREC_EXACT = 2, SAIT_PREC_NONE = 3 };

/* Per-(system, right-hand side) solve report. */
typedef struct {
    int iterations;      /* total inner (Arnoldi) steps */
    int restarts;        /* completed cycles */
    int status;          /* SAIT_OK or SAIT_NOT_CONVERGED */
    double est_relres;   /* last Arnoldi estimate |g_{j+1}| / ||b|| */
    double true_relres;  /* ||b - A x|| / ||b|| at exit */
} sait_solve_info;

void sait_default_build_opts(sait_build_opts *o);
void sait_default_solve_opts(sait_solve_opts *o);

/*
 * Build a preconditioner for A (n x n, host CSR, FP64).
 *   nsys, sys_ptr: A may be a block-diagonal concatenation of nsys
 *     independent systems; sys_ptr (host, nsys+1 entries, sys_ptr[0] = 0,
 *     sys_ptr[nsys] = n, increasing) gives the first row of each.  The
 *     factorisation and SAIT of a block-diagonal matrix are block-diagonal,
 *     so one build serves all systems.  nsys = 1, sys_ptr = NULL otherwise.
 *     No entry of A may couple two systems (SAIT_E_INVALID).
 *   o: options (NULL = defaults); a: allocator (NULL = hipMalloc).
 * Host: A's arrays, sys_ptr, o, a.  The handle copies what it keeps.
 * Steps: host ILU(0) or ILUT (Sec. 3.1), then on the device the Jacobi
 * split T~ = I - D^-1 T (Sec. 2), m passes of W = T~ M + I with dropping
 * (Alg. 2 / 3), the column scaling M <- M D^-1 and the cast to the storage
 * precision, for T = L and T = U.
 * Errors: SAIT_E_INVALID (malformed CSR, tau outside [0,1), m < 0, ...),
 * SAIT_E_ZERO_PIVOT, SAIT_E_NONFINITE, SAIT_E_NOMEM, SAIT_E_DEVICE.
 */
int sait_build(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
               int nsys, const int64_t *sys_ptr, const sait_build_opts *o,
               const sait_allocator *a, void *hip_stream, sait_handle *out);

/*
 * z = M_U (M_L r)            (transpose = 0; Sec. 3.1)
 * z = M_L^T (M_U^T r)        (transpose = 1; needs build_transpose)
 * r, z: device, n x nrhs, leading dimension ld; r and z must not overlap.
 * FP64 factors: FP64 products and sums.  FP32/BF16 factors: r is rounded
 * to binary32, both products accumulate in binary32, the intermediate
 * vector is binary32, z is widened to FP64.
 */
int sait_apply(sait_handle h, const double *r, double *z, int nrhs, int64_t ld, int transpose,
               void *hip_stream);

/*
 * y = A x (transpose = 0) or y = A^T x (transpose = 1, needs build_transpose).
 * x, y: device, n x nrhs with leading dimension ld; must not overlap.
 */
int sait_matvec(sait_handle h, const double *x, double *y, int nrhs, int64_t ld, int transpose,
                void *hip_stream);

/*
 * Solve A x = b (transpose = 0) or A^T x = b (transpose = 1, preconditioned
 * by M_L^T M_U^T) with restarted right-preconditioned GMRES or FGMRES; the
 * Krylov basis, inner products, Hessenberg least squares and the true
 * residual check are FP64 on the device.
 * b: device (n x nrhs, ld); x: device (n x nrhs, ld), holds x0 on entry and
 * the solution on exit.  info: host, nsys*nrhs entries (may be NULL),
 * entry s*nrhs + k for system s, right-hand side k.
 * With nsys > 1 or nrhs > 1 every (system, right-hand side) pair runs its
 * own GMRES in one persistent device launch, converging independently.
 * Returns SAIT_OK when every pair met rtol, SAIT_NOT_CONVERGED otherwise.
 */
int sait_solve(sait_handle h, const double *b, double *x, int nrhs, int64_t ld, int transpose,
               const sait_solve_opts *o, sait_solve_info *info, void *hip_stream);

/*
 * Replace the stored values of A used by sait_matvec, sait_solve and
 * sait_grad_values (and of A^T when built).  val: device, nnz(A) doubles in
 * the CSR order of the matrix given to sait_build (same pattern).  M_L and
 * M_U are not rebuilt: they stay a preconditioner for the new A.
 */
int sait_set_values(sait_handle h, const double *val, void *hip_stream);

/*
 * Gradient of a loss through x = A^-1 b with respect to the stored values
 * of A, given lambda = A^-T (dloss/dx):  grad_val[k] = -lambda[row_k] x[col_k]
 * for the k-th stored entry (row_k, col_k) of A.  (dloss/db = lambda.)
 * lambda, x: device, n entries; grad_val: device, nnz(A) entries.
 */
int sait_grad_values(sait_handle h, const double *lambda, const double *x, double *grad_val,
                     void *hip_stream);

/* Sizes of the stored matrices (any output pointer may be NULL).  The
 * paper's ratio r = nnz(M_T) / nnz(T) (Sec. 3.1) is nnz_ML / nnz_L and
 * nnz_MU / nnz_U. */
int sait_query(sait_handle h, int64_t *n, int64_t *nnz_A, int64_t *nnz_L, int64_t *nnz_U,
               int64_t *nnz_ML, int64_t *nnz_MU);

/*
 * Copy one stored matrix into host buffers sized from sait_query:
 * row_ptr (n+1), col_idx (nnz), val (nnz, FP64; for M_L, M_U the FP64
 * values before the storage cast; any of the three may be NULL).
 * stored (may be NULL): for M_L, M_U the values as stored -- nnz doubles,
 * floats or bfloat16 bit patterns (uint16) per the build precision.
 */
int sait_export(sait_handle h, int which, int32_t *row_ptr, int32_t *col_idx, double *val,
                void *stored);

/*
 * Select the preconditioner of later sait_apply / sait_solve calls on this
 * handle (kind = SAIT_PREC_*; sweeps >= 1 for SAIT_PREC_JACOBI, ignored
 * otherwise).  Builds what the kind needs from the ILU factors on first use
 * (the off-diagonal parts and diagonals for Jacobi, the dependency levels
 * for the exact solves).  Kinds other than SAIT apply to single-system,
 * single right-hand side, non-transposed calls; the others fail with
 * SAIT_E_INVALID while one is selected.  Errors: SAIT_E_INVALID (bad kind,
 * sweeps < 1), SAIT_E_ZERO_PIVOT (zero diagonal in L or U).
 */
int sait_set_preconditioner(sait_handle h, int kind, int sweeps, void *hip_stream);

/* Release the handle and all device memory it owns (NULL is a no-op). */
void sait_destroy(sait_handle h);

/* Thread-local message for the last non-OK status of this thread. */
const char *sait_last_error(void);

/*
 * Apply-kernel shape for M_L and M_U:
 *   SAIT_SHAPE_SELL (-64) / -65: sliced ELL (64-row slices, one row per
 *     lane), 2 / 1 groups of 4 entries per pipeline stage -- the default
 *     when slicing pads at most 1/8 of the entries;
 *   SAIT_SHAPE_STREAM (-16) / -8: LDS-staged CSR with 4088 / 2040-entry
 *     chunks;
 *   a power of two 1..64: wavefront CSR with that many lanes per row.
 * The sliced-ELL and LDS-staged kernels compute each row as the left-to-
 * right sum of separately rounded products in column order.  Blocks of 2-5
 * or 8 right-hand sides with a negative shape use the sliced-ELL block
 * kernel (one row per lane, the same sums per column, so every column equals
 * the one-vector product bit for bit); other block widths use the wavefront
 * kernel (8 lanes per row for a negative shape).  sait_autotune times every
 * candidate on the handle's factors and A (device work on hip_stream,
 * synchronises it) and keeps the fastest; sait_set_apply_lanes overrides
 * (0 = keep); sait_get_apply_lanes reports.
 */
#define SAIT_SHAPE_SELL (-64)
#define SAIT_SHAPE_STREAM (-16)
int sait_autotune(sait_handle h, int nrhs, void *hip_stream);
int sait_set_apply_lanes(sait_handle h, int lanes_L, int lanes_U);
int sait_get_apply_lanes(sait_handle h, int *lanes_L, int *lanes_U);

/*
 * Kernel timing for measurement: runs `reps` applies (transpose = 0,
 * nrhs = 1) on hip_stream, recording HIP events around every SpMV launch,
 * and returns the mean launch durations in milliseconds of the M_L and
 * M_U products and of whole applies.  r, z: device, n entries.
 */
int sait_time_apply(sait_handle h, const double *r, double *z, int reps, void *hip_stream,
                    double *ms_L, double *ms_U, double *ms_apply);

/*
 * Measurement aid: copy `bytes` (a multiple of 16) from src to dst (device,
 * 16-byte aligned, not overlapping) with a plain streaming kernel, on
 * hip_stream.  Its rate is the practically achievable HBM bandwidth the
 * SpMV rates are compared with.
 */
int sait_copy(const void *src, void *dst, size_t bytes, void *hip_stream);

/* LOBPCG options (sait_default_eig_opts fills the defaults in brackets). */
typedef struct {
    int maxit;           /* maximum steps [1000] */
    double tol;          /* stop when every ||A x_j - theta_j x_j||_2 <= tol |theta_j| (||x_j|| = 1) [1e-8] */
} sait_eig_opts;

/* LOBPCG report. */
typedef struct {
    int iterations;      /* Rayleigh-Ritz steps after the one on span(X0) */
    int status;          /* SAIT_OK, SAIT_NOT_CONVERGED or SAIT_BREAKDOWN */
    int p_drops;         /* steps whose Rayleigh-Ritz ran on [X, W] (basis [X, W, P] numerically dependent) */
    double relres;       /* max_j ||A x_j - theta_j x_j|| / |theta_j| at exit */
} sait_eig_info;

void sait_default_eig_opts(sait_eig_opts *o);

/*
 * The k smallest eigenpairs of a symmetric positive definite A by LOBPCG
 * (Knyazev's locally optimal block preconditioned conjugate gradient), the
 * eigensolver of the eigenvalue experiment in Sec. 4.  Every step applies
 * the handle's preconditioner (sait_set_preconditioner; SAIT: W = M_U (M_L R)
 * for the whole n x k residual block, two sparse matrix-matrix products) and
 * A W, forms the Gram matrices of the trial basis [X, W, P] on the device
 * and solves its Rayleigh-Ritz problem (order <= 3k) on the host: if the
 * unit-diagonal scaled S^T S of [X, W, P] has a Cholesky pivot <= 1e-8 that
 * step drops P, and if [X, W] has one <= 1e-14 the solve stops with
 * SAIT_BREAKDOWN.
 * A must be symmetric and the preconditioner symmetric positive definite
 * (SAIT with upper_side = SAIT_SIDE_RIGHT on a symmetric A is); neither is
 * checked.  Single-system handles only.
 * X: device, n x k row-major (ld = k), 1 <= k <= 5, n >= 3k: the start block
 *    (full column rank) on entry, the Ritz vectors (orthonormal) on exit.
 * lambda: host, k Ritz values, ascending.  history: host, maxit + 1 entries
 * or NULL: the residual maximum before every step.  info may be NULL.
 * Returns SAIT_OK, SAIT_NOT_CONVERGED (maxit), SAIT_BREAKDOWN, or an error
 * (SAIT_E_INVALID: bad k, n < 3k, nsys > 1, rank-deficient start block).
 */
int sait_lobpcg(sait_handle h, double *X, int k, double *lambda, double *history, const sait_eig_opts *o,
                sait_eig_info *info, void *hip_stream);

/*
 * Test entry point: one unscaled Horner pass on the device,
 *     M_next = drop(T~ M_prev + I)  (side = SAIT_SIDE_LEFT, Eq. Recursive, Alg. 2)
 *     M_next = drop(M_prev T~ + I)  (side = SAIT_SIDE_RIGHT),  T~ = I - D^-1 T
 * with the threshold rule (tau) and optional cap, for host CSR inputs T
 * (triangular, nonzero diagonal) and M_prev.  Output: host buffers
 * out_row_ptr (n+1), out_col_idx / out_val (capacity entries).  If the
 * result has more than `capacity` entries nothing is written to the
 * column/value buffers, *out_nnz receives the size and SAIT_E_INVALID is
 * returned.
 */
int sait_debug_step(int64_t n, const int32_t *T_row_ptr, const int32_t *T_col_idx, const double *T_val,
                    const int32_t *M_row_ptr, const int32_t *M_col_idx, const double *M_val,
                    double tau, int max_nnz_row, int side, int64_t capacity,
                    int32_t *out_row_ptr, int32_t *out_col_idx, double *out_val, int64_t *out_nnz);

#ifdef __cplusplus
}
#endif

#endif /* SAIT_H */
