/*
 * bnx -- BFGS-preconditioned Inexact Newton eigensolver for one MI355X (gfx950).
 *
 * Computes the p leftmost eigenpairs of a large sparse symmetric positive
 * definite matrix with the DACG-Newton method of Bergamaschi & Martinez,
 * "Efficiently preconditioned Inexact Newton methods for large symmetric
 * eigenvalue problems" (arXiv 1312.1553): each Newton step solves the
 * projected correction equation (eq. (1.2), deflated as in Sec. 3.2)
 *     (I - QQ^T)(A - theta I)(I - QQ^T) s = -(A u - theta u),  s orthogonal to Q,
 * by PCG (Sec. 4.3) preconditioned with an incomplete Cholesky factor updated
 * by the simplified BFGS formula (Sec. 2, eq. (2.2); applied as Alg. 1).
 *
 * Conventions shared by every entry point
 *  - Matrices are CSR with 32-bit indices, both triangles stored, columns
 *    sorted within each row, the diagonal present and positive.
 *  - A block of p vectors of length n is column-major: vector j starts at
 *    element j*n (equivalently a row-major p x n array).
 *  - All work is ordered on the HIP stream given at creation; every call
 *    returns after that stream has been synchronised.
 *  - Errors are returned as bnx_status codes; nothing throws across the ABI.
 *    bnx_last_error() gives the message of the last failing call on a context.
 *  - A context is not thread-safe.  Contexts on one device are independent.
 *  - Precision BNX_FP64 runs every vector and matrix operation in double.
 *    BNX_MIXED runs the correction-equation PCG and DACG (SpMV, triangular
 *    solves, BFGS apply, projection, fused dots) in float with float
 *    accumulation inside a workgroup, and keeps the Rayleigh quotient, the
 *    outer residual, the BFGS scalars s^T r and Gram blocks, and the
 *    re-orthonormalisation of u against converged vectors in double.
 */
#ifndef BNX_H
#define BNX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bnx_ctx bnx_ctx;

typedef enum {
    BNX_OK = 0,
    BNX_NOT_CONVERGED = 1,  /* results written; some pair missed tol within itmax (per-pair relres in stats) */
    BNX_E_ARG = -1,         /* invalid argument, malformed CSR, p or kmax out of range */
    BNX_E_NOT_SPD = -2,     /* non-positive diagonal, or IC(0) breakdown beyond shift_max */
    BNX_E_BREAKDOWN = -3,   /* a device-side wait exceeded its bound, or a non-finite value appeared */
    BNX_E_HIP = -4,         /* a HIP runtime call failed */
    BNX_E_NOMEM = -5,       /* device or host allocation failed */
    BNX_E_STATE = -6        /* call order violated (e.g. solve before factor) */
} bnx_status;

typedef enum { BNX_FP64 = 0, BNX_MIXED = 1 } bnx_precision;

#define BNX_MAX_P 32     /* largest number of eigenpairs per solve */
#define BNX_MAX_KMAX 16  /* largest BFGS window k_max */

/* Solver parameters: Alg. 2 inputs and Table 2 defaults (bnx_default_solve_opts). */
typedef struct {
    int p;              /* number of leftmost eigenpairs (n_eig), 1..BNX_MAX_P            (default 10) */
    double tol;         /* outer test ||A u - theta u|| <= tol * theta (Alg. 2)          (1e-8) */
    int itmax;          /* outer Newton iterations per eigenpair (IMAX)                   (100) */
    double tol_dacg;    /* DACG stop ||A x - q x|| <= tol_dacg * q (Sec. 4.1)            (1e-2) */
    int itmax_dacg;     /* DACG iteration cap                                             (5000) */
    double tol_pcg;     /* PCG exit (i): ||g_l|| <= tol_pcg ||g_0|| (Sec. 4.3)           (1e-2) */
    int itmax_pcg;      /* PCG exit (ii): IMAX_PCG                                        (20) */
    int kmax;           /* BFGS window k_max (Sec. 4.4), 0..BNX_MAX_KMAX                 (5) */
    int precision;      /* bnx_precision                                                  (BNX_FP64) */
    int exit_rule;      /* PCG exit (iv): 0 off, 1 stop when ||g_l|| <= exit_xi * eigres (1) */
    double exit_xi;     /*                                                                (0.1) */
    uint64_t seed;      /* starting block when x0 == NULL: splitmix64 counter generator   (0) */
    const double *x0;   /* optional n x p starting block (host or device per create); NULL = seeded */
    int keep_bfgs;      /* reserved; the backward pass always recomputes its own history  (0) */
    int newton;         /* 1: DACG-Newton (Alg. 2); 0: DACG alone to tol, the DACG rows of
                           Tables 4, 5, 7 and 8; it runs in double in both precision modes
                           (tol is far below the float residual floor); no PCG, outer_its
                           and pcg_its stay 0                                           (1) */
    int bfgs_full;      /* 0: pairs (s_k, r_k) of the simplified update eq. (2.2), y_k ~ -r_k;
                           1: y_k = r_{k+1} - r_k of eq. (2.1), stored as (s_k, r_k - r_{k+1}) and
                           skipped unless s_k^T y_k > 0                                  (0) */
    int jd;             /* 1: Jacobi-Davidson outer iteration (Sec. 6) instead of DACG + Newton:
                           per eigenpair a search space V starts from the start vector (no
                           DACG), Rayleigh-Ritz on V^T A V gives the smallest Ritz pair, the
                           outer test is the one of Alg. 2, V restarts with the jd_mmin smallest
                           Ritz vectors when it holds jd_mmax, and it grows by the correction of
                           the same PCG (same exit tests; the BFGS pairs of the previous
                           correction solves when kmax > 0, the paper's JD when kmax = 0).
                           newton is ignored; dacg_its stay 0; outer_its count corrections  (0) */
    int jd_mmin;        /* (5, Sec. 6); >= 1 */
    int jd_mmax;        /* (10, Sec. 6); jd_mmin < jd_mmax <= 16 */
} bnx_solve_opts;

/* Initial preconditioner P0^ = (L L^T)^{-1} of Sec. 2.  Breakdown policy: on a
 * non-positive pivot the factor is recomputed for A + a*diag(A),
 * a = shift0, 2*shift0, ... <= shift_max. */
typedef struct {
    double shift0;      /* (1e-3) */
    double shift_max;   /* (1.0); shift0 <= 0 disables the retry */
    int ict;            /* 0: IC(0) on the pattern of tril(A), computed on the device (0);
                           1: IC(lfil, tau_ic), the threshold factor the paper uses: at most
                           lfil entries off the diagonal per row of L, entries below tau_ic
                           (relative to the row norm of D^-1/2 A D^-1/2) dropped.  Computed on
                           the host -- its pattern depends on the values row by row -- and
                           installed with its own level sets and block schedules */
    int lfil;           /* (30, Table 2); >= 0 */
    double tau_ic;      /* (1e-2, Table 2); >= 0 */
} bnx_factor_opts;

/* Counters mirroring the columns of the paper's result tables (Tables 4-8). */
typedef struct {
    int dacg_its[BNX_MAX_P];
    int outer_its[BNX_MAX_P];
    int pcg_its[BNX_MAX_P];
    int converged[BNX_MAX_P];
    double relres[BNX_MAX_P];   /* final ||A v - lambda v|| / lambda per pair, in output order */
    long long mvp_dacg;         /* SpMVs with A in DACG */
    long long mvp_newton;       /* SpMVs with A in the Newton phase (1 per PCG iteration + 1 per outer step) */
    int bfgs_skipped;           /* pairs not stored because s^T r >= -1e-12 ||s|| ||r|| */
    int pcg_breakdowns;         /* PCG stops with p^T J p <= 0 */
    int status;                 /* bnx_status of the solve */
    int levels_L, levels_Lt;    /* dependency levels of the triangular systems this solve substituted
                                   (its FP32 solves run level-compressed systems when they apply) */
    double shift_used;          /* IC(0) diagonal shift actually used */
    double t_factor, t_dacg, t_newton;  /* seconds */
    int dacg_restarts;          /* returns from a stalled Newton phase to DACG (see bnx_solve) */
    long long nnz_L;            /* entries of the factor L, diagonal included */
    double fill;                /* fill ratio sigma of Sec. 5: nnz(L) / nnz(tril(A)) */
} bnx_stats;

void bnx_default_solve_opts(bnx_solve_opts *o);
void bnx_default_factor_opts(bnx_factor_opts *o);

/*
 * Create a context for the n x n matrix A (the input matrix of Alg. 2).
 *  rowptr[n+1], col[nnz] (int32), val[nnz] (double): CSR as in the conventions.
 *  device_ptrs: 0 = the three arrays are host memory, 1 = device memory.  The
 *    same flag governs x0/evecs of bnx_solve and the arrays of bnx_backward
 *    and bnx_set_values.
 *  hip_stream: hipStream_t to order all work on (NULL = the null stream).
 * The context copies the arrays; the caller keeps ownership of its memory.
 * Validates: n >= 1, rowptr monotone with rowptr[0] = 0, columns in range and
 * strictly increasing per row, symmetric pattern, diagonal present and > 0.
 * Errors: BNX_E_ARG (malformed), BNX_E_NOT_SPD (diagonal <= 0), BNX_E_NOMEM, BNX_E_HIP.
 * On error *out is NULL.
 */
bnx_status bnx_create_csr(bnx_ctx **out, int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col,
                          const double *val, int device_ptrs, void *hip_stream);

/* Replace the values (same pattern, CSR order).  Invalidates the factor and any
 * stored eigenpairs: call bnx_factor again.  Errors: BNX_E_ARG, BNX_E_NOT_SPD. */
bnx_status bnx_set_values(bnx_ctx *ctx, const double *val);

/*
 * Incomplete Cholesky factor L of the initial preconditioner (Sec. 2,
 * P0^ = (L L^T)^{-1}): IC(0), L L^T = A on the pattern of tril(A), computed on
 * the device level by level; or IC(lfil, tau_ic) (opts->ict = 1).  Also the
 * level sets and LDS block schedules of the L and L^T solves for the pattern of
 * L (rebuilt when the pattern changes).  opts may be NULL (defaults: IC(0)).
 * Errors: BNX_E_ARG (lfil < 0 or tau_ic < 0), BNX_E_NOT_SPD when every shift up
 * to shift_max breaks down.
 */
bnx_status bnx_factor(bnx_ctx *ctx, const bnx_factor_opts *opts);

/* Size of the installed factor (Sec. 5 reports the fill ratio sigma of the
 * initial preconditioner): nnz(L) with the diagonal, sigma = nnz(L)/nnz(tril A),
 * the dependency levels of the factor's L and L^T solves and the diagonal shift used.
 * Any output pointer may be NULL.  Errors: BNX_E_ARG, BNX_E_STATE before bnx_factor. */
bnx_status bnx_factor_info(const bnx_ctx *ctx, long long *nnz_L, double *fill, int *levels_L, int *levels_Lt,
                           double *shift_used);

/*
 * The p leftmost eigenpairs by DACG-Newton (Alg. 2).
 *  evals: host array of p doubles, ascending.
 *  evecs: n x p column-major doubles (host or device per create); column j is
 *         v_{j+1}, unit norm, with its first entry of magnitude above
 *         1e-12 ||v||_inf positive.
 *  stats: may be NULL.
 * When the Newton phase of a pair stalls (a PCG solve takes no step, or the
 * outer residual fails to drop below 0.9x in two consecutive steps) the start
 * was not close enough for Newton (Sec. 4.1): DACG is resumed from the current
 * iterate to 0.005 ||r||/theta (kept within [tol, tol_dacg]), the BFGS history is
 * restarted and Newton continues; at most 5 such returns per pair.
 * Mixed precision (BNX_MIXED) also hands work to double precision where float
 * rounding sets a floor: the float DACG ends when its residual has not dropped
 * by 10 % for 200 iterations within 10x of tol_dacg q, and the double DACG
 * continues from its iterate to tol_dacg; a pair whose outer residual is below
 * 1e-7 theta and has not improved by 10 % for three outer steps is finished by
 * the double DACG to tol.
 * Returns BNX_OK, or BNX_NOT_CONVERGED with results still written.
 * Errors: BNX_E_STATE (no factor), BNX_E_ARG, BNX_E_BREAKDOWN, BNX_E_HIP.
 * The eigenpairs are kept in the context for bnx_backward.
 */
bnx_status bnx_solve(bnx_ctx *ctx, const bnx_solve_opts *opts, double *evals, double *evecs, bnx_stats *stats);

/*
 * Gradient of a scalar loss L(lambda, V) of the last solve's eigenpairs with
 * respect to the CSR values of A (extension; not in the paper).
 *  g_evals: host array of p doubles, dL/dlambda.
 *  g_evecs: n x p column-major dL/dV (host or device per create), or NULL.
 *  g_vals:  nnz doubles (host or device per create), CSR order, written.
 * For each stored entry e = (a,b):
 *  g_vals[e] = sum_i g_evals[i] v_i[a] v_i[b] - 1/2 sum_i (xi_i[a] v_i[b] + v_i[a] xi_i[b]),
 *  xi_i = sum_{j<i} v_j (v_j^T G_i)/(lambda_j - lambda_i) + eta_i, with eta_i
 *  orthogonal to [v_1..v_i] solving the deflated correction-type system
 *  (I - Q_i Q_i^T)(A - lambda_i I)(I - Q_i Q_i^T) eta = (I - Q_i Q_i^T) G_i
 *  (the operator of Sec. 3.2 with theta = lambda_i), by PCG with the IC(0)
 *  preconditioner projected against Q_i, to relative residual tol_adj; in
 *  mixed precision the inner PCG is float and wrapped in double-precision
 *  iterative refinement.
 * Returns BNX_NOT_CONVERGED, with g_vals still written, when an adjoint solve
 * ends with its true projected residual (recomputed in double) above
 * tol_adj ||(I - Q_i Q_i^T) G_i||; bnx_last_error names the pairs.
 * Errors: BNX_E_STATE (no solve since the last factor), BNX_E_ARG.
 */
bnx_status bnx_backward(bnx_ctx *ctx, const double *g_evals, const double *g_evecs, double *g_vals);

/* Tolerance and iteration cap of the adjoint PCG used by bnx_backward (defaults 1e-12, 2000). */
bnx_status bnx_set_adjoint_params(bnx_ctx *ctx, double tol_adj, int itmax_adj);

const char *bnx_last_error(const bnx_ctx *ctx);
void bnx_destroy(bnx_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Step-level entry points.  Each runs one step of the solve path on device
 * vectors (device pointers only, length n unless stated), in the given
 * precision, with the kernels bnx_solve uses.  They require bnx_factor
 * (except bnx_spmv).  Inputs and outputs are double; in BNX_MIXED the inputs
 * are rounded to float, the step runs in float and the result is widened.
 * ------------------------------------------------------------------------- */

/* y = A x: the matrix-vector product (MVP) that is the paper's unit of work. */
bnx_status bnx_spmv(bnx_ctx *ctx, int precision, const double *x, double *y);

/* IC(0) solves for P0^ = (L L^T)^{-1} (Sec. 2): which = 0 solves L x = b,
 * 1 solves L^T x = b, 2 applies both (x = (L L^T)^{-1} b). */
bnx_status bnx_ic_apply(bnx_ctx *ctx, int precision, int which, const double *b, double *x);

/*
 * bnx_ic_apply without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, kernels and results as bnx_ic_apply.
 * The temporaries bnx_ic_apply allocates per call (one n-vector of doubles,
 * or three of floats in BNX_MIXED) live instead in a 12 MiB device array of
 * the library, one copy per device for the life of the process, so
 * n <= 1048576 (larger n: BNX_E_ARG, use bnx_ic_apply).  Every call on a
 * device shares that device's array: calls that overlap in time on one
 * device (different streams or threads) race and must be serialised by the
 * caller.  Nothing in the array needs to start at zero.
 * Errors: as bnx_ic_apply, and BNX_E_ARG when n is too large.
 */
bnx_status bnx_ic_apply_noalloc(bnx_ctx *ctx, int precision, int which, const double *b, double *x);

/*
 * Alg. 1: c = P_k g.  S, R: n x k (column t = pair t, oldest first);
 * alpha_t = s_t^T r_t is formed in double.  Q: n x m projection block (m >= 0,
 * orthonormal columns).  g should be orthogonal to Q (the algorithm omits the
 * right projection).  k <= BNX_MAX_KMAX, m <= BNX_MAX_P + 1.
 */
bnx_status bnx_prec_apply(bnx_ctx *ctx, int precision, int k, const double *S, const double *R, int m,
                          const double *Q, const double *g, double *c);

/*
 * One PCG solve of the correction equation J s = -r (Sec. 4.3) with
 * Q = [Qt, u]: Q is n x m column-major whose last column is the current unit
 * vector u; theta = u^T A u and r = A u - theta u are formed inside.  S, R:
 * n x k stored pairs (oldest first).  Exit tests (i)-(iv) with the given
 * parameters (tau is the outer tolerance used by test (iii)).  Writes s (n),
 * *its (PCG iterations) and *reason (0 cap, 1 tol_pcg, 2 eigen-residual,
 * 3 stagnation rule, 4 p^T J p <= 0).
 */
bnx_status bnx_correction_solve(bnx_ctx *ctx, int precision, int m, const double *Q, int k, const double *S,
                                const double *R, double tol_pcg, int itmax_pcg, double tau, int exit_rule,
                                double exit_xi, double *s, int *its, int *reason);

/*
 * DACG (Sec. 4.1): preconditioned nonlinear CG minimising the Rayleigh
 * quotient on the complement of the m columns of Qt (n x m, orthonormal),
 * from x0, until ||A x - q x|| <= tol q or itmax steps.  Writes the unit
 * vector x and *its.
 */
bnx_status bnx_dacg(bnx_ctx *ctx, int precision, int m, const double *Qt, const double *x0, double tol,
                    int itmax, double *x, int *its);

/* Triangular-solve schedule of the IC(0) solves:
 *  0 = LDS-staged blocks (default): one workgroup per block of consecutive rows
 *      in solve order, the block's solution held in LDS, rows sorted by level
 *      inside the block, dependencies on earlier blocks read from global memory;
 *  1 = one kernel launch per dependency level;
 *  2 = one persistent sync-free kernel over all rows in level order, each row's
 *      completion carried by its solution value in global memory.
 * All three compute the same substitution.  Errors: BNX_E_ARG. */
bnx_status bnx_set_trsv_mode(bnx_ctx *ctx, int mode);

/* Live timing of the hot kernels with HIP events recorded on the context's
 * stream around each launch.  on != 0 clears the counters and starts
 * recording; kernel ids: 0 SpMV fp64, 1 SpMV fp32, 2 forward IC solve fp64,
 * 3 forward fp32, 4 backward IC solve fp64, 5 backward fp32.  bnx_kernel_time
 * synchronises the stream and returns the summed milliseconds and the number
 * of timed launches. */
bnx_status bnx_set_profiling(bnx_ctx *ctx, int on);
bnx_status bnx_kernel_time(bnx_ctx *ctx, int kernel, double *ms_total, long long *launches);

/* Latency probe on the context's device: a chain of `hops` dependent
 * hand-overs (2 <= hops <= 65536), timed with HIP events as one launch.
 * kind 0: between the 16 waves of one workgroup through an LDS flag (the
 * in-block dependency of the LDS-staged triangular solve); kind 1: between
 * workgroups, each polling its predecessor's device-scope flag in global
 * memory (the dependency between two blocks).  The triangular solves are
 * bounded below by levels x the kind-0 figure, which is the latency roofline
 * reported beside the bandwidth one.  *us_per_hop receives microseconds per
 * hand-over.  Waits are bounded: BNX_E_BREAKDOWN if one overflows; BNX_E_ARG
 * on a bad kind or hop count.  The flag buffer (256 KiB) is allocated by the
 * context on first use. */
bnx_status bnx_probe_latency(bnx_ctx *ctx, int kind, int hops, double *us_per_hop);

#ifdef __cplusplus
}
#endif
#endif /* BNX_H */
