/*
 * expm_pfd.h - C ABI of the MI355X (gfx950) library for exp(tA)V, A Hermitian.
 *
 * Method (Hecht, Kaber, Perrin, Plagne, Salomon, "Parallel approximation of the
 * exponential of Hermitian matrices", arXiv 2306.16778):
 *   exp(z) is approximated by R_d(z) = 1/exp_d(-z), exp_d the Taylor polynomial
 *   of even degree d (Sec. 2.2).  Its partial-fraction decomposition
 *   R_d(z) = sum_k a_k/(z + theta_k) over the d roots theta_k of exp_d
 *   (Prop. pro:dec, eqs. yoyo and yoyo2) gives, for Hermitian A,
 *     exp(tA)V ~ R_d(tA)V = sum_k a_k (tA + theta_k I)^{-1} V
 *   (Sec. 3, eqs. equ:ExpoMatRat and equ:expAx): d independent shifted solves.
 *   The roots and residues come in d/2 conjugate pairs and, for Hermitian A,
 *   (tA + conj(theta) I) = (tA + theta I)^H, so one LU factorization serves both
 *   members of a pair (Remark rem:two_time_real_part): the second solve uses the
 *   adjoint of the same factors.
 *
 * Conventions for every entry point
 *   - Complex numbers are interleaved (re, im) doubles: C99 double complex /
 *     std::complex<double> / numpy complex128 layout.
 *   - Matrices are column-major with a leading dimension (LAPACK convention):
 *     element (i, j) of A is A[i + j*lda].
 *   - A is Hermitian and only its LOWER triangle is read (the strictly upper
 *     part is never accessed; the imaginary part of the diagonal is ignored),
 *     or only its UPPER triangle with the option uplo = EXPM_PFD_UPPER.
 *   - Device pointers are HIP device (or managed) memory on the current device.
 *     The caller owns A, V and X; the library never writes A or V and never
 *     keeps a pointer to them after the call returns.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work of a call is enqueued on it and the call returns without
 *     waiting for it, unless the entry point says otherwise.
 *   - Return value: 0 on success, a negative EXPM_PFD_ERR_* code otherwise.
 *     Argument errors are detected before any work is enqueued.
 *   - Spectrum sign is not checked (it would cost an eigensolve).  The error
 *     bounds of the paper (Prop. pro:err, Theorem of Sec. 3) hold for
 *     Spec(tA) in (-inf, 0]; for other spectra the result is still
 *     R_d(tA)V but may be far from exp(tA)V.
 */
#ifndef EXPM_PFD_H
#define EXPM_PFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define EXPM_PFD_OK            0
#define EXPM_PFD_ERR_DEGREE   -1  /* degree odd, < 2 or > EXPM_PFD_MAX_DEGREE */
#define EXPM_PFD_ERR_DIM      -2  /* n < 1, n > EXPM_PFD_MAX_N, m < 1 or m > plan's m_max */
#define EXPM_PFD_ERR_NULL     -3  /* required pointer is NULL */
#define EXPM_PFD_ERR_LD       -4  /* leading dimension smaller than the row count */
#define EXPM_PFD_ERR_OOM      -5  /* device allocation failed */
#define EXPM_PFD_ERR_HIP      -6  /* a HIP runtime call or kernel launch failed */
#define EXPM_PFD_ERR_ARG      -7  /* other invalid argument (precision, t not finite, ...) */
#define EXPM_PFD_ERR_CONST    -8  /* root finding for the constants did not converge */
#define EXPM_PFD_ERR_BUDGET   -9  /* a request can never fit the queue's HBM budget */
#define EXPM_PFD_ERR_TICKET  -10  /* unknown ticket or matrix id */
#define EXPM_PFD_ERR_SYNC    -11  /* a one-launch triangular sweep found its dependency
                                     order broken (a wait hit its cap); results invalid */
#define EXPM_PFD_ERR_SCRATCH -12  /* expm_pfd_apply_noalloc: the problem's workspace does
                                     not fit the fixed scratch array */

#define EXPM_PFD_MAX_DEGREE 64
#define EXPM_PFD_MAX_N      8192

/* ---- options ------------------------------------------------------------ */
#define EXPM_PFD_LOWER 0  /* triangle of A that is read (expm_pfd_opts.uplo) */
#define EXPM_PFD_UPPER 1
#define EXPM_PFD_FP64  0  /* LU, solves and accumulation in complex FP64 */
#define EXPM_PFD_MIXED 1  /* complex FP32 LU and solves on the matrix cores, FP64
                             iterative refinement of every shifted solve and FP64
                             residue-weighted accumulation */

typedef struct expm_pfd_opts {
  int precision;   /* EXPM_PFD_FP64 (default) or EXPM_PFD_MIXED */
  int ir_max_iter; /* MIXED: most refinement sweeps per solve; 0 selects the default
                      (2, or 3 for degree >= 32), a negative value none.  With the
                      convergence test (ir_tol >= 0) fewer run when every solve of
                      a launch has converged. */
  int ir_extended; /* MIXED: how many of the last sweeps accumulate the residual
                      V - (tA + theta I) X in double-double (error-free products and
                      sums; needed when the shifted matrices are ill conditioned,
                      e.g. degree 32 with spectra of width 4e4).  0: automatic (one
                      such sweep for degree >= 32, none below); < 0: none */
  int real_data;   /* nonzero: A and V are real (imaginary parts are not read).
                      Then the conjugate pole's solution is the conjugate of the
                      primal one (Remark rem:two_time_real_part): solves and
                      refinement run for one pole per pair only. */
  int graph;       /* nonzero: expm_pfd_apply and expm_pfd_batch_apply capture their
                      launches into a HIP graph on first use (per plan and
                      right-hand-side width, per batch schedule) and replay it
                      afterwards.  The problem descriptors (A, V, X, t) are
                      uploaded ahead of each replay, so new pointers and times
                      need no recapture.  Launches run directly while tracing is on. */
  int autotune;    /* nonzero: at plan creation, time each LU trailing-update tile
                      shape on the plan's own workspace and keep the fastest
                      (cached per padded order, precision and batch); a batch
                      plan with several groups also times, at its first apply,
                      running the groups one after another against 2 and 4
                      concurrent branches.  Every candidate computes the same
                      bits, so tuning changes speed only. */
  int lu_tile;     /* 0: built-in (64 x 64) or autotuned; k = 1..3 forces tile shape
                      k-1 of {64x64, 128x64, 64x128} (complex elements of C per
                      workgroup).  Other values: EXPM_PFD_ERR_ARG. */
  int uplo;        /* EXPM_PFD_LOWER (0, default): the lower triangle of A is read;
                      EXPM_PFD_UPPER (1): the upper one.  The other triangle is
                      never accessed.  Other values: EXPM_PFD_ERR_ARG. */
  double shift;    /* c of the shifting method (Remark rem:shift): the library
                      computes e^c R_d(tA - cI) V, so spectra of tA up to c are
                      covered by the negative-spectrum error bound of the
                      Theorem of Sec. 3 (relative error controlled when c bounds
                      the spectrum).  Default 0; e^c must be finite (c < 709),
                      otherwise EXPM_PFD_ERR_ARG.  With shift_scale_t, c is in
                      units of A instead. */
  double ir_tol;   /* MIXED: convergence test of the refinement.  After every sweep
                      a solve (one pole of one problem, all its columns) has
                      converged when its largest correction is at most ir_tol
                      times its largest solution entry (max norms); once all
                      solves of a launch have converged the remaining sweeps are
                      skipped on the device (no host round trip; graphs replay
                      it).  A problem with a solve that has not converged after
                      the last sweep gets status 1: the batched entry point
                      expm_pfd_apply_batched and the queue then solve it again on
                      the FP64 path; expm_pfd_batch_apply reports it in `info`,
                      expm_pfd_apply through expm_pfd_plan_check.  0 selects the
                      default 1e-10; a negative value turns the test off (fixed
                      sweep count, status 1 never set).  NaN: EXPM_PFD_ERR_ARG. */
  int shift_scale_t; /* nonzero: `shift` is c in units of A, and problem i is
                      shifted by t_i * c in units of t_i A (one c bounding the
                      spectra of all A_i serves problems of different t_i in a
                      batch or queue): e^(t_i c) R_d(t_i (A_i - cI)) V_i.
                      e^(t_i c) must be finite for every apply (otherwise
                      EXPM_PFD_ERR_ARG from the apply or submit). */
  int tridiag_reuse; /* queue only: a registered matrix named by this many
                      requests is reduced once to tridiagonal form (the route of
                      expm_pfd_tridiag_*), and its later requests are served by
                      that route (FP64, O(n^2) per request).  0: never. */
} expm_pfd_opts;

/* ---- constants (host only) ---------------------------------------------- */
/*
 * expm_pfd_constants: the poles and residues of R_d, one member per conjugate pair.
 *   theta_k: the roots of exp_d (Sec. 2.1), found in binary128 by simultaneous
 *   (Aberth) iteration; a_k = -d!/prod_{j!=k}(theta_k - theta_j) (eq. yoyo2),
 *   evaluated in binary128 and rounded to FP64 (the paper's preferred formula,
 *   Sec. 4).  The member with Im(theta) > 0 is kept; pairs are ordered by
 *   ascending Re(theta).
 *   degree  even, 2 <= degree <= EXPM_PFD_MAX_DEGREE.
 *   theta   host array of degree/2 complex numbers (degree doubles), written.
 *   a       host array of degree/2 complex numbers (degree doubles), written.
 *   Pure host computation; no device is touched.  Thread-safe.
 */
int expm_pfd_constants(int degree, double* theta, double* a);

/* ---- single problem ----------------------------------------------------- */
typedef struct expm_pfd_plan_s* expm_pfd_plan_t;

/*
 * expm_pfd_plan: prepare exp(tA)V ~ R_d(tA)V for matrices of order n
 * (Sec. 3, eq. equ:ExpoMatRat for V = I and eq. equ:expAx otherwise).
 *   out     receives the plan handle.
 *   n       matrix order, 1 <= n <= EXPM_PFD_MAX_N.
 *   degree  even degree d of the approximation (number of poles).
 *   t       the time factor: the method is applied to the matrix tA (finite).
 *   m_max   widest right-hand side block the plan will accept; 0 means n and
 *           also allows V = NULL (V = I, the full matrix R_d(tA)).
 *   opts    NULL for defaults.
 * Allocates all device workspace (degree/2 shifted matrices plus solution
 * blocks) on the current device; nothing is allocated by expm_pfd_apply.
 * Returns EXPM_PFD_ERR_OOM if the workspace does not fit.
 */
int expm_pfd_plan(expm_pfd_plan_t* out, int64_t n, int degree, double t, int64_t m_max,
                  const expm_pfd_opts* opts);

/* Device bytes a plan with these arguments allocates (for admission control). */
int expm_pfd_workspace_bytes(int64_t n, int degree, int64_t m_max, const expm_pfd_opts* opts,
                             size_t* bytes);

/*
 * expm_pfd_apply: X = R_d(tA) V.
 *   A    device, n x n complex, column-major, leading dimension lda >= n;
 *        Hermitian, lower triangle read.
 *   V    device, n x m complex, column-major, ldv >= n; NULL means V = I
 *        (then m must equal n and the plan must have m_max = 0 or n).
 *   X    device, n x m complex, column-major, ldx >= n; written.  Must not
 *        overlap A or V.  For V = NULL, X is Hermitian.
 *   stream  hipStream_t as void*.
 * The plan's workspace is reused: concurrent applies of one plan race.
 */
int expm_pfd_apply(expm_pfd_plan_t plan, const void* A, int64_t lda, const void* V, int64_t ldv,
                   int64_t m, void* X, int64_t ldx, void* stream);

/* Release the plan and its device memory (synchronizes the device first). */
int expm_pfd_destroy(expm_pfd_plan_t plan);

/*
 * expm_pfd_plan_check: synchronizes the device, then reports whether every
 * triangular sweep run with this plan so far kept its dependency order.
 * Thin right-hand sides (at most 64 columns) are solved by one launch per
 * sweep whose workgroups wait on each other's results; each wait is capped,
 * and a capped wait marks the plan.  Returns 0, or EXPM_PFD_ERR_SYNC once a
 * wait has hit its cap (the plan's results since then are invalid and the
 * plan should be destroyed), or EXPM_PFD_ERR_HIP.  For a MIXED plan with the
 * refinement convergence test on (opts.ir_tol >= 0) it returns 1 when a solve
 * of the last apply had not converged after its last sweep (X then holds the
 * refined, unconverged result; apply again with precision FP64).
 */
int expm_pfd_plan_check(expm_pfd_plan_t plan);

/* ---- single problem without device allocation ---------------------------- */
/* Size of the library's fixed device scratch array (one per GPU the library runs
 * on, held until the process ends). */
#define EXPM_PFD_NOALLOC_BYTES ((size_t)128 << 20)

/*
 * expm_pfd_apply_noalloc: X = R_d(tA)V, the same computation (same kernels, same
 * bits) as expm_pfd_plan(n, degree, t, m, opts) + expm_pfd_apply +
 * expm_pfd_destroy, for callers that cannot allocate device memory: code under
 * HIP stream capture, tight serving loops, harnesses that forbid hipMalloc.
 * No hipMalloc, hipFree or other allocating call is made (host memory only for
 * the per-degree constants, computed on the first call of each degree).  The
 * whole workspace is carved from the library's fixed device array of
 * EXPM_PFD_NOALLOC_BYTES bytes; its device address is looked up once per device,
 * on the first call with that device current.  Every launch is a kernel (no
 * memset or copy nodes), so the call may be captured into a graph.
 *   n, degree, t   as for expm_pfd_plan.
 *   A, lda, V, ldv, m, X, ldx   as for expm_pfd_apply (V = NULL: V = I, m = n).
 *   opts    NULL for defaults; precision, ir_sweeps, ir_extended, real_data,
 *           lu_tile, uplo and shift apply; graph and autotune are ignored.
 *   info    device int or NULL: written when the work completes with 0, 2 (X
 *           holds a non-finite value), or EXPM_PFD_ERR_SYNC (a triangular
 *           sweep lost its dependency order; X is invalid).
 *   stream  hipStream_t as void*; the call returns without waiting.
 * Limits: a problem whose workspace (expm_pfd_workspace_bytes with m_max = m,
 * plus at most 13 x 255 bytes of alignment) exceeds EXPM_PFD_NOALLOC_BYTES is
 * rejected with EXPM_PFD_ERR_SCRATCH before any device work.  Largest orders
 * that fit at degree 16: m <= 16, FP64 n <= 896, mixed n <= 1088; V = I, FP64
 * n <= 640, mixed n <= 512.
 * Every call on one GPU uses the same array, which keeps the last call's
 * contents (the parts that must start at zero are cleared by each call): calls
 * that overlap on one GPU (two streams, two host threads) race and give wrong
 * results; calls ordered on one stream are safe.
 */
int expm_pfd_apply_noalloc(int64_t n, int degree, double t, const void* A, int64_t lda, const void* V,
                           int64_t ldv, int64_t m, void* X, int64_t ldx, const expm_pfd_opts* opts, int* info,
                           void* stream);

/* ---- batched ------------------------------------------------------------ */
/*
 * expm_pfd_apply_batched: X_i = R_d(t_i A_i) V_i for count independent problems
 * of possibly different orders (Sec. 3, eq. equ:expAx per problem).
 *   count   number of problems (>= 1).
 *   n, t, lda, m, ldv, ldx   host arrays of length count.
 *   A, V, X host arrays of count device pointers (V[i] may be NULL: V_i = I,
 *           then m[i] must be n[i]).
 *   degree, opts  shared by all problems.
 * Problems are grouped by padded order; every group runs as one sequence of
 * launches whose grids cover all poles of all its problems.  One-shot form of
 * expm_pfd_batch_plan + expm_pfd_batch_apply + expm_pfd_batch_check +
 * expm_pfd_batch_destroy: device workspace is allocated inside the call and
 * released before it returns; the call synchronizes before returning.
 *   info    host array of count ints, or NULL: per-problem status on return,
 *           0 = result finite, 2 = X_i holds a non-finite value (non-finite
 *           input; a zero pivot cannot occur for finite Hermitian A, since
 *           |lambda + theta_k| >= |Im theta_k| > 0), 1 = (MIXED) a shifted
 *           solve's refinement missed opts.ir_tol, so X_i was computed again
 *           on the FP64 path (Sec. 4, Prop. prop:digit: the working precision
 *           must match the accuracy sought).
 */
int expm_pfd_apply_batched(int count, const int64_t* n, const double* t, int degree,
                           const void* const* A, const int64_t* lda, const void* const* V,
                           const int64_t* ldv, const int64_t* m, void* const* X, const int64_t* ldx,
                           const expm_pfd_opts* opts, void* stream, int* info);

/*
 * Batch plans: the workspace of a fixed set of problem shapes, allocated once
 * and reused by every apply, which then allocates nothing and does not wait
 * for the device.
 */
typedef struct expm_pfd_batch_s* expm_pfd_batch_t;

/*
 * expm_pfd_batch_plan: prepare X_i = R_d(t_i A_i) V_i for count problems of
 * orders n[i] (Sec. 3, eq. equ:expAx per problem; all poles of all problems are
 * independent solves).
 *   n, m    host arrays of length count: order of A_i (1..EXPM_PFD_MAX_N) and
 *           columns of V_i (1..n[i]), or m[i] = 0 for V_i = I (the full
 *           R_d(t_i A_i)).
 *   degree, opts  shared by all problems (opts: see expm_pfd_opts; graph and
 *           autotune apply to the whole batch).
 * Problems with the same padded order (a multiple of 64) and right-hand-side
 * kind form one group; every launch of a group covers all poles of all its
 * problems.  Allocates each group's workspace on the current device.
 * Errors: EXPM_PFD_ERR_DIM, _DEGREE, _ARG, _NULL, _OOM, _HIP.
 */
int expm_pfd_batch_plan(expm_pfd_batch_t* out, int count, const int64_t* n, const int64_t* m, int degree,
                        const expm_pfd_opts* opts);

/*
 * expm_pfd_batch_apply: X_i = R_d(t_i A_i) V_i for every problem of the plan.
 *   t, lda, ldv, ldx  host arrays of length count (t finite; lda, ldx >= n[i];
 *           ldv >= n[i] where V[i] is given).
 *   A, V, X host arrays of count device pointers, layouts as in expm_pfd_apply.
 *           V[i] must be NULL exactly where the plan has m[i] = 0.
 *   info    device array of count ints, or NULL: per-problem status written
 *           when the work completes (0 = finite result, 2 = non-finite values
 *           in X_i, 1 = (MIXED) refinement missed opts.ir_tol; X_i holds the
 *           refined result and no FP64 solve is made here).
 * Asynchronous on `stream`: uploads the problem descriptors (from pinned
 * staging the plan owns; it waits only for the previous apply's upload) and
 * enqueues or replays the groups.  Concurrent applies of one batch plan race.
 * Sweep faults are reported by expm_pfd_batch_check.
 */
int expm_pfd_batch_apply(expm_pfd_batch_t b, const double* t, const void* const* A, const int64_t* lda,
                         const void* const* V, const int64_t* ldv, void* const* X, const int64_t* ldx,
                         int* info, void* stream);

/* Synchronizes the device; then 0, or EXPM_PFD_ERR_SYNC if a triangular sweep of
 * any group lost its dependency order (see expm_pfd_plan_check), or _HIP. */
int expm_pfd_batch_check(expm_pfd_batch_t b);

/* Shape of a batch plan: its number of groups, the schedule in use (number of
 * concurrent group branches; 0 before the first apply) and the largest LU tile
 * index among the groups.  Any output pointer may be NULL. */
int expm_pfd_batch_info(expm_pfd_batch_t b, int* groups, int* schedule, int* lu_tile_max);

/* Release a batch plan (synchronizes the device first). */
int expm_pfd_batch_destroy(expm_pfd_batch_t b);

/* ---- tridiagonal route: one reduction of A, many t ------------------------ */
/*
 * The partial fractions combined with a reduction of A to tridiagonal form
 * (the paper's Sec. 1 names such reductions as a complement of the method):
 * A = Q T Q^H once, T real symmetric tridiagonal and Q unitary, then for each t
 *   R_d(tA) V = Q [ sum_k a_k (tT + theta_k I)^{-1} ] Q^H V      (eq. equ:expAx),
 * with one tridiagonal solve (partial pivoting) per pole pair and column for
 * Q^H V and one for its conjugate (T real: (tT + conj(theta) I)^{-1} b =
 * conj((tT + theta I)^{-1} conj(b))), a residue-weighted FP64 sum and one
 * product with Q.  The reduction costs O(n^3) once per matrix; every later t
 * costs O(n^2 m) (two products with the explicit Q) plus O(n d m).  Everything
 * runs in FP64 (opts.precision is accepted and does not change the route).
 */
typedef struct expm_pfd_tri_s* expm_pfd_tri_t;

/* Plan for matrices of order n (1..EXPM_PFD_MAX_N), degree d, right-hand sides
 * of at most m_max columns (1..min(64, n)).  opts: uplo, shift and shift_scale_t
 * apply (see expm_pfd_opts); others are ignored.  Allocates about 2 n^2 x 16
 * bytes (the matrix being reduced and Q) plus O(n d m_max) on the current device.
 * Errors: EXPM_PFD_ERR_DEGREE, _DIM, _ARG, _NULL, _OOM, _HIP. */
int expm_pfd_tridiag_plan(expm_pfd_tri_t* out, int64_t n, int degree, int64_t m_max, const expm_pfd_opts* opts);

/* A = Q T Q^H for the n x n column-major device matrix A (lower triangle read, or
 * the upper one with opts.uplo); A is not kept.  Asynchronous on `stream`; the
 * plan's previous reduction is replaced.  Errors: _NULL, _LD, _HIP. */
int expm_pfd_tridiag_factor(expm_pfd_tri_t tri, const void* A, int64_t lda, void* stream);

/* X = R_d(tA) V with the reduction of the last expm_pfd_tridiag_factor (same
 * stream or ordered after it).  V: device n x m column-major (ldv >= n),
 * 1 <= m <= m_max; X: device n x m (ldx >= n).  Asynchronous on `stream`; calls
 * on one plan must not overlap.  Errors: _NULL, _ARG (not factored, t not
 * finite, e^shift overflows), _DIM, _LD, _HIP. */
int expm_pfd_tridiag_apply(expm_pfd_tri_t tri, double t, const void* V, int64_t ldv, int64_t m, void* X,
                           int64_t ldx, void* stream);

/* Host copies of T: d[0..n) (diagonal) and e[0..n-1) (subdiagonal).  Waits for
 * the device.  Errors: _NULL, _ARG (not factored), _HIP. */
int expm_pfd_tridiag_diagonals(expm_pfd_tri_t tri, double* d, double* e);

/* Release the plan (synchronizes the device first). */
int expm_pfd_tridiag_destroy(expm_pfd_tri_t tri);

/* ---- banded route: Hermitian band matrices -------------------------------- */
/*
 * R_d(tA) V for Hermitian A with kd sub- and superdiagonals: the finite-difference
 * Laplacians of the paper's experiments (Sec. 5: B = 1D, kd = 1; C = 2D on an
 * s x s grid numbered row by row, kd = s) and any other band matrix.  For each
 * pole theta_k the band matrix tA + theta_k I is factored by Gaussian elimination
 * with partial pivoting inside the band (the upper factor gains kd diagonals of
 * fill), the elimination applied to V as it goes, followed by a banded back
 * substitution; then Y = sum_k a_k X_k in FP64 in a fixed pole order
 * (eq. equ:expAx).  Each conjugate pole is solved on its own (tA + conj(theta) I
 * is a different band matrix), or, with opts.real_data, not at all: the result is
 * 2 Re(sum over one member per pair) (Remark rem:two_time_real_part).  Work per
 * pole O(n kd (kd + m)); everything in FP64 (opts.precision is accepted and does
 * not change the route).
 *
 * Band storage (LAPACK's layout), column-major AB with ldab >= kd + 1:
 *   lower (default):  AB[(i - j) + j*ldab] = A(i, j),  j <= i <= min(n-1, j+kd);
 *   upper (opts.uplo): AB[(kd + i - j) + j*ldab] = A(i, j),  max(0, j-kd) <= i <= j.
 * The other triangle is its conjugate and the imaginary part of the diagonal is
 * not read.
 */
typedef struct expm_pfd_band_s* expm_pfd_band_t;

#define EXPM_PFD_BAND_MAX_KD 63       /* widest band (one row per lane of a wave) */
#define EXPM_PFD_BAND_MAX_N  16777216 /* largest order of the banded route */

/* Plan for band matrices of order n (1..EXPM_PFD_BAND_MAX_N) with kd
 * (0..EXPM_PFD_BAND_MAX_KD) sub- and superdiagonals, degree d, right-hand sides of
 * at most m_max columns (1..64).  opts: uplo, real_data, shift and shift_scale_t
 * apply; others are ignored.  Allocates (d, or d/2 with real_data) x n x
 * (2 min(kd, n-1) + 1 + m_max) x 16 bytes on the current device.
 * Errors: EXPM_PFD_ERR_DEGREE, _DIM, _ARG, _NULL, _OOM, _HIP. */
int expm_pfd_band_plan(expm_pfd_band_t* out, int64_t n, int64_t kd, int degree, int64_t m_max,
                       const expm_pfd_opts* opts);

/* X = R_d(tA) V (with the shift: e^c R_d(tA - cI) V).  AB: device band storage
 * as above (ldab >= kd + 1); V: device n x m column-major (ldv >= n),
 * 1 <= m <= m_max; X: device n x m (ldx >= n), not overlapping AB or V.
 * Asynchronous on `stream`; calls on one plan must not overlap.
 * Errors: _NULL, _ARG (t not finite, e^shift overflows), _DIM, _LD, _HIP. */
int expm_pfd_band_apply(expm_pfd_band_t plan, double t, const void* AB, int64_t ldab, const void* V,
                        int64_t ldv, int64_t m, void* X, int64_t ldx, void* stream);

/* Release the plan (synchronizes the device first). */
int expm_pfd_band_destroy(expm_pfd_band_t plan);

/* ---- degree adapted to the arithmetic ------------------------------------ */
/*
 * Sec. 4 (Fig. fig:maple, Prop. prop:digit): with D significant digits the
 * evaluated partial fractions differ from e^x on x <= 0 by at most
 * M_1(d) + M_2(d, D), with M_1(d) = 2^-d (Prop. pro:err) and
 * M_2(d, D) = (C_1(D) + C_2(d, D)) sum_k |a_k| (eq. eq:upper_bound).  M_1 falls
 * and M_2 grows with d, so the precision fixes a best degree.
 *
 * *degree: the smallest even d in [2, EXPM_PFD_MAX_DEGREE] whose bound is at most
 * tol (return 0), or, if none is, the even d with the smallest bound (return 1).
 * *bound (may be NULL): that d's bound.  digits: D, 4..34 (16 for FP64 results,
 * which both precisions deliver).  Host only, no device work.
 * Errors: _NULL, _ARG (digits out of range, tol NaN), _CONST. */
int expm_pfd_choose_degree(double tol, int digits, int* degree, double* bound);

/* ---- tracing ------------------------------------------------------------ */
/* Kernel classes timed by the tracer (one HIP event pair per launch, recorded on
 * the stream the kernel is launched on). */
#define EXPM_PFD_K_FORM        0  /* shifted-matrix formation */
#define EXPM_PFD_K_PANEL       1  /* register-resident panel factorization */
#define EXPM_PFD_K_LU_GEMM     2  /* LU updates C -= L21 U12 inside the outer panels and the narrow
                                      ones a step applies early (64x64 complex tiles) */
#define EXPM_PFD_K_LU_TRSM     3  /* LU U12 = L11^{-1} A12 as a product with the block inverse */
#define EXPM_PFD_K_MOVES       4  /* row moves (left columns, right-hand sides) */
#define EXPM_PFD_K_SOLVE_TRSM  5  /* (unused; diagonal blocks are applied inside the sweeps) */
#define EXPM_PFD_K_SOLVE_GEMM  6  /* triangular sweeps: one-launch chains or block products */
#define EXPM_PFD_K_ACCUM       7  /* residue-weighted accumulation */
#define EXPM_PFD_K_IR_GEMM     8  /* refinement residual product (FP64) */
#define EXPM_PFD_K_ELEMENTWISE 9  /* staging, conversions, shift, correction */
#define EXPM_PFD_K_LU_TRAIL   10  /* LU trailing updates A22 -= L21 U12 over the whole trailing
                                     matrix (two steps at a time: K = 128) */
#define EXPM_PFD_K_COUNT      11

/*
 * expm_pfd_trace: time every later launch of the kernel classes whose bit is set
 * in class_mask (bit EXPM_PFD_K_x; 0 disables tracing), discarding what was
 * recorded before.  Host-side process-wide state; not thread-safe.  Adds two
 * event records per timed launch.
 */
int expm_pfd_trace(int class_mask);

/*
 * expm_pfd_trace_summary: totals for one kernel class over the launches
 * recorded since tracing was enabled.  Waits for the recorded events.
 *   ms        summed kernel durations (milliseconds)
 *   launches  number of launches
 *   flops     algorithmic floating-point operations of those launches
 *             (complex multiply-add = 8)
 *   bytes     algorithmic HBM bytes (reads of the operands once, writes once)
 * Any output pointer may be NULL.
 */
int expm_pfd_trace_summary(int kernel_class, double* ms, int64_t* launches, double* flops, double* bytes);

/* ---- queued serving --------------------------------------------------------- */
/*
 * A queue serves exp(t_i A_i) v_i requests as they arrive (continuous batching;
 * Sec. 3, eq. equ:expAx per request).  A scheduler thread owned by the queue
 * repeatedly takes the oldest pending request and the later ones whose orders
 * are compatible with it (the padded orders of one group stay within a factor 2
 * of each other in LU work, lo^3 >= hi^3 / 2, or all are at most 512), as many
 * as fit the HBM budget (at most max_group), and launches the group as one
 * batched evaluation -- every pole of every request in each launch, the
 * group's order the largest of its requests' (smaller ones are padded with the
 * identity) -- on a free worker stream, so groups overlap on the device and
 * requests arriving meanwhile join the next group.  Completion is observed by
 * one thread per worker stream sleeping on the stream's event (no polling).
 * Latency is host time from submit to that observation.  All requests of a
 * queue share degree and options.
 *
 * Matrices are either registered (copied into queue memory, counted against the
 * budget, reusable by any number of requests with new t and v, released by
 * expm_pfd_unregister_matrix) or passed with each request and read in place.
 * A MIXED request whose refinement misses opts.ir_tol is solved again on the
 * FP64 path before its ticket completes (status 1).
 * Entry points are thread-safe with respect to each other.
 */
typedef struct expm_pfd_queue_s* expm_pfd_queue_t;

typedef struct expm_pfd_queue_stats {
  int64_t submitted;
  int64_t tridiag_requests;  /* requests served by the tridiagonal route (opts.tridiag_reuse) */
  int64_t reductions;        /* matrices reduced to tridiagonal form */
  int64_t completed;         /* requests whose result is in X */
  int64_t failed;            /* requests failed (budget or sweep fault); not in `completed` */
  int64_t fallbacks;         /* requests solved again on the FP64 path (status 1) */
  int64_t groups;            /* batched evaluations launched */
  double p50_ms, p99_ms;     /* latency percentiles of completed requests */
  double mean_ms, max_ms;
  double solves_per_s;       /* completed / (last completion - first submit) */
  double mean_group_size;
  int64_t padded_up;         /* requests evaluated in a group of a larger padded order */
  size_t peak_bytes;         /* peak of registered matrices + in-flight and cached workspace */
  int64_t registered;        /* matrices registered and not yet freed */
  size_t registered_bytes;
} expm_pfd_queue_stats;

/*
 * hbm_budget  device bytes the queue may hold: registered matrices, in-flight
 *             workspace and idle cached workspace (released when needed).  A
 *             request whose workspace alone cannot fit next to the registered
 *             matrices is rejected by expm_pfd_submit with EXPM_PFD_ERR_BUDGET.
 * degree      even degree used for every request.
 * opts        precision, refinement, real-data, uplo and shift options of every
 *             request (graph, autotune: ignored); NULL for defaults.
 * max_group   most requests evaluated together (<= 0: 64).
 * streams     worker streams (<= 0: 3).
 */
int expm_pfd_queue_create(expm_pfd_queue_t* q, size_t hbm_budget, int degree, const expm_pfd_opts* opts,
                          int max_group, int streams);

/*
 * Register the n x n column-major device matrix A (lower triangle read, or the
 * upper one with opts.uplo) with the queue: a copy in queue memory (from the
 * device's stream-ordered pool), made on `stream` after the caller's work
 * already enqueued there, so A may be reused once that stream passes the copy.
 * *mat_id identifies it in expm_pfd_submit.  Returns at once.
 * EXPM_PFD_ERR_BUDGET: the copy does not fit next to the registered matrices
 * and the work in flight (unregister matrices no longer needed).
 */
int expm_pfd_register_matrix(expm_pfd_queue_t q, const void* A, int64_t n, int64_t lda, void* stream,
                             int64_t* mat_id);

/* Release a registered matrix: no new request may name it; its memory returns to
 * the budget once the requests already submitted for it have completed.
 * EXPM_PFD_ERR_TICKET for an unknown or already released id. */
int expm_pfd_unregister_matrix(expm_pfd_queue_t q, int64_t mat_id);

/*
 * Enqueue X = R_d(t A) V.
 *   mat_id, A  A == NULL: the registered matrix mat_id (n and lda are not
 *           read); otherwise (mat_id ignored) the caller's n x n device matrix
 *           A with leading dimension lda, read in place: it must stay valid and
 *           unchanged until the ticket completes.
 *   V       device n x m column-major (ldv >= n), 1 <= m <= 16;
 *   X       device n x m (ldx >= n), written when the ticket completes.  V and X
 *           must stay valid and V unchanged until then.
 *   stream  the caller's stream whose work already enqueued writes A and V
 *           (an event recorded on it orders the request after that work);
 *           NULL: the null stream.
 * Returns at once with *ticket.  EXPM_PFD_ERR_ARG: t not finite or e^(shift)
 * overflows; EXPM_PFD_ERR_TICKET: unknown or released mat_id.
 */
int expm_pfd_submit(expm_pfd_queue_t q, int64_t mat_id, const void* A, int64_t n, int64_t lda, double t,
                    const void* V, int64_t m, int64_t ldv, void* X, int64_t ldx, void* stream, uint64_t* ticket);

/* *done = 1 once the ticket's result is in X (0 otherwise); *info (may be NULL)
 * its status then: 0, 1 (MIXED: refinement missed opts.ir_tol, X solved again
 * on the FP64 path) or 2 (non-finite values in X).  Returns
 * EXPM_PFD_ERR_BUDGET for a request failed because it could no longer fit the
 * budget (matrices registered after it was submitted filled it) and
 * EXPM_PFD_ERR_SYNC for one whose triangular sweeps lost their order. */
int expm_pfd_poll(expm_pfd_queue_t q, uint64_t ticket, int* done, int* info);
/* Block until the ticket completes (same return codes and *info as expm_pfd_poll). */
int expm_pfd_wait(expm_pfd_queue_t q, uint64_t ticket, int* info);
/* Block until every submitted request has completed or failed; returns 0, or
 * the error code of a failed request (EXPM_PFD_ERR_BUDGET, EXPM_PFD_ERR_SYNC). */
int expm_pfd_queue_drain(expm_pfd_queue_t q);
int expm_pfd_queue_stats_get(expm_pfd_queue_t q, expm_pfd_queue_stats* out);
/* Drain, stop the scheduler and free everything the queue owns. */
int expm_pfd_queue_destroy(expm_pfd_queue_t q);

/* Human-readable text for a return code (static storage). */
const char* expm_pfd_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* EXPM_PFD_H */
