/*
 * skfab.h - sketched Krylov approximation of f(A) b on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libskfab.so.  The library evaluates the sketched FOM and sketched
 * GMRES approximants of Guettel & Schweitzer, "Randomized sketching for Krylov
 * approximations of large-scale matrix functions" (arXiv 2208.11447):
 *
 *   Algorithm 1 (Section 2.2)  sketched FOM, closed form (sFOM''') of Section 2.1
 *   Algorithm 2 (Section 4)    sketched GMRES with k-truncated Arnoldi and
 *                              adaptive quadrature (Section 4.1)
 *
 * Problem statement (both algorithms' inputs): a sparse matrix A (N x N), a
 * vector b, a function f, the Krylov dimension m, the truncation length k and
 * the sketch size s with m < s << N.  Output: an approximation of f(A) b.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Memory: every pointer to N-sized data (CSR arrays, b, x, workspace, test
 *    hook outputs) is a DEVICE pointer on the context's device, allocated and
 *    owned by the caller.  Structs passed by pointer (skfab_csr, skfab_params,
 *    skfab_info) are HOST memory.  The library never allocates or frees device
 *    memory in these calls; all scratch lives in the caller's workspace.
 *  - Streams: work is enqueued on the context's HIP stream and is asynchronous
 *    unless stated otherwise.  Calls that fill a host skfab_info synchronise
 *    the stream before returning.
 *  - Errors: return codes only; no C++ exception crosses the ABI.  Argument and
 *    shape errors are detected before anything is enqueued.  Numerical
 *    failures detected on the device (rank deficiency, branch cut, quadrature
 *    non-convergence) are reported through skfab_info.status, which requires a
 *    synchronising call (info != NULL).
 *  - Layouts: dense matrices are column-major with the stated leading
 *    dimension.  CSR uses 0-based int32 row pointers and column indices.
 *  - Precision: values are real; the default path computes in IEEE double.
 */
#ifndef SKFAB_H
#define SKFAB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SKFAB_VERSION_MAJOR 0
#define SKFAB_VERSION_MINOR 1

typedef enum skfab_status {
    SKFAB_OK = 0,
    SKFAB_ERR_ARG = 1,      /* null pointer, unsupported option, bad enum value          */
    SKFAB_ERR_SHAPE = 2,    /* violates 1 <= k <= min(m, 8), m < s <= N, zeta <= s ...   */
    SKFAB_ERR_RANK = 3,     /* sketched basis numerically singular from its first column,
                               or the projected matrix singular (Section 2.1)           */
    SKFAB_ERR_BRANCH = 4,   /* projected matrix has det < 0: an eigenvalue on the branch
                               cut of z^(-1/2) (Section 2.3, sketched Ritz values)       */
    SKFAB_ERR_QUAD = 5,     /* adaptive quadrature did not converge by lmax (Section 4.1) */
    SKFAB_ERR_HIP = 6,      /* a HIP runtime call failed                                  */
    SKFAB_ERR_WORKSPACE = 7,/* workspace pointer null or smaller than required            */
    SKFAB_ERR_TOO_LARGE = 8 /* skfab_solve_noalloc: the problem needs more workspace than
                               SKFAB_NOALLOC_WS_BYTES                                   */
} skfab_status;

/* f in f(A) b.  INVSQRT and INV are Stieltjes functions (Section 1) and work with
 * every method; POLY is evaluated in closed form (SFOM_CLOSED only); EXP in closed
 * form (SFOM_CLOSED) or, with SGMRES_QUAD, by the contour rule of Sections 4.1 and
 * 5.2 (fparam > 0, m <= 200). */
typedef enum skfab_fun {
    SKFAB_F_INVSQRT = 0,    /* z^(-1/2), principal branch                            */
    SKFAB_F_EXP = 1,        /* exp(-fparam * z), fparam >= 0: Pade [13/13] scaling and
                               squaring of the projected matrix (SFOM_CLOSED); sketched
                               GMRES (SGMRES_QUAD, fparam > 0) by Cauchy's integral over
                               a parabola a + i theta - c theta^2 around the negated
                               sketched Ritz values (eigenvalues of H_hat by a
                               Hessenberg QR iteration on the device), trapezoidal rule
                               with K = 32, 64, ..., 1024 intervals under the test of
                               Section 4.1 at quad_tol (info.l_used = K + 1)            */
    SKFAB_F_INV = 2,        /* 1/z (test function)                                   */
    SKFAB_F_POLY = 3        /* sum_i poly[i] z^i, npoly coefficients (test function)  */
} skfab_fun;

typedef enum skfab_method {
    SKFAB_SFOM_CLOSED = 0,  /* Algorithm 1, closed form (sFOM'''): exp by Pade [13/13],
                               1/z and polynomials directly, z^(-1/2) by the adaptive
                               quadrature of Section 4.1 at tol 1e-13 (accepted at the
                               rounding floor 1e-10 when 1e-13 is out of reach of the
                               node solves: info.flags bit 1, info.quad_diff)       */
    SKFAB_SFOM_QUAD = 1,    /* (sFOM) integral form, adaptive quadrature, quad_tol   */
    SKFAB_SGMRES_QUAD = 2   /* Algorithm 2, (sGMRES), adaptive quadrature, quad_tol
                               (Gauss-Chebyshev for the Stieltjes functions, the
                               contour rule for EXP)                                   */
} skfab_method;

/* Precision of the Krylov recurrence (spec precision extension).  In every
 * mode the sketches are accumulated in FP64, the dot products of the recurrence
 * are accumulated in FP64 per thread and reduced in FP64, and the small sketched
 * problem (QR, quadrature / f evaluation) and the assembly x = V_m y (FP64
 * accumulation) stay FP64.  Reduced precisions need zeta = 8 and k <= 4. */
typedef enum skfab_prec {
    SKFAB_PREC_FP64 = 0,           /* A, basis and all arithmetic in IEEE double       */
    SKFAB_PREC_FP32 = 1,           /* A values, basis V_m and A V_m stored in FP32; SpMV
                                      and the basis update in FP32                      */
    SKFAB_PREC_FP32_BF16BASIS = 2  /* as FP32, but V_m stored in bfloat16 (rounded to
                                      nearest even); the rounded vector is the one
                                      multiplied by A and sketched                      */
} skfab_prec;

/* Sketch S of the method (the s x N subspace embedding of Section 1, eq. sketch). */
typedef enum skfab_sketch {
    SKFAB_SKETCH_SPARSE_SIGN = 0,  /* zeta nonzeros +-1/sqrt(zeta) per column, drawn by a
                                      counter-based hash inside the step kernel (see
                                      skfab_sketch_pattern); never stored              */
    SKFAB_SKETCH_SRDCT = 1         /* subsampled randomized DCT S = sqrt(N/s) P F E of
                                      Section 5.1: E = diag(srdct_signs), F the orthonormal
                                      DCT-II, P the srdct_rows of F E; applied to the
                                      stored basis after the recurrence (FP64 matrix
                                      cores); workspace + 8 s N bytes                 */
} skfab_sketch;

typedef enum skfab_valtype {
    SKFAB_VAL_F64 = 0
} skfab_valtype;

/* Sparse matrix A in CSR form (device arrays, caller-owned, read-only). */
typedef struct skfab_csr {
    int64_t n;              /* N: rows = columns                                     */
    int64_t nnz;            /* rowptr[n]                                             */
    const int32_t *rowptr;  /* [n+1], non-decreasing, rowptr[0] = 0                  */
    const int32_t *col;     /* [nnz], column indices in [0, n)                       */
    const void *val;        /* [nnz], element type given by val_type                 */
    int32_t val_type;       /* skfab_valtype                                         */
} skfab_csr;

/* Method parameters (Algorithm 1/2 inputs; host struct). */
typedef struct skfab_params {
    int32_t f;              /* skfab_fun                                             */
    double fparam;          /* tau for SKFAB_F_EXP                                   */
    const double *poly;     /* HOST array of npoly coefficients (lowest degree first) */
    int32_t npoly;          /* 1 <= npoly <= m for SKFAB_F_POLY                       */
    int32_t method;         /* skfab_method                                          */
    int32_t m;              /* Krylov dimension, 1 <= m <= 512                       */
    int32_t k;              /* truncation length, 1 <= k <= min(m, 8)                */
    int32_t s;              /* sketch rows, m < s <= min(N, 1024)                    */
    int32_t zeta;           /* nonzeros per sketch column: 8                         */
    uint64_t seed;          /* sketch seed (SplitMix64 stream, see skfab_sketch_pattern) */
    int32_t l1, l2;         /* starting quadrature orders, l1 < l2 (default 32, 45)  */
    int32_t lmax;           /* largest quadrature order tried (default 1395)         */
    double quad_tol;        /* relative tolerance of the quadrature test (Section 4.1) */
    int32_t prec;           /* skfab_prec                                            */
    double cond_max;        /* largest kappa_F(R_j) = ||R_j||_F ||R_j^-1||_F of the basis
                               prefix the approximant is formed from (Section 2.1 remedy
                               for an extremely ill-conditioned R, see skfab_solve);
                               0 = the default of the precision (SKFAB_COND_MAX_FP64,
                               SKFAB_COND_MAX_FP32, SKFAB_COND_MAX_BF16); else >= 1   */
    int32_t sketch;         /* skfab_sketch (default 0: sparse sign).  SRDCT: skfab_solve
                               with one pass only; zeta and seed are not used           */
    const int8_t *srdct_signs;  /* SRDCT: DEVICE int8[N], the +-1 diagonal of E          */
    const int32_t *srdct_rows;  /* SRDCT: DEVICE int32[s], the rows of F E kept by P,
                               distinct, in [0, N); the draws are the caller's          */
    int32_t two_pass;       /* 1: the two-pass form of Section 4.2 (skfab_solve only): the
                               first pass keeps the k + 1 basis vectors of the window and
                               the sketches, the second reruns the recurrence and adds each
                               regenerated vector to x; workspace O(kN) instead of O(mN),
                               twice the products with A.  0: one pass, V_m kept      */
} skfab_params;

/* Default cond_max per precision.  FP64: rounding of the whitened problem stays near
 * u kappa <= 1e-6.  A basis stored with unit roundoff u_p cannot hold directions below
 * u_p of the rest: kappa of its sketch levels off near 1e2..1e3 / u_p even where the
 * exact basis is dependent, so the reduced precisions stop at 4 / u_p, below that
 * level (u_p = 2^-24 for FP32, 2^-8 for bfloat16). */
#define SKFAB_COND_MAX_FP64 1e10
#define SKFAB_COND_MAX_FP32 67108864.0
#define SKFAB_COND_MAX_BF16 1024.0

/* Filled by synchronising calls (host struct). */
typedef struct skfab_info {
    int32_t status;         /* device-detected numerical status (skfab_status)       */
    int32_t m_used;         /* Krylov dimension actually used (< m after breakdown)  */
    int32_t l_used;         /* quadrature order accepted (0 if none)                 */
    int32_t a_format;       /* storage of A in the Arnoldi steps: 0 CSR (or no product with A),
                               1 SELL-64 with int32 columns, 2 SELL-64 with int16 offsets
                               col - row (chosen when every col - row of A lies in
                               [-32768, 32767]); plus 4 when the SELL-64 copy stores
                               the values as uint8 indices into a table of A's distinct
                               values (at most 256 of them, 0.0 counted; see
                               skfab_set_value_table)                                */
    double eps_est;         /* max_j | ||S v_j||^2 - 1 |  (Section 4.3 monitor)        */
    double rcond_R;         /* 1 / kappa_F(R), R the whitening factor used (kappa_F =
                               ||R||_F ||R^-1||_F)                                     */
    double sigma;           /* spectral scale used by the quadrature                 */
    double beta;            /* ||b||_2                                               */
    double arnoldi_relres;  /* ||S A V_m - [S V_m, S u_{m+1}] Hbar||_F / ||S A V_m||_F: the
                               Arnoldi relation checked in the sketched space          */
    double quad_diff;       /* relative difference ||q_l1 - q_l2|| / ||q_l2|| (whitened
                               coordinates) at the accepted quadrature order; 0 without
                               quadrature                                              */
    int32_t flags;          /* bit 0 (SKFAB_FLAG_TRUNCATED): the basis was cut to its
                               conditioned prefix (Section 2.1 remedy, see skfab_solve);
                               bit 1 (SKFAB_FLAG_QUAD_FLOOR): the quadrature order was
                               accepted at the rounding floor, quad_diff > tol          */
    int32_t m_basis;        /* basis length built (m, or less after a breakdown); m_used
                               is smaller when the remedy cut the basis               */
} skfab_info;

#define SKFAB_FLAG_TRUNCATED 1
#define SKFAB_FLAG_QUAD_FLOOR 2

typedef struct skfab_ctx skfab_ctx;

/* Library version as MAJOR*100 + MINOR. */
int32_t skfab_version(void);

/* Human-readable name of a status code (static string, never NULL). */
const char *skfab_status_string(int32_t status);

/* Create a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL = the default stream).  *ctx receives a host handle.
 * Errors: SKFAB_ERR_ARG (ctx NULL, bad device), SKFAB_ERR_HIP. */
skfab_status skfab_create(skfab_ctx **ctx, int32_t device, void *hip_stream);

/* Rebind the context to another stream on the same device. */
skfab_status skfab_set_stream(skfab_ctx *ctx, void *hip_stream);

/* Destroy a context (does not synchronise; NULL is accepted). */
skfab_status skfab_destroy(skfab_ctx *ctx);

/* Bytes of device workspace skfab_solve (with nrhs right-hand sides) and
 * skfab_arnoldi need for this problem (host computation, no device work).
 * Errors: SKFAB_ERR_ARG (nrhs < 1, null pointers), SKFAB_ERR_SHAPE. */
skfab_status skfab_workspace_bytes(const skfab_csr *A, const skfab_params *p, int32_t nrhs,
                                   size_t *bytes);

/* X[:, r] <- approximation of f(A) B[:, r], r < nrhs (Algorithm 1 for SFOM_*,
 * Algorithm 2 for SGMRES).
 *   b, ldb   device, N x nrhs column-major, column r at b + r ldb (ldb >= N when
 *            nrhs > 1; ignored for nrhs = 1)
 *   x, ldx   device, N x nrhs column-major, column r at x + r ldx; may not alias b
 *   ws       device workspace of at least skfab_workspace_bytes(A, p, nrhs) bytes,
 *            256-byte aligned
 *   info     optional host array of nrhs structs; if non-NULL the call synchronises
 *            the stream and returns the device-detected status of column r in
 *            info[r].status
 * Steps (all on the device): draw S (implicit, hashed), k-truncated Arnoldi with the
 * sketches S v_j and S A v_j formed on the fly and the extension vector u_{m+1},
 * Householder QR of the extended sketch [S V_m, S u_{m+1}] = Q_e R_e, the projected
 * problem from the Arnoldi relation (Hessenberg pencil t R + R_e Hbar; for sFOM the
 * matrix H_m + (R^-1 r) e_m^T of the Section 2.2 remark, similar to Q^T SAV R^-1),
 * f of it or the quadrature of Section 4.1, and the assembly x = V_m y.
 * Extremely ill-conditioned R (the remark after eq. sFOM''' of Section 2.1): the
 * numerical pseudoinverse used is the truncated QR one in basis order, i.e. the
 * approximant is formed from the longest prefix V_j of the basis whose sketch has
 * ||R_j||_F ||R_j^-1||_F <= p->cond_max (info.m_used = j < info.m_basis, flags bit 0).
 * nrhs > 1: for f = z^(-1/2) or 1/z with zeta = 8, k <= 4 and nrhs <= 4 the columns
 * are solved together by the batched form (one step launch per j serves every column,
 * same S for all); otherwise they are solved one after another in the workspace.
 * b = 0 gives x = 0.  Lucky breakdown (Section 4: division by ||w||) stops the
 * recurrence early; info.m_used reports the dimension used. */
skfab_status skfab_solve(skfab_ctx *ctx, const skfab_csr *A, const double *b, int64_t ldb,
                         int32_t nrhs, double *x, int64_t ldx, const skfab_params *p,
                         void *ws, size_t ws_bytes, skfab_info *info);

/* Sketch size chosen by the computation (the conclusions' "responsibly reckless"
 * approach, Section 6): solve with the optimistic p->s first; if the solve fails
 * numerically (info.status nonzero: a sketched Ritz value on the branch cut, a
 * quadrature that does not converge, a singular factor) or the Section 4.3 monitor
 * info.eps_est = max_j | ||S v_j||^2 - 1 | exceeds eps_max, s was too small: the
 * solve is redone with 2 s (S redrawn from the same seed), up to s_max.  One right-
 * hand side; sparse-sign sketch, one-pass form.  ws must hold
 * skfab_workspace_bytes(A, p with s = s_max, 1).  On return x and info are those of
 * the last attempt, *s_used its sketch size (s_max with a nonzero info.status when
 * no attempt succeeded).  Every attempt synchronises to read its info.  Errors:
 * SKFAB_ERR_ARG (null pointers, eps_max <= 0, s_max < p->s, two-pass or SRDCT),
 * the shape checks of skfab_solve at s = s_max, SKFAB_ERR_WORKSPACE. */
skfab_status skfab_solve_reckless(skfab_ctx *ctx, const skfab_csr *A, const double *b, double *x,
                                  const skfab_params *p, int32_t s_max, double eps_max, void *ws,
                                  size_t ws_bytes, skfab_info *info, int32_t *s_used);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): skfab_solve with one right-hand
 * side (ldb = ldx = N) whose workspace is a static device array of
 * SKFAB_NOALLOC_WS_BYTES bytes inside the library, one per device, held until the
 * process ends.  The call allocates and frees nothing.  The array's address is
 * resolved by skfab_create for the context's device.  Problems whose
 * skfab_workspace_bytes(A, p, 1) exceeds the array are refused with
 * SKFAB_ERR_TOO_LARGE before anything is enqueued (the 2D 100 x 100 problem at m = 50,
 * s = 200 needs 26 MiB).  Every call on a device shares that device's array: calls
 * that overlap on one device (two streams, two threads) race and must be ordered by
 * the caller.  Otherwise as skfab_solve (stream-ordered; info synchronises). */
#define SKFAB_NOALLOC_WS_BYTES (64u * 1024u * 1024u)
skfab_status skfab_solve_noalloc(skfab_ctx *ctx, const skfab_csr *A, const double *b, double *x,
                                 const skfab_params *p, skfab_info *info);

/* Test hook: run only the k-truncated Arnoldi recurrence with sketches
 * (Algorithm 2, basis part) and export its state.
 *   V    device, N x m column-major (ld = N), the unit basis vectors v_1..v_m
 *   SV   device, s x m (ld = s), S v_j          SAV  device, s x m, S A v_j
 *   H    device, (m+1) x m (ld = m+1), the truncated MGS coefficients h_ij
 *        (zero outside the band of width k+1)
 * Any of V, SV, SAV, H may be NULL.  info (optional, synchronising) receives
 * m_used, beta and eps_est. */
skfab_status skfab_arnoldi(skfab_ctx *ctx, const skfab_csr *A, const double *b,
                           const skfab_params *p, double *V, double *SV, double *SAV,
                           double *H, void *ws, size_t ws_bytes, skfab_info *info);

/* Test hook: the small sketched problem alone, from Arnoldi data.
 *   SVext  device, s x (m+1) (ld = s): columns 0..m-1 are S v_1..S v_m (unit basis
 *          vectors), column m is S u_{m+1} = h_{m+1,m} S v_{m+1} (unnormalised)
 *   Hbar   device, (m+1) x m (ld = m+1): the Arnoldi coefficients h_ij of
 *          A v_j = sum_i h_ij v_i + u_{j+1}; row m is ignored (taken as e_m^T).
 *          Its band must match p->k (h_ij = 0 unless j-k+1 <= i <= j+1), as the
 *          k-truncated recurrence produces it: the pencil and, for k <= 4, the
 *          square-case node solves (band elimination) use only those entries.
 *   beta   ||b|| (host)
 *   y      device, m: coefficients of the approximant V_m y (Sections 2.1, 3, 4.1)
 * Uses the same device algorithm as skfab_solve after the basis is built. */
skfab_status skfab_small_problem(skfab_ctx *ctx, const double *SVext, const double *Hbar,
                                 double beta, const skfab_params *p, double *y,
                                 void *ws, size_t ws_bytes, skfab_info *info);

/* Workspace bytes for skfab_small_problem alone. */
skfab_status skfab_small_workspace_bytes(const skfab_params *p, size_t *bytes);

/* Test hook: the sparse-sign sketch pattern of columns [col0, col0 + ncols): the
 * s x N subspace embedding S of Section 1, eq. (sketch) (an epsilon-embedding of the
 * Krylov space with high probability), drawn as a sparse sign matrix.
 * rows  device int32 [ncols * zeta]: rows[i*zeta + q] is the row of entry q of
 *       column col0 + i;  signs device int8 [ncols * zeta], +1 or -1.
 * Definition (implemented independently of the CPU reference): SplitMix64
 * (gamma 0x9E3779B97F4A7C15) seeded with `seed`; column i uses outputs
 * 4*ceil(zeta/8)*i + 1 ... ; their 32-bit halves w_q give Floyd's sampling draws
 * r = floor((w_q >> 1)(j+1) / 2^31), j = s - zeta + q (row j on a repeat) and the
 * sign (+1 if bit 0 of w_q is 0).  Each column of S is sum_q sign_q e_row_q / sqrt(zeta).
 * Errors: SKFAB_ERR_SHAPE unless 1 <= zeta <= s and zeta in {2, 4, 8, 16}. */
skfab_status skfab_sketch_pattern(skfab_ctx *ctx, int64_t col0, int64_t ncols, int32_t s,
                                  int32_t zeta, uint64_t seed, int32_t *rows, int8_t *signs);

/* Test hook: Sv <- S v for a device vector v of length n (Sv device, length s), the
 * sketch of Section 1, eq. (sketch), with the pattern of skfab_sketch_pattern.
 * Deterministic (fixed reduction order).  Uses `ws` for per-block partial sums
 * (at least skfab_sketch_ws_bytes(n, s) bytes). */
skfab_status skfab_sketch_apply(skfab_ctx *ctx, int64_t n, int32_t s, int32_t zeta,
                                uint64_t seed, const double *v, double *Sv,
                                void *ws, size_t ws_bytes);
size_t skfab_sketch_ws_bytes(int64_t n, int32_t s);

/* Test hook: SV <- S V for the SRDCT sketch S = sqrt(N/s) P F E (Section 5.1): V device
 * n x ncols column-major (ld ldv >= n), SV device s x ncols (ld s); signs (int8[n], +-1)
 * and rows (int32[s], distinct, in [0, n)) device arrays.  The contraction used by
 * skfab_solve with SKFAB_SKETCH_SRDCT (F_P formed in ws, then FP64 matrix cores, partial
 * tiles summed in a fixed order).  ws: skfab_srdct_ws_bytes(n, s, ncols) bytes.
 * Errors: SKFAB_ERR_ARG (null pointers), SKFAB_ERR_SHAPE (s > n, ldv < n, sizes < 1),
 * SKFAB_ERR_WORKSPACE. */
size_t skfab_srdct_ws_bytes(int64_t n, int32_t s, int32_t ncols);
skfab_status skfab_srdct_apply(skfab_ctx *ctx, int64_t n, int32_t s, const int8_t *signs,
                               const int32_t *rows, const double *V, int64_t ldv, int32_t ncols,
                               double *SV, void *ws, size_t ws_bytes);

/* Value-table storage of A (on by default; FP64 form).  When A has at most 256
 * distinct values (the padding value 0.0 counted), the SELL-64 copy of A made by
 * each FP64 solve stores every entry's value as a uint8 index into a table of those
 * values, which the step kernel holds in LDS: 1 byte per stored entry instead of 8.
 * (The FP32 forms keep their 4-byte values: there the lookup costs more than it
 * saves.)  The values used are the same, so the results are bitwise those of the
 * plain form.  The conversion finds the distinct values itself (an open-addressing
 * set in the workspace); matrices with more of them use the plain form.
 * enable = 0 turns the table form off for later solves on this context (the plain
 * form is then always used), 1 turns it back on.  Errors: SKFAB_ERR_ARG (null ctx,
 * enable other than 0 or 1). */
skfab_status skfab_set_value_table(skfab_ctx *ctx, int32_t enable);

/* Arnoldi relation check.  The small problem builds the projected matrix from the
 * Arnoldi relation of the k-truncated recurrence (the pencil t R + R_e Hbar; the
 * paper's eq. (arnoldi_relation) with the sketch applied), so S A V_m is not needed
 * to solve.  With enable = 1 the step kernels also sketch A u_j into S A V_m and
 * every solve checks the relation: info.arnoldi_relres = ||S A V_m - [S V_m,
 * S u_{m+1}] Hbar||_F / ||S A V_m||_F.  Off (the default) saves 8 of the 16 sketch
 * scatter-adds per row and step; info.arnoldi_relres is then -1.  skfab_arnoldi always
 * forms S A V_m.  Errors: SKFAB_ERR_ARG (null ctx, enable other than 0 or 1). */
skfab_status skfab_set_arnoldi_check(skfab_ctx *ctx, int32_t enable);

/* Kernel timing with HIP events on the context's stream (benchmark support).
 * enable = 0 turns timing off; enable = n >= 1 turns it on.  A run of consecutive
 * launches of a timed kernel class -- the step launches j = 0 .. m-1 of a solve's
 * recurrence, the step launches of a batched solve -- is bracketed by one pair of
 * events and all its launches count (the interval includes the gaps between them);
 * launches that come one at a time (the assembly, the second pass of the two-pass
 * form, the checkpointed recurrence of the adaptive solve) are bracketed every n-th
 * (n = 1: every one; a larger n keeps the events' own cost out of most of them).
 * Negative values are rejected with SKFAB_ERR_ARG.  skfab_timing_read synchronises
 * the stream and returns the summed event durations and the count of timed launches
 * since the last read (then resets).
 *   kernel 0: the fused Arnoldi step kernel (SpMV + orthogonalisation dots +
 *             sparse-sign sketches), kernel 1: the assembly x = V_m y.
 * Events are host runtime objects created by skfab_timing_enable; no device
 * memory is allocated. */
skfab_status skfab_timing_enable(skfab_ctx *ctx, int32_t enable);
skfab_status skfab_timing_read(skfab_ctx *ctx, int32_t kernel, double *total_ms,
                               int64_t *launches);

/* ---------------------------------------------------------------- batches
 * Many independent problems, each with several right-hand sides, solved together:
 * one launch per Arnoldi step covers every (problem, right-hand side) pair whose
 * Krylov dimension has not been reached (the method of Algorithm 1/2 applied to
 * each pair independently; each pair has its own basis and sketches, and the
 * right-hand sides of one problem share its sketch S and its copy of A). */
typedef struct skfab_batch_problem {
    skfab_csr A;            /* device CSR, FP64 values                               */
    const double *B;        /* device, N x nrhs column-major (column r at B + r ldb) */
    double *X;              /* device, N x nrhs column-major: the results (column r at
                               X + r ldx)                                            */
    int32_t m;              /* Krylov dimension of this problem, 1 <= m <= 512       */
    int32_t s;              /* sketch size, m < s <= min(N, 1024)                    */
    uint64_t seed;          /* seed of this problem's sketch S                       */
    int64_t ldb, ldx;       /* leading dimensions of B and X (0 = N; otherwise >= N)  */
} skfab_batch_problem;

/* Launch shape of the batched step kernel: threads per block (256, 512, 1024) and
 * the target number of 64-row SELL slices per wavefront (sets the blocks per
 * (problem, right-hand side) pair, a multiple of 8 and at most 256).  A block size
 * whose per-wave sketch bins (2 s_max doubles each) would not fit the CU's LDS is
 * lowered by halving for the call (the stored tuning is kept); the autotuner skips
 * such sizes.  packed = 1 runs, where it applies, the packed form of the step
 * (default 0; the autotuner tries both): one block per chunk of a problem's rows
 * carries all its right-hand sides, so a row's column offsets, value indices and
 * sketch hash are read or computed once for all of them.  It applies to k = 2,
 * 512-thread blocks, the steps 2 <= j < m of each problem, with the Arnoldi
 * relation check off and the sketch bins of its eight wavefronts (nrhs s_max
 * doubles each) within the LDS; the results are bitwise those of the per-unit
 * form. */
typedef struct skfab_batch_tuning {
    int32_t block;
    int32_t slices_per_wave;
    int32_t packed;         /* 0 or 1 */
} skfab_batch_tuning;

/* Device workspace bytes of skfab_solve_batched / skfab_batch_autotune (host only;
 * independent of the tuning).  p supplies f, method, k, zeta, prec and the
 * quadrature parameters; p->m and p->s are ignored (per problem instead).
 * Errors: SKFAB_ERR_ARG (nprob outside 1..4096, nrhs outside 1..4, f other than
 * z^(-1/2) or 1/z, zeta != 8, k outside 1..4), SKFAB_ERR_SHAPE (a problem's sizes). */
skfab_status skfab_batch_workspace_bytes(int32_t nprob, const skfab_batch_problem *probs,
                                         int32_t nrhs, const skfab_params *p, size_t *bytes);

/* X_p[:, r] <- approximation of f(A_p) B_p[:, r] for every problem p and column r
 * (same method and parameters as skfab_solve).  ws: device workspace of at least
 * skfab_batch_workspace_bytes, 256-byte aligned.  info: optional host array of
 * nprob * nrhs entries (pair (p, r) at p * nrhs + r); if non-NULL the call
 * synchronises.  The per-problem arrays in `probs` are read on the host during the
 * call only.  Asynchronous otherwise, on the context's stream. */
skfab_status skfab_solve_batched(skfab_ctx *ctx, int32_t nprob, const skfab_batch_problem *probs,
                                 int32_t nrhs, const skfab_params *p, void *ws, size_t ws_bytes,
                                 skfab_info *info);

/* Set / read the context's launch shape for batched solves.  Errors: SKFAB_ERR_ARG
 * (null argument, block other than 256/512/1024, slices_per_wave outside 1..64,
 * packed other than 0 or 1). */
skfab_status skfab_batch_set_tuning(skfab_ctx *ctx, const skfab_batch_tuning *t);
skfab_status skfab_batch_get_tuning(skfab_ctx *ctx, skfab_batch_tuning *t);

/* Autotuner: times the batched step kernel on this batch for every candidate
 * shape (block 256/512/1024 x 1/2/4/.../64 slices per wavefront, and the packed form
 * with 512-thread blocks where it applies) over `steps` Arnoldi steps (after an
 * untimed first step), keeps the fastest in the context and returns it in *chosen
 * (may be NULL).  Overwrites the workspace; synchronises. */
skfab_status skfab_batch_autotune(skfab_ctx *ctx, int32_t nprob, const skfab_batch_problem *probs,
                                  int32_t nrhs, const skfab_params *p, void *ws, size_t ws_bytes,
                                  int32_t steps, skfab_batch_tuning *chosen);

/* ------------------------------------------------------------ adaptive m
 * Sketched FOM with the Krylov dimension chosen on the fly (Section 4.3): the
 * recurrence runs up to p->m steps; at the checkpoints m0, m0 + d, ... (< p->m)
 * the approximant of the first m' steps is formed from the nested basis, and the
 * run stops at the first checkpoint whose relative stopping estimate against the
 * previous checkpoint,
 *     || S V_m' (y_m' - [y_prev; 0]) || / || S V_m' y_m' || * sqrt((1+eps)/(1-eps)),
 * eps = max_j | ||S v_j||^2 - 1 |  (the Section 4.3 monitor), is <= tol.  Without
 * such a checkpoint the result is the full p->m solve (its estimate against the
 * last checkpoint is returned).  Every checkpoint synchronises the stream once.
 *   p->method must be SKFAB_SFOM_CLOSED; k <= m0 <= p->m, d >= 1, tol > 0.
 *   m_stop, estimate: optional host outputs; info as for skfab_solve.
 *   ws: at least skfab_adaptive_workspace_bytes, 256-byte aligned. */
skfab_status skfab_adaptive_workspace_bytes(const skfab_csr *A, const skfab_params *p, size_t *bytes);
skfab_status skfab_solve_adaptive(skfab_ctx *ctx, const skfab_csr *A, const double *b, double *x,
                                  const skfab_params *p, int32_t m0, int32_t d, double tol,
                                  void *ws, size_t ws_bytes, skfab_info *info, int32_t *m_stop,
                                  double *estimate);

/* ----------------------------------------------------- learned controller
 * Features and the network of the controller that predicts (m, k, s) for a
 * requested tolerance (the plain adaptive-m solve above is its fallback).
 *
 * bounds[0] = min_i (a_ii - sum_{j != i} |a_ij|), bounds[1] = max_i (a_ii + sum |a_ij|)
 * (Gershgorin discs), device double[2]; ws of skfab_gershgorin_ws_bytes(n) bytes. */
size_t skfab_gershgorin_ws_bytes(int64_t n);
skfab_status skfab_gershgorin(skfab_ctx *ctx, const skfab_csr *A, double *bounds, void *ws,
                              size_t ws_bytes);

/* Network 16 -> 64 -> 64 -> 3, ReLU hidden layers, linear output, FP32.
 * params: device float[skfab_mlp_param_count()] laid out row-major as
 * W1[64][16], b1[64], W2[64][64], b2[64], W3[3][64], b3[3].
 * X: device float[B][16]; Y, T: device float[B][3]; ws: skfab_mlp_ws_bytes(B).
 * loss_grad: grad (device, param_count) of L = (1/(3B)) sum (y - t)^2, and L in
 * *loss (device float, may be NULL).  adam: one Adam step (Kingma & Ba 2015) with
 * step number t >= 1 on params with moment buffers m1, m2 (device, param_count). */
int32_t skfab_mlp_param_count(void);
size_t skfab_mlp_ws_bytes(int32_t batch);
skfab_status skfab_mlp_forward(skfab_ctx *ctx, const float *X, int32_t B, const float *params,
                               float *Y, void *ws, size_t ws_bytes);
skfab_status skfab_mlp_loss_grad(skfab_ctx *ctx, const float *X, const float *T, int32_t B,
                                 const float *params, float *grad, float *loss, void *ws,
                                 size_t ws_bytes);
skfab_status skfab_mlp_adam(skfab_ctx *ctx, float *params, const float *grad, float *m1, float *m2,
                            int32_t t, float lr, float beta1, float beta2, float eps);

#ifdef __cplusplus
}
#endif

#endif /* SKFAB_H */
