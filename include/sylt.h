/*
 * sylt.h -- C ABI of libsylt, an MI355X (gfx950) solver for the
 * N-dimensional Sylvester tensor equation
 *
 *     sum_{k=1..N} A_k x_k X = B,    [A x_k X]_{..i_k..} = sum_m A[i_k, m] X[..m..]
 *
 * (Cuesta & de la Hoz, arXiv 2412.15840, Section 1, eq. e:sylvesterND) by the
 * Schur / Bartels-Stewart route of Section 2: A_k = U_k T_k U_k^*, the chain
 * C = U_N^* x_N ... U_1^* x_1 B (eq. e:CUNU2U1B), one dependency-ordered
 * sweep solving sum_k T_k x_k Y = C (eq. e:TjYC, entrywise eq. e:yi1i2iN) and
 * the chain X = U_N x_N ... U_1 x_1 Y (eq. e:XUNU2U1Y).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Tensors: column-major, mode 1 fastest.  Element (i_1..i_N), 0-based,
 *    sits at sum_j i_j * prod_{l<j} n_l -- the paper's linear index
 *    (Section 2.2, eq. e:index).  Complex values are interleaved (re, im):
 *    complex128 = two doubles (the bytes of torch.complex128), complex64 =
 *    two floats.  A "double*" tensor argument points at complex128 data.
 *  - Matrices: n_k x n_k complex128, column-major (M(i, m) at M[2*(i + n_k*m)]).
 *  - Every tensor / matrix pointer is a DEVICE pointer on the current HIP
 *    device, owned by the caller, 16-byte aligned.  The library never frees
 *    caller memory.
 *  - `stream` is a hipStream_t passed as void* (0 = legacy default stream).
 *    Work is enqueued on it without host synchronisation unless stated.
 *  - Singleton modes (n_k = 1) may appear at any position: A_k is then a
 *    scalar that joins the eigenvalue sums (Section 4, singleton handling).
 *  - Limits: 1 <= N <= 32, 1 <= n_k <= 256, prod n_k < 2^62.
 *  - Return value: a sylt_status code (0 = success).  Argument checks run on
 *    the host before any HIP call and return synchronously.
 *  - A plan owns small device buffers that its calls reuse (reduction
 *    partial sums, the exp(t T_k) of the last evolution).  Calls on one plan
 *    must therefore not run concurrently: issue them on one stream, or order
 *    them.  Distinct plans are independent.
 */
#ifndef SYLT_H
#define SYLT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SYLT_OK = 0,
    SYLT_E_INVALID_ARG = -1,    /* bad N, n_k, null pointer, unknown enum */
    SYLT_E_SINGULAR = -2,       /* some eigenvalue sum lambda_{1,i_1}+..+lambda_{N,i_N} is 0 (Section 2) */
    SYLT_E_NO_CONVERGENCE = -3, /* Schur QR iteration or iterative refinement did not converge */
    SYLT_E_OUT_OF_MEMORY = -4,  /* plan allocation failed */
    SYLT_E_DEVICE = -5,         /* a HIP runtime call failed */
    SYLT_E_UNSUPPORTED = -6,    /* valid problem outside the limits (n_k > 256, N > 32) */
    SYLT_E_WORKSPACE = -7       /* workspace pointer null or smaller than sylt_workspace_bytes() */
} sylt_status;

/* Arithmetic of the solve.  FP64: complex128 everywhere.  MIXED: transforms in
 * FP32 with FP32 accumulation on complex64 intermediates, sweep arithmetic,
 * residual and refinement updates in FP64. */
enum { SYLT_FP64 = 0, SYLT_MIXED = 1 };
/* Direction of sylt_transform: TO_SCHUR applies U_k^* along every mode
 * (eq. e:CUNU2U1B), FROM_SCHUR applies U_k (eq. e:XUNU2U1Y). */
enum { SYLT_TO_SCHUR = 0, SYLT_FROM_SCHUR = 1 };
/* Operator of sylt_sweep: N solves sum_k T_k x_k Y = C (upper triangular,
 * eq. e:yi1i2iN, descending index sums); C solves sum_k T_k^* x_k Y = C (the
 * adjoint, lower triangular, ascending index sums). */
enum { SYLT_OP_N = 0, SYLT_OP_C = 1 };

typedef struct sylt_plan_s *sylt_plan;

typedef struct {
    int precision;   /* SYLT_FP64 or SYLT_MIXED */
    double rtol;     /* MIXED: stop when ||B - sum_k A_k x_k X||_F <= rtol ||B||_F */
    int max_iter;    /* MIXED: maximum number of FP32 correction solves (>= 1) */
} sylt_opts;

typedef struct {
    int status;          /* same as the return value */
    int iterations;      /* MIXED: correction solves performed; FP64: 1 */
    double rel_residual; /* MIXED: final ||R||_F / ||B||_F in FP64; FP64: -1 (not computed) */
    double sep;          /* min over multi-indices of |sum_k lambda_{k,i_k}| */
    /* device time per phase (HIP events on `stream`, summed over the MIXED
     * iterations): both transform chains, the sweep, the FP64 residual
     * passes (0 for FP64) */
    float ms_transform, ms_sweep, ms_residual;
} sylt_info;

/*
 * sylt_schur_factor -- build a plan: complex Schur factors A_k = U_k T_k U_k^*
 * (Section 2; computed on the device by Hessenberg reduction and shifted QR)
 * and the eigenvalue-sum separation sep = min_i |sum_k lambda_{k,i_k}|, the
 * quantity whose non-vanishing is the solvability condition of Section 2.
 *   N        number of modes.
 *   n        host array of N extents n_1..n_N.
 *   A        host array of N device pointers, A[k] -> n_k x n_k complex128
 *            column-major.  Copied into the plan; the caller may free them.
 *   stream   hipStream_t as void*.
 *   out      receives the plan handle (library-owned; free with
 *            sylt_plan_destroy).
 * Synchronises `stream` once.  Errors: INVALID_ARG, UNSUPPORTED,
 * NO_CONVERGENCE (QR iteration cap), SINGULAR (sep == 0), OUT_OF_MEMORY,
 * DEVICE.  On error *out is set to NULL.
 */
int sylt_schur_factor(int N, const int64_t *n, const double *const *A, void *stream,
                      sylt_plan *out);

/*
 * sylt_schur_factor_ex -- sylt_schur_factor with a cap on the shifted-QR
 * iterations: at most qr_iter_per_n * n_k iterations for mode k (<= 0: the
 * default cap of 30 n_k).  A mode whose QR does not deflate within the cap
 * makes the call return NO_CONVERGENCE (its factors are not usable), so the
 * failure path can be exercised from the host with a small cap.
 */
int sylt_schur_factor_ex(int N, const int64_t *n, const double *const *A, int qr_iter_per_n,
                         void *stream, sylt_plan *out);

/*
 * sylt_plan_set_sweep_blocks -- re-plan the sweep's tiling with caller-chosen
 * block sizes.  The sweep cuts every non-singleton mode into blocks; tiles
 * (products of blocks) with equal block-index sums are independent (any order
 * that computes dependencies first is valid, Section 2).  M must equal the
 * number of modes with n_k > 1 and blocks[j] is the block of the j-th such
 * mode (in mode order): 1 <= blocks[j] <= n, and a block shorter than its
 * mode is at most 8.  The result must not depend on the tiling beyond
 * rounding; this call lets tests check that, and pin the shape a workload
 * runs with.  Synchronises the device (earlier calls may use the old tables).
 * Errors: INVALID_ARG (bad M or block), UNSUPPORTED (tile exceeds the LDS
 * budget of one workgroup); the plan keeps its previous tiling on error.
 */
int sylt_plan_set_sweep_blocks(sylt_plan p, int M, const int *blocks);

/*
 * sylt_plan_from_factors -- build a plan from caller-supplied factors instead
 * of computing them (U[k] unitary, T[k] upper triangular, A_k = U T U^*; the
 * library trusts them and uses only the upper triangle of T[k]).  A may be
 * NULL, in which case A_k = U_k T_k U_k^* is not stored and the MIXED solve
 * (which needs A_k for its residual) returns INVALID_ARG.  Same layout,
 * ownership and errors as sylt_schur_factor (no NO_CONVERGENCE).
 */
int sylt_plan_from_factors(int N, const int64_t *n, const double *const *A,
                           const double *const *U, const double *const *T, void *stream,
                           sylt_plan *out);

/* Copies U_k and T_k (0-based k) of the plan into caller device buffers of
 * n_k x n_k complex128 (either may be NULL).  Enqueued on `stream`. */
int sylt_plan_get_factors(sylt_plan p, int k, double *U, double *T, void *stream);

/* Eigenvalue-sum separation computed when the plan was built (host value). */
int sylt_plan_separation(sylt_plan p, double *sep);

/* Frees the plan's device memory (hipFree waits for device work that may
 * still use it). */
int sylt_plan_destroy(sylt_plan p);

/* Bytes of caller workspace sylt_solve / sylt_solve_backward need for
 * `precision` (>= 256; the MIXED solve needs one complex64 tensor).  Returns
 * a negative sylt_status on error. */
int64_t sylt_workspace_bytes(sylt_plan p, int precision);

/*
 * sylt_transform -- in-place chain of mode products with every U_k:
 * dir = TO_SCHUR: X <- U_N^* x_N ( ... (U_1^* x_1 X))   (eq. e:CUNU2U1B)
 * dir = FROM_SCHUR: X <- U_N x_N ( ... (U_1 x_1 X))     (eq. e:XUNU2U1Y)
 * precision = FP64: X is complex128, FP64 arithmetic.  MIXED: X is complex64
 * (FP32 data, U_k rounded to complex64, FP32 accumulation).
 * Singleton modes are identities.  Products on distinct modes commute, so the
 * library fuses runs of modes into single HBM passes.
 */
int sylt_transform(sylt_plan p, int dir, int precision, void *X, void *stream);

/*
 * sylt_sweep -- in-place solve of the triangular system of eq. e:TjYC:
 * op = N: sum_k T_k x_k Y = C, entry by entry with eq. e:yi1i2iN; the entries
 * are processed in descending hyperplanes i_1+..+i_N = s, which are mutually
 * independent (any order that computes dependencies first is valid, Section 2).
 * op = C: sum_k T_k^* x_k Y = C (ascending hyperplanes).
 * If every T_k of the plan is diagonal to rounding (normal A_k, Remark 1), the
 * sweep is the Hadamard product y_i = c_i / sum_k lambda_{k,i_k} (eq.
 * e:yi1i2iNdiag), one streaming pass; sylt_plan_describe reports which form
 * the plan uses.
 * precision = FP64: CY complex128.  MIXED: CY complex64, arithmetic in FP64.
 */
int sylt_sweep(sylt_plan p, int op, int precision, void *CY, void *stream);

/*
 * sylt_residual -- R = B - sum_k A_k x_k X in FP64 (the operator of eq.
 * e:sylvesterND) and, if norms != NULL, norms[0] = ||R||_F^2 and
 * norms[1] = ||B||_F^2 written to the HOST array norms (synchronises
 * `stream`).  B, X, R complex128; R may alias B.  Needs the plan's A_k.
 */
int sylt_residual(sylt_plan p, const double *B, const double *X, double *R, double *norms,
                  void *stream);

/*
 * sylt_solve -- X with sum_k A_k x_k X = B (Algorithm 3: transform, sweep,
 * transform).  FP64: X may alias B.  MIXED: X must not alias B (every
 * residual re-reads B; INVALID_ARG otherwise).  ws: caller device workspace of at least
 * sylt_workspace_bytes(p, o->precision) bytes (may be NULL for FP64).
 * o == NULL means FP64.  MIXED: iterative refinement -- X_0 from an FP32
 * transform solve, then R = B - sum A_k x_k X_i in FP64, stop when
 * ||R||_F <= rtol ||B||_F, else X_{i+1} = X_i + solve_32(R); one host sync per
 * iteration; NO_CONVERGENCE if max_iter solves do not reach rtol (X then holds
 * the last iterate).  If info != NULL it is filled (synchronises `stream`).
 */
int sylt_solve(sylt_plan p, const sylt_opts *o, const double *B, double *X, void *ws,
               size_t ws_bytes, void *stream, sylt_info *info);

/*
 * sylt_solve_backward -- gradients of a real loss L(X) through the solve,
 * reusing the plan's Schur factors.  With the convention
 * grad = dL/dRe + i dL/dIm (so dL = Re<grad, d.>):
 *   GB = A^{-*} GX, i.e. sum_k A_k^* x_k GB = GX (U^* chain, adjoint sweep,
 *        U chain);
 *   GA[k] = -GB_(k) X_(k)^*, i.e. GA[k](a, m) = -sum_{i: i_k = a} GB_i conj(X_{i|i_k->m}).
 * X: the forward solution.  GX: dL/dX.  GB: output (may alias GX).  GA: host
 * array of N device pointers to n_k x n_k complex128 outputs, or NULL to skip
 * the matrix gradients (individual entries may be NULL too).  ws: at least
 * sylt_workspace_bytes(p, SYLT_FP64) bytes.
 */
int sylt_solve_backward(sylt_plan p, const double *X, const double *GX, double *GB,
                        double *const *GA, void *ws, size_t ws_bytes, void *stream);

/*
 * sylt_solve_backward_noalloc -- sylt_solve_backward for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): no workspace argument, and no hipMalloc,
 * hipFree or allocating library call.  The grad-A partial sums go to a fixed
 * 8 MiB scratch array that the library holds on every device it runs on
 * until the process ends; its device address is looked up once per device.
 * Same arguments, layout and results as sylt_solve_backward (results agree
 * to rounding; with large n_k the partial sums use fewer workgroups).
 * Calls on one device share that scratch: calls that overlap on one GPU (on
 * different streams, or from different threads) race; order them.
 * Errors: INVALID_ARG (null pointer), UNSUPPORTED (an n_k x n_k matrix of
 * partial sums would not fit the scratch), DEVICE.
 */
int sylt_solve_backward_noalloc(sylt_plan p, const double *X, const double *GX, double *GB,
                                double *const *GA, void *stream);

/*
 * sylt_evolve -- time evolution by Theorem 1 in Schur form (eqs.
 * e:sylvesterNDG and e:G, from the proof's exp(tA) of a Kronecker sum): the
 * value at time t of the solution of X_t = sum_k A_k x_k X + B, X(0) = X0.
 * With C = U^*-chain(B) and Y(0) = U^*-chain(X0) it forms
 *   G = exp(t T_N) x_N ( ... exp(t T_1) x_1 (sum_k T_k x_k Y(0) + C)) - C,
 * solves sum_k T_k x_k Y = G by the sweep and returns X = U-chain(Y).  The
 * exp(t T_k) (eq. e:exptAj) are formed on the device by scaling and squaring
 * of a Taylor series on the triangular T_k; singleton modes contribute the
 * scalar exp(t a_k).  Uses only the plan's U_k and T_k (works for plans from
 * sylt_plan_from_factors without A).
 * B, X0: complex128 device tensors, not modified.  X: complex128 output; may
 * alias X0 or B.  t: any finite real.  ws: caller device workspace of at least
 * sylt_evolve_workspace_bytes(p) bytes (two complex128 tensors), not
 * overlapping B, X0 or X.  Enqueued on `stream`, no synchronisation.
 * INVALID_ARG for a NULL pointer or non-finite t; WORKSPACE if ws is too small.
 */
int sylt_evolve(sylt_plan p, double t, const double *B, const double *X0, double *X, void *ws,
                size_t ws_bytes, void *stream);

/* Bytes of workspace sylt_evolve needs (negative sylt_status on error). */
int64_t sylt_evolve_workspace_bytes(sylt_plan p);

/*
 * sylt_plan_describe -- writes a NUL-terminated JSON description of the plan
 * (extents, Schur separation, the fused transform passes with their tile
 * shapes and launch counts, the sweep's block sizes, tile levels and local
 * levels) into the caller's host buffer `buf` of `len` bytes.  Returns
 * INVALID_ARG if p or buf is NULL, or if len is too small (buf then holds a
 * truncated, NUL-terminated prefix).
 */
int sylt_plan_describe(sylt_plan p, char *buf, size_t len);

/* Static English description of a status code. */
const char *sylt_status_string(int code);

/* ABI version (major * 100 + minor). */
int sylt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SYLT_H */
