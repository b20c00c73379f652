/*
 * nmf.h -- C ABI of the MI355X (gfx950) E-A-HALS library.
 *
 * Problem (Ang & Gillis, arXiv 1805.06604, Eq. (1)):
 *     min ||X - W H||_F^2  over  W in R^{m x r}, H in R^{r x n},  W, H >= 0,
 * solved by Algorithm 2 (extrapolated two-block NMF) around accelerated HALS
 * (section 1: repeated closed-form row updates of H and column updates of W),
 * with the beta / beta-bar growth-and-restart rule of Algorithm 3 and the
 * error of Remark 1. Every outer iteration runs on the GPU; the host only
 * enqueues work.
 *
 * Conventions
 *   - Host matrices are row-major: X is m x n, W is m x r, H is r x n.
 *   - Every entry point returns nmf_status; no C++ exception crosses the ABI.
 *   - Arguments are validated before any device work; on an error no output
 *     is written and nmf_last_error() describes it.
 *   - A context is bound to the device that was current at nmf_create and is
 *     not thread-safe: use one per thread.
 *   - Streams are passed as `void *` holding a hipStream_t (NULL = the null
 *     stream).
 */
#ifndef NMF_H
#define NMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nmf_ctx nmf_ctx;

typedef enum {
    NMF_OK = 0,
    NMF_E_INVAL = 1,        /* an argument is out of its documented domain   */
    NMF_E_UNSUPPORTED = 2,  /* valid, but not supported by the library       */
    NMF_E_NOMEM = 3,        /* host or device allocation failed              */
    NMF_E_DEVICE = 4,       /* a HIP call failed                             */
    NMF_E_NUMERIC = 5,      /* the initial error e(0) is not finite          */
    NMF_E_STATE = 6,        /* call out of order (e.g. nmf_iterate before
                               nmf_start)                                    */
    NMF_PENDING = 7         /* not an error: the batched problem has not
                               finished yet                                  */
} nmf_status;

typedef enum { NMF_DENSE_ROWMAJOR = 0, NMF_CSR = 1 } nmf_format;

/* Storage type of X on the device. The values are rounded to this type once;
 * how the products then accumulate is set by nmf_prod below (exact integer
 * sums, FP64, or FP32 within a K-chunk), and the objective combination runs
 * in FP64 whatever this is. */
typedef enum { NMF_X_F32 = 0, NMF_X_BF16 = 1, NMF_X_F16 = 2 } nmf_xdtype;

/* How each block subproblem (the NNLS in H with W fixed, then in W with H
 * fixed) is solved. FIXED: A-HALS, inner_k HALS sweeps per block (section 1:
 * the rows of H are updated several times before W, reusing W^T W and W^T X),
 * giving E-A-HALS. EXACT: ANLS, every row's NNLS solved exactly by block
 * principal pivoting (section 1, the active-set method it cites) from the
 * extrapolated warm start, giving E-ANLS; inner_k is then ignored (it must
 * still lie in range). A coordinate with a zero Gram diagonal keeps its warm
 * start projected onto x >= 0; a singular passive-set system or the pivoting
 * cap of 10 r + 20 steps returns the last complete iterate projected onto
 * x >= 0.
 * ADAPTIVE: the inner loop of A-HALS as the cited A-HALS work sets it (the
 * paper only says the rows are updated several times; this rule is recalled
 * from that work): on the W side at most floor(1 + inner_alpha rho_W) sweeps,
 * rho_W = 1 + (mn + nr) / (m (r + 1)) the cost of forming X H^T and H H^T
 * over that of one sweep counted in flops (nnz for mn with sparse X), or
 * inner_rho_w when it is positive (a cost ratio measured on the device, say:
 * 1 + the side's X-pass time over one sweep's), also capped at inner_k;
 * after each sweep l >= 2 the loop stops once ||W^(l) - W^(l-1)||_F <=
 * inner_delta ||W^(1) - W^(0)||_F. The H side swaps m and n (and takes
 * inner_rho_h). Between sweeps
 * the factor is kept in FP64. The sweeps run per iteration can be read with
 * nmf_read_sweeps. ADAPTIVE is not available to batched solves. */
typedef enum { NMF_INNER_FIXED = 0, NMF_INNER_EXACT = 1, NMF_INNER_ADAPTIVE = 2 } nmf_inner;

/* How the two O(mnr) products X^T W and X H^T are computed. Whatever the
 * choice, the products are summed over K-chunks in FP64, and the HALS sweeps,
 * Grams and objective run in FP64 on FP32-stored W and H. MFMA_FAST needs
 * X stored in 16 bits (NMF_E_UNSUPPORTED for FP32 X and for sparse X).
 *   AUTO       : MFMA_EXACT for FP32 X, MFMA_FAST for BF16 and FP16 X.
 *   VALU       : FP64 FMA on the vector ALUs (exact products of the stored
 *                values, FP64 sums): the reference-accuracy path, slowest.
 *   MFMA_EXACT : integer matrix cores. X is stored as four int8 slices per
 *                entry with a power-of-two scale per row (4 bytes per entry,
 *                whatever x_dtype; the x_dtype-rounded values are sliced), the
 *                factor is sliced per column the same way, and the slice
 *                products are summed exactly in int32: products to about
 *                2^-27 of the row and column maxima, no rounding over K.
 *   MFMA_FAST  : 16-bit matrix cores of X's type (BF16 or FP16), X as
 *                stored and the factor split into two parts of that type
 *                once per product (FP16 parts scaled per column by a power
 *                of two), sums in FP32 within a K-chunk. X keeps its x_dtype
 *                storage (2 bytes per entry, which the product streams in its
 *                own fragment order). */
typedef enum {
    NMF_PROD_AUTO = 0,
    NMF_PROD_VALU = 1,
    NMF_PROD_MFMA_EXACT = 2,
    NMF_PROD_MFMA_FAST = 3
} nmf_prod;

/* Flags selecting the alternative readings of Algorithm 3 / Algorithm 2. */
#define NMF_FLAG_BETABAR_LAST_ACCEPTED 1  /* on a restart the upper bound becomes
                                             the beta of the last accepted
                                             iteration instead of beta_{k-1} */
#define NMF_FLAG_CMP_LAST_ACCEPTED 2      /* compare e(k) with the last
                                             accepted error instead of the
                                             previous computed one          */
#define NMF_FLAG_BETA_STAR 4              /* record the diagnostic beta* of
                                             section 4 every iteration (see
                                             nmf_read_beta_star); does not
                                             change the iterates            */

/* Input matrix (host memory; nmf_create copies it). */
typedef struct {
    int32_t fmt;                /* nmf_format                                   */
    int64_t m, n;               /* rows, columns; both >= 1                     */
    const float *dense;         /* DENSE: m*n row-major                         */
    const int64_t *row_ptr;     /* CSR: m+1 offsets, row_ptr[0] = 0             */
    const int32_t *col_idx;     /* CSR: column indices, strictly increasing per row */
    const float *val;           /* CSR: nnz values                              */
    int64_t nnz;                /* CSR: row_ptr[m]                              */
} nmf_matrix;

/* Parameters (Algorithm 2 and 3). nmf_params_default() fills the values of
 * section 5.3.2 for E-A-HALS: hp 3, beta0 0.5, eta 1.5, gamma 1.01,
 * gamma_bar 1.005, 10 inner sweeps, 100 iterations, FP32 X. */
typedef struct {
    int32_t r;                  /* rank, 1..64                                  */
    int32_t hp;                 /* 1, 2 or 3 (Algorithm 2)                      */
    double beta0;               /* beta of iteration 1, in [0, 1); 0 = A-HALS   */
    double gamma, gamma_bar, eta; /* 1 < gamma_bar < gamma < eta (Algorithm 3)  */
    int32_t inner_rule;         /* nmf_inner                                    */
    int32_t inner_k;            /* sweeps per block update, 1..1000             */
    int32_t max_iter;           /* outer iterations, >= 0                       */
    double tol;                 /* > 0: stop after an accepted iteration whose
                                   relative error moved by less than tol        */
    int32_t x_dtype;            /* nmf_xdtype                                   */
    int32_t prod;               /* nmf_prod                                     */
    int32_t flags;              /* NMF_FLAG_*                                   */
    double inner_alpha;         /* ADAPTIVE: cost-ratio weight, >= 0 (0.5)      */
    double inner_delta;         /* ADAPTIVE: stopping ratio, >= 0 (0.1)         */
    double inner_rho_h;         /* ADAPTIVE: cost ratio of the H side, finite,
                                   >= 0; 0 = the flop ratio (0)                 */
    double inner_rho_w;         /* ADAPTIVE: the same for the W side (0)        */
} nmf_params;

void nmf_params_default(nmf_params *p);

/* Validates X and p, uploads X (and the transposed copy the second product
 * streams), converts it to x_dtype and computes ||X||_F^2 in FP64 from the
 * given FP32 values. X may be freed once this returns.
 * Sparse X (NMF_CSR): the CSR arrays are copied, the CSC copy (the CSR form
 * of X^T) is built on the host, and both products run as sparse products
 * whose FP32 x FP32 terms are exact in FP64 and summed in FP64 in a fixed
 * order (rows are split into work items of bounded nonzeros, so a long row
 * costs like many short ones). Sparse X needs x_dtype = NMF_X_F32 and a
 * prod other than NMF_PROD_MFMA_FAST (NMF_E_UNSUPPORTED otherwise); prod is
 * otherwise ignored.
 * Errors: NMF_E_INVAL (shape, malformed CSR, non-finite X, all-zero X, any
 * parameter out of domain), NMF_E_UNSUPPORTED (r > 64; the sparse limits
 * above), NMF_E_NOMEM, NMF_E_DEVICE. On error *out is NULL. */
nmf_status nmf_create(const nmf_matrix *X, const nmf_params *p, nmf_ctx **out);

/* Synchronous solve (Algorithm 2, first step through max_iter iterations).
 * W0 (m*r) and H0 (r*n) are host arrays, finite and >= 0. Outputs, caller
 * allocated host arrays: W (m*r), H (r*n) = the last accepted iterate;
 * trace[0..*n_iter] = ||X - W_n H_y||_F / ||X||_F per iteration (trace[0]
 * is the initial error), trace_cap >= max_iter + 1; accepted and beta
 * (nullable) receive, for k = 1..*n_iter, 1 for an accepted iteration and 0
 * for a restart, and the beta used in iteration k.
 * Errors: NMF_E_INVAL (null or non-finite / negative W0 or H0, small
 * trace_cap), NMF_E_NUMERIC (e(0) not finite), NMF_E_DEVICE. */
nmf_status nmf_solve(nmf_ctx *ctx, const float *W0, const float *H0, float *W,
                     float *H, double *trace, int32_t trace_cap,
                     int32_t *n_iter, uint8_t *accepted, double *beta);

/* Asynchronous interface for callers that own device memory and streams.
 *
 * nmf_start: loads W0 (m*r) and H0 (r*n), from the host (on_device = 0) or
 * from device memory (on_device = 1), resets the beta state and enqueues the
 * computation of e(0) on `stream`. It synchronizes `stream` once to check the
 * inputs and e(0). Errors as for nmf_solve.
 *
 * nmf_iterate: enqueues `iters` outer iterations on `stream` and returns
 * without waiting. Iterations past max_iter, or after the tol stop, do
 * nothing. With NMF_INNER_EXACT, part of each iteration (the inverse of each
 * Gram matrix) runs on a stream of the context, forked from `stream` and
 * joined back within the iteration, so every iteration still starts after
 * the work enqueued on `stream` before it and ends before the work enqueued
 * after it. Errors: NMF_E_STATE before nmf_start, NMF_E_INVAL for iters < 0.
 *
 * nmf_read: waits for `stream`, then copies the last accepted W (m*r) and H
 * (r*n) into host (on_device = 0) or device (on_device = 1) arrays, and the
 * trace, decisions and betas into host arrays (each nullable). */
nmf_status nmf_start(nmf_ctx *ctx, const float *W0, const float *H0,
                     int32_t on_device, void *stream);
nmf_status nmf_iterate(nmf_ctx *ctx, int32_t iters, void *stream);
nmf_status nmf_read(nmf_ctx *ctx, float *W, float *H, int32_t on_device,
                    double *trace, int32_t trace_cap, int32_t *n_iter,
                    uint8_t *accepted, double *beta, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of nmf_create + nmf_solve for dense FP32 X with the exact-integer products
 * and the fixed inner rule, given and returning device arrays only, with no
 * device allocation at all. Its working buffers (the int8 slices of X and
 * X^T, the factor slots, Grams, partial products, the solver state) are
 * carved from one static device array of 128 MiB held by the library on each
 * GPU it runs on until the process ends (a solve needs about 16 m n bytes
 * for X and its copies plus the factor and product buffers, e.g. 95 MiB at
 * m = n = 2048, r = 40; larger problems are refused with NMF_E_NOMEM). Results are
 * those of nmf_solve on the same input, bit for bit.
 *   X (m*n, row-major), W0 (m*r), H0 (r*n): device inputs (W0, H0 >= 0).
 *   W (m*r), H (r*n): device outputs, the last accepted iterate.
 *   trace (device, >= max_iter + 1 doubles): rho(0..n_iter) as for nmf_solve;
 *   accepted (device, >= max_iter bytes) and beta (device, >= max_iter
 *   doubles) are nullable. info (device, 2 int32): info[0] = NMF_OK, or
 *   NMF_E_INVAL for a zero or non-finite X or a negative or non-finite W0 or
 *   H0, or NMF_E_NUMERIC for a non-finite e(0) (no iteration runs then);
 *   info[1] = the completed iterations.
 * Every step is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 * and the call returns without waiting; the outputs are valid once the
 * stream reaches them. Every call on a GPU uses that GPU's one array, and
 * the array keeps the last call's contents: calls that overlap on one GPU
 * (other streams, other threads) race and must be ordered by the caller.
 * Errors (returned, nothing enqueued): NMF_E_INVAL (parameters, NULL
 * pointers, m or n < 1), NMF_E_UNSUPPORTED (other x_dtype, prod or inner
 * rule; flags other than the two readings), NMF_E_NOMEM (beyond the static
 * array), NMF_E_DEVICE. Messages: nmf_last_error(NULL). */
nmf_status nmf_solve_noalloc(const float *X, int64_t m, int64_t n, const nmf_params *p,
                             const float *W0, const float *H0, float *W, float *H,
                             double *trace, uint8_t *accepted, double *beta, int32_t *info,
                             void *stream);

/* Checkpoint and resume. The state of a started solve between outer
 * iterations (the accepted iterate, the warm starts and the iterate slots,
 * their Gram matrices, the beta / beta-bar state and the errors the next
 * test of Algorithm 2 compares with, the iteration count, and the trace,
 * decisions and betas so far) as one host byte array, which a context of
 * the same problem and parameters (same X, r and nmf_params, max_iter
 * included) loads to continue the solve: nmf_iterate after nmf_load_state
 * reproduces the uninterrupted solve bit for bit. The array also records
 * whether the tol rule had stopped the solve.
 * nmf_state_size: the array's length for ctx.
 * nmf_save_state: waits for `stream` and the device, then writes the state
 * after the last completed iteration into buf (cap >= the size).
 * nmf_load_state: checks that buf was saved by this library for the same
 * shape, ||X||_F^2, r and parameters, then makes it the context's state on
 * `stream` (synchronized before returning); nmf_start is not needed.
 * Errors: NMF_E_INVAL (NULL pointers, small cap, a state of another
 * problem, parameters or version, a truncated array), NMF_E_STATE
 * (nmf_save_state before nmf_start), NMF_E_DEVICE. */
nmf_status nmf_state_size(nmf_ctx *ctx, size_t *bytes);
nmf_status nmf_save_state(nmf_ctx *ctx, void *buf, size_t cap, void *stream);
nmf_status nmf_load_state(nmf_ctx *ctx, const void *buf, size_t len, void *stream);

/* Test hook of the restart branch of Algorithm 2 (reading: a non-finite
 * e(k) is a restart and does not replace the previous error; a non-finite
 * e(0) is NMF_E_NUMERIC). From the next nmf_start (or nmf_solve) on, the
 * squared error e(k)^2 of iteration k is multiplied by scale[k] for
 * k < count before it is tested (k = 0: e(0)); a NaN or infinite factor
 * forces the non-finite branch, a large one a forced increase. The host
 * array is copied (count doubles); count = 0 removes the hook. The
 * iterates themselves are not touched. Synchronizes the device.
 * Errors: NMF_E_INVAL (count < 0, or scale NULL with count > 0),
 * NMF_E_DEVICE. */
nmf_status nmf_set_error_scale(nmf_ctx *ctx, const double *scale, int32_t count);

/* Kernels of one outer iteration, in launch order (the phases timed by
 * nmf_profile). The slicing phases run only with the exact-integer products
 * (NMF_PROD_MFMA_EXACT); otherwise they take no time. */
enum nmf_phase {
    NMF_PHASE_SLICE_W = 0,   /* W_y into int8 slices (operand of X^T W_y) */
    NMF_PHASE_PROD_CT = 1,   /* C^T = X^T W_y */
    NMF_PHASE_SWEEP_H = 2,   /* H sweeps, extrapolation, partial Grams */
    NMF_PHASE_FINISH_H = 3,  /* Gram of H_w, its inverse diagonal and column maxima */
    NMF_PHASE_SLICE_H = 4,   /* H_w into int8 slices (operand of X H_w^T) */
    NMF_PHASE_PROD_A = 5,    /* A = X H_w^T */
    NMF_PHASE_SWEEP_W = 6,   /* W sweeps, extrapolation, partial Grams, <W_n, A> */
    NMF_PHASE_FINISH_W = 7,  /* Grams of W_n and W_y', then e(k), accept/restart,
                                beta (two launches) */
    NMF_PHASE_COUNT = 8
};

/* Per-kernel timing. Runs `iters` further outer iterations (they advance the
 * solve like nmf_iterate, within max_iter) launched one kernel at a time on
 * `stream`, with a HIP event recorded on `stream` before and after each
 * kernel, waits for them, and writes the average duration in milliseconds of
 * each phase to ms[0 .. NMF_PHASE_COUNT - 1] (enum nmf_phase).
 * Errors: NMF_E_STATE before nmf_start, NMF_E_INVAL (iters < 1, ms NULL, or
 * fewer than iters iterations left before max_iter), NMF_E_DEVICE. */
nmf_status nmf_profile(nmf_ctx *ctx, int32_t iters, void *stream, double *ms);

/* Sweeps of the inner loop run in each completed iteration: sweeps[2(k-1)]
 * on H and sweeps[2(k-1)+1] on W for k = 1..*n_iter (inner_k for FIXED, the
 * counts of the adaptive loop for ADAPTIVE, 0 for EXACT). sweeps may be NULL
 * (then only *n_iter is set); cap is its length in pairs. Synchronizes the
 * device. Errors: NMF_E_INVAL (NULL ctx, cap < *n_iter), NMF_E_STATE (no
 * successful nmf_start), NMF_E_DEVICE. */
nmf_status nmf_read_sweeps(nmf_ctx *ctx, int32_t *sweeps, int32_t cap, int32_t *n_iter);

/* The diagnostic of section 4: for each iteration k = 1..*n_iter, the beta
 * that would have minimized ||X - (W_n + beta (W_n - W)) H_w||_F, i.e.
 * beta* = <X H_w^T - W_n H_w H_w^T, W_n - W> / <(W_n - W)^T (W_n - W),
 * H_w H_w^T>, from the W_n, W (last accepted) and H_w of that iteration (0
 * when the denominator vanishes), into a host array of capacity cap.
 * Errors: NMF_E_STATE unless the context was created with
 * NMF_FLAG_BETA_STAR and started; NMF_E_INVAL for a small cap. */
nmf_status nmf_read_beta_star(nmf_ctx *ctx, double *beta_star, int32_t cap, int32_t *n_iter);

/* ------------------------------------------------------------------------
 * Batched solves (serving many independent small problems on one GPU).
 *
 * A batch holds a fixed device-memory arena (hbm_budget bytes, allocated at
 * nmf_batch_create) and runs continuous batching: every problem admitted
 * into the arena advances by one outer iteration of Algorithm 2 per batch
 * iteration, all problems of one padded rank sharing each kernel launch
 * (grouped launches); problems join when they fit the arena and leave when
 * they stop (max_iter or the tol rule), between batch iterations. Each
 * problem follows exactly the single-problem algorithm with the exact-integer
 * products (dense FP32 X only).
 * ------------------------------------------------------------------------ */
typedef struct nmf_batch nmf_batch;

typedef struct {
    int64_t hbm_budget;     /* bytes of device memory for the problems, > 0    */
    int32_t max_active;     /* problems advanced together, 1..4096             */
    int32_t check_every;    /* batch iterations between completion checks, >= 1 */
} nmf_batch_params;

/* Errors: NMF_E_INVAL (parameters), NMF_E_NOMEM (the arena), NMF_E_DEVICE.
 * Messages of batch calls: nmf_last_error(NULL). */
nmf_status nmf_batch_create(const nmf_batch_params *bp, nmf_batch **out);

/* Queues one problem: dense FP32 X (m x n), parameters (x_dtype F32; prod is
 * taken as NMF_PROD_MFMA_EXACT), W0 (m*r), H0 (r*n) host arrays, validated
 * as for nmf_create / nmf_solve and copied (the caller may free them on
 * return). *ticket identifies the problem. Nothing runs on the device until
 * nmf_batch_step. Errors: as nmf_create, plus NMF_E_NOMEM if the problem
 * alone exceeds the arena, NMF_E_UNSUPPORTED for CSR X or 16-bit storage. */
nmf_status nmf_batch_submit(nmf_batch *b, const nmf_matrix *X, const nmf_params *p,
                            const float *W0, const float *H0, int64_t *ticket);

/* Admits queued problems in submission order while the arena and max_active
 * allow, runs `iters` batch iterations (check_every at a time, retiring the
 * problems that stopped after each check; a retired problem's result is kept
 * on the host), and returns the numbers of active (admitted ones included),
 * queued and retired-unread problems (each pointer nullable). The set-up of
 * problems admitted while a chunk runs overlaps it; they join at the next
 * chunk. The last chunk of the call is left running on the device when the
 * call returns, so that the caller's own work (submissions, reading results)
 * overlaps it; the next call (or nmf_batch_destroy) waits for it first and
 * retires the problems it finished, so a result can appear one call later.
 * Each chunk is one replay of a graph per padded rank, captured once.
 * Errors: NMF_E_INVAL (iters < 1), NMF_E_DEVICE. */
nmf_status nmf_batch_step(nmf_batch *b, int32_t iters, int32_t *active, int32_t *queued,
                          int32_t *retired);

/* Result of a retired problem into host arrays (each nullable): W (m*r),
 * H (r*n), trace[0..*n_iter] (trace_cap >= *n_iter + 1), and for
 * k = 1..*n_iter the decision (1 accept, 0 restart) and the beta of
 * iteration k; then the problem is forgotten. NMF_PENDING while the problem
 * is queued or active; NMF_E_INVAL for an unknown ticket or a small
 * trace_cap. */
nmf_status nmf_batch_result(nmf_batch *b, int64_t ticket, float *W, float *H, double *trace,
                            int32_t trace_cap, int32_t *n_iter, uint8_t *accepted,
                            double *beta);

/* Frees the arena and every pending problem. NULL is allowed. Waits for the
 * device work of the batch first.
 * Threads: nmf_batch_submit and nmf_batch_result may be called from other
 * threads while nmf_batch_step runs (a serving loop stepping the batch while
 * requests are submitted); calls of nmf_batch_step must not overlap one
 * another, and nmf_batch_destroy must not overlap any call. */
void nmf_batch_destroy(nmf_batch *b);

/* Frees every host and device resource of ctx. NULL is allowed. */
void nmf_destroy(nmf_ctx *ctx);

/* Message of the last failure on ctx, or of the last failed nmf_create on
 * this thread when ctx is NULL. Never NULL. */
const char *nmf_last_error(const nmf_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* NMF_H */
