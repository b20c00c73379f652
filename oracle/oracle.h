/*
 * FP64 reference implementation of extrapolated accelerated HALS (E-A-HALS),
 * Ang & Gillis, "Accelerating Nonnegative Matrix Factorization Algorithms
 * using Extrapolation" (arXiv 1805.06604).
 *
 * TEST INFRASTRUCTURE ONLY. This library is the oracle that the GPU path is
 * checked against. It is plain, single-threaded, double-precision C with
 * fixed summation orders, no BLAS and no fast-math. Only the test suite, the
 * smoke check and the CPU baseline of the benchmark may load it; the GPU
 * library never links or calls it, and the two share no code.
 *
 * Layouts: X is m x n (dense row-major, or CSR with sorted column indices),
 * W is m x r row-major, H is r x n row-major (the paper's notation).
 *
 * Readings of the paper that this code takes (numbered like the list of
 * readings kept with the design notes):
 *   R1  H is r x n (the REQUIRE lines of Algorithms 1 and 2 print m x r).
 *   R2  Alg. 3 sets beta_{k+1} = beta_k / eta on an increase (its printed
 *       line duplicates the left-hand side).
 *   R3  The upper bound grows by gamma_bar on a decrease (Alg. 3; the
 *       prose of section 4 prints gamma there).
 *   R4  beta0 is the beta used in outer iteration 1; the upper bound starts
 *       at 1 once per solve (section 4, first paragraph after Alg. 3).
 *   R5  On an increase the upper bound becomes the beta used in iteration
 *       k-1 (for k = 1: beta0). ORACLE_BETABAR_LAST_ACCEPTED instead uses
 *       the beta of the most recent accepted iteration.
 *   R6  For hp = 1 the W update and e(k) use H_n; H_y = H_n + beta (H_n - H)
 *       is only the warm start of the next H update (section 3, "When
 *       should we perform the extrapolation?").
 *   R7  e(k) is compared with the previous computed finite e, accepted or
 *       not; ORACLE_CMP_LAST_ACCEPTED compares with the last accepted e.
 *   R8  Equality accepts (the test of Alg. 2 is a strict ">").
 *   R9  A non-finite e(k) is a restart and does not replace the previous e;
 *       a non-finite e(0) is an error (ORACLE_ENUMERIC). e is sqrt(max(0,
 *       e^2)) only for a finite e^2 (Remark 1 can round below zero); a NaN
 *       e^2 gives a NaN e and an infinite one +inf, never 0.
 *   R10 A HALS coordinate whose denominator ||W(:,k)||^2 (or ||H(k,:)||^2)
 *       is zero does not enter the objective: it is only projected onto
 *       [0, inf) (kept when already >= 0; the warm start may be negative).
 *       Rows/columns are visited in ascending k.
 *   R11 The output is the last accepted (W, H).
 *   R12 tol > 0 stops after an accepted iteration k with
 *       |rho(k) - rho(k-1)| < tol; rho = e / ||X||_F.
 *   R13 The inner NNLS runs a fixed number K of HALS sweeps per block.
 *   R17 Exact NNLS (E-ANLS): a coordinate whose Gram diagonal is zero does
 *       not enter the objective and keeps max(0, warm start), as in R10. A
 *       singular passive-set system or the pivoting step cap (10 r + 20)
 *       ends the solve with the last complete iterate projected onto x >= 0.
 *   R18 Adaptive inner loop (the A-HALS rule the paper cites for "several
 *       times", not stated in the paper itself; parity unpinned against
 *       the paper): on the W side at most floor(1 + alpha rho_W) sweeps,
 *       rho_W = 1 + (mn + nr) / (m (r + 1)) (the cost of forming X H^T and
 *       H H^T over that of one sweep, counted in flops), or the caller's
 *       cost ratio of the side when given, capped at inner_k; stop after sweep
 *       l >= 2 once ||W^(l) - W^(l-1)||_F <= delta ||W^(1) - W^(0)||_F. The H
 *       side swaps m and n. Sparse X uses nnz for mn.
 *   R16 The diagnostic beta* of section 4 (the beta minimizing
 *       ||X - (W_n + beta (W_n - W)) H_w||_F) is 0 when (W_n - W) H_w = 0.
 */
#ifndef NMF_ORACLE_H
#define NMF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_OK       0
#define ORACLE_EINVAL   1
#define ORACLE_ENUMERIC 2
#define ORACLE_ENOMEM   3

#define ORACLE_BETABAR_LAST_ACCEPTED 1  /* R5 alternative */
#define ORACLE_CMP_LAST_ACCEPTED     2  /* R7 alternative */
#define ORACLE_ERR_REMARK1           4  /* e(k) by Remark 1 instead of the explicit residual */
#define ORACLE_ROUND_F32             8  /* round the stored iterates W_n, H_n, W_y, H_y
                                           to FP32 after each update (conditioning
                                           probe; all arithmetic stays FP64)       */
#define ORACLE_ROUND_F32_RZ         64  /* the same probe with rounding toward
                                           zero (a second, independent
                                           perturbation of the same size)     */
#define ORACLE_ADAPTIVE_INNER       32  /* adaptive A-HALS inner loop (R18) instead of
                                           inner_k sweeps                          */
#define ORACLE_EXACT_NNLS           16  /* E-ANLS: solve each NNLS block exactly
                                           (block principal pivoting) instead of
                                           inner_k HALS sweeps                     */

typedef struct {
    int64_t m, n;
    const double  *dense;    /* m*n row-major, or NULL for CSR          */
    const int64_t *row_ptr;  /* CSR: m+1 offsets                        */
    const int32_t *col_idx;  /* CSR: sorted, unique per row             */
    const double  *val;      /* CSR: nonzero values                     */
} oracle_matrix;

/* The state of a solve between outer iterations (checkpoint / resume).
 * The arrays are caller-allocated: W, Wy m*r; H, Hy r*n. */
typedef struct {
    int     k;                /* completed outer iterations               */
    double *W, *H;            /* last accepted iterate                    */
    double *Wy, *Hy;          /* warm starts of iteration k + 1           */
    double  beta, betabar, beta_prev, beta_acc;   /* Alg. 3 state         */
    double  e_prev, e_acc;    /* errors the next test compares with (R7)  */
    double  rho;              /* rho(k), for the tol rule (R12)           */
} oracle_state;

typedef struct {
    int    hp;                /* 1, 2 or 3 (Alg. 2)                       */
    double beta0, gamma, gamma_bar, eta;  /* Alg. 3                         */
    int    inner_k;           /* HALS sweeps per block update (R13)       */
    int    max_iter;
    double tol;               /* R12; 0 disables                          */
    int    flags;             /* ORACLE_* flags above                     */
    const uint8_t *replay;    /* NULL, or max_iter forced decisions
                                 (1 accept, 0 restart): decision replay   */
    double inner_alpha;       /* R18 (ORACLE_ADAPTIVE_INNER): cost-ratio    */
    double inner_delta;       /*   weight alpha and stopping ratio delta    */
    const int *sweeps_replay; /* NULL, or 2 max_iter forced sweep counts
                                 (H, W per iteration) for the adaptive loop */
    const double *e2_scale;   /* test hook, NULL or e2_scale_n factors:
                                 e(k)^2 is multiplied by e2_scale[k] before
                                 the test of Alg. 2 (k = 0: e(0)); a NaN or
                                 infinite factor drives the non-finite
                                 branch of R9                              */
    int e2_scale_n;
    const oracle_state *resume; /* NULL, or a state saved by an earlier solve
                                 of the same problem and parameters: the
                                 solve continues with iteration resume->k + 1
                                 (trace[0..k] are left as they are)       */
    oracle_state *save;       /* NULL, or receives the state at the end     */
    double inner_rho_h;       /* R18: the cost ratios rho_H, rho_W of the  */
    double inner_rho_w;       /*   sweep caps when > 0 (a measured cost of  */
                              /*   the side's X pass over one sweep, say);  */
                              /*   0 takes the flop ratio                   */
} oracle_params;

/* Full solve (Alg. 2 with Alg. 3). Outputs, all caller-allocated:
 *   sweeps[2(k-1)], sweeps[2(k-1)+1]: HALS sweeps run on H and on W in
 *   iteration k (inner_k, the adaptive count of R18, or 0 for E-ANLS), and
 *   sweep_margin[.]: the closest call of that side's stopping tests,
 *   min |d_l / (delta d_1) - 1| (infinity when none was made);
 *   W (m*r), H (r*n): last accepted iterate;
 *   trace[0..n_iter]: rho(k) = e(k)/||X||_F (capacity max_iter+1);
 *   accepted[k-1], beta_used[k-1], margin[k-1] for k = 1..n_iter, where
 *   margin = (e(k) - e_compared)/||X||_F, and beta_star[k-1], the beta* of
 *   section 4 for the W_n, W and H_w of iteration k (see oracle_beta_star);
 *   each may be NULL.
 * Returns ORACLE_OK, ORACLE_EINVAL or ORACLE_ENUMERIC. */
int oracle_eahals(const oracle_matrix *X, int r, const double *W0,
                  const double *H0, const oracle_params *p, double *W,
                  double *H, double *trace, uint8_t *accepted,
                  double *beta_used, double *margin, int *n_iter,
                  double *beta_star, int *sweeps, double *sweep_margin);

/* Section 4: beta* = argmin_beta ||X - (Wn + beta (Wn - W)) Hw||_F^2 =
 * <X Hw^T - Wn Hw Hw^T, Wn - W> / <(Wn - W)^T (Wn - W), Hw Hw^T> (R16: 0 when
 * the denominator is 0). Wn, W: m*r; Hw: r*n. NaN on invalid input. */
double oracle_beta_star(const oracle_matrix *X, int r, const double *Wn,
                        const double *W, const double *Hw);

/* H-side NNLS by HALS: starting from H (r*n, in/out), run `sweeps` sweeps of
 * the closed-form row updates for min_{H>=0} ||X - W H||_F. */
int oracle_nnls_h(const oracle_matrix *X, int r, const double *W, double *H,
                  int sweeps);

/* Exact NNLS blocks (E-ANLS): every column of H (r*n, in: warm start, out:
 * solution) given W, or every row of W (m*r) given H, by block principal
 * pivoting (R17 for zero Gram diagonals). */
int oracle_nnls_exact_h(const oracle_matrix *X, int r, const double *W, double *H);
int oracle_nnls_exact_w(const oracle_matrix *X, int r, const double *H, double *W);

/* W-side NNLS by HALS: W (m*r, in/out), H fixed. */
int oracle_nnls_w(const oracle_matrix *X, int r, const double *H, double *W,
                  int sweeps);

/* Alg. 3 run on a scripted sequence of outcomes: decreased[k-1] for
 * k = 1..count. Writes the beta used in iteration k and the upper bound
 * after iteration k. */
void oracle_beta_script(int count, const uint8_t *decreased, double beta0,
                        double gamma, double gamma_bar, double eta, int flags,
                        double *beta_used, double *betabar_after);

/* ||X - W H||_F / ||X||_F, explicit. */
double oracle_rel_error(const oracle_matrix *X, int r, const double *W,
                        const double *H);

/* The same quantity by the identity of Remark 1. */
double oracle_rel_error_remark1(const oracle_matrix *X, int r, const double *W,
                                const double *H);

#ifdef __cplusplus
}
#endif
#endif
