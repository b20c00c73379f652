/*
 * FP64 oracle for extrapolated accelerated HALS (E-A-HALS), arXiv 1805.06604.
 * TEST INFRASTRUCTURE ONLY: see oracle.h for the contract and the readings.
 *
 * Every routine is a plain loop nest in double precision, single threaded,
 * with a fixed summation order. Nothing here is blocked, fused or reordered
 * beyond what the paper's formulas state.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- products */

static int is_csr(const oracle_matrix *X) { return X->dense == NULL; }

/* ||X||_F^2 (Remark 1: computed once). */
static double frob2(const oracle_matrix *X)
{
    double s = 0.0;
    if (!is_csr(X)) {
        for (int64_t i = 0; i < X->m * X->n; ++i) s += X->dense[i] * X->dense[i];
    } else {
        for (int64_t p = 0; p < X->row_ptr[X->m]; ++p) s += X->val[p] * X->val[p];
    }
    return s;
}

/* C = W^T X (r x n): the linear term of the H update (section 1). */
static void wt_x(const oracle_matrix *X, int r, const double *W, double *C)
{
    const int64_t m = X->m, n = X->n;
    memset(C, 0, sizeof(double) * (size_t)r * (size_t)n);
    for (int64_t i = 0; i < m; ++i) {
        if (!is_csr(X)) {
            const double *xi = X->dense + i * n;
            for (int k = 0; k < r; ++k) {
                const double w = W[i * r + k];
                double *ck = C + (int64_t)k * n;
                for (int64_t j = 0; j < n; ++j) ck[j] += w * xi[j];
            }
        } else {
            for (int64_t p = X->row_ptr[i]; p < X->row_ptr[i + 1]; ++p) {
                const int64_t j = X->col_idx[p];
                for (int k = 0; k < r; ++k)
                    C[(int64_t)k * n + j] += W[i * r + k] * X->val[p];
            }
        }
    }
}

/* A = X H^T (m x r): the linear term of the W update (Remark 1). */
static void x_ht(const oracle_matrix *X, int r, const double *H, double *A)
{
    const int64_t m = X->m, n = X->n;
    for (int64_t i = 0; i < m; ++i) {
        for (int k = 0; k < r; ++k) {
            const double *hk = H + (int64_t)k * n;
            double s = 0.0;
            if (!is_csr(X)) {
                const double *xi = X->dense + i * n;
                for (int64_t j = 0; j < n; ++j) s += xi[j] * hk[j];
            } else {
                for (int64_t p = X->row_ptr[i]; p < X->row_ptr[i + 1]; ++p)
                    s += X->val[p] * hk[X->col_idx[p]];
            }
            A[i * r + k] = s;
        }
    }
}

/* G = W^T W (r x r), W m x r. */
static void gram_cols(int64_t m, int r, const double *W, double *G)
{
    for (int k = 0; k < r; ++k)
        for (int l = 0; l < r; ++l) {
            double s = 0.0;
            for (int64_t i = 0; i < m; ++i) s += W[i * r + k] * W[i * r + l];
            G[k * r + l] = s;
        }
}

/* B = H H^T (r x r), H r x n. */
static void gram_rows(int64_t n, int r, const double *H, double *B)
{
    for (int k = 0; k < r; ++k)
        for (int l = 0; l < r; ++l) {
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) s += H[k * n + j] * H[l * n + j];
            B[k * r + l] = s;
        }
}

/* ------------------------------------------------------------- HALS sweeps */

/* One pass over the rows of H, each replaced by its exact minimizer with the
 * other rows fixed (the closed form of section 1):
 *   H(k,:) = max(0, (C(k,:) - sum_{j != k} G(k,j) H(j,:)) / G(k,k)),
 * with C = W^T X and G = W^T W. Rows are visited in ascending k and the
 * updated rows are used at once (Gauss-Seidel). A zero G(k,k) means row k
 * does not enter the objective: it is only projected onto H(k,:) >= 0 (R10). */
static void project_row(int64_t len, double *v)
{
    for (int64_t i = 0; i < len; ++i)
        if (!(v[i] >= 0.0)) v[i] = 0.0;
}

static void hals_rows_h(int64_t n, int r, const double *C, const double *G,
                        double *H)
{
    for (int k = 0; k < r; ++k) {
        const double d = G[k * r + k];
        if (!(d > 0.0)) {
            project_row(n, H + (int64_t)k * n);
            continue;
        }
        for (int64_t c = 0; c < n; ++c) {
            double num = C[(int64_t)k * n + c];
            for (int j = 0; j < r; ++j)
                if (j != k) num -= G[k * r + j] * H[(int64_t)j * n + c];
            const double v = num / d;
            H[(int64_t)k * n + c] = v > 0.0 ? v : 0.0;
        }
    }
}

/* The same for the columns of W, by the symmetry ||X - WH|| = ||X^T - H^T W^T||:
 *   W(:,k) = max(0, (A(:,k) - sum_{j != k} W(:,j) B(j,k)) / B(k,k)),
 * with A = X H^T and B = H H^T. */
static void hals_cols_w(int64_t m, int r, const double *A, const double *B,
                        double *W)
{
    for (int k = 0; k < r; ++k) {
        const double d = B[k * r + k];
        if (!(d > 0.0)) {
            for (int64_t i = 0; i < m; ++i)
                if (!(W[i * r + k] >= 0.0)) W[i * r + k] = 0.0;
            continue;
        }
        for (int64_t i = 0; i < m; ++i) {
            double num = A[i * r + k];
            for (int j = 0; j < r; ++j)
                if (j != k) num -= W[i * r + j] * B[j * r + k];
            const double v = num / d;
            W[i * r + k] = v > 0.0 ? v : 0.0;
        }
    }
}

/* ------------------------------------------------------- exact NNLS (ANLS) */

/* Solves M z = b for the symmetric positive definite p x p matrix M (row
 * stride p) by Cholesky factorization; M and b are overwritten. Returns 0 if
 * a pivot is not positive (M not positive definite). */
static int chol_solve(int p, double *M, double *b)
{
    for (int k = 0; k < p; ++k) {
        double d = M[k * p + k];
        for (int j = 0; j < k; ++j) d -= M[k * p + j] * M[k * p + j];
        if (!(d > 0.0)) return 0;
        d = sqrt(d);
        M[k * p + k] = d;
        for (int i = k + 1; i < p; ++i) {
            double v = M[i * p + k];
            for (int j = 0; j < k; ++j) v -= M[i * p + j] * M[k * p + j];
            M[i * p + k] = v / d;
        }
    }
    for (int i = 0; i < p; ++i) {            /* L y = b */
        double v = b[i];
        for (int j = 0; j < i; ++j) v -= M[i * p + j] * b[j];
        b[i] = v / M[i * p + i];
    }
    for (int i = p - 1; i >= 0; --i) {       /* L^T z = y */
        double v = b[i];
        for (int j = i + 1; j < p; ++j) v -= M[j * p + i] * b[j];
        b[i] = v / M[i * p + i];
    }
    return 1;
}

/* One exact NNLS problem, min 1/2 x^T G x - c^T x over x >= 0 (G: r x r
 * symmetric positive semidefinite), by block principal pivoting (the
 * active-set method that section 1 cites for ANLS): the passive set F starts
 * from the support of the warm start x; each step solves the unconstrained
 * problem on F and exchanges the coordinates that violate x_F >= 0 or
 * y = G x - c >= 0 off F: all of them while the count of violations keeps
 * dropping (or at most 3 times without progress), else only the largest
 * index. Reading R17: a coordinate with G_kk = 0 does not enter the
 * objective and keeps max(0, x_k); if a passive-set system is singular or the
 * step cap is reached, the last complete iterate (initially the projected warm
 * start) is returned, projected onto x >= 0. work: r*r + r doubles. */
static void nnls_bpp(int r, const double *G, const double *c, double *x, double *work)
{
    double *M = work, *b = M + r * r;
    double x0[r], y[r];
    int F[r], map[r];
    for (int k = 0; k < r; ++k) {
        x0[k] = x[k] > 0.0 ? x[k] : 0.0;
        F[k] = (G[k * r + k] > 0.0) && x[k] > 0.0;
        x[k] = x0[k];
    }
    int alpha = 3, best = r + 1;
    for (int it = 0; it < 10 * r + 20; ++it) {
        /* x_F from G_FF x_F = c_F; x = 0 off F (R17 coordinates keep x0). */
        int p = 0;
        for (int k = 0; k < r; ++k)
            if (F[k]) map[p++] = k;
        for (int i = 0; i < p; ++i) {
            for (int j = 0; j < p; ++j) M[i * p + j] = G[map[i] * r + map[j]];
            b[i] = c[map[i]];
        }
        if (p > 0 && !chol_solve(p, M, b)) break;
        for (int k = 0; k < r; ++k) x[k] = (G[k * r + k] > 0.0) ? 0.0 : x0[k];
        for (int i = 0; i < p; ++i) x[map[i]] = b[i];
        int nv = 0, vmax = -1;
        for (int k = 0; k < r; ++k) {
            y[k] = 0.0;
            if (!(G[k * r + k] > 0.0)) continue;
            if (!F[k]) {
                double g = -c[k];
                for (int j = 0; j < r; ++j) g += G[k * r + j] * x[j];
                y[k] = g;
            }
            if ((F[k] && x[k] < 0.0) || (!F[k] && y[k] < 0.0)) {
                ++nv;
                vmax = k;
            }
        }
        if (nv == 0) break;
        if (nv < best || alpha > 0) {
            if (nv < best) {
                best = nv;
                alpha = 3;
            } else {
                --alpha;
            }
            for (int k = 0; k < r; ++k)
                if (G[k * r + k] > 0.0 && ((F[k] && x[k] < 0.0) || (!F[k] && y[k] < 0.0)))
                    F[k] = !F[k];
        } else {
            F[vmax] = !F[vmax];
        }
    }
    for (int k = 0; k < r; ++k)
        if (x[k] < 0.0) x[k] = 0.0;
}

/* Exact NNLS of every column of H (r x n) given C = W^T X and G = W^T W. */
static void exact_rows_h(int64_t n, int r, const double *C, const double *G, double *H,
                         double *work)
{
    double c[r], x[r];
    for (int64_t j = 0; j < n; ++j) {
        for (int k = 0; k < r; ++k) {
            c[k] = C[(int64_t)k * n + j];
            x[k] = H[(int64_t)k * n + j];
        }
        nnls_bpp(r, G, c, x, work);
        for (int k = 0; k < r; ++k) H[(int64_t)k * n + j] = x[k];
    }
}

/* Exact NNLS of every row of W (m x r) given A = X H^T and B = H H^T. */
static void exact_cols_w(int64_t m, int r, const double *A, const double *B, double *W,
                         double *work)
{
    for (int64_t i = 0; i < m; ++i) nnls_bpp(r, B, A + i * r, W + i * r, work);
}

/* ------------------------------------------------------------------ errors */

static double explicit_err2(const oracle_matrix *X, int r, const double *W,
                            const double *H)
{
    const int64_t m = X->m, n = X->n;
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        int64_t p = is_csr(X) ? X->row_ptr[i] : 0;
        const int64_t pend = is_csr(X) ? X->row_ptr[i + 1] : 0;
        for (int64_t j = 0; j < n; ++j) {
            double x = 0.0;
            if (!is_csr(X)) {
                x = X->dense[i * n + j];
            } else if (p < pend && X->col_idx[p] == j) {
                x = X->val[p];
                ++p;
            }
            double wh = 0.0;
            for (int k = 0; k < r; ++k) wh += W[i * r + k] * H[(int64_t)k * n + j];
            const double d = x - wh;
            s += d * d;
        }
    }
    return s;
}

/* Remark 1: ||X - WH||^2 = ||X||^2 - 2 <W, X H^T> + <W^T W, H H^T>, given
 * A = X H^T and B = H H^T. Clamped at 0 before the square root. */
static double remark1_err2(int64_t m, int r, double nx2, const double *W,
                           const double *A, const double *B)
{
    double s1 = 0.0;
    for (int64_t i = 0; i < m * r; ++i) s1 += W[i] * A[i];
    double *G = (double *)malloc(sizeof(double) * (size_t)r * (size_t)r);
    gram_cols(m, r, W, G);
    double s2 = 0.0;
    for (int i = 0; i < r * r; ++i) s2 += G[i] * B[i];
    free(G);
    return nx2 - 2.0 * s1 + s2;
}

/* e from e^2 (R9): the Remark-1 combination can round slightly below zero,
 * which is clamped to 0; a non-finite e^2 stays non-finite (NaN stays NaN,
 * an infinite e^2 gives +inf), so that the test of Algorithm 2 sees it and
 * restarts instead of accepting an error of 0. */
static double err_of_sq(double e2)
{
    if (!isfinite(e2)) return fabs(e2);
    return sqrt(e2 > 0.0 ? e2 : 0.0);
}

/* Test hook: e(k)^2 times the caller's factor for iteration k (k = 0 is the
 * initial error); no factor applies past e2_scale_n. */
static double scaled_err2(const oracle_params *p, int k, double e2)
{
    if (p->e2_scale && k < p->e2_scale_n) e2 *= p->e2_scale[k];
    return e2;
}

/* Section 4: the beta that minimizes ||X - (W_n + beta (W_n - W)) H_w||_F^2
 * over beta. With dW = W_n - W, A = X H_w^T and B = H_w H_w^T, the objective
 * is a quadratic in beta whose minimizer is
 *     beta* = <A - W_n B, dW> / <dW^T dW, B>
 * (numerator: <X - W_n H_w, dW H_w>; denominator: ||dW H_w||_F^2). Reading
 * R16: when ||dW H_w|| = 0 there is no direction and beta* is reported as 0. */
static double beta_star_of(int64_t m, int r, const double *A, const double *B,
                           const double *Wn, const double *W)
{
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        for (int k = 0; k < r; ++k) {
            double wb = 0.0, db = 0.0;
            for (int l = 0; l < r; ++l) {
                wb += Wn[i * r + l] * B[l * r + k];
                db += (Wn[i * r + l] - W[i * r + l]) * B[l * r + k];
            }
            const double dk = Wn[i * r + k] - W[i * r + k];
            num += (A[i * r + k] - wb) * dk;
            den += db * dk;
        }
    }
    return den > 0.0 ? num / den : 0.0;
}

/* ---------------------------------------------------------- beta (Alg. 3) */

typedef struct {
    double beta;       /* beta_k: used in the current iteration            */
    double betabar;    /* upper bound                                      */
    double beta_prev;  /* beta_{k-1}                                       */
    double beta_acc;   /* beta of the most recent accepted iteration       */
} beta_state;

static void beta_init(beta_state *s, double beta0)
{
    s->beta = beta0;
    s->betabar = 1.0;          /* R4: once per solve */
    s->beta_prev = beta0;      /* R5: for k = 1, beta_{k-1} is beta0 */
    s->beta_acc = beta0;
}

static void beta_update(beta_state *s, int decreased, double gamma,
                        double gamma_bar, double eta, int flags)
{
    const double bk = s->beta;
    double next;
    if (decreased) {
        next = fmin(s->betabar, gamma * bk);
        s->betabar = fmin(1.0, gamma_bar * s->betabar);   /* R3 */
        s->beta_acc = bk;
    } else {
        next = bk / eta;                                   /* R2 */
        s->betabar = (flags & ORACLE_BETABAR_LAST_ACCEPTED) ? s->beta_acc
                                                            : s->beta_prev;  /* R5 */
    }
    s->beta_prev = bk;
    s->beta = next;
}

void oracle_beta_script(int count, const uint8_t *decreased, double beta0,
                        double gamma, double gamma_bar, double eta, int flags,
                        double *beta_used, double *betabar_after)
{
    beta_state s;
    beta_init(&s, beta0);
    for (int k = 0; k < count; ++k) {
        beta_used[k] = s.beta;
        beta_update(&s, decreased[k] != 0, gamma, gamma_bar, eta, flags);
        betabar_after[k] = s.betabar;
    }
}

/* ------------------------------------------------------------------- solve */

static int valid_matrix(const oracle_matrix *X)
{
    if (X == NULL || X->m < 1 || X->n < 1) return 0;
    if (!is_csr(X)) return 1;
    if (X->row_ptr == NULL || X->row_ptr[0] != 0) return 0;
    for (int64_t i = 0; i < X->m; ++i) {
        if (X->row_ptr[i + 1] < X->row_ptr[i]) return 0;
        for (int64_t p = X->row_ptr[i]; p < X->row_ptr[i + 1]; ++p) {
            if (X->col_idx[p] < 0 || X->col_idx[p] >= X->n) return 0;
            if (p > X->row_ptr[i] && X->col_idx[p] <= X->col_idx[p - 1]) return 0;
        }
    }
    return 1;
}

/* Rounds every entry to the nearest FP32 value (ORACLE_ROUND_F32: models the
 * storage of the iterates in single precision, nothing else). */
static void round_f32(int64_t len, double *v, int flags)
{
    if (flags & ORACLE_ROUND_F32) {
        for (int64_t i = 0; i < len; ++i) v[i] = (double)(float)v[i];
    } else if (flags & ORACLE_ROUND_F32_RZ) {
        for (int64_t i = 0; i < len; ++i) {
            float f = (float)v[i];
            if (fabs((double)f) > fabs(v[i])) f = nextafterf(f, 0.0f);
            v[i] = (double)f;
        }
    }
}

/* Extrapolation: Y = N + beta (N - P), optionally projected onto Y >= 0. */
static void extrapolate(int64_t len, double beta, const double *N,
                        const double *P, double *Y, int project)
{
    for (int64_t i = 0; i < len; ++i) {
        double v = N[i] + beta * (N[i] - P[i]);
        if (project && v < 0.0) v = 0.0;
        Y[i] = v;
    }
}

/* --------------------------------------------- adaptive inner loop (R18) */

/* Sweep cap of one side: floor(1 + alpha rho), rho = 1 + (mn + K r) / (R (r + 1)),
 * R the rows of the factor being updated and K the rows of the fixed one, or
 * the caller's cost ratio of that side when it is positive; capped at inner_k
 * and at least 1. */
static int inner_cap(const oracle_matrix *X, int r, int w_side, const oracle_params *p)
{
    const double m = (double)X->m, n = (double)X->n;
    const double mn = X->dense ? m * n : (double)X->row_ptr[X->m];
    const double given = w_side ? p->inner_rho_w : p->inner_rho_h;
    const double rho = given > 0.0 ? given
                     : w_side ? 1.0 + (mn + n * r) / (m * (r + 1.0))
                              : 1.0 + (mn + m * r) / (n * (r + 1.0));
    double cap = floor(1.0 + p->inner_alpha * rho);
    if (cap > p->inner_k) cap = p->inner_k;
    return cap < 1.0 ? 1 : (int)cap;
}

static double change_norm(int64_t len, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < len; ++i) s += (a[i] - b[i]) * (a[i] - b[i]);
    return sqrt(s);
}

/* HALS sweeps on one side until the cap or the stopping ratio; returns the
 * number of sweeps run. `sweep` applies one sweep to x (len entries).
 * forced > 0 replays that count instead of deciding; *margin receives the
 * closest call among the stopping tests made, min |d_l / (delta d_1) - 1|
 * (infinity when none was made or delta d_1 = 0). */
static int adaptive_sweeps(int64_t len, double *x, double *prev, int cap, double delta,
                           void (*sweep)(int64_t, int, const double *, const double *, double *),
                           int64_t rows, int r, const double *lin, const double *gram,
                           int forced, double *margin)
{
    double eps0 = 0.0;
    *margin = INFINITY;
    if (forced > 0) cap = forced;
    int l;
    for (l = 1; l <= cap; ++l) {
        memcpy(prev, x, sizeof(double) * len);
        sweep(rows, r, lin, gram, x);
        const double d = change_norm(len, x, prev);
        if (l == 1) {
            eps0 = d;
            continue;
        }
        const double bound = delta * eps0;
        if (bound > 0.0 && fabs(d / bound - 1.0) < *margin) *margin = fabs(d / bound - 1.0);
        if (forced > 0 ? l == forced : d <= bound) break;
    }
    return l > cap ? cap : l;
}

int oracle_eahals(const oracle_matrix *X, int r, const double *W0,
                  const double *H0, const oracle_params *p, double *W,
                  double *H, double *trace, uint8_t *accepted,
                  double *beta_used, double *margin, int *n_iter,
                  double *beta_star, int *sweeps, double *sweep_margin)
{
    if (!valid_matrix(X) || r < 1 || p == NULL || p->hp < 1 || p->hp > 3 ||
        p->max_iter < 0 || p->inner_k < 1)
        return ORACLE_EINVAL;
    const int adaptive = (p->flags & ORACLE_ADAPTIVE_INNER) != 0;
    if (adaptive && !(p->inner_alpha >= 0.0 && p->inner_delta >= 0.0 && p->inner_rho_h >= 0.0 &&
                      p->inner_rho_w >= 0.0 && isfinite(p->inner_rho_h) && isfinite(p->inner_rho_w)))
        return ORACLE_EINVAL;
    if (p->resume && (p->resume->k < 0 || p->resume->k > p->max_iter || !p->resume->W ||
                      !p->resume->H || !p->resume->Wy || !p->resume->Hy))
        return ORACLE_EINVAL;
    if (p->save && (!p->save->W || !p->save->H || !p->save->Wy || !p->save->Hy))
        return ORACLE_EINVAL;
    const int64_t m = X->m, n = X->n;
    const int64_t mr = m * r, rn = (int64_t)r * n;
    const double nx2 = frob2(X);
    if (!(nx2 > 0.0) || !isfinite(nx2)) return ORACLE_EINVAL;
    const double nx = sqrt(nx2);

    double *Wy = malloc(sizeof(double) * mr), *Wn = malloc(sizeof(double) * mr);
    double *Wyn = malloc(sizeof(double) * mr), *A = malloc(sizeof(double) * mr);
    double *Hy = malloc(sizeof(double) * rn), *Hn = malloc(sizeof(double) * rn);
    double *Hyn = malloc(sizeof(double) * rn), *C = malloc(sizeof(double) * rn);
    double *G = malloc(sizeof(double) * r * r), *B = malloc(sizeof(double) * r * r);
    double *work = malloc(sizeof(double) * (r * r + r));
    double *prev = malloc(sizeof(double) * (mr > rn ? mr : rn));
    int status = ORACLE_OK;
    if (!Wy || !Wn || !Wyn || !A || !Hy || !Hn || !Hyn || !C || !G || !B || !work || !prev) {
        status = ORACLE_ENOMEM;
        goto done;
    }

    beta_state bs;
    double e_prev, e_acc;
    int k0 = 0;
    if (p->resume) {
        /* Continue a saved solve: its iterates, warm starts, beta state and
         * the errors the next decision compares with. */
        const oracle_state *rs = p->resume;
        k0 = rs->k;
        memcpy(W, rs->W, sizeof(double) * mr);
        memcpy(H, rs->H, sizeof(double) * rn);
        memcpy(Wy, rs->Wy, sizeof(double) * mr);
        memcpy(Hy, rs->Hy, sizeof(double) * rn);
        bs.beta = rs->beta;
        bs.betabar = rs->betabar;
        bs.beta_prev = rs->beta_prev;
        bs.beta_acc = rs->beta_acc;
        e_prev = rs->e_prev;
        e_acc = rs->e_acc;
        trace[k0] = rs->rho;
    } else {
        /* Alg. 2, first step: W_y = W, H_y = H, e(0) = ||X - W H||_F. */
        memcpy(W, W0, sizeof(double) * mr);
        memcpy(H, H0, sizeof(double) * rn);
        memcpy(Wy, W, sizeof(double) * mr);
        memcpy(Hy, H, sizeof(double) * rn);
        double e0sq;
        if (p->flags & ORACLE_ERR_REMARK1) {
            x_ht(X, r, H, A);
            gram_rows(n, r, H, B);
            e0sq = remark1_err2(m, r, nx2, W, A, B);
        } else {
            e0sq = explicit_err2(X, r, W, H);
        }
        const double e0 = err_of_sq(scaled_err2(p, 0, e0sq));
        if (!isfinite(e0)) { status = ORACLE_ENUMERIC; goto done; }
        trace[0] = e0 / nx;
        beta_init(&bs, p->beta0);
        e_prev = e0;
        e_acc = e0;
    }
    int k = 0;
    for (k = k0 + 1; k <= p->max_iter; ++k) {
        const double beta = bs.beta;

        /* H_n: NNLS in H with W_y fixed, warm-started at H_y. */
        wt_x(X, r, Wy, C);
        gram_cols(m, r, Wy, G);
        memcpy(Hn, Hy, sizeof(double) * rn);
        int sw_h = 0, sw_w = 0;
        double mg_h = INFINITY, mg_w = INFINITY;
        if (p->flags & ORACLE_EXACT_NNLS) exact_rows_h(n, r, C, G, Hn, work);
        else if (adaptive)
            sw_h = adaptive_sweeps(rn, Hn, prev, inner_cap(X, r, 0, p), p->inner_delta,
                                   hals_rows_h, n, r, C, G,
                                   p->sweeps_replay ? p->sweeps_replay[2 * (k - 1)] : 0, &mg_h);
        else for (sw_h = 0; sw_h < p->inner_k; ++sw_h) hals_rows_h(n, r, C, G, Hn);
        round_f32(rn, Hn, p->flags);

        /* hp >= 2: extrapolate H now (hp = 3: and project). R6: for hp = 1
         * the same H_y is formed after the W update and only warm-starts the
         * next H update; its value does not depend on that placement. */
        extrapolate(rn, beta, Hn, H, Hyn, p->hp == 3);
        round_f32(rn, Hyn, p->flags);
        const double *Hw = (p->hp == 1) ? Hn : Hyn;

        /* W_n: NNLS in W with H_w fixed, warm-started at W_y. */
        x_ht(X, r, Hw, A);
        gram_rows(n, r, Hw, B);
        memcpy(Wn, Wy, sizeof(double) * mr);
        if (p->flags & ORACLE_EXACT_NNLS) exact_cols_w(m, r, A, B, Wn, work);
        else if (adaptive)
            sw_w = adaptive_sweeps(mr, Wn, prev, inner_cap(X, r, 1, p), p->inner_delta,
                                   hals_cols_w, m, r, A, B,
                                   p->sweeps_replay ? p->sweeps_replay[2 * (k - 1) + 1] : 0, &mg_w);
        else for (sw_w = 0; sw_w < p->inner_k; ++sw_w) hals_cols_w(m, r, A, B, Wn);
        if (sweeps) {
            sweeps[2 * (k - 1)] = sw_h;
            sweeps[2 * (k - 1) + 1] = sw_w;
        }
        if (sweep_margin) {
            sweep_margin[2 * (k - 1)] = mg_h;
            sweep_margin[2 * (k - 1) + 1] = mg_w;
        }
        round_f32(mr, Wn, p->flags);
        if (beta_star) beta_star[k - 1] = beta_star_of(m, r, A, B, Wn, W);

        /* W_y = W_n + beta (W_n - W). */
        extrapolate(mr, beta, Wn, W, Wyn, 0);
        round_f32(mr, Wyn, p->flags);

        /* e(k) = ||X - W_n H_w||_F. */
        const double e2 = (p->flags & ORACLE_ERR_REMARK1)
                              ? remark1_err2(m, r, nx2, Wn, A, B)
                              : explicit_err2(X, r, Wn, Hw);
        const double e = err_of_sq(scaled_err2(p, k, e2));
        trace[k] = e / nx;

        const double e_cmp = (p->flags & ORACLE_CMP_LAST_ACCEPTED) ? e_acc : e_prev;
        int decreased = isfinite(e) && !(e > e_cmp);          /* R7, R8, R9 */
        if (margin) margin[k - 1] = (e - e_cmp) / nx;
        if (p->replay) decreased = p->replay[k - 1] != 0;
        if (beta_used) beta_used[k - 1] = beta;
        if (accepted) accepted[k - 1] = (uint8_t)decreased;

        if (decreased) {
            memcpy(W, Wn, sizeof(double) * mr);
            memcpy(H, Hn, sizeof(double) * rn);
            memcpy(Wy, Wyn, sizeof(double) * mr);
            memcpy(Hy, Hyn, sizeof(double) * rn);
            e_acc = e;
        } else {
            /* Restart: the extrapolated sequence goes back to (W, H). */
            memcpy(Wy, W, sizeof(double) * mr);
            memcpy(Hy, H, sizeof(double) * rn);
        }
        beta_update(&bs, decreased, p->gamma, p->gamma_bar, p->eta, p->flags);
        if (isfinite(e)) e_prev = e;

        if (p->tol > 0.0 && decreased && fabs(trace[k] - trace[k - 1]) < p->tol) {
            ++k;
            break;
        }
    }
    *n_iter = k - 1;
    if (p->save) {
        oracle_state *sv = p->save;
        sv->k = k - 1;
        memcpy(sv->W, W, sizeof(double) * mr);
        memcpy(sv->H, H, sizeof(double) * rn);
        memcpy(sv->Wy, Wy, sizeof(double) * mr);
        memcpy(sv->Hy, Hy, sizeof(double) * rn);
        sv->beta = bs.beta;
        sv->betabar = bs.betabar;
        sv->beta_prev = bs.beta_prev;
        sv->beta_acc = bs.beta_acc;
        sv->e_prev = e_prev;
        sv->e_acc = e_acc;
        sv->rho = trace[k - 1];
    }

done:
    free(Wy); free(Wn); free(Wyn); free(A);
    free(Hy); free(Hn); free(Hyn); free(C);
    free(G); free(B); free(work); free(prev);
    return status;
}

double oracle_beta_star(const oracle_matrix *X, int r, const double *Wn,
                        const double *W, const double *Hw)
{
    if (!valid_matrix(X) || r < 1) return NAN;
    const int64_t mr = X->m * r;
    double *A = malloc(sizeof(double) * mr), *B = malloc(sizeof(double) * r * r);
    if (!A || !B) { free(A); free(B); return NAN; }
    x_ht(X, r, Hw, A);
    gram_rows(X->n, r, Hw, B);
    const double b = beta_star_of(X->m, r, A, B, Wn, W);
    free(A); free(B);
    return b;
}

/* ------------------------------------------------------------ NNLS entries */

int oracle_nnls_exact_h(const oracle_matrix *X, int r, const double *W, double *H)
{
    if (!valid_matrix(X) || r < 1) return ORACLE_EINVAL;
    const int64_t rn = (int64_t)r * X->n;
    double *C = malloc(sizeof(double) * rn), *G = malloc(sizeof(double) * r * r);
    double *work = malloc(sizeof(double) * (r * r + r));
    if (!C || !G || !work) { free(C); free(G); free(work); return ORACLE_ENOMEM; }
    wt_x(X, r, W, C);
    gram_cols(X->m, r, W, G);
    exact_rows_h(X->n, r, C, G, H, work);
    free(C); free(G); free(work);
    return ORACLE_OK;
}

int oracle_nnls_exact_w(const oracle_matrix *X, int r, const double *H, double *W)
{
    if (!valid_matrix(X) || r < 1) return ORACLE_EINVAL;
    const int64_t mr = X->m * r;
    double *A = malloc(sizeof(double) * mr), *B = malloc(sizeof(double) * r * r);
    double *work = malloc(sizeof(double) * (r * r + r));
    if (!A || !B || !work) { free(A); free(B); free(work); return ORACLE_ENOMEM; }
    x_ht(X, r, H, A);
    gram_rows(X->n, r, H, B);
    exact_cols_w(X->m, r, A, B, W, work);
    free(A); free(B); free(work);
    return ORACLE_OK;
}

int oracle_nnls_h(const oracle_matrix *X, int r, const double *W, double *H,
                  int sweeps)
{
    if (!valid_matrix(X) || r < 1) return ORACLE_EINVAL;
    const int64_t rn = (int64_t)r * X->n;
    double *C = malloc(sizeof(double) * rn), *G = malloc(sizeof(double) * r * r);
    if (!C || !G) { free(C); free(G); return ORACLE_ENOMEM; }
    wt_x(X, r, W, C);
    gram_cols(X->m, r, W, G);
    for (int s = 0; s < sweeps; ++s) hals_rows_h(X->n, r, C, G, H);
    free(C); free(G);
    return ORACLE_OK;
}

int oracle_nnls_w(const oracle_matrix *X, int r, const double *H, double *W,
                  int sweeps)
{
    if (!valid_matrix(X) || r < 1) return ORACLE_EINVAL;
    const int64_t mr = X->m * r;
    double *A = malloc(sizeof(double) * mr), *B = malloc(sizeof(double) * r * r);
    if (!A || !B) { free(A); free(B); return ORACLE_ENOMEM; }
    x_ht(X, r, H, A);
    gram_rows(X->n, r, H, B);
    for (int s = 0; s < sweeps; ++s) hals_cols_w(X->m, r, A, B, W);
    free(A); free(B);
    return ORACLE_OK;
}

double oracle_rel_error(const oracle_matrix *X, int r, const double *W,
                        const double *H)
{
    return sqrt(explicit_err2(X, r, W, H) / frob2(X));
}

double oracle_rel_error_remark1(const oracle_matrix *X, int r, const double *W,
                                const double *H)
{
    const int64_t m = X->m;
    double *A = malloc(sizeof(double) * m * r), *B = malloc(sizeof(double) * r * r);
    x_ht(X, r, H, A);
    gram_rows(X->n, r, H, B);
    const double nx2 = frob2(X);
    const double e2 = remark1_err2(m, r, nx2, W, A, B);
    free(A); free(B);
    return err_of_sq(e2) / sqrt(nx2);
}
