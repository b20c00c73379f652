/* Memory and undefined-behaviour check of the oracle (test infrastructure).
 *
 * Built with gcc -fsanitize=address,undefined by tests/test_oracle_asan.py
 * together with oracle.c, and run as a program: every entry point of
 * oracle.h on small dense and CSR problems, ragged and degenerate shapes,
 * every inner rule and flag, replayed decisions, a save and a resume, the
 * error-scale hook with non-finite values, and the invalid-input returns
 * (a non-finite X, an hp out of range).
 * It prints "ok" and exits 0 when no call fails; the sanitizers abort on any
 * out-of-bounds access, use after free, leak or undefined operation. The
 * values themselves are checked elsewhere (tests/test_oracle_pins.py). */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static unsigned long long rng_state = 88172645463325252ULL;

static double uniform(void)  /* xorshift64, in [0, 1) */
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static double *fill(size_t count, double lo, double hi)
{
    double *a = malloc(sizeof(double) * (count ? count : 1));
    for (size_t i = 0; i < count; ++i) a[i] = lo + (hi - lo) * uniform();
    return a;
}

static int failures = 0;

static void expect(int got, int want, const char *what)
{
    if (got != want) {
        fprintf(stderr, "%s: returned %d, expected %d\n", what, got, want);
        ++failures;
    }
}

/* One full solve with every output requested. */
static int solve(const oracle_matrix *X, int r, const double *W0, const double *H0,
                 const oracle_params *p)
{
    const int64_t m = X->m, n = X->n;
    const int cap = p->max_iter > 0 ? p->max_iter : 1;
    double *W = malloc(sizeof(double) * m * r), *H = malloc(sizeof(double) * r * n);
    double *trace = malloc(sizeof(double) * (p->max_iter + 1));
    uint8_t *acc = malloc((size_t)cap);
    double *beta = malloc(sizeof(double) * cap), *margin = malloc(sizeof(double) * cap);
    double *bstar = malloc(sizeof(double) * cap), *smargin = malloc(sizeof(double) * 2 * cap);
    int *sweeps = malloc(sizeof(int) * 2 * cap);
    int n_iter = -1;
    const int st = oracle_eahals(X, r, W0, H0, p, W, H, trace, acc, beta, margin, &n_iter, bstar,
                                 sweeps, smargin);
    free(W); free(H); free(trace); free(acc); free(beta); free(margin); free(bstar);
    free(smargin); free(sweeps);
    return st;
}

static oracle_params params(int hp, int inner_k, int max_iter, int flags)
{
    oracle_params p;
    memset(&p, 0, sizeof(p));
    p.hp = hp;
    p.beta0 = 0.5;
    p.gamma = 1.01;
    p.gamma_bar = 1.005;
    p.eta = 1.5;
    p.inner_k = inner_k;
    p.max_iter = max_iter;
    p.flags = flags;
    p.inner_alpha = 0.5;
    p.inner_delta = 0.1;
    return p;
}

/* CSR copy of a dense m x n array, dropping entries below `cut`. */
static void to_csr(const double *D, int64_t m, int64_t n, double cut, int64_t **rp, int32_t **ci,
                   double **va)
{
    *rp = malloc(sizeof(int64_t) * (m + 1));
    const int64_t cap = m * n > 0 ? m * n : 1;
    *ci = malloc(sizeof(int32_t) * cap);
    *va = malloc(sizeof(double) * cap);
    int64_t z = 0;
    for (int64_t i = 0; i < m; ++i) {
        (*rp)[i] = z;
        for (int64_t j = 0; j < n; ++j)
            if (D[i * n + j] >= cut) {
                (*ci)[z] = (int32_t)j;
                (*va)[z] = D[i * n + j];
                ++z;
            }
    }
    (*rp)[m] = z;
}

static void dense_case(int64_t m, int64_t n, int r)
{
    double *X = fill((size_t)(m * n), 0.0, 1.0);
    double *W0 = fill((size_t)(m * r), 0.0, 1.0), *H0 = fill((size_t)(r * n), 0.0, 1.0);
    oracle_matrix A = {m, n, X, NULL, NULL, NULL};
    const int flag_sets[] = {0, ORACLE_ERR_REMARK1, ORACLE_ROUND_F32, ORACLE_ROUND_F32_RZ,
                             ORACLE_BETABAR_LAST_ACCEPTED | ORACLE_CMP_LAST_ACCEPTED,
                             ORACLE_EXACT_NNLS, ORACLE_ADAPTIVE_INNER,
                             ORACLE_EXACT_NNLS | ORACLE_ERR_REMARK1};
    for (int hp = 1; hp <= 3; ++hp)
        for (size_t f = 0; f < sizeof(flag_sets) / sizeof(flag_sets[0]); ++f) {
            oracle_params p = params(hp, 3, 6, flag_sets[f]);
            expect(solve(&A, r, W0, H0, &p), ORACLE_OK, "dense solve");
        }
    /* tol stop, zero iterations, replayed decisions and sweep counts. */
    oracle_params p = params(3, 2, 8, 0);
    p.tol = 0.5;
    expect(solve(&A, r, W0, H0, &p), ORACLE_OK, "tol");
    p = params(3, 2, 0, 0);
    expect(solve(&A, r, W0, H0, &p), ORACLE_OK, "max_iter 0");
    uint8_t replay[5] = {1, 0, 1, 1, 0};
    int sw[10] = {1, 2, 3, 1, 2, 3, 1, 2, 3, 1};
    p = params(2, 3, 5, ORACLE_ADAPTIVE_INNER);
    p.replay = replay;
    p.sweeps_replay = sw;
    expect(solve(&A, r, W0, H0, &p), ORACLE_OK, "replay");
    /* The error-scale hook: a NaN, an infinity and a large factor. */
    double sc[6] = {1.0, 1.0, NAN, 1e6, INFINITY, 1.0};
    p = params(3, 2, 5, ORACLE_ERR_REMARK1);
    p.e2_scale = sc;
    p.e2_scale_n = 6;
    expect(solve(&A, r, W0, H0, &p), ORACLE_OK, "error scale");
    double sc0[1] = {NAN};
    p.e2_scale = sc0;
    p.e2_scale_n = 1;
    expect(solve(&A, r, W0, H0, &p), ORACLE_ENUMERIC, "non-finite e(0)");
    /* Save after 3 iterations, resume to 6. */
    oracle_state s;
    memset(&s, 0, sizeof(s));
    s.W = malloc(sizeof(double) * m * r);
    s.H = malloc(sizeof(double) * r * n);
    s.Wy = malloc(sizeof(double) * m * r);
    s.Hy = malloc(sizeof(double) * r * n);
    p = params(3, 2, 3, 0);
    p.save = &s;
    expect(solve(&A, r, W0, H0, &p), ORACLE_OK, "save");
    p = params(3, 2, 6, 0);
    p.resume = &s;
    expect(solve(&A, r, W0, H0, &p), ORACLE_OK, "resume");
    free(s.W); free(s.H); free(s.Wy); free(s.Hy);
    /* Block solvers, beta*, errors. */
    double *W = fill((size_t)(m * r), 0.0, 1.0), *H = fill((size_t)(r * n), 0.0, 1.0);
    double *Wn = fill((size_t)(m * r), 0.0, 1.0);
    expect(oracle_nnls_h(&A, r, W, H, 2), ORACLE_OK, "nnls_h");
    expect(oracle_nnls_w(&A, r, H, W, 2), ORACLE_OK, "nnls_w");
    expect(oracle_nnls_exact_h(&A, r, W, H), ORACLE_OK, "nnls_exact_h");
    expect(oracle_nnls_exact_w(&A, r, H, W), ORACLE_OK, "nnls_exact_w");
    (void)oracle_beta_star(&A, r, Wn, W, H);
    (void)oracle_beta_star(&A, r, W, W, H);
    (void)oracle_rel_error(&A, r, W, H);
    (void)oracle_rel_error_remark1(&A, r, W, H);
    /* CSR of the same values with about half the entries. */
    int64_t *rp;
    int32_t *ci;
    double *va;
    to_csr(X, m, n, 0.5, &rp, &ci, &va);
    oracle_matrix C = {m, n, NULL, rp, ci, va};
    p = params(3, 3, 4, ORACLE_ERR_REMARK1);
    expect(solve(&C, r, W0, H0, &p), ORACLE_OK, "csr solve");
    p = params(1, 3, 4, ORACLE_EXACT_NNLS);
    expect(solve(&C, r, W0, H0, &p), ORACLE_OK, "csr exact");
    (void)oracle_beta_star(&C, r, Wn, W, H);
    free(rp); free(ci); free(va);
    free(X); free(W0); free(H0); free(W); free(H); free(Wn);
}

int main(void)
{
    const int64_t shapes[][3] = {{20, 17, 5}, {1, 40, 3}, {40, 1, 3}, {33, 29, 16}, {12, 9, 9}};
    for (size_t i = 0; i < sizeof(shapes) / sizeof(shapes[0]); ++i)
        dense_case(shapes[i][0], shapes[i][1], (int)shapes[i][2]);
    /* Invalid inputs return without touching the outputs. */
    double X[6] = {1, 2, 3, 4, 5, 6}, W0[4] = {1, 1, 1, 1}, H0[6] = {1, 1, 1, 1, 1, 1};
    oracle_matrix A = {2, 3, X, NULL, NULL, NULL};
    oracle_params p = params(3, 2, 3, 0);
    double Xnan[6] = {1, 2, NAN, 4, 5, 6};
    oracle_matrix B = {2, 3, Xnan, NULL, NULL, NULL};
    expect(solve(&B, 2, W0, H0, &p), ORACLE_EINVAL, "NaN in X");
    p.hp = 4;
    expect(solve(&A, 2, W0, H0, &p), ORACLE_EINVAL, "hp 4");
    /* Algorithm 3 on a scripted outcome sequence. */
    uint8_t dec[12] = {1, 1, 0, 1, 1, 1, 0, 0, 1, 1, 1, 1};
    double bu[12], bb[12];
    oracle_beta_script(12, dec, 0.5, 1.05, 1.01, 1.5, 0, bu, bb);
    oracle_beta_script(12, dec, 0.5, 1.05, 1.01, 1.5, ORACLE_BETABAR_LAST_ACCEPTED, bu, bb);
    if (failures) {
        fprintf(stderr, "%d call(s) returned an unexpected status\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
