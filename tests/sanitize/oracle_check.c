/* The oracle's C entry points under AddressSanitizer and
 * UndefinedBehaviorSanitizer: SpMV (plain, conjugate transpose), ILU(0) in
 * every factor precision, both substitutions, inner products, the exact
 * residual and the four methods, real and complex, on small seeded
 * diagonally dominant systems with ragged rows.  Prints "ok" and exits 0
 * when every call returned and the solves converged. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void or_spmv(int64_t n, const int32_t *rp, const int32_t *ci, const double *val, int C, int K,
             const double *x, double *y);
void or_spmv_h(int64_t n, const int32_t *rp, const int32_t *ci, const double *val, int C,
               int K, const double *x, double *y);
int or_ilu0(int64_t n, const int32_t *rp, const int32_t *ci, const double *val, int C, int kf,
            double *f, int64_t *bad_row);
void or_ilu0_apply(int64_t n, const int32_t *rp, const int32_t *ci, const double *f, int C,
                   int kf, int K, const double *r, double *z);
void or_ilu0_apply_h(int64_t n, const int32_t *rp, const int32_t *ci, const double *f, int C,
                     int kf, int K, const double *r, double *z);
void or_dot(int64_t n, int C, int K, const double *a, const double *b, double *out);
void or_residual(int64_t n, const int32_t *rp, const int32_t *ci, const double *val, int C,
                 const double *b, int kb, const double *x, int kx, double *r);
int or_krylov(int method, int64_t n, const int32_t *rp, const int32_t *ci, const double *val,
              int C, int K, int kf, const double *b, double *x, double eps_r, double eps_a,
              int64_t max_iter, int64_t *iters, double *relres_recursive,
              double *relres_true, int64_t *bad_row, double *hist, int64_t hist_len);

static uint64_t rng_state = 0x2504144980ull;
static double urand(void) /* xorshift64*, uniform in [0, 1) */
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (double)((rng_state * 2685821657736338717ull) >> 11) * 0x1.0p-53;
}

/* n rows, 1..maxr off-diagonal entries per row at distinct random columns,
 * diagonal = 1.5 x the row's absolute sum */
static void make(int64_t n, int C, int maxr, int32_t **rp, int32_t **ci, double **val)
{
    int64_t i, cap = n * (maxr + 1), p = 0;
    int32_t *R = malloc(sizeof(int32_t) * (n + 1)), *J = malloc(sizeof(int32_t) * cap);
    double *V = malloc(sizeof(double) * cap * C);
    char *mark = calloc(n, 1);
    R[0] = 0;
    for (i = 0; i < n; ++i) {
        int m = (int)(urand() * maxr) + (i % 7 == 3 ? 0 : 1), k;
        int64_t a = p, j;
        double s = 0;
        mark[i] = 1;
        for (k = 0; k < m; ++k) {
            int64_t c = (int64_t)(urand() * n);
            if (!mark[c]) mark[c] = 1;
        }
        for (j = 0; j < n; ++j)
            if (mark[j]) {
                int c;
                J[p] = (int32_t)j;
                for (c = 0; c < C; ++c) {
                    V[p * C + c] = j == i ? 0.0 : urand() - 0.5;
                    s += fabs(V[p * C + c]);
                }
                ++p;
                mark[j] = 0;
            }
        for (j = a; j < p; ++j)
            if (J[j] == i)
                V[j * C] = 1.5 * s + 1.0;
        R[i + 1] = (int32_t)p;
    }
    free(mark);
    *rp = R;
    *ci = J;
    *val = V;
}

int main(void)
{
    int C, K, kf, m, fails = 0;
    for (C = 1; C <= 2; ++C) {
        int64_t n = C == 1 ? 173 : 131, nnz, i, iters, bad;
        int32_t *rp, *ci;
        double *val;
        make(n, C, 6, &rp, &ci, &val);
        nnz = rp[n];
        for (K = 1; K <= 4; ++K) {
            double *x = malloc(sizeof(double) * n * C * K), *y = malloc(sizeof(double) * n * C * K);
            double *z = malloc(sizeof(double) * n * C * K), d[8], *r = malloc(sizeof(double) * n * C);
            for (i = 0; i < n * C * K; ++i)
                x[i] = (i % K == 0) ? urand() - 0.5 : 0.0;
            or_spmv(n, rp, ci, val, C, K, x, y);
            or_spmv_h(n, rp, ci, val, C, K, x, z);
            or_dot(n, C, K, x, y, d);
            or_residual(n, rp, ci, val, C, y, K, x, K, r);
            for (i = 0; i < n * C; ++i)
                if (fabs(r[i]) > 1e-12)
                    ++fails;
            for (kf = 1; kf <= K; ++kf) {
                double *f = malloc(sizeof(double) * nnz * C * kf);
                if (or_ilu0(n, rp, ci, val, C, kf, f, &bad) != 0)
                    ++fails;
                or_ilu0_apply(n, rp, ci, f, C, kf, K, y, z);
                or_ilu0_apply_h(n, rp, ci, f, C, kf, K, y, z);
                free(f);
            }
            if (K >= 2)
                for (m = 0; m < 4; ++m)
                    for (kf = 0; kf <= 2; ++kf) {
                        double rr, rt, hist[8], tol = K == 2 ? 1e-25 : (K == 3 ? 1e-35 : 1e-50);
                        int st;
                        memset(z, 0, sizeof(double) * n * C * K);
                        st = or_krylov(m, n, rp, ci, val, C, K, kf, y, z, tol, 0.0, 2000, &iters,
                                       &rr, &rt, &bad, hist, 8);
                        if (st != 0 || !(rt <= tol)) {
                            fprintf(stderr, "C=%d K=%d method %d kf %d: status %d relres %g\n",
                                    C, K, m, kf, st, rt);
                            ++fails;
                        }
                    }
            free(x);
            free(y);
            free(z);
            free(r);
        }
        free(rp);
        free(ci);
        free(val);
    }
    if (fails) {
        printf("%d failures\n", fails);
        return 1;
    }
    printf("ok\n");
    return 0;
}
