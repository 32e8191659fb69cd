/*
 * mpk_oracle.c -- plain, slow CPU oracle for ILU(0)-preconditioned
 * multiple-precision Krylov solvers (Kouya, arXiv 2504.14498).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path
 * (the HIP library) never links, calls or includes anything from here, and
 * this file includes nothing from the product.
 *
 * Everything is sequential, in the order the paper (or the cited published
 * algorithm) states.  Numbers with K limbs are arrays double[K], highest
 * limb first.  A vector element holds C*K doubles: the K limbs of the real
 * part, then (C == 2) the K limbs of the imaginary part.  Matrices are CSR
 * (int32 row_ptr[n+1], int32 col_idx[nnz] sorted and unique per row,
 * double val[nnz*C] with (re, im) interleaved when complex).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (no FMA
 * contraction, IEEE binary64 round-to-nearest-even, no flush-to-zero).
 * fma() is called explicitly where an algorithm needs one.
 *
 * Arithmetic (the paper fixes the formats of Section 2 -- DD, TD, QD as
 * 2, 3, 4 binary64 components -- but not their algorithms):
 *   K = 1 : plain binary64.
 *   K = 2 : double-word algorithms of Joldes, Muller, Popescu, "Tight and
 *           rigorous error bounds for basic building blocks of double-word
 *           arithmetic", ACM TOMS 44(2), 2017: AccurateDWPlusDW,
 *           DWTimesFP3, DWTimesDW3, DWDivFP3, DWDivDW2.
 *   K = 3, 4 : floating-point expansions truncated to K terms: exact
 *           partial terms from TwoSum/TwoProd, then renormalisation by
 *           VecSum followed by a VecSumErrBranch-style extraction
 *           (Joldes, Marty, Muller, Popescu, IEEE TC 65(4), 2016), with
 *           the tail beyond K-1 limbs added into the last limb.  Division
 *           is long division with K+1 quotient terms.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define KMAX 4
#define TMAX 32

/* ------------------------------------------------------------------ */
/* Error-free transforms                                               */
/* ------------------------------------------------------------------ */

/* TwoSum (Knuth / Moller): s + e == a + b exactly. */
static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double bb = x - a;
    double ab = x - bb;
    *e = (a - ab) + (b - bb);
    *s = x;
}

/* Fast2Sum (Dekker): exact when the exponent of a is >= that of b. */
static void fast_two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    *e = b - (x - a);
    *s = x;
}

/* TwoProd with FMA: p + e == a * b exactly (barring underflow). */
static void two_prod(double a, double b, double *p, double *e)
{
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* ------------------------------------------------------------------ */
/* Double-word (K = 2)                                                 */
/* ------------------------------------------------------------------ */

/* AccurateDWPlusDW: z = x + y. */
static void dw_add(const double *x, const double *y, double *z)
{
    double sh, sl, th, tl, c, vh, vl, w;
    two_sum(x[0], y[0], &sh, &sl);
    two_sum(x[1], y[1], &th, &tl);
    c = sl + th;
    fast_two_sum(sh, c, &vh, &vl);
    w = tl + vl;
    fast_two_sum(vh, w, &z[0], &z[1]);
}

/* DWTimesFP3: z = x * y, x double-word, y binary64. */
static void dw_mul_fp(const double *x, double y, double *z)
{
    double ch, cl1, cl3;
    two_prod(x[0], y, &ch, &cl1);
    cl3 = fma(x[1], y, cl1);
    fast_two_sum(ch, cl3, &z[0], &z[1]);
}

/* DWTimesDW3: z = x * y, both double-word. */
static void dw_mul(const double *x, const double *y, double *z)
{
    double ch, cl1, tl0, tl1, cl2, cl3;
    two_prod(x[0], y[0], &ch, &cl1);
    tl0 = x[1] * y[1];
    tl1 = fma(x[0], y[1], tl0);
    cl2 = fma(x[1], y[0], tl1);
    cl3 = cl1 + cl2;
    fast_two_sum(ch, cl3, &z[0], &z[1]);
}

/* DWDivFP3: z = x / y, x double-word, y binary64. */
static void dw_div_fp(const double *x, double y, double *z)
{
    double th, ph, pl, dh, dt, d, tl;
    th = x[0] / y;
    two_prod(th, y, &ph, &pl);
    dh = x[0] - ph;
    dt = dh - pl;
    d = dt + x[1];
    tl = d / y;
    fast_two_sum(th, tl, &z[0], &z[1]);
}

/* DWDivDW2: z = x / y, both double-word; the product y * th uses
 * DWTimesFP3. */
static void dw_div(const double *x, const double *y, double *z)
{
    double th, r[2], ph, dl, d, tl;
    th = x[0] / y[0];
    dw_mul_fp(y, th, r);
    ph = x[0] - r[0];
    dl = x[1] - r[1];
    d = ph + dl;
    tl = d / y[0];
    fast_two_sum(th, tl, &z[0], &z[1]);
}

/* ------------------------------------------------------------------ */
/* Truncated expansions (K = 3, 4)                                     */
/* ------------------------------------------------------------------ */

/* Renormalise m terms into K limbs.  Step 1 (VecSum) runs TwoSum from the
 * last term to the first: exact, leaves the rounded total in e[0] and the
 * errors in e[1..m-1].  Step 2 walks e[] from the top, emitting a limb each
 * time TwoSum leaves a nonzero error; once K-1 limbs are out, the rest is
 * added into the last limb. */
static void renorm(const double *t, int m, int K, double *z)
{
    double e[TMAX];
    double s = t[m - 1];
    int i, j;
    for (i = m - 2; i >= 0; --i)
        two_sum(t[i], s, &s, &e[i + 1]);
    e[0] = s;
    for (i = 0; i < K; ++i)
        z[i] = 0.0;
    j = 0;
    s = e[0];
    for (i = 1; i < m; ++i) {
        if (j == K - 1) {
            s = s + e[i];
            continue;
        }
        double r, f;
        two_sum(s, e[i], &r, &f);
        if (f != 0.0) {
            z[j++] = r;
            s = f;
        } else {
            s = r;
        }
    }
    z[j] = s;
}

/* z = x + y: terms interleaved x0, y0, x1, y1, ... then renormalised. */
static void ex_add(int K, const double *x, const double *y, double *z)
{
    double t[2 * KMAX];
    int i;
    for (i = 0; i < K; ++i) {
        t[2 * i] = x[i];
        t[2 * i + 1] = y[i];
    }
    renorm(t, 2 * K, K, z);
}

/* z = x * a, a binary64: TwoProd per limb, terms p0, e0, p1, e1, ... */
static void ex_mul_fp(int K, const double *x, double a, double *z)
{
    double t[2 * KMAX];
    int i;
    for (i = 0; i < K; ++i)
        two_prod(x[i], a, &t[2 * i], &t[2 * i + 1]);
    renorm(t, 2 * K, K, z);
}

/* z = x * y with x of kx limbs, y of ky limbs, result K limbs.  Terms are
 * listed by order class s = i + j: for s < K the exact TwoProd of x_i*y_j
 * (its product in class s, its error in class s+1); for s == K the plain
 * products.  Within a class: errors of class s-1 first, then products in
 * ascending i. */
static void ex_mul(int K, const double *x, int kx, const double *y, int ky, double *z)
{
    double t[TMAX], err[TMAX];
    int nerr = 0, m = 0, s, i, q;
    for (s = 0; s <= K; ++s) {
        int nnew = 0;
        double newerr[TMAX];
        for (q = 0; q < nerr; ++q)
            t[m++] = err[q];
        for (i = 0; i <= s; ++i) {
            int j = s - i;
            if (i >= kx || j >= ky)
                continue;
            if (s < K) {
                double p, e;
                two_prod(x[i], y[j], &p, &e);
                t[m++] = p;
                newerr[nnew++] = e;
            } else {
                t[m++] = x[i] * y[j];
            }
        }
        for (q = 0; q < nnew; ++q)
            err[q] = newerr[q];
        nerr = nnew;
    }
    renorm(t, m, K, z);
}

/* z = x / y, y of ky limbs: long division, K+1 quotient terms. */
static void ex_div(int K, const double *x, const double *y, int ky, double *z)
{
    double r[KMAX], q[KMAX + 1], yk[KMAX], p[KMAX];
    int k, i;
    for (i = 0; i < K; ++i) {
        r[i] = x[i];
        yk[i] = i < ky ? y[i] : 0.0;
    }
    q[0] = r[0] / yk[0];
    for (k = 1; k <= K; ++k) {
        ex_mul_fp(K, yk, q[k - 1], p);
        for (i = 0; i < K; ++i)
            p[i] = -p[i];
        ex_add(K, r, p, r);
        q[k] = r[0] / yk[0];
    }
    renorm(q, K + 1, K, z);
}

/* ------------------------------------------------------------------ */
/* Dispatch over K: the working-precision scalar operations             */
/* ------------------------------------------------------------------ */

static void mp_add(int K, const double *x, const double *y, double *z)
{
    if (K == 1)
        z[0] = x[0] + y[0];
    else if (K == 2)
        dw_add(x, y, z);
    else
        ex_add(K, x, y, z);
}

static void mp_neg(int K, const double *x, double *z)
{
    int i;
    for (i = 0; i < K; ++i)
        z[i] = -x[i];
}

static void mp_sub(int K, const double *x, const double *y, double *z)
{
    double ny[KMAX];
    mp_neg(K, y, ny);
    mp_add(K, x, ny, z);
}

/* x (K limbs) times a binary64 value. */
static void mp_mul_fp(int K, const double *x, double a, double *z)
{
    if (K == 1)
        z[0] = x[0] * a;
    else if (K == 2)
        dw_mul_fp(x, a, z);
    else
        ex_mul_fp(K, x, a, z);
}

/* x (K limbs) times y (ky limbs), ky <= K. */
static void mp_mul_k(int K, const double *x, const double *y, int ky, double *z)
{
    if (ky == 1) {
        mp_mul_fp(K, x, y[0], z);
    } else if (K == 2) {
        dw_mul(x, y, z);
    } else {
        ex_mul(K, x, K, y, ky, z);
    }
}

/* Working-precision product of two K-limb numbers; the first operand is
 * the scalar in scalar*vector updates. */
static void mp_mul(int K, const double *x, const double *y, double *z)
{
    if (K == 1)
        z[0] = x[0] * y[0];
    else if (K == 2)
        dw_mul(x, y, z);
    else
        ex_mul(K, x, K, y, K, z);
}

/* x (K limbs) divided by y (ky limbs), ky <= K. */
static void mp_div_k(int K, const double *x, const double *y, int ky, double *z)
{
    if (K == 1)
        z[0] = x[0] / y[0];
    else if (K == 2 && ky == 1)
        dw_div_fp(x, y[0], z);
    else if (K == 2)
        dw_div(x, y, z);
    else
        ex_div(K, x, y, ky, z);
}

static void mp_div(int K, const double *x, const double *y, double *z)
{
    mp_div_k(K, x, y, K, z);
}

static void mp_zero(int K, double *z)
{
    int i;
    for (i = 0; i < K; ++i)
        z[i] = 0.0;
}

static void mp_copy(int K, const double *x, double *z)
{
    int i;
    for (i = 0; i < K; ++i)
        z[i] = x[i];
}

/* ------------------------------------------------------------------ */
/* Complex (C = 2) over K limbs; element = re[K] then im[K].           */
/* ------------------------------------------------------------------ */

static void el_add(int C, int K, const double *x, const double *y, double *z)
{
    mp_add(K, x, y, z);
    if (C == 2)
        mp_add(K, x + K, y + K, z + K);
}

static void el_sub(int C, int K, const double *x, const double *y, double *z)
{
    mp_sub(K, x, y, z);
    if (C == 2)
        mp_sub(K, x + K, y + K, z + K);
}

/* Product of an element of A or of a binary64 factor (C binary64 values)
 * with a vector element: real part ar*xr - ai*xi, imaginary part
 * ar*xi + ai*xr, each product rounded to K limbs first. */
static void el_mul_fp(int C, int K, const double *a, const double *x, double *z)
{
    if (C == 1) {
        mp_mul_fp(K, x, a[0], z);
    } else {
        double p[KMAX], q[KMAX], zr[KMAX], zi[KMAX];
        mp_mul_fp(K, x, a[0], p);
        mp_mul_fp(K, x + K, a[1], q);
        mp_sub(K, p, q, zr);
        mp_mul_fp(K, x + K, a[0], p);
        mp_mul_fp(K, x, a[1], q);
        mp_add(K, p, q, zi);
        mp_copy(K, zr, z);
        mp_copy(K, zi, z + K);
    }
}

/* Product of a factor value f with kf limbs per component (layout re[kf],
 * im[kf]) and a vector element x: same formula as el_mul_fp. */
static void el_mul_f(int C, int K, const double *f, int kf, const double *x, double *z)
{
    if (kf == 1) {
        double a[2];
        a[0] = f[0];
        a[1] = C == 2 ? f[1] : 0.0;
        el_mul_fp(C, K, a, x, z);
        return;
    }
    if (C == 1) {
        mp_mul_k(K, x, f, kf, z);
    } else {
        double p[KMAX], q[KMAX], zr[KMAX], zi[KMAX];
        mp_mul_k(K, x, f, kf, p);
        mp_mul_k(K, x + K, f + kf, kf, q);
        mp_sub(K, p, q, zr);
        mp_mul_k(K, x + K, f, kf, p);
        mp_mul_k(K, x, f + kf, kf, q);
        mp_add(K, p, q, zi);
        mp_copy(K, zr, z);
        mp_copy(K, zi, z + K);
    }
}

/* Working-precision complex product s*x (s the scalar). */
static void el_mul(int C, int K, const double *s, const double *x, double *z)
{
    if (C == 1) {
        mp_mul(K, s, x, z);
    } else {
        double p[KMAX], q[KMAX], zr[KMAX], zi[KMAX];
        mp_mul(K, s, x, p);
        mp_mul(K, s + K, x + K, q);
        mp_sub(K, p, q, zr);
        mp_mul(K, s, x + K, p);
        mp_mul(K, s + K, x, q);
        mp_add(K, p, q, zi);
        mp_copy(K, zr, z);
        mp_copy(K, zi, z + K);
    }
}

/* Complex conjugate. */
static void el_conj(int C, int K, const double *x, double *z)
{
    mp_copy(K, x, z);
    if (C == 2)
        mp_neg(K, x + K, z + K);
}

/* x / d where d has kd limbs per component: real case is a plain division;
 * complex case is x * conj(d) / |d|^2, all in K limbs, without scaling. */
static void el_div_k_direct(int C, int K, const double *x, const double *d, int kd, double *z)
{
    if (C == 1) {
        mp_div_k(K, x, d, kd, z);
    } else {
        double dr[KMAX], di[KMAX], den[KMAX], p[KMAX], q[KMAX], nr[KMAX], ni[KMAX];
        int i;
        for (i = 0; i < K; ++i) {
            dr[i] = i < kd ? d[i] : 0.0;
            di[i] = i < kd ? d[kd + i] : 0.0;
        }
        mp_mul_k(K, dr, d, kd, p);
        mp_mul_k(K, di, d + kd, kd, q);
        mp_add(K, p, q, den);
        mp_mul_k(K, x, d, kd, p);
        mp_mul_k(K, x + K, d + kd, kd, q);
        mp_add(K, p, q, nr);
        mp_mul_k(K, x + K, d, kd, p);
        mp_mul_k(K, x, d + kd, kd, q);
        mp_sub(K, p, q, ni);
        mp_div(K, nr, den, z);
        mp_div(K, ni, den, z + K);
    }
}

/* x / d.  Complex: x conj(d) / |d|^2, which squares the magnitude of d;
 * when the leading limbs of d lie outside [2^-300, 2^300] (where |d|^2
 * and its lower limbs would leave the binary64 range), d is first scaled
 * by a power of two 2^-e, which is exact, and the quotient by 2^-e
 * afterwards: x / d = (x / (d 2^-e)) 2^-e.  Inside that range the direct
 * formula is used, so its results are unchanged; outside it they are the
 * direct formula's as if the range were unbounded. */
static void el_div_k(int C, int K, const double *x, const double *d, int kd, double *z)
{
    double m = C == 2 ? fmax(fabs(d[0]), fabs(d[kd])) : 0.0;
    if (C == 2 && isfinite(m) && m != 0.0 && (m < 0x1p-300 || m > 0x1p300)) {
        double ds[2 * KMAX];
        int e = ilogb(m), i;
        for (i = 0; i < 2 * kd; ++i)
            ds[i] = ldexp(d[i], -e);
        el_div_k_direct(C, K, x, ds, kd, z);
        for (i = 0; i < 2 * K; ++i)
            z[i] = ldexp(z[i], -e);
        return;
    }
    el_div_k_direct(C, K, x, d, kd, z);
}

static void el_div(int C, int K, const double *x, const double *d, double *z)
{
    el_div_k(C, K, x, d, K, z);
}

/* ------------------------------------------------------------------ */
/* Exported scalar operations, for pinning the arithmetic in tests.    */
/* ------------------------------------------------------------------ */

void or_add(int K, const double *x, const double *y, double *z) { mp_add(K, x, y, z); }
void or_mul(int K, const double *x, const double *y, double *z) { mp_mul(K, x, y, z); }
void or_mul_fp(int K, const double *x, double a, double *z) { mp_mul_fp(K, x, a, z); }
void or_mul_k(int K, const double *x, const double *y, int ky, double *z) { mp_mul_k(K, x, y, ky, z); }
void or_div_k(int K, const double *x, const double *y, int ky, double *z) { mp_div_k(K, x, y, ky, z); }
void or_renorm(const double *t, int m, int K, double *z) { renorm(t, m, K, z); }
void or_two_sum(double a, double b, double *s, double *e) { two_sum(a, b, s, e); }
void or_two_prod(double a, double b, double *p, double *e) { two_prod(a, b, p, e); }
void or_cmul(int K, const double *s, const double *x, double *z) { el_mul(2, K, s, x, z); }
void or_cdiv(int K, const double *x, const double *d, double *z) { el_div(2, K, x, d, z); }

/* ------------------------------------------------------------------ */
/* Sparse kernels                                                       */
/* ------------------------------------------------------------------ */

/* y = A x (Section 2: CRS SpMV with a binary64 matrix and a multi-
 * component vector, the "_d" mixed-precision product of Section 4).
 * Row i accumulates its products in ascending column order, starting from
 * the first product; an empty row gives 0. */
void or_spmv(int64_t n, const int32_t *rp, const int32_t *ci, const double *val,
             int C, int K, const double *x, double *y)
{
    int64_t i, p;
    int E = C * K;
    for (i = 0; i < n; ++i) {
        double acc[2 * KMAX], t[2 * KMAX];
        int first = 1;
        memset(acc, 0, sizeof(acc));
        for (p = rp[i]; p < rp[i + 1]; ++p) {
            el_mul_fp(C, K, val + p * C, x + (int64_t)ci[p] * E, t);
            if (first) {
                memcpy(acc, t, sizeof(double) * E);
                first = 0;
            } else {
                el_add(C, K, acc, t, acc);
            }
        }
        memcpy(y + i * E, acc, sizeof(double) * E);
    }
}

/* Conjugate transpose of a CSR matrix: row j of the result lists the
 * entries (i, j) of A in ascending i, with conjugated values. */
void or_csr_conj_transpose(int64_t n, const int32_t *rp, const int32_t *ci,
                           const double *val, int C, int kv,
                           int32_t *trp, int32_t *tci, double *tval)
{
    int64_t i, p, nnz = rp[n];
    int32_t *cnt = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    int V = C * kv;
    for (p = 0; p < nnz; ++p)
        cnt[ci[p] + 1]++;
    trp[0] = 0;
    for (i = 0; i < n; ++i)
        trp[i + 1] = trp[i] + cnt[i + 1];
    for (i = 0; i < n; ++i)
        cnt[i] = trp[i];
    for (i = 0; i < n; ++i) {
        for (p = rp[i]; p < rp[i + 1]; ++p) {
            int32_t j = ci[p];
            int32_t q = cnt[j]++;
            int v;
            tci[q] = (int32_t)i;
            for (v = 0; v < V; ++v)
                tval[(int64_t)q * V + v] = val[p * V + v];
            if (C == 2)
                for (v = 0; v < kv; ++v)
                    tval[(int64_t)q * V + kv + v] = -val[p * V + kv + v];
        }
    }
    free(cnt);
}

/* y = A^H x by the explicit conjugate transpose (Algorithm 3 uses A^H on
 * the shadow sequence). */
void or_spmv_h(int64_t n, const int32_t *rp, const int32_t *ci, const double *val,
               int C, int K, const double *x, double *y)
{
    int64_t nnz = rp[n];
    int32_t *trp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *tci = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nnz + 1));
    double *tval = (double *)malloc(sizeof(double) * ((size_t)nnz * C + 1));
    or_csr_conj_transpose(n, rp, ci, val, C, 1, trp, tci, tval);
    or_spmv(n, trp, tci, tval, C, K, x, y);
    free(trp);
    free(tci);
    free(tval);
}

/* ILU(0) factorisation (Algorithm 1) on the stored pattern of A, computed
 * row by row (IKJ): for row i and each stored k < i in ascending order,
 * l_ik = a_ik / u_kk, then a_ij -= l_ik * u_kj for each stored j > k of
 * row k that is also stored in row i.  Each entry receives the same
 * updates in the same (ascending k) order as the KIJ loop of Algorithm 1.
 * "A_ij != 0" is read structurally (stored entries).  Values are computed
 * in kf limbs per component (kf = 1: binary64, product then subtraction,
 * two roundings; kf = 2: double-word).  The factor is written in the
 * pattern of A: strictly lower part = L (unit diagonal implied), diagonal
 * and upper part = U.  Returns 0, -5 (a diagonal entry is not stored) or
 * -4 (a zero pivot u_kk), with *bad_row set. */
int or_ilu0(int64_t n, const int32_t *rp, const int32_t *ci, const double *val,
            int C, int kf, double *f, int64_t *bad_row)
{
    int64_t i, p, nnz = rp[n];
    int V = C * kf;
    int64_t *diag = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    *bad_row = -1;
    for (p = 0; p < nnz; ++p) {
        int c, v;
        for (c = 0; c < C; ++c) {
            f[p * V + c * kf] = val[p * C + c];
            for (v = 1; v < kf; ++v)
                f[p * V + c * kf + v] = 0.0;
        }
    }
    for (i = 0; i < n; ++i) {
        diag[i] = -1;
        for (p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] == i)
                diag[i] = p;
        if (diag[i] < 0) {
            *bad_row = i;
            free(diag);
            return -5;
        }
    }
    for (i = 0; i < n; ++i) {
        for (p = rp[i]; p < rp[i + 1] && ci[p] < i; ++p) {
            int64_t k = ci[p], q, r;
            double *lik = f + p * V;
            const double *ukk = f + diag[k] * V;
            double t[2 * KMAX], prod[2 * KMAX];
            int zero = 1, c;
            for (c = 0; c < V; ++c)
                if (ukk[c] != 0.0)
                    zero = 0;
            if (zero) {
                *bad_row = k;
                free(diag);
                return -4;
            }
            el_div_k(C, kf, lik, ukk, kf, t);
            memcpy(lik, t, sizeof(double) * V);
            /* merge row k (entries j > k) with row i (entries j > k) */
            r = p + 1;
            for (q = diag[k] + 1; q < rp[k + 1]; ++q) {
                int32_t j = ci[q];
                while (r < rp[i + 1] && ci[r] < j)
                    ++r;
                if (r < rp[i + 1] && ci[r] == j) {
                    double *aij = f + r * V;
                    if (kf == 1 && C == 1) {
                        double m = lik[0] * f[q];
                        aij[0] = aij[0] - m;
                    } else {
                        el_mul_f(C, kf, f + q * V, kf, lik, prod);
                        el_sub(C, kf, aij, prod, t);
                        memcpy(aij, t, sizeof(double) * V);
                    }
                }
            }
        }
        {
            const double *uii = f + diag[i] * V;
            int zero = 1, c;
            for (c = 0; c < V; ++c)
                if (uii[c] != 0.0)
                    zero = 0;
            if (zero) {
                *bad_row = i;
                free(diag);
                return -4;
            }
        }
    }
    free(diag);
    return 0;
}

/* z = (L U)^{-1} r (Algorithm 2): forward substitution with unit L, then
 * backward substitution with U and a final division by u_ii.  Each sum
 * runs in ascending column order, each term subtracted in turn.  The
 * factor f is in the pattern of A with kf limbs per component. */
void or_ilu0_apply(int64_t n, const int32_t *rp, const int32_t *ci, const double *f,
                   int C, int kf, int K, const double *r, double *z)
{
    int64_t i, p;
    int E = C * K, V = C * kf;
    double *y = (double *)malloc(sizeof(double) * ((size_t)n * E + 1));
    for (i = 0; i < n; ++i) {
        double acc[2 * KMAX], t[2 * KMAX], u[2 * KMAX];
        memcpy(acc, r + i * E, sizeof(double) * E);
        for (p = rp[i]; p < rp[i + 1] && ci[p] < i; ++p) {
            el_mul_f(C, K, f + p * V, kf, y + (int64_t)ci[p] * E, t);
            el_sub(C, K, acc, t, u);
            memcpy(acc, u, sizeof(double) * E);
        }
        memcpy(y + i * E, acc, sizeof(double) * E);
    }
    for (i = n - 1; i >= 0; --i) {
        double acc[2 * KMAX], t[2 * KMAX], u[2 * KMAX];
        int64_t dp = -1;
        memcpy(acc, y + i * E, sizeof(double) * E);
        for (p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] == i)
                dp = p;
            if (ci[p] <= i)
                continue;
            el_mul_f(C, K, f + p * V, kf, z + (int64_t)ci[p] * E, t);
            el_sub(C, K, acc, t, u);
            memcpy(acc, u, sizeof(double) * E);
        }
        el_div_k(C, K, acc, f + dp * V, kf, z + i * E);
    }
    free(y);
}

/* z = (L U)^{-H} r = L^{-H} U^{-H} r (the M^H solve of Algorithm 3):
 * forward substitution with U^H (division by conj(u_ii)), then backward
 * substitution with the unit L^H.  Both use the explicit conjugate
 * transpose, summing in ascending column order of the transposed rows. */
void or_ilu0_apply_h(int64_t n, const int32_t *rp, const int32_t *ci, const double *f,
                     int C, int kf, int K, const double *r, double *z)
{
    int64_t i, p, nnz = rp[n];
    int E = C * K, V = C * kf;
    int32_t *trp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *tci = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nnz + 1));
    double *tf = (double *)malloc(sizeof(double) * ((size_t)nnz * V + 1));
    double *w = (double *)malloc(sizeof(double) * ((size_t)n * E + 1));
    or_csr_conj_transpose(n, rp, ci, f, C, kf, trp, tci, tf);
    /* U^H is lower triangular with diagonal conj(u_ii). */
    for (i = 0; i < n; ++i) {
        double acc[2 * KMAX], t[2 * KMAX], u[2 * KMAX];
        int64_t dp = -1;
        memcpy(acc, r + i * E, sizeof(double) * E);
        for (p = trp[i]; p < trp[i + 1] && tci[p] <= i; ++p) {
            if (tci[p] == i) {
                dp = p;
                continue;
            }
            el_mul_f(C, K, tf + p * V, kf, w + (int64_t)tci[p] * E, t);
            el_sub(C, K, acc, t, u);
            memcpy(acc, u, sizeof(double) * E);
        }
        el_div_k(C, K, acc, tf + dp * V, kf, w + i * E);
    }
    /* L^H is upper triangular with unit diagonal. */
    for (i = n - 1; i >= 0; --i) {
        double acc[2 * KMAX], t[2 * KMAX], u[2 * KMAX];
        memcpy(acc, w + i * E, sizeof(double) * E);
        for (p = trp[i]; p < trp[i + 1]; ++p) {
            if (tci[p] <= i)
                continue;
            el_mul_f(C, K, tf + p * V, kf, z + (int64_t)tci[p] * E, t);
            el_sub(C, K, acc, t, u);
            memcpy(acc, u, sizeof(double) * E);
        }
        memcpy(z + i * E, acc, sizeof(double) * E);
    }
    free(trp);
    free(tci);
    free(tf);
    free(w);
}

/* <a, b> = sum_i conj(a_i) * b_i, accumulated in ascending i in the
 * working precision (Algorithm 3's inner products). */
void or_dot(int64_t n, int C, int K, const double *a, const double *b, double *out)
{
    int64_t i;
    int E = C * K;
    double acc[2 * KMAX], ca[2 * KMAX], t[2 * KMAX];
    memset(acc, 0, sizeof(acc));
    for (i = 0; i < n; ++i) {
        el_conj(C, K, a + i * E, ca);
        el_mul(C, K, ca, b + i * E, t);
        if (i == 0)
            memcpy(acc, t, sizeof(double) * E);
        else
            el_add(C, K, acc, t, acc);
    }
    memcpy(out, acc, sizeof(double) * E);
}

/* ------------------------------------------------------------------ */
/* Exact residual (the check on a solution that Algorithm 3's stopping  */
/* rule asks for, computed without rounding)                            */
/* ------------------------------------------------------------------ */

/* A long fixed-point accumulator in the manner of Kulisch: digit k holds
 * a signed multiple of 2^(32 k + ACC_LOW).  Every binary64 product of two
 * binary64 numbers, and every binary64 number, is an integer of at most
 * 106 bits times a power of two no smaller than 2^-2252 and no larger than
 * 2^1942, so it enters the accumulator exactly; carries are resolved only
 * when the total is read.  Nothing is rounded until the final conversion
 * to binary64. */
#define ACC_LOW (-2272)
#define ACC_WORDS 140

typedef struct {
    int64_t d[ACC_WORDS];
    int lo, hi; /* range of digits touched since the last clear */
} acc_t;

static void acc_clear(acc_t *a)
{
    int k;
    for (k = 0; k < ACC_WORDS; ++k)
        a->d[k] = 0;
    a->lo = ACC_WORDS;
    a->hi = -1;
}

/* a += sign * m * 2^e, m < 2^106 */
static void acc_add_int(acc_t *a, unsigned __int128 m, int e, int neg)
{
    int off = e - ACC_LOW, w = off >> 5, s = off & 31, k;
    for (k = 0; k < 4; ++k) {
        uint64_t c = (uint64_t)(m >> (32 * k)) & 0xFFFFFFFFull;
        uint64_t sh = c << s; /* < 2^63 */
        int64_t lo = (int64_t)(sh & 0xFFFFFFFFull), hi = (int64_t)(sh >> 32);
        if (neg) {
            lo = -lo;
            hi = -hi;
        }
        a->d[w + k] += lo;
        a->d[w + k + 1] += hi;
    }
    if (w < a->lo)
        a->lo = w;
    if (w + 4 > a->hi)
        a->hi = w + 4;
}

/* binary64 x = (-1)^neg * m * 2^e with m an integer below 2^53 */
static void split_double(double x, uint64_t *m, int *e, int *neg)
{
    int ex;
    double f = frexp(fabs(x), &ex);
    *neg = x < 0;
    *m = (uint64_t)ldexp(f, 53);
    *e = ex - 53;
}

static void acc_add(acc_t *a, double x)
{
    uint64_t m;
    int e, neg;
    if (x == 0.0)
        return;
    split_double(x, &m, &e, &neg);
    acc_add_int(a, (unsigned __int128)m, e, neg);
}

/* a += sign * x * y, exactly */
static void acc_add_prod(acc_t *a, double x, double y, int sign)
{
    uint64_t mx, my;
    int ex, ey, nx, ny;
    if (x == 0.0 || y == 0.0)
        return;
    split_double(x, &mx, &ex, &nx);
    split_double(y, &my, &ey, &ny);
    acc_add_int(a, (unsigned __int128)mx * my, ex + ey, (nx ^ ny) ^ (sign < 0));
}

/* The accumulated total rounded to binary64 (to within two units in the
 * last place; not necessarily the nearest). */
static double acc_value(acc_t *a)
{
    int k, top, neg = 0;
    double v;
    if (a->hi < 0)
        return 0.0;
    for (k = a->lo; k < ACC_WORDS - 1 && k <= a->hi; ++k) {
        int64_t carry = a->d[k] >> 32; /* floor division by 2^32 */
        a->d[k] -= carry * ((int64_t)1 << 32);
        a->d[k + 1] += carry;
        if (k == a->hi && carry != 0)
            a->hi = k + 1;
    }
    top = a->hi;
    while (top >= a->lo && a->d[top] == 0)
        --top;
    if (top < a->lo)
        return 0.0;
    if (a->d[top] < 0) {
        /* negative total: negate the digits and resolve the borrows again */
        neg = 1;
        for (k = a->lo; k <= top; ++k)
            a->d[k] = -a->d[k];
        for (k = a->lo; k < top; ++k) {
            int64_t carry = a->d[k] >> 32;
            a->d[k] -= carry * ((int64_t)1 << 32);
            a->d[k + 1] += carry;
        }
        while (top >= a->lo && a->d[top] == 0)
            --top;
    }
    v = 0.0;
    for (k = top; k >= a->lo && k >= top - 2; --k)
        v += ldexp((double)a->d[k], 32 * k + ACC_LOW);
    return neg ? -v : v;
}

/* r = b - A x without rounding, then each component rounded to binary64:
 * r[i*C + c] (C = 2: real then imaginary part).  b has kb limbs and x has
 * kx limbs per component, in the vector layout above; A is binary64 (the
 * complex product uses its four real products).  Used to check a
 * solution's true residual ||b - A x|| independently of the arithmetic
 * the methods run in. */
void or_residual(int64_t n, const int32_t *rp, const int32_t *ci, const double *val, int C,
                 const double *b, int kb, const double *x, int kx, double *r)
{
    int64_t i, p;
    acc_t *acc = (acc_t *)malloc(sizeof(acc_t));
    acc_clear(acc);
    for (i = 0; i < n; ++i) {
        int c, k;
        for (c = 0; c < C; ++c) {
            for (k = 0; k < kb; ++k)
                acc_add(acc, b[(i * C + c) * kb + k]);
            for (p = rp[i]; p < rp[i + 1]; ++p) {
                const double *xj = x + (int64_t)ci[p] * C * kx;
                if (C == 1) {
                    for (k = 0; k < kx; ++k)
                        acc_add_prod(acc, val[p], xj[k], -1);
                } else if (c == 0) {
                    /* re(a x) = a_re x_re - a_im x_im */
                    for (k = 0; k < kx; ++k) {
                        acc_add_prod(acc, val[2 * p], xj[k], -1);
                        acc_add_prod(acc, val[2 * p + 1], xj[kx + k], +1);
                    }
                } else {
                    /* im(a x) = a_re x_im + a_im x_re */
                    for (k = 0; k < kx; ++k) {
                        acc_add_prod(acc, val[2 * p], xj[kx + k], -1);
                        acc_add_prod(acc, val[2 * p + 1], xj[k], -1);
                    }
                }
            }
            r[i * C + c] = acc_value(acc);
            {
                int lo = acc->lo, hi = acc->hi;
                for (k = lo; k <= hi + 1 && k < ACC_WORDS; ++k)
                    acc->d[k] = 0;
                acc->lo = ACC_WORDS;
                acc->hi = -1;
            }
        }
    }
    free(acc);
}

/* ------------------------------------------------------------------ */
/* Krylov methods                                                       */
/* ------------------------------------------------------------------ */

enum { M_BICG = 0, M_CGS = 1, M_BICGSTAB = 2, M_GPBICG = 3 };
enum { ST_OK = 0, ST_NOT_CONVERGED = 1, ST_BREAKDOWN = 2 };

typedef struct {
    int64_t n;
    const int32_t *rp, *ci;
    const double *val;
    int C, K, kf; /* kf = 0: no preconditioner */
    const double *f; /* factor values, pattern of A */
    int E;
} sys_t;

static double *vnew(const sys_t *s)
{
    return (double *)calloc((size_t)s->n * s->E + 1, sizeof(double));
}

static void vcopy(const sys_t *s, const double *x, double *z)
{
    memcpy(z, x, sizeof(double) * (size_t)s->n * s->E);
}

static void precond(const sys_t *s, const double *r, double *z)
{
    if (s->kf == 0)
        vcopy(s, r, z);
    else
        or_ilu0_apply(s->n, s->rp, s->ci, s->f, s->C, s->kf, s->K, r, z);
}

static void precond_h(const sys_t *s, const double *r, double *z)
{
    if (s->kf == 0)
        vcopy(s, r, z);
    else
        or_ilu0_apply_h(s->n, s->rp, s->ci, s->f, s->C, s->kf, s->K, r, z);
}

static void matvec(const sys_t *s, const double *x, double *y)
{
    or_spmv(s->n, s->rp, s->ci, s->val, s->C, s->K, x, y);
}

static void dot(const sys_t *s, const double *a, const double *b, double *out)
{
    or_dot(s->n, s->C, s->K, a, b, out);
}

/* squared 2-norm, leading limb (the stopping test of Algorithm 3 needs
 * only a binary64 comparison). */
static double nrm2sq_hi(const sys_t *s, const double *a)
{
    double d[2 * KMAX];
    dot(s, a, a, d);
    return d[0];
}

static int is_zero(const sys_t *s, const double *x)
{
    int i;
    for (i = 0; i < s->C * s->K; ++i)
        if (x[i] != 0.0)
            return 0;
    return 1;
}

/* z_i = x_i + c * y_i */
static void v_axpy(const sys_t *s, const double *x, const double *c, const double *y, double *z)
{
    int64_t i;
    int E = s->E;
    for (i = 0; i < s->n; ++i) {
        double t[2 * KMAX];
        el_mul(s->C, s->K, c, y + i * E, t);
        el_add(s->C, s->K, x + i * E, t, z + i * E);
    }
}

/* z_i = x_i - c * y_i */
static void v_axmy(const sys_t *s, const double *x, const double *c, const double *y, double *z)
{
    int64_t i;
    int E = s->E;
    for (i = 0; i < s->n; ++i) {
        double t[2 * KMAX];
        el_mul(s->C, s->K, c, y + i * E, t);
        el_sub(s->C, s->K, x + i * E, t, z + i * E);
    }
}

static void v_add(const sys_t *s, const double *x, const double *y, double *z)
{
    int64_t i;
    for (i = 0; i < s->n; ++i)
        el_add(s->C, s->K, x + i * s->E, y + i * s->E, z + i * s->E);
}

static void v_sub(const sys_t *s, const double *x, const double *y, double *z)
{
    int64_t i;
    for (i = 0; i < s->n; ++i)
        el_sub(s->C, s->K, x + i * s->E, y + i * s->E, z + i * s->E);
}

/* Stopping test of Algorithm 3: ||r|| < eps_r ||r_0|| + eps_a, on the
 * leading limbs of the squared norms, in binary64. */
static int stop_test(double nr2, double nr02, double eps_r, double eps_a)
{
    return sqrt(nr2) < eps_r * sqrt(nr02) + eps_a;
}

/* True residual check: ||b - A x|| against the same threshold, with the
 * residual and its norm in the working precision. */
static int true_check(const sys_t *s, const double *b, const double *x, double nr02,
                      double eps_r, double eps_a, double *relres)
{
    double *ax = vnew(s), *rt = vnew(s);
    double nb2, n2;
    matvec(s, x, ax);
    v_sub(s, b, ax, rt);
    n2 = nrm2sq_hi(s, rt);
    nb2 = nrm2sq_hi(s, b);
    *relres = nb2 > 0 ? sqrt(n2 / nb2) : sqrt(n2);
    free(ax);
    free(rt);
    return stop_test(n2, nr02, eps_r, eps_a);
}

typedef struct {
    int64_t iters;
    int32_t status;
    double relres_recursive, relres_true;
} or_info_t;

static void record(double *hist, int64_t hist_len, int64_t k, double nr2)
{
    if (hist && k >= 1 && k <= hist_len)
        hist[k - 1] = nr2;
}

/* Preconditioned BiCG (the method that Algorithm 3 states), written from
 * its defining recurrences.  BiCG builds two coupled sequences, one for A
 * (residuals r_k = b - A x_k) and one for A^H (shadow residuals s_k, with
 * s_0 = r_0), kept biorthogonal through M: <M^-H s_j, r_k> = 0 for j != k.
 * A pass of the pair:
 *   images       (q, q~) = (A d, A^H d~) of the search directions;
 *   step length  alpha = rho / <d~, q>, rho = <M^-H s, r>;
 *   advance      x += alpha d,  r -= alpha q,  s -= conj(alpha) q~;
 *   directions   (z, z~) = (M^-1 r, M^-H s), rho' = <z~, r>,
 *                beta = rho' / rho,  d = z + beta d,  d~ = z~ + conj(beta) d~.
 * The vector operations are the oracle's element-wise ones; each is one
 * pass over the rows, so a pass's rounding does not depend on the order in
 * which independent vectors are updated. */
typedef struct {
    double *r, *s;     /* residual and shadow residual */
    double *z, *zs;    /* their preconditioned forms */
    double *d, *ds;    /* search directions */
    double *q, *qs;    /* images of the directions */
    double rho[2 * KMAX];
} bicg_pair_t;

static void bicg_pair_init(const sys_t *s, bicg_pair_t *P, const double *b, const double *x)
{
    double *ax = vnew(s);
    P->r = vnew(s); P->s = vnew(s); P->z = vnew(s); P->zs = vnew(s);
    P->d = vnew(s); P->ds = vnew(s); P->q = vnew(s); P->qs = vnew(s);
    matvec(s, x, ax);
    v_sub(s, b, ax, P->r);
    vcopy(s, P->r, P->s);
    precond(s, P->r, P->z);
    precond_h(s, P->s, P->zs);
    vcopy(s, P->z, P->d);
    vcopy(s, P->zs, P->ds);
    dot(s, P->zs, P->r, P->rho);
    free(ax);
}

static void bicg_pair_free(bicg_pair_t *P)
{
    free(P->r); free(P->s); free(P->z); free(P->zs);
    free(P->d); free(P->ds); free(P->q); free(P->qs);
}

/* Images of the directions and the step length; 0 on breakdown (a zero
 * <d~, q> or rho). */
static int bicg_step_length(const sys_t *s, bicg_pair_t *P, double *alpha)
{
    double dq[2 * KMAX];
    matvec(s, P->d, P->q);
    or_spmv_h(s->n, s->rp, s->ci, s->val, s->C, s->K, P->ds, P->qs);
    dot(s, P->ds, P->q, dq);
    if (is_zero(s, dq) || is_zero(s, P->rho))
        return 0;
    el_div(s->C, s->K, P->rho, dq, alpha);
    return 1;
}

static void bicg_advance(const sys_t *s, bicg_pair_t *P, const double *alpha, double *x)
{
    double ca[2 * KMAX];
    v_axpy(s, x, alpha, P->d, x);
    v_axmy(s, P->r, alpha, P->q, P->r);
    el_conj(s->C, s->K, alpha, ca);
    v_axmy(s, P->s, ca, P->qs, P->s);
}

static void bicg_new_directions(const sys_t *s, bicg_pair_t *P)
{
    double rho_next[2 * KMAX], beta[2 * KMAX], cb[2 * KMAX];
    precond(s, P->r, P->z);
    precond_h(s, P->s, P->zs);
    dot(s, P->zs, P->r, rho_next);
    el_div(s->C, s->K, rho_next, P->rho, beta);
    v_axpy(s, P->z, beta, P->d, P->d);
    el_conj(s->C, s->K, beta, cb);
    v_axpy(s, P->zs, cb, P->ds, P->ds);
    memcpy(P->rho, rho_next, sizeof(double) * s->E);
}

static int run_bicg(const sys_t *s, const double *b, double *x, int64_t max_iter,
                    double eps_r, double eps_a, or_info_t *info, double *hist, int64_t hlen)
{
    bicg_pair_t P;
    double alpha[2 * KMAX], nr02, nr2 = 0;
    int64_t k;
    int st = ST_NOT_CONVERGED;
    bicg_pair_init(s, &P, b, x);
    nr02 = nrm2sq_hi(s, P.r);
    info->iters = 0;
    for (k = 1; k <= max_iter; ++k) {
        info->iters = k;
        if (!bicg_step_length(s, &P, alpha)) {
            st = ST_BREAKDOWN;
            break;
        }
        bicg_advance(s, &P, alpha, x);
        nr2 = nrm2sq_hi(s, P.r);
        record(hist, hlen, k, nr2);
        if (stop_test(nr2, nr02, eps_r, eps_a) &&
            true_check(s, b, x, nr02, eps_r, eps_a, &info->relres_true)) {
            st = ST_OK;
            break;
        }
        bicg_new_directions(s, &P);
    }
    info->relres_recursive = nr02 > 0 ? sqrt(nr2 / nr02) : sqrt(nr2);
    bicg_pair_free(&P);
    return st;
}

/* Preconditioned CGS: the right-preconditioned form (two M-solves per
 * pass, unpreconditioned residual), shadow vector r~ = r_0. */
static int run_cgs(const sys_t *s, const double *b, double *x, int64_t max_iter,
                   double eps_r, double eps_a, or_info_t *info, double *hist, int64_t hlen)
{
    int E = s->E, C = s->C, K = s->K;
    double *r = vnew(s), *rt = vnew(s), *u = vnew(s), *p = vnew(s), *q = vnew(s),
           *ph = vnew(s), *v = vnew(s), *uh = vnew(s), *w = vnew(s), *tmp = vnew(s);
    double rho[2 * KMAX], rho_old[2 * KMAX], alpha[2 * KMAX], beta[2 * KMAX],
        sigma[2 * KMAX], nr02, nr2 = 0;
    int64_t k;
    int st = ST_NOT_CONVERGED;
    matvec(s, x, tmp);
    v_sub(s, b, tmp, r);
    vcopy(s, r, rt);
    nr02 = nrm2sq_hi(s, r);
    info->iters = 0;
    for (k = 1; k <= max_iter; ++k) {
        dot(s, rt, r, rho);
        if (is_zero(s, rho)) {
            st = ST_BREAKDOWN;
            info->iters = k;
            break;
        }
        if (k == 1) {
            vcopy(s, r, u);
            vcopy(s, u, p);
        } else {
            el_div(C, K, rho, rho_old, beta);
            v_axpy(s, r, beta, q, u);      /* u = r + beta q */
            v_axpy(s, q, beta, p, tmp);    /* tmp = q + beta p */
            v_axpy(s, u, beta, tmp, p);    /* p = u + beta tmp */
        }
        precond(s, p, ph);
        matvec(s, ph, v);
        dot(s, rt, v, sigma);
        if (is_zero(s, sigma)) {
            st = ST_BREAKDOWN;
            info->iters = k;
            break;
        }
        el_div(C, K, rho, sigma, alpha);
        v_axmy(s, u, alpha, v, q);         /* q = u - alpha v */
        v_add(s, u, q, w);                 /* w = u + q */
        precond(s, w, uh);
        v_axpy(s, x, alpha, uh, x);        /* x = x + alpha uh */
        matvec(s, uh, tmp);
        v_axmy(s, r, alpha, tmp, r);       /* r = r - alpha A uh */
        nr2 = nrm2sq_hi(s, r);
        record(hist, hlen, k, nr2);
        info->iters = k;
        if (stop_test(nr2, nr02, eps_r, eps_a)) {
            if (true_check(s, b, x, nr02, eps_r, eps_a, &info->relres_true)) {
                st = ST_OK;
                break;
            }
        }
        memcpy(rho_old, rho, sizeof(double) * E);
    }
    info->relres_recursive = nr02 > 0 ? sqrt(nr2 / nr02) : sqrt(nr2);
    free(r); free(rt); free(u); free(p); free(q); free(ph); free(v); free(uh); free(w); free(tmp);
    return st;
}

/* Preconditioned BiCGSTAB: right-preconditioned form, shadow r~ = r_0,
 * with the early exit on ||s||. */
static int run_bicgstab(const sys_t *s, const double *b, double *x, int64_t max_iter,
                        double eps_r, double eps_a, or_info_t *info, double *hist, int64_t hlen)
{
    int E = s->E, C = s->C, K = s->K;
    double *r = vnew(s), *rt = vnew(s), *p = vnew(s), *ph = vnew(s), *v = vnew(s),
           *sv = vnew(s), *sh = vnew(s), *t = vnew(s), *tmp = vnew(s);
    double rho[2 * KMAX], rho_old[2 * KMAX], alpha[2 * KMAX], beta[2 * KMAX],
        omega[2 * KMAX], sigma[2 * KMAX], ts[2 * KMAX], tt[2 * KMAX], q1[2 * KMAX],
        q2[2 * KMAX], nr02, nr2 = 0;
    int64_t k;
    int st = ST_NOT_CONVERGED;
    matvec(s, x, tmp);
    v_sub(s, b, tmp, r);
    vcopy(s, r, rt);
    nr02 = nrm2sq_hi(s, r);
    info->iters = 0;
    for (k = 1; k <= max_iter; ++k) {
        dot(s, rt, r, rho);
        if (is_zero(s, rho)) {
            st = ST_BREAKDOWN;
            info->iters = k;
            break;
        }
        if (k == 1) {
            vcopy(s, r, p);
        } else {
            el_div(C, K, rho, rho_old, q1);
            el_div(C, K, alpha, omega, q2);
            el_mul(C, K, q1, q2, beta);     /* beta = (rho/rho_old)(alpha/omega) */
            v_axmy(s, p, omega, v, tmp);    /* tmp = p - omega v */
            v_axpy(s, r, beta, tmp, p);     /* p = r + beta tmp */
        }
        precond(s, p, ph);
        matvec(s, ph, v);
        dot(s, rt, v, sigma);
        if (is_zero(s, sigma)) {
            st = ST_BREAKDOWN;
            info->iters = k;
            break;
        }
        el_div(C, K, rho, sigma, alpha);
        v_axmy(s, r, alpha, v, sv);         /* s = r - alpha v */
        nr2 = nrm2sq_hi(s, sv);
        info->iters = k;
        if (stop_test(nr2, nr02, eps_r, eps_a)) {
            v_axpy(s, x, alpha, ph, tmp);   /* candidate x + alpha ph */
            if (true_check(s, b, tmp, nr02, eps_r, eps_a, &info->relres_true)) {
                vcopy(s, tmp, x);
                record(hist, hlen, k, nr2);
                st = ST_OK;
                break;
            }
        }
        precond(s, sv, sh);
        matvec(s, sh, t);
        dot(s, t, sv, ts);
        dot(s, t, t, tt);
        if (is_zero(s, tt)) {
            st = ST_BREAKDOWN;
            break;
        }
        el_div(C, K, ts, tt, omega);
        v_axpy(s, x, alpha, ph, x);         /* x = (x + alpha ph) + omega sh */
        v_axpy(s, x, omega, sh, x);
        v_axmy(s, sv, omega, t, r);         /* r = s - omega t */
        nr2 = nrm2sq_hi(s, r);
        record(hist, hlen, k, nr2);
        if (stop_test(nr2, nr02, eps_r, eps_a)) {
            if (true_check(s, b, x, nr02, eps_r, eps_a, &info->relres_true)) {
                st = ST_OK;
                break;
            }
        }
        if (is_zero(s, omega)) {
            st = ST_BREAKDOWN;
            break;
        }
        memcpy(rho_old, rho, sizeof(double) * E);
    }
    info->relres_recursive = nr02 > 0 ? sqrt(nr2 / nr02) : sqrt(nr2);
    free(r); free(rt); free(p); free(ph); free(v); free(sv); free(sh); free(t); free(tmp);
    return st;
}

/* Preconditioned GPBiCG (Zhang's generalized product-type method), right-
 * preconditioned: M-solves of p and t each pass, the true residual kept,
 * and x updated through z^ = M^{-1} z using A^{-1} y = z_old - alpha t_old
 * - alpha beta p_old + alpha p. */
static int run_gpbicg(const sys_t *s, const double *b, double *x, int64_t max_iter,
                      double eps_r, double eps_a, or_info_t *info, double *hist, int64_t hlen)
{
    int E = s->E, C = s->C, K = s->K;
    double *r = vnew(s), *rt = vnew(s), *p = vnew(s), *ph = vnew(s), *q = vnew(s),
           *y = vnew(s), *t = vnew(s), *th = vnew(s), *sv = vnew(s), *u = vnew(s),
           *vh = vnew(s), *zh = vnew(s), *w = vnew(s), *told = vnew(s), *phold = vnew(s),
           *thold = vnew(s), *tmp = vnew(s), *tmp2 = vnew(s);
    double rho[2 * KMAX], rho_new[2 * KMAX], alpha[2 * KMAX], beta[2 * KMAX],
        zeta[2 * KMAX], eta[2 * KMAX], sig[2 * KMAX], ss[2 * KMAX], yy[2 * KMAX],
        sy[2 * KMAX], ys[2 * KMAX], st_[2 * KMAX], yt[2 * KMAX], a1[2 * KMAX],
        a2[2 * KMAX], den[2 * KMAX], num[2 * KMAX], ab[2 * KMAX], nr02, nr2 = 0;
    int64_t k;
    int st = ST_NOT_CONVERGED;
    matvec(s, x, tmp);
    v_sub(s, b, tmp, r);
    vcopy(s, r, rt);
    nr02 = nrm2sq_hi(s, r);
    memset(beta, 0, sizeof(beta));
    dot(s, rt, r, rho);
    info->iters = 0;
    for (k = 1; k <= max_iter; ++k) {
        if (is_zero(s, rho)) {
            st = ST_BREAKDOWN;
            info->iters = k;
            break;
        }
        v_sub(s, p, u, tmp);                /* p = r + beta (p - u) */
        v_axpy(s, r, beta, tmp, p);
        precond(s, p, ph);
        matvec(s, ph, q);
        dot(s, rt, q, sig);
        if (is_zero(s, sig)) {
            st = ST_BREAKDOWN;
            info->iters = k;
            break;
        }
        el_div(C, K, rho, sig, alpha);
        v_sub(s, told, r, tmp);             /* y = ((t_old - r) - alpha w) + alpha q */
        v_axmy(s, tmp, alpha, w, tmp2);
        v_axpy(s, tmp2, alpha, q, y);
        v_axmy(s, r, alpha, q, t);          /* t = r - alpha q */
        precond(s, t, th);
        matvec(s, th, sv);                  /* s = A t^ */
        dot(s, sv, sv, ss);
        dot(s, sv, t, st_);
        if (k == 1) {
            if (is_zero(s, ss)) {
                st = ST_BREAKDOWN;
                info->iters = k;
                break;
            }
            el_div(C, K, st_, ss, zeta);
            memset(eta, 0, sizeof(eta));
        } else {
            dot(s, y, y, yy);
            dot(s, sv, y, sy);
            dot(s, y, sv, ys);
            dot(s, y, t, yt);
            el_mul(C, K, ss, yy, a1);       /* D = <s,s><y,y> - <s,y><y,s> */
            el_mul(C, K, sy, ys, a2);
            el_sub(C, K, a1, a2, den);
            if (is_zero(s, den)) {
                st = ST_BREAKDOWN;
                info->iters = k;
                break;
            }
            el_mul(C, K, yy, st_, a1);      /* zeta = (<y,y><s,t> - <s,y><y,t>) / D */
            el_mul(C, K, sy, yt, a2);
            el_sub(C, K, a1, a2, num);
            el_div(C, K, num, den, zeta);
            el_mul(C, K, ss, yt, a1);       /* eta = (<s,s><y,t> - <y,s><s,t>) / D */
            el_mul(C, K, ys, st_, a2);
            el_sub(C, K, a1, a2, num);
            el_div(C, K, num, den, eta);
        }
        /* u = zeta q + eta ((t_old - r) + beta u) */
        v_sub(s, told, r, tmp);
        v_axpy(s, tmp, beta, u, tmp2);
        {
            int64_t i;
            for (i = 0; i < s->n; ++i) {
                double a[2 * KMAX], c[2 * KMAX];
                el_mul(C, K, zeta, q + i * E, a);
                el_mul(C, K, eta, tmp2 + i * E, c);
                el_add(C, K, a, c, u + i * E);
            }
        }
        /* v^ = ((z^ - alpha t^_old) - (alpha beta) p^_old) + alpha p^ */
        el_mul(C, K, alpha, beta, ab);
        v_axmy(s, zh, alpha, thold, tmp);
        v_axmy(s, tmp, ab, phold, tmp2);
        v_axpy(s, tmp2, alpha, ph, vh);
        /* z^ = zeta t^ + eta v^ */
        {
            int64_t i;
            for (i = 0; i < s->n; ++i) {
                double a[2 * KMAX], c[2 * KMAX];
                el_mul(C, K, zeta, th + i * E, a);
                el_mul(C, K, eta, vh + i * E, c);
                el_add(C, K, a, c, zh + i * E);
            }
        }
        v_axpy(s, x, alpha, ph, x);         /* x = (x + alpha p^) + z^ */
        v_add(s, x, zh, x);
        v_axmy(s, t, eta, y, tmp);          /* r = (t - eta y) - zeta s */
        v_axmy(s, tmp, zeta, sv, r);
        nr2 = nrm2sq_hi(s, r);
        record(hist, hlen, k, nr2);
        info->iters = k;
        if (stop_test(nr2, nr02, eps_r, eps_a)) {
            if (true_check(s, b, x, nr02, eps_r, eps_a, &info->relres_true)) {
                st = ST_OK;
                break;
            }
        }
        if (is_zero(s, zeta)) {
            st = ST_BREAKDOWN;
            break;
        }
        dot(s, rt, r, rho_new);             /* beta = (alpha/zeta)(rho_new/rho) */
        el_div(C, K, alpha, zeta, a1);
        el_div(C, K, rho_new, rho, a2);
        el_mul(C, K, a1, a2, beta);
        v_axpy(s, sv, beta, q, w);          /* w = s + beta q */
        vcopy(s, t, told);
        vcopy(s, ph, phold);
        vcopy(s, th, thold);
        memcpy(rho, rho_new, sizeof(double) * E);
    }
    info->relres_recursive = nr02 > 0 ? sqrt(nr2 / nr02) : sqrt(nr2);
    free(r); free(rt); free(p); free(ph); free(q); free(y); free(t); free(th); free(sv);
    free(u); free(vh); free(zh); free(w); free(told); free(phold); free(thold); free(tmp);
    free(tmp2);
    return st;
}

/* Solve A x = b.  method: 0 BiCG, 1 CGS, 2 BiCGSTAB, 3 GPBiCG.  kf = 0 runs
 * without a preconditioner; kf = 1, 2 factor A by ILU(0) in that many limbs
 * first.  x holds x_0 on entry.  Returns ST_* (>= 0) or an ILU(0) error
 * (< 0).  hist (optional) receives the leading limb of ||r_k||^2. */
/* The four methods with the ILU(0) factor either computed here (Alg. 1,
 * fgiven == NULL) or supplied by the caller in A's pattern (fgiven: nnz x C
 * x kf values, e.g. a corrected factor); the iteration is the same. */
static int krylov_impl(int method, int64_t n, const int32_t *rp, const int32_t *ci,
                       const double *val, int C, int K, int kf, const double *fgiven,
                       const double *b, double *x, double eps_r, double eps_a,
                       int64_t max_iter, int64_t *iters, double *relres_recursive,
                       double *relres_true, int64_t *bad_row, double *hist, int64_t hist_len)
{
    sys_t s;
    or_info_t info;
    double *f = NULL;
    int st;
    s.n = n;
    s.rp = rp;
    s.ci = ci;
    s.val = val;
    s.C = C;
    s.K = K;
    s.kf = kf;
    s.E = C * K;
    *bad_row = -1;
    if (kf > 0) {
        f = (double *)malloc(sizeof(double) * ((size_t)rp[n] * C * kf + 1));
        if (fgiven) {
            memcpy(f, fgiven, sizeof(double) * (size_t)rp[n] * C * kf);
        } else {
            st = or_ilu0(n, rp, ci, val, C, kf, f, bad_row);
            if (st != 0) {
                free(f);
                return st;
            }
        }
    }
    s.f = f;
    memset(&info, 0, sizeof(info));
    info.relres_true = -1.0;
    switch (method) {
    case M_BICG: st = run_bicg(&s, b, x, max_iter, eps_r, eps_a, &info, hist, hist_len); break;
    case M_CGS: st = run_cgs(&s, b, x, max_iter, eps_r, eps_a, &info, hist, hist_len); break;
    case M_BICGSTAB: st = run_bicgstab(&s, b, x, max_iter, eps_r, eps_a, &info, hist, hist_len); break;
    default: st = run_gpbicg(&s, b, x, max_iter, eps_r, eps_a, &info, hist, hist_len); break;
    }
    *iters = info.iters;
    *relres_recursive = info.relres_recursive;
    *relres_true = info.relres_true;
    free(f);
    return st;
}

int or_krylov(int method, int64_t n, const int32_t *rp, const int32_t *ci,
              const double *val, int C, int K, int kf, const double *b, double *x,
              double eps_r, double eps_a, int64_t max_iter, int64_t *iters,
              double *relres_recursive, double *relres_true, int64_t *bad_row,
              double *hist, int64_t hist_len)
{
    return krylov_impl(method, n, rp, ci, val, C, K, kf, NULL, b, x, eps_r, eps_a, max_iter,
                       iters, relres_recursive, relres_true, bad_row, hist, hist_len);
}

int or_krylov_with_factor(int method, int64_t n, const int32_t *rp, const int32_t *ci,
                          const double *val, int C, int K, int kf, const double *f,
                          const double *b, double *x, double eps_r, double eps_a,
                          int64_t max_iter, int64_t *iters, double *relres_recursive,
                          double *relres_true, int64_t *bad_row, double *hist,
                          int64_t hist_len)
{
    return krylov_impl(method, n, rp, ci, val, C, K, kf, f, b, x, eps_r, eps_a, max_iter,
                       iters, relres_recursive, relres_true, bad_row, hist, hist_len);
}

/* ------------------------------------------------------------------ */
/* Multicolour ordering: a labelled variant beyond the paper's method  */
/* (Section 5 leaves parallelising the ILU(0) routines to future work). */
/* The solve of P A P^T y = P b with ILU(0) of P A P^T is a different   */
/* preconditioner from ILU(0) of A.                                     */
/* ------------------------------------------------------------------ */

/* Greedy colouring of the graph of A + A^T in natural order: vertices i
 * != j are adjacent when a_ij or a_ji is stored, and vertex i = 0, 1, ...
 * takes the smallest colour that no adjacent vertex j < i has.  Writes
 * color[n]; returns the number of colours (0 when n = 0). */
int32_t or_greedy_color(int64_t n, const int32_t *rp, const int32_t *ci, int32_t *color)
{
    int64_t i, p, nnz = rp[n];
    int32_t ncol = 0;
    /* the pattern of A^T: rows j holding column i, listed under i */
    int32_t *trp = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    int32_t *tci = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nnz + 1));
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int64_t *seen = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 2));
    for (p = 0; p < nnz; ++p)
        trp[ci[p] + 1]++;
    for (i = 0; i < n; ++i)
        trp[i + 1] += trp[i];
    for (i = 0; i < n; ++i)
        fill[i] = trp[i];
    for (i = 0; i < n; ++i)
        for (p = rp[i]; p < rp[i + 1]; ++p)
            tci[fill[ci[p]]++] = (int32_t)i;
    /* seen[c] == i: colour c is taken by a neighbour of i numbered below i */
    for (i = 0; i < n + 2; ++i)
        seen[i] = -1;
    for (i = 0; i < n; ++i) {
        int32_t c = 0;
        for (p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] < i)
                seen[color[ci[p]]] = i;
        for (p = trp[i]; p < trp[i + 1]; ++p)
            if (tci[p] < i)
                seen[color[tci[p]]] = i;
        while (seen[c] == i)
            ++c;
        color[i] = c;
        if (c + 1 > ncol)
            ncol = c + 1;
    }
    free(trp);
    free(tci);
    free(fill);
    free(seen);
    return ncol;
}

/* The ordering by colour: perm[k] is the row of A placed at position k;
 * rows are grouped by colour in ascending colour, and keep their order
 * within a colour. */
void or_color_perm(int64_t n, const int32_t *color, int32_t ncol, int32_t *perm)
{
    int64_t i;
    int32_t c, k = 0;
    for (c = 0; c < ncol; ++c)
        for (i = 0; i < n; ++i)
            if (color[i] == c)
                perm[k++] = (int32_t)i;
}

/* B = P A P^T for the permutation perm (perm[k] = the row of A placed at
 * k): b_kl = a_{perm[k], perm[l]}, stored with each row's columns in
 * ascending order.  brp[n+1], bci[nnz], bval[nnz*C]. */
void or_csr_permute(int64_t n, const int32_t *rp, const int32_t *ci, const double *val,
                    int C, const int32_t *perm, int32_t *brp, int32_t *bci, double *bval)
{
    int64_t k, p, q;
    int v;
    int32_t *iperm = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    for (k = 0; k < n; ++k)
        iperm[perm[k]] = (int32_t)k;
    brp[0] = 0;
    for (k = 0; k < n; ++k)
        brp[k + 1] = brp[k] + (rp[perm[k] + 1] - rp[perm[k]]);
    for (k = 0; k < n; ++k) {
        int64_t a = rp[perm[k]], len = rp[perm[k] + 1] - a, o = brp[k];
        /* row perm[k] with its columns renamed, then sorted by insertion */
        for (p = 0; p < len; ++p) {
            int32_t col = iperm[ci[a + p]];
            double w[2];
            for (v = 0; v < C; ++v)
                w[v] = val[(a + p) * C + v];
            q = p;
            while (q > 0 && bci[o + q - 1] > col) {
                bci[o + q] = bci[o + q - 1];
                for (v = 0; v < C; ++v)
                    bval[(o + q) * C + v] = bval[(o + q - 1) * C + v];
                --q;
            }
            bci[o + q] = col;
            for (v = 0; v < C; ++v)
                bval[(o + q) * C + v] = w[v];
        }
    }
    free(iperm);
}
