// mp.hpp -- multi-component binary64 arithmetic for gfx950 (device + host).
//
// A K-limb number is double[K], leading limb first: K = 1 binary64, 2 DD,
// 3 TD, 4 QD (the formats of Section 2 of Kouya, arXiv 2504.14498).  All
// operations are built from the error-free transforms TwoSum and TwoProd
// (the latter with the hardware FMA) on the FP64 vector units.  The whole
// library is compiled with -ffp-contract=off: fma() appears only where an
// algorithm asks for it, and every other operation is one IEEE-rounded
// binary64 operation.
//
//  K = 2 : the double-word algorithms of Joldes, Muller and Popescu (ACM
//          TOMS 44(2), 2017): AccurateDWPlusDW (add), DWTimesFP3 (times a
//          binary64), DWTimesDW3 (times a double-word), DWDivFP3 and DWDivDW2
//          (the latter with DWTimesFP3 for its inner product).
//  K = 3, 4 : truncated floating-point expansions.  Exact partial terms are
//          formed with TwoSum/TwoProd and renormalised to K limbs by VecSum
//          followed by a VecSumErrBranch-style extraction (Joldes, Marty,
//          Muller, Popescu, IEEE TC 65(4), 2016) in which the tail beyond
//          K-1 limbs is added into the last limb.  Division is long division
//          with K+1 quotient terms.
//
// Operand order is part of the definition (several algorithms are not
// symmetric): mul(s, x) with s the scalar of a scalar-vector update;
// mul_f(x, f) with f a matrix/factor value and x the vector operand.
#pragma once
#include <hip/hip_runtime.h>

#define MPK_HD __host__ __device__ __forceinline__

namespace mpk {

// ---------------------------------------------------------------- EFTs
MPK_HD void two_sum(double a, double b, double &s, double &e) {
  double x = a + b;
  double bb = x - a;
  double ab = x - bb;
  e = (a - ab) + (b - bb);
  s = x;
}

MPK_HD void fast_two_sum(double a, double b, double &s, double &e) {
  double x = a + b;
  e = b - (x - a);
  s = x;
}

MPK_HD void two_prod(double a, double b, double &p, double &e) {
  double x = a * b;
  e = __builtin_fma(a, b, -x);
  p = x;
}

template <int K> struct mp { double v[K]; };

template <int K> MPK_HD mp<K> mp_zero() {
  mp<K> z;
#pragma unroll
  for (int i = 0; i < K; ++i) z.v[i] = 0.0;
  return z;
}

template <int K> MPK_HD mp<K> mp_from(double a) {
  mp<K> z = mp_zero<K>();
  z.v[0] = a;
  return z;
}

template <int K> MPK_HD mp<K> neg(const mp<K> &x) {
  mp<K> z;
#pragma unroll
  for (int i = 0; i < K; ++i) z.v[i] = -x.v[i];
  return z;
}

template <int K> MPK_HD bool is_zero(const mp<K> &x) {
  bool z = true;
#pragma unroll
  for (int i = 0; i < K; ++i) z = z && (x.v[i] == 0.0);
  return z;
}

// --------------------------------------------------------- double-word
MPK_HD void dw_add(const double *x, const double *y, double *z) {
  double sh, sl, th, tl, c, vh, vl, w;
  two_sum(x[0], y[0], sh, sl);
  two_sum(x[1], y[1], th, tl);
  c = sl + th;
  fast_two_sum(sh, c, vh, vl);
  w = tl + vl;
  fast_two_sum(vh, w, z[0], z[1]);
}

MPK_HD void dw_mul_fp(const double *x, double y, double *z) {
  double ch, cl1, cl3;
  two_prod(x[0], y, ch, cl1);
  cl3 = __builtin_fma(x[1], y, cl1);
  fast_two_sum(ch, cl3, z[0], z[1]);
}

MPK_HD void dw_mul(const double *x, const double *y, double *z) {
  double ch, cl1, tl0, tl1, cl2, cl3;
  two_prod(x[0], y[0], ch, cl1);
  tl0 = x[1] * y[1];
  tl1 = __builtin_fma(x[0], y[1], tl0);
  cl2 = __builtin_fma(x[1], y[0], tl1);
  cl3 = cl1 + cl2;
  fast_two_sum(ch, cl3, z[0], z[1]);
}

MPK_HD void dw_div_fp(const double *x, double y, double *z) {
  double th, ph, pl, dh, dt, d, tl;
  th = x[0] / y;
  two_prod(th, y, ph, pl);
  dh = x[0] - ph;
  dt = dh - pl;
  d = dt + x[1];
  tl = d / y;
  fast_two_sum(th, tl, z[0], z[1]);
}

MPK_HD void dw_div(const double *x, const double *y, double *z) {
  double th, r[2], ph, dl, d, tl;
  th = x[0] / y[0];
  dw_mul_fp(y, th, r);
  ph = x[0] - r[0];
  dl = x[1] - r[1];
  d = ph + dl;
  tl = d / y[0];
  fast_two_sum(th, tl, z[0], z[1]);
}

// ------------------------------------------------- truncated expansions
// Select-based store into z[j] for a run-time j (keeps z in registers).
template <int K> MPK_HD void put(double *z, int j, double v) {
#pragma unroll
  for (int q = 0; q < K; ++q) z[q] = (q == j) ? v : z[q];
}

// Renormalise M terms into K limbs (VecSum, then limb extraction).
template <int M, int K> MPK_HD mp<K> renorm(const double *t) {
  double e[M];
  double s = t[M - 1];
#pragma unroll
  for (int i = M - 2; i >= 0; --i) two_sum(t[i], s, s, e[i + 1]);
  e[0] = s;
  mp<K> z = mp_zero<K>();
  int j = 0;
  s = e[0];
#pragma unroll
  for (int i = 1; i < M; ++i) {
    if (j == K - 1) {
      s = s + e[i];
    } else {
      double r, f;
      two_sum(s, e[i], r, f);
      if (f != 0.0) {
        put<K>(z.v, j, r);
        ++j;
        s = f;
      } else {
        s = r;
      }
    }
  }
  put<K>(z.v, j, s);
  return z;
}

template <int K> MPK_HD mp<K> ex_add(const mp<K> &x, const mp<K> &y) {
  double t[2 * K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    t[2 * i] = x.v[i];
    t[2 * i + 1] = y.v[i];
  }
  return renorm<2 * K, K>(t);
}

template <int K> MPK_HD mp<K> ex_mul_fp(const mp<K> &x, double a) {
  double t[2 * K];
#pragma unroll
  for (int i = 0; i < K; ++i) two_prod(x.v[i], a, t[2 * i], t[2 * i + 1]);
  return renorm<2 * K, K>(t);
}

// Number of terms of ex_mul for a KX-limb by KY-limb product to K limbs.
template <int K, int KX, int KY> constexpr int ex_mul_terms() {
  int m = 0, nerr = 0;
  for (int s = 0; s <= K; ++s) {
    int nnew = 0;
    m += nerr;
    for (int i = 0; i <= s; ++i) {
      int j = s - i;
      if (i >= KX || j >= KY) continue;
      ++m;
      if (s < K) ++nnew;
    }
    nerr = nnew;
  }
  return m;
}

// Product by order class s = i + j: for s < K the exact TwoProd of x_i y_j
// (product in class s, error in class s + 1), for s == K plain products;
// within a class the errors of class s - 1 come first, then the products
// in ascending i.
template <int K, int KX, int KY>
MPK_HD mp<K> ex_mul(const double *x, const double *y) {
  constexpr int M = ex_mul_terms<K, KX, KY>();
  double t[M];
  double err[K + 1];
  int nerr = 0, m = 0;
#pragma unroll
  for (int s = 0; s <= K; ++s) {
    double nerrv[K + 1];
    int nnew = 0;
#pragma unroll
    for (int q = 0; q < K + 1; ++q)
      if (q < nerr) t[m++] = err[q];
#pragma unroll
    for (int i = 0; i <= s; ++i) {
      const int j = s - i;
      if (i >= KX || j >= KY) continue;
      if (s < K) {
        double p, e;
        two_prod(x[i], y[j], p, e);
        t[m++] = p;
        nerrv[nnew++] = e;
      } else {
        t[m++] = x[i] * y[j];
      }
    }
#pragma unroll
    for (int q = 0; q < K + 1; ++q)
      if (q < nnew) err[q] = nerrv[q];
    nerr = nnew;
  }
  return renorm<M, K>(t);
}

// ------------------------------------------------------ dispatch over K
template <int K> MPK_HD mp<K> add(const mp<K> &x, const mp<K> &y) {
  if constexpr (K == 1) {
    mp<1> z;
    z.v[0] = x.v[0] + y.v[0];
    return z;
  } else if constexpr (K == 2) {
    mp<2> z;
    dw_add(x.v, y.v, z.v);
    return z;
  } else {
    return ex_add<K>(x, y);
  }
}

template <int K> MPK_HD mp<K> sub(const mp<K> &x, const mp<K> &y) { return add<K>(x, neg<K>(y)); }

// x (K limbs) times a binary64 value a.
template <int K> MPK_HD mp<K> mul_fp(const mp<K> &x, double a) {
  if constexpr (K == 1) {
    mp<1> z;
    z.v[0] = x.v[0] * a;
    return z;
  } else if constexpr (K == 2) {
    mp<2> z;
    dw_mul_fp(x.v, a, z.v);
    return z;
  } else {
    return ex_mul_fp<K>(x, a);
  }
}

// x (K limbs) times y (KY <= K limbs).
template <int K, int KY> MPK_HD mp<K> mul_k(const mp<K> &x, const double *y) {
  if constexpr (KY == 1) {
    return mul_fp<K>(x, y[0]);
  } else if constexpr (K == 2) {
    mp<2> z;
    dw_mul(x.v, y, z.v);
    return z;
  } else {
    return ex_mul<K, K, KY>(x.v, y);
  }
}

// Working-precision product (s the scalar operand).
template <int K> MPK_HD mp<K> mul(const mp<K> &s, const mp<K> &x) {
  if constexpr (K == 1) {
    mp<1> z;
    z.v[0] = s.v[0] * x.v[0];
    return z;
  } else if constexpr (K == 2) {
    mp<2> z;
    dw_mul(s.v, x.v, z.v);
    return z;
  } else {
    return ex_mul<K, K, K>(s.v, x.v);
  }
}

// x (K limbs) divided by y (KY <= K limbs).
template <int K, int KY> MPK_HD mp<K> div_k(const mp<K> &x, const double *y) {
  if constexpr (K == 1) {
    mp<1> z;
    z.v[0] = x.v[0] / y[0];
    return z;
  } else if constexpr (K == 2 && KY == 1) {
    mp<2> z;
    dw_div_fp(x.v, y[0], z.v);
    return z;
  } else if constexpr (K == 2) {
    mp<2> z;
    dw_div(x.v, y, z.v);
    return z;
  } else {
    mp<K> r = x, yk = mp_zero<K>();
#pragma unroll
    for (int i = 0; i < KY; ++i) yk.v[i] = y[i];
    double q[K + 1];
    q[0] = r.v[0] / yk.v[0];
#pragma unroll
    for (int k = 1; k <= K; ++k) {
      mp<K> p = ex_mul_fp<K>(yk, q[k - 1]);
      r = ex_add<K>(r, neg<K>(p));
      q[k] = r.v[0] / yk.v[0];
    }
    return renorm<K + 1, K>(q);
  }
}

template <int K> MPK_HD mp<K> div(const mp<K> &x, const mp<K> &y) { return div_k<K, K>(x, y.v); }

// ------------------------------------------------------------ elements
// A vector element: C components (re[, im]) of K limbs.
template <int C, int K> struct el { mp<K> c[C]; };

template <int C, int K> MPK_HD el<C, K> el_zero() {
  el<C, K> z;
#pragma unroll
  for (int c = 0; c < C; ++c) z.c[c] = mp_zero<K>();
  return z;
}

template <int C, int K> MPK_HD el<C, K> el_add(const el<C, K> &x, const el<C, K> &y) {
  el<C, K> z;
#pragma unroll
  for (int c = 0; c < C; ++c) z.c[c] = add<K>(x.c[c], y.c[c]);
  return z;
}

template <int C, int K> MPK_HD el<C, K> el_sub(const el<C, K> &x, const el<C, K> &y) {
  el<C, K> z;
#pragma unroll
  for (int c = 0; c < C; ++c) z.c[c] = sub<K>(x.c[c], y.c[c]);
  return z;
}

template <int C, int K> MPK_HD el<C, K> el_conj(const el<C, K> &x) {
  el<C, K> z = x;
  if constexpr (C == 2) z.c[1] = neg<K>(x.c[1]);
  return z;
}

template <int C, int K> MPK_HD bool el_is_zero(const el<C, K> &x) {
  bool z = true;
#pragma unroll
  for (int c = 0; c < C; ++c) z = z && is_zero<K>(x.c[c]);
  return z;
}

// Product of a matrix or factor value f (C components of KF limbs, layout
// re[KF] then im[KF]) with a vector element x: re = fr*xr - fi*xi and
// im = fr*xi + fi*xr, each product rounded to K limbs first.
template <int C, int K, int KF>
MPK_HD el<C, K> el_mul_f(const double *f, const el<C, K> &x) {
  if constexpr (C == 1) {
    el<1, K> z;
    z.c[0] = mul_k<K, KF>(x.c[0], f);
    return z;
  } else {
    el<2, K> z;
    mp<K> p = mul_k<K, KF>(x.c[0], f);
    mp<K> q = mul_k<K, KF>(x.c[1], f + KF);
    z.c[0] = sub<K>(p, q);
    p = mul_k<K, KF>(x.c[1], f);
    q = mul_k<K, KF>(x.c[0], f + KF);
    z.c[1] = add<K>(p, q);
    return z;
  }
}

// Working-precision product s * x (s the scalar).
template <int C, int K> MPK_HD el<C, K> el_mul(const el<C, K> &s, const el<C, K> &x) {
  if constexpr (C == 1) {
    el<1, K> z;
    z.c[0] = mul<K>(s.c[0], x.c[0]);
    return z;
  } else {
    el<2, K> z;
    mp<K> p = mul<K>(s.c[0], x.c[0]);
    mp<K> q = mul<K>(s.c[1], x.c[1]);
    z.c[0] = sub<K>(p, q);
    p = mul<K>(s.c[0], x.c[1]);
    q = mul<K>(s.c[1], x.c[0]);
    z.c[1] = add<K>(p, q);
    return z;
  }
}

// x / d with d of KD limbs per component: real case a plain division, the
// complex case x conj(d) / |d|^2 in K limbs (no Smith scaling).  Squaring
// |d| leaves the binary64 range when d's leading limbs are outside
// [2^-300, 2^300]; then d is scaled by 2^-e first (exact) and the quotient
// by 2^-e afterwards, x / d = (x / (d 2^-e)) 2^-e.  Inside that range e = 0
// and the scalings are identities, so the direct formula's results stand.
template <int C, int K, int KD>
MPK_HD el<C, K> el_div_k(const el<C, K> &x, const double *d) {
  if constexpr (C == 1) {
    el<1, K> z;
    z.c[0] = div_k<K, KD>(x.c[0], d);
    return z;
  } else {
    const double mg = fmax(fabs(d[0]), fabs(d[KD]));
    const int e = (isfinite(mg) && mg != 0.0 && (mg < 0x1p-300 || mg > 0x1p300)) ? ilogb(mg) : 0;
    double ds[2 * KD];
#pragma unroll
    for (int i = 0; i < 2 * KD; ++i) ds[i] = ldexp(d[i], -e);
    mp<K> dr = mp_zero<K>(), di = mp_zero<K>();
#pragma unroll
    for (int i = 0; i < KD; ++i) {
      dr.v[i] = ds[i];
      di.v[i] = ds[KD + i];
    }
    mp<K> den = add<K>(mul_k<K, KD>(dr, ds), mul_k<K, KD>(di, ds + KD));
    mp<K> nr = add<K>(mul_k<K, KD>(x.c[0], ds), mul_k<K, KD>(x.c[1], ds + KD));
    mp<K> ni = sub<K>(mul_k<K, KD>(x.c[1], ds), mul_k<K, KD>(x.c[0], ds + KD));
    el<2, K> z;
    z.c[0] = div<K>(nr, den);
    z.c[1] = div<K>(ni, den);
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int k = 0; k < K; ++k) z.c[c].v[k] = ldexp(z.c[c].v[k], -e);
    return z;
  }
}

template <int C, int K> MPK_HD el<C, K> el_div(const el<C, K> &x, const el<C, K> &d) {
  double dd[C * K];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int k = 0; k < K; ++k) dd[c * K + k] = d.c[c].v[k];
  return el_div_k<C, K, K>(x, dd);
}

// conj(a) * b, the term of an inner product <a, b> = sum conj(a_i) b_i.
template <int C, int K> MPK_HD el<C, K> el_cdot_term(const el<C, K> &a, const el<C, K> &b) {
  return el_mul<C, K>(el_conj<C, K>(a), b);
}

// ------------------------------------------------------- memory access
template <int C, int K> MPK_HD el<C, K> el_load(const double *p) {
  el<C, K> z;
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int k = 0; k < K; ++k) z.c[c].v[k] = p[c * K + k];
  return z;
}

template <int C, int K> MPK_HD void el_store(double *p, const el<C, K> &x) {
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int k = 0; k < K; ++k) p[c * K + k] = x.c[c].v[k];
}

}  // namespace mpk
