// krylov.hip -- device-driven preconditioned product-type Krylov solvers
// (Section 3: BiCG as Algorithm 3; CGS, BiCGSTAB and GPBiCG in right-
// preconditioned form with the unpreconditioned residual).
//
// Every scalar of a method lives in device memory (KState) and is computed
// by a one-workgroup "scalar" kernel from fixed-order reduction partials,
// so a pass needs no host round trip.  Each kernel returns at once when the
// solve is done; kernels of the true-residual confirmation run only in the
// phase that asked for it.  The host enqueues passes in growing batches and
// polls the done word between batches (or replays a captured hipGraph).
//
// Per-element formulas and the order of the scalar operations follow the
// method statements exactly; the only difference from a sequential
// evaluation is the reduction tree of the inner products.
#include <cmath>
#include <cstdlib>

#include "kernels.hpp"

namespace mpk {

enum { GATE_ANY = -1 };

template <int C, int K> __device__ __forceinline__ el<C, K> sget(const KState *st, int slot) {
  return el_load<C, K>(st->s[slot]);
}
template <int C, int K> __device__ __forceinline__ void sset(KState *st, int slot, const el<C, K> &v) {
  el_store<C, K>(st->s[slot], v);
}
template <int C, int K> __device__ __forceinline__ el<C, K> ld(const double *p, int64_t i) {
  return el_load<C, K>(p + size_t(i) * C * K);
}
template <int C, int K> __device__ __forceinline__ void stv(double *p, int64_t i, const el<C, K> &v) {
  el_store<C, K>(p + size_t(i) * C * K, v);
}

// Stopping rule of Algorithm 3 on leading limbs: ||r|| < eps_r ||r0|| + eps_a.
__device__ __forceinline__ bool stop_test(const KState *st, double nr2) {
  return sqrt(nr2) < st->eps_r * sqrt(st->nr0sq) + st->eps_a;
}

__device__ __forceinline__ void finish(KState *st, int status) {
  st->status = status;
  st->done = 1;
}

__device__ __forceinline__ void record(KState *st, double nr2) {
  st->last_nr2 = nr2;
  if (st->hist && st->iter >= 1 && st->iter <= st->hist_len) st->hist[st->iter - 1] = nr2;
}

// Row kernel with the solve's gating: skipped when done, or when `gate` is
// a phase and the solve is not in it.
template <int C, int K, int ND, class Op>
__global__ __launch_bounds__(BLOCK) void srow_kernel(int64_t n, Op op, const KState *st, int gate,
                                                     double *partials) {
  if (st->done || (gate >= 0 && st->phase != gate)) return;
  const int64_t lb = xcd_block();
  if (lb * BLOCK >= n) return;
  const int64_t i = lb * BLOCK + threadIdx.x;
  el<C, K> d[ND > 0 ? ND : 1];
#pragma unroll
  for (int q = 0; q < (ND > 0 ? ND : 1); ++q) d[q] = el_zero<C, K>();
  if (i < n) op(i, st, d);
  if constexpr (ND > 0) block_reduce<C, K, ND>(d, partials + size_t(lb) * ND * C * K);
}

// ------------------------------------------------------- shared ops
// r = b - A x (written to r and r2 when given); dots ||r||^2, ||b||^2.
template <int C, int K> struct ResidualOp {
  const int32_t *rp, *ci;
  const double *val, *b, *x;
  double *r, *r2;
  __device__ void operator()(int64_t i, const KState *, el<C, K> *d) const {
    el<C, K> bi = ld<C, K>(b, i);
    el<C, K> ri = el_sub<C, K>(bi, row_spmv<C, K>(i, rp, ci, val, x));
    if (r) stv<C, K>(r, i, ri);
    if (r2) stv<C, K>(r2, i, ri);
    d[0] = el_cdot_term<C, K>(ri, ri);
    d[1] = el_cdot_term<C, K>(bi, bi);
  }
};

// y = A x; d0 = <a, y>.
template <int C, int K> struct SpmvDotAY {
  const int32_t *rp, *ci;
  const double *val, *x, *a;
  double *y;
  __device__ void operator()(int64_t i, const KState *, el<C, K> *d) const {
    el<C, K> yi = row_spmv<C, K>(i, rp, ci, val, x);
    stv<C, K>(y, i, yi);
    d[0] = el_cdot_term<C, K>(ld<C, K>(a, i), yi);
  }
};

// y = A x; d0 = <y, a>, d1 = <y, y>.
template <int C, int K> struct SpmvDotYA {
  const int32_t *rp, *ci;
  const double *val, *x, *a;
  double *y;
  __device__ void operator()(int64_t i, const KState *, el<C, K> *d) const {
    el<C, K> yi = row_spmv<C, K>(i, rp, ci, val, x);
    stv<C, K>(y, i, yi);
    d[0] = el_cdot_term<C, K>(yi, ld<C, K>(a, i));
    d[1] = el_cdot_term<C, K>(yi, yi);
  }
};

template <int C, int K> struct ZeroOp {
  double *v[8];
  int nv;
  __device__ void operator()(int64_t i, const KState *, el<C, K> *) const {
    for (int q = 0; q < nv; ++q) stv<C, K>(v[q], i, el_zero<C, K>());
  }
};

// x_tmp = x + alpha p^ (candidate solution of BiCGSTAB's half step).
template <int C, int K> struct AxpyTmpOp {
  const double *x, *ph;
  double *xt;
  __device__ void operator()(int64_t i, const KState *st, el<C, K> *) const {
    el<C, K> al = sget<C, K>(st, S_ALPHA);
    stv<C, K>(xt, i, el_add<C, K>(ld<C, K>(x, i), el_mul<C, K>(al, ld<C, K>(ph, i))));
  }
};

// ------------------------------------------------------- scalar kernels
// One workgroup; modes name the step of a pass.  Partials hold the dots of
// the preceding row kernel.
enum Mode {
  M_INIT = 0,     // d0 = ||r0||^2 = <r~, r0>, d1 = ||b||^2
  M_ALPHA,        // d0 = <r~, v> (BiCGSTAB/CGS/GPBiCG) or <p~, q> (BiCG)
  M_S_TEST,       // BiCGSTAB: d0 = ||s||^2
  M_HALF,         // BiCGSTAB: d0 = ||b - A x_tmp||^2
  M_OMEGA,        // BiCGSTAB: d0 = <t, s>, d1 = <t, t>
  M_R_TEST,       // d0 = ||r||^2, d1 = <r~, r> (not BiCG)
  M_FULL,         // d0 = ||b - A x||^2
  M_BICG_RHO,     // BiCG: d0 = <z~, r>   (first: initial rho)
  M_ZETA          // GPBiCG: d0..d5 = <s,s>, <s,t>, <y,y>, <s,y>, <y,s>, <y,t>
};

// Continuation after a failed (or absent) convergence test at the end of
// a pass: the scalars that start the next pass.
template <int C, int K>
__device__ void continue_pass(KState *st, int method) {
  const el<C, K> rho = sget<C, K>(st, S_RHO);
  const el<C, K> rho_new = sget<C, K>(st, S_D7);
  if (method == MPK_BICGSTAB) {
    const el<C, K> om = sget<C, K>(st, S_OMEGA);
    if (el_is_zero<C, K>(om)) return finish(st, MPK_BREAKDOWN);
  }
  if (method == MPK_GPBICG) {
    const el<C, K> ze = sget<C, K>(st, S_ZETA);
    if (el_is_zero<C, K>(ze)) return finish(st, MPK_BREAKDOWN);
  }
  if (method == MPK_BICGSTAB) {
    el<C, K> q1 = el_div<C, K>(rho_new, rho);
    el<C, K> q2 = el_div<C, K>(sget<C, K>(st, S_ALPHA), sget<C, K>(st, S_OMEGA));
    sset<C, K>(st, S_BETA, el_mul<C, K>(q1, q2));
  } else if (method == MPK_CGS) {
    sset<C, K>(st, S_BETA, el_div<C, K>(rho_new, rho));
  } else if (method == MPK_GPBICG) {
    el<C, K> a1 = el_div<C, K>(sget<C, K>(st, S_ALPHA), sget<C, K>(st, S_ZETA));
    el<C, K> a2 = el_div<C, K>(rho_new, rho);
    sset<C, K>(st, S_BETA, el_mul<C, K>(a1, a2));
  }
  sset<C, K>(st, S_RHO, rho_new);
  st->first = 0;
  st->phase = ST_RUNNING;
  if (el_is_zero<C, K>(rho_new) && st->iter < st->max_iter) {
    st->iter += 1;
    return finish(st, MPK_BREAKDOWN);
  }
}

template <int C, int K, int ND>
__device__ __forceinline__ void get_dots(const double *partials, int nblk, el<C, K> (&d)[ND]) {
  reduce_partials<C, K, ND>(partials, nblk, d);
}

template <int C, int K>
__global__ __launch_bounds__(BLOCK) void scalar_kernel(int mode, int method, KState *st,
                                                       const double *partials, int nblk) {
  if (st->done) return;
  switch (mode) {
    case M_INIT: {
      el<C, K> d[2];
      get_dots<C, K, 2>(partials, nblk, d);
      if (threadIdx.x) return;
      st->nr0sq = d[0].c[0].v[0];
      st->nbsq = d[1].c[0].v[0];
      st->last_nr2 = st->nr0sq;
      st->true_nr2 = -1.0;
      st->iter = 0;
      st->phase = ST_RUNNING;
      st->status = MPK_NOT_CONVERGED;
      st->x_in_tmp = 0;
      st->first = 1;
      sset<C, K>(st, S_RHO, d[0]);
      sset<C, K>(st, S_BETA, el_zero<C, K>());
      if (st->max_iter <= 0) return finish(st, MPK_NOT_CONVERGED);
      if (method != MPK_BICG && el_is_zero<C, K>(d[0])) {
        st->iter = 1;
        return finish(st, MPK_BREAKDOWN);
      }
      return;
    }
    case M_BICG_RHO: {
      el<C, K> d[1];
      get_dots<C, K, 1>(partials, nblk, d);
      if (threadIdx.x) return;
      if (st->first) {
        sset<C, K>(st, S_RHO, d[0]);
        st->first = 0;
      } else {
        sset<C, K>(st, S_BETA, el_div<C, K>(d[0], sget<C, K>(st, S_RHO)));
        sset<C, K>(st, S_RHO, d[0]);
      }
      return;
    }
    case M_ALPHA: {
      el<C, K> d[1];
      get_dots<C, K, 1>(partials, nblk, d);
      if (threadIdx.x) return;
      if (st->iter >= st->max_iter) return finish(st, MPK_NOT_CONVERGED);
      st->iter += 1;
      const el<C, K> rho = sget<C, K>(st, S_RHO);
      if (el_is_zero<C, K>(d[0]) || (method == MPK_BICG && el_is_zero<C, K>(rho)))
        return finish(st, MPK_BREAKDOWN);
      sset<C, K>(st, S_SIGMA, d[0]);
      el<C, K> al = el_div<C, K>(rho, d[0]);
      sset<C, K>(st, S_ALPHA, al);
      if (method == MPK_GPBICG) sset<C, K>(st, S_D6, el_mul<C, K>(al, sget<C, K>(st, S_BETA)));
      return;
    }
    case M_S_TEST: {
      el<C, K> d[1];
      get_dots<C, K, 1>(partials, nblk, d);
      if (threadIdx.x) return;
      const double nr2 = d[0].c[0].v[0];
      st->last_nr2 = nr2;
      if (stop_test(st, nr2)) st->phase = ST_CHECK_HALF;
      return;
    }
    case M_HALF: {
      if (st->phase != ST_CHECK_HALF) return;
      el<C, K> d[2];
      get_dots<C, K, 2>(partials, nblk, d);
      if (threadIdx.x) return;
      st->true_nr2 = d[0].c[0].v[0];
      if (stop_test(st, st->true_nr2)) {
        record(st, st->last_nr2);
        st->x_in_tmp = 1;
        return finish(st, MPK_OK);
      }
      st->phase = ST_RUNNING;
      return;
    }
    case M_OMEGA: {
      el<C, K> d[2];
      get_dots<C, K, 2>(partials, nblk, d);
      if (threadIdx.x) return;
      if (el_is_zero<C, K>(d[1])) return finish(st, MPK_BREAKDOWN);
      sset<C, K>(st, S_OMEGA, el_div<C, K>(d[0], d[1]));
      return;
    }
    case M_R_TEST: {
      el<C, K> d[2];
      get_dots<C, K, 2>(partials, nblk, d);
      if (threadIdx.x) return;
      const double nr2 = d[0].c[0].v[0];
      record(st, nr2);
      if (method == MPK_BICG) {
        if (stop_test(st, nr2)) st->phase = ST_CHECK_FULL;
        return;
      }
      sset<C, K>(st, S_D7, d[1]);
      if (stop_test(st, nr2)) {
        st->phase = ST_CHECK_FULL;
        return;
      }
      continue_pass<C, K>(st, method);
      return;
    }
    case M_FULL: {
      if (st->phase != ST_CHECK_FULL) return;
      el<C, K> d[2];
      get_dots<C, K, 2>(partials, nblk, d);
      if (threadIdx.x) return;
      st->true_nr2 = d[0].c[0].v[0];
      if (stop_test(st, st->true_nr2)) return finish(st, MPK_OK);
      st->phase = ST_RUNNING;
      if (method != MPK_BICG) continue_pass<C, K>(st, method);
      return;
    }
    case M_ZETA: {
      el<C, K> d[6];
      get_dots<C, K, 6>(partials, nblk, d);
      if (threadIdx.x) return;
      const el<C, K> &ss = d[0], &stt = d[1], &yy = d[2], &sy = d[3], &ys = d[4], &yt = d[5];
      if (st->first) {
        if (el_is_zero<C, K>(ss)) return finish(st, MPK_BREAKDOWN);
        sset<C, K>(st, S_ZETA, el_div<C, K>(stt, ss));
        sset<C, K>(st, S_ETA, el_zero<C, K>());
        return;
      }
      el<C, K> den = el_sub<C, K>(el_mul<C, K>(ss, yy), el_mul<C, K>(sy, ys));
      if (el_is_zero<C, K>(den)) return finish(st, MPK_BREAKDOWN);
      el<C, K> num = el_sub<C, K>(el_mul<C, K>(yy, stt), el_mul<C, K>(sy, yt));
      sset<C, K>(st, S_ZETA, el_div<C, K>(num, den));
      num = el_sub<C, K>(el_mul<C, K>(ss, yt), el_mul<C, K>(ys, stt));
      sset<C, K>(st, S_ETA, el_div<C, K>(num, den));
      return;
    }
  }
}

// --------------------------------------------------------- BiCGSTAB ops
template <int C, int K> struct BsP {   // p = r + beta (p - omega v); first pass p = r
  const double *r, *v;
  double *p;
  __device__ void operator()(int64_t i, const KState *st, el<C, K> *) const {
    el<C, K> ri = ld<C, K>(r, i);
    if (st->first) {
      stv<C, K>(p, i, ri);
      return;
    }
    el<C, K> be = sget<C, K>(st, S_BETA), om = sget<C, K>(st, S_OMEGA);
    el<C, K> t = el_sub<C, K>(ld<C, K>(p, i), el_mul<C, K>(om, ld<C, K>(v, i)));
    stv<C, K>(p, i, el_add<C, K>(ri, el_mul<C, K>(be, t)));
  }
};

template <int C, int K> struct BsS {   // s = r - alpha v; d0 = ||s||^2
  const double *r, *v;
  double *s;
  __device__ void operator()(int64_t i, const KState *st, el<C, K> *d) const {
    el<C, K> al = sget<C, K>(st, S_ALPHA);
    el<C, K> si = el_sub<C, K>(ld<C, K>(r, i), el_mul<C, K>(al, ld<C, K>(v, i)));
    stv<C, K>(s, i, si);
    d[0] = el_cdot_term<C, K>(si, si);
  }
};

template <int C, int K> struct BsXR {  // x = (x + alpha p^) + omega s^; r = s - omega t
  const double *ph, *sh, *s, *t, *rt;
  double *x, *r;
  __device__ void operator()(int64_t i, const KState *st, el<C, K> *d) const {
    el<C, K> al = sget<C, K>(st, S_ALPHA), om = sget<C, K>(st, S_OMEGA);
    el<C, K> xi = el_add<C, K>(ld<C, K>(x, i), el_mul<C, K>(al, ld<C, K>(ph, i)));
    xi = el_add<C, K>(xi, el_mul<C, K>(om, ld<C, K>(sh, i)));
    stv<C, K>(x, i, xi);
    el<C, K> ri = el_sub<C, K>(ld<C, K>(s, i), el_mul<C, K>(om, ld<C, K>(t, i)));
    stv<C, K>(r, i, ri);
    d[0] = el_cdot_term<C, K>(ri, ri);
    d[1] = el_cdot_term<C, K>(ld<C, K>(rt, i), ri);
  }
};

// -------------------------------------------------------------- CGS ops
template <int C, int K> struct CgUP {  // u = r + beta q; p = u + beta (q + beta p)
  const double *r, *q;
  double *u, *p;
  __device__ void operator()(int64_t i, const KState *st, el<C, K> *) const {
    el<C, K> ri = ld<C, K>(r, i);
    if (st->first) {
      stv<C, K>(u, i, ri);
      stv<C, K>(p, i, ri);
      return;
    }
    el<C, K> be = sget<C, K>(st, S_BETA), qi = ld<C, K>(q, i);
    el<C, K> ui = el_add<C, K>(ri, el_mul<C, K>(be, qi));
    el<C, K> t = el_add<C, K>(qi, el_mul<C, K>(be, ld<C, K>(p, i)));
    stv<C, K>(u, i, ui);
    stv<C, K>(p, i, el_add<C, K>(ui, el_mul<C, K>(be, t)));
  }
};

template <int C, int K> struct CgQW {  // q = u - alpha v; w = u + q
  const double *u, *v;
  double *q, *w;
  __device__ void operator()(int64_t i, const KState *st, el<C, K> *) const {
    el<C, K> al = sget<C, K>(st, S_ALPHA), ui = ld<C, K>(u, i);
    el<C, K> qi = el_sub<C, K>(ui, el_mul<C, K>(al, ld<C, K>(v, i)));
    stv<C, K>(q, i, qi);
    stv<C, K>(w, i, el_add<C, K>(ui, qi));
  }
};

template <int C, int K> struct CgXR {  // x = x + alpha u^; r = r - alpha A u^
  const int32_t *rp, *ci;
  const double *val, *uh, *rt;
  double *x, *r;
  __device__ void operator()(int64_t i, const KState *st, el<C, K> *d) const {
    el<C, K> al = sget<C, K>(st, S_ALPHA);
    stv<C, K>(x, i, el_add<C, K>(ld<C, K>(x, i), el_mul<C, K>(al, ld<C, K>(uh, i))));
    el<C, K> aui = row_spmv<C, K>(i, rp, ci, val, uh);
    el<C, K> ri = el_sub<C, K>(ld<C, K>(r, i), el_mul<C, K>(al, aui));
    stv<C, K>(r, i, ri);
    d[0] = el_cdot_term<C, K>(ri, ri);
    d[1] = el_cdot_term<C, K>(ld<C, K>(rt, i), ri);
  }
};

// ------------------------------------------------------------- BiCG ops
template <int C, int K> struct BgInit {  // p = z, p~ = z~; d0 = <z~, r>
  const double *z, *zt, *r;
  double *p, *pt;
  __device__ void operator()(int64_t i, const KState *, el<C, K> *d) const {
    el<C, K> zti = ld<C, K>(zt, i);
    stv<C, K>(p, i, ld<C, K>(z, i));
    stv<C, K>(pt, i, zti);
    d[0] = el_cdot_term<C, K>(zti, ld<C, K>(r, i));
  }
};

template <int C, int K> struct BgUpd {  // x += alpha p; r -= alpha q; r~ -= conj(alpha) q~
  const double *p, *q, *qt;
  double *x, *r, *rt;
  __device__ void operator()(int64_t i, const KState *st, el<C, K> *d) const {
    el<C, K> al = sget<C, K>(st, S_ALPHA), ca = el_conj<C, K>(al);
    stv<C, K>(x, i, el_add<C, K>(ld<C, K>(x, i), el_mul<C, K>(al, ld<C, K>(p, i))));
    el<C, K> ri = el_sub<C, K>(ld<C, K>(r, i), el_mul<C, K>(al, ld<C, K>(q, i)));
    stv<C, K>(r, i, ri);
    stv<C, K>(rt, i, el_sub<C, K>(ld<C, K>(rt, i), el_mul<C, K>(ca, ld<C, K>(qt, i))));
    d[0] = el_cdot_term<C, K>(ri, ri);
    d[1] = el_zero<C, K>();
  }
};

template <int C, int K> struct BgDot {   // d0 = <z~, r>
  const double *zt, *r;
  __device__ void operator()(int64_t i, const KState *, el<C, K> *d) const {
    d[0] = el_cdot_term<C, K>(ld<C, K>(zt, i), ld<C, K>(r, i));
  }
};

template <int C, int K> struct BgP {     // p = z + beta p; p~ = z~ + conj(beta) p~
  const double *z, *zt;
  double *p, *pt;
  __device__ void operator()(int64_t i, const KState *st, el<C, K> *) const {
    el<C, K> be = sget<C, K>(st, S_BETA), cb = el_conj<C, K>(be);
    stv<C, K>(p, i, el_add<C, K>(ld<C, K>(z, i), el_mul<C, K>(be, ld<C, K>(p, i))));
    stv<C, K>(pt, i, el_add<C, K>(ld<C, K>(zt, i), el_mul<C, K>(cb, ld<C, K>(pt, i))));
  }
};

// ----------------------------------------------------------- GPBiCG ops
template <int C, int K> struct GpP {     // p = r + beta (p - u)
  const double *r, *u;
  double *p;
  __device__ void operator()(int64_t i, const KState *st, el<C, K> *) const {
    el<C, K> be = sget<C, K>(st, S_BETA);
    el<C, K> t = el_sub<C, K>(ld<C, K>(p, i), ld<C, K>(u, i));
    stv<C, K>(p, i, el_add<C, K>(ld<C, K>(r, i), el_mul<C, K>(be, t)));
  }
};

template <int C, int K> struct GpYT {    // y = ((t_old - r) - alpha w) + alpha q; t = r - alpha q
  const double *told, *r, *w, *q;
  double *y, *t;
  __device__ void operator()(int64_t i, const KState *st, el<C, K> *) const {
    el<C, K> al = sget<C, K>(st, S_ALPHA), ri = ld<C, K>(r, i), qi = ld<C, K>(q, i);
    el<C, K> a = el_sub<C, K>(ld<C, K>(told, i), ri);
    a = el_sub<C, K>(a, el_mul<C, K>(al, ld<C, K>(w, i)));
    stv<C, K>(y, i, el_add<C, K>(a, el_mul<C, K>(al, qi)));
    stv<C, K>(t, i, el_sub<C, K>(ri, el_mul<C, K>(al, qi)));
  }
};

template <int C, int K> struct GpS {     // s = A t^; six inner products
  const int32_t *rp, *ci;
  const double *val, *th, *t, *y;
  double *s;
  __device__ void operator()(int64_t i, const KState *, el<C, K> *d) const {
    el<C, K> si = row_spmv<C, K>(i, rp, ci, val, th);
    stv<C, K>(s, i, si);
    el<C, K> ti = ld<C, K>(t, i), yi = ld<C, K>(y, i);
    d[0] = el_cdot_term<C, K>(si, si);
    d[1] = el_cdot_term<C, K>(si, ti);
    d[2] = el_cdot_term<C, K>(yi, yi);
    d[3] = el_cdot_term<C, K>(si, yi);
    d[4] = el_cdot_term<C, K>(yi, si);
    d[5] = el_cdot_term<C, K>(yi, ti);
  }
};

template <int C, int K> struct GpUpd {
  const double *q, *told, *thold, *phold, *ph, *th, *t, *y, *s, *rt;
  double *u, *zh, *x, *r;
  __device__ void operator()(int64_t i, const KState *st, el<C, K> *d) const {
    const el<C, K> al = sget<C, K>(st, S_ALPHA), be = sget<C, K>(st, S_BETA);
    const el<C, K> ze = sget<C, K>(st, S_ZETA), et = sget<C, K>(st, S_ETA);
    const el<C, K> ab = sget<C, K>(st, S_D6);
    const el<C, K> ri = ld<C, K>(r, i);
    // u = zeta q + eta ((t_old - r) + beta u)
    el<C, K> a = el_sub<C, K>(ld<C, K>(told, i), ri);
    a = el_add<C, K>(a, el_mul<C, K>(be, ld<C, K>(u, i)));
    stv<C, K>(u, i, el_add<C, K>(el_mul<C, K>(ze, ld<C, K>(q, i)), el_mul<C, K>(et, a)));
    // v^ = ((z^ - alpha t^_old) - (alpha beta) p^_old) + alpha p^
    const el<C, K> phi = ld<C, K>(ph, i);
    el<C, K> vh = el_sub<C, K>(ld<C, K>(zh, i), el_mul<C, K>(al, ld<C, K>(thold, i)));
    vh = el_sub<C, K>(vh, el_mul<C, K>(ab, ld<C, K>(phold, i)));
    vh = el_add<C, K>(vh, el_mul<C, K>(al, phi));
    // z^ = zeta t^ + eta v^
    el<C, K> zhi = el_add<C, K>(el_mul<C, K>(ze, ld<C, K>(th, i)), el_mul<C, K>(et, vh));
    stv<C, K>(zh, i, zhi);
    // x = (x + alpha p^) + z^
    el<C, K> xi = el_add<C, K>(ld<C, K>(x, i), el_mul<C, K>(al, phi));
    stv<C, K>(x, i, el_add<C, K>(xi, zhi));
    // r = (t - eta y) - zeta s
    el<C, K> rn = el_sub<C, K>(ld<C, K>(t, i), el_mul<C, K>(et, ld<C, K>(y, i)));
    rn = el_sub<C, K>(rn, el_mul<C, K>(ze, ld<C, K>(s, i)));
    stv<C, K>(r, i, rn);
    d[0] = el_cdot_term<C, K>(rn, rn);
    d[1] = el_cdot_term<C, K>(ld<C, K>(rt, i), rn);
  }
};

template <int C, int K> struct GpW {     // w = s + beta q; shift t, p^, t^ to the "old" slots
  const double *s, *q, *t, *ph, *th;
  double *w, *told, *phold, *thold;
  __device__ void operator()(int64_t i, const KState *st, el<C, K> *) const {
    el<C, K> be = sget<C, K>(st, S_BETA);
    stv<C, K>(w, i, el_add<C, K>(ld<C, K>(s, i), el_mul<C, K>(be, ld<C, K>(q, i))));
    stv<C, K>(told, i, ld<C, K>(t, i));
    stv<C, K>(phold, i, ld<C, K>(ph, i));
    stv<C, K>(thold, i, ld<C, K>(th, i));
  }
};

// ------------------------------------------------------------ the driver
constexpr int NVEC = 16;

struct Layout {
  KState *st = nullptr;
  double *partials = nullptr;
  double *v[NVEC] = {};
  int32_t *abort = nullptr;
  Ilu0 ilu;
  int32_t *t_rp = nullptr, *t_ci = nullptr, *t_src = nullptr;  // A^H (BiCG)
  double *t_val = nullptr;
};

static int nvec_for(int method) {
  switch (method) {
    case MPK_BICG: return 10;
    case MPK_CGS: return 11;
    case MPK_BICGSTAB: return 10;
    default: return 15;
  }
}

// ext_ilu: the preconditioner is a caller's factor, so no ILU(0) part.
static size_t krylov_layout(int method, int C, int K, int KF, int64_t n, int64_t nnz, Bump &b,
                            Layout *L, bool ext_ilu = false) {
  Layout tmp;
  Layout &l = L ? *L : tmp;
  l.st = b.take<KState>(1);
  l.abort = b.take<int32_t>(64);
  l.partials = b.take<double>(size_t(nblocks(n)) * 6 * C * K);
  for (int q = 0; q < nvec_for(method); ++q) l.v[q] = b.take<double>(size_t(n) * C * K);
  if (KF > 0 && !ext_ilu)
    ilu0_layout(n, nnz, C, KF, method == MPK_BICG ? MPK_ILU0_ADJOINT : 0, b, &l.ilu);
  if (method == MPK_BICG) {
    l.t_rp = b.take<int32_t>(size_t(n) + 1);
    l.t_ci = b.take<int32_t>(size_t(nnz));
    l.t_src = b.take<int32_t>(size_t(nnz));
    l.t_val = b.take<double>(size_t(nnz) * C);
  }
  return b.off;
}

template <int C, int K> struct Solver {
  int method;
  int64_t n;
  const mpk_csr *A;
  const double *b;
  double *x;
  Layout L;
  bool precond;
  hipStream_t s;
  int nblk;

  template <int ND, class Op> void rows(Op op, int gate = GATE_ANY) {
    hipLaunchKernelGGL((srow_kernel<C, K, ND, Op>), dim3(xcd_grid(nblk)), dim3(BLOCK), 0, s, n, op,
                       (const KState *)L.st, gate, L.partials);
  }
  void scalar(int mode) {
    hipLaunchKernelGGL((scalar_kernel<C, K>), dim3(1), dim3(BLOCK), 0, s, mode, method, L.st,
                       (const double *)L.partials, nblk);
  }
  void apply(const double *r, double *z, int conj) {
    if (precond) ilu0_apply_launch(L.ilu, K, conj, r, z, nullptr, L.abort, &L.st->done, s);
  }
  double *V(int q) { return L.v[q]; }

  void residual(const double *xv, double *r, double *r2, int gate) {
    rows<2>(ResidualOp<C, K>{A->row_ptr, A->col_idx, A->val, b, xv, r, r2}, gate);
  }

  // ---- BiCGSTAB: v0 r, v1 r~, v2 p, v3 p^, v4 v, v5 s, v6 s^, v7 t, v8 x_tmp
  void setup_bicgstab() {
    residual(x, V(0), V(1), GATE_ANY);
    scalar(M_INIT);
  }
  void pass_bicgstab() {
    double *r = V(0), *rt = V(1), *p = V(2), *v = V(4), *sv = V(5), *t = V(7), *xt = V(8);
    double *ph = precond ? V(3) : p, *sh = precond ? V(6) : sv;
    rows<0>(BsP<C, K>{r, v, p});
    apply(p, ph, 0);
    rows<1>(SpmvDotAY<C, K>{A->row_ptr, A->col_idx, A->val, ph, rt, v});
    scalar(M_ALPHA);
    rows<1>(BsS<C, K>{r, v, sv});
    scalar(M_S_TEST);
    rows<0>(AxpyTmpOp<C, K>{x, ph, xt}, ST_CHECK_HALF);
    residual(xt, nullptr, nullptr, ST_CHECK_HALF);
    scalar(M_HALF);
    apply(sv, sh, 0);
    rows<2>(SpmvDotYA<C, K>{A->row_ptr, A->col_idx, A->val, sh, sv, t});
    scalar(M_OMEGA);
    rows<2>(BsXR<C, K>{ph, sh, sv, t, rt, x, r});
    scalar(M_R_TEST);
    residual(x, nullptr, nullptr, ST_CHECK_FULL);
    scalar(M_FULL);
  }

  // ---- CGS: v0 r, v1 r~, v2 u, v3 p, v4 q, v5 p^, v6 v, v7 u^, v8 w
  void setup_cgs() { setup_bicgstab(); }
  void pass_cgs() {
    double *r = V(0), *rt = V(1), *u = V(2), *p = V(3), *q = V(4), *v = V(6), *w = V(8);
    double *ph = precond ? V(5) : p, *uh = precond ? V(7) : w;
    rows<0>(CgUP<C, K>{r, q, u, p});
    apply(p, ph, 0);
    rows<1>(SpmvDotAY<C, K>{A->row_ptr, A->col_idx, A->val, ph, rt, v});
    scalar(M_ALPHA);
    rows<0>(CgQW<C, K>{u, v, q, w});
    apply(w, uh, 0);
    rows<2>(CgXR<C, K>{A->row_ptr, A->col_idx, A->val, uh, rt, x, r});
    scalar(M_R_TEST);
    residual(x, nullptr, nullptr, ST_CHECK_FULL);
    scalar(M_FULL);
  }

  // ---- BiCG: v0 r, v1 r~, v2 z, v3 z~, v4 p, v5 p~, v6 q, v7 q~
  void setup_bicg() {
    double *r = V(0), *rt = V(1);
    double *z = precond ? V(2) : r, *zt = precond ? V(3) : rt;
    residual(x, r, rt, GATE_ANY);
    scalar(M_INIT);
    apply(r, z, 0);
    apply(rt, zt, 1);
    rows<1>(BgInit<C, K>{z, zt, r, V(4), V(5)});
    scalar(M_BICG_RHO);
  }
  void pass_bicg() {
    double *r = V(0), *rt = V(1), *p = V(4), *pt = V(5), *q = V(6), *qt = V(7);
    double *z = precond ? V(2) : r, *zt = precond ? V(3) : rt;
    rows<1>(SpmvDotAY<C, K>{A->row_ptr, A->col_idx, A->val, p, pt, q});
    rows<0>(SpmvOp2{L.t_rp, L.t_ci, L.t_val, pt, qt});
    scalar(M_ALPHA);
    rows<2>(BgUpd<C, K>{p, q, qt, x, r, rt});
    scalar(M_R_TEST);
    residual(x, nullptr, nullptr, ST_CHECK_FULL);
    scalar(M_FULL);
    apply(r, z, 0);
    apply(rt, zt, 1);
    rows<1>(BgDot<C, K>{zt, r});
    scalar(M_BICG_RHO);
    rows<0>(BgP<C, K>{z, zt, p, pt});
  }
  struct SpmvOp2 {
    const int32_t *rp, *ci;
    const double *val, *xx;
    double *y;
    __device__ void operator()(int64_t i, const KState *, el<C, K> *) const {
      stv<C, K>(y, i, row_spmv<C, K>(i, rp, ci, val, xx));
    }
  };

  // ---- GPBiCG: v0 r, v1 r~, v2 p, v3 p^, v4 q, v5 y, v6 t, v7 t^, v8 s, v9 u,
  //      v10 z^, v11 w, v12 t_old, v13 p^_old, v14 t^_old
  void setup_gpbicg() {
    residual(x, V(0), V(1), GATE_ANY);
    ZeroOp<C, K> z{};
    const int zs[] = {2, 9, 12, 11, 13, 14, 10};
    z.nv = 7;
    for (int q = 0; q < 7; ++q) z.v[q] = V(zs[q]);
    rows<0>(z);
    scalar(M_INIT);
  }
  void pass_gpbicg() {
    double *r = V(0), *rt = V(1), *p = V(2), *q = V(4), *y = V(5), *t = V(6), *sv = V(8),
           *u = V(9), *zh = V(10), *w = V(11), *told = V(12), *phold = V(13), *thold = V(14);
    double *ph = precond ? V(3) : p, *th = precond ? V(7) : t;
    rows<0>(GpP<C, K>{r, u, p});
    apply(p, ph, 0);
    rows<1>(SpmvDotAY<C, K>{A->row_ptr, A->col_idx, A->val, ph, rt, q});
    scalar(M_ALPHA);
    rows<0>(GpYT<C, K>{told, r, w, q, y, t});
    apply(t, th, 0);
    rows<6>(GpS<C, K>{A->row_ptr, A->col_idx, A->val, th, t, y, sv});
    scalar(M_ZETA);
    rows<2>(GpUpd<C, K>{q, told, thold, phold, ph, th, t, y, sv, rt, u, zh, x, r});
    scalar(M_R_TEST);
    residual(x, nullptr, nullptr, ST_CHECK_FULL);
    scalar(M_FULL);
    rows<0>(GpW<C, K>{sv, q, t, ph, th, w, told, phold, thold});
  }

  void setup() {
    switch (method) {
      case MPK_BICG: setup_bicg(); break;
      case MPK_CGS: setup_cgs(); break;
      case MPK_BICGSTAB: setup_bicgstab(); break;
      default: setup_gpbicg(); break;
    }
  }
  void pass() {
    switch (method) {
      case MPK_BICG: pass_bicg(); break;
      case MPK_CGS: pass_cgs(); break;
      case MPK_BICGSTAB: pass_bicgstab(); break;
      default: pass_gpbicg(); break;
    }
  }
};

static bool use_graph(hipStream_t s) {
  const char *e = getenv("MPK_GRAPH");
  if (e && e[0] == '0') return false;
  return s != nullptr;
}

template <int C, int K>
static int krylov_run(int method, int KF, double tol_rel, double tol_abs, int64_t max_iter,
                      const mpk_csr *A, const double *b, double *x, void *ws, size_t ws_bytes,
                      mpk_info *info, hipStream_t s, const Ilu0 *ext = nullptr) {
  const double t0 = now_ms();
  Solver<C, K> S;
  S.method = method;
  S.n = A->n;
  S.A = A;
  S.b = b;
  S.x = x;
  S.s = s;
  S.precond = KF > 0;
  S.nblk = int(nblocks(A->n));
  Bump bump(ws);
  if (krylov_layout(method, C, K, KF, A->n, A->nnz, bump, &S.L, ext != nullptr) > ws_bytes)
    return MPK_EWORKSPACE;
  int st;
  int64_t bad = -1;
  if (ext) {
    // a factor the caller built (and possibly corrected) on A's pattern; its
    // values were checked when it was factored
    S.L.ilu = *ext;
  } else if (KF > 0) {
    mpk_info finfo{};
    // the ILU(0) part of the workspace starts at its first array; carving it
    // again from there reproduces the same offsets
    const size_t used = size_t(reinterpret_cast<char *>(S.L.ilu.words) - static_cast<char *>(ws));
    st = ilu0_factor_impl(C, KF, A,
                          (method == MPK_BICG ? MPK_ILU0_ADJOINT : 0) | MPK_ILU0_VPREC(K),
                          static_cast<void *>(S.L.ilu.words), ws_bytes - used, &S.L.ilu, &finfo, s);
    if (st) {
      if (info) info->bad_row = finfo.bad_row;
      return st;
    }
  } else {
    HostCsr h;
    if ((st = fetch_pattern(A, h, s))) return st;
    if ((st = check_pattern(h, &bad))) {
      if (info) info->bad_row = bad;
      return st;
    }
    if ((st = csr_check_device_values(A, C, S.L.abort, &bad, s))) {
      if (info) info->bad_row = bad;
      return st;
    }
  }
  if (method == MPK_BICG) {
    HostCsr h;
    if ((st = fetch_pattern(A, h, s))) return st;
    IVec trp, tci, tsrc;
    host_transpose(h, trp, tci, tsrc);
    MPK_HIP(hipMemcpyAsync(S.L.t_rp, trp.data(), sizeof(int32_t) * (A->n + 1), hipMemcpyHostToDevice, s));
    MPK_HIP(hipMemcpyAsync(S.L.t_ci, tci.data(), sizeof(int32_t) * A->nnz, hipMemcpyHostToDevice, s));
    MPK_HIP(hipMemcpyAsync(S.L.t_src, tsrc.data(), sizeof(int32_t) * A->nnz, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(gather_vals, dim3(nblocks(A->nnz)), dim3(BLOCK), 0, s, A->nnz, C, 1,
                       (const int32_t *)S.L.t_src, A->val, S.L.t_val, C == 2 ? 1 : 0);
    MPK_HIP(hipStreamSynchronize(s));
  }
  KState init{};
  init.eps_r = tol_rel;
  init.eps_a = tol_abs;
  init.max_iter = max_iter;
  init.hist = info ? info->res_history : nullptr;
  init.hist_len = info && info->res_history ? info->res_history_len : 0;
  init.true_nr2 = -1.0;
  MPK_HIP(hipMemcpyAsync(S.L.st, &init, sizeof(KState), hipMemcpyHostToDevice, s));
  int32_t zero = 0;
  MPK_HIP(hipMemcpyAsync(S.L.abort, &zero, sizeof(int32_t), hipMemcpyHostToDevice, s));
  MPK_HIP(hipStreamSynchronize(s));
  const double t1 = now_ms();
  S.setup();
  MPK_HIP(hipGetLastError());

  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  if (use_graph(s)) {
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      S.pass();
      if (hipStreamEndCapture(s, &graph) != hipSuccess ||
          hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        if (graph) hipGraphDestroy(graph);
        graph = nullptr;
        exec = nullptr;
        (void)hipGetLastError();
      }
    }
  }
  int64_t launched = 0;
  int64_t chunk = 2;
  int32_t done = 0;
  while (launched < max_iter) {
    const int64_t cnt = std::min<int64_t>(chunk, max_iter - launched);
    for (int64_t q = 0; q < cnt; ++q) {
      if (exec)
        MPK_HIP(hipGraphLaunch(exec, s));
      else
        S.pass();
    }
    MPK_HIP(hipGetLastError());
    launched += cnt;
    MPK_HIP(hipMemcpyAsync(&done, &S.L.st->done, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MPK_HIP(hipStreamSynchronize(s));
    if (done) break;
    chunk = std::min<int64_t>(chunk * 2, 64);
  }
  if (exec) hipGraphExecDestroy(exec);
  if (graph) hipGraphDestroy(graph);
  KState fin;
  int32_t abort_word = 0;
  MPK_HIP(hipMemcpyAsync(&fin, S.L.st, sizeof(KState), hipMemcpyDeviceToHost, s));
  MPK_HIP(hipMemcpyAsync(&abort_word, S.L.abort, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPK_HIP(hipStreamSynchronize(s));
  if (fin.x_in_tmp)
    MPK_HIP(hipMemcpyAsync(x, S.L.v[8], sizeof(double) * A->n * C * K, hipMemcpyDeviceToDevice, s));
  MPK_HIP(hipStreamSynchronize(s));
  const double t2 = now_ms();
  int status = fin.done ? fin.status : MPK_NOT_CONVERGED;
  if (abort_word) status = MPK_EWATCHDOG;
  if (info) {
    info->iters = fin.iter;
    info->status = status;
    info->relres_recursive =
        fin.nr0sq > 0 ? std::sqrt(fin.last_nr2 / fin.nr0sq) : std::sqrt(fin.last_nr2);
    info->relres_true = fin.true_nr2 < 0 ? -1.0
                        : (fin.nbsq > 0 ? std::sqrt(fin.true_nr2 / fin.nbsq)
                                        : std::sqrt(fin.true_nr2));
    info->setup_ms = t1 - t0;
    info->solve_ms = t2 - t1;
  }
  return status;
}

static size_t krylov_bytes(int method, int C, int K, int KF, int64_t n, int64_t nnz,
                           bool ext_ilu = false) {
  Bump b(nullptr);
  return krylov_layout(method, C, K, KF, n, nnz, b, nullptr, ext_ilu);
}

// Solve with a factor the caller owns (from mpk_?ilu0_factor, possibly
// corrected): same iteration, no factorisation inside.
static int krylov_solve_precond(int C, mpk_method m, mpk_prec vp, const mpk_ilu0 *Mh,
                                double tol_rel, double tol_abs, int64_t max_iter,
                                const mpk_csr *A, const double *b, double *x, void *ws,
                                size_t ws_bytes, mpk_info *info, void *stream) {
  if (info) {
    info->iters = 0;
    info->bad_row = -1;
    info->relres_recursive = -1;
    info->relres_true = -1;
    info->setup_ms = info->solve_ms = 0;
  }
  const Ilu0 *M = reinterpret_cast<const Ilu0 *>(Mh);
  int st = validate_csr_args(A);
  if (!st && (m < MPK_BICG || m > MPK_GPBICG || vp < MPK_D || vp > MPK_QD || !b || !x || !M ||
              !(tol_rel >= 0) || !(tol_abs >= 0) || max_iter < 0))
    st = MPK_EINVAL;
  // the factor must belong to A, hold enough limbs for K and, for BiCG,
  // carry the adjoint sweeps
  if (!st && (M->C != C || M->n != A->n || M->nnz != A->nnz || M->row_ptr != A->row_ptr ||
              M->col_idx != A->col_idx || M->KF > int(vp) || M->L.kmax < int(vp) ||
              M->U.kmax < int(vp) || (m == MPK_BICG && !(M->flags & MPK_ILU0_ADJOINT))))
    st = MPK_EINVAL;
  if (!st && (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) ||
              ws_bytes < krylov_bytes(m, C, int(vp), M->KF, A->n, A->nnz, true)))
    st = MPK_EWORKSPACE;
  if (!st)
    st = dispatch_ck(C, int(vp), [&]<int CC, int KK>() {
      return krylov_run<CC, KK>(int(m), M->KF, tol_rel, tol_abs, max_iter, A, b, x, ws,
                                ws_bytes, info, (hipStream_t)stream, M);
    });
  if (info) info->status = st;
  return st;
}

static int krylov_solve(int C, mpk_method m, mpk_prec vp, mpk_prec fp, double tol_rel,
                        double tol_abs, int64_t max_iter, const mpk_csr *A, const double *b,
                        double *x, void *ws, size_t ws_bytes, mpk_info *info, void *stream) {
  if (info) {
    info->iters = 0;
    info->bad_row = -1;
    info->relres_recursive = -1;
    info->relres_true = -1;
    info->setup_ms = info->solve_ms = 0;
  }
  int st = validate_csr_args(A);
  if (!st && (m < MPK_BICG || m > MPK_GPBICG || vp < MPK_D || vp > MPK_QD || !b || !x ||
              !(fp == 0 || (fp >= MPK_D && fp <= MPK_QD)) || int(fp) > int(vp) ||
              !(tol_rel >= 0) || !(tol_abs >= 0) || max_iter < 0))
    st = MPK_EINVAL;
  if (!st && (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) ||
              ws_bytes < krylov_bytes(m, C, int(vp), int(fp), A->n, A->nnz)))
    st = MPK_EWORKSPACE;
  if (!st)
    st = dispatch_ck(C, int(vp), [&]<int CC, int KK>() {
      return krylov_run<CC, KK>(int(m), int(fp), tol_rel, tol_abs, max_iter, A, b, x, ws, ws_bytes,
                                info, (hipStream_t)stream);
    });
  if (info) info->status = st;
  return st;
}

}  // namespace mpk

using namespace mpk;

extern "C" {

size_t mpk_krylov_workspace_bytes(mpk_method m, mpk_prec vp, mpk_prec fp, const mpk_csr *A,
                                  int is_complex) {
  if (!A || A->n <= 0 || A->nnz < 0 || m < MPK_BICG || m > MPK_GPBICG || vp < MPK_D ||
      vp > MPK_QD || !(fp == 0 || (fp >= MPK_D && fp <= MPK_QD)))
    return 0;
  return krylov_bytes(m, is_complex ? 2 : 1, int(vp), int(fp), A->n, A->nnz);
}

int mpk_dkrylov_solve(mpk_method m, mpk_prec vp, mpk_prec fp, double tol_rel, double tol_abs,
                      int64_t max_iter, const mpk_csr *A, const double *b, double *x, void *ws,
                      size_t ws_bytes, mpk_info *info, void *stream) {
  return krylov_solve(1, m, vp, fp, tol_rel, tol_abs, max_iter, A, b, x, ws, ws_bytes, info, stream);
}

int mpk_zkrylov_solve(mpk_method m, mpk_prec vp, mpk_prec fp, double tol_rel, double tol_abs,
                      int64_t max_iter, const mpk_csr *A, const double *b, double *x, void *ws,
                      size_t ws_bytes, mpk_info *info, void *stream) {
  return krylov_solve(2, m, vp, fp, tol_rel, tol_abs, max_iter, A, b, x, ws, ws_bytes, info, stream);
}

size_t mpk_krylov_precond_workspace_bytes(mpk_method m, mpk_prec vp, const mpk_csr *A,
                                          int is_complex) {
  if (!A || A->n <= 0 || A->nnz < 0 || m < MPK_BICG || m > MPK_GPBICG || vp < MPK_D ||
      vp > MPK_QD)
    return 0;
  return krylov_bytes(m, is_complex ? 2 : 1, int(vp), 1, A->n, A->nnz, true);
}

int mpk_dkrylov_solve_precond(mpk_method m, mpk_prec vp, const mpk_ilu0 *M, double tol_rel,
                              double tol_abs, int64_t max_iter, const mpk_csr *A, const double *b,
                              double *x, void *ws, size_t ws_bytes, mpk_info *info,
                              void *stream) {
  return krylov_solve_precond(1, m, vp, M, tol_rel, tol_abs, max_iter, A, b, x, ws, ws_bytes,
                              info, stream);
}

int mpk_zkrylov_solve_precond(mpk_method m, mpk_prec vp, const mpk_ilu0 *M, double tol_rel,
                              double tol_abs, int64_t max_iter, const mpk_csr *A, const double *b,
                              double *x, void *ws, size_t ws_bytes, mpk_info *info,
                              void *stream) {
  return krylov_solve_precond(2, m, vp, M, tol_rel, tol_abs, max_iter, A, b, x, ws, ws_bytes,
                              info, stream);
}

}  // extern "C"
