// kernels.hpp -- gfx950 kernels of the mpk library (templated over the
// number of components C, vector limbs K and factor limbs KF).
#pragma once
#include "internal.hpp"

namespace mpk {

// ------------------------------------------------------------ reductions
// Fixed-order reduction of ND element sums over a 256-thread workgroup:
// xor-butterfly inside each wavefront, then wavefronts 0..3 in order.
// The result is a deterministic function of the inputs (no atomics).
template <int C, int K, int ND>
__device__ __forceinline__ void block_reduce(el<C, K> (&d)[ND], double *out) {
  __shared__ double red[BLOCK / WAVE][ND > 0 ? ND : 1][C * K];
#pragma unroll
  for (int off = WAVE / 2; off >= 1; off >>= 1) {
#pragma unroll
    for (int q = 0; q < ND; ++q) {
      el<C, K> o;
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int k = 0; k < K; ++k) o.c[c].v[k] = __shfl_xor(d[q].c[c].v[k], off, WAVE);
      d[q] = el_add<C, K>(d[q], o);
    }
  }
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < ND; ++q)
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int k = 0; k < K; ++k) red[w][q][c * K + k] = d[q].c[c].v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < ND; ++q) {
      el<C, K> s = el_load<C, K>(red[0][q]);
      for (int ww = 1; ww < BLOCK / WAVE; ++ww) s = el_add<C, K>(s, el_load<C, K>(red[ww][q]));
      if (out) el_store<C, K>(out + size_t(q) * C * K, s);
      d[q] = s;
    }
  }
}

// Sum of per-block partials [nblk][ND][C*K] by one workgroup: thread t
// accumulates blocks t, t+256, ... in order, then block_reduce.  The
// totals are valid in thread 0 only.
template <int C, int K, int ND>
__device__ __forceinline__ void reduce_partials(const double *partials, int nblk,
                                                el<C, K> (&tot)[ND]) {
#pragma unroll
  for (int q = 0; q < ND; ++q) tot[q] = el_zero<C, K>();
  for (int b = threadIdx.x; b < nblk; b += BLOCK)
#pragma unroll
    for (int q = 0; q < ND; ++q) {
      el<C, K> v = el_load<C, K>(partials + (size_t(b) * ND + q) * C * K);
      tot[q] = (b == int(threadIdx.x)) ? v : el_add<C, K>(tot[q], v);
    }
  block_reduce<C, K, ND>(tot, nullptr);
}

// ------------------------------------------------------------------ SpMV
// Row i of y = A x: products in ascending column order, accumulated in
// the working precision starting from the first product (empty row: 0).
template <int C, int K>
__device__ __forceinline__ el<C, K> row_spmv(int64_t i, const int32_t *__restrict__ rp,
                                             const int32_t *__restrict__ ci,
                                             const double *__restrict__ val,
                                             const double *__restrict__ x) {
  const int32_t a = rp[i], b = rp[i + 1];
  el<C, K> acc = el_zero<C, K>();
  for (int32_t p = a; p < b; ++p) {
    double f[C];
#pragma unroll
    for (int c = 0; c < C; ++c) f[c] = val[size_t(p) * C + c];
    el<C, K> t = el_mul_f<C, K, 1>(f, el_load<C, K>(x + size_t(ci[p]) * C * K));
    acc = (p == a) ? t : el_add<C, K>(acc, t);
  }
  return acc;
}

// Generic row/element kernel: op(i, dots) for i < n; optional ND fused
// inner-product partials written per workgroup.  Skipped when *done.
template <int C, int K, int ND, class Op>
__global__ __launch_bounds__(BLOCK) void row_kernel(int64_t n, Op op, const int32_t *done,
                                                    double *partials) {
  if (done && *done) return;
  const int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  el<C, K> d[ND > 0 ? ND : 1];
#pragma unroll
  for (int q = 0; q < (ND > 0 ? ND : 1); ++q) d[q] = el_zero<C, K>();
  if (i < n) op(i, d);
  if constexpr (ND > 0) block_reduce<C, K, ND>(d, partials + size_t(blockIdx.x) * ND * C * K);
}

template <int C, int K> struct SpmvOp {
  const int32_t *rp, *ci;
  const double *val, *x;
  double *y;
  __device__ void operator()(int64_t i, el<C, K> *) const {
    el_store<C, K>(y + size_t(i) * C * K, row_spmv<C, K>(i, rp, ci, val, x));
  }
};

// Gathers C binary64 values per entry, conjugating when asked (A^H).
static __global__ void gather_vals(int64_t m, int C, int KF, const int32_t *__restrict__ src,
                            const double *__restrict__ from, double *__restrict__ to, int conj) {
  const int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (i >= m) return;
  const int V = C * KF;
  const double *s = from + size_t(src[i]) * V;
  for (int v = 0; v < V; ++v) to[size_t(i) * V + v] = (conj && v >= KF) ? -s[v] : s[v];
}

// Lowest row holding an Inf/NaN value (atomicMin into *bad, init INT_MAX).
static __global__ void check_finite(int64_t n, int C, const int32_t *__restrict__ rp,
                             const double *__restrict__ val, int32_t *bad) {
  const int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (i >= n) return;
  for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
    for (int c = 0; c < C; ++c) {
      double v = val[size_t(p) * C + c];
      if (!(v - v == 0.0)) {
        atomicMin(bad, int32_t(i));
        return;
      }
    }
}

// ------------------------------------------------------ ILU(0) factor
// One level of the IKJ elimination (Algorithm 1 row by row): for each
// stored k < i in ascending order, l_ik = a_ik / u_kk, then a_ij -= l_ik *
// u_kj for each stored j > k of row k also stored in row i (merge of the
// two sorted rows).  Rows of a level only read rows of earlier levels.
// kf = 1 keeps product-then-subtract in binary64; kf = 2 uses double-word.
template <int C, int KF>
__global__ __launch_bounds__(BLOCK) void ilu0_level(int32_t cnt, const int32_t *__restrict__ rows,
                                                    const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci,
                                                    const int32_t *__restrict__ diag, double *f,
                                                    int32_t *bad) {
  const int t = blockIdx.x * BLOCK + threadIdx.x;
  if (t >= cnt) return;
  const int32_t i = rows[t];
  constexpr int V = C * KF;
  const int32_t ri_end = rp[i + 1];
  for (int32_t p = rp[i]; p < ri_end && ci[p] < i; ++p) {
    const int32_t k = ci[p];
    const double *ukk = f + size_t(diag[k]) * V;
    el<C, KF> lik = el_load<C, KF>(f + size_t(p) * V);
    lik = el_div_k<C, KF, KF>(lik, ukk);
    el_store<C, KF>(f + size_t(p) * V, lik);
    int32_t r = p + 1;
    const int32_t rk_end = rp[k + 1];
    for (int32_t q = diag[k] + 1; q < rk_end; ++q) {
      const int32_t j = ci[q];
      while (r < ri_end && ci[r] < j) ++r;
      if (r < ri_end && ci[r] == j) {
        el<C, KF> aij = el_load<C, KF>(f + size_t(r) * V);
        el<C, KF> prod = el_mul_f<C, KF, KF>(f + size_t(q) * V, lik);
        el_store<C, KF>(f + size_t(r) * V, el_sub<C, KF>(aij, prod));
      }
    }
  }
  if (el_is_zero<C, KF>(el_load<C, KF>(f + size_t(diag[i]) * V))) atomicMin(bad, i);
}

// Copies A's values into the factor array (kf limbs per component, the
// lower limbs zero: the exact promotion of binary64 entries).
static __global__ void promote_vals(int64_t nnz, int C, int KF, const double *__restrict__ val,
                             double *__restrict__ f) {
  const int64_t p = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (p >= nnz) return;
  for (int c = 0; c < C; ++c)
    for (int k = 0; k < KF; ++k) f[(size_t(p) * C + c) * KF + k] = k == 0 ? val[size_t(p) * C + c] : 0.0;
}

// ------------------------------------------------- triangular sweeps
// Sync-free substitution over a level schedule.  Each wavefront takes the
// next segment (<= 64 rows of one level, so no dependencies inside it)
// from a global ticket; segments are handed out in level order, so every
// row a segment waits on belongs to a segment already taken by a running
// wavefront, and the sweep always makes progress.  Results are published
// with agent-scope relaxed stores into an output pre-filled with SENTINEL;
// a consumer spins (agent-scope relaxed loads) until no word of y_j is the
// sentinel.  Every spin is bounded: past the bound the wave raises the
// abort word, every other wave leaves its waits, and the host reports
// MPK_EWATCHDOG.  Row arithmetic: acc = rhs_i; acc -= f_p * y_col(p) for
// the row's entries in ascending column order; then acc / pivot when DIV.
constexpr int SPIN_LIMIT = 1 << 22;

__device__ __forceinline__ uint64_t ld_agent(const double *p) {
  return __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(double *p, double v) {
  unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), b, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

template <int C, int K>
__device__ __forceinline__ bool wait_load(const double *p, el<C, K> &v, int32_t *abort_flag) {
  for (int it = 0;; ++it) {
    bool ok = true;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        uint64_t b = ld_agent(p + c * K + k);
        ok = ok && (b != SENTINEL);
        v.c[c].v[k] = __builtin_bit_cast(double, b);
      }
    if (ok) return true;
    if ((it & 127) == 127 &&
        __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return false;
    if (it >= SPIN_LIMIT) {
      __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

template <int C, int KF, bool CONJ>
__device__ __forceinline__ void load_f(const double *__restrict__ p, double (&f)[C * KF]) {
#pragma unroll
  for (int v = 0; v < C * KF; ++v) f[v] = (CONJ && v >= KF) ? -p[v] : p[v];
}

template <int C, int K, int KF, bool DIV, bool CONJ>
__global__ __launch_bounds__(BLOCK) void trsv_syncfree(
    const int32_t *__restrict__ order, const int32_t *__restrict__ ptr,
    const int32_t *__restrict__ col, const double *__restrict__ val,
    const double *__restrict__ dval, const int32_t *__restrict__ seg, int32_t nseg,
    const double *__restrict__ rhs, double *out, int32_t *ticket, int32_t *abort_flag,
    const int32_t *done) {
  if (done && *done) return;
  const int lane = threadIdx.x & (WAVE - 1);
  constexpr int E = C * K;
  for (;;) {
    int32_t s = 0;
    if (lane == 0) s = atomicAdd(ticket, 1);
    s = __shfl(s, 0, WAVE);
    if (s >= nseg) break;
    const int32_t pos = seg[s] + lane;
    if (pos < seg[s + 1]) {
      const int32_t i = order[pos];
      el<C, K> acc = el_load<C, K>(rhs + size_t(i) * E);
      const int32_t pe = ptr[pos + 1];
      for (int32_t p = ptr[pos]; p < pe; ++p) {
        el<C, K> yj;
        wait_load<C, K>(out + size_t(col[p]) * E, yj, abort_flag);
        double f[C * KF];
        load_f<C, KF, CONJ>(val + size_t(p) * C * KF, f);
        acc = el_sub<C, K>(acc, el_mul_f<C, K, KF>(f, yj));
      }
      if constexpr (DIV) {
        double d[C * KF];
        load_f<C, KF, CONJ>(dval + size_t(pos) * C * KF, d);
        acc = el_div_k<C, K, KF>(acc, d);
      }
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int k = 0; k < K; ++k) {
          double v = acc.c[c].v[k];
          st_agent(out + size_t(i) * E + c * K + k, v != v ? __builtin_nan("") : v);
        }
    }
  }
}

// Prepares one apply: outputs filled with SENTINEL and the two tickets
// reset (a kernel rather than a memset, so the step can be graph-captured).
// The abort word is reset only when abort_reset is non-null: inside a solve
// it persists so the host sees any watchdog event at the end.
static __global__ void trsv_prep(int64_t words, double *out1, double *out2, int32_t *ticket1,
                          int32_t *ticket2, int32_t *abort_reset, const int32_t *done) {
  if (done && *done) return;
  const int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  const double sent = __builtin_bit_cast(double, (unsigned long long)SENTINEL);
  if (i < words) {
    out1[i] = sent;
    out2[i] = sent;
  }
  if (i == 0) {
    *ticket1 = 0;
    *ticket2 = 0;
    if (abort_reset) *abort_reset = 0;
  }
}

}  // namespace mpk
