// kernels.hpp -- gfx950 kernels of the mpk library (templated over the
// number of components C, vector limbs K and factor limbs KF).
#pragma once
#include "internal.hpp"

namespace mpk {

// ------------------------------------------------------------ reductions
// Fixed-order reduction of ND element sums over a workgroup of NT threads
// (256 unless stated): xor-butterfly inside each wavefront, then the
// wavefronts in order.  The result is a deterministic function of the
// inputs (no atomics).
template <int C, int K, int ND, int NT = BLOCK>
__device__ __forceinline__ void block_reduce(el<C, K> (&d)[ND], double *out) {
  __shared__ double red[NT / WAVE][ND > 0 ? ND : 1][C * K];
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
      for (int ww = 1; ww < NT / WAVE; ++ww) s = el_add<C, K>(s, el_load<C, K>(red[ww][q]));
      if (out) el_store<C, K>(out + size_t(q) * C * K, s);
      d[q] = s;
    }
  }
}

// Sum of per-block partials [nblk][ND][C*K] by one workgroup: thread t
// accumulates blocks t, t+256, ... in order, then block_reduce.  The
// totals are valid in thread 0 only.  The loads of U consecutive blocks
// of a thread are issued before their sums, so the memory round trips
// overlap; the summation order stays the same.
template <int C, int K, int ND>
__device__ __forceinline__ void reduce_partials(const double *partials, int nblk,
                                                el<C, K> (&tot)[ND]) {
  constexpr int W = ND * C * K;
  constexpr int U = W <= 4 ? 8 : (W <= 16 ? 4 : 2);
#pragma unroll
  for (int q = 0; q < ND; ++q) tot[q] = el_zero<C, K>();
  for (int b0 = threadIdx.x; b0 < nblk; b0 += U * BLOCK) {
    el<C, K> v[U][ND];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = min(b0 + u * BLOCK, nblk - 1);  // in range; extra copies unused
#pragma unroll
      for (int q = 0; q < ND; ++q) v[u][q] = el_load<C, K>(partials + (size_t(b) * ND + q) * C * K);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = b0 + u * BLOCK;
      if (b < nblk)
#pragma unroll
        for (int q = 0; q < ND; ++q)
          tot[q] = (b == int(threadIdx.x)) ? v[u][q] : el_add<C, K>(tot[q], v[u][q]);
    }
  }
  block_reduce<C, K, ND>(tot, nullptr);
}

// ------------------------------------------------------------------ SpMV
// Entries of a row whose loads are issued together.
template <int C, int K> constexpr int spmv_batch() { return C * K <= 2 ? 8 : 4; }

// Row i of y = A x: products in ascending column order, accumulated in
// the working precision starting from the first product (empty row: 0).
// The first spmv_batch entries' indices, values and x words are requested
// together (indices clamped into the row; the extra words are not used),
// so a short stencil row costs two memory round trips instead of two per
// entry; longer rows continue one entry at a time.
template <int C, int K>
__device__ __forceinline__ el<C, K> row_spmv(int64_t i, const int32_t *__restrict__ rp,
                                             const int32_t *__restrict__ ci,
                                             const double *__restrict__ val,
                                             const double *__restrict__ x) {
  constexpr int U = spmv_batch<C, K>();
  const int32_t a = rp[i], b = rp[i + 1];
  el<C, K> acc = el_zero<C, K>();
  if (b > a) {
    int32_t cj[U];
    double f[U][C];
    el<C, K> xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t p = min(a + u, b - 1);
      cj[u] = ci[p];
#pragma unroll
      for (int c = 0; c < C; ++c) f[u][c] = val[size_t(p) * C + c];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = el_load<C, K>(x + size_t(cj[u]) * C * K);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (a + u < b) {
        const el<C, K> t = el_mul_f<C, K, 1>(f[u], xv[u]);
        acc = u == 0 ? t : el_add<C, K>(acc, t);
      }
    }
    for (int32_t p = a + U; p < b; ++p) {
      double fp[C];
#pragma unroll
      for (int c = 0; c < C; ++c) fp[c] = val[size_t(p) * C + c];
      acc = el_add<C, K>(acc, el_mul_f<C, K, 1>(fp, el_load<C, K>(x + size_t(ci[p]) * C * K)));
    }
  }
  return acc;
}

// Vector-CSR SpMV: G lanes per row (G = 2, 4, 8, 16).  Lane s of a row's
// group loads and multiplies entries a + s, a + s + G, ... (so the group's
// loads of indices and values are contiguous and the gathers of x are
// spread evenly over its lanes); the group then adds the products in
// ascending column order, every lane taking them from their lanes, so all
// lanes of the group end with the row's sum.  The products and the order
// of the additions are row_spmv's, so y is the same bit for bit.  Launch
// with xcd_grid(ceil(n / (BLOCK / G))) workgroups.
template <int C, int K, int G>
__global__ __launch_bounds__(BLOCK) void spmv_vec(int64_t n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci,
                                                  const double *__restrict__ val,
                                                  const double *__restrict__ x,
                                                  double *__restrict__ y, const int32_t *done) {
  static_assert(G >= 2 && G <= 16 && (G & (G - 1)) == 0, "lanes per row");
  if (done && *done) return;
  constexpr int RPB = BLOCK / G;  // rows per workgroup
  const int64_t lb = xcd_block();
  if (lb * RPB >= n) return;
  const int64_t i = lb * RPB + threadIdx.x / G;
  const int s = int(threadIdx.x % G);
  const int g0 = int(threadIdx.x % WAVE) - s;  // the group's first lane in the wavefront
  const bool valid = i < n;
  const int32_t a = valid ? rp[i] : 0, b = valid ? rp[i + 1] : 0;
  el<C, K> acc = el_zero<C, K>();
  for (int32_t q0 = a; q0 < b; q0 += G) {
    const int32_t q = q0 + s < b ? q0 + s : a;  // a lane past the row's end redoes entry a
    double f[C];
#pragma unroll
    for (int c = 0; c < C; ++c) f[c] = val[size_t(q) * C + c];
    const el<C, K> t = el_mul_f<C, K, 1>(f, el_load<C, K>(x + size_t(ci[q]) * C * K));
#pragma unroll
    for (int u = 0; u < G; ++u) {
      el<C, K> tu;
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int kk = 0; kk < K; ++kk) tu.c[c].v[kk] = __shfl(t.c[c].v[kk], g0 + u, WAVE);
      if (q0 + u < b) acc = q0 + u == a ? tu : el_add<C, K>(acc, tu);
    }
  }
  if (valid && s == 0) el_store<C, K>(y + size_t(i) * C * K, acc);
}

// Generic row/element kernel: op(i, dots) for i < n; optional ND fused
// inner-product partials written per row block.  Skipped when *done.
// Launch with xcd_grid(nblocks(n)) workgroups.
template <int C, int K, int ND, class Op>
__global__ __launch_bounds__(BLOCK) void row_kernel(int64_t n, Op op, const int32_t *done,
                                                    double *partials) {
  if (done && *done) return;
  const int64_t lb = xcd_block();
  if (lb * BLOCK >= n) return;
  const int64_t i = lb * BLOCK + threadIdx.x;
  el<C, K> d[ND > 0 ? ND : 1];
#pragma unroll
  for (int q = 0; q < (ND > 0 ? ND : 1); ++q) d[q] = el_zero<C, K>();
  if (i < n) op(i, d);
  if constexpr (ND > 0) block_reduce<C, K, ND>(d, partials + size_t(lb) * ND * C * K);
}

template <int C, int K> struct SpmvOp {
  const int32_t *rp, *ci;
  const double *val, *x;
  double *y;
  __device__ void operator()(int64_t i, el<C, K> *) const {
    el_store<C, K>(y + size_t(i) * C * K, row_spmv<C, K>(i, rp, ci, val, x));
  }
};

// r = b - A x: the row's SpMV sum (row_spmv), then one subtraction from b_i
// in the working precision.
template <int C, int K> struct ResidOp {
  const int32_t *rp, *ci;
  const double *val, *b, *x;
  double *r;
  __device__ void operator()(int64_t i, el<C, K> *) const {
    const el<C, K> bi = el_load<C, K>(b + size_t(i) * C * K);
    el_store<C, K>(r + size_t(i) * C * K, el_sub<C, K>(bi, row_spmv<C, K>(i, rp, ci, val, x)));
  }
};

// Gathers C binary64 values per entry, conjugating when asked (A^H).
static __global__ void gather_vals(int64_t m, int C, int KF, const int32_t *__restrict__ src,
                            const double *__restrict__ from, double *__restrict__ to, int conj) {
  const int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (i >= m) return;
  const int V = C * KF;
  if (src[i] < 0) {
    for (int v = 0; v < V; ++v) to[size_t(i) * V + v] = 0.0;
    return;
  }
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

// ------------------------------------------------- schedule arrays
// Position of the diagonal entry of each row (the pattern was checked, so
// every row has one).
static __global__ void find_diag(int64_t n, const int32_t *__restrict__ rp,
                                 const int32_t *__restrict__ ci, int32_t *diag) {
  const int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (i >= n) return;
  for (int32_t q = rp[i]; q < rp[i + 1]; ++q)
    if (ci[q] == i) diag[i] = q;
}

// Dependencies of the row at each schedule position: the stored columns
// j < i (lower) or j > i of that row of the given CSR.
static __global__ void plan_count(int64_t n, const int32_t *__restrict__ order,
                                  const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                  int lower, int32_t *cnt) {
  const int64_t pos = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (pos >= n) return;
  const int32_t i = order[pos];
  int32_t c = 0;
  for (int32_t q = rp[i]; q < rp[i + 1]; ++q) c += lower ? (ci[q] < i) : (ci[q] > i);
  cnt[pos] = c;
}

// Exclusive scan of n counts into out[0..n] (out[n] = total), three
// phases: 1024-element block scans, a scan of the block sums, offsets.
constexpr int SCAN_ITEMS = 4, SCAN_BLOCK = BLOCK * SCAN_ITEMS;

__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t *total) {
  __shared__ int32_t sh[BLOCK];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < BLOCK; off <<= 1) {
    const int32_t t = threadIdx.x >= unsigned(off) ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  const int32_t incl = sh[threadIdx.x];
  *total = sh[BLOCK - 1];
  __syncthreads();
  return incl - v;
}

static __global__ void scan_blocks(int64_t n, const int32_t *__restrict__ in, int32_t *out,
                                   int32_t *bsum) {
  const int64_t base = int64_t(blockIdx.x) * SCAN_BLOCK + int64_t(threadIdx.x) * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS], s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = base + k < n ? in[base + k] : 0;
    s += v[k];
  }
  int32_t tot;
  int32_t run = block_exclusive_scan(s, &tot);
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

static __global__ void scan_sums(int32_t nb, int32_t *bsum) {
  const int32_t per = (nb + BLOCK - 1) / BLOCK;
  const int32_t a = threadIdx.x * per, e = min(nb, a + per);
  int32_t s = 0;
  for (int32_t q = a; q < e; ++q) s += bsum[q];
  int32_t tot;
  int32_t run = block_exclusive_scan(s, &tot);
  for (int32_t q = a; q < e; ++q) {
    const int32_t v = bsum[q];
    bsum[q] = run;
    run += v;
  }
  if (threadIdx.x == 0) bsum[nb] = tot;
}

static __global__ void scan_add(int64_t n, int32_t *out, const int32_t *__restrict__ bsum,
                                int32_t nb) {
  const int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (i < n) out[i] += bsum[i / SCAN_BLOCK];
  if (i == 0) out[n] = bsum[nb];
}

// Per-position dependency arrays: columns and value sources (positions in
// A's pattern; srcmap maps the rows of A^T back to A) in ascending column
// order, the flat ELLW slots of the blocked sweeps, and the pivot position.
// A flat slot holds the column j of a dependency in another block, or
// -(LDS slot of j + 1) for one in the row's own block (geometry G); each
// position's row, dependency count and own LDS slot go to one 16-byte
// record of ell_meta, fetched with a single load.  xflag (blocked
// schedules, zeroed before) marks every row that a row of another block
// depends on; plan_xmeta copies the mark into the record's last word.
static __global__ void plan_fill(int64_t n, const int32_t *__restrict__ order,
                                 const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                 const int32_t *__restrict__ srcmap, int lower,
                                 const int32_t *__restrict__ ptr, int32_t *col, int32_t *src,
                                 int32_t *ell_nd, int32_t *ell_col, int32_t *ell_src,
                                 int32_t *ell_meta, BlockGeom G,
                                 const int32_t *__restrict__ diag, int32_t *dsrc,
                                 int32_t *xflag) {
  const int64_t pos = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (pos >= n) return;
  const int32_t i = order[pos];
  const int64_t bi = ell_nd ? G.block(i) : 0;
  if (ell_nd) {
    ell_meta[pos * 4] = i;
    ell_meta[pos * 4 + 2] = G.slot(i);
    ell_meta[pos * 4 + 3] = 0;
  }
  int32_t o = ptr[pos], d = 0;
  for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
    const int32_t j = ci[q];
    if (lower ? j < i : j > i) {
      const int32_t sp = srcmap ? srcmap[q] : q;
      col[o] = j;
      src[o] = sp;
      if (ell_nd && d < ELLW) {
        ell_col[pos * ELLW + d] = G.block(j) == bi ? -(G.slot(j) + 1) : j;
        ell_src[pos * ELLW + d] = sp;
      }
      if (xflag && G.block(j) != bi) atomicOr(&xflag[j], 1);
      ++o;
      ++d;
    }
  }
  if (ell_nd) {
    ell_nd[pos] = d;
    ell_meta[pos * 4 + 1] = d;
    for (int32_t k = d; k < ELLW; ++k) {
      ell_col[pos * ELLW + k] = 0;
      ell_src[pos * ELLW + k] = -1;
    }
  }
  if (dsrc) dsrc[pos] = diag[i];
}

// The last word of each position's record: whether a row of another block
// reads this row from memory.
static __global__ void plan_xmeta(int64_t n, const int32_t *__restrict__ order,
                                  const int32_t *__restrict__ xflag, int32_t *ell_meta) {
  const int64_t pos = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (pos < n) ell_meta[pos * 4 + 3] = xflag[order[pos]];
}

// Rows with xflag set, in ascending order, at their exclusive-scan offsets.
static __global__ void plan_xlist(int64_t n, const int32_t *__restrict__ xflag,
                                  const int32_t *__restrict__ off, int32_t *xlist) {
  const int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (i < n && xflag[i]) xlist[off[i]] = int32_t(i);
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
// Substitution over a level schedule in one launch.  Each wavefront takes
// the next segment (<= 64 rows of one level, so no dependencies inside it)
// from a global ticket; segments are handed out in level order, so every
// level a segment waits on was taken by running wavefronts and the sweep
// always progresses.  Before computing, lane 0 waits until every earlier
// level is complete (per-level counters of finished rows, one polled word
// per wavefront instead of one per row, which keeps the polling traffic
// small).  Results are published with agent-scope relaxed stores into an
// output pre-filled with SENTINEL, and each dependency load still spins
// until no word of y_j is the sentinel, so a value is never read before it
// is written.  Every wait is bounded: past the bound the wave raises the
// abort word, every other wave leaves its waits, and the host reports
// MPK_EWATCHDOG.  Row arithmetic: acc = rhs_i; acc -= f_p * y_col(p) over
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
__device__ __forceinline__ int32_t ld_agent_i(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    if ((it & 63) == 63 && ld_agent_i(abort_flag)) return false;
    if (it >= SPIN_LIMIT) {
      __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Lane-0 wait until levels [frontier, L) are complete; returns the new
// frontier (or L on abort).
__device__ __forceinline__ int32_t wait_levels(int32_t frontier, int32_t L,
                                               const int32_t *__restrict__ lev_size,
                                               const int32_t *lev_done, int32_t *abort_flag) {
  int it = 0;
  while (frontier < L) {
    if (ld_agent_i(lev_done + frontier) >= lev_size[frontier]) {
      ++frontier;
      continue;
    }
    if ((++it & 63) == 63 && ld_agent_i(abort_flag)) return L;
    if (it >= SPIN_LIMIT) {
      __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return L;
    }
    __builtin_amdgcn_s_sleep(8);
  }
  return frontier;
}

template <int C, int KF, bool CONJ>
__device__ __forceinline__ void load_f(const double *__restrict__ p, double (&f)[C * KF]) {
#pragma unroll
  for (int v = 0; v < C * KF; ++v) f[v] = (CONJ && v >= KF) ? -p[v] : p[v];
}

// Dependencies are fetched in batches of up to MAXD rows: all their words
// are requested at once (one memory round trip), and only a batch that
// still shows a sentinel falls back to the per-value wait.
template <int E> constexpr int trsv_maxd() { return E <= 2 ? 8 : (E <= 4 ? 4 : 2); }

template <int C, int K, int KF, bool DIV, bool CONJ>
__global__ __launch_bounds__(BLOCK) void trsv_syncfree(
    const int32_t *__restrict__ order, const int32_t *__restrict__ ptr,
    const int32_t *__restrict__ col, const double *__restrict__ val,
    const double *__restrict__ dval, const int32_t *__restrict__ seg,
    const int32_t *__restrict__ seg_level, int32_t nseg, const int32_t *__restrict__ lev_size,
    int32_t *lev_done, const double *__restrict__ rhs, double *out, int32_t *ticket,
    int32_t *abort_flag, const int32_t *done, int32_t xcd_stride) {
  if (done && *done) return;
  // optional placement: only every xcd_stride-th workgroup works, which with
  // round-robin dispatch keeps the sweep on one XCD (a placement choice only)
  if (blockIdx.x % xcd_stride) return;
  constexpr int E = C * K;
  constexpr int MAXD = trsv_maxd<E>();
  constexpr int WPB = BLOCK / WAVE;  // wavefronts per workgroup
  __shared__ int32_t group;
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  int32_t frontier = 0;
  for (;;) {
    // one ticket per workgroup: segments group .. group+WPB-1, one per wave
    if (threadIdx.x == 0) group = atomicAdd(ticket, WPB);
    __syncthreads();
    const int32_t s = group + w;
    __syncthreads();
    if (group >= nseg) break;
    if (s < nseg) {
      const int32_t L = seg_level[s];
      const int32_t p0 = seg[s], p1 = seg[s + 1];
      const int32_t pos = p0 + lane;
      const bool valid = pos < p1;
      int32_t i = 0, pb = 0, pe = 0;
      el<C, K> acc = el_zero<C, K>();
      int32_t cj[MAXD];
      double fv[MAXD][C * KF];
      if (valid) {
        i = order[pos];
        pb = ptr[pos];
        pe = ptr[pos + 1];
        acc = el_load<C, K>(rhs + size_t(i) * E);
#pragma unroll
        for (int d = 0; d < MAXD; ++d)
          if (pb + d < pe) {
            cj[d] = col[pb + d];
            load_f<C, KF, CONJ>(val + size_t(pb + d) * C * KF, fv[d]);
          }
      }
      if (lane == 0) frontier = wait_levels(frontier, L, lev_size, lev_done, abort_flag);
      frontier = __shfl(frontier, 0, WAVE);
      if (valid) {
        for (int32_t q0 = pb; q0 < pe; q0 += MAXD) {
          if (q0 != pb) {
#pragma unroll
            for (int d = 0; d < MAXD; ++d)
              if (q0 + d < pe) {
                cj[d] = col[q0 + d];
                load_f<C, KF, CONJ>(val + size_t(q0 + d) * C * KF, fv[d]);
              }
          }
          el<C, K> yv[MAXD];
          bool ok = true;
#pragma unroll
          for (int d = 0; d < MAXD; ++d) {
            if (q0 + d < pe) {
              const double *yp = out + size_t(cj[d]) * E;
#pragma unroll
              for (int c = 0; c < C; ++c)
#pragma unroll
                for (int k = 0; k < K; ++k) {
                  uint64_t b = ld_agent(yp + c * K + k);
                  ok = ok && (b != SENTINEL);
                  yv[d].c[c].v[k] = __builtin_bit_cast(double, b);
                }
            }
          }
          if (!ok) {
#pragma unroll
            for (int d = 0; d < MAXD; ++d)
              if (q0 + d < pe) wait_load<C, K>(out + size_t(cj[d]) * E, yv[d], abort_flag);
          }
#pragma unroll
          for (int d = 0; d < MAXD; ++d)
            if (q0 + d < pe) acc = el_sub<C, K>(acc, el_mul_f<C, K, KF>(fv[d], yv[d]));
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
      if (lane == 0) atomicAdd(lev_done + L, p1 - p0);
    }
  }
}

// Level-synchronous sweep: one launch per level, one thread per row of
// the level (positions pos0 .. pos0 + cnt - 1 of the level order).  Rows of
// one level depend only on rows of earlier levels, which earlier launches
// on the same stream have finished, so nothing is polled and the loads are
// plain cached loads.  For schedules with few, wide levels (a multicolour
// ordering has one level per colour).  Row arithmetic is the level
// schedule's: right-hand side, then each product subtracted in ascending
// column order, then the division by the pivot (DIV).
template <int C, int K, int KF, bool DIV, bool CONJ>
__global__ __launch_bounds__(BLOCK) void trsv_level(
    int32_t pos0, int32_t cnt, const int32_t *__restrict__ order,
    const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ dval,
    const double *__restrict__ rhs, double *__restrict__ out, const int32_t *done) {
  if (done && *done) return;
  constexpr int E = C * K;
  const int32_t t = int32_t(blockIdx.x) * BLOCK + int32_t(threadIdx.x);
  if (t >= cnt) return;
  const int32_t pos = pos0 + t;
  const int32_t i = order[pos];
  const int32_t pb = ptr[pos], pe = ptr[pos + 1];
  el<C, K> acc = el_load<C, K>(rhs + size_t(i) * E);
  // the first U dependencies' indices and values, then their y words, are
  // requested together (one round trip each); the terms are still
  // subtracted one by one in ascending column order
  constexpr int U = E <= 2 ? 4 : 2;
  if (pe > pb) {
    int32_t cj[U];
    double f[U][C * KF];
    el<C, K> yv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t q = min(pb + u, pe - 1);
      cj[u] = col[q];
      load_f<C, KF, CONJ>(val + size_t(q) * C * KF, f[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) yv[u] = el_load<C, K>(out + size_t(cj[u]) * E);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (pb + u < pe) acc = el_sub<C, K>(acc, el_mul_f<C, K, KF>(f[u], yv[u]));
  }
  for (int32_t q = pb + U; q < pe; ++q) {
    double f[C * KF];
    load_f<C, KF, CONJ>(val + size_t(q) * C * KF, f);
    acc = el_sub<C, K>(acc, el_mul_f<C, K, KF>(f, el_load<C, K>(out + size_t(col[q]) * E)));
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
      const double v = acc.c[c].v[k];
      out[size_t(i) * E + c * K + k] = v != v ? __builtin_nan("") : v;
    }
}

// Blocked schedule: a workgroup takes the next block of rows
// (tickets hand blocks out in the sweep's order, so a block only waits on
// blocks already taken by running workgroups) and walks the block's local
// levels; results of the block stay in LDS for the rows of the same block
// that need them and are published to memory (agent-scope stores) for
// later blocks, which read them with the sentinel-checked wait.  A
// workgroup barrier separates consecutive local levels.  Loads are
// software-pipelined: while level l is computed from LDS, the row data,
// factor values and external y values of level l+1 are already in flight.
// Row arithmetic is identical to the level schedule's.
// ---- blocked sweep ------------------------------------------------------
// Every memory access of a level is one buffer instruction issued by all
// lanes whatever their row: a lane without a row (or a dependency slot
// that is not external) uses an offset past the buffer's end, which the
// hardware turns into a zero load or a dropped store without touching
// memory.  With no memory operation under a lane- or level-dependent
// branch, the compiler counts the loads in flight and waits only for the
// ones a level needs, so the next levels' row data and external values
// stay in flight across the level barriers; loaded words are first used
// when their level is finished.

typedef unsigned int bu2 __attribute__((ext_vector_type(2)));
typedef unsigned int bu4 __attribute__((ext_vector_type(4)));
typedef int bi4 __attribute__((ext_vector_type(4)));
constexpr int BUF_AGENT = 16;               // cache policy: coherent at agent scope (sc1)
constexpr uint32_t BUF_OOB = 0xFFFFFF00u;   // an offset past every buffer's end

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, int(bytes),
                                           0x00020000);
}
template <int AUX>
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, int(off), 0, AUX));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(bu2, v), r, int(off), 0, BUF_AGENT);
}

template <int C, int K, int KF, int MAXD> struct RowPre {
  int32_t i, pos, nd, slot;
  int32_t x;           // read by a row of another block: stored at once
  bool valid;
  // flat slots: column j, or -(LDS slot + 1) inside the block; one 4-word
  // vector, as loaded, so the prefetch stages keep it in one register tuple
  bi4 cj;
  double f[MAXD][C * KF];
  double dv[C * KF];   // pivot (backward sweeps)
  el<C, K> ye[MAXD];   // words of external dependencies (raw)
  el<C, K> rh;         // the row's right-hand side
};

// The buffers of one sweep.
struct SweepBufs {
  __amdgpu_buffer_rsrc_t meta, col, val, dval, rhs, out;
};

// Stage 1 (D levels ahead): row index, dependency count, LDS slot, the
// first ELLW flat dependency slots and factor values, and the pivot, by
// position.
template <int C, int K, int KF, bool DIV, bool CONJ, int MAXD>
__device__ __forceinline__ void row_fetch_meta(RowPre<C, K, KF, MAXD> &r, int32_t pos, bool valid,
                                               const SweepBufs &B) {
  static_assert(MAXD == ELLW, "one slot per flat dependency");
  r.pos = pos;
  r.valid = valid;
  const bu4 m = __builtin_amdgcn_raw_buffer_load_b128(
      B.meta, int(valid ? uint32_t(pos) * 16u : BUF_OOB), 0, 0);
  r.i = int32_t(m.x);
  r.nd = int32_t(m.y);
  r.slot = int32_t(m.z);
  r.x = int32_t(m.w);
  r.cj = __builtin_bit_cast(bi4, __builtin_amdgcn_raw_buffer_load_b128(
                                     B.col, int(valid ? uint32_t(pos) * 4u * ELLW : BUF_OOB), 0, 0));
  const uint32_t fo = valid ? uint32_t(pos) * uint32_t(ELLW * C * KF * 8) : BUF_OOB;
#pragma unroll
  for (int d = 0; d < MAXD; ++d)
#pragma unroll
    for (int v = 0; v < C * KF; ++v) {
      const double x = buf_ld<0>(B.val, fo + uint32_t((d * C * KF + v) * 8));
      r.f[d][v] = (CONJ && v >= KF) ? -x : x;
    }
  if constexpr (DIV) {
    const uint32_t dofs = valid ? uint32_t(pos) * uint32_t(C * KF * 8) : BUF_OOB;
#pragma unroll
    for (int v = 0; v < C * KF; ++v) {
      const double x = buf_ld<0>(B.dval, dofs + uint32_t(v * 8));
      r.dv[v] = (CONJ && v >= KF) ? -x : x;
    }
  }
}

template <int C, int K, int KF, int MAXD>
__device__ __forceinline__ bool dep_external(const RowPre<C, K, KF, MAXD> &r, int d) {
  return r.valid && d < r.nd && r.cj[d] >= 0;
}

// Stage 2 (X levels ahead): the row's right-hand side and the words of
// dependencies outside the block.
template <int C, int K, int KF, int MAXD>
__device__ __forceinline__ void row_fetch_ext(RowPre<C, K, KF, MAXD> &r, const SweepBufs &B) {
  constexpr int E = C * K;
  {
    const uint32_t o = r.valid ? uint32_t(r.i) * uint32_t(E * 8) : BUF_OOB;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int k = 0; k < K; ++k) r.rh.c[c].v[k] = buf_ld<0>(B.rhs, o + uint32_t((c * K + k) * 8));
  }
#pragma unroll
  for (int d = 0; d < MAXD; ++d) {
    const uint32_t o = dep_external<C, K, KF, MAXD>(r, d)
                           ? uint32_t(r.cj[d]) * uint32_t(E * 8) : BUF_OOB;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int k = 0; k < K; ++k)
        r.ye[d].c[c].v[k] = buf_ld<BUF_AGENT>(B.out, o + uint32_t((c * K + k) * 8));
  }
}

// Re-polls the external dependencies whose prefetched words still hold the
// sentinel, all of them in one bounded loop (one copy of the slow path per
// level keeps the unrolled level loop small), until every word is written.
template <int C, int K, int KF, int MAXD>
__device__ __forceinline__ void wait_ext(RowPre<C, K, KF, MAXD> &r, int32_t pe, const SweepBufs &B,
                                      int32_t *abort_flag) {
  constexpr int E = C * K;
  for (int it = 0;; ++it) {
    bool miss = false;
#pragma unroll
    for (int d = 0; d < MAXD; ++d) {
      bool hit = false;
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int k = 0; k < K; ++k)
          hit = hit | (__builtin_bit_cast(uint64_t, r.ye[d].c[c].v[k]) == SENTINEL);
      const bool m = (d < pe) & (r.cj[d] >= 0) & hit;
      miss = miss | m;
      const uint32_t o = m ? uint32_t(r.cj[d]) * uint32_t(E * 8) : BUF_OOB;
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const double v = buf_ld<BUF_AGENT>(B.out, o + uint32_t((c * K + k) * 8));
          r.ye[d].c[c].v[k] = m ? v : r.ye[d].c[c].v[k];
        }
    }
    if (!miss) return;
    if ((it & 63) == 63 && ld_agent_i(abort_flag)) return;
    if (it >= SPIN_LIMIT) {
      __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Finish one row: acc = rhs_i (prefetched with the external values) minus the
// products in ascending column order, divided by the pivot when DIV; the
// result goes to the row's LDS slot, and to out if another block reads it.  A lane without a row uses
// the spare LDS slot `spare` and an out-of-range store.  Dependencies past
// the ELLW flat slots come from the CSR arrays; the host allows them only
// for blocks of one range [r0, r1), where row j sits in slot j - r0.
template <int C, int K, int KF, bool DIV, bool CONJ, int MAXD>
__device__ __forceinline__ void row_finish(RowPre<C, K, KF, MAXD> &r, const int32_t *__restrict__ ptr,
                                           const int32_t *__restrict__ col,
                                           const double *__restrict__ val, double *out,
                                           const SweepBufs &B, double *lds, int32_t r0,
                                           int32_t r1, int32_t spare, int32_t *abort_flag) {
  constexpr int E = C * K;
  const int32_t pe = r.valid ? r.nd : 0;
  const int32_t slot = r.valid ? r.slot : spare;
  el<C, K> acc = r.rh;
  {
    // in-block values from LDS (the spare slot for other slots), kept apart
    // from the prefetched external words: overwriting a register that an
    // LDS read still fills would serialise the reads
    el<C, K> yl[MAXD];
#pragma unroll
    for (int d = 0; d < MAXD; ++d) {
      const int32_t j = r.cj[d];
      yl[d] = el_load<C, K>(lds + size_t(d < pe && j < 0 ? -j - 1 : spare) * E);
    }
    // Any prefetched word still holding the sentinel.  Slots that are not
    // external were loaded from an out-of-range offset and hold zero, so
    // they need no mask here; wait_ext re-checks with the masks.  (Bitwise
    // operators: no short-circuit branches.)
    bool bad = false;
#pragma unroll
    for (int d = 0; d < MAXD; ++d)
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int k = 0; k < K; ++k)
          bad = bad | (__builtin_bit_cast(uint64_t, r.ye[d].c[c].v[k]) == SENTINEL);
    if (bad) wait_ext<C, K, KF, MAXD>(r, pe, B, abort_flag);
#pragma unroll
    for (int d = 0; d < MAXD; ++d)
      if (d < pe) {
        el<C, K> y;
        const bool ext = r.cj[d] >= 0;
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
          for (int k = 0; k < K; ++k) y.c[c].v[k] = ext ? r.ye[d].c[c].v[k] : yl[d].c[c].v[k];
        acc = el_sub<C, K>(acc, el_mul_f<C, K, KF>(r.f[d], y));
      }
  }
  // rows with more than MAXD dependencies: the rest from the CSR arrays
  if (pe > MAXD) {
    const int32_t pb = ptr[r.pos];
    for (int32_t d = MAXD; d < pe; ++d) {
      const int32_t j = col[pb + d];
      el<C, K> yj;
      if (j >= r0 && j < r1)
        yj = el_load<C, K>(lds + size_t(j - r0) * E);
      else
        wait_load<C, K>(out + size_t(j) * E, yj, abort_flag);
      double f[C * KF];
      load_f<C, KF, CONJ>(val + size_t(pb + d) * C * KF, f);
      acc = el_sub<C, K>(acc, el_mul_f<C, K, KF>(f, yj));
    }
  }
  if constexpr (DIV) acc = el_div_k<C, K, KF>(acc, r.dv);
  // only rows that other blocks poll are stored now; the block's other
  // results reach memory when the block ends (trsv_blocked's flush)
  const uint32_t oo = (r.valid && r.x) ? uint32_t(r.i) * uint32_t(E * 8) : BUF_OOB;
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double v = acc.c[c].v[k];
      v = v != v ? __builtin_nan("") : v;
      lds[size_t(slot) * E + c * K + k] = v;
      buf_st(B.out, oo + uint32_t((c * K + k) * 8), v);
    }
}

// Workgroup barrier for data exchanged through LDS only: waits for this
// wave's LDS operations, not for its outstanding global loads and stores
// (a full __syncthreads would drain the prefetch pipeline at every level).
// The asm statement also keeps the compiler from moving memory accesses
// across it.
template <int NT> __device__ __forceinline__ void lds_barrier() {
  if constexpr (NT == WAVE) {
    // one wavefront: its LDS operations execute in program order, so a
    // later read sees an earlier write; only the compiler is fenced
    asm volatile("" ::: "memory");
  } else {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
  }
}

// Prefetch depth (local levels) of the blocked sweep's row data.
template <int E> constexpr int trsv_depth() { return E <= 2 ? 6 : 3; }
template <int E> constexpr int trsv_lead() { return E <= 2 ? 2 : 1; }

// Blocked sweep: a workgroup takes the next block (in sweep order; its
// rows and their LDS slots come from the plan, see BlockGeom: ranges of
// gw-slot width, gt of them, gP rows apart) and walks the block's local
// levels (each at most NT rows: one per lane), separated by LDS-only
// barriers; rows that other blocks read are stored as they are finished,
// and at the end the whole block is copied from LDS to out.  A row's right-hand side is prefetched with its
// external values; in-block results are kept in LDS for the rows that need
// them, and values of other blocks are read from out with the
// sentinel-checked wait.  blk_r holds the first range [r0, r1) of each
// block, used only by rows with more than ELLW dependencies (the host
// allows those only in blocks of one range).  LDS: (spare + 1) * C * K
// doubles, slot `spare` for lanes without a row.  The buffers' byte sizes
// must stay below 2^31 (the host picks the level schedule otherwise).
// About one workgroup per CU (the LDS block decides), so the register
// budget may grow to keep the prefetch stages out of scratch.
// NT threads per workgroup: BLOCK, or one wavefront when no local level
// piece of the plan has more than WAVE rows (no idle wavefronts then
// issue their out-of-range loads beside the working one).
template <int C, int K, int KF, bool DIV, bool CONJ, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 1))) void trsv_blocked(
    int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ dval,
    const int32_t *__restrict__ blk_r, const int32_t *__restrict__ blk_lev,
    const int32_t *__restrict__ loc_pos, int32_t nblk, const int32_t *__restrict__ ell_col,
    const int32_t *__restrict__ ell_meta, const double *__restrict__ ell_val, int32_t spare,
    int64_t gP, int32_t gw, int32_t gt, const double *__restrict__ rhs, double *out,
    int32_t *ticket, int32_t *abort_flag, const int32_t *done) {
  if (done && *done) return;
  extern __shared__ double lds[];
  __shared__ int32_t cur;
  constexpr int E = C * K;
  constexpr int MAXD = ELLW;
  constexpr int D = trsv_depth<E>();
  constexpr int X = trsv_lead<E>();  // levels ahead at which external values are requested
  using RP = RowPre<C, K, KF, MAXD>;
  const int32_t tid = threadIdx.x;
  SweepBufs B;
  B.meta = buf_rsrc(ell_meta, n * 16);
  B.col = buf_rsrc(ell_col, n * 4 * ELLW);
  B.val = buf_rsrc(ell_val, n * ELLW * C * KF * 8);
  B.dval = buf_rsrc(DIV ? dval : ell_val, DIV ? n * C * KF * 8 : 0);
  B.rhs = buf_rsrc(rhs, n * E * 8);
  B.out = buf_rsrc(out, n * E * 8);
  for (;;) {
    if (tid == 0) cur = atomicAdd(ticket, 1);
    __syncthreads();
    const int32_t b = cur;
    __syncthreads();
    if (b >= nblk) break;
    const int32_t r0 = blk_r[2 * b], r1 = blk_r[2 * b + 1];
    const int32_t l0 = blk_lev[b], l1 = blk_lev[b + 1];
    // row data of local level l (empty past the block's last level)
    auto meta = [&](RP &r, int32_t l) {
      const int32_t pb = loc_pos[min(l, l1)], pe = loc_pos[min(l + 1, l1)];
      row_fetch_meta<C, K, KF, DIV, CONJ, MAXD>(r, pb + tid, pb + tid < pe, B);
    };
    // prologue in the steady state's issue pattern (the external values of
    // level l + X, then the row data of level l + D), so the compiler's
    // count of loads in flight at the loop head is the same on both paths
    // and its waits stay partial
    RP st[D];
#pragma unroll
    for (int u = 0; u < D - X; ++u) meta(st[u], l0 + u);
#pragma unroll
    for (int u = D - X; u < D; ++u) {
      row_fetch_ext<C, K, KF, MAXD>(st[u - (D - X)], B);
      meta(st[u], l0 + u);
    }
    __syncthreads();
    // one local level: finish `now`; then request the external values of
    // level l+X (slot `ext`, whose indices arrived D-X stages ago) and
    // refill `now` with the row data of level l+D.  The refill's level
    // bounds come from vector loads issued one stage earlier (all lanes,
    // one address): a scalar load would make every LDS wait of the next
    // level wait for it too, since the two share a counter.
    const __amdgpu_buffer_rsrc_t lp = buf_rsrc(loc_pos, (l1 + 1) * 4);
    auto lp_ld = [&](int32_t l) {
      return int32_t(__builtin_amdgcn_raw_buffer_load_b32(lp, min(l, l1) * 4, 0, 0));
    };
    int32_t vb = lp_ld(l0 + D), ve = lp_ld(l0 + D + 1);
    auto stage = [&](RP &now, RP &ext, int32_t l) {
      row_finish<C, K, KF, DIV, CONJ, MAXD>(now, ptr, col, val, out, B, lds, r0, r1, spare,
                                            abort_flag);
      lds_barrier<NT>();
      row_fetch_ext<C, K, KF, MAXD>(ext, B);
      row_fetch_meta<C, K, KF, DIV, CONJ, MAXD>(now, vb + tid, vb + tid < ve, B);
      vb = ve;
      ve = lp_ld(l + D + 2);
    };
    for (int32_t lv = l0; lv < l1; lv += D) {
#pragma unroll
      for (int u = 0; u < D; ++u) stage(st[u], st[(u + X) % D], lv + u);
    }
    // the block's results from LDS to out, range by range: range k holds
    // rows r0 + k P + c in LDS slots k w + c, and consecutive lanes store
    // consecutive rows
    lds_barrier<NT>();
    const int32_t wb = r1 - r0;
    for (int32_t k = 0; k < gt; ++k) {
      const int64_t a = int64_t(r0) + int64_t(k) * gP;
      if (a >= n) break;
      const int32_t cnt = int32_t(min<int64_t>(wb, n - a));
      for (int32_t c = tid; c < cnt; c += NT) {
        const double *src = lds + size_t(k * gw + c) * E;
#pragma unroll
        for (int e = 0; e < E; ++e) buf_st(B.out, uint32_t((a + c) * E + e) * 8u, src[e]);
      }
    }
    __syncthreads();
  }
}

// ---- grid sweep (mode 3) -------------------------------------------------
// For a matrix whose pattern is the 7-point (3D) or 5-point (2D) stencil of
// an nx x ny x nz grid numbered x fastest, the L sweep (forward) and the U
// sweep (backward, dividing by the pivot) need no schedule arrays: a block
// is BY grid lines in y times BZ in z (BY * BZ = 64, one wavefront), the
// lane of line (yl, zl) is q = zl + BZ yl, and at local level l the lane
// handles x = l - yl - zl.  The dependency on x - 1 is then the lane's own
// value of the previous level, the ones on z - 1 and y - 1 inside the block
// are the previous level's values of lanes q - 1 (a DPP shift) and q - BZ
// (ds_bpermute), and those in the blocks below come from memory with the
// sentinel-checked wait.  The backward sweep runs the same walk on the
// mirrored grid (row n - 1 - i).  Blocks are taken from a ticket in sweep
// order (z-block major), so a block waits only on taken blocks.  Each
// row's terms are subtracted in ascending column order (z, y, x forward;
// x, y, z backward, mirrored) and the row arithmetic is the level
// schedule's.
//
// Memory: the factor values come from records made at setup (grid_gather),
// one per row in processing order (block, level, then active lane), so a
// level's records are contiguous and its loads coalesce.  Rows that a later
// block reads are stored at agent scope as they are finished; the block's
// results also go to LDS (line q at slot q (nx + 1) + x) and are copied to
// memory, line by line, when the block ends (STAGE), or, when the block
// does not fit in LDS, stored at once.

template <int C, int K, int KF> struct GridRow {
  double f[4][C * KF];       // term values in term order; [3] the pivot (backward)
  el<C, K> rh;               // right-hand side
  el<C, K> ye[2];            // external y - 1 and z - 1 values
};

template <int BY> constexpr int grid_bz() { return WAVE / BY; }
// Levels of row data (factor records, right-hand side) requested ahead:
// eight for elements of up to two words (128^3 DD: 0.532, 0.522, 0.508,
// 0.509, 0.505 ms per apply for 4, 6, 8, 10, 12; the unrolled loop runs up
// to depth - 1 levels past a block's last, so 8 gives the best solve).
template <int E> constexpr int grid_depth() { return E <= 2 ? 8 : 4; }
// External values are requested two levels ahead: one level leaves the
// load's latency exposed, three or more ask before the producer has
// stored them and cost a re-poll (128^3 DD: 0.71, 0.59, 0.61, 0.66 ms per
// apply for leads 1 to 4).
template <int E> constexpr int grid_lead() { return 2; }

// Rows of the grid sweep's blocks before block (by, bz): whole z-slabs of
// BZ ny lines below bz, then by blocks of BY x lz lines in slab bz.
__host__ __device__ __forceinline__ int64_t grid_block_start(const GridDims &g, int by_, int bz_,
                                                             int32_t by, int32_t bz) {
  const int64_t lz = min(int64_t(bz_), int64_t(g.nz) - int64_t(bz) * bz_);
  return (int64_t(bz) * bz_ * g.ny + lz * int64_t(by) * by_) * g.nx;
}

// The factor records of a grid sweep: record pos holds the row's three
// term values in term order (zero where the neighbour is outside the grid)
// and, backward, its pivot, C * KF doubles each, at gval[(pos * 4 + slot)
// * C * KF].  pos numbers the rows in processing order: block start, then
// the rows of the block's earlier levels, then the active lanes before the
// row's lane at its level (by = lines per block in y).
static __global__ void grid_gather(int64_t n, GridDims g, int by_, int back, int V,
                                   const int32_t *__restrict__ diag,
                                   const double *__restrict__ f, double *__restrict__ gval) {
  const int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (i >= n) return;
  const int bz_ = WAVE / by_;
  const int64_t s = back ? n - 1 - i : i;  // sweep coordinates
  const int64_t pl = int64_t(g.nx) * g.ny;
  const int64_t x = s % g.nx, y = (s / g.nx) % g.ny, z = s / pl;
  const int32_t by = int32_t(y / by_), bz = int32_t(z / bz_);
  const int yl = int(y % by_), zl = int(z % bz_), q = zl + bz_ * yl;
  const int64_t l = x + yl + zl;
  int64_t pos = grid_block_start(g, by_, bz_, by, bz);
  for (int q2 = 0; q2 < WAVE; ++q2) {
    const int yl2 = q2 / bz_, zl2 = q2 % bz_;
    if (int64_t(by) * by_ + yl2 >= g.ny || int64_t(bz) * bz_ + zl2 >= g.nz) continue;
    const int64_t c = yl2 + zl2;
    pos += min(max(l - c, int64_t(0)), int64_t(g.nx));   // its rows at levels below l
    if (q2 < q && l - c >= 0 && l - c < g.nx) ++pos;      // active before this lane at l
  }
  const bool ex = x > 0, ey = y > 0, ez = z > 0;
  const int64_t dg = diag[i];
  int64_t p[3];
  bool has[3];
  if (!back) {
    // stored lower entries z-1, y-1, x-1 just before the diagonal
    const int nlow = int(ex) + int(ey) + int(ez);
    has[0] = ez;
    has[1] = ey;
    has[2] = ex;
    p[0] = dg - nlow;
    p[1] = dg - nlow + int(ez);
    p[2] = dg - 1;
  } else {
    // stored upper entries x+1, y+1, z+1 just after it (mirrored: x-1, y-1, z-1)
    has[0] = ex;
    has[1] = ey;
    has[2] = ez;
    p[0] = dg + 1;
    p[1] = dg + 1 + int(ex);
    p[2] = dg + 1 + int(ex) + int(ey);
  }
  double *o = gval + pos * 4 * V;
  for (int d = 0; d < 3; ++d)
    for (int v = 0; v < V; ++v) o[d * V + v] = has[d] ? f[p[d] * V + v] : 0.0;
  for (int v = 0; v < V; ++v) o[3 * V + v] = back ? f[dg * V + v] : 0.0;
}

// N doubles from byte offset o of a buffer: 16-byte loads when N is even
// (o a multiple of 16), else 8-byte loads.
template <int N, int AUX>
__device__ __forceinline__ void buf_ld_n(__amdgpu_buffer_rsrc_t r, uint32_t o, double *d) {
  if constexpr (N % 2 == 0) {
#pragma unroll
    for (int j = 0; j < N / 2; ++j) {
      const bu4 w = __builtin_amdgcn_raw_buffer_load_b128(r, int(o + uint32_t(j * 16)), 0, AUX);
      d[2 * j] = __builtin_bit_cast(double, (uint64_t(w.y) << 32) | w.x);
      d[2 * j + 1] = __builtin_bit_cast(double, (uint64_t(w.w) << 32) | w.z);
    }
  } else {
#pragma unroll
    for (int j = 0; j < N; ++j) d[j] = buf_ld<AUX>(r, o + uint32_t(j * 8));
  }
}

template <int C, int K>
__device__ __forceinline__ void el_ld(__amdgpu_buffer_rsrc_t r, uint32_t o, el<C, K> &v) {
  double d[C * K];
  buf_ld_n<C * K, 0>(r, o, d);
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int k = 0; k < K; ++k) v.c[c].v[k] = d[c * K + k];
}

template <int C, int K>
__device__ __forceinline__ void el_ld_agent(__amdgpu_buffer_rsrc_t r, uint32_t o, el<C, K> &v) {
  double d[C * K];
  buf_ld_n<C * K, BUF_AGENT>(r, o, d);
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int k = 0; k < K; ++k) v.c[c].v[k] = d[c * K + k];
}

// Lane q - 1's copy of v (lane 0 gets zero): one DPP move per dword.
template <int C, int K>
__device__ __forceinline__ el<C, K> lane_prev(const el<C, K> &v) {
  el<C, K> r;
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint64_t b = __builtin_bit_cast(uint64_t, v.c[c].v[k]);
      const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b)), 0x138, 0xf, 0xf, true));
      const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b >> 32)), 0x138, 0xf, 0xf, true));
      r.c[c].v[k] = __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
    }
  return r;
}

// Lane src's copy of v (ds_bpermute).
template <int C, int K>
__device__ __forceinline__ el<C, K> lane_read(const el<C, K> &v, int src) {
  el<C, K> r;
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint64_t b = __builtin_bit_cast(uint64_t, v.c[c].v[k]);
      const uint32_t lo = uint32_t(__builtin_amdgcn_ds_bpermute(src * 4, int(uint32_t(b))));
      const uint32_t hi = uint32_t(__builtin_amdgcn_ds_bpermute(src * 4, int(uint32_t(b >> 32))));
      r.c[c].v[k] = __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
    }
  return r;
}

template <int C, int K>
__device__ __forceinline__ bool el_has_sentinel(const el<C, K> &v) {
  bool bad = false;
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int k = 0; k < K; ++k) bad = bad | (__builtin_bit_cast(uint64_t, v.c[c].v[k]) == SENTINEL);
  return bad;
}

template <int C, int K>
__device__ __forceinline__ el<C, K> el_select(bool p, const el<C, K> &a, const el<C, K> &b) {
  el<C, K> r;
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int k = 0; k < K; ++k) r.c[c].v[k] = p ? a.c[c].v[k] : b.c[c].v[k];
  return r;
}

// LDS bytes of a grid sweep block staged in LDS: 64 lines of nx + 1 slots
// (the extra slot keeps consecutive lines in different banks) and a spare
// slot for lanes without a row.
inline size_t grid_lds_bytes(int32_t nx, int E) {
  return (size_t(WAVE) * (size_t(nx) + 1) + 1) * size_t(E) * 8;
}
constexpr size_t GRID_LDS_MAX = 159 * 1024;  // below the 160 KiB of a CU

template <int C, int K, int KF, bool BACK, int BY, bool STAGE>
__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(1, 1))) void trsv_grid(
    int64_t n, GridDims g, const double *__restrict__ gval, const double *__restrict__ rhs,
    double *out, int32_t *ticket, int32_t *abort_flag, const int32_t *done) {
  if (done && *done) return;
  extern __shared__ double lds[];
  constexpr int BZ = grid_bz<BY>();
  constexpr int E = C * K;
  constexpr int V = C * KF;
  constexpr int D = grid_depth<E>();
  constexpr int X = grid_lead<E>();  // levels ahead at which external values are requested
  using GR = GridRow<C, K, KF>;
  __shared__ int32_t cur;
  const int q = int(threadIdx.x);
  const int zl = q % BZ, yl = q / BZ;
  const int64_t plane = int64_t(g.nx) * g.ny;
  const int32_t stride = g.nx + 1;                 // LDS slots per line
  const int32_t spare = WAVE * stride;            // LDS slot of lanes without a row
  const __amdgpu_buffer_rsrc_t Rg = buf_rsrc(gval, n * 4 * V * 8);
  const __amdgpu_buffer_rsrc_t Rr = buf_rsrc(rhs, n * E * 8);
  const __amdgpu_buffer_rsrc_t Ro = buf_rsrc(out, n * E * 8);
  for (;;) {
    if (q == 0) cur = atomicAdd(ticket, 1);
    __syncthreads();
    const int32_t b = cur;
    __syncthreads();
    if (b >= g.nby * g.nbz) break;
    const int32_t by = b % g.nby, bz = b / g.nby;
    // this lane's line, in sweep coordinates (mirrored when BACK)
    const int32_t y = by * BY + yl, z = bz * BZ + zl;
    const bool line = y < g.ny && z < g.nz;
    const int64_t base = int64_t(z) * plane + int64_t(y) * g.nx;  // row of x = 0
    const bool ey = y > 0, ez = z > 0;
    const bool exty = ey && yl == 0, extz = ez && zl == 0;  // neighbour in another block
    // stored at agent scope: read by the next block in y or in z
    const bool pub = line && ((yl == BY - 1 && y < g.ny - 1) || (zl == BZ - 1 && z < g.nz - 1));
    const int32_t nlev = g.nx + (BY - 1) + (BZ - 1);
    auto real = [&](int64_t s) { return BACK ? n - 1 - s : s; };
    // byte offsets of this lane's row at level l (row base + x, mirrored
    // when BACK) and of its neighbours y - 1 and z - 1, as one add each
    constexpr int64_t EB = int64_t(E) * 8;
    const int64_t ob0 = real(base - yl - zl) * EB;  // offset of x = 0 shifted by -(yl + zl)
    const int64_t ostep = BACK ? -EB : EB;          // per level
    const int64_t dy = (BACK ? int64_t(g.nx) : -int64_t(g.nx)) * EB;
    const int64_t dz = (BACK ? plane : -plane) * EB;
    auto row_off = [&](int32_t l) { return ob0 + int64_t(l) * ostep; };
    const int32_t slot0 = q * stride - yl - zl;     // LDS slot of this lane's row at level 0
    // the lane has a row at level l: 0 <= l - yl - zl < nx on a line of the
    // grid, as one unsigned compare (a lane without a line gets an origin
    // past every level used, so l - c0 < 0 for all of them)
    const int32_t c0 = line ? yl + zl : nlev + D;
    auto active = [&](int32_t l) { return uint32_t(l - c0) < uint32_t(g.nx); };
    // position of the next staged level's first record
    int64_t run = grid_block_start(g, BY, BZ, by, bz);
    // row data, D levels ahead: the factor record and the right-hand side
    auto stage_row = [&](GR &r, int32_t l) {
      const bool a = active(l);
      const uint64_t m = __ballot(a);
      const int64_t pos = run + int64_t(__builtin_amdgcn_mbcnt_hi(
                                    uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0)));
      run += __popcll(m);
      const uint32_t og = a ? uint32_t(pos) * uint32_t(4 * V * 8) : BUF_OOB;
      double fr[4 * V];
      buf_ld_n<(BACK ? 4 : 3) * V, 0>(Rg, og, fr);
#pragma unroll
      for (int d = 0; d < (BACK ? 4 : 3); ++d)
#pragma unroll
        for (int v = 0; v < V; ++v) r.f[d][v] = fr[d * V + v];
      const uint32_t o = a ? uint32_t(row_off(l)) : BUF_OOB;
      el_ld<C, K>(Rr, o, r.rh);
    };
    // external neighbours, X levels ahead
    auto stage_ext = [&](GR &r, int32_t l) {
      const bool a = active(l);
      const int64_t o = row_off(l);
      const uint32_t oy = (a && exty) ? uint32_t(o + dy) : BUF_OOB;
      const uint32_t oz = (a && extz) ? uint32_t(o + dz) : BUF_OOB;
      el_ld_agent<C, K>(Ro, oy, r.ye[0]);
      el_ld_agent<C, K>(Ro, oz, r.ye[1]);
    };
    GR st[D];
#pragma unroll
    for (int u = 0; u < D; ++u) stage_row(st[u], u);
#pragma unroll
    for (int u = 0; u < X; ++u) stage_ext(st[u], u);
    el<C, K> prev = el_zero<C, K>();  // this lane's value of the previous level
    // finish level l from its staged data, then request the external values
    // of level l + X and the row data of level l + D
    auto level = [&](GR &now, GR &ext, int32_t l) {
      const bool a = active(l);
      const int32_t x = l - yl - zl;
      // neighbours inside the block: the previous level's values
      el<C, K> vy, vz = el_zero<C, K>();
      if constexpr (BZ == 1) {
        vy = lane_prev<C, K>(prev);
      } else {
        vz = lane_prev<C, K>(prev);
        vy = lane_read<C, K>(prev, q >= BZ ? q - BZ : 0);
      }
      // one wave-uniform test (lane masks in scalar registers, no divergent
      // branch on the common path)
      if (__ballot(el_has_sentinel<C, K>(now.ye[0])) | __ballot(el_has_sentinel<C, K>(now.ye[1]))) {
        // external words not written yet: re-poll them (bounded; keeping a
        // second request in flight made the sweeps slower)
        const int64_t o = row_off(l);
        for (int it = 0;; ++it) {
          const bool my = a && exty && el_has_sentinel<C, K>(now.ye[0]);
          const bool mz = a && extz && el_has_sentinel<C, K>(now.ye[1]);
          if (!(my | mz)) break;
          el<C, K> wy, wz;
          el_ld_agent<C, K>(Ro, my ? uint32_t(o + dy) : BUF_OOB, wy);
          el_ld_agent<C, K>(Ro, mz ? uint32_t(o + dz) : BUF_OOB, wz);
          now.ye[0] = el_select<C, K>(my, wy, now.ye[0]);
          now.ye[1] = el_select<C, K>(mz, wz, now.ye[1]);
          if ((it & 63) == 63 && ld_agent_i(abort_flag)) break;
          if (it >= SPIN_LIMIT) {
            __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
      el<C, K> acc = now.rh;
      // term order: forward z, y, x; backward x, y, z (mirrored)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int which = BACK ? d : 2 - d;  // 0 = x, 1 = y, 2 = z
        bool has;
        el<C, K> yv;
        if (which == 0) {
          has = x > 0;
          yv = prev;
        } else if (which == 1) {
          has = ey;
          yv = el_select<C, K>(exty, now.ye[0], vy);
        } else {
          has = ez;
          yv = el_select<C, K>(extz, now.ye[1], vz);
        }
        const el<C, K> t = el_sub<C, K>(acc, el_mul_f<C, K, KF>(now.f[d], yv));
        acc = el_select<C, K>(has, t, acc);
      }
      if constexpr (BACK) acc = el_div_k<C, K, KF>(acc, now.f[3]);
      const uint32_t o = a ? uint32_t(row_off(l)) : BUF_OOB;
      double *slot = lds + size_t(a ? slot0 + l : spare) * E;
      double w[E];
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int k = 0; k < K; ++k) {
          double v = acc.c[c].v[k];
          v = v != v ? __builtin_nan("") : v;
          acc.c[c].v[k] = v;
          w[c * K + k] = v;
        }
      // the row's words: at agent scope if the next block reads it (16-byte
      // stores when E is even), and to LDS or memory for the block's copy
      const uint32_t op = pub ? o : BUF_OOB;
      if constexpr (E % 2 == 0) {
#pragma unroll
        for (int j = 0; j < E / 2; ++j) {
          const uint64_t u0 = __builtin_bit_cast(uint64_t, w[2 * j]);
          const uint64_t u1 = __builtin_bit_cast(uint64_t, w[2 * j + 1]);
          const bu4 wv = {uint32_t(u0), uint32_t(u0 >> 32), uint32_t(u1), uint32_t(u1 >> 32)};
          __builtin_amdgcn_raw_buffer_store_b128(wv, Ro, int(op + uint32_t(j * 16)), 0, BUF_AGENT);
        }
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e)
          __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(bu2, w[e]), Ro,
                                                int(op + uint32_t(e * 8)), 0, BUF_AGENT);
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if constexpr (STAGE)
          slot[e] = w[e];
        else
          __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(bu2, w[e]), Ro,
                                                int((pub ? BUF_OOB : o) + uint32_t(e * 8)), 0, 0);
      }
      // lanes without a row leave garbage here; no row reads it: a lane's
      // own value is used only for x > 0, a neighbour lane's only when that
      // lane had a row at the previous level
      prev = acc;
      stage_ext(ext, l + X);
      stage_row(now, l + D);
    };
    for (int32_t lv = 0; lv < nlev; lv += D) {
#pragma unroll
      for (int u = 0; u < D; ++u) level(st[u], st[(u + X) % D], lv + u);
    }
    if constexpr (STAGE) {
      // the block's results from LDS to memory, line by line (one wavefront:
      // its LDS operations execute in order, so no barrier is needed)
      asm volatile("" ::: "memory");
      for (int ql = 0; ql < WAVE; ++ql) {
        const int32_t y2 = by * BY + ql / BZ, z2 = bz * BZ + ql % BZ;
        if (y2 >= g.ny || z2 >= g.nz) continue;
        const int64_t b2 = int64_t(z2) * plane + int64_t(y2) * g.nx;
        for (int32_t x2 = q; x2 < g.nx; x2 += WAVE) {
          const double *src = lds + size_t(ql * stride + x2) * E;
          const uint32_t o2 = uint32_t(real(b2 + x2)) * uint32_t(E * 8);
#pragma unroll
          for (int e = 0; e < E; ++e)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(bu2, src[e]), Ro,
                                                  int(o2 + uint32_t(e * 8)), 0, 0);
        }
      }
      asm volatile("" ::: "memory");
    }
    __syncthreads();
  }
}

// ---- grid factorisation -----------------------------------------------
// ILU(0) (Algorithm 1) of a matrix on a 7-point or 5-point grid pattern,
// in one launch with the forward grid sweep's walk (blocks of lines, one
// wavefront, lane q = zl + BZ yl at x = l - yl - zl).  On this pattern no
// update of row i reaches an entry other than its diagonal: for each lower
// neighbour k of row i (z - 1, y - 1, x - 1: ascending column), l_ik =
// a_ik / u_kk, then u_ii -= u_ki l_ik, where u_ki is the (unchanged) entry
// (k, i) of row k, the only entry of row k right of the diagonal that row
// i stores.  These are the operations, in the order, of the row-by-row
// factorisation (ilu0_level), so the factor is the same bit for bit.  u_kk
// comes from the lane's previous level (x - 1), lanes q - 1 and q - BZ
// (z - 1, y - 1), or, across blocks, from `ex` (the pivots of the rows the
// next block reads, pre-filled with the sentinel) with the bounded
// sentinel-checked wait.
//
// Records (in the sweep's processing order, see grid_gather): ra[pos] holds
// the row's three lower entries a_ik in term order and a_ii, each promoted
// to KF limbs; rb[pos] the three entries u_ki.  The kernel overwrites ra
// with l_ik and u_ii; grid_fac_scatter then writes them into the factor.
static __global__ void grid_fac_gather(int64_t n, GridDims g, int by_, int C, int KF,
                                       const int32_t *__restrict__ diag,
                                       const double *__restrict__ val, double *__restrict__ ra,
                                       double *__restrict__ rb) {
  const int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (i >= n) return;
  const int bz_ = WAVE / by_, V = C * KF;
  const int64_t pl = int64_t(g.nx) * g.ny;
  const int64_t x = i % g.nx, y = (i / g.nx) % g.ny, z = i / pl;
  const int32_t by = int32_t(y / by_), bz = int32_t(z / bz_);
  const int yl = int(y % by_), zl = int(z % bz_), q = zl + bz_ * yl;
  const int64_t l = x + yl + zl;
  int64_t pos = grid_block_start(g, by_, bz_, by, bz);
  for (int q2 = 0; q2 < WAVE; ++q2) {
    const int yl2 = q2 / bz_, zl2 = q2 % bz_;
    if (int64_t(by) * by_ + yl2 >= g.ny || int64_t(bz) * bz_ + zl2 >= g.nz) continue;
    const int64_t c = yl2 + zl2;
    pos += min(max(l - c, int64_t(0)), int64_t(g.nx));
    if (q2 < q && l - c >= 0 && l - c < g.nx) ++pos;
  }
  const bool ex = x > 0, ey = y > 0, ez = z > 0;
  const bool xu = x < g.nx - 1, yu = y < g.ny - 1;
  const int64_t dg = diag[i];
  const int nlow = int(ex) + int(ey) + int(ez);
  // term order z, y, x: lower entries of row i, and entries (k, i) of rows k
  const bool has[3] = {ez, ey, ex};
  const int64_t pa[3] = {dg - nlow, dg - nlow + int(ez), dg - 1};
  const int64_t pb[3] = {ez ? diag[i - pl] + 1 + int(xu) + int(yu) : 0,
                         ey ? diag[i - g.nx] + 1 + int(xu) : 0, ex ? diag[i - 1] + 1 : 0};
  double *oa = ra + pos * 4 * V, *ob = rb + pos * 4 * V;
  for (int d = 0; d < 4; ++d)
    for (int c = 0; c < C; ++c)
      for (int k = 0; k < KF; ++k) {
        const double va = d == 3 ? val[dg * C + c] : (has[d] ? val[pa[d] * C + c] : 0.0);
        const double vb = d < 3 && has[d] ? val[pb[d] * C + c] : 0.0;
        oa[d * V + c * KF + k] = k == 0 ? va : 0.0;
        ob[d * V + c * KF + k] = k == 0 ? vb : 0.0;
      }
}

template <int C, int KF, int BY>
__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(1, 1))) void ilu0_grid(
    int64_t n, GridDims g, double *ra, const double *__restrict__ rb, double *ex,
    int32_t *ticket, int32_t *abort_flag, int32_t *bad) {
  constexpr int BZ = grid_bz<BY>();
  constexpr int V = C * KF;
  __shared__ int32_t cur;
  const int q = int(threadIdx.x);
  const int zl = q % BZ, yl = q / BZ;
  const int64_t plane = int64_t(g.nx) * g.ny;
  const __amdgpu_buffer_rsrc_t Ra = buf_rsrc(ra, n * 4 * V * 8);
  const __amdgpu_buffer_rsrc_t Rb = buf_rsrc(rb, n * 4 * V * 8);
  const __amdgpu_buffer_rsrc_t Rx = buf_rsrc(ex, n * V * 8);
  for (;;) {
    if (q == 0) cur = atomicAdd(ticket, 1);
    __syncthreads();
    const int32_t b = cur;
    __syncthreads();
    if (b >= g.nby * g.nbz) break;
    const int32_t by = b % g.nby, bz = b / g.nby;
    const int32_t y = by * BY + yl, z = bz * BZ + zl;
    const bool line = y < g.ny && z < g.nz;
    const int64_t base = int64_t(z) * plane + int64_t(y) * g.nx;
    const bool ey = y > 0, ez = z > 0;
    const bool exty = ey && yl == 0, extz = ez && zl == 0;
    const bool pub = line && ((yl == BY - 1 && y < g.ny - 1) || (zl == BZ - 1 && z < g.nz - 1));
    const int32_t nlev = g.nx + (BY - 1) + (BZ - 1);
    int64_t run = grid_block_start(g, BY, BZ, by, bz);
    el<C, KF> prev = el_zero<C, KF>();
    for (int32_t l = 0; l < nlev; ++l) {
      const int32_t x = l - yl - zl;
      const bool a = line && x >= 0 && x < g.nx;
      const uint64_t m = __ballot(a);
      const int64_t pos = run + int64_t(__builtin_amdgcn_mbcnt_hi(
                                    uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0)));
      run += __popcll(m);
      const uint32_t orec = a ? uint32_t(pos) * uint32_t(4 * V * 8) : BUF_OOB;
      double fa[4 * V], fb[3 * V];
      buf_ld_n<4 * V, 0>(Ra, orec, fa);
      buf_ld_n<3 * V, 0>(Rb, orec, fb);
      // pivots of the lower neighbours
      el<C, KF> vy, vz = el_zero<C, KF>();
      if constexpr (BZ == 1) {
        vy = lane_prev<C, KF>(prev);
      } else {
        vz = lane_prev<C, KF>(prev);
        vy = lane_read<C, KF>(prev, q >= BZ ? q - BZ : 0);
      }
      const int64_t is = base + x;
      const uint32_t oy = (a && exty) ? uint32_t(is - g.nx) * uint32_t(V * 8) : BUF_OOB;
      const uint32_t oz = (a && extz) ? uint32_t(is - plane) * uint32_t(V * 8) : BUF_OOB;
      el<C, KF> wy, wz;
      el_ld_agent<C, KF>(Rx, oy, wy);
      el_ld_agent<C, KF>(Rx, oz, wz);
      for (int it = 0;; ++it) {
        const bool my = a && exty && el_has_sentinel<C, KF>(wy);
        const bool mz = a && extz && el_has_sentinel<C, KF>(wz);
        if (!(my | mz)) break;
        if ((it & 63) == 63 && ld_agent_i(abort_flag)) break;
        if (it >= SPIN_LIMIT) {
          __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(2);
        el<C, KF> ny_, nz_;
        el_ld_agent<C, KF>(Rx, my ? oy : BUF_OOB, ny_);
        el_ld_agent<C, KF>(Rx, mz ? oz : BUF_OOB, nz_);
        wy = el_select<C, KF>(my, ny_, wy);
        wz = el_select<C, KF>(mz, nz_, wz);
      }
      el<C, KF> u;
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int k = 0; k < KF; ++k) u.c[c].v[k] = fa[3 * V + c * KF + k];
      double lo[3][V];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        // term order z, y, x
        bool has;
        el<C, KF> ukk;
        if (d == 0) {
          has = ez;
          ukk = el_select<C, KF>(extz, wz, vz);
        } else if (d == 1) {
          has = ey;
          ukk = el_select<C, KF>(exty, wy, vy);
        } else {
          has = x > 0;
          ukk = prev;
        }
        double dk[V];
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
          for (int k = 0; k < KF; ++k) dk[c * KF + k] = ukk.c[c].v[k];
        el<C, KF> aik;
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
          for (int k = 0; k < KF; ++k) aik.c[c].v[k] = fa[d * V + c * KF + k];
        const el<C, KF> lik = el_div_k<C, KF, KF>(aik, dk);
        const el<C, KF> un = el_sub<C, KF>(u, el_mul_f<C, KF, KF>(fb + d * V, lik));
        u = el_select<C, KF>(has, un, u);
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
          for (int k = 0; k < KF; ++k) lo[d][c * KF + k] = has ? lik.c[c].v[k] : 0.0;
      }
      // results into the record (l_ik, then u_ii); the pivot of a row that
      // the next block reads also to ex, at agent scope
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int v = 0; v < V; ++v)
          __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(bu2, lo[d][v]), Ra,
                                                int(orec + uint32_t((d * V + v) * 8)), 0, 0);
      const uint32_t ox = (a && pub) ? uint32_t(is) * uint32_t(V * 8) : BUF_OOB;
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int k = 0; k < KF; ++k) {
          double v = u.c[c].v[k];
          v = v != v ? __builtin_nan("") : v;
          u.c[c].v[k] = v;
          __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(bu2, v), Ra,
                                                int(orec + uint32_t((3 * V + c * KF + k) * 8)), 0, 0);
          __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(bu2, v), Rx,
                                                int(ox + uint32_t((c * KF + k) * 8)), 0, BUF_AGENT);
        }
      if (a && el_is_zero<C, KF>(u)) atomicMin(bad, int32_t(is));
      prev = el_select<C, KF>(a, u, prev);
    }
    __syncthreads();
  }
}

// The factor from the records of ilu0_grid: row i's lower entries (term
// order z, y, x, the stored ones) and its diagonal, C * KF doubles each.
static __global__ void grid_fac_scatter(int64_t n, GridDims g, int by_, int V,
                                        const int32_t *__restrict__ diag,
                                        const double *__restrict__ ra, double *__restrict__ f) {
  const int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (i >= n) return;
  const int bz_ = WAVE / by_;
  const int64_t pl = int64_t(g.nx) * g.ny;
  const int64_t x = i % g.nx, y = (i / g.nx) % g.ny, z = i / pl;
  const int32_t by = int32_t(y / by_), bz = int32_t(z / bz_);
  const int yl = int(y % by_), zl = int(z % bz_), q = zl + bz_ * yl;
  const int64_t l = x + yl + zl;
  int64_t pos = grid_block_start(g, by_, bz_, by, bz);
  for (int q2 = 0; q2 < WAVE; ++q2) {
    const int yl2 = q2 / bz_, zl2 = q2 % bz_;
    if (int64_t(by) * by_ + yl2 >= g.ny || int64_t(bz) * bz_ + zl2 >= g.nz) continue;
    const int64_t c = yl2 + zl2;
    pos += min(max(l - c, int64_t(0)), int64_t(g.nx));
    if (q2 < q && l - c >= 0 && l - c < g.nx) ++pos;
  }
  const bool has[3] = {z > 0, y > 0, x > 0};
  const int64_t dg = diag[i];
  int64_t p = dg - (int(has[0]) + int(has[1]) + int(has[2]));
  const double *r = ra + pos * 4 * V;
  for (int d = 0; d < 3; ++d)
    if (has[d]) {
      for (int v = 0; v < V; ++v) f[p * V + v] = r[d * V + v];
      ++p;
    }
  for (int v = 0; v < V; ++v) f[dg * V + v] = r[3 * V + v];
}

// Prepares one apply: the words that other workgroups poll filled with
// SENTINEL (rows list1[0..cnt1) of out1 and list2[0..cnt2) of out2, or
// rows 0..cnt-1 when a list is null: the level schedule polls every row),
// the per-level counters zeroed and the two tickets reset (a kernel rather
// than a memset, so the step can be graph-captured).  The abort word is
// reset only when abort_reset is non-null: inside a solve it persists so
// the host sees any watchdog event at the end.
static __global__ void trsv_prep(int E, const int32_t *__restrict__ list1, int64_t cnt1,
                                 double *out1, const int32_t *__restrict__ list2, int64_t cnt2,
                                 double *out2, int32_t nlev1, int32_t *lev1, int32_t nlev2,
                                 int32_t *lev2, int32_t *ticket1, int32_t *ticket2,
                                 int32_t *abort_reset, const int32_t *done) {
  if (done && *done) return;
  const int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  const double sent = __builtin_bit_cast(double, (unsigned long long)SENTINEL);
  const int64_t q = i / E, e = i - q * E;
  if (q < cnt1) out1[(list1 ? int64_t(list1[q]) : q) * E + e] = sent;
  if (q < cnt2) out2[(list2 ? int64_t(list2[q]) : q) * E + e] = sent;
  if (i < nlev1) lev1[i] = 0;
  if (i < nlev2) lev2[i] = 0;
  if (i == 0) {
    *ticket1 = 0;
    *ticket2 = 0;
    if (abort_reset) *abort_reset = 0;
  }
}

}  // namespace mpk
