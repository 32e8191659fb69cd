// batched.hip -- many independent systems of uneven size solved by ILU(0)-
// preconditioned BiCGSTAB in one persistent launch.
//
// Each system is a job for a team of T workgroups that run on one XCD (T = 1
// for small systems, or when teams are off).  The host spreads the jobs over
// one queue per XCD, balanced by stored entries, and lists T tickets per job
// (its members).  A workgroup reads the XCD it runs on and takes tickets
// from that queue only, so a team shares one L2: the vectors a system
// gathers (x in A x, y in the substitutions) stay in that cache instead of
// competing with those of 32 other systems.  Members split every row loop
// and meet at team barriers (an arrival counter in the L2; the L1 of each
// CU is invalidated after it); a team of one uses the workgroup barrier.
// Within a job, in order: pattern checks, forward and backward level
// analysis, the ILU(0) factorisation (Algorithm 1, level by level, IKJ
// rows) and the BiCGSTAB passes with the ILU(0) substitutions (Algorithm 2,
// level by level).  The per-row arithmetic is the single-system path's.
// Inner products are summed per tile of TILE rows (a fixed 256-thread tree)
// and then over the tiles (a fixed tree), so the results are bitwise the
// same for every team size, grid size and job order.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace mpk {

// Per-system descriptor (device array).
struct BSys {
  int64_t n, nnz;
  const int32_t *rp, *ci;
  const double *val, *b;
  double *x;
  double *f;          // factor values [nnz * KF]
  int32_t *diag;      // [n]
  int32_t *lvl;       // [n] level scratch
  int32_t *ordL, *ordU;    // [n] rows by forward / backward level
  int32_t *lptL, *lptU;    // [n + 2] level pointers
  int32_t *cur;       // [n + 2] scatter cursors
  double *vec;        // 9 vectors of n * K doubles
  double *part;       // tile partial sums, two buffers of [ntiles][2][K]
};

// Per-system result (device array).
struct BOut {
  int64_t iters, bad_row;
  int32_t status, pad;
  double relres_recursive, relres_true;
};

// Control words of one job, shared by its team (set by bctl_init before
// the launch; 64 bytes, so jobs do not share a cache line).
struct BCtl {
  int32_t bar;           // team barrier arrivals
  int32_t bad, flag;     // first bad row (INT_MAX) and worst code of the pattern checks
  int32_t maxlL, maxlU;  // highest forward / backward level
  int32_t chg;           // last level-analysis round in which a level changed
  int32_t pivbad;        // first zero pivot (INT_MAX)
  int32_t pad[9];
};

// A queue entry: member `member` of the team of system `sys`.
struct BEnt {
  int32_t sys, member;
};

constexpr int NBV = 9;  // r, r~, p, p^, v, s, s^, t, x (working copy)
constexpr int TILE = 16 * BLOCK;   // rows per inner-product tile
constexpr int TMAX = 64;           // largest team
constexpr int NQ = 16;             // XCD queues (XCC_ID is four bits)
constexpr int QSTRIDE = 16;        // ints between queue tickets (one per 64 bytes)
// A team member waits at most this long (100 MHz clock ticks) for the rest
// of its team; past it the launch is abandoned with MPK_EWATCHDOG.
constexpr uint64_t TEAM_WAIT_TICKS = 1000000000ull;  // 10 s

__host__ __device__ constexpr int64_t ntiles(int64_t n) { return (n + TILE - 1) / TILE; }

// Shared scalars of the system being solved.
template <int K> struct BShared {
  int32_t sys, member, flag, nlevL, nlevU, go;
  double nr0sq, nbsq, nr2;
  double rho[K], alpha[K], omega[K], beta[K];
  double d[2][K];
};

__device__ __forceinline__ bool bstop(double nr2, double nr0sq, double er, double ea) {
  return sqrt(nr2) < er * sqrt(nr0sq) + ea;
}

// Waits until this thread's memory operations (atomics included) are done.
__device__ __forceinline__ void drain() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ __forceinline__ int32_t xcc_id() {
  return int32_t(__builtin_amdgcn_s_getreg((3 << 11) | 20) & 15);  // HW_REG_XCC_ID[3:0]
}

// A team as one member sees it: T workgroups on one XCD, this one number
// m; gen counts the barriers passed (the same sequence in every member).
struct Team {
  BCtl *ctl;
  int32_t T, m, gen;
  int32_t *abort;
  __device__ int64_t gt() const { return int64_t(m) * BLOCK + threadIdx.x; }
  __device__ int64_t gs() const { return int64_t(T) * BLOCK; }
};

// Team barrier: every store of the team issued before it is seen by every
// load after it.  Stores reach the XCD's L2 (the L1 writes through) before
// the arrival is counted; after the barrier each CU drops its L1 lines with
// an agent-scope invalidate (the workgroup-scope one leaves them valid
// outside split-workgroup mode), so loads read the L2 that all members
// share.  Returns false when the launch is abandoned (a member waited past
// TEAM_WAIT_TICKS, here or elsewhere).
template <int K>
__device__ __forceinline__ bool tsync(Team &tm, BShared<K> &sh) {
  if (tm.T == 1) {
    __syncthreads();
    return true;
  }
  drain();
  __syncthreads();
  ++tm.gen;
  if (threadIdx.x == 0) {
    int32_t ok = 1;
    __hip_atomic_fetch_add(&tm.ctl->bar, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t target = tm.gen * tm.T;
    const uint64_t t0 = wall_clock64();
    for (int it = 0; __hip_atomic_load(&tm.ctl->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                     target;
         ++it) {
      if ((it & 63) == 63) {
        if (ld_agent_i(tm.abort)) {
          ok = 0;
          break;
        }
        if (wall_clock64() - t0 > TEAM_WAIT_TICKS) {
          __hip_atomic_store(tm.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
      __builtin_amdgcn_s_sleep(1);
    }
    sh.go = ok;
  }
  __syncthreads();
  asm volatile("buffer_inv sc1" ::: "memory");
  return sh.go != 0;
}

// Tile partial of two per-thread sums: the fixed tree of block_reduce,
// written to dst[2][K] by thread 0.
template <int K>
__device__ __forceinline__ void tile_partial(const mp<K> &a, const mp<K> &c, double *dst) {
  el<1, K> d[2];
  d[0].c[0] = a;
  d[1].c[0] = c;
  block_reduce<1, K, 2>(d, dst);
  __syncthreads();  // block_reduce's LDS is free again
}

// After a team barrier: the sum over the nt tile partials (fixed tree,
// the same in every member) into sh.d.
template <int K>
__device__ __forceinline__ void fold_tiles(const double *part, int64_t nt, BShared<K> &sh) {
  el<1, K> tot[2];
  reduce_partials<1, K, 2>(part, int(nt), tot);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int k = 0; k < K; ++k) sh.d[q][k] = tot[q].c[0].v[k];
  __syncthreads();
}

#define TSYNC()                         \
  do {                                  \
    if (!tsync<K>(tm, sh)) return false; \
  } while (0)

// Levels of one sweep, in chunks of T * BLOCK consecutive rows in the
// sweep's order: dependencies before the chunk are final; those inside it
// are iterated to the fixed point from below until a round changes nothing
// (a team of one in LDS, two workgroup barriers per round; a larger team in
// memory, one team barrier per round: levels only grow, so the values read
// in a round may be old or new).  Then rows are bucketed by level
// (counting sort; the order inside a level is irrelevant because its rows
// are independent).  round counts the team's rounds (the same in every
// member).
template <int K>
__device__ bool blevels(const BSys &S, Team &tm, BShared<K> &sh, bool lower, int32_t *ord,
                        int32_t *lpt, int32_t *maxl_word, int32_t &round, int32_t &nlev_out) {
  const int tid = threadIdx.x;
  const int64_t n = S.n, gt = tm.gt(), GS = tm.gs();
  int32_t mymax = 0;
  __shared__ int32_t tl[BLOCK];  // a team of one iterates its chunk in LDS
  for (int64_t c = 0; c < n; c += GS) {
    const int64_t t = c + gt;
    const int64_t i = lower ? t : n - 1 - t;
    const bool valid = t < n;
    int32_t ext = 0;
    if (valid) {
      for (int32_t q = S.rp[i]; q < S.rp[i + 1]; ++q) {
        const int32_t j = S.ci[q];
        const bool dep = lower ? j < i : j > i;
        const int64_t tj = lower ? j : n - 1 - j;
        if (dep && tj < c) ext = max(ext, S.lvl[j] + 1);
      }
    }
    int32_t cur = ext;
    if (tm.T == 1) {
      tl[tid] = ext;
      __syncthreads();
      for (;;) {
        int32_t l = ext;
        if (valid) {
          for (int32_t q = S.rp[i]; q < S.rp[i + 1]; ++q) {
            const int32_t j = S.ci[q];
            const bool dep = lower ? j < i : j > i;
            const int64_t tj = lower ? j : n - 1 - j;
            if (dep && tj >= c) l = max(l, tl[tj - c] + 1);
          }
        }
        __syncthreads();  // every read of tl in this round is done
        const bool ch = valid && l != tl[tid];
        if (ch) tl[tid] = l;
        if (!__syncthreads_or(ch)) break;
      }
      cur = tl[tid];
      if (valid) S.lvl[i] = cur;
      __syncthreads();
    } else {
      if (valid) S.lvl[i] = ext;
      TSYNC();
      for (;;) {
        int32_t l = ext;
        if (valid) {
          for (int32_t q = S.rp[i]; q < S.rp[i + 1]; ++q) {
            const int32_t j = S.ci[q];
            const bool dep = lower ? j < i : j > i;
            const int64_t tj = lower ? j : n - 1 - j;
            if (dep && tj >= c) l = max(l, S.lvl[j] + 1);
          }
        }
        l = max(l, cur);  // levels only grow
        const bool ch = valid && l != cur;
        if (ch) {
          S.lvl[i] = l;
          cur = l;
        }
        if (__syncthreads_or(ch) && tid == 0) {
          atomicMax(&tm.ctl->chg, round + 1);
          drain();
        }
        TSYNC();
        // a member already in the next round may have raised chg further; a
        // member enters that round only after some level changed in this one
        const bool again = ld_agent_i(&tm.ctl->chg) >= round + 1;
        ++round;
        if (!again) break;
      }
    }
    mymax = max(mymax, cur);
  }
  if (mymax > 0) atomicMax(maxl_word, mymax);
  drain();
  TSYNC();
  const int32_t nlev = ld_agent_i(maxl_word) + 1;
  for (int64_t l = gt; l <= nlev; l += GS) lpt[l] = 0;
  TSYNC();
  for (int64_t i = gt; i < n; i += GS) atomicAdd(&lpt[S.lvl[i] + 1], 1);
  drain();
  TSYNC();
  if (tm.m == 0 && tid == 0)
    for (int32_t l = 0; l < nlev; ++l) lpt[l + 1] += lpt[l];
  TSYNC();
  for (int64_t l = gt; l < nlev; l += GS) S.cur[l] = lpt[l];
  TSYNC();
  for (int64_t i = gt; i < n; i += GS) ord[atomicAdd(&S.cur[S.lvl[i]], 1)] = int32_t(i);
  drain();
  TSYNC();
  nlev_out = nlev;
  return true;
}

// Row i of the factorisation (Algorithm 1, IKJ): for each k < i stored in
// row i (ascending), l_ik = a_ik / u_kk, then a_ij -= l_ik u_kj for every
// stored j > k of row k that row i also stores.  Rows of at most RCACHE
// entries keep their column indices in the thread's LDS slice, so the
// search for j is an LDS walk; row k's upper part is read eight entries at
// a time and the matched a_ij are loaded together.  Longer rows take the
// entry-by-entry path.  Both perform the same operations in the same order.
constexpr int RCACHE = 32;

template <int KF>
__device__ __forceinline__ void bfactor_row(const BSys &S, int32_t i, int32_t *lc,
                                            int32_t *bad) {
  const int32_t a = S.rp[i], e = S.rp[i + 1], di = S.diag[i];
  if (e - a <= RCACHE) {
    for (int32_t b0 = a; b0 < e; b0 += 8) {
      int32_t cb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) cb[u] = S.ci[min(b0 + u, e - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (b0 + u < e) lc[b0 + u - a] = cb[u];
    }
    for (int32_t p = a; p < di; ++p) {
      const int32_t k = lc[p - a];
      const int32_t dk = S.diag[k], q1 = S.rp[k + 1];
      el<1, KF> lik = el_load<1, KF>(S.f + size_t(p) * KF);
      lik = el_div_k<1, KF, KF>(lik, S.f + size_t(dk) * KF);
      el_store<1, KF>(S.f + size_t(p) * KF, lik);
      int32_t r = p + 1 - a;  // walk position in row i
      for (int32_t qb = dk + 1; qb < q1; qb += 8) {
        int32_t cq[8], rm[8];
        double fk[8][KF];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int32_t q = min(qb + u, q1 - 1);
          cq[u] = S.ci[q];
#pragma unroll
          for (int v = 0; v < KF; ++v) fk[u][v] = S.f[size_t(q) * KF + v];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          rm[u] = -1;
          if (qb + u < q1) {
            while (r < e - a && lc[r] < cq[u]) ++r;
            if (r < e - a && lc[r] == cq[u]) rm[u] = r;
          }
        }
        el<1, KF> aij[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          aij[u] = el_load<1, KF>(S.f + size_t(a + (rm[u] >= 0 ? rm[u] : 0)) * KF);
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (rm[u] >= 0)
            el_store<1, KF>(S.f + size_t(a + rm[u]) * KF,
                            el_sub<1, KF>(aij[u], el_mul_f<1, KF, KF>(fk[u], lik)));
      }
    }
  } else {
    for (int32_t p = a; p < e && S.ci[p] < i; ++p) {
      const int32_t k = S.ci[p];
      el<1, KF> lik = el_load<1, KF>(S.f + size_t(p) * KF);
      lik = el_div_k<1, KF, KF>(lik, S.f + size_t(S.diag[k]) * KF);
      el_store<1, KF>(S.f + size_t(p) * KF, lik);
      int32_t r = p + 1;
      for (int32_t q = S.diag[k] + 1; q < S.rp[k + 1]; ++q) {
        const int32_t j = S.ci[q];
        while (r < e && S.ci[r] < j) ++r;
        if (r < e && S.ci[r] == j) {
          el<1, KF> aij = el_load<1, KF>(S.f + size_t(r) * KF);
          el<1, KF> prod = el_mul_f<1, KF, KF>(S.f + size_t(q) * KF, lik);
          el_store<1, KF>(S.f + size_t(r) * KF, el_sub<1, KF>(aij, prod));
        }
      }
    }
  }
  if (el_is_zero<1, KF>(el_load<1, KF>(S.f + size_t(di) * KF))) atomicMin(bad, i);
}


template <int K, int KF>
__device__ bool bfactor(const BSys &S, Team &tm, BShared<K> &sh, int32_t nlev, int32_t *lcols) {
  const int64_t gt = tm.gt(), GS = tm.gs();
  for (int64_t p = gt; p < S.nnz; p += GS) {
    S.f[p * KF] = S.val[p];
    if constexpr (KF == 2) S.f[p * KF + 1] = 0.0;
  }
  TSYNC();
  for (int32_t l = 0; l < nlev; ++l) {
    for (int64_t pos = S.lptL[l] + gt; pos < S.lptL[l + 1]; pos += GS)
      bfactor_row<KF>(S, S.ordL[pos], lcols + threadIdx.x * RCACHE, &tm.ctl->pivbad);
    TSYNC();
  }
  drain();  // zero-pivot reports, read back after the barrier
  TSYNC();
  return true;
}

// acc - sum over p in [p0, p1) of f_p v_{ci[p]}, subtracted in ascending p.
// Entries are taken eight at a time: their indices, factor values and
// vector words are requested together (indices clamped into the range;
// the extra words are not used), so a row costs two memory round trips per
// eight entries instead of two per entry.
template <int K, int KF>
__device__ __forceinline__ el<1, K> bsub_products(el<1, K> acc, int32_t p0, int32_t p1,
                                                  const int32_t *__restrict__ ci,
                                                  const double *__restrict__ f, const double *v) {
  constexpr int U = 8;
  for (int32_t pb = p0; pb < p1; pb += U) {
    int32_t cj[U];
    double fv[U][KF];
    el<1, K> yv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t p = min(pb + u, p1 - 1);
      cj[u] = ci[p];
#pragma unroll
      for (int q = 0; q < KF; ++q) fv[u][q] = f[size_t(p) * KF + q];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) yv[u] = el_load<1, K>(v + size_t(cj[u]) * K);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (pb + u < p1) acc = el_sub<1, K>(acc, el_mul_f<1, K, KF>(fv[u], yv[u]));
  }
  return acc;
}

// The same for two rows at once (rows w = 0, 1 with entry ranges
// [p0[w], p1[w])): both rows' loads are issued before either is used, so a
// thread keeps twice as many requests in flight.  Each row's products are
// subtracted in its own ascending order, as above.
template <int K> constexpr int bpair_batch() { return K <= 2 ? 8 : 4; }

template <int K, int KF>
__device__ __forceinline__ void bsub_products2(el<1, K> (&acc)[2], const int32_t (&p0)[2],
                                               const int32_t (&p1)[2],
                                               const int32_t *__restrict__ ci,
                                               const double *__restrict__ f, const double *v) {
  constexpr int U = bpair_batch<K>();
  int32_t pb[2] = {p0[0], p0[1]};
  while (pb[0] < p1[0] || pb[1] < p1[1]) {
    int32_t cj[2][U];
    double fv[2][U][KF];
    el<1, K> yv[2][U];
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t p = pb[w] < p1[w] ? min(pb[w] + u, p1[w] - 1) : 0;
        cj[w][u] = ci[p];
#pragma unroll
        for (int q = 0; q < KF; ++q) fv[w][u][q] = f[size_t(p) * KF + q];
      }
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
      for (int u = 0; u < U; ++u) yv[w][u] = el_load<1, K>(v + size_t(cj[w][u]) * K);
#pragma unroll
    for (int w = 0; w < 2; ++w) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (pb[w] + u < p1[w]) acc[w] = el_sub<1, K>(acc[w], el_mul_f<1, K, KF>(fv[w][u], yv[w][u]));
      pb[w] += U;
    }
  }
}

// Two rows of y = A x (as row_spmv: products in ascending column order,
// accumulated from the first product; an empty row gives 0).
template <int K>
__device__ __forceinline__ void bspmv_rows2(const BSys &S, const int64_t (&i)[2], const bool (&ok)[2],
                                            const double *x, mp<K> (&y)[2]) {
  constexpr int U = bpair_batch<K>();
  int32_t pb[2], pe[2], p0[2];
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    p0[w] = ok[w] ? S.rp[i[w]] : 0;
    pe[w] = ok[w] ? S.rp[i[w] + 1] : 0;
    pb[w] = p0[w];
    y[w] = mp_zero<K>();
  }
  while (pb[0] < pe[0] || pb[1] < pe[1]) {
    int32_t cj[2][U];
    double fv[2][U][1];
    el<1, K> xv[2][U];
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t p = pb[w] < pe[w] ? min(pb[w] + u, pe[w] - 1) : 0;
        cj[w][u] = S.ci[p];
        fv[w][u][0] = S.val[p];
      }
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
      for (int u = 0; u < U; ++u) xv[w][u] = el_load<1, K>(x + size_t(cj[w][u]) * K);
#pragma unroll
    for (int w = 0; w < 2; ++w) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (pb[w] + u < pe[w]) {
          const el<1, K> t = el_mul_f<1, K, 1>(fv[w][u], xv[w][u]);
          y[w] = (pb[w] + u == p0[w]) ? t.c[0] : el_add<1, K>(el<1, K>{{y[w]}}, t).c[0];
        }
      pb[w] += U;
    }
  }
}

// z = (L U)^{-1} r with the level orders; y (intermediate) and z are
// vectors of the system.  Row arithmetic as Algorithm 2: the strict lower
// part of row i is [rp_i, diag_i), the strict upper part (diag_i, rp_i+1).
// Each thread takes two rows of a level per step (positions pos and
// pos + T * BLOCK); a team barrier ends every level.
template <int K, int KF>
__device__ bool bapply(const BSys &S, Team &tm, BShared<K> &sh, const double *r, double *y,
                       double *z) {
  const int64_t gt = tm.gt(), GS = tm.gs();
  for (int32_t l = 0; l < sh.nlevL; ++l) {
    const int64_t pe = S.lptL[l + 1];
    for (int64_t pos = S.lptL[l] + gt; pos < pe; pos += 2 * GS) {
      const bool two = pos + GS < pe;
      const int32_t i0 = S.ordL[pos], i1 = two ? S.ordL[pos + GS] : i0;
      el<1, K> acc[2] = {el_load<1, K>(r + size_t(i0) * K), el_load<1, K>(r + size_t(i1) * K)};
      const int32_t a[2] = {S.rp[i0], two ? S.rp[i1] : 0};
      const int32_t b[2] = {S.diag[i0], two ? S.diag[i1] : 0};
      bsub_products2<K, KF>(acc, a, b, S.ci, S.f, y);
      el_store<1, K>(y + size_t(i0) * K, acc[0]);
      if (two) el_store<1, K>(y + size_t(i1) * K, acc[1]);
    }
    TSYNC();
  }
  for (int32_t l = 0; l < sh.nlevU; ++l) {
    const int64_t pe = S.lptU[l + 1];
    for (int64_t pos = S.lptU[l] + gt; pos < pe; pos += 2 * GS) {
      const bool two = pos + GS < pe;
      const int32_t i0 = S.ordU[pos], i1 = two ? S.ordU[pos + GS] : i0;
      el<1, K> acc[2] = {el_load<1, K>(y + size_t(i0) * K), el_load<1, K>(y + size_t(i1) * K)};
      const int32_t a[2] = {S.diag[i0] + 1, two ? S.diag[i1] + 1 : 0};
      const int32_t b[2] = {S.rp[i0 + 1], two ? S.rp[i1 + 1] : 0};
      bsub_products2<K, KF>(acc, a, b, S.ci, S.f, z);
      acc[0] = el_div_k<1, K, KF>(acc[0], S.f + size_t(S.diag[i0]) * KF);
      el_store<1, K>(z + size_t(i0) * K, acc[0]);
      if (two) {
        acc[1] = el_div_k<1, K, KF>(acc[1], S.f + size_t(S.diag[i1]) * KF);
        el_store<1, K>(z + size_t(i1) * K, acc[1]);
      }
    }
    TSYNC();
  }
  return true;
}

template <int K>
__device__ __forceinline__ mp<K> bspmv_row(const BSys &S, int64_t i, const double *x) {
  return row_spmv<1, K>(i, S.rp, S.ci, S.val, x).c[0];
}

template <int K> __device__ __forceinline__ mp<K> ldk(const double *p, int64_t i) {
  mp<K> v;
#pragma unroll
  for (int k = 0; k < K; ++k) v.v[k] = p[size_t(i) * K + k];
  return v;
}
template <int K> __device__ __forceinline__ void stk(double *p, int64_t i, const mp<K> &v) {
#pragma unroll
  for (int k = 0; k < K; ++k) p[size_t(i) * K + k] = v.v[k];
}
template <int K> __device__ __forceinline__ mp<K> shk(const double (&a)[K]) {
  mp<K> v;
#pragma unroll
  for (int k = 0; k < K; ++k) v.v[k] = a[k];
  return v;
}
template <int K> __device__ __forceinline__ void setk(double (&a)[K], const mp<K> &v) {
#pragma unroll
  for (int k = 0; k < K; ++k) a[k] = v.v[k];
}

// The next tile-partial buffer (two, used in turn: a member may write the
// next reduction's partials while another still reads the previous one's,
// never the one before).
template <int K>
__device__ __forceinline__ double *next_part(const BSys &S, int32_t &rcnt) {
  return S.part + size_t(rcnt++ & 1) * size_t(ntiles(S.n)) * 2 * K;
}

// Residual r = b - A x (stored when r != nullptr, and in r2 when r2 !=
// nullptr), with ||r||^2 and ||b||^2 into sh.d.
template <int K>
__device__ bool bresidual(const BSys &S, Team &tm, BShared<K> &sh, int32_t &rcnt, const double *x,
                          double *r, double *r2) {
  const int64_t nt = ntiles(S.n);
  double *part = next_part<K>(S, rcnt);
  for (int64_t c = tm.m; c < nt; c += tm.T) {
    mp<K> a = mp_zero<K>(), cc = mp_zero<K>();
    for (int k = 0; k < TILE / BLOCK; ++k) {
      const int64_t i = c * TILE + k * BLOCK + threadIdx.x;
      if (i < S.n) {
        mp<K> bi = ldk<K>(S.b, i);
        mp<K> ri = sub<K>(bi, bspmv_row<K>(S, i, x));
        if (r) stk<K>(r, i, ri);
        if (r2) stk<K>(r2, i, ri);
        mp<K> t1 = mul<K>(ri, ri), t2 = mul<K>(bi, bi);
        a = k == 0 ? t1 : add<K>(a, t1);
        cc = k == 0 ? t2 : add<K>(cc, t2);
      }
    }
    tile_partial<K>(a, cc, part + size_t(c) * 2 * K);
  }
  TSYNC();
  fold_tiles<K>(part, nt, sh);
  return true;
}

// y = A x over the tiles of this member with one inner product per row,
// dot(i, y_i) (its first value taken as is).  Two rows per thread and step.
template <int K, class Dot>
__device__ bool bspmv_dot(const BSys &S, Team &tm, BShared<K> &sh, int32_t &rcnt, const double *x,
                          double *y, Dot dot) {
  const int64_t n = S.n, nt = ntiles(n);
  double *part = next_part<K>(S, rcnt);
  for (int64_t c = tm.m; c < nt; c += tm.T) {
    mp<K> a = mp_zero<K>(), cc = mp_zero<K>();
    for (int k = 0; k < TILE / BLOCK; k += 2) {
      const int64_t i0 = c * TILE + k * BLOCK + threadIdx.x;
      const int64_t ii[2] = {i0, i0 + BLOCK};
      const bool ok[2] = {i0 < n, i0 + BLOCK < n};
      mp<K> yy[2];
      bspmv_rows2<K>(S, ii, ok, x, yy);
#pragma unroll
      for (int w = 0; w < 2; ++w)
        if (ok[w]) {
          stk<K>(y, ii[w], yy[w]);
          dot(ii[w], yy[w], k + w == 0, a, cc);
        }
    }
    tile_partial<K>(a, cc, part + size_t(c) * 2 * K);
  }
  TSYNC();
  fold_tiles<K>(part, nt, sh);
  return true;
}

// An elementwise row update over the tiles of this member with two inner
// products per row: upd(i, first, a, c).
template <int K, class Upd>
__device__ bool brows_dot(const BSys &S, Team &tm, BShared<K> &sh, int32_t &rcnt, Upd upd) {
  const int64_t n = S.n, nt = ntiles(n);
  double *part = next_part<K>(S, rcnt);
  for (int64_t c = tm.m; c < nt; c += tm.T) {
    mp<K> a = mp_zero<K>(), cc = mp_zero<K>();
    for (int k = 0; k < TILE / BLOCK; ++k) {
      const int64_t i = c * TILE + k * BLOCK + threadIdx.x;
      if (i < n) upd(i, k == 0, a, cc);
    }
    tile_partial<K>(a, cc, part + size_t(c) * 2 * K);
  }
  TSYNC();
  fold_tiles<K>(part, nt, sh);
  return true;
}

// One system, as member tm.m of its team.  Returns false when the launch
// is abandoned (watchdog).
template <int K, int KF>
__device__ bool run_job(const BSys &S, Team &tm, BShared<K> &sh, int32_t *lcols, BOut *out,
                        int32_t sid, double er, double ea, int64_t max_iter, int copy_x) {
  const int tid = threadIdx.x;
  const int64_t n = S.n, gt = tm.gt(), GS = tm.gs();
  const bool lead = tm.m == 0 && tid == 0;  // writes the report
  BOut o{};
  o.bad_row = -1;
  o.relres_true = -1.0;
  // ---- pattern checks: sorted unique columns, diagonal stored, finite
  {
    int32_t wbad = INT_MAX, wflag = 0;
    for (int64_t i = gt; i < n; i += GS) {
      int32_t dg = -1, code = 0;
      for (int32_t q = S.rp[i]; q < S.rp[i + 1]; ++q) {
        const int32_t j = S.ci[q];
        if (j < 0 || j >= n || (q > S.rp[i] && j <= S.ci[q - 1])) code = 1;
        if (j == i) dg = q;
        const double v = S.val[q];
        if (!(v - v == 0.0)) code = code ? code : 3;
      }
      if (dg < 0 && !code) code = 2;
      S.diag[i] = dg;
      if (code) {
        wbad = min(wbad, int32_t(i));
        wflag = max(wflag, code);
      }
    }
    if (wflag) {
      atomicMin(&tm.ctl->bad, wbad);
      atomicMax(&tm.ctl->flag, wflag);
      drain();  // read back after the barrier
    }
  }
  TSYNC();
  const int32_t pflag = ld_agent_i(&tm.ctl->flag);
  if (pflag) {
    if (lead) {
      o.status = pflag == 1 ? MPK_EPATTERN : (pflag == 2 ? MPK_ENO_DIAG : MPK_ENONFINITE);
      o.bad_row = ld_agent_i(&tm.ctl->bad);
      out[sid] = o;
    }
    return true;
  }
  // ---- analysis and factorisation
  int32_t round = 0, rcnt = 0;
  if constexpr (KF > 0) {
    int32_t nl = 0;
    if (!blevels<K>(S, tm, sh, true, S.ordL, S.lptL, &tm.ctl->maxlL, round, nl)) return false;
    if (tid == 0) sh.nlevL = nl;
    if (!blevels<K>(S, tm, sh, false, S.ordU, S.lptU, &tm.ctl->maxlU, round, nl)) return false;
    if (tid == 0) sh.nlevU = nl;
    __syncthreads();
    if (!bfactor<K, KF>(S, tm, sh, sh.nlevL, lcols)) return false;
    const int32_t pb = ld_agent_i(&tm.ctl->pivbad);
    if (pb != INT_MAX) {
      if (lead) {
        o.status = MPK_EZERO_PIVOT;
        o.bad_row = pb;
        out[sid] = o;
      }
      return true;
    }
  }
  // ---- BiCGSTAB (right-preconditioned, shadow r~ = r0)
  double *r = S.vec, *rt = S.vec + n * K, *p = S.vec + 2 * n * K, *ph = S.vec + 3 * n * K,
         *v = S.vec + 4 * n * K, *sv = S.vec + 5 * n * K, *shv = S.vec + 6 * n * K,
         *t = S.vec + 7 * n * K, *xw = S.vec + 8 * n * K;
  if (KF == 0) {
    ph = p;
    shv = sv;
  }
  for (int64_t i = gt; i < n * K; i += GS) xw[i] = S.x[i];
  TSYNC();
  if (!bresidual<K>(S, tm, sh, rcnt, xw, r, rt)) return false;
  if (tid == 0) {
    sh.nr0sq = sh.d[0][0];
    sh.nbsq = sh.d[1][0];
    sh.nr2 = sh.nr0sq;
    for (int k = 0; k < K; ++k) sh.rho[k] = sh.d[0][k];
    sh.flag = 0;
  }
  __syncthreads();
  int status = MPK_NOT_CONVERGED;
  int64_t it = 0;
  double true_nr2 = -1.0;
  if (is_zero<K>(shk<K>(sh.rho))) {
    status = MPK_BREAKDOWN;
    it = 1;
  }
  while (status == MPK_NOT_CONVERGED && it < max_iter) {
    ++it;
    // p = r (first pass) or r + beta (p - omega v)
    {
      const mp<K> om = shk<K>(sh.omega), be = shk<K>(sh.beta);
      for (int64_t i = gt; i < n; i += GS) {
        mp<K> ri = ldk<K>(r, i);
        if (it == 1) {
          stk<K>(p, i, ri);
        } else {
          mp<K> tt = sub<K>(ldk<K>(p, i), mul<K>(om, ldk<K>(v, i)));
          stk<K>(p, i, add<K>(ri, mul<K>(be, tt)));
        }
      }
    }
    TSYNC();
    if constexpr (KF > 0)
      if (!bapply<K, KF>(S, tm, sh, p, t, ph)) return false;
    // v = A p^, sigma = <r~, v>
    if (!bspmv_dot<K>(S, tm, sh, rcnt, ph, v,
                      [&](int64_t i, const mp<K> &vi, bool first, mp<K> &a, mp<K> &) {
                        mp<K> tt = mul<K>(ldk<K>(rt, i), vi);
                        a = first ? tt : add<K>(a, tt);
                      }))
      return false;
    if (tid == 0) {
      mp<K> sig = shk<K>(sh.d[0]);
      sh.flag = is_zero<K>(sig) ? 1 : 0;
      if (!sh.flag) setk<K>(sh.alpha, div<K>(shk<K>(sh.rho), sig));
    }
    __syncthreads();
    if (sh.flag) {
      status = MPK_BREAKDOWN;
      break;
    }
    // s = r - alpha v, ||s||^2
    {
      const mp<K> al = shk<K>(sh.alpha);
      if (!brows_dot<K>(S, tm, sh, rcnt, [&](int64_t i, bool first, mp<K> &a, mp<K> &) {
            mp<K> si = sub<K>(ldk<K>(r, i), mul<K>(al, ldk<K>(v, i)));
            stk<K>(sv, i, si);
            mp<K> tt = mul<K>(si, si);
            a = first ? tt : add<K>(a, tt);
          }))
        return false;
    }
    const double nr2s = sh.d[0][0];
    if (bstop(nr2s, sh.nr0sq, er, ea)) {
      // candidate x + alpha p^ (held in t, unused until A s^) checked on
      // the true residual
      const mp<K> al = shk<K>(sh.alpha);
      for (int64_t i = gt; i < n; i += GS)
        stk<K>(t, i, add<K>(ldk<K>(xw, i), mul<K>(al, ldk<K>(ph, i))));
      TSYNC();
      if (!bresidual<K>(S, tm, sh, rcnt, t, nullptr, nullptr)) return false;
      true_nr2 = sh.d[0][0];
      if (bstop(true_nr2, sh.nr0sq, er, ea)) {
        for (int64_t i = gt; i < n * K; i += GS) xw[i] = t[i];
        __syncthreads();
        if (tid == 0) sh.nr2 = nr2s;
        status = MPK_OK;
        break;
      }
    }
    if constexpr (KF > 0)
      if (!bapply<K, KF>(S, tm, sh, sv, t, shv)) return false;
    // t = A s^, <t, s>, <t, t>
    if (!bspmv_dot<K>(S, tm, sh, rcnt, shv, t,
                      [&](int64_t i, const mp<K> &ti, bool first, mp<K> &a, mp<K> &c) {
                        mp<K> t1 = mul<K>(ti, ldk<K>(sv, i)), t2 = mul<K>(ti, ti);
                        a = first ? t1 : add<K>(a, t1);
                        c = first ? t2 : add<K>(c, t2);
                      }))
      return false;
    if (tid == 0) {
      mp<K> tt = shk<K>(sh.d[1]);
      sh.flag = is_zero<K>(tt) ? 1 : 0;
      if (!sh.flag) setk<K>(sh.omega, div<K>(shk<K>(sh.d[0]), tt));
    }
    __syncthreads();
    if (sh.flag) {
      status = MPK_BREAKDOWN;
      break;
    }
    // x = (x + alpha p^) + omega s^; r = s - omega t; ||r||^2, <r~, r>
    {
      const mp<K> al = shk<K>(sh.alpha), om = shk<K>(sh.omega);
      if (!brows_dot<K>(S, tm, sh, rcnt, [&](int64_t i, bool first, mp<K> &a, mp<K> &c) {
            mp<K> xi = add<K>(ldk<K>(xw, i), mul<K>(al, ldk<K>(ph, i)));
            stk<K>(xw, i, add<K>(xi, mul<K>(om, ldk<K>(shv, i))));
            mp<K> ri = sub<K>(ldk<K>(sv, i), mul<K>(om, ldk<K>(t, i)));
            stk<K>(r, i, ri);
            mp<K> t1 = mul<K>(ri, ri), t2 = mul<K>(ldk<K>(rt, i), ri);
            a = first ? t1 : add<K>(a, t1);
            c = first ? t2 : add<K>(c, t2);
          }))
        return false;
    }
    const double nr2 = sh.d[0][0];
    mp<K> rho_new = shk<K>(sh.d[1]);
    __syncthreads();
    if (tid == 0) sh.nr2 = nr2;
    if (bstop(nr2, sh.nr0sq, er, ea)) {
      if (!bresidual<K>(S, tm, sh, rcnt, xw, nullptr, nullptr)) return false;
      true_nr2 = sh.d[0][0];
      if (bstop(true_nr2, sh.nr0sq, er, ea)) {
        status = MPK_OK;
        break;
      }
    }
    if (is_zero<K>(shk<K>(sh.omega))) {
      status = MPK_BREAKDOWN;
      break;
    }
    if (it < max_iter && is_zero<K>(rho_new)) {
      status = MPK_BREAKDOWN;
      ++it;
      break;
    }
    __syncthreads();
    if (tid == 0) {
      mp<K> q1 = div<K>(rho_new, shk<K>(sh.rho));
      mp<K> q2 = div<K>(shk<K>(sh.alpha), shk<K>(sh.omega));
      setk<K>(sh.beta, mul<K>(q1, q2));
      setk<K>(sh.rho, rho_new);
    }
    __syncthreads();
  }
  __syncthreads();
  if (copy_x)
    for (int64_t i = gt; i < n * K; i += GS) S.x[i] = xw[i];
  if (lead) {
    o.iters = it;
    o.status = status;
    o.relres_recursive = sh.nr0sq > 0 ? sqrt(sh.nr2 / sh.nr0sq) : sqrt(sh.nr2);
    o.relres_true = true_nr2 < 0 ? -1.0 : (sh.nbsq > 0 ? sqrt(true_nr2 / sh.nbsq) : sqrt(true_nr2));
    out[sid] = o;
  }
  __syncthreads();
  return true;
}

#undef TSYNC

template <int K, int KF>
__global__ __launch_bounds__(BLOCK) void batched_bicgstab(
    const BSys *__restrict__ sys, BCtl *ctl, const int32_t *__restrict__ team,
    const BEnt *__restrict__ ent, const int32_t *__restrict__ qstart, int32_t *qticket,
    const int32_t *__restrict__ qmap, BOut *out, double er, double ea, int64_t max_iter,
    int copy_x, int32_t *abort) {
  __shared__ BShared<K> sh;
  __shared__ int32_t lcols[BLOCK * RCACHE];
  const int tid = threadIdx.x;
  const int32_t q = qmap[xcc_id()];
  if (q < 0) return;  // no queue for this XCD (not planned for)
  const int32_t q0 = qstart[q], qlen = qstart[q + 1] - q0;
  for (;;) {
    if (tid == 0) {
      const int32_t tk = atomicAdd(&qticket[q * QSTRIDE], 1);
      sh.sys = -1;
      if (tk < qlen && !ld_agent_i(abort)) {
        const BEnt e = ent[q0 + tk];
        sh.sys = e.sys;
        sh.member = e.member;
      }
    }
    __syncthreads();
    const int32_t sid = sh.sys, mem = sh.member;
    __syncthreads();
    if (sid < 0) break;
    const BSys S = sys[sid];
    Team tm{ctl + sid, team[sid], mem, 0, abort};
    if (!run_job<K, KF>(S, tm, sh, lcols, out, sid, er, ea, max_iter, copy_x)) return;
  }
}

// Job control words, queue tickets and the watchdog word; every report
// starts as MPK_EWATCHDOG, so a job the launch never ran is reported.
static __global__ void bctl_init(int32_t nsys, BCtl *ctl, BOut *out, int32_t *qticket,
                                 int32_t *abort) {
  const int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (i < nsys) {
    BCtl c{};
    c.bad = INT_MAX;
    c.pivbad = INT_MAX;
    ctl[i] = c;
    BOut o{};
    o.bad_row = -1;
    o.status = MPK_EWATCHDOG;
    o.relres_recursive = o.relres_true = -1.0;
    out[i] = o;
  }
  if (i < NQ * QSTRIDE) qticket[i] = 0;
  if (i < 16) abort[i] = 0;
}

static __global__ void xcc_probe(int32_t *out) {
  if (threadIdx.x == 0) out[blockIdx.x] = xcc_id();
}

// ------------------------------------------------------------- host side
constexpr unsigned PROBE_MAX = 4096;  // largest grid

struct BLayout {
  BSys *sys = nullptr;
  BOut *out = nullptr;
  BCtl *ctl = nullptr;
  int32_t *team = nullptr;
  BEnt *ent = nullptr;
  int32_t *qstart = nullptr, *qticket = nullptr, *qmap = nullptr, *abort = nullptr;
  int32_t *probe = nullptr;
};

// Workspace: descriptors, results, job control, queues, then per-system
// arrays.
static size_t blayout(int32_t nsys, const int64_t *ns, const int64_t *nnzs, int K, int KF, Bump &b,
                      BLayout *L, std::vector<BSys> *hs) {
  BLayout tmp;
  BLayout &l = L ? *L : tmp;
  l.sys = b.take<BSys>(size_t(nsys));
  l.out = b.take<BOut>(size_t(nsys));
  l.ctl = b.take<BCtl>(size_t(nsys));
  l.team = b.take<int32_t>(size_t(nsys));
  l.ent = b.take<BEnt>(size_t(nsys) * TMAX);
  l.qstart = b.take<int32_t>(NQ + 1);
  l.qticket = b.take<int32_t>(NQ * QSTRIDE);
  l.qmap = b.take<int32_t>(NQ);
  l.abort = b.take<int32_t>(16);
  l.probe = b.take<int32_t>(PROBE_MAX);
  for (int32_t q = 0; q < nsys; ++q) {
    BSys s{};
    const int64_t n = ns[q], nnz = nnzs[q];
    s.f = KF ? b.take<double>(size_t(nnz) * KF) : nullptr;
    s.diag = b.take<int32_t>(size_t(n));
    s.lvl = b.take<int32_t>(size_t(n));
    s.ordL = b.take<int32_t>(size_t(n));
    s.ordU = b.take<int32_t>(size_t(n));
    s.lptL = b.take<int32_t>(size_t(n) + 2);
    s.lptU = b.take<int32_t>(size_t(n) + 2);
    s.cur = b.take<int32_t>(size_t(n) + 2);
    s.vec = b.take<double>(size_t(NBV) * n * K);
    s.part = b.take<double>(size_t(ntiles(n)) * 2 * 2 * K);
    s.n = n;
    s.nnz = nnz;
    if (hs) hs->push_back(s);
  }
  return b.off;
}

// A schedule: the persistent grid size, the order jobs are considered in
// (largest nnz first, or as given) and the rows per team member
// (team_rows = 0: one workgroup per system).  None changes the arithmetic.
struct BSched {
  unsigned grid;
  bool lpt;
  int64_t team_rows;
};

static bool parse_sched(const char *str, BSched &sc) {
  // "grid=<n>,order=lpt|given[,team=<rows per member>]"
  std::string s(str);
  size_t g = s.find("grid="), o = s.find("order="), t = s.find("team=");
  if (g == std::string::npos || o == std::string::npos) return false;
  sc.grid = unsigned(atoi(s.c_str() + g + 5));
  sc.lpt = s.compare(o + 6, 3, "lpt") == 0;
  sc.team_rows = t == std::string::npos ? 0 : atoll(s.c_str() + t + 5);
  return sc.grid > 0 && sc.team_rows >= 0;
}

static std::map<std::string, BSched> &tune_cache() {
  static std::map<std::string, BSched> m;
  return m;
}

template <int K, int KF> static const void *bkernel() {
  return reinterpret_cast<const void *>(&batched_bicgstab<K, KF>);
}

static const void *bkernel_of(int K, int KF) {
#define MPK_BK(k, kf) \
  if (K == k && KF == kf) return bkernel<k, kf>()
  MPK_BK(1, 0); MPK_BK(1, 1); MPK_BK(2, 0); MPK_BK(2, 1); MPK_BK(2, 2);
  MPK_BK(3, 0); MPK_BK(3, 1); MPK_BK(3, 2); MPK_BK(4, 0); MPK_BK(4, 1); MPK_BK(4, 2);
#undef MPK_BK
  return nullptr;
}

// The XCD of every workgroup of a cooperative grid of this size (probed
// once per device and size with the solver's launch path).  Only the plan
// relies on it: a workgroup always serves the queue of the XCD it runs on.
static int xcc_map(const BLayout &L, unsigned grid, hipStream_t s, std::vector<int32_t> &xcc) {
  static std::map<std::pair<int, unsigned>, std::vector<int32_t>> cache;
  int dev = 0;
  MPK_HIP(hipGetDevice(&dev));
  auto key = std::make_pair(dev, grid);
  auto it = cache.find(key);
  if (it != cache.end()) {
    xcc = it->second;
    return MPK_OK;
  }
  int32_t *a0 = L.probe;
  void *args[] = {&a0};
  MPK_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&xcc_probe), dim3(grid),
                                     dim3(BLOCK), args, 0, s));
  xcc.assign(grid, 0);
  MPK_HIP(hipMemcpyAsync(xcc.data(), L.probe, sizeof(int32_t) * grid, hipMemcpyDeviceToHost, s));
  MPK_HIP(hipStreamSynchronize(s));
  cache[key] = xcc;
  return MPK_OK;
}

// Jobs to queues: one queue per XCD that the grid reaches; team sizes from
// team_rows (at most the workgroups of the smallest queue, so every team
// can meet); each job, in the schedule's order, to the queue with the least
// work so far (stored entries per workgroup); T tickets per job.
struct BPlan {
  std::vector<int32_t> team, qstart, qmap;
  std::vector<BEnt> ent;
};

static void plan_queues(int32_t nsys, const int64_t *ns, const int64_t *nz, const BSched &sc,
                        const std::vector<int32_t> &xcc, const std::vector<int32_t> *only,
                        BPlan &P) {
  if (only) {
    // one queue that every XCD serves, one workgroup per job
    P.qmap.assign(NQ, 0);
    P.team.assign(size_t(nsys), 1);
    P.ent.clear();
    for (int32_t j : *only) P.ent.push_back(BEnt{j, 0});
    P.qstart.assign(NQ + 1, int32_t(P.ent.size()));
    P.qstart[0] = 0;
    return;
  }
  int cnt[NQ] = {0};
  for (int32_t x : xcc) cnt[x & (NQ - 1)]++;
  P.qmap.assign(NQ, -1);
  std::vector<int> W;
  for (int x = 0; x < NQ; ++x)
    if (cnt[x]) {
      P.qmap[x] = int32_t(W.size());
      W.push_back(cnt[x]);
    }
  const int nq = int(W.size());
  const int tcap = std::min(*std::min_element(W.begin(), W.end()), TMAX);
  P.team.assign(size_t(nsys), 1);
  if (sc.team_rows > 0)
    for (int32_t q = 0; q < nsys; ++q)
      P.team[q] = int32_t(std::max<int64_t>(
          1, std::min<int64_t>(tcap, (ns[q] + sc.team_rows - 1) / sc.team_rows)));
  std::vector<int32_t> order(static_cast<size_t>(nsys));
  for (int32_t q = 0; q < nsys; ++q) order[q] = q;
  if (sc.lpt)
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return nz[a] > nz[c]; });
  std::vector<std::vector<int32_t>> qjobs(static_cast<size_t>(nq));
  std::vector<double> load(static_cast<size_t>(nq), 0.0);
  for (int32_t j : order) {
    int best = 0;
    for (int q = 1; q < nq; ++q)
      if (load[q] < load[best]) best = q;
    qjobs[best].push_back(j);
    load[best] += double(nz[j]) / W[best];
  }
  P.ent.clear();
  P.qstart.assign(NQ + 1, 0);
  for (int q = 0; q < nq; ++q) {
    P.qstart[q] = int32_t(P.ent.size());
    for (int32_t j : qjobs[q])
      for (int32_t m = 0; m < P.team[j]; ++m) P.ent.push_back(BEnt{j, m});
  }
  for (int q = nq; q <= NQ; ++q) P.qstart[q] = int32_t(P.ent.size());
}

// Workgroups of the kernel that fit on the device at once (the launch is
// cooperative: every workgroup is resident, so team members can wait for
// one another).
static int bresident(int K, int KF, unsigned *per_cu, unsigned *cus) {
  int dev = 0, nb = 0;
  MPK_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  MPK_HIP(hipGetDeviceProperties(&prop, dev));
  MPK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, bkernel_of(K, KF), BLOCK, 0));
  *per_cu = unsigned(std::max(nb, 1));
  *cus = unsigned(prop.multiProcessorCount);
  return MPK_OK;
}

// One launch for the jobs of the schedule (only != nullptr: just these
// jobs, one workgroup each, from one queue).  Asynchronous; the reports
// start as MPK_EWATCHDOG until a job ends.
static int run_batched(int K, int KF, const BLayout &L, int32_t nsys, const int64_t *ns,
                       const int64_t *nz, BSched sc, const std::vector<int32_t> *only, double er,
                       double ea, int64_t max_iter, int copy_x, hipStream_t s) {
  unsigned per_cu = 1, cus = 1;
  int st = bresident(K, KF, &per_cu, &cus);
  if (st) return st;
  sc.grid = std::min({sc.grid, per_cu * cus, PROBE_MAX});
  if (sc.team_rows == 0 || only)
    sc.grid = std::min<unsigned>(sc.grid, unsigned(only ? only->size() : size_t(nsys)));
  std::vector<int32_t> xcc;
  if (!only && (st = xcc_map(L, sc.grid, s, xcc))) return st;
  BPlan P;
  plan_queues(nsys, ns, nz, sc, xcc, only, P);
  MPK_HIP(hipMemcpyAsync(L.team, P.team.data(), sizeof(int32_t) * P.team.size(),
                         hipMemcpyHostToDevice, s));
  MPK_HIP(hipMemcpyAsync(L.ent, P.ent.data(), sizeof(BEnt) * P.ent.size(), hipMemcpyHostToDevice,
                         s));
  MPK_HIP(hipMemcpyAsync(L.qstart, P.qstart.data(), sizeof(int32_t) * P.qstart.size(),
                         hipMemcpyHostToDevice, s));
  MPK_HIP(hipMemcpyAsync(L.qmap, P.qmap.data(), sizeof(int32_t) * P.qmap.size(),
                         hipMemcpyHostToDevice, s));
  const unsigned ig = unsigned((std::max<int64_t>(nsys, NQ * QSTRIDE) + BLOCK - 1) / BLOCK);
  hipLaunchKernelGGL(bctl_init, dim3(ig), dim3(BLOCK), 0, s, nsys, L.ctl, L.out, L.qticket,
                     L.abort);
  MPK_HIP(hipGetLastError());
  MPK_HIP(hipStreamSynchronize(s));  // the plan's host buffers are released on return
  const BSys *a0 = L.sys;
  BCtl *a1 = L.ctl;
  const int32_t *a2 = L.team;
  const BEnt *a3 = L.ent;
  const int32_t *a4 = L.qstart;
  int32_t *a5 = L.qticket;
  const int32_t *a6 = L.qmap;
  BOut *a7 = L.out;
  double a8 = er, a9 = ea;
  int64_t a10 = max_iter;
  int a11 = copy_x;
  int32_t *a12 = L.abort;
  void *args[] = {&a0, &a1, &a2, &a3, &a4, &a5, &a6, &a7, &a8, &a9, &a10, &a11, &a12};
  MPK_HIP(hipLaunchCooperativeKernel(bkernel_of(K, KF), dim3(sc.grid), dim3(BLOCK), args, 0, s));
  return MPK_OK;
}

// The reports of the last launch (after the stream has drained) and the
// jobs it did not finish (never reached, or left when a team waited past
// its bound).
static int breports(const BLayout &L, int32_t nsys, hipStream_t s, std::vector<BOut> &outs,
                    std::vector<int32_t> &unfinished) {
  outs.resize(static_cast<size_t>(nsys));
  MPK_HIP(hipMemcpyAsync(outs.data(), L.out, sizeof(BOut) * nsys, hipMemcpyDeviceToHost, s));
  MPK_HIP(hipStreamSynchronize(s));
  unfinished.clear();
  for (int32_t q = 0; q < nsys; ++q)
    if (outs[q].status == MPK_EWATCHDOG) unfinished.push_back(q);
  return MPK_OK;
}

}  // namespace mpk

using namespace mpk;

extern "C" {

size_t mpk_krylov_batched_workspace_bytes(mpk_method m, mpk_prec vp, mpk_prec fp, int32_t nsys,
                                          const mpk_csr *A) {
  if (m != MPK_BICGSTAB || vp < MPK_D || vp > MPK_QD || !(fp == 0 || fp == MPK_D || fp == MPK_DD) ||
      int(fp) > int(vp) || nsys <= 0 || !A)
    return 0;
  std::vector<int64_t> ns(static_cast<size_t>(nsys)), nz(static_cast<size_t>(nsys));
  for (int32_t q = 0; q < nsys; ++q) {
    if (A[q].n <= 0 || A[q].nnz < 0) return 0;
    ns[q] = A[q].n;
    nz[q] = A[q].nnz;
  }
  Bump b(nullptr);
  return blayout(nsys, ns.data(), nz.data(), int(vp), int(fp), b, nullptr, nullptr);
}

int mpk_dkrylov_solve_batched(mpk_method m, mpk_prec vp, mpk_prec fp, double tol_rel,
                              double tol_abs, int64_t max_iter, int32_t nsys, const mpk_csr *A,
                              const double *const *b, double *const *x, void *ws, size_t ws_bytes,
                              mpk_info *info, const char *schedule, void *stream) {
  if (m != MPK_BICGSTAB) return MPK_EUNSUPPORTED;
  if (vp < MPK_D || vp > MPK_QD || !(fp == 0 || fp == MPK_D || fp == MPK_DD) ||
      int(fp) > int(vp) || nsys <= 0 || !A || !b || !x || !(tol_rel >= 0) || !(tol_abs >= 0) ||
      max_iter < 0)
    return MPK_EINVAL;
  for (int32_t q = 0; q < nsys; ++q)
    if (validate_csr_args(&A[q]) || !b[q] || !x[q]) return MPK_EINVAL;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) ||
      ws_bytes < mpk_krylov_batched_workspace_bytes(m, vp, fp, nsys, A))
    return MPK_EWORKSPACE;
  BSched sc{0, true, 0};
  if (schedule && !parse_sched(schedule, sc)) return MPK_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const double t0 = now_ms();
  const int K = int(vp), KF = int(fp);
  std::vector<int64_t> ns(static_cast<size_t>(nsys)), nz(static_cast<size_t>(nsys));
  for (int32_t q = 0; q < nsys; ++q) {
    ns[q] = A[q].n;
    nz[q] = A[q].nnz;
  }
  Bump bump(ws);
  BLayout L;
  std::vector<BSys> hs;
  blayout(nsys, ns.data(), nz.data(), K, KF, bump, &L, &hs);
  for (int32_t q = 0; q < nsys; ++q) {
    hs[q].rp = A[q].row_ptr;
    hs[q].ci = A[q].col_idx;
    hs[q].val = A[q].val;
    hs[q].b = b[q];
    hs[q].x = x[q];
  }
  MPK_HIP(hipMemcpyAsync(L.sys, hs.data(), sizeof(BSys) * nsys, hipMemcpyHostToDevice, s));
  int st = MPK_OK;
  std::vector<BOut> outs;
  std::vector<int32_t> unfinished;
  if (!schedule) {
    // autotune on the first call for this batch shape: a few passes of each
    // candidate (x untouched), fastest kept
    char key[96];
    int64_t tot = 0;
    for (auto v : nz) tot += v;
    snprintf(key, sizeof key, "%d/%lld/%d/%d", nsys, (long long)(tot >> 16), K, KF);
    auto it = tune_cache().find(key);
    if (it != tune_cache().end()) {
      sc = it->second;
    } else {
      unsigned per_cu = 1, cus = 1;
      if ((st = bresident(K, KF, &per_cu, &cus))) return st;
      std::vector<BSched> cand;
      for (unsigned g = 1; g <= std::min(per_cu, 2u); ++g)
        for (int64_t tr : {int64_t(0), int64_t(32768), int64_t(16384), int64_t(8192)})
          cand.push_back(BSched{g * cus, true, tr});
      double best = 1e300;
      sc = cand[0];
      for (const BSched &c : cand) {
        const double a = now_ms();
        if ((st = run_batched(K, KF, L, nsys, ns.data(), nz.data(), c, nullptr, tol_rel, tol_abs,
                              std::min<int64_t>(max_iter, 3), 0, s)))
          return st;
        if ((st = breports(L, nsys, s, outs, unfinished))) return st;
        const double tm = now_ms() - a;
        if (unfinished.empty() && tm < best) {
          best = tm;
          sc = c;
        }
      }
      tune_cache()[key] = sc;
    }
  }
  const double t1 = now_ms();
  if ((st = run_batched(K, KF, L, nsys, ns.data(), nz.data(), sc, nullptr, tol_rel, tol_abs,
                        max_iter, 1, s)))
    return st;
  if ((st = breports(L, nsys, s, outs, unfinished))) return st;
  if (!unfinished.empty()) {
    // jobs a team could not finish (a queue got fewer workgroups than
    // planned) run again, one workgroup each; their x is written only when
    // a job ends, so they restart from the caller's x
    const std::vector<int32_t> redo = unfinished;
    std::vector<BOut> outs2;
    if ((st = run_batched(K, KF, L, nsys, ns.data(), nz.data(), sc, &redo, tol_rel, tol_abs,
                          max_iter, 1, s)))
      return st;
    if ((st = breports(L, nsys, s, outs2, unfinished))) return st;
    for (int32_t q : redo) {
      if (outs2[q].status == MPK_EWATCHDOG) return MPK_EWATCHDOG;
      outs[q] = outs2[q];
    }
  }
  const double t2 = now_ms();
  int worst = MPK_OK;
  for (int32_t q = 0; q < nsys; ++q) {
    if (info) {
      info[q].iters = outs[q].iters;
      info[q].bad_row = outs[q].bad_row;
      info[q].status = outs[q].status;
      info[q].relres_recursive = outs[q].relres_recursive;
      info[q].relres_true = outs[q].relres_true;
      info[q].setup_ms = t1 - t0;
      info[q].solve_ms = t2 - t1;
    }
    if (outs[q].status < 0 && (worst >= 0 || outs[q].status < worst)) worst = outs[q].status;
    if (outs[q].status > 0 && worst == MPK_OK) worst = outs[q].status;
  }
  return worst;
}

}  // extern "C"
