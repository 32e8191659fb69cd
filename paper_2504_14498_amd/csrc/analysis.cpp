// analysis.cpp -- host-side checks of a CSR pattern and the dependency
// schedules (level sets) of the ILU(0) factorisation and substitutions.
//
// Level sets: in the forward substitution of Algorithm 2 row i needs every
// y_j with a stored l_ij (j < i), so lvl(i) = 1 + max lvl(j) over those j
// (0 if none); rows of one level are independent.  The backward
// substitution mirrors this over the stored u_ij (j > i), and the M^H
// solve uses the columns of U and L instead of their rows.  The schedules
// only decide which rows run together; each row's own arithmetic keeps the
// ascending column order of Algorithm 2.
#include <algorithm>
#include <cstdlib>
#include <map>
#include <thread>

#include "internal.hpp"

namespace mpk {

// The pattern is copied into a page-locked buffer of the calling thread,
// kept (and grown when needed) across calls: device-to-host copies into
// pageable memory go through a staging copy and run several times slower.
namespace {
struct PinnedStage {
  int32_t *p = nullptr;
  size_t cap = 0;  // int32 words
};
thread_local PinnedStage pinned_stage;
}  // namespace

int fetch_pattern(const mpk_csr *A, HostCsr &h, hipStream_t s) {
  h.n = A->n;
  h.nnz = A->nnz;
  const size_t need = size_t(A->n) + 1 + size_t(std::max<int64_t>(A->nnz, 1));
  PinnedStage &st = pinned_stage;
  if (st.cap < need) {
    if (st.p) (void)hipHostFree(st.p);
    st.p = nullptr;
    st.cap = 0;
    void *q = nullptr;
    if (hipHostMalloc(&q, sizeof(int32_t) * need, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      // no page-locked memory: fall back to the thread's own arrays
      h.own_rp.resize(size_t(A->n) + 1);
      h.own_ci.resize(size_t(std::max<int64_t>(A->nnz, 1)));
      h.own();
      MPK_HIP(hipMemcpyAsync(h.own_rp.data(), A->row_ptr, sizeof(int32_t) * (A->n + 1),
                             hipMemcpyDeviceToHost, s));
      if (A->nnz > 0)
        MPK_HIP(hipMemcpyAsync(h.own_ci.data(), A->col_idx, sizeof(int32_t) * A->nnz,
                               hipMemcpyDeviceToHost, s));
      MPK_HIP(hipStreamSynchronize(s));
      return MPK_OK;
    }
    st.p = static_cast<int32_t *>(q);
    st.cap = need;
  }
  int32_t *rp = st.p, *ci = st.p + (size_t(A->n) + 1);
  MPK_HIP(hipMemcpyAsync(rp, A->row_ptr, sizeof(int32_t) * (A->n + 1), hipMemcpyDeviceToHost, s));
  if (A->nnz > 0)
    MPK_HIP(hipMemcpyAsync(ci, A->col_idx, sizeof(int32_t) * A->nnz, hipMemcpyDeviceToHost, s));
  MPK_HIP(hipStreamSynchronize(s));
  h.rp = rp;
  h.ci = ci;
  return MPK_OK;
}

int check_pattern(const HostCsr &h, int64_t *bad_row) {
  *bad_row = -1;
  if (h.rp[0] != 0 || h.rp[h.n] != h.nnz) return MPK_EPATTERN;
  // rows in up to 8 contiguous chunks on host threads; the first chunk
  // (in row order) that finds a bad row reports the lowest one
  const int T = int(std::min<int64_t>(8, std::max<int64_t>(1, h.n / 65536)));
  std::vector<int64_t> bad(size_t(T), -1);
  std::vector<int> code(size_t(T), MPK_OK);
  auto work = [&](int t) {
    const int64_t i0 = h.n * t / T, i1 = h.n * (t + 1) / T;
    for (int64_t i = i0; i < i1; ++i) {
      const int32_t a = h.rp[i], b = h.rp[i + 1];
      if (b < a || a < 0 || b > h.nnz) {
        bad[t] = i;
        code[t] = MPK_EPATTERN;
        return;
      }
      bool diag = false;
      for (int32_t p = a; p < b; ++p) {
        const int32_t j = h.ci[p];
        if (j < 0 || j >= h.n || (p > a && j <= h.ci[p - 1])) {
          bad[t] = i;
          code[t] = MPK_EPATTERN;
          return;
        }
        diag |= (j == i);
      }
      if (!diag) {
        bad[t] = i;
        code[t] = MPK_ENO_DIAG;
        return;
      }
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < T; ++t) th.emplace_back(work, t);
  work(0);
  for (auto &x : th) x.join();
  for (int t = 0; t < T; ++t)
    if (bad[t] >= 0) {
      *bad_row = bad[t];
      return code[t];
    }
  return MPK_OK;
}

void host_diag(const HostCsr &h, std::vector<int32_t> &diag) {
  diag.assign(size_t(h.n), -1);
  for (int64_t i = 0; i < h.n; ++i)
    for (int32_t p = h.rp[i]; p < h.rp[i + 1]; ++p)
      if (h.ci[p] == i) diag[i] = p;
}

void host_transpose(const HostCsr &h, IVec &trp, IVec &tci, IVec &tsrc) {
  const int64_t n = h.n, nnz = h.nnz;
  trp.assign(size_t(n) + 1, 0);
  tci.resize(size_t(std::max<int64_t>(nnz, 1)));
  tsrc.resize(size_t(std::max<int64_t>(nnz, 1)));
  for (int64_t p = 0; p < nnz; ++p) trp[h.ci[p] + 1]++;
  for (int64_t i = 0; i < n; ++i) trp[i + 1] += trp[i];
  std::vector<int32_t> next(trp.begin(), trp.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t p = h.rp[i]; p < h.rp[i + 1]; ++p) {
      int32_t q = next[h.ci[p]]++;
      tci[q] = int32_t(i);
      tsrc[q] = p;
    }
}

// Greedy colouring of the graph of A + A^T in natural order: rows i != j
// are adjacent when a_ij or a_ji is stored, and row i = 0, 1, ... takes
// the smallest colour that no adjacent row j < i has.  Its neighbours
// below i come from the lower part of row i and from the rows j < i that
// store column i (the lower part of row i of A^T).  Returns the number of
// colours.
int32_t greedy_color(const HostCsr &h, IVec &color) {
  const int64_t n = h.n, nnz = h.nnz;
  // A structurally symmetric pattern (every stored a_ij has a stored a_ji,
  // checked on up to 8 host threads) needs only its lower part: row i's
  // neighbours below i are its columns below i.
  bool sym = true;
  {
    const int T = int(std::min<int64_t>(8, std::max<int64_t>(1, n / 65536)));
    std::vector<char> ok(size_t(T), 1);
    auto work = [&](int t) {
      const int64_t i0 = n * t / T, i1 = n * (t + 1) / T;
      for (int64_t i = i0; i < i1 && ok[t]; ++i)
        for (int32_t p = h.rp[i + 1] - 1; p >= h.rp[i] && h.ci[p] > i; --p) {
          const int32_t j = h.ci[p];
          if (!std::binary_search(h.ci + h.rp[j], h.ci + h.rp[j + 1], int32_t(i))) {
            ok[t] = 0;
            break;
          }
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < T; ++t) th.emplace_back(work, t);
    work(0);
    for (auto &x : th) x.join();
    for (int t = 0; t < T; ++t) sym = sym && ok[t];
  }
  // otherwise the lower part of A^T as well: row c lists the rows j < c
  // that store column c (their upper entries), ascending j
  IVec trp(size_t(n) + 1, 0), tci(size_t(std::max<int64_t>(sym ? 1 : nnz, 1)));
  if (!sym) {
    for (int64_t j = 0; j < n; ++j)
      for (int32_t p = h.rp[j + 1] - 1; p >= h.rp[j] && h.ci[p] > j; --p) trp[h.ci[p] + 1]++;
    for (int64_t i = 0; i < n; ++i) trp[i + 1] += trp[i];
    IVec next(trp.begin(), trp.end() - 1);
    for (int64_t j = 0; j < n; ++j)
      for (int32_t p = h.rp[j]; p < h.rp[j + 1]; ++p)
        if (h.ci[p] > j) tci[next[h.ci[p]]++] = int32_t(j);
  }
  color.resize(size_t(n));  // each entry is written before it is read
  // the colours of row i's neighbours below i: a bit mask while they are
  // below 64, else seen[c] == i marks colour c as taken
  IVec seen;
  int32_t ncol = 0;
  for (int64_t i = 0; i < n; ++i) {
    uint64_t mask = 0;
    auto take = [&](int32_t c) {
      if (c < 64) mask |= uint64_t(1) << c;
    };
    for (int32_t p = h.rp[i]; p < h.rp[i + 1] && h.ci[p] < i; ++p) take(color[h.ci[p]]);
    for (int32_t p = trp[i]; p < trp[i + 1]; ++p) take(color[tci[p]]);
    int32_t c;
    if (~mask != 0) {
      c = __builtin_ctzll(~mask);  // smallest colour not taken (below 64)
    } else {
      if (seen.empty()) seen.assign(size_t(n) + 2, -1);
      const int32_t me = int32_t(i);
      for (int32_t p = h.rp[i]; p < h.rp[i + 1] && h.ci[p] < i; ++p) seen[color[h.ci[p]]] = me;
      for (int32_t p = trp[i]; p < trp[i + 1]; ++p) seen[color[tci[p]]] = me;
      c = 64;
      while (seen[c] == me) ++c;
    }
    color[i] = c;
    ncol = std::max(ncol, c + 1);
  }
  return ncol;
}

bool grid_dims_from_last_row(int64_t n, const int32_t *cols, int64_t len, int32_t &nx,
                             int32_t &ny, int32_t &nz) {
  if (n < 4) return false;
  // strides of the last row's lower neighbours: 1, nx (2D) and nx ny (3D)
  std::vector<int64_t> d;
  for (int64_t k = 0; k < len && cols[k] < n - 1; ++k) d.push_back(n - 1 - cols[k]);
  std::sort(d.begin(), d.end());
  if (d.empty() || d[0] != 1) return false;
  int64_t gx, gy, gz;
  if (d.size() == 2) {
    gx = d[1];
    if (gx < 2 || n % gx) return false;
    gy = n / gx;
    gz = 1;
  } else if (d.size() == 3) {
    gx = d[1];
    const int64_t pl = d[2];
    if (gx < 2 || pl % gx || n % pl) return false;
    gy = pl / gx;
    gz = n / pl;
    if (gz < 2) return false;
  } else {
    return false;
  }
  if (gy < 2) return false;
  nx = int32_t(gx);
  ny = int32_t(gy);
  nz = int32_t(gz);
  return true;
}

bool detect_grid(const HostCsr &h, int32_t &nx, int32_t &ny, int32_t &nz) {
  const int64_t n = h.n;
  if (n < 4) return false;
  // the pattern may not have been checked: every read below stays inside
  // [0, nnz) (a row is read only when its bounds lie there)
  if (h.rp[0] != 0 || h.rp[n] != h.nnz || h.rp[n - 1] < 0 || h.rp[n - 1] > h.rp[n]) return false;
  int32_t ex, ey, ez;
  if (!grid_dims_from_last_row(n, h.ci + h.rp[n - 1], h.rp[n] - h.rp[n - 1], ex, ey, ez))
    return false;
  const int64_t gx = ex, gy = ey, gz = ez;
  const int64_t pl = gx * gy;
  // every row stores exactly its neighbours inside the grid (and its
  // diagonal), ascending; checked on up to 8 host threads
  const int T = int(std::min<int64_t>(8, std::max<int64_t>(1, n / 65536)));
  std::vector<char> ok(size_t(T), 1);
  auto work = [&](int t) {
    const int64_t i0 = n * t / T, i1 = n * (t + 1) / T;
    int64_t x = i0 % gx, y = (i0 / gx) % gy, z = i0 / pl;  // advanced row by row below
    for (int64_t i = i0; i < i1; ++i) {
      int64_t want[7];
      int m = 0;
      if (z > 0) want[m++] = i - pl;
      if (y > 0) want[m++] = i - gx;
      if (x > 0) want[m++] = i - 1;
      want[m++] = i;
      if (x < gx - 1) want[m++] = i + 1;
      if (y < gy - 1) want[m++] = i + gx;
      if (z < gz - 1) want[m++] = i + pl;
      if (h.rp[i] < 0 || h.rp[i + 1] > h.nnz || h.rp[i + 1] - h.rp[i] != m) {
        ok[t] = 0;
        return;
      }
      for (int k = 0; k < m; ++k)
        if (h.ci[h.rp[i] + k] != want[k]) {
          ok[t] = 0;
          return;
        }
      if (++x == gx) {
        x = 0;
        if (++y == gy) {
          y = 0;
          ++z;
        }
      }
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < T; ++t) th.emplace_back(work, t);
  work(0);
  for (auto &x : th) x.join();
  for (int t = 0; t < T; ++t)
    if (!ok[t]) return false;
  nx = int32_t(gx);
  ny = int32_t(gy);
  nz = int32_t(gz);
  return true;
}

void grid_levels(const GridDims &g, std::vector<int32_t> &levptr, std::vector<int32_t> &order) {
  const int64_t nx = g.nx, ny = g.ny, nz = g.nz, n = nx * ny * nz;
  const int32_t nlev = int32_t(nx + ny + nz - 2);
  // rows per level from the lines: line (y, z) holds levels y+z .. y+z+nx-1
  auto count = [&](int64_t z0, int64_t z1, std::vector<int64_t> &cnt) {
    std::vector<int64_t> diff(size_t(nlev) + 1, 0);
    for (int64_t z = z0; z < z1; ++z)
      for (int64_t y = 0; y < ny; ++y) {
        diff[size_t(y + z)] += 1;
        diff[size_t(y + z + nx)] -= 1;
      }
    cnt.assign(size_t(nlev), 0);
    int64_t run = 0;
    for (int32_t l = 0; l < nlev; ++l) cnt[l] = (run += diff[l]);
  };
  // z-slabs on up to 8 host threads: each fills its rows, level by level, at
  // the offsets left by the slabs before it (ascending row within a level)
  const int T = int(std::min<int64_t>(8, std::max<int64_t>(1, nz)));
  std::vector<std::vector<int64_t>> cnt(static_cast<size_t>(T));
  auto zb = [&](int t) { return nz * t / T; };
  {
    std::vector<std::thread> th;
    for (int t = 1; t < T; ++t) th.emplace_back([&, t] { count(zb(t), zb(t + 1), cnt[t]); });
    count(zb(0), zb(1), cnt[0]);
    for (auto &x : th) x.join();
  }
  levptr.assign(size_t(nlev) + 1, 0);
  for (int32_t l = 0; l < nlev; ++l) {
    int64_t s = 0;
    for (int t = 0; t < T; ++t) s += cnt[t][l];
    levptr[l + 1] = levptr[l] + int32_t(s);
  }
  order.resize(size_t(n));
  auto fill = [&](int t) {
    std::vector<int64_t> next(static_cast<size_t>(nlev));
    for (int32_t l = 0; l < nlev; ++l) {
      int64_t o = levptr[l];
      for (int u = 0; u < t; ++u) o += cnt[u][l];
      next[l] = o;
    }
    for (int64_t z = zb(t); z < zb(t + 1); ++z)
      for (int64_t y = 0; y < ny; ++y)
        for (int64_t x = 0; x < nx; ++x) order[size_t(next[size_t(x + y + z)]++)] =
            int32_t((z * ny + y) * nx + x);
  };
  std::vector<std::thread> th;
  for (int t = 1; t < T; ++t) th.emplace_back(fill, t);
  fill(0);
  for (auto &x : th) x.join();
}

void build_plan_grid(int64_t n, int kind, HostPlan &p) {
  GridDims &g = p.grid;
  const int by = g.nz > 1 ? 8 : 64, bz = 64 / by;
  p.grid_by = by;
  g.nby = (g.ny + by - 1) / by;
  g.nbz = (g.nz + bz - 1) / bz;
  p.nblk = g.nby * g.nbz;
  // rows that the next block in y or in z reads, in the sweep's (for U
  // mirrored) coordinates: the last line of a block in y or in z
  const int64_t pl = int64_t(g.nx) * g.ny;
  auto pub = [&](int64_t y, int64_t z) {
    return (y % by == by - 1 && y < g.ny - 1) || (z % bz == bz - 1 && z < g.nz - 1);
  };
  int64_t lines = 0;
  for (int64_t z = 0; z < g.nz; ++z)
    for (int64_t y = 0; y < g.ny; ++y) lines += pub(y, z);
  p.xlist.resize(size_t(lines * g.nx));  // sized once, then filled in place
  int32_t *o = p.xlist.data();
  for (int64_t z = 0; z < g.nz; ++z)
    for (int64_t y = 0; y < g.ny; ++y) {
      if (!pub(y, z)) continue;
      const int64_t s0 = z * pl + y * g.nx;
      if (kind == 1)
        for (int64_t x = 0; x < g.nx; ++x) *o++ = int32_t(n - 1 - (s0 + x));
      else
        for (int64_t x = 0; x < g.nx; ++x) *o++ = int32_t(s0 + x);
    }
}

// Rows per block of the blocked schedule: the block's results live in LDS,
// at most 128 KiB for quad-double (K = 4).
int default_block_rows(int C, int kmax) {
  const char *e = getenv("MPK_TRSV_BLOCK_ROWS");
  if (e) {
    int rows = 64;  // a power of two (block shapes are built with shifts)
    while (rows * 2 <= atoi(e)) rows *= 2;
    return rows;
  }
  // largest power of two with rows * C * kmax doubles within 128 KiB
  int rows = 64;
  while (int64_t(rows) * 2 * C * kmax * 8 <= 131072) rows *= 2;
  return rows;
}

// Dependency lists of the four sweeps, read straight from a CSR (rows of
// A for L and U, rows of A^T for U^H and L^H): row i depends on the stored
// columns j < i (forward kinds 0, 2) or j > i (backward kinds 1, 3).
struct DepView {
  const int32_t *rp, *ci;
  bool lower;
  // rows are sorted: the lower part is a prefix, the upper part a suffix
  template <class F> void each(int64_t i, F &&f) const {
    if (lower) {
      for (int32_t q = rp[i]; q < rp[i + 1] && ci[q] < i; ++q) f(ci[q]);
    } else {
      for (int32_t q = rp[i + 1] - 1; q >= rp[i] && ci[q] > i; --q) f(ci[q]);
    }
  }
};

// Block geometry of a blocked sweep with cap LDS slots per block: plain
// ranges of cap consecutive rows, or blocks t periods deep when most rows
// share a long dependency offset P (one plane of a grid numbered plane by
// plane).  A dependency chain through the whole matrix crosses about
// (periods / t - 1) + (chunks per period - 1) block boundaries, against
// n / cap - 1 for plain ranges, and each crossing is a value written by one
// workgroup and polled by another.  The deep shape with the fewest
// crossings is returned only if it cuts them by a third; the caller still
// checks that no dependency leads to a block processed later.
static BlockGeom plain_geom(int64_t n, int cap) {
  BlockGeom g;
  g.P = std::max<int64_t>(n, 1);
  g.w = cap;
  g.t = 1;
  g.nch = (g.P + cap - 1) / cap;
  return g;
}

static BlockGeom deep_geom(const DepView &dv, int64_t n, int cap) {
  const BlockGeom plain = plain_geom(n, cap);
  if (const char *e = getenv("MPK_TRSV_DEEP"))
    if (e[0] == '0') return plain;
  // dependency offsets over a window of rows in the middle of the matrix
  const int64_t W = std::min<int64_t>(n, 4096), i0 = (n - W) / 2;
  std::map<int64_t, int64_t> cnt;
  for (int64_t i = i0; i < i0 + W; ++i)
    dv.each(i, [&](int32_t j) { cnt[i > j ? i - j : j - i]++; });
  std::vector<int64_t> periods;
  for (auto it = cnt.rbegin(); it != cnt.rend() && periods.size() < 3; ++it)
    if (4 * it->second >= W && it->first >= 2 && it->first < n) periods.push_back(it->first);
  const int64_t base = (n + cap - 1) / cap - 1;
  int64_t best = -1;
  BlockGeom g = plain;
  for (const int64_t P : periods) {
    const int64_t nper = (n + P - 1) / P;
    for (int32_t t = 2; t <= cap && t <= nper; t *= 2) {
      const int32_t w = cap / t;
      if (w > P) continue;
      const int64_t nch = (P + w - 1) / w;
      const int64_t cost = ((nper + t - 1) / t - 1) + (nch - 1);
      if (3 * cost <= 2 * base && (best < 0 || cost < best)) {
        best = cost;
        g.P = P;
        g.w = w;
        g.t = t;
        g.nch = nch;
      }
    }
  }
  return g;
}

// Schedule of a sweep: blocked (mode 1) when at least half of the
// dependencies stay inside blocks of blk_rows consecutive rows, else the
// level schedule (mode 0, which build_plan_levels turns into mode 2, one
// launch per level, when the levels are few and wide).  One pass over the
// pattern on up to 8 host threads.
int plan_mode(const HostCsr &h, const HostCsr *ht, int kind, int blk_rows) {
  int mode = 0;
  if (blk_rows > 0) {
    const int64_t n = h.n;
    const HostCsr &g = (kind >= 2) ? *ht : h;
    const DepView dv{g.rp, g.ci, kind == 0 || kind == 2};
    int shift = 0;
    while ((int64_t(1) << shift) < blk_rows) ++shift;
    const int T = int(std::min<int64_t>(8, std::max<int64_t>(1, n / 65536)));
    std::vector<int64_t> internal(size_t(T), 0), total(size_t(T), 0);
    auto work = [&](int t) {
      const int64_t i0 = n * t / T, i1 = n * (t + 1) / T;
      int64_t in = 0, tot = 0;
      for (int64_t i = i0; i < i1; ++i) {
        const int64_t bi = i >> shift;
        dv.each(i, [&](int32_t j) {
          ++tot;
          in += (int64_t(j) >> shift) == bi;
        });
      }
      internal[t] = in;
      total[t] = tot;
    };
    std::vector<std::thread> th;
    for (int t = 1; t < T; ++t) th.emplace_back(work, t);
    work(0);
    for (auto &x : th) x.join();
    int64_t in = 0, tot = 0;
    for (int t = 0; t < T; ++t) in += internal[t], tot += total[t];
    mode = (tot > 0 && 2 * in >= tot) ? 1 : 0;
  }
  // MPK_TRSV_MODE: b = blocked, l = polling level schedule, s = one launch
  // per level (both level schedules start as mode 0 here)
  if (const char *e = getenv("MPK_TRSV_MODE"))
    mode = (e[0] == 'b') ? 1 : ((e[0] == 'l' || e[0] == 's') ? 0 : mode);
  if (blk_rows <= 0) mode = 0;  // blocked schedule not available
  return mode;
}

void build_plan_levels(const HostCsr &h, const HostCsr *ht, int kind, int blk_rows,
                       HostPlan &p) {
  // p.mode was set by plan_mode.  Global levels are needed by the level
  // schedule and, for the L sweep, by the factorisation; a blocked sweep
  // of U, U^H or L^H needs none.
  if ((p.mode == 1 || p.mode == 3) && kind != 0) {
    p.nlev = 0;
    return;
  }
  const int64_t n = h.n;
  const HostCsr &g = (kind >= 2) ? *ht : h;
  const DepView dv{g.rp, g.ci, kind == 0 || kind == 2};
  const bool forward = (kind == 0 || kind == 2);
  std::vector<int32_t> lvl(size_t(n), 0);
  int32_t nlev = n > 0 ? 1 : 0;
  for (int64_t t = 0; t < n; ++t) {
    const int64_t i = forward ? t : n - 1 - t;
    int32_t l = 0;
    dv.each(i, [&](int32_t j) { l = std::max(l, lvl[j] + 1); });
    lvl[i] = l;
    nlev = std::max(nlev, l + 1);
  }
  (void)blk_rows;
  p.nlev = nlev;
  auto counting_order = [&](std::vector<int32_t> &levptr, std::vector<int32_t> &order) {
    levptr.assign(size_t(nlev) + 1, 0);
    for (int64_t i = 0; i < n; ++i) levptr[lvl[i] + 1]++;
    for (int32_t l = 0; l < nlev; ++l) levptr[l + 1] += levptr[l];
    order.resize(size_t(std::max<int64_t>(n, 1)));
    std::vector<int32_t> next(levptr.begin(), levptr.end() - 1);
    for (int64_t i = 0; i < n; ++i) order[next[lvl[i]]++] = int32_t(i);
  };
  if (kind == 0) counting_order(p.glob_levptr, p.glob_order);
  if (p.mode == 0) {
    // few, wide levels (at least 16384 rows each on average, at most 64):
    // one launch per level (mode 2) instead of one polling launch
    const char *e = getenv("MPK_TRSV_MODE");
    const bool force = e && e[0] == 's', forbid = e && e[0] == 'l';
    if (force || (!forbid && nlev <= 64 && n >= int64_t(nlev) * 16384)) p.mode = 2;
  }
  if (p.mode == 0 || p.mode == 2) {
    counting_order(p.levptr, p.order);
    p.seg.clear();
    p.seg_level.clear();
    for (int32_t l = 0; l < nlev; ++l)
      for (int32_t s = p.levptr[l]; s < p.levptr[l + 1]; s += WAVE) {
        p.seg.push_back(s);
        p.seg_level.push_back(l);
      }
    p.seg.push_back(int32_t(n));
  }
}

void build_plan_blocks(const HostCsr &h, const HostCsr *ht, int kind, int blk_rows,
                       HostPlan &p) {
  if (p.mode != 1) return;
  const int64_t n = h.n;
  const HostCsr &g = (kind >= 2) ? *ht : h;
  const DepView dv{g.rp, g.ci, kind == 0 || kind == 2};
  const bool forward = (kind == 0 || kind == 2);
  // blocked schedule: blocks (plain row ranges or a few periods deep, see
  // deep_geom) taken in the sweep's direction, each ordered by its local
  // (block-internal) levels
  p.blk_rows = blk_rows;
  BlockGeom G = deep_geom(dv, n, blk_rows);
  int lw = 0, lt = 0;
  while ((1 << lw) < G.w) ++lw;
  while ((1 << lt) < G.t) ++lt;
  // block id and LDS slot of every row of a deep geometry (plain ranges
  // use the shifts directly), on up to 8 host threads
  IVec blk_of, slot_of;
  const int T8 = int(std::min<int64_t>(8, std::max<int64_t>(1, n / 65536)));
  auto par = [&](auto &&f) {
    std::vector<std::thread> th;
    for (int t = 1; t < T8; ++t) th.emplace_back(f, t);
    f(0);
    for (auto &x : th) x.join();
  };
  if (G.t > 1) {
    blk_of.resize(size_t(n));
    slot_of.resize(size_t(n));
    par([&](int t) {
      const int64_t a0 = n * t / T8, a1 = n * (t + 1) / T8;
      int64_t z = a0 / G.P, a = a0 - z * G.P;
      for (int64_t i = a0; i < a1; ++i) {
        blk_of[i] = int32_t((z >> lt) * G.nch + (a >> lw));
        slot_of[i] = int32_t(((z & (G.t - 1)) << lw) | (a & (G.w - 1)));
        if (++a == G.P) {
          a = 0;
          ++z;
        }
      }
    });
    // every dependency must stay in its block or lead to a block processed
    // earlier, and every row must fit the flat dependency slots
    std::vector<char> ok(size_t(T8), 1);
    par([&](int t) {
      const int64_t a0 = n * t / T8, a1 = n * (t + 1) / T8;
      for (int64_t i = a0; i < a1 && ok[t]; ++i) {
        int nd = 0;
        dv.each(i, [&](int32_t j) {
          ++nd;
          if (forward ? blk_of[j] > blk_of[i] : blk_of[j] < blk_of[i]) ok[t] = 0;
        });
        if (nd > ELLW) ok[t] = 0;
      }
    });
    if (std::find(ok.begin(), ok.end(), 0) != ok.end()) {
      G = plain_geom(n, blk_rows);
      lw = lt = 0;
      while ((1 << lw) < G.w) ++lw;
    }
  }
  const bool deep = G.t > 1;
  auto BLK = [&](int64_t i) -> int64_t { return deep ? blk_of[i] : (i >> lw); };
  auto SLOT = [&](int64_t i) -> int32_t { return deep ? slot_of[i] : int32_t(i & (G.w - 1)); };
  p.geom = G;
  {
    const int64_t nper = (n + G.P - 1) / G.P, nzg = (nper + G.t - 1) / G.t;
    const int64_t rest = n - (nzg - 1) * G.t * G.P;
    p.nblk = int32_t((nzg - 1) * G.nch + std::min<int64_t>(G.nch, (rest + G.w - 1) / G.w));
  }
  p.blk_r.assign(size_t(2) * p.nblk, 0);
  p.blk_lev.assign(size_t(p.nblk) + 1, 0);
  p.loc_pos.clear();
  p.order.assign(size_t(std::max<int64_t>(n, 1)), 0);
  // block (by id): first row and width of its ranges; range k starts k * P
  // rows later, all clipped to n
  auto ranges = [&](int64_t id, int64_t &r0, int64_t &wb) {
    const int64_t bz = id / G.nch, ba = id - bz * G.nch;
    r0 = bz * G.t * G.P + ba * G.w;
    wb = std::min<int64_t>(G.w, G.P - ba * G.w);
  };
  // blocks are independent: their local levels are computed on up to 8
  // host threads, then the level boundaries are concatenated in block
  // order.  Block b's positions start after those of the blocks processed
  // before it (in the backward direction the first one is the short tail).
  std::vector<std::vector<int32_t>> bpos(size_t(p.nblk));
  std::vector<int32_t> bbase(size_t(p.nblk) + 1, 0), bwide(size_t(p.nblk), 0);
  for (int32_t b = 0; b < p.nblk; ++b) {
    const int64_t id = forward ? b : p.nblk - 1 - b;
    int64_t r0, wb, rows = 0;
    ranges(id, r0, wb);
    for (int32_t k = 0; k < G.t; ++k) {
      const int64_t a = r0 + k * G.P;
      if (a >= n) break;
      rows += std::min<int64_t>(a + wb, n) - a;
    }
    bbase[size_t(b) + 1] = bbase[size_t(b)] + int32_t(rows);
  }
  auto do_block = [&](int32_t b, std::vector<int32_t> &loc, std::vector<int32_t> &cnt) {
    const int64_t id = forward ? b : p.nblk - 1 - b;
    int64_t r0, wb;
    ranges(id, r0, wb);
    const int32_t base = bbase[size_t(b)];
    p.blk_r[2 * b] = int32_t(r0);
    p.blk_r[2 * b + 1] = int32_t(std::min<int64_t>(r0 + wb, n));
    int32_t nk = 0;
    while (nk < G.t && r0 + nk * G.P < n) ++nk;
    // the block's rows in the sweep's direction
    auto each_row = [&](auto &&f) {
      for (int32_t kk = 0; kk < nk; ++kk) {
        const int32_t k = forward ? kk : nk - 1 - kk;
        const int64_t a = r0 + k * G.P, e = std::min<int64_t>(a + wb, n);
        if (forward)
          for (int64_t i = a; i < e; ++i) f(i);
        else
          for (int64_t i = e - 1; i >= a; --i) f(i);
      }
    };
    int32_t nl = 1;
    each_row([&](int64_t i) {
      int32_t l = 0;
      dv.each(i, [&](int32_t j) {
        if (BLK(j) == id) l = std::max(l, loc[SLOT(j)] + 1);
      });
      loc[SLOT(i)] = l;
      nl = std::max(nl, l + 1);
    });
    cnt.assign(size_t(nl) + 1, 0);
    each_row([&](int64_t i) { cnt[loc[SLOT(i)] + 1]++; });
    for (int32_t l = 0; l < nl; ++l) cnt[l + 1] += cnt[l];
    // a local level wider than a workgroup is cut into pieces of at most
    // BLOCK rows (its rows are independent), so a lane owns one row
    std::vector<int32_t> &bp = bpos[size_t(b)];
    int32_t widest = 0;
    for (int32_t l = 0; l < nl; ++l) {
      widest = std::max(widest, std::min(BLOCK, cnt[l + 1] - cnt[l]));
      for (int32_t q = cnt[l]; q < cnt[l + 1]; q += BLOCK) bp.push_back(base + q);
    }
    bwide[size_t(b)] = widest;
    each_row([&](int64_t i) { p.order[base + cnt[loc[SLOT(i)]]++] = int32_t(i); });
  };
  {
    const int T = int(std::min<int64_t>(8, std::max<int32_t>(1, p.nblk / 4)));
    auto work = [&](int t) {
      std::vector<int32_t> loc(size_t(blk_rows), 0), cnt;
      for (int32_t b = t; b < p.nblk; b += T) do_block(b, loc, cnt);
    };
    std::vector<std::thread> th;
    for (int t = 1; t < T; ++t) th.emplace_back(work, t);
    work(0);
    for (auto &x : th) x.join();
  }
  p.max_piece = p.nblk ? *std::max_element(bwide.begin(), bwide.end()) : 0;
  for (int32_t b = 0; b < p.nblk; ++b) {
    p.blk_lev[b] = int32_t(p.loc_pos.size());
    p.loc_pos.insert(p.loc_pos.end(), bpos[size_t(b)].begin(), bpos[size_t(b)].end());
  }
  p.blk_lev[p.nblk] = int32_t(p.loc_pos.size());
  p.loc_pos.push_back(int32_t(n));
  p.levptr.assign(2, 0);
  p.levptr[1] = int32_t(n);
  p.seg.assign(1, int32_t(n));
  p.seg_level.assign(1, 0);
}

void build_plan(const HostCsr &h, const HostCsr *ht, int kind, int blk_rows, HostPlan &p) {
  p.mode = plan_mode(h, ht, kind, blk_rows);
  build_plan_levels(h, ht, kind, blk_rows, p);
  build_plan_blocks(h, ht, kind, blk_rows, p);
}

size_t plan_bytes(int64_t n, int64_t nnz_bound, int C, int KF, bool div, Bump &b, Plan *out) {
  Plan tmp;
  Plan &p = out ? *out : tmp;
  p.order = b.take<int32_t>(size_t(n));
  p.ptr = b.take<int32_t>(size_t(n) + 1);
  p.col = b.take<int32_t>(size_t(nnz_bound));
  p.src = b.take<int32_t>(size_t(nnz_bound));
  p.seg = b.take<int32_t>(size_t(n) + size_t(n) / WAVE + 2);
  p.seg_level = b.take<int32_t>(size_t(n) + size_t(n) / WAVE + 2);
  p.lev_size = b.take<int32_t>(size_t(n) + 1);
  p.lev_done = b.take<int32_t>(size_t(n) + 1);
  p.val = b.take<double>(size_t(nnz_bound) * C * KF);
  if (div) {
    p.dsrc = b.take<int32_t>(size_t(n));
    p.dval = b.take<double>(size_t(n) * C * KF);
  }
  p.sync = b.take<int32_t>(64);
  p.ell_nd = b.take<int32_t>(size_t(n));
  p.ell_col = b.take<int32_t>(size_t(n) * ELLW);
  p.ell_meta = b.take<int32_t>(size_t(n) * 4);
  p.ell_src = b.take<int32_t>(size_t(n) * ELLW);
  p.ell_val = b.take<double>(size_t(n) * ELLW * C * KF);
  p.blk_r = b.take<int32_t>(2 * size_t(n) + 2);
  p.blk_lev = b.take<int32_t>(size_t(n) + 1);
  p.loc_pos = b.take<int32_t>(size_t(n) + 1);
  p.xflag = b.take<int32_t>(size_t(n) + 1);
  p.xlist = b.take<int32_t>(size_t(n) + 1);
  p.div = div;
  return b.off;
}

int upload_plan(const HostPlan &hp, Plan &p, hipStream_t s) {
  const int64_t n = int64_t(hp.order.size()) > 0 ? int64_t(hp.order.size()) : 0;
  p.nlev = hp.nlev;
  p.nseg = int32_t(hp.seg.size()) - 1;
  p.h_levptr = hp.levptr;
  p.mode = hp.mode;
  p.nblk = hp.nblk;
  p.blk_rows = hp.blk_rows;
  p.max_piece = hp.max_piece;
  p.geom = hp.geom;
  (void)n;
  if (hp.mode != 3)
    MPK_HIP(hipMemcpyAsync(p.order, hp.order.data(), sizeof(int32_t) * p.n,
                           hipMemcpyHostToDevice, s));
  if (hp.mode == 3) {
    p.grid = hp.grid;
    p.grid_by = hp.grid_by;
    p.nx = int64_t(hp.xlist.size());
    p.h_blk.assign(hp.xlist.begin(), hp.xlist.end());
    if (p.nx > 0)
      MPK_HIP(hipMemcpyAsync(p.xlist, p.h_blk.data(), sizeof(int32_t) * size_t(p.nx),
                             hipMemcpyHostToDevice, s));
    return MPK_OK;
  }
  if (hp.mode == 1) {
    p.nloc = int32_t(hp.loc_pos.size()) - 1;
    p.h_blk.clear();
    p.h_blk.insert(p.h_blk.end(), hp.blk_r.begin(), hp.blk_r.end());
    p.h_blk.insert(p.h_blk.end(), hp.blk_lev.begin(), hp.blk_lev.end());
    p.h_blk.insert(p.h_blk.end(), hp.loc_pos.begin(), hp.loc_pos.end());
    const int32_t *hb = p.h_blk.data();
    MPK_HIP(hipMemcpyAsync(p.blk_r, hb, sizeof(int32_t) * hp.blk_r.size(), hipMemcpyHostToDevice, s));
    hb += hp.blk_r.size();
    MPK_HIP(hipMemcpyAsync(p.blk_lev, hb, sizeof(int32_t) * hp.blk_lev.size(),
                           hipMemcpyHostToDevice, s));
    hb += hp.blk_lev.size();
    MPK_HIP(hipMemcpyAsync(p.loc_pos, hb, sizeof(int32_t) * hp.loc_pos.size(),
                           hipMemcpyHostToDevice, s));
  } else {
    MPK_HIP(hipMemcpyAsync(p.seg, hp.seg.data(), sizeof(int32_t) * hp.seg.size(),
                           hipMemcpyHostToDevice, s));
    MPK_HIP(hipMemcpyAsync(p.seg_level, hp.seg_level.data(),
                           sizeof(int32_t) * hp.seg_level.size(), hipMemcpyHostToDevice, s));
    std::vector<int32_t> sz(size_t(hp.nlev) + 1, 0);
    for (int32_t l = 0; l < hp.nlev; ++l) sz[l] = hp.levptr[l + 1] - hp.levptr[l];
    p.h_levsize = sz;
    MPK_HIP(hipMemcpyAsync(p.lev_size, p.h_levsize.data(), sizeof(int32_t) * sz.size(),
                           hipMemcpyHostToDevice, s));
  }
  return MPK_OK;
}

}  // namespace mpk
