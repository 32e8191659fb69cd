// The library's host-side pattern checks and sweep schedules under
// AddressSanitizer and UndefinedBehaviorSanitizer (no device is touched):
// check_pattern, host_transpose and the four sweeps' plans (level and
// blocked schedules, plain and several-planes-deep blocks) on seeded
// patterns: 2D and 3D stencils, random patterns with ragged rows, a
// tridiagonal matrix and single-row and empty-dependency cases.  For every
// plan it checks that the rows form a permutation and that every
// dependency of a row is scheduled before the piece of work holding it.
// The greedy colouring of the multicolour ordering is checked on the same
// patterns: no two adjacent rows share a colour, and every colour below a
// row's own is taken by a neighbour numbered before it.
// Prints "ok" and exits 0 when all hold.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2504_14498_amd/csrc/internal.hpp"

using namespace mpk;

namespace {

struct Pattern {
  int64_t n = 0;
  IVec rp, ci;
};

Pattern stencil(int nx, int ny, int nz) {
  Pattern p;
  p.n = int64_t(nx) * ny * nz;
  p.rp.push_back(0);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int64_t i = (int64_t(z) * ny + y) * nx + x;
        if (z > 0) p.ci.push_back(int32_t(i - int64_t(nx) * ny));
        if (y > 0) p.ci.push_back(int32_t(i - nx));
        if (x > 0) p.ci.push_back(int32_t(i - 1));
        p.ci.push_back(int32_t(i));
        if (x + 1 < nx) p.ci.push_back(int32_t(i + 1));
        if (y + 1 < ny) p.ci.push_back(int32_t(i + nx));
        if (z + 1 < nz) p.ci.push_back(int32_t(i + int64_t(nx) * ny));
        p.rp.push_back(int32_t(p.ci.size()));
      }
  return p;
}

Pattern random_pattern(int64_t n, int maxr, unsigned seed) {
  std::mt19937_64 g(seed);
  Pattern p;
  p.n = n;
  p.rp.push_back(0);
  std::vector<char> mark(size_t(n), 0);
  for (int64_t i = 0; i < n; ++i) {
    std::vector<int32_t> cols{int32_t(i)};
    mark[i] = 1;
    const int m = int(g() % (maxr + 1));
    for (int k = 0; k < m; ++k) {
      const int32_t j = int32_t(g() % n);
      if (!mark[j]) {
        mark[j] = 1;
        cols.push_back(j);
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int32_t j : cols) {
      mark[j] = 0;
      p.ci.push_back(j);
    }
    p.rp.push_back(int32_t(p.ci.size()));
  }
  return p;
}

HostCsr view(const Pattern &p) {
  HostCsr h;
  h.n = p.n;
  h.nnz = int64_t(p.ci.size());
  h.rp = p.rp.data();
  h.ci = p.ci.data();
  return h;
}

int fails = 0;
int plans_of_mode[3] = {0, 0, 0};
#define EXPECT(c)                                                                \
  do {                                                                           \
    if (!(c)) {                                                                  \
      std::fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #c);               \
      ++fails;                                                                   \
      return;                                                                    \
    }                                                                            \
  } while (0)

// Dependencies of row i in sweep `kind` (0: L, 1: U, 2: U^H, 3: L^H).
template <class F> void deps(const HostCsr &h, const HostCsr &t, int kind, int64_t i, F &&f) {
  const HostCsr &g = kind >= 2 ? t : h;
  const bool lower = kind == 0 || kind == 2;
  for (int32_t q = g.rp[i]; q < g.rp[i + 1]; ++q) {
    const int32_t j = g.ci[q];
    if (lower ? j < i : j > i) f(j);
  }
}

void check_plan(const HostCsr &h, const HostCsr &t, int kind, const HostPlan &p) {
  const int64_t n = h.n;
  std::vector<int32_t> pos(size_t(n), -1);
  for (int64_t q = 0; q < n; ++q) {
    const int32_t i = p.order[q];
    EXPECT(i >= 0 && i < n && pos[i] < 0);
    pos[i] = int32_t(q);
  }
  // start position of the unit of work holding each position: a level
  // segment (level schedule) or a local-level piece (blocked schedule)
  std::vector<int32_t> start(size_t(n), 0);
  if (p.mode != 1) {
    EXPECT(p.levptr.size() == size_t(p.nlev) + 1 && p.levptr[p.nlev] == n);
    for (int32_t l = 0; l < p.nlev; ++l)
      for (int32_t q = p.levptr[l]; q < p.levptr[l + 1]; ++q) start[q] = p.levptr[l];
    for (size_t s = 0; s + 1 < p.seg.size(); ++s) {
      EXPECT(p.seg[s + 1] - p.seg[s] <= WAVE && p.seg[s] < p.seg[s + 1]);
      const int32_t l = p.seg_level[s];
      EXPECT(p.seg[s] >= p.levptr[l] && p.seg[s + 1] <= p.levptr[l + 1]);
    }
  } else {
    EXPECT(p.blk_lev.size() == size_t(p.nblk) + 1);
    EXPECT(p.loc_pos.back() == n);
    for (int32_t b = 0; b < p.nblk; ++b)
      for (int32_t k = p.blk_lev[b]; k < p.blk_lev[b + 1]; ++k) {
        const int32_t s = p.loc_pos[k], e = p.loc_pos[k + 1];
        EXPECT(s < e && e - s <= BLOCK && e <= n);
        for (int32_t q = s; q < e; ++q) start[q] = s;
      }
    EXPECT(p.max_piece >= 1 && p.max_piece <= BLOCK);
  }
  for (int64_t i = 0; i < n; ++i)
    deps(h, t, kind, i, [&](int32_t j) {
      if (pos[j] >= start[pos[i]]) {
        std::fprintf(stderr, "kind %d mode %d: row %lld (pos %d) depends on %d (pos %d)\n", kind,
                     p.mode, (long long)i, pos[i], j, pos[j]);
        ++fails;
      }
    });
}

void check_color(const HostCsr &h, const HostCsr &t) {
  IVec color;
  const int32_t ncol = greedy_color(h, color);
  int32_t top = -1;
  for (int64_t i = 0; i < h.n; ++i) top = std::max(top, color[i]);
  EXPECT(ncol == top + 1);
  std::vector<char> taken;
  for (int64_t i = 0; i < h.n; ++i) {
    taken.assign(size_t(color[i]) + 1, 0);
    // neighbours in A + A^T: the columns of row i of A and of A^T
    for (const HostCsr *g : {&h, &t})
      for (int32_t q = g->rp[i]; q < g->rp[i + 1]; ++q) {
        const int32_t j = g->ci[q];
        if (j == i) continue;
        EXPECT(color[j] != color[i]);
        if (j < i && color[j] < color[i]) taken[color[j]] = 1;
      }
    for (int32_t c = 0; c < color[i]; ++c) EXPECT(taken[c]);
  }
}

// Grid sweeps: detect_grid on stencils (with the grid's shape) and on
// other patterns (rejected); the rows a grid sweep's blocks read from
// other blocks (the y - 1 and z - 1 neighbours of a block's first lines,
// in the sweep's coordinates) are all in the plan's list, and the list
// holds rows in range, each once.
void check_grid(const HostCsr &h, int nx, int ny, int nz, bool expect) {
  int32_t gx = -1, gy = -1, gz = -1;
  const bool got = detect_grid(h, gx, gy, gz);
  EXPECT(got == expect);
  if (!got) return;
  EXPECT(gx == nx && gy == ny && gz == nz);
  {
    // closed-form levels of the grid = the levels found from the pattern
    HostPlan ref;
    ref.mode = plan_mode(h, nullptr, 0, 0);
    build_plan_levels(h, nullptr, 0, 0, ref);
    GridDims gd;
    gd.nx = gx;
    gd.ny = gy;
    gd.nz = gz;
    std::vector<int32_t> levptr, order;
    grid_levels(gd, levptr, order);
    EXPECT(levptr == ref.glob_levptr);
    EXPECT(order == ref.glob_order);
  }
  for (int kind = 0; kind < 2; ++kind) {
    HostPlan hp;
    hp.mode = 3;
    hp.grid.nx = gx;
    hp.grid.ny = gy;
    hp.grid.nz = gz;
    build_plan_grid(h.n, kind, hp);
    const int by = hp.grid_by, bz = 64 / by;
    EXPECT(by * bz == 64 && hp.grid.nby * by >= ny && hp.grid.nbz * bz >= nz);
    std::vector<char> in(size_t(h.n), 0);
    for (int32_t r : hp.xlist) {
      EXPECT(r >= 0 && r < h.n && !in[r]);
      in[r] = 1;
    }
    const int64_t pl = int64_t(nx) * ny;
    for (int64_t z = 0; z < nz; ++z)
      for (int64_t y = 0; y < ny; ++y)
        for (int64_t x = 0; x < nx; ++x) {
          const int64_t s = z * pl + y * nx + x;
          auto real = [&](int64_t v) { return kind == 1 ? h.n - 1 - v : v; };
          if (y > 0 && y % by == 0) EXPECT(in[real(s - nx)]);
          if (z > 0 && z % bz == 0) EXPECT(in[real(s - pl)]);
        }
  }
}

void run(const Pattern &pat, const char *name) {
  const HostCsr h = view(pat);
  int64_t bad = -2;
  if (check_pattern(h, &bad) != MPK_OK || bad != -1) {
    std::fprintf(stderr, "%s: pattern rejected (row %lld)\n", name, (long long)bad);
    ++fails;
    return;
  }
  IVec trp, tci, tsrc;
  host_transpose(h, trp, tci, tsrc);
  HostCsr t;
  t.n = h.n;
  t.nnz = h.nnz;
  t.rp = trp.data();
  t.ci = tci.data();
  for (int64_t p = 0; p < h.nnz; ++p)
    if (tsrc[p] < 0 || tsrc[p] >= h.nnz) ++fails;
  check_color(h, t);
  // the one-launch-per-level schedule, forced
  setenv("MPK_TRSV_MODE", "s", 1);
  for (int kind = 0; kind < 4; ++kind) {
    HostPlan hp;
    build_plan(h, &t, kind, 1024, hp);
    EXPECT(hp.mode == 2);
    plans_of_mode[hp.mode]++;
    check_plan(h, t, kind, hp);
  }
  unsetenv("MPK_TRSV_MODE");
  for (int rows : {0, 64, 256, 1024, 8192})
    for (int kind = 0; kind < 4; ++kind) {
      HostPlan hp;
      build_plan(h, &t, kind, rows, hp);
      plans_of_mode[hp.mode]++;
      check_plan(h, t, kind, hp);
    }
}

void bad_patterns() {
  // unsorted columns, a missing diagonal, an out-of-range column
  Pattern p;
  p.n = 3;
  p.rp = {0, 2, 3, 5};
  p.ci = {1, 0, 1, 0, 2};
  int64_t bad = -2;
  HostCsr h = view(p);
  if (check_pattern(h, &bad) != MPK_EPATTERN || bad != 0) ++fails;
  p.ci = {0, 1, 0, 0, 2};
  h = view(p);
  if (check_pattern(h, &bad) != MPK_ENO_DIAG || bad != 1) ++fails;
  p.ci = {0, 1, 1, 0, 3};
  h = view(p);
  if (check_pattern(h, &bad) != MPK_EPATTERN || bad != 2) ++fails;
}

}  // namespace

int main() {
  check_grid(view(stencil(20, 13, 9)), 20, 13, 9, true);
  check_grid(view(stencil(9, 17, 16)), 9, 17, 16, true);
  check_grid(view(stencil(45, 33, 1)), 45, 33, 1, true);
  check_grid(view(stencil(64, 70, 1)), 64, 70, 1, true);
  check_grid(view(stencil(37, 1, 1)), 37, 1, 1, false);   // 1D: not a grid sweep
  check_grid(view(random_pattern(3001, 9, 5)), 0, 0, 0, false);
  {
    // a stencil with one entry missing is not a grid
    Pattern p = stencil(12, 12, 12);
    p.ci.erase(p.ci.begin() + 5000);
    for (size_t k = 0; k < p.rp.size(); ++k)
      if (p.rp[k] > 5000) --p.rp[k];
    check_grid(view(p), 0, 0, 0, false);
  }
  {
    // detect_grid runs before the pattern checks: malformed row pointers
    // (negative, decreasing, past nnz, a wrong total) are rejected with
    // every read inside the arrays (the sanitizers see any other read)
    const Pattern base = stencil(10, 9, 8);
    const size_t n = base.rp.size() - 1;
    const int32_t nnz = base.rp.back();
    for (int c = 0; c < 6; ++c) {
      Pattern p = base;
      if (c == 0) p.rp[n / 2] = -7;
      if (c == 1) p.rp[n / 2] = nnz + 40;
      if (c == 2) std::swap(p.rp[n / 3], p.rp[n / 3 + 1]);
      if (c == 3) p.rp[n] = nnz - 1;
      if (c == 4) p.rp[n - 1] = nnz + 3;
      if (c == 5) p.rp[0] = 2;
      check_grid(view(p), 0, 0, 0, false);
    }
  }
  run(stencil(37, 1, 1), "tridiagonal");
  run(stencil(1, 1, 1), "one row");
  run(stencil(45, 33, 1), "5-point 45x33");
  run(stencil(20, 20, 20), "7-point 20^3");
  run(stencil(64, 64, 9), "7-point 64x64x9");
  run(random_pattern(3001, 9, 5), "random 3001");
  run(random_pattern(700, 30, 6), "random 700");
  bad_patterns();
  // both schedules were built and checked
  if (plans_of_mode[0] == 0 || plans_of_mode[1] == 0 || plans_of_mode[2] == 0) ++fails;
  if (fails) {
    std::printf("%d failures\n", fails);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
