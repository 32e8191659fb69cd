// ops.hip -- SpMV, inner product and ILU(0) (factor, apply) behind the
// C-ABI declared in include/mpk.h.
#include <chrono>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <thread>

#include "kernels.hpp"

namespace mpk {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

int validate_csr_args(const mpk_csr *A) {
  if (!A || A->n <= 0 || A->nnz < A->n || A->nnz >= (int64_t(1) << 31) || A->n >= (int64_t(1) << 31))
    return MPK_EINVAL;
  if (!A->row_ptr || !A->col_idx || !A->val) return MPK_EINVAL;
  return MPK_OK;
}

int csr_check_device_values(const mpk_csr *A, int C, int32_t *word, int64_t *bad_row,
                            hipStream_t s) {
  int32_t init = INT_MAX, got = INT_MAX;
  MPK_HIP(hipMemcpyAsync(word, &init, sizeof(int32_t), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(check_finite, dim3(nblocks(A->n)), dim3(BLOCK), 0, s, A->n, C, A->row_ptr,
                     A->val, word);
  MPK_HIP(hipGetLastError());
  MPK_HIP(hipMemcpyAsync(&got, word, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPK_HIP(hipStreamSynchronize(s));
  if (got != INT_MAX) {
    *bad_row = got;
    return MPK_ENONFINITE;
  }
  return MPK_OK;
}

int spmv_launch(int C, int K, int64_t n, const int32_t *rp, const int32_t *ci, const double *val,
                const double *x, double *y, const int32_t *done, hipStream_t s, int lanes) {
  if (n == 0) return MPK_OK;
  return dispatch_ck(C, K, [&]<int CC, int KK>() {
    auto vec = [&]<int G>() {
      const unsigned nb = unsigned((n + BLOCK / G - 1) / (BLOCK / G));
      hipLaunchKernelGGL((spmv_vec<CC, KK, G>), dim3(xcd_grid(nb)), dim3(BLOCK), 0, s, n, rp, ci,
                         val, x, y, done);
    };
    switch (lanes) {
      case 2: vec.template operator()<2>(); break;
      case 4: vec.template operator()<4>(); break;
      case 8: vec.template operator()<8>(); break;
      case 16: vec.template operator()<16>(); break;
      default: {
        SpmvOp<CC, KK> op{rp, ci, val, x, y};
        hipLaunchKernelGGL((row_kernel<CC, KK, 0, SpmvOp<CC, KK>>), dim3(xcd_grid(nblocks(n))),
                           dim3(BLOCK), 0, s, n, op, done, (double *)nullptr);
      }
    }
    return hipGetLastError() == hipSuccess ? MPK_OK : MPK_EDEVICE;
  });
}

// Lanes per row of the standalone SpMV, per matrix (its three device
// arrays and n): set by mpk_spmv_set_lanes or mpk_spmv_tune; 1 (one lane
// per row) otherwise.
namespace {
struct LanesKey {
  const void *rp, *ci, *val;
  int64_t n;
  bool operator<(const LanesKey &o) const {
    return std::tie(rp, ci, val, n) < std::tie(o.rp, o.ci, o.val, o.n);
  }
};
std::mutex lanes_mu;
std::map<LanesKey, int> lanes_table;
LanesKey lanes_key(const mpk_csr *A) { return {A->row_ptr, A->col_idx, A->val, A->n}; }
}  // namespace

int spmv_lanes(const mpk_csr *A) {
  std::lock_guard<std::mutex> lock(lanes_mu);
  auto it = lanes_table.find(lanes_key(A));
  return it == lanes_table.end() ? 1 : it->second;
}

// ------------------------------------------------------------- ILU(0)
size_t ilu0_layout(int64_t n, int64_t nnz, int C, int KF, int flags, Bump &b, Ilu0 *M) {
  Ilu0 tmp;
  Ilu0 &m = M ? *M : tmp;
  m.words = b.take<int32_t>(64);
  m.diag = b.take<int32_t>(size_t(n));
  m.f = b.take<double>(size_t(nnz) * C * KF);
  plan_bytes(n, nnz, C, KF, false, b, &m.L);
  plan_bytes(n, nnz, C, KF, true, b, &m.U);
  if (flags & MPK_ILU0_ADJOINT) {
    plan_bytes(n, nnz, C, KF, true, b, &m.UH);
    plan_bytes(n, nnz, C, KF, false, b, &m.LH);
  }
  m.tmp = b.take<double>(size_t(n) * C * 4);
  m.fac_order = b.take<int32_t>(size_t(n));
  m.scan_tmp = b.take<int32_t>(size_t(n) / SCAN_BLOCK + 2);
  if (flags & MPK_ILU0_ADJOINT) {
    m.t_rp = b.take<int32_t>(size_t(n) + 1);
    m.t_ci = b.take<int32_t>(size_t(nnz));
    m.t_src = b.take<int32_t>(size_t(nnz));
  }
  return b.off;
}

template <int C, int KF>
static int ilu0_levels(const Ilu0 &M, hipStream_t s) {
  const int32_t nlev = int32_t(M.h_fac_levptr.size()) - 1;
  for (int32_t l = 0; l < nlev; ++l) {
    const int32_t a = M.h_fac_levptr[l], cnt = M.h_fac_levptr[l + 1] - a;
    hipLaunchKernelGGL((ilu0_level<C, KF>), dim3(nblocks(cnt)), dim3(BLOCK), 0, s, cnt,
                       M.fac_order + a, M.row_ptr, M.col_idx, M.diag, M.f, M.words + 1);
  }
  MPK_HIP(hipGetLastError());
  return MPK_OK;
}

// ILU(0) of a recognised grid in one launch (ilu0_grid): the records from
// A, the sentinel on the pivots the next blocks read, the factorisation,
// then the factor written into A's pattern.  Uses the L plan (grid, lines
// per block, the list of those rows), the two plans' record arrays and
// tmp; words[4] is its watchdog word, words[1] the zero-pivot row.
template <int C, int KF>
static int ilu0_grid_run(const Ilu0 &M, const double *val, hipStream_t s) {
  const Plan &P = M.L;
  const int64_t n = M.n;
  const int V = C * KF;
  hipLaunchKernelGGL(grid_fac_gather, dim3(nblocks(n)), dim3(BLOCK), 0, s, n, P.grid, P.grid_by,
                     C, KF, (const int32_t *)M.diag, val, M.L.ell_val, M.U.ell_val);
  hipLaunchKernelGGL(trsv_prep, dim3(nblocks(std::max<int64_t>(P.nx * V, 1))), dim3(BLOCK), 0, s,
                     V, (const int32_t *)P.xlist, P.nx, M.tmp, (const int32_t *)nullptr,
                     int64_t(0), (double *)nullptr, 0, (int32_t *)nullptr, 0, (int32_t *)nullptr,
                     M.L.sync, M.U.sync, M.words + 4, (const int32_t *)nullptr);
  const unsigned grid = unsigned(std::max<int64_t>(1, std::min<int64_t>(P.nblk, 512)));
  if (P.grid_by == 8)
    hipLaunchKernelGGL((ilu0_grid<C, KF, 8>), dim3(grid), dim3(WAVE), 0, s, n, P.grid,
                       M.L.ell_val, (const double *)M.U.ell_val, M.tmp, M.L.sync, M.words + 4,
                       M.words + 1);
  else
    hipLaunchKernelGGL((ilu0_grid<C, KF, 64>), dim3(grid), dim3(WAVE), 0, s, n, P.grid,
                       M.L.ell_val, (const double *)M.U.ell_val, M.tmp, M.L.sync, M.words + 4,
                       M.words + 1);
  hipLaunchKernelGGL(grid_fac_scatter, dim3(nblocks(n)), dim3(BLOCK), 0, s, n, P.grid,
                     P.grid_by, V, (const int32_t *)M.diag, (const double *)M.L.ell_val, M.f);
  MPK_HIP(hipGetLastError());
  return MPK_OK;
}

// Per-position schedule arrays of a plan, built on the device from the
// uploaded row order (count, scan, fill).
static int device_plan_arrays(Plan &P, const Ilu0 &M, int kind, hipStream_t s) {
  if (P.mode == 3) {
    // grid sweeps need only their factor records (gather_plan)
    P.nnz = 0;
    return MPK_OK;
  }
  const int64_t n = P.n;
  const bool tr = kind >= 2;
  const int32_t *rp = tr ? M.t_rp : M.row_ptr, *ci = tr ? M.t_ci : M.col_idx;
  const int lower = (kind == 0 || kind == 2) ? 1 : 0;
  const unsigned g = nblocks(n);
  // counts land in ptr[0..n), then the scan rewrites ptr in place
  hipLaunchKernelGGL(plan_count, dim3(g), dim3(BLOCK), 0, s, n, P.order, rp, ci, lower, P.ptr);
  const int32_t nb = int32_t((n + SCAN_BLOCK - 1) / SCAN_BLOCK);
  hipLaunchKernelGGL(scan_blocks, dim3(nb), dim3(BLOCK), 0, s, n, (const int32_t *)P.ptr, P.ptr,
                     M.scan_tmp);
  hipLaunchKernelGGL(scan_sums, dim3(1), dim3(BLOCK), 0, s, nb, M.scan_tmp);
  hipLaunchKernelGGL(scan_add, dim3(g), dim3(BLOCK), 0, s, n, P.ptr, (const int32_t *)M.scan_tmp,
                     nb);
  const bool ell = P.mode == 1;
  if (ell) MPK_HIP(hipMemsetAsync(P.xflag, 0, sizeof(int32_t) * size_t(n), s));
  hipLaunchKernelGGL(plan_fill, dim3(g), dim3(BLOCK), 0, s, n, P.order, rp, ci,
                     tr ? (const int32_t *)M.t_src : nullptr, lower, (const int32_t *)P.ptr, P.col,
                     P.src, ell ? P.ell_nd : nullptr, ell ? P.ell_col : nullptr,
                     ell ? P.ell_src : nullptr, ell ? P.ell_meta : nullptr, P.geom,
                     (const int32_t *)M.diag, P.div ? P.dsrc : nullptr, ell ? P.xflag : nullptr);
  if (ell) {
    // the rows other blocks read: marked in the records, and listed (their
    // scan offsets go to lev_done, which only the level schedule uses)
    hipLaunchKernelGGL(plan_xmeta, dim3(g), dim3(BLOCK), 0, s, n, (const int32_t *)P.order,
                       (const int32_t *)P.xflag, P.ell_meta);
    hipLaunchKernelGGL(scan_blocks, dim3(nb), dim3(BLOCK), 0, s, n, (const int32_t *)P.xflag,
                       P.lev_done, M.scan_tmp);
    hipLaunchKernelGGL(scan_sums, dim3(1), dim3(BLOCK), 0, s, nb, M.scan_tmp);
    hipLaunchKernelGGL(scan_add, dim3(g), dim3(BLOCK), 0, s, n, P.lev_done,
                       (const int32_t *)M.scan_tmp, nb);
    hipLaunchKernelGGL(plan_xlist, dim3(g), dim3(BLOCK), 0, s, n, (const int32_t *)P.xflag,
                       (const int32_t *)P.lev_done, P.xlist);
  }
  MPK_HIP(hipGetLastError());
  int32_t tot[2] = {0, 0};
  MPK_HIP(hipMemcpyAsync(&tot[0], P.ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  if (ell) MPK_HIP(hipMemcpyAsync(&tot[1], P.lev_done + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPK_HIP(hipStreamSynchronize(s));
  P.nnz = tot[0];
  P.nx = ell ? tot[1] : n;
  return MPK_OK;
}

static int gather_plan(const Plan &P, const Ilu0 &M, hipStream_t s) {
  if (P.mode == 3) {
    // grid sweep: each row's term values (and pivot) in one record
    if (P.n > 0)
      hipLaunchKernelGGL(grid_gather, dim3(nblocks(P.n)), dim3(BLOCK), 0, s, P.n, P.grid,
                         P.grid_by, P.div ? 1 : 0, M.C * M.KF, (const int32_t *)M.diag,
                         (const double *)M.f, P.ell_val);
    MPK_HIP(hipGetLastError());
    return MPK_OK;
  }
  if (P.mode == 1 && P.n > 0)
    hipLaunchKernelGGL(gather_vals, dim3(nblocks(P.n * ELLW)), dim3(BLOCK), 0, s, P.n * ELLW, M.C,
                       M.KF, P.ell_src, M.f, P.ell_val, 0);
  if (P.nnz > 0)
    hipLaunchKernelGGL(gather_vals, dim3(nblocks(P.nnz)), dim3(BLOCK), 0, s, P.nnz, M.C, M.KF,
                       P.src, M.f, P.val, 0);
  if (P.div)
    hipLaunchKernelGGL(gather_vals, dim3(nblocks(P.n)), dim3(BLOCK), 0, s, P.n, M.C, M.KF, P.dsrc,
                       M.f, P.dval, 0);
  MPK_HIP(hipGetLastError());
  return MPK_OK;
}

int ilu0_regather(const Ilu0 &M, hipStream_t s) {
  int st;
  if ((st = gather_plan(M.L, M, s)) || (st = gather_plan(M.U, M, s))) return st;
  if (M.flags & MPK_ILU0_ADJOINT)
    if ((st = gather_plan(M.UH, M, s)) || (st = gather_plan(M.LH, M, s))) return st;
  return MPK_OK;
}

static bool timing_on() {
  static const bool on = getenv("MPK_TIMING") != nullptr;
  return on;
}
#define MPK_PHASE(name)                                                          \
  do {                                                                           \
    if (timing_on()) {                                                           \
      hipStreamSynchronize(s);                                                   \
      const double t_ = now_ms();                                                \
      fprintf(stderr, "[mpk] %-22s %8.2f ms\n", name, t_ - tp);                  \
      tp = t_;                                                                   \
    }                                                                            \
  } while (0)

// Row i against the stencil of an nx x ny x nz grid numbered x fastest: it
// stores exactly its in-grid neighbours and itself, ascending (the host's
// detect_grid test, one thread per row); otherwise *bad is set.  A row is
// read only when its bounds lie inside [0, nnz).
static __global__ void grid_check(int64_t n, int32_t nx, int32_t ny, int32_t nz, int64_t nnz,
                                  const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                  int32_t *bad) {
  const int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (i >= n) return;
  const int64_t pl = int64_t(nx) * ny;
  const int64_t x = i % nx, y = (i / nx) % ny, z = i / pl;
  int64_t want[7];
  int m = 0;
  if (z > 0) want[m++] = i - pl;
  if (y > 0) want[m++] = i - nx;
  if (x > 0) want[m++] = i - 1;
  want[m++] = i;
  if (x < nx - 1) want[m++] = i + 1;
  if (y < ny - 1) want[m++] = i + nx;
  if (z < nz - 1) want[m++] = i + pl;
  const int32_t a = rp[i], e = rp[i + 1];
  bool ok = a >= 0 && e <= nnz && e - a == m;
  for (int k = 0; ok && k < m; ++k) ok = ci[a + k] == want[k];
  if (!ok) atomicOr(bad, 1);
}

// A grid recognised on the device, the pattern left there: the extents
// from the last row (a few words copied), then every row checked by
// grid_check.  yes is false (and nothing else done) when A is no grid.
static int device_grid(const mpk_csr *A, int32_t *word, int32_t &gx, int32_t &gy, int32_t &gz,
                       bool &yes, hipStream_t s) {
  yes = false;
  const int64_t n = A->n;
  if (n < 4) return MPK_OK;
  int32_t r[3] = {-1, -1, -1};
  MPK_HIP(hipMemcpyAsync(&r[0], A->row_ptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPK_HIP(hipMemcpyAsync(&r[1], A->row_ptr + n - 1, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPK_HIP(hipStreamSynchronize(s));
  if (r[0] != 0 || r[2] != A->nnz || r[1] < 0 || r[1] > r[2] || r[2] - r[1] > 7) return MPK_OK;
  int32_t last[7];
  if (r[2] > r[1]) {
    MPK_HIP(hipMemcpyAsync(last, A->col_idx + r[1], sizeof(int32_t) * size_t(r[2] - r[1]),
                           hipMemcpyDeviceToHost, s));
    MPK_HIP(hipStreamSynchronize(s));
  }
  if (!grid_dims_from_last_row(n, last, r[2] - r[1], gx, gy, gz)) return MPK_OK;
  const int32_t zero = 0;
  MPK_HIP(hipMemcpyAsync(word, &zero, sizeof(int32_t), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(grid_check, dim3(nblocks(n)), dim3(BLOCK), 0, s, n, gx, gy, gz, A->nnz,
                     A->row_ptr, A->col_idx, word);
  MPK_HIP(hipGetLastError());
  int32_t bad = 1;
  MPK_HIP(hipMemcpyAsync(&bad, word, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPK_HIP(hipStreamSynchronize(s));
  yes = bad == 0;
  return MPK_OK;
}

int ilu0_factor_impl(int C, int KF, const mpk_csr *A, int flags, void *ws, size_t ws_bytes,
                     Ilu0 *M, mpk_info *info, hipStream_t s) {
  const double t0 = now_ms();
  double tp = t0;
  int64_t bad = -1;
  if (info) info->bad_row = -1;
  Bump b(ws);
  if (ilu0_layout(A->n, A->nnz, C, KF, flags, b, M) > ws_bytes) return MPK_EWORKSPACE;
  M->n = A->n;
  M->nnz = A->nnz;
  M->C = C;
  M->KF = KF;
  M->flags = flags;
  M->row_ptr = A->row_ptr;
  M->col_idx = A->col_idx;
  HostCsr h;
  int st = MPK_OK;
  const int kmax = (flags >> 4) & 7 ? (flags >> 4) & 7 : 4;
  // the blocked sweeps address their arrays with 32-bit buffer offsets
  const int64_t big = int64_t(A->n) * std::max(ELLW * C * KF, C * kmax) * 8;
  const int br = big < (int64_t(1) << 31) ? default_block_rows(C, kmax) : 0;
  const bool adj = (flags & MPK_ILU0_ADJOINT) != 0;
  // A 7-point or 5-point grid numbered x fastest gets grid sweeps for L and
  // U and the one-launch grid factorisation (MPK_TRSV_MODE forces the other
  // schedules and the level-by-level factorisation).  Recognising it checks
  // every row against the stencil, so its pattern needs no other check; and
  // without adjoint schedules nothing else needs the pattern on the host, so
  // it is recognised on the device and not copied.
  const char *force = getenv("MPK_TRSV_MODE");
  int32_t gx = 0, gy = 0, gz = 0;
  const bool grid_ok = br > 0 && !(force && (force[0] == 'b' || force[0] == 'l' || force[0] == 's')) &&
                       A->nnz * int64_t(C * KF) * 8 < (int64_t(1) << 31) &&
                       A->n * int64_t(C * kmax) * 8 < (int64_t(1) << 31);
  bool grid = false;
  if (grid_ok && !adj && (st = device_grid(A, M->words + 8, gx, gy, gz, grid, s))) return st;
  if (grid) {
    h.n = A->n;  // the pattern stays on the device
    h.nnz = A->nnz;
  } else {
    if ((st = fetch_pattern(A, h, s))) return st;
    MPK_PHASE("fetch pattern");
    grid = grid_ok && detect_grid(h, gx, gy, gz);
    if (!grid) {
      st = check_pattern(h, &bad);
      if (st) {
        if (info) info->bad_row = bad;
        return st;
      }
    }
  }
  st = csr_check_device_values(A, C, M->words + 2, &bad, s);
  if (st) {
    if (info) info->bad_row = bad;
    return st;
  }
  MPK_PHASE("check pattern+values");
  hipLaunchKernelGGL(find_diag, dim3(nblocks(A->n)), dim3(BLOCK), 0, s, A->n, A->row_ptr,
                     A->col_idx, M->diag);
  HostPlan hp[4];
  HostCsr ht;
  {
    // the schedules of the two (four) sweeps are independent: the backward
    // (and adjoint) ones are built on other host threads.  The forward
    // sweep's global levels give the factorisation order, so the level-by-
    // level factorisation is launched as soon as they exist and runs on the
    // device while the blocked schedules are built on the host; the forward
    // sweep's blocked schedule needs only the schedule choice and is built
    // on its own thread meanwhile.  The grid factorisation needs no levels.
    if (grid) {
      for (int k = 0; k < 2; ++k) {
        hp[k].mode = 3;
        hp[k].grid.nx = gx;
        hp[k].grid.ny = gy;
        hp[k].grid.nz = gz;
      }
      // the L plan first: the grid factorisation uses its block shape and
      // its list of the rows the next blocks read
      build_plan_grid(h.n, 0, hp[0]);
      M->L.n = A->n;
      if ((st = upload_plan(hp[0], M->L, s))) return st;
    } else {
      hp[0].mode = plan_mode(h, nullptr, 0, br);
    }
    std::thread t0([&] {
      if (!grid) build_plan_blocks(h, nullptr, 0, br, hp[0]);
    });
    std::thread t1([&] {
      if (grid)
        build_plan_grid(h.n, 1, hp[1]);
      else
        build_plan(h, nullptr, 1, br, hp[1]);
    });
    std::thread t2;
    if (adj) {
      t2 = std::thread([&] {
        IVec tsrc;
        ht.n = h.n;
        ht.nnz = h.nnz;
        host_transpose(h, ht.own_rp, ht.own_ci, tsrc);
        ht.own();
        std::thread t4([&] { build_plan(h, &ht, 3, br, hp[3]); });
        build_plan(h, &ht, 2, br, hp[2]);
        t4.join();
      });
    }
    if (!grid) {
      build_plan_levels(h, nullptr, 0, br, hp[0]);
      M->h_fac_levptr = hp[0].glob_levptr;
      if (hipMemcpyAsync(M->fac_order, hp[0].glob_order.data(), sizeof(int32_t) * A->n,
                         hipMemcpyHostToDevice, s) != hipSuccess)
        st = MPK_EDEVICE;
    }
    int32_t init[3] = {0, INT_MAX, INT_MAX};
    if (!st && hipMemcpyAsync(M->words, init, sizeof(init), hipMemcpyHostToDevice, s) != hipSuccess)
      st = MPK_EDEVICE;
    if (!st) {
      hipLaunchKernelGGL(promote_vals, dim3(nblocks(A->nnz)), dim3(BLOCK), 0, s, A->nnz, C, KF,
                         A->val, M->f);
      st = hipGetLastError() != hipSuccess ? MPK_EDEVICE : MPK_OK;
    }
    // the level-by-level factorisation, or on a grid the one-launch one
    if (!st)
      st = dispatch_ck(C, KF, [&]<int CC, int KK>() {
        return grid ? ilu0_grid_run<CC, KK>(*M, A->val, s) : ilu0_levels<CC, KK>(*M, s);
      });
    t0.join();
    t1.join();
    if (adj) t2.join();
    if (st) return st;
  }
  MPK_PHASE("levels, factor launch, plans (host)");
  Plan *P[4] = {&M->L, &M->U, &M->UH, &M->LH};
  for (int k = 0; k < (adj ? 4 : 2); ++k) P[k]->n = A->n;
  if ((!grid && (st = upload_plan(hp[0], M->L, s))) || (st = upload_plan(hp[1], M->U, s)))
    return st;
  M->U.div = true;
  M->L.div = false;
  M->L.kmax = M->U.kmax = M->UH.kmax = M->LH.kmax = kmax;
  if (adj) {
    // transposed pattern for the adjoint schedules: rows of A^T with the
    // source position of each entry in A's pattern
    IVec trp, tci, tsrc;
    host_transpose(h, trp, tci, tsrc);
    MPK_HIP(hipMemcpyAsync(M->t_rp, trp.data(), sizeof(int32_t) * (A->n + 1), hipMemcpyHostToDevice, s));
    MPK_HIP(hipMemcpyAsync(M->t_ci, tci.data(), sizeof(int32_t) * A->nnz, hipMemcpyHostToDevice, s));
    MPK_HIP(hipMemcpyAsync(M->t_src, tsrc.data(), sizeof(int32_t) * A->nnz, hipMemcpyHostToDevice, s));
    if ((st = upload_plan(hp[2], M->UH, s)) || (st = upload_plan(hp[3], M->LH, s))) return st;
    M->UH.div = true;
    M->LH.div = false;
    M->UH.conj = M->LH.conj = true;
    for (int k = 0; k < 4; ++k)
      if ((st = device_plan_arrays(*P[k], *M, k, s))) return st;
    MPK_HIP(hipStreamSynchronize(s));
  } else {
    for (int k = 0; k < 2; ++k)
      if ((st = device_plan_arrays(*P[k], *M, k, s))) return st;
  }
  MPK_PHASE("upload plans (after the factorisation)");
  int32_t badpiv = INT_MAX, fac_abort = 0;
  MPK_HIP(hipMemcpyAsync(&badpiv, M->words + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  if (grid)
    MPK_HIP(hipMemcpyAsync(&fac_abort, M->words + 4, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPK_HIP(hipStreamSynchronize(s));
  if (fac_abort) return MPK_EWATCHDOG;
  if (badpiv != INT_MAX) {
    if (info) info->bad_row = badpiv;
    return MPK_EZERO_PIVOT;
  }
  if ((st = gather_plan(M->L, *M, s)) || (st = gather_plan(M->U, *M, s))) return st;
  if (flags & MPK_ILU0_ADJOINT)
    if ((st = gather_plan(M->UH, *M, s)) || (st = gather_plan(M->LH, *M, s))) return st;
  MPK_HIP(hipStreamSynchronize(s));
  MPK_PHASE("gather values");
  if (info) info->setup_ms = now_ms() - t0;
  return MPK_OK;
}

int ilu0_apply_launch(const Ilu0 &M, int K, int conj, const double *r, double *z,
                      int32_t *abort_reset, int32_t *abort_flag, const int32_t *done,
                      hipStream_t s) {
  if (K < M.KF || K < 1 || K > 4) return MPK_EUNSUPPORTED;
  if (K > M.L.kmax) return MPK_EUNSUPPORTED;
  if (conj && !(M.flags & MPK_ILU0_ADJOINT)) return MPK_EUNSUPPORTED;
  return dispatch_ck(M.C, K, [&]<int C, int KK>() {
    return ilu0_apply_ck<C, KK>(M, conj, r, z, abort_reset, abort_flag, done, s);
  });
}

// --------------------------------------------------------------- dots
template <int C, int K> struct DotOp {
  const double *a, *b;
  __device__ void operator()(int64_t i, el<C, K> *d) const {
    d[0] = el_cdot_term<C, K>(el_load<C, K>(a + size_t(i) * C * K),
                              el_load<C, K>(b + size_t(i) * C * K));
  }
};

template <int C, int K>
__global__ __launch_bounds__(BLOCK) void dot_final(const double *partials, int nblk, double *out) {
  el<C, K> tot[1];
  reduce_partials<C, K, 1>(partials, nblk, tot);
  if (threadIdx.x == 0) el_store<C, K>(out, tot[0]);
}

// Fixed device scratch of the inner product that allocates nothing: the
// per-workgroup partials of one mpk_dot_noalloc call.  Every GPU the library
// runs on holds one copy until the process ends; calls on one GPU share it.
constexpr size_t DOT_SCRATCH_DOUBLES = size_t(1) << 19;  // 4 MiB
__device__ __align__(256) double dot_scratch[DOT_SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex dot_scratch_mu;
double *dot_scratch_ptr[MAX_DEVICES];

// The device address of this GPU's dot_scratch, looked up once per device
// (with that device current) on the first call.  The array's name is a
// host-side stand-in, never passed to a kernel.
int dot_scratch_address(double **out) {
  int dev = 0;
  MPK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return MPK_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(dot_scratch_mu);
  if (!dot_scratch_ptr[dev]) {
    void *p = nullptr;
    MPK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(dot_scratch)));
    if (!p) return MPK_EDEVICE;
    dot_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *out = dot_scratch_ptr[dev];
  return MPK_OK;
}

}  // namespace mpk

using namespace mpk;

extern "C" {

const char *mpk_status_str(int status) {
  switch (status) {
    case MPK_OK: return "ok";
    case MPK_NOT_CONVERGED: return "not converged (max_iter reached)";
    case MPK_BREAKDOWN: return "breakdown (a method scalar became zero)";
    case MPK_EINVAL: return "invalid argument";
    case MPK_EDEVICE: return "HIP runtime error";
    case MPK_EWORKSPACE: return "workspace missing, misaligned or too small";
    case MPK_EZERO_PIVOT: return "zero pivot in ILU(0)";
    case MPK_ENO_DIAG: return "diagonal entry not stored";
    case MPK_EUNSUPPORTED: return "unsupported combination";
    case MPK_ENONFINITE: return "non-finite matrix entry";
    case MPK_EPATTERN: return "CSR pattern not strictly ascending or out of range";
    case MPK_EWATCHDOG: return "device dependency wait exceeded its bound";
  }
  return "unknown status";
}

int mpk_version(void) { return 100; }

size_t mpk_spmv_workspace_bytes(const mpk_csr *A, int is_complex, int trans) {
  if (!A || A->n <= 0 || A->nnz < 0) return 0;
  if (!trans) return 0;
  Bump b(nullptr);
  b.take<int32_t>(size_t(A->n) + 1);
  b.take<int32_t>(size_t(A->nnz));
  b.take<int32_t>(size_t(A->nnz));
  b.take<double>(size_t(A->nnz) * (is_complex ? 2 : 1));
  return b.off;
}

static int csr_spmv(int C, mpk_prec xp, const mpk_csr *A, int trans, const double *x, double *y,
                    void *ws, size_t ws_bytes, void *stream) {
  int st = validate_csr_args(A);
  if (st) return st;
  if (xp < MPK_D || xp > MPK_QD || !x || !y) return MPK_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (!trans)
    return spmv_launch(C, int(xp), A->n, A->row_ptr, A->col_idx, A->val, x, y, nullptr, s,
                       spmv_lanes(A));
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) ||
      ws_bytes < mpk_spmv_workspace_bytes(A, C == 2, 1))
    return MPK_EWORKSPACE;
  HostCsr h;
  if ((st = fetch_pattern(A, h, s))) return st;
  int64_t bad;
  if ((st = check_pattern(h, &bad))) return st;
  IVec trp, tci, tsrc;
  host_transpose(h, trp, tci, tsrc);
  Bump b(ws);
  int32_t *d_rp = b.take<int32_t>(size_t(A->n) + 1), *d_ci = b.take<int32_t>(size_t(A->nnz)),
          *d_src = b.take<int32_t>(size_t(A->nnz));
  double *d_val = b.take<double>(size_t(A->nnz) * C);
  MPK_HIP(hipMemcpyAsync(d_rp, trp.data(), sizeof(int32_t) * (A->n + 1), hipMemcpyHostToDevice, s));
  MPK_HIP(hipMemcpyAsync(d_ci, tci.data(), sizeof(int32_t) * A->nnz, hipMemcpyHostToDevice, s));
  MPK_HIP(hipMemcpyAsync(d_src, tsrc.data(), sizeof(int32_t) * A->nnz, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(gather_vals, dim3(nblocks(A->nnz)), dim3(BLOCK), 0, s, A->nnz, C, 1, d_src,
                     A->val, d_val, C == 2 ? 1 : 0);
  MPK_HIP(hipGetLastError());
  st = spmv_launch(C, int(xp), A->n, d_rp, d_ci, d_val, x, y, nullptr, s);
  MPK_HIP(hipStreamSynchronize(s));
  return st;
}

int mpk_dcsr_spmv(mpk_prec xp, const mpk_csr *A, int trans, const double *x, double *y, void *ws,
                  size_t ws_bytes, void *stream) {
  return csr_spmv(1, xp, A, trans, x, y, ws, ws_bytes, stream);
}

int mpk_zcsr_spmv(mpk_prec xp, const mpk_csr *A, int conj_trans, const double *x, double *y,
                  void *ws, size_t ws_bytes, void *stream) {
  return csr_spmv(2, xp, A, conj_trans, x, y, ws, ws_bytes, stream);
}

size_t mpk_ilu0_workspace_bytes(const mpk_csr *A, mpk_prec fp, int is_complex, int flags) {
  if (!A || A->n <= 0 || A->nnz < 0 || fp < MPK_D || fp > MPK_QD) return 0;
  Bump b(nullptr);
  return ilu0_layout(A->n, A->nnz, is_complex ? 2 : 1, int(fp), flags, b, nullptr);
}

static int ilu0_factor(int C, mpk_prec fp, const mpk_csr *A, int flags, void *ws, size_t ws_bytes,
                       mpk_ilu0 **M, mpk_info *info, void *stream) {
  int st = validate_csr_args(A);
  if (st) return st;
  if (fp < MPK_D || fp > MPK_QD || !M || (flags & ~(MPK_ILU0_ADJOINT | (7 << 4))) ||
      ((flags >> 4) & 7) > 4 || (((flags >> 4) & 7) && ((flags >> 4) & 7) < int(fp)))
    return MPK_EINVAL;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) ||
      ws_bytes < mpk_ilu0_workspace_bytes(A, fp, C == 2, flags))
    return MPK_EWORKSPACE;
  Ilu0 *h = new Ilu0();
  st = ilu0_factor_impl(C, int(fp), A, flags, ws, ws_bytes, h, info, (hipStream_t)stream);
  if (info) info->status = st;
  if (st) {
    delete h;
    *M = nullptr;
    return st;
  }
  *M = reinterpret_cast<mpk_ilu0 *>(h);
  return MPK_OK;
}

int mpk_dilu0_factor(mpk_prec fp, const mpk_csr *A, int flags, void *ws, size_t ws_bytes,
                     mpk_ilu0 **M, mpk_info *info, void *stream) {
  return ilu0_factor(1, fp, A, flags, ws, ws_bytes, M, info, stream);
}

int mpk_zilu0_factor(mpk_prec fp, const mpk_csr *A, int flags, void *ws, size_t ws_bytes,
                     mpk_ilu0 **M, mpk_info *info, void *stream) {
  return ilu0_factor(2, fp, A, flags, ws, ws_bytes, M, info, stream);
}

static int ilu0_apply(int C, const mpk_ilu0 *Mh, mpk_prec vp, int conj_trans, const double *r,
                      double *z, void *stream) {
  const Ilu0 *M = reinterpret_cast<const Ilu0 *>(Mh);
  if (!M || !r || !z || M->C != C || vp < MPK_D || vp > MPK_QD) return MPK_EINVAL;
  return ilu0_apply_launch(*M, int(vp), conj_trans ? 1 : 0, r, z, M->words, M->words,
                           nullptr, (hipStream_t)stream);
}

int mpk_dilu0_apply(const mpk_ilu0 *M, mpk_prec vp, int conj_trans, const double *r, double *z,
                    void *stream) {
  return ilu0_apply(1, M, vp, conj_trans, r, z, stream);
}

int mpk_zilu0_apply(const mpk_ilu0 *M, mpk_prec vp, int conj_trans, const double *r, double *z,
                    void *stream) {
  return ilu0_apply(2, M, vp, conj_trans, r, z, stream);
}

void mpk_ilu0_destroy(mpk_ilu0 *M) { delete reinterpret_cast<Ilu0 *>(M); }

size_t mpk_dot_workspace_bytes(int64_t n, int is_complex, mpk_prec p) {
  if (n <= 0 || p < MPK_D || p > MPK_QD) return 0;
  Bump b(nullptr);
  b.take<double>(size_t(nblocks(n)) * (is_complex ? 2 : 1) * int(p));
  return b.off;
}

int mpk_dot(mpk_prec p, int is_complex, int64_t n, const double *a, const double *b, double *out,
            void *ws, size_t ws_bytes, void *stream) {
  if (n <= 0 || p < MPK_D || p > MPK_QD || !a || !b || !out) return MPK_EINVAL;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) ||
      ws_bytes < mpk_dot_workspace_bytes(n, is_complex, p))
    return MPK_EWORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  double *part = static_cast<double *>(ws);
  const int nb = int(nblocks(n));
  return dispatch_ck(is_complex ? 2 : 1, int(p), [&]<int C, int K>() {
    DotOp<C, K> op{a, b};
    hipLaunchKernelGGL((row_kernel<C, K, 1, DotOp<C, K>>), dim3(xcd_grid(nb)), dim3(BLOCK), 0, s, n, op,
                       (const int32_t *)nullptr, part);
    hipLaunchKernelGGL((dot_final<C, K>), dim3(1), dim3(BLOCK), 0, s, (const double *)part, nb,
                       out);
    return hipGetLastError() == hipSuccess ? MPK_OK : MPK_EDEVICE;
  });
}

size_t mpk_dot_noalloc_max_elements(int is_complex, mpk_prec p) {
  if (p < MPK_D || p > MPK_QD) return 0;
  return DOT_SCRATCH_DOUBLES / size_t((is_complex ? 2 : 1) * int(p)) * BLOCK;
}

int mpk_dot_noalloc(mpk_prec p, int is_complex, int64_t n, const double *a, const double *b,
                    double *out, void *stream) {
  if (n <= 0 || p < MPK_D || p > MPK_QD || !a || !b || !out) return MPK_EINVAL;
  if (size_t(n) > mpk_dot_noalloc_max_elements(is_complex, p)) return MPK_EWORKSPACE;
  double *part = nullptr;
  int st = dot_scratch_address(&part);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  const int nb = int(nblocks(n));
  return dispatch_ck(is_complex ? 2 : 1, int(p), [&]<int C, int K>() {
    DotOp<C, K> op{a, b};
    hipLaunchKernelGGL((row_kernel<C, K, 1, DotOp<C, K>>), dim3(xcd_grid(nb)), dim3(BLOCK), 0, s, n, op,
                       (const int32_t *)nullptr, part);
    hipLaunchKernelGGL((dot_final<C, K>), dim3(1), dim3(BLOCK), 0, s, (const double *)part, nb,
                       out);
    return hipGetLastError() == hipSuccess ? MPK_OK : MPK_EDEVICE;
  });
}

static int csr_residual(int C, mpk_prec p, const mpk_csr *A, const double *b, const double *x,
                        double *r, void *stream) {
  int st = validate_csr_args(A);
  if (st) return st;
  if (p < MPK_D || p > MPK_QD || !b || !x || !r) return MPK_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = A->n;
  return dispatch_ck(C, int(p), [&]<int CC, int KK>() {
    ResidOp<CC, KK> op{A->row_ptr, A->col_idx, A->val, b, x, r};
    hipLaunchKernelGGL((row_kernel<CC, KK, 0, ResidOp<CC, KK>>), dim3(xcd_grid(nblocks(n))),
                       dim3(BLOCK), 0, s, n, op, (const int32_t *)nullptr, (double *)nullptr);
    return hipGetLastError() == hipSuccess ? MPK_OK : MPK_EDEVICE;
  });
}

int mpk_dcsr_residual(mpk_prec p, const mpk_csr *A, const double *b, const double *x, double *r,
                      void *stream) {
  return csr_residual(1, p, A, b, x, r, stream);
}

int mpk_zcsr_residual(mpk_prec p, const mpk_csr *A, const double *b, const double *x, double *r,
                      void *stream) {
  return csr_residual(2, p, A, b, x, r, stream);
}

int mpk_spmv_set_lanes(const mpk_csr *A, int lanes) {
  if (validate_csr_args(A)) return MPK_EINVAL;
  if (!(lanes == 0 || lanes == 1 || lanes == 2 || lanes == 4 || lanes == 8 || lanes == 16))
    return MPK_EINVAL;
  std::lock_guard<std::mutex> lock(lanes_mu);
  if (lanes == 0)
    lanes_table.erase(lanes_key(A));
  else
    lanes_table[lanes_key(A)] = lanes;
  return MPK_OK;
}

int mpk_spmv_tune(mpk_prec xp, const mpk_csr *A, int is_complex, const double *x, double *y,
                  int *lanes, double *ms, void *stream) {
  if (validate_csr_args(A) || xp < MPK_D || xp > MPK_QD || !x || !y) return MPK_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int C = is_complex ? 2 : 1;
  const int cand[] = {1, 2, 4, 8, 16};
  hipEvent_t e0, e1;
  MPK_HIP(hipEventCreate(&e0));
  MPK_HIP(hipEventCreate(&e1));
  int best = 1, st = MPK_OK;
  float best_ms = 0;
  for (int k = 0; k < 5 && !st; ++k) {
    const int g = cand[k];
    float t = 0;
    st = spmv_launch(C, int(xp), A->n, A->row_ptr, A->col_idx, A->val, x, y, nullptr, s, g);
    if (!st && hipEventRecord(e0, s) != hipSuccess) st = MPK_EDEVICE;
    for (int r = 0; r < 3 && !st; ++r)
      st = spmv_launch(C, int(xp), A->n, A->row_ptr, A->col_idx, A->val, x, y, nullptr, s, g);
    if (!st && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&t, e0, e1) != hipSuccess))
      st = MPK_EDEVICE;
    if (!st && (k == 0 || t < best_ms)) {
      best_ms = t;
      best = g;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  {
    std::lock_guard<std::mutex> lock(lanes_mu);
    lanes_table[lanes_key(A)] = best;
  }
  if (lanes) *lanes = best;
  if (ms) *ms = best_ms / 3;
  return MPK_OK;
}

}  // extern "C"
