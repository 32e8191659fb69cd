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

#include "internal.hpp"

namespace mpk {

int fetch_pattern(const mpk_csr *A, HostCsr &h, hipStream_t s) {
  h.n = A->n;
  h.nnz = A->nnz;
  h.rp.resize(size_t(A->n) + 1);
  h.ci.resize(size_t(std::max<int64_t>(A->nnz, 1)));
  MPK_HIP(hipMemcpyAsync(h.rp.data(), A->row_ptr, sizeof(int32_t) * (A->n + 1),
                         hipMemcpyDeviceToHost, s));
  if (A->nnz > 0)
    MPK_HIP(hipMemcpyAsync(h.ci.data(), A->col_idx, sizeof(int32_t) * A->nnz,
                           hipMemcpyDeviceToHost, s));
  MPK_HIP(hipStreamSynchronize(s));
  return MPK_OK;
}

int check_pattern(const HostCsr &h, int64_t *bad_row) {
  *bad_row = -1;
  if (h.rp[0] != 0 || h.rp[h.n] != h.nnz) return MPK_EPATTERN;
  for (int64_t i = 0; i < h.n; ++i) {
    int32_t a = h.rp[i], b = h.rp[i + 1];
    if (b < a) {
      *bad_row = i;
      return MPK_EPATTERN;
    }
    bool diag = false;
    for (int32_t p = a; p < b; ++p) {
      int32_t j = h.ci[p];
      if (j < 0 || j >= h.n || (p > a && j <= h.ci[p - 1])) {
        *bad_row = i;
        return MPK_EPATTERN;
      }
      diag |= (j == i);
    }
    if (!diag) {
      *bad_row = i;
      return MPK_ENO_DIAG;
    }
  }
  return MPK_OK;
}

void host_diag(const HostCsr &h, std::vector<int32_t> &diag) {
  diag.assign(size_t(h.n), -1);
  for (int64_t i = 0; i < h.n; ++i)
    for (int32_t p = h.rp[i]; p < h.rp[i + 1]; ++p)
      if (h.ci[p] == i) diag[i] = p;
}

void host_transpose(const HostCsr &h, std::vector<int32_t> &trp, std::vector<int32_t> &tci,
                    std::vector<int32_t> &tsrc) {
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

// Rows per block of the blocked schedule: the block's results live in LDS,
// at most 128 KiB for quad-double (K = 4).
int default_block_rows(int C, int kmax) {
  const char *e = getenv("MPK_TRSV_BLOCK_ROWS");
  if (e) return std::max(64, atoi(e));
  // largest power of two with rows * C * kmax doubles within 128 KiB
  int rows = 64;
  while (int64_t(rows) * 2 * C * kmax * 8 <= 131072) rows *= 2;
  return rows;
}

void build_plan(const HostCsr &h, const std::vector<int32_t> &diag, int kind, int blk_rows,
                HostPlan &p) {
  const int64_t n = h.n;
  // dependency lists per row: (column, source position), ascending column
  std::vector<int32_t> dptr(size_t(n) + 1, 0), dcol, dsrcv;
  if (kind == 0 || kind == 1) {
    for (int64_t i = 0; i < n; ++i) {
      int cnt = 0;
      for (int32_t q = h.rp[i]; q < h.rp[i + 1]; ++q)
        if (kind == 0 ? h.ci[q] < i : h.ci[q] > i) ++cnt;
      dptr[i + 1] = dptr[i] + cnt;
    }
    dcol.resize(size_t(dptr[n]) + 1);
    dsrcv.resize(size_t(dptr[n]) + 1);
    for (int64_t i = 0; i < n; ++i) {
      int32_t o = dptr[i];
      for (int32_t q = h.rp[i]; q < h.rp[i + 1]; ++q)
        if (kind == 0 ? h.ci[q] < i : h.ci[q] > i) {
          dcol[o] = h.ci[q];
          dsrcv[o] = q;
          ++o;
        }
    }
  } else {
    std::vector<int32_t> trp, tci, tsrc;
    host_transpose(h, trp, tci, tsrc);
    for (int64_t i = 0; i < n; ++i) {
      int cnt = 0;
      for (int32_t q = trp[i]; q < trp[i + 1]; ++q)
        if (kind == 2 ? tci[q] < i : tci[q] > i) ++cnt;
      dptr[i + 1] = dptr[i] + cnt;
    }
    dcol.resize(size_t(dptr[n]) + 1);
    dsrcv.resize(size_t(dptr[n]) + 1);
    for (int64_t i = 0; i < n; ++i) {
      int32_t o = dptr[i];
      for (int32_t q = trp[i]; q < trp[i + 1]; ++q)
        if (kind == 2 ? tci[q] < i : tci[q] > i) {
          dcol[o] = tci[q];
          dsrcv[o] = tsrc[q];
          ++o;
        }
    }
  }
  const bool forward = (kind == 0 || kind == 2);
  std::vector<int32_t> lvl(size_t(n), 0);
  int32_t nlev = n > 0 ? 1 : 0;
  for (int64_t t = 0; t < n; ++t) {
    int64_t i = forward ? t : n - 1 - t;
    int32_t l = 0;
    for (int32_t q = dptr[i]; q < dptr[i + 1]; ++q) l = std::max(l, lvl[dcol[q]] + 1);
    lvl[i] = l;
    nlev = std::max(nlev, l + 1);
  }
  // blocked schedule: blocks of blk_rows consecutive rows, taken in the
  // sweep's direction; used when most dependencies stay inside a block
  p.mode = 0;
  {
    int64_t internal = 0, total = dptr[n];
    for (int64_t i = 0; i < n; ++i)
      for (int32_t q = dptr[i]; q < dptr[i + 1]; ++q)
        internal += (dcol[q] / blk_rows) == (i / blk_rows);
    const char *e = getenv("MPK_TRSV_MODE");
    if (e && e[0] == 'b')
      p.mode = 1;
    else if (e && e[0] == 'l')
      p.mode = 0;
    else
      p.mode = (total > 0 && 2 * internal >= total) ? 1 : 0;
  }
  if (kind == 0) {
    // the factorisation walks the global forward levels
    p.glob_levptr.assign(size_t(nlev) + 1, 0);
    for (int64_t i = 0; i < n; ++i) p.glob_levptr[lvl[i] + 1]++;
    for (int32_t l = 0; l < nlev; ++l) p.glob_levptr[l + 1] += p.glob_levptr[l];
    p.glob_order.resize(size_t(std::max<int64_t>(n, 1)));
    std::vector<int32_t> next(p.glob_levptr.begin(), p.glob_levptr.end() - 1);
    for (int64_t i = 0; i < n; ++i) p.glob_order[next[lvl[i]]++] = int32_t(i);
  }
  if (p.mode == 1) {
    p.blk_rows = blk_rows;
    p.nblk = int32_t((n + blk_rows - 1) / blk_rows);
    p.blk_r.assign(size_t(2) * p.nblk, 0);
    p.blk_lev.assign(size_t(p.nblk) + 1, 0);
    p.loc_pos.clear();
    p.order.clear();
    std::vector<int32_t> loc(size_t(blk_rows), 0);
    for (int32_t b = 0; b < p.nblk; ++b) {
      // processing order: ascending blocks forward, descending backward
      const int32_t nb = forward ? b : p.nblk - 1 - b;
      const int64_t r0 = int64_t(nb) * blk_rows, r1 = std::min<int64_t>(n, r0 + blk_rows);
      p.blk_r[2 * b] = int32_t(r0);
      p.blk_r[2 * b + 1] = int32_t(r1);
      int32_t nl = 1;
      for (int64_t t = 0; t < r1 - r0; ++t) {
        const int64_t i = forward ? r0 + t : r1 - 1 - t;
        int32_t l = 0;
        for (int32_t q = dptr[i]; q < dptr[i + 1]; ++q) {
          const int32_t j = dcol[q];
          if (j >= r0 && j < r1) l = std::max(l, loc[j - r0] + 1);
        }
        loc[i - r0] = l;
        nl = std::max(nl, l + 1);
      }
      p.blk_lev[b] = int32_t(p.loc_pos.size());
      std::vector<int32_t> cnt(size_t(nl) + 1, 0);
      for (int64_t i = r0; i < r1; ++i) cnt[loc[i - r0] + 1]++;
      for (int32_t l = 0; l < nl; ++l) cnt[l + 1] += cnt[l];
      const int32_t base = int32_t(p.order.size());
      for (int32_t l = 0; l < nl; ++l) p.loc_pos.push_back(base + cnt[l]);
      p.order.resize(size_t(base) + size_t(r1 - r0));
      for (int64_t i = r0; i < r1; ++i) p.order[base + cnt[loc[i - r0]]++] = int32_t(i);
    }
    p.blk_lev[p.nblk] = int32_t(p.loc_pos.size());
    p.loc_pos.push_back(int32_t(n));
    p.nlev = nlev;
    p.levptr.assign(2, 0);
    p.levptr[1] = int32_t(n);
    p.seg.assign(1, int32_t(n));
    p.seg_level.assign(1, 0);
    goto fill;
  }
  p.nlev = nlev;
  p.levptr.assign(size_t(nlev) + 1, 0);
  for (int64_t i = 0; i < n; ++i) p.levptr[lvl[i] + 1]++;
  for (int32_t l = 0; l < nlev; ++l) p.levptr[l + 1] += p.levptr[l];
  p.order.resize(size_t(std::max<int64_t>(n, 1)));
  {
    std::vector<int32_t> next(p.levptr.begin(), p.levptr.end() - 1);
    for (int64_t i = 0; i < n; ++i) p.order[next[lvl[i]]++] = int32_t(i);
  }
  p.seg.clear();
  p.seg_level.clear();
  for (int32_t l = 0; l < nlev; ++l)
    for (int32_t s = p.levptr[l]; s < p.levptr[l + 1]; s += WAVE) {
      p.seg.push_back(s);
      p.seg_level.push_back(l);
    }
  p.seg.push_back(int32_t(n));
fill:
  p.ptr.assign(size_t(n) + 1, 0);
  for (int64_t pos = 0; pos < n; ++pos) {
    int32_t i = p.order[pos];
    p.ptr[pos + 1] = p.ptr[pos] + (dptr[i + 1] - dptr[i]);
  }
  p.col.resize(size_t(p.ptr[n]) + 1);
  p.src.resize(size_t(p.ptr[n]) + 1);
  for (int64_t pos = 0; pos < n; ++pos) {
    int32_t i = p.order[pos];
    int32_t o = p.ptr[pos];
    for (int32_t q = dptr[i]; q < dptr[i + 1]; ++q, ++o) {
      p.col[o] = dcol[q];
      p.src[o] = dsrcv[q];
    }
  }
  if (p.mode == 1) {
    p.ell_nd.assign(size_t(std::max<int64_t>(n, 1)), 0);
    p.ell_col.assign(size_t(std::max<int64_t>(n, 1)) * ELLW, 0);
    p.ell_src.assign(size_t(std::max<int64_t>(n, 1)) * ELLW, -1);
    for (int64_t pos = 0; pos < n; ++pos) {
      const int32_t a = p.ptr[pos], e = p.ptr[pos + 1];
      p.ell_nd[pos] = e - a;
      for (int32_t d = 0; d < ELLW && a + d < e; ++d) {
        p.ell_col[pos * ELLW + d] = p.col[a + d];
        p.ell_src[pos * ELLW + d] = p.src[a + d];
      }
    }
  }
  p.dsrc.clear();
  if (kind == 1 || kind == 2) {
    p.dsrc.resize(size_t(std::max<int64_t>(n, 1)));
    for (int64_t pos = 0; pos < n; ++pos) p.dsrc[pos] = diag[p.order[pos]];
  }
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
  p.ell_src = b.take<int32_t>(size_t(n) * ELLW);
  p.ell_val = b.take<double>(size_t(n) * ELLW * C * KF);
  p.blk_r = b.take<int32_t>(2 * size_t(n) + 2);
  p.blk_lev = b.take<int32_t>(size_t(n) + 1);
  p.loc_pos = b.take<int32_t>(size_t(n) + 1);
  p.div = div;
  return b.off;
}

int upload_plan(const HostPlan &hp, Plan &p, hipStream_t s) {
  const int64_t n = int64_t(hp.ptr.size()) - 1;
  p.n = n;
  p.nnz = hp.ptr[n];
  p.nlev = hp.nlev;
  p.nseg = int32_t(hp.seg.size()) - 1;
  p.h_levptr = hp.levptr;
  p.mode = hp.mode;
  p.nblk = hp.nblk;
  p.blk_rows = hp.blk_rows;
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
    MPK_HIP(hipMemcpyAsync(p.ell_nd, hp.ell_nd.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    MPK_HIP(hipMemcpyAsync(p.ell_col, hp.ell_col.data(), sizeof(int32_t) * n * ELLW,
                           hipMemcpyHostToDevice, s));
    MPK_HIP(hipMemcpyAsync(p.ell_src, hp.ell_src.data(), sizeof(int32_t) * n * ELLW,
                           hipMemcpyHostToDevice, s));
  }
  MPK_HIP(hipMemcpyAsync(p.order, hp.order.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
  MPK_HIP(hipMemcpyAsync(p.ptr, hp.ptr.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, s));
  if (p.nnz > 0) {
    MPK_HIP(hipMemcpyAsync(p.col, hp.col.data(), sizeof(int32_t) * p.nnz, hipMemcpyHostToDevice, s));
    MPK_HIP(hipMemcpyAsync(p.src, hp.src.data(), sizeof(int32_t) * p.nnz, hipMemcpyHostToDevice, s));
  }
  MPK_HIP(hipMemcpyAsync(p.seg, hp.seg.data(), sizeof(int32_t) * hp.seg.size(),
                         hipMemcpyHostToDevice, s));
  MPK_HIP(hipMemcpyAsync(p.seg_level, hp.seg_level.data(), sizeof(int32_t) * hp.seg_level.size(),
                         hipMemcpyHostToDevice, s));
  {
    std::vector<int32_t> sz(size_t(hp.nlev) + 1, 0);
    for (int32_t l = 0; l < hp.nlev; ++l) sz[l] = hp.levptr[l + 1] - hp.levptr[l];
    p.h_levsize = sz;
    MPK_HIP(hipMemcpyAsync(p.lev_size, p.h_levsize.data(), sizeof(int32_t) * sz.size(),
                           hipMemcpyHostToDevice, s));
  }
  if (p.div && n > 0)
    MPK_HIP(hipMemcpyAsync(p.dsrc, hp.dsrc.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
  return MPK_OK;
}

}  // namespace mpk
