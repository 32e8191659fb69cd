// apply.hpp -- launch of the two sweeps of one ILU(0) apply (Algorithm 2,
// or the M^H solve of Algorithm 3) for one element type: the kernels of
// kernels.hpp instantiated per (components, limbs); each pair is compiled
// in its own translation unit (apply_c<C>k<K>.hip) so the library builds
// in parallel.
#pragma once
#include <algorithm>
#include <cstdlib>

#include "kernels.hpp"

namespace mpk {

template <int C, int K, int KF, bool DIV, bool CONJ>
inline void launch_trsv(const Plan &P, const double *rhs, double *out, int32_t *abort_flag,
                        const int32_t *done, hipStream_t s) {
  if constexpr (!CONJ) {
    if (P.mode == 3) {
      // grid sweep: the forward one for L, the backward one (dividing) for U
      static const int64_t gcap = [] {
        const char *e = getenv("MPK_TRSV_GGRID");
        return e ? std::max<int64_t>(1, atoll(e)) : int64_t(512);
      }();
      const unsigned grid = unsigned(std::max<int64_t>(1, std::min<int64_t>(P.nblk, gcap)));
      // the block's results staged in LDS when they fit
      const size_t lds = grid_lds_bytes(P.grid.nx, C * K);
      const bool stage = lds <= GRID_LDS_MAX;
      auto go = [&]<int BY, bool ST>() {
        hipLaunchKernelGGL((trsv_grid<C, K, KF, DIV, BY, ST>), dim3(grid), dim3(WAVE),
                           ST ? lds : 0, s, P.n, P.grid, (const double *)P.ell_val, rhs, out,
                           P.sync, abort_flag, done);
      };
      if (P.grid_by == 8) {
        if (stage)
          go.template operator()<8, true>();
        else
          go.template operator()<8, false>();
      } else {
        if (stage)
          go.template operator()<64, true>();
        else
          go.template operator()<64, false>();
      }
      return;
    }
  }
  if (P.mode == 2) {
    // one launch per level, in order
    for (int32_t l = 0; l < P.nlev; ++l) {
      const int32_t a = P.h_levptr[l], cnt = P.h_levptr[l + 1] - a;
      if (cnt <= 0) continue;
      hipLaunchKernelGGL((trsv_level<C, K, KF, DIV, CONJ>), dim3((cnt + BLOCK - 1) / BLOCK),
                         dim3(BLOCK), 0, s, a, cnt, P.order, P.ptr, P.col, P.val, P.dval, rhs,
                         out, done);
    }
    return;
  }
  if (P.mode == 1) {
    static const int64_t bcap = [] {
      const char *e = getenv("MPK_TRSV_BGRID");
      return e ? std::max<int64_t>(1, atoll(e)) : int64_t(512);
    }();
    const unsigned grid = unsigned(std::min<int64_t>(P.nblk, bcap));
    const size_t lds = size_t(P.blk_rows + 1) * C * K * sizeof(double);
    static const bool one_wave = [] {
      const char *e = getenv("MPK_TRSV_ONE_WAVE");
      return !e || e[0] != '0';
    }();
    if (one_wave && P.max_piece <= WAVE)
      hipLaunchKernelGGL((trsv_blocked<C, K, KF, DIV, CONJ, WAVE>), dim3(grid ? grid : 1),
                         dim3(WAVE), lds, s, P.n, P.ptr, P.col, P.val, P.dval, P.blk_r,
                         P.blk_lev, P.loc_pos, P.nblk, P.ell_col, P.ell_meta,
                         P.ell_val, P.blk_rows, P.geom.P, P.geom.w, P.geom.t, rhs, out, P.sync,
                         abort_flag, done);
    else
      hipLaunchKernelGGL((trsv_blocked<C, K, KF, DIV, CONJ, BLOCK>), dim3(grid ? grid : 1),
                         dim3(BLOCK), lds, s, P.n, P.ptr, P.col, P.val, P.dval, P.blk_r,
                         P.blk_lev, P.loc_pos, P.nblk, P.ell_col, P.ell_meta,
                         P.ell_val, P.blk_rows, P.geom.P, P.geom.w, P.geom.t, rhs, out, P.sync,
                         abort_flag, done);
    return;
  }
  static const int64_t cap = [] {
    const char *e = getenv("MPK_TRSV_GRID");
    return e ? std::max<int64_t>(1, atoll(e)) : int64_t(512);
  }();
  static const int32_t xcd = [] {
    const char *e = getenv("MPK_TRSV_XCD");
    return e ? std::max(1, atoi(e)) : 1;
  }();
  const unsigned grid = unsigned(std::min<int64_t>((P.nseg + 3) / 4, cap)) * unsigned(xcd);
  hipLaunchKernelGGL((trsv_syncfree<C, K, KF, DIV, CONJ>), dim3(grid ? grid : 1), dim3(BLOCK), 0,
                     s, P.order, P.ptr, P.col, P.val, P.dval, P.seg, P.seg_level, P.nseg,
                     P.lev_size, P.lev_done, rhs, out, P.sync, abort_flag, done, xcd);
}

template <int C, int K, int KF>
inline int apply_ckf(const Ilu0 &M, int conj, const double *r, double *z, int32_t *abort_reset,
                     int32_t *abort_flag, const int32_t *done, hipStream_t s) {
  const Plan &P1 = conj ? M.UH : M.L;
  const Plan &P2 = conj ? M.LH : M.U;
  // blocked and grid sweeps poll only listed rows; level-synchronous
  // sweeps (mode 2) poll nothing
  const bool x1 = P1.mode == 1 || P1.mode == 3, x2 = P2.mode == 1 || P2.mode == 3;
  const int32_t *l1 = x1 ? P1.xlist : nullptr, *l2 = x2 ? P2.xlist : nullptr;
  const int64_t c1 = x1 ? P1.nx : (P1.mode == 2 ? 0 : M.n),
                c2 = x2 ? P2.nx : (P2.mode == 2 ? 0 : M.n);
  const int64_t cover = std::max<int64_t>(std::max(c1, c2) * C * K, std::max(P1.nlev, P2.nlev));
  hipLaunchKernelGGL(trsv_prep, dim3(nblocks(std::max<int64_t>(cover, 1))), dim3(BLOCK), 0, s,
                     C * K, l1, c1, M.tmp, l2, c2, z, P1.nlev, P1.lev_done, P2.nlev, P2.lev_done,
                     P1.sync, P2.sync, abort_reset, done);
  if (!conj) {
    launch_trsv<C, K, KF, false, false>(P1, r, M.tmp, abort_flag, done, s);
    launch_trsv<C, K, KF, true, false>(P2, M.tmp, z, abort_flag, done, s);
  } else {
    launch_trsv<C, K, KF, true, true>(P1, r, M.tmp, abort_flag, done, s);
    launch_trsv<C, K, KF, false, true>(P2, M.tmp, z, abort_flag, done, s);
  }
  return hipGetLastError() == hipSuccess ? MPK_OK : MPK_EDEVICE;
}

// z = M^{-1} r (or M^{-H} r) for vectors of C components of K limbs, with
// the factor's own limb count.
template <int C, int K>
int ilu0_apply_ck(const Ilu0 &M, int conj, const double *r, double *z, int32_t *abort_reset,
                  int32_t *abort_flag, const int32_t *done, hipStream_t s) {
  if constexpr (K >= 4) {
    if (M.KF == 4) return apply_ckf<C, K, 4>(M, conj, r, z, abort_reset, abort_flag, done, s);
  }
  if constexpr (K >= 3) {
    if (M.KF == 3) return apply_ckf<C, K, 3>(M, conj, r, z, abort_reset, abort_flag, done, s);
  }
  if constexpr (K >= 2) {
    if (M.KF == 2) return apply_ckf<C, K, 2>(M, conj, r, z, abort_reset, abort_flag, done, s);
  }
  return apply_ckf<C, K, 1>(M, conj, r, z, abort_reset, abort_flag, done, s);
}

}  // namespace mpk
