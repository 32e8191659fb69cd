// order.hip -- multicolour ordering behind the C-ABI in include/mpk.h.
//
// A labelled variant beyond the paper's method (its Section 5 leaves the
// parallelisation of the ILU(0) routines to future work): the rows are
// coloured greedily and ordered by colour, B = P A P^T is formed, and
// ILU(0) of B preconditions the solve of B y = P b, x = P^T y.  ILU(0) of
// B is a different preconditioner from ILU(0) of A.  In B a row of colour
// c has stored lower entries only in columns of colours below c, so each
// substitution has at most one level per colour, each level a set of
// independent rows.
#include <climits>

#include "kernels.hpp"

namespace mpk {

// perm checks and B's row lengths: iperm[perm[k]] = k (iperm filled with
// -1 before), bit 0 of *word when perm is out of range or repeats a row,
// bit 1 when a row of A has a negative length; cnt[k] = length of row
// perm[k] of A.
static __global__ void perm_invert(int64_t n, const int32_t *__restrict__ perm,
                                   const int32_t *__restrict__ rp, int32_t *iperm, int32_t *cnt,
                                   int32_t *word) {
  const int64_t k = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (k >= n) return;
  const int32_t p = perm[k];
  int32_t len = 0;
  if (p < 0 || p >= n) {
    atomicOr(word, 1);
  } else {
    if (atomicExch(&iperm[p], int32_t(k)) != -1) atomicOr(word, 1);
    len = rp[p + 1] - rp[p];
    if (len < 0) {
      atomicOr(word, 2);
      len = 0;
    }
  }
  cnt[k] = len;
}

static __global__ void fill_i32(int64_t n, int32_t *a, int32_t v) {
  const int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (i < n) a[i] = v;
}

// Row k of B: row perm[k] of A with its columns renamed by iperm, sorted
// by insertion (one thread per row; rows of a sparse matrix are short).
// A column outside [0, n) sets bit 1 of *word and is stored as column 0.
template <int C>
__global__ void perm_rows(int64_t n, const int32_t *__restrict__ perm,
                          const int32_t *__restrict__ iperm, const int32_t *__restrict__ rp,
                          const int32_t *__restrict__ ci, const double *__restrict__ val,
                          const int32_t *__restrict__ brp, int32_t *__restrict__ bci,
                          double *__restrict__ bval, int32_t *word) {
  const int64_t k = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (k >= n) return;
  const int32_t p = perm[k];
  const int32_t a = rp[p], len = brp[k + 1] - brp[k];
  const int64_t o = brp[k];
  for (int32_t t = 0; t < len; ++t) {
    const int32_t j = ci[a + t];
    int32_t col = 0;
    if (j < 0 || j >= n)
      atomicOr(word, 2);
    else
      col = iperm[j];
    double w[C];
#pragma unroll
    for (int c = 0; c < C; ++c) w[c] = val[int64_t(a + t) * C + c];
    int32_t q = t;
    while (q > 0 && bci[o + q - 1] > col) {
      bci[o + q] = bci[o + q - 1];
#pragma unroll
      for (int c = 0; c < C; ++c) bval[(o + q) * C + c] = bval[(o + q - 1) * C + c];
      --q;
    }
    bci[o + q] = col;
#pragma unroll
    for (int c = 0; c < C; ++c) bval[(o + q) * C + c] = w[c];
  }
}

// y[k] = x[perm[k]] (gather) or y[perm[k]] = x[k] (scatter), E doubles
// per element; one thread per double, consecutive threads on consecutive
// doubles of the side that is read or written in order.  An entry of perm
// outside [0, n) is skipped.
static __global__ void vec_perm(int64_t n, int E, const int32_t *__restrict__ perm, int inverse,
                                const double *__restrict__ x, double *__restrict__ y) {
  const int64_t t = int64_t(blockIdx.x) * BLOCK + threadIdx.x;
  if (t >= n * E) return;
  const int64_t k = t / E, e = t - k * E;
  const int64_t p = perm[k];
  if (p < 0 || p >= n) return;  // not a row: nothing is read or written
  if (inverse)
    y[p * E + e] = x[t];
  else
    y[t] = x[p * E + e];
}

static unsigned grid_for(int64_t count) {
  return unsigned((count + BLOCK - 1) / BLOCK);
}

static int csr_permute(int C, const mpk_csr *A, const int32_t *perm, int32_t *b_rp, int32_t *b_ci,
                       double *b_val, void *ws, size_t ws_bytes, void *stream);

}  // namespace mpk

using namespace mpk;

extern "C" {

int mpk_multicolor_order(const mpk_csr *A, int32_t *perm, int32_t *ncolors, void *stream) {
  int st = validate_csr_args(A);
  if (st) return st;
  if (!perm || !ncolors) return MPK_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  HostCsr h;
  if ((st = fetch_pattern(A, h, s))) return st;
  int64_t bad;
  if ((st = check_pattern(h, &bad))) return st;
  IVec color;
  const int32_t ncol = greedy_color(h, color);
  // the ordering by colour: a stable counting sort
  IVec start(size_t(ncol) + 1, 0), hperm(size_t(A->n));
  for (int64_t i = 0; i < A->n; ++i) start[color[i] + 1]++;
  for (int32_t c = 0; c < ncol; ++c) start[c + 1] += start[c];
  for (int64_t i = 0; i < A->n; ++i) hperm[start[color[i]]++] = int32_t(i);
  MPK_HIP(hipMemcpyAsync(perm, hperm.data(), sizeof(int32_t) * size_t(A->n),
                         hipMemcpyHostToDevice, s));
  MPK_HIP(hipStreamSynchronize(s));
  *ncolors = ncol;
  return MPK_OK;
}

size_t mpk_csr_permute_workspace_bytes(int64_t n) {
  if (n <= 0) return 0;
  Bump b(nullptr);
  b.take<int32_t>(size_t(n));                   // iperm
  b.take<int32_t>(size_t(n) / SCAN_BLOCK + 2);  // scan block sums
  b.take<int32_t>(4);                           // status word
  return b.off;
}

int mpk_dcsr_permute(const mpk_csr *A, const int32_t *perm, int32_t *b_row_ptr,
                     int32_t *b_col_idx, double *b_val, void *ws, size_t ws_bytes, void *stream) {
  return csr_permute(1, A, perm, b_row_ptr, b_col_idx, b_val, ws, ws_bytes, stream);
}

int mpk_zcsr_permute(const mpk_csr *A, const int32_t *perm, int32_t *b_row_ptr,
                     int32_t *b_col_idx, double *b_val, void *ws, size_t ws_bytes, void *stream) {
  return csr_permute(2, A, perm, b_row_ptr, b_col_idx, b_val, ws, ws_bytes, stream);
}

int mpk_vec_permute(mpk_prec vp, int is_complex, int64_t n, const int32_t *perm, int inverse,
                    const double *x, double *y, void *stream) {
  if (vp < MPK_D || vp > MPK_QD || n < 0 || n >= (int64_t(1) << 31) || (n > 0 && (!perm || !x || !y)))
    return MPK_EINVAL;
  if (n == 0) return MPK_OK;
  const int E = (is_complex ? 2 : 1) * int(vp);
  hipLaunchKernelGGL(vec_perm, dim3(grid_for(n * E)), dim3(BLOCK), 0, (hipStream_t)stream, n, E,
                     perm, inverse ? 1 : 0, x, y);
  MPK_HIP(hipGetLastError());
  return MPK_OK;
}

}  // extern "C"

namespace mpk {

static int csr_permute(int C, const mpk_csr *A, const int32_t *perm, int32_t *b_rp, int32_t *b_ci,
                       double *b_val, void *ws, size_t ws_bytes, void *stream) {
  int st = validate_csr_args(A);
  if (st) return st;
  if (!perm || !b_rp || !b_ci || !b_val) return MPK_EINVAL;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) ||
      ws_bytes < mpk_csr_permute_workspace_bytes(A->n))
    return MPK_EWORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = A->n;
  Bump b(ws);
  int32_t *iperm = b.take<int32_t>(size_t(n));
  int32_t *bsum = b.take<int32_t>(size_t(n) / SCAN_BLOCK + 2);
  int32_t *word = b.take<int32_t>(4);
  const unsigned g = grid_for(n);
  hipLaunchKernelGGL(fill_i32, dim3(g), dim3(BLOCK), 0, s, n, iperm, -1);
  hipLaunchKernelGGL(fill_i32, dim3(1), dim3(BLOCK), 0, s, int64_t(1), word, 0);
  hipLaunchKernelGGL(perm_invert, dim3(g), dim3(BLOCK), 0, s, n, perm, A->row_ptr, iperm, b_rp,
                     word);
  // row lengths in b_rp[0..n) become offsets, b_rp[n] the total
  const int32_t nb = int32_t((n + SCAN_BLOCK - 1) / SCAN_BLOCK);
  hipLaunchKernelGGL(scan_blocks, dim3(nb), dim3(BLOCK), 0, s, n, (const int32_t *)b_rp, b_rp,
                     bsum);
  hipLaunchKernelGGL(scan_sums, dim3(1), dim3(BLOCK), 0, s, nb, bsum);
  hipLaunchKernelGGL(scan_add, dim3(g), dim3(BLOCK), 0, s, n, b_rp, (const int32_t *)bsum, nb);
  MPK_HIP(hipGetLastError());
  int32_t chk[4] = {0, 0, 0, 0};
  MPK_HIP(hipMemcpyAsync(&chk[0], word, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPK_HIP(hipMemcpyAsync(&chk[1], b_rp + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPK_HIP(hipMemcpyAsync(&chk[2], A->row_ptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPK_HIP(hipMemcpyAsync(&chk[3], A->row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPK_HIP(hipStreamSynchronize(s));
  if (chk[0] & 1) return MPK_EINVAL;  // not a permutation
  // every row inside [0, nnz): row_ptr starts at 0, ends at nnz, no row negative
  if ((chk[0] & 2) || chk[1] != A->nnz || chk[2] != 0 || chk[3] != A->nnz) return MPK_EPATTERN;
  if (C == 1)
    hipLaunchKernelGGL(perm_rows<1>, dim3(g), dim3(BLOCK), 0, s, n, perm, (const int32_t *)iperm,
                       A->row_ptr, A->col_idx, A->val, (const int32_t *)b_rp, b_ci, b_val, word);
  else
    hipLaunchKernelGGL(perm_rows<2>, dim3(g), dim3(BLOCK), 0, s, n, perm, (const int32_t *)iperm,
                       A->row_ptr, A->col_idx, A->val, (const int32_t *)b_rp, b_ci, b_val, word);
  MPK_HIP(hipGetLastError());
  MPK_HIP(hipMemcpyAsync(&chk[0], word, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPK_HIP(hipStreamSynchronize(s));
  return (chk[0] & 2) ? MPK_EPATTERN : MPK_OK;
}

}  // namespace mpk
