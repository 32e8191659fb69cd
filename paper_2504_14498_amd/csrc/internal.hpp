// internal.hpp -- shared host/device definitions of the mpk library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <utility>
#include <vector>

#include "../../include/mpk.h"
#include "mp.hpp"

namespace mpk {

constexpr int BLOCK = 256;          // threads per workgroup for row/element kernels
constexpr int WAVE = 64;            // CDNA wavefront
constexpr int MAX_PARTIAL_BLOCKS = 8192;
constexpr int MAXE = 8;             // max doubles per element (C * K)
constexpr int ELLW = 4;             // flat dependency slots per row (blocked sweeps)

// Bit pattern marking "not yet computed" in the outputs of the sync-free
// triangular solves: a NaN payload that arithmetic never produces (stored
// results are canonicalised first).
constexpr uint64_t SENTINEL = 0x7FF4C0DE5E1A7100ull;

// Device-side status of a running solve, in workspace memory.  Every
// kernel of an iteration reads `done` first and returns if it is set, so
// work enqueued past convergence or breakdown is a no-op.
enum : int32_t { ST_RUNNING = 0, ST_CHECK_HALF = 1, ST_CHECK_FULL = 2 };

struct KState {
  double s[16][MAXE];        // method scalars (K-limb, complex layout re[K] im[K])
  double nr0sq;              // leading limb of ||r_0||^2
  double nbsq;               // leading limb of ||b||^2
  double eps_r, eps_a;
  double last_nr2;           // leading limb of the last recursive ||r||^2
  double true_nr2;           // leading limb of the last true ||b - A x||^2
  int64_t iter;              // passes started
  int64_t max_iter;
  int64_t hist_len;
  double *hist;
  int32_t done;              // 0 running; 1 finished (see status)
  int32_t status;            // MPK_OK / MPK_NOT_CONVERGED / MPK_BREAKDOWN
  int32_t phase;             // ST_RUNNING / ST_CHECK_HALF / ST_CHECK_FULL
  int32_t x_in_tmp;          // solution left in the temporary vector
  int32_t first;             // 1 during the first pass
  int32_t pad[3];
};

// Scalar slots in KState::s.
enum {
  S_RHO = 0, S_RHO_OLD, S_ALPHA, S_BETA, S_OMEGA, S_ZETA, S_ETA, S_SIGMA,
  S_D0, S_D1, S_D2, S_D3, S_D4, S_D5, S_D6, S_D7
};

// Bump allocator over the caller's workspace.  With base == nullptr it only
// measures, so the same layout code sizes and carves the workspace.
struct Bump {
  char *base;
  size_t off;
  explicit Bump(void *b) : base(static_cast<char *>(b)), off(0) {}
  template <class T> T *take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += sizeof(T) * (count ? count : 1);
    return p;
  }
};

// Block geometry of the blocked sweeps.  A block is t ranges of w
// consecutive rows, one range in each of t consecutive periods of P rows:
// the rows z * P + a with z in [bz * t, bz * t + t) and a in
// [ba * w, ba * w + w), a < P.  Blocks are numbered bz * nch + ba (nch
// chunks per period), which is the forward sweep's processing order.  A
// row's LDS slot in its block is (z mod t) * w + (a mod w).  With t = 1
// and P = n a block is a plain range of w consecutive rows.  On a grid
// numbered plane by plane, P = one plane and t > 1 gives blocks a few
// planes deep, so a dependency chain through the grid crosses fewer
// blocks.  w and t are powers of two.
struct BlockGeom {
  int64_t P = 1;    // period (rows)
  int32_t w = 1;    // rows of one range
  int32_t t = 1;    // ranges (periods) per block
  int64_t nch = 1;  // chunks per period: ceil(P / w)
  __host__ __device__ int64_t block(int64_t i) const {
    const int64_t z = i / P, a = i - z * P;
    return (z / t) * nch + a / w;
  }
  __host__ __device__ int32_t slot(int64_t i) const {
    const int64_t z = i / P, a = i - z * P;
    return int32_t((z % t) * w + a % w);
  }
};

// A dependency-ordered schedule for one triangular sweep: rows grouped by
// level; `seg` splits each level into runs of at most WAVE rows (the work
// unit of one wavefront, free of internal dependencies).
// Grid of a grid sweep (mode 3): nx x ny x nz points numbered x fastest
// (nz = 1 in 2D), cut into nby x nbz blocks of lines.
struct GridDims {
  int32_t nx = 0, ny = 0, nz = 0;
  int32_t nby = 0, nbz = 0;
};

struct Plan {
  int64_t n = 0, nnz = 0;      // rows, dependency entries
  int32_t nlev = 0, nseg = 0;
  int32_t *order = nullptr;    // [n] row at each position
  int32_t *ptr = nullptr;      // [n+1] entry range of each position
  int32_t *col = nullptr;      // [nnz] dependency column
  int32_t *src = nullptr;      // [nnz] index of the value in A's pattern
  int32_t *dsrc = nullptr;     // [n] diagonal position (division plans)
  int32_t *seg = nullptr;      // [nseg+1] first position of each segment
  int32_t *seg_level = nullptr;  // [nseg] level of each segment
  int32_t *lev_size = nullptr;   // [nlev] rows per level
  int32_t *lev_done = nullptr;   // [nlev] rows of each level finished (per sweep)
  double *val = nullptr;       // [nnz * C * KF] gathered factor values
  double *dval = nullptr;      // [n * C * KF] gathered pivots
  int32_t *sync = nullptr;     // [0] ticket, [1] watchdog abort
  // blocked schedule (mode 1): contiguous row blocks in processing order,
  // each with its own local levels; positions are block-major
  int32_t mode = 0;            // 0 level schedule, 1 blocked schedule, 2 one launch per level,
                               // 3 grid sweep
  // grid sweep (mode 3): the grid and the lines per block in y (8 in 3D,
  // 64 in 2D); ell_val holds each row's factor record (4 slots)
  GridDims grid;
  int32_t grid_by = 0;
  int32_t nblk = 0, nloc = 0;  // blocks, local levels in total
  int32_t kmax = 4;            // largest vector precision the blocks are sized for
  int32_t blk_rows = 0;        // LDS slots per block (t * w)
  int32_t max_piece = 0;       // rows of the widest local level piece
  BlockGeom geom;              // block shape
  int32_t *blk_r = nullptr;    // [2*nblk] first range [r0, r1) of each block
  int32_t *blk_lev = nullptr;  // [nblk+1] first local level of each block
  int32_t *loc_pos = nullptr;  // [nloc+1] first position of each local level
  // rows that rows of other blocks read from memory (blocked schedule):
  // the only ones polled, so the only ones given the sentinel and stored
  // as soon as they are finished; the other rows reach memory when their
  // block ends
  int32_t *xflag = nullptr;    // [n] 1 if read by another block
  int32_t *xlist = nullptr;    // [nx] those rows
  int64_t nx = 0;
  // flat per-position dependency slots (blocked schedule): up to ELLW
  // dependencies of the row at position pos live at [pos * ELLW + d]
  int32_t *ell_nd = nullptr;   // [n] dependencies of each position
  int32_t *ell_col = nullptr;  // [n * ELLW] column j, or -(slot + 1) if j is in the row's block
  int32_t *ell_meta = nullptr; // [n * 4] row, dependency count, LDS slot, 0 (blocked sweeps)
  int32_t *ell_src = nullptr;  // [n * ELLW] value source in A's pattern (-1 pad)
  double *ell_val = nullptr;   // [n * ELLW * C * KF]
  std::vector<int32_t> h_blk;  // host copies kept alive for the uploads
  std::vector<int32_t> h_ell;
  std::vector<int32_t> h_levptr;   // level boundaries (host)
  std::vector<int32_t> h_levsize;  // level sizes (host copy kept alive for the upload)
  bool div = false, conj = false;
};

struct Ilu0 {
  int64_t n = 0, nnz = 0;
  int C = 1, KF = 1;
  int flags = 0;
  const int32_t *row_ptr = nullptr, *col_idx = nullptr;
  int32_t *diag = nullptr;     // [n]
  double *f = nullptr;         // [nnz * C * KF] factor in A's pattern
  Plan L, U, UH, LH;
  double *tmp = nullptr;       // [n * C * 4] intermediate of an apply
  int32_t *fac_order = nullptr;  // [n] rows by global forward level (factorisation)
  int32_t *scan_tmp = nullptr;   // [n / 1024 + 2] block sums of the schedule scans
  int32_t *t_rp = nullptr, *t_ci = nullptr, *t_src = nullptr;  // A^T pattern (adjoint)
  std::vector<int32_t> h_fac_levptr;
  int32_t *words = nullptr;    // device: [0] abort of standalone applies,
                               // [1] zero-pivot row, [2] non-finite row
};

// Host launchers shared by the C-ABI and the solvers (ops.hip).
size_t ilu0_layout(int64_t n, int64_t nnz, int C, int KF, int flags, Bump &b, Ilu0 *M);
int ilu0_factor_impl(int C, int KF, const mpk_csr *A, int flags, void *ws, size_t ws_bytes,
                     Ilu0 *M, mpk_info *info, hipStream_t s);
// Re-gather the sweep plans' values after the factor values in A's pattern
// changed (same pattern).
int ilu0_regather(const Ilu0 &M, hipStream_t s);
// Defined in apply.hpp, instantiated for every (C, K) in apply_c<C>k<K>.hip.
template <int C, int K>
int ilu0_apply_ck(const Ilu0 &M, int conj, const double *r, double *z, int32_t *abort_reset,
                  int32_t *abort_flag, const int32_t *done, hipStream_t s);
int ilu0_apply_launch(const Ilu0 &M, int K, int conj, const double *r, double *z,
                      int32_t *abort_reset, int32_t *abort_flag, const int32_t *done,
                      hipStream_t s);
int spmv_launch(int C, int K, int64_t n, const int32_t *rp, const int32_t *ci, const double *val,
                const double *x, double *y, const int32_t *done, hipStream_t s,
                int lanes = 1);
// Lanes per row of the standalone SpMV chosen for A (1 unless set or tuned).
int spmv_lanes(const mpk_csr *A);
int validate_csr_args(const mpk_csr *A);
int csr_check_device_values(const mpk_csr *A, int C, int32_t *word, int64_t *bad_row,
                            hipStream_t s);
inline unsigned nblocks(int64_t n) { return unsigned((n + BLOCK - 1) / BLOCK); }

// Workgroups are dispatched to the 8 XCDs in turn.  Row kernels renumber
// them so that each XCD walks one contiguous range of row blocks: rows that
// share x values (stencil neighbours) then meet in the same L2.  The grid
// is padded to a multiple of 8; padding blocks do nothing.
constexpr unsigned NXCD = 8;
inline unsigned xcd_grid(unsigned nb) { return (nb + NXCD - 1) / NXCD * NXCD; }
__device__ __forceinline__ int64_t xcd_block() {
  const unsigned b = blockIdx.x, per = gridDim.x / NXCD;
  return int64_t(b % NXCD) * per + b / NXCD;
}
double now_ms();

// Launch error check for host code.
#define MPK_HIP(call)                                  \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return MPK_EDEVICE;          \
  } while (0)

template <class F> int dispatch_ck(int C, int K, F &&f) {
  switch (C * 10 + K) {
    case 11: return f.template operator()<1, 1>();
    case 12: return f.template operator()<1, 2>();
    case 13: return f.template operator()<1, 3>();
    case 14: return f.template operator()<1, 4>();
    case 21: return f.template operator()<2, 1>();
    case 22: return f.template operator()<2, 2>();
    case 23: return f.template operator()<2, 3>();
    case 24: return f.template operator()<2, 4>();
  }
  return MPK_EINVAL;
}

// Host-side CSR checks and schedules (analysis.cpp).
// Host index arrays that are overwritten at once: allocated without the
// zero fill of std::vector<int32_t>::resize.
template <class T> struct NoInitAlloc : std::allocator<T> {
  template <class U> struct rebind { using other = NoInitAlloc<U>; };
  NoInitAlloc() = default;
  template <class U> NoInitAlloc(const NoInitAlloc<U> &) {}
  template <class U, class... A> void construct(U *p, A &&...a) {
    if constexpr (sizeof...(A) == 0)
      ::new (static_cast<void *>(p)) U;
    else
      ::new (static_cast<void *>(p)) U(std::forward<A>(a)...);
  }
};
using IVec = std::vector<int32_t, NoInitAlloc<int32_t>>;

// A CSR pattern on the host.  rp/ci point either into own_rp/own_ci or
// into the calling thread's page-locked staging buffer (fetch_pattern),
// which stays valid until that thread's next fetch.
struct HostCsr {
  int64_t n = 0, nnz = 0;
  const int32_t *rp = nullptr, *ci = nullptr;
  IVec own_rp, own_ci;
  void own() {
    rp = own_rp.data();
    ci = own_ci.data();
  }
};
int fetch_pattern(const mpk_csr *A, HostCsr &h, hipStream_t s);
int check_pattern(const HostCsr &h, int64_t *bad_row);
void host_diag(const HostCsr &h, std::vector<int32_t> &diag);

struct HostPlan {
  std::vector<int32_t> order, ptr, col, src, dsrc, seg, seg_level, levptr;
  int32_t nlev = 0;
  int32_t mode = 0, nblk = 0, blk_rows = 0, max_piece = 0;
  BlockGeom geom;
  std::vector<int32_t> blk_r, blk_lev, loc_pos;
  std::vector<int32_t> glob_order, glob_levptr;  // global level order (factorisation)
  GridDims grid;                 // grid sweep (mode 3)
  int32_t grid_by = 0;
  std::vector<int32_t> xlist;    // grid sweep: rows read by later blocks
};
// kind: 0 = L (strict lower of rows, forward), 1 = U (strict upper, backward,
// divides), 2 = U^H (columns of the upper part, forward, divides),
// 3 = L^H (columns of the strict lower part, backward).
// ht: the transposed pattern (needed for kinds 2 and 3 only).
void build_plan(const HostCsr &h, const HostCsr *ht, int kind, int blk_rows, HostPlan &p);
// The parts of build_plan: the schedule choice (plan_mode, whose result
// goes to p.mode first); global levels where needed (the factorisation
// order of kind 0, the level schedule); the blocked schedule when it was
// chosen.  With p.mode set, the last two touch different fields of p and
// may run on different threads.
int plan_mode(const HostCsr &h, const HostCsr *ht, int kind, int blk_rows);
// The pattern is the 7-point (3D) or 5-point (2D) stencil of an nx x ny x
// nz grid numbered x fastest (every row stores exactly its neighbours
// inside the grid): the L and U sweeps can be grid sweeps (mode 3).
// The extents of a grid numbered x fastest from the stored columns of its
// last row (lower neighbours at strides 1, nx and nx ny); false when they do
// not describe a 2D or 3D grid.
bool grid_dims_from_last_row(int64_t n, const int32_t *cols, int64_t len, int32_t &nx,
                             int32_t &ny, int32_t &nz);
bool detect_grid(const HostCsr &h, int32_t &nx, int32_t &ny, int32_t &nz);
// Grid sweep plan of the L (kind 0) or U (kind 1) sweep: block counts and
// the rows that later blocks read (p.mode = 3 and the grid set before).
void build_plan_grid(int64_t n, int kind, HostPlan &p);
// The forward levels of a grid (row (x, y, z) is on level x + y + z) and
// the rows in level order, ascending within a level: the factorisation's
// order, without a pass over the pattern.
void grid_levels(const GridDims &g, std::vector<int32_t> &levptr, std::vector<int32_t> &order);
void build_plan_levels(const HostCsr &h, const HostCsr *ht, int kind, int blk_rows,
                       HostPlan &p);
void build_plan_blocks(const HostCsr &h, const HostCsr *ht, int kind, int blk_rows,
                       HostPlan &p);
int default_block_rows(int C, int kmax);
size_t plan_bytes(int64_t n, int64_t nnz_bound, int C, int KF, bool div, Bump &b, Plan *out);
int upload_plan(const HostPlan &hp, Plan &p, hipStream_t s);

// Transposed pattern with source map (for A^T / A^H products).
void host_transpose(const HostCsr &h, IVec &trp, IVec &tci, IVec &tsrc);

// Greedy colouring of the graph of A + A^T in natural order (row i takes
// the smallest colour no adjacent row j < i has); returns the number of
// colours.
int32_t greedy_color(const HostCsr &h, IVec &color);

}  // namespace mpk
