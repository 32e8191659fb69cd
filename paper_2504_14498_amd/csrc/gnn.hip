// gnn.hip -- learned correction to the ILU(0) factor: a small message-passing
// network on A's sparsity graph (nodes = rows, edges = stored entries in CSR
// order), its training kernels, the factor loss and the guarded correction.
//
// The paper has no learned part: the network is defined on top of its
// ILU(0) (Alg. 1) and Krylov methods (Sec. 3) and must leave their arithmetic
// alone.  Hidden width 32, three layers; weights are float32 (master copy),
// activations are stored as bfloat16; the dense per-edge and per-node layers
// run on MFMA (bf16 inputs with float32 accumulation forward, float32 inputs
// backward); gathers and segment sums are plain HBM-bound loops.
//
// Layer l (h: node states, e: edge states, q = (i, j)):
//   z_q = Wm [h_i; h_j; e_q] + bm,  m_q = R(relu(z_q)),
//   g_i = R(mean_{q in row i} m_q),  u_i = Wu [h_i; g_i] + bu,
//   h_i <- R(h_i + relu(u_i)),  e_q <- R(e_q + m_q)
// with R() round-to-nearest-even to bf16; encoders are 4 -> 32 float32
// affine maps with relu, the decoder a float32 dot of [h_i; h_j; e_q].

#include <cmath>

#include "internal.hpp"

namespace mpk {
namespace {

constexpr int HID = 32;
constexpr int NLAYER = 3;
constexpr int FN = 4, FE = 4;
constexpr double C_OFF = 0.5;
constexpr double PIVOT_MIN = 1e-8, PIVOT_MAX = 1e8;

// parameter offsets (float32, row-major [out][in])
constexpr int P_WN = 0;
constexpr int P_BN = P_WN + HID * FN;
constexpr int P_WE = P_BN + HID;
constexpr int P_BE = P_WE + HID * FE;
constexpr int P_L0 = P_BE + HID;
constexpr int L_WM = 0;
constexpr int L_BM = L_WM + HID * 3 * HID;
constexpr int L_WU = L_BM + HID;
constexpr int L_BU = L_WU + HID * 2 * HID;
constexpr int L_SIZE = L_BU + HID;
constexpr int P_WD = P_L0 + NLAYER * L_SIZE;
constexpr int P_BD = P_WD + 3 * HID;
constexpr int NPARAM = P_BD + 1;

constexpr int GRID_MAX = 1024;          // persistent grid of the tile kernels
constexpr int NWAVE_MAX = GRID_MAX * (BLOCK / WAVE);
constexpr int PART_MAX = HID * 3 * HID + HID;  // largest weight group (Wm + bm)

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }
__device__ __forceinline__ float bf2f(short h) { return bf2f(uint16_t(h)); }
__device__ __forceinline__ bf4 ld4(const uint16_t *p) { return *reinterpret_cast<const bf4 *>(p); }
__device__ __forceinline__ void st4(uint16_t *p, bf4 v) { *reinterpret_cast<bf4 *>(p) = v; }
__device__ __forceinline__ f4 ldf4(const float *p) { return *reinterpret_cast<const f4 *>(p); }
__device__ __forceinline__ void stf4(float *p, f4 v) { *reinterpret_cast<f4 *>(p) = v; }
__device__ __forceinline__ float rbf(float w) { return bf2f(f2bf(w)); }  // weight as used by MFMA

// ---- graph, activations and loss workspaces -----------------------------

struct GGraph {
  int32_t *row = nullptr;    // [E] row of each edge
  int32_t *t_rp = nullptr;   // [n+1] edges ending at each node ...
  int32_t *t_src = nullptr;  // [E] ... as positions in CSR order
  int32_t *diag = nullptr;   // [n] diagonal position
  float *x = nullptr;        // [n][FN] node inputs
  float *y = nullptr;        // [E][FE] edge inputs
};

size_t graph_layout(int64_t n, int64_t E, Bump &b, GGraph *G) {
  GGraph t;
  GGraph &g = G ? *G : t;
  g.row = b.take<int32_t>(size_t(E));
  g.t_rp = b.take<int32_t>(size_t(n) + 1);
  g.t_src = b.take<int32_t>(size_t(E));
  g.diag = b.take<int32_t>(size_t(n));
  g.x = b.take<float>(size_t(n) * FN);
  g.y = b.take<float>(size_t(E) * FE);
  return b.off;
}

struct GWork {
  uint16_t *h[NLAYER + 1];   // [n][HID] node states
  uint16_t *e[NLAYER + 1];   // [E][HID] edge states
  uint16_t *m[NLAYER];       // [E][HID] messages
  uint16_t *g[NLAYER];       // [n][HID] aggregates
  uint16_t *r[NLAYER];       // [n][HID] relu(u) (its sign is the backward mask)
  float *dh, *dh2, *dg, *du; // [n][HID]
  float *de, *dz, *ci, *cj;  // [E][HID]
  float *part;               // [NWAVE_MAX][PART_MAX] per-wave partial sums
};

size_t work_layout(int64_t n, int64_t E, Bump &b, GWork *W) {
  GWork t;
  GWork &w = W ? *W : t;
  for (int l = 0; l <= NLAYER; ++l) {
    w.h[l] = b.take<uint16_t>(size_t(n) * HID);
    w.e[l] = b.take<uint16_t>(size_t(E) * HID);
  }
  for (int l = 0; l < NLAYER; ++l) {
    w.m[l] = b.take<uint16_t>(size_t(E) * HID);
    w.g[l] = b.take<uint16_t>(size_t(n) * HID);
    w.r[l] = b.take<uint16_t>(size_t(n) * HID);
  }
  w.dh = b.take<float>(size_t(n) * HID);
  w.dh2 = b.take<float>(size_t(n) * HID);
  w.dg = b.take<float>(size_t(n) * HID);
  w.du = b.take<float>(size_t(n) * HID);
  w.de = b.take<float>(size_t(E) * HID);
  w.dz = b.take<float>(size_t(E) * HID);
  w.ci = b.take<float>(size_t(E) * HID);
  w.cj = b.take<float>(size_t(E) * HID);
  w.part = b.take<float>(size_t(NWAVE_MAX) * PART_MAX);
  return b.off;
}

struct LWork {
  double *aw, *y, *e, *gy;   // [P][n]
  double *coef;              // [P]
  double *part;              // [nblk][2P]
};

size_t loss_layout(int64_t n, int P, Bump &b, LWork *L) {
  LWork t;
  LWork &w = L ? *L : t;
  w.aw = b.take<double>(size_t(P) * n);
  w.y = b.take<double>(size_t(P) * n);
  w.e = b.take<double>(size_t(P) * n);
  w.gy = b.take<double>(size_t(P) * n);
  w.coef = b.take<double>(size_t(P));
  w.part = b.take<double>(size_t(nblocks(n)) * 2 * P);
  return b.off;
}

unsigned tile_grid(int64_t rows) {
  const int64_t tiles = (rows + 15) / 16;
  const int64_t blocks = (tiles + (BLOCK / WAVE) - 1) / (BLOCK / WAVE);
  return unsigned(std::max<int64_t>(1, std::min<int64_t>(blocks, GRID_MAX)));
}

// ---- inputs ---------------------------------------------------------------

__global__ void node_inputs(int64_t n, const int32_t *rp, const double *val, const double *f,
                            const int32_t *diag, float *x) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t d = diag[i];
  const double aii = fabs(val[d]), uii = fabs(f[d]);
  double off = 0.0;
  for (int32_t q = rp[i]; q < rp[i + 1]; ++q) off += q == d ? 0.0 : fabs(val[q]);
  x[i * FN + 0] = float(log(aii));
  x[i * FN + 1] = float(off / aii);
  x[i * FN + 2] = float(log(uii / aii));
  x[i * FN + 3] = float(double(rp[i + 1] - rp[i]) / 8.0);
}

__global__ void edge_inputs(int64_t E, const int32_t *row, const int32_t *ci, const double *val,
                            const double *f, const int32_t *diag, float *y) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= E) return;
  const int32_t i = row[q], j = ci[q];
  const double aii = fabs(val[diag[i]]);
  y[q * FE + 0] = float(val[q] / aii);
  y[q * FE + 1] = float(j < i ? f[q] : f[q] / aii);
  y[q * FE + 2] = j < i ? 1.0f : 0.0f;
  y[q * FE + 3] = j > i ? 1.0f : 0.0f;
}

// ---- forward ----------------------------------------------------------------

// out[r][o] = R(relu(b[o] + sum_k W[o][k] in[r][k])) for a 4-input encoder
__global__ void encode(int64_t rows, const float *in, const float *W, const float *bias,
                       uint16_t *out) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= rows * HID) return;
  const int64_t r = t / HID;
  const int o = int(t % HID);
  float acc = bias[o];
  for (int k = 0; k < 4; ++k) acc = fmaf(W[o * 4 + k], in[r * 4 + k], acc);
  out[t] = f2bf(acc > 0.0f ? acc : 0.0f);
}

// One wavefront per tile of 16 edges: z^T = Wm X^T on MFMA (A = weights in
// registers, B = the gathered [h_i; h_j; e_q] rows), then bias, relu and the
// bf16 stores of m and of the new edge state.
__global__ __launch_bounds__(BLOCK) void edge_layer(int64_t E, const int32_t *row,
                                                   const int32_t *col, const uint16_t *h,
                                                   const uint16_t *e_in, const float *W,
                                                   const float *bias, uint16_t *m_out,
                                                   uint16_t *e_out) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int r16 = lane & 15, g4 = lane >> 4;
  const int64_t wave = (int64_t(blockIdx.x) * BLOCK + threadIdx.x) / WAVE;
  const int64_t nwave = int64_t(gridDim.x) * (BLOCK / WAVE);
  bf4 wa[2][6];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int s = 0; s < 6; ++s)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        wa[t][s][u] = short(f2bf(W[(16 * t + r16) * (3 * HID) + 16 * s + 4 * g4 + u]));
  float bo[2][4];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) bo[t][v] = bias[16 * t + 4 * g4 + v];
  const int64_t ntile = (E + 15) / 16;
  for (int64_t tile = wave; tile < ntile; tile += nwave) {
    const int64_t q = tile * 16 + r16;
    const bool ok = q < E;
    const int64_t qc = ok ? q : E - 1;
    const int64_t i = row[qc], j = col[qc];
    bf4 b[6];
    b[0] = ld4(h + i * HID + 4 * g4);
    b[1] = ld4(h + i * HID + 16 + 4 * g4);
    b[2] = ld4(h + j * HID + 4 * g4);
    b[3] = ld4(h + j * HID + 16 + 4 * g4);
    b[4] = ld4(e_in + qc * HID + 4 * g4);
    b[5] = ld4(e_in + qc * HID + 16 + 4 * g4);
    f4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int s = 0; s < 6; ++s)
#pragma unroll
      for (int t = 0; t < 2; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[t][s], b[s], acc[t], 0, 0, 0);
    if (ok) {
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int o = 16 * t + 4 * g4;
        const bf4 eo = ld4(e_in + q * HID + o);
        bf4 mo, en;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float z = acc[t][v] + bo[t][v];
          const uint16_t mb = f2bf(z > 0.0f ? z : 0.0f);
          mo[v] = short(mb);
          en[v] = short(f2bf(bf2f(eo[v]) + bf2f(mb)));
        }
        st4(m_out + q * HID + o, mo);
        st4(e_out + q * HID + o, en);
      }
    }
  }
}

// One wavefront per tile of 16 nodes: the mean of the row's messages (in
// CSR order, float32), then u^T = Wu [h; g]^T on MFMA, relu, residual add.
__global__ __launch_bounds__(BLOCK) void node_layer(int64_t n, const int32_t *rp,
                                                   const uint16_t *h, const uint16_t *m,
                                                   const float *W, const float *bias,
                                                   uint16_t *g_out, uint16_t *r_out,
                                                   uint16_t *h_out) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int r16 = lane & 15, g4 = lane >> 4;
  const int64_t wave = (int64_t(blockIdx.x) * BLOCK + threadIdx.x) / WAVE;
  const int64_t nwave = int64_t(gridDim.x) * (BLOCK / WAVE);
  bf4 wa[2][4];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        wa[t][s][u] = short(f2bf(W[(16 * t + r16) * (2 * HID) + 16 * s + 4 * g4 + u]));
  float bo[2][4];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) bo[t][v] = bias[16 * t + 4 * g4 + v];
  const int64_t ntile = (n + 15) / 16;
  for (int64_t tile = wave; tile < ntile; tile += nwave) {
    const int64_t i = tile * 16 + r16;
    const bool ok = i < n;
    const int64_t ic = ok ? i : n - 1;
    bf4 b[4];
    b[0] = ld4(h + ic * HID + 4 * g4);
    b[1] = ld4(h + ic * HID + 16 + 4 * g4);
    float s0[4] = {0.f, 0.f, 0.f, 0.f}, s1[4] = {0.f, 0.f, 0.f, 0.f};
    const int32_t q0 = rp[ic], q1 = rp[ic + 1];
    for (int32_t q = q0; q < q1; ++q) {
      const bf4 a0 = ld4(m + int64_t(q) * HID + 4 * g4);
      const bf4 a1 = ld4(m + int64_t(q) * HID + 16 + 4 * g4);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        s0[v] += bf2f(a0[v]);
        s1[v] += bf2f(a1[v]);
      }
    }
    const float deg = float(q1 - q0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      b[2][v] = short(f2bf(s0[v] / deg));
      b[3][v] = short(f2bf(s1[v] / deg));
    }
    f4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 2; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[t][s], b[s], acc[t], 0, 0, 0);
    if (ok) {
      st4(g_out + i * HID + 4 * g4, b[2]);
      st4(g_out + i * HID + 16 + 4 * g4, b[3]);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int o = 16 * t + 4 * g4;
        const bf4 ho = ld4(h + i * HID + o);
        bf4 ro, hn;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float u = acc[t][v] + bo[t][v];
          const float ru = u > 0.0f ? u : 0.0f;
          ro[v] = short(f2bf(ru));
          hn[v] = short(f2bf(bf2f(ho[v]) + ru));
        }
        st4(r_out + i * HID + o, ro);
        st4(h_out + i * HID + o, hn);
      }
    }
  }
}

__global__ void decode(int64_t E, const int32_t *row, const int32_t *col, const uint16_t *h,
                       const uint16_t *e, const float *wd, const float *bd, float *delta) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= E) return;
  const int64_t i = row[q], j = col[q];
  float acc = bd[0];
  for (int k = 0; k < HID; ++k) acc = fmaf(wd[k], bf2f(h[i * HID + k]), acc);
  for (int k = 0; k < HID; ++k) acc = fmaf(wd[HID + k], bf2f(h[j * HID + k]), acc);
  for (int k = 0; k < HID; ++k) acc = fmaf(wd[2 * HID + k], bf2f(e[q * HID + k]), acc);
  delta[q] = acc;
}

// ---- backward -----------------------------------------------------------------

// Decoder: de[q] = g_q wd[64:96]; dh[i] = wd[0:32] sum_{row i} g + wd[32:64] sum_{col i} g
__global__ void decode_bwd_edges(int64_t E, const float *gd, const float *wd, float *de) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= E * HID) return;
  de[t] = gd[t / HID] * wd[2 * HID + int(t % HID)];
}

__global__ void decode_bwd_nodes(int64_t n, const int32_t *rp, const int32_t *t_rp,
                                 const int32_t *t_src, const float *gd, const float *wd,
                                 float *dh) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * HID) return;
  const int64_t i = t / HID;
  const int k = int(t % HID);
  float sr = 0.0f, sc = 0.0f;
  for (int32_t q = rp[i]; q < rp[i + 1]; ++q) sr += gd[q];
  for (int32_t p = t_rp[i]; p < t_rp[i + 1]; ++p) sc += gd[t_src[p]];
  dh[t] = wd[k] * sr + wd[HID + k] * sc;
}

// Per-block partial sums over a chunk of edges of g_q [h_i; h_j; e_q; 1]
__global__ void decode_bwd_weights(int64_t E, const int32_t *row, const int32_t *col,
                                   const uint16_t *h, const uint16_t *e, const float *gd,
                                   float *part) {
  const int k = threadIdx.x;  // 0..96
  const int64_t per = (E + gridDim.x - 1) / gridDim.x;
  const int64_t q0 = int64_t(blockIdx.x) * per, q1 = std::min<int64_t>(E, q0 + per);
  if (k > 3 * HID) return;
  float acc = 0.0f;
  for (int64_t q = q0; q < q1; ++q) {
    float xv;
    if (k < HID) xv = bf2f(h[int64_t(row[q]) * HID + k]);
    else if (k < 2 * HID) xv = bf2f(h[int64_t(col[q]) * HID + k - HID]);
    else if (k < 3 * HID) xv = bf2f(e[q * HID + k - 2 * HID]);
    else xv = 1.0f;
    acc = fmaf(gd[q], xv, acc);
  }
  part[int64_t(blockIdx.x) * (3 * HID + 1) + k] = acc;
}

// out[e] = sum over parts p (in order) of part[p * stride + e]
__global__ void reduce_parts(int64_t nparts, int stride, int count, const float *part,
                             float *out) {
  const int e = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= count) return;
  float s = 0.0f;
  for (int64_t p = 0; p < nparts; ++p) s += part[p * stride + e];
  out[e] = s;
}

// du = dh * [r > 0]
__global__ void node_du(int64_t n, const float *dh, const uint16_t *r, float *du) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * HID) return;
  du[t] = bf2f(r[t]) > 0.0f ? dh[t] : 0.0f;
}

// dz = (de + dg_i / deg_i) * [m > 0]
__global__ void edge_dz(int64_t E, const int32_t *rp, const int32_t *row, const float *de,
                        const float *dg, const uint16_t *m, float *dz) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= E * HID) return;
  const int64_t q = t / HID;
  const int k = int(t % HID);
  const int64_t i = row[q];
  const float deg = float(rp[i + 1] - rp[i]);
  dz[t] = bf2f(m[t]) > 0.0f ? de[t] + dg[i * HID + k] / deg : 0.0f;
}

// Where the 16-column groups of a layer's input gradient go: out[c] (row
// stride HID), plus add[c] when given (may alias out[c]: each lane reads its
// own elements before it writes them).
struct DxOut {
  float *out[6];
  const float *add[6];
};

// Input gradient of a 32-output layer on MFMA (float32):  dX^T = W^T dY^T for
// a tile of 16 rows; W [32][NIN] rounded to bf16 as in the forward, dY
// [rows][32].
template <int NIN>
__global__ __launch_bounds__(BLOCK) void layer_dx(int64_t rows, const float *W, const float *dY,
                                                 DxOut o) {
  constexpr int NC = NIN / 16;
  const int lane = threadIdx.x & (WAVE - 1);
  const int r16 = lane & 15, g4 = lane >> 4;
  const int64_t wave = (int64_t(blockIdx.x) * BLOCK + threadIdx.x) / WAVE;
  const int64_t nwave = int64_t(gridDim.x) * (BLOCK / WAVE);
  // A[r][k] = W[k][r]: lane holds r = 16c + r16, k = 4s + g4
  float wa[NC][8];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int s = 0; s < 8; ++s) wa[c][s] = rbf(W[(4 * s + g4) * NIN + 16 * c + r16]);
  const int64_t ntile = (rows + 15) / 16;
  for (int64_t tile = wave; tile < ntile; tile += nwave) {
    const int64_t q = tile * 16 + r16;
    const bool ok = q < rows;
    const int64_t qc = ok ? q : rows - 1;
    float b[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) b[s] = ok ? dY[qc * HID + 4 * s + g4] : 0.0f;
    f4 acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      acc[c] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 8; ++s)
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[c][s], b[s], acc[c], 0, 0, 0);
    }
    if (ok) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        // lane holds dX[q][16c + 4 g4 + v], v = 0..3
        f4 v = acc[c];
        if (o.add[c]) v = v + ldf4(o.add[c] + q * HID + 4 * g4);
        stf4(o.out[c] + q * HID + 4 * g4, v);
      }
    }
  }
}

// The input rows of a layer as 16-column groups of bf16 sources: group c is
// src[c][idx[c] ? idx[c][r] : r][off[c] .. off[c] + 15].
struct DwIn {
  const uint16_t *src[6];
  const int32_t *idx[6];
  int off[6];
};

// Weight gradient of a 32-output layer on MFMA (float32): per wavefront, the
// sum over its row tiles of dY^T [X | 1] (the ones column gives the bias),
// written to its own slot of `part` as [o][NIN] followed by [o].
template <int NIN>
__global__ __launch_bounds__(BLOCK) void layer_dw(int64_t rows, const float *dY, DwIn x,
                                                 float *part) {
  constexpr int NC = NIN / 16;
  const int lane = threadIdx.x & (WAVE - 1);
  const int r16 = lane & 15, g4 = lane >> 4;
  const int64_t wave = (int64_t(blockIdx.x) * BLOCK + threadIdx.x) / WAVE;
  const int64_t nwave = int64_t(gridDim.x) * (BLOCK / WAVE);
  f4 acc[2][NC + 1];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int c = 0; c <= NC; ++c) acc[t][c] = f4{0.f, 0.f, 0.f, 0.f};
  const int64_t ntile = (rows + 15) / 16;
  for (int64_t tile = wave; tile < ntile; tile += nwave) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      // the k index of this step is the row tile*16 + 4s + g4
      const int64_t r = tile * 16 + 4 * s + g4;
      const bool ok = r < rows;
      const int64_t rc = ok ? r : rows - 1;
      float a[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) a[t] = ok ? dY[rc * HID + 16 * t + r16] : 0.0f;
      float b[NC + 1];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int64_t src = x.idx[c] ? int64_t(x.idx[c][rc]) : rc;
        b[c] = bf2f(x.src[c][src * HID + x.off[c] + r16]);
      }
      b[NC] = r16 == 0 ? 1.0f : 0.0f;
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int c = 0; c <= NC; ++c)
          acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], b[c], acc[t][c], 0, 0, 0);
    }
  }
  // D[o = 16t + 4g4 + v][col = 16c + r16]
  float *P = part + wave * PART_MAX;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int o = 16 * t + 4 * g4 + v;
#pragma unroll
      for (int c = 0; c < NC; ++c) P[o * NIN + 16 * c + r16] = acc[t][c][v];
      if (r16 == 0) P[HID * NIN + o] = acc[t][NC][v];
    }
}

// dh_new[i] = dh_mid[i] + sum_{q in row i} ci[q] + sum_{q in col i} cj[q]
__global__ void node_gather(int64_t n, const int32_t *rp, const int32_t *t_rp,
                            const int32_t *t_src, const float *dh_mid, const float *ci,
                            const float *cj, float *dh_new) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * HID) return;
  const int64_t i = t / HID;
  const int k = int(t % HID);
  float s = dh_mid[t];
  for (int32_t q = rp[i]; q < rp[i + 1]; ++q) s += ci[int64_t(q) * HID + k];
  for (int32_t p = t_rp[i]; p < t_rp[i + 1]; ++p) s += cj[int64_t(t_src[p]) * HID + k];
  dh_new[t] = s;
}

// Encoder weights: per block, sum over a chunk of rows of dz[r][o] [x[r]; 1]
__global__ void encode_bwd(int64_t rows, const float *dY, const uint16_t *hout, const float *x,
                           float *part) {
  const int t = threadIdx.x;  // o * 5 + k
  if (t >= HID * 5) return;
  const int o = t / 5, k = t % 5;
  const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = int64_t(blockIdx.x) * per, r1 = std::min<int64_t>(rows, r0 + per);
  float acc = 0.0f;
  for (int64_t r = r0; r < r1; ++r) {
    const float dz = bf2f(hout[r * HID + o]) > 0.0f ? dY[r * HID + o] : 0.0f;
    acc = fmaf(dz, k < 4 ? x[r * 4 + k] : 1.0f, acc);
  }
  // weights [o][4] then bias [o]
  part[int64_t(blockIdx.x) * (HID * 5) + (k < 4 ? o * 4 + k : HID * 4 + o)] = acc;
}

// ---- Adam -----------------------------------------------------------------------

__global__ void adam_step(int64_t count, float lr, float b1, float b2, float eps, float c1,
                          float c2, float *p, const float *g, float *m, float *v) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const float gt = g[t];
  const float mt = b1 * m[t] + (1.0f - b1) * gt;
  const float vt = b2 * v[t] + (1.0f - b2) * gt * gt;
  m[t] = mt;
  v[t] = vt;
  p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

// ---- factor loss (float64) -------------------------------------------------------

__device__ __forceinline__ double corr_value(double f, float d, bool diag) {
  const double dd = double(d);
  return diag ? f * exp(dd) : f * (1.0 + C_OFF * tanh(dd));
}

// Aw = A w, y = U~ w for every probe
__global__ void loss_upper(int64_t n, int P, const int32_t *rp, const int32_t *ci,
                           const double *val, const double *f, const float *delta,
                           const double *w, double *aw, double *y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int p = 0; p < P; ++p) {
    const double *wp = w + int64_t(p) * n;
    double sa = 0.0, sy = 0.0;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
      const int32_t j = ci[q];
      sa += val[q] * wp[j];
      if (j >= i) sy += corr_value(f[q], delta[q], j == i) * wp[j];
    }
    aw[int64_t(p) * n + i] = sa;
    y[int64_t(p) * n + i] = sy;
  }
}

// e = A w - L~ y; per-block partial sums of ||e||^2 and ||A w||^2
__global__ void loss_lower(int64_t n, int P, const int32_t *rp, const int32_t *ci,
                           const double *f, const float *delta, const double *aw,
                           const double *y, double *e, double *part) {
  __shared__ double red[BLOCK];
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (int p = 0; p < P; ++p) {
    double ee = 0.0, aa = 0.0;
    if (i < n) {
      const double *yp = y + int64_t(p) * n;
      double z = yp[i];
      for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        const int32_t j = ci[q];
        if (j < i) z += corr_value(f[q], delta[q], false) * yp[j];
      }
      const double a = aw[int64_t(p) * n + i];
      const double ev = a - z;
      e[int64_t(p) * n + i] = ev;
      ee = ev * ev;
      aa = a * a;
    }
    for (int which = 0; which < 2; ++which) {
      red[threadIdx.x] = which ? aa : ee;
      __syncthreads();
      for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
      }
      if (threadIdx.x == 0) part[int64_t(blockIdx.x) * 2 * P + 2 * p + which] = red[0];
      __syncthreads();
    }
  }
}

__global__ void loss_scalar(int64_t nblk, int P, const double *part, double *coef,
                            double *loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double tot = 0.0;
  for (int p = 0; p < P; ++p) {
    double ee = 0.0, aa = 0.0;
    for (int64_t b = 0; b < nblk; ++b) {
      ee += part[b * 2 * P + 2 * p];
      aa += part[b * 2 * P + 2 * p + 1];
    }
    tot += ee / aa;
    coef[p] = -2.0 / (aa * P);
  }
  loss[0] = tot / P;
}

// gy = L~^T gz with gz = coef e (columns of the strict lower part through the
// transposed pattern)
__global__ void loss_gy(int64_t n, int P, const int32_t *t_rp, const int32_t *t_src,
                        const int32_t *row, const double *f, const float *delta,
                        const double *coef, const double *e, double *gy) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int p = 0; p < P; ++p) {
    const double *ep = e + int64_t(p) * n;
    double s = coef[p] * ep[j];
    for (int32_t t = t_rp[j]; t < t_rp[j + 1]; ++t) {
      const int32_t q = t_src[t];
      const int32_t i = row[q];
      if (i > j) s += corr_value(f[q], delta[q], false) * (coef[p] * ep[i]);
    }
    gy[int64_t(p) * n + j] = s;
  }
}

__global__ void loss_grad(int64_t E, int P, int64_t n, const int32_t *row, const int32_t *ci,
                          const double *f, const float *delta, const double *coef,
                          const double *e, const double *y, const double *gy, const double *w,
                          float *gd) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= E) return;
  const int32_t i = row[q], j = ci[q];
  double s = 0.0;
  for (int p = 0; p < P; ++p) {
    const int64_t o = int64_t(p) * n;
    s += j < i ? (coef[p] * e[o + i]) * y[o + j] : gy[o + i] * w[o + j];
  }
  const double d = double(delta[q]);
  double dv;
  if (j == i) {
    dv = f[q] * exp(d);
  } else {
    const double th = tanh(d);
    dv = f[q] * C_OFF * (1.0 - th * th);
  }
  gd[q] = float(s * dv);
}

// ---- guarded correction ------------------------------------------------------------

// row of CSR position q (binary search in row_ptr)
__device__ __forceinline__ int64_t row_of(const int32_t *rp, int64_t n, int64_t q) {
  int64_t lo = 0, hi = n;  // rp[lo] <= q < rp[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (rp[mid] <= q) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ void correct_check(int64_t E, const int32_t *rp, int64_t n, const int32_t *ci,
                              const double *f, const float *delta, int32_t *flag) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= E) return;
  const bool dg = row_of(rp, n, q) == ci[q];
  const double d = double(delta[q]);
  const double v = corr_value(f[q], delta[q], dg);
  bool bad = !isfinite(d) || !isfinite(v);
  if (dg && !bad) {
    const double ratio = exp(d);
    bad = !(ratio >= PIVOT_MIN && ratio <= PIVOT_MAX);
  }
  if (bad) atomicOr(flag, 1);
}

__global__ void correct_apply(int64_t E, const int32_t *rp, int64_t n, const int32_t *ci,
                              double *f, const float *delta) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= E) return;
  f[q] = corr_value(f[q], delta[q], row_of(rp, n, q) == ci[q]);
}

__global__ void edge_rows(int64_t n, const int32_t *rp, int32_t *row) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int32_t q = rp[i]; q < rp[i + 1]; ++q) row[q] = int32_t(i);
}

inline unsigned nb(int64_t work) { return unsigned((work + BLOCK - 1) / BLOCK); }

// host-side parameter initialisation: splitmix64 stream, uniform in
// [-1/sqrt(fan_in), 1/sqrt(fan_in)] for weights, zero biases, zero decoder
uint64_t splitmix(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void init_block(std::vector<float> &p, int off, int rows, int cols, uint64_t &s) {
  const double a = 1.0 / std::sqrt(double(cols));
  for (int k = 0; k < rows * cols; ++k) {
    const double u = double(splitmix(s) >> 11) * 0x1.0p-53;
    p[size_t(off + k)] = float((2.0 * u - 1.0) * a);
  }
}

}  // namespace

}  // namespace mpk

using namespace mpk;

namespace {

int check_graph_args(const mpk_csr *A, const void *graph, size_t graph_bytes) {
  if (validate_csr_args(A) || !graph) return MPK_EINVAL;
  if (reinterpret_cast<uintptr_t>(graph) & 255) return MPK_EWORKSPACE;
  Bump b(nullptr);
  if (graph_layout(A->n, A->nnz, b, nullptr) > graph_bytes) return MPK_EWORKSPACE;
  return MPK_OK;
}

GGraph graph_of(const mpk_csr *A, const void *graph) {
  GGraph G;
  Bump b(const_cast<void *>(graph));
  graph_layout(A->n, A->nnz, b, &G);
  return G;
}

}  // namespace

extern "C" {

int64_t mpk_gnn_param_count(void) { return NPARAM; }

int mpk_gnn_init(float *params, uint64_t seed, void *stream) {
  if (!params) return MPK_EINVAL;
  std::vector<float> p(size_t(NPARAM), 0.0f);
  uint64_t s = seed;
  init_block(p, P_WN, HID, FN, s);
  init_block(p, P_WE, HID, FE, s);
  for (int l = 0; l < NLAYER; ++l) {
    init_block(p, P_L0 + l * L_SIZE + L_WM, HID, 3 * HID, s);
    init_block(p, P_L0 + l * L_SIZE + L_WU, HID, 2 * HID, s);
  }
  hipStream_t st = (hipStream_t)stream;
  MPK_HIP(hipMemcpyAsync(params, p.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice, st));
  MPK_HIP(hipStreamSynchronize(st));
  return MPK_OK;
}

size_t mpk_gnn_graph_bytes(const mpk_csr *A) {
  if (!A || A->n <= 0 || A->nnz < 0) return 0;
  Bump b(nullptr);
  return graph_layout(A->n, A->nnz, b, nullptr);
}

int mpk_gnn_graph_setup(const mpk_csr *A, const mpk_ilu0 *Mh, void *graph, size_t graph_bytes,
                        void *stream) {
  int st = check_graph_args(A, graph, graph_bytes);
  if (st) return st;
  const Ilu0 *M = reinterpret_cast<const Ilu0 *>(Mh);
  if (!M) return MPK_EINVAL;
  if (M->C != 1 || M->KF != 1) return MPK_EUNSUPPORTED;
  if (M->n != A->n || M->nnz != A->nnz || M->row_ptr != A->row_ptr || M->col_idx != A->col_idx)
    return MPK_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  GGraph G = graph_of(A, graph);
  HostCsr h;
  if ((st = fetch_pattern(A, h, s))) return st;
  IVec trp, tci, tsrc;
  host_transpose(h, trp, tci, tsrc);
  MPK_HIP(hipMemcpyAsync(G.t_rp, trp.data(), sizeof(int32_t) * (A->n + 1), hipMemcpyHostToDevice,
                         s));
  if (A->nnz > 0)
    MPK_HIP(hipMemcpyAsync(G.t_src, tsrc.data(), sizeof(int32_t) * A->nnz, hipMemcpyHostToDevice,
                           s));
  MPK_HIP(hipMemcpyAsync(G.diag, M->diag, sizeof(int32_t) * A->n, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(edge_rows, dim3(nb(A->n)), dim3(BLOCK), 0, s, A->n, A->row_ptr, G.row);
  hipLaunchKernelGGL(node_inputs, dim3(nb(A->n)), dim3(BLOCK), 0, s, A->n, A->row_ptr, A->val,
                     (const double *)M->f, (const int32_t *)G.diag, G.x);
  if (A->nnz > 0)
    hipLaunchKernelGGL(edge_inputs, dim3(nb(A->nnz)), dim3(BLOCK), 0, s, A->nnz,
                       (const int32_t *)G.row, A->col_idx, A->val, (const double *)M->f,
                       (const int32_t *)G.diag, G.y);
  MPK_HIP(hipGetLastError());
  MPK_HIP(hipStreamSynchronize(s));
  return MPK_OK;
}

size_t mpk_gnn_workspace_bytes(const mpk_csr *A) {
  if (!A || A->n <= 0 || A->nnz < 0) return 0;
  Bump b(nullptr);
  return work_layout(A->n, A->nnz, b, nullptr);
}

int mpk_gnn_forward(const mpk_csr *A, const void *graph, const float *params, float *delta,
                    void *ws, size_t ws_bytes, void *stream) {
  if (!params || !delta) return MPK_EINVAL;
  int st = check_graph_args(A, graph, ~size_t(0));
  if (st) return st;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) || ws_bytes < mpk_gnn_workspace_bytes(A))
    return MPK_EWORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = A->n, E = A->nnz;
  const GGraph G = graph_of(A, graph);
  GWork W;
  Bump b(ws);
  work_layout(n, E, b, &W);
  hipLaunchKernelGGL(encode, dim3(nb(n * HID)), dim3(BLOCK), 0, s, n, (const float *)G.x,
                     params + P_WN, params + P_BN, W.h[0]);
  hipLaunchKernelGGL(encode, dim3(nb(E * HID)), dim3(BLOCK), 0, s, E, (const float *)G.y,
                     params + P_WE, params + P_BE, W.e[0]);
  for (int l = 0; l < NLAYER; ++l) {
    const float *P = params + P_L0 + l * L_SIZE;
    hipLaunchKernelGGL(edge_layer, dim3(tile_grid(E)), dim3(BLOCK), 0, s, E,
                       (const int32_t *)G.row, A->col_idx, (const uint16_t *)W.h[l],
                       (const uint16_t *)W.e[l], P + L_WM, P + L_BM, W.m[l], W.e[l + 1]);
    hipLaunchKernelGGL(node_layer, dim3(tile_grid(n)), dim3(BLOCK), 0, s, n, A->row_ptr,
                       (const uint16_t *)W.h[l], (const uint16_t *)W.m[l], P + L_WU, P + L_BU,
                       W.g[l], W.r[l], W.h[l + 1]);
  }
  hipLaunchKernelGGL(decode, dim3(nb(E)), dim3(BLOCK), 0, s, E, (const int32_t *)G.row,
                     A->col_idx, (const uint16_t *)W.h[NLAYER], (const uint16_t *)W.e[NLAYER],
                     params + P_WD, params + P_BD, delta);
  MPK_HIP(hipGetLastError());
  return MPK_OK;
}

int mpk_gnn_backward(const mpk_csr *A, const void *graph, const float *params,
                     const float *ddelta, float *dparams, void *ws, size_t ws_bytes,
                     void *stream) {
  if (!params || !ddelta || !dparams) return MPK_EINVAL;
  int st = check_graph_args(A, graph, ~size_t(0));
  if (st) return st;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) || ws_bytes < mpk_gnn_workspace_bytes(A))
    return MPK_EWORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = A->n, E = A->nnz;
  const GGraph G = graph_of(A, graph);
  GWork W;
  Bump b(ws);
  work_layout(n, E, b, &W);
  const int32_t *row = G.row, *col = A->col_idx, *rp = A->row_ptr;
  const int nwE = int(tile_grid(E)) * (BLOCK / WAVE), nwN = int(tile_grid(n)) * (BLOCK / WAVE);
  // decoder
  const int dgrid = int(std::min<int64_t>(std::max<int64_t>(1, (E + 4095) / 4096), GRID_MAX));
  hipLaunchKernelGGL(decode_bwd_weights, dim3(dgrid), dim3(128), 0, s, E, row, col,
                     (const uint16_t *)W.h[NLAYER], (const uint16_t *)W.e[NLAYER], ddelta,
                     W.part);
  hipLaunchKernelGGL(reduce_parts, dim3(1), dim3(128), 0, s, int64_t(dgrid), 3 * HID + 1,
                     3 * HID + 1, (const float *)W.part, dparams + P_WD);
  hipLaunchKernelGGL(decode_bwd_edges, dim3(nb(E * HID)), dim3(BLOCK), 0, s, E, ddelta,
                     params + P_WD, W.de);
  hipLaunchKernelGGL(decode_bwd_nodes, dim3(nb(n * HID)), dim3(BLOCK), 0, s, n, rp,
                     (const int32_t *)G.t_rp, (const int32_t *)G.t_src, ddelta, params + P_WD,
                     W.dh);
  for (int l = NLAYER - 1; l >= 0; --l) {
    const float *P = params + P_L0 + l * L_SIZE;
    float *dP = dparams + P_L0 + l * L_SIZE;
    // node update: du, [dh_mid | dg] = du Wu, dWu
    hipLaunchKernelGGL(node_du, dim3(nb(n * HID)), dim3(BLOCK), 0, s, n, (const float *)W.dh,
                       (const uint16_t *)W.r[l], W.du);
    DxOut on{{W.dh2, W.dh2 + 16, W.dg, W.dg + 16, nullptr, nullptr},
             {W.dh, W.dh + 16, nullptr, nullptr, nullptr, nullptr}};
    hipLaunchKernelGGL((layer_dx<2 * HID>), dim3(tile_grid(n)), dim3(BLOCK), 0, s, n,
                       P + L_WU, (const float *)W.du, on);
    DwIn xn{{W.h[l], W.h[l], W.g[l], W.g[l], nullptr, nullptr},
            {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr},
            {0, 16, 0, 16, 0, 0}};
    hipLaunchKernelGGL((layer_dw<2 * HID>), dim3(tile_grid(n)), dim3(BLOCK), 0, s, n,
                       (const float *)W.du, xn, W.part);
    hipLaunchKernelGGL(reduce_parts, dim3((HID * 2 * HID + HID + 255) / 256), dim3(256), 0, s,
                       int64_t(nwN), PART_MAX, HID * 2 * HID + HID, (const float *)W.part,
                       dP + L_WU);
    // edge layer: dz, [ci | cj | de] = dz Wm, dWm
    hipLaunchKernelGGL(edge_dz, dim3(nb(E * HID)), dim3(BLOCK), 0, s, E, rp, row,
                       (const float *)W.de, (const float *)W.dg, (const uint16_t *)W.m[l],
                       W.dz);
    DxOut oe{{W.ci, W.ci + 16, W.cj, W.cj + 16, W.de, W.de + 16},
             {nullptr, nullptr, nullptr, nullptr, W.de, W.de + 16}};
    hipLaunchKernelGGL((layer_dx<3 * HID>), dim3(tile_grid(E)), dim3(BLOCK), 0, s, E,
                       P + L_WM, (const float *)W.dz, oe);
    DwIn xe{{W.h[l], W.h[l], W.h[l], W.h[l], W.e[l], W.e[l]},
            {row, row, col, col, nullptr, nullptr},
            {0, 16, 0, 16, 0, 16}};
    hipLaunchKernelGGL((layer_dw<3 * HID>), dim3(tile_grid(E)), dim3(BLOCK), 0, s, E,
                       (const float *)W.dz, xe, W.part);
    hipLaunchKernelGGL(reduce_parts, dim3((HID * 3 * HID + HID + 255) / 256), dim3(256), 0, s,
                       int64_t(nwE), PART_MAX, HID * 3 * HID + HID, (const float *)W.part,
                       dP + L_WM);
    hipLaunchKernelGGL(node_gather, dim3(nb(n * HID)), dim3(BLOCK), 0, s, n, rp,
                       (const int32_t *)G.t_rp, (const int32_t *)G.t_src, (const float *)W.dh2,
                       (const float *)W.ci, (const float *)W.cj, W.dh);
  }
  // encoders
  const int gN = int(std::min<int64_t>(std::max<int64_t>(1, (n + 1023) / 1024), GRID_MAX));
  const int gE = int(std::min<int64_t>(std::max<int64_t>(1, (E + 1023) / 1024), GRID_MAX));
  hipLaunchKernelGGL(encode_bwd, dim3(gN), dim3(HID * 5), 0, s, n, (const float *)W.dh,
                     (const uint16_t *)W.h[0], (const float *)G.x, W.part);
  hipLaunchKernelGGL(reduce_parts, dim3(1), dim3(HID * 5), 0, s, int64_t(gN), HID * 5, HID * 5,
                     (const float *)W.part, dparams + P_WN);
  hipLaunchKernelGGL(encode_bwd, dim3(gE), dim3(HID * 5), 0, s, E, (const float *)W.de,
                     (const uint16_t *)W.e[0], (const float *)G.y, W.part);
  hipLaunchKernelGGL(reduce_parts, dim3(1), dim3(HID * 5), 0, s, int64_t(gE), HID * 5, HID * 5,
                     (const float *)W.part, dparams + P_WE);
  MPK_HIP(hipGetLastError());
  return MPK_OK;
}

int mpk_gnn_saved(const mpk_csr *A, const void *ws, size_t ws_bytes, int which, int layer,
                  uint16_t *out, void *stream) {
  if (validate_csr_args(A) || !ws || !out) return MPK_EINVAL;
  if ((reinterpret_cast<uintptr_t>(ws) & 255) || ws_bytes < mpk_gnn_workspace_bytes(A))
    return MPK_EWORKSPACE;
  const int nlayer = (which <= 1) ? NLAYER + 1 : NLAYER;
  if (which < 0 || which > 4 || layer < 0 || layer >= nlayer) return MPK_EINVAL;
  GWork W;
  Bump b(const_cast<void *>(ws));
  work_layout(A->n, A->nnz, b, &W);
  const uint16_t *src = nullptr;
  int64_t rows = A->n;
  switch (which) {
    case 0: src = W.h[layer]; break;
    case 1: src = W.e[layer]; rows = A->nnz; break;
    case 2: src = W.m[layer]; rows = A->nnz; break;
    case 3: src = W.g[layer]; break;
    default: src = W.r[layer]; break;
  }
  MPK_HIP(hipMemcpyAsync(out, src, sizeof(uint16_t) * size_t(rows) * HID,
                         hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return MPK_OK;
}

size_t mpk_gnn_loss_workspace_bytes(const mpk_csr *A, int32_t nprobe) {
  if (!A || A->n <= 0 || A->nnz < 0 || nprobe <= 0) return 0;
  Bump b(nullptr);
  return loss_layout(A->n, nprobe, b, nullptr);
}

int mpk_gnn_factor_loss(const mpk_csr *A, const mpk_ilu0 *Mh, const void *graph,
                        const float *delta, int32_t nprobe, const double *probes, double *loss,
                        float *ddelta, void *ws, size_t ws_bytes, void *stream) {
  int st = check_graph_args(A, graph, ~size_t(0));
  if (st) return st;
  const Ilu0 *M = reinterpret_cast<const Ilu0 *>(Mh);
  if (!M || !delta || !probes || !loss || nprobe <= 0) return MPK_EINVAL;
  if (M->C != 1 || M->KF != 1) return MPK_EUNSUPPORTED;
  if (M->n != A->n || M->nnz != A->nnz) return MPK_EINVAL;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) ||
      ws_bytes < mpk_gnn_loss_workspace_bytes(A, nprobe))
    return MPK_EWORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = A->n, E = A->nnz;
  const GGraph G = graph_of(A, graph);
  LWork L;
  Bump b(ws);
  loss_layout(n, nprobe, b, &L);
  const double *f = M->f;
  hipLaunchKernelGGL(loss_upper, dim3(nb(n)), dim3(BLOCK), 0, s, n, int(nprobe), A->row_ptr,
                     A->col_idx, A->val, f, delta, probes, L.aw, L.y);
  hipLaunchKernelGGL(loss_lower, dim3(nb(n)), dim3(BLOCK), 0, s, n, int(nprobe), A->row_ptr,
                     A->col_idx, f, delta, (const double *)L.aw, (const double *)L.y, L.e,
                     L.part);
  hipLaunchKernelGGL(loss_scalar, dim3(1), dim3(64), 0, s, int64_t(nb(n)), int(nprobe),
                     (const double *)L.part, L.coef, loss);
  if (ddelta) {
    hipLaunchKernelGGL(loss_gy, dim3(nb(n)), dim3(BLOCK), 0, s, n, int(nprobe),
                       (const int32_t *)G.t_rp, (const int32_t *)G.t_src,
                       (const int32_t *)G.row, f, delta, (const double *)L.coef,
                       (const double *)L.e, L.gy);
    if (E > 0)
      hipLaunchKernelGGL(loss_grad, dim3(nb(E)), dim3(BLOCK), 0, s, E, int(nprobe), n,
                         (const int32_t *)G.row, A->col_idx, f, delta, (const double *)L.coef,
                         (const double *)L.e, (const double *)L.y, (const double *)L.gy,
                         probes, ddelta);
  }
  MPK_HIP(hipGetLastError());
  return MPK_OK;
}

int mpk_ilu0_correct(mpk_ilu0 *Mh, const float *delta, int32_t *fell_back, void *stream) {
  Ilu0 *M = reinterpret_cast<Ilu0 *>(Mh);
  if (!M || !delta || !fell_back) return MPK_EINVAL;
  if (M->C != 1 || M->KF != 1) return MPK_EUNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  const int64_t E = M->nnz;
  *fell_back = 0;
  if (E == 0) return MPK_OK;
  // the guard word: words[3] of the factor's workspace
  int32_t *flag = M->words + 3;
  int32_t h_flag = 0;
  MPK_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
  hipLaunchKernelGGL(correct_check, dim3(nb(E)), dim3(BLOCK), 0, s, E, M->row_ptr, M->n,
                     M->col_idx, (const double *)M->f, delta, flag);
  MPK_HIP(hipGetLastError());
  MPK_HIP(hipMemcpyAsync(&h_flag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPK_HIP(hipStreamSynchronize(s));
  if (h_flag) {
    *fell_back = 1;
    return MPK_OK;
  }
  hipLaunchKernelGGL(correct_apply, dim3(nb(E)), dim3(BLOCK), 0, s, E, M->row_ptr, M->n,
                     M->col_idx, M->f, delta);
  MPK_HIP(hipGetLastError());
  int st = ilu0_regather(*M, s);
  if (st) return st;
  MPK_HIP(hipStreamSynchronize(s));
  return MPK_OK;
}

int mpk_gnn_adam(int64_t count, int64_t step, float lr, float beta1, float beta2, float eps,
                 float *params, const float *grad, float *m, float *v, void *stream) {
  if (count <= 0 || step <= 0 || !params || !grad || !m || !v || !(lr >= 0) ||
      !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return MPK_EINVAL;
  const float c1 = float(1.0 - std::pow(double(beta1), double(step)));
  const float c2 = float(1.0 - std::pow(double(beta2), double(step)));
  hipLaunchKernelGGL(adam_step, dim3(nb(count)), dim3(BLOCK), 0, (hipStream_t)stream, count,
                     lr, beta1, beta2, eps, c1, c2, params, grad, m, v);
  MPK_HIP(hipGetLastError());
  return MPK_OK;
}

}  // extern "C"
