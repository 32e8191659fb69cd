/*
 * mpk.h -- C-ABI of the MI355X (gfx950) library for ILU(0)-preconditioned
 * multiple-precision Krylov solvers (Kouya, "Assessing the Performance of
 * Mixed-Precision ILU(0)-Preconditioned Multiple-Precision Real and Complex
 * Krylov Subspace Methods", arXiv 2504.14498).
 *
 * Problem (Section 3, the linear system equation): A x = b with A an n x n
 * sparse non-singular matrix, real or complex, stored in CRS with binary64
 * entries (the paper's matrices are binary64; Section 3, last paragraph),
 * and x, b in a multi-component precision.  x0 is taken from x on entry.
 *
 * Conventions shared by every call:
 *  - All array pointers are DEVICE pointers (memory of the current HIP
 *    device) unless stated otherwise.  The caller owns every buffer; the
 *    library never allocates or frees device memory.  Calls that need
 *    scratch space take a caller-provided workspace sized by the matching
 *    *_workspace_bytes query, aligned to 256 bytes.
 *  - Precision: mpk_prec = number of binary64 limbs K (1 = binary64 "D",
 *    2 = double-double "DD", 3 = triple-double "TD", 4 = quad-double "QD";
 *    Section 2's multi-component types).  A vector of n elements is an array
 *    of n * C * K doubles, element-major: element i holds the K limbs of the
 *    real part (leading limb first), then (complex, C = 2) the K limbs of the
 *    imaginary part.
 *  - CSR: row_ptr int32[n+1], col_idx int32[nnz] strictly ascending within
 *    each row, every diagonal entry stored; val: nnz doubles (real) or
 *    2*nnz doubles ((re, im) interleaved, complex).  nnz < 2^31.
 *  - stream: a hipStream_t (NULL = the default stream).  Kernels are
 *    enqueued on it; calls documented as synchronous wait for it.
 *  - Return value: MPK_OK or a status code below.  Invalid arguments are
 *    rejected before any device work, leaving outputs untouched.  No call
 *    aborts or throws.
 */
#ifndef MPK_H
#define MPK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { MPK_D = 1, MPK_DD = 2, MPK_TD = 3, MPK_QD = 4 } mpk_prec;

/* The four product-type methods of Section 3 (Algorithm 3 is BiCG). */
typedef enum { MPK_BICG = 0, MPK_CGS = 1, MPK_BICGSTAB = 2, MPK_GPBICG = 3 } mpk_method;

enum {
  MPK_OK = 0,
  MPK_NOT_CONVERGED = 1,  /* max_iter reached; x holds the last iterate      */
  MPK_BREAKDOWN = 2,      /* a method scalar became exactly zero; x = last  */
  MPK_EINVAL = -1,        /* bad argument (null pointer, size, precision)    */
  MPK_EDEVICE = -2,       /* a HIP runtime call failed                       */
  MPK_EWORKSPACE = -3,    /* workspace missing, too small or misaligned      */
  MPK_EZERO_PIVOT = -4,   /* ILU(0) met u_kk = 0 (bad_row = k)               */
  MPK_ENO_DIAG = -5,      /* a diagonal entry is not stored (bad_row = i)    */
  MPK_EUNSUPPORTED = -6,  /* valid but unsupported combination              */
  MPK_ENONFINITE = -7,    /* a matrix entry is Inf or NaN (bad_row = i)      */
  MPK_EPATTERN = -8,      /* columns not strictly ascending or out of range  */
  MPK_EWATCHDOG = -9      /* a device dependency wait exceeded its bound     */
};

/* CSR matrix, binary64 values; all pointers device, borrowed. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int32_t *row_ptr;
  const int32_t *col_idx;
  const double *val;
} mpk_csr;

/* Solve / factor report (host struct, filled by the library). */
typedef struct {
  int64_t iters;            /* passes of the main loop run                    */
  int64_t bad_row;          /* row of a zero pivot / missing diagonal, else -1 */
  int32_t status;           /* same as the return value                        */
  double relres_recursive;  /* ||r_k|| / ||r_0||, recursive residual           */
  double relres_true;       /* ||b - A x|| / ||b||, checked in the working
                               precision; -1 if never evaluated                 */
  double setup_ms;          /* validation, analysis and ILU(0) factorisation   */
  double solve_ms;          /* iterations and true-residual checks             */
  double *res_history;      /* optional DEVICE buffer: leading limb of
                               ||r_k||^2 for k = 1..res_history_len            */
  int64_t res_history_len;
} mpk_info;

typedef struct mpk_ilu0 mpk_ilu0; /* opaque, host-side handle */

const char *mpk_status_str(int status);
int mpk_version(void);

/* ------------------------------------------------------------------ SpMV
 * y = A x, or y = A^T x (real, trans = 1), or y = A^H x (complex,
 * conj_trans = 1): the CRS SpMV with binary64 A and a K-limb vector (the
 * mixed-precision "_d" product of Section 4).  Row i accumulates its
 * products in ascending column order in the working precision, starting
 * from the first product; the transposed product uses the explicit
 * (conjugate) transpose, whose rows list the entries in ascending original
 * row.  The transposed form needs ws of mpk_spmv_workspace_bytes(A, C, 1)
 * bytes and synchronizes the stream (it copies the pattern to the host to
 * build the transpose); the plain form needs no workspace (ws may be NULL)
 * and is asynchronous.  x and y must not overlap. */
size_t mpk_spmv_workspace_bytes(const mpk_csr *A, int is_complex, int trans);
int mpk_dcsr_spmv(mpk_prec xp, const mpk_csr *A, int trans, const double *x, double *y,
                  void *ws, size_t ws_bytes, void *stream);
int mpk_zcsr_spmv(mpk_prec xp, const mpk_csr *A, int conj_trans, const double *x, double *y,
                  void *ws, size_t ws_bytes, void *stream);

/* r = b - A x in the working precision p (the true residual that the
 * solvers check, Algorithm 3's stopping rule): row i forms (A x)_i as the
 * SpMV above, then subtracts it from b_i once.  b, x, r: device vectors of
 * n elements of (z: 2, d: 1) * p doubles; r must not overlap x.
 * Asynchronous on stream. */
int mpk_dcsr_residual(mpk_prec p, const mpk_csr *A, const double *b, const double *x, double *r,
                      void *stream);
int mpk_zcsr_residual(mpk_prec p, const mpk_csr *A, const double *b, const double *x, double *r,
                      void *stream);

/* Lanes per row of the plain (non-transposed) SpMV for one matrix, keyed
 * by its row_ptr, col_idx and val pointers and n: 1 = one lane per row
 * (the default), 2, 4, 8 or 16 = vector CSR, where that many lanes load and
 * multiply a row's entries (contiguous loads of indices and values) and
 * then add the products in ascending column order.  y is identical for
 * every choice.  0 forgets the choice.  Host-side only; MPK_EINVAL for
 * other values. */
int mpk_spmv_set_lanes(const mpk_csr *A, int lanes);
/* Times y = A x on stream with each lanes-per-row choice (1, 2, 4, 8, 16:
 * one warm-up launch, then three timed) and keeps the fastest for A; *lanes
 * and *ms (either may be NULL) receive it and its mean time per launch.
 * x and y as for mpk_?csr_spmv (y is overwritten).  Synchronous. */
int mpk_spmv_tune(mpk_prec xp, const mpk_csr *A, int is_complex, const double *x, double *y,
                  int *lanes, double *ms, void *stream);

/* ------------------------------------------------- multicolour ordering
 * A labelled variant beyond the paper's method: Section 5 leaves the
 * parallelisation of the ILU(0) routines to future work.  The rows are
 * coloured and ordered by colour, B = P A P^T is formed, and B y = P b is
 * solved with ILU(0) of B; x = P^T y.  ILU(0) of B is a different
 * preconditioner from ILU(0) of A (usually more passes), but in B a row of
 * colour c has stored lower entries only in columns of colours below c,
 * so each substitution runs at most one level per colour, each a set of
 * independent rows.
 *
 * mpk_multicolor_order: the greedy colouring of the graph of A + A^T in
 * natural order (rows i != j are adjacent when a_ij or a_ji is stored; row
 * i = 0, 1, ... takes the smallest colour that no adjacent row j < i has)
 * and the ordering by colour: perm[k] = the row of A placed at position k,
 * colours ascending, rows in their original order within a colour.
 * perm: device int32[n], written; *ncolors (host) receives the number of
 * colours.  The pattern is checked as for ILU(0) (MPK_EPATTERN,
 * MPK_ENO_DIAG).  The colouring runs on the host (the pattern is copied
 * there).  Synchronous. */
int mpk_multicolor_order(const mpk_csr *A, int32_t *perm, int32_t *ncolors, void *stream);
/* B = P A P^T for a permutation perm (device int32[n], perm[k] = the row
 * of A placed at k): b_kl = a_{perm[k], perm[l]}, each row's columns in
 * ascending order, values copied exactly.  b_row_ptr[n+1], b_col_idx[nnz]
 * and b_val[nnz*C] are device arrays of the caller, written here (B has
 * A's n and nnz).  ws: mpk_csr_permute_workspace_bytes(n) bytes of device
 * memory, 256-byte aligned (MPK_EWORKSPACE otherwise).  MPK_EINVAL when
 * perm does not hold every row exactly once; MPK_EPATTERN when A's
 * row_ptr or col_idx are out of range.  Synchronous. */
size_t mpk_csr_permute_workspace_bytes(int64_t n);
int mpk_dcsr_permute(const mpk_csr *A, const int32_t *perm, int32_t *b_row_ptr,
                     int32_t *b_col_idx, double *b_val, void *ws, size_t ws_bytes, void *stream);
int mpk_zcsr_permute(const mpk_csr *A, const int32_t *perm, int32_t *b_row_ptr,
                     int32_t *b_col_idx, double *b_val, void *ws, size_t ws_bytes, void *stream);
/* y = P x (inverse = 0: y[k] = x[perm[k]]) or y = P^T x (inverse = 1:
 * y[perm[k]] = x[k]) for device vectors of n elements of (is_complex ? 2 :
 * 1) * vp doubles.  perm should be a permutation (mpk_?csr_permute checks
 * one); an entry outside [0, n) is skipped, nothing is read or written
 * for it.  x and y must not overlap.  Asynchronous on stream. */
int mpk_vec_permute(mpk_prec vp, int is_complex, int64_t n, const int32_t *perm, int inverse,
                    const double *x, double *y, void *stream);

/* --------------------------------------------------------------- ILU(0)
 * ILU(0) factorisation (Algorithm 1) on the stored pattern of A, in factor
 * precision fp = MPK_D (binary64: the "_d_ILU(0)" factor of Section 4) or
 * MPK_DD, MPK_TD, MPK_QD (A promoted exactly to fp limbs and factored in
 * that arithmetic: the full-precision "ILU(0)" factors of Section 4,
 * Tables 1 and 2).  "A_ij != 0" is read
 * structurally.  Rows are eliminated in IKJ order, level by level; each
 * entry receives the updates of Algorithm 1 in ascending k, so the factor
 * is identical to the KIJ loop's.  Zero pivots are reported
 * (MPK_EZERO_PIVOT, bad_row = k), never skipped.  ws (caller-owned, kept
 * alive until mpk_ilu0_destroy) receives the factor and the level
 * schedules; *M receives a host handle pointing into it.  flags:
 * MPK_ILU0_ADJOINT also prepares the M^H solve (needed by
 * conj_trans = 1 and by BiCG); MPK_ILU0_VPREC(k) declares the largest
 * vector precision used with it.  Synchronous; info may be NULL. */
#define MPK_ILU0_ADJOINT 1
/* Largest vector precision (limbs, 1..4) the factor will be applied with;
 * it sizes the on-chip blocks of the substitutions.  0 (the default) means
 * MPK_QD.  Applying with more limbs than declared returns MPK_EUNSUPPORTED. */
#define MPK_ILU0_VPREC(k) ((k) << 4)
size_t mpk_ilu0_workspace_bytes(const mpk_csr *A, mpk_prec fp, int is_complex, int flags);
int mpk_dilu0_factor(mpk_prec fp, const mpk_csr *A, int flags, void *ws, size_t ws_bytes,
                     mpk_ilu0 **M, mpk_info *info, void *stream);
int mpk_zilu0_factor(mpk_prec fp, const mpk_csr *A, int flags, void *ws, size_t ws_bytes,
                     mpk_ilu0 **M, mpk_info *info, void *stream);

/* z = M^{-1} r with M = L U (Algorithm 2: unit-lower forward substitution,
 * then backward substitution with a division by u_ii), or z = M^{-H} r
 * (conj_trans = 1: forward with U^H dividing by conj(u_ii), then backward
 * with the unit L^H; Algorithm 3's M^H solve).  Sums run in ascending
 * column order, each term subtracted in turn.  Vector precision vp >= the
 * factor precision.  Asynchronous on stream; r and z must not overlap and
 * must not be in use by another apply of the same handle. */
int mpk_dilu0_apply(const mpk_ilu0 *M, mpk_prec vp, int conj_trans, const double *r, double *z,
                    void *stream);
int mpk_zilu0_apply(const mpk_ilu0 *M, mpk_prec vp, int conj_trans, const double *r, double *z,
                    void *stream);
/* Frees the host handle only; the workspace stays the caller's. */
void mpk_ilu0_destroy(mpk_ilu0 *M);

/* --------------------------------------------------------------- solvers
 * Solve A x = b with a preconditioned product-type method (Section 3):
 * BiCG exactly as Algorithm 3; CGS, BiCGSTAB and GPBiCG in right-
 * preconditioned form (unpreconditioned residual, two M-solves per pass).
 * vp: vector precision (MPK_D..MPK_QD).  fp: 0 = no preconditioner,
 * MPK_D..vp = ILU(0) factor precision.  Stopping rule of Algorithm 3,
 * ||r|| < tol_rel ||r_0|| + tol_abs, on the recursive residual; when it
 * passes, the true residual ||b - A x|| is evaluated in the working
 * precision and must pass the same test, otherwise the recursion goes on.
 * max_iter bounds the passes.  x: in x0, out the solution (or last
 * iterate).  Synchronous.  info may be NULL. */
size_t mpk_krylov_workspace_bytes(mpk_method m, mpk_prec vp, mpk_prec fp, const mpk_csr *A,
                                  int is_complex);
int mpk_dkrylov_solve(mpk_method m, mpk_prec vp, mpk_prec fp, double tol_rel, double tol_abs,
                      int64_t max_iter, const mpk_csr *A, const double *b, double *x, void *ws,
                      size_t ws_bytes, mpk_info *info, void *stream);
int mpk_zkrylov_solve(mpk_method m, mpk_prec vp, mpk_prec fp, double tol_rel, double tol_abs,
                      int64_t max_iter, const mpk_csr *A, const double *b, double *x, void *ws,
                      size_t ws_bytes, mpk_info *info, void *stream);

/* The same methods with a preconditioner the caller built with
 * mpk_?ilu0_factor on this A (same row_ptr and col_idx pointers), possibly
 * changed since by mpk_ilu0_correct: nothing is factored here.  The factor
 * must have been built with MPK_ILU0_VPREC(k), k >= vp (or 0), and with
 * MPK_ILU0_ADJOINT for BiCG; otherwise MPK_EINVAL.  The handle's sweeps
 * use its own workspace, so one factor serves one solve at a time.  The
 * workspace here holds the vectors only. */
size_t mpk_krylov_precond_workspace_bytes(mpk_method m, mpk_prec vp, const mpk_csr *A,
                                          int is_complex);
int mpk_dkrylov_solve_precond(mpk_method m, mpk_prec vp, const mpk_ilu0 *M, double tol_rel,
                              double tol_abs, int64_t max_iter, const mpk_csr *A, const double *b,
                              double *x, void *ws, size_t ws_bytes, mpk_info *info,
                              void *stream);
int mpk_zkrylov_solve_precond(mpk_method m, mpk_prec vp, const mpk_ilu0 *M, double tol_rel,
                              double tol_abs, int64_t max_iter, const mpk_csr *A, const double *b,
                              double *x, void *ws, size_t ws_bytes, mpk_info *info,
                              void *stream);

/* --------------------------------------------------------- batched solve
 * nsys independent real systems A[q] x[q] = b[q] of any sizes, each solved
 * by ILU(0)-preconditioned BiCGSTAB (the only method offered batched) with
 * the semantics of mpk_dkrylov_solve, in ONE persistent (cooperative)
 * kernel launch: a team of workgroups on one XCD takes the next system,
 * checks its pattern, builds its level schedules, factors it (Algorithm 1)
 * and runs the passes with the substitutions of Algorithm 2, synchronising
 * only inside the team.  A, b, x: host arrays of nsys entries holding
 * device pointers.  info: host array of nsys reports (may be NULL).
 * schedule: NULL = autotune (on the first call for a batch shape a few
 * passes of each candidate schedule are timed, x untouched, and the
 * fastest is cached), or "grid=<workgroups>,order=lpt|given[,team=<rows>]"
 * (lpt: systems considered largest first; team: rows per team member, a
 * system of n rows gets ceil(n / rows) workgroups up to the workgroups of
 * an XCD; absent or 0: one workgroup per system).  The grid is capped at
 * the workgroups that fit on the device at once.  Schedules only map work
 * to workgroups: inner products are summed over fixed row tiles, so results
 * are bitwise identical for every schedule.  A system that a launch did not
 * finish (a team that waited past its bound) is solved again with one
 * workgroup, from the caller's x.  Returns MPK_OK when every system
 * converged, otherwise the most severe per-system status.  Synchronous. */
size_t mpk_krylov_batched_workspace_bytes(mpk_method m, mpk_prec vp, mpk_prec fp, int32_t nsys,
                                          const mpk_csr *A);
int mpk_dkrylov_solve_batched(mpk_method m, mpk_prec vp, mpk_prec fp, double tol_rel,
                              double tol_abs, int64_t max_iter, int32_t nsys, const mpk_csr *A,
                              const double *const *b, double *const *x, void *ws, size_t ws_bytes,
                              mpk_info *info, const char *schedule, void *stream);

/* ------------------------------------------- learned ILU(0) correction
 * Not in the paper: a correction of the binary64 ILU(0) factor (Algorithm
 * 1) predicted by a small graph network, applied without touching the
 * methods' arithmetic or their stopping test; plain ILU(0) stays the
 * fallback.  Real matrices with a binary64 (MPK_D) factor only.
 *
 * Graph: nodes are the rows of A, edges its stored entries q = (i, j) in
 * CSR order, diagonal included, so the output delta[nnz] lies on the
 * ILU(0) pattern.  Inputs, from A and the plain factor (l below the
 * diagonal, u on and above it):
 *   node i: log|a_ii|, sum_{j != i}|a_ij| / |a_ii|, log(|u_ii| / |a_ii|),
 *           (stored entries of row i) / 8
 *   edge q: a_ij / |a_ii|, (l_ij if j < i, else u_ij / |a_ii|), [j < i], [j > i]
 * Network, hidden width 32, three message-passing layers; R() rounds to
 * bfloat16 (nearest even), the type activations are stored in:
 *   h_i = R(relu(Wn x_i + bn)),  e_q = R(relu(We y_q + be))
 *   per layer: m_q = R(relu(Wm [h_i; h_j; e_q] + bm)),
 *              g_i = R(mean of m_q over row i),
 *              h_i <- R(h_i + relu(Wu [h_i; g_i] + bu)),  e_q <- R(e_q + m_q)
 *   delta_q = wd . [h_i; h_j; e_q] + bd
 * Wm and Wu are rounded to bfloat16 for the matrix cores (float32
 * accumulation); the encoders and the decoder use the float32 weights.
 * Parameters: one float32 vector of mpk_gnn_param_count() = 15969 values,
 * row-major [out][in]: Wn[32][4], bn[32], We[32][4], be[32], then per layer
 * Wm[32][96], bm[32], Wu[32][64], bu[32], then wd[96], bd[1].
 *
 * Correction: u_ii <- u_ii exp(delta_ii) (sign kept, never zero); every
 * other value v <- v (1 + tanh(delta_q) / 2).
 *
 * All device pointers; all calls on `stream`; setup, loss (its host part)
 * and correct synchronize, forward, backward and adam are asynchronous. */
int64_t mpk_gnn_param_count(void);
/* Initial parameters from seed: weights uniform in +-1/sqrt(fan_in), biases
 * zero, decoder zero (so the first prediction is delta = 0, the plain
 * factor). */
int mpk_gnn_init(float *params, uint64_t seed, void *stream);
/* Per-matrix graph data (edge rows, transposed pattern, inputs), built
 * from A and its plain binary64 factor M (from mpk_dilu0_factor on this
 * A, before any correction).  graph: caller-owned, 256-byte aligned, at
 * least mpk_gnn_graph_bytes(A). */
size_t mpk_gnn_graph_bytes(const mpk_csr *A);
int mpk_gnn_graph_setup(const mpk_csr *A, const mpk_ilu0 *M, void *graph, size_t graph_bytes,
                        void *stream);
/* delta[nnz] (float32) = network(params) on a set-up graph.  ws (at least
 * mpk_gnn_workspace_bytes(A)) keeps the activations for backward. */
size_t mpk_gnn_workspace_bytes(const mpk_csr *A);
int mpk_gnn_forward(const mpk_csr *A, const void *graph, const float *params, float *delta,
                    void *ws, size_t ws_bytes, void *stream);
/* dparams = d(sum_q ddelta_q delta_q)/dparams for the activations the last
 * forward left in ws (bfloat16 rounding taken as the identity).  Writes
 * (does not accumulate) all mpk_gnn_param_count() values. */
int mpk_gnn_backward(const mpk_csr *A, const void *graph, const float *params,
                     const float *ddelta, float *dparams, void *ws, size_t ws_bytes,
                     void *stream);
/* Copies an activation the last mpk_gnn_forward left in ws to out (device,
 * bfloat16 bit patterns, rows x 32, row-major), so that a check of the
 * backward pass can start from exactly the values it uses.  which: 0 =
 * node states h (layer 0..3: the encoder output, then after each message-
 * passing layer; n rows), 1 = edge states e (layer 0..3; nnz rows), 2 =
 * messages m (layer 0..2; nnz rows), 3 = row means g (layer 0..2; n
 * rows), 4 = relu of the node update, R(relu(Wu [h; g] + bu)) (layer
 * 0..2; n rows).  Asynchronous; MPK_EINVAL for another which or layer. */
int mpk_gnn_saved(const mpk_csr *A, const void *ws, size_t ws_bytes, int which, int layer,
                  uint16_t *out, void *stream);
/* Training loss of a correction delta on probe vectors w_p (nprobe rows of
 * n doubles, e.g. normalised residuals of the plain method), in binary64:
 *   loss = mean_p ||A w_p - L~ U~ w_p||^2 / ||A w_p||^2
 * with L~ (unit lower) and U~ from the plain factor M corrected by delta
 * as above.  loss: device double; ddelta (may be NULL): d loss / d delta as
 * float32.  M must be uncorrected. */
size_t mpk_gnn_loss_workspace_bytes(const mpk_csr *A, int32_t nprobe);
int mpk_gnn_factor_loss(const mpk_csr *A, const mpk_ilu0 *M, const void *graph,
                        const float *delta, int32_t nprobe, const double *probes, double *loss,
                        float *ddelta, void *ws, size_t ws_bytes, void *stream);
/* One Adam step (Kingma and Ba, with bias correction) over count values;
 * step counts from 1. */
int mpk_gnn_adam(int64_t count, int64_t step, float lr, float beta1, float beta2, float eps,
                 float *params, const float *grad, float *m, float *v, void *stream);
/* Apply delta to the factor in place (and to its sweep schedules), with
 * guards: if any delta or corrected value is non-finite, or a pivot ratio
 * exp(delta_ii) falls outside [1e-8, 1e8], nothing changes and
 * *fell_back (host int) = 1; otherwise 0.  Corrections compound if called
 * twice.  Synchronous. */
int mpk_ilu0_correct(mpk_ilu0 *M, const float *delta, int32_t *fell_back, void *stream);

/* --------------------------------------------------------- inner product
 * out = <a, b> = sum_i conj(a_i) b_i in the working precision (the inner
 * products of Algorithm 3), reduced by a fixed tree (deterministic for a
 * given n).  out: DEVICE pointer to C*K doubles.  ws: at least
 * mpk_dot_workspace_bytes(n, C, K) bytes.  Asynchronous. */
size_t mpk_dot_workspace_bytes(int64_t n, int is_complex, mpk_prec p);
int mpk_dot(mpk_prec p, int is_complex, int64_t n, const double *a, const double *b,
            double *out, void *ws, size_t ws_bytes, void *stream);

/* The same inner product for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no workspace argument; the partials go to a fixed 4 MiB
 * device array of the library (one per GPU, held until the process ends,
 * its address looked up on the first call on each device).  Same kernels
 * and reduction tree as mpk_dot, so the result is bitwise identical.
 * n may be at most mpk_dot_noalloc_max_elements(is_complex, p) (2^27 /
 * (C K) rounded to whole workgroups of 256), otherwise MPK_EWORKSPACE
 * before any device work.  Calls on one GPU share the array: calls that
 * overlap in time on one GPU (different streams, or host threads) race and
 * must be serialised by the caller.  Calls no hipMalloc/hipFree.
 * Asynchronous on stream. */
size_t mpk_dot_noalloc_max_elements(int is_complex, mpk_prec p);
int mpk_dot_noalloc(mpk_prec p, int is_complex, int64_t n, const double *a, const double *b,
                    double *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MPK_H */
