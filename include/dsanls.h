/*
 * dsanls.h -- C ABI of the MI355X (gfx950) sketched-ANLS library.
 *
 * The library runs the per-node hot path of DSANLS (Alg. 2 of "Fast and
 * Secure Distributed Nonnegative Matrix Factorization", arXiv 2009.02845) on
 * one GPU, for the problem min_{U>=0, V>=0} ||M - U V^T||_F (eq. problem):
 *
 *   update_U(t):  S^t (n x d) random sketch            (Sec. 3.4)
 *                 A = M S^t,  B = V^T S^t              (eq. def_A_B)
 *                 G = B B^T,  R = A B^T                (eq. gradient_descent)
 *                 U <- prox-CD sweep(s) or PGD step    (Alg. 3 / eq. gradient_descent)
 *   update_V(t):  the same on M^T with S'^t (m x d') and the current U.
 *   objective:    ||M - U V^T||_F / ||M||_F            (Sec. 5.2)
 *
 * Conventions (all entry points):
 *   - Matrices are row-major.  "Device" pointers are HIP device memory owned
 *     by the caller; the library never allocates or frees device memory: all
 *     scratch space lives in the caller's workspace.
 *   - Work is enqueued on the caller's HIP stream (hip_stream may be NULL
 *     for the null stream) and is asynchronous unless stated otherwise.
 *     With a subsampling sketch a context also owns one stream of its own
 *     (default priority), on which the other side's next subsample and its
 *     sketched rows are prepared ahead (they need only M, the seed and t);
 *     events order that work against the caller's stream, so results are
 *     as if everything ran on the caller's stream in call order.
 *   - Every call returns a dsanls_status; nothing is thrown across the ABI.
 *     dsanls_last_error() returns a message for the calling thread's last
 *     failure.  A context is not thread-safe; separate contexts on separate
 *     streams are independent.
 */
#ifndef DSANLS_H
#define DSANLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DSANLS_OK = 0,
  DSANLS_E_INVALID_ARG = 1,  /* bad pointer, enum or parameter value           */
  DSANLS_E_SHAPE = 2,        /* inconsistent or unsupported sizes              */
  DSANLS_E_WORKSPACE = 3,    /* workspace missing, misaligned or too small     */
  DSANLS_E_HIP = 4,          /* a HIP runtime call failed                      */
  DSANLS_E_NONFINITE = 5,    /* NaN/Inf found in M, U or V                     */
  DSANLS_E_STATE = 6,        /* call out of order (e.g. before init)           */
  DSANLS_E_UNSUPPORTED = 7,  /* valid request the library does not implement   */
  DSANLS_E_INTERNAL = 8      /* a device-side step failed (reported later, see
                                dsanls_objective)                              */
} dsanls_status;

/* Kind of random sketch (Sec. 3.4).  IDENTITY (S = I, needs d = n and
 * d' = m) turns the method into exact-product ANLS and is meant for tests.
 * COUNT and SRHT are the further kinds the last paragraph of Sec. 3.4 names
 * (both satisfy Assumption 1, E[S S^T] = I):
 *   COUNT: row j of S has one nonzero s_j = +-1 in column h_j (uniform over
 *          d); A = M S costs one pass over M (dense or CSR).  Needs
 *          d >= n_global / 1024 (and d' >= m_global / 1024).
 *   SRHT:  S[j, c] = s_j H[j, p_c] / sqrt(d), H the Sylvester Hadamard matrix
 *          of order N = max(1024, 2^ceil(log2 n_global)), p the d sampled
 *          columns of H (without replacement).  Dense input, N <= 32768.
 * Signs, buckets and sampled columns come from Philox counters
 * (0, j, side | kind << 8, t) with kind 2 (count), 3 (SRHT signs) and 4
 * (SRHT columns, the subsampling rule over N). */
typedef enum {
  DSANLS_SKETCH_GAUSSIAN = 0,   /* i.i.d. N(0, 1/d) entries                   */
  DSANLS_SKETCH_SUBSAMPLE = 1,  /* d columns e_j without replacement, x sqrt(n/d) */
  DSANLS_SKETCH_IDENTITY = 2,
  DSANLS_SKETCH_COUNT = 3,      /* count sketch                               */
  DSANLS_SKETCH_SRHT = 4        /* subsampled randomised Hadamard transform   */
} dsanls_sketch;

/* Subproblem solver (Sec. 3.5). */
typedef enum {
  DSANLS_SOLVER_PROX_CD = 0,    /* proximal coordinate descent, Alg. 3        */
  DSANLS_SOLVER_PGD = 1         /* one projected-gradient step                */
} dsanls_solver;

/* Arithmetic of the dense sketch product A = M S. */
typedef enum {
  DSANLS_PREC_FP32 = 0,         /* FP32 MFMA, FP32 accumulation               */
  DSANLS_PREC_BF16_SKETCH = 1   /* M and S rounded to BF16, BF16 MFMA, FP32
                                   accumulation; B, G, R and the solver FP32  */
} dsanls_precision;

typedef enum { DSANLS_DENSE = 0, DSANLS_CSR = 1 } dsanls_format;

/*
 * Problem and method parameters.
 *   m, n       M is m x n; U is m x k and V is n x k (row-major, ld = k).
 *   d, d_prime sketch sizes of the U- and V-subproblems (eq. sketched_u/v).
 *   alpha,beta proximal weight mu_t = alpha + beta * t (Sec. 5.2), used by
 *              prox-CD and, through the step 1/(2(L_t + mu_t)), by PGD.
 *   sweeps     prox-CD sweeps per update (the paper uses 1); 0 sweeps each
 *              row until its relative KKT residual <= tol or max_sweeps.
 *   clip_upper nonzero clips U, V to sqrt(2 ||M||_F) (eq. extra_con).
 *   seed       key of the counter-based generator: equal seeds give equal
 *              S^t on every node (Sec. 3.4).
 *   warm_hidden hidden width of the warm-start network that
 *              dsanls_set_warm_start may install later (0: none); it sizes
 *              the workspace.  Warm starts apply to CSR input with a
 *              subsampling sketch in to-tolerance mode (sweeps = 0).
 *   row_offset, col_offset, m_global, n_global
 *              a node's share (Sec. 3.1, eq. u_block; Alg. 2): M is the block
 *              [row_offset, row_offset + m) x [col_offset, col_offset + n)
 *              of an m_global x n_global matrix (m_global = 0 or n_global = 0
 *              mean m or n: the whole matrix, the one-node case).  U holds
 *              the block's rows of U and V its rows of V.  The sketches are
 *              drawn at global indices from the one shared seed (Sec. 3.4):
 *              row j of S^t is row col_offset + j of the whole S^t, row i of
 *              S'^t row row_offset + i of the whole S'^t, and subsampling
 *              picks d of n_global (d' of m_global) indices with scale
 *              sqrt(n_global / d) (sqrt(m_global / d')).  So a block that
 *              spans all columns (col_offset = 0, n = n_global) computes node
 *              r's U update of Alg. 2 exactly, its A = M_{I_r:} S^t being
 *              those rows of the whole product; on a block of columns
 *              update_U forms the node's partial products A_r = M S_{J_r} and
 *              B_r = V^T S_{J_r}, whose sum over the column blocks is the
 *              whole A and B (the all-reduce of Alg. 2, read back with
 *              dsanls_debug_fetch).  Mirrored for update_V.  The identity
 *              sketch and the warm start need the whole matrix.
 */
typedef struct {
  int64_t m, n, k, d, d_prime;
  int32_t sketch;      /* dsanls_sketch    */
  int32_t solver;      /* dsanls_solver    */
  int32_t precision;   /* dsanls_precision */
  int32_t sweeps;
  int32_t max_sweeps;
  int32_t clip_upper;
  double tol;
  double alpha, beta;
  uint64_t seed;
  int32_t warm_hidden;
  int32_t reserved;
  int64_t row_offset, col_offset;
  int64_t m_global, n_global;
} dsanls_config;

/*
 * The local data of one node: Alg. 2 takes both M_{I_r:} and M_{:J_r} as
 * input; with one node these are M and M^T.
 *   DENSE: dense (m x n, leading dimension ld >= n).  dense_t (n x m, ld_t)
 *          may be NULL, in which case init builds M^T in the workspace.
 *   CSR:   rowptr[m+1] (int64), colidx[nnz] (int32, sorted within each row,
 *          no duplicates, all < n), vals[nnz], nnz < 2^31; plus the same
 *          arrays of CSR(M^T) (t_rowptr[n+1], t_colidx, t_vals).  With
 *          t_rowptr NULL, init builds CSR(M^T) in the workspace on the GPU
 *          (rows of M^T sorted; deterministic).
 * All arrays are device memory, read-only, and must outlive the context.
 */
typedef struct {
  int32_t format;      /* dsanls_format */
  const float* dense;
  int64_t ld;
  const float* dense_t;
  int64_t ld_t;
  const int64_t* rowptr;
  const int32_t* colidx;
  const float* vals;
  int64_t nnz;
  const int64_t* t_rowptr;
  const int32_t* t_colidx;
  const float* t_vals;
} dsanls_matrix;

typedef struct dsanls_ctx dsanls_ctx;

/* Counters accumulated since init (read with dsanls_get_stats). */
typedef struct {
  int64_t updates;          /* half-iterations run                           */
  int64_t rows_updated;     /* NNLS rows solved                              */
  int64_t sweeps_total;     /* prox-CD row-sweeps run (to-tol mode: counted) */
  int64_t rows_unconverged; /* to-tol rows that hit max_sweeps               */
  int64_t warm_fallbacks;   /* warm-start rows that started from U^t instead */
} dsanls_stats;

/* Size in bytes of the device workspace init needs for (cfg, M). */
dsanls_status dsanls_workspace_bytes(const dsanls_config* cfg, const dsanls_matrix* M,
                                     size_t* bytes);

/*
 * Validate the problem, carve the workspace (device memory of at least
 * dsanls_workspace_bytes, 256-byte aligned), prepare M^T / BF16 copies and
 * ||M||_F^2, and return a context.  U (m x k) and V (n x k) are device
 * arrays holding U^0 >= 0 and V^0 >= 0; they are updated in place by the
 * update calls.  Synchronises the stream once (for ||M||_F^2).
 * Errors: INVALID_ARG (null pointers, alpha/beta < 0, alpha = mu_0 = 0
 * outside to-tolerance mode, bad enums), SHAPE (sizes, a block outside the
 * global matrix, d > n_global for subsampling, d != n for identity),
 * WORKSPACE, UNSUPPORTED (Gaussian or SRHT sketch on CSR input, BF16 on
 * CSR input or with a sketch other than Gaussian, the size limits of COUNT
 * and SRHT above, k > 512, k > 128 with PGD, to-tolerance sweeps or a warm
 * start), HIP.  NONFINITE: M, U or V holds NaN or Inf.
 */
dsanls_status dsanls_init(const dsanls_config* cfg, const dsanls_matrix* M, float* U, float* V,
                          void* workspace, size_t workspace_bytes, void* hip_stream,
                          dsanls_ctx** out);

/* One U half-iteration at outer iteration t (Alg. 2, U-side, N = 1):
 * U <- update(M, U, V).  Asynchronous. */
dsanls_status dsanls_sketch_update_U(dsanls_ctx* ctx, int64_t t);

/* One V half-iteration at outer iteration t on M^T with the current U
 * (which is U^{t+1} after update_U(t), as in Alg. 1).  Asynchronous. */
dsanls_status dsanls_sketch_update_V(dsanls_ctx* ctx, int64_t t);

/* Relative error ||M - U V^T||_F / ||M||_F of the current U, V (Sec. 5.2).
 * Synchronises the stream.  Returns NONFINITE if U, V or the residual hold
 * NaN/Inf: the NNLS updates never project a non-finite value to 0 (a row
 * whose right-hand side, centre, start or Gram is not finite comes out NaN
 * in every entry), so a non-finite input of any update since init shows up
 * here.  Returns INTERNAL if a subsample selection since the last objective
 * failed (its results are then wrong).  The device flags behind both are
 * cleared by each call. */
dsanls_status dsanls_objective(dsanls_ctx* ctx, double* rel_err);

dsanls_status dsanls_get_stats(dsanls_ctx* ctx, dsanls_stats* out);

/* Install (params != NULL) or remove (NULL) the learned warm start.  params
 * is the packed network of the dsanls_mlp_* calls below (device memory,
 * caller-owned, read at each update), with d = cfg.d = cfg.d_prime, k = cfg.k
 * and hidden = cfg.warm_hidden; residual selects the network's form as in
 * those calls (0: the plain two-layer network).  With a warm start, each
 * to-tolerance update first forms the sketched rows a_i of A = X S (CSR), runs the network on
 * [a_i; u_i^t] for every row and starts prox-CD from its output, with the
 * proximal centre kept at u_i^t.  A row starts from u_i^t instead when the
 * network's output is not finite, or misses the tolerance and has the larger
 * relative projected-gradient norm of the two (counted in
 * dsanls_stats.warm_fallbacks).
 * Errors: STATE (the context cannot take a warm start), SHAPE. */
dsanls_status dsanls_set_warm_start(dsanls_ctx* ctx, const float* params, int32_t hidden, int32_t residual);

/* Keep the sketched rows A = X S (CSR form) of every subsampling update on
 * CSR input, for dsanls_gather_sketched_rows (used to build training pairs
 * for the warm-start network).  Warm-start updates keep them anyway. */
dsanls_status dsanls_set_keep_sketched_rows(dsanls_ctx* ctx, int32_t enable);

/* Copy rows sel[0..nsel) (device int32, indices into the last update's
 * rows) of the last update's sketched matrix A into a packed CSR: offsets
 * out_rowptr[nsel + 1], column indices (sketch columns, ascending) and
 * values, all device arrays; capacity bounds the entries.  Synchronises;
 * *nnz (host) receives the entry count.  Errors: STATE (rows not kept),
 * WORKSPACE (capacity too small: nothing is copied beyond the offsets). */
dsanls_status dsanls_gather_sketched_rows(dsanls_ctx* ctx, const int32_t* sel, int64_t nsel,
                                          int32_t* out_rowptr, int32_t* out_cols, float* out_vals,
                                          int64_t capacity, int64_t* nnz);

/* Per-phase GPU time of the updates run while timing was enabled, from HIP
 * events recorded on the context's stream around each phase:
 *   sketch   -- drawing S^t (Philox Gaussian sketch or subsample selection)
 *   product  -- the sketch product: A = M S on MFMA (dense), the gathered
 *               columns (dense subsample), or R from the CSR stream (sparse)
 *   small    -- B = W^T S, G = B B^T, R = A B^T and the transposes
 *   nnls     -- the batched NNLS update (prox-CD or PGD)
 * launches counts the half-iterations timed.  get_timing synchronises.
 * With the environment variable DSANLS_TRACE set (to anything but "" or
 * "0") when dsanls_init runs, timing is on from the start and
 * dsanls_destroy writes one line to stderr with these four totals and the
 * update count. */
typedef struct {
  double sketch_ms, product_ms, small_ms, nnls_ms;
  int64_t launches;
} dsanls_timing;
dsanls_status dsanls_set_timing(dsanls_ctx* ctx, int32_t enable);
dsanls_status dsanls_get_timing(dsanls_ctx* ctx, dsanls_timing* out);

/* Copy an intermediate of the last update to host memory (synchronises).
 * which: 0 = S^T as d x n (Gaussian) or sampled indices (int32, subsample),
 *        1 = A (rows x d, dense paths), 2 = B (k x d), 3 = G (k x k),
 *        4 = R (rows x k).  bytes must equal the object's size. */
dsanls_status dsanls_debug_fetch(dsanls_ctx* ctx, int32_t which, void* dst, size_t bytes);

/* Release the context (host memory, and its own stream after that stream's
 * pending work has finished; caller buffers untouched).  The workspace may
 * be reused or freed once this returns. */
dsanls_status dsanls_destroy(dsanls_ctx* ctx);

const char* dsanls_status_string(dsanls_status s);
const char* dsanls_last_error(void);

/* ---------------------------------------------------------------------------
 * Stand-alone kernels of the path, exported for tests and benchmarks.
 * ------------------------------------------------------------------------- */

/* Philox4x32-10 block function (Salmon et al., SC'11) on count counters:
 * ctr[4*count], key[2*count] in, out[4*count] out (device, uint32). */
dsanls_status dsanls_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out,
                                   int64_t count, void* hip_stream);

/* Gaussian sketch S (n x d, N(0, 1/d), Sec. 3.4) written transposed: St is
 * d x n with leading dimension ld_st >= n (device, FP32).  Row j of S uses
 * counters (q, j, side, t) with key = seed. */
dsanls_status dsanls_gaussian_sketch_t(uint64_t seed, int64_t t, int32_t side, int64_t n,
                                       int64_t d, float* St, int64_t ld_st, void* hip_stream);

/* Subsampling sketch (Sec. 3.4): the d indices of [0, n) with the smallest
 * 64-bit Philox keys (ties by index), written ascending to idx[d] (device
 * int32).  workspace: device memory of dsanls_subsample_workspace_bytes(n). */
size_t dsanls_subsample_workspace_bytes(int64_t n);
dsanls_status dsanls_subsample_indices(uint64_t seed, int64_t t, int32_t side, int64_t n,
                                       int64_t d, int32_t* idx, void* workspace,
                                       size_t workspace_bytes, void* hip_stream);

/* C = X Y^T (FP32 MFMA, FP32 accumulation): X is rows x K (ldx), Y is
 * cols x K (ldy), C is rows x cols (ldc); all device FP32.  X and Y may be
 * NULL when K = 0 (C is then set to zero).  workspace may be NULL (no
 * split-K) or hold dsanls_gemm_workspace_bytes(rows, cols, K) bytes. */
size_t dsanls_gemm_workspace_bytes(int64_t rows, int64_t cols, int64_t K);
dsanls_status dsanls_gemm_nt(const float* X, int64_t ldx, const float* Y, int64_t ldy, float* C,
                             int64_t ldc, int64_t rows, int64_t cols, int64_t K, void* workspace,
                             size_t workspace_bytes, void* hip_stream);

/* C = X Y^T with BF16 operands (raw bfloat16 bit patterns, rows x K and
 * cols x K, row-major) and FP32 accumulation on MFMA; C is FP32 rows x cols.
 * The precision form of the sketch product A = M S. */
dsanls_status dsanls_gemm_nt_bf16(const void* X, int64_t ldx, const void* Y, int64_t ldy, float* C,
                                  int64_t ldc, int64_t rows, int64_t cols, int64_t K,
                                  void* hip_stream);

/* ---- warm-start network: h = ReLU(a W1a + W1u u + b1), y = ReLU(W2 h + b2);
 *      with residual != 0 the variant y = ReLU(u + W2 h + b2) (its second
 *      layer predicts a correction to the cold start u)
 * Packed FP32 parameters: W1a (d x H, row c = input column c) | W1u (H x k)
 * | b1 (H) | W2 (k x H) | b2 (k), dsanls_mlp_param_count(d, k, H) floats.
 * A batch: a as CSR (a_rowptr[rows + 1], a_cols, a_vals; int32 offsets),
 * and for gradients also its CSC form (c_colptr[d + 1], c_rows, c_vals);
 * U and Y (labels) are rows x k.  All device memory. */
int64_t dsanls_mlp_param_count(int32_t d, int32_t k, int32_t hidden);
size_t dsanls_mlp_workspace_bytes(int32_t d, int32_t k, int32_t hidden, int64_t rows);
/* out (rows x k) = network(a, U). */
dsanls_status dsanls_mlp_forward(int32_t d, int32_t k, int32_t hidden, int32_t residual,
                                 const float* params, int64_t rows, const int32_t* a_rowptr, const int32_t* a_cols,
                                 const float* a_vals, const float* U, float* out, void* workspace,
                                 size_t workspace_bytes, void* hip_stream);
/* grads (packed like params) of L = (1/rows) sum_b ||y_b - Y_b||^2; loss
 * (device, 2 floats) receives L as a (hi, lo) pair. */
dsanls_status dsanls_mlp_gradients(int32_t d, int32_t k, int32_t hidden, int32_t residual,
                                   const float* params, float* grads, int64_t rows, const int32_t* a_rowptr,
                                   const int32_t* a_cols, const float* a_vals,
                                   const int32_t* c_colptr, const int32_t* c_rows,
                                   const float* c_vals, const float* U, const float* Y,
                                   float* loss, void* workspace, size_t workspace_bytes,
                                   void* hip_stream);
/* gradients, then one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, step
 * t >= 1) on params with moments adam_m, adam_v (packed like params). */
dsanls_status dsanls_mlp_train_step(int32_t d, int32_t k, int32_t hidden, int32_t residual, float* params,
                                    float* grads, float* adam_m, float* adam_v, int64_t step,
                                    float lr, int64_t rows, const int32_t* a_rowptr,
                                    const int32_t* a_cols, const float* a_vals,
                                    const int32_t* c_colptr, const int32_t* c_rows,
                                    const float* c_vals, const float* U, const float* Y,
                                    float* loss, void* workspace, size_t workspace_bytes,
                                    void* hip_stream);

/* Batched row-wise NNLS of the regularised sketched subproblem (eq. reg_sub):
 * for every row i of U (rows x k, in place), starting from U[i] and with
 * proximal centre C[i] (C may equal U), run prox-CD sweeps (Alg. 3) on
 * min_{u>=0} u G u^T - 2 r_i u^T + mu ||u - c_i||^2 with G (k x k; column j
 * of G is used for coordinate j) and R (rows x k).  sweeps >= 1: exactly
 * that many; sweeps = 0: until the relative KKT residual
 * ||pg|| / ||r_i + mu c_i|| <= tol or max_sweeps.  sweeps_used (device
 * int32[rows]) may be NULL.  upper > 0 clips entries to upper.  1 <= k <= 512
 * (else UNSUPPORTED); above 128 only fixed sweeps (sweeps >= 1), in blocks
 * of 16 coordinates coupled on the matrix cores.  workspace: device memory of
 * dsanls_nnls_workspace_bytes(k) bytes for the prepared Gram.  A row whose
 * right-hand side, centre, start or Gram entries are not finite is written
 * as NaN in every entry (never projected to 0); the call is asynchronous and
 * does not itself report it. */
size_t dsanls_nnls_workspace_bytes(int32_t k);
dsanls_status dsanls_nnls_prox_cd(const float* G, const float* R, const float* C, float* U,
                                  int64_t rows, int32_t k, float mu, int32_t sweeps, float tol,
                                  int32_t max_sweeps, float upper, int32_t* sweeps_used,
                                  void* workspace, size_t workspace_bytes, void* hip_stream);

/* The same batched NNLS update as dsanls_nnls_prox_cd, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops
 * that forbid allocation): no workspace argument and no allocation of any
 * kind.  The prepared Gram lives in a static device array of
 * dsanls_nnls_noalloc_scratch_bytes() bytes, one copy on each GPU the
 * library runs on, held until the process ends; its device address is
 * looked up on the first call on each device (the stream must belong to the
 * current device).  Every call on one GPU shares that array: calls that
 * overlap on one GPU (other streams, other threads) race and give wrong
 * results.  Arguments, layout and results as dsanls_nnls_prox_cd;
 * UNSUPPORTED if k > 128 or the prepared Gram would not fit the array. */
size_t dsanls_nnls_noalloc_scratch_bytes(void);
dsanls_status dsanls_nnls_prox_cd_noalloc(const float* G, const float* R, const float* C, float* U,
                                          int64_t rows, int32_t k, float mu, int32_t sweeps, float tol,
                                          int32_t max_sweeps, float upper, int32_t* sweeps_used,
                                          void* hip_stream);

/* One projected-gradient step (eq. gradient_descent) with eta computed on
 * the device as 1 / (2 (max_j sum_l |G_lj| + mu)):
 * U <- max(U - 2 eta (U G - R), 0), in place.  Workspace as above.  The
 * projection keeps a NaN (and turns -Inf into NaN) instead of returning 0. */
dsanls_status dsanls_pgd_step(const float* G, const float* R, float* U, int64_t rows, int32_t k,
                              float mu, float upper, void* workspace, size_t workspace_bytes,
                              void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* DSANLS_H */
