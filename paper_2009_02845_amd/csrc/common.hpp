// Internal declarations shared by the HIP translation units of libdsanls.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <algorithm>
#include <cmath>
#include <string>

#include "../../include/dsanls.h"

namespace dsanls {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
dsanls_status fail(dsanls_status s, const std::string& msg);
dsanls_status hip_fail(hipError_t e, const char* what);

#define DSANLS_HIP(call)                                          \
  do {                                                            \
    hipError_t e_ = (call);                                       \
    if (e_ != hipSuccess) return ::dsanls::hip_fail(e_, #call);   \
  } while (0)

// Check the launch that was just enqueued.
#define DSANLS_LAUNCHED(name)                                        \
  do {                                                               \
    hipError_t e_ = hipGetLastError();                               \
    if (e_ != hipSuccess) return ::dsanls::hip_fail(e_, name);       \
  } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Number of XCDs of an MI355X: workgroups are dispatched round-robin over
// them and each has its own L2, so tile schedules remap workgroup ids.
constexpr int kNumXcd = 8;

// ---------------------------------------------------------------- philox.hip
// S^T (d x n) of rows j0 .. j0 + n - 1 of the Gaussian sketch (and its
// BF16 rounding when St_bf16 is not null).
dsanls_status launch_gaussian_sketch_t(uint64_t seed, uint32_t t, int side, int64_t j0, int64_t n, int64_t d,
                                       float* St, int64_t ld, __hip_bfloat16* St_bf16, int64_t ld_bf16,
                                       hipStream_t s);
// Workspace layout of the subsample selection.
size_t subsample_ws_bytes(int64_t n);
// idx[d] ascending; slot (may be null) gets slot[j] = column of index j or -1.
// idx_win (may be null): idx[c] - win_off where that lies in [0, win_len),
// else -1 (the sampled columns seen by a block of the long dimension).
// kind selects the counter stream (1: the subsampling sketch, 4: the SRHT's
// sampled Hadamard columns).
constexpr uint32_t kSrhtSampleKind = 4;
dsanls_status launch_subsample(uint64_t seed, uint32_t t, int side, int64_t n, int64_t d,
                               int32_t* idx, int32_t* slot, void* ws, size_t ws_bytes,
                               int* err_flag, hipStream_t s, int64_t win_off = 0, int64_t win_len = 0,
                               int32_t* idx_win = nullptr, uint32_t kind = 1);

// ---------------------------------------------------------------- sketches.hip
// Count sketch of one side: bucket h_j and sign s_j of each row j of S (n
// rows, global index j0 + j), bucket offsets off[d + 1] and the rows of
// each bucket in ascending order (list); cnt holds 2 (d + 1) ints (counts,
// cursors), tmp n ints, scan_ws scan_ws_bytes(d); a bucket over the
// ordering kernel's capacity sets bit 4 of *err.
struct CountSketch {
  int32_t* bucket = nullptr;
  float* sign = nullptr;
  int32_t* cnt = nullptr;
  int32_t* off = nullptr;
  int32_t* scan_ws = nullptr;
  int32_t* tmp = nullptr;
  int32_t* list = nullptr;
  int* err = nullptr;
};
dsanls_status launch_count_sketch_hash(uint64_t seed, uint32_t t, int side, int64_t j0, int64_t n, int64_t d,
                                       const CountSketch& cs, hipStream_t s);
// Out (d x cols, ldo) = S^T X^T for X^T (n x cols, ldx): bucket sums of the
// signed rows of X^T.
dsanls_status launch_count_sketch_rows(const float* Xt, int64_t ldx, int64_t cols, int64_t d, const CountSketch& cs,
                                       float* Out, int64_t ldo, hipStream_t s);
// SRHT: transform length N = max(1024, 2^ceil(log2 n)); signs of rows
// j0 .. j0 + n - 1; Out (rows x d) = X S for the rows of X (rows x lng, a
// block starting at global column j0), p the d sampled Hadamard columns.
int64_t srht_length(int64_t n);
dsanls_status launch_srht_signs(uint64_t seed, uint32_t t, int side, int64_t j0, int64_t n, float* sign,
                                hipStream_t s);
dsanls_status launch_srht_rows(const float* X, int64_t ldx, int64_t rows, int64_t lng, int64_t j0, int64_t N,
                               const float* sign, const int32_t* p, int64_t d, float* Out, int64_t ldo,
                               hipStream_t s);

// ---------------------------------------------------------------- gemm.hip
// C[rows x cols] = X[rows x K] * Y[cols x K]^T, FP32 MFMA.
size_t gemm_ws_bytes(int64_t rows, int64_t cols, int64_t K);
dsanls_status launch_gemm_nt(const float* X, int64_t ldx, const float* Y, int64_t ldy, float* C,
                             int64_t ldc, int64_t rows, int64_t cols, int64_t K, void* ws,
                             size_t ws_bytes, hipStream_t s);
// Two independent products C = X Y^T in one launch (both K-contiguous);
// element type FP32 or BF16 (raw bits), FP32 output.  A product with
// rows == 0 is skipped.
struct GemmDesc {
  const void* X;
  int64_t ldx;
  const void* Y;
  int64_t ldy;
  float* C;
  int64_t ldc;
  int64_t rows, cols, K;
};
dsanls_status launch_gemm_grouped(const GemmDesc& a, const GemmDesc& b, bool bf16, hipStream_t s);
// BF16 operands, FP32 accumulation.
dsanls_status launch_gemm_nt_bf16(const __hip_bfloat16* X, int64_t ldx, const __hip_bfloat16* Y,
                                  int64_t ldy, float* C, int64_t ldc, int64_t rows, int64_t cols,
                                  int64_t K, hipStream_t s);
// Sum over (M - U V^T)^2 into partials (2 floats per workgroup: sum, compensation).
int64_t residual_partials(int64_t m, int64_t n);
dsanls_status launch_residual_sq(const float* M, int64_t ldm, const float* U, const float* V,
                                 int64_t m, int64_t n, int64_t k, float* partials, hipStream_t s);

// ---------------------------------------------------------------- small.hip
dsanls_status launch_transpose(const float* X, int64_t ldx, float* Y, int64_t ldy, int64_t rows,
                               int64_t cols, hipStream_t s);
// Y = bf16(X) (rows x cols, round to nearest even), zeros in columns cols .. ldy - 1
dsanls_status launch_to_bf16(const float* X, int64_t ldx, __hip_bfloat16* Y, int64_t ldy,
                             int64_t rows, int64_t cols, hipStream_t s);
// G = B B^T (k x k) with compensated FP32 sums; B is k x d (ld).
dsanls_status launch_gram(const float* B, int64_t ld, int64_t k, int64_t d, float* G,
                          hipStream_t s);
// Sum of squares of a dense matrix into partials (sum, comp pairs), npart blocks.
int64_t sumsq_partials(int64_t rows, int64_t cols);
dsanls_status launch_sumsq(const float* X, int64_t ld, int64_t rows, int64_t cols,
                           float* partials, hipStream_t s);
// Combine npart (sum, comp) pairs in a fixed order into out[0..1] (hi, lo)
// and flag non-finite values.
dsanls_status launch_combine_partials(const float* partials, int64_t npart, int64_t stride,
                                      float* out, int* err_flag, hipStream_t s);
// out[0..1] = compensated sum of X[i] * Y[i] over count entries (one block).
dsanls_status launch_frob_dot(const float* X, const float* Y, int64_t count, float* out,
                              hipStream_t s);
// A[i, c] = scale * X[i, idx[c]] (rows x d), gathered columns (0 where idx[c] < 0).
dsanls_status launch_gather_cols(const float* X, int64_t ldx, const int32_t* idx, int64_t rows,
                                 int64_t d, float scale, float* A, int64_t lda, hipStream_t s);
// B[l, c] = scale * W[idx[c], l] (k x d) from W (rows x k); 0 where idx[c] < 0.
dsanls_status launch_gather_rows_t(const float* W, int64_t k, const int32_t* idx, int64_t d,
                                   float scale, float* B, int64_t ldb, hipStream_t s);
dsanls_status launch_check_finite(const float* X, int64_t count, int* err_flag, hipStream_t s);
// out[0..n] = exclusive prefix sums of in[0..n) (out[n] = total); ws holds
// scan_ws_bytes(n) bytes.
size_t scan_ws_bytes(int64_t n);
dsanls_status launch_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* ws,
                                    hipStream_t s);

// ---------------------------------------------------------------- nnls.hip
// Largest rank of the NNLS kernels, and the floats of the prepared Gram for
// a padded rank KC (KC x KC, four vectors of KC, 64 spare).
constexpr int kNnlsMaxRank = 128;
constexpr size_t nnls_prep_floats(int KC) { return static_cast<size_t>(KC) * KC + 4 * static_cast<size_t>(KC) + 64; }
size_t nnls_ws_bytes(int k);
// Ranks 129 .. 512 (fixed prox-CD sweeps): the wide kernel's padded rank
// (0 past the largest) and its launch on the prepared Gram gp (KC x KC, row j
// = column j of G, zero diagonal) and inv (1 / (G_jj + mu), zero padding).
constexpr int kNnlsMaxRankWide = 512;
int nnls_kc_wide(int k);
dsanls_status launch_prox_cd_wide(const float* gp, const float* inv, int KC, const float* R, const float* C, float* U,
                                  int64_t rows, int k, float mu, int sweeps, float upper, int32_t* sweeps_used,
                                  hipStream_t s);
// Workspace of the to-tolerance mode's compacted passes (rows = the most
// rows of any update; nw = ceil(rows / 64)): per-row sweep counts and flags,
// per-wave pending counts (nw), their scan (nw + 1), pending rows per wave
// (64 nw), two row lists (rows each), the scan's own workspace and a copy
// of the centre (rows x k).
struct TolWork {
  unsigned long long* counters;  // may be null: [0] += row-sweeps, [1] += unconverged rows,
                                 // [2] += rows that started cold although a warm start was given
  int32_t* used;
  int32_t* flags;
  int32_t* wave_cnt;
  int32_t* wave_off;
  int32_t* wave_rows;
  int32_t* list[2];
  int32_t* scan_ws;
  float* centre;                 // rows x k: a copy of C when C aliases U (U changes between passes)
};
// pgd = false: prox-CD (sweeps >= 1, or 0 = to tol); pgd = true: one PGD step.
// tw (to-tolerance mode; may be null: one pass to the end, no counts): the
// compaction workspace.  start (may be null: start from U) is a warm start
// for the to-tolerance mode; a row starts from C instead when its warm start
// is not finite or has the larger projected-gradient norm.
dsanls_status launch_nnls(bool pgd, const float* G, const float* R, const float* C, float* U,
                          int64_t rows, int k, float mu, int sweeps, float tol, int max_sweeps,
                          float upper, int32_t* sweeps_used, const TolWork* tw, void* ws,
                          size_t ws_bytes, hipStream_t s, const float* start = nullptr);

// ---------------------------------------------------------------- sparse.hip
// Longest run of nnz one wave streams in the segmented CSR kernels.
constexpr int64_t kCsrSegment = 4096;
// Segment table of a CSR matrix (device arrays, built at init): segment s
// covers nnz [seg_beg[s], min(seg_beg[s] + kCsrSegment, rowptr[row + 1]))
// of row seg_row[s]; seg_part[s] = -1 for a single-segment row, else the
// index of its partial vector.  Rows with several segments are listed in
// multi_row with their partials [multi_part[i], multi_part[i + 1]).
struct CsrSegments {
  int32_t* seg_row = nullptr;
  int64_t* seg_beg = nullptr;
  int32_t* seg_part = nullptr;
  int32_t* multi_row = nullptr;
  int32_t* multi_part = nullptr;
  int64_t nseg = 0, nmulti = 0, nparts = 0;
};
// Upper bounds used to size the table before it is built.
inline int64_t csr_seg_bound(int64_t rows, int64_t nnz) { return rows + nnz / kCsrSegment + 1; }
inline int64_t csr_part_bound(int64_t nnz) { return 2 * (nnz / kCsrSegment) + 2; }
// Sketched rows a_i of A = X S (subsampling) as CSR over the segment table:
// seg_cnt and seg_pos hold nseg and nseg + 1 ints, scan_ws scan_ws_bytes(nseg).
// Largest sketch size d of the sampled-column gather (a row of A then
// holds at most d entries, which one workgroup sorts in LDS).
constexpr int64_t kGatherMaxD = 4096;
// Sketched rows A = X S (CSR, int32 offsets, values scaled) of a
// subsampling sketch, gathered from the rows idx[0..d) of X^T
// (t_rowptr/t_colidx/t_vals).  Rows longer than 8 entries leave sorted by
// slot; launch_a_rhs sorts the others.  Needs nnz(X) < 2^31 and
// d <= kGatherMaxD.
// cnt: rows + 1 ints; offs: d + 1 ints; long_rows: rows ints; nlong: 1 int.
dsanls_status launch_sampled_rows(const int64_t* t_rowptr, const int32_t* t_colidx, const float* t_vals,
                                  int64_t rows, const int32_t* idx, int64_t d, float scale, int32_t* cnt,
                                  int32_t* offs, int32_t* scan_ws, int32_t* a_rowptr, int32_t* a_cols,
                                  float* a_vals, int32_t* long_rows, int32_t* nlong, hipStream_t s);
// R[i, :] = scale * sum_e a_vals[e] W[idx[a_cols[e]], :] over row i of A, in
// slot order; sorts (in place) the rows launch_sampled_rows left unsorted;
// long_rows/nlong are launch_sampled_rows' list of the rows it sorted.
dsanls_status launch_a_rhs(const int32_t* a_rowptr, int32_t* a_cols, float* a_vals, int64_t rows,
                           const int32_t* idx, const float* W, int64_t k, float scale, const int32_t* long_rows,
                           const int32_t* nlong, float* R, hipStream_t s);
dsanls_status launch_sketched_rows(const int64_t* rowptr, const int32_t* colidx, const float* vals,
                                   int64_t rows, const CsrSegments& sg, const int32_t* slot, float scale,
                                   int32_t* seg_cnt, int32_t* seg_pos, int32_t* scan_ws,
                                   int32_t* a_rowptr, int32_t* a_cols, float* a_vals, hipStream_t s);
// hbucket/hsign (count sketch): W is then B^T (d x k), read at the bucket of
// each entry's column, the entry scaled by the column's sign.
dsanls_status launch_csr_rhs_seg(const int64_t* rowptr, const int32_t* colidx, const float* vals,
                                 const CsrSegments& sg, const int32_t* slot, const float* W, int64_t k,
                                 float scale, float* R, float* P, hipStream_t s,
                                 const int32_t* hbucket = nullptr, const float* hsign = nullptr);
// R[i, :] = scale * sum_{e in row i, slot[col_e] >= 0} val_e * W[col_e, :]
// (slot == nullptr: every column).  CSR rows x ncols, W is ncols x k.
dsanls_status launch_csr_sketch_rhs(const int64_t* rowptr, const int32_t* colidx,
                                    const float* vals, int64_t rows, const int32_t* slot,
                                    const float* W, int64_t k, float scale, float* R,
                                    hipStream_t s);
// Rows of the sketched matrix A = X S for a subsampling sketch, as CSR:
// row i holds (slot[col], scale * val) for the sampled columns of row i of
// X, in ascending column order.  count: cnt[i] = hits of row i; fill:
// writes them at a_rowptr[i].
dsanls_status launch_csr_hits_count(const int64_t* rowptr, const int32_t* colidx, int64_t rows,
                                    const int32_t* slot, int32_t* cnt, hipStream_t s);
dsanls_status launch_csr_hits_fill(const int64_t* rowptr, const int32_t* colidx, const float* vals,
                                   int64_t rows, const int32_t* slot, float scale,
                                   const int32_t* a_rowptr, int32_t* a_cols, float* a_vals,
                                   hipStream_t s);
// Copy rows sel[0..nsel) of a CSR with nrows rows (int32 offsets) into a
// packed CSR whose offsets out_rowptr come from a scan of the selected row
// lengths; indices outside [0, nrows) select an empty row.
dsanls_status launch_csr_select_len(const int32_t* rowptr, int64_t nrows, const int32_t* sel,
                                    int64_t nsel, int32_t* len, hipStream_t s);
dsanls_status launch_csr_select_copy(const int32_t* rowptr, int64_t nrows, const int32_t* cols,
                                     const float* vals, const int32_t* sel, int64_t nsel,
                                     const int32_t* out_rowptr, int32_t* out_cols, float* out_vals,
                                     hipStream_t s);
// CSR(M^T) (t_rowptr n + 1 int64, t_colidx, t_vals) from CSR(M) (rows x n,
// nnz < 2^31), each row of M^T in ascending column order; workspace of
// csr_transpose_ws_bytes(n) bytes (csr_transpose.hip).
size_t csr_transpose_ws_bytes(int64_t n);
dsanls_status launch_csr_transpose(const int64_t* rowptr, const int32_t* colidx, const float* vals, int64_t rows,
                                   int64_t n, int64_t nnz, int64_t* t_rowptr, int32_t* t_colidx, float* t_vals,
                                   void* ws, size_t ws_bytes, hipStream_t s);
// MLP (mlp.hip)
int64_t mlp_param_count(int d, int k, int hd);
size_t mlp_ws_bytes(int d, int k, int hd, int64_t rows, bool forward_only);
dsanls_status mlp_forward(int d, int k, int hd, bool residual, const float* params, int64_t rows,
                          const int32_t* a_rowptr, const int32_t* a_cols, const float* a_vals,
                          const float* U, float* out, void* ws, size_t ws_bytes, hipStream_t s);
// Sparse objective pieces: sum_nnz M_ij <u_i, v_j> and sum_nnz M_ij^2 as
// compensated partials.
int64_t csr_cross_partials(int64_t rows);
dsanls_status launch_csr_cross(const int64_t* rowptr, const int32_t* colidx, const float* vals,
                               int64_t rows, const float* U, const float* V, int64_t k,
                               float* partials, hipStream_t s);

}  // namespace dsanls
