// CSR(M^T) from CSR(M) on the GPU (init only), for callers that pass CSR(M)
// alone: Alg. 2 reads both M_{I_r:} and M_{:J_r}, and the V half-iteration
// streams the rows of M^T.
//
// Deterministic and with every row of M^T sorted by column (= row of M)
// without a sort: the rows of M are cut into P contiguous blocks; the
// entries of column j that block p holds land at
//     t_rowptr[j] + (entries of column j in blocks before p) + (earlier
//     entries of column j in block p),
// so each block, walking its own rows in order, writes its part of every
// row of M^T in ascending row order, after the parts of the blocks before
// it.  Counts per (block, column) use integer atomics (order-free), and the
// positions inside a block are taken row after row.
#include "common.hpp"

namespace dsanls {

namespace {

constexpr int kTBlocks = 128;   // row blocks P (the count table is P x n ints)

__global__ __launch_bounds__(256) void ct_zero_kernel(int32_t* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += gridDim.x * 256ll) p[i] = 0;
}

// cnt[p * n + j] = entries of column j in row block p
__global__ __launch_bounds__(256) void ct_count_kernel(const int64_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ colidx, int64_t rows,
                                                       int64_t rows_per_block, int64_t n, int32_t* __restrict__ cnt) {
  const int p = blockIdx.x;
  const int64_t r0 = p * rows_per_block, r1 = r0 + rows_per_block < rows ? r0 + rows_per_block : rows;
  if (r0 >= r1) return;
  int32_t* c = cnt + static_cast<int64_t>(p) * n;
  for (int64_t e = rowptr[r0] + threadIdx.x; e < rowptr[r1]; e += 256) atomicAdd(&c[colidx[e]], 1);
}

// total[j] = sum over the blocks of cnt[p * n + j]
__global__ __launch_bounds__(256) void ct_total_kernel(const int32_t* __restrict__ cnt, int64_t n, int nblk,
                                                       int32_t* __restrict__ total) {
  const int64_t j = blockIdx.x * 256ll + threadIdx.x;
  if (j >= n) return;
  int32_t s = 0;
  for (int p = 0; p < nblk; ++p) s += cnt[static_cast<int64_t>(p) * n + j];
  total[j] = s;
}

// cnt[p * n + j] <- t_rowptr[j] + entries of column j in blocks before p
// (the start of block p's part of row j of M^T); t_rowptr as int64
__global__ __launch_bounds__(256) void ct_start_kernel(int32_t* __restrict__ cnt, const int32_t* __restrict__ off,
                                                       int64_t n, int nblk, int64_t* __restrict__ t_rowptr) {
  const int64_t j = blockIdx.x * 256ll + threadIdx.x;
  if (j > n) return;
  t_rowptr[j] = off[j];
  if (j == n) return;
  int32_t s = off[j];
  for (int p = 0; p < nblk; ++p) {
    int32_t* c = cnt + static_cast<int64_t>(p) * n + j;
    const int32_t v = *c;
    *c = s;
    s += v;
  }
}

// Block p walks its rows in order; the entries of a row have distinct
// columns, so each takes its column's next position without conflict, and
// the barrier makes the cursors of one row visible to the next.
__global__ __launch_bounds__(256) void ct_fill_kernel(const int64_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colidx,
                                                      const float* __restrict__ vals, int64_t rows,
                                                      int64_t rows_per_block, int64_t n, int32_t* __restrict__ cur,
                                                      int32_t* __restrict__ t_colidx, float* __restrict__ t_vals) {
  const int p = blockIdx.x;
  const int64_t r0 = p * rows_per_block, r1 = r0 + rows_per_block < rows ? r0 + rows_per_block : rows;
  int32_t* c = cur + static_cast<int64_t>(p) * n;
  for (int64_t r = r0; r < r1; ++r) {
    for (int64_t e = rowptr[r] + threadIdx.x; e < rowptr[r + 1]; e += 256) {
      const int32_t j = colidx[e];
      const int32_t pos = c[j]++;
      t_colidx[pos] = static_cast<int32_t>(r);
      t_vals[pos] = vals[e];
    }
    __syncthreads();
  }
}

}  // namespace

size_t csr_transpose_ws_bytes(int64_t n) {
  return align_up(sizeof(int32_t) * kTBlocks * static_cast<size_t>(n), 256) +
         2 * align_up(sizeof(int32_t) * static_cast<size_t>(n + 1), 256) + align_up(scan_ws_bytes(n), 256);
}

dsanls_status launch_csr_transpose(const int64_t* rowptr, const int32_t* colidx, const float* vals, int64_t rows,
                                   int64_t n, int64_t nnz, int64_t* t_rowptr, int32_t* t_colidx, float* t_vals,
                                   void* ws, size_t ws_bytes, hipStream_t s) {
  if (ws_bytes < csr_transpose_ws_bytes(n)) return fail(DSANLS_E_WORKSPACE, "csr_transpose: workspace too small");
  if (nnz >= (int64_t{1} << 31)) return fail(DSANLS_E_UNSUPPORTED, "csr_transpose: nnz must be < 2^31");
  char* base = static_cast<char*>(ws);
  int32_t* cnt = reinterpret_cast<int32_t*>(base);
  base += align_up(sizeof(int32_t) * kTBlocks * static_cast<size_t>(n), 256);
  int32_t* total = reinterpret_cast<int32_t*>(base);
  base += align_up(sizeof(int32_t) * static_cast<size_t>(n + 1), 256);
  int32_t* off = reinterpret_cast<int32_t*>(base);
  base += align_up(sizeof(int32_t) * static_cast<size_t>(n + 1), 256);
  int32_t* scan_ws = reinterpret_cast<int32_t*>(base);
  const int64_t rpb = ceil_div(std::max<int64_t>(rows, 1), kTBlocks);
  const int64_t tab = static_cast<int64_t>(kTBlocks) * n;
  ct_zero_kernel<<<static_cast<unsigned>(std::min<int64_t>(ceil_div(tab, 256), 8192)), 256, 0, s>>>(cnt, tab);
  DSANLS_LAUNCHED("ct_zero_kernel");
  ct_count_kernel<<<kTBlocks, 256, 0, s>>>(rowptr, colidx, rows, rpb, n, cnt);
  DSANLS_LAUNCHED("ct_count_kernel");
  ct_total_kernel<<<static_cast<unsigned>(ceil_div(n, 256)), 256, 0, s>>>(cnt, n, kTBlocks, total);
  DSANLS_LAUNCHED("ct_total_kernel");
  dsanls_status st = launch_exclusive_scan(total, off, n, scan_ws, s);
  if (st != DSANLS_OK) return st;
  ct_start_kernel<<<static_cast<unsigned>(ceil_div(n + 1, 256)), 256, 0, s>>>(cnt, off, n, kTBlocks, t_rowptr);
  DSANLS_LAUNCHED("ct_start_kernel");
  ct_fill_kernel<<<kTBlocks, 256, 0, s>>>(rowptr, colidx, vals, rows, rpb, n, cnt, t_colidx, t_vals);
  DSANLS_LAUNCHED("ct_fill_kernel");
  return DSANLS_OK;
}

}  // namespace dsanls
