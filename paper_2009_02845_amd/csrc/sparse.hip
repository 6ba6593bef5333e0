// Sparse (CSR) side of the path: the sketch right-hand side R = A B^T for a
// subsampling sketch, and the nnz term of the sparse objective.
//
// With S = sqrt(n/d) [e_{j_1} .. e_{j_d}], A = M S keeps only the sampled
// columns of M and B = V^T S the sampled rows of V, so
//     R[i, :] = (A B^T)[i, :] = (n/d) * sum_{j sampled, M_ij != 0} M_ij V[j, :]
// (Sec. 3.4: subsampling keeps the sparsity of M).  One wave streams the
// nnz of a row in coalesced 64-entry chunks, tests each column against the
// sampled-slot map, and folds the hits, in ascending column order, into a
// k-vector held across the lanes (two components per lane for k <= 128).
#include "common.hpp"

namespace dsanls {

namespace {

constexpr int64_t kSeg = kCsrSegment;

__device__ __forceinline__ void neumaier(float& s, float& c, float x) {
  const float t = s + x;
  c += fabsf(s) >= fabsf(x) ? (s - t) + x : (x - t) + s;
  s = t;
}

__global__ __launch_bounds__(256) void csr_rhs_kernel(const int64_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colidx,
                                                      const float* __restrict__ vals,
                                                      int64_t rows,
                                                      const int32_t* __restrict__ slot,
                                                      const float* __restrict__ W, int k,
                                                      float scale, float* __restrict__ R) {
  const int64_t row = blockIdx.x * 4ll + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= rows) return;
  const int64_t beg = rowptr[row], end = rowptr[row + 1];
  float a0 = 0.f, a1 = 0.f;
  for (int64_t base = beg; base < end; base += 64) {
    const int64_t e = base + lane;
    int32_t col = -1;
    float v = 0.f;
    if (e < end) {
      col = colidx[e];
      if (slot != nullptr && slot[col] < 0) col = -1;
      if (col >= 0) v = vals[e];
    }
    unsigned long long mask = __ballot(col >= 0);
    while (mask != 0ull) {
      const int b = __ffsll(mask) - 1;
      mask &= mask - 1ull;
      const int32_t c = __shfl(col, b, 64);
      const float x = __shfl(v, b, 64);
      const float* w = W + (int64_t)c * k;
      if (lane < k) a0 += x * w[lane];
      if (lane + 64 < k) a1 += x * w[lane + 64];
    }
  }
  float* r = R + row * k;
  if (lane < k) r[lane] = scale * a0;
  if (lane + 64 < k) r[lane + 64] = scale * a1;
}

// Segmented form of the stream: rows longer than kSeg nnz are split into
// segments (built once at init, the CSR structure being fixed), one wave
// per segment, so a Zipf-popular column of M^T (hundreds of thousands of
// entries) is shared by many waves instead of serialising one.  A segment
// of a single-segment row writes R directly; the segments of a longer row
// write partial k-vectors that a fixup sums in segment order.
// HASHED (count sketch): every entry counts, and entry (i, j) adds
// M_ij s_j T[h_j, :] with T = B^T (d x k) read at the bucket h_j of its
// column, instead of M_ij W[j, :] over the sampled columns.
template <bool HASHED>
__global__ __launch_bounds__(256) void csr_rhs_seg_kernel(const int64_t* __restrict__ rowptr,
                                                          const int32_t* __restrict__ colidx,
                                                          const float* __restrict__ vals,
                                                          const int32_t* __restrict__ seg_row,
                                                          const int64_t* __restrict__ seg_beg,
                                                          const int32_t* __restrict__ seg_part,
                                                          int64_t nseg,
                                                          const int32_t* __restrict__ slot,
                                                          const float* __restrict__ W, int k, int64_t ldw,
                                                          float scale, float* __restrict__ R, int64_t ldr,
                                                          float* __restrict__ P,
                                                          const int32_t* __restrict__ hbucket,
                                                          const float* __restrict__ hsign) {
  const int64_t sg = blockIdx.x * 4ll + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (sg >= nseg) return;
  const int64_t row = seg_row[sg];
  const int64_t beg = seg_beg[sg];
  const int64_t rend = rowptr[row + 1];
  const int64_t end = beg + kSeg < rend ? beg + kSeg : rend;
  float a0 = 0.f, a1 = 0.f;
  for (int64_t base = beg; base < end; base += 64) {
    const int64_t e = base + lane;
    int32_t col = -1;
    float v = 0.f;
    if (e < end) {
      col = colidx[e];
      if (HASHED) {
        v = vals[e] * hsign[col];
        col = hbucket[col];
      } else {
        if (slot != nullptr && slot[col] < 0) col = -1;
        if (col >= 0) v = vals[e];
      }
    }
    unsigned long long mask = __ballot(col >= 0);
    while (mask != 0ull) {
      // up to 8 hits at a time (wave-uniform: read from their lanes into
      // scalar registers), their rows of W loaded together so that the
      // loads overlap; the FMAs follow in the hits' order
      constexpr int U = 8;
      int32_t cs[U];
      float xs[U];
      int cnt = 0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        cs[u] = 0;
        xs[u] = 0.f;
        if (mask != 0ull) {
          const int b = __ffsll(mask) - 1;
          mask &= mask - 1ull;
          cs[u] = __builtin_amdgcn_readlane(col, b);
          xs[u] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), b));
          cnt = u + 1;
        }
      }
      float w0[U], w1[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const float* w = W + (int64_t)cs[u] * ldw;
        w0[u] = u < cnt && lane < k ? w[lane] : 0.f;
        w1[u] = u < cnt && lane + 64 < k ? w[lane + 64] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (u < cnt) {
          a0 += xs[u] * w0[u];
          a1 += xs[u] * w1[u];
        }
      }
    }
  }
  const int32_t part = seg_part[sg];
  float* out = part < 0 ? R + row * ldr : P + (int64_t)part * k;
  const float sc = part < 0 ? scale : 1.0f;
  if (lane < k) out[lane] = sc * a0;
  if (lane + 64 < k) out[lane + 64] = sc * a1;
}

// R[row] = scale * sum of the row's segment partials, in segment order.
__global__ __launch_bounds__(256) void csr_rhs_fixup_kernel(const int32_t* __restrict__ multi_row,
                                                            const int32_t* __restrict__ multi_part,
                                                            int64_t nmulti, int k, float scale,
                                                            const float* __restrict__ P,
                                                            float* __restrict__ R, int64_t ldr) {
  const int64_t i = blockIdx.x * 4ll + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= nmulti) return;
  const int64_t row = multi_row[i];
  const int32_t p0 = multi_part[i], p1 = multi_part[i + 1];
  float a0 = 0.f, a1 = 0.f;
  for (int32_t p = p0; p < p1; ++p) {
    if (lane < k) a0 += P[(int64_t)p * k + lane];
    if (lane + 64 < k) a1 += P[(int64_t)p * k + lane + 64];
  }
  if (lane < k) R[row * ldr + lane] = scale * a0;
  if (lane + 64 < k) R[row * ldr + lane + 64] = scale * a1;
}

// Sketched rows per segment: count the sampled hits of every segment, then
// (after a scan over segments, which are in row-major order) write them.
__global__ __launch_bounds__(256) void seg_hits_count_kernel(const int64_t* __restrict__ rowptr,
                                                             const int32_t* __restrict__ colidx,
                                                             const int32_t* __restrict__ seg_row,
                                                             const int64_t* __restrict__ seg_beg,
                                                             int64_t nseg,
                                                             const int32_t* __restrict__ slot,
                                                             int32_t* __restrict__ cnt) {
  const int64_t sg = blockIdx.x * 4ll + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (sg >= nseg) return;
  const int64_t beg = seg_beg[sg], rend = rowptr[seg_row[sg] + 1];
  const int64_t end = beg + kSeg < rend ? beg + kSeg : rend;
  int32_t c = 0;
  for (int64_t base = beg; base < end; base += 64) {
    const int64_t e = base + lane;
    c += __popcll(__ballot(e < end && slot[colidx[e]] >= 0));
  }
  if (lane == 0) cnt[sg] = c;
}

// a_rowptr[row] = start of the row's first segment; a_rowptr[rows] = total.
__global__ __launch_bounds__(256) void seg_rowptr_kernel(const int64_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ seg_row,
                                                         const int64_t* __restrict__ seg_beg,
                                                         int64_t nseg, int64_t rows,
                                                         const int32_t* __restrict__ spos,
                                                         int32_t* __restrict__ a_rowptr) {
  const int64_t sg = blockIdx.x * 256ll + threadIdx.x;
  if (sg < nseg) {
    const int32_t r = seg_row[sg];
    if (seg_beg[sg] == rowptr[r]) a_rowptr[r] = spos[sg];
  }
  if (sg == 0) a_rowptr[rows] = spos[nseg];
}

__global__ __launch_bounds__(256) void seg_hits_fill_kernel(const int64_t* __restrict__ rowptr,
                                                            const int32_t* __restrict__ colidx,
                                                            const float* __restrict__ vals,
                                                            const int32_t* __restrict__ seg_row,
                                                            const int64_t* __restrict__ seg_beg,
                                                            int64_t nseg,
                                                            const int32_t* __restrict__ slot,
                                                            float scale,
                                                            const int32_t* __restrict__ spos,
                                                            int32_t* __restrict__ a_cols,
                                                            float* __restrict__ a_vals) {
  const int64_t sg = blockIdx.x * 4ll + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (sg >= nseg) return;
  const int64_t beg = seg_beg[sg], rend = rowptr[seg_row[sg] + 1];
  const int64_t end = beg + kSeg < rend ? beg + kSeg : rend;
  int32_t pos = spos[sg];
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int64_t base = beg; base < end; base += 64) {
    const int64_t e = base + lane;
    int32_t sl = -1;
    if (e < end) sl = slot[colidx[e]];
    const unsigned long long mask = __ballot(sl >= 0);
    if (sl >= 0) {
      const int32_t at = pos + __popcll(mask & below);
      a_cols[at] = sl;
      a_vals[at] = scale * vals[e];
    }
    pos += __popcll(mask);
  }
}

__global__ __launch_bounds__(256) void csr_hits_count_kernel(const int64_t* __restrict__ rowptr,
                                                             const int32_t* __restrict__ colidx,
                                                             int64_t rows,
                                                             const int32_t* __restrict__ slot,
                                                             int32_t* __restrict__ cnt) {
  const int64_t row = blockIdx.x * 4ll + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= rows) return;
  const int64_t beg = rowptr[row], end = rowptr[row + 1];
  int32_t c = 0;
  for (int64_t base = beg; base < end; base += 64) {
    const int64_t e = base + lane;
    const bool hit = e < end && slot[colidx[e]] >= 0;
    c += __popcll(__ballot(hit));
  }
  if (lane == 0) cnt[row] = c;
}

__global__ __launch_bounds__(256) void csr_hits_fill_kernel(const int64_t* __restrict__ rowptr,
                                                            const int32_t* __restrict__ colidx,
                                                            const float* __restrict__ vals,
                                                            int64_t rows,
                                                            const int32_t* __restrict__ slot,
                                                            float scale,
                                                            const int32_t* __restrict__ a_rowptr,
                                                            int32_t* __restrict__ a_cols,
                                                            float* __restrict__ a_vals) {
  const int64_t row = blockIdx.x * 4ll + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= rows) return;
  const int64_t beg = rowptr[row], end = rowptr[row + 1];
  int32_t pos = a_rowptr[row];
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int64_t base = beg; base < end; base += 64) {
    const int64_t e = base + lane;
    int32_t sl = -1;
    if (e < end) sl = slot[colidx[e]];
    const unsigned long long mask = __ballot(sl >= 0);
    if (sl >= 0) {
      const int32_t at = pos + __popcll(mask & below);
      a_cols[at] = sl;
      a_vals[at] = scale * vals[e];
    }
    pos += __popcll(mask);
  }
}

__global__ __launch_bounds__(256) void select_len_kernel(const int32_t* __restrict__ rowptr,
                                                         int64_t nrows,
                                                         const int32_t* __restrict__ sel, int64_t nsel,
                                                         int32_t* __restrict__ len) {
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= nsel) return;
  const int32_t r = sel[i];
  len[i] = (r >= 0 && r < nrows) ? rowptr[r + 1] - rowptr[r] : 0;
}

__global__ __launch_bounds__(256) void select_copy_kernel(const int32_t* __restrict__ rowptr,
                                                          int64_t nrows,
                                                          const int32_t* __restrict__ cols,
                                                          const float* __restrict__ vals,
                                                          const int32_t* __restrict__ sel,
                                                          int64_t nsel,
                                                          const int32_t* __restrict__ out_rowptr,
                                                          int32_t* __restrict__ out_cols,
                                                          float* __restrict__ out_vals) {
  const int64_t i = blockIdx.x * 4ll + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= nsel) return;
  const int32_t r = sel[i];
  if (r < 0 || r >= nrows) return;
  const int32_t beg = rowptr[r], len = rowptr[r + 1] - beg, dst = out_rowptr[i];
  for (int32_t e = lane; e < len; e += 64) {
    out_cols[dst + e] = cols[beg + e];
    out_vals[dst + e] = vals[beg + e];
  }
}

constexpr int kCrossBlocks = 2048;

// Per wave, rows i = wave_id, wave_id + total_waves, ...: (M V)_i is
// accumulated across the lanes, dotted with u_i, and added (compensated)
// to the wave's running sum; sum of M_ij^2 alongside.  Partials: four
// floats per block (cross sum, comp, square sum, comp).
__global__ __launch_bounds__(256) void csr_cross_kernel(const int64_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ colidx,
                                                        const float* __restrict__ vals,
                                                        int64_t rows, const float* __restrict__ U,
                                                        const float* __restrict__ V, int k,
                                                        float* __restrict__ partials) {
  __shared__ float red[4 * 4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nw = (int64_t)gridDim.x * 4;
  float cs = 0.f, cc = 0.f, qs = 0.f, qc = 0.f;
  for (int64_t row = blockIdx.x * 4ll + wave; row < rows; row += nw) {
    const int64_t beg = rowptr[row], end = rowptr[row + 1];
    float sq = 0.f, sqc = 0.f, dot = 0.f;
    // the lanes hold two columns each: ranks above 128 in chunks of 128
    for (int c0 = 0; c0 < k; c0 += 128) {
      const int kc = k - c0 < 128 ? k - c0 : 128;
      float a0 = 0.f, a1 = 0.f;
      for (int64_t base = beg; base < end; base += 64) {
        const int64_t e = base + lane;
        int32_t col = 0;
        float v = 0.f;
        if (e < end) {
          col = colidx[e];
          v = vals[e];
        }
        if (c0 == 0) neumaier(sq, sqc, v * v);
        const int cnt = static_cast<int>(end - base < 64 ? end - base : 64);
        for (int b = 0; b < cnt; ++b) {
          const int32_t c = __shfl(col, b, 64);
          const float x = __shfl(v, b, 64);
          const float* w = V + (int64_t)c * k + c0;
          if (lane < kc) a0 += x * w[lane];
          if (lane + 64 < kc) a1 += x * w[lane + 64];
        }
      }
      const float* u = U + row * k + c0;
      if (lane < kc) dot += u[lane] * a0;
      if (lane + 64 < kc) dot += u[lane + 64] * a1;
    }
    for (int off = 32; off > 0; off >>= 1) dot += __shfl_down(dot, off, 64);
    for (int off = 32; off > 0; off >>= 1) {
      const float os = __shfl_down(sq, off, 64), oc = __shfl_down(sqc, off, 64);
      neumaier(sq, sqc, os);
      sqc += oc;
    }
    if (lane == 0) {
      neumaier(cs, cc, dot);
      neumaier(qs, qc, sq);
      qc += sqc;
    }
  }
  if (lane == 0) {
    red[4 * wave] = cs;
    red[4 * wave + 1] = cc;
    red[4 * wave + 2] = qs;
    red[4 * wave + 3] = qc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = red[0], ac = red[1], b = red[2], bc = red[3];
    for (int w = 1; w < 4; ++w) {
      neumaier(a, ac, red[4 * w]);
      ac += red[4 * w + 1];
      neumaier(b, bc, red[4 * w + 2]);
      bc += red[4 * w + 3];
    }
    partials[4 * blockIdx.x] = a;
    partials[4 * blockIdx.x + 1] = ac;
    partials[4 * blockIdx.x + 2] = b;
    partials[4 * blockIdx.x + 3] = bc;
  }
}


// ---------------------------------------------------------------------------
// Sampled-column gather.  The sketched rows A = X S of a subsampling sketch
// hold only the sampled columns X[:, idx[c]] (scaled), and column idx[c] of X
// is row idx[c] of the transposed CSR: reading those rows touches about d/n
// of the nnz instead of streaming all of them.  The entries are bucketed by
// row (count, scan, fill), then every row is sorted by slot c (= ascending
// column of X, the subsample being in index order), which makes the result
// independent of the order the atomics ran in.

// Rows of A with up to kShortRow entries are sorted by a_rhs_kernel itself
// (one lane each, in registers); longer ones (at most d <= kLongCap) by
// row_sort_long_kernel first.
constexpr int kShortRow = 8;
constexpr int kLongCap = 4096;

// len[c] = nnz of column idx[c] of X (row idx[c] of X^T).
__global__ __launch_bounds__(256) void gather_len_kernel(const int64_t* __restrict__ t_rowptr,
                                                         const int32_t* __restrict__ idx, int d,
                                                         int32_t* __restrict__ len) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  // a sampled column outside this block (idx[c] < 0) has no entries here
  if (c < d) len[c] = idx[c] >= 0 ? static_cast<int32_t>(t_rowptr[idx[c] + 1] - t_rowptr[idx[c]]) : 0;
}

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += gridDim.x * 256ll) p[i] = v;
}

// Walks the E = offs[d] sampled entries as one flat range, 64 per wave step
// (offs = exclusive scan of len): COUNT adds one to cnt[row] per entry; the
// fill pass takes a slot of its row from the back (cnt counts down), writes
// (c, scale * value) there and lists the rows longer than kShortRow.
template <bool COUNT>
__global__ __launch_bounds__(256) void gather_entries_kernel(const int64_t* __restrict__ t_rowptr,
                                                             const int32_t* __restrict__ t_colidx,
                                                             const float* __restrict__ t_vals,
                                                             const int32_t* __restrict__ idx,
                                                             const int32_t* __restrict__ offs, int d,
                                                             int32_t* __restrict__ cnt,
                                                             const int32_t* __restrict__ a_rowptr,
                                                             int32_t* __restrict__ a_cols,
                                                             float* __restrict__ a_vals, float scale,
                                                             int32_t* __restrict__ long_rows,
                                                             int32_t* __restrict__ nlong) {
  const int lane = threadIdx.x & 63;
  const int32_t E = offs[d];
  const int64_t step = static_cast<int64_t>(gridDim.x) * 4;
  for (int64_t tile = blockIdx.x * 4ll + (threadIdx.x >> 6); tile * 64 < E; tile += step) {
    const int32_t fb = static_cast<int32_t>(tile * 64);
    // column of the tile's first entry: the last c with offs[c] <= fb
    int lo = 0, hi = d - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (offs[mid] <= fb) lo = mid;
      else hi = mid - 1;
    }
    const int32_t f = fb + lane;
    if (f >= E) continue;
    int c = lo;
    while (offs[c + 1] <= f) ++c;
    const int64_t e = t_rowptr[idx[c]] + (f - offs[c]);
    const int32_t row = t_colidx[e];
    if (COUNT) {
      atomicAdd(&cnt[row], 1);
    } else {
      const int32_t left = atomicSub(&cnt[row], 1) - 1;
      const int32_t pos = a_rowptr[row] + left;
      a_cols[pos] = c;
      a_vals[pos] = scale * t_vals[e];
      // the entry that takes a row's last free slot lists the row if it is
      // longer than a_rhs_kernel sorts itself
      if (left == 0 && a_rowptr[row + 1] - a_rowptr[row] > kShortRow) long_rows[atomicAdd(nlong, 1)] = row;
    }
  }
}

// Listed rows of kShortRow < length <= kMidRow entries (most of the listed
// rows): one wave each, a bitonic sort of (slot, value) by slot in
// registers, lane i holding entry i and its partner reached by a shuffle
// (no barriers); the waves walk the list.  Slots within a row are distinct.
constexpr int kMidRow = 64;
__global__ __launch_bounds__(256) void row_sort_mid_kernel(const int32_t* __restrict__ a_rowptr,
                                                           int32_t* __restrict__ a_cols,
                                                           float* __restrict__ a_vals,
                                                           const int32_t* __restrict__ long_rows,
                                                           const int32_t* __restrict__ nlong) {
  const int lane = threadIdx.x & 63;
  const int n_long = *nlong;
  const int64_t nw = gridDim.x * 4ll;
  for (int64_t li = blockIdx.x * 4ll + (threadIdx.x >> 6); li < n_long; li += nw) {
    const int32_t i = long_rows[li];
    const int32_t b = a_rowptr[i], n = a_rowptr[i + 1] - b;
    if (n > kMidRow) continue;
    int32_t key = lane < n ? a_cols[b + lane] : 0x7fffffff;
    float val = lane < n ? a_vals[b + lane] : 0.f;
#pragma unroll
    for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        const int32_t ok = __shfl_xor(key, stride, 64);
        const float ov = __shfl_xor(val, stride, 64);
        // the pair's lower lane keeps the smaller key in an ascending block
        // (lane & size == 0) and the larger in a descending one
        const bool up = (lane & size) == 0, lower = (lane & stride) == 0;
        if (lower == up ? ok < key : ok > key) {
          key = ok;
          val = ov;
        }
      }
    }
    if (lane < n) {
      a_cols[b + lane] = key;
      a_vals[b + lane] = val;
    }
  }
}

// Listed rows of kMidRow < length <= kLongCap entries: one workgroup per
// row (the workgroups walk the list).  The slots of a row are distinct
// columns of the subsample, below d <= kLongCap, so the row is put in slot
// order by counting: each entry marks its slot in an LDS map of d words,
// then every thread takes a contiguous run of slots and writes the marked
// ones at its exclusive prefix count (O(d + n) per row; the bitonic network
// it replaces took 66 barrier-separated stages for a 2000-entry row).  A
// row whose slots repeat (a CSR with duplicate entries, outside the
// interface's contract) is sorted by a bitonic network instead, so no entry
// is ever lost.
__global__ __launch_bounds__(256) void row_sort_long_kernel(const int32_t* __restrict__ a_rowptr,
                                                            int32_t* __restrict__ a_cols,
                                                            float* __restrict__ a_vals,
                                                            const int32_t* __restrict__ long_rows,
                                                            const int32_t* __restrict__ nlong, int d) {
  __shared__ int32_t key[kLongCap];
  __shared__ float val[kLongCap];
  __shared__ int32_t at[kLongCap];   // slot -> entry of the row, or -1
  __shared__ int32_t wsum[4];
  __shared__ int dup;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int run = (d + 255) / 256;   // slots per thread
  const int n_long = *nlong;
  for (int r = blockIdx.x; r < n_long; r += gridDim.x) {
    const int32_t i = long_rows[r];
    const int32_t b = a_rowptr[i], n = a_rowptr[i + 1] - b;
    if (n <= kMidRow || n > kLongCap) continue;   // the wave sort's, or (duplicate CSR entries) too long
    __syncthreads();
    for (int c = tid; c < d; c += 256) at[c] = -1;
    if (tid == 0) dup = 0;
    __syncthreads();
    for (int e = tid; e < n; e += 256) {
      const int32_t c = a_cols[b + e];
      val[e] = a_vals[b + e];
      key[e] = c;
      if (c < 0 || c >= d || atomicExch(&at[c], e) >= 0) dup = 1;
    }
    __syncthreads();
    if (!dup) {
      const int c0 = tid * run, c1 = c0 + run < d ? c0 + run : d;
      int cnt = 0;
      for (int c = c0; c < c1; ++c) cnt += at[c] >= 0;
      int incl = cnt;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
      }
      if (lane == 63) wsum[w] = incl;
      __syncthreads();
      int pos = incl - cnt;
      for (int q = 0; q < w; ++q) pos += wsum[q];
      for (int c = c0; c < c1; ++c) {
        const int32_t e = at[c];
        if (e >= 0) {
          a_cols[b + pos] = c;
          a_vals[b + pos] = val[e];
          ++pos;
        }
      }
      continue;
    }
    int P = 1;
    while (P < n) P <<= 1;
    for (int t = n + tid; t < P; t += 256) {
      key[t] = 0x7fffffff;
      val[t] = 0.f;
    }
    for (int size = 2; size <= P; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        __syncthreads();
        for (int t = tid; t < (P >> 1); t += 256) {
          const int lo = 2 * stride * (t / stride) + (t % stride), hi = lo + stride;
          const bool up = (lo & size) == 0;
          if ((key[lo] > key[hi]) == up) {
            const int32_t kt = key[lo];
            key[lo] = key[hi];
            key[hi] = kt;
            const float vt = val[lo];
            val[lo] = val[hi];
            val[hi] = vt;
          }
        }
      }
    }
    __syncthreads();
    for (int t = tid; t < n; t += 256) {
      a_cols[b + t] = key[t];
      a_vals[b + t] = val[t];
    }
  }
}

// R[i, :] = scale * sum over row i of A, in slot order, of a_vals[e] *
// W[idx[a_cols[e]], :] (W row-major, row length k <= 128), 64 rows per wave
// and the lanes over the columns of R (lane, lane + 64).
//  * A row of at most kShortRow entries arrives in fill order: its lane
//    sorts it in registers (odd-even transposition), writes it back (so A
//    leaves sorted) and puts (W row, value, row) into the wave's flat entry
//    list in LDS, rows in order.  The wave walks the list four entries at a
//    time, the four W rows loaded before their FMAs, and writes each R row
//    (zero for a row without short entries) when the list moves past it.
//  * A longer row (listed and sorted by row_sort_long_kernel) gets a zero
//    row here and its value from a_rhs_long_kernel afterwards.
__global__ __launch_bounds__(256) void a_rhs_kernel(const int32_t* __restrict__ a_rowptr,
                                                    int32_t* __restrict__ a_cols,
                                                    float* __restrict__ a_vals, int64_t rows,
                                                    const int32_t* __restrict__ idx,
                                                    const float* __restrict__ W, int k, int64_t ldw,
                                                    float scale, float* __restrict__ R, int64_t ldr) {
  __shared__ int32_t s_j[4][64 * kShortRow];
  __shared__ float s_v[4][64 * kShortRow];
  __shared__ int32_t s_r[4][64 * kShortRow];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t row0 = (blockIdx.x * 4ll + w) * 64;
  if (row0 >= rows) return;   // whole waves only; no block barrier below
  const int nrows = static_cast<int>(rows - row0 < 64 ? rows - row0 : 64);
  int32_t b = 0, n = 0;
  if (lane < nrows) {
    b = a_rowptr[row0 + lane];
    n = a_rowptr[row0 + lane + 1] - b;
  }
  const bool is_short = n <= kShortRow;
  const int ns = is_short ? n : 0;
  int32_t c[kShortRow];
  float v[kShortRow];
  // unconditional loads (entry q clamped into the row, or the lane's row
  // start, always inside A) so that they are all in flight at once
#pragma unroll
  for (int q = 0; q < kShortRow; ++q) {
    const int32_t e = b + (q < ns ? q : 0);
    const int32_t cq = a_cols[e];
    const float vq = a_vals[e];
    c[q] = q < ns ? cq : 0x7fffffff;
    v[q] = q < ns ? vq : 0.f;
  }
#pragma unroll
  for (int round = 0; round < kShortRow; ++round) {
#pragma unroll
    for (int q = round & 1; q + 1 < kShortRow; q += 2) {
      if (c[q] > c[q + 1]) {
        const int32_t ct = c[q];
        c[q] = c[q + 1];
        c[q + 1] = ct;
        const float vt = v[q];
        v[q] = v[q + 1];
        v[q + 1] = vt;
      }
    }
  }
  // flat offset of this lane's entries: exclusive scan of ns over the lanes
  int incl = ns;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  const int off = incl - ns;
  const int total = __shfl(incl, 63, 64);
#pragma unroll
  for (int q = 0; q < kShortRow; ++q) {
    if (q < ns) {
      if (ns > 1) {
        a_cols[b + q] = c[q];
        a_vals[b + q] = v[q];
      }
      s_j[w][off + q] = idx[c[q]];
      s_v[w][off + q] = v[q];
      s_r[w][off + q] = lane;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const bool in0 = lane < k, in1 = lane + 64 < k;
  const int col0 = in0 ? lane : k - 1, col1 = in1 ? lane + 64 : k - 1;   // in-row load columns
  float* Rw = R + row0 * ldr;
  float a0 = 0.f, a1 = 0.f;
  int cur = 0;   // next R row of the wave to write
  for (int t0 = 0; t0 < total; t0 += 4) {
    float x0[4], x1[4], vv[4];
    int rr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = t0 + q < total ? t0 + q : t0;
      const float* wr = W + static_cast<int64_t>(s_j[w][t]) * ldw;
      const float y0 = wr[col0], y1 = wr[col1];
      x0[q] = in0 ? y0 : 0.f;
      x1[q] = in1 ? y1 : 0.f;
      vv[q] = s_v[w][t];
      rr[q] = __builtin_amdgcn_readfirstlane(s_r[w][t]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (t0 + q < total) {
        while (cur < rr[q]) {
          if (in0) Rw[static_cast<int64_t>(cur) * ldr + lane] = scale * a0;
          if (in1) Rw[static_cast<int64_t>(cur) * ldr + lane + 64] = scale * a1;
          a0 = a1 = 0.f;
          ++cur;
        }
        a0 += vv[q] * x0[q];
        a1 += vv[q] * x1[q];
      }
    }
  }
  while (cur < nrows) {
    if (in0) Rw[static_cast<int64_t>(cur) * ldr + lane] = scale * a0;
    if (in1) Rw[static_cast<int64_t>(cur) * ldr + lane + 64] = scale * a1;
    a0 = a1 = 0.f;
    ++cur;
  }
}

// R rows of the listed (long, sorted) rows of A with min_len <= length <=
// max_len: one workgroup per row, the row's entries split into NWV
// consecutive parts, one per wave (four waves up to kVeryLongRow entries,
// sixteen beyond, so that a 2000-entry row is not one wave's 500-step
// chain); a wave loads 64 entries at a time (slot, value, W row), then walks
// them with the lanes over the columns of R, kLongBatch W rows in flight.
// The partial sums are added in wave order, so the result depends only on
// the row.
constexpr int kLongBatch = 8;      // W rows in flight per wave (16: 1.2x slower)
constexpr int kVeryLongRow = 512;  // longer rows get four times the waves
template <int NWV>
__global__ __launch_bounds__(64 * NWV) void a_rhs_long_kernel(const int32_t* __restrict__ a_rowptr,
                                                              const int32_t* __restrict__ a_cols,
                                                              const float* __restrict__ a_vals,
                                                              const int32_t* __restrict__ idx,
                                                              const float* __restrict__ W, int k, int64_t ldw,
                                                              float scale, const int32_t* __restrict__ long_rows,
                                                              const int32_t* __restrict__ nlong, int min_len,
                                                              int max_len, float* __restrict__ R, int64_t ldr) {
  __shared__ float part[NWV][128];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool in0 = lane < k, in1 = lane + 64 < k;
  const int col0 = in0 ? lane : k - 1, col1 = in1 ? lane + 64 : k - 1;
  const int n_long = *nlong;
  for (int li = blockIdx.x; li < n_long; li += gridDim.x) {
    const int32_t row = long_rows[li];
    const int32_t rb = a_rowptr[row], n = a_rowptr[row + 1] - rb;
    if (n < min_len || n > max_len) continue;
    const int32_t qn = (n + NWV - 1) / NWV;
    const int32_t beg = rb + (w * qn < n ? w * qn : n), end = rb + ((w + 1) * qn < n ? (w + 1) * qn : n);
    float a0 = 0.f, a1 = 0.f;
    for (int32_t e0 = beg; e0 < end; e0 += 64) {
      const int cn = end - e0 < 64 ? end - e0 : 64;
      const int32_t e = e0 + (lane < cn ? lane : 0);
      const int32_t j = idx[a_cols[e]];
      const float v = a_vals[e];
      for (int r0 = 0; r0 < cn; r0 += kLongBatch) {
        float x0[kLongBatch], x1[kLongBatch], vv[kLongBatch];
#pragma unroll
        for (int q = 0; q < kLongBatch; ++q) {
          const int r = r0 + q < cn ? r0 + q : r0;
          const float* wr = W + static_cast<int64_t>(__shfl(j, r, 64)) * ldw;
          const float y0 = wr[col0], y1 = wr[col1];
          x0[q] = in0 ? y0 : 0.f;
          x1[q] = in1 ? y1 : 0.f;
          vv[q] = r0 + q < cn ? __shfl(v, r, 64) : 0.f;
        }
#pragma unroll
        for (int q = 0; q < kLongBatch; ++q) {
          if (r0 + q < cn) {
            a0 += vv[q] * x0[q];
            a1 += vv[q] * x1[q];
          }
        }
      }
    }
    __syncthreads();
    part[w][lane] = a0;
    part[w][lane + 64] = a1;
    __syncthreads();
    if (w == 0) {
      float s0 = part[0][lane], s1 = part[0][lane + 64];
#pragma unroll
      for (int q = 1; q < NWV; ++q) {
        s0 += part[q][lane];
        s1 += part[q][lane + 64];
      }
      if (in0) R[static_cast<int64_t>(row) * ldr + lane] = scale * s0;
      if (in1) R[static_cast<int64_t>(row) * ldr + lane + 64] = scale * s1;
    }
  }
}

}  // namespace

dsanls_status launch_csr_sketch_rhs(const int64_t* rowptr, const int32_t* colidx, const float* vals,
                                    int64_t rows, const int32_t* slot, const float* W, int64_t k,
                                    float scale, float* R, hipStream_t s) {
  if (rows <= 0) return DSANLS_OK;
  if (k > 128) return fail(DSANLS_E_UNSUPPORTED, "CSR path supports k <= 128");
  csr_rhs_kernel<<<static_cast<unsigned>(ceil_div(rows, 4)), 256, 0, s>>>(
      rowptr, colidx, vals, rows, slot, W, static_cast<int>(k), scale, R);
  DSANLS_LAUNCHED("csr_rhs_kernel");
  return DSANLS_OK;
}

dsanls_status launch_csr_rhs_seg(const int64_t* rowptr, const int32_t* colidx, const float* vals,
                                 const CsrSegments& sg, const int32_t* slot, const float* W, int64_t k,
                                 float scale, float* R, float* P, hipStream_t s, const int32_t* hbucket,
                                 const float* hsign) {
  if (sg.nseg <= 0) return DSANLS_OK;
  const unsigned g = static_cast<unsigned>(ceil_div(sg.nseg, 4));
  // columns of R in chunks of 128 (two per lane); the partials of long rows
  // are laid out per chunk
  for (int64_t c0 = 0; c0 < k; c0 += 128) {
    const int kc = static_cast<int>(std::min<int64_t>(128, k - c0));
    if (hbucket != nullptr)
      csr_rhs_seg_kernel<true><<<g, 256, 0, s>>>(rowptr, colidx, vals, sg.seg_row, sg.seg_beg, sg.seg_part,
                                                 sg.nseg, nullptr, W + c0, kc, k, scale, R + c0, k, P, hbucket,
                                                 hsign);
    else
      csr_rhs_seg_kernel<false><<<g, 256, 0, s>>>(rowptr, colidx, vals, sg.seg_row, sg.seg_beg, sg.seg_part,
                                                  sg.nseg, slot, W + c0, kc, k, scale, R + c0, k, P, nullptr,
                                                  nullptr);
    DSANLS_LAUNCHED("csr_rhs_seg_kernel");
    if (sg.nmulti > 0) {
      csr_rhs_fixup_kernel<<<static_cast<unsigned>(ceil_div(sg.nmulti, 4)), 256, 0, s>>>(
          sg.multi_row, sg.multi_part, sg.nmulti, kc, scale, P, R + c0, k);
      DSANLS_LAUNCHED("csr_rhs_fixup_kernel");
    }
  }
  return DSANLS_OK;
}


dsanls_status launch_sampled_rows(const int64_t* t_rowptr, const int32_t* t_colidx, const float* t_vals,
                                  int64_t rows, const int32_t* idx, int64_t d, float scale, int32_t* cnt,
                                  int32_t* offs, int32_t* scan_ws, int32_t* a_rowptr, int32_t* a_cols,
                                  float* a_vals, int32_t* long_rows, int32_t* nlong, hipStream_t s) {
  if (d < 1 || d > kGatherMaxD) return fail(DSANLS_E_UNSUPPORTED, "sampled-column gather needs 1 <= d <= 4096");
  // column lengths (into a_rowptr, free until the row scan) -> offs
  gather_len_kernel<<<static_cast<unsigned>(ceil_div(d, 256)), 256, 0, s>>>(t_rowptr, idx, static_cast<int>(d),
                                                                           a_rowptr);
  DSANLS_LAUNCHED("gather_len_kernel");
  dsanls_status st = launch_exclusive_scan(a_rowptr, offs, d, scan_ws, s);
  if (st != DSANLS_OK) return st;
  const unsigned zg = static_cast<unsigned>(std::min<int64_t>(ceil_div(rows + 1, 256), 4096));
  fill_i32_kernel<<<zg, 256, 0, s>>>(cnt, rows + 1, 0);
  DSANLS_LAUNCHED("fill_i32_kernel");
  fill_i32_kernel<<<1, 256, 0, s>>>(nlong, 1, 0);
  DSANLS_LAUNCHED("fill_i32_kernel");
  const unsigned eg = 2048;
  gather_entries_kernel<true><<<eg, 256, 0, s>>>(t_rowptr, t_colidx, t_vals, idx, offs, static_cast<int>(d), cnt,
                                                 nullptr, nullptr, nullptr, scale, nullptr, nullptr);
  DSANLS_LAUNCHED("gather_entries_kernel");
  if ((st = launch_exclusive_scan(cnt, a_rowptr, rows, scan_ws, s)) != DSANLS_OK) return st;
  gather_entries_kernel<false><<<eg, 256, 0, s>>>(t_rowptr, t_colidx, t_vals, idx, offs, static_cast<int>(d), cnt,
                                                  a_rowptr, a_cols, a_vals, scale, long_rows, nlong);
  DSANLS_LAUNCHED("gather_entries_kernel");
  if (rows > 0) {
    row_sort_mid_kernel<<<1024, 256, 0, s>>>(a_rowptr, a_cols, a_vals, long_rows, nlong);
    DSANLS_LAUNCHED("row_sort_mid_kernel");
    row_sort_long_kernel<<<1024, 256, 0, s>>>(a_rowptr, a_cols, a_vals, long_rows, nlong, static_cast<int>(d));
    DSANLS_LAUNCHED("row_sort_long_kernel");
  }
  return DSANLS_OK;
}

dsanls_status launch_a_rhs(const int32_t* a_rowptr, int32_t* a_cols, float* a_vals, int64_t rows,
                           const int32_t* idx, const float* W, int64_t k, float scale, const int32_t* long_rows,
                           const int32_t* nlong, float* R, hipStream_t s) {
  if (rows <= 0) return DSANLS_OK;
  // the lanes hold two columns of R each: columns in chunks of 128 (the
  // first chunk also leaves the short rows of A sorted; later ones find
  // them so)
  for (int64_t c0 = 0; c0 < k; c0 += 128) {
    const int kc = static_cast<int>(std::min<int64_t>(128, k - c0));
    a_rhs_kernel<<<static_cast<unsigned>(ceil_div(rows, 256)), 256, 0, s>>>(a_rowptr, a_cols, a_vals, rows, idx,
                                                                           W + c0, kc, k, scale, R + c0, k);
    DSANLS_LAUNCHED("a_rhs_kernel");
    a_rhs_long_kernel<4><<<1024, 256, 0, s>>>(a_rowptr, a_cols, a_vals, idx, W + c0, kc, k, scale, long_rows,
                                              nlong, kShortRow + 1, kVeryLongRow, R + c0, k);
    DSANLS_LAUNCHED("a_rhs_long_kernel");
    a_rhs_long_kernel<16><<<256, 1024, 0, s>>>(a_rowptr, a_cols, a_vals, idx, W + c0, kc, k, scale,
                                               long_rows, nlong, kVeryLongRow + 1, 0x7fffffff, R + c0, k);
    DSANLS_LAUNCHED("a_rhs_long_kernel");
  }
  return DSANLS_OK;
}

dsanls_status launch_sketched_rows(const int64_t* rowptr, const int32_t* colidx, const float* vals,
                                   int64_t rows, const CsrSegments& sg, const int32_t* slot, float scale,
                                   int32_t* seg_cnt, int32_t* seg_pos, int32_t* scan_ws,
                                   int32_t* a_rowptr, int32_t* a_cols, float* a_vals, hipStream_t s) {
  if (sg.nseg <= 0) return DSANLS_OK;
  const unsigned g4 = static_cast<unsigned>(ceil_div(sg.nseg, 4));
  seg_hits_count_kernel<<<g4, 256, 0, s>>>(rowptr, colidx, sg.seg_row, sg.seg_beg, sg.nseg, slot, seg_cnt);
  DSANLS_LAUNCHED("seg_hits_count_kernel");
  dsanls_status st = launch_exclusive_scan(seg_cnt, seg_pos, sg.nseg, scan_ws, s);
  if (st != DSANLS_OK) return st;
  seg_rowptr_kernel<<<static_cast<unsigned>(ceil_div(sg.nseg, 256)), 256, 0, s>>>(
      rowptr, sg.seg_row, sg.seg_beg, sg.nseg, rows, seg_pos, a_rowptr);
  DSANLS_LAUNCHED("seg_rowptr_kernel");
  seg_hits_fill_kernel<<<g4, 256, 0, s>>>(rowptr, colidx, vals, sg.seg_row, sg.seg_beg, sg.nseg, slot, scale,
                                          seg_pos, a_cols, a_vals);
  DSANLS_LAUNCHED("seg_hits_fill_kernel");
  return DSANLS_OK;
}

dsanls_status launch_csr_hits_count(const int64_t* rowptr, const int32_t* colidx, int64_t rows,
                                    const int32_t* slot, int32_t* cnt, hipStream_t s) {
  if (rows <= 0) return DSANLS_OK;
  csr_hits_count_kernel<<<static_cast<unsigned>(ceil_div(rows, 4)), 256, 0, s>>>(rowptr, colidx, rows, slot,
                                                                                 cnt);
  DSANLS_LAUNCHED("csr_hits_count_kernel");
  return DSANLS_OK;
}

dsanls_status launch_csr_hits_fill(const int64_t* rowptr, const int32_t* colidx, const float* vals,
                                   int64_t rows, const int32_t* slot, float scale,
                                   const int32_t* a_rowptr, int32_t* a_cols, float* a_vals,
                                   hipStream_t s) {
  if (rows <= 0) return DSANLS_OK;
  csr_hits_fill_kernel<<<static_cast<unsigned>(ceil_div(rows, 4)), 256, 0, s>>>(
      rowptr, colidx, vals, rows, slot, scale, a_rowptr, a_cols, a_vals);
  DSANLS_LAUNCHED("csr_hits_fill_kernel");
  return DSANLS_OK;
}

dsanls_status launch_csr_select_len(const int32_t* rowptr, int64_t nrows, const int32_t* sel,
                                    int64_t nsel, int32_t* len, hipStream_t s) {
  if (nsel <= 0) return DSANLS_OK;
  select_len_kernel<<<static_cast<unsigned>(ceil_div(nsel, 256)), 256, 0, s>>>(rowptr, nrows, sel, nsel, len);
  DSANLS_LAUNCHED("select_len_kernel");
  return DSANLS_OK;
}

dsanls_status launch_csr_select_copy(const int32_t* rowptr, int64_t nrows, const int32_t* cols,
                                     const float* vals, const int32_t* sel, int64_t nsel,
                                     const int32_t* out_rowptr, int32_t* out_cols, float* out_vals,
                                     hipStream_t s) {
  if (nsel <= 0) return DSANLS_OK;
  select_copy_kernel<<<static_cast<unsigned>(ceil_div(nsel, 4)), 256, 0, s>>>(rowptr, nrows, cols, vals, sel,
                                                                               nsel, out_rowptr, out_cols,
                                                                               out_vals);
  DSANLS_LAUNCHED("select_copy_kernel");
  return DSANLS_OK;
}

int64_t csr_cross_partials(int64_t) { return kCrossBlocks; }

dsanls_status launch_csr_cross(const int64_t* rowptr, const int32_t* colidx, const float* vals,
                               int64_t rows, const float* U, const float* V, int64_t k,
                               float* partials, hipStream_t s) {
  csr_cross_kernel<<<kCrossBlocks, 256, 0, s>>>(rowptr, colidx, vals, rows, U, V,
                                                static_cast<int>(k), partials);
  DSANLS_LAUNCHED("csr_cross_kernel");
  return DSANLS_OK;
}

}  // namespace dsanls
