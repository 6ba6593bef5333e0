// Sparse (CSR) side of the path: the sketch right-hand side R = A B^T for a
// subsampling sketch, and the nnz term of the sparse objective.
//
// With S = sqrt(n/d) [e_{j_1} .. e_{j_d}], A = M S keeps only the sampled
// columns of M and B = V^T S the sampled rows of V, so
//     R[i, :] = (A B^T)[i, :] = (n/d) * sum_{j sampled, M_ij != 0} M_ij V[j, :]
// (Sec. 3.3: subsampling keeps the sparsity of M).  One wave streams the
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
__global__ __launch_bounds__(256) void csr_rhs_seg_kernel(const int64_t* __restrict__ rowptr,
                                                          const int32_t* __restrict__ colidx,
                                                          const float* __restrict__ vals,
                                                          const int32_t* __restrict__ seg_row,
                                                          const int64_t* __restrict__ seg_beg,
                                                          const int32_t* __restrict__ seg_part,
                                                          int64_t nseg,
                                                          const int32_t* __restrict__ slot,
                                                          const float* __restrict__ W, int k,
                                                          float scale, float* __restrict__ R,
                                                          float* __restrict__ P) {
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
  const int32_t part = seg_part[sg];
  float* out = part < 0 ? R + row * k : P + (int64_t)part * k;
  const float sc = part < 0 ? scale : 1.0f;
  if (lane < k) out[lane] = sc * a0;
  if (lane + 64 < k) out[lane + 64] = sc * a1;
}

// R[row] = scale * sum of the row's segment partials, in segment order.
__global__ __launch_bounds__(256) void csr_rhs_fixup_kernel(const int32_t* __restrict__ multi_row,
                                                            const int32_t* __restrict__ multi_part,
                                                            int64_t nmulti, int k, float scale,
                                                            const float* __restrict__ P,
                                                            float* __restrict__ R) {
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
  if (lane < k) R[row * k + lane] = scale * a0;
  if (lane + 64 < k) R[row * k + lane + 64] = scale * a1;
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
    float a0 = 0.f, a1 = 0.f, sq = 0.f, sqc = 0.f;
    for (int64_t base = beg; base < end; base += 64) {
      const int64_t e = base + lane;
      int32_t col = 0;
      float v = 0.f;
      if (e < end) {
        col = colidx[e];
        v = vals[e];
      }
      neumaier(sq, sqc, v * v);
      const int cnt = static_cast<int>(end - base < 64 ? end - base : 64);
      for (int b = 0; b < cnt; ++b) {
        const int32_t c = __shfl(col, b, 64);
        const float x = __shfl(v, b, 64);
        const float* w = V + (int64_t)c * k;
        if (lane < k) a0 += x * w[lane];
        if (lane + 64 < k) a1 += x * w[lane + 64];
      }
    }
    const float* u = U + row * k;
    float dot = 0.f;
    if (lane < k) dot += u[lane] * a0;
    if (lane + 64 < k) dot += u[lane + 64] * a1;
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
                                 float scale, float* R, float* P, hipStream_t s) {
  if (sg.nseg <= 0) return DSANLS_OK;
  if (k > 128) return fail(DSANLS_E_UNSUPPORTED, "CSR path supports k <= 128");
  csr_rhs_seg_kernel<<<static_cast<unsigned>(ceil_div(sg.nseg, 4)), 256, 0, s>>>(
      rowptr, colidx, vals, sg.seg_row, sg.seg_beg, sg.seg_part, sg.nseg, slot, W, static_cast<int>(k), scale, R,
      P);
  DSANLS_LAUNCHED("csr_rhs_seg_kernel");
  if (sg.nmulti > 0) {
    csr_rhs_fixup_kernel<<<static_cast<unsigned>(ceil_div(sg.nmulti, 4)), 256, 0, s>>>(
        sg.multi_row, sg.multi_part, sg.nmulti, static_cast<int>(k), scale, P, R);
    DSANLS_LAUNCHED("csr_rhs_fixup_kernel");
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
  if (k > 128) return fail(DSANLS_E_UNSUPPORTED, "CSR path supports k <= 128");
  csr_cross_kernel<<<kCrossBlocks, 256, 0, s>>>(rowptr, colidx, vals, rows, U, V,
                                                static_cast<int>(k), partials);
  DSANLS_LAUNCHED("csr_cross_kernel");
  return DSANLS_OK;
}

}  // namespace dsanls
