// Small and memory-bound helpers of the path: transposes, the k x k Gram
// G = B B^T with compensated sums, gathers for the subsampling sketch, and
// compensated reductions.
#include "common.hpp"

#include <hip/hip_bf16.h>

namespace dsanls {

namespace {

__device__ __forceinline__ void neumaier(float& s, float& c, float x) {
  const float t = s + x;
  c += fabsf(s) >= fabsf(x) ? (s - t) + x : (x - t) + s;
  s = t;
}

// 64 x 64 tiles through LDS (padded against bank conflicts); reads and
// writes are both coalesced along the fast index.
template <typename TOut, typename Cvt>
__global__ __launch_bounds__(256) void transpose_kernel(const float* __restrict__ X, int64_t ldx,
                                                        TOut* __restrict__ Y, int64_t ldy,
                                                        int64_t rows, int64_t cols, Cvt cvt) {
  __shared__ float tile[64][65];
  const int64_t r0 = blockIdx.y * 64ll, c0 = blockIdx.x * 64ll;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int64_t r = r0 + i, c = c0 + tx;
    tile[i][tx] = (r < rows && c < cols) ? X[r * ldx + c] : 0.f;
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < cols && r < rows) Y[c * ldy + r] = cvt(tile[tx][i]);
  }
}

struct Id {
  __device__ float operator()(float x) const { return x; }
};
struct ToBf16 {
  __device__ __hip_bfloat16 operator()(float x) const { return __float2bfloat16(x); }
};

// Y = bf16(X) on rows x cols, zeros in columns cols .. ldy - 1
__global__ __launch_bounds__(256) void to_bf16_kernel(const float* __restrict__ X, int64_t ldx,
                                                      __hip_bfloat16* __restrict__ Y, int64_t ldy,
                                                      int64_t rows, int64_t cols) {
  const int64_t total = rows * ldy;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / ldy, c = i % ldy;
    Y[i] = c < cols ? __float2bfloat16(X[r * ldx + c]) : __float2bfloat16(0.0f);
  }
}

// G[a][b] = sum_c B[a][c] B[b][c] for a <= b, mirrored.  One wave per
// (a, b) pair: lanes stride over c, each with a compensated partial, then a
// fixed-order compensated tree across the wave.
__global__ __launch_bounds__(256) void gram_kernel(const float* __restrict__ B, int64_t ld,
                                                   int64_t k, int64_t d, float* __restrict__ G) {
  const int64_t pair = blockIdx.x * 4ll + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t npairs = k * (k + 1) / 2;
  if (pair >= npairs) return;
  // pair -> (a, b) with a <= b, row-major over the upper triangle
  int64_t a = 0, rem = pair;
  while (rem >= k - a) {
    rem -= k - a;
    ++a;
  }
  const int64_t b = a + rem;
  const float* pa = B + a * ld;
  const float* pb = B + b * ld;
  float s = 0.f, c = 0.f;
  for (int64_t i = lane; i < d; i += 64) neumaier(s, c, pa[i] * pb[i]);
  for (int off = 32; off > 0; off >>= 1) {
    const float os = __shfl_down(s, off, 64), oc = __shfl_down(c, off, 64);
    neumaier(s, c, os);
    c += oc;
  }
  if (lane == 0) {
    const float v = s + c;
    G[a * k + b] = v;
    G[b * k + a] = v;
  }
}

constexpr int kRedBlock = 256;
constexpr int64_t kRedChunk = 1 << 16;   // elements per partial

__global__ __launch_bounds__(kRedBlock) void sumsq_kernel(const float* __restrict__ X, int64_t ld,
                                                          int64_t rows, int64_t cols,
                                                          float* __restrict__ partials) {
  __shared__ float red[2 * kRedBlock / 64];
  const int64_t total = rows * cols;
  const int64_t beg = blockIdx.x * kRedChunk;
  const int64_t end = beg + kRedChunk < total ? beg + kRedChunk : total;
  float s = 0.f, c = 0.f;
  for (int64_t i = beg + threadIdx.x; i < end; i += kRedBlock) {
    const float x = X[(i / cols) * ld + (i % cols)];
    neumaier(s, c, x * x);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    const float os = __shfl_down(s, off, 64), oc = __shfl_down(c, off, 64);
    neumaier(s, c, os);
    c += oc;
  }
  if (lane == 0) {
    red[2 * wave] = s;
    red[2 * wave + 1] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float ts = red[0], tc = red[1];
    for (int w = 1; w < kRedBlock / 64; ++w) {
      neumaier(ts, tc, red[2 * w]);
      tc += red[2 * w + 1];
    }
    partials[2 * blockIdx.x] = ts;
    partials[2 * blockIdx.x + 1] = tc;
  }
}

// One block: combine (sum, comp) partials in a fixed order into a
// double-float (hi, lo) pair; flag NaN/Inf.
__global__ __launch_bounds__(256) void combine_kernel(const float* __restrict__ partials,
                                                      int64_t npart, int64_t stride,
                                                      float* __restrict__ out, int* err_flag) {
  __shared__ float red[2 * 256];
  float s = 0.f, c = 0.f;
  for (int64_t i = threadIdx.x; i < npart; i += 256) {
    neumaier(s, c, partials[stride * i]);
    c += partials[stride * i + 1];
  }
  red[2 * threadIdx.x] = s;
  red[2 * threadIdx.x + 1] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    float ts = 0.f, tc = 0.f;
    for (int w = 0; w < 256; ++w) {
      neumaier(ts, tc, red[2 * w]);
      tc += red[2 * w + 1];
    }
    // renormalise (ts, tc) into hi + lo
    const float hi = ts + tc;
    const float lo = tc - (hi - ts);
    out[0] = hi;
    out[1] = lo;
    if (!isfinite(hi)) atomicOr(err_flag, 1);
  }
}

__global__ __launch_bounds__(256) void gather_cols_kernel(const float* __restrict__ X, int64_t ldx,
                                                          const int32_t* __restrict__ idx,
                                                          int64_t rows, int64_t d, float scale,
                                                          float* __restrict__ A, int64_t lda) {
  const int64_t total = rows * d;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const int64_t r = i / d, c = i % d;
    const int32_t j = idx[c];
    A[r * lda + c] = j >= 0 ? scale * X[r * ldx + j] : 0.f;
  }
}

__global__ __launch_bounds__(256) void gather_rows_t_kernel(const float* __restrict__ W, int64_t k,
                                                            const int32_t* __restrict__ idx,
                                                            int64_t d, float scale,
                                                            float* __restrict__ B, int64_t ldb) {
  const int64_t c = blockIdx.x * 256ll + threadIdx.x;
  const int64_t l = blockIdx.y;
  if (c >= d) return;
  const int32_t j = idx[c];
  B[l * ldb + c] = j >= 0 ? scale * W[(int64_t)j * k + l] : 0.f;
}

__global__ __launch_bounds__(256) void finite_kernel(const float* __restrict__ X, int64_t count,
                                                     int* err_flag) {
  bool bad = false;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
    bad |= !isfinite(X[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(err_flag, 1);
}

__global__ __launch_bounds__(256) void frob_dot_kernel(const float* __restrict__ X,
                                                       const float* __restrict__ Y, int64_t count,
                                                       float* __restrict__ out) {
  __shared__ float red[2 * 256];
  float s = 0.f, c = 0.f;
  for (int64_t i = threadIdx.x; i < count; i += 256) neumaier(s, c, X[i] * Y[i]);
  red[2 * threadIdx.x] = s;
  red[2 * threadIdx.x + 1] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    float ts = 0.f, tc = 0.f;
    for (int w = 0; w < 256; ++w) {
      neumaier(ts, tc, red[2 * w]);
      tc += red[2 * w + 1];
    }
    const float hi = ts + tc;
    out[0] = hi;
    out[1] = tc - (hi - ts);
  }
}

constexpr int kScanTile = 2048;   // 256 threads x 8 items

// Inclusive sum of a block's 256 thread values (wave scans + LDS).
__device__ __forceinline__ int32_t block_scan_incl(int32_t x, int32_t* wsum) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  int32_t before = 0;
  for (int w = 0; w < wave; ++w) before += wsum[w];
  __syncthreads();
  return x + before;
}

__global__ __launch_bounds__(256) void scan_sums_kernel(const int32_t* __restrict__ in, int64_t n,
                                                        int32_t* __restrict__ sums) {
  __shared__ int32_t wsum[4];
  const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * 8;
  int32_t t = 0;
  for (int e = 0; e < 8; ++e)
    if (base + e < n) t += in[base + e];
  t = block_scan_incl(t, wsum);
  if (threadIdx.x == 255) sums[blockIdx.x] = t;
}

// exclusive scan of the tile sums in place (one block, any length)
__global__ __launch_bounds__(256) void scan_tiles_kernel(int32_t* sums, int64_t ntiles) {
  __shared__ int32_t wsum[4];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < ntiles; b0 += 256) {
    const int64_t i = b0 + threadIdx.x;
    const int32_t v = i < ntiles ? sums[i] : 0;
    const int32_t incl = block_scan_incl(v, wsum);
    if (i < ntiles) sums[i] = carry + incl - v;
    __syncthreads();
    if (threadIdx.x == 255) carry += incl;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void scan_apply_kernel(const int32_t* __restrict__ in, int64_t n,
                                                         const int32_t* __restrict__ sums,
                                                         int32_t* __restrict__ out) {
  __shared__ int32_t wsum[4];
  const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * 8;
  int32_t v[8];
  int32_t t = 0;
  for (int e = 0; e < 8; ++e) {
    v[e] = base + e < n ? in[base + e] : 0;
    t += v[e];
  }
  const int32_t incl = block_scan_incl(t, wsum);
  int32_t run = sums[blockIdx.x] + incl - t;
  for (int e = 0; e < 8; ++e) {
    if (base + e < n) out[base + e] = run;
    run += v[e];
  }
  const int64_t last = (static_cast<int64_t>(gridDim.x) - 1) * kScanTile + 255 * 8;
  if (base == last) out[n] = run;   // total, written by the last thread of the grid
}

unsigned grid_for(int64_t total, int64_t per_block, int64_t cap) {
  int64_t g = ceil_div(total, per_block);
  if (g > cap) g = cap;
  return static_cast<unsigned>(g < 1 ? 1 : g);
}

}  // namespace

dsanls_status launch_transpose(const float* X, int64_t ldx, float* Y, int64_t ldy, int64_t rows,
                               int64_t cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return DSANLS_OK;
  if (ceil_div(rows, 64) > 65535) return fail(DSANLS_E_SHAPE, "transpose: too many rows");
  dim3 grid(static_cast<unsigned>(ceil_div(cols, 64)), static_cast<unsigned>(ceil_div(rows, 64)));
  transpose_kernel<float, Id><<<grid, 256, 0, s>>>(X, ldx, Y, ldy, rows, cols, Id{});
  DSANLS_LAUNCHED("transpose_kernel");
  return DSANLS_OK;
}

dsanls_status launch_to_bf16(const float* X, int64_t ldx, __hip_bfloat16* Y, int64_t ldy,
                             int64_t rows, int64_t cols, hipStream_t s) {
  if (rows <= 0 || ldy <= 0) return DSANLS_OK;
  if (cols > ldy) return fail(DSANLS_E_SHAPE, "to_bf16: cols exceed the leading dimension");
  to_bf16_kernel<<<grid_for(rows * ldy, 256 * 8, 1 << 20), 256, 0, s>>>(X, ldx, Y, ldy, rows, cols);
  DSANLS_LAUNCHED("to_bf16_kernel");
  return DSANLS_OK;
}

dsanls_status launch_gram(const float* B, int64_t ld, int64_t k, int64_t d, float* G,
                          hipStream_t s) {
  const int64_t npairs = k * (k + 1) / 2;
  gram_kernel<<<static_cast<unsigned>(ceil_div(npairs, 4)), 256, 0, s>>>(B, ld, k, d, G);
  DSANLS_LAUNCHED("gram_kernel");
  return DSANLS_OK;
}

int64_t sumsq_partials(int64_t rows, int64_t cols) {
  return std::max<int64_t>(1, ceil_div(rows * cols, kRedChunk));
}

dsanls_status launch_sumsq(const float* X, int64_t ld, int64_t rows, int64_t cols, float* partials,
                           hipStream_t s) {
  const int64_t np = sumsq_partials(rows, cols);
  sumsq_kernel<<<static_cast<unsigned>(np), kRedBlock, 0, s>>>(X, ld, rows, cols, partials);
  DSANLS_LAUNCHED("sumsq_kernel");
  return DSANLS_OK;
}

dsanls_status launch_combine_partials(const float* partials, int64_t npart, int64_t stride,
                                      float* out, int* err_flag, hipStream_t s) {
  combine_kernel<<<1, 256, 0, s>>>(partials, npart, stride, out, err_flag);
  DSANLS_LAUNCHED("combine_kernel");
  return DSANLS_OK;
}

dsanls_status launch_gather_cols(const float* X, int64_t ldx, const int32_t* idx, int64_t rows,
                                 int64_t d, float scale, float* A, int64_t lda, hipStream_t s) {
  if (rows <= 0 || d <= 0) return DSANLS_OK;
  gather_cols_kernel<<<grid_for(rows * d, 256 * 4, 1 << 20), 256, 0, s>>>(X, ldx, idx, rows, d,
                                                                          scale, A, lda);
  DSANLS_LAUNCHED("gather_cols_kernel");
  return DSANLS_OK;
}

dsanls_status launch_gather_rows_t(const float* W, int64_t k, const int32_t* idx, int64_t d,
                                   float scale, float* B, int64_t ldb, hipStream_t s) {
  if (k <= 0 || d <= 0) return DSANLS_OK;
  dim3 grid(static_cast<unsigned>(ceil_div(d, 256)), static_cast<unsigned>(k));
  gather_rows_t_kernel<<<grid, 256, 0, s>>>(W, k, idx, d, scale, B, ldb);
  DSANLS_LAUNCHED("gather_rows_t_kernel");
  return DSANLS_OK;
}

dsanls_status launch_frob_dot(const float* X, const float* Y, int64_t count, float* out,
                              hipStream_t s) {
  frob_dot_kernel<<<1, 256, 0, s>>>(X, Y, count, out);
  DSANLS_LAUNCHED("frob_dot_kernel");
  return DSANLS_OK;
}

size_t scan_ws_bytes(int64_t n) { return sizeof(int32_t) * (ceil_div(n, kScanTile) + 1); }

dsanls_status launch_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* ws,
                                    hipStream_t s) {
  if (n <= 0) {
    DSANLS_HIP(hipMemsetAsync(out, 0, sizeof(int32_t), s));
    return DSANLS_OK;
  }
  const int64_t nt = ceil_div(n, kScanTile);
  scan_sums_kernel<<<static_cast<unsigned>(nt), 256, 0, s>>>(in, n, ws);
  DSANLS_LAUNCHED("scan_sums_kernel");
  scan_tiles_kernel<<<1, 256, 0, s>>>(ws, nt);
  DSANLS_LAUNCHED("scan_tiles_kernel");
  scan_apply_kernel<<<static_cast<unsigned>(nt), 256, 0, s>>>(in, n, ws, out);
  DSANLS_LAUNCHED("scan_apply_kernel");
  return DSANLS_OK;
}

dsanls_status launch_check_finite(const float* X, int64_t count, int* err_flag, hipStream_t s) {
  if (count <= 0) return DSANLS_OK;
  finite_kernel<<<grid_for(count, 256 * 16, 4096), 256, 0, s>>>(X, count, err_flag);
  DSANLS_LAUNCHED("finite_kernel");
  return DSANLS_OK;
}

}  // namespace dsanls
