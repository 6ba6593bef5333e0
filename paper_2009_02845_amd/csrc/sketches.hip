// The further sketch kinds of Sec. 3.4 (its closing paragraph): the count
// sketch and the subsampled randomised Hadamard transform (SRHT).  Both
// satisfy Assumption 1 (E[S S^T] = I) and, like the Gaussian and
// subsampling sketches, are pure functions of (seed, t, side, global row
// index) through Philox4x32-10, so every node draws the same S^t.
//
// Count sketch: row j of S (n x d) has one nonzero, s_j in {+1, -1}, in
// column h_j (bucket), both from the counter (0, j, side | 2 << 8, t):
// h_j = hi32(x0 * d), s_j = top bit of x1.  Then
//     (A^T)[c, :] = sum_{j : h_j = c} s_j X^T[j, :],
// so with X^T resident each bucket streams its rows of X^T once: forming
// A = X S reads X exactly once (HBM-bound, no matrix cores needed).  The
// rows of a bucket are summed in ascending j (bucket lists built by a
// counting sort, then ordered within each bucket), so results do not depend
// on scheduling.  On CSR input R = A B^T is folded straight from the nnz
// stream: R[i, :] = sum_e M_ij s_j B^T[h_j, :].
//
// SRHT: with N = 2^ceil(log2 n) (at least 1024), signs s_j from counter
// (0, j, side | 3 << 8, t) and d sampled Hadamard columns p_c (the d
// smallest keys of counter (0, b, side | 4 << 8, t) over b < N, ascending),
// S[j, c] = s_j H[j, p_c] / sqrt(d), H the Sylvester Hadamard matrix.  Row i
// of A = X S is the Walsh-Hadamard transform of the signed, zero-padded row
// x_i, read at p and scaled: one workgroup transforms one row in LDS.
#include "common.hpp"

namespace dsanls {

namespace {

constexpr uint32_t kPhM0 = 0xD2511F53u, kPhM1 = 0xCD9E8D57u;
constexpr uint32_t kPhW0 = 0x9E3779B9u, kPhW1 = 0xBB67AE85u;

struct W4 { uint32_t x0, x1, x2, x3; };

// Philox4x32-10 block function (Salmon et al., SC'11).
__device__ __forceinline__ W4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                     uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kPhW0;
      k1 += kPhW1;
    }
    const uint32_t hi0 = __umulhi(kPhM0, c0), lo0 = kPhM0 * c0;
    const uint32_t hi1 = __umulhi(kPhM1, c2), lo1 = kPhM1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return {c0, c1, c2, c3};
}

// ----------------------------------------------------------------- count sketch

__global__ __launch_bounds__(256) void cs_zero_kernel(int32_t* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += gridDim.x * 256ll) p[i] = 0;
}

// Bucket and sign of rows j0 .. j0 + n - 1, and the bucket counts.
__global__ __launch_bounds__(256) void cs_hash_kernel(uint32_t k0, uint32_t k1, uint32_t t, uint32_t side_word,
                                                      int64_t j0, int64_t n, uint32_t d,
                                                      int32_t* __restrict__ bucket, float* __restrict__ sign,
                                                      int32_t* __restrict__ cnt) {
  const int64_t j = blockIdx.x * 256ll + threadIdx.x;
  if (j >= n) return;
  const W4 w = philox(0u, static_cast<uint32_t>(j0 + j), side_word, t, k0, k1);
  const int32_t b = static_cast<int32_t>(__umulhi(w.x0, d));
  bucket[j] = b;
  sign[j] = (w.x1 >> 31) ? -1.0f : 1.0f;
  atomicAdd(&cnt[b], 1);
}

// Scatter j into its bucket's segment (any order; ordered below).
__global__ __launch_bounds__(256) void cs_fill_kernel(const int32_t* __restrict__ bucket, int64_t n,
                                                      const int32_t* __restrict__ off, int32_t* __restrict__ cursor,
                                                      int32_t* __restrict__ tmp) {
  const int64_t j = blockIdx.x * 256ll + threadIdx.x;
  if (j >= n) return;
  const int32_t b = bucket[j];
  tmp[off[b] + atomicAdd(&cursor[b], 1)] = static_cast<int32_t>(j);
}

// One workgroup per bucket: its (distinct) rows in ascending order, each
// written at its rank.  A bucket longer than kCsBucketCap (far beyond its
// expected length, which the configuration bounds by 1024) keeps its rows
// unordered, still valid indices, and sets bit 4 of err.
constexpr int kCsBucketCap = 4096;
__global__ __launch_bounds__(256) void cs_order_kernel(const int32_t* __restrict__ off, const int32_t* __restrict__ tmp,
                                                       int32_t* __restrict__ list, int* __restrict__ err) {
  __shared__ int32_t e[kCsBucketCap];
  const int c = blockIdx.x;
  const int32_t b0 = off[c], len = off[c + 1] - b0;
  if (len > kCsBucketCap) {
    for (int i = threadIdx.x; i < len; i += 256) list[b0 + i] = tmp[b0 + i];
    if (threadIdx.x == 0) atomicOr(err, 4);
    return;
  }
  for (int i = threadIdx.x; i < len; i += 256) e[i] = tmp[b0 + i];
  __syncthreads();
  for (int i = threadIdx.x; i < len; i += 256) {
    const int32_t v = e[i];
    int rank = 0;
    for (int q = 0; q < len; ++q) rank += e[q] < v;
    list[b0 + rank] = v;
  }
}

// Out[c, col] = sum over the rows j of bucket c (ascending) of
// sign[j] * X^T[j, col]: grid (column chunks of 1024, buckets, strided by
// gridDim.y), four columns per thread.  VEC: X^T rows and Out rows 16-byte
// aligned (float4 loads).
template <bool VEC>
__global__ __launch_bounds__(256) void cs_rows_kernel(const float* __restrict__ Xt, int64_t ldx, int64_t cols,
                                                      int64_t nb, const int32_t* __restrict__ off,
                                                      const int32_t* __restrict__ list,
                                                      const float* __restrict__ sign, float* __restrict__ Out,
                                                      int64_t ldo) {
  const int64_t col = (blockIdx.x * 256ll + threadIdx.x) * 4;
  if (col >= cols) return;
  for (int64_t c = blockIdx.y; c < nb; c += gridDim.y) {
    const int32_t e0 = off[c], e1 = off[c + 1];
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    if (VEC && col + 4 <= cols) {
      for (int32_t e = e0; e < e1; ++e) {
        const int32_t j = list[e];
        const float s = sign[j];
        const float4 x = *reinterpret_cast<const float4*>(Xt + j * ldx + col);
        a0 += s * x.x;
        a1 += s * x.y;
        a2 += s * x.z;
        a3 += s * x.w;
      }
      *reinterpret_cast<float4*>(Out + c * ldo + col) = make_float4(a0, a1, a2, a3);
      continue;
    }
    const int nc = cols - col < 4 ? static_cast<int>(cols - col) : 4;
    for (int32_t e = e0; e < e1; ++e) {
      const int32_t j = list[e];
      const float s = sign[j];
      const float* x = Xt + j * ldx + col;
      a0 += s * x[0];
      if (nc > 1) a1 += s * x[1];
      if (nc > 2) a2 += s * x[2];
      if (nc > 3) a3 += s * x[3];
    }
    float* o = Out + c * ldo + col;
    o[0] = a0;
    if (nc > 1) o[1] = a1;
    if (nc > 2) o[2] = a2;
    if (nc > 3) o[3] = a3;
  }
}

// ----------------------------------------------------------------- SRHT

__global__ __launch_bounds__(256) void srht_sign_kernel(uint32_t k0, uint32_t k1, uint32_t t, uint32_t side_word,
                                                        int64_t j0, int64_t n, float* __restrict__ sign) {
  const int64_t j = blockIdx.x * 256ll + threadIdx.x;
  if (j >= n) return;
  const W4 w = philox(0u, static_cast<uint32_t>(j0 + j), side_word, t, k0, k1);
  sign[j] = (w.x0 >> 31) ? -1.0f : 1.0f;
}

// LDS position of element i of the transform: the XOR of bits 5..9 into
// bits 0..4 spreads each access pattern of the three passes over distinct
// banks (32 consecutive lanes never collide).
__device__ __forceinline__ int hswz(int i) { return i ^ ((i >> 5) & 31); }

// In-register butterflies over the R values of one thread (a Walsh-Hadamard
// transform of length R): v[r] and v[r + h] -> (sum, difference).
template <int R>
__device__ __forceinline__ void fwht_regs(float (&v)[R]) {
#pragma unroll
  for (int h = 1; h < R; h <<= 1)
#pragma unroll
    for (int r = 0; r < R; ++r)
      if ((r & h) == 0) {
        const float a = v[r], b = v[r + h];
        v[r] = a + b;
        v[r + h] = a - b;
      }
}

// One workgroup of 1024 threads per row of X: the signed row, placed at its
// global offset j0 in a zero vector of N = 1024 E, is transformed in place
// (bits 10.. of the index in registers straight from HBM, bits 5..9 and
// then bits 0..4 in registers between LDS passes), and the d sampled
// entries p_c are written, scaled, to Out[row, c].
template <int LOGE>
__global__ __launch_bounds__(1024) void srht_rows_kernel(const float* __restrict__ X, int64_t ldx, int64_t lng,
                                                         int64_t j0, const float* __restrict__ sign,
                                                         const int32_t* __restrict__ p, int d, float scale,
                                                         float* __restrict__ Out, int64_t ldo) {
  constexpr int E = 1 << LOGE, N = 1024 * E;
  __shared__ float sx[N];
  const int tid = threadIdx.x;
  const int64_t row = blockIdx.x;
  const float* x = X + row * ldx;
  {
    float v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int64_t jl = static_cast<int64_t>(tid + 1024 * r) - j0;
      v[r] = jl >= 0 && jl < lng ? x[jl] * sign[jl] : 0.f;
    }
    fwht_regs<E>(v);
#pragma unroll
    for (int r = 0; r < E; ++r) sx[hswz(tid + 1024 * r)] = v[r];
  }
  __syncthreads();
  if (tid < 32 * E) {
    const int base = 1024 * (tid >> 5) + (tid & 31);
    float v[32];
#pragma unroll
    for (int r = 0; r < 32; ++r) v[r] = sx[hswz(base + 32 * r)];
    fwht_regs<32>(v);
#pragma unroll
    for (int r = 0; r < 32; ++r) sx[hswz(base + 32 * r)] = v[r];
  }
  __syncthreads();
  if (tid < 32 * E) {
    float v[32];
#pragma unroll
    for (int r = 0; r < 32; ++r) v[r] = sx[hswz(32 * tid + r)];
    fwht_regs<32>(v);
#pragma unroll
    for (int r = 0; r < 32; ++r) sx[hswz(32 * tid + r)] = v[r];
  }
  __syncthreads();
  for (int c = tid; c < d; c += 1024) Out[row * ldo + c] = scale * sx[hswz(p[c])];
}

}  // namespace

int64_t srht_length(int64_t n) {
  int64_t N = 1024;
  while (N < n) N <<= 1;
  return N;
}

dsanls_status launch_count_sketch_hash(uint64_t seed, uint32_t t, int side, int64_t j0, int64_t n, int64_t d,
                                       const CountSketch& cs, hipStream_t s) {
  if (d < 1 || d > INT32_MAX || n < 1) return fail(DSANLS_E_SHAPE, "count sketch: bad sizes");
  const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
  const uint32_t side_word = (static_cast<uint32_t>(side) & 0xFFu) | (2u << 8);
  const unsigned gn = static_cast<unsigned>(ceil_div(n, 256));
  // counts and cursors (a fill kernel: the update may run under graph capture)
  cs_zero_kernel<<<static_cast<unsigned>(std::min<int64_t>(ceil_div(2 * (d + 1), 256), 1024)), 256, 0, s>>>(
      cs.cnt, 2 * (d + 1));
  DSANLS_LAUNCHED("cs_zero_kernel");
  cs_hash_kernel<<<gn, 256, 0, s>>>(k0, k1, t, side_word, j0, n, static_cast<uint32_t>(d), cs.bucket, cs.sign,
                                    cs.cnt);
  DSANLS_LAUNCHED("cs_hash_kernel");
  dsanls_status st = launch_exclusive_scan(cs.cnt, cs.off, d, cs.scan_ws, s);
  if (st != DSANLS_OK) return st;
  cs_fill_kernel<<<gn, 256, 0, s>>>(cs.bucket, n, cs.off, cs.cnt + (d + 1), cs.tmp);
  DSANLS_LAUNCHED("cs_fill_kernel");
  cs_order_kernel<<<static_cast<unsigned>(d), 256, 0, s>>>(cs.off, cs.tmp, cs.list, cs.err);
  DSANLS_LAUNCHED("cs_order_kernel");
  return DSANLS_OK;
}

dsanls_status launch_count_sketch_rows(const float* Xt, int64_t ldx, int64_t cols, int64_t d, const CountSketch& cs,
                                       float* Out, int64_t ldo, hipStream_t s) {
  if (cols <= 0) return DSANLS_OK;
  dim3 grid(static_cast<unsigned>(ceil_div(cols, 1024)), static_cast<unsigned>(std::min<int64_t>(d, 65535)));
  const bool vec = ldx % 4 == 0 && ldo % 4 == 0 && (reinterpret_cast<uintptr_t>(Xt) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(Out) & 15) == 0;
  if (vec)
    cs_rows_kernel<true><<<grid, 256, 0, s>>>(Xt, ldx, cols, d, cs.off, cs.list, cs.sign, Out, ldo);
  else
    cs_rows_kernel<false><<<grid, 256, 0, s>>>(Xt, ldx, cols, d, cs.off, cs.list, cs.sign, Out, ldo);
  DSANLS_LAUNCHED("cs_rows_kernel");
  return DSANLS_OK;
}

dsanls_status launch_srht_signs(uint64_t seed, uint32_t t, int side, int64_t j0, int64_t n, float* sign,
                                hipStream_t s) {
  const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
  const uint32_t side_word = (static_cast<uint32_t>(side) & 0xFFu) | (3u << 8);
  srht_sign_kernel<<<static_cast<unsigned>(ceil_div(n, 256)), 256, 0, s>>>(k0, k1, t, side_word, j0, n, sign);
  DSANLS_LAUNCHED("srht_sign_kernel");
  return DSANLS_OK;
}

dsanls_status launch_srht_rows(const float* X, int64_t ldx, int64_t rows, int64_t lng, int64_t j0, int64_t N,
                               const float* sign, const int32_t* p, int64_t d, float* Out, int64_t ldo,
                               hipStream_t s) {
  if (rows <= 0) return DSANLS_OK;
  if (j0 + lng > N) return fail(DSANLS_E_SHAPE, "srht: block outside the transform length");
  const float scale = static_cast<float>(1.0 / std::sqrt(static_cast<double>(d)));
  const unsigned g = static_cast<unsigned>(rows);
  switch (N) {
#define DSANLS_SRHT(LOGE)                                                                                      \
  case 1024 << LOGE:                                                                                           \
    srht_rows_kernel<LOGE><<<g, 1024, 0, s>>>(X, ldx, lng, j0, sign, p, static_cast<int>(d), scale, Out, ldo); \
    DSANLS_LAUNCHED("srht_rows_kernel");                                                                       \
    return DSANLS_OK;
    DSANLS_SRHT(0)
    DSANLS_SRHT(1)
    DSANLS_SRHT(2)
    DSANLS_SRHT(3)
    DSANLS_SRHT(4)
    DSANLS_SRHT(5)
#undef DSANLS_SRHT
  }
  return fail(DSANLS_E_UNSUPPORTED, "SRHT supports a long dimension of at most 32768 (transform in LDS)");
}

}  // namespace dsanls
