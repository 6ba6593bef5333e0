// Random sketch matrices (Sec. 3.4) from a counter-based generator.
//
// All nodes must draw the same S^t from one shared seed; a counter-based
// generator makes S^t a pure function of (seed, t, side, row, column), so
// any GPU (or the CPU) can produce any block of it without communication.
// Generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
// Counter = (q, j, side | kind << 8, t), key = (seed lo, seed hi).
#include "common.hpp"

#include <hip/hip_bf16.h>

namespace dsanls {

namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;
constexpr uint32_t kKindGaussian = 0;
constexpr uint32_t kKindSubsample = 1;

struct Words { uint32_t x0, x1, x2, x3; };

__device__ __forceinline__ Words philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint32_t hi0 = __umulhi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
    const uint32_t hi1 = __umulhi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return {c0, c1, c2, c3};
}

// (x >> 9) + 1/2, scaled by 2^-23: exact in binary32, strictly inside (0, 1).
__device__ __forceinline__ float open01(uint32_t x) {
  return (static_cast<float>(x >> 9) + 0.5f) * 0x1p-23f;
}

__global__ void philox_kernel(const uint32_t* __restrict__ ctr, const uint32_t* __restrict__ key,
                              uint32_t* __restrict__ out, int64_t count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  const Words w = philox10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3],
                           key[2 * i], key[2 * i + 1]);
  out[4 * i] = w.x0;
  out[4 * i + 1] = w.x1;
  out[4 * i + 2] = w.x2;
  out[4 * i + 3] = w.x3;
}

// One thread per (row j of S, group q of four columns).  Box-Muller maps
// (x0, x1) to columns 4q, 4q+1 and (x2, x3) to 4q+2, 4q+3.  S is stored
// transposed (St[c * ld + j]) so that it is the K-contiguous operand of the
// sketch GEMM; consecutive threads write consecutive j (coalesced).
// Row j of the block is row j0 + j of the whole sketch (a node's share of the
// long dimension draws the same values as the one-node sketch).
__global__ void gaussian_t_kernel(uint32_t k0, uint32_t k1, uint32_t t, uint32_t side_word,
                                  int64_t j0, int64_t n, int64_t d, float scale, float* __restrict__ St,
                                  int64_t ld, __hip_bfloat16* __restrict__ Sb, int64_t ldb) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const uint32_t q = blockIdx.y;
  if (j >= n) return;
  const Words w = philox10(q, static_cast<uint32_t>(j0 + j), side_word, t, k0, k1);
  float z[4];
  {
    const float rad = sqrtf(-2.0f * logf(open01(w.x0)));
    float sn, cs;
    sincospif(2.0f * open01(w.x1), &sn, &cs);
    z[0] = rad * cs;
    z[1] = rad * sn;
  }
  {
    const float rad = sqrtf(-2.0f * logf(open01(w.x2)));
    float sn, cs;
    sincospif(2.0f * open01(w.x3), &sn, &cs);
    z[2] = rad * cs;
    z[3] = rad * sn;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t c = 4 * (int64_t)q + e;
    if (c < d) {
      float v = z[e] * scale;
      if (Sb != nullptr) {
        const __hip_bfloat16 b = __float2bfloat16(v);  // round to nearest even
        Sb[c * ldb + j] = b;
        v = __bfloat162float(b);
      }
      St[c * ld + j] = v;
    }
  }
}

// ---------------------------------------------------------------- subsampling
//
// The sampled set is the d indices with the smallest (key, index) pairs,
// where key is the 64-bit word x0:x1 of counter (0, j, side | 1 << 8, t).
// It is found by a radix select on the top 16 key bits followed by an exact
// sort of the one boundary bucket; the output is the indicator of the set,
// compacted in ascending index order by a prefix sum.

constexpr int kHistBins = 1 << 16;
constexpr int kCandCap = 4096;   // boundary-bucket capacity (sorted in LDS)
constexpr int kScanItems = 8;    // indices per thread in the count/write passes
constexpr int kScanBlock = 256;

struct SelectState {
  uint32_t bin;        // top-16-bit bucket holding the d-th smallest key
  uint32_t need;       // how many of that bucket are taken
  uint32_t cand_count; // candidates collected from the bucket
  uint32_t pad;
  uint64_t tkey;       // (tkey, tidx) = the d-th smallest (key, index)
  int64_t tidx;
};

__global__ void sub_keys_kernel(uint32_t k0, uint32_t k1, uint32_t t, uint32_t side_word,
                                int64_t n, uint64_t* __restrict__ keys,
                                uint32_t* __restrict__ hist) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const Words w = philox10(0u, static_cast<uint32_t>(j), side_word, t, k0, k1);
  const uint64_t key = (static_cast<uint64_t>(w.x0) << 32) | w.x1;
  keys[j] = key;
  atomicAdd(&hist[key >> 48], 1u);
}

// One block of 1024 threads: find the bucket where the running count of
// keys crosses d.
__global__ __launch_bounds__(1024) void sub_select_kernel(const uint32_t* __restrict__ hist,
                                                          int64_t d, SelectState* st) {
  constexpr int kPer = kHistBins / 1024;
  __shared__ uint32_t part[1024];
  const int tid = threadIdx.x;
  uint32_t s = 0;
  for (int i = 0; i < kPer; ++i) s += hist[tid * kPer + i];
  part[tid] = s;
  __syncthreads();
  // inclusive Hillis-Steele scan of the 1024 partial sums
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t v = tid >= off ? part[tid - off] : 0u;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  const uint32_t before = tid > 0 ? part[tid - 1] : 0u;
  if (before < static_cast<uint64_t>(d) && static_cast<uint64_t>(d) <= part[tid]) {
    uint32_t cum = before;
    for (int i = 0; i < kPer; ++i) {
      const uint32_t h = hist[tid * kPer + i];
      if (static_cast<uint64_t>(d) <= cum + h) {
        st->bin = tid * kPer + i;
        st->need = static_cast<uint32_t>(d - cum);
        break;
      }
      cum += h;
    }
  }
}

__global__ void sub_collect_kernel(const uint64_t* __restrict__ keys, int64_t n,
                                   SelectState* st, uint64_t* __restrict__ cand_key,
                                   int64_t* __restrict__ cand_idx) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const uint64_t key = keys[j];
  if ((key >> 48) == st->bin) {
    const uint32_t pos = atomicAdd(&st->cand_count, 1u);
    if (pos < kCandCap) {
      cand_key[pos] = key;
      cand_idx[pos] = j;
    }
  }
}

__device__ __forceinline__ bool pair_less(uint64_t ka, int64_t ia, uint64_t kb, int64_t ib) {
  return ka < kb || (ka == kb && ia < ib);
}

// One block: bitonic sort of the boundary bucket by (key, index); the
// need-th smallest is the selection threshold.
__global__ __launch_bounds__(1024) void sub_resolve_kernel(const uint64_t* __restrict__ cand_key,
                                                           const int64_t* __restrict__ cand_idx,
                                                           SelectState* st, int* err_flag) {
  __shared__ uint64_t sk[kCandCap];
  __shared__ int64_t si[kCandCap];
  const uint32_t total = st->cand_count;
  if (total > kCandCap) {
    if (threadIdx.x == 0) atomicOr(err_flag, 2);
    return;
  }
  int p2 = 1;
  while (p2 < static_cast<int>(total)) p2 <<= 1;
  for (int i = threadIdx.x; i < p2; i += blockDim.x) {
    if (i < static_cast<int>(total)) {
      sk[i] = cand_key[i];
      si[i] = cand_idx[i];
    } else {
      sk[i] = ~0ull;
      si[i] = INT64_MAX;
    }
  }
  __syncthreads();
  for (int size = 2; size <= p2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < p2; i += blockDim.x) {
        const int partner = i ^ stride;
        if (partner > i) {
          const bool up = (i & size) == 0;
          const bool gt = pair_less(sk[partner], si[partner], sk[i], si[i]);
          if (gt == up) {
            const uint64_t tk = sk[i];
            sk[i] = sk[partner];
            sk[partner] = tk;
            const int64_t ti = si[i];
            si[i] = si[partner];
            si[partner] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    const uint32_t need = st->need;
    st->tkey = sk[need - 1];
    st->tidx = si[need - 1];
  }
}

__device__ __forceinline__ bool selected(const uint64_t* keys, int64_t j, const SelectState* st) {
  const uint64_t key = keys[j];
  return key < st->tkey || (key == st->tkey && j <= st->tidx);
}

__global__ __launch_bounds__(kScanBlock) void sub_count_kernel(const uint64_t* __restrict__ keys,
                                                               int64_t n, const SelectState* st,
                                                               uint32_t* __restrict__ blk) {
  __shared__ uint32_t red[kScanBlock / 64];
  const int64_t base = blockIdx.x * (int64_t)(kScanBlock * kScanItems);
  uint32_t c = 0;
  for (int e = 0; e < kScanItems; ++e) {
    const int64_t j = base + e * kScanBlock + threadIdx.x;
    if (j < n && selected(keys, j, st)) ++c;
  }
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int w = 0; w < kScanBlock / 64; ++w) s += red[w];
    blk[blockIdx.x] = s;
  }
}

// Exclusive scan of the per-block counts, in place (one block, any length).
__global__ __launch_bounds__(1024) void sub_blockscan_kernel(uint32_t* blk, int64_t nblk) {
  __shared__ uint32_t part[1024];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nblk; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const uint32_t v = i < nblk ? blk[i] : 0u;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const uint32_t u = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
      __syncthreads();
      part[threadIdx.x] += u;
      __syncthreads();
    }
    if (i < nblk) blk[i] = carry + part[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += part[1023];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kScanBlock) void sub_write_kernel(const uint64_t* __restrict__ keys,
                                                               int64_t n, const SelectState* st,
                                                               const uint32_t* __restrict__ blk,
                                                               int32_t* __restrict__ idx,
                                                               int32_t* __restrict__ slot) {
  __shared__ uint32_t wsum[kScanBlock / 64];
  const int64_t base = blockIdx.x * (int64_t)(kScanBlock * kScanItems);
  uint32_t offset = blk[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int e = 0; e < kScanItems; ++e) {
    const int64_t j = base + e * kScanBlock + threadIdx.x;
    const bool f = j < n && selected(keys, j, st);
    // block-wide exclusive prefix of f in thread order
    uint32_t x = f ? 1u : 0u;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int w = 0; w < kScanBlock / 64; ++w) {
      if (w < wave) before += wsum[w];
      total += wsum[w];
    }
    const uint32_t pos = offset + before + x - (f ? 1u : 0u);
    if (j < n) {
      if (f) idx[pos] = static_cast<int32_t>(j);
      if (slot != nullptr) slot[j] = f ? static_cast<int32_t>(pos) : -1;
    }
    offset += total;
    __syncthreads();
  }
}

struct SubWs {
  uint64_t* keys;
  uint32_t* hist;
  SelectState* st;
  uint64_t* cand_key;
  int64_t* cand_idx;
  uint32_t* blk;
  size_t bytes;
};

SubWs carve_sub(void* base, int64_t n) {
  SubWs w{};
  size_t off = 0;
  auto take = [&](size_t b) {
    char* p = static_cast<char*>(base) + off;
    off = align_up(off + b, 256);
    return p;
  };
  w.keys = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * n));
  w.hist = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * kHistBins + sizeof(SelectState)));
  w.st = reinterpret_cast<SelectState*>(w.hist + kHistBins);
  w.cand_key = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * kCandCap));
  w.cand_idx = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * kCandCap));
  w.blk = reinterpret_cast<uint32_t*>(
      take(sizeof(uint32_t) * ceil_div(n, kScanBlock * kScanItems)));
  w.bytes = off;
  return w;
}

}  // namespace

dsanls_status launch_gaussian_sketch_t(uint64_t seed, uint32_t t, int side, int64_t j0, int64_t n, int64_t d,
                                       float* St, int64_t ld, __hip_bfloat16* St_bf16, int64_t ld_bf16,
                                       hipStream_t s) {
  if (n <= 0 || d <= 0) return DSANLS_OK;
  const int64_t nq = ceil_div(d, 4);
  if (nq > 65535 || n > 0xFFFFFFFFll) return fail(DSANLS_E_SHAPE, "gaussian sketch: d or n too large");
  const float scale = static_cast<float>(1.0 / std::sqrt(static_cast<double>(d)));
  dim3 grid(static_cast<unsigned>(ceil_div(n, 256)), static_cast<unsigned>(nq));
  gaussian_t_kernel<<<grid, 256, 0, s>>>(static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), t,
                                         (static_cast<uint32_t>(side) & 0xFFu) | (kKindGaussian << 8), j0,
                                         n, d, scale, St, ld, St_bf16, ld_bf16);
  DSANLS_LAUNCHED("gaussian_t_kernel");
  return DSANLS_OK;
}

size_t subsample_ws_bytes(int64_t n) {
  return carve_sub(nullptr, n).bytes;
}

// idx_win[c] = idx[c] - off for the sampled indices inside [off, off + len),
// -1 for the others: the sampled columns as seen by a block of the long
// dimension (a node's share).
__global__ void sub_window_kernel(const int32_t* __restrict__ idx, int64_t d, int64_t off, int64_t len,
                                  int32_t* __restrict__ idx_win) {
  const int64_t c = blockIdx.x * 256ll + threadIdx.x;
  if (c >= d) return;
  const int64_t j = static_cast<int64_t>(idx[c]) - off;
  idx_win[c] = j >= 0 && j < len ? static_cast<int32_t>(j) : -1;
}

dsanls_status launch_subsample(uint64_t seed, uint32_t t, int side, int64_t n, int64_t d,
                               int32_t* idx, int32_t* slot, void* ws, size_t ws_bytes,
                               int* err_flag, hipStream_t s, int64_t win_off, int64_t win_len,
                               int32_t* idx_win, uint32_t kind) {
  if (d < 1 || d > n) return fail(DSANLS_E_SHAPE, "subsampling needs 1 <= d <= n");
  if (n > (int64_t(1) << 27)) return fail(DSANLS_E_UNSUPPORTED, "subsampling supports n <= 2^27");
  SubWs w = carve_sub(ws, n);
  if (ws_bytes < w.bytes) return fail(DSANLS_E_WORKSPACE, "subsample workspace too small");
  const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
  const uint32_t side_word = (static_cast<uint32_t>(side) & 0xFFu) | (kind << 8);
  DSANLS_HIP(hipMemsetAsync(w.hist, 0, sizeof(uint32_t) * kHistBins + sizeof(SelectState), s));
  const unsigned g = static_cast<unsigned>(ceil_div(n, 256));
  sub_keys_kernel<<<g, 256, 0, s>>>(k0, k1, t, side_word, n, w.keys, w.hist);
  DSANLS_LAUNCHED("sub_keys_kernel");
  sub_select_kernel<<<1, 1024, 0, s>>>(w.hist, d, w.st);
  DSANLS_LAUNCHED("sub_select_kernel");
  sub_collect_kernel<<<g, 256, 0, s>>>(w.keys, n, w.st, w.cand_key, w.cand_idx);
  DSANLS_LAUNCHED("sub_collect_kernel");
  sub_resolve_kernel<<<1, 1024, 0, s>>>(w.cand_key, w.cand_idx, w.st, err_flag);
  DSANLS_LAUNCHED("sub_resolve_kernel");
  const int64_t nblk = ceil_div(n, kScanBlock * kScanItems);
  sub_count_kernel<<<static_cast<unsigned>(nblk), kScanBlock, 0, s>>>(w.keys, n, w.st, w.blk);
  DSANLS_LAUNCHED("sub_count_kernel");
  sub_blockscan_kernel<<<1, 1024, 0, s>>>(w.blk, nblk);
  DSANLS_LAUNCHED("sub_blockscan_kernel");
  sub_write_kernel<<<static_cast<unsigned>(nblk), kScanBlock, 0, s>>>(w.keys, n, w.st, w.blk, idx,
                                                                      slot);
  DSANLS_LAUNCHED("sub_write_kernel");
  if (idx_win != nullptr) {
    sub_window_kernel<<<static_cast<unsigned>(ceil_div(d, 256)), 256, 0, s>>>(idx, d, win_off, win_len, idx_win);
    DSANLS_LAUNCHED("sub_window_kernel");
  }
  return DSANLS_OK;
}

}  // namespace dsanls

// ------------------------------------------------------------------ C ABI
using namespace dsanls;

extern "C" dsanls_status dsanls_philox4x32_10(const uint32_t* ctr, const uint32_t* key,
                                              uint32_t* out, int64_t count, void* hip_stream) {
  if (count < 0 || (count > 0 && (!ctr || !key || !out)))
    return fail(DSANLS_E_INVALID_ARG, "philox: null pointer or negative count");
  if (count == 0) return DSANLS_OK;
  philox_kernel<<<static_cast<unsigned>(ceil_div(count, 256)), 256, 0,
                  static_cast<hipStream_t>(hip_stream)>>>(ctr, key, out, count);
  DSANLS_LAUNCHED("philox_kernel");
  return DSANLS_OK;
}

extern "C" dsanls_status dsanls_gaussian_sketch_t(uint64_t seed, int64_t t, int32_t side, int64_t n,
                                                  int64_t d, float* St, int64_t ld_st,
                                                  void* hip_stream) {
  if (!St || n < 1 || d < 1 || ld_st < n || t < 0 || side < 0 || side > 255)
    return fail(DSANLS_E_INVALID_ARG, "gaussian_sketch_t: bad arguments");
  return launch_gaussian_sketch_t(seed, static_cast<uint32_t>(t), side, 0, n, d, St, ld_st, nullptr, 0,
                                  static_cast<hipStream_t>(hip_stream));
}

extern "C" size_t dsanls_subsample_workspace_bytes(int64_t n) {
  return subsample_ws_bytes(n < 1 ? 1 : n) + 256;
}

extern "C" dsanls_status dsanls_subsample_indices(uint64_t seed, int64_t t, int32_t side, int64_t n,
                                                  int64_t d, int32_t* idx, void* workspace,
                                                  size_t workspace_bytes, void* hip_stream) {
  if (!idx || !workspace || t < 0 || side < 0 || side > 255)
    return fail(DSANLS_E_INVALID_ARG, "subsample_indices: bad arguments");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(DSANLS_E_WORKSPACE, "subsample_indices: workspace must be 256-byte aligned");
  // error flag lives in the last 256 bytes of the caller's workspace
  const size_t need = subsample_ws_bytes(n);
  if (workspace_bytes < need + 256) return fail(DSANLS_E_WORKSPACE, "subsample workspace too small");
  int* flag = reinterpret_cast<int*>(static_cast<char*>(workspace) + need);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  DSANLS_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
  return launch_subsample(seed, static_cast<uint32_t>(t), side, n, d, idx, nullptr, workspace, need,
                          flag, s);
}
