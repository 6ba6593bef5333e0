// Dense products of the path on MFMA: the sketch product A = M S (and
// A' = M^T S'), B = W^T S, R = A B^T, and the residual of the objective.
//
// Every product is expressed as C = X Y^T with X (rows x K) and Y (cols x K)
// both row-major and K-contiguous: S is generated transposed (d x n) and
// M^T is kept resident next to M, as the paper's node keeps both its row
// block and its column block of M (Alg. 2 input).
//
// The sketch products run on LDS-ring kernels (gemm_nt_f32_dma_kernel,
// gemm_nt_bf16_dma_kernel, below) when K and the rows allow; otherwise, and
// for the other products:
//
// Tiling (FP32): 256 threads = 4 waves in a 2 x 2 grid; a workgroup owns a
// BM x BN tile and each wave a (BM/2) x (BN/2) sub-tile made of 32 x 32
// v_mfma_f32_32x32x2f32 blocks.  K advances in stages of 32 through a double
// buffered LDS tile (row stride 36 floats, so the 16-byte fragment reads of
// 16 consecutive lanes land on distinct banks).  Each lane reads four
// consecutive k of its row in one ds_read_b128 and feeds them to four MFMAs;
// lanes 0-31 and 32-63 take interleaved k blocks (k and k+4), which is a
// permutation of the contraction index shared by X and Y and so leaves the
// product unchanged.
#include "common.hpp"

#include <hip/hip_bf16.h>

namespace dsanls {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kBK = 32;
constexpr int kLds = kBK + 4;

// Workgroups are dispatched round-robin over the XCDs; give each XCD a
// contiguous run of tiles so the tiles sharing a row block of X meet in the
// same L2.
__device__ __forceinline__ int xcd_remap(int wg, int ntiles) {
  const int xcd = wg % kNumXcd, local = wg / kNumXcd;
  const int per = ntiles / kNumXcd, rem = ntiles % kNumXcd;
  return xcd * per + (xcd < rem ? xcd : rem) + local;
}

template <int BM, int BN>
struct TileMap {
  int row0, col0;
  __device__ TileMap(int tiles_m, int tiles_n) {
    const int logical = xcd_remap(blockIdx.x, tiles_m * tiles_n);
    row0 = (logical / tiles_n) * BM;
    col0 = (logical % tiles_n) * BN;
  }
};

// One of the (up to two) products of a grouped launch.
template <typename T>
struct Problem {
  const T* X;
  int64_t ldx;
  const T* Y;
  int64_t ldy;
  float* C;
  int64_t ldc;
  int rows, cols, K, tiles_n, ntiles;
};

// Pick the problem and tile of this workgroup in a grouped launch.  Each XCD
// (workgroup id mod 8) owns a contiguous chunk of the first product's tiles
// followed by a contiguous chunk of the second's, so every XCD gets the same
// share of both (the host orders the products longest-K first); grid =
// 8 * (c0 + c1) with c = ceil(ntiles / 8), and the few surplus workgroups
// return at once.
template <int BM, int BN, typename T>
__device__ __forceinline__ bool pick(const Problem<T>& p0, const Problem<T>& p1, Problem<T>& p,
                                     int& row0, int& col0) {
  const int wg = blockIdx.x;
  const int xcd = wg % kNumXcd, local = wg / kNumXcd;
  const int c0 = (p0.ntiles + kNumXcd - 1) / kNumXcd, c1 = (p1.ntiles + kNumXcd - 1) / kNumXcd;
  int t;
  if (local < c0) {
    t = xcd * c0 + local;
    if (t >= p0.ntiles) return false;
    p = p0;
  } else {
    t = xcd * c1 + (local - c0);
    if (local - c0 >= c1 || t >= p1.ntiles) return false;
    p = p1;
  }
  row0 = (t / p.tiles_n) * BM;
  col0 = (t % p.tiles_n) * BN;
  return true;
}

inline int grouped_grid(int n0, int n1) {
  return kNumXcd * ((n0 + kNumXcd - 1) / kNumXcd + (n1 + kNumXcd - 1) / kNumXcd);
}

template <int NV, bool VEC>
__device__ __forceinline__ void load_stage(const float* __restrict__ P, int64_t ld, int r0,
                                           int nrows, int k0, int kend, floatx4 (&reg)[NV]) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int id = v * 256 + threadIdx.x;
    const int r = id >> 3, kq = (id & 7) * 4;
    const int gr = r0 + r, gk = k0 + kq;
    floatx4 x = {0.f, 0.f, 0.f, 0.f};
    if (gr < nrows) {
      const float* p = P + (int64_t)gr * ld + gk;
      if (VEC && gk + 3 < kend) {
        x = *reinterpret_cast<const floatx4*>(p);
      } else {
        if (gk + 0 < kend) x[0] = p[0];
        if (gk + 1 < kend) x[1] = p[1];
        if (gk + 2 < kend) x[2] = p[2];
        if (gk + 3 < kend) x[3] = p[3];
      }
    }
    reg[v] = x;
  }
}

template <int NV>
__device__ __forceinline__ void store_stage(float* __restrict__ s, const floatx4 (&reg)[NV]) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int id = v * 256 + threadIdx.x;
    const int r = id >> 3, kq = (id & 7) * 4;
    *reinterpret_cast<floatx4*>(s + r * kLds + kq) = reg[v];
  }
}

// Main loop: acc += X[row0.., kbeg..kend) * Y[col0.., kbeg..kend)^T.
template <int BM, int BN, bool VEC>
__device__ __forceinline__ void mainloop(const float* __restrict__ X, int64_t ldx,
                                         const float* __restrict__ Y, int64_t ldy, int rows,
                                         int cols, int kbeg, int kend, int row0, int col0,
                                         float* sX, float* sY,
                                         floatx16 (&acc)[BM / 64][BN / 64]) {
  constexpr int FM = BM / 64, FN = BN / 64;
  constexpr int XV = BM * kBK / 4 / 256, YV = BN * kBK / 4 / 256;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lrow = lane & 31, lk = (lane >> 5) * 4;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  if (kbeg >= kend) return;

  floatx4 rx[XV], ry[YV];
  load_stage<XV, VEC>(X, ldx, row0, rows, kbeg, kend, rx);
  load_stage<YV, VEC>(Y, ldy, col0, cols, kbeg, kend, ry);
  store_stage<XV>(sX, rx);
  store_stage<YV>(sY, ry);
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += kBK) {
    const bool more = k0 + kBK < kend;
    if (more) {
      load_stage<XV, VEC>(X, ldx, row0, rows, k0 + kBK, kend, rx);
      load_stage<YV, VEC>(Y, ldy, col0, cols, k0 + kBK, kend, ry);
    }
    const float* cx = sX + buf * (BM * kLds);
    const float* cy = sY + buf * (BN * kLds);
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 8) {
      floatx4 a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        a[i] = *reinterpret_cast<const floatx4*>(cx + (wm * (BM / 2) + i * 32 + lrow) * kLds + kk + lk);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        b[j] = *reinterpret_cast<const floatx4*>(cy + (wn * (BN / 2) + j * 32 + lrow) * kLds + kk + lk);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
    }
    if (more) {
      store_stage<XV>(sX + (buf ^ 1) * (BM * kLds), rx);
      store_stage<YV>(sY + (buf ^ 1) * (BN * kLds), ry);
    }
    __syncthreads();
    buf ^= 1;
  }
}

// Row of element r of a 32x32 MFMA accumulator held by this lane.
__device__ __forceinline__ int acc_row(int r, int lane) {
  return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

template <int BM, int BN, bool VEC>
__global__ __launch_bounds__(256, 2) void gemm_nt_grouped_kernel(Problem<float> p0, Problem<float> p1) {
  __shared__ __attribute__((aligned(16))) float sX[2 * BM * kLds];
  __shared__ __attribute__((aligned(16))) float sY[2 * BN * kLds];
  constexpr int FM = BM / 64, FN = BN / 64;
  int row0, col0;
  Problem<float> p;
  if (!pick<BM, BN>(p0, p1, p, row0, col0)) return;
  floatx16 acc[FM][FN];
  mainloop<BM, BN, VEC>(p.X, p.ldx, p.Y, p.ldy, p.rows, p.cols, 0, p.K, row0, col0, sX, sY, acc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = col0 + wn * (BN / 2) + j * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = row0 + wm * (BM / 2) + i * 32 + acc_row(r, lane);
        if (row < p.rows && col < p.cols) p.C[(int64_t)row * p.ldc + col] = acc[i][j][r];
      }
    }
}

template <int BM, int BN, bool VEC>
__global__ __launch_bounds__(256, 2) void gemm_nt_kernel(const float* __restrict__ X, int64_t ldx,
                                                         const float* __restrict__ Y, int64_t ldy,
                                                         float* __restrict__ C, int64_t ldc,
                                                         int64_t split_stride, int rows, int cols,
                                                         int K, int kchunk, int tiles_m,
                                                         int tiles_n) {
  __shared__ __attribute__((aligned(16))) float sX[2 * BM * kLds];
  __shared__ __attribute__((aligned(16))) float sY[2 * BN * kLds];
  constexpr int FM = BM / 64, FN = BN / 64;
  const TileMap<BM, BN> tile(tiles_m, tiles_n);
  const int kbeg = blockIdx.y * kchunk;
  const int kend = min(K, kbeg + kchunk);
  floatx16 acc[FM][FN];
  mainloop<BM, BN, VEC>(X, ldx, Y, ldy, rows, cols, kbeg, kend, tile.row0, tile.col0, sX, sY, acc);
  float* Cz = C + blockIdx.y * split_stride;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = tile.col0 + wn * (BN / 2) + j * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = tile.row0 + wm * (BM / 2) + i * 32 + acc_row(r, lane);
        if (row < rows && col < cols) Cz[(int64_t)row * ldc + col] = acc[i][j][r];
      }
    }
}

// Fixed-order compensated sum over the split-K partials.
__global__ void splitk_reduce_kernel(const float* __restrict__ P, int64_t split_stride, int splits,
                                     int rows, int cols, float* __restrict__ C, int64_t ldc) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows * cols) return;
  const int r = static_cast<int>(i / cols), c = static_cast<int>(i % cols);
  float s = 0.f, comp = 0.f;
  for (int z = 0; z < splits; ++z) {
    const float x = P[z * split_stride + i];
    const float t = s + x;
    comp += fabsf(s) >= fabsf(x) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  C[(int64_t)r * ldc + c] = s + comp;
}

// Neumaier update of (s, c) with x.
__device__ __forceinline__ void neumaier(float& s, float& c, float x) {
  const float t = s + x;
  c += fabsf(s) >= fabsf(x) ? (s - t) + x : (x - t) + s;
  s = t;
}

// Sum over the tile of (M - U V^T)^2; one compensated (sum, comp) pair per
// workgroup.  The residual is formed entry by entry, so a near-exact fit
// does not lose its digits to cancellation.
template <int BM, int BN, bool VEC>
__global__ __launch_bounds__(256, 2) void residual_kernel(const float* __restrict__ U,
                                                          const float* __restrict__ V, int k,
                                                          const float* __restrict__ M,
                                                          int64_t ldm, int rows, int cols,
                                                          int tiles_m, int tiles_n,
                                                          float* __restrict__ partials) {
  __shared__ __attribute__((aligned(16))) float sX[2 * BM * kLds];
  __shared__ __attribute__((aligned(16))) float sY[2 * BN * kLds];
  __shared__ float red[2 * 4];
  constexpr int FM = BM / 64, FN = BN / 64;
  const TileMap<BM, BN> tile(tiles_m, tiles_n);
  floatx16 acc[FM][FN];
  mainloop<BM, BN, VEC>(U, k, V, k, rows, cols, 0, k, tile.row0, tile.col0, sX, sY, acc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  float s = 0.f, c = 0.f;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = tile.col0 + wn * (BN / 2) + j * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = tile.row0 + wm * (BM / 2) + i * 32 + acc_row(r, lane);
        if (row < rows && col < cols) {
          const float e = M[(int64_t)row * ldm + col] - acc[i][j][r];
          neumaier(s, c, e * e);
        }
      }
    }
  // wave tree of compensated pairs, then the four waves in order
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
    for (int w = 1; w < 4; ++w) {
      neumaier(ts, tc, red[2 * w]);
      tc += red[2 * w + 1];
    }
    const int64_t b = blockIdx.x;
    partials[2 * b] = ts;
    partials[2 * b + 1] = tc;
  }
}


// ---------------------------------------------------------------- BF16
// A = M S with M and S rounded to BF16 (the precision form) on
// v_mfma_f32_32x32x16_bf16 (FP32 accumulation).  General kernel (any K,
// leading dimension or alignment): operands staged through registers.
// K advances 64 bf16 (128 bytes per row) per stage; the LDS row stride of
// 72 bf16 (36 dwords) keeps 16-byte fragment reads conflict-free.  Lane
// halves take k blocks 0-7 and 8-15 of each 16-wide step for both operands.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushortx8 __attribute__((ext_vector_type(8)));

constexpr int kBKh = 64;
constexpr int kLdsh = kBKh + 8;
// BF16 block tile 256 x 256 in eight waves of 128 x 64 (4 x 2 MFMA tiles):
// two waves per SIMD, so one wave's MFMAs cover the other's wait for its
// next stage (1.12x over four waves of 128 x 128 at one wave per SIMD),
// while every fragment read from LDS still feeds two to four MFMAs (a
// 64 x 64 wave tile would need 128 B/clk of LDS reads per CU at the MFMA
// rate, the whole port).
constexpr int kBMh = 256, kBNh = 256;
constexpr int kWvMh = 2, kWvNh = 4;

template <int NV, bool VEC, int NT = 256>
__device__ __forceinline__ void load_stage_h(const unsigned short* __restrict__ P, int64_t ld, int r0,
                                             int nrows, int k0, int kend, ushortx8 (&reg)[NV]) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int id = v * NT + threadIdx.x;
    const int r = id >> 3, kq = (id & 7) * 8;
    const int gr = r0 + r, gk = k0 + kq;
    ushortx8 x = {0, 0, 0, 0, 0, 0, 0, 0};
    if (gr < nrows) {
      const unsigned short* p = P + (int64_t)gr * ld + gk;
      if (VEC && gk + 7 < kend) {
        x = *reinterpret_cast<const ushortx8*>(p);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (gk + e < kend) x[e] = p[e];
      }
    }
    reg[v] = x;
  }
}

template <int NV, int NT = 256>
__device__ __forceinline__ void store_stage_h(unsigned short* __restrict__ s, const ushortx8 (&reg)[NV]) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int id = v * NT + threadIdx.x;
    const int r = id >> 3, kq = (id & 7) * 8;
    *reinterpret_cast<ushortx8*>(s + r * kLdsh + kq) = reg[v];
  }
}

template <int BM, int BN, bool VEC, int WVM = 2, int WVN = 2>
__global__ __launch_bounds__(64 * WVM * WVN, 1) void gemm_nt_bf16_kernel(Problem<unsigned short> p0,
                                                              Problem<unsigned short> p1) {
  __shared__ __attribute__((aligned(16))) unsigned short sX[2 * BM * kLdsh];
  __shared__ __attribute__((aligned(16))) unsigned short sY[2 * BN * kLdsh];
  // WVM x WVN waves, each a (BM / WVM) x (BN / WVN) tile of 32 x 32 MFMA tiles
  constexpr int NT = 64 * WVM * WVN, TM = BM / WVM, TN = BN / WVN;
  constexpr int FM = TM / 32, FN = TN / 32;
  constexpr int XV = BM * kBKh / 8 / NT, YV = BN * kBKh / 8 / NT;
  int row0, col0;
  Problem<unsigned short> p;
  if (!pick<BM, BN>(p0, p1, p, row0, col0)) return;
  const unsigned short* X = p.X;
  const unsigned short* Y = p.Y;
  const int64_t ldx = p.ldx, ldy = p.ldy;
  const int rows = p.rows, cols = p.cols, K = p.K;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WVN, wn = wave % WVN;
  const int lrow = lane & 31, lk = (lane >> 5) * 8;
  floatx16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  if (K > 0) {
    ushortx8 rx[XV], ry[YV];
    load_stage_h<XV, VEC, NT>(X, ldx, row0, rows, 0, K, rx);
    load_stage_h<YV, VEC, NT>(Y, ldy, col0, cols, 0, K, ry);
    store_stage_h<XV, NT>(sX, rx);
    store_stage_h<YV, NT>(sY, ry);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < K; k0 += kBKh) {
      const bool more = k0 + kBKh < K;
      if (more) {
        load_stage_h<XV, VEC, NT>(X, ldx, row0, rows, k0 + kBKh, K, rx);
        load_stage_h<YV, VEC, NT>(Y, ldy, col0, cols, k0 + kBKh, K, ry);
      }
      const unsigned short* cx = sX + buf * (BM * kLdsh);
      const unsigned short* cy = sY + buf * (BN * kLdsh);
#pragma unroll
      for (int kk = 0; kk < kBKh; kk += 16) {
        bf16x8 a[FM], b[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
          a[i] = *reinterpret_cast<const bf16x8*>(cx + (wm * TM + i * 32 + lrow) * kLdsh + kk + lk);
#pragma unroll
        for (int j = 0; j < FN; ++j)
          b[j] = *reinterpret_cast<const bf16x8*>(cy + (wn * TN + j * 32 + lrow) * kLdsh + kk + lk);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
      }
      if (more) {
        store_stage_h<XV, NT>(sX + (buf ^ 1) * (BM * kLdsh), rx);
        store_stage_h<YV, NT>(sY + (buf ^ 1) * (BN * kLdsh), ry);
      }
      __syncthreads();
      buf ^= 1;
    }
  }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = col0 + wn * TN + j * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = row0 + wm * TM + i * 32 + acc_row(r, lane);
        if (row < rows && col < cols) p.C[(int64_t)row * p.ldc + col] = acc[i][j][r];
      }
    }
}

// Fast BF16 kernel, for K a multiple of 32 and 16-byte aligned rows (the
// method pads its BF16 copies of M and S with zero columns to that).  The
// operands go from HBM straight into LDS (global_load_lds_dwordx4, no
// register staging) through a ring of NS stages of 32 k each: while one
// stage feeds the MFMAs, the next NS - 1 are in flight, so a load has NS - 1
// stage times to arrive (the register-staged kernel gives it one).  One DMA
// load writes 64 consecutive 16-byte slots (16 tile rows of 32 bf16), so the
// rows cannot be padded apart; instead chunk c of tile row r lives in slot
// c ^ f(r), and each lane fetches the chunk that belongs in its slot.  With
// bits r1, r2, r3 of r, f(r) = r2 | (r1 ^ r3) << 1 puts the eight lanes that
// a 16-byte LDS read serves together on distinct banks whether those are
// eight consecutive lanes or two quads q, q ^ x (x odd) of a half-wave; the
// 0 bank-conflict cycles it measures compare with 1.5e9 per launch for
// ((r >> 1) ^ (r >> 3)) & 3, which only spreads consecutive lanes (a 2.4%
// difference in time).  Tile rows past the end of an operand re-read its
// last row (their results are not stored).  The compiler orders neither the
// DMA writes before the fragment reads nor the reads before the next DMA
// into the same stage, so the waits are explicit: vmcnt for this wave's own
// loads, then lgkmcnt(0) and a barrier for every wave's.
constexpr int kBKd = 32;
// four stages (128 KB of LDS): 1.01x over three, 1.01x over five
constexpr int kRingd = 4;

__device__ __forceinline__ int swz64(int r) { return ((r >> 2) & 1) | ((((r >> 1) ^ (r >> 3)) & 1) << 1); }

template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N == 0 || N == 3 || N == 4 || N == 6 || N == 8 || N == 16 || N == 32, "vmcnt immediate");
  if constexpr (N == 0) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  else if constexpr (N == 3) asm volatile("s_waitcnt vmcnt(3)" ::: "memory");
  else if constexpr (N == 6) asm volatile("s_waitcnt vmcnt(6)" ::: "memory");
  else if constexpr (N == 4) asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
  else if constexpr (N == 8) asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
  else if constexpr (N == 16) asm volatile("s_waitcnt vmcnt(16)" ::: "memory");
  else asm volatile("s_waitcnt vmcnt(32)" ::: "memory");
}

// every wave's LDS reads done, then all waves meet
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// ROWS tile rows of one operand, 64 bytes of k each (32 bf16 or 16 floats),
// into a stage: ROWS / 16 DMA loads of 16 rows, spread over the NW waves.
template <typename T, int ROWS, int NW>
__device__ __forceinline__ void dma_tile(const T* __restrict__ P, int64_t ld, int r0, int nrows, int k0,
                                         T* lds) {
  constexpr int RowE = 64 / sizeof(T), ChE = 16 / sizeof(T);
  static_assert((ROWS / 16) % NW == 0, "tile split");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < ROWS / 16 / NW; ++i) {
    const int blk = i * NW + wave;
    const int r = blk * 16 + (lane >> 2);
    const int c = (lane & 3) ^ swz64(r);
    const int gr = min(r0 + r, nrows - 1);
    __builtin_amdgcn_global_load_lds(P + (int64_t)gr * ld + k0 + c * ChE, lds + blk * 16 * RowE, 16, 0, 0);
  }
}

template <int WVM, int WVN, int NS>
__global__ __launch_bounds__(64 * WVM * WVN, 1) void gemm_nt_bf16_dma_kernel(Problem<unsigned short> p0,
                                                                             Problem<unsigned short> p1) {
  constexpr int BM = 256, BN = 256, NW = WVM * WVN, TM = BM / WVM, TN = BN / WVN;
  constexpr int FM = TM / 32, FN = TN / 32;
  constexpr int STAGE = (BM + BN) * kBKd;   // bf16 per stage (X tile, then Y tile)
  constexpr int IPW = 2 * 16 / NW;          // DMA loads per wave per stage
  static_assert(16 % NW == 0 && NS >= 2, "tile split");
  __shared__ __attribute__((aligned(1024))) unsigned short sm[NS * STAGE];
  int row0, col0;
  Problem<unsigned short> p;
  if (!pick<BM, BN>(p0, p1, p, row0, col0)) return;
  const unsigned short* X = p.X;
  const unsigned short* Y = p.Y;
  const int64_t ldx = p.ldx, ldy = p.ldy;
  const int rows = p.rows, cols = p.cols, nk = p.K / kBKd;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WVN, wn = wave % WVN;
  const int lrow = lane & 31, hi = lane >> 5;
  // tile rows of a fragment are 32-aligned, so the slot swizzle depends on lrow only
  const int sw = swz64(lrow);
  const int off0 = lrow * kBKd + ((hi ^ sw) << 3), off1 = lrow * kBKd + (((2 + hi) ^ sw) << 3);
  floatx16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
#pragma unroll
  for (int st = 0; st < NS - 1; ++st)
    if (st < nk) {
      dma_tile<unsigned short, BM, NW>(X, ldx, row0, rows, st * kBKd, sm + st * STAGE);
      dma_tile<unsigned short, BN, NW>(Y, ldy, col0, cols, st * kBKd, sm + st * STAGE + BM * kBKd);
    }
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + NS - 2 < nk)
      wait_vm<(NS - 2) * IPW>();
    else
      wait_vm<0>();
    lds_barrier();
    const int nx = kt + NS - 1;
    if (nx < nk) {
      unsigned short* dst = sm + (nx % NS) * STAGE;
      dma_tile<unsigned short, BM, NW>(X, ldx, row0, rows, nx * kBKd, dst);
      dma_tile<unsigned short, BN, NW>(Y, ldy, col0, cols, nx * kBKd, dst + BM * kBKd);
    }
    const unsigned short* sx = sm + (kt % NS) * STAGE + wm * TM * kBKd;
    const unsigned short* sy = sm + (kt % NS) * STAGE + BM * kBKd + wn * TN * kBKd;
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const int off = kk == 0 ? off0 : off1;
      bf16x8 a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = *reinterpret_cast<const bf16x8*>(sx + i * 32 * kBKd + off);
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = *reinterpret_cast<const bf16x8*>(sy + j * 32 * kBKd + off);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = col0 + wn * TN + j * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = row0 + wm * TM + i * 32 + acc_row(r, lane);
        if (row < rows && col < cols) p.C[(int64_t)row * p.ldc + col] = acc[i][j][r];
      }
    }
}

// FP32 sketch product on the same LDS ring: 128 x 64 WVN tile, 2 WVN waves
// of 64 x 64 (2 x 2 v_mfma_f32_32x32x2f32), stages of 16 k (64-byte rows,
// the same chunk swizzle).
// A lane reads four consecutive k of its row (one 16-byte chunk) and feeds
// them to four MFMAs; lanes 0-31 and 32-63 take chunks 2g and 2g + 1, a
// permutation of the contraction index shared by both operands.  Used when
// K is a multiple of 16 with 16-byte aligned rows.
constexpr int kBKf = 16;
// 128 x 256 tiles in eight waves of 64 x 64 (kWvNf = 4 along N) and three
// stages of 24 KB (two workgroups, sixteen waves per CU): 0.862 of the FP32
// MFMA peak on the 20000 x 10000 sketch product (two stages: 0.869, four:
// 0.837); 128 x 128 tiles in four waves reached 0.821, the register-staged
// kernel 0.748
constexpr int kRingf = 3;
constexpr int kWvNf = 4;   // waves along N (tile 128 x 64 kWvNf)

template <int NS, int WVN>
__global__ __launch_bounds__(128 * WVN, WVN <= 4 ? 2 : 1) void gemm_nt_f32_dma_kernel(Problem<float> p0, Problem<float> p1) {
  constexpr int BM = 128, BN = 64 * WVN, NW = 2 * WVN, FM = 2, FN = 2;
  constexpr int STAGE = (BM + BN) * kBKf;   // floats per stage (X tile, then Y tile)
  constexpr int IPW = (BM + BN) / 16 / NW;  // DMA loads per wave per stage
  __shared__ __attribute__((aligned(1024))) float sm[NS * STAGE];
  int row0, col0;
  Problem<float> p;
  if (!pick<BM, BN>(p0, p1, p, row0, col0)) return;
  const float* X = p.X;
  const float* Y = p.Y;
  const int64_t ldx = p.ldx, ldy = p.ldy;
  const int rows = p.rows, cols = p.cols, nk = p.K / kBKf;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WVN, wn = wave % WVN;
  const int lrow = lane & 31, hi = lane >> 5;
  const int sw = swz64(lrow);
  const int off0 = lrow * kBKf + ((hi ^ sw) << 2), off1 = lrow * kBKf + (((2 + hi) ^ sw) << 2);
  floatx16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
#pragma unroll
  for (int st = 0; st < NS - 1; ++st)
    if (st < nk) {
      dma_tile<float, BM, NW>(X, ldx, row0, rows, st * kBKf, sm + st * STAGE);
      dma_tile<float, BN, NW>(Y, ldy, col0, cols, st * kBKf, sm + st * STAGE + BM * kBKf);
    }
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + NS - 2 < nk)
      wait_vm<(NS - 2) * IPW>();
    else
      wait_vm<0>();
    lds_barrier();
    const int nx = kt + NS - 1;
    if (nx < nk) {
      float* dst = sm + (nx % NS) * STAGE;
      dma_tile<float, BM, NW>(X, ldx, row0, rows, nx * kBKf, dst);
      dma_tile<float, BN, NW>(Y, ldy, col0, cols, nx * kBKf, dst + BM * kBKf);
    }
    const float* sx = sm + (kt % NS) * STAGE + wm * (BM / 2) * kBKf;
    const float* sy = sm + (kt % NS) * STAGE + BM * kBKf + wn * 64 * kBKf;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int off = g == 0 ? off0 : off1;
      floatx4 a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = *reinterpret_cast<const floatx4*>(sx + i * 32 * kBKf + off);
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = *reinterpret_cast<const floatx4*>(sy + j * 32 * kBKf + off);
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][s4], b[j][s4], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = col0 + wn * 64 + j * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = row0 + wm * (BM / 2) + i * 32 + acc_row(r, lane);
        if (row < rows && col < cols) p.C[(int64_t)row * p.ldc + col] = acc[i][j][r];
      }
    }
}

template <int BM, int BN>
dsanls_status gemm_dispatch(const float* X, int64_t ldx, const float* Y, int64_t ldy, float* C,
                            int64_t ldc, int64_t split_stride, int rows, int cols, int K,
                            int splits, int kchunk, hipStream_t s) {
  const int tm = static_cast<int>(ceil_div(rows, BM)), tn = static_cast<int>(ceil_div(cols, BN));
  dim3 grid(tm * tn, splits);
  const bool vec = (ldx % 4 == 0) && (ldy % 4 == 0) && (reinterpret_cast<uintptr_t>(X) % 16 == 0) &&
                   (reinterpret_cast<uintptr_t>(Y) % 16 == 0);
  if (vec)
    gemm_nt_kernel<BM, BN, true><<<grid, 256, 0, s>>>(X, ldx, Y, ldy, C, ldc, split_stride, rows,
                                                      cols, K, kchunk, tm, tn);
  else
    gemm_nt_kernel<BM, BN, false><<<grid, 256, 0, s>>>(X, ldx, Y, ldy, C, ldc, split_stride, rows,
                                                       cols, K, kchunk, tm, tn);
  DSANLS_LAUNCHED("gemm_nt_kernel");
  return DSANLS_OK;
}

struct SplitPlan {
  int splits, kchunk;
};

SplitPlan plan_split(int64_t rows, int64_t cols, int64_t K, int bm, int bn) {
  if (K <= 0) return {1, kBK};
  const int64_t tiles = ceil_div(rows, bm) * ceil_div(cols, bn);
  int64_t splits = 1;
  // fewer tiles than half the workgroup slots of the chip and a long K:
  // split K so that about 512 workgroups run, each with >= 8 stages
  if (tiles < 256 && K >= 16 * kBK) {
    splits = std::min<int64_t>(ceil_div(512, tiles), K / (8 * kBK));
    splits = std::max<int64_t>(1, std::min<int64_t>(splits, 64));
  }
  int64_t kchunk = ceil_div(ceil_div(K, splits), kBK) * kBK;
  splits = ceil_div(K, kchunk);
  return {static_cast<int>(splits), static_cast<int>(kchunk)};
}

}  // namespace

size_t gemm_ws_bytes(int64_t rows, int64_t cols, int64_t K) {
  const int bn = cols <= 64 ? 64 : 128;
  const SplitPlan p = plan_split(rows, cols, K, 128, bn);
  return p.splits > 1 ? sizeof(float) * p.splits * rows * cols : 0;
}

dsanls_status launch_gemm_nt(const float* X, int64_t ldx, const float* Y, int64_t ldy, float* C,
                             int64_t ldc, int64_t rows, int64_t cols, int64_t K, void* ws,
                             size_t ws_bytes, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return DSANLS_OK;
  if (rows > INT32_MAX || cols > INT32_MAX || K > INT32_MAX)
    return fail(DSANLS_E_SHAPE, "gemm: dimension exceeds int32");
  if (ceil_div(rows, 64) * ceil_div(cols, 64) > INT32_MAX) return fail(DSANLS_E_SHAPE, "gemm: too many tiles");
  const int bn = cols <= 64 ? 64 : 128;
  SplitPlan p = plan_split(rows, cols, K, 128, bn);
  const size_t need = p.splits > 1 ? sizeof(float) * p.splits * rows * cols : 0;
  if (p.splits > 1 && (ws == nullptr || ws_bytes < need)) p = {1, static_cast<int>(ceil_div(K, kBK) * kBK)};
  if (p.splits == 1) {
    const int kchunk = static_cast<int>(std::max<int64_t>(kBK, ceil_div(K, kBK) * kBK));
    if (bn == 64)
      return gemm_dispatch<128, 64>(X, ldx, Y, ldy, C, ldc, 0, (int)rows, (int)cols, (int)K, 1, kchunk, s);
    return gemm_dispatch<128, 128>(X, ldx, Y, ldy, C, ldc, 0, (int)rows, (int)cols, (int)K, 1, kchunk, s);
  }
  float* P = static_cast<float*>(ws);
  const int64_t stride = rows * cols;
  dsanls_status st;
  if (bn == 64)
    st = gemm_dispatch<128, 64>(X, ldx, Y, ldy, P, cols, stride, (int)rows, (int)cols, (int)K, p.splits, p.kchunk, s);
  else
    st = gemm_dispatch<128, 128>(X, ldx, Y, ldy, P, cols, stride, (int)rows, (int)cols, (int)K, p.splits, p.kchunk, s);
  if (st != DSANLS_OK) return st;
  splitk_reduce_kernel<<<static_cast<unsigned>(ceil_div(stride, 256)), 256, 0, s>>>(
      P, stride, p.splits, (int)rows, (int)cols, C, ldc);
  DSANLS_LAUNCHED("splitk_reduce_kernel");
  return DSANLS_OK;
}

int64_t residual_partials(int64_t m, int64_t n) { return ceil_div(m, 128) * ceil_div(n, 128); }

dsanls_status launch_residual_sq(const float* M, int64_t ldm, const float* U, const float* V,
                                 int64_t m, int64_t n, int64_t k, float* partials, hipStream_t s) {
  const int tm = static_cast<int>(ceil_div(m, 128)), tn = static_cast<int>(ceil_div(n, 128));
  const bool vec = (k % 4 == 0) && (reinterpret_cast<uintptr_t>(U) % 16 == 0) &&
                   (reinterpret_cast<uintptr_t>(V) % 16 == 0);
  if (vec)
    residual_kernel<128, 128, true><<<tm * tn, 256, 0, s>>>(U, V, (int)k, M, ldm, (int)m, (int)n, tm, tn, partials);
  else
    residual_kernel<128, 128, false><<<tm * tn, 256, 0, s>>>(U, V, (int)k, M, ldm, (int)m, (int)n, tm, tn, partials);
  DSANLS_LAUNCHED("residual_kernel");
  return DSANLS_OK;
}

namespace {

template <typename T>
bool make_problem(const GemmDesc& g, int elems_per_vec, Problem<T>& p, bool& vec, int bm = 128, int bn = 128) {
  if (g.rows <= 0 || g.cols <= 0) {
    p = Problem<T>{nullptr, 0, nullptr, 0, nullptr, 0, 0, 0, 0, 1, 0};
    return true;
  }
  if (g.rows > INT32_MAX || g.cols > INT32_MAX || g.K > INT32_MAX) return false;
  const int tm = static_cast<int>(ceil_div(g.rows, bm)), tn = static_cast<int>(ceil_div(g.cols, bn));
  p = Problem<T>{static_cast<const T*>(g.X), g.ldx, static_cast<const T*>(g.Y), g.ldy, g.C, g.ldc,
                 static_cast<int>(g.rows), static_cast<int>(g.cols), static_cast<int>(g.K), tn, tm * tn};
  vec = vec && (g.ldx % elems_per_vec == 0) && (g.ldy % elems_per_vec == 0) &&
        (reinterpret_cast<uintptr_t>(g.X) % 16 == 0) && (reinterpret_cast<uintptr_t>(g.Y) % 16 == 0);
  return true;
}

}  // namespace

dsanls_status launch_gemm_grouped(const GemmDesc& a_in, const GemmDesc& b_in, bool bf16,
                                  hipStream_t s) {
  // longest-K product first, so each XCD starts its longest tiles first
  const bool swap = b_in.rows > 0 && b_in.cols > 0 && b_in.K > a_in.K;
  const GemmDesc& a = swap ? b_in : a_in;
  const GemmDesc& b = swap ? a_in : b_in;
  bool vec = true;
  if (bf16) {
    Problem<unsigned short> p0, p1;
    if (!make_problem(a, 8, p0, vec, kBMh, kBNh) || !make_problem(b, 8, p1, vec, kBMh, kBNh))
      return fail(DSANLS_E_SHAPE, "gemm: dimension exceeds int32");
    if (p0.ntiles + p1.ntiles == 0) return DSANLS_OK;
    const int grid = grouped_grid(p0.ntiles, p1.ntiles);
    const bool dma = vec && p0.K % kBKd == 0 && (p1.ntiles == 0 || p1.K % kBKd == 0);
    if (dma) {
      gemm_nt_bf16_dma_kernel<kWvMh, kWvNh, kRingd><<<grid, 64 * kWvMh * kWvNh, 0, s>>>(p0, p1);
      DSANLS_LAUNCHED("gemm_nt_bf16_dma_kernel");
      return DSANLS_OK;
    }
    if (vec)
      gemm_nt_bf16_kernel<kBMh, kBNh, true, kWvMh, kWvNh><<<grid, 64 * kWvMh * kWvNh, 0, s>>>(p0, p1);
    else
      gemm_nt_bf16_kernel<kBMh, kBNh, false, kWvMh, kWvNh><<<grid, 64 * kWvMh * kWvNh, 0, s>>>(p0, p1);
    DSANLS_LAUNCHED("gemm_nt_bf16_kernel");
    return DSANLS_OK;
  }
  Problem<float> p0, p1;
  {
    Problem<float> q0, q1;
    if (!make_problem(a, 4, q0, vec, 128, 64 * kWvNf) || !make_problem(b, 4, q1, vec, 128, 64 * kWvNf))
      return fail(DSANLS_E_SHAPE, "gemm: dimension exceeds int32");
    if (q0.ntiles + q1.ntiles == 0) return DSANLS_OK;
    if (vec && (q0.ntiles == 0 || q0.K % kBKf == 0) && (q1.ntiles == 0 || q1.K % kBKf == 0)) {
      gemm_nt_f32_dma_kernel<kRingf, kWvNf><<<grouped_grid(q0.ntiles, q1.ntiles), 128 * kWvNf, 0, s>>>(q0, q1);
      DSANLS_LAUNCHED("gemm_nt_f32_dma_kernel");
      return DSANLS_OK;
    }
  }
  vec = true;
  if (!make_problem(a, 4, p0, vec) || !make_problem(b, 4, p1, vec))
    return fail(DSANLS_E_SHAPE, "gemm: dimension exceeds int32");
  const int grid = grouped_grid(p0.ntiles, p1.ntiles);
  if (vec)
    gemm_nt_grouped_kernel<128, 128, true><<<grid, 256, 0, s>>>(p0, p1);
  else
    gemm_nt_grouped_kernel<128, 128, false><<<grid, 256, 0, s>>>(p0, p1);
  DSANLS_LAUNCHED("gemm_nt_grouped_kernel");
  return DSANLS_OK;
}

dsanls_status launch_gemm_nt_bf16(const __hip_bfloat16* X, int64_t ldx, const __hip_bfloat16* Y,
                                  int64_t ldy, float* C, int64_t ldc, int64_t rows, int64_t cols,
                                  int64_t K, hipStream_t s) {
  const GemmDesc a{X, ldx, Y, ldy, C, ldc, rows, cols, K};
  const GemmDesc none{nullptr, 0, nullptr, 0, nullptr, 0, 0, 0, 0};
  return launch_gemm_grouped(a, none, true, s);
}

}  // namespace dsanls

using namespace dsanls;

extern "C" size_t dsanls_gemm_workspace_bytes(int64_t rows, int64_t cols, int64_t K) {
  return gemm_ws_bytes(rows, cols, K);
}

extern "C" dsanls_status dsanls_gemm_nt(const float* X, int64_t ldx, const float* Y, int64_t ldy,
                                        float* C, int64_t ldc, int64_t rows, int64_t cols,
                                        int64_t K, void* workspace, size_t workspace_bytes,
                                        void* hip_stream) {
  if (rows < 0 || cols < 0 || K < 0) return fail(DSANLS_E_SHAPE, "gemm_nt: negative size");
  if (rows == 0 || cols == 0) return DSANLS_OK;
  if ((K > 0 && (!X || !Y)) || !C || ldx < K || ldy < K || ldc < cols)
    return fail(DSANLS_E_INVALID_ARG, "gemm_nt: null pointer or leading dimension too small");
  return launch_gemm_nt(X, ldx, Y, ldy, C, ldc, rows, cols, K, workspace, workspace_bytes,
                        static_cast<hipStream_t>(hip_stream));
}

extern "C" dsanls_status dsanls_gemm_nt_bf16(const void* X, int64_t ldx, const void* Y, int64_t ldy,
                                             float* C, int64_t ldc, int64_t rows, int64_t cols,
                                             int64_t K, void* hip_stream) {
  if (rows < 0 || cols < 0 || K < 0) return fail(DSANLS_E_SHAPE, "gemm_nt_bf16: negative size");
  if (rows == 0 || cols == 0) return DSANLS_OK;
  if ((K > 0 && (!X || !Y)) || !C || ldx < K || ldy < K || ldc < cols)
    return fail(DSANLS_E_INVALID_ARG, "gemm_nt_bf16: null pointer or leading dimension too small");
  return launch_gemm_nt_bf16(static_cast<const __hip_bfloat16*>(X), ldx,
                             static_cast<const __hip_bfloat16*>(Y), ldy, C, ldc, rows, cols, K,
                             static_cast<hipStream_t>(hip_stream));
}
