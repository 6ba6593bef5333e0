// Prox-CD sweeps (Alg. 3, eq. entry_sol) for ranks above 128, where neither
// a row of U nor the Gram fits the lane-per-row kernels: 16 rows per wave,
// the rank padded to KP = 16 NBK and split into NBK blocks of 16
// coordinates.  For coordinate j of block b,
//     sum_{l != j} G_lj u_l = T_j + sum_{l in b, l != j} G_lj u_l,
//     T_j = sum_{l outside b} G_lj u_l,
// the blocks before b already holding this sweep's values (Gauss-Seidel
// order, as in Alg. 3).  T for the block's 16 coordinates and the wave's 16
// rows is one product (16 x (KP - 16)) x ((KP - 16) x 16) on
// v_mfma_f32_16x16x4f32 (2 (KP - 16) 16 * 16 flops per block); the 16
// coordinates then run one lane per row, with the block's own 16 x 16 part
// of G read by broadcast.
//
// Registers hold the iterate in the MFMA B-operand layout: lane (m, g) =
// (lane % 16, lane / 16) holds u[row m][4 q + g] in slot q (NQ = 4 NBK
// slots); the slots rotate by one block after each block, so block b always
// sits in slots 0..3 while the block loop runs at run time.  G (prepared:
// row j = column j of G, zero diagonal, KP x KP) is staged block by block
// (16 rows of KP) into LDS, double buffered and shared by the workgroup's
// four waves, so one block of G read from L2 serves 64 rows.
#include "common.hpp"

namespace dsanls {

namespace {

__device__ __forceinline__ void wguard(float& g, float x) { g = __builtin_fmaf(x, 0.f, g); }

template <int NBK>
__global__ __launch_bounds__(256) void prox_cd_wide_kernel(const float* __restrict__ gp, const float* __restrict__ inv,
                                                           const float* __restrict__ R, const float* C, float* U,
                                                           int64_t rows, int k, float mu, int sweeps, float upper,
                                                           int32_t* __restrict__ sweeps_used) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  // a G block is 16 x KP floats = 4 KP float4s, NG per thread (the last
  // round partial when KP is not a multiple of 64)
  constexpr int KP = 16 * NBK, NQ = 4 * NBK, GS = KP + 4, NG4 = 4 * KP, NG = (NG4 + 255) / 256;
  __shared__ __attribute__((aligned(16))) float gl[2][16 * GS];
  __shared__ float sinv[KP];
  __shared__ float tx[4][16 * 17];
  __shared__ float ux[4][16 * 17];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, m = lane & 15, g = lane >> 4;
  const int64_t row0 = (blockIdx.x * 4ll + w) * 16;
  // a wave past the last row still takes part in every barrier
  const int nrows = rows - row0 <= 0 ? 0 : (rows - row0 < 16 ? static_cast<int>(rows - row0) : 16);
  const float ubnd = upper > 0.f ? upper : INFINITY;
  for (int i = tid; i < KP; i += 256) sinv[i] = inv[i];

  float u[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int c = 4 * q + g;
    u[q] = m < nrows && c < k ? U[(row0 + m) * k + c] : 0.f;
  }

  // G block b (rows 16 b .. 16 b + 15 of the prepared Gram) in flight in
  // registers, then into LDS buffer buf
  const f4* gp4 = reinterpret_cast<const f4*>(gp);
  f4 gs[NG];
  auto load_g = [&](int b) {
#pragma unroll
    for (int r = 0; r < NG; ++r) {
      const int e = tid + 256 * r, i = e / (KP / 4), l4 = e % (KP / 4);
      if (NG4 % 256 == 0 || e < NG4) gs[r] = gp4[(16 * b + i) * (KP / 4) + l4];
    }
  };
  auto store_g = [&](int buf) {
#pragma unroll
    for (int r = 0; r < NG; ++r) {
      const int e = tid + 256 * r, i = e / (KP / 4), l4 = e % (KP / 4);
      if (NG4 % 256 == 0 || e < NG4) *reinterpret_cast<f4*>(&gl[buf][i * GS + 4 * l4]) = gs[r];
    }
  };
  load_g(0);
  store_g(0);
  __syncthreads();

  float gd = 0.f;   // non-finite guard of row `lane` (lanes < 16)
  int buf = 0;
  for (int s = 0; s < sweeps; ++s) {
    const bool c_is_u = s == 0 && C == U;
    for (int b = 0; b < NBK; ++b) {
      const bool more = b + 1 < NBK || s + 1 < sweeps;
      if (more) load_g(b + 1 < NBK ? b + 1 : 0);
      // right-hand side of the block for the row of this lane (lanes < 16)
      float qv[16];
      const bool rl = lane < nrows;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const int c = 16 * b + jj;
        const bool in = rl && c < k;
        const int64_t o = in ? (row0 + lane) * k + c : 0;
        float v = in ? R[o] : 0.f;
        if (!c_is_u && in) v += mu * C[o];
        qv[jj] = v;
      }
      // T of the block's coordinates from every other block
      const float* ga = gl[buf] + (lane & 15) * GS + (lane >> 4);
      f4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int sl = 4; sl < NQ; ++sl) {
        int q = 4 * b + sl;
        q = q >= NQ ? q - NQ : q;
        const float a = ga[4 * q];
        if (sl & 1)
          acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, u[sl], acc1, 0, 0, 0);
        else
          acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, u[sl], acc0, 0, 0, 0);
      }
      const f4 acc = acc0 + acc1;
      // lane (m, g) holds T[coordinate 4 g + i][row m]; the block's u in
      // slots 0..3 are coordinates 4 qq + g of row m
      float* T = tx[w];
      float* X = ux[w];
#pragma unroll
      for (int i = 0; i < 4; ++i) T[m * 17 + 4 * g + i] = acc[i];
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) X[m * 17 + 4 * qq + g] = u[qq];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (lane < 16) {
        float tt[16], uu[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
          tt[jj] = T[lane * 17 + jj];
          uu[jj] = X[lane * 17 + jj];
        }
        const float* gb = gl[buf] + 16 * b;   // row jj of the block at gb + jj * GS
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
          float t0 = tt[jj], t1 = 0.f;
#pragma unroll
          for (int ll = 0; ll < 16; ++ll) {
            if (ll == jj) continue;
            const float gv = gb[jj * GS + ll];
            if (ll & 1)
              t1 += gv * uu[ll];
            else
              t0 += gv * uu[ll];
          }
          const float q = c_is_u ? qv[jj] + mu * uu[jj] : qv[jj];
          const float x = (q - (t0 + t1)) * sinv[16 * b + jj];
          wguard(gd, x);
          uu[jj] = fminf(fmaxf(x, 0.f), ubnd);
        }
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) X[lane * 17 + jj] = uu[jj];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      float nb[4];
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) nb[qq] = X[m * 17 + 4 * qq + g];
      // rotate: block b + 1 into slots 0..3, block b's new values last
#pragma unroll
      for (int sl = 0; sl + 4 < NQ; ++sl) u[sl] = u[sl + 4];
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) u[NQ - 4 + qq] = nb[qq];
      if (more) store_g(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  const unsigned long long badm = __ballot(gd != gd);
  const bool bad = (badm >> m) & 1ull;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int c = 4 * q + g;
    if (m < nrows && c < k) U[(row0 + m) * k + c] = bad ? __builtin_nanf("") : u[q];
  }
  if (lane < nrows && sweeps_used != nullptr) sweeps_used[row0 + lane] = sweeps;
}

}  // namespace

int nnls_kc_wide(int k) {
  static const int sizes[] = {208, 256, 384, 512};
  for (int kc : sizes)
    if (k <= kc) return kc;
  return 0;
}

dsanls_status launch_prox_cd_wide(const float* gp, const float* inv, int KC, const float* R, const float* C, float* U,
                                  int64_t rows, int k, float mu, int sweeps, float upper, int32_t* sweeps_used,
                                  hipStream_t s) {
  if (rows == 0) return DSANLS_OK;
  if ((reinterpret_cast<uintptr_t>(gp) & 15) != 0)
    return fail(DSANLS_E_WORKSPACE, "NNLS workspace must be 16-byte aligned");
  const unsigned grid = static_cast<unsigned>(ceil_div(rows, 64));
  switch (KC) {
#define DSANLS_WIDE(KCV)                                                                                   \
  case KCV:                                                                                                \
    prox_cd_wide_kernel<KCV / 16><<<grid, 256, 0, s>>>(gp, inv, R, C, U, rows, k, mu, sweeps, upper,       \
                                                        sweeps_used);                                      \
    DSANLS_LAUNCHED("prox_cd_wide_kernel");                                                                \
    return DSANLS_OK;
    DSANLS_WIDE(208)
    DSANLS_WIDE(256)
    DSANLS_WIDE(384)
    DSANLS_WIDE(512)
#undef DSANLS_WIDE
  }
  return fail(DSANLS_E_UNSUPPORTED, "NNLS: no wide kernel for this rank");
}

}  // namespace dsanls
