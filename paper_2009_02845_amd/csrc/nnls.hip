// Batched row-wise NNLS updates of the sketched subproblem (Sec. 3.4).
//
// Every row i of U solves its own k-dimensional problem (the subproblem is
// row-independent, eq. u_block), all sharing G = B B^T.  Layout: one lane
// per row, the row's iterate u and q = r + mu c held in registers, and the
// Gram read as wave-uniform scalar operands: G is first copied into a padded
// KC x KC block (column j of G stored as row j) so that every G_lj in the
// fully unrolled coordinate loop has a compile-time offset and is fetched by
// scalar loads (s_load) instead of one LDS read per lane.  The k^2 FMAs of a
// row-sweep are then plain VALU work with no reductions; 64 rows per wave
// share every G value.
#include "common.hpp"

namespace dsanls {

namespace {

// Prepared Gram: gp[j * KC + l] = G[l][j] (zero outside k x k), den[j] =
// G_jj + mu, inv[j] = 1 / den[j] (zero in the padding), eta for PGD.
struct Prep {
  float* gp;
  float* den;
  float* inv;
  float* eta;
};

template <int KC>
size_t prep_bytes() {
  return sizeof(float) * (KC * KC + 3 * KC + 64);
}

template <int KC>
Prep carve_prep(void* ws) {
  float* p = static_cast<float*>(ws);
  return {p, p + KC * KC, p + KC * KC + KC, p + KC * KC + 2 * KC};
}

__global__ __launch_bounds__(256) void prep_kernel(const float* __restrict__ G, int k, int KC,
                                                   float mu, float* __restrict__ gp,
                                                   float* __restrict__ den,
                                                   float* __restrict__ inv,
                                                   float* __restrict__ eta) {
  __shared__ float colsum[256];
  for (int i = threadIdx.x; i < KC * KC; i += blockDim.x) {
    const int j = i / KC, l = i % KC;
    gp[i] = (j < k && l < k) ? G[l * k + j] : 0.f;
  }
  float best = 0.f;
  for (int j = threadIdx.x; j < KC; j += blockDim.x) {
    if (j < k) {
      const float dj = G[j * k + j] + mu;
      den[j] = dj;
      inv[j] = 1.0f / dj;
      float sabs = 0.f;
      for (int l = 0; l < k; ++l) sabs += fabsf(G[l * k + j]);
      best = fmaxf(best, sabs);
    } else {
      den[j] = 1.f;
      inv[j] = 0.f;
    }
  }
  colsum[threadIdx.x] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    float L = 0.f;
    for (int i = 0; i < 256; ++i) L = fmaxf(L, colsum[i]);
    // eta = 1 / (2 (L + mu)): at most the inverse Lipschitz constant of the
    // sketched gradient 2 (U G - R), shrinking as mu_t grows.
    eta[0] = 1.0f / (2.0f * (L + mu));
  }
}

template <int KC>
__device__ __forceinline__ void load_row(const float* __restrict__ P, int64_t row, int k,
                                         float (&x)[KC]) {
  const float* p = P + row * k;
#pragma unroll
  for (int l = 0; l < KC; ++l) x[l] = (l < k) ? p[l] : 0.f;
}

// sum_j u_j Q[j][l] - q_l for all l, then the relative projected-gradient
// norm of the row (zero exactly at the row's minimiser).
template <int KC>
__device__ __forceinline__ float kkt(const float* __restrict__ gp0, const float* __restrict__ den,
                                     const float (&u)[KC], const float (&q)[KC]) {
  float pg2 = 0.f, q2 = 0.f;
#pragma unroll
  for (int l = 0; l < KC; ++l) {
    const float* gp = gp0;
    float g0 = den[l] * u[l] - q[l], g1 = 0.f;
#pragma unroll
    for (int j = 0; j < KC; j += 2) {
      if (j != l) g0 += gp[l * KC + j] * u[j];
      if (j + 1 < KC && j + 1 != l) g1 += gp[l * KC + j + 1] * u[j + 1];
    }
    float g = g0 + g1;
    if (!(u[l] > 0.f)) g = fminf(g, 0.f);
    pg2 += g * g;
    q2 += q[l] * q[l];
  }
  return sqrtf(pg2) / fmaxf(sqrtf(q2), 1e-30f);
}

// One Gauss-Seidel sweep over the coordinates (Alg. 3 / eq. entry_sol):
// u_j <- max((q_j - sum_{l != j} G_lj u_l) / (G_jj + mu), 0), j ascending,
// with u_l already updated for l < j.
template <int KC>
__device__ __forceinline__ void sweep(const float* __restrict__ gp0, const float* __restrict__ inv,
                                      float upper, float (&u)[KC], const float (&q)[KC]) {
#pragma unroll
  for (int j = 0; j < KC; ++j) {
    const float* gp = gp0;
    float t0 = q[j], t1 = 0.f;
#pragma unroll
    for (int l = 0; l < KC; l += 2) {
      if (l != j) t0 -= gp[j * KC + l] * u[l];
      if (l + 1 < KC && l + 1 != j) t1 -= gp[j * KC + l + 1] * u[l + 1];
    }
    float v = fmaxf((t0 + t1) * inv[j], 0.f);
    if (upper > 0.f) v = fminf(v, upper);
    u[j] = v;
  }
}

template <int KC, bool TO_TOL>
__global__ __launch_bounds__(64) void prox_cd_kernel(const float* __restrict__ gp,
                                                     const float* __restrict__ den,
                                                     const float* __restrict__ inv,
                                                     const float* __restrict__ R,
                                                     const float* __restrict__ C,
                                                     float* __restrict__ U, int64_t rows, int k,
                                                     float mu, int sweeps, float tol,
                                                     int max_sweeps, float upper,
                                                     int32_t* __restrict__ sweeps_used,
                                                     unsigned long long* __restrict__ counters,
                                                     int zero) {
  // The Gram is read at gp + sweep * zero (zero is 0 at run time): G is
  // invariant across sweeps, and without the opaque offset the compiler
  // hoists all k^2 scalar loads out of the sweep loop and spills SGPRs.
  const int64_t row = blockIdx.x * 64ll + threadIdx.x;
  const bool valid = row < rows;
  float u[KC], q[KC];
  if (valid) {
    float c[KC];
    load_row<KC>(U, row, k, u);
    load_row<KC>(C, row, k, c);
    load_row<KC>(R, row, k, q);
#pragma unroll
    for (int l = 0; l < KC; ++l) q[l] += mu * c[l];
  } else {
#pragma unroll
    for (int l = 0; l < KC; ++l) u[l] = q[l] = 0.f;
  }
  int used = 0;
  bool unconverged = false;
  if (valid) {
    if (!TO_TOL) {
      for (int s = 0; s < sweeps; ++s) sweep<KC>(gp + s * zero, inv, upper, u, q);
      used = sweeps;
    } else {
      bool active = kkt<KC>(gp, den, u, q) > tol;
      while (active && used < max_sweeps) {
        sweep<KC>(gp + (2 * used + 1) * zero, inv, upper, u, q);
        ++used;
        active = kkt<KC>(gp + (2 * used) * zero, den, u, q) > tol;
      }
      unconverged = active;
    }
    float* p = U + row * k;
#pragma unroll
    for (int l = 0; l < KC; ++l)
      if (l < k) p[l] = u[l];
    if (sweeps_used != nullptr) sweeps_used[row] = used;
  }
  if (counters != nullptr) {
    // wave totals, one integer atomic per wave (exact, order-free)
    unsigned long long a = static_cast<unsigned long long>(used);
    unsigned long long b = unconverged ? 1ull : 0ull;
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_down(a, off, 64);
      b += __shfl_down(b, off, 64);
    }
    if (threadIdx.x == 0) {
      atomicAdd(&counters[0], a);
      atomicAdd(&counters[1], b);
    }
  }
}

// One projected-gradient step (eq. gradient_descent), all coordinates from
// the old iterate: u_j <- max(u_j - 2 eta ((u G)_j - r_j), 0).
template <int KC>
__global__ __launch_bounds__(64) void pgd_kernel(const float* __restrict__ gp0,
                                                 const float* __restrict__ eta_p,
                                                 const float* __restrict__ R,
                                                 float* __restrict__ U, int64_t rows, int k,
                                                 float upper) {
  const int64_t row = blockIdx.x * 64ll + threadIdx.x;
  if (row >= rows) return;
  float u[KC], r[KC];
  load_row<KC>(U, row, k, u);
  load_row<KC>(R, row, k, r);
  const float two_eta = 2.0f * eta_p[0];
  float* p = U + row * k;
#pragma unroll
  for (int j = 0; j < KC; ++j) {
    const float* gp = gp0;
    float g0 = -r[j], g1 = 0.f;
#pragma unroll
    for (int l = 0; l < KC; l += 2) {
      g0 += gp[j * KC + l] * u[l];
      if (l + 1 < KC) g1 += gp[j * KC + l + 1] * u[l + 1];
    }
    float v = fmaxf(u[j] - two_eta * (g0 + g1), 0.f);
    if (upper > 0.f) v = fminf(v, upper);
    if (j < k) p[j] = v;
  }
}

template <int KC>
dsanls_status run_kc(bool pgd, const float* G, const float* R, const float* C, float* U,
                     int64_t rows, int k, float mu, int sweeps, float tol, int max_sweeps,
                     float upper, int32_t* sweeps_used, unsigned long long* counters, void* ws,
                     hipStream_t s) {
  Prep p = carve_prep<KC>(ws);
  prep_kernel<<<1, 256, 0, s>>>(G, k, KC, mu, p.gp, p.den, p.inv, p.eta);
  DSANLS_LAUNCHED("prep_kernel");
  if (rows == 0) return DSANLS_OK;
  const unsigned grid = static_cast<unsigned>(ceil_div(rows, 64));
  if (pgd) {
    pgd_kernel<KC><<<grid, 64, 0, s>>>(p.gp, p.eta, R, U, rows, k, upper);
    DSANLS_LAUNCHED("pgd_kernel");
  } else {
    if (sweeps > 0)
      prox_cd_kernel<KC, false><<<grid, 64, 0, s>>>(p.gp, p.den, p.inv, R, C, U, rows, k, mu, sweeps,
                                                    tol, max_sweeps, upper, sweeps_used, counters, 0);
    else
      prox_cd_kernel<KC, true><<<grid, 64, 0, s>>>(p.gp, p.den, p.inv, R, C, U, rows, k, mu, sweeps,
                                                   tol, max_sweeps, upper, sweeps_used, counters, 0);
    DSANLS_LAUNCHED("prox_cd_kernel");
  }
  return DSANLS_OK;
}

}  // namespace

// Largest k handled by the NNLS kernels.
constexpr int kMaxK = 128;

int nnls_kc(int k) {
  if (k <= 8) return 8;
  if (k <= 16) return 16;
  if (k <= 32) return 32;
  if (k <= 64) return 64;
  if (k <= 100) return 100;
  return 128;
}

size_t nnls_ws_bytes(int k) {
  switch (nnls_kc(k)) {
    case 8: return prep_bytes<8>();
    case 16: return prep_bytes<16>();
    case 32: return prep_bytes<32>();
    case 64: return prep_bytes<64>();
    case 100: return prep_bytes<100>();
    default: return prep_bytes<128>();
  }
}

dsanls_status launch_nnls(bool pgd, const float* G, const float* R, const float* C, float* U,
                          int64_t rows, int k, float mu, int sweeps, float tol, int max_sweeps,
                          float upper, int32_t* sweeps_used, unsigned long long* counters,
                          void* ws, size_t ws_bytes, hipStream_t s) {
  if (k < 1 || k > kMaxK) return fail(DSANLS_E_UNSUPPORTED, "NNLS supports 1 <= k <= 128");
  if (ws_bytes < nnls_ws_bytes(k)) return fail(DSANLS_E_WORKSPACE, "NNLS workspace too small");
  switch (nnls_kc(k)) {
#define DSANLS_KC(KC)                                                                          \
  case KC:                                                                                     \
    return run_kc<KC>(pgd, G, R, C, U, rows, k, mu, sweeps, tol, max_sweeps, upper, sweeps_used, \
                      counters, ws, s);
    DSANLS_KC(8)
    DSANLS_KC(16)
    DSANLS_KC(32)
    DSANLS_KC(64)
    DSANLS_KC(100)
    DSANLS_KC(128)
#undef DSANLS_KC
  }
  return fail(DSANLS_E_UNSUPPORTED, "NNLS: no kernel for this k");
}

}  // namespace dsanls

using namespace dsanls;

extern "C" size_t dsanls_nnls_workspace_bytes(int32_t k) {
  return k < 1 || k > kMaxK ? 0 : align_up(nnls_ws_bytes(k), 256);
}

extern "C" dsanls_status dsanls_nnls_prox_cd(const float* G, const float* R, const float* C,
                                             float* U, int64_t rows, int32_t k, float mu,
                                             int32_t sweeps, float tol, int32_t max_sweeps,
                                             float upper, int32_t* sweeps_used, void* workspace,
                                             size_t workspace_bytes, void* hip_stream) {
  if (rows < 0 || !G || (rows > 0 && (!R || !C || !U)) || !workspace)
    return fail(DSANLS_E_INVALID_ARG, "nnls_prox_cd: null pointer or negative rows");
  if (sweeps < 0 || (sweeps == 0 && (max_sweeps < 1 || !(tol >= 0.f))) || !(mu >= 0.f))
    return fail(DSANLS_E_INVALID_ARG, "nnls_prox_cd: bad sweeps/tol/mu");
  return launch_nnls(false, G, R, C, U, rows, k, mu, sweeps, tol, max_sweeps, upper, sweeps_used,
                     nullptr, workspace, workspace_bytes, static_cast<hipStream_t>(hip_stream));
}

extern "C" dsanls_status dsanls_pgd_step(const float* G, const float* R, float* U, int64_t rows,
                                         int32_t k, float mu, float upper, void* workspace,
                                         size_t workspace_bytes, void* hip_stream) {
  if (rows < 0 || !G || (rows > 0 && (!R || !U)) || !workspace || !(mu >= 0.f))
    return fail(DSANLS_E_INVALID_ARG, "pgd_step: bad arguments");
  return launch_nnls(true, G, R, nullptr, U, rows, k, mu, 1, 0.f, 1, upper, nullptr, nullptr,
                     workspace, workspace_bytes, static_cast<hipStream_t>(hip_stream));
}
