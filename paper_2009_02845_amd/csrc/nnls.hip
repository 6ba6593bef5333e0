// Batched row-wise NNLS updates of the sketched subproblem (Sec. 3.4).
//
// Every row i of U solves its own k-dimensional problem (the subproblem is
// row-independent, eq. u_block), all sharing G = B B^T.  Layout: one lane
// per row, 64 rows per wave.  The row's iterate u lives in registers as
// W-wide vector blocks; the Gram is copied once into a padded KC x KC block
// (column j of G stored as row j, zero diagonal) so that coordinate j reads
// row j with wave-uniform scalar loads (s_load_dwordx16) and the k FMAs of
// its dot product take G as a scalar operand: 64 rows share every G value
// and no lane reads G through LDS.  The coordinate loop runs at run time
// inside each (statically unrolled) block, so the one dynamic register
// access per coordinate, u_j <- new value, is an indexed register move.
// The per-row right-hand side q_j = r_j + mu c_j is loaded per coordinate
// (the load is issued ahead of the dot product that hides it).
#include "common.hpp"

namespace dsanls {

namespace {

// Prepared Gram: gp[j * KC + l] = G[l][j] for l != j (zero on the diagonal
// and outside k x k); gdiag[j] = G_jj; den[j] = G_jj + mu; inv[j] =
// 1 / den[j] (zero in the padding); eta = PGD step.
struct Prep {
  float* gp;
  float* gdiag;
  float* den;
  float* inv;
  float* eta;
};

constexpr int kMaxKC = 128;

size_t prep_floats(int KC) { return static_cast<size_t>(KC) * KC + 4 * KC + 64; }

Prep carve_prep(void* ws, int KC) {
  float* p = static_cast<float*>(ws);
  return {p, p + KC * KC, p + KC * KC + KC, p + KC * KC + 2 * KC, p + KC * KC + 3 * KC};
}

__global__ __launch_bounds__(256) void prep_kernel(const float* __restrict__ G, int k, int KC,
                                                   float mu, float* __restrict__ gp,
                                                   float* __restrict__ gdiag,
                                                   float* __restrict__ den,
                                                   float* __restrict__ inv,
                                                   float* __restrict__ eta) {
  __shared__ float colsum[256];
  for (int i = threadIdx.x; i < KC * KC; i += blockDim.x) {
    const int j = i / KC, l = i % KC;
    gp[i] = (j < k && l < k && l != j) ? G[l * k + j] : 0.f;
  }
  float best = 0.f;
  for (int j = threadIdx.x; j < KC; j += blockDim.x) {
    if (j < k) {
      const float gj = G[j * k + j];
      const float dj = gj + mu;
      gdiag[j] = gj;
      den[j] = dj;
      // a zero denominator (G_jj = 0 and mu = 0) leaves the coordinate at 0
      inv[j] = dj != 0.f ? 1.0f / dj : 0.f;
      float sabs = 0.f;
      for (int l = 0; l < k; ++l) sabs += fabsf(G[l * k + j]);
      best = fmaxf(best, sabs);
    } else {
      gdiag[j] = 0.f;
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

template <int KC, int W>
struct RowBlocks {
  static constexpr int NB = (KC + W - 1) / W;
  typedef float vec __attribute__((ext_vector_type(W)));
  vec b[NB];
};

// sum_l g[l] * u_l over the padded row (static offsets: scalar loads).
template <int KC, int W>
__device__ __forceinline__ float dot_row(const float* __restrict__ g, const RowBlocks<KC, W>& u) {
  float t0 = 0.f, t1 = 0.f;
#pragma unroll
  for (int l = 0; l < KC; l += 2) {
    t0 += g[l] * u.b[l / W][l % W];
    if (l + 1 < KC) t1 += g[l + 1] * u.b[(l + 1) / W][(l + 1) % W];
  }
  return t0 + t1;
}

template <int KC, int W>
__device__ __forceinline__ void load_row(const float* __restrict__ P, int64_t row, int k, bool valid,
                                         RowBlocks<KC, W>& x) {
  const float* p = P + row * k;
#pragma unroll
  for (int l = 0; l < KC; ++l) x.b[l / W][l % W] = (valid && l < k) ? p[l] : 0.f;
}

// q_j = r_j + mu c_j for the W coordinates of block jb of this lane's row
// (zero in the padding), loaded once per block so that the per-coordinate
// access is a register read rather than a strided global load.
template <int KC, int W>
__device__ __forceinline__ typename RowBlocks<KC, W>::vec rhs_block(const float* __restrict__ R,
                                                                     const float* __restrict__ C,
                                                                     int64_t off, int jb, int k,
                                                                     float mu, bool valid) {
  typename RowBlocks<KC, W>::vec q;
#pragma unroll
  for (int e = 0; e < W; ++e) {
    const int j = jb * W + e;
    q[e] = (valid && j < k) ? R[off + j] + mu * C[off + j] : 0.f;
  }
  return q;
}

// One Gauss-Seidel sweep over the coordinates (Alg. 3 / eq. entry_sol):
// u_j <- max((q_j - sum_{l != j} G_lj u_l) / (G_jj + mu), 0), j ascending,
// with u_l already updated for l < j.
template <int KC, int W>
__device__ __forceinline__ void sweep(const float* __restrict__ gp, const float* __restrict__ inv,
                                      const float* __restrict__ R, const float* __restrict__ C,
                                      int64_t off, int k, float mu, bool valid, float upper,
                                      RowBlocks<KC, W>& u) {
  constexpr int NB = RowBlocks<KC, W>::NB;
#pragma unroll
  for (int jb = 0; jb < NB; ++jb) {
    const int jn = (jb + 1) * W <= KC ? W : KC - jb * W;
    const auto qb = rhs_block<KC, W>(R, C, off, jb, k, mu, valid);
#pragma nounroll
    for (int je = 0; je < jn; ++je) {
      const int j = jb * W + je;
      const float q = qb[je];
      const float t = dot_row<KC, W>(gp + j * KC, u);
      float v = fmaxf((q - t) * inv[j], 0.f);
      if (upper > 0.f) v = fminf(v, upper);
      u.b[jb][je] = v;
    }
  }
}

// Relative projected-gradient norm of the row problem
// min_{u >= 0} 1/2 u Q u^T - q u^T, Q = G + mu I: zero exactly at its
// minimiser.
template <int KC, int W>
__device__ __forceinline__ float kkt(const float* __restrict__ gp, const float* __restrict__ den,
                                     const float* __restrict__ R, const float* __restrict__ C,
                                     int64_t off, int k, float mu, bool valid,
                                     const RowBlocks<KC, W>& u) {
  constexpr int NB = RowBlocks<KC, W>::NB;
  float pg2 = 0.f, q2 = 0.f;
#pragma unroll
  for (int lb = 0; lb < NB; ++lb) {
    const int ln = (lb + 1) * W <= KC ? W : KC - lb * W;
    const auto qb = rhs_block<KC, W>(R, C, off, lb, k, mu, valid);
#pragma nounroll
    for (int le = 0; le < ln; ++le) {
      const int l = lb * W + le;
      const float q = qb[le];
      const float ul = u.b[lb][le];
      float g = dot_row<KC, W>(gp + l * KC, u) + den[l] * ul - q;
      if (!(ul > 0.f)) g = fminf(g, 0.f);
      if (l < k) {
        pg2 += g * g;
        q2 += q * q;
      }
    }
  }
  return sqrtf(pg2) / fmaxf(sqrtf(q2), 1e-30f);
}

template <int KC, int W, bool TO_TOL>
__global__ __launch_bounds__(64) void prox_cd_kernel(const float* __restrict__ gp,
                                                     const float* __restrict__ den,
                                                     const float* __restrict__ inv,
                                                     const float* __restrict__ R,
                                                     const float* C, const float* start, float* U,
                                                     int64_t rows, int k, float mu, int sweeps,
                                                     float tol, int max_sweeps, float upper,
                                                     int32_t* __restrict__ sweeps_used,
                                                     unsigned long long* __restrict__ counters) {
  // C (the proximal centre) may alias U: every lane reads its own row of C
  // before it writes that row of U, at the end.  start (to-tolerance mode
  // only) is a warm start; without it the solve starts from U.
  const int64_t row = blockIdx.x * 64ll + threadIdx.x;
  const bool valid = row < rows;
  const int64_t off = row * k;
  RowBlocks<KC, W> u;
  load_row<KC, W>(TO_TOL && start != nullptr ? start : U, row, k, valid, u);
  int used = 0;
  bool unconverged = false, fell_back = false;
  if (!TO_TOL) {
    for (int s = 0; s < sweeps; ++s) sweep<KC, W>(gp, inv, R, C, off, k, mu, valid, upper, u);
    used = sweeps;
  } else if (valid) {
    bool ok = true;
    if (start != nullptr) {
#pragma unroll
      for (int l = 0; l < KC; ++l) ok = ok && isfinite(u.b[l / W][l % W]);
    }
    bool active = ok && kkt<KC, W>(gp, den, R, C, off, k, mu, valid, u) > tol;
    while (active && used < max_sweeps) {
      sweep<KC, W>(gp, inv, R, C, off, k, mu, valid, upper, u);
      ++used;
      active = kkt<KC, W>(gp, den, R, C, off, k, mu, valid, u) > tol;
    }
    if (start != nullptr && (!ok || active)) {
      // the warm start failed: restart from the cold start, the centre U^t
      fell_back = true;
      load_row<KC, W>(C, row, k, valid, u);
      int cold = 0;
      active = kkt<KC, W>(gp, den, R, C, off, k, mu, valid, u) > tol;
      while (active && cold < max_sweeps) {
        sweep<KC, W>(gp, inv, R, C, off, k, mu, valid, upper, u);
        ++cold;
        active = kkt<KC, W>(gp, den, R, C, off, k, mu, valid, u) > tol;
      }
      used += cold;
    }
    unconverged = active;
  }
  if (valid) {
    float* p = U + off;
#pragma unroll
    for (int l = 0; l < KC; ++l)
      if (l < k) p[l] = u.b[l / W][l % W];
    if (sweeps_used != nullptr) sweeps_used[row] = used;
  } else {
    used = 0;
  }
  if (counters != nullptr) {
    // wave totals, one integer atomic per wave (exact, order-free)
    unsigned long long a = static_cast<unsigned long long>(used);
    unsigned long long b = unconverged ? 1ull : 0ull;
    unsigned long long f = fell_back ? 1ull : 0ull;
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_down(a, o, 64);
      b += __shfl_down(b, o, 64);
      f += __shfl_down(f, o, 64);
    }
    if (threadIdx.x == 0) {
      atomicAdd(&counters[0], a);
      atomicAdd(&counters[1], b);
      atomicAdd(&counters[2], f);
    }
  }
}

// One projected-gradient step (eq. gradient_descent), every coordinate from
// the old iterate: u_j <- max(u_j - 2 eta ((u G)_j - r_j), 0), written out
// as it is formed.
template <int KC, int W>
__global__ __launch_bounds__(64) void pgd_kernel(const float* __restrict__ gp,
                                                 const float* __restrict__ gdiag,
                                                 const float* __restrict__ eta_p,
                                                 const float* __restrict__ R, float* U,
                                                 int64_t rows, int k, float upper) {
  const int64_t row = blockIdx.x * 64ll + threadIdx.x;
  const bool valid = row < rows;
  const int64_t off = row * k;
  RowBlocks<KC, W> u;
  load_row<KC, W>(U, row, k, valid, u);
  const float two_eta = 2.0f * eta_p[0];
  constexpr int NB = RowBlocks<KC, W>::NB;
#pragma unroll
  for (int jb = 0; jb < NB; ++jb) {
    const int jn = (jb + 1) * W <= KC ? W : KC - jb * W;
#pragma nounroll
    for (int je = 0; je < jn; ++je) {
      const int j = jb * W + je;
      if (j >= k) break;
      const float uj = u.b[jb][je];
      const float r = valid ? R[off + j] : 0.f;
      const float g = dot_row<KC, W>(gp + j * KC, u) + gdiag[j] * uj - r;
      float v = fmaxf(uj - two_eta * g, 0.f);
      if (upper > 0.f) v = fminf(v, upper);
      if (valid) U[off + j] = v;
    }
  }
}

template <int KC, int W>
dsanls_status run_kc(bool pgd, const float* G, const float* R, const float* C, float* U,
                     int64_t rows, int k, float mu, int sweeps, float tol, int max_sweeps,
                     float upper, int32_t* sweeps_used, unsigned long long* counters, void* ws,
                     hipStream_t s, const float* start) {
  Prep p = carve_prep(ws, KC);
  prep_kernel<<<1, 256, 0, s>>>(G, k, KC, mu, p.gp, p.gdiag, p.den, p.inv, p.eta);
  DSANLS_LAUNCHED("prep_kernel");
  if (rows == 0) return DSANLS_OK;
  const unsigned grid = static_cast<unsigned>(ceil_div(rows, 64));
  if (pgd) {
    pgd_kernel<KC, W><<<grid, 64, 0, s>>>(p.gp, p.gdiag, p.eta, R, U, rows, k, upper);
    DSANLS_LAUNCHED("pgd_kernel");
  } else if (sweeps > 0) {
    prox_cd_kernel<KC, W, false><<<grid, 64, 0, s>>>(p.gp, p.den, p.inv, R, C, nullptr, U, rows, k, mu,
                                                     sweeps, tol, max_sweeps, upper, sweeps_used, counters);
    DSANLS_LAUNCHED("prox_cd_kernel");
  } else {
    prox_cd_kernel<KC, W, true><<<grid, 64, 0, s>>>(p.gp, p.den, p.inv, R, C, start, U, rows, k, mu,
                                                    sweeps, tol, max_sweeps, upper, sweeps_used, counters);
    DSANLS_LAUNCHED("prox_cd_kernel");
  }
  return DSANLS_OK;
}

// Padded size of the prepared Gram for rank k (exact for the ranks the
// workloads use, otherwise the next size up; the padding costs FMAs only).
int nnls_kc(int k) {
  static const int sizes[] = {4, 8, 10, 16, 32, 48, 64, 96, 100, 128};
  for (int kc : sizes)
    if (k <= kc) return kc;
  return 0;
}

}  // namespace

constexpr int kMaxK = 128;

size_t nnls_ws_bytes(int k) {
  const int kc = nnls_kc(k < 1 ? 1 : k);
  return sizeof(float) * prep_floats(kc > 0 ? kc : kMaxKC);
}

dsanls_status launch_nnls(bool pgd, const float* G, const float* R, const float* C, float* U,
                          int64_t rows, int k, float mu, int sweeps, float tol, int max_sweeps,
                          float upper, int32_t* sweeps_used, unsigned long long* counters,
                          void* ws, size_t ws_bytes, hipStream_t s, const float* start) {
  if (k < 1 || k > kMaxK) return fail(DSANLS_E_UNSUPPORTED, "NNLS supports 1 <= k <= 128");
  if (ws_bytes < nnls_ws_bytes(k)) return fail(DSANLS_E_WORKSPACE, "NNLS workspace too small");
  switch (nnls_kc(k)) {
#define DSANLS_KC(KC, W)                                                                             \
  case KC:                                                                                           \
    return run_kc<KC, W>(pgd, G, R, C, U, rows, k, mu, sweeps, tol, max_sweeps, upper, sweeps_used, \
                         counters, ws, s, start);
    DSANLS_KC(4, 4)
    DSANLS_KC(8, 8)
    DSANLS_KC(10, 16)
    DSANLS_KC(16, 16)
    DSANLS_KC(32, 32)
    DSANLS_KC(48, 16)
    DSANLS_KC(64, 32)
    DSANLS_KC(96, 32)
    DSANLS_KC(100, 32)
    DSANLS_KC(128, 32)
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
