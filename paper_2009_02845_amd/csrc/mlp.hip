// Warm-start network for the to-tolerance NNLS solves: forward, backward
// and Adam, all on the GPU.
//
//   h = ReLU(a W1a + W1u u + b1),  y = ReLU(W2 h + b2)
//
// a is the sketched row (sparse CSR for a subsampling sketch), u the
// current factor row.  The residual variant adds u to the output
// pre-activation, y = ReLU(u + W2 h + b2), so that its second layer
// predicts a correction to u (the cold start of the NNLS solve).  Parameters are one packed FP32 vector:
//   W1a (d x H, row c = weights of input column c) | W1u (H x k) | b1 (H)
//   | W2 (k x H) | b2 (k)
// The dense layers run on the FP32 MFMA GEMM (C = X Y^T); the sparse part
// of layer 1 gathers rows of W1a (one wave per batch row, lanes over H);
// its weight gradient is a deterministic gather over the batch's CSC form.
#include "common.hpp"

namespace dsanls {

namespace {

// ReLU that propagates NaN (like the definition max(x, 0) evaluated in IEEE
// arithmetic by the reference), so a broken network is detected downstream.
__device__ __forceinline__ float relu(float x) { return x > 0.f || x != x ? x : 0.f; }

__device__ __forceinline__ void neumaier(float& s, float& c, float x) {
  const float t = s + x;
  c += fabsf(s) >= fabsf(x) ? (s - t) + x : (x - t) + s;
  s = t;
}

struct Params {
  const float* W1a;
  const float* W1u;
  const float* b1;
  const float* W2;
  const float* b2;
};

struct Grads {
  float* W1a;
  float* W1u;
  float* b1;
  float* W2;
  float* b2;
};

template <typename P, typename T>
P split(T* base, int d, int k, int h) {
  T* p = base;
  T* W1a = p;
  p += static_cast<int64_t>(d) * h;
  T* W1u = p;
  p += static_cast<int64_t>(h) * k;
  T* b1 = p;
  p += h;
  T* W2 = p;
  p += static_cast<int64_t>(k) * h;
  T* b2 = p;
  return P{W1a, W1u, b1, W2, b2};
}

// H[b, :] = ReLU(H[b, :] + sum_e val_e W1a[col_e, :] + b1), H holding
// u_b W1u^T on entry.  One wave per four batch rows (sketched rows hold a
// few entries each, so a wave per row spent its time waiting on three
// dependent loads): the four rows' H values and their entries (one range,
// 64 at a time, one per lane, walked through shuffles) are read together,
// each entry adding to the accumulators of its row, each lane holding the
// hidden units h = lane + 64 q (hd <= 256; larger widths take one row and
// one segment at a time).  Every sum runs in the row's entry order.
constexpr int kL1Rows = 4;
__global__ __launch_bounds__(256) void l1_sparse_kernel(const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ cols,
                                                        const float* __restrict__ vals,
                                                        const float* __restrict__ W1a,
                                                        const float* __restrict__ b1,
                                                        float* __restrict__ H, int64_t rows,
                                                        int hd) {
  const int64_t r0 = (blockIdx.x * 4ll + (threadIdx.x >> 6)) * kL1Rows;
  const int lane = threadIdx.x & 63;
  if (r0 >= rows) return;
  const int nr = rows - r0 < kL1Rows ? static_cast<int>(rows - r0) : kL1Rows;
  if (hd <= 256) {
    // row boundaries; past the last row they repeat its end
    int rp[kL1Rows + 1];
#pragma unroll
    for (int i = 0; i <= kL1Rows; ++i) rp[i] = rowptr[r0 + (i < nr ? i : nr)];
    float acc[kL1Rows][4];
#pragma unroll
    for (int rr = 0; rr < kL1Rows; ++rr)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        acc[rr][q] = rr < nr && lane + 64 * q < hd ? H[(r0 + rr) * hd + lane + 64 * q] : 0.f;
    for (int e0 = rp[0]; e0 < rp[kL1Rows]; e0 += 64) {
      const int cnt = rp[kL1Rows] - e0 < 64 ? rp[kL1Rows] - e0 : 64;
      int c = 0;
      float v = 0.f;
      if (lane < cnt) {
        c = cols[e0 + lane];
        v = vals[e0 + lane];
      }
      for (int i = 0; i < cnt; ++i) {
        const int e = e0 + i;
        const float* w = W1a + static_cast<int64_t>(__shfl(c, i, 64)) * hd;
        const float vi = __shfl(v, i, 64);
        float x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = lane + 64 * q < hd ? w[lane + 64 * q] : 0.f;
        // the entry's row (wave-uniform)
        const int rr = (e >= rp[1]) + (e >= rp[2]) + (e >= rp[3]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (rr == 0)
            acc[0][q] += vi * x[q];
          else if (rr == 1)
            acc[1][q] += vi * x[q];
          else if (rr == 2)
            acc[2][q] += vi * x[q];
          else
            acc[3][q] += vi * x[q];
        }
      }
    }
#pragma unroll
    for (int rr = 0; rr < kL1Rows; ++rr)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (rr < nr && lane + 64 * q < hd)
          H[(r0 + rr) * hd + lane + 64 * q] = relu(acc[rr][q] + b1[lane + 64 * q]);
    return;
  }
  for (int rr = 0; rr < nr; ++rr) {
    const int64_t r = r0 + rr;
    const int beg = rowptr[r], end = rowptr[r + 1];
    for (int h = lane; h < hd; h += 64) {
      float acc = H[r * hd + h];
      for (int e = beg; e < end; ++e) acc += vals[e] * W1a[static_cast<int64_t>(cols[e]) * hd + h];
      H[r * hd + h] = relu(acc + b1[h]);
    }
  }
}

// X = ReLU(X + b), or ReLU(R + X + b) with the residual input R (not null).
__global__ __launch_bounds__(256) void bias_relu_kernel(float* __restrict__ X,
                                                        const float* __restrict__ b,
                                                        const float* __restrict__ R, int64_t rows,
                                                        int cols) {
  const int64_t n = rows * cols;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    X[i] = relu((R != nullptr ? R[i] : 0.f) + X[i] + b[i % cols]);
}

// dY = (2/B) (Yhat - Y) [Yhat > 0]; per-block compensated partial sums of
// (Yhat - Y)^2 / B for the loss.
__global__ __launch_bounds__(256) void mse_grad_kernel(const float* __restrict__ Yhat,
                                                       const float* __restrict__ Y,
                                                       float* __restrict__ dY, int64_t n,
                                                       float scale, float inv_rows,
                                                       float* __restrict__ partials) {
  __shared__ float red[2 * 4];
  float s = 0.f, c = 0.f;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float e = Yhat[i] - Y[i];
    neumaier(s, c, e * e * inv_rows);
    dY[i] = Yhat[i] > 0.f ? scale * e : 0.f;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) {
    const float os = __shfl_down(s, o, 64), oc = __shfl_down(c, o, 64);
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
    partials[2 * blockIdx.x] = ts;
    partials[2 * blockIdx.x + 1] = tc;
  }
}

__global__ __launch_bounds__(256) void relu_mask_kernel(float* __restrict__ dH,
                                                        const float* __restrict__ H, int64_t n) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    if (!(H[i] > 0.f)) dH[i] = 0.f;
}

// out[c] = sum_r X[r, c] for X (rows x cols): one wave per column, lanes
// over rows, fixed-order tree.
__global__ __launch_bounds__(256) void colsum_kernel(const float* __restrict__ X, int64_t rows,
                                                     int cols, float* __restrict__ out) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= cols) return;
  float s = 0.f, comp = 0.f;
  for (int64_t r = lane; r < rows; r += 64) neumaier(s, comp, X[r * cols + c]);
  for (int o = 32; o > 0; o >>= 1) {
    const float os = __shfl_down(s, o, 64), oc = __shfl_down(comp, o, 64);
    neumaier(s, comp, os);
    comp += oc;
  }
  if (lane == 0) out[c] = s + comp;
}

// dW1a[c, :] = sum_{e in column c} val_e dH[row_e, :] over the batch's CSC
// form: one wave per input column, lanes over the hidden units.
__global__ __launch_bounds__(256) void csc_grad_kernel(const int32_t* __restrict__ colptr,
                                                       const int32_t* __restrict__ rowidx,
                                                       const float* __restrict__ vals,
                                                       const float* __restrict__ dH, int hd, int d,
                                                       float* __restrict__ dW1a) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= d) return;
  const int beg = colptr[c], end = colptr[c + 1];
  for (int h = lane; h < hd; h += 64) {
    float acc = 0.f;
    for (int e = beg; e < end; ++e) acc += vals[e] * dH[static_cast<int64_t>(rowidx[e]) * hd + h];
    dW1a[static_cast<int64_t>(c) * hd + h] = acc;
  }
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   int64_t n, float lr, float beta1, float beta2,
                                                   float eps, float bc1, float bc2) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

unsigned grid_of(int64_t n) {
  int64_t g = ceil_div(n, 256 * 4);
  return static_cast<unsigned>(g < 1 ? 1 : (g > 65535 ? 65535 : g));
}

constexpr int kLossBlocks = 256;

struct MlpWs {
  float* H;      // B x hd
  float* Y;      // B x k (layer-2 output)
  float* dY;     // B x k
  float* dYt;    // k x B
  float* Ht;     // hd x B
  float* W2t;    // hd x k
  float* dH;     // B x hd
  float* dHt;    // hd x B
  float* Ut;     // k x B
  float* partials;
  void* gemm_ws;
  size_t gemm_ws_bytes;
  size_t total;
};

MlpWs carve(void* base, int d, int k, int hd, int64_t B, bool forward_only = false) {
  MlpWs w{};
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? static_cast<char*>(base) + off : nullptr;
    off = align_up(off + bytes, 256);
    return p;
  };
  auto f = [&](int64_t n) { return reinterpret_cast<float*>(take(sizeof(float) * n)); };
  w.H = f(B * hd);
  w.Y = f(B * k);
  if (forward_only) {
    w.gemm_ws_bytes = std::max(gemm_ws_bytes(B, hd, k), gemm_ws_bytes(B, k, hd));
    w.gemm_ws = w.gemm_ws_bytes ? take(w.gemm_ws_bytes) : nullptr;
    w.total = off;
    return w;
  }
  w.dY = f(B * k);
  w.dYt = f(k * B);
  w.Ht = f(hd * B);
  w.W2t = f(static_cast<int64_t>(hd) * k);
  w.dH = f(B * hd);
  w.dHt = f(hd * B);
  w.Ut = f(k * B);
  w.partials = f(2 * kLossBlocks + 8);
  size_t g = 0;
  g = std::max(g, gemm_ws_bytes(B, hd, k));
  g = std::max(g, gemm_ws_bytes(B, k, hd));
  g = std::max(g, gemm_ws_bytes(k, hd, B));
  g = std::max(g, gemm_ws_bytes(B, hd, k));
  g = std::max(g, gemm_ws_bytes(hd, k, B));
  w.gemm_ws_bytes = g;
  w.gemm_ws = g ? take(g) : nullptr;
  w.total = off;
  (void)d;
  return w;
}

}  // namespace

int64_t mlp_param_count(int d, int k, int hd) {
  return static_cast<int64_t>(d) * hd + static_cast<int64_t>(hd) * k + hd +
         static_cast<int64_t>(k) * hd + k;
}

size_t mlp_ws_bytes(int d, int k, int hd, int64_t rows, bool forward_only) {
  return carve(nullptr, d, k, hd, rows, forward_only).total;
}

// Forward pass: out (rows x k) = network(a, u).  H (rows x hd) is left in
// the workspace for the backward pass.
dsanls_status mlp_forward(int d, int k, int hd, bool residual, const float* params, int64_t rows,
                          const int32_t* a_rowptr, const int32_t* a_cols, const float* a_vals,
                          const float* U, float* out, void* ws, size_t ws_bytes, hipStream_t s) {
  MlpWs w = carve(ws, d, k, hd, rows, /*forward_only=*/true);
  if (ws_bytes < w.total) return fail(DSANLS_E_WORKSPACE, "mlp: workspace too small");
  if (rows == 0) return DSANLS_OK;
  const Params p = split<Params>(params, d, k, hd);
  dsanls_status st;
  // layer 1: H = U W1u^T (MFMA), then + sparse a W1a + b1, ReLU
  if ((st = launch_gemm_nt(U, k, p.W1u, k, w.H, hd, rows, hd, k, w.gemm_ws, w.gemm_ws_bytes, s)) != DSANLS_OK)
    return st;
  l1_sparse_kernel<<<static_cast<unsigned>(ceil_div(rows, 4 * kL1Rows)), 256, 0, s>>>(a_rowptr, a_cols, a_vals, p.W1a,
                                                                            p.b1, w.H, rows, hd);
  DSANLS_LAUNCHED("l1_sparse_kernel");
  // layer 2: out = ReLU(H W2^T + b2) (+ U in the residual variant)
  if ((st = launch_gemm_nt(w.H, hd, p.W2, hd, out, k, rows, k, hd, w.gemm_ws, w.gemm_ws_bytes, s)) != DSANLS_OK)
    return st;
  bias_relu_kernel<<<grid_of(rows * k), 256, 0, s>>>(out, p.b2, residual ? U : nullptr, rows, k);
  DSANLS_LAUNCHED("bias_relu_kernel");
  return DSANLS_OK;
}

// Gradients of L = (1/B) sum_b ||yhat_b - y_b||^2; loss_out[0..1] gets the
// loss before any update as a (hi, lo) pair.
dsanls_status mlp_gradients(int d, int k, int hd, bool residual, const float* params, float* grads, int64_t rows,
                            const int32_t* a_rowptr, const int32_t* a_cols, const float* a_vals,
                            const int32_t* c_colptr, const int32_t* c_rows, const float* c_vals,
                            const float* U, const float* Ylab, float* loss_out, void* ws,
                            size_t ws_bytes, int* err_flag, hipStream_t s) {
  MlpWs w = carve(ws, d, k, hd, rows);
  if (ws_bytes < w.total) return fail(DSANLS_E_WORKSPACE, "mlp: workspace too small");
  if (rows < 1) return fail(DSANLS_E_SHAPE, "mlp: empty batch");
  dsanls_status st;
  // H and Y sit at the same offsets in the forward-only layout; its GEMM
  // scratch overlaps dY and later buffers, which are written only after the
  // forward pass has finished on this stream.
  if ((st = mlp_forward(d, k, hd, residual, params, rows, a_rowptr, a_cols, a_vals, U, w.Y, ws, ws_bytes, s)) !=
      DSANLS_OK)
    return st;
  const Params p = split<Params>(params, d, k, hd);
  const Grads g = split<Grads>(grads, d, k, hd);
  const int64_t nY = rows * k;
  mse_grad_kernel<<<kLossBlocks, 256, 0, s>>>(w.Y, Ylab, w.dY, nY, 2.0f / static_cast<float>(rows),
                                              1.0f / static_cast<float>(rows), w.partials);
  DSANLS_LAUNCHED("mse_grad_kernel");
  int* flag = err_flag ? err_flag : reinterpret_cast<int*>(w.partials + 2 * kLossBlocks);
  if ((st = launch_combine_partials(w.partials, kLossBlocks, 2, loss_out, flag, s)) != DSANLS_OK) return st;
  // dW2 = dY^T H  (k x hd), db2 = column sums of dY
  if ((st = launch_transpose(w.dY, k, w.dYt, rows, rows, k, s)) != DSANLS_OK) return st;
  if ((st = launch_transpose(w.H, hd, w.Ht, rows, rows, hd, s)) != DSANLS_OK) return st;
  if ((st = launch_gemm_nt(w.dYt, rows, w.Ht, rows, g.W2, hd, k, hd, rows, w.gemm_ws, w.gemm_ws_bytes, s)) != DSANLS_OK)
    return st;
  colsum_kernel<<<static_cast<unsigned>(ceil_div(k, 4)), 256, 0, s>>>(w.dY, rows, k, g.b2);
  DSANLS_LAUNCHED("colsum_kernel");
  // dH = (dY W2) [H > 0]
  if ((st = launch_transpose(p.W2, hd, w.W2t, k, k, hd, s)) != DSANLS_OK) return st;
  if ((st = launch_gemm_nt(w.dY, k, w.W2t, k, w.dH, hd, rows, hd, k, w.gemm_ws, w.gemm_ws_bytes, s)) != DSANLS_OK)
    return st;
  relu_mask_kernel<<<grid_of(rows * hd), 256, 0, s>>>(w.dH, w.H, rows * hd);
  DSANLS_LAUNCHED("relu_mask_kernel");
  // dW1u = dH^T U  (hd x k), db1 = column sums of dH, dW1a from the CSC form
  if ((st = launch_transpose(w.dH, hd, w.dHt, rows, rows, hd, s)) != DSANLS_OK) return st;
  if ((st = launch_transpose(U, k, w.Ut, rows, rows, k, s)) != DSANLS_OK) return st;
  if ((st = launch_gemm_nt(w.dHt, rows, w.Ut, rows, g.W1u, k, hd, k, rows, w.gemm_ws, w.gemm_ws_bytes, s)) != DSANLS_OK)
    return st;
  colsum_kernel<<<static_cast<unsigned>(ceil_div(hd, 4)), 256, 0, s>>>(w.dH, rows, hd, g.b1);
  DSANLS_LAUNCHED("colsum_kernel");
  csc_grad_kernel<<<static_cast<unsigned>(ceil_div(d, 4)), 256, 0, s>>>(c_colptr, c_rows, c_vals, w.dH, hd, d,
                                                                        g.W1a);
  DSANLS_LAUNCHED("csc_grad_kernel");
  return DSANLS_OK;
}

dsanls_status mlp_adam(float* params, const float* grads, float* m, float* v, int64_t n, int64_t t,
                       float lr, hipStream_t s) {
  const double beta1 = 0.9, beta2 = 0.999;
  const float bc1 = static_cast<float>(1.0 - std::pow(beta1, static_cast<double>(t)));
  const float bc2 = static_cast<float>(1.0 - std::pow(beta2, static_cast<double>(t)));
  adam_kernel<<<grid_of(n), 256, 0, s>>>(params, grads, m, v, n, lr, static_cast<float>(beta1),
                                         static_cast<float>(beta2), 1e-8f, bc1, bc2);
  DSANLS_LAUNCHED("adam_kernel");
  return DSANLS_OK;
}

}  // namespace dsanls

using namespace dsanls;

extern "C" int64_t dsanls_mlp_param_count(int32_t d, int32_t k, int32_t hidden) {
  return (d < 1 || k < 1 || hidden < 1) ? 0 : mlp_param_count(d, k, hidden);
}

extern "C" size_t dsanls_mlp_workspace_bytes(int32_t d, int32_t k, int32_t hidden, int64_t rows) {
  return (d < 1 || k < 1 || hidden < 1 || rows < 0) ? 0 : mlp_ws_bytes(d, k, hidden, rows, false);
}

extern "C" dsanls_status dsanls_mlp_forward(int32_t d, int32_t k, int32_t hidden, int32_t residual,
                                            const float* params, int64_t rows, const int32_t* a_rowptr,
                                            const int32_t* a_cols, const float* a_vals,
                                            const float* U, float* out, void* workspace,
                                            size_t workspace_bytes, void* hip_stream) {
  if (d < 1 || k < 1 || hidden < 1 || rows < 0) return fail(DSANLS_E_SHAPE, "mlp_forward: bad sizes");
  if (rows > 0 && (!params || !a_rowptr || !U || !out || !workspace))
    return fail(DSANLS_E_INVALID_ARG, "mlp_forward: null pointer");
  return mlp_forward(d, k, hidden, residual != 0, params, rows, a_rowptr, a_cols, a_vals, U, out, workspace,
                     workspace_bytes, static_cast<hipStream_t>(hip_stream));
}

extern "C" dsanls_status dsanls_mlp_gradients(int32_t d, int32_t k, int32_t hidden, int32_t residual,
                                              const float* params, float* grads, int64_t rows,
                                              const int32_t* a_rowptr,
                                              const int32_t* a_cols, const float* a_vals,
                                              const int32_t* c_colptr, const int32_t* c_rows,
                                              const float* c_vals, const float* U, const float* Y,
                                              float* loss_out, void* workspace,
                                              size_t workspace_bytes, void* hip_stream) {
  if (d < 1 || k < 1 || hidden < 1 || rows < 1) return fail(DSANLS_E_SHAPE, "mlp_gradients: bad sizes");
  if (!params || !grads || !a_rowptr || !c_colptr || !U || !Y || !loss_out || !workspace)
    return fail(DSANLS_E_INVALID_ARG, "mlp_gradients: null pointer");
  return mlp_gradients(d, k, hidden, residual != 0, params, grads, rows, a_rowptr, a_cols, a_vals, c_colptr,
                       c_rows, c_vals, U, Y, loss_out, workspace, workspace_bytes, nullptr,
                       static_cast<hipStream_t>(hip_stream));
}

extern "C" dsanls_status dsanls_mlp_train_step(int32_t d, int32_t k, int32_t hidden, int32_t residual,
                                               float* params,
                                               float* grads, float* adam_m, float* adam_v,
                                               int64_t step, float lr, int64_t rows,
                                               const int32_t* a_rowptr, const int32_t* a_cols,
                                               const float* a_vals, const int32_t* c_colptr,
                                               const int32_t* c_rows, const float* c_vals,
                                               const float* U, const float* Y, float* loss_out,
                                               void* workspace, size_t workspace_bytes,
                                               void* hip_stream) {
  if (step < 1 || !(lr > 0.f)) return fail(DSANLS_E_INVALID_ARG, "mlp_train_step: step >= 1 and lr > 0");
  if (!adam_m || !adam_v) return fail(DSANLS_E_INVALID_ARG, "mlp_train_step: null Adam state");
  dsanls_status st = dsanls_mlp_gradients(d, k, hidden, residual, params, grads, rows, a_rowptr, a_cols, a_vals,
                                          c_colptr, c_rows, c_vals, U, Y, loss_out, workspace,
                                          workspace_bytes, hip_stream);
  if (st != DSANLS_OK) return st;
  return mlp_adam(params, grads, adam_m, adam_v, mlp_param_count(d, k, hidden), step, lr,
                  static_cast<hipStream_t>(hip_stream));
}
