// Host side of the C ABI: validation, workspace planning and the sequence
// of kernels of one half-iteration (Alg. 2 with N = 1).
#include "common.hpp"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

namespace dsanls {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

dsanls_status fail(dsanls_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

dsanls_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return DSANLS_E_HIP;
}

namespace {

// Largest rank: 512 (ranks above 128 take the wide NNLS kernel, fixed
// prox-CD sweeps only)
constexpr int64_t kMaxRank = kNnlsMaxRankWide;

int64_t r4(int64_t x) { return (x + 3) / 4 * 4; }
int64_t r8(int64_t x) { return (x + 7) / 8 * 8; }
// BF16 operands of the sketch product: rows padded with zeros to 32 bf16, so
// the product runs on the ring kernel with K rounded up to 32 (zeros add nothing)
int64_t r32(int64_t x) { return (x + 31) / 32 * 32; }

// Device buffers carved from the caller's workspace.
struct Layout {
  float* Mt = nullptr;              // n x ldmt, resident M^T (dense, when not supplied)
  int64_t ldmt = 0;
  // CSR(M^T) built at init when the caller passes CSR(M) alone
  int64_t* t_rowptr = nullptr;
  int32_t* t_colidx = nullptr;
  float* t_vals = nullptr;
  void* ct_ws = nullptr;
  size_t ct_ws_bytes = 0;
  __hip_bfloat16* Mb = nullptr;     // m x ldmb (BF16 copy of M)
  __hip_bfloat16* Mtb = nullptr;    // n x ldmtb
  int64_t ldmb = 0, ldmtb = 0;
  float* St[2] = {nullptr, nullptr};            // per side: d x lds, sketch transposed
  __hip_bfloat16* Sb[2] = {nullptr, nullptr};   // per side: d x ldsb (BF16 form)
  float* A[2] = {nullptr, nullptr};             // per side: rows x lda
  float* Wt = nullptr;              // k x ldw, fixed factor transposed
  float* B = nullptr;               // k x ldb
  float* G = nullptr;               // k x k
  float* Gobj = nullptr;            // 2 x k x k (objective Grams)
  float* R = nullptr;               // rows x k
  void* gemm_ws = nullptr;
  size_t gemm_ws_bytes = 0;
  void* nnls_ws = nullptr;
  size_t nnls_ws_bytes = 0;
  int32_t* idx[2] = {nullptr, nullptr};    // per side: subsample indices (d, global) ...
  int32_t* idx_win[2] = {nullptr, nullptr};  // ... the same seen by this block (-1: outside), shares only
  int32_t* slot[2] = {nullptr, nullptr};   // ... and slot map (lng); one set per side so that the
                                           // next side's selection can run ahead on the side stream
  // sketched rows of A (CSR input, subsampling): counts, offsets, entries
  // sketched rows of A, one set per side (the next side's gather can run
  // ahead on the side stream while this side's are still in use)
  int32_t* a_cnt[2] = {nullptr, nullptr};      // per-row or per-segment counts
  int32_t* a_pos[2] = {nullptr, nullptr};      // per-segment start positions / column offsets
  int32_t* long_rows[2] = {nullptr, nullptr};  // rows of A longer than a lane sorts
  int32_t* nlong[2] = {nullptr, nullptr};
  int32_t* a_rowptr[2] = {nullptr, nullptr};
  int32_t* a_cols[2] = {nullptr, nullptr};
  float* a_vals[2] = {nullptr, nullptr};
  int32_t* scan_ws[2] = {nullptr, nullptr};
  float* ustart = nullptr;          // warm start, rows x k
  // count sketch: per side the hash and bucket lists; At (d x rows, the
  // product before its transpose) and Bt (d x k) shared by the sides
  CountSketch cs[2];
  float* At = nullptr;
  int64_t ldat = 0;
  float* Bt = nullptr;
  // SRHT: per side the signs and the sampled Hadamard columns
  float* hsign[2] = {nullptr, nullptr};
  int32_t* hcol[2] = {nullptr, nullptr};
  int64_t hlen[2] = {0, 0};          // transform length N of each side
  // segment tables of CSR(M) (side 0) and CSR(M^T) (side 1), partial sums
  CsrSegments seg[2];
  int64_t seg_cap[2] = {0, 0}, multi_cap[2] = {0, 0};
  float* seg_partials = nullptr;
  void* mlp_ws = nullptr;
  size_t mlp_ws_bytes = 0;
  void* sub_ws[2] = {nullptr, nullptr};
  size_t sub_ws_bytes = 0;
  float* partials = nullptr;
  float* red = nullptr;             // 64 floats of small results
  int* err = nullptr;               // 16 ints of device flags
  unsigned long long* counters = nullptr;
  TolWork tol{};                    // to-tolerance passes (null pointers when unused)
  size_t total = 0;
};

bool dense(const dsanls_matrix* M) { return M->format == DSANLS_DENSE; }

// The whole matrix of which this context holds the block: m_global x
// n_global (0 means the block's own size), the block starting at
// (row_offset, col_offset).  Side 0's long dimension is the columns, side
// 1's the rows.
int64_t m_glob(const dsanls_config& c) { return c.m_global > 0 ? c.m_global : c.m; }
int64_t n_glob(const dsanls_config& c) { return c.n_global > 0 ? c.n_global : c.n; }
bool is_share(const dsanls_config& c) {
  return c.row_offset != 0 || c.col_offset != 0 || m_glob(c) != c.m || n_glob(c) != c.n;
}

Layout plan(const dsanls_config& c, const dsanls_matrix& M, char* base) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off = align_up(off + bytes, 256);
    return p;
  };
  const int64_t m = c.m, n = c.n, k = c.k;
  const int64_t lngmax = std::max(m, n), rowsmax = std::max(m, n), dmax = std::max(c.d, c.d_prime);
  const int64_t lngglob = std::max(m_glob(c), n_glob(c));
  const bool is_dense = dense(&M);
  const bool gauss = c.sketch == DSANLS_SKETCH_GAUSSIAN;
  const bool sub = c.sketch == DSANLS_SKETCH_SUBSAMPLE;
  const bool count = c.sketch == DSANLS_SKETCH_COUNT;
  const bool srht = c.sketch == DSANLS_SKETCH_SRHT;
  const bool bf16 = c.precision == DSANLS_PREC_BF16_SKETCH;
  if (is_dense && M.dense_t == nullptr) {
    L.ldmt = r4(m);
    L.Mt = reinterpret_cast<float*>(take(sizeof(float) * n * L.ldmt));
  }
  if (!is_dense && M.t_rowptr == nullptr) {
    const int64_t nnz = std::max<int64_t>(M.nnz, 1);
    L.t_rowptr = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * (n + 1)));
    L.t_colidx = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * nnz));
    L.t_vals = reinterpret_cast<float*>(take(sizeof(float) * nnz));
    L.ct_ws_bytes = csr_transpose_ws_bytes(n);
    L.ct_ws = take(L.ct_ws_bytes);
  }
  if (is_dense && bf16) {
    L.ldmb = r32(n);
    L.ldmtb = r32(m);
    L.Mb = reinterpret_cast<__hip_bfloat16*>(take(2 * m * L.ldmb));
    L.Mtb = reinterpret_cast<__hip_bfloat16*>(take(2 * n * L.ldmtb));
  }
  // Side 0 (U-subproblem): S is n x d, A is m x d; side 1: S' is m x d', A' is n x d'.
  const int64_t side_rows[2] = {m, n}, side_lng[2] = {n, m}, side_d[2] = {c.d, c.d_prime};
  for (int sd = 0; sd < 2; ++sd) {
    if (gauss) {
      L.St[sd] = reinterpret_cast<float*>(take(sizeof(float) * side_d[sd] * r4(side_lng[sd])));
      if (bf16) L.Sb[sd] = reinterpret_cast<__hip_bfloat16*>(take(2 * side_d[sd] * r32(side_lng[sd])));
    }
    if (is_dense && (gauss || sub || count || srht))
      L.A[sd] = reinterpret_cast<float*>(take(sizeof(float) * side_rows[sd] * r4(side_d[sd])));
    if (count) {
      const int64_t lng = side_lng[sd], dd = side_d[sd];
      CountSketch& q = L.cs[sd];
      q.bucket = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * lng));
      q.sign = reinterpret_cast<float*>(take(sizeof(float) * lng));
      q.cnt = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * 2 * (dd + 1)));
      q.off = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (dd + 1)));
      q.scan_ws = reinterpret_cast<int32_t*>(take(scan_ws_bytes(dd)));
      q.tmp = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * lng));
      q.list = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * lng));
    }
    if (srht) {
      L.hsign[sd] = reinterpret_cast<float*>(take(sizeof(float) * side_lng[sd]));
      L.hcol[sd] = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * side_d[sd]));
    }
  }
  if (count) {
    L.ldat = r4(rowsmax);
    if (is_dense) L.At = reinterpret_cast<float*>(take(sizeof(float) * dmax * L.ldat));
    L.Bt = reinterpret_cast<float*>(take(sizeof(float) * dmax * k));
  }
  if (srht) {
    L.hlen[0] = srht_length(n_glob(c));
    L.hlen[1] = srht_length(m_glob(c));
    L.sub_ws_bytes = subsample_ws_bytes(std::max(L.hlen[0], L.hlen[1]));
    for (int sd = 0; sd < 2; ++sd) L.sub_ws[sd] = take(L.sub_ws_bytes);
  }
  L.Wt = reinterpret_cast<float*>(take(sizeof(float) * k * r4(lngmax)));
  L.B = reinterpret_cast<float*>(take(sizeof(float) * k * r4(dmax)));
  L.G = reinterpret_cast<float*>(take(sizeof(float) * k * k));
  L.Gobj = reinterpret_cast<float*>(take(sizeof(float) * 2 * k * k));
  L.R = reinterpret_cast<float*>(take(sizeof(float) * rowsmax * k));
  size_t gws = 0;
  for (int side = 0; side < 2; ++side) {
    const int64_t rows = side == 0 ? m : n, lng = side == 0 ? n : m, d = side == 0 ? c.d : c.d_prime;
    const int64_t kdim = c.sketch == DSANLS_SKETCH_IDENTITY ? lng : d;
    gws = std::max(gws, gemm_ws_bytes(rows, d, lng));
    gws = std::max(gws, gemm_ws_bytes(k, d, lng));
    gws = std::max(gws, gemm_ws_bytes(rows, k, kdim));
  }
  L.gemm_ws_bytes = gws;
  L.gemm_ws = gws ? take(gws) : nullptr;
  L.nnls_ws_bytes = align_up(nnls_ws_bytes(static_cast<int>(std::min<int64_t>(k, kMaxRank))), 256);
  L.nnls_ws = take(L.nnls_ws_bytes);
  if (sub) {
    // the selection runs over the whole long dimension (global indices)
    L.sub_ws_bytes = subsample_ws_bytes(lngglob);
    for (int sd = 0; sd < 2; ++sd) {
      L.idx[sd] = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * dmax));
      if (is_share(c)) L.idx_win[sd] = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * dmax));
      L.slot[sd] = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * lngglob));
      L.sub_ws[sd] = take(L.sub_ws_bytes);
    }
  }
  if (!is_dense) {
    const int64_t nnz = std::max<int64_t>(M.nnz, 0);
    int64_t parts = 0;
    for (int sd = 0; sd < 2; ++sd) {
      const int64_t rows = sd == 0 ? m : n;
      L.seg_cap[sd] = csr_seg_bound(rows, nnz);
      L.multi_cap[sd] = nnz / kCsrSegment + 1;
      L.seg[sd].seg_row = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * L.seg_cap[sd]));
      L.seg[sd].seg_beg = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * L.seg_cap[sd]));
      L.seg[sd].seg_part = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * L.seg_cap[sd]));
      L.seg[sd].multi_row = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * L.multi_cap[sd]));
      L.seg[sd].multi_part = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (L.multi_cap[sd] + 1)));
      parts = std::max(parts, csr_part_bound(nnz));
    }
    L.seg_partials = reinterpret_cast<float*>(take(sizeof(float) * parts * k));
  }
  if (!is_dense && sub) {
    const int64_t cnt_len = std::max({rowsmax + 1, L.seg_cap[0] + 1, L.seg_cap[1] + 1});
    for (int sd = 0; sd < 2; ++sd) {
      L.a_cnt[sd] = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * cnt_len));
      L.a_pos[sd] = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * cnt_len));
      L.a_rowptr[sd] = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (rowsmax + 1)));
      L.a_cols[sd] = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * std::max<int64_t>(M.nnz, 1)));
      L.a_vals[sd] = reinterpret_cast<float*>(take(sizeof(float) * std::max<int64_t>(M.nnz, 1)));
      L.scan_ws[sd] = reinterpret_cast<int32_t*>(take(scan_ws_bytes(cnt_len)));
      L.long_rows[sd] = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * rowsmax));
      L.nlong[sd] = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * 4));
    }
    if (c.warm_hidden > 0) {
      L.ustart = reinterpret_cast<float*>(take(sizeof(float) * rowsmax * k));
      L.mlp_ws_bytes = mlp_ws_bytes(static_cast<int>(c.d), static_cast<int>(k), c.warm_hidden, rowsmax, true);
      L.mlp_ws = take(L.mlp_ws_bytes);
    }
  }
  int64_t np = std::max<int64_t>(sumsq_partials(is_dense ? m : 1, is_dense ? n : std::max<int64_t>(M.nnz, 1)),
                                 csr_cross_partials(m));
  if (is_dense) np = std::max(np, residual_partials(m, n));
  L.partials = reinterpret_cast<float*>(take(sizeof(float) * 4 * np));
  L.red = reinterpret_cast<float*>(take(sizeof(float) * 64));
  L.err = reinterpret_cast<int*>(take(sizeof(int) * 16));
  // (a sizing pass has no base: no pointer arithmetic on null)
  for (int sd = 0; sd < 2; ++sd) L.cs[sd].err = L.err != nullptr ? L.err + 1 : nullptr;
  L.counters = reinterpret_cast<unsigned long long*>(take(sizeof(unsigned long long) * 8));
  L.tol.counters = L.counters;
  if (c.solver == DSANLS_SOLVER_PROX_CD && c.sweeps == 0) {
    const int64_t nw = (rowsmax + 15) / 16;   // waves of 16 to 64 rows, 64 slots each
    L.tol.used = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * rowsmax));
    L.tol.flags = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * rowsmax));
    L.tol.wave_cnt = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * nw));
    L.tol.wave_off = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (nw + 1)));
    L.tol.wave_rows = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * nw * 64));
    L.tol.list[0] = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * rowsmax));
    L.tol.list[1] = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * rowsmax));
    L.tol.scan_ws = reinterpret_cast<int32_t*>(take(scan_ws_bytes(nw)));
    L.tol.centre = reinterpret_cast<float*>(take(sizeof(float) * rowsmax * k));
  }
  L.total = off;
  return L;
}

dsanls_status validate(const dsanls_config* c, const dsanls_matrix* M) {
  if (!c || !M) return fail(DSANLS_E_INVALID_ARG, "config or matrix is NULL");
  if (c->m < 1 || c->n < 1 || c->k < 1 || c->d < 1 || c->d_prime < 1)
    return fail(DSANLS_E_SHAPE, "m, n, k, d, d_prime must be >= 1");
  if (c->k > kMaxRank) return fail(DSANLS_E_UNSUPPORTED, "k > 512 is not supported");
  if (c->k > kNnlsMaxRank && !(c->solver == DSANLS_SOLVER_PROX_CD && c->sweeps >= 1))
    return fail(DSANLS_E_UNSUPPORTED, "ranks above 128 support prox-CD with a fixed number of sweeps only");
  if (c->k > kNnlsMaxRank && c->warm_hidden > 0)
    return fail(DSANLS_E_UNSUPPORTED, "the warm start supports ranks up to 128");
  if (c->m > INT32_MAX || c->n > INT32_MAX) return fail(DSANLS_E_SHAPE, "m and n must fit int32");
  if (c->sketch < 0 || c->sketch > 4) return fail(DSANLS_E_INVALID_ARG, "bad sketch kind");
  if (c->solver < 0 || c->solver > 1) return fail(DSANLS_E_INVALID_ARG, "bad solver");
  if (c->precision < 0 || c->precision > 1) return fail(DSANLS_E_INVALID_ARG, "bad precision");
  if (c->row_offset < 0 || c->col_offset < 0 || c->m_global < 0 || c->n_global < 0)
    return fail(DSANLS_E_SHAPE, "row_offset, col_offset, m_global and n_global must be >= 0");
  if (c->row_offset + c->m > m_glob(*c) || c->col_offset + c->n > n_glob(*c))
    return fail(DSANLS_E_SHAPE, "the block [row_offset, +m) x [col_offset, +n) must lie inside m_global x n_global");
  if (m_glob(*c) > INT32_MAX || n_glob(*c) > INT32_MAX) return fail(DSANLS_E_SHAPE, "m_global and n_global must fit int32");
  if (c->sketch == DSANLS_SKETCH_SUBSAMPLE && (c->d > n_glob(*c) || c->d_prime > m_glob(*c)))
    return fail(DSANLS_E_SHAPE, "subsampling needs d <= n_global and d_prime <= m_global");
  if (c->sketch == DSANLS_SKETCH_IDENTITY && (c->d != c->n || c->d_prime != c->m))
    return fail(DSANLS_E_SHAPE, "identity sketch needs d == n and d_prime == m");
  if (c->sketch == DSANLS_SKETCH_IDENTITY && is_share(*c))
    return fail(DSANLS_E_UNSUPPORTED, "identity sketch applies to the whole matrix only");
  if (c->sketch == DSANLS_SKETCH_COUNT && (c->d * 1024 < n_glob(*c) || c->d_prime * 1024 < m_glob(*c)))
    return fail(DSANLS_E_UNSUPPORTED, "count sketch needs d >= n_global / 1024 and d_prime >= m_global / 1024 "
                                      "(bucket lists of at most a few thousand rows)");
  if (c->sketch == DSANLS_SKETCH_SRHT) {
    if (M->format != DSANLS_DENSE) return fail(DSANLS_E_UNSUPPORTED, "SRHT applies to dense input only");
    if (srht_length(n_glob(*c)) > 32768 || srht_length(m_glob(*c)) > 32768)
      return fail(DSANLS_E_UNSUPPORTED, "SRHT supports m_global, n_global <= 32768 (the transform runs in LDS)");
    if (c->d > srht_length(n_glob(*c)) || c->d_prime > srht_length(m_glob(*c)))
      return fail(DSANLS_E_SHAPE, "SRHT needs d <= N = max(1024, 2^ceil(log2 n_global)), and d_prime likewise");
  }
  if ((c->sketch == DSANLS_SKETCH_COUNT || c->sketch == DSANLS_SKETCH_SRHT) && c->precision != DSANLS_PREC_FP32)
    return fail(DSANLS_E_UNSUPPORTED, "the BF16 form applies to the Gaussian sketch GEMM only");
  if (c->sketch == DSANLS_SKETCH_GAUSSIAN && std::max(c->d, c->d_prime) > 4 * 65535)
    return fail(DSANLS_E_SHAPE, "Gaussian sketch supports d <= 262140");
  if (c->warm_hidden < 0 || c->warm_hidden > 4096) return fail(DSANLS_E_INVALID_ARG, "warm_hidden out of range");
  if (c->warm_hidden > 0 && (c->d != c->d_prime || M->format != DSANLS_CSR || c->sketch != DSANLS_SKETCH_SUBSAMPLE))
    return fail(DSANLS_E_UNSUPPORTED, "warm start needs CSR input, a subsampling sketch and d == d_prime");
  if (c->warm_hidden > 0 && is_share(*c)) return fail(DSANLS_E_UNSUPPORTED, "warm start applies to the whole matrix only");
  if (!(c->alpha >= 0.0) || !(c->beta >= 0.0) || !std::isfinite(c->alpha) || !std::isfinite(c->beta))
    return fail(DSANLS_E_INVALID_ARG, "alpha and beta must be finite and >= 0");
  if (c->solver == DSANLS_SOLVER_PROX_CD) {
    if (c->sweeps < 0) return fail(DSANLS_E_INVALID_ARG, "sweeps must be >= 0");
    if (c->sweeps == 0 && (c->max_sweeps < 1 || !(c->tol >= 0.0)))
      return fail(DSANLS_E_INVALID_ARG, "to-tolerance mode needs max_sweeps >= 1 and tol >= 0");
  }
  // mu_0 = alpha must be positive for the one-step updates: a coordinate
  // with G_jj = 0 would have no defined step (fixed sweeps) and the PGD step
  // 1 / (2 (L + mu)) no bound; only the exact (to-tolerance) solve, which
  // then solves plain NNLS, may run with alpha = 0
  if (!(c->alpha > 0.0) && !(c->solver == DSANLS_SOLVER_PROX_CD && c->sweeps == 0))
    return fail(DSANLS_E_INVALID_ARG, "alpha (mu_0) must be > 0 outside to-tolerance mode");
  if (M->format == DSANLS_DENSE) {
    if (!M->dense || M->ld < c->n) return fail(DSANLS_E_INVALID_ARG, "dense M: NULL or ld < n");
    if (M->dense_t && M->ld_t < c->m) return fail(DSANLS_E_INVALID_ARG, "dense M^T: ld_t < m");
  } else if (M->format == DSANLS_CSR) {
    if (!M->rowptr || M->nnz < 0 || (M->nnz > 0 && (!M->colidx || !M->vals)))
      return fail(DSANLS_E_INVALID_ARG, "CSR M: rowptr, colidx and vals are required");
    if (M->t_rowptr != nullptr && M->nnz > 0 && (!M->t_colidx || !M->t_vals))
      return fail(DSANLS_E_INVALID_ARG, "CSR M^T: t_rowptr given without t_colidx or t_vals");
    if (c->sketch == DSANLS_SKETCH_GAUSSIAN || c->sketch == DSANLS_SKETCH_SRHT)
      return fail(DSANLS_E_UNSUPPORTED, "Gaussian and SRHT sketches on CSR input are not supported");
    if (c->precision != DSANLS_PREC_FP32)
      return fail(DSANLS_E_UNSUPPORTED, "BF16 sketch applies to dense input only");
  } else {
    return fail(DSANLS_E_INVALID_ARG, "bad matrix format");
  }
  return DSANLS_OK;
}

}  // namespace
}  // namespace dsanls

using namespace dsanls;

struct dsanls_ctx {
  dsanls_config cfg;
  dsanls_matrix mat;
  float* U;
  float* V;
  hipStream_t stream;
  Layout L;
  const float* Mt;  // resident M^T (caller's or ours)
  int64_t ldmt;
  double normM2;
  float upper;
  // record of the last update, for debug_fetch
  int last_side = -1;
  int64_t last_rows = 0, last_d = 0, last_lds = 0, last_lda = 0, last_ldb = 0;
  const float* last_A = nullptr;
  const float* last_B = nullptr;
  dsanls_stats stats{};
  // phase timing: per phase, event pairs recorded while timing is on
  bool timing = false;
  // DSANLS_TRACE in the environment at init: timing on from the start and a
  // per-phase summary on stderr when the context is released
  bool trace = false;
  std::vector<hipEvent_t> ev[4];
  int64_t timed_updates = 0;
  // outer iteration whose V-side sketch product A' = M^T S'^t is already in
  // A[1] (computed together with the U side), or -1
  int64_t lookahead_t = -1;
  // subsampling: the selection of the other side's next sketch (V side of
  // the same t after a U update, U side of t + 1 after a V update) is
  // launched on a side stream, where it overlaps this side's products and
  // NNLS; sel_t[side] is the iteration it was drawn for (-1: none usable),
  // ev_sel signals its end, ev_used the end of the last main-stream use of
  // that side's index buffers
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_sel[2] = {nullptr, nullptr};
  hipEvent_t ev_used[2] = {nullptr, nullptr};
  bool used_recorded[2] = {false, false};
  int64_t sel_t[2] = {-1, -1};
  bool gathered_ahead[2] = {false, false};   // the run-ahead also built the sketched rows
  bool ahead_pending[2] = {false, false};    // side-stream work on that side's buffers may be in flight
  // learned warm start (device parameters, caller-owned) and sketched rows
  const float* warm = nullptr;
  bool warm_residual = false;
  bool keep_rows = false;
  int64_t rows_kept = -1;   // rows of the kept sketched matrix, -1 if none
  ~dsanls_ctx() {
    for (auto& v : ev)
      for (hipEvent_t e : v) (void)hipEventDestroy(e);
    if (side_stream != nullptr) (void)hipStreamSynchronize(side_stream);
    for (int sd = 0; sd < 2; ++sd) {
      if (ev_sel[sd] != nullptr) (void)hipEventDestroy(ev_sel[sd]);
      if (ev_used[sd] != nullptr) (void)hipEventDestroy(ev_used[sd]);
    }
    if (side_stream != nullptr) (void)hipStreamDestroy(side_stream);
  }
};

namespace {

enum Phase { kPhSketch = 0, kPhProduct = 1, kPhSmall = 2, kPhNnls = 3 };

// Split the rows of a CSR matrix (device rowptr) into segments of at most
// kCsrSegment nnz and upload the table (init only; synchronous copies).
dsanls_status build_segments(const int64_t* d_rowptr, int64_t rows, int64_t cap, int64_t multi_cap,
                             CsrSegments& sg, hipStream_t s) {
  std::vector<int64_t> rp(rows + 1);
  DSANLS_HIP(hipMemcpyAsync(rp.data(), d_rowptr, sizeof(int64_t) * (rows + 1), hipMemcpyDeviceToHost, s));
  DSANLS_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> row, part, mrow, mpart;
  std::vector<int64_t> beg;
  row.reserve(rows);
  beg.reserve(rows);
  part.reserve(rows);
  int32_t np = 0;
  for (int64_t i = 0; i < rows; ++i) {
    const int64_t len = rp[i + 1] - rp[i];
    if (len < 0) return fail(DSANLS_E_INVALID_ARG, "CSR rowptr is not non-decreasing");
    const int64_t ns = len <= kCsrSegment ? 1 : (len + kCsrSegment - 1) / kCsrSegment;
    if (ns > 1) {
      mrow.push_back(static_cast<int32_t>(i));
      mpart.push_back(np);
    }
    for (int64_t q = 0; q < ns; ++q) {
      row.push_back(static_cast<int32_t>(i));
      beg.push_back(rp[i] + q * kCsrSegment);
      part.push_back(ns > 1 ? np++ : -1);
    }
  }
  mpart.push_back(np);
  if (static_cast<int64_t>(row.size()) > cap || static_cast<int64_t>(mrow.size()) > multi_cap)
    return fail(DSANLS_E_SHAPE, "CSR segment table exceeds its bound (rowptr inconsistent with nnz?)");
  sg.nseg = static_cast<int64_t>(row.size());
  sg.nmulti = static_cast<int64_t>(mrow.size());
  sg.nparts = np;
  DSANLS_HIP(hipMemcpyAsync(sg.seg_row, row.data(), sizeof(int32_t) * row.size(), hipMemcpyHostToDevice, s));
  DSANLS_HIP(hipMemcpyAsync(sg.seg_beg, beg.data(), sizeof(int64_t) * beg.size(), hipMemcpyHostToDevice, s));
  DSANLS_HIP(hipMemcpyAsync(sg.seg_part, part.data(), sizeof(int32_t) * part.size(), hipMemcpyHostToDevice, s));
  if (!mrow.empty())
    DSANLS_HIP(hipMemcpyAsync(sg.multi_row, mrow.data(), sizeof(int32_t) * mrow.size(), hipMemcpyHostToDevice, s));
  DSANLS_HIP(hipMemcpyAsync(sg.multi_part, mpart.data(), sizeof(int32_t) * mpart.size(), hipMemcpyHostToDevice, s));
  DSANLS_HIP(hipStreamSynchronize(s));
  return DSANLS_OK;
}

// Record an event on the stream (start or end of a phase) when timing is on.
dsanls_status mark(dsanls_ctx* ctx, int phase) {
  if (!ctx->timing) return DSANLS_OK;
  hipEvent_t e;
  DSANLS_HIP(hipEventCreate(&e));
  ctx->ev[phase].push_back(e);
  DSANLS_HIP(hipEventRecord(e, ctx->stream));
  return DSANLS_OK;
}

// Device flag words: err[0] non-finite values met by the checks of init and
// objective, err[1] and err[2] a subsample selection that failed (its
// boundary bucket over capacity) on the caller's stream and on the side
// stream.  read_scalars copies the first three back; objective clears them
// after reading, so each objective reports what happened since the last.
dsanls_status read_scalars(dsanls_ctx* ctx, float* host_red, int n_red, int* host_err) {
  hipStream_t s = ctx->stream;
  DSANLS_HIP(hipMemcpyAsync(host_red, ctx->L.red, sizeof(float) * n_red, hipMemcpyDeviceToHost, s));
  DSANLS_HIP(hipMemcpyAsync(host_err, ctx->L.err, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
  DSANLS_HIP(hipStreamSynchronize(s));
  return DSANLS_OK;
}

// Status of the flag words read by read_scalars, then cleared on the stream.
dsanls_status report_flags(dsanls_ctx* ctx, const int* err, const char* where) {
  DSANLS_HIP(hipMemsetAsync(ctx->L.err, 0, 3 * sizeof(int), ctx->stream));
  if (err[0]) return fail(DSANLS_E_NONFINITE, std::string(where) + ": non-finite values in U, V or the residual");
  if (err[1] | err[2])
    return fail(DSANLS_E_INTERNAL, std::string(where) + ": a subsample selection or a count-sketch bucket list "
                                                        "exceeded its capacity");
  return DSANLS_OK;
}

// One half-iteration: side 0 updates U from (M, V) with S^t (n x d), side 1
// updates V from (M^T, U) with S'^t (m x d').
dsanls_status half_iteration(dsanls_ctx* ctx, int side, int64_t t) {
  const dsanls_config& c = ctx->cfg;
  const Layout& L = ctx->L;
  hipStream_t s = ctx->stream;
  const bool is_dense = ctx->mat.format == DSANLS_DENSE;
  const bool bf16 = c.precision == DSANLS_PREC_BF16_SKETCH;
  const int64_t k = c.k;
  const int64_t rows = side == 0 ? c.m : c.n;
  const int64_t lng = side == 0 ? c.n : c.m;
  const int64_t d = side == 0 ? c.d : c.d_prime;
  float* Wself = side == 0 ? ctx->U : ctx->V;
  const float* Wother = side == 0 ? ctx->V : ctx->U;
  const float* X = side == 0 ? ctx->mat.dense : ctx->Mt;
  const int64_t ldx = side == 0 ? ctx->mat.ld : ctx->ldmt;
  const int64_t* rowptr = side == 0 ? ctx->mat.rowptr : ctx->mat.t_rowptr;
  const int32_t* colidx = side == 0 ? ctx->mat.colidx : ctx->mat.t_colidx;
  const float* vals = side == 0 ? ctx->mat.vals : ctx->mat.t_vals;
  const uint32_t tt = static_cast<uint32_t>(t);
  const double mu = c.alpha + c.beta * static_cast<double>(t);
  const int64_t lds = r4(lng), lda = r4(d), ldb = r4(d), ldw = r4(lng);
  // the long dimension of the whole matrix and where this block starts in
  // it: rows of the sketch (and the subsample) are drawn at global indices
  const int64_t lng_g = side == 0 ? n_glob(c) : m_glob(c);
  const int64_t off = side == 0 ? c.col_offset : c.row_offset;
  const bool share = is_share(c);
  dsanls_status st = DSANLS_OK;
#define CHECK(x)                      \
  do {                                \
    if ((st = (x)) != DSANLS_OK) return st; \
  } while (0)

  bool gathered = false;   // sketched rows of this side already built on the side stream
  const float* Bp = L.B;
  int64_t Bld = ldb, Bk = d;   // B is k x Bk with leading dimension Bld
  const float* Ap = L.A[side];
  int64_t Ald = lda;
  if (c.sketch == DSANLS_SKETCH_GAUSSIAN) {
    // S^t transposed (d x lng) and A = X S (rows x d) on MFMA.  A' = M^T S'^t
    // of the V side needs only M and t, so the U-side call draws both
    // sketches and runs both products as one grouped launch (filling the
    // machine with both tile sets); the V-side call of the same t reuses A'.
    const bool both = side == 0;
    if (both || ctx->lookahead_t != t) {
      CHECK(mark(ctx, kPhSketch));
      for (int sd = both ? 0 : 1; sd < 2; ++sd) {
        const int64_t lng_s = sd == 0 ? c.n : c.m, d_s = sd == 0 ? c.d : c.d_prime;
        const int64_t off_s = sd == 0 ? c.col_offset : c.row_offset;
        CHECK(launch_gaussian_sketch_t(c.seed, tt, sd, off_s, lng_s, d_s, L.St[sd], r4(lng_s),
                                       bf16 ? L.Sb[sd] : nullptr, r32(lng_s), s));
      }
      CHECK(mark(ctx, kPhSketch));
      CHECK(mark(ctx, kPhProduct));
      GemmDesc g[2];
      for (int sd = 0; sd < 2; ++sd) {
        const int64_t rows_s = sd == 0 ? c.m : c.n, lng_s = sd == 0 ? c.n : c.m;
        const int64_t d_s = sd == 0 ? c.d : c.d_prime;
        if (bf16)
          g[sd] = GemmDesc{sd == 0 ? L.Mb : L.Mtb, sd == 0 ? L.ldmb : L.ldmtb, L.Sb[sd], r32(lng_s), L.A[sd],
                           r4(d_s), rows_s, d_s, r32(lng_s)};
        else
          g[sd] = GemmDesc{sd == 0 ? ctx->mat.dense : ctx->Mt, sd == 0 ? ctx->mat.ld : ctx->ldmt, L.St[sd],
                           r4(lng_s), L.A[sd], r4(d_s), rows_s, d_s, lng_s};
      }
      if (!both) g[0].rows = 0;
      CHECK(launch_gemm_grouped(g[0], g[1], bf16, s));
      CHECK(mark(ctx, kPhProduct));
      ctx->lookahead_t = t;
    }
    // B = W^T S (k x d), split over the long dimension
    CHECK(mark(ctx, kPhSmall));
    CHECK(launch_transpose(Wother, k, L.Wt, ldw, lng, k, s));
    CHECK(launch_gemm_nt(L.Wt, ldw, L.St[side], lds, L.B, ldb, k, d, lng, L.gemm_ws, L.gemm_ws_bytes, s));
  } else if (c.sketch == DSANLS_SKETCH_SUBSAMPLE) {
    CHECK(mark(ctx, kPhSketch));
    // a selection launched ahead on the side stream: used if it is for this
    // t; otherwise waited for (it writes the same buffers) and redone here
    if (ctx->ahead_pending[side]) DSANLS_HIP(hipStreamWaitEvent(s, ctx->ev_sel[side], 0));
    ctx->ahead_pending[side] = false;
    if (ctx->sel_t[side] != t)
      CHECK(launch_subsample(c.seed, tt, side, lng_g, d, L.idx[side], is_dense ? nullptr : L.slot[side],
                             L.sub_ws[side], L.sub_ws_bytes, L.err + 1, s, off, lng, L.idx_win[side]));
    else
      gathered = ctx->gathered_ahead[side];
    ctx->sel_t[side] = -1;
    CHECK(mark(ctx, kPhSketch));
    // d of the lng_g columns, each scaled by sqrt(lng_g / d); a block sees
    // the sampled columns inside it (idx_win, -1 elsewhere)
    const float scale = static_cast<float>(std::sqrt(static_cast<double>(lng_g) / static_cast<double>(d)));
    const int32_t* idx_b = share ? L.idx_win[side] : L.idx[side];
    if (is_dense) {
      CHECK(mark(ctx, kPhProduct));
      CHECK(launch_gather_cols(X, ldx, idx_b, rows, d, scale, L.A[side], lda, s));
      CHECK(mark(ctx, kPhProduct));
    }
    CHECK(mark(ctx, kPhSmall));
    CHECK(launch_gather_rows_t(Wother, k, idx_b, d, scale, L.B, ldb, s));
  } else if (c.sketch == DSANLS_SKETCH_COUNT) {
    // hash and bucket lists of this side's rows of S (global row indices),
    // then A^T = S^T X^T bucket by bucket (reads X once) and B^T = S^T W
    const CountSketch& q = L.cs[side];
    CHECK(mark(ctx, kPhSketch));
    CHECK(launch_count_sketch_hash(c.seed, tt, side, off, lng, d, L.cs[side], s));
    CHECK(mark(ctx, kPhSketch));
    if (is_dense) {
      const float* Xt = side == 0 ? ctx->Mt : ctx->mat.dense;
      const int64_t ldxt = side == 0 ? ctx->ldmt : ctx->mat.ld;
      CHECK(mark(ctx, kPhProduct));
      CHECK(launch_count_sketch_rows(Xt, ldxt, rows, d, q, L.At, L.ldat, s));
      CHECK(launch_transpose(L.At, L.ldat, L.A[side], lda, d, rows, s));
      CHECK(mark(ctx, kPhProduct));
    }
    CHECK(mark(ctx, kPhSmall));
    CHECK(launch_count_sketch_rows(Wother, k, k, d, q, L.Bt, k, s));
    CHECK(launch_transpose(L.Bt, k, L.B, ldb, d, k, s));
  } else if (c.sketch == DSANLS_SKETCH_SRHT) {
    // signs of this side's rows and the d sampled Hadamard columns, then
    // A = X S and B = W^T S by one transform per row
    const int64_t N = L.hlen[side];
    CHECK(mark(ctx, kPhSketch));
    CHECK(launch_srht_signs(c.seed, tt, side, off, lng, L.hsign[side], s));
    CHECK(launch_subsample(c.seed, tt, side, N, d, L.hcol[side], nullptr, L.sub_ws[side], L.sub_ws_bytes, L.err + 1,
                           s, 0, 0, nullptr, kSrhtSampleKind));
    CHECK(mark(ctx, kPhSketch));
    CHECK(mark(ctx, kPhProduct));
    CHECK(launch_srht_rows(X, ldx, rows, lng, off, N, L.hsign[side], L.hcol[side], d, L.A[side], lda, s));
    CHECK(mark(ctx, kPhProduct));
    CHECK(mark(ctx, kPhSmall));
    CHECK(launch_transpose(Wother, k, L.Wt, ldw, lng, k, s));
    CHECK(launch_srht_rows(L.Wt, ldw, k, lng, off, N, L.hsign[side], L.hcol[side], d, L.B, ldb, s));
  } else {
    // identity: A = X, B = W^T
    CHECK(mark(ctx, kPhSmall));
    CHECK(launch_transpose(Wother, k, L.Wt, ldw, lng, k, s));
    Bp = L.Wt;
    Bld = ldw;
    Bk = lng;
    Ap = X;
    Ald = ldx;
  }
  CHECK(launch_gram(Bp, Bld, k, Bk, L.G, s));
  if (is_dense) {
    CHECK(launch_gemm_nt(Ap, Ald, Bp, Bld, L.R, k, rows, k, Bk, L.gemm_ws, L.gemm_ws_bytes, s));
    CHECK(mark(ctx, kPhSmall));
  } else {
    CHECK(mark(ctx, kPhSmall));
    const bool sub = c.sketch == DSANLS_SKETCH_SUBSAMPLE;
    ctx->rows_kept = -1;
    CHECK(mark(ctx, kPhProduct));
    if (sub && d <= kGatherMaxD && ctx->mat.nnz < (int64_t{1} << 31)) {
      // sketched rows a_i of A = X S (slot, sqrt(lng/d) * value) from the
      // sampled columns of X, i.e. rows idx of X^T, then R = A B^T with
      // B = sqrt(lng/d) W[idx]^T
      const int64_t* xt_rowptr = side == 0 ? ctx->mat.t_rowptr : ctx->mat.rowptr;
      const int32_t* xt_colidx = side == 0 ? ctx->mat.t_colidx : ctx->mat.colidx;
      const float* xt_vals = side == 0 ? ctx->mat.t_vals : ctx->mat.vals;
      const float scale = static_cast<float>(std::sqrt(static_cast<double>(lng_g) / static_cast<double>(d)));
      const int32_t* idx_b = share ? L.idx_win[side] : L.idx[side];
      if (!gathered)
        CHECK(launch_sampled_rows(xt_rowptr, xt_colidx, xt_vals, rows, idx_b, d, scale, L.a_cnt[side],
                                  L.a_pos[side], L.scan_ws[side], L.a_rowptr[side], L.a_cols[side],
                                  L.a_vals[side], L.long_rows[side], L.nlong[side], s));
      CHECK(launch_a_rhs(L.a_rowptr[side], L.a_cols[side], L.a_vals[side], rows, idx_b, Wother, k, scale,
                         L.long_rows[side], L.nlong[side], L.R,
                         s));
      ctx->rows_kept = rows;
    } else if (c.sketch == DSANLS_SKETCH_COUNT) {
      // the CSR stream, each entry (i, j) adding M_ij s_j B^T[h_j, :]
      CHECK(launch_csr_rhs_seg(rowptr, colidx, vals, L.seg[side], nullptr, L.Bt, k, 1.0f, L.R, L.seg_partials, s,
                               L.cs[side].bucket, L.cs[side].sign));
    } else {
      // the CSR stream: every nnz of X, the sampled ones (or all, identity)
      // folded into R
      // (the slot map covers the whole long dimension: this block's columns
      // start at off)
      const float scale = sub ? static_cast<float>(static_cast<double>(lng_g) / static_cast<double>(d)) : 1.0f;
      CHECK(launch_csr_rhs_seg(rowptr, colidx, vals, L.seg[side], sub ? L.slot[side] + off : nullptr, Wother, k,
                               scale, L.R, L.seg_partials, s));
    }
    CHECK(mark(ctx, kPhProduct));
  }
  const bool pgd = c.solver == DSANLS_SOLVER_PGD;
  const bool warm = ctx->warm != nullptr && !is_dense && c.sketch == DSANLS_SKETCH_SUBSAMPLE &&
                    !pgd && c.sweeps == 0;
  if (is_dense) ctx->rows_kept = -1;
  if (!is_dense && c.sketch == DSANLS_SKETCH_SUBSAMPLE && (warm || ctx->keep_rows) && ctx->rows_kept < 0) {
    // sketched rows from the CSR stream (d too large for the gather)
    CHECK(mark(ctx, kPhProduct));
    const float scale = static_cast<float>(std::sqrt(static_cast<double>(lng_g) / static_cast<double>(d)));
    CHECK(launch_sketched_rows(rowptr, colidx, vals, rows, L.seg[side], L.slot[side] + off, scale, L.a_cnt[side],
                               L.a_pos[side], L.scan_ws[side], L.a_rowptr[side], L.a_cols[side], L.a_vals[side],
                               s));
    CHECK(mark(ctx, kPhProduct));
    ctx->rows_kept = rows;
  }
  const float* start = nullptr;
  if (warm) {
    CHECK(mark(ctx, kPhSmall));
    CHECK(mlp_forward(static_cast<int>(d), static_cast<int>(k), c.warm_hidden, ctx->warm_residual, ctx->warm, rows,
                      L.a_rowptr[side],
                      L.a_cols[side], L.a_vals[side], Wself, L.ustart, L.mlp_ws, L.mlp_ws_bytes, s));
    CHECK(mark(ctx, kPhSmall));
    start = L.ustart;
  }
  CHECK(mark(ctx, kPhNnls));
  CHECK(launch_nnls(pgd, L.G, L.R, Wself, Wself, rows, static_cast<int>(k), static_cast<float>(mu),
                    c.sweeps, static_cast<float>(c.tol), c.max_sweeps, ctx->upper, nullptr,
                    L.tol.used != nullptr ? &L.tol : nullptr, L.nnls_ws, L.nnls_ws_bytes, s, start));
  if (!pgd && c.sweeps > 0) ctx->stats.sweeps_total += rows * c.sweeps;
  CHECK(mark(ctx, kPhNnls));
  if (ctx->timing) ctx->timed_updates += 1;
  if (ctx->side_stream != nullptr) {
    // this side's index buffers are free once the main stream gets here
    DSANLS_HIP(hipEventRecord(ctx->ev_used[side], s));
    ctx->used_recorded[side] = true;
    const int ns = 1 - side;
    const int64_t nt = side == 0 ? t : t + 1;
    if (nt <= UINT32_MAX) {
      const int64_t nlng = ns == 0 ? c.n : c.m, nd = ns == 0 ? c.d : c.d_prime;
      const int64_t nlng_g = ns == 0 ? n_glob(c) : m_glob(c), noff = ns == 0 ? c.col_offset : c.row_offset;
      if (ctx->ahead_pending[ns]) DSANLS_HIP(hipStreamWaitEvent(ctx->side_stream, ctx->ev_sel[ns], 0));
      if (ctx->used_recorded[ns]) DSANLS_HIP(hipStreamWaitEvent(ctx->side_stream, ctx->ev_used[ns], 0));
      dsanls_status ast = launch_subsample(c.seed, static_cast<uint32_t>(nt), ns, nlng_g, nd, L.idx[ns],
                                           is_dense ? nullptr : L.slot[ns], L.sub_ws[ns], L.sub_ws_bytes,
                                           L.err + 2, ctx->side_stream, noff, nlng, L.idx_win[ns]);
      // the sketched rows of that side need only M and the indices
      const bool gather = !is_dense && nd <= kGatherMaxD && ctx->mat.nnz < (int64_t{1} << 31);
      if (ast == DSANLS_OK && gather) {
        const int64_t nrows = ns == 0 ? c.m : c.n;
        const float nscale = static_cast<float>(std::sqrt(static_cast<double>(nlng_g) / static_cast<double>(nd)));
        ast = launch_sampled_rows(ns == 0 ? ctx->mat.t_rowptr : ctx->mat.rowptr,
                                  ns == 0 ? ctx->mat.t_colidx : ctx->mat.colidx,
                                  ns == 0 ? ctx->mat.t_vals : ctx->mat.vals, nrows,
                                  share ? L.idx_win[ns] : L.idx[ns], nd, nscale,
                                  L.a_cnt[ns], L.a_pos[ns], L.scan_ws[ns], L.a_rowptr[ns], L.a_cols[ns],
                                  L.a_vals[ns], L.long_rows[ns], L.nlong[ns], ctx->side_stream);
      }
      // the event covers whatever went out, even after a failure, and the
      // next use of these buffers waits for it; the result is used only if
      // everything went out
      DSANLS_HIP(hipEventRecord(ctx->ev_sel[ns], ctx->side_stream));
      ctx->ahead_pending[ns] = true;
      ctx->gathered_ahead[ns] = ast == DSANLS_OK && gather;
      ctx->sel_t[ns] = ast == DSANLS_OK ? nt : -1;
      if (ast != DSANLS_OK) return ast;
    }
  }
#undef CHECK
  ctx->last_side = side;
  ctx->last_rows = rows;
  ctx->last_d = Bk;
  ctx->last_lds = lds;
  ctx->last_A = is_dense ? Ap : nullptr;
  ctx->last_lda = Ald;
  ctx->last_B = Bp;
  ctx->last_ldb = Bld;
  ctx->stats.updates += 1;
  ctx->stats.rows_updated += rows;
  return DSANLS_OK;
}

}  // namespace

extern "C" {

const char* dsanls_status_string(dsanls_status s) {
  switch (s) {
    case DSANLS_OK: return "ok";
    case DSANLS_E_INVALID_ARG: return "invalid argument";
    case DSANLS_E_SHAPE: return "bad shape";
    case DSANLS_E_WORKSPACE: return "workspace too small or misaligned";
    case DSANLS_E_HIP: return "HIP runtime error";
    case DSANLS_E_NONFINITE: return "non-finite value";
    case DSANLS_E_STATE: return "call out of order";
    case DSANLS_E_UNSUPPORTED: return "unsupported";
    case DSANLS_E_INTERNAL: return "internal failure";
  }
  return "unknown status";
}

const char* dsanls_last_error(void) { return g_last_error.c_str(); }

dsanls_status dsanls_workspace_bytes(const dsanls_config* cfg, const dsanls_matrix* M, size_t* bytes) {
  if (!bytes) return fail(DSANLS_E_INVALID_ARG, "bytes is NULL");
  const dsanls_status st = validate(cfg, M);
  if (st != DSANLS_OK) return st;
  *bytes = plan(*cfg, *M, nullptr).total;
  return DSANLS_OK;
}

dsanls_status dsanls_init(const dsanls_config* cfg, const dsanls_matrix* M, float* U, float* V,
                          void* workspace, size_t workspace_bytes, void* hip_stream,
                          dsanls_ctx** out) {
  if (!out) return fail(DSANLS_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  dsanls_status st = validate(cfg, M);
  if (st != DSANLS_OK) return st;
  if (!U || !V) return fail(DSANLS_E_INVALID_ARG, "U or V is NULL");
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(DSANLS_E_WORKSPACE, "workspace must be non-NULL and 256-byte aligned");
  const size_t need = plan(*cfg, *M, nullptr).total;
  if (workspace_bytes < need)
    return fail(DSANLS_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  dsanls_ctx* ctx = new (std::nothrow) dsanls_ctx();
  if (!ctx) return fail(DSANLS_E_INVALID_ARG, "out of host memory");
  ctx->cfg = *cfg;
  ctx->mat = *M;
  ctx->U = U;
  ctx->V = V;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  if (const char* tr = std::getenv("DSANLS_TRACE"); tr != nullptr && tr[0] != '\0' && std::strcmp(tr, "0") != 0)
    ctx->timing = ctx->trace = true;
  ctx->L = plan(*cfg, *M, static_cast<char*>(workspace));
  const Layout& L = ctx->L;
  hipStream_t s = ctx->stream;
  const dsanls_config& c = *cfg;
  auto bail = [&](dsanls_status e) {
    delete ctx;
    return e;
  };
  if (c.sketch == DSANLS_SKETCH_SUBSAMPLE) {
    // side stream (default priority) and events for the selection run-ahead
    if (hipStreamCreateWithFlags(&ctx->side_stream, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(DSANLS_E_HIP, "init: side stream creation failed"));
    for (int sd = 0; sd < 2; ++sd)
      if (hipEventCreateWithFlags(&ctx->ev_sel[sd], hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&ctx->ev_used[sd], hipEventDisableTiming) != hipSuccess)
        return bail(fail(DSANLS_E_HIP, "init: event creation failed"));
  }

  if (hipMemsetAsync(L.err, 0, sizeof(int) * 16, s) != hipSuccess ||
      hipMemsetAsync(L.counters, 0, sizeof(unsigned long long) * 8, s) != hipSuccess)
    return bail(fail(DSANLS_E_HIP, "init: memset failed"));
  if (M->format == DSANLS_DENSE) {
    if (M->dense_t) {
      ctx->Mt = M->dense_t;
      ctx->ldmt = M->ld_t;
    } else {
      if ((st = launch_transpose(M->dense, M->ld, L.Mt, L.ldmt, c.m, c.n, s)) != DSANLS_OK) return bail(st);
      ctx->Mt = L.Mt;
      ctx->ldmt = L.ldmt;
    }
    if (c.precision == DSANLS_PREC_BF16_SKETCH) {
      if ((st = launch_to_bf16(M->dense, M->ld, L.Mb, L.ldmb, c.m, c.n, s)) != DSANLS_OK) return bail(st);
      if ((st = launch_to_bf16(ctx->Mt, ctx->ldmt, L.Mtb, L.ldmtb, c.n, c.m, s)) != DSANLS_OK) return bail(st);
      // the sketch kernel writes columns < lng of S^T only: zero the padding once
      for (int sd = 0; sd < 2; ++sd)
        if (L.Sb[sd] != nullptr) {
          const int64_t lng_s = sd == 0 ? c.n : c.m, d_s = sd == 0 ? c.d : c.d_prime;
          if ((st = launch_to_bf16(nullptr, 0, L.Sb[sd], r32(lng_s), d_s, 0, s)) != DSANLS_OK) return bail(st);
        }
    }
    if ((st = launch_sumsq(M->dense, M->ld, c.m, c.n, L.partials, s)) != DSANLS_OK) return bail(st);
    if ((st = launch_combine_partials(L.partials, sumsq_partials(c.m, c.n), 2, L.red, L.err, s)) != DSANLS_OK)
      return bail(st);
  } else {
    if (M->nnz > INT32_MAX) return bail(fail(DSANLS_E_SHAPE, "CSR input supports nnz < 2^31"));
    if (M->t_rowptr == nullptr) {
      // CSR(M^T) from CSR(M), rows of M^T sorted
      if ((st = launch_csr_transpose(M->rowptr, M->colidx, M->vals, c.m, c.n, M->nnz, L.t_rowptr, L.t_colidx,
                                     L.t_vals, L.ct_ws, L.ct_ws_bytes, s)) != DSANLS_OK)
        return bail(st);
      ctx->mat.t_rowptr = L.t_rowptr;
      ctx->mat.t_colidx = L.t_colidx;
      ctx->mat.t_vals = L.t_vals;
    }
    for (int sd = 0; sd < 2; ++sd) {
      if ((st = build_segments(sd == 0 ? M->rowptr : ctx->mat.t_rowptr, sd == 0 ? c.m : c.n, L.seg_cap[sd],
                               L.multi_cap[sd], ctx->L.seg[sd], s)) != DSANLS_OK)
        return bail(st);
    }
    const int64_t nnz = std::max<int64_t>(M->nnz, 1);
    if (M->nnz > 0) {
      if ((st = launch_sumsq(M->vals, nnz, 1, nnz, L.partials, s)) != DSANLS_OK) return bail(st);
      if ((st = launch_combine_partials(L.partials, sumsq_partials(1, nnz), 2, L.red, L.err, s)) != DSANLS_OK)
        return bail(st);
    } else if (hipMemsetAsync(L.red, 0, 2 * sizeof(float), s) != hipSuccess) {
      return bail(fail(DSANLS_E_HIP, "init: memset failed"));
    }
  }
  if ((st = launch_check_finite(U, c.m * c.k, L.err, s)) != DSANLS_OK) return bail(st);
  if ((st = launch_check_finite(V, c.n * c.k, L.err, s)) != DSANLS_OK) return bail(st);
  float red[2];
  int err[3] = {0, 0, 0};
  if ((st = read_scalars(ctx, red, 2, err)) != DSANLS_OK) return bail(st);
  if (err[0]) return bail(fail(DSANLS_E_NONFINITE, "init: M, U or V holds NaN/Inf"));
  ctx->normM2 = static_cast<double>(red[0]) + static_cast<double>(red[1]);
  ctx->upper = c.clip_upper ? static_cast<float>(std::sqrt(2.0 * std::sqrt(ctx->normM2))) : 0.0f;
  *out = ctx;
  return DSANLS_OK;
}

dsanls_status dsanls_sketch_update_U(dsanls_ctx* ctx, int64_t t) {
  if (!ctx) return fail(DSANLS_E_STATE, "update_U: context is NULL");
  if (t < 0 || t > UINT32_MAX) return fail(DSANLS_E_INVALID_ARG, "update_U: t out of range");
  return half_iteration(ctx, 0, t);
}

dsanls_status dsanls_sketch_update_V(dsanls_ctx* ctx, int64_t t) {
  if (!ctx) return fail(DSANLS_E_STATE, "update_V: context is NULL");
  if (t < 0 || t > UINT32_MAX) return fail(DSANLS_E_INVALID_ARG, "update_V: t out of range");
  return half_iteration(ctx, 1, t);
}

dsanls_status dsanls_objective(dsanls_ctx* ctx, double* rel_err) {
  if (!ctx) return fail(DSANLS_E_STATE, "objective: context is NULL");
  if (!rel_err) return fail(DSANLS_E_INVALID_ARG, "objective: rel_err is NULL");
  const dsanls_config& c = ctx->cfg;
  const Layout& L = ctx->L;
  hipStream_t s = ctx->stream;
  dsanls_status st;
  // the side stream's selections report into err[2]: they end before it is read
  for (int sd = 0; sd < 2; ++sd)
    if (ctx->ahead_pending[sd]) DSANLS_HIP(hipStreamWaitEvent(s, ctx->ev_sel[sd], 0));
  if ((st = launch_check_finite(ctx->U, c.m * c.k, L.err, s)) != DSANLS_OK) return st;
  if ((st = launch_check_finite(ctx->V, c.n * c.k, L.err, s)) != DSANLS_OK) return st;
  double resid = 0.0;
  if (ctx->mat.format == DSANLS_DENSE) {
    if ((st = launch_residual_sq(ctx->mat.dense, ctx->mat.ld, ctx->U, ctx->V, c.m, c.n, c.k, L.partials, s)) != DSANLS_OK)
      return st;
    if ((st = launch_combine_partials(L.partials, residual_partials(c.m, c.n), 2, L.red, L.err, s)) != DSANLS_OK)
      return st;
    float red[2];
    int err[3] = {0, 0, 0};
    if ((st = read_scalars(ctx, red, 2, err)) != DSANLS_OK) return st;
    if ((st = report_flags(ctx, err, "objective")) != DSANLS_OK) return st;
    resid = static_cast<double>(red[0]) + static_cast<double>(red[1]);
  } else {
    // ||M||^2 - 2 sum_nnz M_ij <u_i, v_j> + <U^T U, V^T V>
    const int64_t k = c.k;
    if ((st = launch_csr_cross(ctx->mat.rowptr, ctx->mat.colidx, ctx->mat.vals, c.m, ctx->U, ctx->V, k,
                               L.partials, s)) != DSANLS_OK)
      return st;
    if ((st = launch_combine_partials(L.partials, csr_cross_partials(c.m), 4, L.red, L.err, s)) != DSANLS_OK)
      return st;
    float* GU = L.Gobj;
    float* GV = L.Gobj + k * k;
    if ((st = launch_transpose(ctx->U, k, L.Wt, r4(c.m), c.m, k, s)) != DSANLS_OK) return st;
    if ((st = launch_gram(L.Wt, r4(c.m), k, c.m, GU, s)) != DSANLS_OK) return st;
    if ((st = launch_transpose(ctx->V, k, L.Wt, r4(c.n), c.n, k, s)) != DSANLS_OK) return st;
    if ((st = launch_gram(L.Wt, r4(c.n), k, c.n, GV, s)) != DSANLS_OK) return st;
    if ((st = launch_frob_dot(GU, GV, k * k, L.red + 4, s)) != DSANLS_OK) return st;
    float red[6];
    int err[3] = {0, 0, 0};
    if ((st = read_scalars(ctx, red, 6, err)) != DSANLS_OK) return st;
    if ((st = report_flags(ctx, err, "objective")) != DSANLS_OK) return st;
    const double cross = static_cast<double>(red[0]) + static_cast<double>(red[1]);
    const double gg = static_cast<double>(red[4]) + static_cast<double>(red[5]);
    resid = std::max(0.0, ctx->normM2 - 2.0 * cross + gg);
  }
  if (!std::isfinite(resid)) return fail(DSANLS_E_NONFINITE, "objective: residual is not finite");
  *rel_err = ctx->normM2 > 0 ? std::sqrt(resid / ctx->normM2) : std::sqrt(resid);
  return DSANLS_OK;
}

dsanls_status dsanls_get_stats(dsanls_ctx* ctx, dsanls_stats* out) {
  if (!ctx) return fail(DSANLS_E_STATE, "get_stats: context is NULL");
  if (!out) return fail(DSANLS_E_INVALID_ARG, "get_stats: out is NULL");
  unsigned long long cnt[3] = {0, 0, 0};
  DSANLS_HIP(hipMemcpyAsync(cnt, ctx->L.counters, sizeof(cnt), hipMemcpyDeviceToHost, ctx->stream));
  DSANLS_HIP(hipStreamSynchronize(ctx->stream));
  *out = ctx->stats;
  out->sweeps_total = ctx->stats.sweeps_total + static_cast<int64_t>(cnt[0]);
  out->rows_unconverged = static_cast<int64_t>(cnt[1]);
  out->warm_fallbacks = static_cast<int64_t>(cnt[2]);
  return DSANLS_OK;
}

dsanls_status dsanls_set_warm_start(dsanls_ctx* ctx, const float* params, int32_t hidden, int32_t residual) {
  if (!ctx) return fail(DSANLS_E_STATE, "set_warm_start: context is NULL");
  if (params == nullptr) {
    ctx->warm = nullptr;
    return DSANLS_OK;
  }
  if (ctx->cfg.warm_hidden <= 0 || ctx->L.mlp_ws == nullptr)
    return fail(DSANLS_E_STATE, "set_warm_start: the context was created with warm_hidden = 0");
  if (hidden != ctx->cfg.warm_hidden) return fail(DSANLS_E_SHAPE, "set_warm_start: hidden != cfg.warm_hidden");
  ctx->warm = params;
  ctx->warm_residual = residual != 0;
  return DSANLS_OK;
}

dsanls_status dsanls_set_keep_sketched_rows(dsanls_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(DSANLS_E_STATE, "set_keep_sketched_rows: context is NULL");
  if (enable && ctx->L.a_rowptr[0] == nullptr)
    return fail(DSANLS_E_STATE, "set_keep_sketched_rows: needs CSR input and a subsampling sketch");
  ctx->keep_rows = enable != 0;
  return DSANLS_OK;
}

dsanls_status dsanls_gather_sketched_rows(dsanls_ctx* ctx, const int32_t* sel, int64_t nsel,
                                          int32_t* out_rowptr, int32_t* out_cols, float* out_vals,
                                          int64_t capacity, int64_t* nnz) {
  if (!ctx) return fail(DSANLS_E_STATE, "gather_sketched_rows: context is NULL");
  if (ctx->rows_kept < 0) return fail(DSANLS_E_STATE, "gather_sketched_rows: the last update kept no rows");
  if (nsel < 0 || (nsel > 0 && (!sel || !out_cols || !out_vals)) || !out_rowptr || !nnz)
    return fail(DSANLS_E_INVALID_ARG, "gather_sketched_rows: bad arguments");
  if (nsel > std::max(ctx->cfg.m, ctx->cfg.n)) return fail(DSANLS_E_SHAPE, "gather_sketched_rows: nsel > max(m, n)");
  const Layout& L = ctx->L;
  hipStream_t s = ctx->stream;
  const int sd = ctx->last_side;
  dsanls_status st;
  // lengths into out_rowptr, scanned in place through the count buffer
  if ((st = launch_csr_select_len(L.a_rowptr[sd], ctx->rows_kept, sel, nsel, L.a_cnt[sd], s)) != DSANLS_OK)
    return st;
  if ((st = launch_exclusive_scan(L.a_cnt[sd], out_rowptr, nsel, L.scan_ws[sd], s)) != DSANLS_OK) return st;
  int32_t total = 0;
  DSANLS_HIP(hipMemcpyAsync(&total, out_rowptr + nsel, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  DSANLS_HIP(hipStreamSynchronize(s));
  *nnz = total;
  if (total > capacity) return fail(DSANLS_E_WORKSPACE, "gather_sketched_rows: capacity too small");
  st = launch_csr_select_copy(L.a_rowptr[sd], ctx->rows_kept, L.a_cols[sd], L.a_vals[sd], sel, nsel, out_rowptr,
                              out_cols, out_vals, s);
  // this side's rows are in use until here: a run-ahead gather into them waits
  if (st == DSANLS_OK && ctx->side_stream != nullptr) DSANLS_HIP(hipEventRecord(ctx->ev_used[sd], s));
  return st;
}

dsanls_status dsanls_set_timing(dsanls_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(DSANLS_E_STATE, "set_timing: context is NULL");
  ctx->timing = enable != 0;
  return DSANLS_OK;
}

dsanls_status dsanls_get_timing(dsanls_ctx* ctx, dsanls_timing* out) {
  if (!ctx) return fail(DSANLS_E_STATE, "get_timing: context is NULL");
  if (!out) return fail(DSANLS_E_INVALID_ARG, "get_timing: out is NULL");
  DSANLS_HIP(hipStreamSynchronize(ctx->stream));
  double ms[4] = {0, 0, 0, 0};
  for (int p = 0; p < 4; ++p) {
    auto& v = ctx->ev[p];
    for (size_t i = 0; i + 1 < v.size(); i += 2) {
      float e = 0.f;
      DSANLS_HIP(hipEventElapsedTime(&e, v[i], v[i + 1]));
      ms[p] += e;
    }
  }
  out->sketch_ms = ms[kPhSketch];
  out->product_ms = ms[kPhProduct];
  out->small_ms = ms[kPhSmall];
  out->nnls_ms = ms[kPhNnls];
  out->launches = ctx->timed_updates;
  return DSANLS_OK;
}

dsanls_status dsanls_debug_fetch(dsanls_ctx* ctx, int32_t which, void* dst, size_t bytes) {
  if (!ctx) return fail(DSANLS_E_STATE, "debug_fetch: context is NULL");
  if (!dst) return fail(DSANLS_E_INVALID_ARG, "debug_fetch: dst is NULL");
  if (ctx->last_side < 0) return fail(DSANLS_E_STATE, "debug_fetch: no update has run");
  const dsanls_config& c = ctx->cfg;
  const int64_t k = c.k, rows = ctx->last_rows, d = ctx->last_d;
  const int64_t lng = ctx->last_side == 0 ? c.n : c.m;
  hipStream_t s = ctx->stream;
  auto copy2d = [&](const void* src, int64_t ld_elems, int64_t h, int64_t w, size_t esz) -> dsanls_status {
    if (bytes != static_cast<size_t>(h * w) * esz) return fail(DSANLS_E_INVALID_ARG, "debug_fetch: wrong byte count");
    DSANLS_HIP(hipMemcpy2DAsync(dst, w * esz, src, ld_elems * esz, w * esz, h, hipMemcpyDeviceToHost, s));
    DSANLS_HIP(hipStreamSynchronize(s));
    return DSANLS_OK;
  };
  switch (which) {
    case 0:
      if (c.sketch == DSANLS_SKETCH_GAUSSIAN)
        return copy2d(ctx->L.St[ctx->last_side], ctx->last_lds, d, lng, sizeof(float));
      if (c.sketch == DSANLS_SKETCH_SUBSAMPLE) return copy2d(ctx->L.idx[ctx->last_side], d, 1, d, sizeof(int32_t));
      return fail(DSANLS_E_UNSUPPORTED, "debug_fetch: S is stored for the Gaussian and subsampling sketches only");
    case 1:
      if (!ctx->last_A) return fail(DSANLS_E_UNSUPPORTED, "debug_fetch: A is not formed on the CSR path");
      return copy2d(ctx->last_A, ctx->last_lda, rows, d, sizeof(float));
    case 2: return copy2d(ctx->last_B, ctx->last_ldb, k, d, sizeof(float));
    case 3: return copy2d(ctx->L.G, k, k, k, sizeof(float));
    case 4: return copy2d(ctx->L.R, k, rows, k, sizeof(float));
  }
  return fail(DSANLS_E_INVALID_ARG, "debug_fetch: bad selector");
}

dsanls_status dsanls_destroy(dsanls_ctx* ctx) {
  if (!ctx) return fail(DSANLS_E_STATE, "destroy: context is NULL");
  if (ctx->trace) {
    dsanls_timing t{};
    if (dsanls_get_timing(ctx, &t) == DSANLS_OK) {
      std::fprintf(stderr,
                   "[dsanls] %lld updates: sketch %.3f ms, product %.3f ms, small %.3f ms, nnls %.3f ms\n",
                   static_cast<long long>(t.launches), t.sketch_ms, t.product_ms, t.small_ms, t.nnls_ms);
      std::fflush(stderr);
    }
  }
  delete ctx;
  return DSANLS_OK;
}

}  // extern "C"
