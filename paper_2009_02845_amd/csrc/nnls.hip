// Batched row-wise NNLS updates of the sketched subproblem (Sec. 3.5).
//
// Every row i of U solves its own k-dimensional problem (the subproblem is
// row-independent, eq. u_block), all sharing G = B B^T.  Layout: one lane
// per row, 64 rows per wave.  The row's iterate u lives in registers as
// W-wide vector blocks; the Gram is prepared once as a padded KC x KC block
// (column j of G stored as row j, zero diagonal), copied into LDS by each
// workgroup and read by coordinate j as row j with broadcast loads, so 64
// rows share every G value.  The coordinate loop runs at run time inside
// each (statically unrolled) block, so the one dynamic register access per
// coordinate, u_j <- new value, is an indexed register write.  Rows of U
// move between HBM and the lanes through LDS panels of SW columns, loaded
// and stored by the whole wave with coalesced row runs; the right-hand side
// q = r + mu c streams into LDS one panel ahead of the coordinates that use
// it.  For fixed sweeps at the larger ranks a second kernel moves the
// coupling between coordinate blocks onto the matrix cores (see
// prox_cd_mfma_kernel).
#include "common.hpp"

namespace dsanls {

namespace {

// Prepared Gram: gp[j * KC + l] = G[l][j] for l != j (zero on the diagonal
// and outside k x k); gdiag[j] = G_jj; den[j] = G_jj + mu; inv[j] =
// 1 / den[j] (zero in the padding); colsum[j] = sum_l |G_lj| (for the PGD
// step size).
struct Prep {
  float* gp;
  float* gdiag;
  float* den;
  float* inv;
  float* colsum;
};

constexpr int kMaxKC = 128;

// Lane within the wave (a workgroup is one wave of 64 rows).
__device__ __forceinline__ int lane_id() { return static_cast<int>(threadIdx.x & 63); }

size_t prep_floats(int KC) { return nnls_prep_floats(KC); }

Prep carve_prep(void* ws, int KC) {
  float* p = static_cast<float*>(ws);
  return {p, p + KC * KC, p + KC * KC + KC, p + KC * KC + 2 * KC, p + KC * KC + 3 * KC};
}

// One wave per prepared row j (grid = KC).
__global__ __launch_bounds__(64) void prep_kernel(const float* __restrict__ G, int k, int KC,
                                                  float mu, float* __restrict__ gp,
                                                  float* __restrict__ gdiag,
                                                  float* __restrict__ den,
                                                  float* __restrict__ inv,
                                                  float* __restrict__ colsum) {
  const int j = blockIdx.x;
  float sabs = 0.f;
  for (int l = threadIdx.x; l < KC; l += 64) {
    const bool in = j < k && l < k;
    const float g = in ? G[static_cast<int64_t>(l) * k + j] : 0.f;
    gp[j * KC + l] = l != j ? g : 0.f;
    sabs += fabsf(g);
  }
  for (int o = 32; o > 0; o >>= 1) sabs += __shfl_xor(sabs, o, 64);
  if (threadIdx.x == 0) {
    if (j < k) {
      const float gj = G[static_cast<int64_t>(j) * k + j];
      const float dj = gj + mu;
      gdiag[j] = gj;
      den[j] = dj;
      // a zero denominator (G_jj = 0 and mu = 0) leaves the coordinate at 0
      inv[j] = dj != 0.f ? 1.0f / dj : 0.f;
      colsum[j] = sabs;
    } else {
      gdiag[j] = 0.f;
      den[j] = 1.f;
      inv[j] = 0.f;
      colsum[j] = 0.f;
    }
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

// The same dot product with the row in LDS (broadcast reads).  The row's
// address goes through an opaque VGPR copy so that every read is that one
// register plus an immediate offset (the compiler otherwise materialises
// each address in an SGPR and moves it to a VGPR, two instructions a read).
template <int KC, int W>
__device__ __forceinline__ float dot_row_lds(const float* g, const RowBlocks<KC, W>& u) {
  typedef __attribute__((address_space(3))) const float* lds_ptr;
  uint32_t a = static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_ptr)g));
  asm volatile("" : "+v"(a));
  const lds_ptr gl = reinterpret_cast<lds_ptr>(static_cast<uintptr_t>(a));
  float t0 = 0.f, t1 = 0.f;
  if constexpr (KC % 4 == 0) {
    // rows start 16-byte aligned: four values per read
    typedef float f4 __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(3))) const f4* lds_ptr4;
    const lds_ptr4 g4 = reinterpret_cast<lds_ptr4>(gl);
#pragma unroll
    for (int l = 0; l < KC; l += 4) {
      const f4 g = g4[l / 4];
      t0 += g[0] * u.b[l / W][l % W];
      t1 += g[1] * u.b[(l + 1) / W][(l + 1) % W];
      t0 += g[2] * u.b[(l + 2) / W][(l + 2) % W];
      t1 += g[3] * u.b[(l + 3) / W][(l + 3) % W];
    }
  } else {
#pragma unroll
    for (int l = 0; l < KC; l += 2) {
      t0 += gl[l] * u.b[l / W][l % W];
      if (l + 1 < KC) t1 += gl[l + 1] * u.b[(l + 1) / W][(l + 1) % W];
    }
  }
  return t0 + t1;
}

// The 64 rows of a wave move between HBM and registers through an LDS panel
// of SW columns (SW divides 64): row r of the panel starts at word r * STR,
// STR odd, so the 64 lanes reading one column of their own rows hit 64
// distinct banks, and the global side reads and writes runs of SW
// consecutive floats per row (64 / SW rows per instruction, coalesced)
// instead of one strided element per lane.
template <int SW>
struct Panel {
  static_assert(64 % SW == 0, "a load step covers whole panel rows");
  static constexpr int STR = SW | 1;
  static constexpr int WORDS = 64 * STR;
  static constexpr int RPS = 64 / SW;  // panel rows per load step
};

// panel <- columns [c0, c0 + SW) of rows [row0, row0 + nrows) of the
// row-major matrix P (row length k), plus mu times the same entries of C
// when ADD; entries outside the matrix are zero.  Every load is issued
// before the first LDS write; a load outside the matrix reads the panel's
// corner instead (in bounds) and is then discarded.
template <int SW, bool ADD>
__device__ __forceinline__ void stage(float* __restrict__ panel, const float* __restrict__ P,
                                      const float* __restrict__ C, float mu, int64_t row0,
                                      int nrows, int k, int c0, const int32_t* rmap = nullptr) {
  constexpr int STR = Panel<SW>::STR, RPS = Panel<SW>::RPS;
  // The inputs do not change during the kernel, so the compiler would hoist
  // every panel's loads (and their addresses) out of the sweep loop and keep
  // them all in registers; opaque copies of the corner and the lane index
  // keep the loads where they are.
  int64_t corner = row0 * k + c0;
  int lane = lane_id();
  asm volatile("" : "+s"(corner));
  asm volatile("" : "+v"(lane));
  const int rl = lane / SW, cl = lane % SW;
  float* dst = panel + rl * STR + cl;
  if (c0 >= k || nrows <= 0) {
#pragma unroll
    for (int s = 0; s < SW; ++s) dst[s * RPS * STR] = 0.f;
    return;
  }
  float x[SW];
  if (rmap != nullptr) {
    // listed rows (a compacted pass): row r of the panel is rmap[r]
    const bool col_ok = c0 + cl < k;
#pragma unroll
    for (int s = 0; s < SW; ++s) {
      const int r = s * RPS + rl;
      const bool ok = col_ok && r < nrows;
      const int64_t o = static_cast<int64_t>(rmap[ok ? r : 0]) * k + (ok ? c0 + cl : 0);
      float v = P[o];
      if (ADD) v += mu * C[o];
      x[s] = ok ? v : 0.f;
    }
#pragma unroll
    for (int s = 0; s < SW; ++s) dst[s * RPS * STR] = x[s];
    return;
  }
  const float* p = P + corner;
  const float* c = ADD ? C + corner : nullptr;
  const unsigned lane_off = static_cast<unsigned>(rl * k + cl) * 4u;
  const int64_t step = static_cast<int64_t>(RPS) * k;
  if (nrows == 64 && c0 + SW <= k) {
    // whole panel inside the matrix: a wave-uniform row base per step plus
    // the lane's 32-bit byte offset
#pragma unroll
    for (int s = 0; s < SW; ++s) {
      float v = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(p + s * step) + lane_off);
      if (ADD) v += mu * *reinterpret_cast<const float*>(reinterpret_cast<const char*>(c + s * step) + lane_off);
      x[s] = v;
    }
  } else {
    const bool col_ok = c0 + cl < k;
    const unsigned bstep = static_cast<unsigned>(step) * 4u;
#pragma unroll
    for (int s = 0; s < SW; ++s) {
      const bool ok = col_ok && s * RPS + rl < nrows;
      const unsigned o = ok ? lane_off + s * bstep : 0u;
      float v = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(p) + o);
      if (ADD) v += mu * *reinterpret_cast<const float*>(reinterpret_cast<const char*>(c) + o);
      x[s] = ok ? v : 0.f;
    }
  }
#pragma unroll
  for (int s = 0; s < SW; ++s) dst[s * RPS * STR] = x[s];
}

// Columns [c0, c0 + SW) of rows [row0, row0 + nrows) of P <- panel.
template <int SW>
__device__ __forceinline__ void unstage(const float* __restrict__ panel, float* P, int64_t row0,
                                        int nrows, int k, int c0, const int32_t* rmap = nullptr) {
  constexpr int STR = Panel<SW>::STR, RPS = Panel<SW>::RPS;
  int64_t corner = row0 * k + c0;
  int lane = lane_id();
  asm volatile("" : "+s"(corner));
  asm volatile("" : "+v"(lane));
  const int rl = lane / SW, cl = lane % SW;
  if (c0 >= k || c0 + cl >= k) return;
  const float* src = panel + rl * STR + cl;
  if (rmap != nullptr) {
#pragma unroll
    for (int s = 0; s < SW; ++s) {
      const int r = s * RPS + rl;
      if (r < nrows) P[static_cast<int64_t>(rmap[r]) * k + c0 + cl] = src[s * RPS * STR];
    }
    return;
  }
  char* p = reinterpret_cast<char*>(P + corner);
  const unsigned lane_off = static_cast<unsigned>(rl * k + cl) * 4u;
  const unsigned step = static_cast<unsigned>(RPS * k) * 4u;
#pragma unroll
  for (int s = 0; s < SW; ++s)
    if (s * RPS + rl < nrows) *reinterpret_cast<float*>(p + lane_off + s * step) = src[s * RPS * STR];
}

// The right-hand side q = r + mu c of the sweeps and the KKT test moves in
// panels of SW columns straight from HBM into LDS (global_load_lds_dword:
// no registers in between), one panel ahead of the coordinates that use
// it: the lanes read panel pc into registers, then issue panel pc + 1 into
// the same LDS and work through the coordinates of pc while it arrives.
// Lane l of load step s writes LDS word 64 s + l, i.e. row r = RPS s + l / SW
// of the panel at slot l % SW, which holds column (l % SW) ^ f(r): the
// swizzle f makes the 64 lanes reading one column of their own rows hit 64
// distinct banks (and 32 distinct within each half-wave).
template <int SW>
__device__ __forceinline__ int swz(int r) {
  constexpr int RPS = Panel<SW>::RPS;
  return (r / RPS) ^ ((SW / 2) * ((2 * r / RPS) & 1));
}

template <int SW>
struct QPanel {
  float r[64 * SW];
  float c[64 * SW];
};

// The compiler does not order the LDS reads of a panel after its
// global_load_lds writes (nor the next panel's writes after the reads), so
// the two waits are explicit, and compiler barriers too.
__device__ __forceinline__ void wait_lds_reads() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void wait_panel_loads() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
// Between the LDS writes and reads of one wave (the workgroup is one wave)
// a wait for the wave's own LDS traffic is enough: no barrier, and no wait
// for its global stores still in flight.
__device__ __forceinline__ void lds_order() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Issue the loads of columns [c0, c0 + SW) of rows [row0, row0 + nrows) of R
// and C into qp.  An entry outside the matrix loads the panel's corner
// instead (in bounds; its q is never used: padding coordinates have
// 1 / (G_jj + mu) = 0 and rows past nrows are not stored).
template <int SW>
__device__ __forceinline__ void q_issue(QPanel<SW>& qp, const float* __restrict__ R,
                                        const float* __restrict__ C, int64_t row0, int nrows, int k,
                                        int c0, bool with_c, const int32_t* rmap = nullptr) {
  constexpr int RPS = Panel<SW>::RPS;
  if (c0 >= k || nrows <= 0) return;
  // opaque copies, or the compiler hoists every panel's addresses out of the
  // sweep loop and keeps them all in registers
  int64_t corner = row0 * k + c0;
  int lane = lane_id();
  asm volatile("" : "+s"(corner));
  asm volatile("" : "+v"(lane));
  if (rmap != nullptr) {
    // listed rows (a compacted pass): row r of the panel is rmap[r]
#pragma unroll
    for (int s = 0; s < SW; ++s) {
      const int r = RPS * s + lane / SW;
      const int c = (lane % SW) ^ swz<SW>(r);
      const bool ok = r < nrows && c0 + c < k;
      const int64_t off = static_cast<int64_t>(rmap[ok ? r : 0]) * k + c0 + (ok ? c : 0);
      __builtin_amdgcn_global_load_lds(R + off, qp.r + 64 * s, 4, 0, 0);
      if (with_c) __builtin_amdgcn_global_load_lds(C + off, qp.c + 64 * s, 4, 0, 0);
    }
    return;
  }
  const float* rb = R + corner;
  const float* cb = C + corner;
#pragma unroll
  for (int s = 0; s < SW; ++s) {
    const int r = RPS * s + lane / SW;
    const int c = (lane % SW) ^ swz<SW>(r);
    const int off = r < nrows && c0 + c < k ? r * k + c : 0;
    __builtin_amdgcn_global_load_lds(rb + off, qp.r + 64 * s, 4, 0, 0);
    if (with_c) __builtin_amdgcn_global_load_lds(cb + off, qp.c + 64 * s, 4, 0, 0);
  }
}

// q[e] = r + mu c of this lane's row at panel column e (r alone without c).
template <int SW>
__device__ __forceinline__ void q_read(const QPanel<SW>& qp, float mu, int c0, int k, bool with_c,
                                       typename RowBlocks<SW, SW>::vec& q) {
  int lane = lane_id();
  asm volatile("" : "+v"(lane));
  const int f = swz<SW>(lane);
  wait_panel_loads();
  if (c0 >= k) {
#pragma unroll
    for (int e = 0; e < SW; ++e) q[e] = 0.f;
    return;
  }
  float x[SW], y[SW];
#pragma unroll
  for (int e = 0; e < SW; ++e) {
    x[e] = qp.r[SW * lane + (e ^ f)];
    y[e] = with_c ? qp.c[SW * lane + (e ^ f)] : 0.f;
  }
  if (c0 + SW > k) {
    // the last panel of a rank that is not a multiple of SW: its columns
    // past k hold the corner's value (see q_issue); they read as exact
    // zeros, so that the padding coordinates see finite values
#pragma unroll
    for (int e = 0; e < SW; ++e)
      if (c0 + e >= k) x[e] = y[e] = 0.f;
  }
#pragma unroll
  for (int e = 0; e < SW; ++e) q[e] = x[e] + mu * y[e];
}

// Non-finite guard of a row: g = fma(x, 0, g) stays +0 while every x folded
// in is finite and becomes NaN as soon as one is NaN or +-Inf (x * 0 is NaN
// for those).  The projection max(x, 0) would map a NaN to 0; instead a row
// whose guard is NaN is written out as NaN in every entry, so a non-finite
// right-hand side, centre, start or Gram never turns into a silent zero.
__device__ __forceinline__ void guard(float& g, float x) { g = __builtin_fmaf(x, 0.f, g); }

// A lane's row with a NaN guard becomes NaN in every entry.
template <int KC, int W>
__device__ __forceinline__ void poison_row(RowBlocks<KC, W>& u, float gd) {
  const bool bad = gd != gd;
#pragma unroll
  for (int l = 0; l < RowBlocks<KC, W>::NB * W; ++l) u.b[l / W][l % W] = bad ? __builtin_nanf("") : u.b[l / W][l % W];
}

// u <- this lane's row of P on the lanes where take holds.  A first load
// (u not yet live) of rows of 16 B multiples: per-lane float4 loads, all
// in flight at once; a reload (MASKED: u stays live, and 25 float4s beside
// it would cost occupancy) goes through the LDS panel, a cooperative load
// in which every lane of the wave takes part.
template <int KC, int W, int SW, bool MASKED = false>
__device__ __forceinline__ void load_rows(float* __restrict__ panel, const float* __restrict__ P,
                                          int64_t row0, int nrows, int k, bool take,
                                          RowBlocks<KC, W>& u, const int32_t* rmap = nullptr) {
  constexpr int NB = RowBlocks<KC, W>::NB, BPP = SW / W, NP = (KC + SW - 1) / SW;
  if (!MASKED && nrows <= 0) {   // a wave without rows (last workgroup)
#pragma unroll
    for (int l = 0; l < NB * W; ++l) u.b[l / W][l % W] = 0.f;
    return;
  }
  if (!MASKED && k % 4 == 0 && (reinterpret_cast<uintptr_t>(P) & 15) == 0) {
    // rows of 16 B multiples: each lane reads its own row as float4s (a
    // lane's row is contiguous, so every line is fetched once), all loads
    // in flight together; lanes past nrows read the last row and drop it
    constexpr int NQ = (KC + 3) / 4;
    const int rl = lane_id() < nrows ? lane_id() : nrows - 1;
    const int64_t grow = rmap != nullptr ? static_cast<int64_t>(rmap[rl]) : row0 + rl;
    const float4* src = reinterpret_cast<const float4*>(P + grow * k);
    const int kq = k / 4;
    float4 x[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) x[q] = src[q < kq ? q : kq - 1];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const bool in = q < kq;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int l = 4 * q + e;
        const float v = in ? (e == 0 ? x[q].x : e == 1 ? x[q].y : e == 2 ? x[q].z : x[q].w) : 0.f;
        if (take) u.b[l / W][l % W] = v;
      }
    }
#pragma unroll
    for (int l = 4 * NQ; l < NB * W; ++l)
      if (take) u.b[l / W][l % W] = 0.f;
    return;
  }
  const float* mine = panel + lane_id() * Panel<SW>::STR;
#pragma unroll
  for (int pc = 0; pc < NP; ++pc) {
    lds_order();
    stage<SW, false>(panel, P, nullptr, 0.f, row0, nrows, k, pc * SW, rmap);
    lds_order();
#pragma unroll
    for (int b = 0; b < BPP; ++b) {
      const int jb = pc * BPP + b;
      if (jb < NB) {
#pragma unroll
        for (int e = 0; e < W; ++e)
          if (take) u.b[jb][e] = mine[b * W + e];
      }
    }
  }
}

template <int KC, int W, int SW>
__device__ __forceinline__ void store_rows(float* __restrict__ panel, float* P, int64_t row0,
                                           int nrows, int k, const RowBlocks<KC, W>& u,
                                           const int32_t* rmap = nullptr) {
  constexpr int NB = RowBlocks<KC, W>::NB, BPP = SW / W, NP = (KC + SW - 1) / SW;
  if (k % 4 == 0 && (reinterpret_cast<uintptr_t>(P) & 15) == 0) {
    // each lane writes its own row as float4s (every line written whole by
    // one lane)
    constexpr int NQ = (KC + 3) / 4;
    if (lane_id() >= nrows) return;
    const int64_t grow = rmap != nullptr ? static_cast<int64_t>(rmap[lane_id()]) : row0 + lane_id();
    float4* dst = reinterpret_cast<float4*>(P + grow * k);
    const int kq = k / 4;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (q < kq)
        dst[q] = make_float4(u.b[(4 * q) / W][(4 * q) % W], u.b[(4 * q + 1) / W][(4 * q + 1) % W],
                             u.b[(4 * q + 2) / W][(4 * q + 2) % W], u.b[(4 * q + 3) / W][(4 * q + 3) % W]);
    return;
  }
  float* mine = panel + lane_id() * Panel<SW>::STR;
#pragma unroll
  for (int pc = 0; pc < NP; ++pc) {
    lds_order();
#pragma unroll
    for (int b = 0; b < BPP; ++b) {
      const int jb = pc * BPP + b;
      if (jb < NB) {
#pragma unroll
        for (int e = 0; e < W; ++e) mine[b * W + e] = u.b[jb][e];
      }
    }
    lds_order();
    unstage<SW>(panel, P, row0, nrows, k, pc * SW, rmap);
  }
}

// One Gauss-Seidel sweep over the coordinates (Alg. 3 / eq. entry_sol):
// u_j <- max((q_j - sum_{l != j} G_lj u_l) / (G_jj + mu), 0), j ascending,
// with u_l already updated for l < j, q = r + mu c one panel at a time,
// clipped at ub (+inf without a bound).  Only lanes with act set change
// their row.
template <int KC, int W, int SW, bool GLDS = false>
__device__ __forceinline__ void sweep(QPanel<SW>& qp, const float* __restrict__ gp,
                                      const float* __restrict__ inv, const float* __restrict__ R,
                                      const float* __restrict__ C, int64_t row0, int nrows, int k,
                                      float mu, float ub, bool act, bool c_is_u,
                                      RowBlocks<KC, W>& u, float& gd, const int32_t* rmap = nullptr) {
  // c_is_u: the centre is the iterate this sweep starts from, so c_j is
  // u_j as it stands when coordinate j is reached, and C is not read
  constexpr int NB = RowBlocks<KC, W>::NB, BPP = SW / W, NP = (KC + SW - 1) / SW;
  wait_lds_reads();
  q_issue<SW>(qp, R, C, row0, nrows, k, 0, !c_is_u, rmap);
#pragma unroll
  for (int pc = 0; pc < NP; ++pc) {
    typename RowBlocks<SW, SW>::vec qb;
    q_read<SW>(qp, mu, pc * SW, k, !c_is_u, qb);
    wait_lds_reads();
    if (pc + 1 < NP) q_issue<SW>(qp, R, C, row0, nrows, k, (pc + 1) * SW, !c_is_u, rmap);
#pragma unroll
    for (int b = 0; b < BPP; ++b) {
      const int jb = pc * BPP + b;
      if (jb < NB) {
        const int jn = (jb + 1) * W <= KC ? W : KC - jb * W;
#pragma nounroll
        for (int je = 0; je < jn; ++je) {
          const int j = jb * W + je;
          const float q = c_is_u ? qb[b * W + je] + mu * u.b[jb][je] : qb[b * W + je];
          const float t = GLDS ? dot_row_lds<KC, W>(gp + j * KC, u) : dot_row<KC, W>(gp + j * KC, u);
          const float x = (q - t) * inv[j];
          guard(gd, x);
          const float v = fminf(fmaxf(x, 0.f), ub);
          if (act) u.b[jb][je] = v;
        }
      }
    }
  }
}

// Relative projected-gradient norm of the row problem
// min_{u >= 0} 1/2 u Q u^T - q u^T, Q = G + mu I: zero exactly at its
// minimiser.
template <int KC, int W, int SW, bool GLDS = false>
__device__ __forceinline__ float kkt(QPanel<SW>& qp, const float* __restrict__ gp,
                                     const float* __restrict__ den, const float* __restrict__ R,
                                     const float* __restrict__ C, int64_t row0, int nrows, int k,
                                     float mu, const RowBlocks<KC, W>& u, float& gd,
                                     const int32_t* rmap = nullptr) {
  constexpr int NB = RowBlocks<KC, W>::NB, BPP = SW / W, NP = (KC + SW - 1) / SW;
  float pg2 = 0.f, q2 = 0.f;
  wait_lds_reads();
  q_issue<SW>(qp, R, C, row0, nrows, k, 0, true, rmap);
#pragma unroll
  for (int pc = 0; pc < NP; ++pc) {
    typename RowBlocks<SW, SW>::vec qb;
    q_read<SW>(qp, mu, pc * SW, k, true, qb);
    wait_lds_reads();
    if (pc + 1 < NP) q_issue<SW>(qp, R, C, row0, nrows, k, (pc + 1) * SW, true, rmap);
#pragma unroll
    for (int b = 0; b < BPP; ++b) {
      const int lb = pc * BPP + b;
      if (lb < NB) {
        const int ln = (lb + 1) * W <= KC ? W : KC - lb * W;
#pragma nounroll
        for (int le = 0; le < ln; ++le) {
          const int l = lb * W + le;
          const float q = qb[b * W + le];
          const float ul = u.b[lb][le];
          float g = (GLDS ? dot_row_lds<KC, W>(gp + l * KC, u) : dot_row<KC, W>(gp + l * KC, u)) + den[l] * ul - q;
          guard(gd, g);
          if (!(ul > 0.f)) g = fminf(g, 0.f);
          if (l < k) {
            pg2 += g * g;
            q2 += q * q;
          }
        }
      }
    }
  }
  return sqrtf(pg2) / fmaxf(sqrtf(q2), 1e-30f);
}

// Fixed number of sweeps (the paper's one, or s).  C (the proximal centre)
// may alias U: the rows of C are read only before U is written, at the end.
// A workgroup of NWV waves (each with its own 64 rows, panels and
// right-hand-side stream) copies the padded G into LDS once and reads its
// rows with broadcast LDS loads; fetching every row through the scalar
// cache instead, which the 100 x 100 Gram of the text workload overflows,
// was 1.32x slower.
template <int KC, int W, int SW, int NWV>
__global__ __launch_bounds__(64 * NWV) void prox_cd_lds_kernel(const float* __restrict__ gp,
                                                               const float* __restrict__ inv,
                                                               const float* __restrict__ R, const float* C,
                                                               float* U, int64_t rows, int k, float mu,
                                                               int sweeps, float upper,
                                                               int32_t* __restrict__ sweeps_used) {
  constexpr int kWords = Panel<SW>::WORDS > 2 * 64 * SW ? Panel<SW>::WORDS : 2 * 64 * SW;
  __shared__ __attribute__((aligned(16))) float sg[KC * KC];
  __shared__ float lds[NWV][kWords];
  {
    // every chunk of a thread loaded before the first is stored
    constexpr int N4 = KC * KC / 4, P = (N4 + 64 * NWV - 1) / (64 * NWV);
    float4 t[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int i = threadIdx.x + 64 * NWV * p;
      if (i < N4) t[p] = reinterpret_cast<const float4*>(gp)[i];
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int i = threadIdx.x + 64 * NWV * p;
      if (i < N4) reinterpret_cast<float4*>(sg)[i] = t[p];
    }
  }
  __syncthreads();
  // wave-uniform (scalar) wave index: the row addressing lives in SGPRs
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int64_t row0 = (blockIdx.x * static_cast<int64_t>(NWV) + wave) * 64;
  if (row0 >= rows) return;
  float* panel = lds[wave];
  QPanel<SW>& qp = *reinterpret_cast<QPanel<SW>*>(panel);
  const int nrows = static_cast<int>(rows - row0 < 64 ? rows - row0 : 64);
  const bool valid = lane_id() < nrows;
  const float ub = upper > 0.f ? upper : INFINITY;
  RowBlocks<KC, W> u;
  float gd = 0.f;
  load_rows<KC, W, SW>(panel, U, row0, nrows, k, true, u);
  for (int s = 0; s < sweeps; ++s)
    sweep<KC, W, SW, true>(qp, sg, inv, R, C, row0, nrows, k, mu, ub, true, s == 0 && C == U, u, gd);
  poison_row(u, gd);
  store_rows<KC, W, SW>(panel, U, row0, nrows, k, u);
  if (valid && sweeps_used != nullptr) sweeps_used[row0 + lane_id()] = sweeps;
}

// Fixed sweeps for the larger ranks, with the coordinates in blocks of 16
// and the coupling between blocks on the matrix cores.  The sweep is the
// same Gauss-Seidel pass in the same coordinate order: for a coordinate j
// of block b,
//   sum_{l != j} G_lj u_l = T_j + sum_{l in b, l != j} G_lj u_l,
//   T_j = sum_{l outside b} G_lj u_l,
// where the blocks before b already hold this sweep's values and the blocks
// after it the previous ones.  T for the 16 coordinates of block b and the
// wave's 64 rows is one product (16 x (KP - 16)) x ((KP - 16) x 64), taken
// with v_mfma_f32_16x16x4f32 right before the block is swept (its G
// operand read from L2 one block ahead); the 16 coordinates themselves run
// one lane per row on the VALU, with the block's own 16 x 16 part of G
// read from LDS by broadcast.  So per row and sweep the VALU does 16 k
// FMAs instead of k^2, and G is no longer read once per coordinate.
//
// Registers hold u in the MFMA operand layout: lane (m, g) = (lane % 16,
// lane / 16) holds, for each row quarter r, the values of row 16 r + m at
// coordinates 16 b + 4 g + e (e = 0..3) of every block b, which is also the
// layout in which the product leaves T.  A block's u and T move to one lane
// per row, and the new u back, through a 64 x 16 LDS tile whose 4-float
// chunks are XOR-swizzled by row.  Only for k % 4 == 0 and 16-byte aligned
// U and G (rows enter and leave as float4s in the operand layout; the
// to-tolerance passes also need C, the warm start and R aligned).
template <int KC>
struct MfmaCd {
  static constexpr int NBK = (KC + 15) / 16;   // coordinate blocks
  static constexpr int KP = 16 * NBK;          // padded rank
  static constexpr int NWV = 2;                // waves per workgroup
};

__device__ __forceinline__ int cd_chunk(int n, int c) { return 16 * n + 4 * (c ^ ((n >> 1) & 3)); }

// Coordinates j0 .. j0 + NJ - 1 of one lane's row, in order: t = T_j plus
// the block's own part of the dot product, then the proximal step.  The
// block's rows of G (gb: row jj at gb + jj * GS, zero diagonal) and
// 1 / (G_jj + mu) (ib) are read from LDS with broadcast reads, which the
// compiler can issue ahead of the coordinates that use them (scalar loads
// cannot be waited for one at a time).
template <int NJ, int GS, typename F4, typename QV>
__device__ __forceinline__ void cd_block(const float* gb, const float* ib, float mu, float ubnd,
                                         bool c_is_u, bool act, const QV& qb, const F4 (&tr)[4],
                                         F4 (&ur)[4], float& gd) {
  F4 gr[4], gn[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) gr[c] = *reinterpret_cast<const F4*>(gb + 4 * c);
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
    // the next coordinate's row is in flight while this one computes
    if (jj + 1 < NJ) {
#pragma unroll
      for (int c = 0; c < 4; ++c) gn[c] = *reinterpret_cast<const F4*>(gb + (jj + 1) * GS + 4 * c);
    }
    float t0 = tr[jj / 4][jj % 4], t1 = 0.f;
#pragma unroll
    for (int l = 0; l < NJ; ++l) {
      if (l == jj) continue;
      if (l & 1)
        t1 += gr[l / 4][l % 4] * ur[l / 4][l % 4];
      else
        t0 += gr[l / 4][l % 4] * ur[l / 4][l % 4];
    }
    const float q = c_is_u ? qb[jj] + mu * ur[jj / 4][jj % 4] : qb[jj];
    const float x = (q - (t0 + t1)) * ib[jj];
    guard(gd, x);
    const float v = fminf(fmaxf(x, 0.f), ubnd);
    if (act) ur[jj / 4][jj % 4] = v;
    if (jj + 1 < NJ) {
#pragma unroll
      for (int c = 0; c < 4; ++c) gr[c] = gn[c];
    }
  }
}

// Projected-gradient terms of coordinates j0 .. j0 + NJ - 1 of one lane's
// row (the KKT test of the to-tolerance solve): g_j = T_j + the block's
// own part of (G u)_j + (G_jj + mu) u_j - q_j, clipped at 0 from above where
// u_j = 0; sums of g_j^2 and q_j^2 over the coordinates below k.
template <int NJ, typename F4, typename QV>
__device__ __forceinline__ void kkt_block(const float* gb, const float* db, int j0, int k, const QV& qb,
                                          const F4 (&tr)[4], const F4 (&ur)[4], float& pg2, float& q2,
                                          float& gd) {
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
    F4 gr[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) gr[c] = *reinterpret_cast<const F4*>(gb + jj * 16 + 4 * c);
    float t0 = tr[jj / 4][jj % 4], t1 = 0.f;
#pragma unroll
    for (int l = 0; l < NJ; ++l) {
      if (l == jj) continue;
      if (l & 1)
        t1 += gr[l / 4][l % 4] * ur[l / 4][l % 4];
      else
        t0 += gr[l / 4][l % 4] * ur[l / 4][l % 4];
    }
    const float uj = ur[jj / 4][jj % 4];
    float gj = (t0 + t1) + db[jj] * uj - qb[jj];
    guard(gd, gj);
    if (!(uj > 0.f)) gj = fminf(gj, 0.f);
    if (j0 + jj < k) {
      pg2 += gj * gj;
      q2 += qb[jj] * qb[jj];
    }
  }
}

template <int KC>
__global__ __launch_bounds__(64 * MfmaCd<KC>::NWV) void prox_cd_mfma_kernel(
    const float* __restrict__ gp, const float* __restrict__ inv, const float* __restrict__ R,
    const float* C, float* U, int64_t rows, int k, float mu, int sweeps, float upper,
    int32_t* __restrict__ sweeps_used) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  constexpr int NBK = MfmaCd<KC>::NBK, KP = MfmaCd<KC>::KP, NWV = MfmaCd<KC>::NWV;
  // LDS: the 16 x 16 diagonal blocks of G (block b row jj at sd + (16 b +
  // jj) * 16, zero past KC), 1 / (G_jj + mu), and per wave a right-hand-side
  // panel and the transpose tile; about 15 KB a wave, so that several
  // workgroups share a CU and one's loads and stores overlap another's
  // arithmetic
  __shared__ __attribute__((aligned(16))) float sd[NBK * 256];
  __shared__ float sinv[KP];
  __shared__ QPanel<16> qps[NWV];
  __shared__ __attribute__((aligned(16))) float xs[NWV][64 * 16];
  {
    // 16-byte chunks (G rows are 16-byte aligned, KC % 4 == 0), every
    // chunk of a thread loaded before the first is stored: one round of L2
    // latency per workgroup instead of one per element
    constexpr int N4 = NBK * 64, P = (N4 + 64 * NWV - 1) / (64 * NWV);
    f4 t[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int i = 4 * (threadIdx.x + 64 * NWV * p);
      const int bk = i >> 8, j = 16 * bk + ((i >> 4) & 15), l = 16 * bk + (i & 15);
      t[p] = i < 4 * N4 && j < KC && l < KC ? *reinterpret_cast<const f4*>(gp + j * KC + l)
                                             : f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int i = 4 * (threadIdx.x + 64 * NWV * p);
      if (i < 4 * N4) *reinterpret_cast<f4*>(sd + i) = t[p];
    }
  }
  for (int i = threadIdx.x; i < KP; i += 64 * NWV) sinv[i] = i < KC ? inv[i] : 0.f;
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int64_t row0 = (blockIdx.x * static_cast<int64_t>(NWV) + wave) * 64;
  if (row0 >= rows) return;
  const int nrows = static_cast<int>(rows - row0 < 64 ? rows - row0 : 64);
  const int lane = lane_id(), m = lane & 15, g = lane >> 4;
  QPanel<16>& qp = qps[wave];
  float* X = xs[wave];
  const float ubnd = upper > 0.f ? upper : INFINITY;

  f4 ub[NBK][4];
#pragma unroll
  for (int b = 0; b < NBK; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = 16 * r + m, c = 16 * b + 4 * g;
      ub[b][r] = n < nrows && c < k ? *reinterpret_cast<const f4*>(U + (row0 + n) * k + c) : f4{0.f, 0.f, 0.f, 0.f};
    }

  // The blocks rotate through ub: while block b is swept it sits in ub[0]
  // and ub[i] holds block (b + i) mod NBK, so every register index is
  // static while the block loop runs at run time; after a sweep the order
  // is the original one again.
  // The MFMA's A operand for block b, rotated block i: G values of row
  // 16 b + m at coordinates 16 bb + 4 g .. + 3, bb = (b + i) mod NBK, read
  // from the prepared G in global memory (L2-resident) during the previous
  // block's coordinates; zero outside KC x KC.
  f4 an[NBK - 1];
  auto fetch_a = [&](int b) {
#pragma unroll
    for (int i = 1; i < NBK; ++i) {
      const int bb = b + i < NBK ? b + i : b + i - NBK;
      const int j = 16 * b + m, l = 16 * bb + 4 * g;
      const bool in = j < KC && l < KC;
      an[i - 1] = *reinterpret_cast<const f4*>(gp + (in ? j * KC + l : 0));
      if (!in) an[i - 1] = f4{0.f, 0.f, 0.f, 0.f};
    }
  };
  fetch_a(0);
  float gd = 0.f;   // non-finite guard of this lane's row (one lane per row in cd_block)
  for (int s = 0; s < sweeps; ++s) {
    const bool c_is_u = s == 0 && C == U;
    wait_lds_reads();
    q_issue<16>(qp, R, C, row0, nrows, k, 0, !c_is_u);
#pragma nounroll
    for (int b = 0; b < NBK; ++b) {
      f4 a[NBK - 1];
#pragma unroll
      for (int i = 0; i + 1 < NBK; ++i) a[i] = an[i];
      // T of block b's coordinates from every other block
      f4 acc[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 1; i < NBK; ++i) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i - 1][e], ub[i][r][e], acc[r], 0, 0, 0);
      }
      // the block's u and T to one lane per row (one wave's LDS accesses
      // are carried out in order, so the tile is reused without waits: the
      // compiler waits only where the values read are used)
      f4 ur[4], tr[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) *reinterpret_cast<f4*>(X + cd_chunk(16 * r + m, g)) = ub[0][r];
#pragma unroll
      for (int c = 0; c < 4; ++c) ur[c] = *reinterpret_cast<const f4*>(X + cd_chunk(lane, c));
#pragma unroll
      for (int r = 0; r < 4; ++r) *reinterpret_cast<f4*>(X + cd_chunk(16 * r + m, g)) = acc[r];
#pragma unroll
      for (int c = 0; c < 4; ++c) tr[c] = *reinterpret_cast<const f4*>(X + cd_chunk(lane, c));
      typename RowBlocks<16, 16>::vec qb;
      q_read<16>(qp, mu, 16 * b, k, !c_is_u, qb);
      wait_lds_reads();
      if (b + 1 < NBK) q_issue<16>(qp, R, C, row0, nrows, k, 16 * (b + 1), !c_is_u);
      // the next block's operands, issued after the panel wait above (which
      // waits for every load in flight)
      fetch_a(b + 1 < NBK ? b + 1 : 0);
      // the block's coordinates in order (the last block of a rank that is
      // not a multiple of 16 has only KC % 16 of them)
      const float* gb = sd + 256 * b;
      if (KC % 16 != 0 && b == NBK - 1)
        cd_block<(KC % 16 != 0 ? KC % 16 : 16), 16>(gb, sinv + 16 * b, mu, ubnd, c_is_u, true, qb, tr, ur, gd);
      else
        cd_block<16, 16>(gb, sinv + 16 * b, mu, ubnd, c_is_u, true, qb, tr, ur, gd);
      // the new values back to the operand layout, then rotate
#pragma unroll
      for (int c = 0; c < 4; ++c) *reinterpret_cast<f4*>(X + cd_chunk(lane, c)) = ur[c];
      f4 nb[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) nb[r] = *reinterpret_cast<const f4*>(X + cd_chunk(16 * r + m, g));
#pragma unroll
      for (int i = 0; i + 1 < NBK; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) ub[i][r] = ub[i + 1][r];
#pragma unroll
      for (int r = 0; r < 4; ++r) ub[NBK - 1][r] = nb[r];
    }
  }
  // rows whose guard is NaN leave as NaN (bit n of badm: row n)
  const unsigned long long badm = __ballot(gd != gd);
  const f4 nanv = f4{__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""), __builtin_nanf("")};
#pragma unroll
  for (int b = 0; b < NBK; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = 16 * r + m, c = 16 * b + 4 * g;
      if (n < nrows && c < k) *reinterpret_cast<f4*>(U + (row0 + n) * k + c) = (badm >> n) & 1ull ? nanv : ub[b][r];
    }
  if (lane < nrows && sweeps_used != nullptr) sweeps_used[row0 + lane] = sweeps;
}

// One pass of the to-tolerance solve.  Sweeps run on the lanes whose row is
// pending (relative projected-gradient norm above tol) until every row of
// the wave has converged, spent max_sweeps, or spent this pass's budget; the
// loop is wave-uniform (the panels are loaded by the whole wave) and a lane
// that is done keeps its row.  The first pass takes the rows in order and
// picks their start: with a warm start, each row starts from whichever of
// the warm start and the cold start (the centre U^t) has the smaller
// projected-gradient norm, and a start that is not finite is never taken.
// A row still pending when the budget runs out is listed (per wave, in lane
// order) for the next pass, which takes only listed rows and resumes from
// the row's current iterate and sweep count: a wave then waits only for
// rows as slow as its own, not for the slowest row of 64 neighbours.  The
// arithmetic of every row is the same as in one pass to the end.
struct TolPass {
  const int32_t* list_in;    // rows of this pass (null: all rows in order, first pass)
  const int32_t* count_in;   // number of listed rows (device)
  int budget;                // sweeps per row in this pass
  int32_t* used;             // per row: sweeps so far (may be null in a single pass)
  int32_t* flags;            // per row: bit 0 unconverged, bit 1 started cold (may be null)
  int32_t* wave_cnt;         // per wave: rows left pending (null: last pass, none kept)
  int32_t* wave_rows;        // per wave: those rows, 64 slots
};

template <int KC, int W, int SW, int NWV>
__global__ __launch_bounds__(64 * NWV) void prox_cd_tol_kernel(const float* __restrict__ gp,
                                                         const float* __restrict__ den,
                                                         const float* __restrict__ inv,
                                                         const float* __restrict__ R, const float* C,
                                                         const float* start, float* U, int64_t rows,
                                                         int k, float mu, float tol, int max_sweeps,
                                                         float upper, TolPass pass) {
  // the Gram in LDS, shared by the NWV waves of the workgroup (as in the
  // fixed-sweep kernel); every wave is otherwise on its own
  constexpr int kWords = Panel<SW>::WORDS > 2 * 64 * SW ? Panel<SW>::WORDS : 2 * 64 * SW;
  __shared__ __attribute__((aligned(16))) float sg[KC * KC];
  __shared__ float lds[NWV][kWords];
  {
    // every chunk of a thread loaded before the first is stored
    constexpr int N4 = KC * KC / 4, P = (N4 + 64 * NWV - 1) / (64 * NWV);
    float4 t[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int i = threadIdx.x + 64 * NWV * p;
      if (i < N4) t[p] = reinterpret_cast<const float4*>(gp)[i];
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int i = threadIdx.x + 64 * NWV * p;
      if (i < N4) reinterpret_cast<float4*>(sg)[i] = t[p];
    }
  }
  __syncthreads();
  const int wib = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int64_t wave = blockIdx.x * static_cast<int64_t>(NWV) + wib;
  if (wave * 64 >= rows) return;   // past the last wave (its per-wave slots do not exist)
  float* panel = lds[wib];
  QPanel<SW>& qp = *reinterpret_cast<QPanel<SW>*>(panel);
  const int lane = lane_id();
  int64_t row0 = wave * 64;
  const int32_t* rmap = nullptr;
  int nrows;
  if (pass.list_in != nullptr) {
    const int64_t cnt = *pass.count_in;
    if (row0 >= cnt) {
      if (pass.wave_cnt != nullptr && lane == 0) pass.wave_cnt[wave] = 0;
      return;
    }
    nrows = static_cast<int>(cnt - row0 < 64 ? cnt - row0 : 64);
    rmap = pass.list_in + row0;
  } else {
    nrows = static_cast<int>(rows - row0 < 64 ? rows - row0 : 64);
  }
  const bool valid = lane < nrows;
  const int64_t myrow = valid ? (rmap != nullptr ? static_cast<int64_t>(rmap[lane]) : row0 + lane) : 0;
  const float ub = upper > 0.f ? upper : INFINITY;
  RowBlocks<KC, W> u;
  int used = 0;
  bool fell_back = false;
  float res = INFINITY;   // a listed row is pending
  float gd = 0.f;         // non-finite guard (a warm start's own values are not folded in)
  if (rmap == nullptr) {
    load_rows<KC, W, SW>(panel, start != nullptr ? start : U, row0, nrows, k, true, u);
    bool ok = valid;
    if (start != nullptr) {
#pragma unroll
      for (int l = 0; l < KC; ++l) ok = ok && isfinite(u.b[l / W][l % W]);
    }
    float res_w = 0.f, res_c = 0.f;
    const int ncand = start != nullptr ? 2 : 1;
#pragma nounroll
    for (int c = 0; c < ncand; ++c) {
      if (c == 1 && !__any(valid && !(ok && res_w <= tol))) {
        // every row keeps its warm start (finite and within tolerance): the
        // cold candidate's KKT pass is skipped
        res_c = INFINITY;
        break;
      }
      if (c == 1) load_rows<KC, W, SW, true>(panel, C, row0, nrows, k, true, u);
      float gc = 0.f;
      const float r = kkt<KC, W, SW, true>(qp, sg, den, R, C, row0, nrows, k, mu, u, gc);
      if (c + 1 == ncand) gd += gc;   // the cold start (or the only start)
      if (c == 0) res_w = r;
      else res_c = r;
    }
    res = res_w;
    if (start != nullptr) {
      // a finite warm start within tolerance is kept; otherwise the
      // candidate with the smaller residual
      const bool warm = ok && (res_w <= tol || res_w < res_c);
      fell_back = valid && !warm;
      if (__any(warm)) load_rows<KC, W, SW, true>(panel, start, row0, nrows, k, warm, u);
      res = warm ? res_w : res_c;
    }
  } else {
    load_rows<KC, W, SW>(panel, U, row0, nrows, k, true, u, rmap);
    used = valid && pass.used != nullptr ? pass.used[myrow] : 0;
  }
  int here = 0;
  bool pend = false;
  for (;;) {
    if (valid) pend = res > tol;
    const bool run = valid && pend && used < max_sweeps && here < pass.budget;
    if (!__any(run)) break;
    sweep<KC, W, SW, true>(qp, sg, inv, R, C, row0, nrows, k, mu, ub, run, false, u, gd, rmap);
    if (run) {
      ++used;
      ++here;
    }
    res = kkt<KC, W, SW, true>(qp, sg, den, R, C, row0, nrows, k, mu, u, gd, rmap);
  }
  poison_row(u, gd);
  store_rows<KC, W, SW>(panel, U, row0, nrows, k, u, rmap);
  const bool keep = valid && pend && used < max_sweeps && pass.wave_cnt != nullptr;
  if (valid) {
    if (pass.used != nullptr) pass.used[myrow] = used;
    if (pass.flags != nullptr) {
      const int32_t unconv = !keep && pend ? 1 : 0;
      if (rmap == nullptr) pass.flags[myrow] = (fell_back ? 2 : 0) | unconv;
      else if (unconv) pass.flags[myrow] |= 1;
    }
  }
  if (pass.wave_cnt != nullptr) {
    const unsigned long long m = __ballot(keep);
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    if (keep) pass.wave_rows[wave * 64 + rank] = static_cast<int32_t>(myrow);
    if (lane == 0) pass.wave_cnt[wave] = __popcll(m);
  }
}

// Q = R + mu C over n4 float4s (16-byte aligned): the right-hand side of
// every pass of a to-tolerance solve in the block form, formed once.
__global__ __launch_bounds__(256) void qsum_kernel(const float4* __restrict__ R, const float4* C, float mu,
                                                   int64_t n4, float4* __restrict__ Q) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n4; i += gridDim.x * 256ll) {
    const float4 r = R[i], c = C[i];
    Q[i] = make_float4(r.x + mu * c.x, r.y + mu * c.y, r.z + mu * c.z, r.w + mu * c.w);
  }
}

// One pass of the to-tolerance solve in the block form, carrying each row's
// gradient g = u Q - q (Q = G + mu I, the row problem of eq. reg_sub
// divided by 2) in registers instead of re-forming it for every stopping
// test.  The passes, start choice, per-row stopping and bookkeeping are
// those of prox_cd_tol_kernel.  Coordinate j's prox-CD step (eq. entry_sol)
// is u_j <- max(u_j - g_j / Q_jj, 0) with g_j current, the same Gauss-Seidel
// update written through the gradient.  Per coordinate block b (16
// coordinates, all in order):
//   - the block's u and g go to one lane per row through the LDS tile; the
//     16 coordinates step in order, each step delta_j moving the g of the
//     block's later coordinates by delta_j Q_jl (the block's own 16 x 16 part
//     of Q read by LDS broadcast);
//   - the block's new u returns to the operand layout, and every block of g
//     takes g_bb += delta_b Q_{b,bb}, one (16 x 16) x (16 x 64) product per
//     block on v_mfma_f32_16x16x4f32 (16 MFMAs each, the operand read from Q
//     in LDS).
// After the sweep g is exact (up to rounding) at the new iterate, so the
// stopping test, ||pg|| / ||q|| <= tol with pg_j = g_j where u_j > 0 and
// min(g_j, 0) where u_j = 0, costs O(k) per row instead of a pass of 2 k^2
// flop.  Each pass forms g afresh (the same products, from u and q), so the
// rounding carried in g is that of at most one pass's sweeps.  Rows that are
// done (or out of budget) enter the products with delta = 0 and keep their
// values (a step clamped to [u_j, u_j]).  A non-finite value anywhere in a
// row's problem reaches its g, which every stopping test folds into the
// row's guard.  Registers: u and g of the wave's 16 RQ rows in the operand
// layout (lane (m, g) holds rows 16 r + m, r < RQ, coordinates 16 b + 4 g ..
// + 3), 2 RQ KP / 4 floats a lane, one wave per SIMD; the block loop is
// unrolled so every index is static.  With WITHC, q = r + mu c is read from
// R and C when g is formed; without, R already holds q.  C (the cold start
// of the first pass) is read before the wave writes its rows, so it may
// alias U.
template <int KC, bool WITHC, int RQ>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(1, 1))) void prox_cd_grad_tol_kernel(
    const float* __restrict__ gp, const float* __restrict__ den, const float* __restrict__ inv,
    const float* __restrict__ R, const float* C, const float* start, float* U, int64_t rows, int k,
    float mu, float tol, int max_sweeps, float upper, TolPass pass) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  constexpr int NBK = MfmaCd<KC>::NBK, KP = MfmaCd<KC>::KP, NWV = 2, QS = KP + 4, NR = 16 * RQ;
  // Q (row j: G_jl, G_jj + mu on the diagonal, zero outside KC x KC; rows
  // padded to QS floats), its diagonal blocks for the coordinate steps, and
  // one transpose tile per wave
  __shared__ __attribute__((aligned(16))) float sq[KP * QS];
  __shared__ __attribute__((aligned(16))) float sdb[NBK * 16 * 20];
  __shared__ __attribute__((aligned(16))) float xs[NWV][NR * 16];
  // a workgroup past the pass's rows leaves before staging Q
  if (blockIdx.x * static_cast<int64_t>(NWV * NR) >= (pass.list_in != nullptr ? *pass.count_in : rows)) {
    if (pass.wave_cnt != nullptr && threadIdx.x % 64 == 0) {
      const int64_t w = blockIdx.x * static_cast<int64_t>(NWV) + threadIdx.x / 64;
      if (w * NR < rows) pass.wave_cnt[w] = 0;
    }
    return;
  }
  {
    // Both copies in 16-byte chunks, every chunk of a thread loaded before
    // the first is stored (one round of L2 latency per workgroup instead of
    // one per element).  Rows of the prepared Gram are 16-byte aligned
    // (KC % 4 == 0); a chunk lies wholly inside or outside KC.  sdb: row j =
    // 16 b + jj at sdb + 20 j: Q_jl for l != j in the block, 1 / Q_jj (0: a
    // zero Q_jj, or past k) on the diagonal.
    constexpr int C1 = QS / 4, N1 = KP * C1, C2 = 5, N2 = NBK * 16 * C2;
    constexpr int P1 = (N1 + 64 * NWV - 1) / (64 * NWV), P2 = (N2 + 64 * NWV - 1) / (64 * NWV);
    f4 t1[P1], t2[P2];
#pragma unroll
    for (int p = 0; p < P1; ++p) {
      const int i = threadIdx.x + 64 * NWV * p, j = i / C1, l = 4 * (i - j * C1);
      f4 v = f4{0.f, 0.f, 0.f, 0.f};
      if (i < N1 && j < KC && l < KC) {
        v = *reinterpret_cast<const f4*>(gp + j * KC + l);
        if (j >= l && j < l + 4) v[j - l] = den[j];
      }
      t1[p] = v;
    }
#pragma unroll
    for (int p = 0; p < P2; ++p) {
      const int i = threadIdx.x + 64 * NWV * p, j = i / C2, c = i - j * C2, l = 16 * (j / 16) + 4 * c;
      f4 v = f4{0.f, 0.f, 0.f, 0.f};
      if (i < N2 && c < 4 && j < KC && l < KC) {
        v = *reinterpret_cast<const f4*>(gp + j * KC + l);
        if (j >= l && j < l + 4) v[j - l] = inv[j];
      }
      t2[p] = v;
    }
#pragma unroll
    for (int p = 0; p < P1; ++p) {
      const int i = threadIdx.x + 64 * NWV * p;
      if (i < N1) *reinterpret_cast<f4*>(sq + 4 * i) = t1[p];
    }
#pragma unroll
    for (int p = 0; p < P2; ++p) {
      const int i = threadIdx.x + 64 * NWV * p;
      if (i < N2) *reinterpret_cast<f4*>(sdb + 4 * i) = t2[p];
    }
  }
  __syncthreads();
  const int wib = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int64_t wave = blockIdx.x * static_cast<int64_t>(NWV) + wib;
  if (wave * NR >= rows) return;   // past the last wave (its per-wave slots do not exist)
  const int lane = lane_id(), m = lane & 15, g = lane >> 4;
  const int64_t row0 = wave * NR;
  const int32_t* rmap = nullptr;
  int nrows;
  if (pass.list_in != nullptr) {
    const int64_t cnt = *pass.count_in;
    if (row0 >= cnt) {
      if (pass.wave_cnt != nullptr && lane == 0) pass.wave_cnt[wave] = 0;
      return;
    }
    nrows = static_cast<int>(cnt - row0 < NR ? cnt - row0 : NR);
    rmap = pass.list_in + row0;
  } else {
    nrows = static_cast<int>(rows - row0 < NR ? rows - row0 : NR);
  }
  const bool valid = lane < nrows;
  const int64_t myrow = valid ? (rmap != nullptr ? static_cast<int64_t>(rmap[lane]) : row0 + lane) : 0;
  const float ubnd = upper > 0.f ? upper : INFINITY;
  float* X = xs[wib];

  // offset of row 16 r + m of the wave in the row-major matrices (-1: past
  // the wave's rows)
  int64_t roff[RQ];
#pragma unroll
  for (int r = 0; r < RQ; ++r) {
    const int n = 16 * r + m;
    roff[r] = n < nrows ? (rmap != nullptr ? static_cast<int64_t>(rmap[n]) : row0 + n) * k : -1;
  }
  f4 ub[NBK][RQ], gb[NBK][RQ];
  // every row into the operand layout: from P1 where the row's bit is set in
  // take, else from P0 (one load per value either way)
  auto load_ub = [&](const float* P0, const float* P1, unsigned long long take) {
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
      const float* P = (take >> (16 * r + m)) & 1ull ? P1 : P0;
#pragma unroll
      for (int b = 0; b < NBK; ++b) {
        const int c = 16 * b + 4 * g;
        ub[b][r] = roff[r] >= 0 && c < k ? *reinterpret_cast<const f4*>(P + roff[r] + c) : f4{0.f, 0.f, 0.f, 0.f};
      }
    }
  };
  // per-row sums (lane per row) of per-(lane, quarter) partial sums: the
  // four lanes of a row quarter add up, lane 16 g + m keeps quarter g
  auto row_sum = [&](float (&s)[RQ]) -> float {
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
      s[r] += __shfl_xor(s[r], 16, 64);
      s[r] += __shfl_xor(s[r], 32, 64);
    }
    float v = 0.f;
#pragma unroll
    for (int r = 0; r < RQ; ++r)
      if (g == r) v = s[r];
    return v;
  };
  // g = u Q - q for the wave's rows, and ||q||^2 of each row (lane per row)
  float q2 = 0.f;
  auto form_g = [&]() {
    float qs[RQ];
#pragma unroll
    for (int r = 0; r < RQ; ++r) qs[r] = 0.f;
#pragma unroll
    for (int bb = 0; bb < NBK; ++bb) {
#pragma unroll
      for (int r = 0; r < RQ; ++r) {
        const int c = 16 * bb + 4 * g;
        f4 q = f4{0.f, 0.f, 0.f, 0.f};
        if (roff[r] >= 0 && c < k) {
          q = *reinterpret_cast<const f4*>(R + roff[r] + c);
          if (WITHC) q += mu * *reinterpret_cast<const f4*>(C + roff[r] + c);
        }
        qs[r] += (q[0] * q[0] + q[1] * q[1]) + (q[2] * q[2] + q[3] * q[3]);
        gb[bb][r] = -q;
      }
#pragma unroll
      for (int b = 0; b < NBK; ++b) {
        const f4 a = *reinterpret_cast<const f4*>(sq + (16 * bb + m) * QS + 16 * b + 4 * g);
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int r = 0; r < RQ; ++r)
            gb[bb][r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], ub[b][r][e], gb[bb][r], 0, 0, 0);
      }
      // one block of g at a time (the scheduler would otherwise hoist every
      // block's loads, beyond the register file)
      __builtin_amdgcn_sched_barrier(0);
    }
    q2 = row_sum(qs);
  };
  // relative projected-gradient norm of each row (lane per row) from the
  // carried g; gk takes the non-finite guard of the row's g
  auto kkt = [&](float& gk) -> float {
    float s[RQ], z[RQ];
#pragma unroll
    for (int r = 0; r < RQ; ++r) s[r] = z[r] = 0.f;
#pragma unroll
    for (int bb = 0; bb < NBK; ++bb)
#pragma unroll
      for (int r = 0; r < RQ; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          // coordinates past k hold g = 0 exactly
          const float gv = gb[bb][r][e];
          z[r] = __builtin_fmaf(gv, 0.f, z[r]);
          const float pg = ub[bb][r][e] > 0.f ? gv : fminf(gv, 0.f);
          s[r] = __builtin_fmaf(pg, pg, s[r]);
        }
    guard(gk, row_sum(z));
    return sqrtf(row_sum(s)) / fmaxf(sqrtf(q2), 1e-30f);
  };
  float gd = 0.f;   // non-finite guard of this lane's row (a warm start's own values are not folded in)
  auto sweep = [&](bool run) {
#pragma unroll
    for (int b = 0; b < NBK; ++b) {
      // (lanes past the wave's NR rows read row lane % NR and write nothing)
      f4 ur[4], gr[4];
      const int me = lane & (NR - 1);
#pragma unroll
      for (int r = 0; r < RQ; ++r) *reinterpret_cast<f4*>(X + cd_chunk(16 * r + m, g)) = ub[b][r];
#pragma unroll
      for (int c = 0; c < 4; ++c) ur[c] = *reinterpret_cast<const f4*>(X + cd_chunk(me, c));
#pragma unroll
      for (int r = 0; r < RQ; ++r) *reinterpret_cast<f4*>(X + cd_chunk(16 * r + m, g)) = gb[b][r];
#pragma unroll
      for (int c = 0; c < 4; ++c) gr[c] = *reinterpret_cast<const f4*>(X + cd_chunk(me, c));
      // the block's coordinates in order (the last block of a rank that is
      // not a multiple of 16 has only KC % 16 of them)
      constexpr int NL = KC % 16 != 0 ? KC % 16 : 16;
      const int nj = b == NBK - 1 ? NL : 16;
      // row jj of the block's part of Q (1 / Q_jj on the diagonal), one row
      // ahead of its use, alternating between two buffers
      const float* qb = sdb + (16 * b) * 20;
      f4 qv[2][4];
#pragma unroll
      for (int c = 0; c < 4; ++c) qv[0][c] = *reinterpret_cast<const f4*>(qb + 4 * c);
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        if (jj < nj) {
          if (jj + 1 < nj) {
#pragma unroll
            for (int c = (jj + 1) / 4; c < 4; ++c)
              qv[(jj + 1) & 1][c] = *reinterpret_cast<const f4*>(qb + (jj + 1) * 20 + 4 * c);
          }
          const f4(&q)[4] = qv[jj & 1];
          const float uj = ur[jj / 4][jj % 4];
          const float iv = q[jj / 4][jj % 4];
          // off the chain: a zero 1 / Q_jj sets the coordinate to 0, and a
          // row that does not run keeps u_j (clamped to [u_j, u_j])
          const float u0 = iv != 0.f ? uj : 0.f;
          const float lo = run ? 0.f : uj, hi = run ? ubnd : uj;
          // (a non-finite step comes from a non-finite g, caught by the
          // stopping test's guard after the sweep)
          const float x = __builtin_fmaf(-gr[jj / 4][jj % 4], iv, u0);
          const float v = __builtin_amdgcn_fmed3f(x, lo, hi);
          const float dl = v - uj;
          ur[jj / 4][jj % 4] = v;
          // the later coordinates of the block see the step
#pragma unroll
          for (int l = jj + 1; l < 16; ++l)
            if (l < nj) gr[l / 4][l % 4] = __builtin_fmaf(dl, q[l / 4][l % 4], gr[l / 4][l % 4]);
          // one coordinate at a time (hoisting the later rows' reads would
          // outgrow the registers)
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      // the new values back to the operand layout; the step of the block
      if (lane < NR) {
#pragma unroll
        for (int c = 0; c < 4; ++c) *reinterpret_cast<f4*>(X + cd_chunk(lane, c)) = ur[c];
      }
      f4 dlt[RQ];
#pragma unroll
      for (int r = 0; r < RQ; ++r) {
        const f4 nb = *reinterpret_cast<const f4*>(X + cd_chunk(16 * r + m, g));
        dlt[r] = nb - ub[b][r];
        ub[b][r] = nb;
      }
      // g_bb += delta_b Q_{b, bb} for every block (the operand: Q[16 bb +
      // m][16 b + 4 g + e], by symmetry)
#pragma unroll
      for (int bb = 0; bb < NBK; ++bb) {
        const f4 a = *reinterpret_cast<const f4*>(sq + (16 * bb + m) * QS + 16 * b + 4 * g);
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int r = 0; r < RQ; ++r)
            gb[bb][r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], dlt[r][e], gb[bb][r], 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  int used = 0;
  bool fell_back = false;
  float res = INFINITY;   // a listed row is pending
  // g of the start.  A listed row resumes (pending).  In the first pass
  // with a warm start: the warm start's g and test, then (unless every row
  // keeps its finite warm start, within tolerance) the cold start's, then
  // (rows mixed) g of the chosen starts.  Each phase loads every row anew.
  const bool cand = rmap == nullptr && start != nullptr;
  const float* src0 = cand ? start : U;
  const float* src1 = nullptr;
  unsigned long long take = 0ull;
  bool ok = valid;
  float gw = 0.f, res_w = 0.f;
  for (int phase = 0;; ++phase) {
    load_ub(src0, src1, take);
    if (cand && phase == 0) {
      // a row is finite when none of its four lanes' values is not
      unsigned long long bad[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
      for (int r = 0; r < RQ; ++r) {
        bool fin = true;
#pragma unroll
        for (int b = 0; b < NBK; ++b)
#pragma unroll
          for (int e = 0; e < 4; ++e) fin = fin && isfinite(ub[b][r][e]);
        bad[r] = __ballot(!fin);
      }
      const int rr = lane >> 4, mm = lane & 15;
      const unsigned long long br = rr == 0 ? bad[0] : rr == 1 ? bad[1] : rr == 2 ? bad[2] : bad[3];
      const unsigned long long mine = (br >> mm) | (br >> (mm + 16)) | (br >> (mm + 32)) | (br >> (mm + 48));
      ok = ok && !(mine & 1ull);
    }
    form_g();
    if (rmap != nullptr) {
      used = valid && pass.used != nullptr ? pass.used[myrow] : 0;
      break;
    }
    if (phase == 2) break;
    const float r = kkt(cand && phase == 0 ? gw : gd);
    if (!cand) {
      res = r;
      break;
    }
    if (phase == 0) {
      res_w = r;
      res = r;
      if (!__any(valid && !(ok && res_w <= tol))) break;
      src0 = C;
      continue;
    }
    // a finite warm start within tolerance is kept; otherwise the
    // candidate with the smaller residual
    const bool warm = ok && (res_w <= tol || res_w < r);
    fell_back = valid && !warm;
    res = warm ? res_w : r;
    take = __ballot(warm);
    if (take == 0ull) break;
    src1 = start;
  }
  int here = 0;
  bool pend = false;
  for (;;) {
    if (valid) pend = res > tol;
    const bool run = valid && pend && used < max_sweeps && here < pass.budget;
    if (!__any(run)) break;
    sweep(run);
    if (run) {
      ++used;
      ++here;
    }
    res = kkt(gd);
  }
  const unsigned long long badm = __ballot(gd != gd);
  const f4 nanv = f4{__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""), __builtin_nanf("")};
#pragma unroll
  for (int b = 0; b < NBK; ++b)
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
      const int c = 16 * b + 4 * g;
      if (roff[r] >= 0 && c < k) *reinterpret_cast<f4*>(U + roff[r] + c) = (badm >> (16 * r + m)) & 1ull ? nanv : ub[b][r];
    }
  const bool keep = valid && pend && used < max_sweeps && pass.wave_cnt != nullptr;
  if (valid) {
    if (pass.used != nullptr) pass.used[myrow] = used;
    if (pass.flags != nullptr) {
      const int32_t unconv = !keep && pend ? 1 : 0;
      if (rmap == nullptr) pass.flags[myrow] = (fell_back ? 2 : 0) | unconv;
      else if (unconv) pass.flags[myrow] |= 1;
    }
  }
  if (pass.wave_cnt != nullptr) {
    const unsigned long long mk = __ballot(keep);
    const int rank = __popcll(mk & ((1ull << lane) - 1ull));
    if (keep) pass.wave_rows[wave * 64 + rank] = static_cast<int32_t>(myrow);
    if (lane == 0) pass.wave_cnt[wave] = __popcll(mk);
  }
}

// list[wave_off[w] + r] = wave_rows[64 w + r] for r < wave_cnt[w]: the rows
// left pending, in wave order.
__global__ __launch_bounds__(256) void tol_compact_kernel(const int32_t* __restrict__ wave_cnt,
                                                          const int32_t* __restrict__ wave_off,
                                                          const int32_t* __restrict__ wave_rows,
                                                          int64_t nwaves, int32_t* __restrict__ list) {
  const int64_t t = blockIdx.x * 256ll + threadIdx.x;
  const int64_t w = t >> 6;
  const int r = static_cast<int>(t & 63);
  if (w < nwaves && r < wave_cnt[w]) list[wave_off[w] + r] = wave_rows[t];
}

// counters += (sum of used, rows with bit 0, rows with bit 1) over all rows.
// Integer sums, so the order does not matter: each block sums a grid-stride
// share through its waves and adds it with one atomic per counter.
__global__ __launch_bounds__(256) void tol_stats_kernel(const int32_t* __restrict__ used,
                                                        const int32_t* __restrict__ flags,
                                                        int64_t rows,
                                                        unsigned long long* __restrict__ counters) {
  __shared__ unsigned long long part[3][4];
  unsigned long long a = 0, b = 0, f = 0;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < rows; i += gridDim.x * 256ll) {
    a += static_cast<unsigned long long>(used[i]);
    b += flags[i] & 1;
    f += (flags[i] >> 1) & 1;
  }
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
    f += __shfl_xor(f, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[0][w] = a;
    part[1][w] = b;
    part[2][w] = f;
  }
  __syncthreads();
  if (threadIdx.x < 3)
    atomicAdd(&counters[threadIdx.x], part[threadIdx.x][0] + part[threadIdx.x][1] + part[threadIdx.x][2] +
                                          part[threadIdx.x][3]);
}

// One projected-gradient step (eq. gradient_descent), every coordinate from
// the old iterate: u_j <- max(u_j - 2 eta ((u G)_j - r_j), 0), with
// eta = 1 / (2 (L + mu)), L = max_j sum_l |G_lj| (at most the inverse
// Lipschitz constant of the sketched gradient 2 (U G - R)).  The new values
// replace r in the panel and leave through it.
template <int KC, int W, int SW>
__global__ __launch_bounds__(64) void pgd_kernel(const float* __restrict__ gp,
                                                 const float* __restrict__ gdiag,
                                                 const float* __restrict__ colsum,
                                                 const float* __restrict__ R, float* U,
                                                 int64_t rows, int k, float mu, float upper) {
  constexpr int NB = RowBlocks<KC, W>::NB, BPP = SW / W, NP = (KC + SW - 1) / SW;
  __shared__ float panel[Panel<SW>::WORDS];
  const int64_t row0 = blockIdx.x * 64ll;
  const int nrows = static_cast<int>(rows - row0 < 64 ? rows - row0 : 64);
  float* mine = panel + threadIdx.x * Panel<SW>::STR;
  RowBlocks<KC, W> u;
  load_rows<KC, W, SW>(panel, U, row0, nrows, k, true, u);
  float L = 0.f;
#pragma unroll
  for (int j = 0; j < KC; ++j) L = fmaxf(L, colsum[j]);
  const float two_eta = 1.0f / (L + mu);
  const float ub = upper > 0.f ? upper : INFINITY;
#pragma unroll
  for (int pc = 0; pc < NP; ++pc) {
    lds_order();
    stage<SW, false>(panel, R, nullptr, 0.f, row0, nrows, k, pc * SW);
    lds_order();
#pragma unroll
    for (int b = 0; b < BPP; ++b) {
      const int jb = pc * BPP + b;
      if (jb < NB) {
        const int jn = (jb + 1) * W <= KC ? W : KC - jb * W;
#pragma nounroll
        for (int je = 0; je < jn; ++je) {
          const int j = jb * W + je;
          const float uj = u.b[jb][je];
          const float g = dot_row<KC, W>(gp + j * KC, u) + gdiag[j] * uj - mine[b * W + je];
          // max(x, 0) that keeps a NaN (and makes -Inf a NaN): x - x is 0
          // for finite x and NaN otherwise
          const float x = uj - two_eta * g;
          mine[b * W + je] = x > 0.f ? fminf(x, ub) : x - x;
        }
      }
    }
    lds_order();
    unstage<SW>(panel, U, row0, nrows, k, pc * SW);
  }
}

template <int KC, int W, int SW>
dsanls_status run_kc(bool pgd, const float* G, const float* R, const float* C, float* U,
                     int64_t rows, int k, float mu, int sweeps, float tol, int max_sweeps,
                     float upper, int32_t* sweeps_used, const TolWork* tw, void* ws, hipStream_t s,
                     const float* start) {
  static_assert(SW % W == 0, "a panel holds whole register blocks");
  Prep p = carve_prep(ws, KC);
  prep_kernel<<<KC, 64, 0, s>>>(G, k, KC, mu, p.gp, p.gdiag, p.den, p.inv, p.colsum);
  DSANLS_LAUNCHED("prep_kernel");
  if (rows == 0) return DSANLS_OK;
  const int64_t nw = ceil_div(rows, 64);
  const unsigned grid = static_cast<unsigned>(nw);
  // NNLS workgroups of four waves (64 rows each) sharing the Gram in LDS:
  // two workgroups share a CU, so the two waves on a SIMD come from
  // different workgroups and do not wait for the LDS in step (eight waves
  // in one workgroup: 1.57x slower at k = 100; two waves, one wave per
  // SIMD: 2.7x slower)
  constexpr int NWV = 4;
  const unsigned gl = static_cast<unsigned>(ceil_div(nw, NWV));
  if (pgd) {
    pgd_kernel<KC, W, SW><<<grid, 64, 0, s>>>(p.gp, p.gdiag, p.colsum, R, U, rows, k, mu, upper);
    DSANLS_LAUNCHED("pgd_kernel");
    return DSANLS_OK;
  }
  if constexpr (KC == 96 || KC == 100) {
    if (sweeps > 0 && k % 4 == 0 && ((reinterpret_cast<uintptr_t>(U) | reinterpret_cast<uintptr_t>(p.gp)) & 15) == 0) {
      constexpr int NM = MfmaCd<KC>::NWV;
      prox_cd_mfma_kernel<KC><<<static_cast<unsigned>(ceil_div(nw, NM)), 64 * NM, 0, s>>>(
          p.gp, p.inv, R, C, U, rows, k, mu, sweeps, upper, sweeps_used);
      DSANLS_LAUNCHED("prox_cd_mfma_kernel");
      return DSANLS_OK;
    }
  }
  if (sweeps > 0) {
    prox_cd_lds_kernel<KC, W, SW, NWV><<<gl, 64 * NWV, 0, s>>>(p.gp, p.inv, R, C, U, rows, k, mu, sweeps, upper,
                                                               sweeps_used);
    DSANLS_LAUNCHED("prox_cd_lds_kernel");
    return DSANLS_OK;
  }
  // one pass of the to-tolerance solve: in the block form carrying the
  // gradient (coupling on the matrix cores) where the fixed sweeps take the
  // block form and every row source is 16-byte aligned, else one dot
  // product per coordinate
  // row quarters (16 rows) per wave of prox_cd_grad_tol_kernel (waves of
  // 16 rows in the passes after the first cut a wave's latency per sweep
  // but cost throughput where many rows remain: slower overall on the
  // sparse text workload)
  constexpr int kRQ = 4;
  bool block = false;
  if constexpr (KC == 96 || KC == 100) {
    const uintptr_t al = reinterpret_cast<uintptr_t>(U) | reinterpret_cast<uintptr_t>(C) |
                         reinterpret_cast<uintptr_t>(start) | reinterpret_cast<uintptr_t>(p.gp) |
                         reinterpret_cast<uintptr_t>(R) |
                         reinterpret_cast<uintptr_t>(tw != nullptr ? tw->centre : nullptr);
    block = k % 4 == 0 && (al & 15) == 0;
  }
  const float* Rq = R;
  bool qc = true;
  auto tol_pass = [&](const TolPass& ps, const float* Cc) -> dsanls_status {
    if constexpr (KC == 96 || KC == 100) {
      if (block) {
        // waves per workgroup of prox_cd_grad_tol_kernel: two (a workgroup
        // holds its LDS until its last wave ends, so with one wave per SIMD a
        // slow wave keeps fewer SIMDs idle than with four: 75.3 vs 71.8 it/s
        // on the sparse warm-start workload, cold)
        constexpr int NG = 2;
        const unsigned gg = static_cast<unsigned>(ceil_div(ceil_div(rows, 16 * kRQ), NG));
        if (qc)
          prox_cd_grad_tol_kernel<KC, true, kRQ><<<gg, 64 * NG, 0, s>>>(
              p.gp, p.den, p.inv, Rq, Cc, start, U, rows, k, mu, tol, max_sweeps, upper, ps);
        else
          prox_cd_grad_tol_kernel<KC, false, kRQ><<<gg, 64 * NG, 0, s>>>(
              p.gp, p.den, p.inv, Rq, Cc, start, U, rows, k, mu, tol, max_sweeps, upper, ps);
        DSANLS_LAUNCHED("prox_cd_grad_tol_kernel");
        return DSANLS_OK;
      }
    }
    prox_cd_tol_kernel<KC, W, SW, NWV><<<gl, 64 * NWV, 0, s>>>(p.gp, p.den, p.inv, R, Cc, start, U, rows, k,
                                                               mu, tol, max_sweeps, upper, ps);
    DSANLS_LAUNCHED("prox_cd_tol_kernel");
    return DSANLS_OK;
  };
  if (tw == nullptr) {
    // one pass to the end (no compaction workspace)
    const TolPass one{nullptr, nullptr, max_sweeps, sweeps_used, nullptr, nullptr, nullptr};
    return tol_pass(one, C);
  }
  // passes with budgets 8, 8, 16, 32, 64, ... sweeps (on the sparse text
  // workload 8% faster than 16, 16, 32, ...; 4, 4, 8, ... and 32, 32, 64,
  // ... were slower); the last pass runs to max_sweeps and lists nothing.
  // Each pass writes U, so a centre that aliases U is copied first.
  if (block) {
    // q = r + mu c once for all passes (each pass reads it when it forms
    // the gradient)
    const int64_t n4 = rows * k / 4;
    const unsigned qg = static_cast<unsigned>(std::min<int64_t>(ceil_div(n4, 256), 4096));
    qsum_kernel<<<qg, 256, 0, s>>>(reinterpret_cast<const float4*>(R), reinterpret_cast<const float4*>(C), mu, n4,
                                   reinterpret_cast<float4*>(tw->centre));
    DSANLS_LAUNCHED("qsum_kernel");
    Rq = tw->centre;
    qc = false;
  } else if (C == U) {
    DSANLS_HIP(hipMemcpyAsync(tw->centre, C, sizeof(float) * rows * k, hipMemcpyDeviceToDevice, s));
    C = tw->centre;
  }
  // waves of the passes (16 kRQ rows in the block form; every wave has 64
  // slots in wave_rows)
  auto waves = [&](int) -> int64_t { return block ? ceil_div(rows, 16 * kRQ) : nw; };
  int budget = 8, spent = 0;
  for (int pass_no = 0;; ++pass_no) {
    const bool last = spent + budget >= max_sweeps;
    const int64_t nwp = waves(pass_no);
    TolPass ps{pass_no == 0 ? nullptr : tw->list[pass_no & 1], pass_no == 0 ? nullptr : tw->wave_off + waves(pass_no - 1),
               last ? max_sweeps : budget, tw->used, tw->flags, last ? nullptr : tw->wave_cnt, tw->wave_rows};
    dsanls_status st = tol_pass(ps, C);
    if (st != DSANLS_OK) return st;
    if (last) break;
    st = launch_exclusive_scan(tw->wave_cnt, tw->wave_off, nwp, tw->scan_ws, s);
    if (st != DSANLS_OK) return st;
    tol_compact_kernel<<<static_cast<unsigned>(ceil_div(nwp * 64, 256)), 256, 0, s>>>(
        tw->wave_cnt, tw->wave_off, tw->wave_rows, nwp, tw->list[(pass_no + 1) & 1]);
    DSANLS_LAUNCHED("tol_compact_kernel");
    spent += budget;
    if (pass_no > 0) budget *= 2;
  }
  if (tw->counters != nullptr) {
    const unsigned sg = static_cast<unsigned>(std::min<int64_t>(ceil_div(rows, 1024), 1024));
    tol_stats_kernel<<<sg, 256, 0, s>>>(tw->used, tw->flags, rows, tw->counters);
    DSANLS_LAUNCHED("tol_stats_kernel");
  }
  if (sweeps_used != nullptr)
    DSANLS_HIP(hipMemcpyAsync(sweeps_used, tw->used, sizeof(int32_t) * rows, hipMemcpyDeviceToDevice, s));
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

constexpr int kMaxK = kNnlsMaxRank;

size_t nnls_ws_bytes(int k) {
  const int kc = k > kMaxK ? nnls_kc_wide(k) : nnls_kc(k < 1 ? 1 : k);
  return sizeof(float) * prep_floats(kc > 0 ? kc : kMaxKC);
}

namespace {

// Ranks 129 .. kNnlsMaxRankWide: the Gram prepared at the padded rank of the
// wide kernel (fixed sweeps of prox-CD only).
dsanls_status run_wide(bool pgd, const float* G, const float* R, const float* C, float* U, int64_t rows, int k,
                       float mu, int sweeps, float upper, int32_t* sweeps_used, void* ws, hipStream_t s) {
  if (pgd || sweeps < 1)
    return fail(DSANLS_E_UNSUPPORTED, "ranks above 128 support prox-CD with a fixed number of sweeps only");
  const int KC = nnls_kc_wide(k);
  Prep p = carve_prep(ws, KC);
  prep_kernel<<<KC, 64, 0, s>>>(G, k, KC, mu, p.gp, p.gdiag, p.den, p.inv, p.colsum);
  DSANLS_LAUNCHED("prep_kernel");
  return launch_prox_cd_wide(p.gp, p.inv, KC, R, C, U, rows, k, mu, sweeps, upper, sweeps_used, s);
}

}  // namespace

dsanls_status launch_nnls(bool pgd, const float* G, const float* R, const float* C, float* U,
                          int64_t rows, int k, float mu, int sweeps, float tol, int max_sweeps,
                          float upper, int32_t* sweeps_used, const TolWork* tw, void* ws,
                          size_t ws_bytes, hipStream_t s, const float* start) {
  if (k < 1 || k > kNnlsMaxRankWide) return fail(DSANLS_E_UNSUPPORTED, "NNLS supports 1 <= k <= 512");
  if (ws_bytes < nnls_ws_bytes(k)) return fail(DSANLS_E_WORKSPACE, "NNLS workspace too small");
  if (k > kMaxK) return run_wide(pgd, G, R, C, U, rows, k, mu, sweeps, upper, sweeps_used, ws, s);
  switch (nnls_kc(k)) {
#define DSANLS_KC(KC, W, SW)                                                                         \
  case KC:                                                                                           \
    return run_kc<KC, W, SW>(pgd, G, R, C, U, rows, k, mu, sweeps, tol, max_sweeps, upper,          \
                             sweeps_used, tw, ws, s, start);
    DSANLS_KC(4, 4, 4)
    DSANLS_KC(8, 8, 8)
    DSANLS_KC(10, 16, 16)
    DSANLS_KC(16, 16, 16)
    DSANLS_KC(32, 16, 16)
    DSANLS_KC(48, 16, 16)
    DSANLS_KC(64, 16, 16)
    DSANLS_KC(96, 16, 16)
    DSANLS_KC(100, 16, 16)
    DSANLS_KC(128, 16, 16)
#undef DSANLS_KC
  }
  return fail(DSANLS_E_UNSUPPORTED, "NNLS: no kernel for this k");
}

}  // namespace dsanls

using namespace dsanls;

extern "C" size_t dsanls_nnls_workspace_bytes(int32_t k) {
  return k < 1 || k > kNnlsMaxRankWide ? 0 : align_up(nnls_ws_bytes(k), 256);
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
