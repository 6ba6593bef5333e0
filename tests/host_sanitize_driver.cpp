// Host-only driver for the sanitizer build of the library's host code: runs
// the argument checks and workspace planning of the C ABI over a grid of
// configurations (dense and CSR matrices, every sketch and solver, fixed
// sweeps and to-tolerance, node shares, warm-start sizes) and the error
// paths of the entry points that return before any device call.  Device
// pointers are opaque, non-null values that the host code never reads.
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "dsanls.h"

int main() {
  const float* fake = reinterpret_cast<const float*>(uintptr_t{0x10000});
  dsanls_matrix dense;
  std::memset(&dense, 0, sizeof dense);
  dense.format = DSANLS_DENSE;
  dense.dense = fake;
  dsanls_matrix csr;
  std::memset(&csr, 0, sizeof csr);
  csr.format = DSANLS_CSR;
  csr.rowptr = reinterpret_cast<const int64_t*>(fake);
  csr.colidx = reinterpret_cast<const int32_t*>(fake);
  csr.vals = fake;
  csr.t_rowptr = reinterpret_cast<const int64_t*>(fake);
  csr.t_colidx = reinterpret_cast<const int32_t*>(fake);
  csr.t_vals = fake;
  long ok = 0, rejected = 0;
  const int64_t shapes[][2] = {{1, 1}, {200, 150}, {5000, 3000}, {500000, 200000}};
  for (const auto& sh : shapes)
    for (int fmt = 0; fmt < 2; ++fmt)
      for (int64_t k : {1, 10, 33, 100, 128, 129, 300, 512, 513})
        for (int sk = 0; sk < 5; ++sk)
          for (int sol = 0; sol < 2; ++sol)
            for (int sweeps : {0, 1, 3})
              for (int hidden : {0, 256})
                for (int share = 0; share < 2; ++share) {
                  dsanls_config c;
                  std::memset(&c, 0, sizeof c);
                  c.m = sh[0];
                  c.n = sh[1];
                  c.k = k;
                  c.d = sk == DSANLS_SKETCH_IDENTITY ? c.n : (c.n > 40 ? 40 : c.n);
                  c.d_prime = sk == DSANLS_SKETCH_IDENTITY ? c.m : (c.m > 40 ? 40 : c.m);
                  c.sketch = sk;
                  c.solver = sol;
                  c.sweeps = sweeps;
                  c.max_sweeps = 100;
                  c.tol = 1e-4f;
                  c.alpha = 0.1f;
                  c.beta = 1.f;
                  c.warm_hidden = hidden;
                  if (share) {
                    c.row_offset = c.m;
                    c.col_offset = 0;
                    c.m_global = 2 * c.m;
                    c.n_global = c.n;
                  }
                  dsanls_matrix M = fmt ? csr : dense;
                  if (fmt) M.nnz = c.m * 3; else M.ld = c.n;
                  size_t bytes = 0;
                  if (dsanls_workspace_bytes(&c, &M, &bytes) == DSANLS_OK) {
                    ++ok;
                    if (bytes == 0 || bytes % 256 != 0) {
                      std::printf("bad workspace size %zu\n", bytes);
                      return 1;
                    }
                  } else {
                    ++rejected;
                    if (std::strlen(dsanls_last_error()) == 0) return 1;
                  }
                }
  // error paths that return before any device call
  dsanls_config c;
  std::memset(&c, 0, sizeof c);
  c.m = 200; c.n = 150; c.k = 10; c.d = 40; c.d_prime = 40; c.sweeps = 1; c.max_sweeps = 100;
  c.tol = 1e-4f; c.alpha = 0.1f; c.beta = 1.f;
  dense.ld = 150;
  size_t need = 0;
  if (dsanls_workspace_bytes(&c, &dense, &need) != DSANLS_OK) return 2;
  if (dsanls_workspace_bytes(nullptr, &dense, &need) == DSANLS_OK) return 3;
  if (dsanls_workspace_bytes(&c, &dense, nullptr) == DSANLS_OK) return 4;
  dsanls_ctx* ctx = nullptr;
  float* U = const_cast<float*>(fake);
  if (dsanls_init(&c, &dense, U, U, nullptr, need, nullptr, &ctx) == DSANLS_OK || ctx != nullptr) return 5;
  void* ws = reinterpret_cast<void*>(uintptr_t{0x20000});
  if (dsanls_init(&c, &dense, U, U, ws, need - 1, nullptr, &ctx) == DSANLS_OK || ctx != nullptr) return 6;
  if (dsanls_init(&c, &dense, nullptr, U, ws, need, nullptr, &ctx) == DSANLS_OK || ctx != nullptr) return 7;
  if (dsanls_sketch_update_U(nullptr, 0) == DSANLS_OK) return 8;
  if (dsanls_destroy(nullptr) == DSANLS_OK) return 9;
  std::printf("sanitized host checks: %ld accepted, %ld rejected\n", ok, rejected);
  return 0;
}
