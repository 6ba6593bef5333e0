// Allocation-free entry point of the batched NNLS update: the same kernels
// as dsanls_nnls_prox_cd, with the prepared Gram in a file-scope device
// array instead of a caller's workspace.
#include "common.hpp"

#include <mutex>

namespace dsanls {
namespace {

// One copy per device, held until the process ends: the prepared Gram of
// the largest rank the NNLS kernels take.
constexpr size_t kScratchFloats = nnls_prep_floats(kNnlsMaxRank);
__device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (looked up once per device, with
// that device current; the array's name is not a device address on the host).
dsanls_status scratch_for_current_device(float** out) {
  int dev = 0;
  DSANLS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(DSANLS_E_UNSUPPORTED, "nnls_prox_cd_noalloc: device index >= 64");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (p == nullptr) return fail(DSANLS_E_HIP, "nnls_prox_cd_noalloc: scratch has no device address");
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return DSANLS_OK;
}

}  // namespace
}  // namespace dsanls

using namespace dsanls;

extern "C" size_t dsanls_nnls_noalloc_scratch_bytes(void) { return sizeof(float) * kScratchFloats; }

extern "C" dsanls_status dsanls_nnls_prox_cd_noalloc(const float* G, const float* R, const float* C, float* U,
                                                     int64_t rows, int32_t k, float mu, int32_t sweeps, float tol,
                                                     int32_t max_sweeps, float upper, int32_t* sweeps_used,
                                                     void* hip_stream) {
  if (rows < 0 || !G || (rows > 0 && (!R || !C || !U)))
    return fail(DSANLS_E_INVALID_ARG, "nnls_prox_cd_noalloc: null pointer or negative rows");
  if (sweeps < 0 || (sweeps == 0 && (max_sweeps < 1 || !(tol >= 0.f))) || !(mu >= 0.f))
    return fail(DSANLS_E_INVALID_ARG, "nnls_prox_cd_noalloc: bad sweeps/tol/mu");
  if (k < 1 || k > kNnlsMaxRank || nnls_ws_bytes(k) > sizeof(float) * kScratchFloats)
    return fail(DSANLS_E_UNSUPPORTED, "nnls_prox_cd_noalloc: k must be in [1, " + std::to_string(kNnlsMaxRank) +
                                          "] (the prepared Gram must fit the " +
                                          std::to_string(sizeof(float) * kScratchFloats) + "-byte scratch)");
  float* ws = nullptr;
  const dsanls_status st = scratch_for_current_device(&ws);
  if (st != DSANLS_OK) return st;
  return launch_nnls(false, G, R, C, U, rows, k, mu, sweeps, tol, max_sweeps, upper, sweeps_used, nullptr, ws,
                     sizeof(float) * kScratchFloats, static_cast<hipStream_t>(hip_stream));
}
