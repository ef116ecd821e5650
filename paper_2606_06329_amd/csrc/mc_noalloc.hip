// mc_curvature_fast_noalloc: mc_curvature_fast for callers that cannot allocate (code under
// HIP graph capture, tight serving loops).  The two-pass kernels' per-point state lives in a
// file-scope device array of MC_NOALLOC_SCRATCH_BYTES instead of a caller workspace.
//
// The array's name is a host-side stand-in in host code, not a device address: the address
// is taken once per device with hipGetSymbolAddress (with that device current) on the
// entry point's first call there, and only that pointer is ever handed to the kernels.
#include <mutex>

#include <hip/hip_runtime.h>

#include "../../include/mecuco.h"

namespace {

__device__ __align__(256) unsigned char scratch[MC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// This device's copy of the scratch array (nullptr if its address cannot be taken).
void* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" int mc_curvature_fast_noalloc(const float* X, int64_t n, int64_t m, int64_t ldx,
                                         const int32_t* idx, int32_t k, int32_t precision,
                                         int32_t variant, uint32_t flags, float* kappa_out,
                                         uint8_t* flags_out, void* stream) {
  const size_t need = mc_workspace_bytes(MC_OP_FAST, n, m, k, precision, 1);
  if (need == 0) {
    // invalid or unsupported sizes: the regular entry point returns the precise code
    return mc_curvature_fast(X, n, m, ldx, idx, k, precision, variant, flags, kappa_out, flags_out,
                             nullptr, 0, stream);
  }
  if (need > (size_t)MC_NOALLOC_SCRATCH_BYTES) return MC_ESCRATCH;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return MC_EDEVICE;
  }
  void* ws = scratch_ptr(dev);
  if (!ws) return MC_EDEVICE;
  return mc_curvature_fast(X, n, m, ldx, idx, k, precision, variant, flags, kappa_out, flags_out, ws,
                           (size_t)MC_NOALLOC_SCRATCH_BYTES, stream);
}
