// extern "C" entry points of libmecuco.so: argument validation (host only, before
// anything is enqueued), workspace sizing, dispatch to the gfx950 kernels.
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "../../include/mecuco.h"
#include "mc_internal.h"

namespace {

constexpr int64_t kIdxMax = 2147483647;  // neighbour indices are int32

bool misaligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) != 0; }

// Shared checks of the (X, n, m, ldx, k) description of a point cloud.
int check_cloud(const float* X, int64_t n, int64_t m, int64_t ldx, int32_t k) {
  if (!X) return MC_EINVAL;
  if (n <= 0 || m <= 0 || ldx < m) return MC_EINVAL;
  if (k < 2 || k > MC_KMAX || (int64_t)k >= n) return MC_EINVAL;
  if (n > kIdxMax) return MC_ESHAPE;
  int64_t elems = 0;
  if (__builtin_mul_overflow(n, ldx, &elems)) return MC_ESHAPE;   // n x ldx floats addressable
  return MC_OK;
}

int check_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return MC_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MC_EDEVICE;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return MC_EDEVICE;
  return MC_OK;
}

int strict_check(const uint8_t* flags, int64_t n, uint8_t mask, hipStream_t s) {
  if (!flags) return MC_OK;
  if (hipStreamSynchronize(s) != hipSuccess) return MC_ELAUNCH;
  // copy in bounded chunks to a small host buffer
  uint8_t buf[4096];
  for (int64_t o = 0; o < n; o += (int64_t)sizeof(buf)) {
    const size_t c = (size_t)((n - o) < (int64_t)sizeof(buf) ? (n - o) : (int64_t)sizeof(buf));
    if (hipMemcpy(buf, flags + o, c, hipMemcpyDeviceToHost) != hipSuccess) return MC_ELAUNCH;
    for (size_t t = 0; t < c; ++t)
      if (buf[t] & mask) return MC_ENUMERIC;
  }
  return MC_OK;
}

}  // namespace

extern "C" {

int mc_version(void) { return MC_VERSION; }

const char* mc_status_string(int status) {
  switch (status) {
    case MC_OK: return "ok";
    case MC_EINVAL: return "invalid argument (null pointer, k out of [2, 32] or >= n, n or m <= 0, ldx < m, bad enum)";
    case MC_ESHAPE: return "size beyond a supported range (int32 indices; on-chip buffers of exact mode, float64 Fast mode or the adjoint)";
    case MC_EPRECISION: return "precision not available for this operation";
    case MC_EWORKSPACE: return "workspace too small or not 256-byte aligned";
    case MC_ELAUNCH: return "kernel launch failed";
    case MC_ENUMERIC: return "MC_STRICT: a point carries a numerical flag";
    case MC_EDEVICE: return "no gfx950 device is current";
    case MC_ESCRATCH: return "sizes need more per-point state than the static scratch of the no-allocation entry point (MC_NOALLOC_SCRATCH_BYTES)";
    default: return "unknown status";
  }
}

size_t mc_workspace_bytes(int32_t op, int64_t n, int64_t m, int32_t k, int32_t precision,
                          int32_t rerank_factor) {
  if (op == MC_OP_NORMALIZE) return n > 0 ? mc::normalize_ws_bytes() : 0;
  if (n <= 0 || m <= 0 || k < 2 || k > MC_KMAX || (int64_t)k >= n) return 0;
  int64_t elems = 0;   // the calls reject these shapes (ldx >= m, so n x ldx would overflow too)
  if (n > kIdxMax || __builtin_mul_overflow(n, m, &elems)) return 0;
  switch (op) {
    case MC_OP_KNN: {
      if (precision != MC_FP32 && precision != MC_BF16 && precision != MC_FP8) return 0;
      if (rerank_factor < 1 || rerank_factor > 4) return 0;
      const int kc = k * rerank_factor;
      if (kc > 64 || (int64_t)kc >= n) return 0;
      return mc::knn_plan(n, m, k, kc, precision).total;
    }
    case MC_OP_FAST:
      if (precision != MC_FP32 && precision != MC_BF16 && precision != MC_FP64) return 0;
      if (precision == MC_FP64 && k > MC_FAST_FP64_KMAX) return 0;
      // the single-pass kernel keeps everything on chip; the two-pass form hands per-point
      // k x k state between its kernels
      return k <= mc::FAST_SINGLE_PASS_KMAX ? 256 : mc::curv_fast2_ws_bytes(n, k, precision);
    case MC_OP_EXACT:
      if (!mc::curv_exact_fits(m, k)) return 0;
      return mc::curv_exact_ws_bytes(n, m, k);
    case MC_OP_BACKWARD:
      if (k > 16) return 0;
      return 256;
    default:
      return 0;
  }
}

int mc_knn(const float* X, int64_t n, int64_t m, int64_t ldx, int32_t k, int32_t precision,
           int32_t rerank_factor, uint32_t flags, int32_t* idx_out, float* d2_out,
           uint8_t* knn_flags, void* ws, size_t ws_bytes, void* stream) {
  int st = check_cloud(X, n, m, ldx, k);
  if (st) return st;
  if (!idx_out || !ws) return MC_EINVAL;
  if (flags & ~(MC_INCLUDE_SELF | MC_STRICT)) return MC_EINVAL;
  if (precision == MC_FP64) return MC_EPRECISION;
  if (precision != MC_FP32 && precision != MC_BF16 && precision != MC_FP8) return MC_EINVAL;
  if (rerank_factor < 1 || rerank_factor > 4) return MC_EINVAL;
  const int kc = k * rerank_factor;
  if (kc > 64 || (int64_t)kc >= n) return MC_EINVAL;
  if (precision != MC_FP32 && rerank_factor < 2) return MC_EINVAL;
  const mc::KnnPlan plan = mc::knn_plan(n, m, k, kc, precision);
  if (ws_bytes < plan.total || misaligned(ws)) return MC_EWORKSPACE;
  st = check_device();
  if (st) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (mc::launch_knn(X, n, m, ldx, k, kc, precision, (flags & MC_INCLUDE_SELF) != 0, idx_out,
                     d2_out, knn_flags, ws, plan, s) != hipSuccess)
    return MC_ELAUNCH;
  if (flags & MC_STRICT) return strict_check(knn_flags, n, (uint8_t)~MC_PF_KNN_AMBIGUOUS, s);
  return MC_OK;
}

int mc_curvature_fast(const float* X, int64_t n, int64_t m, int64_t ldx, const int32_t* idx,
                      int32_t k, int32_t precision, int32_t variant, uint32_t flags,
                      float* kappa_out, uint8_t* flags_out, void* ws, size_t ws_bytes,
                      void* stream) {
  int st = check_cloud(X, n, m, ldx, k);
  if (st) return st;
  if (!idx || !kappa_out) return MC_EINVAL;
  if (variant != MC_FAST_PAPER && variant != MC_FAST_HAAR) return MC_EINVAL;
  if (flags & ~MC_STRICT) return MC_EINVAL;
  if (precision != MC_FP32 && precision != MC_BF16 && precision != MC_FP64) {
    return precision == MC_FP8 ? MC_EPRECISION : MC_EINVAL;
  }
  if (precision == MC_FP64 && k > MC_FAST_FP64_KMAX) return MC_ESHAPE;
  if (k > mc::FAST_SINGLE_PASS_KMAX) {
    if (!ws) return MC_EINVAL;
    if (ws_bytes < mc::curv_fast2_ws_bytes(n, k, precision) || misaligned(ws)) return MC_EWORKSPACE;
  }
  st = check_device();
  if (st) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (mc::launch_curv_fast(X, n, m, ldx, idx, k, precision, variant, kappa_out, flags_out, ws, s) !=
      hipSuccess)
    return MC_ELAUNCH;
  if (flags & MC_STRICT) return strict_check(flags_out, n, (uint8_t)~MC_PF_EIGEN_FP64, s);
  return MC_OK;
}

int mc_curvature_exact(const float* X, int64_t n, int64_t m, int64_t ldx, const int32_t* idx,
                       int32_t k, int32_t precision, uint32_t flags, float* kappa_out,
                       uint8_t* flags_out, void* ws, size_t ws_bytes, void* stream) {
  int st = check_cloud(X, n, m, ldx, k);
  if (st) return st;
  if (!idx || !kappa_out || !ws) return MC_EINVAL;
  if (flags & ~MC_STRICT) return MC_EINVAL;
  if (precision != MC_FP32) {
    return (precision == MC_BF16 || precision == MC_FP8 || precision == MC_FP64) ? MC_EPRECISION
                                                                                : MC_EINVAL;
  }
  if (ws_bytes < mc::curv_exact_ws_bytes(n, m, k) || misaligned(ws)) return MC_EWORKSPACE;
  if (!mc::curv_exact_fits(m, k)) return MC_ESHAPE;
  st = check_device();
  if (st) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (mc::launch_curv_exact(X, n, m, ldx, idx, k, kappa_out, flags_out, ws, s) != hipSuccess)
    return MC_ELAUNCH;
  if (flags & MC_STRICT) return strict_check(flags_out, n, 0xFF, s);
  return MC_OK;
}

int mc_curvature_backward(const float* X, int64_t n, int64_t m, int64_t ldx, const int32_t* idx,
                          int32_t k, int32_t variant, const float* grad_kappa, float gap_eps,
                          float* grad_X, void* ws, size_t ws_bytes, void* stream) {
  int st = check_cloud(X, n, m, ldx, k);
  if (st) return st;
  if (!idx || !grad_kappa || !grad_X) return MC_EINVAL;
  if (variant != MC_FAST_PAPER && variant != MC_FAST_HAAR) return MC_EINVAL;
  if (!(gap_eps >= 0.0f) || gap_eps > 1.0f) return MC_EINVAL;
  if (k > 16) return MC_ESHAPE;   // the adjoint keeps its k x k(k+1)/2 third-moment adjoint in LDS
  (void)ws;
  (void)ws_bytes;
  st = check_device();
  if (st) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (mc::launch_curv_backward(X, n, m, ldx, idx, k, variant, grad_kappa, gap_eps, grad_X, s) !=
      hipSuccess)
    return MC_ELAUNCH;
  return MC_OK;
}

int mc_normalize_minmax(const float* kappa, int64_t n, float* out, void* ws, size_t ws_bytes, void* stream) {
  if (!kappa || !out || !ws || n <= 0) return MC_EINVAL;
  if (ws_bytes < mc::normalize_ws_bytes() || misaligned(ws)) return MC_EWORKSPACE;
  const int st = check_device();
  if (st) return st;
  if (mc::launch_normalize(kappa, n, out, ws, reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
    return MC_ELAUNCH;
  return MC_OK;
}

}  // extern "C"
