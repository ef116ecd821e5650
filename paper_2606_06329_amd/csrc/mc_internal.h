// Internal launcher interface between the C-ABI layer (mc_abi.cpp) and the
// HIP kernels.  Host code only; no device code is declared here.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <atomic>

#include <hip/hip_runtime_api.h>

namespace mc {

// Runs the idempotent `fn` (e.g. a kernel attribute setter) once per device, keyed by the
// current device's ordinal (< 64); thread-safe: concurrent first calls may both run it.
template <class F>
void once_per_device(std::atomic<uint64_t>& done, F fn) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    fn();
    return;
  }
  const uint64_t bit = 1ull << dev;
  if (done.load(std::memory_order_acquire) & bit) return;
  fn();
  done.fetch_or(bit, std::memory_order_release);
}

// Stage timers (mc_timing.cpp): no-ops unless mc_timing_enable(1) was called.
void timing_begin(int stage, hipStream_t s);
void timing_end(int stage, hipStream_t s);

// Workspace layout helpers (bytes, 256-aligned pieces).
inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct KnnPlan {
  int64_t n, m;
  int k, kc;          // neighbours, candidates kept per query (rerank_factor * k)
  int precision;
  int64_t tiles;      // 128-point tiles
  int sym;            // 1: symmetric tile-pair schedule (row side + column side), 0: full
  int64_t pairs_a;    // tile pairs of the GEMM/top-k (row side) stage
  int64_t groups;     // its workgroups
  int smax;           // its list segments reserved per row tile
  int64_t pairs_b;    // transposed tiles of the column-side stage (0 unless sym)
  int64_t groups_b;   // its workgroups
  int smax_b;         // its list segments reserved per column tile
  size_t off_xc, off_norm, off_colsum, off_stats, off_cand_s, off_cand_j, off_xlow, off_scale;
  size_t off_cap, off_thr, off_rescan, off_tbuf, total;
};

KnnPlan knn_plan(int64_t n, int64_t m, int k, int kc, int precision);

// Fast curvature: the fused single-pass kernel (k <= 12, no workspace) or the two-pass
// kernels (k >= 13), which keep per-point k x k state in the workspace.
hipError_t launch_curv_fast(const float* X, int64_t n, int64_t m, int64_t ldx, const int32_t* idx,
                            int k, int precision, int variant, float* kappa, uint8_t* flags, void* ws,
                            hipStream_t stream);
hipError_t launch_curv_fast2(const float* X, int64_t n, int64_t m, int64_t ldx, const int32_t* idx, int k,
                             int precision, int variant, float* kappa, uint8_t* flags, void* ws,
                             hipStream_t stream);
size_t curv_fast2_ws_bytes(int64_t n, int k, int precision);
constexpr int FAST_SINGLE_PASS_KMAX = 12;   // largest k of the single-pass form

hipError_t launch_curv_exact(const float* X, int64_t n, int64_t m, int64_t ldx, const int32_t* idx,
                             int k, float* kappa, uint8_t* flags, void* ws, hipStream_t stream);

size_t curv_exact_ws_bytes(int64_t n, int64_t m, int k);
bool curv_exact_fits(int64_t m, int k);   // patch and V_r fit the exact kernel's LDS

hipError_t launch_curv_backward(const float* X, int64_t n, int64_t m, int64_t ldx,
                                const int32_t* idx, int k, int variant, const float* gk,
                                float gap_eps, float* grad, hipStream_t stream);

// Min-max normalisation of a score vector to [0, 1] (mc_normalize.hip).
size_t normalize_ws_bytes();
hipError_t launch_normalize(const float* kappa, int64_t n, float* out, void* ws, hipStream_t stream);

hipError_t launch_knn(const float* X, int64_t n, int64_t m, int64_t ldx, int k, int kc,
                      int precision, bool include_self, int32_t* idx, float* d2, uint8_t* kflags,
                      void* ws, const KnnPlan& plan, hipStream_t stream);

}  // namespace mc
