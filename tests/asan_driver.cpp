// Host-side paths of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer: every
// call below is rejected by the argument checks before any device work, or is a pure query
// (workspace sizes, status and stage strings).  Built and run by test_host_sanitizer.py.
#include <stdint.h>
#include <stdio.h>

#include "mecuco.h"

static int failures = 0;
#define EXPECT(call, code)                                                               \
  do {                                                                                   \
    const int st_ = (call);                                                              \
    if (st_ != (code)) {                                                                 \
      printf("line %d: %s returned %d, expected %d\n", __LINE__, #call, st_, (int)(code)); \
      ++failures;                                                                        \
    }                                                                                    \
  } while (0)

int main() {
  alignas(256) static unsigned char ws_mem[4096];
  float fx[64] = {0};
  int32_t ix[64] = {0};
  float gk[64] = {0};
  void* ws = ws_mem;
  const int64_t big = INT64_MAX / 2;

  // mc_knn
  EXPECT(mc_knn(nullptr, 100, 4, 4, 5, MC_FP32, 2, 0, ix, nullptr, nullptr, ws, 1 << 20, nullptr), MC_EINVAL);
  EXPECT(mc_knn(fx, 100, 4, 4, 5, MC_FP32, 2, 0, nullptr, nullptr, nullptr, ws, 1 << 20, nullptr), MC_EINVAL);
  EXPECT(mc_knn(fx, 100, 4, 2, 5, MC_FP32, 2, 0, ix, nullptr, nullptr, ws, 1 << 20, nullptr), MC_EINVAL);
  EXPECT(mc_knn(fx, 100, 4, 4, 1, MC_FP32, 2, 0, ix, nullptr, nullptr, ws, 1 << 20, nullptr), MC_EINVAL);
  EXPECT(mc_knn(fx, 100, 4, 4, 33, MC_FP32, 2, 0, ix, nullptr, nullptr, ws, 1 << 20, nullptr), MC_EINVAL);
  EXPECT(mc_knn(fx, 100, 4, 4, 5, MC_FP64, 2, 0, ix, nullptr, nullptr, ws, 1 << 20, nullptr), MC_EPRECISION);
  EXPECT(mc_knn(fx, 100, 4, 4, 5, 17, 2, 0, ix, nullptr, nullptr, ws, 1 << 20, nullptr), MC_EINVAL);
  EXPECT(mc_knn(fx, 100, 4, 4, 5, MC_FP32, 5, 0, ix, nullptr, nullptr, ws, 1 << 20, nullptr), MC_EINVAL);
  EXPECT(mc_knn(fx, 100, 4, 4, 5, MC_BF16, 1, 0, ix, nullptr, nullptr, ws, 1 << 20, nullptr), MC_EINVAL);
  EXPECT(mc_knn(fx, 100, 4, 4, 5, MC_FP32, 2, 0x80, ix, nullptr, nullptr, ws, 1 << 20, nullptr), MC_EINVAL);
  EXPECT(mc_knn(fx, 100, 4, 4, 5, MC_FP32, 2, 0, ix, nullptr, nullptr, ws, 16, nullptr), MC_EWORKSPACE);
  EXPECT(mc_knn(fx, 100, 4, 4, 5, MC_FP32, 2, 0, ix, nullptr, nullptr, ws_mem + 8, 1 << 20, nullptr), MC_EWORKSPACE);
  EXPECT(mc_knn(fx, (int64_t)1 << 32, 4, 4, 5, MC_FP32, 2, 0, ix, nullptr, nullptr, ws, 1 << 20, nullptr), MC_ESHAPE);
  EXPECT(mc_knn(fx, 1 << 20, big, big, 5, MC_FP32, 2, 0, ix, nullptr, nullptr, ws, 1 << 20, nullptr), MC_ESHAPE);

  // mc_curvature_fast
  EXPECT(mc_curvature_fast(nullptr, 100, 4, 4, ix, 5, MC_FP32, 0, 0, fx, nullptr, ws, 1 << 20, nullptr), MC_EINVAL);
  EXPECT(mc_curvature_fast(fx, 100, 4, 4, nullptr, 5, MC_FP32, 0, 0, fx, nullptr, ws, 1 << 20, nullptr), MC_EINVAL);
  EXPECT(mc_curvature_fast(fx, 100, 4, 4, ix, 5, MC_FP32, 2, 0, fx, nullptr, ws, 1 << 20, nullptr), MC_EINVAL);
  EXPECT(mc_curvature_fast(fx, 100, 4, 4, ix, 5, MC_FP8, 0, 0, fx, nullptr, ws, 1 << 20, nullptr), MC_EPRECISION);
  EXPECT(mc_curvature_fast(fx, 100, 4, 4, ix, 29, MC_FP64, 0, 0, fx, nullptr, ws, 1 << 20, nullptr), MC_ESHAPE);
  EXPECT(mc_curvature_fast(fx, 100, 4, 4, ix, 20, MC_FP32, 0, 0, fx, nullptr, nullptr, 1 << 20, nullptr), MC_EINVAL);
  EXPECT(mc_curvature_fast(fx, 100, 4, 4, ix, 20, MC_FP32, 0, 0, fx, nullptr, ws, 16, nullptr), MC_EWORKSPACE);
  EXPECT(mc_curvature_fast(fx, 100, 4, 4, ix, 5, MC_FP32, 0, 4, fx, nullptr, ws, 1 << 20, nullptr), MC_EINVAL);

  // mc_curvature_exact
  EXPECT(mc_curvature_exact(fx, 100, 4, 4, ix, 5, MC_BF16, 0, fx, nullptr, ws, 1 << 20, nullptr), MC_EPRECISION);
  EXPECT(mc_curvature_exact(fx, 100, 4, 4, ix, 5, MC_FP32, 0, fx, nullptr, nullptr, 1 << 20, nullptr), MC_EINVAL);
  EXPECT(mc_curvature_exact(fx, 100, 4, 4, ix, 5, MC_FP32, 0, fx, nullptr, ws, 0, nullptr), MC_EWORKSPACE);
  EXPECT(mc_curvature_exact(fx, 100, 100000, 100000, ix, 5, MC_FP32, 0, fx, nullptr, ws, (size_t)1 << 40, nullptr), MC_ESHAPE);

  // mc_curvature_backward
  EXPECT(mc_curvature_backward(fx, 100, 4, 4, ix, 20, 0, gk, 0.0f, fx, ws, 1 << 20, nullptr), MC_ESHAPE);
  EXPECT(mc_curvature_backward(fx, 100, 4, 4, ix, 5, 0, gk, -1.0f, fx, ws, 1 << 20, nullptr), MC_EINVAL);
  EXPECT(mc_curvature_backward(fx, 100, 4, 4, ix, 5, 0, nullptr, 0.0f, fx, ws, 1 << 20, nullptr), MC_EINVAL);
  EXPECT(mc_curvature_backward(fx, 100, 4, 4, ix, 5, 3, gk, 0.0f, fx, ws, 1 << 20, nullptr), MC_EINVAL);

  // mc_normalize_minmax and the no-allocation Fast entry point
  EXPECT(mc_normalize_minmax(nullptr, 10, fx, ws, 4096, nullptr), MC_EINVAL);
  EXPECT(mc_normalize_minmax(fx, 10, fx, ws, 1, nullptr), MC_EWORKSPACE);
  EXPECT(mc_curvature_fast_noalloc(fx, 100, 4, 4, ix, 1, MC_FP32, 0, 0, fx, nullptr, nullptr), MC_EINVAL);

  // pure queries over a grid of sizes, including the edges of every accepted range
  const int64_t ns[] = {-1, 0, 1, 2, 3, 33, 100, 131072, 140000, (int64_t)1 << 31, (int64_t)1 << 40, big};
  const int64_t ms[] = {-1, 0, 1, 20, 784, 4096, 54621, (int64_t)1 << 31, big};
  const int32_t ks[] = {-1, 0, 1, 2, 11, 12, 13, 16, 17, 28, 29, 32, 33};
  size_t sink = 0;
  for (int32_t op = -1; op <= 5; ++op)
    for (int64_t n : ns)
      for (int64_t m : ms)
        for (int32_t k : ks)
          for (int32_t prec = -1; prec <= 4; ++prec)
            for (int32_t rr = 0; rr <= 5; ++rr) sink += mc_workspace_bytes(op, n, m, k, prec, rr);
  for (int s = -2; s <= 12; ++s) sink += (size_t)mc_status_string(s)[0];
  for (int s = -2; s <= MC_STAGE_COUNT + 1; ++s) sink += (size_t)mc_stage_name(s)[0];
  sink += (size_t)mc_version();
  printf("host sanitizer driver: %d failures (checksum %zu)\n", failures, sink % 1000);
  return failures == 0 ? 0 : 1;
}
