// Min-max normalisation of curvature scores to [0, 1] over the whole point set: the
// per-dataset normalised output of the paper's normalised-score experiment (Table 3).
// Two launches on the caller's stream: per-block minima and maxima of the finite scores,
// then every block reduces those partials (order-free, so deterministic) and writes
// (kappa - min) / (max - min) with an IEEE division.  Non-finite scores stay NaN; a constant
// score vector maps to 0; with no finite score every output is NaN.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mc_device.h"
#include "mc_internal.h"

namespace mc {

constexpr int NORM_BLOCKS = 256;
constexpr int NORM_THREADS = 256;

__global__ __launch_bounds__(NORM_THREADS) void norm_partials_kernel(const float* __restrict__ kappa, int64_t n,
                                                                     float* __restrict__ part) {
  float mn = INFINITY, mx = -INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * NORM_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * NORM_THREADS) {
    const float v = kappa[i];
    if (isfinite(v)) {
      mn = fminf(mn, v);
      mx = fmaxf(mx, v);
    }
  }
  __shared__ float smn[NORM_THREADS / WAVE], smx[NORM_THREADS / WAVE];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mn = fminf(mn, __shfl_xor(mn, o, WAVE));
    mx = fmaxf(mx, __shfl_xor(mx, o, WAVE));
  }
  if (threadIdx.x % WAVE == 0) {
    smn[threadIdx.x / WAVE] = mn;
    smx[threadIdx.x / WAVE] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < NORM_THREADS / WAVE; ++w) {
      mn = fminf(mn, smn[w]);
      mx = fmaxf(mx, smx[w]);
    }
    part[2 * blockIdx.x] = mn;
    part[2 * blockIdx.x + 1] = mx;
  }
}

// kappa and out may be the same array: each element is read and written by one thread
__global__ __launch_bounds__(NORM_THREADS) void norm_apply_kernel(const float* kappa, int64_t n,
                                                                  const float* __restrict__ part, int nparts,
                                                                  float* out) {
  __shared__ float lim[2];
  if (threadIdx.x < WAVE) {
    float mn = INFINITY, mx = -INFINITY;
    for (int p = threadIdx.x; p < nparts; p += WAVE) {
      mn = fminf(mn, part[2 * p]);
      mx = fmaxf(mx, part[2 * p + 1]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      mn = fminf(mn, __shfl_xor(mn, o, WAVE));
      mx = fmaxf(mx, __shfl_xor(mx, o, WAVE));
    }
    if (threadIdx.x == 0) {
      lim[0] = mn;
      lim[1] = mx;
    }
  }
  __syncthreads();
  const float mn = lim[0], mx = lim[1];
  const float range = mx - mn;
  for (int64_t i = (int64_t)blockIdx.x * NORM_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * NORM_THREADS) {
    const float v = kappa[i];
    float r;
    if (!isfinite(v) || !(mn <= mx)) r = __builtin_nanf("");
    else if (range == 0.0f) r = 0.0f;
    else r = (v - mn) / range;
    out[i] = r;
  }
}

size_t normalize_ws_bytes() { return align256((size_t)NORM_BLOCKS * 2 * sizeof(float)); }

hipError_t launch_normalize(const float* kappa, int64_t n, float* out, void* ws, hipStream_t stream) {
  const int64_t want = (n + NORM_THREADS - 1) / NORM_THREADS;
  const int blocks = (int)(want < NORM_BLOCKS ? want : NORM_BLOCKS);
  float* part = reinterpret_cast<float*>(ws);
  hipLaunchKernelGGL(norm_partials_kernel, dim3(blocks), dim3(NORM_THREADS), 0, stream, kappa, n, part);
  hipLaunchKernelGGL(norm_apply_kernel, dim3(blocks), dim3(NORM_THREADS), 0, stream, kappa, n,
                     (const float*)part, blocks, out);
  return hipGetLastError();
}

}  // namespace mc
