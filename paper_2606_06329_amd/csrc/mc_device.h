// Device helpers shared by the gfx950 kernels of libmecuco (wave64, MFMA, LDS).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mc {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef short shortx8 __attribute__((ext_vector_type(8)));
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef int intx8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

constexpr int WAVE = 64;

// Per-point flag bits (mirror MC_PF_* of the public header).
constexpr uint8_t PF_NONFINITE = 1u;
constexpr uint8_t PF_DEGENERATE = 2u;
constexpr uint8_t PF_RANK_DEFICIENT = 4u;
constexpr uint8_t PF_JACOBI_MAXSWEEPS = 8u;
constexpr uint8_t PF_KNN_AMBIGUOUS = 16u;
constexpr uint8_t PF_KNN_UNCERTIFIED = 32u;
constexpr uint8_t PF_EIGEN_FP64 = 64u;
constexpr uint8_t PF_PRECISION_LIMIT = 128u;

// Fast mode: whether the point's error estimate exceeds its precision's budget: bf16 moments
// on rows narrower than 256 (their 8-bit products exceed 2e-2 on strongly curved patches
// there), or a centred patch whose Gram matrix is too ill-conditioned for the moments.  The
// Gram matrix's relative rounding u (prec_class 0: float32 moments, 2^-24; 1: bf16 moments
// with a float32 Gram, 2^-24; 3: bf16 moments with the Gram from split bf16 products,
// 3 * 2^-16, what a product of two hi + lo splits can drop; 2: float64, 2^-53) turns the
// weakest kept direction by about u cond, cond = sigma_1 / sigma_pe, towards the null space,
// which moves the null-space term by that angle spread over its q = m - pe directions:
// estimate 2 u cond / q (2 u cond when q = 0), against the path's budget (1e-4 float32,
// 2e-2 bf16, 1e-6 float64).
__device__ __forceinline__ bool beyond_precision(double sig_max, double sig_min, int k, int64_t m, int pe,
                                                 int prec_class) {
  (void)k;
  const bool bf16 = prec_class == 1 || prec_class == 3;
  if (bf16 && m < 256) return true;
  if (!(sig_min > 0.0)) return pe > 0;
  const double u = prec_class == 2 ? 0x1p-53 : (prec_class == 3 ? 0x1.8p-15 : 0x1p-24);
  const double budget = prec_class == 0 ? 1e-4 : (bf16 ? 2e-2 : 1e-6);
  const int64_t q = m - pe;
  return 2.0 * u * (sig_max / sig_min) / (double)(q > 0 ? q : 1) > budget;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, WAVE));
  return v;
}

// Round-to-nearest-even float -> bfloat16 bits (gfx950 converts in hardware, two values
// per v_cvt_pk_bf16_f32 when adjacent conversions pair up).
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Round-to-nearest-even float -> IEEE binary16 bits.
__device__ __forceinline__ uint16_t f2h(float f) { return __builtin_bit_cast(uint16_t, (_Float16)f); }

// D(16x16) += A(16x4) * B(4x16), fp32.  Lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; it receives D[4*(l/16)+r][l%16], r = 0..3.
__device__ __forceinline__ floatx4 mfma16x16x4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// D(16x16) += A(16x4) * B(4x16), fp64.  Inputs as the fp32 16x16x4 form (lane l supplies
// A[l%16][l/16] and B[l/16][l%16]), but the result is interleaved differently: lane l
// receives D[l/16 + 4r][l%16], r = 0..3 (checked on gfx950).
__device__ __forceinline__ doublex4 mfma16x16x4f64(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// D(32x32) += A(32x2) * B(2x32), fp32.  Lane l supplies A[l%32][l/32] and
// B[l/32][l%32]; it receives D[8*(r/4) + 4*(l/32) + r%4][l%32], r = 0..15.
__device__ __forceinline__ floatx16 mfma32x32x2(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// D(16x16) += A(16x32) * B(32x16), binary16 in, fp32 accumulate.  Lane l supplies
// A[l%16][8*(l/16)+e] and B[8*(l/16)+e][l%16], e = 0..7.
__device__ __forceinline__ floatx4 mfma16x16x32f16(halfx8 a, halfx8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// D(16x16) += A(16x32) * B(32x16), bf16 in, fp32 accumulate, operands as the binary16 form.
__device__ __forceinline__ floatx4 mfma16x16x32bf16(shortx8 a, shortx8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(__attribute__((ext_vector_type(8))) __bf16, a),
                                                 __builtin_bit_cast(__attribute__((ext_vector_type(8))) __bf16, b),
                                                 c, 0, 0, 0);
}

}  // namespace mc
