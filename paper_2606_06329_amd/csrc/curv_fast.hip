// Fused Fast-mode mean curvature, one point per wave (k <= 20) or per workgroup (gfx950).
// Moments in float32 (default), bf16 with a float32 Gram, or float64 (precision 3).
//
// What is computed (Fast branch of Algorithm 1, eqs. tnull/tA/tB/fast_curv):
// for the centred k x m patch X_c of point i,
//   tau     = ||X_c||_F^2/(k-1)
//   t_range = ||X_c V_r^{o2}||_F^2/(k-1)
//   t_A     = ||X_c d_P||^2/(k-1),  d_P = 1 - (V_r o V_r) 1
//   t_S     = ||X_c V_r||_F^2/(k-1)                       (printed t_B middle term)
//   t_D     = sum_{j,a} X_c[j,a]^2 h_a/(k-1), h = (V_r o V_r) 1 (Haar middle term)
//   g       = ||G_tens||_F^2/(k-1),  G_tens[j,l1,l2] = sum_a X_c[j,a] V[a,l1] V[a,l2]
//   kappa   = |(t_range + t_null)/2 + tau/2|
//
// How (Gram-space evaluation, one pass over the patch):
// with K = X_c X_c^T = U diag(sigma) U^T and Ut = U_p diag(sigma_p^{-1/2}),
// V_r = X_c^T Ut (eq. svd_cov), so every term reduces to k x k objects:
//   G_j = Ut^T T_j Ut,  t_range = sum_j sum_l G_j[l,l]^2,  g = sum_j ||G_j||^2,
//   (X_c d_P)_j = r_j - tr G_j,  t_S = sum_l ||K ut_l||^2,  t_D = sum_l ut_l^T Q ut_l
// (each divided by k-1), with the moments T, Q, r, K of curv_core.h.
#include "curv_core.h"
#include "mc_internal.h"

namespace mc {

template <int KMAX, int PREC>
struct FastCfgSel {
  static constexpr int NW = KMAX <= 20 ? 1 : (KMAX <= 26 ? 2 : 4);
  // float64 moments double the staged chunk and the moment rows: two points per workgroup
  static constexpr int PPW = NW == 1 ? (PREC == MOM_FP64 ? 2 : 4) : 1;
  using C = CurvCfg<KMAX, NW, PPW, 0, PREC == MOM_FP64 ? 8 : 4>;
};

// Largest k whose float64-moment per-point state fits the 160 KiB of LDS.
constexpr int FAST_FP64_KMAX = 28;

// Gram-space terms of the Fast branch.  part[0..4] = (k-1) * (t_range, g, t_A, t_S, t_D).
template <int KMAX, class C, int PREC>
__device__ __forceinline__ void fast_terms(const PointLds& P, int k, int pe, int tg,
                                           double (&part)[5]) {
  const int np = k * (k + 1) / 2;
  using MT = MomT<PREC>;
  const MT* mom = reinterpret_cast<const MT*>(P.mom);
  const MT* Krow = mom + (k + 1) * C::NPAD;
  const MT* Qrow = mom + k * C::NPAD;
  const double* UT = P.UT;
  double* YB = P.YB;
#pragma unroll
  for (int t = 0; t < 5; ++t) part[t] = 0.0;
  // t_S = sum_l ||K ut_l||^2 ; t_D = sum_l ut_l^T Q ut_l
  for (int e = tg; e < k * pe; e += C::NTG) {
    const int a = e / pe, l = e % pe;
    double kv = 0.0, qv = 0.0;
    for (int b = 0; b < k; ++b) {
      const int pb = P.PIDX[a * KMAX + b];
      const double u = UT[b * KMAX + l];
      kv = fma((double)Krow[pb], u, kv);
      qv = fma((double)Qrow[pb], u, qv);
    }
    part[3] = fma(kv, kv, part[3]);
    part[4] = fma(UT[a * KMAX + l], qv, part[4]);
  }
  for (int j = 0; j < k; ++j) {
    const MT* Tj = mom + j * C::NPAD;
    for (int e = tg; e < k * pe; e += C::NTG) {
      const int a = e / pe, l = e % pe;
      double yv = 0.0;
      for (int b = 0; b < k; ++b) yv = fma((double)Tj[P.PIDX[a * KMAX + b]], UT[b * KMAX + l], yv);
      YB[a * KMAX + l] = yv;
    }
    gsync<C::NW>();
    double trg = 0.0;
    for (int e = tg; e < pe * pe; e += C::NTG) {
      const int l1 = e / pe, l2 = e % pe;
      double gv = 0.0;
      for (int a = 0; a < k; ++a) gv = fma(UT[a * KMAX + l1], YB[a * KMAX + l2], gv);
      part[1] = fma(gv, gv, part[1]);
      if (l1 == l2) {
        part[0] = fma(gv, gv, part[0]);
        trg += gv;
      }
    }
    double tv[1] = {trg};
    group_sum<C::NW, 1>(tv, P.RED, tg);
    if (tg == 0) {
      const double bj = (double)mom[j * C::NPAD + np] - tv[0];   // (X_c d_P)_j
      part[2] = fma(bj, bj, part[2]);
    }
    gsync<C::NW>();
  }
  group_sum<C::NW, 5>(part, P.RED, tg);
}

// kappa from the raw sums (all float64); returns |inner| and stores inner.
__device__ __forceinline__ double fast_combine(const double (&part)[5], double tauk, int k,
                                               int64_t m, int pe, int variant, double* inner) {
  const double km1 = (double)(k - 1);
  const double tau = tauk / km1;
  const double t_range = part[0] / km1, g = part[1] / km1, t_A = part[2] / km1;
  const double t_S = part[3] / km1, t_D = part[4] / km1;
  const int64_t q = m - pe;
  double t_null = 0.0;
  if (q > 0) {
    if (variant == 0)
      t_null = (t_A + 2.0 * (tau - 2.0 * t_S + g)) / (double)q;
    else
      t_null = (t_A + 2.0 * (tau - 2.0 * t_D + g)) / (double)(q + 2);
  }
  const double in = 0.5 * (t_range + t_null) + 0.5 * tau;
  if (inner) *inner = in;
  return fabs(in);
}

template <int KMAX, int PREC>
__global__ __launch_bounds__((FastCfgSel<KMAX, PREC>::C::NT)) void curv_fast_kernel(
    const float* __restrict__ X, int64_t n, int64_t m, int64_t ldx, const int32_t* __restrict__ idx,
    int k, int variant, float* __restrict__ kappa_out, uint8_t* __restrict__ flags_out) {
  using C = typename FastCfgSel<KMAX, PREC>::C;
  extern __shared__ __align__(16) unsigned char smem_all[];
  const int gid = threadIdx.x / C::NTG;            // point group inside the workgroup
  const int tg = threadIdx.x % C::NTG;             // thread inside the group
  const int64_t i = (int64_t)blockIdx.x * C::PPW + gid;
  if (i >= n) return;                              // whole group exits together
  const PointLds P = point_lds<C>(smem_all + (size_t)gid * C::BYTES);

  double tauk, sig0;
  int pe, sweep;
  const uint8_t bad = patch_front<KMAX, C, PREC>(P, X, n, m, ldx, idx, k, i, tg, tauk, sig0, pe, sweep);
  if (bad) {
    if (tg == 0) {
      kappa_out[i] = __builtin_nanf("");
      if (flags_out) flags_out[i] = bad;
    }
    return;
  }
  double part[5];
  fast_terms<KMAX, C, PREC>(P, k, pe, tg, part);

  if (tg == 0) {
    uint8_t fl = 0;
    double kap;
    if (!(sig0 > 0.0) || tauk == 0.0) {
      kap = 0.0;
      fl |= PF_DEGENERATE;
    } else {
      kap = fast_combine(part, tauk, k, m, pe, variant, nullptr);
    }
    const int plim = (int)((int64_t)(k - 1) < m ? (int64_t)(k - 1) : m);
    if (pe < plim) fl |= PF_RANK_DEFICIENT;
    if (sweep >= JAC_MAX_SWEEPS) fl |= PF_JACOBI_MAXSWEEPS;
    kappa_out[i] = (float)kap;
    if (flags_out) flags_out[i] = fl;
  }
}

template <int KMAX, int PREC>
static hipError_t launch_fast_kp(const float* X, int64_t n, int64_t m, int64_t ldx,
                                 const int32_t* idx, int k, int variant, float* kappa,
                                 uint8_t* flags, hipStream_t stream) {
  using C = typename FastCfgSel<KMAX, PREC>::C;
  static_assert(C::PPW * C::BYTES <= 160 * 1024, "per-workgroup LDS exceeds the 160 KiB of a CU");
  static bool attr_set = false;   // LDS beyond 64 KiB needs the opt-in attribute
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&curv_fast_kernel<KMAX, PREC>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)(C::PPW * C::BYTES));
    (void)hipGetLastError();
    attr_set = true;
  }
  const unsigned grid = (unsigned)((n + C::PPW - 1) / C::PPW);
  timing_begin(6, stream);
  hipLaunchKernelGGL((curv_fast_kernel<KMAX, PREC>), dim3(grid), dim3(C::NT), C::PPW * C::BYTES, stream,
                     X, n, m, ldx, idx, k, variant, kappa, flags);
  timing_end(6, stream);
  return hipGetLastError();
}

template <int KMAX>
static hipError_t launch_fast_k(const float* X, int64_t n, int64_t m, int64_t ldx,
                                const int32_t* idx, int k, int precision, int variant, float* kappa,
                                uint8_t* flags, hipStream_t stream) {
  if (precision == 1)
    return launch_fast_kp<KMAX, MOM_BF16>(X, n, m, ldx, idx, k, variant, kappa, flags, stream);
  if (precision == 3) {
    if constexpr (KMAX <= FAST_FP64_KMAX)
      return launch_fast_kp<KMAX, MOM_FP64>(X, n, m, ldx, idx, k, variant, kappa, flags, stream);
    return hipErrorInvalidValue;
  }
  return launch_fast_kp<KMAX, MOM_FP32>(X, n, m, ldx, idx, k, variant, kappa, flags, stream);
}

hipError_t launch_curv_fast(const float* X, int64_t n, int64_t m, int64_t ldx, const int32_t* idx,
                            int k, int precision, int variant, float* kappa, uint8_t* flags,
                            hipStream_t stream) {
  if (k <= 4) return launch_fast_k<4>(X, n, m, ldx, idx, k, precision, variant, kappa, flags, stream);
  if (k <= 8) return launch_fast_k<8>(X, n, m, ldx, idx, k, precision, variant, kappa, flags, stream);
  if (k <= 12) return launch_fast_k<12>(X, n, m, ldx, idx, k, precision, variant, kappa, flags, stream);
  if (k <= 16) return launch_fast_k<16>(X, n, m, ldx, idx, k, precision, variant, kappa, flags, stream);
  if (k <= 20) return launch_fast_k<20>(X, n, m, ldx, idx, k, precision, variant, kappa, flags, stream);
  if (k <= 24) return launch_fast_k<24>(X, n, m, ldx, idx, k, precision, variant, kappa, flags, stream);
  if (k <= 28) return launch_fast_k<28>(X, n, m, ldx, idx, k, precision, variant, kappa, flags, stream);
  return launch_fast_k<32>(X, n, m, ldx, idx, k, precision, variant, kappa, flags, stream);
}

}  // namespace mc
