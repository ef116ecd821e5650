// Fused Fast-mode mean curvature (gfx950): one point per wave (k <= 20) or per workgroup.
// Moments in float32 (default), bf16 with a float32 Gram, or float64.
//
// What is computed (Fast branch of Algorithm 1, eqs. tnull/tA/tB/fast_curv):
// for the centred k x m patch X_c of point i,
//   tau     = ||X_c||_F^2/(k-1)
//   t_range = ||X_c V_r^{o2}||_F^2/(k-1)
//   t_A     = ||X_c d_P||^2/(k-1),  d_P = 1 - h,  h = (V_r o V_r) 1
//   t_S     = ||X_c V_r||_F^2/(k-1)                       (printed t_B middle term)
//   t_D     = sum_{j,a} X_c[j,a]^2 h_a/(k-1)               (Haar middle term)
//   g       = ||G_tens||_F^2/(k-1),  G_tens[j,l1,l2] = sum_a X_c[j,a] V[a,l1] V[a,l2]
//   kappa   = |(t_range + t_null)/2 + tau/2|
// With K = X_c X_c^T = U diag(sigma) U^T and Ut = U_p diag(sigma_p^{-1/2}), V_r = X_c^T Ut
// (eq. svd_cov).  Two evaluations, chosen by k:
//
// Single pass (k <= 12): one MFMA GEMM over the patch gives the third moments
//   T_j[a][b] = sum_c X_c[j,c] X_c[a,c] X_c[b,c], Q, r and K; after the eigen-solve every term
//   is k x k algebra: G_j = Ut^T T_j Ut, t_range = sum_j sum_l G_j[l,l]^2, g = sum_j ||G_j||^2,
//   (X_c d_P)_j = r_j - tr G_j, t_S = sum_l ||K ut_l||^2, t_D = sum_l ut_l^T Q ut_l.
//   The moments take k (k+1)/2 + 1 columns per point in LDS, which grows as k^3.
//
// Two passes (k >= 13):
//  1. K = X_c X_c^T on MFMA (and tau in float64); float64 Jacobi gives Ut.
//  2. Per 64-column chunk: the chunk of V_r^T = Ut^T X_c on MFMA, then one MFMA GEMM
//        X_c (k x chunk)  x  [V[:,l1] o V[:,l2] (l1 <= l2) | h | 1]  (chunk x p(p+1)/2 + 2)
//     whose columns are G_tens (pairs), tr G_j = (X_c h)_j and r_j = (X_c 1)_j; t_D comes
//     from sum_c q_c h_c with q_c = sum_j X_c[j,c]^2.
//   Only reductions of the accumulators leave registers, so the per-point LDS is two staged
//   chunks plus the k x k eigen-solve, and the patch is read twice.
#include "curv_core.h"
#include "mc_internal.h"

namespace mc {

// Largest k accepted with float64 moments (MC_FAST_FP64_KMAX in the public header).
constexpr int FAST_FP64_KMAX = 28;
// Largest k taken by the single-pass form; larger k use the two-pass form.
constexpr int FAST1_KMAX = FAST_SINGLE_PASS_KMAX;

// ---- single-pass form (k <= 12) -------------------------------------------------------
template <int KMAX, int PREC>
struct Fast1CfgSel {
  static constexpr int NW = KMAX <= 20 ? 1 : (KMAX <= 26 ? 2 : 4);
  // float64 moments double the staged chunk and the moment rows: two points per workgroup
  static constexpr int PPW = NW == 1 ? (PREC == MOM_FP64 ? 2 : 4) : 1;
  using C = CurvCfg<KMAX, NW, PPW, 0, PREC == MOM_FP64 ? 8 : 4>;
};

// Y = M Ut for a symmetric k x k moment matrix M held as packed pairs (row `mrow` of the
// moments), on v_mfma_f64_16x16x4f64.  The k index of step s in block bb is
// 16 bb + 4 s + lane/16 for both operands; ub[bb][s][lb] holds Ut[16bb+4s+lane/16][16lb+lane%16]
// (0 outside k x pe) and pix[ab][bb][s] the pair index of M[16ab+lane%16][16bb+4s+lane/16]
// (-1 outside k x k).  Block (ab, lb) of Y comes back in the MFMA result layout: element r
// holds Y[16ab + lane/16 + 4r][16lb + lane%16].
template <int KB, class MT>
__device__ __forceinline__ void gram_times_ut(const MT* __restrict__ mrow, const int (&pix)[KB][KB][4],
                                              const double (&ub)[KB][4][KB], doublex4 (&y)[KB][KB]) {
#pragma unroll
  for (int ab = 0; ab < KB; ++ab)
#pragma unroll
    for (int lb = 0; lb < KB; ++lb) y[ab][lb] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ab = 0; ab < KB; ++ab)
#pragma unroll
    for (int bb = 0; bb < KB; ++bb)
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int pi = pix[ab][bb][st];
        const double mv = pi >= 0 ? (double)mrow[pi] : 0.0;
#pragma unroll
        for (int lb = 0; lb < KB; ++lb) y[ab][lb] = mfma16x16x4f64(mv, ub[bb][st][lb], y[ab][lb]);
      }
}

// Gram-space terms of the Fast branch.  part[0..4] = (k-1) * (t_range, g, t_A, t_S, t_D).
// Per neighbour j, G_j = Ut^T (T_j Ut) is two chained f64 MFMA products: the result layout
// of T_j Ut is exactly the B-operand layout of the second product, so G_j never leaves
// registers.  The waves of a point take the j in turn; the diagonals of the G_j go to LDS
// (over the Jacobi matrix, no longer needed) for the traces in b_j = r_j - tr G_j.
template <int KMAX, class C, int PREC>
__device__ __forceinline__ void fast_terms(const PointLds& P, int k, int pe, int tg,
                                           double (&part)[5]) {
  constexpr int KB = (KMAX + 15) / 16;
  const int np = k * (k + 1) / 2;
  const int w = tg / WAVE, lane = tg % WAVE;
  using MT = MomT<PREC>;
  const MT* mom = reinterpret_cast<const MT*>(P.mom);
  const double* UT = P.UT;
  double* Dg = P.JA;                   // Dg[j * JLD + l] = G_j[l][l]
  int pix[KB][KB][4];
  double ub[KB][4][KB];
#pragma unroll
  for (int ab = 0; ab < KB; ++ab)
#pragma unroll
    for (int bb = 0; bb < KB; ++bb)
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int a = 16 * ab + lane % 16, b = 16 * bb + 4 * st + lane / 16;
        pix[ab][bb][st] = (a < k && b < k) ? (int)P.PIDX[a * KMAX + b] : -1;
      }
#pragma unroll
  for (int bb = 0; bb < KB; ++bb)
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
      for (int lb = 0; lb < KB; ++lb) {
        const int b = 16 * bb + 4 * st + lane / 16, l = 16 * lb + lane % 16;
        ub[bb][st][lb] = (b < k && l < pe) ? UT[b * KMAX + l] : 0.0;
      }
#pragma unroll
  for (int t = 0; t < 5; ++t) part[t] = 0.0;
  doublex4 y[KB][KB];
  // t_S = sum_l ||K ut_l||^2 (wave 0);  t_D = sum_l ut_l^T Q ut_l (wave 1 % NW)
  if (w == 0) {
    gram_times_ut<KB>(mom + (k + 1) * C::NPAD, pix, ub, y);
#pragma unroll
    for (int ab = 0; ab < KB; ++ab)
#pragma unroll
      for (int lb = 0; lb < KB; ++lb)
#pragma unroll
        for (int r = 0; r < 4; ++r) part[3] = fma(y[ab][lb][r], y[ab][lb][r], part[3]);
  }
  if (w == 1 % C::NW) {
    gram_times_ut<KB>(mom + k * C::NPAD, pix, ub, y);
#pragma unroll
    for (int ab = 0; ab < KB; ++ab)
#pragma unroll
      for (int lb = 0; lb < KB; ++lb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = 16 * ab + lane / 16 + 4 * r, l = 16 * lb + lane % 16;
          const double u = (a < k && l < pe) ? UT[a * KMAX + l] : 0.0;
          part[4] = fma(u, y[ab][lb][r], part[4]);
        }
  }
  for (int j = w; j < k; j += C::NW) {
    gram_times_ut<KB>(mom + j * C::NPAD, pix, ub, y);
    // G_j = Ut^T Y: A operand Ut^T[16 l1b + lane%16][16 ab + 4 s + lane/16] = ub[ab][s][l1b]
#pragma unroll
    for (int l1b = 0; l1b < KB; ++l1b)
#pragma unroll
      for (int l2b = 0; l2b < KB; ++l2b) {
        doublex4 g = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ab = 0; ab < KB; ++ab)
#pragma unroll
          for (int st = 0; st < 4; ++st) g = mfma16x16x4f64(ub[ab][st][l1b], y[ab][l2b][st], g);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          part[1] = fma(g[r], g[r], part[1]);
          const int l1 = 16 * l1b + lane / 16 + 4 * r, l2 = 16 * l2b + lane % 16;
          if (l1 == l2) {
            part[0] = fma(g[r], g[r], part[0]);
            if (l1 < pe) Dg[j * C::JLD + l1] = g[r];
          }
        }
      }
  }
  gsync<C::NW>();
  for (int j = tg; j < k; j += C::NTG) {
    double tr = 0.0;
    for (int l = 0; l < pe; ++l) tr += Dg[j * C::JLD + l];
    const double bj = (double)mom[j * C::NPAD + np] - tr;   // (X_c d_P)_j
    part[2] = fma(bj, bj, part[2]);
  }
  group_sum<C::NW, 5>(part, P.RED, tg);
}

template <int KMAX, int PREC>
__global__ __launch_bounds__((Fast1CfgSel<KMAX, PREC>::C::NT)) void curv_fast1_kernel(
    const float* __restrict__ X, int64_t n, int64_t m, int64_t ldx, const int32_t* __restrict__ idx,
    int k, int variant, float* __restrict__ kappa_out, uint8_t* __restrict__ flags_out) {
  using C = typename Fast1CfgSel<KMAX, PREC>::C;
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
  // the smallest kept eigenvalue, read before fast_terms reuses the Jacobi storage
  const double sig_min = pe > 0 ? P.JA[P.ord[pe - 1] * C::JLD + P.ord[pe - 1]] : 0.0;
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
    if (P.misc[5]) fl |= PF_EIGEN_FP64;
    if (!(fl & PF_DEGENERATE) && beyond_precision(sig0, sig_min, k, m, pe, PREC == MOM_FP64 ? 2 : (PREC == MOM_BF16 ? 1 : 0)))
      fl |= PF_PRECISION_LIMIT;
    kappa_out[i] = (float)kap;
    if (flags_out) flags_out[i] = fl;
  }
}

template <int KMAX, int PREC>
static hipError_t launch_fast_kp(const float* X, int64_t n, int64_t m, int64_t ldx,
                                 const int32_t* idx, int k, int variant, float* kappa,
                                 uint8_t* flags, hipStream_t stream) {
  using C = typename Fast1CfgSel<KMAX, PREC>::C;
  static_assert(C::PPW * C::BYTES <= 160 * 1024, "per-workgroup LDS exceeds the 160 KiB of a CU");
  const void* fn = reinterpret_cast<const void*>(&curv_fast1_kernel<KMAX, PREC>);
  static std::atomic<uint64_t> attr_set{0};   // LDS beyond 64 KiB needs the opt-in attribute
  once_per_device(attr_set, [&] {
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(C::PPW * C::BYTES));
    (void)hipGetLastError();
  });
  const unsigned grid = (unsigned)((n + C::PPW - 1) / C::PPW);
  timing_begin(6, stream);
  hipLaunchKernelGGL((curv_fast1_kernel<KMAX, PREC>), dim3(grid), dim3(C::NT), C::PPW * C::BYTES,
                     stream, X, n, m, ldx, idx, k, variant, kappa, flags);
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
                            int k, int precision, int variant, float* kappa, uint8_t* flags, void* ws,
                            hipStream_t stream) {
  if (k <= 4) return launch_fast_k<4>(X, n, m, ldx, idx, k, precision, variant, kappa, flags, stream);
  if (k <= 8) return launch_fast_k<8>(X, n, m, ldx, idx, k, precision, variant, kappa, flags, stream);
  if (k <= 12) return launch_fast_k<12>(X, n, m, ldx, idx, k, precision, variant, kappa, flags, stream);
  return launch_curv_fast2(X, n, m, ldx, idx, k, precision, variant, kappa, flags, ws, stream);
}

}  // namespace mc
