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
constexpr int FAST1_KMAX = 12;

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
    kappa_out[i] = (float)kap;
    if (flags_out) flags_out[i] = fl;
  }
}

// ---- two-pass form (k >= 13) ----------------------------------------------------------
// Per-point LDS layout of the two-pass Fast kernel.  ESZ: bytes per staged value (4 or 8).
template <int KMAX, int NW_, int PPW_, int ESZ_>
struct FastCfg {
  static constexpr int KM = KMAX;
  static constexpr int KB = (KMAX + 15) / 16;               // 16-row blocks of the patch
  static constexpr int NW = NW_, PPW = PPW_, NTG = NW * WAVE, NT = PPW * NTG;
  static constexpr int ESZ = ESZ_;
  static constexpr int NCOLMAX = (KMAX - 1) * KMAX / 2 + 2; // pairs (l1 <= l2 < k-1), h, ones
  static constexpr int NB = (NCOLMAX + 15) / 16;
  static constexpr int NPAD = NB * 16;
  static constexpr int NBW = (NB + NW - 1) / NW;            // column blocks per wave
  static constexpr int KK = (KMAX + 1) & ~1;                // even Jacobi size
  static constexpr int JLD = KK + 1;
  static constexpr int XQ = 16 * KB, XONE = 16 * KB + 1, XROWS = 16 * KB + 2;   // patch chunk rows
  static constexpr int VH = 16 * KB, VONE = 16 * KB + 1, VZERO = 16 * KB + 2;   // range chunk rows
  static constexpr int VROWS = 16 * KB + 3;
  static constexpr int VBLK = KB * (FCH / 16);              // blocks of the V_r^T chunk product
  static constexpr int VBW = (VBLK + NW - 1) / NW;
  static constexpr int KBLK = KB * KB;                      // blocks of the Gram product
  static constexpr int KBW = (KBLK + NW - 1) / NW;
  static constexpr size_t OFF_XS = 0;
  static constexpr size_t OFF_VS = ((size_t)XROWS * FLDX * ESZ + 15) & ~(size_t)15;
  static constexpr size_t OFF_JA = (OFF_VS + (size_t)VROWS * FLDX * ESZ + 15) & ~(size_t)15;
  static constexpr size_t OFF_JV = OFF_JA + (size_t)KK * JLD * 8;
  static constexpr size_t OFF_UT = OFF_JV + (size_t)KK * JLD * 8;
  static constexpr size_t OFF_YB = OFF_UT + (size_t)KMAX * KMAX * 8;    // copy of K
  static constexpr size_t OFF_RED = OFF_YB + (size_t)KMAX * KMAX * 8;
  static constexpr size_t OFF_ROT = OFF_RED + (size_t)16 * NW * 8;
  static constexpr size_t OFF_BJ = OFF_ROT + (size_t)KK * 8;            // tr G_j, r_j
  static constexpr size_t OFF_INT = OFF_BJ + (size_t)2 * KMAX * 8;
  static constexpr size_t N_INT = KMAX + KK + 8;                         // nb, ord, misc
  static constexpr size_t OFF_PAIR = OFF_INT + N_INT * 4;
  static constexpr size_t OFF_PJ = OFF_PAIR + (size_t)(KK - 1) * (KK / 2) * 2;
  static constexpr size_t BYTES = (OFF_PJ + 2 * NPAD + 15) & ~(size_t)15;
};

template <int KMAX, int PREC>
struct Fast2CfgSel {
  static constexpr int NW = KMAX <= 20 ? 1 : (KMAX <= 26 ? 2 : 4);
  static constexpr int PPW = NW == 1 ? (PREC == MOM_FP64 ? 2 : 4) : 1;
  using C = FastCfg<KMAX, NW, PPW, PREC == MOM_FP64 ? 8 : 4>;
};

template <int KMAX, int PREC>
__global__ __launch_bounds__((Fast2CfgSel<KMAX, PREC>::C::NT)) void curv_fast2_kernel(
    const float* __restrict__ X, int64_t n, int64_t m, int64_t ldx, const int32_t* __restrict__ idx,
    int k, int variant, float* __restrict__ kappa_out, uint8_t* __restrict__ flags_out) {
  using C = typename Fast2CfgSel<KMAX, PREC>::C;
  using ST = typename std::conditional<PREC == MOM_FP64, double, float>::type;   // staged values
  using AccT = typename std::conditional<PREC == MOM_FP64, doublex4, floatx4>::type;
  constexpr int KB = C::KB;
  extern __shared__ __align__(16) unsigned char smem_all[];
  const int gid = threadIdx.x / C::NTG;            // point group inside the workgroup
  const int tg = threadIdx.x % C::NTG;             // thread inside the group
  const int w = tg / WAVE, lane = tg % WAVE;
  const int64_t i = (int64_t)blockIdx.x * C::PPW + gid;
  if (i >= n) return;                              // whole group exits together
  unsigned char* sm = smem_all + (size_t)gid * C::BYTES;
  ST* XS = reinterpret_cast<ST*>(sm + C::OFF_XS);
  ST* VS = reinterpret_cast<ST*>(sm + C::OFF_VS);
  double* BJ = reinterpret_cast<double*>(sm + C::OFF_BJ);
  unsigned char* pj1 = sm + C::OFF_PJ;
  unsigned char* pj2 = pj1 + C::NPAD;
  PointLds P{};
  P.JA = reinterpret_cast<double*>(sm + C::OFF_JA);
  P.JV = reinterpret_cast<double*>(sm + C::OFF_JV);
  P.UT = reinterpret_cast<double*>(sm + C::OFF_UT);
  P.YB = reinterpret_cast<double*>(sm + C::OFF_YB);
  P.RED = reinterpret_cast<double*>(sm + C::OFF_RED);
  P.ROT = reinterpret_cast<double*>(sm + C::OFF_ROT);
  int* IN = reinterpret_cast<int*>(sm + C::OFF_INT);
  P.nb = IN;
  P.ord = IN + C::KM;
  P.misc = P.ord + C::KK;
  P.pairs = reinterpret_cast<uint16_t*>(sm + C::OFF_PAIR);
  int* nb = P.nb;
  int* misc = P.misc;
  const int npair = (k - 1) * k / 2;
  const int ncol = npair + 2;
  const int nbr = (ncol + 15) / 16;                // column blocks in use

  // ---- setup: neighbour rows, column tables, zero rows -----------------------------
  if (tg < 8) misc[tg] = 0;
  gsync<C::NW>();
  if (tg < k) {
    int v = idx[i * k + tg];
    if (v < 0 || (int64_t)v >= n) { misc[0] = 1; v = 0; }
    nb[tg] = v;
  }
  for (int t = tg; t < C::NPAD; t += C::NTG) {
    int a = C::VZERO, b = C::VZERO;                // padding column: zero row
    if (t < npair) {
      int r = t;
      a = 0;
      while (r >= k - 1 - a) { r -= k - 1 - a; ++a; }
      b = a + r;
    } else if (t == npair) {
      a = C::VH;                                   // h column: h o 1
      b = C::VONE;
    } else if (t == npair + 1) {
      a = b = C::VONE;                             // ones column
    }
    pj1[t] = (unsigned char)a;
    pj2[t] = (unsigned char)b;
  }
  for (int t = tg; t < (16 * KB - k) * FLDX; t += C::NTG) XS[k * FLDX + t] = (ST)0;
  for (int t = tg; t < FLDX; t += C::NTG) VS[C::VZERO * FLDX + t] = (ST)0;
  gsync<C::NW>();
  if (misc[0]) {
    if (tg == 0) {
      kappa_out[i] = __builtin_nanf("");
      if (flags_out) flags_out[i] = PF_NONFINITE;
    }
    return;
  }

  // staging of one chunk by wave 0: centred rows, q row, ones row
  float xr[KMAX];
  auto stage = [&](int64_t c0, double& tau64, bool& nonfinite) {
    if constexpr (PREC == MOM_FP64) {
      double xc[KMAX];
      centre_column_f64<KMAX>(xr, xc, k);
      double q = 0.0;
#pragma unroll
      for (int j = 0; j < KMAX; ++j)
        if (j < k) {
          nonfinite |= !isfinite(xr[j]);
          q = fma(xc[j], xc[j], q);
          XS[j * FLDX + lane] = xc[j];
        }
      tau64 += q;
      XS[C::XQ * FLDX + lane] = q;
    } else {
#pragma unroll
      for (int j = 0; j < KMAX; ++j)
        if (j < k) nonfinite |= !isfinite(xr[j]);
      centre_column<KMAX>(xr, k);
      float q = 0.0f;
#pragma unroll
      for (int j = 0; j < KMAX; ++j)
        if (j < k) {
          q = fmaf(xr[j], xr[j], q);
          tau64 = fma((double)xr[j], (double)xr[j], tau64);
          XS[j * FLDX + lane] = xr[j];
        }
      XS[C::XQ * FLDX + lane] = q;
    }
    XS[C::XONE * FLDX + lane] = (c0 + lane < m) ? (ST)1 : (ST)0;
  };
  auto steps16 = [&](int64_t c0) { return m - c0 >= FCH ? FCH / 16 : (int)((m - c0 + 15) / 16); };

  // ---- pass 1: K = X_c X_c^T on MFMA, tau in float64 ----------------------------------
  double tau64 = 0.0;
  bool nonfinite = false;
  {
    AccT kacc[C::KBW];
#pragma unroll
    for (int t = 0; t < C::KBW; ++t) kacc[t] = AccT{0, 0, 0, 0};
    if (w == 0) load_chunk<KMAX>(xr, X, ldx, nb, k, m, 0, lane);
    for (int64_t c0 = 0; c0 < m; c0 += FCH) {
      if (w == 0) stage(c0, tau64, nonfinite);
      gsync<C::NW>();
      if (w == 0 && c0 + FCH < m) load_chunk<KMAX>(xr, X, ldx, nb, k, m, c0 + FCH, lane);
      const int ng = steps16(c0);
      for (int g = 0; g < ng; ++g) {
        const int col = 16 * g + 4 * (lane / 16);   // lane supplies columns col .. col+3
#pragma unroll
        for (int t = 0; t < C::KBW; ++t) {
          const int kb = w + C::NW * t;
          if (kb < C::KBLK) {
            const int ab = kb / KB, bb = kb % KB;
            const ST* pa = XS + (16 * ab + lane % 16) * FLDX + col;
            const ST* pb = XS + (16 * bb + lane % 16) * FLDX + col;
#pragma unroll
            for (int st = 0; st < 4; ++st) {
              if constexpr (PREC == MOM_FP64) kacc[t] = mfma16x16x4f64(pa[st], pb[st], kacc[t]);
              else kacc[t] = mfma16x16x4(pa[st], pb[st], kacc[t]);
            }
          }
        }
      }
      gsync<C::NW>();
    }
    // K into the Jacobi matrix (padded with zeros) and its copy; V = identity
#pragma unroll
    for (int t = 0; t < C::KBW; ++t) {
      const int kb = w + C::NW * t;
      if (kb < C::KBLK) {
        const int ab = kb / KB, bb = kb % KB;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int x = 16 * ab + (PREC == MOM_FP64 ? lane / 16 + 4 * r : 4 * (lane / 16) + r);
          const int y = 16 * bb + lane % 16;
          if (x < C::KK && y < C::KK) {
            const double v = (x < k && y < k) ? (double)kacc[t][r] : 0.0;
            P.JA[x * C::JLD + y] = v;
            if (x < KMAX && y < KMAX) P.YB[x * KMAX + y] = v;
          }
        }
      }
    }
    for (int e = tg; e < C::KK * C::KK; e += C::NTG) {
      const int x = e / C::KK, y = e % C::KK;
      P.JV[x * C::JLD + y] = (x == y) ? 1.0 : 0.0;
    }
    if (w == 0) {
      tau64 = wave_sum(tau64);
      const int nf = __any(nonfinite);
      if (lane == 0) {
        P.RED[15 * C::NW] = tau64;
        misc[1] = nf;
      }
    }
    gsync<C::NW>();
  }
  const double tauk = P.RED[15 * C::NW];
  if (misc[1]) {
    if (tg == 0) {
      kappa_out[i] = __builtin_nanf("");
      if (flags_out) flags_out[i] = PF_NONFINITE;
    }
    return;
  }

  // ---- eigen-solve: Ut = U_p diag(sigma_p^(-1/2)) ------------------------------------
  double sig0;
  int pe, sweep;
  jacobi_eigen<KMAX, C, PREC != MOM_FP64>(P, k, m, tg, PREC == MOM_FP64 ? 0x1p-44 : 0x1p-24, sig0, pe, sweep);
  const int plim = (int)((int64_t)(k - 1) < m ? (int64_t)(k - 1) : m);
  uint8_t fl = 0;
  if (pe < plim) fl |= PF_RANK_DEFICIENT;
  if (sweep >= JAC_MAX_SWEEPS) fl |= PF_JACOBI_MAXSWEEPS;
  if (misc[5]) fl |= PF_EIGEN_FP64;
  if (!(sig0 > 0.0) || tauk == 0.0 || pe == 0) {   // locally flat: kappa = 0
    if (tg == 0) {
      kappa_out[i] = 0.0f;
      if (flags_out) flags_out[i] = fl | PF_DEGENERATE;
    }
    return;
  }

  // ---- pass 2: range chunks and the G_tens / trace / r GEMM ----------------------------
  // Ut^T operand of the V_r^T chunk product: A[l][j] = Ut[j][l] at row l = 16 lb + lane%16,
  // k index j = 16 jb + 4 s + lane/16
  ST ua[KB][KB][4];
#pragma unroll
  for (int lb = 0; lb < KB; ++lb)
#pragma unroll
    for (int jb = 0; jb < KB; ++jb)
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int l = 16 * lb + lane % 16, j = 16 * jb + 4 * st + lane / 16;
        ua[lb][jb][st] = (l < pe && j < k) ? (ST)P.UT[j * KMAX + l] : (ST)0;
      }
  int off1[C::NBW], off2[C::NBW];
#pragma unroll
  for (int b = 0; b < C::NBW; ++b) {
    const int nbg = w + C::NW * b;
    const int pc = nbg * 16 + lane % 16 < C::NPAD ? nbg * 16 + lane % 16 : C::NPAD - 1;
    off1[b] = pj1[pc] * FLDX;
    off2[b] = pj2[pc] * FLDX;
  }
  AccT acc[KB][C::NBW];
#pragma unroll
  for (int a = 0; a < KB; ++a)
#pragma unroll
    for (int b = 0; b < C::NBW; ++b) acc[a][b] = AccT{0, 0, 0, 0};
  double tD = 0.0;
  double dummy = 0.0;
  bool nf2 = false;
  if (w == 0) load_chunk<KMAX>(xr, X, ldx, nb, k, m, 0, lane);
  for (int64_t c0 = 0; c0 < m; c0 += FCH) {
    if (w == 0) stage(c0, dummy, nf2);
    gsync<C::NW>();
    if (w == 0 && c0 + FCH < m) load_chunk<KMAX>(xr, X, ldx, nb, k, m, c0 + FCH, lane);
    // V_r^T chunk = Ut^T X_c (rows l, columns c of the chunk)
#pragma unroll
    for (int t = 0; t < C::VBW; ++t) {
      const int vb = w + C::NW * t;
      if (vb < C::VBLK) {
        const int lb = vb / (FCH / 16), cb = vb % (FCH / 16);
        AccT v = AccT{0, 0, 0, 0};
#pragma unroll
        for (int jb = 0; jb < KB; ++jb)
#pragma unroll
          for (int st = 0; st < 4; ++st) {
            const ST bv = XS[(16 * jb + 4 * st + lane / 16) * FLDX + 16 * cb + lane % 16];
            if constexpr (PREC == MOM_FP64) v = mfma16x16x4f64(ua[lb][jb][st], bv, v);
            else v = mfma16x16x4(ua[lb][jb][st], bv, v);
          }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int l = 16 * lb + (PREC == MOM_FP64 ? lane / 16 + 4 * r : 4 * (lane / 16) + r);
          VS[l * FLDX + 16 * cb + lane % 16] = (ST)v[r];
        }
      }
    }
    gsync<C::NW>();
    // h_c = sum_l V[c, l]^2, the ones row, and t_D's sum_c q_c h_c
    if (w == 0) {
      ST h = 0;
      for (int l = 0; l < pe; ++l) {
        const ST v = VS[l * FLDX + lane];
        h += v * v;
      }
      VS[C::VH * FLDX + lane] = h;
      VS[C::VONE * FLDX + lane] = (c0 + lane < m) ? (ST)1 : (ST)0;
      tD = fma((double)XS[C::XQ * FLDX + lane], (double)h, tD);
    }
    gsync<C::NW>();
    if constexpr (PREC == MOM_FP64) {
      const int st4 = m - c0 >= FCH ? FCH / 4 : (int)((m - c0 + 3) / 4);
      for (int s4 = 0; s4 < st4; ++s4) {
        const int col = 4 * s4 + lane / 16;
        double av[KB];
#pragma unroll
        for (int a = 0; a < KB; ++a) av[a] = XS[(16 * a + lane % 16) * FLDX + col];
#pragma unroll
        for (int b = 0; b < C::NBW; ++b) {
          if (w + C::NW * b < nbr) {
            const double bv = VS[off1[b] + col] * VS[off2[b] + col];
#pragma unroll
            for (int a = 0; a < KB; ++a) acc[a][b] = mfma16x16x4f64(av[a], bv, acc[a][b]);
          }
        }
      }
    } else if constexpr (PREC == MOM_FP32) {
      const int ng = steps16(c0);
      for (int g = 0; g < ng; ++g) {
        const int col = 16 * g + 4 * (lane / 16);
        floatx4 av[KB];
#pragma unroll
        for (int a = 0; a < KB; ++a)
          av[a] = *reinterpret_cast<const floatx4*>(XS + (16 * a + lane % 16) * FLDX + col);
#pragma unroll
        for (int b = 0; b < C::NBW; ++b) {
          if (w + C::NW * b < nbr) {
            const floatx4 x1 = *reinterpret_cast<const floatx4*>(VS + off1[b] + col);
            const floatx4 x2 = *reinterpret_cast<const floatx4*>(VS + off2[b] + col);
            const floatx4 bv = x1 * x2;
#pragma unroll
            for (int st = 0; st < 4; ++st)
#pragma unroll
              for (int a = 0; a < KB; ++a) acc[a][b] = mfma16x16x4(av[a][st], bv[st], acc[a][b]);
          }
        }
      }
    } else {
      // bf16 operands, 32-column steps: lane l supplies columns 32 s + 8 (l / 16) + e
      const int st32 = m - c0 >= FCH ? FCH / 32 : (int)((m - c0 + 31) / 32);
      for (int s32 = 0; s32 < st32; ++s32) {
        const int col0 = 32 * s32 + 8 * (lane / 16);
        shortx8 abf[KB];
#pragma unroll
        for (int a = 0; a < KB; ++a) {
          const floatx4 x0 = *reinterpret_cast<const floatx4*>(XS + (16 * a + lane % 16) * FLDX + col0);
          const floatx4 x1 = *reinterpret_cast<const floatx4*>(XS + (16 * a + lane % 16) * FLDX + col0 + 4);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            abf[a][e] = (short)f2bf(x0[e]);
            abf[a][4 + e] = (short)f2bf(x1[e]);
          }
        }
#pragma unroll
        for (int b = 0; b < C::NBW; ++b) {
          if (w + C::NW * b < nbr) {
            const floatx4 p0 = *reinterpret_cast<const floatx4*>(VS + off1[b] + col0);
            const floatx4 p1 = *reinterpret_cast<const floatx4*>(VS + off1[b] + col0 + 4);
            const floatx4 q0 = *reinterpret_cast<const floatx4*>(VS + off2[b] + col0);
            const floatx4 q1 = *reinterpret_cast<const floatx4*>(VS + off2[b] + col0 + 4);
            shortx8 bbf;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              bbf[e] = (short)f2bf(p0[e] * q0[e]);
              bbf[4 + e] = (short)f2bf(p1[e] * q1[e]);
            }
#pragma unroll
            for (int a = 0; a < KB; ++a) acc[a][b] = mfma16x16x32bf16(abf[a], bbf, acc[a][b]);
          }
        }
      }
    }
    gsync<C::NW>();
  }

  // ---- reductions: raw sums (k-1) * (t_range, g, t_A, t_S, t_D) ------------------------
  double part[5] = {0.0, 0.0, 0.0, 0.0, tD};
#pragma unroll
  for (int b = 0; b < C::NBW; ++b) {
    const int nbg = w + C::NW * b;
    if (nbg < nbr) {
      const int col = nbg * 16 + lane % 16;
#pragma unroll
      for (int a = 0; a < KB; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = 16 * a + (PREC == MOM_FP64 ? lane / 16 + 4 * r : 4 * (lane / 16) + r);
          if (j < k && col < ncol) {
            const double v = (double)acc[a][b][r];
            if (col < npair) {
              const bool diag = pj1[col] == pj2[col];
              part[1] = fma(diag ? v : 2.0 * v, v, part[1]);
              if (diag) part[0] = fma(v, v, part[0]);
            } else {
              BJ[(col - npair) * KMAX + j] = v;      // tr G_j (h column), r_j (ones column)
            }
          }
        }
    }
  }
  // t_S = sum_l ||K ut_l||^2 from the copy of K
  for (int e = tg; e < KMAX * KMAX; e += C::NTG) {
    const int a = e / KMAX, l = e % KMAX;
    if (a < k && l < pe) {
      double sv = 0.0;
      for (int b = 0; b < k; ++b) sv = fma(P.YB[a * KMAX + b], P.UT[b * KMAX + l], sv);
      part[3] = fma(sv, sv, part[3]);
    }
  }
  gsync<C::NW>();
  for (int j = tg; j < k; j += C::NTG) {
    const double bj = BJ[KMAX + j] - BJ[j];       // (X_c d_P)_j = r_j - tr G_j
    part[2] = fma(bj, bj, part[2]);
  }
  group_sum<C::NW, 5>(part, P.RED, tg);

  if (tg == 0) {
    kappa_out[i] = (float)fast_combine(part, tauk, k, m, pe, variant, nullptr);
    if (flags_out) flags_out[i] = fl;
  }
}

template <int KMAX, int PREC>
static hipError_t launch_fast_kp(const float* X, int64_t n, int64_t m, int64_t ldx,
                                 const int32_t* idx, int k, int variant, float* kappa,
                                 uint8_t* flags, hipStream_t stream) {
  using C = typename std::conditional<(KMAX <= FAST1_KMAX), typename Fast1CfgSel<KMAX, PREC>::C,
                                      typename Fast2CfgSel<KMAX, PREC>::C>::type;
  static_assert(C::PPW * C::BYTES <= 160 * 1024, "per-workgroup LDS exceeds the 160 KiB of a CU");
  const void* fn;
  if constexpr (KMAX <= FAST1_KMAX) fn = reinterpret_cast<const void*>(&curv_fast1_kernel<KMAX, PREC>);
  else fn = reinterpret_cast<const void*>(&curv_fast2_kernel<KMAX, PREC>);
  static std::atomic<uint64_t> attr_set{0};   // LDS beyond 64 KiB needs the opt-in attribute
  once_per_device(attr_set, [&] {
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(C::PPW * C::BYTES));
    (void)hipGetLastError();
  });
  const unsigned grid = (unsigned)((n + C::PPW - 1) / C::PPW);
  timing_begin(6, stream);
  if constexpr (KMAX <= FAST1_KMAX) {
    hipLaunchKernelGGL((curv_fast1_kernel<KMAX, PREC>), dim3(grid), dim3(C::NT), C::PPW * C::BYTES,
                       stream, X, n, m, ldx, idx, k, variant, kappa, flags);
  } else {
    hipLaunchKernelGGL((curv_fast2_kernel<KMAX, PREC>), dim3(grid), dim3(C::NT), C::PPW * C::BYTES,
                       stream, X, n, m, ldx, idx, k, variant, kappa, flags);
  }
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
