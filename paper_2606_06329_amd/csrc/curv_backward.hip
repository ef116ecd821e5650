// Adjoint of the Fast curvature (float64 moments and adjoint algebra) with respect to the point coordinates,
// neighbour lists held fixed: grad_X += d(sum_i gk_i kappa_i)/dX.
//
// The forward value is evaluated in Gram space (see curv_fast.hip):
//   R = Ut Ut^T (= K^+ on the range), G_j = Ut^T T_j Ut, d_jl = G_j[l,l]
//   T_range = sum_jl d_jl^2, T_g = sum_j tr(T_j R T_j R), b_j = r_j - tr(R T_j), T_A = sum_j b_j^2,
//   T_S = tr(R K K) (printed reading), T_D = tr(R Q) (Haar reading), T_tau = ||X_c||^2,
// all raw sums = (k-1) * the paper's terms.  Reverse mode:
//   * terms that depend on X_c only through R (g, t_A, t_S, t_D) use dR = -R dK R: the
//     centring null vector of K is fixed under centred perturbations, so there are no
//     eigen-gap factors;
//   * t_range depends on the individual range eigenvectors; their derivative uses the
//     regularised gap factors Delta / (Delta^2 + eta^2), eta = gap_eps * sigma_1;
//   * the k x k adjoints (K_bar, Q_bar, T_bar, r_bar) are turned into column gradients in a
//     second pass over the patch, un-centred, and scatter-added into grad_X.
#include "curv_core.h"
#include "mc_internal.h"

namespace mc {

template <int KMAX>
struct BwdExtra {
  static constexpr int NPM = KMAX * (KMAX + 1) / 2;
  static constexpr size_t KK2 = (size_t)KMAX * KMAX;
  // doubles: Rm, Rb, Kb, Qb, W1, W2, Ub, Db, Tb (KMAX x NPM), misc 64
  static constexpr size_t OFF_RM = 0;
  static constexpr size_t OFF_RB = OFF_RM + KK2 * 8;
  static constexpr size_t OFF_KB = OFF_RB + KK2 * 8;
  static constexpr size_t OFF_QB = OFF_KB + KK2 * 8;
  static constexpr size_t OFF_W1 = OFF_QB + KK2 * 8;
  static constexpr size_t OFF_W2 = OFF_W1 + KK2 * 8;
  static constexpr size_t OFF_UB = OFF_W2 + KK2 * 8;
  static constexpr size_t OFF_DB = OFF_UB + KK2 * 8;
  static constexpr size_t OFF_TB = OFF_DB + KK2 * 8;
  static constexpr size_t OFF_SC = OFF_TB + (size_t)KMAX * NPM * 8;   // 64 doubles of scalars
  // doubles for the column pass: Theta (NPM x KMAX), Kbf, Qbf (KMAX x KMAX), rbf (KMAX)
  static constexpr size_t OFF_TH = OFF_SC + 64 * 8;
  static constexpr size_t OFF_KBF = OFF_TH + (size_t)NPM * KMAX * 8;
  static constexpr size_t OFF_QBF = OFF_KBF + KK2 * 8;
  static constexpr size_t OFF_RBF = OFF_QBF + KK2 * 8;
  static constexpr size_t BYTES = OFF_RBF + (size_t)KMAX * 8 + 16;
};

template <int KMAX>
struct BwdCfgSel {
  using C = CurvCfg<KMAX, 2, 1, BwdExtra<KMAX>::BYTES, 8>;   // float64 moments
};

// out[a][b] = sum_c A[a][c] B[c][b] for k x k row-major (stride KMAX) float64 matrices,
// spread over the group's threads.
template <int KMAX, int NTG>
__device__ __forceinline__ void mat_mul(double* out, const double* A, const double* B, int k, int tg) {
  for (int e = tg; e < k * k; e += NTG) {
    const int a = e / k, b = e % k;
    double s = 0.0;
    for (int c = 0; c < k; ++c) s = fma(A[a * KMAX + c], B[c * KMAX + b], s);
    out[a * KMAX + b] = s;
  }
}

template <int KMAX>
__global__ __launch_bounds__(BwdCfgSel<KMAX>::C::NT) void curv_backward_kernel(
    const float* __restrict__ X, int64_t n, int64_t m, int64_t ldx, const int32_t* __restrict__ idx,
    int k, int variant, const float* __restrict__ gkap, float gap_eps, float* __restrict__ grad) {
  using C = typename BwdCfgSel<KMAX>::C;
  using E = BwdExtra<KMAX>;
  extern __shared__ __align__(16) unsigned char smem_all[];
  const int tg = threadIdx.x;
  const int w = tg / WAVE, lane = tg % WAVE;
  const int64_t i = blockIdx.x;
  const PointLds P = point_lds<C>(smem_all);
  double* Rm = reinterpret_cast<double*>(P.extra + E::OFF_RM);
  double* Rb = reinterpret_cast<double*>(P.extra + E::OFF_RB);
  double* Kb = reinterpret_cast<double*>(P.extra + E::OFF_KB);
  double* Qb = reinterpret_cast<double*>(P.extra + E::OFF_QB);
  double* W1 = reinterpret_cast<double*>(P.extra + E::OFF_W1);
  double* W2 = reinterpret_cast<double*>(P.extra + E::OFF_W2);
  double* Ub = reinterpret_cast<double*>(P.extra + E::OFF_UB);
  double* Db = reinterpret_cast<double*>(P.extra + E::OFF_DB);
  double* Tb = reinterpret_cast<double*>(P.extra + E::OFF_TB);
  double* SC = reinterpret_cast<double*>(P.extra + E::OFF_SC);
  double* TH = reinterpret_cast<double*>(P.extra + E::OFF_TH);
  double* Kbf = reinterpret_cast<double*>(P.extra + E::OFF_KBF);
  double* Qbf = reinterpret_cast<double*>(P.extra + E::OFF_QBF);
  double* rbf = reinterpret_cast<double*>(P.extra + E::OFF_RBF);

  const float gk = gkap[i];
  if (gk == 0.0f) return;
  double tauk, sig0;
  int pe, sweep;
  if (patch_front<KMAX, C, MOM_FP64>(P, X, n, m, ldx, idx, k, i, tg, tauk, sig0, pe, sweep)) return;
  if (!(sig0 > 0.0) || tauk == 0.0 || pe == 0) return;   // degenerate: kappa = 0 locally flat

  const int np = k * (k + 1) / 2;
  const double* mom = reinterpret_cast<const double*>(P.mom);
  const double* Krow = mom + (k + 1) * C::NPAD;
  const double* Qrow = mom + k * C::NPAD;
  const double* UT = P.UT;
  double* YB = P.YB;
  const uint16_t* PIDX = P.PIDX;
  auto Tj_at = [&](int j, int a, int b) -> double { return (double)mom[j * C::NPAD + PIDX[a * KMAX + b]]; };
  auto K_at = [&](int a, int b) -> double { return (double)Krow[PIDX[a * KMAX + b]]; };
  auto Q_at = [&](int a, int b) -> double { return (double)Qrow[PIDX[a * KMAX + b]]; };

  // ---- forward values: R, d_jl, b_j, sums ---------------------------------------------
  for (int e = tg; e < k * k; e += C::NTG) {
    const int a = e / k, b = e % k;
    double s = 0.0;
    for (int l = 0; l < pe; ++l) s = fma(UT[a * KMAX + l], UT[b * KMAX + l], s);
    Rm[a * KMAX + b] = s;
  }
  double part[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int e = tg; e < k * pe; e += C::NTG) {
    const int a = e / pe, l = e % pe;
    double kv = 0.0, qv = 0.0;
    for (int b = 0; b < k; ++b) {
      const double u = UT[b * KMAX + l];
      kv = fma(K_at(a, b), u, kv);
      qv = fma(Q_at(a, b), u, qv);
    }
    part[3] = fma(kv, kv, part[3]);
    part[4] = fma(UT[a * KMAX + l], qv, part[4]);
  }
  for (int j = 0; j < k; ++j) {
    for (int e = tg; e < k * pe; e += C::NTG) {
      const int a = e / pe, l = e % pe;
      double yv = 0.0;
      for (int b = 0; b < k; ++b) yv = fma(Tj_at(j, a, b), UT[b * KMAX + l], yv);
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
        Db[j * KMAX + l1] = gv;                      // d_jl (forward value for now)
      }
    }
    double tv[1] = {trg};
    group_sum<C::NW, 1>(tv, P.RED, tg);
    if (tg == 0) {
      const double bj = (double)mom[j * C::NPAD + np] - tv[0];
      SC[16 + j] = bj;                               // b_j
      part[2] = fma(bj, bj, part[2]);
    }
    gsync<C::NW>();
  }
  group_sum<C::NW, 5>(part, P.RED, tg);

  // ---- scalar adjoints -----------------------------------------------------------------
  const double km1 = (double)(k - 1);
  const int64_t q = m - pe;
  const double qq = variant == 0 ? (double)q : (double)(q + 2);
  const double tau = tauk / km1;
  double t_null = 0.0;
  if (q > 0) {
    const double tM = variant == 0 ? part[3] : part[4];
    t_null = (part[2] + 2.0 * (tauk - 2.0 * tM + part[1])) / (km1 * qq);
  }
  const double inner = 0.5 * (part[0] / km1 + t_null) + 0.5 * tau;
  const double sgn = inner > 0.0 ? 1.0 : (inner < 0.0 ? -1.0 : 0.0);
  const double a_in = (double)gk * sgn;
  const double cR = 0.5 * a_in / km1;
  double cA = 0.0, cG = 0.0, cM = 0.0, cT = 0.5 * a_in / km1;
  if (q > 0) {
    cA = 0.5 * a_in / (km1 * qq);
    cG = a_in / (km1 * qq);
    cM = -2.0 * a_in / (km1 * qq);
    cT += a_in / (km1 * qq);
  }

  // ---- R_bar, T_bar ---------------------------------------------------------------------
  // R_bar = -sum_j bb_j T_j + 2 cG sum_j T_j R T_j + cM (K K | Q),  bb_j = 2 cA b_j
  // T_bar_j = -bb_j R + 2 cG R T_j R + Ut diag(2 cR d_j) Ut^T
  for (int e = tg; e < k * k; e += C::NTG) {
    const int a = e / k, b = e % k;
    double s = 0.0;
    if (variant == 0) {
      for (int c = 0; c < k; ++c) s = fma(K_at(a, c), K_at(c, b), s);
    } else {
      s = Q_at(a, b);
    }
    Rb[a * KMAX + b] = cM * s;
  }
  gsync<C::NW>();
  for (int j = 0; j < k; ++j) {
    const double bb = 2.0 * cA * SC[16 + j];
    // W1 = T_j R
    for (int e = tg; e < k * k; e += C::NTG) {
      const int a = e / k, b = e % k;
      double s = 0.0;
      for (int c = 0; c < k; ++c) s = fma(Tj_at(j, a, c), Rm[c * KMAX + b], s);
      W1[a * KMAX + b] = s;
    }
    gsync<C::NW>();
    // R_bar += 2 cG W1 T_j - bb T_j ;  T_bar_j = -bb R + 2 cG R W1 + Ut diag(2 cR d_j) Ut^T
    for (int e = tg; e < k * k; e += C::NTG) {
      const int a = e / k, b = e % k;
      double s1 = 0.0, s2 = 0.0, s3 = 0.0;
      for (int c = 0; c < k; ++c) {
        s1 = fma(W1[a * KMAX + c], Tj_at(j, c, b), s1);
        s2 = fma(Rm[a * KMAX + c], W1[c * KMAX + b], s2);
      }
      for (int l = 0; l < pe; ++l) s3 = fma(UT[a * KMAX + l] * (2.0 * cR * Db[j * KMAX + l]), UT[b * KMAX + l], s3);
      Rb[a * KMAX + b] += 2.0 * cG * s1 - bb * Tj_at(j, a, b);
      if (a <= b) Tb[j * E::NPM + pair_index(a, b, k)] = -bb * Rm[a * KMAX + b] + 2.0 * cG * s2 + s3;
    }
    gsync<C::NW>();
  }
  // r_bar_j = bb_j
  if (tg < k) rbf[tg] = 2.0 * cA * SC[16 + tg];

  // ---- Ut_bar from t_range: Ut_bar[:, l] = sum_j 4 cR d_jl T_j ut_l ----------------------------
  for (int e = tg; e < k * pe; e += C::NTG) {
    const int a = e / pe, l = e % pe;
    double s = 0.0;
    for (int j = 0; j < k; ++j) {
      double y = 0.0;
      for (int b = 0; b < k; ++b) y = fma(Tj_at(j, a, b), UT[b * KMAX + l], y);
      s = fma(4.0 * cR * Db[j * KMAX + l], y, s);
    }
    Ub[a * KMAX + l] = s;
  }
  gsync<C::NW>();

  // ---- eigen adjoint: K_bar += U (diag(sig_bar) + F o (U^T U_bar)) U^T, F regularised ------
  // U columns in eigen order: column l of U is JV[:, ord[l]]; U_bar[:, l] = Ut_bar[:, l] sigma_l^{-1/2}
  constexpr int KK = C::KK;                         // every eigen column of the padded solve
  const double eta = (double)gap_eps * sig0;
  for (int e = tg; e < KK * pe; e += C::NTG) {
    const int x = e / pe, l = e % pe;                // M[x][l], x over all eigen columns
    const int ox = P.ord[x], ol = P.ord[l];
    const double sl = P.JA[ol * C::JLD + ol];
    const double isq = 1.0 / sqrt(sl);
    double a = 0.0;                                  // (U^T Ut_bar)[x][l]
    for (int r = 0; r < k; ++r) a = fma(P.JV[r * C::JLD + ox], Ub[r * KMAX + l], a);
    double v;
    if (x == l) {
      v = -0.5 * isq / sl * a;                       // sig_bar_l
    } else {
      const double sx = P.JA[ox * C::JLD + ox];
      const double dlt = sl - sx;
      v = dlt / (dlt * dlt + eta * eta) * (a * isq);
    }
    W2[x * KMAX + l] = v;
  }
  gsync<C::NW>();
  // Kb = U M U^T (M has nonzero columns l < pe only), symmetrised below
  for (int e = tg; e < k * k; e += C::NTG) {
    const int a = e / k, b = e % k;
    double s = 0.0;
    for (int l = 0; l < pe; ++l) {
      double t = 0.0;
      for (int x = 0; x < KK; ++x) t = fma(P.JV[a * C::JLD + P.ord[x]], W2[x * KMAX + l], t);
      s = fma(t, P.JV[b * C::JLD + P.ord[l]], s);
    }
    Kb[a * KMAX + b] = s;
  }
  gsync<C::NW>();
  // ---- K_bar += -R R_bar_sym R (+ cM (R K + K R) on the printed reading); Q_bar = cM R -------
  for (int e = tg; e < k * k; e += C::NTG) {
    const int a = e / k, b = e % k;
    double s = 0.0;
    for (int c = 0; c < k; ++c) s = fma(Rm[a * KMAX + c], 0.5 * (Rb[c * KMAX + b] + Rb[b * KMAX + c]), s);
    W1[a * KMAX + b] = s;                            // R R_bar_sym
  }
  gsync<C::NW>();
  for (int e = tg; e < k * k; e += C::NTG) {
    const int a = e / k, b = e % k;
    double s = 0.0, t = 0.0;
    for (int c = 0; c < k; ++c) {
      s = fma(W1[a * KMAX + c], Rm[c * KMAX + b], s);
      if (variant == 0) t = fma(Rm[a * KMAX + c], K_at(c, b), fma(K_at(a, c), Rm[c * KMAX + b], t));
    }
    W2[a * KMAX + b] = -s + cM * t;
  }
  gsync<C::NW>();
  for (int e = tg; e < k * k; e += C::NTG) {
    const int a = e / k, b = e % k;
    const double kb = 0.5 * (Kb[a * KMAX + b] + Kb[b * KMAX + a]) + 0.5 * (W2[a * KMAX + b] + W2[b * KMAX + a]);
    Kbf[a * KMAX + b] = kb;
    Qbf[a * KMAX + b] = variant == 0 ? 0.0 : cM * Rm[a * KMAX + b];
  }
  // ---- Theta[pair(a,b)][i] = w_ab (T_bar_i[a][b] + T_bar_a[i][b] + T_bar_b[i][a]) ----------------
  for (int e = tg; e < np * k; e += C::NTG) {
    const int pi = e / k, ii = e % k;
    int r = pi, a = 0;
    while (r >= k - a) { r -= k - a; ++a; }
    const int b = a + r;
    const double th = Tb[ii * E::NPM + pi] + Tb[a * E::NPM + pair_index(ii, b, k)] +
                      Tb[b * E::NPM + pair_index(ii, a, k)];
    TH[pi * KMAX + ii] = (a == b ? 1.0 : 2.0) * th;
  }
  gsync<C::NW>();

  // ---- second pass over the patch: column gradients, un-centring, scatter-add ----------------
  // float64 throughout: the terms cancel strongly on thin patches (small m, large k).
  const double cT2 = 2.0 * cT;
  for (int64_t c0 = (int64_t)w * WAVE; c0 < m; c0 += (int64_t)C::NW * WAVE) {
    const int64_t c = c0 + lane;
    float xf[KMAX];
    load_chunk<KMAX>(xf, X, ldx, P.nb, k, m, c0, lane);
    double xr[KMAX];
    centre_column_f64<KMAX>(xf, xr, k);              // the forward moments' centred values
    double qc = 0.0;
#pragma unroll
    for (int a = 0; a < KMAX; ++a) qc = fma(xr[a], xr[a], qc);
    double g[KMAX];
#pragma unroll
    for (int a = 0; a < KMAX; ++a) g[a] = 0.0;
    // sum_{a<=b} Theta[ab][i] x_a x_b
    int pi = 0;
#pragma unroll
    for (int a = 0; a < KMAX; ++a) {
      if (a < k) {
#pragma unroll
        for (int b = a; b < KMAX; ++b) {
          if (b < k) {
            const double pab = xr[a] * xr[b];
            const double* th = TH + pi * KMAX;
#pragma unroll
            for (int ii = 0; ii < KMAX; ++ii) g[ii] = fma(th[ii], pab, g[ii]);
            ++pi;
          }
        }
      }
    }
    // + 2 (K_bar x)_i + 2 q (Q_bar x)_i + 2 x_i (x^T Q_bar x) + r_bar_i + 2 cT x_i
    double xqx = 0.0;
    double qx[KMAX];
#pragma unroll
    for (int a = 0; a < KMAX; ++a) {
      double kx = 0.0, qa = 0.0;
#pragma unroll
      for (int b = 0; b < KMAX; ++b) {
        if (a < k && b < k) {
          kx = fma(Kbf[a * KMAX + b], xr[b], kx);
          qa = fma(Qbf[a * KMAX + b], xr[b], qa);
        }
      }
      qx[a] = qa;
      g[a] += 2.0 * kx + rbf[a] * (a < k ? 1.0 : 0.0) + cT2 * xr[a];
      xqx = fma(xr[a], qa, xqx);
    }
    double mean = 0.0;
#pragma unroll
    for (int a = 0; a < KMAX; ++a) {
      if (a < k) {
        g[a] += 2.0 * qc * qx[a] + 2.0 * xr[a] * xqx;
        mean += g[a];
      }
    }
    mean /= (double)k;
    if (c < m) {
#pragma unroll
      for (int a = 0; a < KMAX; ++a)
        if (a < k) unsafeAtomicAdd(grad + (int64_t)P.nb[a] * ldx + c, (float)(g[a] - mean));
    }
  }
}

template <int KMAX>
static hipError_t launch_bwd_k(const float* X, int64_t n, int64_t m, int64_t ldx,
                               const int32_t* idx, int k, int variant, const float* gk,
                               float gap_eps, float* grad, hipStream_t stream) {
  using C = typename BwdCfgSel<KMAX>::C;
  static std::atomic<uint64_t> attr_set{0};   // LDS beyond 64 KiB needs the opt-in attribute
  once_per_device(attr_set, [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&curv_backward_kernel<KMAX>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::BYTES);
    (void)hipGetLastError();
  });
  timing_begin(8, stream);
  hipLaunchKernelGGL(curv_backward_kernel<KMAX>, dim3((unsigned)n), dim3(C::NT), C::BYTES, stream, X,
                     n, m, ldx, idx, k, variant, gk, gap_eps, grad);
  timing_end(8, stream);
  return hipGetLastError();
}

hipError_t launch_curv_backward(const float* X, int64_t n, int64_t m, int64_t ldx,
                                const int32_t* idx, int k, int variant, const float* gk,
                                float gap_eps, float* grad, hipStream_t stream) {
  if (k <= 4) return launch_bwd_k<4>(X, n, m, ldx, idx, k, variant, gk, gap_eps, grad, stream);
  if (k <= 8) return launch_bwd_k<8>(X, n, m, ldx, idx, k, variant, gk, gap_eps, grad, stream);
  if (k <= 12) return launch_bwd_k<12>(X, n, m, ldx, idx, k, variant, gk, gap_eps, grad, stream);
  if (k <= 16) return launch_bwd_k<16>(X, n, m, ldx, idx, k, variant, gk, gap_eps, grad, stream);
  return hipErrorInvalidValue;
}

}  // namespace mc
