// Exact-mode curvature (Theorem 1, eq. kappa_final) with a canonical null basis (gfx950).
//
// kappa = |1/2 v^T (C o C) 1 + 1/2 sum v| with C = W^T (W o W), W = [V_r | Q_null] and
// v = (lambda_r, 0, ..., 0).  Splitting the columns of W into the range and the null
// space (eq. split) gives kappa = |(t_range + t_null^W)/2 + tau/2| with
//   t_range  = ||X_c V_r^{o2}||_F^2 / (k-1)
//   t_null^W = sum_{l >= p} ||X_c (w_l o w_l)||^2 / (k-1),
// because sum_s lambda_s v_s v_s^T = X_c^T X_c/(k-1).  The paper's Exact branch takes
// the null columns from an m x m eigensolver, which makes kappa depend on that solver
// whenever m > rank.  Here Q_null is fixed: the trailing m - p columns of the Householder
// QR of V_r in LAPACK's convention (dlarfg: beta = -sign(alpha) ||x||, tau = (beta -
// alpha)/beta), held in compact WY form Q = I - Y T Y^T, so w_l = e_l - Y T y_l with y_l
// row l of Y.  Cost O((k + p) m^2) per point instead of the eigensolver's O(m^3).
//
// One workgroup (4 waves) per point.  V_r (float64), the gathered rows (float32) and the
// per-column means (float64) live in LDS, which bounds m * (8 p + 4 k + 8) (checked on the
// host).  Centred values are formed in float64 exactly as in the moment pass.
#include "curv_core.h"
#include "mc_internal.h"

namespace mc {

constexpr size_t EXACT_LDS_MAX = 150 * 1024;   // bytes for V_r + patch + T on top of the core

template <int KMAX>
struct ExactCfgSel {
  using C = CurvCfg<KMAX, 4, 1, 0, 8>;   // float64 moments: an exact Gram for the basis
};

__device__ __forceinline__ double block_sum256(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  const double s = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return s;
}

template <int KMAX>
__global__ __launch_bounds__(256) void curv_exact_kernel(
    const float* __restrict__ X, int64_t n, int64_t m, int64_t ldx, const int32_t* __restrict__ idx,
    int k, float* __restrict__ kappa_out, uint8_t* __restrict__ flags_out) {
  using C = typename ExactCfgSel<KMAX>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tg = threadIdx.x;
  const int64_t i = blockIdx.x;
  const PointLds P = point_lds<C>(smem);
  double tauk, sig0;
  int pe, sweep;
  const uint8_t bad = patch_front<KMAX, C, MOM_FP64>(P, X, n, m, ldx, idx, k, i, tg, tauk, sig0, pe, sweep);
  if (bad) {
    if (tg == 0) {
      kappa_out[i] = __builtin_nanf("");
      if (flags_out) flags_out[i] = bad;
    }
    return;
  }
  const int plim = (int)((int64_t)(k - 1) < m ? (int64_t)(k - 1) : m);
  uint8_t fl = 0;
  if (pe < plim) fl |= PF_RANK_DEFICIENT;
  if (sweep >= JAC_MAX_SWEEPS) fl |= PF_JACOBI_MAXSWEEPS;
  if (!(sig0 > 0.0) || tauk == 0.0 || pe == 0) {
    if (tg == 0) {
      kappa_out[i] = 0.0f;
      if (flags_out) flags_out[i] = fl | PF_DEGENERATE;
    }
    return;
  }
  // exact-mode buffers after the core region
  double* Vd = reinterpret_cast<double*>(smem + C::BYTES);                 // m x pe, row-major
  float* Xs = reinterpret_cast<float*>(smem + C::BYTES + (size_t)m * pe * 8);   // k x m, raw rows
  double* mu = reinterpret_cast<double*>(smem + C::BYTES + (size_t)m * pe * 8 +
                                         (((size_t)k * m * 4 + 15) & ~(size_t)15));   // m column means
  double* Tf = mu + m;
  double* tau_h = Tf + KMAX * KMAX;                                        // reflector scalars
  double* red = tau_h + KMAX;                                              // 4 doubles
  double* wv = red + 8;                                                    // KMAX doubles

  // ---- gathered rows and column means into LDS ----------------------------------------------
  // X_c[j, c] = (Xs[j, c] - Xs[0, c]) - mu[c] in float64: the same values as the moment pass.
  for (int64_t c0 = (int64_t)(tg / WAVE) * WAVE; c0 < m; c0 += 256) {
    float xr[KMAX];
    load_chunk<KMAX>(xr, X, ldx, P.nb, k, m, c0, tg % WAVE);
    const int64_t c = c0 + tg % WAVE;
    if (c < m) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < KMAX; ++j)
        if (j < k) {
          Xs[(int64_t)j * m + c] = xr[j];
          s += (double)xr[j] - (double)xr[0];
        }
      mu[c] = s / (double)k;
    }
  }
  __syncthreads();
  auto xcen = [&](int j, int64_t a) -> double {
    return ((double)Xs[(int64_t)j * m + a] - (double)Xs[a]) - mu[a];
  };
  const int lane = tg % WAVE, wid = tg / WAVE;
  const int li = lane % 16, lq = lane / 16;
  const int mm = (int)m;                       // m * pe values fit the LDS, so int indices
  const int pp = pe;
  // the staged-chunk / moment storage of patch_front is free from here on: small products
  // and reductions go there
  constexpr int MT = (KMAX + 15) / 16;         // 16-wide tiles of a KMAX-sized index
  constexpr int SLD = 16 * MT;                 // row stride of a small product in scr
  static_assert(C::U0_B >= sizeof(double) * SLD * SLD, "scratch for the small products");
  static_assert(C::U0_B >= sizeof(double) * 4 * KMAX, "scratch for the vector reductions");
  double* scr = reinterpret_cast<double*>(P.lhs);
  // scr[i][n] = sum_{a < m} fa(i, a) fb(n, a) for i, n < SLD on float64 MFMA: wave w takes the
  // K-steps a0 = 16 t + 4 w (lane l supplies A[l%16][l/16] and B[l/16][l%16]), and the four
  // partial products are added in wave order (deterministic).  fa, fb are 0 out of range.
  auto small_product = [&](auto fa, auto fb) {
    doublex4 acc[MT][MT];
#pragma unroll
    for (int ti = 0; ti < MT; ++ti)
#pragma unroll
      for (int tn = 0; tn < MT; ++tn) acc[ti][tn] = doublex4{0.0, 0.0, 0.0, 0.0};
    for (int a0 = 4 * wid; a0 < mm; a0 += 16) {
      const int a = a0 + lq;
      double av[MT], bv[MT];
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        av[t] = a < mm ? fa(16 * t + li, a) : 0.0;
        bv[t] = a < mm ? fb(16 * t + li, a) : 0.0;
      }
#pragma unroll
      for (int ti = 0; ti < MT; ++ti)
#pragma unroll
        for (int tn = 0; tn < MT; ++tn) acc[ti][tn] = mfma16x16x4f64(av[ti], bv[tn], acc[ti][tn]);
    }
    for (int w = 0; w < 4; ++w) {
      if (wid == w) {
#pragma unroll
        for (int ti = 0; ti < MT; ++ti)
#pragma unroll
          for (int tn = 0; tn < MT; ++tn)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              double& cell = scr[(16 * ti + lq + 4 * r) * SLD + 16 * tn + li];
              cell = (w == 0 ? 0.0 : cell) + acc[ti][tn][r];
            }
      }
      __syncthreads();
    }
  };
  // ---- V_r = X_c^T Ut (float64), and t_range = ||X_c V_r^{o2}||^2 ------------------------
  for (int64_t e = tg; e < m * pe; e += 256) {
    const int64_t a = e / pe;
    const int l = (int)(e % pe);
    double s = 0.0;
    for (int j = 0; j < k; ++j) s = fma(xcen(j, a), P.UT[j * KMAX + l], s);
    Vd[a * pe + l] = s;
  }
  __syncthreads();
  small_product([&](int i, int a) { return i < k ? xcen(i, a) : 0.0; },
                [&](int n, int a) {
                  const double v = n < pp ? Vd[a * pp + n] : 0.0;
                  return v * v;
                });
  double trange = 0.0;
  for (int e = tg; e < k * pe; e += 256) {
    const double v = scr[(e / pe) * SLD + e % pe];
    trange = fma(v, v, trange);
  }
  trange = block_sum256(trange, red);

  // ---- Householder QR of V_r in place (LAPACK geqr2 / dlarfg convention) --------------------
  // Step j: one pass gives ||x||^2 (c = j) and the column products dots[c] = sum_{a > j}
  // V[a][j] V[a][c] (c > j) of the unscaled reflector, one vector reduction sums them, and
  // with v = scal V[:, j] (v_j = 1) the update is V[:, c] -= tau (V[j][c] + scal dots[c]) v.
  for (int j = 0; j < pe; ++j) {
    double part[KMAX], vjc[KMAX];
#pragma unroll
    for (int c = 0; c < KMAX; ++c) part[c] = 0.0;
    for (int a = j + 1 + tg; a < mm; a += 256) {
      const double vj = Vd[a * pp + j];
#pragma unroll
      for (int c = 0; c < KMAX; ++c)
        if (c >= j && c < pp) part[c] = fma(vj, Vd[a * pp + c], part[c]);
    }
    // V[j][c] before the reduction's barriers: thread 0 rewrites the row below
#pragma unroll
    for (int c = 0; c < KMAX; ++c) vjc[c] = (c > j && c < pp) ? Vd[j * pp + c] : 0.0;
#pragma unroll
    for (int c = 0; c < KMAX; ++c) {
      const double ws = (c >= j && c < pp) ? wave_sum(part[c]) : 0.0;
      if (lane == 0) scr[wid * KMAX + c] = ws;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
      part[c] = (scr[c] + scr[KMAX + c]) + (scr[2 * KMAX + c] + scr[3 * KMAX + c]);
    const double alpha = Vd[j * pp + j];
    __syncthreads();   // everyone has read scr and alpha
    double xnorm2 = 0.0;
#pragma unroll
    for (int c = 0; c < KMAX; ++c) xnorm2 = c == j ? part[c] : xnorm2;
    double tauj = 0.0, scal = 0.0, beta = alpha;
    if (xnorm2 > 0.0) {
      const double nrm = sqrt(alpha * alpha + xnorm2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tauj = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    double f[KMAX];
#pragma unroll
    for (int c = 0; c < KMAX; ++c) f[c] = (c > j && c < pp) ? tauj * (vjc[c] + scal * part[c]) : 0.0;
    if (tauj != 0.0) {
      for (int a = j + 1 + tg; a < mm; a += 256) {
        const double va = Vd[a * pp + j] * scal;   // v below the diagonal
        Vd[a * pp + j] = va;
#pragma unroll
        for (int c = 0; c < KMAX; ++c)
          if (c > j && c < pp) Vd[a * pp + c] -= f[c] * va;
      }
    }
    if (tg == 0) {
      Vd[j * pp + j] = beta;
      tau_h[j] = tauj;
#pragma unroll
      for (int c = 0; c < KMAX; ++c)
        if (c > j && c < pp) Vd[j * pp + c] = vjc[c] - f[c];
    }
    __syncthreads();
  }
  // ---- compact WY factor T (LAPACK dlarft, forward, columnwise) -----------------------------
  // Y[:, j] = (0..0, 1, Vd[j+1:, j]);  T[j][j] = tau_j;  T[0:j, j] = -tau_j T[0:j, 0:j] (Y^T y_j)[0:j],
  // with the Gram Y^T Y from one float64 MFMA product
  auto yval = [&](int s, int a) -> double {
    if (s >= pp) return 0.0;
    return a > s ? Vd[a * pp + s] : (a == s ? 1.0 : 0.0);
  };
  small_product(yval, yval);
  for (int j = 0; j < pe; ++j) {
    if (tg < j) wv[tg] = -tau_h[j] * scr[tg * SLD + j];
    __syncthreads();
    if (tg < j) {
      double t = 0.0;
      for (int s = tg; s < j; ++s) t = fma(Tf[tg * KMAX + s], wv[s], t);   // T upper triangular
      Tf[tg * KMAX + j] = t;
    }
    if (tg == 0) Tf[j * KMAX + j] = tau_h[j];
    __syncthreads();
  }
  // ---- null columns: w_l = e_l - Y z_l, z_l = T y_l,  t_null^W = sum_l ||X_c (w_l o w_l)||^2 ----------
  // Two float64 MFMA products per block of 16 null columns: D = Y Z_blk over 16-row blocks of
  // a (K = pe, padded to 4 KS1), W2 = (E - D)^2 in registers, then acc += X_c W2 (K = the
  // block's 16 rows).  The 16x16x4 f64 product leaves lane l holding rows l/16 + 4r of column
  // l%16, which is exactly the B operand of the r-th K-step of the second product, so W2
  // never leaves the registers.  Each wave takes NCB column blocks at once (blocks
  // 4 (NCB g + c) + w): they share every Y and X_c operand, and their MFMA chains are
  // independent.  Operands are read at clamped (always valid) LDS addresses and masked.
  constexpr int KS1 = (KMAX + 3) / 4;          // K-steps over the reflectors
  constexpr int JT = (KMAX + 15) / 16;         // 16-row tiles of X_c
  constexpr int NCB = 4;                       // column blocks per wave and pass
  const int ncb = (mm - pp + 15) / 16, nrb = (mm + 15) / 16;
  double tnull = 0.0;
  for (int g0 = 0; g0 * 4 * NCB < ncb; ++g0) {
    int ln[NCB];
    double zb[NCB][KS1];
    doublex4 acc2[NCB][JT];
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
      const int cb = 4 * (NCB * g0 + c) + wid;
      ln[c] = pp + 16 * cb + li;                 // null column of this lane's B operands
      const int lnc = ln[c] < mm ? ln[c] : mm - 1;
      // z_l[s] = sum_{u >= s} T[s][u] y_l[u], y_l = row l of Y (below the diagonal: l >= pe > u)
#pragma unroll
      for (int st = 0; st < KS1; ++st) {
        const int sidx = 4 * st + lq;
        double t = 0.0;
        if (sidx < pp && ln[c] < mm)
          for (int u = sidx; u < pp; ++u) t = fma(Tf[sidx * KMAX + u], Vd[lnc * pp + u], t);
        zb[c][st] = t;
      }
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) acc2[c][jt] = doublex4{0.0, 0.0, 0.0, 0.0};
    }
    for (int rb = 0; rb < nrb; ++rb) {
      const int a0 = 16 * rb;
      // A operands of the first product: Y[a0 + li][4 st + lq]
      double yv[KS1];
      {
        const int a = a0 + li, ac = a < mm ? a : mm - 1;
#pragma unroll
        for (int st = 0; st < KS1; ++st) {
          const int sidx = 4 * st + lq, sc = sidx < pp ? sidx : pp - 1;
          const double raw = Vd[ac * pp + sc];
          yv[st] = (sidx < pp && a < mm) ? (a > sidx ? raw : (a == sidx ? 1.0 : 0.0)) : 0.0;
        }
      }
      // A operands of the second product: X_c[16 jt + li][a0 + 4 r + lq]
      double xa[4][JT];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ax = a0 + 4 * r + lq, axc = ax < mm ? ax : mm - 1;
        const double x0 = (double)Xs[axc], mua = mu[axc];
#pragma unroll
        for (int jt = 0; jt < JT; ++jt) {
          const int jj = 16 * jt + li, jc = jj < k ? jj : k - 1;
          const double v = ((double)Xs[jc * mm + axc] - x0) - mua;
          xa[r][jt] = (jj < k && ax < mm) ? v : 0.0;
        }
      }
      // the NCB chains interleave step by step: D for every block, then W2, then X_c W2
      doublex4 d[NCB];
#pragma unroll
      for (int c = 0; c < NCB; ++c) d[c] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int st = 0; st < KS1; ++st)
#pragma unroll
        for (int c = 0; c < NCB; ++c) d[c] = mfma16x16x4f64(yv[st], zb[c][st], d[c]);
      // W2 = (E - D)^2 on this lane's rows a0 + lq + 4 r of column ln[c]
      double w2[NCB][4];
#pragma unroll
      for (int c = 0; c < NCB; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = a0 + lq + 4 * r;
          double wa = (a == ln[c] ? 1.0 : 0.0) - d[c][r];
          if (a >= mm || ln[c] >= mm) wa = 0.0;
          w2[c][r] = wa * wa;
        }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int jt = 0; jt < JT; ++jt)
#pragma unroll
          for (int c = 0; c < NCB; ++c) acc2[c][jt] = mfma16x16x4f64(xa[r][jt], w2[c][r], acc2[c][jt]);
    }
    // rows past k and columns past m are zero
#pragma unroll
    for (int c = 0; c < NCB; ++c)
#pragma unroll
      for (int jt = 0; jt < JT; ++jt)
#pragma unroll
        for (int r = 0; r < 4; ++r) tnull = fma(acc2[c][jt][r], acc2[c][jt][r], tnull);
  }
  tnull = block_sum256(tnull, red);

  if (tg == 0) {
    const double km1 = (double)(k - 1);
    const double kap = fabs(0.5 * (trange / km1 + tnull / km1) + 0.5 * tauk / km1);
    kappa_out[i] = (float)kap;
    if (flags_out) flags_out[i] = fl;
  }
}

template <int KMAX>
static size_t exact_lds_bytes(int64_t m, int k) {
  using C = typename ExactCfgSel<KMAX>::C;
  const int p = k - 1;
  return C::BYTES + (size_t)m * p * 8 + (((size_t)k * m * 4 + 15) & ~(size_t)15) + (size_t)m * 8 +
         (size_t)(KMAX * KMAX + KMAX + 8 + KMAX) * 8;
}

static size_t exact_bytes(int64_t m, int k) {
  if (k <= 4) return exact_lds_bytes<4>(m, k);
  if (k <= 8) return exact_lds_bytes<8>(m, k);
  if (k <= 12) return exact_lds_bytes<12>(m, k);
  if (k <= 16) return exact_lds_bytes<16>(m, k);
  if (k <= 20) return exact_lds_bytes<20>(m, k);
  if (k <= 24) return exact_lds_bytes<24>(m, k);
  if (k <= 28) return exact_lds_bytes<28>(m, k);
  return exact_lds_bytes<32>(m, k);
}

bool curv_exact_fits(int64_t m, int k) { return exact_bytes(m, k) <= EXACT_LDS_MAX; }

size_t curv_exact_ws_bytes(int64_t, int64_t, int) { return 256; }

template <int KMAX>
static hipError_t launch_exact_k(const float* X, int64_t n, int64_t m, int64_t ldx,
                                 const int32_t* idx, int k, float* kappa, uint8_t* flags,
                                 hipStream_t stream) {
  const size_t lds = exact_lds_bytes<KMAX>(m, k);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&curv_exact_kernel<KMAX>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)hipGetLastError();
  timing_begin(7, stream);
  hipLaunchKernelGGL(curv_exact_kernel<KMAX>, dim3((unsigned)n), dim3(256), lds, stream, X, n, m, ldx,
                     idx, k, kappa, flags);
  timing_end(7, stream);
  return hipGetLastError();
}

hipError_t launch_curv_exact(const float* X, int64_t n, int64_t m, int64_t ldx, const int32_t* idx,
                             int k, float* kappa, uint8_t* flags, void* ws, hipStream_t stream) {
  (void)ws;
  if (k <= 4) return launch_exact_k<4>(X, n, m, ldx, idx, k, kappa, flags, stream);
  if (k <= 8) return launch_exact_k<8>(X, n, m, ldx, idx, k, kappa, flags, stream);
  if (k <= 12) return launch_exact_k<12>(X, n, m, ldx, idx, k, kappa, flags, stream);
  if (k <= 16) return launch_exact_k<16>(X, n, m, ldx, idx, k, kappa, flags, stream);
  if (k <= 20) return launch_exact_k<20>(X, n, m, ldx, idx, k, kappa, flags, stream);
  if (k <= 24) return launch_exact_k<24>(X, n, m, ldx, idx, k, kappa, flags, stream);
  if (k <= 28) return launch_exact_k<28>(X, n, m, ldx, idx, k, kappa, flags, stream);
  return launch_exact_k<32>(X, n, m, ldx, idx, k, kappa, flags, stream);
}

}  // namespace mc
