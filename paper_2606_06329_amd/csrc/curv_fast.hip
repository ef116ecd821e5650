// Fused Fast-mode mean curvature, one point per wave (k <= 20) or per workgroup (gfx950).
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
//   T[j][a][b] = sum_c X_c[j,c] X_c[a,c] X_c[b,c]    (third moments)
//   Q[a][b]    = sum_c q_c X_c[a,c] X_c[b,c],  q_c = sum_j X_c[j,c]^2
//   r_j        = sum_c X_c[j,c]
//   G_j = Ut^T T_j Ut,  t_range = sum_j sum_l G_j[l,l]^2,  g = sum_j ||G_j||^2,
//   (X_c d_P)_j = r_j - tr G_j,  t_S = sum_l ||K ut_l||^2,  t_D = sum_l ut_l^T Q ut_l
// (each divided by k-1).  The moments are one MFMA GEMM over the m columns:
//   [X_c ; q ; 1] (k+2 x m)  times  [X_c[a] o X_c[b] (a<=b) | 1] (m x k(k+1)/2+1).
// The m loop streams the patch through LDS in chunks of 64 columns (coalesced
// row reads of the k gathered rows); the k x k eigen-solve is a parallel-order
// cyclic Jacobi in float64 and the combination is float64.
#include <math.h>

#include "mc_device.h"
#include "mc_internal.h"

namespace mc {

constexpr int FCH = 64;        // patch columns per staged chunk
constexpr int FLDX = FCH + 1;  // LDS row stride (floats) of a staged chunk
constexpr int JAC_MAX_SWEEPS = 40;

template <int KMAX>
struct FastCfg {
  static constexpr int MB = (KMAX + 2 + 15) / 16;           // 16-row blocks of the LHS
  static constexpr int ROWS = (16 * MB > KMAX + 3) ? 16 * MB : KMAX + 3;
  static constexpr int NPC = KMAX * (KMAX + 1) / 2 + 1;     // pair columns + ones column
  static constexpr int NB = (NPC + 15) / 16;                // 16-column blocks of the RHS
  static constexpr int NW = KMAX <= 20 ? 1 : (KMAX <= 26 ? 2 : 4);   // waves per point
  static constexpr int PPW = NW == 1 ? 4 : 1;               // points per workgroup
  static constexpr int NTG = NW * WAVE;                     // threads per point
  static constexpr int NT = PPW * NTG;                      // threads per workgroup
  static constexpr int NBW = (NB + NW - 1) / NW;            // RHS blocks per wave
  static constexpr int KK = (KMAX + 1) & ~1;                // even Jacobi size
  static constexpr int JLD = KK + 1;                        // Jacobi row stride (doubles)
  static constexpr int NPAD = NB * 16;
  // LDS layout of one point (bytes); the staged chunk and the moments share storage.
  static constexpr size_t LHS_B = (size_t)ROWS * FLDX * 4;
  static constexpr size_t MOM_B = (size_t)(KMAX + 2) * NPAD * 4;
  static constexpr size_t U0_B = LHS_B > MOM_B ? LHS_B : MOM_B;
  static constexpr size_t OFF_JA = (U0_B + 15) & ~(size_t)15;
  static constexpr size_t OFF_JV = OFF_JA + (size_t)KK * JLD * 8;
  static constexpr size_t OFF_UT = OFF_JV + (size_t)KK * JLD * 8;
  static constexpr size_t OFF_Y = OFF_UT + (size_t)KMAX * KMAX * 8;
  static constexpr size_t OFF_RED = OFF_Y + (size_t)KMAX * KMAX * 8;     // 16 doubles x NW
  static constexpr size_t OFF_ROT = OFF_RED + (size_t)16 * NW * 8;        // c, s per pair
  static constexpr size_t OFF_INT = OFF_ROT + (size_t)KK * 8;
  static constexpr size_t N_INT = KMAX + KK + 8;                          // nb, ord, misc
  static constexpr size_t OFF_PIDX = OFF_INT + N_INT * 4;
  static constexpr size_t OFF_PJ = OFF_PIDX + (size_t)KMAX * KMAX * 2;
  static constexpr size_t BYTES = (OFF_PJ + 2 * NPAD + 15) & ~(size_t)15;
};

// Index of pair (a, b), a <= b, in row-major upper-triangular order of a k x k matrix.
__device__ __forceinline__ int pair_index(int a, int b, int k) {
  if (a > b) { int t = a; a = b; b = t; }
  return a * k - (a * (a - 1)) / 2 + (b - a);
}

// Synchronise the threads of one point: a single wave needs only an LDS fence.
template <int NW>
__device__ __forceinline__ void gsync() {
  if constexpr (NW == 1) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Sum of NV doubles over the threads of one point; result valid in every thread.
template <int NW, int NV>
__device__ __forceinline__ void group_sum(double (&v)[NV], double* red, int tg) {
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if constexpr (NW > 1) {
    const int w = tg / WAVE, l = tg % WAVE;
    __syncthreads();
    if (l == 0) {
#pragma unroll
      for (int i = 0; i < NV; ++i) red[w * 16 + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int ww = 0; ww < NW; ++ww) s += red[ww * 16 + i];
      v[i] = s;
    }
    __syncthreads();
  }
}

// Lane `lane` of the staging wave holds column c0+lane of the k gathered rows in xr.
template <int KMAX>
__device__ __forceinline__ void load_chunk(float (&xr)[KMAX], const float* __restrict__ X,
                                           int64_t ldx, const int* nb, int k, int64_t m,
                                           int64_t c0, int lane) {
  const int64_t c = c0 + lane;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    float v = 0.0f;
    if (j < k && c < m) v = X[(int64_t)nb[j] * ldx + c];
    xr[j] = v;
  }
}

// Player at round-robin position `pos` in round r of the circle schedule on KK players.
__device__ __forceinline__ int rr_player(int pos, int r, int KK) {
  if (pos == 0) return 0;
  int t = pos - 1 + r;
  if (t >= KK - 1) t -= KK - 1;
  return t + 1;
}

template <int KMAX>
__global__ __launch_bounds__(FastCfg<KMAX>::NT) void curv_fast_kernel(
    const float* __restrict__ X, int64_t n, int64_t m, int64_t ldx, const int32_t* __restrict__ idx,
    int k, int variant, float* __restrict__ kappa_out, uint8_t* __restrict__ flags_out) {
  using C = FastCfg<KMAX>;
  extern __shared__ __align__(16) unsigned char smem_all[];
  const int gid = threadIdx.x / C::NTG;            // point group inside the workgroup
  const int tg = threadIdx.x % C::NTG;             // thread inside the group
  const int w = tg / WAVE;
  const int lane = tg % WAVE;
  const int64_t i = (int64_t)blockIdx.x * C::PPW + gid;
  if (i >= n) return;                              // whole group exits together
  unsigned char* smem = smem_all + (size_t)gid * C::BYTES;
  float* lhs = reinterpret_cast<float*>(smem);     // ROWS x FLDX (during the m loop)
  float* mom = reinterpret_cast<float*>(smem);     // (k+2) x NPAD (after the m loop)
  double* JA = reinterpret_cast<double*>(smem + C::OFF_JA);
  double* JV = reinterpret_cast<double*>(smem + C::OFF_JV);
  double* UT = reinterpret_cast<double*>(smem + C::OFF_UT);
  double* YB = reinterpret_cast<double*>(smem + C::OFF_Y);
  double* RED = reinterpret_cast<double*>(smem + C::OFF_RED);
  double* ROT = reinterpret_cast<double*>(smem + C::OFF_ROT);   // c[KK/2], s[KK/2]
  int* IN = reinterpret_cast<int*>(smem + C::OFF_INT);
  int* nb = IN;                       // [KMAX] neighbour rows
  int* ord = IN + KMAX;               // [KK] eigen order
  int* misc = ord + C::KK;            // [8] flags / counters
  uint16_t* PIDX = reinterpret_cast<uint16_t*>(smem + C::OFF_PIDX);
  unsigned char* pj1 = smem + C::OFF_PJ;
  unsigned char* pj2 = pj1 + C::NPAD;

  const int np = k * (k + 1) / 2;
  const int npc = np + 1;
  const int nbr = (npc + 15) / 16;    // RHS blocks in use

  // ---- setup: neighbour rows, pair tables, zero rows --------------------------------
  if (tg < 8) misc[tg] = 0;
  gsync<C::NW>();
  if (tg < k) {
    int v = idx[i * k + tg];
    if (v < 0 || (int64_t)v >= n) { misc[0] = 1; v = 0; }
    nb[tg] = v;
  }
  for (int t = tg; t < C::NPAD; t += C::NTG) {
    int a = k + 2, b = k + 2;          // zero row
    if (t < np) {
      int r = t;
      a = 0;
      while (r >= k - a) { r -= k - a; ++a; }
      b = a + r;
    } else if (t == np) {
      a = b = k + 1;                   // ones row: the column of ones
    }
    pj1[t] = (unsigned char)a;
    pj2[t] = (unsigned char)b;
  }
  for (int t = tg; t < k * k; t += C::NTG) PIDX[(t / k) * KMAX + t % k] = (uint16_t)pair_index(t / k, t % k, k);
  for (int t = tg; t < (C::ROWS - (k + 2)) * FLDX; t += C::NTG) lhs[(k + 2) * FLDX + t] = 0.0f;
  gsync<C::NW>();
  if (misc[0]) {
    if (tg == 0) {
      kappa_out[i] = __builtin_nanf("");
      if (flags_out) flags_out[i] = PF_NONFINITE;
    }
    return;
  }

  // ---- pass over the patch: moments on MFMA --------------------------------------
  floatx4 acc[C::MB][C::NBW];
#pragma unroll
  for (int a = 0; a < C::MB; ++a)
#pragma unroll
    for (int b = 0; b < C::NBW; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

  int off1[C::NBW], off2[C::NBW];
#pragma unroll
  for (int b = 0; b < C::NBW; ++b) {
    const int nbg = w + C::NW * b;
    const int pi = nbg * 16 + (lane % 16);
    const int pc = pi < C::NPAD ? pi : C::NPAD - 1;
    off1[b] = pj1[pc] * FLDX;
    off2[b] = pj2[pc] * FLDX;
  }

  float xr[KMAX];
  double tau64 = 0.0;
  bool nonfinite = false;
  if (w == 0) load_chunk<KMAX>(xr, X, ldx, nb, k, m, 0, lane);

  for (int64_t c0 = 0; c0 < m; c0 += FCH) {
    if (w == 0) {
      // centre the column at the patch mean (float32), written as the mean of the
      // offsets from the first row: equal rows give exactly zero, and the offsets
      // carry no cancellation from the magnitude of the coordinates
#pragma unroll
      for (int j = KMAX - 1; j >= 0; --j)
        if (j < k) xr[j] -= xr[0];
      float s = 0.0f;
#pragma unroll
      for (int j = 0; j < KMAX; ++j)
        if (j < k) s += xr[j];
      const float mean = s / (float)k;
      float q = 0.0f;
#pragma unroll
      for (int j = 0; j < KMAX; ++j) {
        if (j < k) {
          nonfinite |= !isfinite(xr[j]);
          const float xc = xr[j] - mean;
          q = fmaf(xc, xc, q);
          tau64 = fma((double)xc, (double)xc, tau64);
          lhs[j * FLDX + lane] = xc;
        }
      }
      lhs[k * FLDX + lane] = q;
      lhs[(k + 1) * FLDX + lane] = (c0 + lane < m) ? 1.0f : 0.0f;
    }
    gsync<C::NW>();
    if (w == 0 && c0 + FCH < m) load_chunk<KMAX>(xr, X, ldx, nb, k, m, c0 + FCH, lane);

    const int64_t rem = m - c0;
    const int steps = rem >= FCH ? FCH / 4 : (int)((rem + 3) / 4);
    for (int s = 0; s < steps; ++s) {
      const int col = 4 * s + lane / 16;
      float av[C::MB];
#pragma unroll
      for (int a = 0; a < C::MB; ++a) av[a] = lhs[(16 * a + lane % 16) * FLDX + col];
#pragma unroll
      for (int b = 0; b < C::NBW; ++b) {
        if (w + C::NW * b < nbr) {
          const float bv = lhs[off1[b] + col] * lhs[off2[b] + col];
#pragma unroll
          for (int a = 0; a < C::MB; ++a) acc[a][b] = mfma16x16x4(av[a], bv, acc[a][b]);
        }
      }
    }
    gsync<C::NW>();
  }

  // ---- moments to LDS ------------------------------------------------------------
  if (w == 0) {
    tau64 = wave_sum(tau64);
    const int nf = __any(nonfinite);
    if (lane == 0) {
      RED[15 * C::NW] = tau64;
      misc[1] = nf;
    }
  }
#pragma unroll
  for (int b = 0; b < C::NBW; ++b) {
    const int nbg = w + C::NW * b;
    if (nbg < nbr) {
      const int col = nbg * 16 + lane % 16;
#pragma unroll
      for (int a = 0; a < C::MB; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * a + 4 * (lane / 16) + r;
          if (row < k + 2 && col < npc) mom[row * C::NPAD + col] = acc[a][b][r];
        }
    }
  }
  gsync<C::NW>();
  const double tauk = RED[15 * C::NW];   // (k-1) * tau, float64 accumulation
  if (misc[1]) {
    if (tg == 0) {
      kappa_out[i] = __builtin_nanf("");
      if (flags_out) flags_out[i] = PF_NONFINITE;
    }
    return;
  }

  // ---- k x k eigen-solve: cyclic Jacobi, parallel (round-robin) order, float64 -------
  // Each round rotates KK/2 disjoint planes.  The update works on 2 x 2 blocks of A
  // (pair i x pair i') and on row x of V restricted to one pair, so every thread
  // reads and writes the same cells and the update runs in place.
  const int KK = (k + 1) & ~1;
  const int HP = KK / 2;
  const float* Krow = mom + (k + 1) * C::NPAD;
  double trace = 0.0;
  for (int e = tg; e < KK * KK; e += C::NTG) {
    const int x = e / KK, y = e % KK;
    JA[x * C::JLD + y] = (x < k && y < k) ? (double)Krow[PIDX[x * KMAX + y]] : 0.0;
    JV[x * C::JLD + y] = (x == y) ? 1.0 : 0.0;
  }
  for (int x = 0; x < k; ++x) trace += (double)Krow[PIDX[x * KMAX + x]];
  gsync<C::NW>();
  const double floor_abs = trace * 0x1p-100;
  int sweep = 0;
  for (; sweep < JAC_MAX_SWEEPS; ++sweep) {
    if (tg == 0) misc[2] = 0;
    for (int r = 0; r < KK - 1; ++r) {
      if (tg < HP) {
        const int pa = rr_player(tg, r, KK), pb = rr_player(KK - 1 - tg, r, KK);
        const int p = pa < pb ? pa : pb, q = pa < pb ? pb : pa;
        const double app = JA[p * C::JLD + p], aqq = JA[q * C::JLD + q], apq = JA[p * C::JLD + q];
        double c = 1.0, s = 0.0;
        const double thr = fmax(0x1p-52 * sqrt(fabs(app) * fabs(aqq)), floor_abs);
        if (fabs(apq) > thr) {
          const double theta = (aqq - app) / (2.0 * apq);
          const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
          misc[2] = 1;
        }
        ROT[tg] = c;
        ROT[C::KK / 2 + tg] = s;
      }
      gsync<C::NW>();
      // A <- J^T A J on 2 x 2 blocks; V <- V J on row pairs
      for (int u = tg; u < HP * HP + KK * HP; u += C::NTG) {
        if (u < HP * HP) {
          const int bi = u / HP, bj = u % HP;
          const int pa = rr_player(bi, r, KK), pb = rr_player(KK - 1 - bi, r, KK);
          const int p = pa < pb ? pa : pb, q = pa < pb ? pb : pa;
          const int qa = rr_player(bj, r, KK), qb = rr_player(KK - 1 - bj, r, KK);
          const int p2 = qa < qb ? qa : qb, q2 = qa < qb ? qb : qa;
          const double c = ROT[bi], s = ROT[C::KK / 2 + bi];
          const double c2 = ROT[bj], s2 = ROT[C::KK / 2 + bj];
          const double a00 = JA[p * C::JLD + p2], a01 = JA[p * C::JLD + q2];
          const double a10 = JA[q * C::JLD + p2], a11 = JA[q * C::JLD + q2];
          // columns: (p2, q2) <- (c2 a_p2 - s2 a_q2, s2 a_p2 + c2 a_q2)
          const double m00 = c2 * a00 - s2 * a01, m01 = s2 * a00 + c2 * a01;
          const double m10 = c2 * a10 - s2 * a11, m11 = s2 * a10 + c2 * a11;
          // rows: (p, q) <- (c m_p - s m_q, s m_p + c m_q)
          double n00 = c * m00 - s * m10, n01 = c * m01 - s * m11;
          double n10 = s * m00 + c * m10, n11 = s * m01 + c * m11;
          if (bi == bj && s != 0.0) {
            n01 = 0.0;
            n10 = 0.0;
          }
          JA[p * C::JLD + p2] = n00;
          JA[p * C::JLD + q2] = n01;
          JA[q * C::JLD + p2] = n10;
          JA[q * C::JLD + q2] = n11;
        } else {
          const int v = u - HP * HP;
          const int x = v / HP, bj = v % HP;
          const int qa = rr_player(bj, r, KK), qb = rr_player(KK - 1 - bj, r, KK);
          const int p2 = qa < qb ? qa : qb, q2 = qa < qb ? qb : qa;
          const double c2 = ROT[bj], s2 = ROT[C::KK / 2 + bj];
          const double v0 = JV[x * C::JLD + p2], v1 = JV[x * C::JLD + q2];
          JV[x * C::JLD + p2] = c2 * v0 - s2 * v1;
          JV[x * C::JLD + q2] = s2 * v0 + c2 * v1;
        }
      }
      gsync<C::NW>();
    }
    const int any = misc[2];
    gsync<C::NW>();
    if (!any) break;
  }

  // ---- eigen order, numerical rank, Ut = U_p / sqrt(sigma) -------------------------------
  if (tg < KK) {
    const double dx = JA[tg * C::JLD + tg];
    int rk = 0;
    for (int y = 0; y < KK; ++y) {
      const double dy = JA[y * C::JLD + y];
      rk += (dy > dx) || (dy == dx && y < tg);
    }
    ord[rk] = tg;
  }
  gsync<C::NW>();
  const double sig0 = JA[ord[0] * C::JLD + ord[0]];
  const int plim = (int)((int64_t)(k - 1) < m ? (int64_t)(k - 1) : m);
  const double rtol = (double)(m > k ? m : k) * 0x1p-24;
  int pe = 0;
  if (sig0 > 0.0) {
    while (pe < plim && JA[ord[pe] * C::JLD + ord[pe]] > rtol * sig0) ++pe;
  }
  for (int e = tg; e < k * pe; e += C::NTG) {
    const int a = e / pe, l = e % pe;
    const int x = ord[l];
    UT[a * KMAX + l] = JV[a * C::JLD + x] / sqrt(JA[x * C::JLD + x]);
  }
  gsync<C::NW>();

  // ---- Gram-space terms -------------------------------------------------------------
  // part: 0 t_range, 1 g, 2 t_A, 3 t_S, 4 t_D  (each times k-1)
  double part[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const float* Qrow = mom + k * C::NPAD;
  // t_S = sum_l ||K ut_l||^2 ; t_D = sum_l ut_l^T Q ut_l
  for (int e = tg; e < k * pe; e += C::NTG) {
    const int a = e / pe, l = e % pe;
    double kv = 0.0, qv = 0.0;
    for (int b = 0; b < k; ++b) {
      const int pb = PIDX[a * KMAX + b];
      const double u = UT[b * KMAX + l];
      kv = fma((double)Krow[pb], u, kv);
      qv = fma((double)Qrow[pb], u, qv);
    }
    part[3] = fma(kv, kv, part[3]);
    part[4] = fma(UT[a * KMAX + l], qv, part[4]);
  }
  for (int j = 0; j < k; ++j) {
    const float* Tj = mom + j * C::NPAD;
    for (int e = tg; e < k * pe; e += C::NTG) {
      const int a = e / pe, l = e % pe;
      double yv = 0.0;
      for (int b = 0; b < k; ++b) yv = fma((double)Tj[PIDX[a * KMAX + b]], UT[b * KMAX + l], yv);
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
    group_sum<C::NW, 1>(tv, RED, tg);
    if (tg == 0) {
      const double bj = (double)mom[j * C::NPAD + np] - tv[0];   // (X_c d_P)_j
      part[2] = fma(bj, bj, part[2]);
    }
    gsync<C::NW>();
  }
  group_sum<C::NW, 5>(part, RED, tg);

  if (tg == 0) {
    uint8_t fl = 0;
    const double km1 = (double)(k - 1);
    const double tau = tauk / km1;
    double kap;
    if (!(sig0 > 0.0) || tauk == 0.0) {
      kap = 0.0;
      fl |= PF_DEGENERATE;
    } else {
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
      kap = fabs(0.5 * (t_range + t_null) + 0.5 * tau);
    }
    if (pe < plim) fl |= PF_RANK_DEFICIENT;
    if (sweep >= JAC_MAX_SWEEPS) fl |= PF_JACOBI_MAXSWEEPS;
    kappa_out[i] = (float)kap;
    if (flags_out) flags_out[i] = fl;
  }
}

template <int KMAX>
static hipError_t launch_fast_k(const float* X, int64_t n, int64_t m, int64_t ldx,
                                const int32_t* idx, int k, int variant, float* kappa,
                                uint8_t* flags, hipStream_t stream) {
  using C = FastCfg<KMAX>;
  static bool attr_set = false;   // LDS beyond 64 KiB needs the opt-in attribute
  if (!attr_set) {
    hipFuncSetAttribute(reinterpret_cast<const void*>(&curv_fast_kernel<KMAX>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)(C::PPW * C::BYTES));
    (void)hipGetLastError();
    attr_set = true;
  }
  const unsigned grid = (unsigned)((n + C::PPW - 1) / C::PPW);
  timing_begin(6, stream);
  hipLaunchKernelGGL(curv_fast_kernel<KMAX>, dim3(grid), dim3(C::NT), C::PPW * C::BYTES, stream, X,
                     n, m, ldx, idx, k, variant, kappa, flags);
  timing_end(6, stream);
  return hipGetLastError();
}

hipError_t launch_curv_fast(const float* X, int64_t n, int64_t m, int64_t ldx, const int32_t* idx,
                            int k, int precision, int variant, float* kappa, uint8_t* flags,
                            hipStream_t stream) {
  (void)precision;
  if (k <= 4) return launch_fast_k<4>(X, n, m, ldx, idx, k, variant, kappa, flags, stream);
  if (k <= 8) return launch_fast_k<8>(X, n, m, ldx, idx, k, variant, kappa, flags, stream);
  if (k <= 12) return launch_fast_k<12>(X, n, m, ldx, idx, k, variant, kappa, flags, stream);
  if (k <= 16) return launch_fast_k<16>(X, n, m, ldx, idx, k, variant, kappa, flags, stream);
  if (k <= 20) return launch_fast_k<20>(X, n, m, ldx, idx, k, variant, kappa, flags, stream);
  if (k <= 24) return launch_fast_k<24>(X, n, m, ldx, idx, k, variant, kappa, flags, stream);
  if (k <= 28) return launch_fast_k<28>(X, n, m, ldx, idx, k, variant, kappa, flags, stream);
  return launch_fast_k<32>(X, n, m, ldx, idx, k, variant, kappa, flags, stream);
}

}  // namespace mc
