// Shared front half of the per-point curvature kernels (gfx950): patch gather and
// centring, the moment GEMM on MFMA, the k x k Jacobi eigen-solve and the range
// basis Ut = U_p diag(sigma_p^{-1/2}).  Used by the Fast forward and its adjoint.
//
// Moments of the centred patch X_c (k x m), one MFMA GEMM over the m columns:
//   [X_c ; q ; 1] (k+2 x m)  times  [X_c[a] o X_c[b] (a<=b) | 1] (m x k(k+1)/2+1)
// gives, in `mom` (row-major, stride NPAD):
//   row j < k : T[j][pair(a,b)] = sum_c X_c[j,c] X_c[a,c] X_c[b,c],  T[j][np] = r_j = sum_c X_c[j,c]
//   row k     : Q[pair(a,b)]    = sum_c q_c X_c[a,c] X_c[b,c],  q_c = sum_j X_c[j,c]^2
//   row k+1   : K[pair(a,b)]    = sum_c X_c[a,c] X_c[b,c]
// tau * (k-1) = ||X_c||_F^2 is accumulated separately in float64.
#pragma once

#include <math.h>

#include <type_traits>

#include "mc_device.h"

namespace mc {

constexpr int FCH = 64;        // patch columns per staged chunk
constexpr int FLDX = FCH + 4;  // LDS row stride of a staged chunk: 16-byte rows for vector reads,
                               // rows 4 banks apart so 8 lanes of a 128-bit read never collide
constexpr int JAC_MAX_SWEEPS = 40;

// MOMSZ: bytes per stored moment and per staged patch value (4: float32, 8: float64).
template <int KMAX, int NW_, int PPW_, size_t EXTRA_B = 0, int MOMSZ = 4>
struct CurvCfg {
  static constexpr int KM = KMAX;
  static constexpr int MB = (KMAX + 2 + 15) / 16;           // 16-row blocks of the LHS
  static constexpr int ROWS = (16 * MB > KMAX + 3) ? 16 * MB : KMAX + 3;
  static constexpr int NPC = KMAX * (KMAX + 1) / 2 + 1;     // pair columns + ones column
  static constexpr int NB = (NPC + 15) / 16;                // 16-column blocks of the RHS
  static constexpr int NW = NW_;                            // waves per point
  static constexpr int PPW = PPW_;                          // points per workgroup
  static constexpr int NTG = NW * WAVE;                     // threads per point
  static constexpr int NT = PPW * NTG;                      // threads per workgroup
  static constexpr int NBW = (NB + NW - 1) / NW;            // RHS blocks per wave
  static constexpr int KK = (KMAX + 1) & ~1;                // even Jacobi size
  static constexpr int JLD = KK + 1;                        // Jacobi row stride (doubles)
  static constexpr int NPAD = NB * 16;
  // LDS layout of one point (bytes); the staged chunk and the moments share storage.
  static constexpr size_t LHS_B = (size_t)ROWS * FLDX * MOMSZ;
  static constexpr size_t MOM_B = (size_t)(KMAX + 2) * NPAD * MOMSZ;
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
  static constexpr size_t OFF_PAIR = (OFF_PJ + 2 * NPAD + 1) & ~(size_t)1;  // Jacobi pair table
  static constexpr size_t OFF_EXTRA = (OFF_PAIR + (size_t)(KK - 1) * (KK / 2) * 2 + 15) & ~(size_t)15;
  static constexpr size_t BYTES = (OFF_EXTRA + EXTRA_B + 15) & ~(size_t)15;
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

// Centre one column of the patch in float32: the mean is taken of the offsets from the
// first row, so equal rows give exactly zero and large coordinates cause no cancellation.
// On return xr[j] holds X_c[j, c].
template <int KMAX>
__device__ __forceinline__ void centre_column(float (&xr)[KMAX], int k) {
#pragma unroll
  for (int j = KMAX - 1; j >= 0; --j)
    if (j < k) xr[j] -= xr[0];
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < KMAX; ++j)
    if (j < k) s += xr[j];
  const float mean = s / (float)k;
#pragma unroll
  for (int j = 0; j < KMAX; ++j)
    if (j < k) xr[j] -= mean;
}

// Float64 centring of one column: offsets from the first row are exact in float64, so the
// centred values carry only the rounding of the mean.  xc[j] = X_c[j, c] (0 for j >= k).
template <int KMAX>
__device__ __forceinline__ void centre_column_f64(const float (&xr)[KMAX], double (&xc)[KMAX], int k) {
  const double x0 = (double)xr[0];
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    xc[j] = j < k ? (double)xr[j] - x0 : 0.0;
    s += xc[j];
  }
  const double mean = s / (double)k;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) xc[j] = j < k ? xc[j] - mean : 0.0;
}

// 1/sqrt(x) for normal x > 0: hardware estimate refined by two Newton steps (float64).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  y = y * fma(-0.5 * x * y, y, 1.5);
  return y;
}

// Player at round-robin position `pos` in round r of the circle schedule on KK players.
__device__ __forceinline__ int rr_player(int pos, int r, int KK) {
  if (pos == 0) return 0;
  int t = pos - 1 + r;
  if (t >= KK - 1) t -= KK - 1;
  return t + 1;
}

// Pointers into one point's LDS region.
struct PointLds {
  float* lhs;
  void* mom;          // float or double moments (row-major, stride NPAD)
  double* JA;
  double* JV;
  double* UT;
  double* YB;
  double* RED;
  double* ROT;
  int* nb;
  int* ord;
  int* misc;
  uint16_t* PIDX;
  unsigned char* pj1;
  unsigned char* pj2;
  uint16_t* pairs;    // round r, slot i: p | q << 8 (p < q) of the round-robin schedule
  unsigned char* extra;
};

template <class C>
__device__ __forceinline__ PointLds point_lds(unsigned char* smem) {
  PointLds P;
  P.lhs = reinterpret_cast<float*>(smem);
  P.mom = smem;
  P.JA = reinterpret_cast<double*>(smem + C::OFF_JA);
  P.JV = reinterpret_cast<double*>(smem + C::OFF_JV);
  P.UT = reinterpret_cast<double*>(smem + C::OFF_UT);
  P.YB = reinterpret_cast<double*>(smem + C::OFF_Y);
  P.RED = reinterpret_cast<double*>(smem + C::OFF_RED);
  P.ROT = reinterpret_cast<double*>(smem + C::OFF_ROT);
  int* IN = reinterpret_cast<int*>(smem + C::OFF_INT);
  P.nb = IN;
  P.ord = IN + C::KM;
  P.misc = P.ord + C::KK;
  P.PIDX = reinterpret_cast<uint16_t*>(smem + C::OFF_PIDX);
  P.pj1 = smem + C::OFF_PJ;
  P.pj2 = P.pj1 + C::NPAD;
  P.pairs = reinterpret_cast<uint16_t*>(smem + C::OFF_PAIR);
  P.extra = smem + C::OFF_EXTRA;
  return P;
}

__device__ __forceinline__ float rsqrt_nr(float x) {
  float y = __builtin_amdgcn_rsqf(x);
  return y * fmaf(-0.5f * x * y, y, 1.5f);
}

// Cyclic Jacobi sweeps in parallel (round-robin) order on the KK x KK matrix A (row stride
// C::JLD, working type JT), accumulating the rotations into V.  The matrix is padded to
// KK = KMAX (even) with zero rows and columns, which never rotate, so every loop bound is a
// compile-time constant.  Each round rotates KK/2 disjoint planes; the update works on 2 x 2
// blocks of A (pair i x pair i') and on row x of V restricted to one pair, so every thread
// reads and writes the same cells and the update runs in place.  A round whose planes are
// all below threshold (|a_pq| <= eps sqrt(|a_pp a_qq|), or the absolute floor) skips its
// update.  Returns the sweeps used (JAC_MAX_SWEEPS when the limit was hit).
template <class C, class JT>
__device__ int jacobi_sweeps(const PointLds& P, JT* JA, JT* JV, int k, int tg, JT eps) {
  int* misc = P.misc;
  constexpr int KK = C::KK;
  constexpr int HP = KK / 2;
  JT* ROT = reinterpret_cast<JT*>(P.ROT);
  JT trace = 0;
  for (int x = 0; x < k; ++x) trace += JA[x * C::JLD + x];
  const JT floor_abs = trace * (JT)0x1p-100;
  int sweep = 0;
  for (; sweep < JAC_MAX_SWEEPS; ++sweep) {
    int swept = 0;
    for (int r = 0; r < KK - 1; ++r) {
      const uint16_t* pr = P.pairs + r * HP;
      int rot = 0;
      if (tg < HP) {
        const int pq = pr[tg];
        const int p = pq & 0xff, q = pq >> 8;
        const JT app = JA[p * C::JLD + p], aqq = JA[q * C::JLD + q], apq = JA[p * C::JLD + q];
        JT c = 1, sn = 0;
        const JT thr = fmax(eps * sqrt(fabs(app) * fabs(aqq)), floor_abs);
        if (fabs(apq) > thr) {
          // t = tan(phi), the smaller root of t^2 + 2 t (aqq - app)/(2 apq) - 1 = 0
          const JT d = aqq - app, e2 = 2 * apq;
          const JT t0 = e2 / (fabs(d) + sqrt(fma(d, d, e2 * e2)));
          const JT t = d < 0 ? -t0 : t0;
          c = rsqrt_nr(fma(t, t, (JT)1));
          sn = t * c;
          rot = 1;
        }
        ROT[tg] = c;
        ROT[C::KK / 2 + tg] = sn;
      }
      rot = __any(rot);                   // the rotating lanes all sit in wave 0
      if constexpr (C::NW > 1) {
        if (tg == 0) misc[3 + (r & 1)] = rot;   // two slots: a skipped round has no second barrier
      }
      gsync<C::NW>();
      if constexpr (C::NW > 1) rot = misc[3 + (r & 1)];
      if (!rot) continue;                 // nothing rotates in this round
      swept = 1;
      // A <- J^T A J on 2 x 2 blocks.  When the thread count is a multiple of HP, a thread's
      // column block bj is the same for all its blocks: its plane and rotation are read once.
      constexpr bool FIXJ = C::NTG % HP == 0;
      int pqj = 0;
      JT cj = 0, sj = 0;
      if constexpr (FIXJ) {
        pqj = pr[tg % HP];
        cj = ROT[tg % HP];
        sj = ROT[C::KK / 2 + tg % HP];
      }
      for (int u = tg; u < HP * HP; u += C::NTG) {
        const int bi = u / HP, bj = u % HP;
        const int pq1 = pr[bi], pq2 = FIXJ ? pqj : pr[bj];
        const int p = pq1 & 0xff, q = pq1 >> 8, p2 = pq2 & 0xff, q2 = pq2 >> 8;
        const JT c = ROT[bi], sn = ROT[C::KK / 2 + bi];
        const JT c2 = FIXJ ? cj : ROT[bj], s2 = FIXJ ? sj : ROT[C::KK / 2 + bj];
        const JT a00 = JA[p * C::JLD + p2], a01 = JA[p * C::JLD + q2];
        const JT a10 = JA[q * C::JLD + p2], a11 = JA[q * C::JLD + q2];
        // columns: (p2, q2) <- (c2 a_p2 - s2 a_q2, s2 a_p2 + c2 a_q2)
        const JT m00 = c2 * a00 - s2 * a01, m01 = s2 * a00 + c2 * a01;
        const JT m10 = c2 * a10 - s2 * a11, m11 = s2 * a10 + c2 * a11;
        // rows: (p, q) <- (c m_p - s m_q, s m_p + c m_q)
        JT n00 = c * m00 - sn * m10, n01 = c * m01 - sn * m11;
        JT n10 = sn * m00 + c * m10, n11 = sn * m01 + c * m11;
        if (bi == bj && sn != 0) {
          n01 = 0;
          n10 = 0;
        }
        JA[p * C::JLD + p2] = n00;
        JA[p * C::JLD + q2] = n01;
        JA[q * C::JLD + p2] = n10;
        JA[q * C::JLD + q2] = n11;
      }
      // V <- V J on the rows of the real matrix (padded rows stay unit vectors)
      for (int u = tg; u < KK * HP; u += C::NTG) {
        const int x = u / HP, bj = u % HP;
        if (x < k) {
          const int pq2 = FIXJ ? pqj : pr[bj];
          const int p2 = pq2 & 0xff, q2 = pq2 >> 8;
          const JT c2 = FIXJ ? cj : ROT[bj], s2 = FIXJ ? sj : ROT[C::KK / 2 + bj];
          const JT v0 = JV[x * C::JLD + p2], v1 = JV[x * C::JLD + q2];
          JV[x * C::JLD + p2] = c2 * v0 - s2 * v1;
          JV[x * C::JLD + q2] = s2 * v0 + c2 * v1;
        }
      }
      gsync<C::NW>();
    }
    if (!swept) break;
  }
  return sweep;
}

// k x k eigen-solve of the Gram matrix K.  On entry JA holds K (float64, k x k, zero-padded
// to KK) and JV the identity.
//  * F32 = false: float64 Jacobi sweeps to a relative 2^-52.
//  * F32 = true (float32 and bf16 moments): float32 sweeps to 2^-23 on a float32 copy held
//    in the JV storage.  Jacobi is accurate relative to its data, and the moments' own
//    rounding (2^-24 sigma_1 and more for float32, 2^-9 sigma_1 for bf16) dominates the
//    solve's.  A kept spectrum with a near-degenerate pair (sigma_x, sigma_y within a
//    relative 2^-13 of each other) is re-solved in float64 from the untouched JA; misc[5]
//    records that.
// On return: eigen order in P.ord, sig0 = sigma_1, pe = numerical rank (eigenvalues above
// max(k, m) * unit * sigma_1 among the first min(k-1, m)), sweep = sweeps used, and
// P.UT = U_p diag(sigma_p^(-1/2)).
template <int KMAX, class C, bool F32 = false>
__device__ void jacobi_eigen(const PointLds& P, int k, int64_t m, int tg, double unit, double& sig0,
                             int& pe, int& sweep) {
  double* JA = P.JA;
  double* JV = P.JV;
  int* misc = P.misc;
  constexpr int KK = C::KK;
  constexpr int HP = KK / 2;
  for (int e = tg; e < (KK - 1) * HP; e += C::NTG) {
    const int r = e / HP, i = e % HP;
    const int pa = rr_player(i, r, KK), pb = rr_player(KK - 1 - i, r, KK);
    P.pairs[e] = (uint16_t)((pa < pb ? pa : pb) | ((pa < pb ? pb : pa) << 8));
  }
  if constexpr (F32) {
    float* A32 = reinterpret_cast<float*>(JV);   // the two float32 matrices fill JV's storage
    float* V32 = A32 + KK * C::JLD;
    for (int e = tg; e < KK * KK; e += C::NTG) {
      const int x = e / KK, y = e % KK;
      A32[x * C::JLD + y] = (float)JA[x * C::JLD + y];
      V32[x * C::JLD + y] = x == y ? 1.0f : 0.0f;
    }
    gsync<C::NW>();
    sweep = jacobi_sweeps<C, float>(P, A32, V32, k, tg, 0x1p-23f);
    // near-degenerate pair among the kept eigenvalues (wave 0 holds the KK diagonal lanes)
    if (tg < WAVE) {
      bool near = false;
      if (tg < k) {
        float s1 = 0.0f;
        for (int y = 0; y < k; ++y) s1 = fmaxf(s1, A32[y * C::JLD + y]);
        const float keep = (float)((double)(m > k ? m : k) * unit) * s1;
        const float lx = A32[tg * C::JLD + tg];
        if (lx > keep) {
          for (int y = 0; y < k; ++y) {
            const float ly = A32[y * C::JLD + y];
            near |= y != tg && ly > keep && fabsf(lx - ly) < 0x1p-13f * fmaxf(lx, ly);
          }
        }
      }
      const int anyv = __any(near);
      if (tg == 0) misc[5] = anyv;
    }
    gsync<C::NW>();
    if (misc[5]) {
      for (int e = tg; e < KK * KK; e += C::NTG) {
        const int x = e / KK, y = e % KK;
        JV[x * C::JLD + y] = (x == y) ? 1.0 : 0.0;
      }
      gsync<C::NW>();
      sweep = jacobi_sweeps<C, double>(P, JA, JV, k, tg, 0x1p-52);
    } else {
      // float32 results into the float64 arrays (JA's diagonal, JV), read all before writing
      constexpr int NPT = (KK * KK + C::NTG - 1) / C::NTG;
      float vv[NPT];
#pragma unroll
      for (int t = 0; t < NPT; ++t) {
        const int e = tg + t * C::NTG;
        vv[t] = e < KK * KK ? V32[(e / KK) * C::JLD + e % KK] : 0.0f;
      }
      const float dg = tg < KK ? A32[tg * C::JLD + tg] : 0.0f;
      gsync<C::NW>();
#pragma unroll
      for (int t = 0; t < NPT; ++t) {
        const int e = tg + t * C::NTG;
        if (e < KK * KK) JV[(e / KK) * C::JLD + e % KK] = (double)vv[t];
      }
      if (tg < KK) JA[tg * C::JLD + tg] = (double)dg;
      gsync<C::NW>();
    }
  } else {
    gsync<C::NW>();
    sweep = jacobi_sweeps<C, double>(P, JA, JV, k, tg, 0x1p-52);
  }

  // ---- eigen order, numerical rank, Ut = U_p / sqrt(sigma) -------------------------------
  if (tg < KK) {
    const double dx = JA[tg * C::JLD + tg];
    int rk = 0;
    for (int y = 0; y < KK; ++y) {
      const double dy = JA[y * C::JLD + y];
      rk += (dy > dx) || (dy == dx && y < tg);
    }
    P.ord[rk] = tg;
  }
  gsync<C::NW>();
  sig0 = JA[P.ord[0] * C::JLD + P.ord[0]];
  const int plim = (int)((int64_t)(k - 1) < m ? (int64_t)(k - 1) : m);
  // relative floor of the Gram eigenvalues: the rounding level of the accumulated moments
  const double rtol = (double)(m > k ? m : k) * unit;
  pe = 0;
  if (sig0 > 0.0) {
    while (pe < plim && JA[P.ord[pe] * C::JLD + P.ord[pe]] > rtol * sig0) ++pe;
  }
  for (int e = tg; e < KMAX * KMAX; e += C::NTG) {
    const int a = e / KMAX, l = e % KMAX;
    if (a < k && l < pe) {
      const int x = P.ord[l];
      P.UT[a * KMAX + l] = JV[a * C::JLD + x] / sqrt(JA[x * C::JLD + x]);
    }
  }
  gsync<C::NW>();
}

// Moment precision of patch_front: float32 MFMA, bf16 MFMA (float32 Gram), float64 MFMA.
constexpr int MOM_FP32 = 0;
constexpr int MOM_BF16 = 1;
constexpr int MOM_FP64 = 2;

template <int PREC>
using MomT = typename std::conditional<PREC == MOM_FP64, double, float>::type;

// Front half for point i: setup, moments, Jacobi, eigen order, numerical rank and Ut.
// Returns 0 on success, or PF_NONFINITE (bad index or non-finite patch value).
// Outputs (valid in every thread of the group): tauk = ||X_c||^2, sig0 = sigma_1,
// pe = numerical rank, sweep = Jacobi sweeps used.  With MOM_FP64 the patch is centred,
// staged and multiplied in float64 (centre_column_f64).
template <int KMAX, class C, int PREC = MOM_FP32>
__device__ uint8_t patch_front(const PointLds& P, const float* __restrict__ X, int64_t n, int64_t m,
                               int64_t ldx, const int32_t* __restrict__ idx, int k, int64_t i,
                               int tg, double& tauk, double& sig0, int& pe, int& sweep) {
  static_assert(PREC != MOM_FP64 || sizeof(MomT<PREC>) * C::NPAD * (KMAX + 2) <= C::U0_B,
                "float64 moments need a CurvCfg with MOMSZ = 8");
  const int w = tg / WAVE;
  const int lane = tg % WAVE;
  MomT<PREC>* lhs = reinterpret_cast<MomT<PREC>*>(P.lhs);   // staged chunk: float64 with MOM_FP64
  MomT<PREC>* mom = reinterpret_cast<MomT<PREC>*>(P.mom);
  double* JA = P.JA;
  double* JV = P.JV;
  int* misc = P.misc;
  int* nb = P.nb;
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
    P.pj1[t] = (unsigned char)a;
    P.pj2[t] = (unsigned char)b;
  }
  for (int t = tg; t < k * k; t += C::NTG)
    P.PIDX[(t / k) * KMAX + t % k] = (uint16_t)pair_index(t / k, t % k, k);
  for (int t = tg; t < (C::ROWS - (k + 2)) * FLDX; t += C::NTG) lhs[(k + 2) * FLDX + t] = 0;
  gsync<C::NW>();
  if (misc[0]) return PF_NONFINITE;

  // ---- pass over the patch: moments on MFMA --------------------------------------
  using AccT = typename std::conditional<PREC == MOM_FP64, doublex4, floatx4>::type;
  AccT acc[C::MB][C::NBW];
#pragma unroll
  for (int a = 0; a < C::MB; ++a)
#pragma unroll
    for (int b = 0; b < C::NBW; ++b) acc[a][b] = AccT{0, 0, 0, 0};

  int off1[C::NBW], off2[C::NBW];
#pragma unroll
  for (int b = 0; b < C::NBW; ++b) {
    const int nbg = w + C::NW * b;
    const int pi = nbg * 16 + (lane % 16);
    const int pc = pi < C::NPAD ? pi : C::NPAD - 1;
    off1[b] = P.pj1[pc] * FLDX;
    off2[b] = P.pj2[pc] * FLDX;
  }

  // bf16 path: K = X_c X_c^T stays float32 (it feeds the eigen-solve and the rank test);
  // KB x KB blocks of 16 x 16 on v_mfma_f32_16x16x4f32, fed by the same staged values.
  constexpr int KB = (KMAX + 15) / 16;
  floatx4 kacc[KB][KB];
#pragma unroll
  for (int a = 0; a < KB; ++a)
#pragma unroll
    for (int b = 0; b < KB; ++b) kacc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

  float xr[KMAX];
  double tau64 = 0.0;
  bool nonfinite = false;
  if (w == 0) load_chunk<KMAX>(xr, X, ldx, nb, k, m, 0, lane);

  for (int64_t c0 = 0; c0 < m; c0 += FCH) {
    if (w == 0) {
#pragma unroll
      for (int j = 0; j < KMAX; ++j)
        if (j < k) nonfinite |= !isfinite(xr[j]);
      if constexpr (PREC == MOM_FP64) {
        double xc[KMAX];
        centre_column_f64<KMAX>(xr, xc, k);
        double q = 0.0;
#pragma unroll
        for (int j = 0; j < KMAX; ++j) {
          if (j < k) {
            q = fma(xc[j], xc[j], q);
            lhs[j * FLDX + lane] = xc[j];
          }
        }
        tau64 += q;
        lhs[k * FLDX + lane] = q;
      } else {
        centre_column<KMAX>(xr, k);
        float q = 0.0f;
#pragma unroll
        for (int j = 0; j < KMAX; ++j) {
          if (j < k) {
            const float xc = xr[j];
            q = fmaf(xc, xc, q);
            tau64 = fma((double)xc, (double)xc, tau64);
            lhs[j * FLDX + lane] = xc;
          }
        }
        lhs[k * FLDX + lane] = q;
      }
      lhs[(k + 1) * FLDX + lane] = (c0 + lane < m) ? 1 : 0;
    }
    gsync<C::NW>();
    if (w == 0 && c0 + FCH < m) load_chunk<KMAX>(xr, X, ldx, nb, k, m, c0 + FCH, lane);

    const int64_t rem = m - c0;
    if constexpr (PREC == MOM_FP64) {
      const int steps = rem >= FCH ? FCH / 4 : (int)((rem + 3) / 4);
      for (int s = 0; s < steps; ++s) {
        const int col = 4 * s + lane / 16;
        double av[C::MB];
#pragma unroll
        for (int a = 0; a < C::MB; ++a) av[a] = lhs[(16 * a + lane % 16) * FLDX + col];
#pragma unroll
        for (int b = 0; b < C::NBW; ++b) {
          if (w + C::NW * b < nbr) {
            const double bv = lhs[off1[b] + col] * lhs[off2[b] + col];
#pragma unroll
            for (int a = 0; a < C::MB; ++a) acc[a][b] = mfma16x16x4f64(av[a], bv, acc[a][b]);
          }
        }
      }
    } else if constexpr (PREC == MOM_FP32) {
      // 16-column groups; lane l supplies column 4 (l / 16) + s of the group at step s, so
      // each operand row is one 128-bit read per group (A and B use the same column order)
      const int ngrp = rem >= FCH ? FCH / 16 : (int)((rem + 15) / 16);
      for (int g = 0; g < ngrp; ++g) {
        const int col = 16 * g + 4 * (lane / 16);
        floatx4 av[C::MB];
#pragma unroll
        for (int a = 0; a < C::MB; ++a)
          av[a] = *reinterpret_cast<const floatx4*>(lhs + (16 * a + lane % 16) * FLDX + col);
#pragma unroll
        for (int b = 0; b < C::NBW; ++b) {
          if (w + C::NW * b < nbr) {
            const floatx4 x1 = *reinterpret_cast<const floatx4*>(lhs + off1[b] + col);
            const floatx4 x2 = *reinterpret_cast<const floatx4*>(lhs + off2[b] + col);
            const floatx4 bv = x1 * x2;
#pragma unroll
            for (int st = 0; st < 4; ++st)
#pragma unroll
              for (int a = 0; a < C::MB; ++a) acc[a][b] = mfma16x16x4(av[a][st], bv[st], acc[a][b]);
          }
        }
      }
    } else {
      // 32-column steps; lane l supplies columns 32 s + 8 (l / 16) + e, e = 0..7
      const int steps = rem >= FCH ? FCH / 32 : (int)((rem + 31) / 32);
      for (int s = 0; s < steps; ++s) {
        const int col0 = 32 * s + 8 * (lane / 16);
        float xa[C::MB][8];
        shortx8 abf[C::MB];
#pragma unroll
        for (int a = 0; a < C::MB; ++a)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            xa[a][e] = lhs[(16 * a + lane % 16) * FLDX + col0 + e];
            abf[a][e] = (short)f2bf(xa[a][e]);
          }
        if (w == 0) {
#pragma unroll
          for (int e = 0; e < 8; ++e)
#pragma unroll
            for (int a = 0; a < KB; ++a)
#pragma unroll
              for (int b = 0; b < KB; ++b) kacc[a][b] = mfma16x16x4(xa[a][e], xa[b][e], kacc[a][b]);
        }
#pragma unroll
        for (int b = 0; b < C::NBW; ++b) {
          if (w + C::NW * b < nbr) {
            shortx8 bbf;
#pragma unroll
            for (int e = 0; e < 8; ++e) bbf[e] = (short)f2bf(lhs[off1[b] + col0 + e] * lhs[off2[b] + col0 + e]);
#pragma unroll
            for (int a = 0; a < C::MB; ++a) acc[a][b] = mfma16x16x32bf16(abf[a], bbf, acc[a][b]);
          }
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
      P.RED[15 * C::NW] = tau64;
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
          const int row = 16 * a + (PREC == MOM_FP64 ? lane / 16 + 4 * r : 4 * (lane / 16) + r);
          if (row < (PREC == MOM_BF16 ? k + 1 : k + 2) && col < npc) mom[row * C::NPAD + col] = acc[a][b][r];
        }
    }
  }
  if constexpr (PREC == MOM_BF16) {
    if (w == 0) {
#pragma unroll
      for (int a = 0; a < KB; ++a)
#pragma unroll
        for (int b = 0; b < KB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int x = 16 * a + 4 * (lane / 16) + r, y = 16 * b + lane % 16;
            if (x <= y && y < k) mom[(k + 1) * C::NPAD + P.PIDX[x * KMAX + y]] = kacc[a][b][r];
          }
    }
  }
  gsync<C::NW>();
  tauk = P.RED[15 * C::NW];
  if (misc[1]) return PF_NONFINITE;

  // ---- k x k eigen-solve (Jacobi: float32 sweeps unless the moments are float64) on K --
  {
    constexpr int KK = C::KK;
    const MomT<PREC>* Krow = mom + (k + 1) * C::NPAD;
    for (int e = tg; e < KK * KK; e += C::NTG) {
      const int x = e / KK, y = e % KK;
      JA[x * C::JLD + y] = (x < k && y < k) ? (double)Krow[P.PIDX[x * KMAX + y]] : 0.0;
      JV[x * C::JLD + y] = (x == y) ? 1.0 : 0.0;
    }
  }
  jacobi_eigen<KMAX, C, PREC != MOM_FP64>(P, k, m, tg, PREC == MOM_FP64 ? 0x1p-44 : 0x1p-24, sig0, pe, sweep);
  gsync<C::NW>();
  return 0;
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

}  // namespace mc
