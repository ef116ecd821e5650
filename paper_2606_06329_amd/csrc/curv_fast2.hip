// Two-pass Fast-mode mean curvature for k >= 13 (gfx950), split into four kernels that
// hand per-point k x k state to each other through the caller's workspace.
//
// What is computed is the Fast branch of Algorithm 1 (eqs. svd_cov, tA, tB, tnull,
// fast_curv), evaluated as in curv_fast.hip's two-pass form:
//   1. curv_gram:  K = X_c X_c^T on MFMA from one pass over the centred patch (split
//                  bf16 products on the bf16 path), and tau (k-1) = ||X_c||_F^2 in float64.
//   2. curv_eigen: the k x k eigen-solve of K (parallel-order Jacobi) gives
//                  Ut = U_p diag(sigma_p^{-1/2}), the numerical rank and
//                  (k-1) t_S = sum_l ||K ut_l||^2.  Float32 sweeps on the float32/bf16
//                  paths; a point whose kept spectrum has a near-degenerate pair is marked
//                  and re-solved in float64 by a second launch of the same kernel.
//   3. curv_range: a second pass over the patch forms each 64-column chunk of
//                  V_r^T = Ut^T X_c on MFMA and one GEMM
//                  X_c (k x chunk) x [V[:,l1] o V[:,l2] (l1 <= l2) | h | 1]
//                  whose columns give G_tens, tr G_j = (X_c h)_j and r_j = (X_c 1)_j;
//                  t_D = sum_c q_c h_c with q_c = sum_j X_c[j,c]^2; then the float64
//                  combination.  On the bf16 path that GEMM runs on binary16 operands: the
//                  patch rows scaled by powers of two from K's diagonal, and packed
//                  binary16 products of the range rows.
// Each stage runs at its own occupancy: the eigen-solve, a chain of dependent rounds, runs
// one wave per point with only its two k x k matrices in LDS, so many points hide each
// other's latency; the patch passes spread the staging of a chunk over all waves of a point.
#include "curv_core.h"
#include "mc_internal.h"

namespace mc {

// rank slot value marking a point whose float32 eigen-solve found a near-degenerate kept pair
constexpr int PE_NEED_FP64 = -1;

// Workspace layout: structure of arrays over the n points.  KMAX is the kernel's k bucket.
struct Fast2Ws {
  int kmax;
  size_t esz_k, esz_u;      // bytes per stored K entry and per Ut entry
  size_t off_k, off_ut, off_tau, off_ts, off_pe, off_fl, total;
};

static int fast2_kmax(int k) { return k <= 16 ? 16 : (k <= 20 ? 20 : (k <= 24 ? 24 : (k <= 28 ? 28 : 32))); }

Fast2Ws fast2_ws(int64_t n, int k, int precision) {
  Fast2Ws L{};
  L.kmax = fast2_kmax(k);
  const size_t kk = (size_t)L.kmax * L.kmax;
  const bool f64 = precision == 3;
  L.esz_k = f64 ? 8 : 4;
  L.esz_u = f64 ? 8 : 4;
  size_t off = 0;
  L.off_k = off;   off += align256((size_t)n * kk * L.esz_k);
  L.off_ut = off;  off += align256((size_t)n * kk * L.esz_u);
  L.off_tau = off; off += align256((size_t)n * 8);
  L.off_ts = off;  off += align256((size_t)n * 8);
  L.off_pe = off;  off += align256((size_t)n * 4);
  L.off_fl = off;  off += align256((size_t)n);
  L.total = off;
  return L;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane exchanges across 16-lane rows without the LDS crossbar (gfx950 permlane swaps):
// permlane16_swap(v, v) yields, in every lane, the values of its row pair in row order, and
// permlane32_swap(v, v) those of its half pair; their sum is the xor-16 (xor-32) butterfly sum,
// the same in both lanes of a pair (the two addends in a fixed order).
__device__ __forceinline__ float xsum16(float x) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float xsum32(float x) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// sum over the lanes l' with l' % CPW == l % CPW (CPW = 64 / number of lane groups)
template <int CPW>
__device__ __forceinline__ float group_sum_f(float x) {
#pragma unroll
  for (int o = CPW; o < 16 && o < WAVE; o <<= 1) x += __shfl_xor(x, o, WAVE);
  if constexpr (CPW <= 16) x = xsum16(x);
  if constexpr (CPW <= 32) x = xsum32(x);
  return x;
}
// the value of lane l % CPW in every lane (row 0's copy of each column)
template <int CPW>
__device__ __forceinline__ float group_bcast_f(float x) {
  if constexpr (CPW == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    const auto t = __builtin_amdgcn_permlane32_swap(r[0], r[0], false, false);
    return __uint_as_float(t[0]);
  } else if constexpr (CPW == 32) {
    const auto t = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(t[0]);
  } else if constexpr (CPW == WAVE) {
    return x;
  } else {
    return __shfl(x, lane_id() % CPW, WAVE);
  }
}

// ---- 1. Gram pass: one wave per point, four points per workgroup ------------------------
template <int KMAX, int PREC>
struct GramCfg {
  static constexpr int KB = (KMAX + 15) / 16;
  static constexpr int ROWS = 16 * KB;
  static constexpr int NUB = KB * (KB + 1) / 2;       // upper-triangular 16 x 16 blocks of K
  static constexpr int PPW = PREC == MOM_FP64 ? 2 : 4;
  static constexpr int ESZ = PREC == MOM_FP64 ? 8 : 4;
  // bf16 moments stage the centred chunk as bf16 high and low parts, x ~ hi + lo, in two
  // arrays of ROWS x FLDG (16-byte rows, the row stride of the range pass's 16-bit copy)
  static constexpr bool SPLIT = PREC == MOM_BF16;
  static constexpr int FLDG = FCH + 8;
  static constexpr size_t BYTES = SPLIT ? (size_t)2 * ROWS * FLDG * 2
                                        : ((size_t)ROWS * FLDX * ESZ + 15) & ~(size_t)15;
};

template <int KMAX, int PREC>
__global__ __launch_bounds__(256) void curv_gram_kernel(const float* __restrict__ X, int64_t n, int64_t m,
                                                        int64_t ldx, const int32_t* __restrict__ idx, int k,
                                                        unsigned char* __restrict__ ws, Fast2Ws L) {
  using C = GramCfg<KMAX, PREC>;
  using ST = typename std::conditional<PREC == MOM_FP64, double, float>::type;
  using AccT = typename std::conditional<PREC == MOM_FP64, doublex4, floatx4>::type;
  constexpr int KB = C::KB;
  extern __shared__ __align__(16) unsigned char smem_all[];
  const int gid = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int64_t i = (int64_t)blockIdx.x * C::PPW + gid;
  if (i >= n) return;                                // whole wave exits together
  ST* XS = reinterpret_cast<ST*>(smem_all + (size_t)gid * C::BYTES);
  double* TAU = reinterpret_cast<double*>(ws + L.off_tau);
  uint8_t* FL = ws + L.off_fl;
  MomT<PREC>* Kout = reinterpret_cast<MomT<PREC>*>(ws + L.off_k) + (size_t)i * KMAX * KMAX;

  const int nbv = lane < k ? idx[i * k + lane] : 0;
  if (__any(lane < k && (nbv < 0 || (int64_t)nbv >= n))) {
    if (lane == 0) {
      FL[i] = PF_NONFINITE;
      TAU[i] = 0.0;
    }
    return;
  }
  uint16_t* XH = reinterpret_cast<uint16_t*>(smem_all + (size_t)gid * C::BYTES);   // split staging
  uint16_t* XL = XH + C::ROWS * C::FLDG;
  if constexpr (C::SPLIT) {
    for (int t = lane; t < (C::ROWS - k) * C::FLDG; t += WAVE) {
      XH[k * C::FLDG + t] = 0;
      XL[k * C::FLDG + t] = 0;
    }
  } else {
    for (int t = lane; t < (C::ROWS - k) * FLDX; t += WAVE) XS[k * FLDX + t] = (ST)0;
  }

  AccT acc[C::NUB];
#pragma unroll
  for (int b = 0; b < C::NUB; ++b) acc[b] = AccT{0, 0, 0, 0};
  double tau64 = 0.0;
  bool nonfinite = false;
  // the MFMA pass over one staged chunk (K's upper-triangular 16 x 16 blocks)
  auto products = [&](int64_t c0) {
    if constexpr (C::SPLIT) {
      // K = sum over 32-column steps of hi hi^T + hi lo^T + lo hi^T on bf16 MFMA (products
      // exact, float32 sums), plus lo lo^T on the diagonal blocks.  With x = hi + lo + r,
      // |lo| <= 2^-8 |x| and |r| <= 2^-16 |x|, a product drops lo_i lo_j and the r terms, at
      // most 3 * 2^-16 |x_i x_j|; on the diagonal blocks only the r terms, whose sign follows
      // the second rounding, so the trace carries no one-sided error
      const int ns = m - c0 >= FCH ? FCH / 32 : (int)((m - c0 + 31) / 32);
      for (int st = 0; st < ns; ++st) {
        const int col = 32 * st + 8 * (lane / 16);   // lane supplies columns col .. col + 7
        shortx8 ah[KB], al[KB];
#pragma unroll
        for (int ab = 0; ab < KB; ++ab) {
          ah[ab] = *reinterpret_cast<const shortx8*>(XH + (16 * ab + lane % 16) * C::FLDG + col);
          al[ab] = *reinterpret_cast<const shortx8*>(XL + (16 * ab + lane % 16) * C::FLDG + col);
        }
        int b = 0;
#pragma unroll
        for (int ab = 0; ab < KB; ++ab)
#pragma unroll
          for (int bb = ab; bb < KB; ++bb, ++b) {
            if (ab == bb) acc[b] = mfma16x16x32bf16(al[ab], al[bb], acc[b]);
            acc[b] = mfma16x16x32bf16(ah[ab], al[bb], acc[b]);
            acc[b] = mfma16x16x32bf16(al[ab], ah[bb], acc[b]);
            acc[b] = mfma16x16x32bf16(ah[ab], ah[bb], acc[b]);
          }
      }
      return;
    }
    const int ng = m - c0 >= FCH ? FCH / 16 : (int)((m - c0 + 15) / 16);
    for (int g = 0; g < ng; ++g) {
      const int col = 16 * g + 4 * (lane / 16);      // lane supplies columns col .. col+3
      int b = 0;
#pragma unroll
      for (int ab = 0; ab < KB; ++ab)
#pragma unroll
        for (int bb = ab; bb < KB; ++bb, ++b) {
          const ST* pa = XS + (16 * ab + lane % 16) * FLDX + col;
          const ST* pb = XS + (16 * bb + lane % 16) * FLDX + col;
#pragma unroll
          for (int st = 0; st < 4; ++st) {
            if constexpr (PREC == MOM_FP64) acc[b] = mfma16x16x4f64(pa[st], pb[st], acc[b]);
            else acc[b] = mfma16x16x4(pa[st], pb[st], acc[b]);
          }
        }
    }
  };
  if constexpr (PREC == MOM_FP64) {
    float xr[KMAX];
    auto load = [&](int64_t c0) {
      const int64_t c = c0 + lane;
#pragma unroll
      for (int j = 0; j < KMAX; ++j) {
        float v = 0.0f;
        if (j < k && c < m) v = X[(int64_t)__builtin_amdgcn_readlane(nbv, j) * ldx + c];
        xr[j] = v;
      }
    };
    load(0);
    for (int64_t c0 = 0; c0 < m; c0 += FCH) {
#pragma unroll
      for (int j = 0; j < KMAX; ++j)
        if (j < k) nonfinite |= !isfinite(xr[j]);
      double xc[KMAX];
      centre_column_f64<KMAX>(xr, xc, k);
#pragma unroll
      for (int j = 0; j < KMAX; ++j)
        if (j < k) {
          tau64 = fma(xc[j], xc[j], tau64);
          XS[j * FLDX + lane] = xc[j];
        }
      wave_sync();
      if (c0 + FCH < m) load(c0 + FCH);
      products(c0);
      wave_sync();
    }
  } else {
    // Lane (g, c4) = (lane / 16, lane % 16) gathers columns 4 c4 .. 4 c4 + 3 of the rows
    // j = 4 t + g, one 16-byte load per row (four rows per instruction), from row pointers it
    // keeps for the whole pass.  The column's offsets from its first row and their mean are
    // reduced over the four lane groups.  tau's float64 sum turns non-finite when a gathered
    // value is (a NaN, or an infinity minus an infinity, reaches the centred entries of its
    // column) or a centred value overflows, so one test at the end replaces a test per value.
    constexpr int RT = KMAX / 4;
    static_assert(KMAX % 4 == 0, "row groups of four");
    const int g = lane / 16, c4 = lane % 16;
    const bool vec = (ldx % 4 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
    const float* rp[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int j = 4 * t + g;
      const int r = __shfl(nbv, j < k ? j : 0, WAVE);
      rp[t] = X + (int64_t)r * ldx;
    }
    // Two instances of the pass: FULL when k fills the bucket (no row tests), and the
    // general one.  A chunk that lies inside the rows (and 16-byte rows) is gathered with
    // unconditional vector loads; rows j >= k read row 0 and are never used (the centring,
    // tau and the staging skip them), so nothing waits for the loads before the products.
    floatx4 xv[RT];
    auto load = [&](int64_t c0, auto full_tag) {
      constexpr bool FULL = decltype(full_tag)::value;
      const int64_t c = c0 + 4 * c4;
      if (vec && c0 + FCH <= m) {
#pragma unroll
        for (int t = 0; t < RT; ++t) xv[t] = *reinterpret_cast<const floatx4*>(rp[t] + c);
        return;
      }
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        floatx4 v = {0.f, 0.f, 0.f, 0.f};
        if (FULL || 4 * t + g < k) {
          if (vec && c + 3 < m) {
            v = *reinterpret_cast<const floatx4*>(rp[t] + c);
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (c + e < m) v[e] = rp[t][c + e];
          }
        }
        xv[t] = v;
      }
    };
    auto pass = [&](auto full_tag) {
    constexpr bool FULL = decltype(full_tag)::value;
    load(0, full_tag);
    for (int64_t c0 = 0; c0 < m; c0 += FCH) {
      floatx4 x0, sm = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int e = 0; e < 4; ++e) x0[e] = __shfl(xv[0][e], c4, WAVE);   // row 0 sits in group 0
#pragma unroll
      for (int t = 0; t < RT; ++t)
        if (FULL || 4 * t + g < k) {
          xv[t] -= x0;
          sm += xv[t];
        }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        sm[e] += __shfl_xor(sm[e], 16, WAVE);
        sm[e] += __shfl_xor(sm[e], 32, WAVE);
      }
      const floatx4 mean = sm / (float)k;
#pragma unroll
      for (int t = 0; t < RT; ++t)
        if (FULL || 4 * t + g < k) {
          const floatx4 xc = xv[t] - mean;
#pragma unroll
          for (int e = 0; e < 4; ++e) tau64 = fma((double)xc[e], (double)xc[e], tau64);
          if constexpr (C::SPLIT) {
            uint16_t hi[4], lo[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              hi[e] = f2bf(xc[e]);
              lo[e] = f2bf(xc[e] - bf2f(hi[e]));
            }
            const int o = (4 * t + g) * C::FLDG + 4 * c4;
            *reinterpret_cast<uint2*>(XH + o) = make_uint2(hi[0] | ((uint32_t)hi[1] << 16), hi[2] | ((uint32_t)hi[3] << 16));
            *reinterpret_cast<uint2*>(XL + o) = make_uint2(lo[0] | ((uint32_t)lo[1] << 16), lo[2] | ((uint32_t)lo[3] << 16));
          } else {
            *reinterpret_cast<floatx4*>(XS + (4 * t + g) * FLDX + 4 * c4) = xc;
          }
        }
      wave_sync();
      if (c0 + FCH < m) load(c0 + FCH, full_tag);
      products(c0);
      wave_sync();
    }
    };
    if (k == KMAX) pass(std::true_type{});
    else pass(std::false_type{});
  }
  // K (both triangles) to the workspace, each entry from the upper triangle: the split
  // products sum a diagonal block's (x, y) and (y, x) terms in different orders, and the
  // eigen-solve expects K exactly symmetric
  int b = 0;
#pragma unroll
  for (int ab = 0; ab < KB; ++ab)
#pragma unroll
    for (int bb = ab; bb < KB; ++bb, ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x = 16 * ab + (PREC == MOM_FP64 ? lane / 16 + 4 * r : 4 * (lane / 16) + r);
        const int y = 16 * bb + lane % 16;
        if (x < k && y < k && x <= y) {
          Kout[x * KMAX + y] = (MomT<PREC>)acc[b][r];
          Kout[y * KMAX + x] = (MomT<PREC>)acc[b][r];
        }
      }
  tau64 = wave_sum(tau64);
  const int nf = __any(nonfinite) || !isfinite(tau64);
  if (lane == 0) {
    TAU[i] = tau64;
    FL[i] = nf ? PF_NONFINITE : 0;
  }
}

// ---- 2. eigen-solve: one wave per point -------------------------------------------------
template <int KMAX, class JT>
struct EigCfg {
  static constexpr int KM = KMAX;
  static constexpr int KK = (KMAX + 1) & ~1;
  static constexpr int JLD = KK + 1;
  static constexpr int NW = 1, NTG = WAVE;
  static constexpr int PPW = sizeof(JT) == 8 ? 2 : 4;
  static constexpr size_t OFF_A = 0;
  static constexpr size_t OFF_V = OFF_A + (size_t)KK * JLD * sizeof(JT);
  static constexpr size_t OFF_ROT = (OFF_V + (size_t)KK * JLD * sizeof(JT) + 7) & ~(size_t)7;
  static constexpr size_t OFF_PAIR = OFF_ROT + (size_t)KK * 8;
  static constexpr size_t OFF_INT = (OFF_PAIR + (size_t)(KK - 1) * (KK / 2) * 2 + 15) & ~(size_t)15;
  static constexpr size_t BYTES = (OFF_INT + (size_t)(KK + 8) * 4 + 15) & ~(size_t)15;
};

// F64: float64 sweeps to 2^-52 (float64 moments, or the re-solve of a marked point); else
// float32 sweeps to 2^-23, marking points with a near-degenerate kept pair (two eigenvalues
// above the rank floor within a relative 2^-13) for the float64 launch.  resolve_only: work
// only on marked points.
template <int KMAX, int PREC, bool F64>
__global__ __launch_bounds__(256) void curv_eigen_kernel(int64_t n, int64_t m, int k, int resolve_only,
                                                         unsigned char* __restrict__ ws, Fast2Ws L) {
  using JT = typename std::conditional<F64, double, float>::type;
  using C = EigCfg<KMAX, JT>;
  using ST = typename std::conditional<PREC == MOM_FP64, double, float>::type;
  constexpr int KK = C::KK;
  constexpr int HP = KK / 2;
  extern __shared__ __align__(16) unsigned char smem_all[];
  const int gid = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int64_t i = (int64_t)blockIdx.x * C::PPW + gid;
  if (i >= n) return;
  uint8_t* FL = ws + L.off_fl;
  const uint8_t fl0 = FL[i];
  if (fl0 & PF_NONFINITE) return;
  int* PE = reinterpret_cast<int*>(ws + L.off_pe);
  if (resolve_only && PE[i] != PE_NEED_FP64) return;
  unsigned char* sm = smem_all + (size_t)gid * C::BYTES;
  JT* A = reinterpret_cast<JT*>(sm + C::OFF_A);
  JT* V = reinterpret_cast<JT*>(sm + C::OFF_V);
  PointLds P{};
  P.ROT = reinterpret_cast<double*>(sm + C::OFF_ROT);
  P.pairs = reinterpret_cast<uint16_t*>(sm + C::OFF_PAIR);
  int* ord = reinterpret_cast<int*>(sm + C::OFF_INT);
  P.misc = ord + KK;
  const MomT<PREC>* Kin = reinterpret_cast<const MomT<PREC>*>(ws + L.off_k) + (size_t)i * KMAX * KMAX;

  for (int e = lane; e < KK * KK; e += WAVE) {
    const int x = e / KK, y = e % KK;
    A[x * C::JLD + y] = (x < k && y < k) ? (JT)Kin[x * KMAX + y] : (JT)0;
    V[x * C::JLD + y] = x == y ? (JT)1 : (JT)0;
  }
  for (int e = lane; e < (KK - 1) * HP; e += WAVE) {
    const int r = e / HP, s = e % HP;
    const int pa = rr_player(s, r, KK), pb = rr_player(KK - 1 - s, r, KK);
    P.pairs[e] = (uint16_t)((pa < pb ? pa : pb) | ((pa < pb ? pb : pa) << 8));
  }
  wave_sync();
  const int sweep = jacobi_sweeps<C, JT>(P, A, V, k, lane, F64 ? (JT)0x1p-52 : (JT)0x1p-23);
  const double unit = PREC == MOM_FP64 ? 0x1p-44 : 0x1p-24;   // rounding level of the moments
  const double rtol = (double)(m > k ? m : k) * unit;
  if constexpr (!F64) {
    // near-degenerate pair among the kept eigenvalues: leave it to the float64 launch
    bool near = false;
    if (lane < k) {
      JT s1 = 0;
      for (int y = 0; y < k; ++y) s1 = fmax(s1, A[y * C::JLD + y]);
      const JT keep = (JT)rtol * s1;
      const JT lx = A[lane * C::JLD + lane];
      if (lx > keep) {
        for (int y = 0; y < k; ++y) {
          const JT ly = A[y * C::JLD + y];
          near |= y != lane && ly > keep && fabs(lx - ly) < (JT)0x1p-13 * fmax(lx, ly);
        }
      }
    }
    if (__any(near)) {
      if (lane == 0) PE[i] = PE_NEED_FP64;
      return;
    }
  }
  // eigen order (descending), numerical rank, Ut, t_S
  if (lane < KK) {
    const JT dx = A[lane * C::JLD + lane];
    int rk = 0;
    for (int y = 0; y < KK; ++y) {
      const JT dy = A[y * C::JLD + y];
      rk += (dy > dx) || (dy == dx && y < lane);
    }
    ord[rk] = lane;
  }
  wave_sync();
  const double sig0 = (double)A[ord[0] * C::JLD + ord[0]];
  const int plim = (int)((int64_t)(k - 1) < m ? (int64_t)(k - 1) : m);
  int pe = 0;
  if (sig0 > 0.0)
    while (pe < plim && (double)A[ord[pe] * C::JLD + ord[pe]] > rtol * sig0) ++pe;
  ST* UT = reinterpret_cast<ST*>(ws + L.off_ut) + (size_t)i * KMAX * KMAX;
  // lane l < pe: column l of Ut and ||K ut_l||^2 in float64 (K from the workspace: the
  // addresses are uniform over the wave, so they are scalar loads)
  double ts = 0.0;
  {
    const int l = lane;
    const int x = l < pe ? ord[l] : 0;
    const double isq = l < pe ? 1.0 / sqrt((double)A[x * C::JLD + x]) : 0.0;
    for (int a = 0; a < k; ++a) {
      if (l < pe) UT[a * KMAX + l] = (ST)((double)V[a * C::JLD + x] * isq);
      double sv = 0.0;
      for (int bb = 0; bb < k; ++bb) sv = fma((double)Kin[a * KMAX + bb], (double)V[bb * C::JLD + x], sv);
      sv *= isq;
      ts = fma(sv, sv, ts);
    }
  }
  ts = wave_sum(ts);
  if (lane == 0) {
    const double tauk = reinterpret_cast<const double*>(ws + L.off_tau)[i];
    uint8_t fl = fl0;
    if (pe < plim) fl |= PF_RANK_DEFICIENT;
    if (sweep >= JAC_MAX_SWEEPS) fl |= PF_JACOBI_MAXSWEEPS;
    if (F64 && PREC != MOM_FP64) fl |= PF_EIGEN_FP64;
    if (!(sig0 > 0.0) || tauk == 0.0 || pe == 0) {
      fl |= PF_DEGENERATE;
    } else {
      const double smin = (double)A[ord[pe - 1] * C::JLD + ord[pe - 1]];
      if (beyond_precision(sig0, smin, k, m, pe, PREC == MOM_FP64 ? 2 : (PREC == MOM_BF16 ? 3 : 0)))
        fl |= PF_PRECISION_LIMIT;
    }
    reinterpret_cast<double*>(ws + L.off_ts)[i] = ts;
    PE[i] = pe;
    FL[i] = fl;
  }
}

// ---- 3. range pass: NW waves per point ---------------------------------------------------
template <int KMAX, int NW_, int PPW_, int ESZ_, bool BFA>
struct RangeCfg {
  static constexpr int KB = (KMAX + 15) / 16;               // 16-row blocks of the patch
  static constexpr int NW = NW_, PPW = PPW_, NTG = NW * WAVE, NT = PPW * NTG;
  static constexpr int ESZ = ESZ_;
  static constexpr int NCOLMAX = (KMAX - 1) * KMAX / 2 + 2; // pairs (l1 <= l2 < k-1), h, ones
  static constexpr int NB = (NCOLMAX + 15) / 16;
  static constexpr int NPAD = NB * 16;
  static constexpr int NBW = (NB + NW - 1) / NW;            // column blocks per wave
  // bf16 moments with several waves per point form V_r^T from bf16 high/low parts (VBF)
  static constexpr bool VBF = BFA && NW_ > 1;
  // patch chunk rows: the centred rows, q and ones (with VBF only q and ones stay in XS: the
  // patch goes to XB and, transposed and split into bf16 high and low parts, to XT)
  static constexpr int XQ = VBF ? 0 : 16 * KB, XONE = XQ + 1, XROWS = XQ + 2;
  static constexpr int VH = 16 * KB, VONE = 16 * KB + 1, VZERO = 16 * KB + 2;   // range chunk rows
  static constexpr int VROWS = 16 * KB + 3;
  static constexpr int VBLK = KB * (FCH / 16);              // blocks of the V_r^T chunk product
  static constexpr int VBW = (VBLK + NW - 1) / NW;
  // staging: each wave takes CPW columns of a chunk; its lanes split them into NW row groups
  static constexpr int CPW = FCH / NW;
  static constexpr int RPG = (KMAX + NW - 1) / NW;          // patch rows per group
  static constexpr int VPG = 16 * KB / NW;                  // range rows per group (h)
  // With several waves per point (float32 staging) the staged chunk (XS, XB) and its range
  // rows (VS) are double buffered: chunk c + 1 is staged while other waves still read chunk c, so a chunk needs two
  // barriers (staged; range rows formed).  h_c is formed from the V_r^T product's registers
  // when every wave holds all range rows of its columns (NW divides FCH / 16).
  static constexpr int NBUF = (NW > 1 && ESZ == 4) ? 2 : 1;   // float64 staging: 64 KiB cap
  static constexpr bool HREG = (FCH / 16) % NW == 0;
  static constexpr size_t XS_B = ((size_t)XROWS * FLDX * ESZ + 15) & ~(size_t)15;
  static constexpr size_t VS_B = ((size_t)VROWS * FLDX * ESZ + 15) & ~(size_t)15;
  static constexpr size_t OFF_XS = 0;
  static constexpr size_t OFF_VS = NBUF * XS_B;
  static constexpr size_t OFF_RED = OFF_VS + NBUF * VS_B;
  static constexpr size_t OFF_BJ = OFF_RED + (size_t)16 * NW * 8;          // tr G_j, r_j
  static constexpr size_t OFF_NB = OFF_BJ + (size_t)2 * KMAX * 8;
  static constexpr size_t OFF_PJ = OFF_NB + (size_t)KMAX * 4;
  static constexpr size_t OFF_RS = OFF_PJ + 2 * NPAD;                     // row scales 2^-e_j
  // bf16 moments: the staged patch rows again as binary16 (row j scaled by 2^-e_j, below),
  // the A operand of the range GEMM
  // (rows of FLDB = 72 elements: 144 bytes, so 16 lanes' 16-byte reads hit distinct banks)
  static constexpr int FLDB = FCH + 8;
  static constexpr size_t XB_B = BFA ? (((size_t)16 * KB * FLDB * 2 + 15) & ~(size_t)15) : 0;
  static constexpr size_t OFF_XB = (OFF_RS + (size_t)KMAX * 4 + 15) & ~(size_t)15;
  // XT[c][j] (high part, then low part): the B operand of the bf16 V_r^T product, K = j; rows of
  // FLDT = 40 elements (80 bytes: 16 lanes' 16-byte reads hit distinct banks)
  static constexpr int FLDT = 40;
  static constexpr size_t XT_B = VBF ? (size_t)2 * FCH * FLDT * 2 : 0;
  static constexpr size_t OFF_XT = OFF_XB + NBUF * XB_B;
  static constexpr size_t BYTES = OFF_XT + NBUF * XT_B;
  // bf16 moments keep the range rows (and h, ones, zero) as binary16 in the VS buffers, rows of
  // FLDH = 72 halves: the B operand of the range GEMM is formed by packed binary16 products
  static constexpr int FLDH = FCH + 8;
  static_assert(!BFA || (size_t)VROWS * FLDH * 2 <= VS_B, "binary16 range rows fit the VS buffer");
  static_assert(!BFA || HREG, "bf16 moments form h in registers");
};

// Binary16 staging of the bf16 path's range GEMM: row j of the centred patch is scaled by
// 2^-e_j, e_j the exponent with sqrt(K_jj) < 2^e_j (K_jj = ||X_c[j, :]||^2 from the Gram pass),
// so every staged value has magnitude at most about 1; the range rows are scaled by 16, so
// the pairwise products stay below 256.  The GEMM's row j is then rescaled by 2^(e_j - 8).
__device__ __forceinline__ int range_row_exp(float kjj) {
  int e = 0;
  if (kjj > 0.0f) (void)frexpf(sqrtf(kjj), &e);
  return e;
}

template <int KMAX, int PREC>
struct RangeCfgSel {
  // waves per point: past k = 26 the float32 pass splits a point over 8 waves, whose
  // registers then fit four waves per SIMD (60.8 against 63.8 ms at k = 32, m = 4096); the
  // bf16 pass measured no gain from it (21.0 against 20.5 ms) and keeps 4
  static constexpr int NW = KMAX <= 16 ? 1 : (KMAX <= 26 ? 2 : (PREC == MOM_FP32 ? 8 : 4));
  // waves per SIMD the register allocation aims for
  static constexpr int WPE = PREC == MOM_FP64 ? 1 : (NW == 8 ? 4 : 2);
  static constexpr int PPW = NW == 1 ? (PREC == MOM_FP64 ? 2 : 4) : 1;
  using C = RangeCfg<KMAX, NW, PPW, PREC == MOM_FP64 ? 8 : 4, PREC == MOM_BF16>;
};

template <int KMAX, int PREC>
__global__ __launch_bounds__((RangeCfgSel<KMAX, PREC>::C::NT))
__attribute__((amdgpu_waves_per_eu(RangeCfgSel<KMAX, PREC>::WPE, 8))) void curv_range_kernel(
    const float* __restrict__ X, int64_t n, int64_t m, int64_t ldx, const int32_t* __restrict__ idx,
    int k, int variant, const unsigned char* __restrict__ ws, Fast2Ws L, float* __restrict__ kappa_out,
    uint8_t* __restrict__ flags_out) {
  using C = typename RangeCfgSel<KMAX, PREC>::C;
  using ST = typename std::conditional<PREC == MOM_FP64, double, float>::type;   // staged values
  using AccT = typename std::conditional<PREC == MOM_FP64, doublex4, floatx4>::type;
  constexpr int KB = C::KB;
  extern __shared__ __align__(16) unsigned char smem_all[];
  const int gid = threadIdx.x / C::NTG;            // point group inside the workgroup
  const int tg = threadIdx.x % C::NTG;             // thread inside the group
  const int w = tg / WAVE, lane = tg % WAVE;
  const int64_t i = (int64_t)blockIdx.x * C::PPW + gid;
  if (i >= n) return;                              // whole group exits together
  const uint8_t fl = ws[L.off_fl + i];
  if (fl & (PF_NONFINITE | PF_DEGENERATE)) {
    if (tg == 0) {
      kappa_out[i] = (fl & PF_NONFINITE) ? __builtin_nanf("") : 0.0f;
      if (flags_out) flags_out[i] = fl;
    }
    return;
  }
  unsigned char* sm = smem_all + (size_t)gid * C::BYTES;
  ST* XS0 = reinterpret_cast<ST*>(sm + C::OFF_XS);
  ST* VS0 = reinterpret_cast<ST*>(sm + C::OFF_VS);
  constexpr int XSE = (int)(C::XS_B / sizeof(ST)), VSE = (int)(C::VS_B / sizeof(ST));   // buffer strides
  double* RED = reinterpret_cast<double*>(sm + C::OFF_RED);
  double* BJ = reinterpret_cast<double*>(sm + C::OFF_BJ);
  int* nb = reinterpret_cast<int*>(sm + C::OFF_NB);
  unsigned char* pj1 = sm + C::OFF_PJ;
  unsigned char* pj2 = pj1 + C::NPAD;
  uint16_t* XB0 = reinterpret_cast<uint16_t*>(sm + C::OFF_XB);
  constexpr int XBE = (int)(C::XB_B / 2);
  uint16_t* XT0 = reinterpret_cast<uint16_t*>(sm + C::OFF_XT);
  constexpr int XTE = (int)(C::XT_B / 2), XTLO = FCH * C::FLDT;   // buffer stride, low-part offset
  const int pe = reinterpret_cast<const int*>(ws + L.off_pe)[i];
  const double tauk = reinterpret_cast<const double*>(ws + L.off_tau)[i];
  const double tS = reinterpret_cast<const double*>(ws + L.off_ts)[i];
  const ST* UT = reinterpret_cast<const ST*>(ws + L.off_ut) + (size_t)i * KMAX * KMAX;
  const int npair = (k - 1) * k / 2;
  const int ncol = npair + 2;
  const int nbr = (ncol + 15) / 16;                // column blocks in use

  float* RSF = reinterpret_cast<float*>(sm + C::OFF_RS);   // binary16 row scales (bf16 moments)
  const float* KD = reinterpret_cast<const float*>(ws + L.off_k) + (size_t)i * KMAX * KMAX;

  // ---- setup: neighbour rows, column tables, zero rows -----------------------------
  if (tg < k) {
    nb[tg] = idx[i * k + tg];                      // checked by the Gram pass
    if constexpr (PREC == MOM_BF16) RSF[tg] = ldexpf(1.0f, -range_row_exp(KD[tg * KMAX + tg]));
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
#pragma unroll
  for (int bf = 0; bf < C::NBUF; ++bf) {
    if constexpr (!C::VBF)
      for (int t = tg; t < (16 * KB - k) * FLDX; t += C::NTG) XS0[bf * XSE + k * FLDX + t] = (ST)0;
    if constexpr (PREC == MOM_BF16)
      for (int t = tg; t < (16 * KB - k) * C::FLDB; t += C::NTG) XB0[bf * XBE + k * C::FLDB + t] = 0;
    if constexpr (C::VBF) {
      for (int t = tg; t < 2 * FCH * (32 - k); t += C::NTG) {   // XT entries j >= k, both parts
        const int pl = t / (FCH * (32 - k)), r = t % (FCH * (32 - k));
        XT0[bf * XTE + pl * XTLO + (r / (32 - k)) * C::FLDT + k + r % (32 - k)] = 0;
      }
    }
    for (int t = tg; t < FLDX; t += C::NTG) VS0[bf * VSE + C::VZERO * FLDX + t] = (ST)0;
    if constexpr (PREC == MOM_BF16)
      for (int t = tg; t < C::FLDH; t += C::NTG)
        reinterpret_cast<uint16_t*>(VS0 + bf * VSE)[C::VZERO * C::FLDH + t] = 0;
  }
  // Ut^T operand of the V_r^T chunk product: A[l][j] = Ut[j][l] at row l = 16 lb + lane%16,
  // k index j = 16 jb + st + 4 (lane/16): the four lane groups read patch rows four apart,
  // 16 banks apart in LDS, so the B operand's reads are conflict-free
  constexpr int UAK = C::VBF ? 1 : KB;
  ST ua[KB][UAK][4];
  // VBF: Ut^T split into bf16 high and low parts, A[l][j] with k index j = 8 (lane/16) + e of
  // one 16x16x32 step (k <= 32)
  shortx8 uah[KB], ual[KB];
  if constexpr (C::VBF) {
#pragma unroll
    for (int lb = 0; lb < KB; ++lb)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int l = 16 * lb + lane % 16, j = 8 * (lane / 16) + e;
        const float u = (l < pe && j < k) ? (float)UT[j * KMAX + l] : 0.0f;
        const uint16_t hi = f2bf(u);
        uah[lb][e] = (short)hi;
        ual[lb][e] = (short)f2bf(u - __uint_as_float((uint32_t)hi << 16));
      }
  } else {
#pragma unroll
    for (int lb = 0; lb < KB; ++lb)
#pragma unroll
      for (int jb = 0; jb < KB; ++jb)
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int l = 16 * lb + lane % 16, j = 16 * jb + st + 4 * (lane / 16);
          ua[lb][jb][st] = (l < pe && j < k) ? UT[j * KMAX + l] : (ST)0;
        }
  }
  gsync<C::NW>();
  // column blocks past the point's ncol columns read the zero row, so every wave runs all NBW
  // blocks without a branch and the compiler can interleave their loads
  int off1[C::NBW], off2[C::NBW];
#pragma unroll
  for (int b = 0; b < C::NBW; ++b) {
    const int nbg = w + C::NW * b;
    const int pc = nbg * 16 + lane % 16 < C::NPAD ? nbg * 16 + lane % 16 : C::NPAD - 1;
    off1[b] = pj1[pc] * (PREC == MOM_BF16 ? C::FLDH : FLDX);
    off2[b] = pj2[pc] * (PREC == MOM_BF16 ? C::FLDH : FLDX);
  }

  // staging: lane (cl, g) of wave w holds rows g*RPG + r of column w*CPW + cl of the chunk
  const int cl = lane % C::CPW, grp = lane / C::CPW;
  const int colw = w * C::CPW + cl;                // column inside the chunk
  int nbr_[C::RPG];
#pragma unroll
  for (int r = 0; r < C::RPG; ++r) {
    const int j = grp * C::RPG + r;
    nbr_[r] = j < k ? nb[j] : 0;
  }
  ST* XS = XS0;          // the current chunk's buffers (the lambdas below read these)
  ST* VS = VS0;
  uint16_t* XB = XB0;
  uint16_t* XT = XT0;
  float xr[C::RPG];
  // unconditional gather (rows j >= k read row nbr_ = 0, columns past m the last column, both
  // in bounds); the staging zeroes those entries where it uses them, so nothing waits for
  // this chunk's loads before the products that run behind them
  auto load = [&](int64_t c0) {
    const int64_t c = c0 + colw;
    const int64_t cc = c < m ? c : m - 1;
#pragma unroll
    for (int r = 0; r < C::RPG; ++r) xr[r] = X[(int64_t)nbr_[r] * ldx + cc];
  };
  // the centred chunk: offsets from the first row, minus their mean (as centre_column), and
  // q_c = sum_j X_c[j, c]^2, reduced over the lanes that share the column
  auto stage = [&](int64_t c0) {
    if constexpr (PREC == MOM_FP64) {
      const bool cin = c0 + colw < m;
      const double x0 = (double)__shfl(xr[0], cl, WAVE);
      double d[C::RPG];
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < C::RPG; ++r) {
        const int j = grp * C::RPG + r;
        d[r] = (j < k && cin) ? (double)xr[r] - x0 : 0.0;
        s += d[r];
      }
#pragma unroll
      for (int o = C::CPW; o < WAVE; o <<= 1) s += __shfl_xor(s, o, WAVE);
      const double mean = s / (double)k;
      double q = 0.0;
#pragma unroll
      for (int r = 0; r < C::RPG; ++r) {
        const int j = grp * C::RPG + r;
        if (j < k) {
          const double xc = d[r] - mean;
          q = fma(xc, xc, q);
          XS[j * FLDX + colw] = xc;
        }
      }
#pragma unroll
      for (int o = C::CPW; o < WAVE; o <<= 1) q += __shfl_xor(q, o, WAVE);
      if (grp == 0) XS[C::XQ * FLDX + colw] = q;
    } else {
      const bool cin = c0 + colw < m;
      const float x0 = group_bcast_f<C::CPW>(xr[0]);
      float d[C::RPG];
      float s = 0.0f;
#pragma unroll
      for (int r = 0; r < C::RPG; ++r) {
        const int j = grp * C::RPG + r;
        d[r] = (j < k && cin) ? xr[r] - x0 : 0.0f;
        s += d[r];
      }
      s = group_sum_f<C::CPW>(s);
      const float mean = s / (float)k;
      float q = 0.0f;
      // with eight rows per group the transposed high and low parts of the group's rows are
      // eight consecutive entries of XT: one 16-byte store each (zeros past row k)
      constexpr bool XT8 = C::VBF && C::RPG == 8;
      shortx8 th = {0, 0, 0, 0, 0, 0, 0, 0}, tl = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < C::RPG; ++r) {
        const int j = grp * C::RPG + r;
        if (j < k) {
          const float xc = d[r] - mean;
          q = fmaf(xc, xc, q);
          if constexpr (C::VBF) {
            const uint16_t hi = f2bf(xc);
            const uint16_t lo = f2bf(xc - __uint_as_float((uint32_t)hi << 16));
            XB[j * C::FLDB + colw] = f2h(xc * RSF[j]);
            if constexpr (XT8) {
              th[r % 8] = (short)hi;
              tl[r % 8] = (short)lo;
            } else {
              XT[colw * C::FLDT + j] = hi;
              XT[XTLO + colw * C::FLDT + j] = lo;
            }
          } else {
            XS[j * FLDX + colw] = xc;
            if constexpr (PREC == MOM_BF16) XB[j * C::FLDB + colw] = f2h(xc * RSF[j]);
          }
        }
      }
      if constexpr (XT8) {
        *reinterpret_cast<shortx8*>(XT + colw * C::FLDT + 8 * grp) = th;
        *reinterpret_cast<shortx8*>(XT + XTLO + colw * C::FLDT + 8 * grp) = tl;
      }
      q = group_sum_f<C::CPW>(q);
      if (grp == 0) XS[C::XQ * FLDX + colw] = q;
    }
    if (grp == 0) XS[C::XONE * FLDX + colw] = (c0 + colw < m) ? (ST)1 : (ST)0;
  };

  AccT acc[KB][C::NBW];
#pragma unroll
  for (int a = 0; a < KB; ++a)
#pragma unroll
    for (int b = 0; b < C::NBW; ++b) acc[a][b] = AccT{0, 0, 0, 0};
  double tD = 0.0;
  load(0);
  int buf = 0;
  for (int64_t c0 = 0; c0 < m; c0 += FCH) {
    XS = XS0 + buf * XSE;
    VS = VS0 + buf * VSE;
    XB = XB0 + buf * XBE;
    XT = XT0 + buf * XTE;
    if constexpr (C::NBUF == 2) buf ^= 1;
    stage(c0);
    gsync<C::NW>();
    if (c0 + FCH < m) load(c0 + FCH);
    // V_r^T chunk = Ut^T X_c (rows l, columns c of the chunk); with HREG each wave also sums
    // h over the rows it formed, for its columns 16 cb .. 16 cb + 15
    ST hsum[C::VBW];
#pragma unroll
    for (int t = 0; t < C::VBW; ++t) hsum[t] = 0;
#pragma unroll
    for (int t = 0; t < C::VBW; ++t) {
      const int vb = w + C::NW * t;
      if (vb < C::VBLK) {
        const int lb = vb / (FCH / 16), cb = vb % (FCH / 16);
        AccT v = AccT{0, 0, 0, 0};
        if constexpr (C::VBF) {
          // three bf16 products (high x low, low x high, high x high, the small terms first):
          // Ut^T X_c to about 2^-16 of the terms, far inside the binary16 range products' 2^-11
          const uint16_t* xt = XT + (16 * cb + lane % 16) * C::FLDT + 8 * (lane / 16);
          const shortx8 xh = *reinterpret_cast<const shortx8*>(xt);
          const shortx8 xl = *reinterpret_cast<const shortx8*>(xt + XTLO);
          v = mfma16x16x32bf16(uah[lb], xl, v);
          v = mfma16x16x32bf16(ual[lb], xh, v);
          v = mfma16x16x32bf16(uah[lb], xh, v);
        } else {
#pragma unroll
          for (int jb = 0; jb < KB; ++jb)
#pragma unroll
            for (int st = 0; st < 4; ++st) {
              const ST bv = XS[(16 * jb + st + 4 * (lane / 16)) * FLDX + 16 * cb + lane % 16];
              if constexpr (PREC == MOM_FP64) v = mfma16x16x4f64(ua[lb][jb][st], bv, v);
              else v = mfma16x16x4(ua[lb][jb][st], bv, v);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int l = 16 * lb + (PREC == MOM_FP64 ? lane / 16 + 4 * r : 4 * (lane / 16) + r);
          const ST vr = (ST)v[r];
          if constexpr (PREC == MOM_BF16)
            reinterpret_cast<uint16_t*>(VS)[l * C::FLDH + 16 * cb + lane % 16] = f2h(16.0f * vr);
          else
            VS[l * FLDX + 16 * cb + lane % 16] = vr;
          hsum[t] += vr * vr;
        }
      }
    }
    if constexpr (C::HREG) {
      // wave w's blocks t cover column block cb = (w + NW t) % (FCH / 16) for every row block:
      // h_c (rows l >= pe hold zeros), the ones row and t_D's sum_c q_c h_c without a barrier
#pragma unroll
      for (int t = 0; t < C::VBW; ++t) {
        const int vb = w + C::NW * t;
        if (vb < FCH / 16) {          // the first row block of each of the wave's columns
          ST h = 0;
#pragma unroll
          for (int t2 = 0; t2 < C::VBW; ++t2)
            if ((w + C::NW * t2) % (FCH / 16) == vb) h += hsum[t2];
          if constexpr (PREC == MOM_FP64) {
            h += __shfl_xor(h, 16, WAVE);
            h += __shfl_xor(h, 32, WAVE);
          } else {
            h = xsum32(xsum16(h));
          }
          if (lane < 16) {
            const int col = 16 * vb + lane;
            if constexpr (PREC == MOM_BF16) {
              uint16_t* VSh = reinterpret_cast<uint16_t*>(VS);
              VSh[C::VH * C::FLDH + col] = f2h(16.0f * h);
              VSh[C::VONE * C::FLDH + col] = (c0 + col < m) ? f2h(16.0f) : (uint16_t)0;
            } else {
              VS[C::VH * FLDX + col] = h;
              VS[C::VONE * FLDX + col] = (c0 + col < m) ? (ST)1 : (ST)0;
            }
            tD = fma((double)XS[C::XQ * FLDX + col], (double)h, tD);
          }
        }
      }
    }
    gsync<C::NW>();
    // h_c = sum_l V[c, l]^2 (rows l >= pe hold zeros), the ones row, and t_D's sum_c q_c h_c
    if constexpr (!C::HREG) {
      ST h = 0;
#pragma unroll
      for (int r = 0; r < C::VPG; ++r) {
        const ST v = VS[(grp * C::VPG + r) * FLDX + colw];
        h += v * v;
      }
#pragma unroll
      for (int o = C::CPW; o < WAVE; o <<= 1) h += __shfl_xor(h, o, WAVE);
      if (grp == 0) {
        VS[C::VH * FLDX + colw] = h;
        VS[C::VONE * FLDX + colw] = (c0 + colw < m) ? (ST)1 : (ST)0;
        tD = fma((double)XS[C::XQ * FLDX + colw], (double)h, tD);
      }
      gsync<C::NW>();
    }
    if constexpr (PREC == MOM_FP64) {
      const int st4 = m - c0 >= FCH ? FCH / 4 : (int)((m - c0 + 3) / 4);
      for (int s4 = 0; s4 < st4; ++s4) {
        const int col = 4 * s4 + lane / 16;
        double av[KB];
#pragma unroll
        for (int a = 0; a < KB; ++a) av[a] = XS[(16 * a + lane % 16) * FLDX + col];
#pragma unroll
        for (int b = 0; b < C::NBW; ++b) {
          const double bv = VS[off1[b] + col] * VS[off2[b] + col];
#pragma unroll
          for (int a = 0; a < KB; ++a) acc[a][b] = mfma16x16x4f64(av[a], bv, acc[a][b]);
        }
      }
    } else if constexpr (PREC == MOM_FP32) {
      auto gstep = [&](int g) {
        const int col = 16 * g + 4 * (lane / 16);
        floatx4 av[KB];
#pragma unroll
        for (int a = 0; a < KB; ++a)
          av[a] = *reinterpret_cast<const floatx4*>(XS + (16 * a + lane % 16) * FLDX + col);
#pragma unroll
        for (int b = 0; b < C::NBW; ++b) {
          const floatx4 x1 = *reinterpret_cast<const floatx4*>(VS + off1[b] + col);
          const floatx4 x2 = *reinterpret_cast<const floatx4*>(VS + off2[b] + col);
          const floatx4 bv = x1 * x2;
#pragma unroll
          for (int st = 0; st < 4; ++st)
#pragma unroll
            for (int a = 0; a < KB; ++a) acc[a][b] = mfma16x16x4(av[a][st], bv[st], acc[a][b]);
        }
      };
      const int ng = m - c0 >= FCH ? FCH / 16 : (int)((m - c0 + 15) / 16);
      for (int g = 0; g < ng; ++g) gstep(g);
    } else {
      // binary16 operands, 32-column steps: lane l supplies columns 32 s + 8 (l / 16) + e; the
      // A operand is the scaled patch, the B operand the pairwise products of the scaled range
      // rows, eight per lane from four packed binary16 multiplies.  Both are stored as 16-bit
      // integers and read as such (a binary16 pointer would not alias those stores).
      // The lane's column part 8 (l / 16) goes into the bases and the two steps are unrolled, so
      // a step's column offset is an immediate of the LDS reads.
      const uint16_t* VSh = reinterpret_cast<const uint16_t*>(VS) + 8 * (lane / 16);
      const uint16_t* XBl = XB + 8 * (lane / 16);
      auto ld8 = [](const uint16_t* p) { return __builtin_bit_cast(halfx8, *reinterpret_cast<const shortx8*>(p)); };
      auto gstep = [&](int s32) {
        const int col0 = 32 * s32;
        halfx8 ahf[KB];
#pragma unroll
        for (int a = 0; a < KB; ++a) ahf[a] = ld8(XBl + (16 * a + lane % 16) * C::FLDB + col0);
        if constexpr (C::NW == 2 || C::NW == 4) {
          // the operand rows of block b + 1 are in flight while block b's products are formed
          constexpr int PD = 1, RING = PD + 1;
          halfx8 pq[RING][2];
          auto rd = [&](halfx8 (&d)[2], int b) {
            d[0] = ld8(VSh + off1[b] + col0);
            d[1] = ld8(VSh + off2[b] + col0);
          };
#pragma unroll
          for (int b = 0; b < PD && b < C::NBW; ++b) rd(pq[b], b);
#pragma unroll
          for (int b = 0; b < C::NBW; ++b) {
            if (b + PD < C::NBW) rd(pq[(b + PD) % RING], b + PD);
            const halfx8 bv = pq[b % RING][0] * pq[b % RING][1];
#pragma unroll
            for (int a = 0; a < KB; ++a) acc[a][b] = mfma16x16x32f16(ahf[a], bv, acc[a][b]);
          }
        } else {
#pragma unroll
          for (int b = 0; b < C::NBW; ++b) {
            const halfx8 p = ld8(VSh + off1[b] + col0);
            const halfx8 q = ld8(VSh + off2[b] + col0);
            const halfx8 bv = p * q;
#pragma unroll
            for (int a = 0; a < KB; ++a) acc[a][b] = mfma16x16x32f16(ahf[a], bv, acc[a][b]);
          }
        }
      };
      const int st32 = m - c0 >= FCH ? FCH / 32 : (int)((m - c0 + 31) / 32);
#pragma unroll
      for (int s32 = 0; s32 < FCH / 32; ++s32)
        if (s32 < st32) gstep(s32);
    }
    // single buffers: the next chunk's staging overwrites what this GEMM reads
    if constexpr (C::NBUF == 1) gsync<C::NW>();
  }
  gsync<C::NW>();
  if constexpr (PREC == MOM_BF16) {
    // undo the binary16 scales: row j of the GEMM by 2^(e_j - 8)
#pragma unroll
    for (int a = 0; a < KB; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = 16 * a + 4 * (lane / 16) + r;
        const float sc = j < k ? 1.0f / (256.0f * RSF[j]) : 0.0f;   // 2^(e_j - 8), exact
#pragma unroll
        for (int b = 0; b < C::NBW; ++b) acc[a][b][r] *= sc;
      }
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
  gsync<C::NW>();
  for (int j = tg; j < k; j += C::NTG) {
    const double bj = BJ[KMAX + j] - BJ[j];       // (X_c d_P)_j = r_j - tr G_j
    part[2] = fma(bj, bj, part[2]);
  }
  if (tg == 0) part[3] = tS;
  group_sum<C::NW, 5>(part, RED, tg);

  if (tg == 0) {
    kappa_out[i] = (float)fast_combine(part, tauk, k, m, pe, variant, nullptr);
    if (flags_out) flags_out[i] = fl;
  }
}

template <int KMAX, int PREC>
static hipError_t launch_fast2_kp(const float* X, int64_t n, int64_t m, int64_t ldx, const int32_t* idx,
                                  int k, int variant, float* kappa, uint8_t* flags, unsigned char* ws,
                                  const Fast2Ws& L, hipStream_t stream) {
  using G = GramCfg<KMAX, PREC>;
  using E32 = EigCfg<KMAX, float>;
  using E64 = EigCfg<KMAX, double>;
  using R = typename RangeCfgSel<KMAX, PREC>::C;
  static_assert(G::PPW * G::BYTES <= 64 * 1024 && E32::PPW * E32::BYTES <= 64 * 1024 &&
                    E64::PPW * E64::BYTES <= 64 * 1024 && R::PPW * R::BYTES <= 64 * 1024,
                "per-workgroup LDS of the two-pass kernels stays within 64 KiB");
  timing_begin(11, stream);
  hipLaunchKernelGGL((curv_gram_kernel<KMAX, PREC>), dim3((unsigned)((n + G::PPW - 1) / G::PPW)), dim3(G::PPW * WAVE),
                     G::PPW * G::BYTES, stream, X, n, m, ldx, idx, k, ws, L);
  timing_end(11, stream);
  timing_begin(12, stream);
  if constexpr (PREC != MOM_FP64) {
    hipLaunchKernelGGL((curv_eigen_kernel<KMAX, PREC, false>), dim3((unsigned)((n + E32::PPW - 1) / E32::PPW)),
                       dim3(E32::PPW * WAVE), E32::PPW * E32::BYTES, stream, n, m, k, 0, ws, L);
  }
  hipLaunchKernelGGL((curv_eigen_kernel<KMAX, PREC, true>), dim3((unsigned)((n + E64::PPW - 1) / E64::PPW)),
                     dim3(E64::PPW * WAVE), E64::PPW * E64::BYTES, stream, n, m, k,
                     PREC == MOM_FP64 ? 0 : 1, ws, L);
  timing_end(12, stream);
  timing_begin(13, stream);
  hipLaunchKernelGGL((curv_range_kernel<KMAX, PREC>), dim3((unsigned)((n + R::PPW - 1) / R::PPW)), dim3(R::NT),
                     R::PPW * R::BYTES, stream, X, n, m, ldx, idx, k, variant, (const unsigned char*)ws, L,
                     kappa, flags);
  timing_end(13, stream);
  return hipGetLastError();
}

template <int KMAX>
static hipError_t launch_fast2_k(const float* X, int64_t n, int64_t m, int64_t ldx, const int32_t* idx, int k,
                                 int precision, int variant, float* kappa, uint8_t* flags, unsigned char* ws,
                                 const Fast2Ws& L, hipStream_t stream) {
  if (precision == 1)
    return launch_fast2_kp<KMAX, MOM_BF16>(X, n, m, ldx, idx, k, variant, kappa, flags, ws, L, stream);
  if (precision == 3) {
    if constexpr (KMAX <= 28)
      return launch_fast2_kp<KMAX, MOM_FP64>(X, n, m, ldx, idx, k, variant, kappa, flags, ws, L, stream);
    return hipErrorInvalidValue;
  }
  return launch_fast2_kp<KMAX, MOM_FP32>(X, n, m, ldx, idx, k, variant, kappa, flags, ws, L, stream);
}

hipError_t launch_curv_fast2(const float* X, int64_t n, int64_t m, int64_t ldx, const int32_t* idx, int k,
                             int precision, int variant, float* kappa, uint8_t* flags, void* ws,
                             hipStream_t stream) {
  const Fast2Ws L = fast2_ws(n, k, precision);
  unsigned char* w = reinterpret_cast<unsigned char*>(ws);
  switch (L.kmax) {
    case 16: return launch_fast2_k<16>(X, n, m, ldx, idx, k, precision, variant, kappa, flags, w, L, stream);
    case 20: return launch_fast2_k<20>(X, n, m, ldx, idx, k, precision, variant, kappa, flags, w, L, stream);
    case 24: return launch_fast2_k<24>(X, n, m, ldx, idx, k, precision, variant, kappa, flags, w, L, stream);
    case 28: return launch_fast2_k<28>(X, n, m, ldx, idx, k, precision, variant, kappa, flags, w, L, stream);
    default: return launch_fast2_k<32>(X, n, m, ldx, idx, k, precision, variant, kappa, flags, w, L, stream);
  }
}

size_t curv_fast2_ws_bytes(int64_t n, int k, int precision) { return fast2_ws(n, k, precision).total; }

}  // namespace mc
