// Brute-force k nearest neighbours on gfx950 (Step 1 of the method, eq. knn;
// the kNN-Graph step of Algorithm 1).
//
// Pipeline (all on one stream, workspace owned by the caller):
//  1. knn_colsum / knn_center: subtract the column mean (distances are
//     translation invariant; centring shrinks ||x||^2 and with it the
//     cancellation in ||x||^2 + ||y||^2 - 2 x.y), write the centred copy with a
//     zero-padded row stride, float32 norms, a per-row rounding radius for the
//     candidate certificate, and a bf16 copy when asked.
//  2. knn_gemm_topk: query tile x database tile scores s = ||y||^2 - 2 x.y on
//     MFMA (fp32 32x32x2 or bf16 16x16x32), written to LDS, then each wave keeps
//     a sorted list of the K' best (score, index) per query row in registers
//     (lane r holds rank r); candidates are filtered against the K'-th score
//     with a ballot and inserted with a wave-wide shift.  The database range is
//     split over blockIdx.y so that the grid fills the chip.
//  3. knn_rerank: merge the split lists, recompute the K' distances in float32
//     difference form sum_a (x_a - y_a)^2 from the original X, order by
//     (distance, index), keep k, and flag ambiguous gaps and candidate sets
//     that cannot be certified complete.
#include <float.h>
#include <limits.h>
#include <math.h>

#include "mc_device.h"
#include "mc_internal.h"

namespace mc {

constexpr int KBQ = 128;   // queries per tile
constexpr int KBN = 128;   // database points per tile
constexpr int KNT = 256;   // threads per GEMM workgroup
constexpr int SLD = KBN + 4;  // score-tile row stride (floats)
constexpr int KCMAX = 64;  // largest candidate list

// ------------------------------------------------------------------------------------
// prep
// ------------------------------------------------------------------------------------
// Partial column sums over a block of rows (deterministic two-level reduction).
__global__ __launch_bounds__(256) void knn_colsum_kernel(const float* __restrict__ X, int64_t n,
                                                         int64_t m, int64_t ldx, int64_t rows_per,
                                                         double* __restrict__ part) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= m) return;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per;
  const int64_t r1 = r0 + rows_per < n ? r0 + rows_per : n;
  double s = 0.0;
  for (int64_t r = r0; r < r1; ++r) s += (double)X[r * ldx + c];
  part[(int64_t)blockIdx.y * m + c] = s;
}

__global__ __launch_bounds__(256) void knn_mean_kernel(const double* __restrict__ part, int64_t m,
                                                       int nparts, int64_t n, float* __restrict__ mu) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= m) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += part[(int64_t)p * m + c];
  mu[c] = (float)(s / (double)n);
}

// One wave per row: centred float32 copy (row stride mp, zero padded), bf16 copy
// (optional), norm ||xc||^2 (float32, from a float64 sum), rounding radius.
__global__ __launch_bounds__(256) void knn_center_kernel(
    const float* __restrict__ X, int64_t n, int64_t m, int64_t ldx, int64_t mp,
    const float* __restrict__ mu, float* __restrict__ xc, uint16_t* __restrict__ xb,
    float* __restrict__ norms, float* __restrict__ radius, int precision) {
  const int64_t r = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
  const int lane = threadIdx.x % WAVE;
  if (r >= n) return;
  double s = 0.0, e = 0.0;
  for (int64_t c = lane; c < mp; c += WAVE) {
    float v = 0.0f;
    if (c < m) v = X[r * ldx + c] - mu[c];
    xc[r * mp + c] = v;
    s = fma((double)v, (double)v, s);
    if (precision == 1) {
      const uint16_t h = f2bf(v);
      xb[r * mp + c] = h;
      const double d = (double)bf2f(h) - (double)v;
      e = fma(d, d, e);
    }
  }
  s = wave_sum(s);
  e = wave_sum(e);
  if (lane == 0) {
    norms[r] = (float)s;
    radius[r] = (float)sqrt(e);    // ||bf16(xc) - xc|| (0 on the fp32 path)
  }
}

// stats[0] = max_i sqrt(norm_i), stats[1] = max_i radius_i  (one workgroup)
__global__ __launch_bounds__(256) void knn_stats_kernel(const float* __restrict__ norms,
                                                        const float* __restrict__ radius, int64_t n,
                                                        float* __restrict__ stats) {
  __shared__ float red[2][4];
  float a = 0.0f, b = 0.0f;
  for (int64_t r = threadIdx.x; r < n; r += 256) {
    a = fmaxf(a, sqrtf(norms[r]));
    b = fmaxf(b, radius[r]);
  }
  a = wave_max(a);
  b = wave_max(b);
  if (threadIdx.x % WAVE == 0) {
    red[0][threadIdx.x / WAVE] = a;
    red[1][threadIdx.x / WAVE] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    stats[0] = fmaxf(fmaxf(red[0][0], red[0][1]), fmaxf(red[0][2], red[0][3]));
    stats[1] = fmaxf(fmaxf(red[1][0], red[1][1]), fmaxf(red[1][2], red[1][3]));
  }
}

// ------------------------------------------------------------------------------------
// wave-level sorted list: lane r holds the r-th smallest (score, index), r < kc
// ------------------------------------------------------------------------------------
__device__ __forceinline__ float rdlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ void list_insert(float& ls, int& lj, float s, int j, uint64_t kmask) {
  const int lane = lane_id();
  const bool less = (ls < s) || (ls == s && lj < j);
  const int pos = __popcll(__ballot(less) & kmask);
  const float us = __shfl_up(ls, 1, WAVE);
  const int uj = __shfl_up(lj, 1, WAVE);
  if (lane > pos) {
    ls = us;
    lj = uj;
  } else if (lane == pos) {
    ls = s;
    lj = j;
  }
}

// Filter one 128-wide score row against the list and insert what passes.
__device__ __forceinline__ void row_update(float& ls, int& lj, float v0, float v1, int64_t j0,
                                           int kc, uint64_t kmask) {
  float th = rdlane(ls, kc - 1);
  uint64_t m0 = __ballot(v0 < th), m1 = __ballot(v1 < th);
  while (m0 | m1) {
    float sv;
    int jv;
    if (m0) {
      const int src = __ffsll((unsigned long long)m0) - 1;
      m0 &= m0 - 1;
      sv = rdlane(v0, src);
      jv = (int)(j0 + src);
    } else {
      const int src = __ffsll((unsigned long long)m1) - 1;
      m1 &= m1 - 1;
      sv = rdlane(v1, src);
      jv = (int)(j0 + 64 + src);
    }
    if (sv < th) {
      list_insert(ls, lj, sv, jv, kmask);
      th = rdlane(ls, kc - 1);
    }
  }
}

// ------------------------------------------------------------------------------------
// GEMM + top-K'.  PREC 0: fp32 MFMA 32x32x2, BK = 16; PREC 1: bf16 MFMA 16x16x32, BK = 64.
// ------------------------------------------------------------------------------------
template <int PREC>
struct GemmCfg;
template <>
struct GemmCfg<0> {
  static constexpr int BK = 16;                 // columns per stage
  static constexpr int ALD = BK + 4;            // staging row stride (elements)
  static constexpr int ESZ = 4;
  static constexpr size_t STAGE_B = (size_t)2 * (KBQ + KBN) * ALD * ESZ;
};
template <>
struct GemmCfg<1> {
  static constexpr int BK = 64;
  static constexpr int ALD = BK + 8;
  static constexpr int ESZ = 2;
  static constexpr size_t STAGE_B = (size_t)2 * (KBQ + KBN) * ALD * ESZ;
};

template <int PREC>
constexpr size_t gemm_lds_bytes() {
  return GemmCfg<PREC>::STAGE_B > (size_t)KBQ * SLD * 4 ? GemmCfg<PREC>::STAGE_B
                                                         : (size_t)KBQ * SLD * 4;
}

template <int PREC>
__global__ __launch_bounds__(KNT) void knn_gemm_topk_kernel(
    const void* __restrict__ xsrc, int64_t mp, const float* __restrict__ norms, int64_t n, int kc,
    int tiles_per_split, int include_self, float* __restrict__ cand_s, int* __restrict__ cand_j) {
  using G = GemmCfg<PREC>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int w = tid / WAVE, lane = tid % WAVE;
  const int64_t q0 = (int64_t)blockIdx.x * KBQ;
  const int split = blockIdx.y;
  const int64_t ntiles = (n + KBN - 1) / KBN;
  const int64_t t_begin = (int64_t)split * tiles_per_split;
  const int64_t t_end = t_begin + tiles_per_split < ntiles ? t_begin + tiles_per_split : ntiles;
  const uint64_t kmask = kc >= 64 ? ~0ull : ((1ull << kc) - 1ull);

  float ls[32];
  int lj[32];
#pragma unroll
  for (int r = 0; r < 32; ++r) {
    ls[r] = INFINITY;
    lj[r] = INT_MAX;
  }

  const int wr = w / 2, wc = w % 2;      // wave tile: rows 64*wr.., cols 64*wc..
  float* Ss = reinterpret_cast<float*>(smem);
  const int nch = (int)(mp / G::BK);

  for (int64_t t = t_begin; t < t_end; ++t) {
    const int64_t j0 = t * KBN;
    if constexpr (PREC == 0) {
      const float* xs = reinterpret_cast<const float*>(xsrc);
      float* As = reinterpret_cast<float*>(smem);
      floatx16 acc[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
      // staging: 128 query rows + 128 db rows, 16 floats each = 1024 float4; 4 per thread
      float4 pre[4];
      auto gload = [&](int ch) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int f = tid + u * KNT;
          const int row = (f / 4) % 128;
          const int c4 = f % 4;
          const bool isq = f < 512;
          const int64_t g = isq ? q0 + row : j0 + row;
          float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
          if (g < n) v = *reinterpret_cast<const float4*>(xs + g * mp + (int64_t)ch * G::BK + 4 * c4);
          pre[u] = v;
        }
      };
      auto sstore = [&](int buf) {
        float* base = As + (size_t)buf * (KBQ + KBN) * G::ALD;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int f = tid + u * KNT;
          const int row = f / 4;         // 0..255: queries then db rows
          const int c4 = f % 4;
          *reinterpret_cast<float4*>(base + row * G::ALD + 4 * c4) = pre[u];
        }
      };
      gload(0);
      sstore(0);
      __syncthreads();
      for (int ch = 0; ch < nch; ++ch) {
        if (ch + 1 < nch) gload(ch + 1);
        const float* base = As + (size_t)(ch & 1) * (KBQ + KBN) * G::ALD;
        const int h = lane / 32;
        float av[2][8], bv[2][8];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const float* pa = base + (64 * wr + 32 * a + lane % 32) * G::ALD + 8 * h;
          const float4 x0 = *reinterpret_cast<const float4*>(pa);
          const float4 x1 = *reinterpret_cast<const float4*>(pa + 4);
          av[a][0] = x0.x; av[a][1] = x0.y; av[a][2] = x0.z; av[a][3] = x0.w;
          av[a][4] = x1.x; av[a][5] = x1.y; av[a][6] = x1.z; av[a][7] = x1.w;
          const float* pb = base + (KBQ + 64 * wc + 32 * a + lane % 32) * G::ALD + 8 * h;
          const float4 y0 = *reinterpret_cast<const float4*>(pb);
          const float4 y1 = *reinterpret_cast<const float4*>(pb + 4);
          bv[a][0] = y0.x; bv[a][1] = y0.y; bv[a][2] = y0.z; bv[a][3] = y0.w;
          bv[a][4] = y1.x; bv[a][5] = y1.y; bv[a][6] = y1.z; bv[a][7] = y1.w;
        }
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = mfma32x32x2(av[a][s], bv[b][s], acc[a][b]);
        if (ch + 1 < nch) sstore((ch + 1) & 1);
        __syncthreads();
      }
      // scores to LDS: D[i][j] with i = query row, j = db column
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int col = 64 * wc + 32 * b + lane % 32;
          const int64_t gj = j0 + col;
          const float nj = gj < n ? norms[gj] : 0.0f;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = 64 * wr + 32 * a + 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
            const int64_t gi = q0 + row;
            float sc = fmaf(-2.0f, acc[a][b][r], nj);
            if (gj >= n || (!include_self && gj == gi)) sc = INFINITY;
            Ss[row * SLD + col] = sc;
          }
        }
    } else {
      const uint16_t* xs = reinterpret_cast<const uint16_t*>(xsrc);
      uint16_t* As = reinterpret_cast<uint16_t*>(smem);
      // 4 waves as 2 x 2, each 64 x 64 = 4 x 4 blocks of 16 x 16
      floatx4 acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
      // staging: 256 rows x 64 bf16 = 256 x 8 chunks of 16 B = 2048; 8 per thread
      uint4 pre[8];
      auto gload = [&](int ch) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int f = tid + u * KNT;
          const int row = f / 8;
          const int c8 = f % 8;
          const bool isq = row < 128;
          const int64_t g = isq ? q0 + row : j0 + (row - 128);
          uint4 v = make_uint4(0u, 0u, 0u, 0u);
          if (g < n) v = *reinterpret_cast<const uint4*>(xs + g * mp + (int64_t)ch * G::BK + 8 * c8);
          pre[u] = v;
        }
      };
      auto sstore = [&](int buf) {
        uint16_t* base = As + (size_t)buf * (KBQ + KBN) * G::ALD;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int f = tid + u * KNT;
          const int row = f / 8;
          const int c8 = f % 8;
          *reinterpret_cast<uint4*>(base + row * G::ALD + 8 * c8) = pre[u];
        }
      };
      gload(0);
      sstore(0);
      __syncthreads();
      for (int ch = 0; ch < nch; ++ch) {
        if (ch + 1 < nch) gload(ch + 1);
        const uint16_t* base = As + (size_t)(ch & 1) * (KBQ + KBN) * G::ALD;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {           // two 32-wide k steps per stage
          shortx8 av[4], bv[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            const uint16_t* pa = base + (64 * wr + 16 * a + lane % 16) * G::ALD + 32 * kk + 8 * (lane / 16);
            av[a] = *reinterpret_cast<const shortx8*>(pa);
            const uint16_t* pb = base + (KBQ + 64 * wc + 16 * a + lane % 16) * G::ALD + 32 * kk + 8 * (lane / 16);
            bv[a] = *reinterpret_cast<const shortx8*>(pb);
          }
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = mfma16x16x32bf16(av[a], bv[b], acc[a][b]);
        }
        if (ch + 1 < nch) sstore((ch + 1) & 1);
        __syncthreads();
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int col = 64 * wc + 16 * b + lane % 16;
          const int64_t gj = j0 + col;
          const float nj = gj < n ? norms[gj] : 0.0f;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 64 * wr + 16 * a + 4 * (lane / 16) + r;
            const int64_t gi = q0 + row;
            float sc = fmaf(-2.0f, acc[a][b][r], nj);
            if (gj >= n || (!include_self && gj == gi)) sc = INFINITY;
            Ss[row * SLD + col] = sc;
          }
        }
    }
    __syncthreads();
    // top-K' update: wave w owns query rows 32w .. 32w+31
#pragma unroll
    for (int rr = 0; rr < 32; ++rr) {
      const int row = 32 * w + rr;
      const float v0 = Ss[row * SLD + lane];
      const float v1 = Ss[row * SLD + 64 + lane];
      row_update(ls[rr], lj[rr], v0, v1, j0, kc, kmask);
    }
    __syncthreads();
  }
  // write this split's lists
#pragma unroll
  for (int rr = 0; rr < 32; ++rr) {
    const int64_t gi = q0 + 32 * w + rr;
    if (gi < n && lane < kc) {
      const int64_t o = ((int64_t)split * n + gi) * kc + lane;
      cand_s[o] = ls[rr];
      cand_j[o] = lj[rr];
    }
  }
}

// ------------------------------------------------------------------------------------
// merge + float32 re-rank + certificate.  One wave per query, 4 queries per block.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void knn_rerank_kernel(
    const float* __restrict__ X, int64_t n, int64_t m, int64_t ldx, int k, int kc, int splits,
    const float* __restrict__ cand_s, const int* __restrict__ cand_j, const float* __restrict__ norms,
    const float* __restrict__ radius, const float* __restrict__ stats, int precision,
    int include_self, int32_t* __restrict__ idx_out, float* __restrict__ d2_out,
    uint8_t* __restrict__ kflags) {
  __shared__ float sh_s[4][4 * KCMAX];
  __shared__ int sh_j[4][4 * KCMAX];
  __shared__ float sel_s[4][KCMAX];
  __shared__ int sel_j[4][KCMAX];
  const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int64_t qraw = (int64_t)blockIdx.x * 4 + wv;
  const bool valid = qraw < n;
  const int64_t qi = valid ? qraw : n - 1;   // tail waves mirror the last query, write nothing
  const int tot = splits * kc;
  // gather the split lists
  for (int t = lane; t < tot; t += WAVE) {
    const int sp = t / kc, r = t % kc;
    const int64_t o = ((int64_t)sp * n + qi) * kc + r;
    sh_s[wv][t] = cand_s[o];
    sh_j[wv][t] = cand_j[o];
  }
  __syncthreads();
  // rank every gathered candidate by (score, index, slot); keep rank < kc
  for (int t = lane; t < tot; t += WAVE) {
    const float s = sh_s[wv][t];
    const int j = sh_j[wv][t];
    int rk = 0;
    for (int u = 0; u < tot; ++u) {
      const float su = sh_s[wv][u];
      const int ju = sh_j[wv][u];
      rk += (su < s) || (su == s && (ju < j || (ju == j && u < t)));
    }
    if (rk < kc) {
      sel_s[wv][rk] = s;
      sel_j[wv][rk] = j;
    }
  }
  __syncthreads();
  const float s_last = sel_s[wv][kc - 1];   // worst kept GEMM score
  // exact float32 difference-form distances of the kc candidates
  float myd = INFINITY;
  int myj = INT_MAX;
  const float* xq = X + qi * ldx;
  for (int r = 0; r < kc; ++r) {
    const int j = sel_j[wv][r];
    float d = INFINITY;
    if (j >= 0 && (int64_t)j < n) {
      const float* xj = X + (int64_t)j * ldx;
      float acc = 0.0f;
      for (int64_t c = lane; c < m; c += WAVE) {
        const float df = xq[c] - xj[c];
        acc = fmaf(df, df, acc);
      }
      d = wave_sum(acc);
    }
    if (lane == r) {
      myd = d;
      myj = (j >= 0 && (int64_t)j < n) ? j : INT_MAX;
    }
  }
  // the point itself (MC_INCLUDE_SELF) always comes first
  float key = myd;
  if (include_self && myj == (int)qi) key = -1.0f;
  // rank by (distance, index)
  int rk = 0;
  for (int u = 0; u < kc; ++u) {
    const float ku = __shfl(key, u, WAVE);
    const int ju = __shfl(myj, u, WAVE);
    rk += (ku < key) || (ku == key && ju < myj);
  }
  if (valid && lane < kc && rk < k) {
    idx_out[qi * k + rk] = myj;
    if (d2_out) d2_out[qi * k + rk] = myd;
  }
  // k-th and (k+1)-th distances
  float dk = 0.0f, dk1 = INFINITY;
  {
    const uint64_t bk = __ballot(lane < kc && rk == k - 1);
    const uint64_t bk1 = __ballot(lane < kc && rk == k);
    if (bk) dk = rdlane(myd, __ffsll((unsigned long long)bk) - 1);
    if (bk1) dk1 = rdlane(myd, __ffsll((unsigned long long)bk1) - 1);
  }
  if (valid && lane == 0 && kflags) {
    uint8_t fl = 0;
    const double u = 0x1p-24;
    const double gam = (double)(m + 2) * u / (1.0 - (double)(m + 2) * u);
    if (kc > k && isfinite(dk1) && (double)dk1 - (double)dk <= 2.0 * gam * (double)dk1)
      fl |= PF_KNN_AMBIGUOUS;
    // certificate: every non-candidate y has GEMM score >= s_last; bound its true distance
    // from below and compare with the k-th re-ranked distance.
    bool cert = true;
    if (tot < n - (include_self ? 0 : 1) && isfinite(s_last)) {
      const double ni = (double)norms[qi], rn = sqrt(ni);
      const double nmax = (double)stats[0], emax = (double)stats[1], ei = (double)radius[qi];
      const double gm = (double)(m + 8) * u / (1.0 - (double)(m + 8) * u);
      // |gemm d2 - ||xc_i - xc_j||^2| <= E (dot rounding of the low-precision copy + fp32 sums)
      double E = 2.0 * (ei * (nmax + emax) + rn * emax) + 2.0 * gm * (rn + ei) * (nmax + emax) +
                 4.0 * u * (ni + nmax * nmax) + gm * (ni + nmax * nmax);
      (void)precision;
      const double lo2 = ni + (double)s_last - E;
      // centring rounding: | ||xc_i - xc_j|| - ||x_i - x_j|| | <= u (||xc_i|| + ||xc_j||) (1+u)
      const double lo = (lo2 > 0.0 ? sqrt(lo2) : 0.0) - 1.0001 * u * (rn + nmax);
      const double dk_hi = (double)dk / (1.0 - gam);
      cert = lo > 0.0 && lo * lo > dk_hi;
    }
    if (!cert) fl |= PF_KNN_UNCERTIFIED;
    kflags[qi] = fl;
  }
}

// ------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------
static int64_t knn_mp(int64_t m, int precision) {
  const int64_t bk = precision == 0 ? GemmCfg<0>::BK : GemmCfg<1>::BK;
  return ((m + bk - 1) / bk) * bk;
}

static int knn_splits(int64_t n, int kc) {
  const int64_t qt = (n + KBQ - 1) / KBQ;
  const int64_t nt = (n + KBN - 1) / KBN;
  int64_t s = (1024 + qt - 1) / qt;   // aim for >= 1024 workgroups (4 per CU)
  if (s > 16) s = 16;
  if (s > (4 * KCMAX) / kc) s = (4 * KCMAX) / kc;   // merged lists must fit the re-rank LDS
  if (s > nt) s = nt;
  if (s < 1) s = 1;
  return (int)s;
}

KnnPlan knn_plan(int64_t n, int64_t m, int k, int kc, int precision) {
  KnnPlan p{};
  p.n = n;
  p.m = m;
  p.k = k;
  p.kc = kc;
  p.precision = precision;
  p.splits = knn_splits(n, kc);
  const int64_t mp = knn_mp(m, precision);
  const int64_t parts = 64;
  size_t off = 0;
  p.off_xc = off;     off += align256((size_t)n * mp * 4);
  p.off_norm = off;   off += align256((size_t)n * 4);
  p.off_colsum = off; off += align256((size_t)parts * m * 8 + (size_t)m * 4);
  p.off_stats = off;  off += align256((size_t)n * 4 + 64);
  p.off_cand_s = off; off += align256((size_t)p.splits * n * kc * 4);
  p.off_cand_j = off; off += align256((size_t)p.splits * n * kc * 4);
  p.off_xlow = off;   off += precision == 1 ? align256((size_t)n * mp * 2) : 0;
  p.off_scale = off;
  p.total = off;
  return p;
}

hipError_t launch_knn(const float* X, int64_t n, int64_t m, int64_t ldx, int k, int kc,
                      int precision, bool include_self, int32_t* idx, float* d2, uint8_t* kflags,
                      void* ws, const KnnPlan& plan, hipStream_t stream) {
  unsigned char* base = reinterpret_cast<unsigned char*>(ws);
  const int64_t mp = knn_mp(m, precision);
  float* xc = reinterpret_cast<float*>(base + plan.off_xc);
  float* norms = reinterpret_cast<float*>(base + plan.off_norm);
  double* part = reinterpret_cast<double*>(base + plan.off_colsum);
  float* mu = reinterpret_cast<float*>(base + plan.off_colsum + (size_t)64 * m * 8);
  float* radius = reinterpret_cast<float*>(base + plan.off_stats);
  float* stats = radius + n;
  float* cand_s = reinterpret_cast<float*>(base + plan.off_cand_s);
  int* cand_j = reinterpret_cast<int*>(base + plan.off_cand_j);
  uint16_t* xb = reinterpret_cast<uint16_t*>(base + plan.off_xlow);

  const int64_t parts = 64;
  const int64_t rows_per = (n + parts - 1) / parts;
  const unsigned gx = (unsigned)((m + 255) / 256);
  timing_begin(0, stream);
  hipLaunchKernelGGL(knn_colsum_kernel, dim3(gx, (unsigned)parts), dim3(256), 0, stream, X, n, m,
                     ldx, rows_per, part);
  timing_end(0, stream);
  timing_begin(1, stream);
  hipLaunchKernelGGL(knn_mean_kernel, dim3(gx), dim3(256), 0, stream, part, m, (int)parts, n, mu);
  timing_end(1, stream);
  timing_begin(2, stream);
  hipLaunchKernelGGL(knn_center_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream, X, n,
                     m, ldx, mp, mu, xc, xb, norms, radius, precision);
  timing_end(2, stream);
  timing_begin(3, stream);
  hipLaunchKernelGGL(knn_stats_kernel, dim3(1), dim3(256), 0, stream, norms, radius, n, stats);
  timing_end(3, stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;

  const int64_t nt = (n + KBN - 1) / KBN;
  const int splits = plan.splits;
  const int tps = (int)((nt + splits - 1) / splits);
  const dim3 grid((unsigned)((n + KBQ - 1) / KBQ), (unsigned)splits);
  static bool attr_set = false;   // LDS beyond 64 KiB needs the opt-in attribute
  if (!attr_set) {
    hipFuncSetAttribute(reinterpret_cast<const void*>(&knn_gemm_topk_kernel<0>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm_lds_bytes<0>());
    hipFuncSetAttribute(reinterpret_cast<const void*>(&knn_gemm_topk_kernel<1>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm_lds_bytes<1>());
    (void)hipGetLastError();
    attr_set = true;
  }
  timing_begin(4, stream);
  if (precision == 0) {
    hipLaunchKernelGGL(knn_gemm_topk_kernel<0>, grid, dim3(KNT), gemm_lds_bytes<0>(), stream,
                       (const void*)xc, mp, norms, n, kc, tps, include_self ? 1 : 0, cand_s, cand_j);
  } else {
    hipLaunchKernelGGL(knn_gemm_topk_kernel<1>, grid, dim3(KNT), gemm_lds_bytes<1>(), stream,
                       (const void*)xb, mp, norms, n, kc, tps, include_self ? 1 : 0, cand_s, cand_j);
  }
  timing_end(4, stream);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  timing_begin(5, stream);
  hipLaunchKernelGGL(knn_rerank_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream, X, n, m,
                     ldx, k, kc, splits, cand_s, cand_j, norms, radius, stats, precision,
                     include_self ? 1 : 0, idx, d2, kflags);
  timing_end(5, stream);
  return hipGetLastError();
}

}  // namespace mc
