// Brute-force k nearest neighbours on gfx950 (Step 1 of the method, eq. knn;
// the kNN-Graph step of Algorithm 1).
//
// Pipeline (all on one stream, workspace owned by the caller):
//  1. knn_colsum / knn_center: subtract the column mean (distances are
//     translation invariant; centring shrinks ||x||^2 and with it the
//     cancellation in ||x||^2 + ||y||^2 - 2 x.y) and write the centred copy in
//     the GEMM's input format (float32, bf16, or fp8 e4m3 with per-row scales)
//     with a zero-padded row stride, float32 norms, and a per-row rounding
//     radius of the low-precision copy for the candidate certificate.
//  2. knn_gemm_topk: query tile x database tile scores s = ||y||^2 - 2 x.y on
//     MFMA (fp32 32x32x2, bf16 16x16x32 or fp8 16x16x32), written to LDS; each
//     wave keeps a sorted 64-entry list of (score, index) per query row across
//     its lanes, filters every row against its K'-th entry (and the smallest one
//     any workgroup has published for that query) with a ballot and takes in
//     survivors by a DPP shift (few) or a bitonic sort and merge (many).  The
//     list of tile pairs is cut into equal contiguous ranges, one per workgroup.
//     The distance matrix is symmetric: under the symmetric schedule each
//     unordered tile pair is scored once and its transposed scores go to the
//     workspace for the other tile's queries.
//  3. knn_rowcap / knn_column_topk (symmetric schedule): bound each query's final
//     K'-th key by its merged row-side lists, then stream the transposed tiles
//     through the same list code (the column side).
//  4. knn_rerank: merge all list segments, recompute the K' distances in float32
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
constexpr int KNT = 512;   // threads per GEMM workgroup (8 waves)
constexpr int RPW = KBQ / (KNT / 64);   // query rows owned by one wave in the top-k stage
constexpr int SLD = KBN + 4;  // score-tile row stride (floats)
constexpr int KCMAX = 64;  // largest candidate list
constexpr int KPARTS = 256; // row blocks of the column-mean reduction
constexpr int RESCAN_CMAX = 256;   // candidates the rescan collects per uncertified query

// Per-query state of the rescan of uncertified queries (workspace arrays).
struct RescanWs {
  float* act_thr;        // score threshold of the quick test (-inf: query not rescanned)
  float* act_T;          // distance threshold T of the exact test
  float* act_a;          // lower-bound offset a (sqrt(s + a) bounds the copies' distance)
  int* cnt;              // collected candidates
  int* cbuf;             // n x RESCAN_CMAX candidate indices
  float* p1d;            // n x KCMAX exact distances of the first pass's candidates
  int* p1j;              // n x KCMAX their indices
  uint32_t* tile_active; // per 128-point tile: some query of the tile is rescanned
};

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

// Column means from the partial sums: a block takes 16 columns, its 256 threads take 16
// partial sums each (16 groups), then the groups are added in a fixed order (deterministic).
__global__ __launch_bounds__(256) void knn_mean_kernel(const double* __restrict__ part, int64_t m,
                                                       int nparts, int64_t n, float* __restrict__ mu,
                                                       uint32_t* __restrict__ stats) {
  __shared__ double red[16][17];
  if (blockIdx.x == 0 && threadIdx.x < 2) stats[threadIdx.x] = 0u;   // for knn_stats' atomic maxima
  const int cl = threadIdx.x % 16, grp = threadIdx.x / 16;
  const int64_t c = (int64_t)blockIdx.x * 16 + cl;
  double s = 0.0;
  if (c < m) {
    for (int p = grp; p < nparts; p += 16) s += part[(int64_t)p * m + c];
  }
  red[grp][cl] = s;
  __syncthreads();
  if (grp == 0 && c < m) {
    double t = 0.0;
#pragma unroll
    for (int g = 0; g < 16; ++g) t += red[g][cl];
    mu[c] = (float)(t / (double)n);
  }
}

// One wave per row: the centred row xc = fl(x - mu) in the GEMM's input format (float32,
// bf16, or fp8 e4m3 with the per-row scale s = max|xc| / 448), zero padded to the row
// stride mp; the norm of that copy, ||lowp(xc)||^2 (float32, from a float64 sum); and the
// rounding radius ||lowp(xc) - xc|| of the low-precision copy (0 on the float32 path).
__global__ __launch_bounds__(256) void knn_center_kernel(
    const float* __restrict__ X, int64_t n, int64_t m, int64_t ldx, int64_t mp,
    const float* __restrict__ mu, void* __restrict__ xout, float* __restrict__ scales,
    float* __restrict__ norms, float* __restrict__ radius, int precision, uint32_t* __restrict__ thr,
    uint32_t* __restrict__ tile_active) {
  const int64_t r = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
  const int lane = threadIdx.x % WAVE;
  if (r >= n) return;
  double s = 0.0, e = 0.0, sh = 0.0;
  float amax = 0.0f;
  for (int64_t c = lane; c < m; c += WAVE) {
    const float v = X[r * ldx + c] - mu[c];
    s = fma((double)v, (double)v, s);
    amax = fmaxf(amax, fabsf(v));
  }
  amax = wave_max(amax);
  const float sc = amax > 0.0f ? amax / 448.0f : 1.0f;
  const float isc = 1.0f / sc;
  for (int64_t c = lane; c < mp; c += WAVE) {
    const float v = c < m ? X[r * ldx + c] - mu[c] : 0.0f;
    if (precision == 0) {
      reinterpret_cast<float*>(xout)[r * mp + c] = v;
    } else if (precision == 1) {
      const uint16_t h = f2bf(v);
      reinterpret_cast<uint16_t*>(xout)[r * mp + c] = h;
      const double vh = (double)bf2f(h);
      const double d = vh - (double)v;
      e = fma(d, d, e);
      sh = fma(vh, vh, sh);
    } else {
      const int pk = __builtin_amdgcn_cvt_pk_fp8_f32(v * isc, 0.0f, 0, false);
      reinterpret_cast<uint8_t*>(xout)[r * mp + c] = (uint8_t)(pk & 0xff);
      const double vh = (double)sc * (double)__builtin_amdgcn_cvt_f32_fp8(pk, 0);
      const double d = vh - (double)v;
      e = fma(d, d, e);
      sh = fma(vh, vh, sh);
    }
  }
  s = wave_sum(s);
  e = wave_sum(e);
  sh = wave_sum(sh);
  if (lane == 0) {
    // the GEMM scores use the norm of the copy it multiplies, so that score + norm_i is the
    // squared distance of the two copies up to float32 rounding
    norms[r] = (float)(precision == 0 ? s : sh);
    if (r % KBQ == 0) tile_active[r / KBQ] = 0u;
    radius[r] = (float)(sqrt(e) * (1.0 + 0x1p-20));   // rounded up: it bounds an error
    if (scales) scales[r] = sc;
    thr[r] = 0xFFFFFFFFu;   // no K'-th key published yet
  }
}

// stats[0] = max_i sqrt(norm_i), stats[1] = max_i radius_i: every workgroup reduces a strided
// share of the rows, then one atomic maximum per value (both are non-negative, so their
// float32 bit patterns order like the values; knn_mean zeroes them first)
__global__ __launch_bounds__(256) void knn_stats_kernel(const float* __restrict__ norms,
                                                        const float* __restrict__ radius, int64_t n,
                                                        uint32_t* __restrict__ stats) {
  __shared__ float red[2][4];
  float a = 0.0f, b = 0.0f;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256) {
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
    atomicMax(stats, __float_as_uint(fmaxf(fmaxf(red[0][0], red[0][1]), fmaxf(red[0][2], red[0][3]))));
    atomicMax(stats + 1, __float_as_uint(fmaxf(fmaxf(red[1][0], red[1][1]), fmaxf(red[1][2], red[1][3]))));
  }
}

// ------------------------------------------------------------------------------------
// wave-level sorted list: lane r holds the r-th smallest key of a row, r = 0..63, and the
// row's threshold is the entry of lane kc-1.  A key is the 64-bit integer
// (ord(score) << 32) | index, with ord the order-preserving map of float32 onto uint32,
// so one unsigned compare orders by (score, index) without branches.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ float rdlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ uint32_t rdlane_u(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// a < b as float32  <=>  f2ord(a) < f2ord(b) as uint32 (NaN-free inputs; +inf maps highest)
__device__ __forceinline__ uint32_t f2ord(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float ord2f(uint32_t o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

__device__ __forceinline__ uint64_t mkkey(uint32_t hi, uint32_t lo) {
  return ((uint64_t)hi << 32) | (uint64_t)lo;
}

constexpr uint32_t KEY_PAD_HI = 0xFF800000u;   // ord(+inf)
constexpr uint32_t KEY_PAD_LO = 0x7FFFFFFFu;   // INT_MAX index

// Value of lane (lane ^ JJ): DPP quad permutes for 1 and 2, DPP row rotate for 8,
// ds_swizzle (no memory access) for 4 and 16, ds_bpermute for 32.
template <int JJ>
__device__ __forceinline__ uint32_t xshfl(uint32_t v) {
  if constexpr (JJ == 1) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  } else if constexpr (JJ == 2) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  } else if constexpr (JJ == 4) {
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x101F);              // xor 4 in 32 lanes
  } else if constexpr (JJ == 8) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);  // row_ror:8
  } else if constexpr (JJ == 16) {
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F);              // xor 16 in 32 lanes
  } else {
    static_assert(JJ == 32, "lane distance");
    return (uint32_t)__builtin_amdgcn_ds_bpermute((lane_id() ^ 32) << 2, (int)v);
  }
}

// Insert one key that beats the threshold: lanes at or after its rank shift up by one.
__device__ __forceinline__ void list_insert(uint32_t& hi, uint32_t& lo, uint32_t nhi, uint32_t nlo) {
  const int lane = lane_id();
  const int pos = __popcll(__ballot(mkkey(hi, lo) < mkkey(nhi, nlo)));
  const uint32_t uh = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi, 0x138, 0xf, 0xf, false);   // wave_shr:1
  const uint32_t ul = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo, 0x138, 0xf, 0xf, false);
  hi = lane > pos ? uh : (lane == pos ? nhi : hi);
  lo = lane > pos ? ul : (lane == pos ? nlo : lo);
}

// Compare-exchange with lane ^ JJ: the lower lane keeps the smaller key when `asc`, the
// larger otherwise (keys are distinct, so one unsigned compare decides both lanes).
template <int JJ>
__device__ __forceinline__ void cmpx(uint32_t& hi, uint32_t& lo, bool asc) {
  const uint32_t oh = xshfl<JJ>(hi), ol = xshfl<JJ>(lo);
  const bool lower = (lane_id() & JJ) == 0;
  const bool take = (mkkey(oh, ol) < mkkey(hi, lo)) != (lower != asc);
  hi = take ? oh : hi;
  lo = take ? ol : lo;
}

// Bitonic sort of one key per lane, ascending (ASC) or descending.
template <bool ASC>
__device__ __forceinline__ void wave_sort64(uint32_t& hi, uint32_t& lo) {
  const int lane = lane_id();
#define MC_STAGE(KK, JJ) cmpx<JJ>(hi, lo, ((lane & (KK)) == 0) == ASC)
  MC_STAGE(2, 1);
  MC_STAGE(4, 2); MC_STAGE(4, 1);
  MC_STAGE(8, 4); MC_STAGE(8, 2); MC_STAGE(8, 1);
  MC_STAGE(16, 8); MC_STAGE(16, 4); MC_STAGE(16, 2); MC_STAGE(16, 1);
  MC_STAGE(32, 16); MC_STAGE(32, 8); MC_STAGE(32, 4); MC_STAGE(32, 2); MC_STAGE(32, 1);
  MC_STAGE(64, 32); MC_STAGE(64, 16); MC_STAGE(64, 8); MC_STAGE(64, 4); MC_STAGE(64, 2); MC_STAGE(64, 1);
#undef MC_STAGE
}

// The 64 smallest of an ascending list and a DESCENDING b, ascending, into (hi, lo):
// the lane-wise minimum of the two is bitonic, and six stages sort it.
__device__ __forceinline__ void wave_merge64(uint32_t& hi, uint32_t& lo, uint32_t bh, uint32_t bl) {
  const bool take = mkkey(bh, bl) < mkkey(hi, lo);
  hi = take ? bh : hi;
  lo = take ? bl : lo;
  cmpx<32>(hi, lo, true);
  cmpx<16>(hi, lo, true);
  cmpx<8>(hi, lo, true);
  cmpx<4>(hi, lo, true);
  cmpx<2>(hi, lo, true);
  cmpx<1>(hi, lo, true);
}

constexpr int INSERT_MAX = 12;   // up to this many survivors go in one by one; more: sort + merge

__device__ __forceinline__ uint32_t umin32(uint32_t a, uint32_t b) { return a < b ? a : b; }

// Filter 64 candidate keys (one per lane) against the row list (and below `cap`) and take
// in what passes.
__device__ __forceinline__ void half_update(uint32_t& hi, uint32_t& lo, uint32_t vh, uint32_t vl, int kc,
                                            uint32_t cap) {
  uint32_t th = umin32(rdlane_u(hi, kc - 1), cap);
  uint64_t msk = __ballot(vh < th);
  if (!msk) return;
  if (__popcll(msk) <= INSERT_MAX) {
    while (msk) {
      const int src = __ffsll((unsigned long long)msk) - 1;
      msk &= msk - 1;
      const uint32_t sh = rdlane_u(vh, src);
      if (sh < th) {
        list_insert(hi, lo, sh, rdlane_u(vl, src));
        th = umin32(rdlane_u(hi, kc - 1), cap);
      }
    }
  } else {
    uint32_t bh = vh < th ? vh : 0xFFFFFFFFu;
    uint32_t bl = vh < th ? vl : 0xFFFFFFFFu;
    wave_sort64<false>(bh, bl);
    wave_merge64(hi, lo, bh, bl);
  }
}

// Take in the survivors of a row's 128 candidates (two 64-lane halves): keys below both the
// list's K'-th key and `cap`.  Few survivors go in one by one; up to 64 are packed into one
// vector (forward permute), sorted and merged once; more than 64 (early tiles) fall back to
// one sort + merge per half.
__device__ __forceinline__ void row_update(uint32_t& hi, uint32_t& lo, uint32_t vh0, uint32_t vl0,
                                           uint32_t vh1, uint32_t vl1, int kc, uint32_t cap) {
  uint32_t th = umin32(rdlane_u(hi, kc - 1), cap);
  const uint64_t m0 = __ballot(vh0 < th), m1 = __ballot(vh1 < th);
  const int c0 = __popcll(m0), c = c0 + __popcll(m1);
  if (c == 0) return;
  if (c <= INSERT_MAX) {
#pragma nounroll
    for (int h = 0; h < 2; ++h) {
      uint64_t msk = h == 0 ? m0 : m1;
      const uint32_t vh = h == 0 ? vh0 : vh1, vl = h == 0 ? vl0 : vl1;
      while (msk) {
        const int src = __ffsll((unsigned long long)msk) - 1;
        msk &= msk - 1;
        const uint32_t sh = rdlane_u(vh, src);
        if (sh < th) {
          list_insert(hi, lo, sh, rdlane_u(vl, src));
          th = umin32(rdlane_u(hi, kc - 1), cap);
        }
      }
    }
  } else if (c <= WAVE) {
    const int lane = lane_id();
    const uint64_t below = (1ull << lane) - 1ull;
    const bool s0 = (m0 >> lane) & 1ull, s1 = (m1 >> lane) & 1ull;
    // survivor ranks: half 0 fills lanes [0, c0), half 1 fills [c0, c); others go to a lane
    // whose received value is ignored
    const int d0 = s0 ? __popcll(m0 & below) : WAVE - 1;
    const int d1 = s1 ? c0 + __popcll(m1 & below) : (c0 > 0 ? 0 : WAVE - 1);
    const uint32_t p0h = (uint32_t)__builtin_amdgcn_ds_permute(d0 << 2, (int)vh0);
    const uint32_t p0l = (uint32_t)__builtin_amdgcn_ds_permute(d0 << 2, (int)vl0);
    const uint32_t p1h = (uint32_t)__builtin_amdgcn_ds_permute(d1 << 2, (int)vh1);
    const uint32_t p1l = (uint32_t)__builtin_amdgcn_ds_permute(d1 << 2, (int)vl1);
    uint32_t bh = lane < c0 ? p0h : (lane < c ? p1h : 0xFFFFFFFFu);
    uint32_t bl = lane < c0 ? p0l : (lane < c ? p1l : 0xFFFFFFFFu);
    wave_sort64<false>(bh, bl);
    wave_merge64(hi, lo, bh, bl);
  } else {
    half_update(hi, lo, vh0, vl0, kc, cap);
    half_update(hi, lo, vh1, vl1, kc, cap);
  }
}

// ------------------------------------------------------------------------------------
// GEMM + top-K'.  PREC 0: fp32 MFMA 32x32x2, BK = 16; PREC 1: bf16 MFMA 16x16x32, BK = 64;
// PREC 2: fp8 e4m3 MFMA 16x16x128 with per-row scales, BK = 128.
//
// Work is a list of (query tile, database tile) pairs in query-major order (the tile-pair
// schedules below).  Workgroup L takes the contiguous range [L*P/G, (L+1)*P/G): every
// workgroup does the same amount of MFMA work, a query tile is cut into at most a few
// segments (each refills its lists once), and because G >= the tile count a range touches
// at most two query tiles.  Workgroups are dispatched round-robin over the 8 XCDs, so the
// logical id is remapped to give each XCD a block of consecutive ranges: its workgroups
// then share query tiles in their own L2.
// ------------------------------------------------------------------------------------
template <int PREC>
struct GemmCfg;
template <>
struct GemmCfg<0> {
  static constexpr int ESZ = 4;                 // bytes per element
  static constexpr int BK = 16;                 // columns per stage
  static constexpr int ALD = BK + 4;            // staging row stride (elements)
};
template <>
struct GemmCfg<1> {
  static constexpr int ESZ = 2;
  static constexpr int BK = 64;
  static constexpr int ALD = BK + 8;
};
template <>
struct GemmCfg<2> {
  static constexpr int ESZ = 1;
  static constexpr int BK = 128;                // fp8 bytes per row per stage
  static constexpr int ALD = BK + 16;
};

// One stage of the staged operands: 256 rows (queries, then database points) of BK
// elements, moved as 16-byte chunks, NPRE per thread.
template <int PREC>
struct Stage {
  using G = GemmCfg<PREC>;
  static constexpr int CPR = G::BK * G::ESZ / 16;                  // chunks per row
  static constexpr int NPRE = (KBQ + KBN) * CPR / KNT;
  static constexpr size_t BUF_B = (size_t)(KBQ + KBN) * G::ALD * G::ESZ;
  static constexpr size_t STAGE_B = 2 * BUF_B;                     // double buffered
};

// Global -> registers: stage `ch` of query tile q0 and database tile j0 (rows past n are 0).
template <int PREC>
__device__ __forceinline__ void stage_load(uint4 (&pre)[Stage<PREC>::NPRE], const void* __restrict__ xsrc,
                                           int64_t mp, int64_t n, int64_t q0, int64_t j0, int ch) {
  using S = Stage<PREC>;
  using G = GemmCfg<PREC>;
  const unsigned char* xs = reinterpret_cast<const unsigned char*>(xsrc);
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < S::NPRE; ++u) {
    const int f = tid + u * KNT;
    const int row = f / S::CPR, c = f % S::CPR;
    const int64_t g = row < KBQ ? q0 + row : j0 + (row - KBQ);
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (g < n)
      v = *reinterpret_cast<const uint4*>(xs + (g * mp + (int64_t)ch * G::BK) * G::ESZ + 16 * c);
    pre[u] = v;
  }
}

// Registers -> LDS staging buffer `buf`.
template <int PREC>
__device__ __forceinline__ void stage_store(const uint4 (&pre)[Stage<PREC>::NPRE], unsigned char* smem, int buf) {
  using S = Stage<PREC>;
  using G = GemmCfg<PREC>;
  unsigned char* base = smem + (size_t)buf * S::BUF_B;
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < S::NPRE; ++u) {
    const int f = tid + u * KNT;
    *reinterpret_cast<uint4*>(base + (f / S::CPR) * (G::ALD * G::ESZ) + 16 * (f % S::CPR)) = pre[u];
  }
}

// Branch-free stage_load for the prefetches (the next stage inside a tile, stage 0 of the next
// pair behind the top-K' work): rows past n read row n - 1 (in bounds) instead of zeros, so no
// load sits behind a branch and every wait on the loads issued before it counts exactly the
// memory operations issued after them.  An output of the tile depends only on its own row and
// column, and those rows only reach query rows whose lists are never written or published
// and database columns the score epilogue sets to +inf, whose transposed scores add the +inf
// norm of a row past n.
template <int PREC>
__device__ __forceinline__ void stage_load_clamped(uint4 (&pre)[Stage<PREC>::NPRE], const void* __restrict__ xsrc,
                                                   int64_t mp, int64_t n, int64_t q0, int64_t j0, int ch = 0) {
  using S = Stage<PREC>;
  using G = GemmCfg<PREC>;
  const unsigned char* xs = reinterpret_cast<const unsigned char*>(xsrc);
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < S::NPRE; ++u) {
    const int f = tid + u * KNT;
    const int row = f / S::CPR, c = f % S::CPR;
    int64_t g = row < KBQ ? q0 + row : j0 + (row - KBQ);
    g = g < n ? g : n - 1;
    pre[u] = *reinterpret_cast<const uint4*>(xs + (g * mp + (int64_t)ch * G::BK) * G::ESZ + 16 * c);
  }
}

template <int PREC>
constexpr size_t gemm_lds_bytes() {
  return Stage<PREC>::STAGE_B > (size_t)KBQ * SLD * 4 ? Stage<PREC>::STAGE_B
                                                       : (size_t)KBQ * SLD * 4;
}

// Workgroup holding tile pair t under the range schedule (floor((t+1)G - 1)/P).
__host__ __device__ __forceinline__ int64_t range_owner(int64_t t, int64_t G, int64_t P) {
  return ((t + 1) * G - 1) / P;
}

// Tile-pair schedules.  Pairs are numbered row tile by row tile: row tile i owns a_len(i)
// consecutive pairs from a_start(i), pair (i, d) scoring query tile i against database
// tile a_db(i, d).
//  * full (sym = 0): every row tile meets all T tiles, d = 0 .. T-1.
//  * symmetric (sym = 1): the score matrix is symmetric, so each unordered tile pair is
//    scored once.  Row tile i meets the tiles (i + d) mod T, d = 0 .. h (plus d = T/2 for
//    i < T/2 when T is even): the circulant half of the pairs, about T/2 per row tile.
//    The transposed tile of every off-diagonal pair serves the queries of its database
//    tile (the column side); column tile j receives the pairs ((j - d) mod T, j),
//    d = 1 .. b_len(j), numbered column tile by column tile from b_start(j).
struct TileSched {
  int64_t T;   // 128-point tiles
  int64_t h;   // off-diagonal pairs of every row tile in the symmetric schedule, (T - 1) / 2
  int64_t e;   // row tiles with one more (T even: T / 2, else 0)
  int sym;
};

__host__ __device__ __forceinline__ TileSched make_sched(int64_t n, int sym) {
  TileSched s;
  s.T = (n + KBQ - 1) / KBQ;
  s.h = (s.T - 1) / 2;
  s.e = (s.T % 2 == 0) ? s.T / 2 : 0;
  s.sym = sym;
  return s;
}
__host__ __device__ __forceinline__ int64_t a_len(const TileSched& s, int64_t i) {
  return s.sym ? s.h + 1 + (i < s.e ? 1 : 0) : s.T;
}
__host__ __device__ __forceinline__ int64_t a_start(const TileSched& s, int64_t i) {
  return s.sym ? i * (s.h + 1) + (i < s.e ? i : s.e) : i * s.T;
}
__host__ __device__ __forceinline__ int64_t a_pairs(const TileSched& s) {
  return s.sym ? s.T * (s.h + 1) + s.e : s.T * s.T;
}
__host__ __device__ __forceinline__ void a_pair(const TileSched& s, int64_t t, int64_t& i, int64_t& d) {
  if (!s.sym) {
    i = t / s.T;
    d = t % s.T;
    return;
  }
  const int64_t lead = s.e * (s.h + 2);   // the e row tiles of h + 2 pairs come first
  if (t < lead) {
    i = t / (s.h + 2);
    d = t % (s.h + 2);
  } else {
    const int64_t u = t - lead;
    i = s.e + u / (s.h + 1);
    d = u % (s.h + 1);
  }
}
__host__ __device__ __forceinline__ int64_t a_db(const TileSched& s, int64_t i, int64_t d) {
  return s.sym ? (i + d >= s.T ? i + d - s.T : i + d) : d;   // d < T
}
// the pair after (i, d) in schedule order
__host__ __device__ __forceinline__ void a_next(const TileSched& s, int64_t& i, int64_t& d) {
  if (++d == a_len(s, i)) {
    ++i;
    d = 0;
  }
}
__host__ __device__ __forceinline__ int64_t b_len(const TileSched& s, int64_t j) {
  return s.h + (j >= s.T - s.e ? 1 : 0);
}
__host__ __device__ __forceinline__ int64_t b_start(const TileSched& s, int64_t j) {
  return j * s.h + (j > s.T - s.e ? j - (s.T - s.e) : 0);
}
__host__ __device__ __forceinline__ int64_t b_pairs(const TileSched& s) { return s.T * s.h + s.e; }
__host__ __device__ __forceinline__ void b_pair(const TileSched& s, int64_t t, int64_t& j, int64_t& d) {
  const int64_t lead = (s.T - s.e) * s.h;   // column tiles with h pairs come first
  if (t < lead) {
    j = t / s.h;
    d = 1 + t % s.h;
  } else {
    const int64_t u = t - lead;
    j = (s.T - s.e) + u / (s.h + 1);
    d = 1 + u % (s.h + 1);
  }
}
// column-side number (and transposed-tile slot) of the off-diagonal pair (i, d), d >= 1
__host__ __device__ __forceinline__ int64_t b_index(const TileSched& s, int64_t i, int64_t d) {
  return b_start(s, a_db(s, i, d)) + d - 1;
}
// list segments of one row (column) tile: workgroups whose ranges meet [first, first + len)
__host__ __device__ __forceinline__ int64_t segments(int64_t first, int64_t len, int64_t G, int64_t P) {
  return len > 0 ? range_owner(first + len - 1, G, P) - range_owner(first, G, P) + 1 : 0;
}

// Cross terms D[i][j] = -2 x_i . y_j of one 128 x 128 tile into Ss (LDS); +inf past column n
// and, unless include_self, on the diagonal.  The score of y_j for query x_i is then
// ||y_j||^2 + D[i][j] and that of x_i for query y_j is ||x_i||^2 + D[i][j]; for the float32
// and bf16 copies each equals the fused fmaf(-2, dot, norm), as -2 dot is exact.
// 8 waves as 2 (query rows) x 4 (db columns); wave tile 64 x 32.  On entry `pre` holds
// stage 0 of this tile (the caller loads it early, behind the previous tile's top-K').
// 32 bytes of LDS at a 16-byte aligned address, as the eight dwords of an MFMA operand.
__device__ __forceinline__ intx8 lds_load32(const uint8_t* p) {
  const uint4 lo = *reinterpret_cast<const uint4*>(p);
  const uint4 hi = *reinterpret_cast<const uint4*>(p + 16);
  return intx8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
}

template <int PREC>
__device__ __forceinline__ void tile_scores(const void* __restrict__ xsrc, int64_t mp,
                                            const float* __restrict__ norms,
                                            const float* __restrict__ scales, int64_t n, int64_t q0,
                                            int64_t j0, int include_self, unsigned char* smem,
                                            uint4 (&pre)[Stage<PREC>::NPRE]) {
  using G = GemmCfg<PREC>;
  const int tid = threadIdx.x;
  const int w = tid / WAVE, lane = tid % WAVE;
  const int wr = w / 4, wc = w % 4;      // wave tile: rows 64*wr.., cols 32*wc..
  float* Ss = reinterpret_cast<float*>(smem);
  const int nch = (int)(mp / G::BK);
  if constexpr (PREC == 0) {
    float* As = reinterpret_cast<float*>(smem);
    floatx16 acc[2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][r] = 0.0f;
    stage_store<PREC>(pre, smem, 0);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
      stage_load_clamped<PREC>(pre, xsrc, mp, n, q0, j0, ch + 1 < nch ? ch + 1 : ch);
      const float* base = As + (size_t)(ch & 1) * (KBQ + KBN) * G::ALD;
      const int h = lane / 32;
      float av[2][8], bv[8];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const float* pa = base + (64 * wr + 32 * a + lane % 32) * G::ALD + 8 * h;
        const float4 x0 = *reinterpret_cast<const float4*>(pa);
        const float4 x1 = *reinterpret_cast<const float4*>(pa + 4);
        av[a][0] = x0.x; av[a][1] = x0.y; av[a][2] = x0.z; av[a][3] = x0.w;
        av[a][4] = x1.x; av[a][5] = x1.y; av[a][6] = x1.z; av[a][7] = x1.w;
      }
      {
        const float* pb = base + (KBQ + 32 * wc + lane % 32) * G::ALD + 8 * h;
        const float4 y0 = *reinterpret_cast<const float4*>(pb);
        const float4 y1 = *reinterpret_cast<const float4*>(pb + 4);
        bv[0] = y0.x; bv[1] = y0.y; bv[2] = y0.z; bv[3] = y0.w;
        bv[4] = y1.x; bv[5] = y1.y; bv[6] = y1.z; bv[7] = y1.w;
      }
      // k order inside a stage: lane half h supplies column 8h+s at step s, for A and B alike
#pragma unroll
      for (int st = 0; st < 8; ++st)
#pragma unroll
        for (int a = 0; a < 2; ++a) acc[a] = mfma32x32x2(av[a][st], bv[st], acc[a]);
      stage_store<PREC>(pre, smem, (ch + 1) & 1);
      __syncthreads();
    }
    const int col = 32 * wc + lane % 32;
    const int64_t gj = j0 + col;
    const bool colok = gj < n;
    const int dq = (int)(j0 - q0) + col;   // column index relative to the query tile (int32)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 64 * wr + 32 * a + 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
        float sc = -2.0f * acc[a][r];
        if (!colok || (!include_self && dq == row)) sc = INFINITY;
        Ss[row * SLD + col] = sc;
      }
  } else if constexpr (PREC == 1) {
    uint16_t* As = reinterpret_cast<uint16_t*>(smem);
    floatx4 acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    stage_store<PREC>(pre, smem, 0);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
      stage_load_clamped<PREC>(pre, xsrc, mp, n, q0, j0, ch + 1 < nch ? ch + 1 : ch);
      const uint16_t* base = As + (size_t)(ch & 1) * (KBQ + KBN) * G::ALD;
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {           // two 32-wide k steps per stage
        shortx8 av[4], bv[2];
#pragma unroll
        for (int a = 0; a < 4; ++a)
          av[a] = *reinterpret_cast<const shortx8*>(
              base + (64 * wr + 16 * a + lane % 16) * G::ALD + 32 * kk + 8 * (lane / 16));
#pragma unroll
        for (int b = 0; b < 2; ++b)
          bv[b] = *reinterpret_cast<const shortx8*>(
              base + (KBQ + 32 * wc + 16 * b + lane % 16) * G::ALD + 32 * kk + 8 * (lane / 16));
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = mfma16x16x32bf16(av[a], bv[b], acc[a][b]);
      }
      stage_store<PREC>(pre, smem, (ch + 1) & 1);
      __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = 32 * wc + 16 * b + lane % 16;
      const int64_t gj = j0 + col;
      const bool colok = gj < n;
      const int dq = (int)(j0 - q0) + col;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 64 * wr + 16 * a + 4 * (lane / 16) + r;
          float sc = -2.0f * acc[a][b][r];
          if (!colok || (!include_self && dq == row)) sc = INFINITY;
          Ss[row * SLD + col] = sc;
        }
    }
  } else {
    // fp8 e4m3 (OCP) with per-row scales: x ~ s_i * x8_i, dot = s_i s_j (x8_i . x8_j).  One
    // 16x16x128 MFMA per fragment pair and stage, each from a zero accumulator: the fp8 MFMA
    // rounds its sum (its accumulator input included) well short of float32, so the stage
    // results are added in float32 and that error does not compound over the stages.
    uint8_t* As = reinterpret_cast<uint8_t*>(smem);
    floatx4 acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    const floatx4 zero4 = {0.f, 0.f, 0.f, 0.f};
    stage_store<PREC>(pre, smem, 0);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
      // one basic block per stage: the last stage reloads itself and stores it to the idle
      // buffer (never read), so the scheduler sees the loads, products and sums together
      stage_load_clamped<PREC>(pre, xsrc, mp, n, q0, j0, ch + 1 < nch ? ch + 1 : ch);
      const uint8_t* base = As + (size_t)(ch & 1) * (KBQ + KBN) * G::ALD + 32 * (lane / 16);
      // lane l supplies row l % 16, bytes 32 (l / 16) .. + 31 of the stage, for A and B alike
      intx8 bv[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = lds_load32(base + (KBQ + 32 * wc + 16 * b + lane % 16) * G::ALD);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const intx8 av = lds_load32(base + (64 * wr + 16 * a + lane % 16) * G::ALD);
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] += __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv[b], zero4, 0, 0, 0, 0, 0, 0);
        // two products in flight per wave (the other waves of the SIMD fill the MFMA pipe):
        // the results need no more registers than that
        __builtin_amdgcn_sched_barrier(0);
      }
      stage_store<PREC>(pre, smem, (ch + 1) & 1);
      __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = 32 * wc + 16 * b + lane % 16;
      const int64_t gj = j0 + col;
      const bool colok = gj < n;
      const int dq = (int)(j0 - q0) + col;
      const float sj = colok ? scales[gj] : 0.0f;
      const float* sq = scales + q0;                // row scales of the query tile
      const int nq = (int)(n - q0 < KBQ ? n - q0 : KBQ);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 64 * wr + 16 * a + 4 * (lane / 16) + r;
          const float si = row < nq ? sq[row] : 0.0f;
          float sc = (-2.0f * si * sj) * acc[a][b][r];
          if (!colok || (!include_self && dq == row)) sc = INFINITY;
          Ss[row * SLD + col] = sc;
        }
    }
  }
}

// Top-K' update of the RPW rows a wave owns against 128 new candidates c0 .. c0 + 127, in
// two steps.  lists_filter: a cheap, unrolled pass marks the rows with any score below
// their threshold (the list's K'-th key and lane rr of capv, the caller's upper bound for
// row rr);
// score(rr, h) is row rr's score of candidate c0 + 64 h + lane, rr a compile-time index.
// lists_apply: only the marked rows are swapped into working registers and updated (one
// copy of the code); score(rr, h) is read again with rr a run-time index.
template <class F>
__device__ __forceinline__ uint32_t lists_filter(const uint32_t (&lh)[RPW], const F& score, int kc,
                                                 uint32_t capv) {
  uint32_t need = 0;
#pragma unroll
  for (int rr = 0; rr < RPW; ++rr) {
    const uint32_t own = rdlane_u(lh[rr], kc - 1);
    const uint32_t th = umin32(own, rdlane_u(capv, rr));
    // no short-circuit: every score load is issued up front
    const bool hit = (f2ord(score(rr, 0)) < th) | (f2ord(score(rr, 1)) < th);
    need |= (__ballot(hit) != 0ull ? 1u : 0u) << rr;
  }
  return need;
}

template <class F>
__device__ __forceinline__ void lists_apply(uint32_t (&lh)[RPW], uint32_t (&ll)[RPW], uint32_t need,
                                            const F& score, uint32_t c0, int kc, int lane,
                                            uint32_t capv) {
  while (need) {
    const int rr = __ffs(need) - 1;
    need &= need - 1;
    uint32_t wh = lh[0], wl = ll[0];
#pragma unroll
    for (int r = 1; r < RPW; ++r) {
      wh = rr == r ? lh[r] : wh;
      wl = rr == r ? ll[r] : wl;
    }
    const uint32_t cp = rdlane_u(capv, rr);
    row_update(wh, wl, f2ord(score(rr, 0)), c0 + (uint32_t)lane, f2ord(score(rr, 1)),
               c0 + 64u + (uint32_t)lane, kc, cp);
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      lh[r] = rr == r ? wh : lh[r];
      ll[r] = rr == r ? wl : ll[r];
    }
  }
}

// Distance GEMM + per-row top-K' over the row side of a tile-pair schedule, cut into G
// equal ranges of pairs.  Each workgroup keeps the lists of the current row tile's 128
// queries in registers (wave w: rows RPW w .. RPW w + RPW - 1) and writes them to list
// slot (its rank among the workgroups sharing that row tile) when the row tile changes.
// The workgroups sharing a row tile run at the same time: each publishes an updated row's
// K'-th key to thr[q] (atomic minimum) and filters against the smallest one published.
// Any list's K'-th key bounds the final one from above, so a candidate skipped this way
// scores at least the final merged K'-th key, which is all the re-rank's certificate needs.
// Under the symmetric schedule every off-diagonal pair also leaves its transposed tile in
// tbuf for the column pass.
template <int PREC>
__global__ __launch_bounds__(KNT) __attribute__((amdgpu_waves_per_eu(4, 4))) void knn_gemm_topk_kernel(
    const void* __restrict__ xsrc, int64_t mp, const float* __restrict__ norms,
    const float* __restrict__ scales, int64_t n, int kc, int sym, int64_t G, int nslot,
    int include_self, float* __restrict__ cand_s, int* __restrict__ cand_j, float* __restrict__ tbuf,
    uint32_t* __restrict__ thr) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int w = tid / WAVE, lane = tid % WAVE;
  const TileSched S = make_sched(n, sym);
  const int64_t P = a_pairs(S);
  // XCD-aware logical id: dispatch order bid -> XCD bid % 8
  const int64_t bid = blockIdx.x;
  const int64_t L = (G % 8 == 0) ? (bid % 8) * (G / 8) + bid / 8 : bid;
  const int64_t tb = (L * P) / G, te = ((L + 1) * P) / G;
  const float* Ss = reinterpret_cast<const float*>(smem);

  uint32_t lh[RPW], ll[RPW];   // per-row sorted key lists (score order bits, index)
  int64_t cur_qt = -1;
  auto flush = [&]() {
    if (cur_qt < 0) return;
    const int64_t seg = L - range_owner(a_start(S, cur_qt), G, P);
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
      const int64_t gi = cur_qt * KBQ + RPW * w + rr;
      if (gi < n && lane < kc) {
        const int64_t o = ((cur_qt * nslot + seg) * KBQ + RPW * w + rr) * kc + lane;
        cand_s[o] = ord2f(lh[rr]);
        cand_j[o] = (int)ll[rr];
      }
    }
  };
  int64_t qt = 0, d = 0;
  uint4 pre[Stage<PREC>::NPRE];
  if (tb < te) {
    a_pair(S, tb, qt, d);
    stage_load<PREC>(pre, xsrc, mp, n, qt * KBQ, a_db(S, qt, d) * KBN, 0);
  }
  for (int64_t t = tb; t < te; ++t) {
    if (qt != cur_qt) {
      flush();
      cur_qt = qt;
#pragma unroll
      for (int rr = 0; rr < RPW; ++rr) {
        lh[rr] = KEY_PAD_HI;
        ll[rr] = KEY_PAD_LO;
      }
    }
    const int64_t j0 = a_db(S, qt, d) * KBN;
    const int64_t q0 = qt * KBQ;
    const int64_t gq = q0 + RPW * w + lane;
    tile_scores<PREC>(xsrc, mp, norms, scales, n, q0, j0, include_self, smem, pre);
    __syncthreads();
    // Norms of the query rows (transposed store) and database columns (filter), then stage 0
    // of the next pair, all unconditional (clamped rows): no later wait on memory before the
    // next pair's first LDS store.
    const int64_t nl = n - 1;
    const float njr0 = norms[j0 + lane < n ? j0 + lane : nl];
    const float njr1 = norms[j0 + 64 + lane < n ? j0 + 64 + lane : nl];
    // lane rr < RPW: the smallest K'-th key any workgroup has published for row RPW w + rr,
    // read after the pair's GEMM (the later, the smaller)
    const uint32_t thrr = thr[gq < n ? gq : nl];
    const float nxr0 = norms[q0 + lane < n ? q0 + lane : nl];
    const float nxr1 = norms[q0 + 64 + lane < n ? q0 + 64 + lane : nl];
    const float nx0 = q0 + lane < n ? nxr0 : INFINITY;
    const float nx1 = q0 + 64 + lane < n ? nxr1 : INFINITY;
    const float nj0 = j0 + lane < n ? njr0 : 0.0f;
    const float nj1 = j0 + 64 + lane < n ? njr1 : 0.0f;
    const uint32_t capv = lane < RPW && gq < n ? thrr : 0xFFFFFFFFu;
    // an empty statement that takes these values completes their loads here, ahead of the
    // stage load: a later wait for them (the store branch below is conditional) would also
    // wait for the stage load and the transposed stores
    __asm__ volatile("" ::"v"(nx0), "v"(nx1), "v"(nj0), "v"(nj1), "v"(capv));
    __builtin_amdgcn_sched_barrier(0);
    int64_t nqt = qt, nd = d;
    a_next(S, nqt, nd);
    if (t + 1 >= te) {   // last pair: reload this one (never used)
      nqt = qt;
      nd = d;
    }
    stage_load_clamped<PREC>(pre, xsrc, mp, n, nqt * KBQ, a_db(S, nqt, nd) * KBN);
    // the symmetric schedule's off-diagonal pairs leave the transposed scores for the column
    // pass: tbuf[pair][c][r] = ||x_r||^2 + D[r][c] (+inf past row n); wave w writes columns
    // 16 w .. 16 w + 15, lanes over rows
    if (sym && d > 0) {
      // the column base is wave-uniform (scalar address + 32-bit lane offset)
      const int c0 = 16 * __builtin_amdgcn_readfirstlane(w);
      float* tout = tbuf + b_index(S, qt, d) * (KBQ * KBN) + c0 * KBQ;
#pragma unroll 4
      for (int cc = 0; cc < 16; ++cc) {
        tout[cc * KBQ + lane] = Ss[lane * SLD + c0 + cc] + nx0;
        tout[cc * KBQ + 64 + lane] = Ss[(64 + lane) * SLD + c0 + cc] + nx1;
      }
    }
    const float* srow = Ss + RPW * w * SLD + lane;
    const auto score = [&](int rr, int h) { return srow[rr * SLD + 64 * h] + (h ? nj1 : nj0); };
    const uint32_t need = lists_filter(lh, score, kc, capv);
    lists_apply(lh, ll, need, score, (uint32_t)j0, kc, lane, capv);
    if (need) {
      // publish the updated rows' K'-th keys (lane rr: row RPW w + rr)
      uint32_t mine = 0xFFFFFFFFu;
#pragma unroll
      for (int rr = 0; rr < RPW; ++rr) {
        const uint32_t kth = rdlane_u(lh[rr], kc - 1);
        mine = lane == rr ? kth : mine;
      }
      if (lane < RPW && ((need >> lane) & 1u) && gq < n && mine < capv) atomicMin(thr + gq, mine);
    }
    __syncthreads();
    qt = nqt;
    d = nd;
  }
  flush();
}

// The diagonal tile pairs' scores for the rescan of uncertified queries: tile qt against
// itself, computed by the same code as in the GEMM kernel (so with the same roundings) and
// stored like a transposed tile after the off-diagonal ones; only tiles holding a rescanned
// query are computed.
template <int PREC>
__global__ __launch_bounds__(KNT) void knn_diag_tiles_kernel(const void* __restrict__ xsrc, int64_t mp,
                                                             const float* __restrict__ norms,
                                                             const float* __restrict__ scales, int64_t n,
                                                             int include_self, float* __restrict__ tbuf,
                                                             const uint32_t* __restrict__ tile_active) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t qt = blockIdx.x;
  if (tile_active[qt] == 0u) return;             // uniform over the workgroup
  const TileSched S = make_sched(n, 1);
  const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int64_t q0 = qt * KBQ;
  uint4 pre[Stage<PREC>::NPRE];
  stage_load<PREC>(pre, xsrc, mp, n, q0, q0, 0);
  tile_scores<PREC>(xsrc, mp, norms, scales, n, q0, q0, include_self, smem, pre);
  __syncthreads();
  const float* Ss = reinterpret_cast<const float*>(smem);
  const float nx0 = q0 + lane < n ? norms[q0 + lane] : INFINITY;
  const float nx1 = q0 + 64 + lane < n ? norms[q0 + 64 + lane] : INFINITY;
  const int c0 = 16 * w;
  float* tout = tbuf + (b_pairs(S) + qt) * (KBQ * KBN) + c0 * KBQ;
  for (int cc = 0; cc < 16; ++cc) {
    tout[cc * KBQ + lane] = Ss[lane * SLD + c0 + cc] + nx0;
    tout[cc * KBQ + 64 + lane] = Ss[(64 + lane) * SLD + c0 + cc] + nx1;
  }
}

// The row-side lists of the symmetric schedule are complete once the GEMM kernel ends: the
// K'-th key of their merge (one wave per query; each list ascending, read in reverse) bounds
// the query's final K'-th key from above.
__global__ __launch_bounds__(256) void knn_rowcap_kernel(int64_t n, int kc, int64_t GA, int nslot,
                                                          const float* __restrict__ cand_s,
                                                          const int* __restrict__ cand_j,
                                                          uint32_t* __restrict__ rowcap) {
  const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int64_t q = (int64_t)blockIdx.x * 4 + wv;
  if (q >= n) return;                       // whole wave exits together
  const TileSched S = make_sched(n, 1);
  const int64_t qt = q / KBQ, row = q % KBQ;
  const int64_t na = segments(a_start(S, qt), a_len(S, qt), GA, a_pairs(S));
  const int src = WAVE - 1 - lane;
  uint32_t lh = KEY_PAD_HI, ll = KEY_PAD_LO;
  for (int64_t sg = 0; sg < na; ++sg) {
    const int64_t o = ((qt * nslot + sg) * KBQ + row) * kc + src;
    uint32_t bh = 0xFFFFFFFFu, bl = 0xFFFFFFFFu;
    if (src < kc) {
      bh = f2ord(cand_s[o]);
      bl = (uint32_t)cand_j[o];
    }
    wave_merge64(lh, ll, bh, bl);
  }
  if (lane == 0) rowcap[q] = rdlane_u(lh, kc - 1);
}

// Column side of the symmetric schedule: the queries of column tile j scan the transposed
// tiles of the pairs ((j - d) mod T, j), d = 1 .. b_len(j), with the register lists of the
// GEMM kernel; their lists go to slots slot0 + (rank among the workgroups sharing j).
// Streams the tiles once (the next pair's scores load behind the current top-K' work) and
// does no arithmetic on X.  rowcap[q] (knn_rowcap_kernel) bounds query q's final K'-th key
// from above; candidates at or above it are skipped.  Everything skipped scores at least
// the final merged K'-th key, which is what the re-rank's certificate needs.
__global__ __launch_bounds__(KNT) __attribute__((amdgpu_waves_per_eu(4, 4))) void knn_column_topk_kernel(
    const float* __restrict__ tbuf, int64_t n, int kc, int64_t G, int slot0, int nslot,
    const uint32_t* __restrict__ rowcap, float* __restrict__ cand_s, int* __restrict__ cand_j) {
  const int tid = threadIdx.x;
  const int w = tid / WAVE, lane = tid % WAVE;
  const TileSched S = make_sched(n, 1);
  const int64_t P = b_pairs(S);
  const int64_t bid = blockIdx.x;
  const int64_t L = (G % 8 == 0) ? (bid % 8) * (G / 8) + bid / 8 : bid;
  const int64_t tb = (L * P) / G, te = ((L + 1) * P) / G;

  uint32_t lh[RPW], ll[RPW];
  uint32_t capv = 0xFFFFFFFFu;   // lane rr: the bound of row RPW w + rr
  int64_t cur_j = -1;
  auto flush = [&]() {
    if (cur_j < 0) return;
    const int64_t seg = slot0 + L - range_owner(b_start(S, cur_j), G, P);
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
      const int64_t gi = cur_j * KBQ + RPW * w + rr;
      if (gi < n && lane < kc) {
        const int64_t o = ((cur_j * nslot + seg) * KBQ + RPW * w + rr) * kc + lane;
        cand_s[o] = ord2f(lh[rr]);
        cand_j[o] = (int)ll[rr];
      }
    }
  };
  // wave w's rows of transposed tile t (rows RPW w + rr, candidates lane and 64 + lane) go
  // global -> registers (loaded one pair ahead) -> the wave's own LDS rows, which the filter
  // and the list updates read like the GEMM kernel's score tile
  __shared__ float rows_lds[KNT / WAVE][RPW][KBN];
  float (*my)[KBN] = rows_lds[w];
  float c0[RPW], c1[RPW];
  auto fetch = [&](int64_t t) {
    const float* trow = tbuf + t * (KBQ * KBN) + RPW * w * KBN + lane;
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
      c0[rr] = trow[rr * KBN];
      c1[rr] = trow[rr * KBN + 64];
    }
  };
  int64_t j = 0, d = 1;
  if (tb < te) {
    b_pair(S, tb, j, d);
    fetch(tb);
  }
  for (int64_t t = tb; t < te; ++t) {
    if (j != cur_j) {
      flush();
      cur_j = j;
#pragma unroll
      for (int rr = 0; rr < RPW; ++rr) {
        lh[rr] = KEY_PAD_HI;
        ll[rr] = KEY_PAD_LO;
      }
      // lane rr < RPW holds row RPW w + rr's bound (rows past n are never flushed)
      const int64_t gq = j * KBQ + RPW * w + lane;
      capv = lane < RPW && gq < n ? rowcap[gq] : 0xFFFFFFFFu;
    }
    // only this wave touches its LDS rows, and its earlier reads are complete (in order)
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
      my[rr][lane] = c0[rr];
      my[rr][64 + lane] = c1[rr];
    }
    const uint32_t need = lists_filter(lh, [&](int rr, int h) { return h ? c1[rr] : c0[rr]; }, kc, capv);
    if (t + 1 < te) fetch(t + 1);
    const int64_t i = (j - d + S.T) % S.T;   // the pair's row tile: the candidates
    lists_apply(lh, ll, need, [&](int rr, int h) { return my[rr][64 * h + lane]; }, (uint32_t)(i * KBQ),
                kc, lane, capv);
    if (++d > b_len(S, j)) {
      ++j;
      d = 1;
    }
  }
  flush();
}

// ------------------------------------------------------------------------------------
// float32 difference-form distances sum_a (x_a - y_a)^2 from the original X of the
// candidates held by lanes 0 .. kc-1 (index lj, valid_j) to query qi: every lane keeps a
// partial sum per candidate (lanes over columns), then one transpose-reduction leaves the
// total for candidate r in lane r.  Lanes past kc or with an invalid index get +inf.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ float cand_exact_d2(const float* __restrict__ X, int64_t m, int64_t ldx, int64_t qi,
                                               int lj, bool valid_j, int kc, int lane) {
  const int jsafe = valid_j ? lj : (int)qi;
  float acc[KCMAX];
#pragma unroll
  for (int r = 0; r < KCMAX; ++r) acc[r] = 0.0f;
  const float* xq = X + qi * ldx;
  if ((ldx & 3) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0) {
    // 16-byte rows: each lane reads four consecutive columns per candidate row
    for (int64_t c0 = 0; c0 < m; c0 += 4 * WAVE) {
      const int64_t c = c0 + 4 * lane;
      float4 xv = make_float4(0.f, 0.f, 0.f, 0.f);
      if (c + 3 < m) {
        xv = *reinterpret_cast<const float4*>(xq + c);
      } else if (c < m) {
        xv.x = xq[c];
        if (c + 1 < m) xv.y = xq[c + 1];
        if (c + 2 < m) xv.z = xq[c + 2];
      }
#pragma unroll
      for (int r = 0; r < KCMAX; ++r) {
        if (r < kc) {
          const float* yr = X + (int64_t)__builtin_amdgcn_readlane(jsafe, r) * ldx;
          float4 yv = make_float4(0.f, 0.f, 0.f, 0.f);
          if (c + 3 < m) {
            yv = *reinterpret_cast<const float4*>(yr + c);
          } else if (c < m) {
            yv.x = yr[c];
            if (c + 1 < m) yv.y = yr[c + 1];
            if (c + 2 < m) yv.z = yr[c + 2];
          }
          const float d0 = xv.x - yv.x, d1 = xv.y - yv.y, d2 = xv.z - yv.z, d3 = xv.w - yv.w;
          acc[r] = fmaf(d3, d3, fmaf(d2, d2, fmaf(d1, d1, fmaf(d0, d0, acc[r]))));
        }
      }
    }
  } else {
    for (int64_t c0 = 0; c0 < m; c0 += WAVE) {
      const int64_t c = c0 + lane;
      const bool in = c < m;
      const float xv = in ? xq[c] : 0.0f;
#pragma unroll
      for (int r = 0; r < KCMAX; ++r) {
        if (r < kc) {
          const int j = __builtin_amdgcn_readlane(jsafe, r);
          const float df = xv - (in ? X[(int64_t)j * ldx + c] : 0.0f);
          acc[r] = fmaf(df, df, acc[r]);
        }
      }
    }
  }
#pragma unroll
  for (int wdt = 32; wdt >= 1; wdt >>= 1) {
    const bool upper = (lane & wdt) != 0;
#pragma unroll
    for (int t = 0; t < wdt; ++t) {
      const float send = upper ? acc[t] : acc[t + wdt];
      const float keep = upper ? acc[t + wdt] : acc[t];
      acc[t] = keep + __shfl_xor(send, wdt, WAVE);
    }
  }
  return (lane < kc && valid_j) ? acc[0] : INFINITY;
}

// Rounding bounds shared by the certificate and the rescan.  A query's GEMM score of a
// point j, s = fl(||y_j||^2 - 2 x_i . y_j) on the copies y = lowp(x - mu) the GEMM
// multiplies, differs from ||y_j||^2 - 2 y_i . y_j by at most E: float32 norms, the dot
// product's error g sum |y_ia y_ja| <= g ||y_i|| ||y_j|| (knn_dot_err: float32 accumulation
// of exact products for the float32 and bf16 MFMAs, the fp8 MFMA's own rounding plus the
// float32 sum of its per-stage results for fp8), the fp8 scale products, the final add, and
// the re-association of a transposed score (fl(||y_r||^2 + D) - ||y_r||^2 + ||y_c||^2).  With the stored norms rounded too,
//   ||y_i - y_j|| >= sqrt(max(0, s + ||y_i||^2 - E)),
// and by the triangle inequality the centred rows xc = fl(x - mu) are at least
// e_i + e_j closer than that at most (e = ||y - xc||, the rounding radius), the originals
// at most cen_i + cen_j more (cen = 1.0001 u (||y|| + e), the rounding of the centring).
struct CertBounds {
  double a;      // s + a = the lower bound on ||y_i - y_j||^2 (a = ||y_i||^2 - E)
  double slack;  // e_i + cen_i
  double emax;   // e_j + cen_j over all j
};

__device__ __forceinline__ CertBounds cert_bounds(double ni, double ei, double nmax, double emax, double gdot) {
  const double u = 0x1p-24;
  const double rn = sqrt(ni);
  const double E = 4.0 * u * ni + 5.0 * u * nmax * nmax + (2.0 * gdot + 14.0 * u) * rn * nmax;
  CertBounds b;
  b.a = ni - E;
  b.slack = ei + 1.0001 * u * (rn + ei);
  b.emax = emax + 1.0001 * u * (nmax + emax);
  return b;
}

// ------------------------------------------------------------------------------------
// merge + float32 re-rank + certificate.  One wave per query, 4 queries per block.
// A query is certified when every point outside its K' candidates is provably farther than
// its k-th re-ranked neighbour; under the symmetric schedule an uncertified one is handed to
// the rescan (knn_collect + knn_rerank2) with its exact candidate distances and thresholds.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void knn_rerank_kernel(
    const float* __restrict__ X, int64_t n, int64_t m, int64_t ldx, int k, int kc, int sym,
    int64_t GA, int64_t GB, int slotb, int nslot, const float* __restrict__ cand_s,
    const int* __restrict__ cand_j,
    const float* __restrict__ norms, const float* __restrict__ radius,
    const float* __restrict__ stats, int include_self, int32_t* __restrict__ idx_out,
    float* __restrict__ d2_out, uint8_t* __restrict__ kflags, double gdot, RescanWs rs) {
  const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int64_t qi = (int64_t)blockIdx.x * 4 + wv;
  if (qi >= n) return;                      // whole wave exits together
  const TileSched S = make_sched(n, sym);
  const int64_t qt = qi / KBQ, row = qi % KBQ;
  // list segments: row side (slots 0 ..), column side (slots slotb ..)
  const int64_t na = segments(a_start(S, qt), a_len(S, qt), GA, a_pairs(S));
  const int64_t nb = sym ? segments(b_start(S, qt), b_len(S, qt), GB, b_pairs(S)) : 0;
  // merge the segment lists (each ascending; read in reverse, so descending) into the 64 best;
  // eight lists' loads are in flight before their merges
  uint32_t lh = KEY_PAD_HI, ll = KEY_PAD_LO;
  const int src = WAVE - 1 - lane;
  for (int64_t s0 = 0; s0 < na + nb; s0 += 8) {
    uint32_t bh[8], bl[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t sg = s0 + u;
      const int64_t slot = sg < na ? sg : slotb + (sg - na);
      const int64_t o = ((qt * nslot + slot) * KBQ + row) * kc;
      const bool in = sg < na + nb && src < kc;
      bh[u] = in ? f2ord(cand_s[o + src]) : 0xFFFFFFFFu;
      bl[u] = in ? (uint32_t)cand_j[o + src] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (s0 + u < na + nb) wave_merge64(lh, ll, bh[u], bl[u]);
  }
  const int lj = (int)ll;
  const float s_last = ord2f(rdlane_u(lh, kc - 1));   // every non-candidate scores >= s_last
  const bool valid_j = lj >= 0 && (int64_t)lj < n;
  const float myd = cand_exact_d2(X, m, ldx, qi, lj, valid_j, kc, lane);
  const int myj = (lane < kc && valid_j) ? lj : INT_MAX;
  // order by (distance, index); the point itself (MC_INCLUDE_SELF) comes first
  uint32_t sh = f2ord(lane < kc ? myd : INFINITY);
  uint32_t sl = (uint32_t)(lane < kc ? myj : INT_MAX);
  if (include_self && (int)sl == (int)qi) sh = f2ord(-1.0f);
  wave_sort64<true>(sh, sl);
  // after the sort, lane r holds rank r; recover its distance
  const int kj = (int)sl;
  float dr = ord2f(sh);
  if (include_self && kj == (int)qi) dr = 0.0f;
  if (lane < k) {
    idx_out[qi * k + lane] = kj;
    if (d2_out) d2_out[qi * k + lane] = dr;
  }
  const float dk = rdlane(dr, k - 1);
  const float dk1 = kc > k ? rdlane(dr, k) : INFINITY;
  const double u = 0x1p-24;
  const double gam = (double)(m + 2) * u / (1.0 - (double)(m + 2) * u);
  // certificate: every non-candidate y has GEMM score >= s_last
  bool cert = true;
  CertBounds cb{};
  const double dk_hi = (double)dk / (1.0 - gam);   // the true k-th distance is at most this
  if ((int64_t)kc < n - (include_self ? 0 : 1) && isfinite(s_last)) {
    cb = cert_bounds((double)norms[qi], (double)radius[qi], (double)stats[0], (double)stats[1], gdot);
    const double lo2 = (double)s_last + cb.a;
    const double lo = (lo2 > 0.0 ? sqrt(lo2) : 0.0) - cb.slack - cb.emax;
    cert = lo > 0.0 && lo * lo > dk_hi;
  }
  if (lane == 0) {
    if (kflags) {
      uint8_t fl = 0;
      if (kc > k && isfinite(dk1) && (double)dk1 - (double)dk <= 2.0 * gam * (double)dk1)
        fl |= PF_KNN_AMBIGUOUS;
      if (!cert) fl |= PF_KNN_UNCERTIFIED;
      kflags[qi] = fl;
    }
    rs.cnt[qi] = 0;
  }
  // hand an uncertified query to the rescan: a point j can be among the true k nearest only
  // if its score s satisfies sqrt(max(0, s + a)) - e_j - cen_j <= sqrt(dk_hi) + e_i + cen_i = T
  float thr = -INFINITY;
  if (!cert && sym && isfinite(dk)) {
    const double T = sqrt(dk_hi) * (1.0 + 4.0 * u) + cb.slack;
    const double tq = (T + cb.emax) * (T + cb.emax) * (1.0 + 4.0 * u) - cb.a;
    thr = (float)tq * (1.0f + 0x1p-22f);
    if (lane == 0) {
      rs.act_T[qi] = (float)T * (1.0f + 0x1p-22f);
      rs.act_a[qi] = (float)cb.a * (cb.a > 0.0 ? 1.0f - 0x1p-22f : 1.0f + 0x1p-22f);
      atomicOr(rs.tile_active + qt, 1u);
    }
    if (lane < kc) {
      rs.p1d[qi * KCMAX + lane] = dr;
      rs.p1j[qi * KCMAX + lane] = kj;
    }
  }
  if (lane == 0) rs.act_thr[qi] = thr;
}

// ------------------------------------------------------------------------------------
// Rescan of uncertified queries (symmetric schedule).  The transposed tiles hold every
// score of the distance matrix once: tile [c][r] = ||y_r||^2 + D[r][c] scores candidate r
// (row tile) for query c (column tile), and ||y_c||^2 + D[r][c] = tile - ||y_r||^2 + ||y_c||^2
// scores c for query r; the diagonal tiles cover a tile against itself.  knn_collect streams
// them once and appends every candidate that passes an active query's test to that query's
// buffer; knn_rerank2 evaluates the new ones in float32 and re-selects the k nearest.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void knn_collect_kernel(const float* __restrict__ tbuf, int64_t n, int64_t G,
                                                          const float* __restrict__ norms,
                                                          const float* __restrict__ radius, RescanWs rs) {
  const TileSched S = make_sched(n, 1);
  const int64_t PB = b_pairs(S), P = PB + S.T;
  const int64_t L = blockIdx.x;
  const int64_t tb = (L * P) / G, te = ((L + 1) * P) / G;
  __shared__ __align__(16) float q_thr[2][KBQ], q_T[2][KBQ], q_a[2][KBQ], q_n[2][KBQ], q_e[2][KBQ];
  const int tid = threadIdx.x;
  const double u = 0x1p-24;
  for (int64_t t = tb; t < te; ++t) {
    int64_t ct, rt;                          // column tile (queries of the stored rows), row tile
    if (t < PB) {
      int64_t d;
      b_pair(S, t, ct, d);
      rt = (ct - d + S.T) % S.T;
    } else {
      ct = rt = t - PB;
    }
    const bool act_c = rs.tile_active[ct] != 0u, act_r = t < PB && rs.tile_active[rt] != 0u;
    if (!act_c && !act_r) continue;          // uniform over the workgroup
    __syncthreads();
    if (tid < 2 * KBQ) {
      const int side = tid / KBQ, o = tid % KBQ;
      const int64_t q = (side == 0 ? ct : rt) * KBQ + o;
      const bool in = q < n;
      q_thr[side][o] = in ? rs.act_thr[q] : -INFINITY;
      q_T[side][o] = in ? rs.act_T[q] : 0.0f;
      q_a[side][o] = in ? rs.act_a[q] : 0.0f;
      q_n[side][o] = in ? norms[q] : 0.0f;
      const float e = in ? radius[q] : 0.0f;
      // e + cen of the point (the centring slack of cert_bounds)
      q_e[side][o] = in ? (float)((double)e + 1.0001 * u * (sqrt((double)q_n[side][o]) + (double)e)) * (1.0f + 0x1p-22f)
                        : 0.0f;
    }
    __syncthreads();
    const float* tile = tbuf + t * (int64_t)(KBQ * KBN);
    // pass v: thread tid reads the 16 bytes at float4 index tid + 256 v (row c, columns r..r+3),
    // so every load instruction of a wave covers 1 KiB of consecutive memory; eight passes are
    // in flight at a time
#pragma unroll 8
    for (int v = 0; v < KBQ * KBN / (4 * 256); ++v) {
      const int f = tid + 256 * v;
      const int c = f / (KBN / 4), rb = 4 * (f % (KBN / 4));
      const float4 s4 = *reinterpret_cast<const float4*>(tile + 4 * (int64_t)f);
      const float sv[4] = {s4.x, s4.y, s4.z, s4.w};
      const int64_t qc = ct * KBQ + c;
      const float thc = q_thr[0][c];
      const float nc = q_n[0][c], ec = q_e[0][c];
      // the four row queries' thresholds and norms: one 16-byte LDS read each
      const float4 thr4 = *reinterpret_cast<const float4*>(&q_thr[1][rb]);
      const float4 nr4 = *reinterpret_cast<const float4*>(&q_n[1][rb]);
      const float thrv[4] = {thr4.x, thr4.y, thr4.z, thr4.w};
      const float nrv[4] = {nr4.x, nr4.y, nr4.z, nr4.w};
      // candidates r for query c: the 32 lanes of a half wave share c, so their hits take one
      // counter increment per half wave, each lane writing at the base plus its rank among
      // the half wave's hits (in e4, then lane order)
      const unsigned hsh = lane_id() & 32u;                 // 0 or 32: the half wave
      const uint64_t below = ((1ull << (lane_id() & 31u)) - 1ull) << hsh;
      bool hit[4];
      int rank[4], tot = 0;
#pragma unroll
      for (int e4 = 0; e4 < 4; ++e4) {
        const int r = rb + e4;
        const int64_t qr = rt * KBQ + r;
        const float s = sv[e4];
        bool h = s <= thc && qc < n && qr < n;
        if (h) h = sqrtf(fmaxf(0.0f, s + q_a[0][c])) * (1.0f - 0x1p-22f) - q_e[1][r] <= q_T[0][c];
        const uint64_t mk = __ballot(h);
        hit[e4] = h;
        rank[e4] = tot + (int)__popcll(mk & below);
        tot += (int)__popcll((mk >> hsh) & 0xFFFFFFFFull);
      }
      int base = 0;
      if ((lane_id() & 31u) == 0 && tot > 0) base = atomicAdd(rs.cnt + qc, tot);
      base = __shfl(base, (int)hsh, WAVE);
#pragma unroll
      for (int e4 = 0; e4 < 4; ++e4) {
        const int slot = base + rank[e4];
        if (hit[e4] && slot < RESCAN_CMAX) rs.cbuf[qc * RESCAN_CMAX + slot] = (int)(rt * KBQ + rb + e4);
      }
#pragma unroll
      for (int e4 = 0; e4 < 4; ++e4) {
        const int r = rb + e4;
        const int64_t qr = rt * KBQ + r;
        const float s = sv[e4];
        // candidate c for query r (off-diagonal tiles): re-associate the stored score
        if (t < PB && qr < n && qc < n) {
          const float thr = thrv[e4];
          if (thr > -INFINITY) {
            const float s2 = (s - nrv[e4]) + nc;
            if (s2 <= thr) {
              const float lb = sqrtf(fmaxf(0.0f, s2 + q_a[1][r])) * (1.0f - 0x1p-22f) - ec;
              if (lb <= q_T[1][r]) {
                const int slot = atomicAdd(rs.cnt + qr, 1);
                if (slot < RESCAN_CMAX) rs.cbuf[qr * RESCAN_CMAX + slot] = (int)qc;
              }
            }
          }
        }
      }
    }
  }
}

// One wave per query handed to the rescan: the pass's exact candidate distances plus the
// float32 distances of every collected point not among them, re-selected by (d^2, index).
// A query whose buffer overflowed keeps its first result and its UNCERTIFIED flag.
__global__ __launch_bounds__(256) void knn_rerank2_kernel(const float* __restrict__ X, int64_t n, int64_t m,
                                                          int64_t ldx, int k, int kc, int include_self,
                                                          int32_t* __restrict__ idx_out,
                                                          float* __restrict__ d2_out,
                                                          uint8_t* __restrict__ kflags, RescanWs rs) {
  const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int64_t qi = (int64_t)blockIdx.x * 4 + wv;
  if (qi >= n) return;
  if (!(rs.act_thr[qi] > -INFINITY)) return;      // certified, or full schedule
  const int cnt = rs.cnt[qi];
  if (cnt > RESCAN_CMAX) return;
  // the first pass's kc candidates (ranks in lanes), exact float32 distances
  const int pj = lane < kc ? rs.p1j[qi * KCMAX + lane] : INT_MAX;
  const float pd = lane < kc ? rs.p1d[qi * KCMAX + lane] : INFINITY;
  uint32_t lh = f2ord(pd), ll = (uint32_t)pj;
  if (include_self && pj == (int)qi) lh = f2ord(-1.0f);
  for (int b0 = 0; b0 < cnt; b0 += WAVE) {
    const int cj = b0 + lane < cnt ? rs.cbuf[qi * RESCAN_CMAX + b0 + lane] : -1;
    bool dup = cj < 0;
    for (int r = 0; r < kc; ++r) dup |= cj == __builtin_amdgcn_readlane(pj, r);
    const uint64_t fresh = __ballot(!dup);
    const int nn = __popcll(fresh);
    if (nn == 0) continue;
    // compact the new candidates into lanes 0 .. nn-1
    const int dst = !dup ? __popcll(fresh & ((1ull << lane) - 1ull)) : WAVE - 1;
    int nj = __builtin_amdgcn_ds_permute(dst << 2, cj);
    if (lane >= nn) nj = -1;
    const bool valid = nj >= 0 && (int64_t)nj < n;
    const float d = cand_exact_d2(X, m, ldx, qi, nj, valid, nn, lane);
    uint32_t bh = lane < nn && valid ? f2ord(d) : 0xFFFFFFFFu;
    uint32_t bl = lane < nn && valid ? (uint32_t)nj : 0xFFFFFFFFu;
    if (include_self && (int)bl == (int)qi) bh = f2ord(-1.0f);
    wave_sort64<false>(bh, bl);
    wave_merge64(lh, ll, bh, bl);
  }
  const int kj = (int)ll;
  float dr = ord2f(lh);
  if (include_self && kj == (int)qi) dr = 0.0f;
  if (lane < k) {
    idx_out[qi * k + lane] = kj;
    if (d2_out) d2_out[qi * k + lane] = dr;
  }
  const float dk = rdlane(dr, k - 1);
  const float dk1 = rdlane(dr, k);
  if (lane == 0 && kflags) {
    const double u = 0x1p-24;
    const double gam = (double)(m + 2) * u / (1.0 - (double)(m + 2) * u);
    uint8_t fl = 0;
    if (isfinite(dk1) && (double)dk1 - (double)dk <= 2.0 * gam * (double)dk1) fl |= PF_KNN_AMBIGUOUS;
    kflags[qi] = fl;
  }
}

// ------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------
// Bound g on the GEMM's dot-product error relative to ||y_i|| ||y_j||.  The float32 and bf16
// MFMAs accumulate exact products in float32 (gamma_{m+2}).  The fp8 MFMA does not: on gfx950
// one 16x16x128 fp8 instruction was measured at up to 2^-12.8 of sum |p| (its accumulator
// input rounded alike), so each stage starts from zero and the bound takes 2^-9 per stage
// (a margin of 14x) plus the float32 sum of the mp / 128 stage results.
constexpr double FP8_MFMA_REL = 0x1p-9;
static double knn_dot_err(int64_t m, int64_t mp, int precision) {
  const double u = 0x1p-24;
  if (precision == 2) {
    const double r = (double)(mp / GemmCfg<2>::BK) + 2.0;
    return FP8_MFMA_REL + r * u / (1.0 - r * u);
  }
  const double t = (double)(m + 2);
  return t * u / (1.0 - t * u);
}

static int64_t knn_mp(int64_t m, int precision) {
  const int64_t bk = precision == 0 ? GemmCfg<0>::BK : (precision == 1 ? GemmCfg<1>::BK : GemmCfg<2>::BK);
  return ((m + bk - 1) / bk) * bk;
}

// Workgroups of a list stage over P tile pairs: 2 resident per CU (register and LDS bound),
// so a whole number of 512-workgroup waves (no part-full last wave), never fewer than the
// row tiles; a multiple of 8 for the XCD map.
static int64_t knn_groups(int64_t P, int64_t T) {
  constexpr int64_t RESIDENT = 512;
  int64_t G = (T + RESIDENT - 1) / RESIDENT * RESIDENT;
  if (G > P) G = P;
  if (G >= 8) G = (G + 7) / 8 * 8;
  if (G > P) G = P;
  return G;
}

// The symmetric schedule keeps one transposed 64 KiB score tile per off-diagonal pair in
// the workspace (20 GB at n = 100000, against 288 GB of HBM); beyond this many bytes (n above
// 131072) the full schedule runs.
constexpr size_t KNN_SYM_MAX_BYTES = (size_t)32 << 30;

KnnPlan knn_plan(int64_t n, int64_t m, int k, int kc, int precision) {
  KnnPlan p{};
  p.n = n;
  p.m = m;
  p.k = k;
  p.kc = kc;
  p.precision = precision;
  const int64_t T = (n + KBQ - 1) / KBQ;
  const size_t tile_b = (size_t)KBQ * KBN * 4;
  p.tiles = T;
  p.sym = (T >= 2 && (size_t)(T * (T - 1) / 2) * tile_b <= KNN_SYM_MAX_BYTES) ? 1 : 0;
  const TileSched S = make_sched(n, p.sym);
  p.pairs_a = a_pairs(S);
  p.groups = knn_groups(p.pairs_a, T);
  p.smax = 1;
  for (int64_t i = 0; i < T; ++i) {
    const int64_t c = segments(a_start(S, i), a_len(S, i), p.groups, p.pairs_a);
    if (c > p.smax) p.smax = (int)c;
  }
  p.pairs_b = p.sym ? b_pairs(S) : 0;
  p.groups_b = p.pairs_b > 0 ? knn_groups(p.pairs_b, T) : 0;
  p.smax_b = 0;
  for (int64_t j = 0; p.pairs_b > 0 && j < T; ++j) {
    const int64_t c = segments(b_start(S, j), b_len(S, j), p.groups_b, p.pairs_b);
    if (c > p.smax_b) p.smax_b = (int)c;
  }
  const int64_t mp = knn_mp(m, precision);
  const int64_t parts = KPARTS;
  const size_t esz = precision == 0 ? 4 : (precision == 1 ? 2 : 1);
  size_t off = 0;
  p.off_xc = off;     off += align256((size_t)n * mp * esz);     // the GEMM's input copy
  p.off_norm = off;   off += align256((size_t)n * 4);
  p.off_colsum = off; off += align256((size_t)parts * m * 8 + (size_t)m * 4);
  p.off_stats = off;  off += align256((size_t)n * 4 + 64);
  const size_t cand = (size_t)T * (p.smax + p.smax_b) * KBQ * kc * 4;
  p.off_cand_s = off; off += align256(cand);
  p.off_cand_j = off; off += align256(cand);
  p.off_xlow = off;
  p.off_scale = off;  off += precision == 2 ? align256((size_t)n * 4) : 0;
  p.off_cap = off;    off += p.sym ? align256((size_t)n * 4) : 0;
  p.off_thr = off;    off += align256((size_t)n * 4);
  // rescan state (per query), then the transposed tiles (plus the diagonal ones)
  p.off_rescan = off;
  off += align256((size_t)n * 4) * 4;                        // act_thr, act_T, act_a, cnt
  off += align256((size_t)n * RESCAN_CMAX * 4);              // cbuf
  off += align256((size_t)n * KCMAX * 4) * 2;                // p1d, p1j
  off += align256((size_t)T * 4);                            // tile_active
  p.off_tbuf = off;   off += p.sym ? (size_t)(p.pairs_b + T) * tile_b : 0;
  p.total = off;
  return p;
}

static RescanWs rescan_ws(unsigned char* base, const KnnPlan& p) {
  RescanWs r;
  const int64_t n = p.n;
  size_t off = p.off_rescan;
  r.act_thr = reinterpret_cast<float*>(base + off); off += align256((size_t)n * 4);
  r.act_T = reinterpret_cast<float*>(base + off);   off += align256((size_t)n * 4);
  r.act_a = reinterpret_cast<float*>(base + off);   off += align256((size_t)n * 4);
  r.cnt = reinterpret_cast<int*>(base + off);       off += align256((size_t)n * 4);
  r.cbuf = reinterpret_cast<int*>(base + off);      off += align256((size_t)n * RESCAN_CMAX * 4);
  r.p1d = reinterpret_cast<float*>(base + off);     off += align256((size_t)n * KCMAX * 4);
  r.p1j = reinterpret_cast<int*>(base + off);       off += align256((size_t)n * KCMAX * 4);
  r.tile_active = reinterpret_cast<uint32_t*>(base + off);
  return r;
}

hipError_t launch_knn(const float* X, int64_t n, int64_t m, int64_t ldx, int k, int kc,
                      int precision, bool include_self, int32_t* idx, float* d2, uint8_t* kflags,
                      void* ws, const KnnPlan& plan, hipStream_t stream) {
  unsigned char* base = reinterpret_cast<unsigned char*>(ws);
  const int64_t mp = knn_mp(m, precision);
  void* xc = base + plan.off_xc;
  float* scales = precision == 2 ? reinterpret_cast<float*>(base + plan.off_scale) : nullptr;
  float* norms = reinterpret_cast<float*>(base + plan.off_norm);
  double* part = reinterpret_cast<double*>(base + plan.off_colsum);
  float* mu = reinterpret_cast<float*>(base + plan.off_colsum + (size_t)KPARTS * m * 8);
  float* radius = reinterpret_cast<float*>(base + plan.off_stats);
  float* stats = radius + n;
  float* cand_s = reinterpret_cast<float*>(base + plan.off_cand_s);
  int* cand_j = reinterpret_cast<int*>(base + plan.off_cand_j);

  const int64_t parts = KPARTS;
  const int64_t rows_per = (n + parts - 1) / parts;
  const unsigned gx = (unsigned)((m + 255) / 256);
  timing_begin(0, stream);
  hipLaunchKernelGGL(knn_colsum_kernel, dim3(gx, (unsigned)parts), dim3(256), 0, stream, X, n, m,
                     ldx, rows_per, part);
  timing_end(0, stream);
  timing_begin(1, stream);
  hipLaunchKernelGGL(knn_mean_kernel, dim3((unsigned)((m + 15) / 16)), dim3(256), 0, stream, part, m,
                     (int)parts, n, mu, reinterpret_cast<uint32_t*>(stats));
  timing_end(1, stream);
  timing_begin(2, stream);
  uint32_t* thr = reinterpret_cast<uint32_t*>(base + plan.off_thr);
  const RescanWs rs = rescan_ws(base, plan);
  hipLaunchKernelGGL(knn_center_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream, X, n,
                     m, ldx, mp, mu, xc, scales, norms, radius, precision, thr, rs.tile_active);
  timing_end(2, stream);
  timing_begin(3, stream);
  const unsigned sgrid = (unsigned)((n + 255) / 256 < 64 ? (n + 255) / 256 : 64);
  hipLaunchKernelGGL(knn_stats_kernel, dim3(sgrid), dim3(256), 0, stream, norms, radius, n,
                     reinterpret_cast<uint32_t*>(stats));
  timing_end(3, stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;

  static std::atomic<uint64_t> attr_set{0};   // LDS beyond 64 KiB needs the opt-in attribute
  once_per_device(attr_set, [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&knn_gemm_topk_kernel<0>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm_lds_bytes<0>());
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&knn_gemm_topk_kernel<1>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm_lds_bytes<1>());
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&knn_gemm_topk_kernel<2>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm_lds_bytes<2>());
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&knn_diag_tiles_kernel<0>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm_lds_bytes<0>());
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&knn_diag_tiles_kernel<1>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm_lds_bytes<1>());
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&knn_diag_tiles_kernel<2>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm_lds_bytes<2>());
    (void)hipGetLastError();
  });
  float* tbuf = reinterpret_cast<float*>(base + plan.off_tbuf);
  const int nslot = plan.smax + plan.smax_b;
  const int self = include_self ? 1 : 0;
  const dim3 grid((unsigned)plan.groups);
  timing_begin(4, stream);
  if (precision == 0) {
    hipLaunchKernelGGL(knn_gemm_topk_kernel<0>, grid, dim3(KNT), gemm_lds_bytes<0>(), stream,
                       (const void*)xc, mp, norms, scales, n, kc, plan.sym, plan.groups, nslot, self,
                       cand_s, cand_j, tbuf, thr);
  } else if (precision == 1) {
    hipLaunchKernelGGL(knn_gemm_topk_kernel<1>, grid, dim3(KNT), gemm_lds_bytes<1>(), stream,
                       (const void*)xc, mp, norms, scales, n, kc, plan.sym, plan.groups, nslot, self,
                       cand_s, cand_j, tbuf, thr);
  } else {
    hipLaunchKernelGGL(knn_gemm_topk_kernel<2>, grid, dim3(KNT), gemm_lds_bytes<2>(), stream,
                       (const void*)xc, mp, norms, scales, n, kc, plan.sym, plan.groups, nslot, self,
                       cand_s, cand_j, tbuf, thr);
  }
  timing_end(4, stream);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (plan.pairs_b > 0) {
    uint32_t* rowcap = reinterpret_cast<uint32_t*>(base + plan.off_cap);
    timing_begin(9, stream);
    hipLaunchKernelGGL(knn_rowcap_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream, n, kc,
                       plan.groups, nslot, (const float*)cand_s, (const int*)cand_j, rowcap);
    hipLaunchKernelGGL(knn_column_topk_kernel, dim3((unsigned)plan.groups_b), dim3(KNT), 0, stream,
                       (const float*)tbuf, n, kc, plan.groups_b, plan.smax, nslot,
                       (const uint32_t*)rowcap, cand_s, cand_j);
    timing_end(9, stream);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  timing_begin(5, stream);
  hipLaunchKernelGGL(knn_rerank_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream, X, n, m,
                     ldx, k, kc, plan.sym, plan.groups, plan.groups_b, plan.smax, nslot, cand_s, cand_j,
                     norms, radius, stats, self, idx, d2, kflags, knn_dot_err(m, mp, precision), rs);
  timing_end(5, stream);
  e = hipGetLastError();
  if (e != hipSuccess || !plan.sym) return e;
  // rescan of the queries the certificate could not close (symmetric schedule: every score
  // is in the transposed and diagonal tiles)
  timing_begin(10, stream);
  if (precision == 0) {
    hipLaunchKernelGGL(knn_diag_tiles_kernel<0>, dim3((unsigned)plan.tiles), dim3(KNT), gemm_lds_bytes<0>(), stream,
                       (const void*)xc, mp, norms, scales, n, self, tbuf, (const uint32_t*)rs.tile_active);
  } else if (precision == 1) {
    hipLaunchKernelGGL(knn_diag_tiles_kernel<1>, dim3((unsigned)plan.tiles), dim3(KNT), gemm_lds_bytes<1>(), stream,
                       (const void*)xc, mp, norms, scales, n, self, tbuf, (const uint32_t*)rs.tile_active);
  } else {
    hipLaunchKernelGGL(knn_diag_tiles_kernel<2>, dim3((unsigned)plan.tiles), dim3(KNT), gemm_lds_bytes<2>(), stream,
                       (const void*)xc, mp, norms, scales, n, self, tbuf, (const uint32_t*)rs.tile_active);
  }
  const int64_t ptiles = plan.pairs_b + plan.tiles;
  const int64_t gc = ptiles < 2048 ? ptiles : 2048;
  hipLaunchKernelGGL(knn_collect_kernel, dim3((unsigned)gc), dim3(256), 0, stream, (const float*)tbuf, n, gc,
                     (const float*)norms, (const float*)radius, rs);
  hipLaunchKernelGGL(knn_rerank2_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream, X, n, m, ldx, k,
                     kc, self, idx, d2, kflags, rs);
  timing_end(10, stream);
  return hipGetLastError();
}

}  // namespace mc
