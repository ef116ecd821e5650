/*
 * mecuco.h -- C ABI of libmecuco.so, the MI355X (gfx950) mean-curvature hot path.
 *
 * The method (Levada, "Efficient Mean Curvature Computation on High-Dimensional
 * Data Manifolds", arXiv 2606.06329) takes a point cloud X in R^{n x m} and a
 * neighbourhood size k and returns one mean-curvature score per point
 * (Algorithm 1, "MeCuCo").  The library splits that call at its natural seam:
 *
 *   mc_knn               the kNN graph (Step 1, eq. knn; Algorithm 1 kNN-Graph)
 *   mc_curvature_fast    the Fast branch of Algorithm 1 per point (eq. fast_curv)
 *   mc_curvature_exact   Theorem 1 per point with a canonical null-space basis
 *   mc_curvature_backward  gradient of sum_i w_i kappa_i w.r.t. X (lists held fixed)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array pointer is a DEVICE pointer owned by the caller.  The library
 *    allocates nothing; scratch memory is the caller's workspace `ws` of at
 *    least mc_workspace_bytes(...) bytes (256-byte aligned).
 *  - X is float32, row-major, n rows of m values with row stride ldx >= m
 *    (in elements).  Neighbour lists are int32, n rows of k entries.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls only enqueue
 *    work on it; they never synchronise (except MC_STRICT, below).
 *  - All argument checks run on the host before anything is enqueued; a
 *    failing check returns a positive MC_E* code and enqueues nothing.
 *  - Numerical trouble never fails a call: it is reported per point through
 *    the optional uint8 flag arrays (MC_PF_* bits).  With MC_STRICT in `flags`
 *    the call synchronises the stream and returns MC_ENUMERIC if any point
 *    carries a flag bit other than the informational MC_PF_KNN_AMBIGUOUS and
 *    MC_PF_EIGEN_FP64.
 *  - Calls on different streams are independent; calls sharing a workspace
 *    must be ordered on one stream.
 *
 * Readings of the paper fixed by this ABI (the paper is silent on them)
 *  - A point is not its own neighbour (MC_INCLUDE_SELF makes it the first
 *    entry, followed by k-1 others); ties in distance go to the smaller index.
 *  - The patch is centred at the mean of its k rows; covariances use 1/(k-1).
 *  - p = k-1 range directions, reduced to the numerical rank when the patch is
 *    rank deficient (flag MC_PF_RANK_DEFICIENT); q = m - p_eff; q = 0 gives
 *    t_null = 0.
 */
#ifndef MECUCO_H
#define MECUCO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MC_VERSION 100 /* 1.0.0 */
#define MC_KMAX 32     /* largest supported k */

/* status codes */
#define MC_OK 0
#define MC_EINVAL 1      /* null pointer, k < 2, k > MC_KMAX, k >= n, n or m <= 0, ldx < m, bad enum */
#define MC_ESHAPE 2      /* size beyond the int32 index range or an on-chip limit of the operation */
#define MC_EPRECISION 3  /* precision not available for this operation */
#define MC_EWORKSPACE 4  /* ws_bytes smaller than mc_workspace_bytes(...) or ws misaligned */
#define MC_ELAUNCH 5     /* a kernel launch failed (hipGetLastError) */
#define MC_ENUMERIC 6    /* MC_STRICT: some point carries a flag */
#define MC_EDEVICE 7     /* no usable gfx950 device current */
#define MC_ESCRATCH 8    /* sizes need more than the static scratch of a no-allocation entry point */

/* precision of the MFMA stages (distance GEMM, patch moments) */
#define MC_FP32 0 /* float32 inputs, float32 accumulation */
#define MC_BF16 1 /* bfloat16 inputs, float32 accumulation */
#define MC_FP8 2  /* OCP e4m3 inputs with per-row scales (mc_knn only), float32 accumulation */
#define MC_FP64 3 /* float64 centring and moments (mc_curvature_fast only, k <= MC_FAST_FP64_KMAX) */
#define MC_FAST_FP64_KMAX 28 /* the float64 moments of one point must fit in LDS */

/* reading of the Fast-mode null-space term */
#define MC_FAST_PAPER 0 /* Algorithm 1 / eqs. tnull, tA, tB as printed: t_B uses ||X_c V_r||^2, denominator D-p */
#define MC_FAST_HAAR 1  /* exact expectation of eq. gnull_exp: t_B uses sum X_c^2 (V_r o V_r)1, denominator D-p+2 */

/* flags argument bits */
#define MC_INCLUDE_SELF 1u /* mc_knn: the point itself is its first neighbour */
#define MC_STRICT 2u       /* turn per-point flags into MC_ENUMERIC (synchronises) */

/* per-point flag bits (uint8) */
#define MC_PF_NONFINITE 1u       /* a patch value is NaN/Inf, or idx out of range; kappa = NaN */
#define MC_PF_DEGENERATE 2u      /* tau = 0 (all k points equal); kappa = 0 */
#define MC_PF_RANK_DEFICIENT 4u  /* numerical rank of the patch below k-1 */
#define MC_PF_JACOBI_MAXSWEEPS 8u /* k x k eigen-solve hit its sweep limit */
#define MC_PF_KNN_AMBIGUOUS 16u  /* k-th and (k+1)-th distances within float32 rounding of each other */
#define MC_PF_KNN_UNCERTIFIED 32u /* the candidate set could not be proven to contain the k nearest */
#define MC_PF_EIGEN_FP64 64u     /* (information) Fast mode: the float32 eigen-solve found two kept
                                    eigenvalues within a relative 2^-13 and was redone in float64 */
#define MC_PF_PRECISION_LIMIT 128u /* Fast mode: the point's error estimate exceeds the precision's
                                      budget (an ill-conditioned Gram matrix, or bf16 moments on rows
                                      narrower than 256; see mc_curvature_fast); kappa is still
                                      written; MC_FP64 moments hold where this is set */

/* operations for mc_workspace_bytes */
#define MC_OP_KNN 0
#define MC_OP_FAST 1
#define MC_OP_EXACT 2
#define MC_OP_BACKWARD 3
#define MC_OP_NORMALIZE 4 /* mc_normalize_minmax (only n is read) */

/*
 * mc_knn -- k nearest neighbours of every point by brute force (Step 1, eq. knn).
 *
 * Distances are Euclidean.  A tiled MFMA GEMM on globally mean-centred copies of
 * X (precision: MC_FP32, MC_BF16, or MC_FP8 with per-row scales) proposes
 * K' = rerank_factor * k candidates per point; they are re-ranked with float32
 * difference-form distances sum_a (x_a - y_a)^2 on the original X and the k
 * smallest are kept, ordered by (distance, index).  With rerank_factor == 1 the
 * GEMM distances decide (MC_FP32 only).  The distance matrix is symmetric: while
 * the workspace for it stays within 32 GiB (n up to 131072), each unordered pair
 * of 128-point tiles is scored once and its transposed 64 KiB score tile serves
 * the other tile's queries, so the workspace then holds about n^2 / 2 floats
 * (0.8 GB at n = 20000, 20 GB at n = 100000).
 *
 *   X            [n x ldx] float32, device
 *   n, m, ldx    points, dimensions, row stride (elements)
 *   k            neighbours per point, 2 <= k <= MC_KMAX, k < n
 *   precision    MC_FP32 | MC_BF16 | MC_FP8
 *   rerank_factor 1..4 (K' = rerank_factor * k must not exceed 64 and must be < n)
 *   flags        MC_INCLUDE_SELF | MC_STRICT
 *   idx_out      [n x k] int32, device, written
 *   d2_out       [n x k] float32 squared distances (float32 difference form), or NULL
 *   knn_flags    [n] uint8 (MC_PF_KNN_* bits), or NULL
 *   ws, ws_bytes workspace, >= mc_workspace_bytes(MC_OP_KNN, n, m, k, precision, rerank_factor)
 *   stream       hipStream_t
 */
int mc_knn(const float* X, int64_t n, int64_t m, int64_t ldx, int32_t k, int32_t precision,
           int32_t rerank_factor, uint32_t flags, int32_t* idx_out, float* d2_out,
           uint8_t* knn_flags, void* ws, size_t ws_bytes, void* stream);

/*
 * mc_curvature_fast -- Fast branch of Algorithm 1 for every point (eq. fast_curv).
 *
 * For point i the patch is X[idx[i][0..k-1]], centred at its mean.  tau, the
 * range term t_range = ||X_c V_r^{o2}||^2/(k-1), t_A, t_B and t_null are those
 * of Algorithm 1 in the reading `variant`; kappa_i = |(t_range + t_null)/2 + tau/2|.
 * The truncated SVD comes from the k x k Gram matrix X_c X_c^T (eq. svd_cov);
 * all terms are evaluated in Gram space from one pass over the patch.
 *
 *   X, n, m, ldx  as in mc_knn (any float32 matrix; need not be the kNN input)
 *   idx          [n x k] int32 neighbour lists, device; entries outside [0, n)
 *                give kappa = NaN and MC_PF_NONFINITE for that point
 *   k            2 <= k <= MC_KMAX
 *   precision    MC_FP32 | MC_BF16 | MC_FP64 (patch moments on MFMA; the
 *                combination is float64 in all three; the k x k eigen-solve is
 *                float32 Jacobi for MC_FP32 and MC_BF16, redone in float64 when a
 *                kept eigenvalue pair is near-degenerate (flag MC_PF_EIGEN_FP64),
 *                and float64 Jacobi for MC_FP64).  MC_BF16 at k >= 13 forms the Gram
 *                matrix and V_r^T from split bf16 products (x = hi + lo) and runs the
 *                third-moment GEMM on binary16 operands (patch rows scaled by powers of
 *                two, packed binary16 pair products), float32 accumulation throughout;
 *                at k <= 12 it takes bf16 operands with a float32 Gram.  MC_FP64 centres
 *                and accumulates in float64 (v_mfma_f64_16x16x4f64): use it for
 *                thin or noisy patches whose Gram matrix is ill-conditioned, where
 *                float32 moments lose digits.  k > MC_FAST_FP64_KMAX -> MC_ESHAPE.
 *                A point is flagged MC_PF_PRECISION_LIMIT when 2 u cond / max(q, 1) exceeds
 *                the path's error budget, with cond = sigma_1 / sigma_pe of the Gram matrix,
 *                q = m - pe, u = 2^-24 for MC_FP32 and for MC_BF16 at k <= 12 (float32
 *                Gram), 3 * 2^-16 for MC_BF16 at k >= 13 (Gram from split bf16 products,
 *                x = hi + lo), 2^-53 for MC_FP64, and budgets 1e-4, 2e-2 and 1e-6: the
 *                moments' rounding turns the weakest kept direction by about u cond
 *                towards the null space, whose term spreads that over its q directions.
 *                MC_BF16 moments on rows narrower than 256 flag every point
 *                MC_PF_PRECISION_LIMIT (their 8-bit products exceed the 2e-2 budget on
 *                strongly curved patches there)
 *   variant      MC_FAST_PAPER | MC_FAST_HAAR
 *   kappa_out    [n] float32, device, written
 *   flags_out    [n] uint8 (MC_PF_* bits), or NULL
 *   flags        0 | MC_STRICT
 */
int mc_curvature_fast(const float* X, int64_t n, int64_t m, int64_t ldx, const int32_t* idx,
                      int32_t k, int32_t precision, int32_t variant, uint32_t flags,
                      float* kappa_out, uint8_t* flags_out, void* ws, size_t ws_bytes,
                      void* stream);

/*
 * mc_curvature_exact -- Theorem 1 (eq. kappa_final) for every point with
 * W = [V_r | Q_null], where Q_null is the canonical completion of V_r: the
 * trailing m - p_eff columns of the Householder QR of V_r (LAPACK reflector
 * convention beta = -sign(alpha) ||x||).  The paper's Exact branch uses
 * whatever null basis its eigensolver returns; because only columns with a
 * non-zero eigenvalue are weighted, kappa depends on that choice whenever
 * m > rank, and this ABI fixes it so results are reproducible.
 *
 * Arguments as mc_curvature_fast without `variant`; precision MC_FP32 only.
 * V_r (float64), the gathered rows (float32) and the column means (float64) are
 * held on chip: m * (8 (k-1) + 4 k + 8) bytes plus about 16 KiB of per-point state
 * must stay within 150 KiB (e.g. m <= 1038 at k = 11), else MC_ESHAPE.  Centring,
 * moments and the eigen-solve run in float64.
 */
int mc_curvature_exact(const float* X, int64_t n, int64_t m, int64_t ldx, const int32_t* idx,
                       int32_t k, int32_t precision, uint32_t flags, float* kappa_out,
                       uint8_t* flags_out, void* ws, size_t ws_bytes, void* stream);

/*
 * mc_curvature_backward -- adjoint of mc_curvature_fast (MC_FP32 path):
 * grad_X += d(sum_i grad_kappa[i] * kappa_i)/dX with the neighbour lists held
 * fixed.  The derivative of the eigenvectors of the Gram matrix uses
 * regularised gap factors Delta/(Delta^2 + eta^2), eta = gap_eps * sigma_1;
 * gap_eps = 0 gives the exact derivative.  The patch moments, the eigen-solve
 * and the adjoint algebra run in float64 (thin patches cancel strongly); only
 * the scatter-add into grad_X is float32.
 *
 *   grad_kappa   [n] float32, device
 *   grad_X       [n x ldx] float32, device, ACCUMULATED into (atomic adds, so the
 *                summation order, and the last bits, vary from run to run)
 *   k            2 <= k <= 16 (MC_ESHAPE above)
 * Points whose patch is degenerate (tau = 0) or non-finite contribute nothing.
 */
int mc_curvature_backward(const float* X, int64_t n, int64_t m, int64_t ldx, const int32_t* idx,
                          int32_t k, int32_t variant, const float* grad_kappa, float gap_eps,
                          float* grad_X, void* ws, size_t ws_bytes, void* stream);

/*
 * mc_normalize_minmax -- out[i] = (kappa[i] - min) / (max - min), min and max over the finite
 * scores of all n points: the per-dataset normalisation to [0, 1] of the paper's
 * normalised-score experiment (Table 3), which keeps the ranking and removes the scale.
 *
 *   kappa        [n] float32 scores, device (e.g. mc_curvature_fast's output)
 *   out          [n] float32, device, written (may alias kappa): non-finite scores give NaN,
 *                a constant score vector gives 0, no finite score at all gives NaN everywhere
 *   ws, ws_bytes workspace, >= mc_workspace_bytes(MC_OP_NORMALIZE, n, ...)
 * The division is IEEE float32, so the result equals (k - min) / (max - min) evaluated in
 * float32 on the host.
 */
int mc_normalize_minmax(const float* kappa, int64_t n, float* out, void* ws, size_t ws_bytes, void* stream);

/*
 * mc_curvature_fast_noalloc -- mc_curvature_fast without a workspace argument, for callers
 * that cannot allocate device memory (code under HIP graph capture, serving loops, harnesses
 * that forbid allocation).  Arguments and results are those of mc_curvature_fast.
 *
 * The per-point state that the two-pass form (k >= 13) keeps between its kernels goes to a
 * static device array of MC_NOALLOC_SCRATCH_BYTES inside the library instead (each GPU the
 * library runs on holds its own copy until the process ends; its address is taken on the
 * first call on that device).  The call allocates nothing.  Sizes whose state exceeds the
 * array (mc_workspace_bytes(MC_OP_FAST, ...) > MC_NOALLOC_SCRATCH_BYTES: n above about 7900
 * at k = 32 with float32 moments, about 28000 at k = 16) return MC_ESCRATCH and enqueue
 * nothing; k <= 12 needs no state and takes any n.  All calls on one GPU share its array:
 * calls that overlap in time on one GPU (different streams or threads) race and must be
 * serialised by the caller.
 */
#define MC_NOALLOC_SCRATCH_BYTES (64u << 20)
int mc_curvature_fast_noalloc(const float* X, int64_t n, int64_t m, int64_t ldx, const int32_t* idx,
                              int32_t k, int32_t precision, int32_t variant, uint32_t flags,
                              float* kappa_out, uint8_t* flags_out, void* stream);

/*
 * Stage timers (instrumentation, off by default).  While enabled, every kernel
 * the library launches is bracketed by a pair of hipEvents recorded on the
 * stream it is launched on.  mc_timing_read synchronises those events, returns
 * the summed duration (ms) and launch count of one stage since the last read
 * of that stage, and resets it.  Stages are numbered 0 .. MC_STAGE_COUNT-1.
 */
#define MC_STAGE_KNN_COLSUM 0
#define MC_STAGE_KNN_MEAN 1
#define MC_STAGE_KNN_CENTER 2
#define MC_STAGE_KNN_STATS 3
#define MC_STAGE_KNN_GEMM_TOPK 4
#define MC_STAGE_KNN_RERANK 5
#define MC_STAGE_CURV_FAST 6
#define MC_STAGE_CURV_EXACT 7
#define MC_STAGE_CURV_BACKWARD 8
#define MC_STAGE_KNN_COLUMN_TOPK 9
#define MC_STAGE_KNN_RESCAN 10
#define MC_STAGE_CURV_GRAM 11   /* Fast mode, k >= 13: the three kernels of the two-pass form */
#define MC_STAGE_CURV_EIGEN 12  /*   (k <= 12: MC_STAGE_CURV_FAST, one fused kernel) */
#define MC_STAGE_CURV_RANGE 13
#define MC_STAGE_COUNT 14
int mc_timing_enable(int on);
int mc_timing_read(int32_t stage, double* total_ms, int64_t* launches);
const char* mc_stage_name(int32_t stage);

/* Workspace bytes needed by operation `op` (MC_OP_*) for these sizes; 0 if the
 * arguments are invalid or the operation does not support them (the same cases
 * in which the operation itself returns MC_EINVAL, MC_ESHAPE or MC_EPRECISION),
 * so a 0 doubles as the support query. */
size_t mc_workspace_bytes(int32_t op, int64_t n, int64_t m, int32_t k, int32_t precision,
                          int32_t rerank_factor);

/* Static, NUL-terminated description of a status code. */
const char* mc_status_string(int status);

/* MC_VERSION of the loaded library. */
int mc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MECUCO_H */
