// rn_filter.hip -- filter (Alg. filter; Sec. 3.5 pre-filtering of the
// pattern, Sec. 3.7 post-filtering of P) on node blocks, and the compaction
// of the kept entries.
//
// The matrix G (n DOF rows, m DOFs per node) is stored on a pattern whose DOF
// rows m I .. m I + m - 1 share the node structure of node row I (DOF
// columns m a + c' of node column a).  A node entry's magnitude is the
// largest |G| of its m x m block.  The entry of the row's own aggregate
// (node column agg[I]) takes the place of the diagonal: it is kept and is
// not an off entry.  An off entry is dropped when k > 0 and at least k off
// entries of the row are strictly larger (it lies below the k-th largest),
// or when theta > 0 and it lies below theta times the largest off entry.
// Rows of root nodes are kept whole.  Integer decisions on FP64 magnitudes:
// the same comparisons, in the same precision, as any evaluation of the
// definition, so the kept pattern is exact.
#include <climits>
#include <cstring>

#include "rn_internal.h"

// Block magnitude of node entry q of node row I (DOF rows i0 .. i0 + m - 1).
template <int M>
__device__ inline double blk_mag(const int32_t *__restrict__ Np, const double *__restrict__ G, int i0, int q) {
  double v = 0.0;
#pragma unroll
  for (int c = 0; c < M; ++c) {
    const int64_t base = (int64_t)Np[i0 + c] + (int64_t)M * q;
#pragma unroll
    for (int cc = 0; cc < M; ++cc) v = fmax(v, fabs(G[base + cc]));
  }
  return v;
}

// One lane per stored DOF entry: keep[e] = 1 when the entry survives.
template <int M>
__global__ __launch_bounds__(RN_BLOCK) void k_filter_mark(int32_t n, int64_t nnz, const int32_t *__restrict__ Np,
                                                         const int32_t *__restrict__ Nj,
                                                         const double *__restrict__ G,
                                                         const uint8_t *__restrict__ is_root,
                                                         const int32_t *__restrict__ agg, int32_t k, double theta,
                                                         uint8_t *__restrict__ keep,
                                                         const int32_t *__restrict__ guard) {
  const int64_t e = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x;
  if (e >= nnz || *guard) return;
  // the row holding e: last i with Np[i] <= e
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)Np[mid] <= e) lo = mid; else hi = mid;
  }
  const int i = lo, I = i / M, i0 = M * I;
  bool root = false;
  if (is_root)
#pragma unroll
    for (int c = 0; c < M; ++c) root = root || is_root[i0 + c] != 0;
  const int q = (int)(e - Np[i]) / M;
  const int own = agg[I];
  if (root || Nj[(int64_t)Np[i0] + (int64_t)M * q] / M == own) {
    keep[e] = 1;
    return;
  }
  const double g = blk_mag<M>(Np, G, i0, q);
  const int len = (Np[i0 + 1] - Np[i0]) / M;
  double offmax = 0.0;
  int greater = 0;
  for (int t = 0; t < len; ++t) {
    if (Nj[(int64_t)Np[i0] + (int64_t)M * t] / M == own) continue;
    const double v = blk_mag<M>(Np, G, i0, t);
    offmax = fmax(offmax, v);
    greater += v > g;
  }
  bool kp = true;
  if (k > 0 && greater >= k) kp = false;
  if (theta > 0.0 && g < theta * offmax) kp = false;
  keep[e] = kp ? 1 : 0;
}

// Node-blocked input: the DOF rows of a node that is not a root must have
// equal lengths divisible by m (they share the node structure).
__global__ __launch_bounds__(RN_BLOCK) void k_filter_check_blocks(int32_t nn, int32_t m,
                                                                 const int32_t *__restrict__ Np,
                                                                 const uint8_t *__restrict__ is_root,
                                                                 int32_t *__restrict__ guard) {
  const int I = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (I >= nn || *guard) return;
  bool root = false;
  if (is_root)
    for (int c = 0; c < m; ++c) root = root || is_root[m * I + c] != 0;
  if (root) return;
  const int l0 = Np[m * I + 1] - Np[m * I];
  bool bad = l0 % m != 0;
  for (int c = 1; c < m; ++c) bad = bad || (Np[m * I + c + 1] - Np[m * I + c]) != l0;
  if (bad) atomicOr(guard, GUARD_N);
}

__global__ __launch_bounds__(RN_BLOCK) void k_filter_count(int32_t n, const int32_t *__restrict__ Np,
                                                          const uint8_t *__restrict__ keep,
                                                          int32_t *__restrict__ cnt,
                                                          const int32_t *__restrict__ guard) {
  const int i = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (i >= n) return;
  int c = 0;
  if (!*guard)
    for (int p = Np[i]; p < Np[i + 1]; ++p) c += keep[p];
  cnt[i] = c;
}

// One lane per stored entry: kept entries move to their place in the
// compacted row (the count of kept entries before them in the row).
__global__ __launch_bounds__(RN_BLOCK) void k_filter_fill(int32_t n, int64_t nnz, const int32_t *__restrict__ Np,
                                                         const int32_t *__restrict__ Nj,
                                                         const double *__restrict__ G,
                                                         const uint8_t *__restrict__ keep,
                                                         const int32_t *__restrict__ Fp, int32_t *__restrict__ Fj,
                                                         double *__restrict__ Fv) {
  const int64_t e = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x;
  if (e >= nnz || !keep[e]) return;
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)Np[mid] <= e) lo = mid; else hi = mid;
  }
  int before = 0;
  for (int64_t p = Np[lo]; p < e; ++p) before += keep[p];
  const int64_t w = (int64_t)Fp[lo] + before;
  Fj[w] = Nj[e];
  if (Fv) Fv[w] = G[e];
}

extern "C" rn_status rn_filter(rn_ctx *ctx, int32_t n, int32_t block_m, const int32_t *N_rowptr,
                               const int32_t *N_colind, int64_t nnz_N, const uint8_t *is_root, const int32_t *agg,
                               const double *vals, int32_t k, double theta, int32_t *F_rowptr, int32_t *F_colind,
                               double *F_vals, int64_t *nnz_F) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  const int m = block_m;
  if ((m != 1 && m != 2) || n < 0 || n % m || nnz_N < 0 || k < 0 || !(theta >= 0.0) || !nnz_F)
    return rn_fail(ctx, RN_EINVAL, "rn_filter: bad argument (n %d, block_m %d, k %d, theta %g)", n, m, k, theta);
  if (nnz_N >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_filter: nnz_N >= 2^31");
  if (n > 0 && (!N_rowptr || !agg || !F_rowptr)) return rn_fail(ctx, RN_EINVAL, "rn_filter: null argument");
  if (nnz_N > 0 && (!N_colind || !vals)) return rn_fail(ctx, RN_EINVAL, "rn_filter: null argument");
  rn_status st = RN_OK;
  uint8_t *keep = (uint8_t *)rn_scratch(ctx, SLOT_FLT_KEEP, (size_t)nnz_N + 1, &st);
  if (!keep) return st;
  if (F_colind) {  // phase 2: the kept entries of the mask phase 1 left
    if (ctx->flt_n != n || ctx->flt_nnz_in != nnz_N)
      return rn_fail(ctx, RN_EINVAL, "rn_filter: phase 2 without a matching phase 1");
    if (nnz_N > 0) {
      hipLaunchKernelGGL(k_filter_fill, dim3(rn_div_up(nnz_N, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, n, nnz_N,
                         N_rowptr, N_colind, vals, keep, F_rowptr, F_colind, F_vals);
      LAUNCH_CHECK(ctx);
    }
    *nnz_F = ctx->flt_nnz;
    ctx->flt_n = -1;
    return RN_OK;
  }
  int32_t *guard = rn_guard_begin(ctx, &st);
  if (!guard) return st;
  int32_t *cnt = (int32_t *)rn_scratch(ctx, SLOT_FLT_CNT, (size_t)(n + 1) * sizeof(int32_t), &st);
  if (!cnt) return st;
  RnChecks v{};
  v.csr[0] = {n, INT_MAX, nnz_N, N_rowptr, N_colind, GUARD_N};
  v.ncsr = 1;
  RN_TRY(rn_validate(ctx, v, guard));
  if (m > 1 && n > 0) {
    hipLaunchKernelGGL(k_filter_check_blocks, dim3(rn_div_up(n / m, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream,
                       n / m, m, N_rowptr, is_root, guard);
    LAUNCH_CHECK(ctx);
  }
  if (nnz_N > 0) {
    const dim3 g(rn_div_up(nnz_N, RN_BLOCK)), b(RN_BLOCK);
    if (m == 1)
      hipLaunchKernelGGL(k_filter_mark<1>, g, b, 0, ctx->stream, n, nnz_N, N_rowptr, N_colind, vals, is_root, agg,
                         k, theta, keep, guard);
    else
      hipLaunchKernelGGL(k_filter_mark<2>, g, b, 0, ctx->stream, n, nnz_N, N_rowptr, N_colind, vals, is_root, agg,
                         k, theta, keep, guard);
    LAUNCH_CHECK(ctx);
  }
  if (n > 0) {
    hipLaunchKernelGGL(k_filter_count, dim3(rn_div_up(n, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, n, N_rowptr,
                       keep, cnt, guard);
    LAUNCH_CHECK(ctx);
  }
  RN_TRY(rn_scan_counts(ctx, cnt, F_rowptr, n, nullptr));
  int64_t *total = (int64_t *)rn_scratch(ctx, SLOT_SCAN_TOTAL, sizeof(int64_t), &st);
  if (!total) return st;
  int64_t tot = 0;
  RN_TRY(rn_read_guard_i64(ctx, guard, total, &tot, "rn_filter"));
  ctx->flt_n = n;
  ctx->flt_nnz_in = nnz_N;
  ctx->flt_nnz = tot;
  *nnz_F = tot;
  return RN_OK;
}
