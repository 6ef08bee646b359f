// rn_pattern.hip -- strength of connection (Sec. 3.2) and the interpolation
// pattern N = S^d C with unamalgamation and root rows (Sec. 3.4).
// Integer work: results are bit-exact by construction (sorted, unique rows).
#include <cstring>
#include <climits>
#include "rn_internal.h"

// ---------------------------------------------------------------------------
// strength
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RN_BLOCK) void k_diag_csr(int n, const int32_t *__restrict__ Ap,
                                                      const int32_t *__restrict__ Aj,
                                                      const double *__restrict__ Ax, double *__restrict__ diag,
                                                      const int32_t *__restrict__ guard) {
  const int i = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (i >= n || *guard) return;
  double d = 0.0;
  for (int p = Ap[i]; p < Ap[i + 1]; ++p)
    if (Aj[p] == i) d = Ax[p];
  diag[i] = d;
}


// strong when a^2 >= theta^2 |a_ii a_jj| (rounded products, no FMA); the
// diagonal is always strong.
__device__ inline bool rn_is_strong(double a, double di, double dj, double th2, bool on_diag) {
  return on_diag || (__dmul_rn(a, a) >= __dmul_rn(th2, fabs(__dmul_rn(di, dj))));
}

__global__ __launch_bounds__(RN_BLOCK) void k_strong_csr(int n, const int32_t *__restrict__ Ap,
                                                        const int32_t *__restrict__ Aj,
                                                        const double *__restrict__ Ax,
                                                        const double *__restrict__ diag, double th2,
                                                        uint8_t *__restrict__ mask,
                                                        const int32_t *__restrict__ guard) {
  const int i = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (i >= n || *guard) return;
  const double di = diag[i];
  for (int p = Ap[i]; p < Ap[i + 1]; ++p) {
    const int j = Aj[p];
    mask[p] = rn_is_strong(Ax[p], di, diag[j], th2, i == j);
  }
}


__global__ __launch_bounds__(RN_BLOCK) void k_gather_u8(const uint8_t *__restrict__ src,
                                                       const int32_t *__restrict__ idx, int64_t n,
                                                       uint8_t *__restrict__ dst,
                                                       const int32_t *__restrict__ guard) {
  if (*guard) return;
  for (int64_t q = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; q < n; q += (int64_t)gridDim.x * RN_BLOCK)
    dst[q] = src[idx[q]];
}

// Node row I of S u S^T u {I}: a three-way merge of the strong entries of row
// I of A, of row I of A^T and of the diagonal.  FILL = false counts.
template <bool FILL>
__global__ __launch_bounds__(RN_BLOCK) void k_sym_merge(int nn, const int32_t *__restrict__ Ap,
                                                       const int32_t *__restrict__ Aj,
                                                       const uint8_t *__restrict__ mask,
                                                       const int32_t *__restrict__ Tp,
                                                       const int32_t *__restrict__ Tj,
                                                       const uint8_t *__restrict__ tmask,
                                                       int32_t *__restrict__ cnt_or_ptr,
                                                       int32_t *__restrict__ Sj,
                                                       const int32_t *__restrict__ guard) {
  const int I = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (I >= nn) return;
  if (*guard) {
    if (!FILL) cnt_or_ptr[I] = 0;
    return;
  }
  int p = Ap[I], pe = Ap[I + 1], q = Tp[I], qe = Tp[I + 1];
  const int INF = 0x7fffffff;
  bool dtodo = true;
  int last = -1, c = 0, w = FILL ? cnt_or_ptr[I] : 0;
  while (true) {
    while (p < pe && !mask[p]) ++p;
    while (q < qe && !tmask[q]) ++q;
    const int a = p < pe ? Aj[p] : INF;
    const int b = q < qe ? Tj[q] : INF;
    const int d = dtodo ? I : INF;
    const int v = min(a, min(b, d));
    if (v == INF) break;
    if (v != last) {
      if (FILL) Sj[w + c] = v;
      ++c;
      last = v;
    }
    if (a == v) ++p;
    if (b == v) ++q;
    if (d == v) dtodo = false;
  }
  if (!FILL) cnt_or_ptr[I] = c;
}

__global__ __launch_bounds__(RN_BLOCK) void k_copy_i32(const int32_t *__restrict__ src, int64_t n,
                                                      int32_t *__restrict__ dst) {
  for (int64_t q = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; q < n; q += (int64_t)gridDim.x * RN_BLOCK)
    dst[q] = src[q];
}

static unsigned grid_for(int64_t n, unsigned cap = 8192) {
  unsigned g = rn_div_up(n, RN_BLOCK);
  if (g == 0) g = 1;
  return g > cap ? cap : g;
}

// Row-wise kernels below give each row a group of SG lanes that read the
// row's entries side by side (SG consecutive entries per load instead of one
// entry of SG different rows).
#define SG 8
#define SRPB (RN_BLOCK / SG)

// diagonal of a scalar CSR matrix (0 where it is not stored)
__global__ __launch_bounds__(RN_BLOCK) void k_diag_csr_g(int n, const int32_t *__restrict__ Ap,
                                                        const int32_t *__restrict__ Aj,
                                                        const double *__restrict__ Ax, double *__restrict__ diag,
                                                        const int32_t *__restrict__ guard) {
  const int g = threadIdx.x / SG, l = threadIdx.x % SG;
  const int i = blockIdx.x * SRPB + g;
  if (i >= n || *guard) return;
  double d = 0.0;
  bool hit = false;
  for (int p = Ap[i] + l; p < Ap[i + 1]; p += SG)
    if (Aj[p] == i) {
      d = Ax[p];
      hit = true;
    }
  // a stored diagonal is unique in its (sorted, duplicate-free) row
  const unsigned long long who = __ballot(hit);
  const int base = threadIdx.x & (RN_WAVE - 1) & ~(SG - 1);
  const unsigned long long mine = (who >> base) & ((1ull << SG) - 1);
  if (l == 0 && !mine) diag[i] = 0.0;
  if (hit) diag[i] = d;
}

// diagonal of a node-blocked (2x2) matrix: both DOFs' entries of the
// diagonal block (0 where the block is not stored)
__global__ __launch_bounds__(RN_BLOCK) void k_diag_bsr(int nn, const int32_t *__restrict__ Ap,
                                                      const int32_t *__restrict__ Aj,
                                                      const double *__restrict__ Ax, double *__restrict__ diag,
                                                      const int32_t *__restrict__ guard) {
  const int I = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (I >= nn || *guard) return;
  double d0 = 0.0, d1 = 0.0;
  for (int p = Ap[I]; p < Ap[I + 1]; ++p)
    if (Aj[p] == I) {
      d0 = Ax[4 * (int64_t)p + 0];
      d1 = Ax[4 * (int64_t)p + 3];
    }
  diag[2 * I] = d0;
  diag[2 * I + 1] = d1;
}

// node-blocked strength: block (I,J) is strong when any of its four DOF
// entries is (the boolean OR of the amalgamation); the SG lanes of row I take
// its blocks side by side
__global__ __launch_bounds__(RN_BLOCK) void k_strong_bsr(int nn, const int32_t *__restrict__ Ap,
                                                        const int32_t *__restrict__ Aj,
                                                        const double *__restrict__ Ax,
                                                        const double *__restrict__ diag, double th2,
                                                        uint8_t *__restrict__ mask,
                                                        const int32_t *__restrict__ guard) {
  const int g = threadIdx.x / SG, l = threadIdx.x % SG;
  const int I = blockIdx.x * SRPB + g;
  if (I >= nn || *guard) return;
  const double di[2] = {diag[2 * I], diag[2 * I + 1]};
  for (int p = Ap[I] + l; p < Ap[I + 1]; p += SG) {
    const int J = Aj[p];
    const double *a = Ax + 4 * (int64_t)p;
    const double a4[4] = {a[0], a[1], a[2], a[3]};
    const double dj[2] = {diag[2 * J], diag[2 * J + 1]};
    bool s = false;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) s |= rn_is_strong(a4[2 * c + cc], di[c], dj[cc], th2, (2 * I + c) == (2 * J + cc));
    mask[p] = s;
  }
}

// Strong set of node row I made symmetric through A's own structure: entry
// (I,J) is kept when it or its partner (J,I) is strong.  Valid when A is
// structurally symmetric; a missing partner sets *asym (the caller then takes
// the transpose path).  cnt[I] counts the kept entries plus the diagonal when
// it is not stored.  INL: block_m = 1, the strength tested inline from A's
// values and diagonal (no mask array); otherwise the node mask of
// k_strong_bsr.
template <bool INL>
__global__ __launch_bounds__(RN_BLOCK) void k_partner_g(int nn, const int32_t *__restrict__ Ap,
                                                       const int32_t *__restrict__ Aj,
                                                       const double *__restrict__ Ax,
                                                       const double *__restrict__ diag, double th2,
                                                       const uint8_t *__restrict__ mask,
                                                       uint8_t *__restrict__ symmask, int32_t *__restrict__ cnt,
                                                       int32_t *__restrict__ asym,
                                                       const int32_t *__restrict__ guard) {
  const int g = threadIdx.x / SG, l = threadIdx.x % SG;
  const int I = blockIdx.x * SRPB + g;
  if (*guard) {
    if (I < nn && l == 0) cnt[I] = 0;
    return;
  }
  bool missing = false, hasd = false;
  int c = 0;
  if (I < nn) {
    const double di = INL ? diag[I] : 0.0;
    for (int p = Ap[I] + l; p < Ap[I + 1]; p += SG) {
      const int J = Aj[p];
      bool s;
      if (J == I) {
        hasd = true;
        s = INL ? true : mask[p];
      } else {
        const double dj = INL ? diag[J] : 0.0;
        s = INL ? rn_is_strong(Ax[p], di, dj, th2, false) : mask[p];
        int lo = Ap[J], hi = Ap[J + 1];
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (Aj[mid] < I) lo = mid + 1; else hi = mid;
        }
        if (lo < Ap[J + 1] && Aj[lo] == I) s = s || (INL ? rn_is_strong(Ax[lo], dj, di, th2, false) : mask[lo]);
        else missing = true;
      }
      symmask[p] = s;
      c += s;
    }
  }
#pragma unroll
  for (int off = SG / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, SG);
  const unsigned long long dh = __ballot(hasd);
  const int base = threadIdx.x & (RN_WAVE - 1) & ~(SG - 1);
  const bool rowd = ((dh >> base) & ((1ull << SG) - 1)) != 0;
  if (I < nn && l == 0) cnt[I] = c + (rowd ? 0 : 1);
  if (__any(missing) && (threadIdx.x & (RN_WAVE - 1)) == 0) atomicOr(asym, 1);
}

// Row I of S: the kept entries in order, the diagonal inserted before the
// first column above I when A does not store it.
__global__ __launch_bounds__(RN_BLOCK) void k_partner_fill_g(int nn, const int32_t *__restrict__ Ap,
                                                            const int32_t *__restrict__ Aj,
                                                            const uint8_t *__restrict__ symmask,
                                                            const int32_t *__restrict__ Sp,
                                                            int32_t *__restrict__ Sj,
                                                            const int32_t *__restrict__ guard) {
  if (guard && *guard) return;  // (queued before the checks were read back)
  const int g = threadIdx.x / SG, l = threadIdx.x % SG;
  const int I = blockIdx.x * SRPB + g;
  const bool ok = I < nn;
  const int s = ok ? Ap[I] : 0, e = ok ? Ap[I + 1] : 0;
  const int base = threadIdx.x & (RN_WAVE - 1) & ~(SG - 1);
  const unsigned long long gm = ((1ull << SG) - 1) << base;
  // is the diagonal stored?
  bool hd = false;
  for (int p = s + l; p < e; p += SG) hd = hd || Aj[p] == I;
  const bool rowd = (__ballot(hd) & gm) != 0;
  int w = ok ? Sp[I] : 0;
  int nless = 0;  // kept entries below the diagonal (where the missing one goes)
  for (int c0 = s; c0 < e; c0 += SG) {
    const int p = c0 + l;
    int J = 0;
    bool keep = false;
    if (p < e) {
      J = Aj[p];
      keep = symmask[p] || J == I;
    }
    const unsigned long long kb = __ballot(keep) & gm;
    const int before = __popcll(kb & ((1ull << (base + l)) - 1) & gm);
    if (keep) {
      const int ins = (!rowd && J > I) ? 1 : 0;
      Sj[w + before + ins] = J;
      if (J < I) ++nless;
    }
    w += __popcll(kb);
  }
#pragma unroll
  for (int off = SG / 2; off > 0; off >>= 1) nless += __shfl_xor(nless, off, SG);
  if (ok && !rowd && l == 0) Sj[Sp[I] + nless] = I;
}

static rn_status strength_transpose_path(rn_ctx *ctx, const rn_matrix *A, double theta, int32_t *S_rowptr,
                                         int32_t *S_colind, int64_t *nnz_S);
static rn_status strength_sym_launch(rn_ctx *ctx, const rn_matrix *A, double theta, int32_t *S_rowptr,
                                     int32_t *guard, int32_t **asym_out);

extern "C" rn_status rn_strength(rn_ctx *ctx, const rn_matrix *A, double theta, int32_t *S_rowptr,
                                 int32_t *S_colind, int64_t *nnz_S) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (!A || !S_rowptr || !nnz_S) return rn_fail(ctx, RN_EINVAL, "rn_strength: null argument");
  const int m = A->block_m;
  if ((m != 1 && m != 2) || A->n < 0 || A->n % m || A->nnz < 0 || !A->rowptr || (A->nnz && (!A->colind || !A->vals)))
    return rn_fail(ctx, RN_EINVAL, "rn_strength: bad matrix descriptor");
  if (!(theta >= 0.0)) return rn_fail(ctx, RN_EINVAL, "rn_strength: theta must be >= 0");
  if (A->nnz >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_strength: nnz >= 2^31");
  if (S_colind && ctx->str_direct) {  // phase 2, symmetric structure: fill S from the kept-entry mask
    const int nn = A->n / m;
    if (ctx->str_nnz < 0 || ctx->str_nodes != nn)
      return rn_fail(ctx, RN_EINVAL, "rn_strength: phase 2 without a matching phase 1");
    if (nn > 0) {
      hipLaunchKernelGGL(k_partner_fill_g, dim3(rn_div_up(nn, SRPB)), dim3(RN_BLOCK), 0, ctx->stream, nn, A->rowptr,
                         A->colind, (const uint8_t *)ctx->slot[SLOT_STR_TMASK].ptr, S_rowptr, S_colind,
                         (const int32_t *)nullptr);
      LAUNCH_CHECK(ctx);
    }
    *nnz_S = ctx->str_nnz;
    ctx->str_nnz = -1;
    ctx->str_direct = false;
    return RN_OK;
  }
  if (S_colind) return strength_transpose_path(ctx, A, theta, S_rowptr, S_colind, nnz_S);  // phase 2 copy
  const int nn = A->n / m;
  rn_status st = RN_OK;
  int32_t *guard = rn_guard_begin(ctx, &st);
  if (!guard) return st;
  int32_t *asym = nullptr;
  RN_TRY(strength_sym_launch(ctx, A, theta, S_rowptr, guard, &asym));
  // one synchronisation: total, guard and the structural-asymmetry flag
  const RnFetch it[3] = {{ctx->slot[SLOT_SCAN_TOTAL].ptr, sizeof(int64_t)}, {guard, 4}, {asym, 4}};
  const unsigned char *hb = nullptr;
  size_t off[3];
  RN_TRY(rn_fetch(ctx, 3, it, &hb, off));
  int64_t total = 0;
  int32_t gword = 0, hasym = 0;
  memcpy(&total, hb + off[0], 8);
  memcpy(&gword, hb + off[1], 4);
  memcpy(&hasym, hb + off[2], 4);
  RN_TRY(rn_guard_status(ctx, gword, "rn_strength"));
  if (hasym) return strength_transpose_path(ctx, A, theta, S_rowptr, nullptr, nnz_S);
  // the columns are written by phase 2 straight into the caller's array
  ctx->str_nnz = total;
  ctx->str_nodes = nn;
  ctx->str_direct = true;
  *nnz_S = total;
  return RN_OK;
}

// Phase 1 of the strength for a structurally symmetric A, queued on guard
// (not reset here): diagonal, kept-entry mask (SLOT_STR_TMASK), row sizes
// and their scan into S_rowptr; *asym_out receives the device flag set when
// an entry has no partner (A not structurally symmetric).
static rn_status strength_sym_launch(rn_ctx *ctx, const rn_matrix *A, double theta, int32_t *S_rowptr,
                                     int32_t *guard, int32_t **asym_out) {
  const int m = A->block_m;
  const int nn = A->n / m;
  const int64_t nz = A->nnz;
  rn_status st = RN_OK;
  double *diag = (double *)rn_scratch(ctx, SLOT_STR_DIAG, (size_t)(A->n + 1) * sizeof(double), &st);
  uint8_t *mask = (uint8_t *)rn_scratch(ctx, SLOT_STR_MASK, (size_t)(nz + 1), &st);
  uint8_t *symmask = (uint8_t *)rn_scratch(ctx, SLOT_STR_TMASK, (size_t)(nz + 1), &st);
  int32_t *cnt = (int32_t *)rn_scratch(ctx, SLOT_STR_CNT, (size_t)(nn + 1) * sizeof(int32_t), &st);
  int32_t *asym = guard + GS_ASYM;
  if (!diag || !mask || !symmask || !cnt) return st;
  RN_TRY(rn_validate_csr(ctx, nn, nn, nz, A->rowptr, A->colind, guard, GUARD_A));
  const double th2 = theta * theta;
  const dim3 g(rn_div_up(nn > 0 ? nn : 1, RN_BLOCK)), b(RN_BLOCK);
  const dim3 gg(rn_div_up(nn > 0 ? nn : 1, SRPB));
  if (nn > 0) {
    if (m == 1) {
      hipLaunchKernelGGL(k_diag_csr_g, gg, b, 0, ctx->stream, nn, A->rowptr, A->colind, A->vals, diag, guard);
      hipLaunchKernelGGL(k_partner_g<true>, gg, b, 0, ctx->stream, nn, A->rowptr, A->colind,
                         (const double *)A->vals, diag, th2, (const uint8_t *)nullptr, symmask, cnt, asym, guard);
    } else {
      hipLaunchKernelGGL(k_diag_bsr, g, b, 0, ctx->stream, nn, A->rowptr, A->colind, A->vals, diag, guard);
      hipLaunchKernelGGL(k_strong_bsr, gg, b, 0, ctx->stream, nn, A->rowptr, A->colind, A->vals, diag, th2, mask,
                         guard);
      hipLaunchKernelGGL(k_partner_g<false>, gg, b, 0, ctx->stream, nn, A->rowptr, A->colind,
                         (const double *)nullptr, (const double *)nullptr, th2, mask, symmask, cnt, asym, guard);
    }
    LAUNCH_CHECK(ctx);
  }
  RN_TRY(rn_scan_counts(ctx, cnt, S_rowptr, nn, nullptr));
  *asym_out = asym;
  return RN_OK;
}

// General path: S u S^T through an explicit transpose of the strong set.
static rn_status strength_transpose_path(rn_ctx *ctx, const rn_matrix *A, double theta, int32_t *S_rowptr,
                                         int32_t *S_colind, int64_t *nnz_S) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (!A || !S_rowptr || !nnz_S) return rn_fail(ctx, RN_EINVAL, "rn_strength: null argument");
  const int m = A->block_m;
  if ((m != 1 && m != 2) || A->n < 0 || A->n % m || A->nnz < 0 || !A->rowptr || (A->nnz && (!A->colind || !A->vals)))
    return rn_fail(ctx, RN_EINVAL, "rn_strength: bad matrix descriptor");
  if (!(theta >= 0.0)) return rn_fail(ctx, RN_EINVAL, "rn_strength: theta must be >= 0");
  if (A->nnz >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_strength: nnz >= 2^31");
  const int nn = A->n / m;
  if (S_colind) {  // phase 2
    if (ctx->str_nnz < 0 || ctx->str_nodes != nn)
      return rn_fail(ctx, RN_EINVAL, "rn_strength: phase 2 without a matching phase 1");
    if (ctx->str_nnz > 0)
      HIP_TRY(ctx, hipMemcpyAsync(S_colind, ctx->slot[SLOT_STR_SJ].ptr, (size_t)ctx->str_nnz * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, ctx->stream));
    *nnz_S = ctx->str_nnz;
    ctx->str_nnz = -1;
    return RN_OK;
  }
  rn_status st = RN_OK;
  const int64_t nz = A->nnz;
  double *diag = (double *)rn_scratch(ctx, SLOT_STR_DIAG, (size_t)(A->n + 1) * sizeof(double), &st);
  if (!diag) return st;
  uint8_t *mask = (uint8_t *)rn_scratch(ctx, SLOT_STR_MASK, (size_t)(nz + 1), &st);
  if (!mask) return st;
  int32_t *Tp = (int32_t *)rn_scratch(ctx, SLOT_STR_TP, (size_t)(nn + 1) * sizeof(int32_t), &st);
  if (!Tp) return st;
  int32_t *Tj = (int32_t *)rn_scratch(ctx, SLOT_STR_TJ, (size_t)(nz + 1) * sizeof(int32_t), &st);
  if (!Tj) return st;
  int32_t *Tperm = (int32_t *)rn_scratch(ctx, SLOT_STR_TPERM, (size_t)(nz + 1) * sizeof(int32_t), &st);
  if (!Tperm) return st;
  uint8_t *tmask = (uint8_t *)rn_scratch(ctx, SLOT_STR_TMASK, (size_t)(nz + 1), &st);
  if (!tmask) return st;
  int32_t *cnt = (int32_t *)rn_scratch(ctx, SLOT_STR_CNT, (size_t)(nn + 1) * sizeof(int32_t), &st);
  if (!cnt) return st;
  int32_t *guard = rn_guard_begin(ctx, &st);
  if (!guard) return st;
  RN_TRY(rn_validate_csr(ctx, nn, nn, nz, A->rowptr, A->colind, guard, GUARD_A));
  const double th2 = theta * theta;
  if (nn > 0) {
    if (m == 1) {
      hipLaunchKernelGGL(k_diag_csr, dim3(rn_div_up(nn, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, nn, A->rowptr,
                         A->colind, A->vals, diag, guard);
      LAUNCH_CHECK(ctx);
      hipLaunchKernelGGL(k_strong_csr, dim3(rn_div_up(nn, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, nn,
                         A->rowptr, A->colind, A->vals, diag, th2, mask, guard);
    } else {
      hipLaunchKernelGGL(k_diag_bsr, dim3(rn_div_up(nn, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, nn, A->rowptr,
                         A->colind, A->vals, diag, guard);
      LAUNCH_CHECK(ctx);
      hipLaunchKernelGGL(k_strong_bsr, dim3(rn_div_up(nn, SRPB)), dim3(RN_BLOCK), 0, ctx->stream, nn,
                         A->rowptr, A->colind, A->vals, diag, th2, mask, guard);
    }
    LAUNCH_CHECK(ctx);
  }
  RN_TRY(rn_transpose_structure(ctx, nn, nn, nz, A->rowptr, A->colind, Tp, Tj, Tperm, guard));
  if (nz > 0) {
    hipLaunchKernelGGL(k_gather_u8, dim3(grid_for(nz)), dim3(RN_BLOCK), 0, ctx->stream, mask, Tperm, nz, tmask, guard);
    LAUNCH_CHECK(ctx);
  }
  if (nn > 0) {
    hipLaunchKernelGGL(k_sym_merge<false>, dim3(rn_div_up(nn, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, nn,
                       A->rowptr, A->colind, mask, Tp, Tj, tmask, cnt, (int32_t *)nullptr, guard);
    LAUNCH_CHECK(ctx);
  }
  RN_TRY(rn_scan_counts(ctx, cnt, S_rowptr, nn, nullptr));
  int64_t total = 0;
  RN_TRY(rn_read_guard_i64(ctx, guard, ctx->slot[SLOT_SCAN_TOTAL].ptr, &total, "rn_strength"));
  int32_t *Sj = (int32_t *)rn_scratch(ctx, SLOT_STR_SJ, (size_t)(total + 1) * sizeof(int32_t), &st);
  if (!Sj) return st;
  if (nn > 0) {
    hipLaunchKernelGGL(k_sym_merge<true>, dim3(rn_div_up(nn, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, nn,
                       A->rowptr, A->colind, mask, Tp, Tj, tmask, S_rowptr, Sj, guard);
    LAUNCH_CHECK(ctx);
  }
  ctx->str_nnz = total;
  ctx->str_nodes = nn;
  ctx->str_direct = false;
  *nnz_S = total;
  return RN_OK;
}

// ---------------------------------------------------------------------------
// pattern expansion: X_{t+1}(I) = sorted unique union of X_t(J), J in S(I).
// A group of EG lanes owns one node row; its candidates (the concatenated
// rows X_t(J)) are staged in an LDS window of ECAP entries, deduplicated by
// first occurrence and placed by rank.  Rows with more candidates go to a
// device-side list that a second kernel works through with one block per
// row and a window of BCAP entries.
// A level is held either as CSR (row pointers) or padded: row J at J * PCAP
// with its length in a count array (level 0, C itself, is the aggregate map:
// stride 1, length 1).  Modes: EX_COUNT writes row sizes, EX_FILL the sorted
// columns of a CSR level whose row pointers are known, EX_PAD the sorted
// columns and the size of a padded level in one pass (no host round trip
// between levels); a padded row longer than PCAP raises *pflag and the
// caller redoes the expansion with CSR levels.
// ---------------------------------------------------------------------------
#define EG 8
#define ECAP 64
#define ERPB (RN_BLOCK / EG)
#define BCAP 6144
#define PCAP 64
enum { EX_COUNT = 0, EX_FILL = 1, EX_PAD = 2 };

__device__ inline void x_row(const XRows &X, int J, int64_t &s, int &len) {
  if (X.p) {
    s = X.p[J];
    len = X.p[J + 1] - (int)s;
  } else {
    s = (int64_t)J * X.stride;
    len = X.c ? X.c[J] : 1;
  }
}

template <int MODE>
__global__ __launch_bounds__(RN_BLOCK) void k_expand(int nn, const int32_t *__restrict__ Sp,
                                                    const int32_t *__restrict__ Sj, const XRows X,
                                                    int32_t *__restrict__ cnt_or_ptr,
                                                    int32_t *__restrict__ Yj, int32_t *__restrict__ ovf,
                                                    int32_t *__restrict__ ovf_n,
                                                    const int32_t *__restrict__ guard) {
  __shared__ int32_t cand[ERPB][ECAP];
  __shared__ uint8_t first[ERPB][ECAP];
  const int g = threadIdx.x / EG, l = threadIdx.x % EG;
  const int I = blockIdx.x * ERPB + g;
  if (*guard) {
    if (MODE != EX_FILL && I < nn && l == 0) cnt_or_ptr[I] = 0;
    return;
  }
  const bool ok = I < nn;
  int L = 0;
  if (ok) {
    const int s = Sp[I], e = Sp[I + 1];
    for (int c0 = s; c0 < e; c0 += EG) {
      const int p = c0 + l;
      int len = 0;
      int64_t xs = 0;
      if (p < e) x_row(X, Sj[p], xs, len);
      int inc = len;
#pragma unroll
      for (int off = 1; off < EG; off <<= 1) {
        const int t = __shfl_up(inc, off, EG);
        if (l >= off) inc += t;
      }
      const int excl = L + inc - len;
      const int tot = __shfl(inc, EG - 1, EG);
      for (int q = 0; q < len; ++q) {
        const int pos = excl + q;
        if (pos < ECAP) cand[g][pos] = X.v[xs + q];
      }
      L += tot;
    }
  }
  const int Lc = L < ECAP ? L : ECAP;
  __syncthreads();
  // Candidates spanning fewer than 64*EG values: a bitmap, one 64-bit word per
  // lane, gives the distinct values in ascending order in O(L) per lane.
  // Wider rows: first occurrences and ranks by comparison.
  int vmin = INT_MAX, vmax = -1;
  for (int c = l; c < Lc; c += EG) {
    const int v = cand[g][c];
    vmin = min(vmin, v);
    vmax = max(vmax, v);
  }
#pragma unroll
  for (int off = EG / 2; off > 0; off >>= 1) {
    vmin = min(vmin, __shfl_xor(vmin, off, EG));
    vmax = max(vmax, __shfl_xor(vmax, off, EG));
  }
  const bool bm = Lc > 0 && vmax - vmin < 64 * EG;  // the same in every lane of the row
  if (!bm) {
    for (int c = l; c < Lc; c += EG) {
      const int v = cand[g][c];
      uint8_t f = 1;
      for (int u = 0; u < c; ++u)
        if (cand[g][u] == v) { f = 0; break; }
      first[g][c] = f;
    }
  }
  __syncthreads();
  if (!ok) return;
  if (L > ECAP) {  // the large-window kernel takes the row
    if (MODE != EX_FILL && l == 0) {
      cnt_or_ptr[I] = 0;
      ovf[atomicAdd(ovf_n, 1)] = I;
    }
    return;
  }
  // (a padded row here holds at most L <= ECAP = PCAP columns)
  if (bm) {
    unsigned long long bits = 0ull;
    for (int c = 0; c < Lc; ++c) {
      const int v = cand[g][c] - vmin;
      if ((v >> 6) == l) bits |= 1ull << (v & 63);
    }
    const int cl = __popcll(bits);
    int inc = cl;
#pragma unroll
    for (int off = 1; off < EG; off <<= 1) {
      const int t = __shfl_up(inc, off, EG);
      if (l >= off) inc += t;
    }
    if (MODE != EX_FILL && l == EG - 1) cnt_or_ptr[I] = inc;
    if (MODE != EX_COUNT) {
      int64_t pos = (MODE == EX_FILL ? (int64_t)cnt_or_ptr[I] : (int64_t)I * PCAP) + inc - cl;
      while (bits) {
        const int bit = __ffsll(bits) - 1;
        bits &= bits - 1ull;
        Yj[pos++] = vmin + 64 * l + bit;
      }
    }
    return;
  }
  if (MODE != EX_FILL) {
    int mc = 0;
    for (int c = l; c < Lc; c += EG) mc += first[g][c];
#pragma unroll
    for (int off = EG / 2; off > 0; off >>= 1) mc += __shfl_xor(mc, off, EG);
    if (l == 0) cnt_or_ptr[I] = mc;
  }
  if (MODE != EX_COUNT) {
    const int64_t base = MODE == EX_FILL ? (int64_t)cnt_or_ptr[I] : (int64_t)I * PCAP;
    for (int c = l; c < Lc; c += EG) {
      if (!first[g][c]) continue;
      const int v = cand[g][c];
      int rank = 0;
      for (int u = 0; u < Lc; ++u) rank += (first[g][u] && cand[g][u] < v);
      Yj[base + rank] = v;
    }
  }
}

// The rows listed by k_expand: one block per row, grid-stride over the list
// (its length is read on the device, so no host round trip).  A row with
// more than BCAP candidates sets GUARD_LIMIT (CSR levels) or *pflag (padded
// levels, which are then redone as CSR).
template <int MODE>
__global__ __launch_bounds__(RN_BLOCK) void k_expand_big(const int32_t *__restrict__ Sp,
                                                        const int32_t *__restrict__ Sj, const XRows X,
                                                        int32_t *__restrict__ cnt_or_ptr,
                                                        int32_t *__restrict__ Yj,
                                                        const int32_t *__restrict__ ovf,
                                                        const int32_t *__restrict__ ovf_n,
                                                        int32_t *__restrict__ guard, int32_t *__restrict__ pflag) {
  __shared__ int32_t cand[BCAP];
  __shared__ uint8_t first[BCAP];
  __shared__ int s_len[RN_BLOCK];
  __shared__ int s_red[RN_BLOCK / RN_WAVE];
  const int t = threadIdx.x;
  const int nov = *ovf_n;
  for (int q = blockIdx.x; q < nov; q += gridDim.x) {
    const int I = ovf[q];
    const int s = Sp[I], e = Sp[I + 1];
    // candidates: rows of the S-neighbours, concatenated in S order
    int L = 0;
    for (int c0 = s; c0 < e; c0 += RN_BLOCK) {
      const int p = c0 + t;
      int len = 0;
      int64_t xs = 0;
      if (p < e) x_row(X, Sj[p], xs, len);
      __syncthreads();
      s_len[t] = len;
      __syncthreads();
      int excl = 0, tot = 0;  // block-wide exclusive prefix of len (small: RN_BLOCK terms)
      for (int u = 0; u < RN_BLOCK; ++u) {
        const int v = s_len[u];
        if (u < t) excl += v;
        tot += v;
      }
      for (int w = 0; w < len; ++w) {
        const int pos = L + excl + w;
        if (pos < BCAP) cand[pos] = X.v[xs + w];
      }
      L += tot;
    }
    __syncthreads();
    if (L > BCAP) {
      if (t == 0) {
        if (MODE == EX_PAD) atomicOr(pflag, 1);
        else atomicOr(guard, GUARD_LIMIT);
        if (MODE != EX_FILL) cnt_or_ptr[I] = 0;
      }
      continue;
    }
    for (int c = t; c < L; c += RN_BLOCK) {
      const int v = cand[c];
      uint8_t f = 1;
      for (int u = 0; u < c; ++u)
        if (cand[u] == v) { f = 0; break; }
      first[c] = f;
    }
    __syncthreads();
    int total = 0;
    if (MODE != EX_FILL) {
      int mc = 0;
      for (int c = t; c < L; c += RN_BLOCK) mc += first[c];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) mc += __shfl_xor(mc, off, RN_WAVE);
      if ((t & (RN_WAVE - 1)) == 0) s_red[t / RN_WAVE] = mc;
      __syncthreads();
      total = s_red[0] + s_red[1] + s_red[2] + s_red[3];
      if (t == 0) cnt_or_ptr[I] = (MODE == EX_PAD && total > PCAP) ? 0 : total;
      if (MODE == EX_PAD && total > PCAP && t == 0) atomicOr(pflag, 1);
    }
    if (MODE == EX_FILL || (MODE == EX_PAD && total <= PCAP)) {
      const int64_t base = MODE == EX_FILL ? (int64_t)cnt_or_ptr[I] : (int64_t)I * PCAP;
      for (int c = t; c < L; c += RN_BLOCK) {
        if (!first[c]) continue;
        const int v = cand[c];
        int rank = 0;
        for (int u = 0; u < L; ++u) rank += (first[u] && cand[u] < v);
        Yj[base + rank] = v;
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(RN_BLOCK) void k_iota(int n, int32_t *__restrict__ out) {
  const int i = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (i <= n) out[i] = i;
}

__global__ __launch_bounds__(RN_BLOCK) void k_dof_count(int n, int m, const XRows X, const int32_t *__restrict__ agg,
                                                       const int32_t *__restrict__ roots, int n_agg,
                                                       int32_t *__restrict__ cnt, uint8_t *__restrict__ is_root,
                                                       int32_t *__restrict__ flag,
                                                       const int32_t *__restrict__ guard) {
  const int i = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (i >= n) return;
  if (*guard) {
    cnt[i] = 0;
    is_root[i] = 0;
    return;
  }
  const int I = i / m, a = agg[I];
  if (a < 0 || a >= n_agg) {  // malformed aggregation: reported, row left empty
    atomicOr(flag, GUARD_AGG);
    cnt[i] = 0;
    is_root[i] = 0;
    return;
  }
  const bool root = roots[a] == I;
  is_root[i] = root;
  int64_t s;
  int len;
  x_row(X, I, s, len);
  cnt[i] = root ? 1 : m * len;
}

// one group of SG lanes per DOF row, the lanes over the row's node columns
__global__ __launch_bounds__(RN_BLOCK) void k_dof_fill(int n, int m, const XRows X, const int32_t *__restrict__ agg,
                                                      const int32_t *__restrict__ Np,
                                                      const uint8_t *__restrict__ is_root,
                                                      int32_t *__restrict__ Nj) {
  // runs only after phase 1 reported success, so its inputs were validated
  const int g = threadIdx.x / SG, l = threadIdx.x % SG;
  const int i = blockIdx.x * SRPB + g;
  if (i >= n) return;
  const int I = i / m, c = i % m;
  const int w = Np[i];
  if (is_root[i]) {
    if (l == 0) Nj[w] = m * agg[I] + c;
    return;
  }
  int64_t s;
  int len;
  x_row(X, I, s, len);
  for (int q = l; q < len; q += SG) {
    const int v = X.v[s + q];
    for (int cc = 0; cc < m; ++cc) Nj[w + m * q + cc] = m * v + cc;
  }
}

// padded levels unless the context's RN_OPT_PADDED_PATTERN is 0
static bool pattern_pad_on(const rn_ctx *ctx) { return ctx->opt[RN_OPT_PADDED_PATTERN] != 0; }

// Expansion with padded levels (no host round trip between levels), then the
// DOF row sizes and their scan into Np, queued on guard; *pflag_out
// receives the device flag raised when a padded row outgrew PCAP, *xout the
// final level.
static rn_status pattern_padded_launch(rn_ctx *ctx, int nn, int n, int m, const int32_t *Sp, const int32_t *Sj,
                                       const int32_t *agg, const int32_t *roots, int n_agg, int degree, int32_t *Np,
                                       uint8_t *is_root, int32_t *cnt, int32_t *ovf, int32_t *guard,
                                       int32_t **pflag_out, XRows *xout) {
  rn_status st = RN_OK;
  int32_t *pflag = guard + GS_PFLAG;
  XRows X{nullptr, agg, nullptr, 1};  // X_0 = C
  int cur = 0;
  const unsigned g = rn_div_up(nn, ERPB) ? rn_div_up(nn, ERPB) : 1;
  for (int t = 0; t < degree; ++t) {
    const size_t vb = (size_t)nn * PCAP * sizeof(int32_t) + 16;
    int32_t *Yv = (int32_t *)rn_scratch(ctx, cur ? SLOT_PAT_XJ0 : SLOT_PAT_XJ1, vb, &st);
    if (!Yv) return st;
    int32_t *Yc = (int32_t *)rn_scratch(ctx, cur ? SLOT_PAT_XP0 : SLOT_PAT_XP1, (size_t)(nn + 1) * sizeof(int32_t),
                                        &st);
    if (!Yc) return st;
    // wide-row counter of this power: a guard slot (already zero) for the
    // first GS_NPOW powers, else cleared here
    int32_t *ctr = t < GS_NPOW ? guard + GS_POW0 + t : ovf;
    if (t >= GS_NPOW) HIP_TRY(ctx, hipMemsetAsync(ovf, 0, sizeof(int32_t), ctx->stream));
    hipLaunchKernelGGL(k_expand<EX_PAD>, dim3(g), dim3(RN_BLOCK), 0, ctx->stream, nn, Sp, Sj, X, Yc, Yv, ovf + 1,
                       ctr, guard);
    hipLaunchKernelGGL(k_expand_big<EX_PAD>, dim3(256), dim3(RN_BLOCK), 0, ctx->stream, Sp, Sj, X, Yc, Yv,
                       ovf + 1, ctr, guard, pflag);
    LAUNCH_CHECK(ctx);
    X = XRows{nullptr, Yv, Yc, PCAP};
    cur ^= 1;
  }
  if (n > 0) {
    hipLaunchKernelGGL(k_dof_count, dim3(rn_div_up(n, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, n, m, X, agg,
                       roots, n_agg, cnt, is_root, guard, guard);
    LAUNCH_CHECK(ctx);
  }
  RN_TRY(rn_scan_counts(ctx, cnt, Np, n, nullptr));
  *pflag_out = pflag;
  *xout = X;
  return RN_OK;
}

// The same with its synchronisation: *ok is false when a padded row outgrew
// PCAP (nothing is published then).
static rn_status pattern_padded(rn_ctx *ctx, int nn, int n, int m, const int32_t *Sp, const int32_t *Sj,
                                const int32_t *agg, const int32_t *roots, int n_agg, int degree, int32_t *Np,
                                uint8_t *is_root, int32_t *cnt, int32_t *ovf, int32_t *guard, int64_t *total,
                                bool *ok) {
  *ok = false;
  int32_t *pflag = nullptr;
  XRows X{};
  RN_TRY(pattern_padded_launch(ctx, nn, n, m, Sp, Sj, agg, roots, n_agg, degree, Np, is_root, cnt, ovf, guard,
                               &pflag, &X));
  // one synchronisation: total, guard, padded overflow
  const RnFetch it[3] = {{ctx->slot[SLOT_SCAN_TOTAL].ptr, sizeof(int64_t)}, {guard, 4}, {pflag, 4}};
  const unsigned char *hb = nullptr;
  size_t off[3];
  RN_TRY(rn_fetch(ctx, 3, it, &hb, off));
  int32_t gword = 0, pf = 0;
  memcpy(total, hb + off[0], 8);
  memcpy(&gword, hb + off[1], 4);
  memcpy(&pf, hb + off[2], 4);
  RN_TRY(rn_guard_status(ctx, gword, "rn_pattern"));
  if (pf) return RN_OK;
  ctx->pat_x = X;
  *ok = true;
  return RN_OK;
}

extern "C" rn_status rn_pattern(rn_ctx *ctx, int32_t nn, const int32_t *Sp, const int32_t *Sj, const int32_t *agg,
                                const int32_t *roots, int32_t n_agg, int32_t degree, int32_t m, int32_t *Np,
                                int32_t *Nj, uint8_t *is_root, int64_t *nnz_N) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (!nnz_N || !Np || (nn > 0 && (!Sp || !Sj || !agg || !is_root)) || (n_agg > 0 && !roots))
    return rn_fail(ctx, RN_EINVAL, "rn_pattern: null argument");
  if (nn < 0 || n_agg < 0 || degree < 0 || (m != 1 && m != 2))
    return rn_fail(ctx, RN_EINVAL, "rn_pattern: bad size (n_nodes %d, n_agg %d, degree %d, m %d)", nn, n_agg,
                   degree, m);
  if ((int64_t)nn * m >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_pattern: rows >= 2^31");
  const int n = nn * m;
  if (Nj) {  // phase 2
    if (ctx->pat_nnz < 0 || ctx->pat_n != n || ctx->pat_m != m)
      return rn_fail(ctx, RN_EINVAL, "rn_pattern: phase 2 without a matching phase 1");
    XRows X = ctx->pat_x;
    if (!X.p && !X.c) X.v = agg;  // degree 0 on padded levels: the aggregate map itself
    if (n > 0) {
      hipLaunchKernelGGL(k_dof_fill, dim3(rn_div_up(n, SRPB)), dim3(RN_BLOCK), 0, ctx->stream, n, m, X, agg, Np,
                         is_root, Nj);
      LAUNCH_CHECK(ctx);
    }
    *nnz_N = ctx->pat_nnz;
    ctx->pat_nnz = -1;
    return RN_OK;
  }
  rn_status st = RN_OK;
  int32_t *cnt = (int32_t *)rn_scratch(ctx, SLOT_PAT_CNT, (size_t)(n + 1) * sizeof(int32_t), &st);
  if (!cnt) return st;
  // rows with more than ECAP candidates: [0] = count, [1..] = node rows
  int32_t *ovf = (int32_t *)rn_scratch(ctx, SLOT_PAT_OVF, (size_t)(nn + 2) * sizeof(int32_t), &st);
  if (!ovf) return st;
  int32_t *guard = rn_guard_begin(ctx, &st);
  if (!guard) return st;
  // S is validated against its own last row pointer (nnz = -1)
  {
    RnChecks v{};
    v.csr[0] = {nn, nn, -1, Sp, Sj, GUARD_S};
    v.ncsr = 1;
    v.range[0] = {nn, agg, 0, n_agg, GUARD_AGG};
    v.range[1] = {n_agg, roots, 0, nn, GUARD_ROOTS};
    v.nrange = 2;
    RN_TRY(rn_validate(ctx, v, guard));
  }
  int64_t total = 0;
  if ((int64_t)nn * PCAP < ((int64_t)1 << 31) && pattern_pad_on(ctx)) {
    bool ok = false;
    RN_TRY(pattern_padded(ctx, nn, n, m, Sp, Sj, agg, roots, n_agg, degree, Np, is_root, cnt, ovf, guard, &total,
                          &ok));
    if (ok) {
      if (total >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_pattern: pattern nnz reaches 2^31");
      ctx->pat_nnz = total;
      ctx->pat_n = n;
      ctx->pat_m = m;
      *nnz_N = total;
      return RN_OK;
    }
  }
  // CSR levels: each level's row sizes, a scan and a host round trip for its
  // length, then its columns
  int cur = 0;
  {
    int32_t *Xp = (int32_t *)rn_scratch(ctx, SLOT_PAT_XP0, (size_t)(nn + 1) * sizeof(int32_t), &st);
    if (!Xp) return st;
    int32_t *Xj = (int32_t *)rn_scratch(ctx, SLOT_PAT_XJ0, (size_t)(nn + 1) * sizeof(int32_t), &st);
    if (!Xj) return st;
    hipLaunchKernelGGL(k_iota, dim3(rn_div_up(nn + 1, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, nn, Xp);
    LAUNCH_CHECK(ctx);
    if (nn > 0) {
      hipLaunchKernelGGL(k_copy_i32, dim3(grid_for(nn)), dim3(RN_BLOCK), 0, ctx->stream, agg, (int64_t)nn, Xj);
      LAUNCH_CHECK(ctx);
    }
  }
  for (int t = 0; t < degree; ++t) {
    const XRows X{(const int32_t *)ctx->slot[cur ? SLOT_PAT_XP1 : SLOT_PAT_XP0].ptr,
                  (const int32_t *)ctx->slot[cur ? SLOT_PAT_XJ1 : SLOT_PAT_XJ0].ptr, nullptr, 0};
    int32_t *Yp = (int32_t *)rn_scratch(ctx, cur ? SLOT_PAT_XP0 : SLOT_PAT_XP1, (size_t)(nn + 1) * sizeof(int32_t),
                                        &st);
    if (!Yp) return st;
    const unsigned g = rn_div_up(nn, ERPB) ? rn_div_up(nn, ERPB) : 1;
    const unsigned gb = 256;
    HIP_TRY(ctx, hipMemsetAsync(ovf, 0, sizeof(int32_t), ctx->stream));
    hipLaunchKernelGGL(k_expand<EX_COUNT>, dim3(g), dim3(RN_BLOCK), 0, ctx->stream, nn, Sp, Sj, X, cnt,
                       (int32_t *)nullptr, ovf + 1, ovf, guard);
    hipLaunchKernelGGL(k_expand_big<EX_COUNT>, dim3(gb), dim3(RN_BLOCK), 0, ctx->stream, Sp, Sj, X, cnt,
                       (int32_t *)nullptr, ovf + 1, ovf, guard, (int32_t *)nullptr);
    LAUNCH_CHECK(ctx);
    RN_TRY(rn_scan_counts(ctx, cnt, Yp, nn, nullptr));
    int64_t lt = 0;
    st = rn_read_guard_i64(ctx, guard, ctx->slot[SLOT_SCAN_TOTAL].ptr, &lt, "rn_pattern");
    if (st == RN_ELIMIT)
      return rn_fail(ctx, RN_ELIMIT, "rn_pattern: a node row gathers more than %d candidates in step %d", BCAP,
                     t + 1);
    RN_TRY(st);
    if (lt >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_pattern: nodal pattern reaches 2^31");
    int32_t *Yj = (int32_t *)rn_scratch(ctx, cur ? SLOT_PAT_XJ0 : SLOT_PAT_XJ1, (size_t)(lt + 1) * sizeof(int32_t),
                                        &st);
    if (!Yj) return st;
    hipLaunchKernelGGL(k_expand<EX_FILL>, dim3(g), dim3(RN_BLOCK), 0, ctx->stream, nn, Sp, Sj, X, Yp, Yj, ovf + 1,
                       ovf, guard);
    hipLaunchKernelGGL(k_expand_big<EX_FILL>, dim3(gb), dim3(RN_BLOCK), 0, ctx->stream, Sp, Sj, X, Yp, Yj, ovf + 1,
                       ovf, guard, (int32_t *)nullptr);
    LAUNCH_CHECK(ctx);
    cur ^= 1;
  }
  const XRows X{(const int32_t *)ctx->slot[cur ? SLOT_PAT_XP1 : SLOT_PAT_XP0].ptr,
                (const int32_t *)ctx->slot[cur ? SLOT_PAT_XJ1 : SLOT_PAT_XJ0].ptr, nullptr, 0};
  if (n > 0) {
    hipLaunchKernelGGL(k_dof_count, dim3(rn_div_up(n, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, n, m, X, agg,
                       roots, n_agg, cnt, is_root, guard, guard);
    LAUNCH_CHECK(ctx);
  }
  RN_TRY(rn_scan_counts(ctx, cnt, Np, n, nullptr));
  RN_TRY(rn_read_guard_i64(ctx, guard, ctx->slot[SLOT_SCAN_TOTAL].ptr, &total, "rn_pattern"));
  if (total >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_pattern: pattern nnz reaches 2^31");
  ctx->pat_nnz = total;
  ctx->pat_n = n;
  ctx->pat_m = m;
  ctx->pat_x = X;
  *nnz_N = total;
  return RN_OK;
}

// Strength and phase 1 of the pattern with one synchronisation (for
// rn_setup): the strength assumes a structurally symmetric A and fills S
// into Sj (room for nnz(A) + n/block_m entries) before its checks are read
// back, then the pattern expands with padded levels.  *done is false when A
// turned out not to be structurally symmetric or a padded row outgrew its
// room: the caller then runs rn_strength and rn_pattern.  With *done true,
// S is complete, Np / is_root hold the pattern's phase 1 and rn_pattern's
// phase 2 fills N's columns.
rn_status rn_strength_pattern(rn_ctx *ctx, const rn_matrix *A, double theta, int32_t *Sp, int32_t *Sj,
                              const int32_t *agg, const int32_t *roots, int32_t n_agg, int32_t degree, int32_t *Np,
                              uint8_t *is_root, int64_t *nnz_S, int64_t *nnz_N, bool *done) {
  *done = false;
  const int m = A->block_m;
  if ((m != 1 && m != 2) || A->n < 0 || A->n % m || A->nnz < 0 || !A->rowptr || (A->nnz && (!A->colind || !A->vals)))
    return rn_fail(ctx, RN_EINVAL, "rn_strength: bad matrix descriptor");
  if (!(theta >= 0.0)) return rn_fail(ctx, RN_EINVAL, "rn_strength: theta must be >= 0");
  if (A->nnz >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_strength: nnz >= 2^31");
  const int nn = A->n / m, n = A->n;
  if (n_agg < 0 || degree < 0) return rn_fail(ctx, RN_EINVAL, "rn_pattern: bad size");
  if ((int64_t)nn * PCAP >= ((int64_t)1 << 31) || !pattern_pad_on(ctx)) return RN_OK;
  rn_status st = RN_OK;
  int32_t *cnt = (int32_t *)rn_scratch(ctx, SLOT_PAT_CNT, (size_t)(n + 1) * sizeof(int32_t), &st);
  int32_t *ovf = (int32_t *)rn_scratch(ctx, SLOT_PAT_OVF, (size_t)(nn + 2) * sizeof(int32_t), &st);
  if (!cnt || !ovf) return st;
  int32_t *guard = rn_guard_begin(ctx, &st);
  if (!guard) return st;
  int32_t *asym = nullptr;
  RN_TRY(strength_sym_launch(ctx, A, theta, Sp, guard, &asym));
  if (nn > 0) {
    hipLaunchKernelGGL(k_partner_fill_g, dim3(rn_div_up(nn, SRPB)), dim3(RN_BLOCK), 0, ctx->stream, nn, A->rowptr,
                       A->colind, (const uint8_t *)ctx->slot[SLOT_STR_TMASK].ptr, Sp, Sj, guard);
    LAUNCH_CHECK(ctx);
  }
  {
    RnChecks v{};
    v.range[0] = {nn, agg, 0, n_agg, GUARD_AGG};
    v.range[1] = {n_agg, roots, 0, nn, GUARD_ROOTS};
    v.nrange = 2;
    RN_TRY(rn_validate(ctx, v, guard));
  }
  int32_t *pflag = nullptr;
  XRows X{};
  RN_TRY(pattern_padded_launch(ctx, nn, n, m, Sp, Sj, agg, roots, n_agg, degree, Np, is_root, cnt, ovf, guard,
                               &pflag, &X));
  // one synchronisation: nnz(S), guard, asymmetry, nnz(N), padded overflow
  const RnFetch it[5] = {{Sp + nn, 4}, {guard, 4}, {asym, 4}, {ctx->slot[SLOT_SCAN_TOTAL].ptr, 8}, {pflag, 4}};
  const unsigned char *hb = nullptr;
  size_t off[5];
  RN_TRY(rn_fetch(ctx, 5, it, &hb, off));
  int32_t ns = 0, gword = 0, hasym = 0, pf = 0;
  int64_t total = 0;
  memcpy(&ns, hb + off[0], 4);
  memcpy(&gword, hb + off[1], 4);
  memcpy(&hasym, hb + off[2], 4);
  memcpy(&total, hb + off[3], 8);
  memcpy(&pf, hb + off[4], 4);
  RN_TRY(rn_guard_status(ctx, gword, "rn_setup (strength, pattern)"));
  if (hasym || pf) return RN_OK;
  if (total >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_pattern: pattern nnz reaches 2^31");
  ctx->pat_nnz = total;
  ctx->pat_n = n;
  ctx->pat_m = m;
  ctx->pat_x = X;
  *nnz_S = ns;
  *nnz_N = total;
  *done = true;
  return RN_OK;
}

// ---------------------------------------------------------------------------
// strength values (Eq. soc) and the DOF pattern of a given nodal pattern
// ---------------------------------------------------------------------------
// position of column c in the sorted row [s, e) of Aj, or -1
__device__ inline int find_sorted(const int32_t *__restrict__ Aj, int s, int e, int c) {
  int a = s, b = e;
  while (a < b) {
    const int mid = (a + b) >> 1;
    if (Aj[mid] < c) a = mid + 1; else b = mid;
  }
  return (a < e && Aj[a] == c) ? a : -1;
}

// One lane per entry (I, J) of S: the largest |a| over the strong DOF
// entries of blocks (I, J) and (J, I) of A (M x M blocks, row-major); the
// diagonal entry gets 1.  Rows are normalised by k_sval_norm.
template <int M>
__global__ __launch_bounds__(RN_BLOCK) void k_sval(int32_t nn, int64_t nnzS, const int32_t *__restrict__ Sp,
                                                  const int32_t *__restrict__ Sj, const int32_t *__restrict__ Ap,
                                                  const int32_t *__restrict__ Aj, const double *__restrict__ Ax,
                                                  const double *__restrict__ diag, double th2,
                                                  double *__restrict__ Sv, const int32_t *__restrict__ guard) {
  const int64_t e = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x;
  if (e >= nnzS || *guard) return;
  int lo = 0, hi = nn;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)Sp[mid] <= e) lo = mid; else hi = mid;
  }
  const int I = lo, J = Sj[e];
  if (I == J) {
    Sv[e] = 1.0;
    return;
  }
  double v = 0.0;
  const int p = find_sorted(Aj, Ap[I], Ap[I + 1], J);
  if (p >= 0)
#pragma unroll
    for (int r = 0; r < M; ++r)
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const double a = Ax[(int64_t)p * M * M + r * M + c];
        if (rn_is_strong(a, diag[M * I + r], diag[M * J + c], th2, false)) v = fmax(v, fabs(a));
      }
  const int q = find_sorted(Aj, Ap[J], Ap[J + 1], I);
  if (q >= 0)
#pragma unroll
    for (int r = 0; r < M; ++r)
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const double a = Ax[(int64_t)q * M * M + r * M + c];
        if (rn_is_strong(a, diag[M * J + r], diag[M * I + c], th2, false)) v = fmax(v, fabs(a));
      }
  Sv[e] = v;
}

// Eq. soc: each row divided by its largest off-diagonal value (rows whose off
// values are all 0 keep them), diagonal 1.
__global__ __launch_bounds__(RN_BLOCK) void k_sval_norm(int32_t nn, const int32_t *__restrict__ Sp,
                                                       const int32_t *__restrict__ Sj, double *__restrict__ Sv,
                                                       const int32_t *__restrict__ guard) {
  const int I = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (I >= nn || *guard) return;
  double mx = 0.0;
  for (int q = Sp[I]; q < Sp[I + 1]; ++q)
    if (Sj[q] != I) mx = fmax(mx, Sv[q]);
  for (int q = Sp[I]; q < Sp[I + 1]; ++q)
    if (Sj[q] != I && mx > 0.0) Sv[q] = Sv[q] / mx;
}

extern "C" rn_status rn_strength_values(rn_ctx *ctx, const rn_matrix *A, double theta, const int32_t *S_rowptr,
                                        const int32_t *S_colind, int64_t nnz_S, double *S_vals) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (!A || !S_rowptr) return rn_fail(ctx, RN_EINVAL, "rn_strength_values: null argument");
  const int m = A->block_m;
  if ((m != 1 && m != 2) || A->n < 0 || A->n % m || A->nnz < 0 || !A->rowptr || (A->nnz && (!A->colind || !A->vals)))
    return rn_fail(ctx, RN_EINVAL, "rn_strength_values: bad matrix descriptor");
  if (!(theta >= 0.0) || nnz_S < 0 || (nnz_S > 0 && (!S_colind || !S_vals)))
    return rn_fail(ctx, RN_EINVAL, "rn_strength_values: bad argument");
  if (A->nnz >= ((int64_t)1 << 31) || nnz_S >= ((int64_t)1 << 31))
    return rn_fail(ctx, RN_ELIMIT, "rn_strength_values: 2^31 entries or more");
  const int nn = A->n / m;
  rn_status st = RN_OK;
  int32_t *guard = rn_guard_begin(ctx, &st);
  if (!guard) return st;
  double *diag = (double *)rn_scratch(ctx, SLOT_STR_DIAG, (size_t)(A->n + 1) * sizeof(double), &st);
  if (!diag) return st;
  RnChecks v{};
  v.csr[0] = {nn, nn, A->nnz, A->rowptr, A->colind, GUARD_A};
  v.csr[1] = {nn, nn, nnz_S, S_rowptr, S_colind, GUARD_S};
  v.ncsr = 2;
  RN_TRY(rn_validate(ctx, v, guard));
  if (nn > 0) {
    if (m == 1)
      hipLaunchKernelGGL(k_diag_csr, dim3(rn_div_up(nn, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, nn, A->rowptr,
                         A->colind, A->vals, diag, guard);
    else
      hipLaunchKernelGGL(k_diag_bsr, dim3(rn_div_up(nn, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, nn, A->rowptr,
                         A->colind, A->vals, diag, guard);
    LAUNCH_CHECK(ctx);
  }
  const double th2 = theta * theta;
  if (nnz_S > 0) {
    const dim3 g(rn_div_up(nnz_S, RN_BLOCK)), b(RN_BLOCK);
    if (m == 1)
      hipLaunchKernelGGL(k_sval<1>, g, b, 0, ctx->stream, nn, nnz_S, S_rowptr, S_colind, A->rowptr, A->colind,
                         A->vals, diag, th2, S_vals, guard);
    else
      hipLaunchKernelGGL(k_sval<2>, g, b, 0, ctx->stream, nn, nnz_S, S_rowptr, S_colind, A->rowptr, A->colind,
                         A->vals, diag, th2, S_vals, guard);
    LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_sval_norm, dim3(rn_div_up(nn, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, nn, S_rowptr,
                       S_colind, S_vals, guard);
    LAUNCH_CHECK(ctx);
  }
  return rn_check_guard(ctx, guard, "rn_strength_values");
}

extern "C" rn_status rn_pattern_dofs(rn_ctx *ctx, int32_t nn, const int32_t *Nn_rowptr, const int32_t *Nn_colind,
                                     int64_t nnz_Nn, const int32_t *agg, const int32_t *roots, int32_t n_agg,
                                     int32_t m, int32_t *N_rowptr, int32_t *N_colind, uint8_t *is_root,
                                     int64_t *nnz_N) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (!nnz_N || !N_rowptr || (nn > 0 && (!Nn_rowptr || !agg || !is_root)) || (n_agg > 0 && !roots) ||
      (nnz_Nn > 0 && !Nn_colind))
    return rn_fail(ctx, RN_EINVAL, "rn_pattern_dofs: null argument");
  if (nn < 0 || n_agg < 0 || nnz_Nn < 0 || (m != 1 && m != 2))
    return rn_fail(ctx, RN_EINVAL, "rn_pattern_dofs: bad size (n_nodes %d, n_agg %d, m %d)", nn, n_agg, m);
  if ((int64_t)nn * m >= ((int64_t)1 << 31) || nnz_Nn >= ((int64_t)1 << 31))
    return rn_fail(ctx, RN_ELIMIT, "rn_pattern_dofs: 2^31 rows or entries");
  const int n = nn * m;
  XRows X{Nn_rowptr, Nn_colind, nullptr, 0};
  if (N_colind) {  // phase 2
    if (ctx->pat_nnz < 0 || ctx->pat_n != n || ctx->pat_m != m)
      return rn_fail(ctx, RN_EINVAL, "rn_pattern_dofs: phase 2 without a matching phase 1");
    if (n > 0) {
      hipLaunchKernelGGL(k_dof_fill, dim3(rn_div_up(n, SRPB)), dim3(RN_BLOCK), 0, ctx->stream, n, m, X, agg,
                         N_rowptr, is_root, N_colind);
      LAUNCH_CHECK(ctx);
    }
    *nnz_N = ctx->pat_nnz;
    ctx->pat_nnz = -1;
    return RN_OK;
  }
  rn_status st = RN_OK;
  int32_t *cnt = (int32_t *)rn_scratch(ctx, SLOT_PAT_CNT, (size_t)(n + 1) * sizeof(int32_t), &st);
  if (!cnt) return st;
  int32_t *guard = rn_guard_begin(ctx, &st);
  if (!guard) return st;
  RnChecks v{};
  v.csr[0] = {nn, n_agg, nnz_Nn, Nn_rowptr, Nn_colind, GUARD_N};
  v.ncsr = 1;
  v.range[0] = {nn, agg, 0, n_agg, GUARD_AGG};
  v.range[1] = {n_agg, roots, 0, nn, GUARD_ROOTS};
  v.nrange = 2;
  RN_TRY(rn_validate(ctx, v, guard));
  if (n > 0) {
    hipLaunchKernelGGL(k_dof_count, dim3(rn_div_up(n, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, n, m, X, agg, roots,
                       n_agg, cnt, is_root, guard, guard);
    LAUNCH_CHECK(ctx);
  }
  RN_TRY(rn_scan_counts(ctx, cnt, N_rowptr, n, nullptr));
  int64_t total = 0;
  RN_TRY(rn_read_guard_i64(ctx, guard, ctx->slot[SLOT_SCAN_TOTAL].ptr, &total, "rn_pattern_dofs"));
  if (total >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_pattern_dofs: pattern nnz reaches 2^31");
  ctx->pat_nnz = total;
  ctx->pat_n = n;
  ctx->pat_m = m;
  *nnz_N = total;
  return RN_OK;
}
