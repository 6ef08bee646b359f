// rn_product.hip -- general sparse product C = X Y and the Galerkin coarse
// operator A_c = R A P (Sec. 3.8, the last line of Alg. root_node_setup).
//
// Symbolic: a group of SG_G lanes per row of X merges the sorted rows of Y
// that the row selects (a k-way merge: each lane owns lists t = lane + SG_G r,
// their cursors in LDS, or for rows of more than SG_LCAP entries in a global
// array with one slot per entry of X; the group's minimum head is the next
// column, and the lists holding it advance), so a row costs one step per
// output column and needs no candidate buffer.  Numeric: one lane per output
// entry (i, j) adds X_it Y_kj over the row of X in its order (binary search
// of j in row k of Y), the order in which a row-by-row accumulation adds
// them: results are deterministic and independent of the launch shape.
#include <climits>
#include <cstring>

#include "rn_internal.h"

#define SG_G 16       // lanes per row of X
#define SG_LCAP 128   // cursors per row kept in LDS (longer rows: global slots)
#define SG_BLOCK 256

__global__ __launch_bounds__(SG_BLOCK) void k_sg_sym(int32_t rows, const int32_t *__restrict__ Xp,
                                                    const int32_t *__restrict__ Xj, const int32_t *__restrict__ Yp,
                                                    const int32_t *__restrict__ Yj, int2 *__restrict__ gcur,
                                                    int32_t *__restrict__ cnt, const int32_t *__restrict__ Cp,
                                                    int32_t *__restrict__ Cj, const int32_t *__restrict__ guard) {
  __shared__ int2 lcur[SG_BLOCK / SG_G][SG_LCAP];
  const int grp = threadIdx.x / SG_G, gl = threadIdx.x % SG_G;
  const int row = blockIdx.x * (SG_BLOCK / SG_G) + grp;
  int L = 0, s0 = 0;
  const bool active = row < rows && *guard == 0;
  if (active) {
    s0 = Xp[row];
    L = Xp[row + 1] - s0;
  }
  int2 *cur = L <= SG_LCAP ? &lcur[grp][0] : gcur + s0;
  // each lane touches only its own lists: no exchange through memory
  for (int t = gl; t < L; t += SG_G) {
    const int k = Xj[s0 + t];
    cur[t] = make_int2(Yp[k], Yp[k + 1]);
  }
  const int64_t wbase = (Cj && active) ? (int64_t)Cp[row] : 0;
  int count = 0;
  while (true) {
    int mn = INT_MAX;
    for (int t = gl; t < L; t += SG_G) {
      const int2 c = cur[t];
      if (c.x < c.y) mn = min(mn, Yj[c.x]);
    }
#pragma unroll
    for (int off = SG_G / 2; off > 0; off >>= 1) mn = min(mn, __shfl_xor(mn, off, RN_WAVE));
    if (mn == INT_MAX) break;  // uniform within the group
    if (Cj && gl == 0) Cj[wbase + count] = mn;
    ++count;
    for (int t = gl; t < L; t += SG_G) {
      const int2 c = cur[t];
      if (c.x < c.y && Yj[c.x] == mn) cur[t].x = c.x + 1;
    }
  }
  if (cnt && gl == 0 && row < rows) cnt[row] = count;
}

// One lane per entry of C: C_ij = sum over t of X_it Y_(k_t) j, in the order
// of the row of X.
__global__ __launch_bounds__(RN_BLOCK) void k_sg_num(int32_t rows, int64_t nnzC, const int32_t *__restrict__ Xp,
                                                    const int32_t *__restrict__ Xj, const double *__restrict__ Xv,
                                                    const int32_t *__restrict__ Yp, const int32_t *__restrict__ Yj,
                                                    const double *__restrict__ Yv, const int32_t *__restrict__ Cp,
                                                    const int32_t *__restrict__ Cj, double *__restrict__ Cv,
                                                    const int32_t *__restrict__ guard) {
  const int64_t e = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x;
  if (e >= nnzC || *guard) return;
  int lo = 0, hi = rows;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)Cp[mid] <= e) lo = mid; else hi = mid;
  }
  const int j = Cj[e];
  double s = 0.0;
  for (int t = Xp[lo]; t < Xp[lo + 1]; ++t) {
    const int k = Xj[t];
    int a = Yp[k], b = Yp[k + 1];
    while (a < b) {
      const int mid = (a + b) >> 1;
      if (Yj[mid] < j) a = mid + 1; else b = mid;
    }
    if (a < Yp[k + 1] && Yj[a] == j) s += Xv[t] * Yv[a];
  }
  Cv[e] = s;
}

// Scalar CSR of a node-blocked operator (2 x 2 blocks, row-major inside a
// block): DOF row 2I + r holds (2J + c, block value (r, c)) for every block
// (I, J) of node row I, in order.
__global__ __launch_bounds__(RN_BLOCK) void k_bsr2_rows(int32_t nn, const int32_t *__restrict__ Bp,
                                                       int32_t *__restrict__ cnt) {
  const int I = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (I >= nn) return;
  const int l = 2 * (Bp[I + 1] - Bp[I]);
  cnt[2 * I] = l;
  cnt[2 * I + 1] = l;
}

__global__ __launch_bounds__(RN_BLOCK) void k_bsr2_fill(int32_t nn, const int32_t *__restrict__ Bp,
                                                       const int32_t *__restrict__ Bj, const double *__restrict__ Bv,
                                                       const int32_t *__restrict__ Sp, int32_t *__restrict__ Sj,
                                                       double *__restrict__ Sv, const int32_t *__restrict__ guard) {
  const int I = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (I >= nn || *guard) return;
  for (int r = 0; r < 2; ++r) {
    int64_t w = Sp[2 * I + r];
    for (int b = Bp[I]; b < Bp[I + 1]; ++b) {
      const int J = Bj[b];
      for (int c = 0; c < 2; ++c) {
        Sj[w] = 2 * J + c;
        Sv[w] = Bv[(int64_t)b * 4 + r * 2 + c];
        ++w;
      }
    }
  }
}

// Symbolic pass of C = X Y (X with nnzX entries): counts into cnt (Cj NULL)
// or columns into Cj.
static rn_status sg_symbolic(rn_ctx *ctx, int32_t rows, int64_t nnzX, const int32_t *Xp, const int32_t *Xj,
                             const int32_t *Yp, const int32_t *Yj, int32_t *cnt, const int32_t *Cp, int32_t *Cj,
                             int32_t *guard) {
  if (rows <= 0) return RN_OK;
  rn_status st = RN_OK;
  int2 *gcur = (int2 *)rn_scratch(ctx, SLOT_PRD_CUR, (size_t)(nnzX + 1) * sizeof(int2), &st);
  if (!gcur) return st;
  hipLaunchKernelGGL(k_sg_sym, dim3(rn_div_up(rows, SG_BLOCK / SG_G)), dim3(SG_BLOCK), 0, ctx->stream, rows, Xp, Xj,
                     Yp, Yj, gcur, cnt, Cp, Cj, guard);
  LAUNCH_CHECK(ctx);
  return RN_OK;
}

static rn_status sg_numeric(rn_ctx *ctx, int32_t rows, int64_t nnzC, const int32_t *Xp, const int32_t *Xj,
                            const double *Xv, const int32_t *Yp, const int32_t *Yj, const double *Yv,
                            const int32_t *Cp, const int32_t *Cj, double *Cv, const int32_t *guard) {
  if (nnzC <= 0) return RN_OK;
  hipLaunchKernelGGL(k_sg_num, dim3(rn_div_up(nnzC, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, rows, nnzC, Xp, Xj,
                     Xv, Yp, Yj, Yv, Cp, Cj, Cv, guard);
  LAUNCH_CHECK(ctx);
  return RN_OK;
}

// Symbolic count, scan, fill and (when values are given) numeric pass of
// C = X Y into context scratch slots; returns nnz(C) after one
// synchronisation (guard read with it).
static rn_status sg_full(rn_ctx *ctx, int32_t rows, int64_t nnzX, const int32_t *Xp, const int32_t *Xj,
                         const double *Xv, const int32_t *Yp, const int32_t *Yj, const double *Yv, int slot_p,
                         int slot_j, int slot_v,
                         int32_t **Cp_out, int32_t **Cj_out, double **Cv_out, int64_t *nnz, int32_t *guard,
                         const char *what) {
  rn_status st = RN_OK;
  int32_t *Cp = (int32_t *)rn_scratch(ctx, slot_p, (size_t)(rows + 1) * sizeof(int32_t), &st);
  int32_t *cnt = (int32_t *)rn_scratch(ctx, SLOT_PRD_CNT, (size_t)(rows + 1) * sizeof(int32_t), &st);
  if (!Cp || !cnt) return st;
  RN_TRY(sg_symbolic(ctx, rows, nnzX, Xp, Xj, Yp, Yj, cnt, nullptr, nullptr, guard));
  RN_TRY(rn_scan_counts(ctx, cnt, Cp, rows, nullptr));
  int64_t *total = (int64_t *)rn_scratch(ctx, SLOT_SCAN_TOTAL, sizeof(int64_t), &st);
  if (!total) return st;
  RN_TRY(rn_read_guard_i64(ctx, guard, total, nnz, what));
  int32_t *Cj = (int32_t *)rn_scratch(ctx, slot_j, (size_t)(*nnz + 1) * sizeof(int32_t), &st);
  double *Cv = Xv ? (double *)rn_scratch(ctx, slot_v, (size_t)(*nnz + 1) * sizeof(double), &st) : nullptr;
  if (!Cj || (Xv && !Cv)) return st;
  RN_TRY(sg_symbolic(ctx, rows, nnzX, Xp, Xj, Yp, Yj, nullptr, Cp, Cj, guard));
  if (Xv) RN_TRY(sg_numeric(ctx, rows, *nnz, Xp, Xj, Xv, Yp, Yj, Yv, Cp, Cj, Cv, guard));
  *Cp_out = Cp;
  *Cj_out = Cj;
  if (Cv_out) *Cv_out = Cv;
  return RN_OK;
}

extern "C" rn_status rn_spgemm(rn_ctx *ctx, int32_t rows, int32_t inner, int32_t cols, const int32_t *X_rowptr,
                               const int32_t *X_colind, const double *X_vals, int64_t nnz_X,
                               const int32_t *Y_rowptr, const int32_t *Y_colind, const double *Y_vals,
                               int64_t nnz_Y, int32_t *C_rowptr, int32_t *C_colind, double *C_vals,
                               int64_t *nnz_C) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (rows < 0 || inner < 0 || cols < 0 || nnz_X < 0 || nnz_Y < 0 || !nnz_C || !C_rowptr)
    return rn_fail(ctx, RN_EINVAL, "rn_spgemm: bad argument");
  if (nnz_X >= ((int64_t)1 << 31) || nnz_Y >= ((int64_t)1 << 31))
    return rn_fail(ctx, RN_ELIMIT, "rn_spgemm: an operand has 2^31 entries or more");
  if ((rows > 0 && !X_rowptr) || (inner > 0 && !Y_rowptr) || (nnz_X > 0 && !X_colind) || (nnz_Y > 0 && !Y_colind))
    return rn_fail(ctx, RN_EINVAL, "rn_spgemm: null argument");
  if (C_vals && ((nnz_X > 0 && !X_vals) || (nnz_Y > 0 && !Y_vals)))
    return rn_fail(ctx, RN_EINVAL, "rn_spgemm: values of C need values of X and Y");
  rn_status st = RN_OK;
  int32_t *guard = rn_guard_begin(ctx, &st);
  if (!guard) return st;
  if (!C_colind) {  // phase 1: validation, counts, scan
    RnChecks v{};
    v.csr[0] = {rows, inner, nnz_X, X_rowptr, X_colind, GUARD_A};
    v.csr[1] = {inner, cols, nnz_Y, Y_rowptr, Y_colind, GUARD_N};
    v.ncsr = 2;
    RN_TRY(rn_validate(ctx, v, guard));
    int32_t *cnt = (int32_t *)rn_scratch(ctx, SLOT_PRD_CNT, (size_t)(rows + 1) * sizeof(int32_t), &st);
    if (!cnt) return st;
    RN_TRY(sg_symbolic(ctx, rows, nnz_X, X_rowptr, X_colind, Y_rowptr, Y_colind, cnt, nullptr, nullptr, guard));
    RN_TRY(rn_scan_counts(ctx, cnt, C_rowptr, rows, nullptr));
    int64_t *total = (int64_t *)rn_scratch(ctx, SLOT_SCAN_TOTAL, sizeof(int64_t), &st);
    if (!total) return st;
    RN_TRY(rn_read_guard_i64(ctx, guard, total, nnz_C, "rn_spgemm"));
    ctx->prd_rows = rows;
    ctx->prd_nnz = *nnz_C;
    return RN_OK;
  }
  // phase 2: the operands were validated in phase 1
  if (ctx->prd_rows != rows) return rn_fail(ctx, RN_EINVAL, "rn_spgemm: phase 2 without a matching phase 1");
  RN_TRY(sg_symbolic(ctx, rows, nnz_X, X_rowptr, X_colind, Y_rowptr, Y_colind, nullptr, C_rowptr, C_colind,
                     guard));
  if (C_vals)
    RN_TRY(sg_numeric(ctx, rows, ctx->prd_nnz, X_rowptr, X_colind, X_vals, Y_rowptr, Y_colind, Y_vals, C_rowptr,
                      C_colind, C_vals, guard));
  *nnz_C = ctx->prd_nnz;
  ctx->prd_rows = -1;
  return rn_check_guard(ctx, guard, "rn_spgemm");
}

rn_status rn_scalar_view(rn_ctx *ctx, const rn_matrix *A, const int32_t **Sp_out, const int32_t **Sj_out,
                         const double **Sv_out, int32_t *guard);

extern "C" rn_status rn_galerkin(rn_ctx *ctx, const rn_matrix *A, int32_t n_cols, const int32_t *N_rowptr,
                                 const int32_t *N_colind, int64_t nnz_N, const double *P, const double *RT,
                                 int32_t *Ac_rowptr, int32_t *Ac_colind, double *Ac_vals, int64_t *nnz_Ac) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (!A || !nnz_Ac || !Ac_rowptr || n_cols < 0 || nnz_N < 0 || (A->block_m != 1 && A->block_m != 2) || A->n < 0 ||
      A->n % A->block_m || A->nnz < 0)
    return rn_fail(ctx, RN_EINVAL, "rn_galerkin: bad argument");
  if (A->n > 0 && (!A->rowptr || !A->vals || !N_rowptr)) return rn_fail(ctx, RN_EINVAL, "rn_galerkin: null argument");
  if ((A->nnz > 0 && !A->colind) || (nnz_N > 0 && (!N_colind || !P)))
    return rn_fail(ctx, RN_EINVAL, "rn_galerkin: null argument");
  const int64_t mm = (int64_t)A->block_m * A->block_m;
  if (A->nnz * mm >= ((int64_t)1 << 31) || nnz_N >= ((int64_t)1 << 31))
    return rn_fail(ctx, RN_ELIMIT, "rn_galerkin: 2^31 entries or more");
  const int32_t n = A->n;
  rn_status st = RN_OK;
  int32_t *guard = rn_guard_begin(ctx, &st);
  if (!guard) return st;
  if (Ac_colind) {  // phase 2: R (A P) from the intermediates phase 1 left
    if (ctx->gal_nc != n_cols || ctx->gal_n != n)
      return rn_fail(ctx, RN_EINVAL, "rn_galerkin: phase 2 without a matching phase 1");
    RN_TRY(sg_symbolic(ctx, n_cols, nnz_N, ctx->gal_R[0], ctx->gal_R[1], ctx->gal_AP[0], ctx->gal_AP[1], nullptr,
                       Ac_rowptr, Ac_colind, guard));
    if (Ac_vals)
      RN_TRY(sg_numeric(ctx, n_cols, ctx->gal_nnz, ctx->gal_R[0], ctx->gal_R[1], ctx->gal_Rv, ctx->gal_AP[0],
                        ctx->gal_AP[1], ctx->gal_APv, Ac_rowptr, Ac_colind, Ac_vals, guard));
    *nnz_Ac = ctx->gal_nnz;
    ctx->gal_n = -1;
    return rn_check_guard(ctx, guard, "rn_galerkin");
  }
  // phase 1
  const int32_t nn = n / A->block_m;
  RnChecks v{};
  v.csr[0] = {nn, nn, A->nnz, A->rowptr, A->colind, GUARD_A};
  v.csr[1] = {n, n_cols, nnz_N, N_rowptr, N_colind, GUARD_N};
  v.ncsr = 2;
  RN_TRY(rn_validate(ctx, v, guard));
  // scalar CSR of A
  const int32_t *Sp = nullptr, *Sj = nullptr;
  const double *Sv = nullptr;
  RN_TRY(rn_scalar_view(ctx, A, &Sp, &Sj, &Sv, guard));
  // A P (n x n_cols)
  int32_t *APp = nullptr, *APj = nullptr;
  double *APv = nullptr;
  int64_t nnzAP = 0;
  RN_TRY(sg_full(ctx, n, A->nnz * mm, Sp, Sj, Sv, N_rowptr, N_colind, P, SLOT_GAL_APP, SLOT_GAL_APJ,
                 SLOT_GAL_APV, &APp, &APj, &APv, &nnzAP, guard, "rn_galerkin"));
  // R = (R^T)^T, R^T = P when no R^T is given (n_cols x n)
  int32_t *Rp = (int32_t *)rn_scratch(ctx, SLOT_GAL_RP, (size_t)(n_cols + 1) * sizeof(int32_t), &st);
  int32_t *Rj = (int32_t *)rn_scratch(ctx, SLOT_GAL_RJ, (size_t)(nnz_N + 1) * sizeof(int32_t), &st);
  double *Rv = (double *)rn_scratch(ctx, SLOT_GAL_RV, (size_t)(nnz_N + 1) * sizeof(double), &st);
  int32_t *perm = (int32_t *)rn_scratch(ctx, SLOT_GAL_PERM, (size_t)(nnz_N + 1) * sizeof(int32_t), &st);
  if (!Rp || !Rj || !Rv || !perm) return st;
  RN_TRY(rn_transpose_structure(ctx, n, n_cols, nnz_N, N_rowptr, N_colind, Rp, Rj, perm, guard));
  RN_TRY(rn_gather_values(ctx, RT ? RT : P, perm, nnz_N, Rv));
  // counts of R (A P)
  int32_t *cnt = (int32_t *)rn_scratch(ctx, SLOT_PRD_CNT, (size_t)(n_cols + 1) * sizeof(int32_t), &st);
  if (!cnt) return st;
  RN_TRY(sg_symbolic(ctx, n_cols, nnz_N, Rp, Rj, APp, APj, cnt, nullptr, nullptr, guard));
  RN_TRY(rn_scan_counts(ctx, cnt, Ac_rowptr, n_cols, nullptr));
  int64_t *total = (int64_t *)rn_scratch(ctx, SLOT_SCAN_TOTAL, sizeof(int64_t), &st);
  if (!total) return st;
  RN_TRY(rn_read_guard_i64(ctx, guard, total, nnz_Ac, "rn_galerkin"));
  ctx->gal_n = n;
  ctx->gal_nc = n_cols;
  ctx->gal_nnz = *nnz_Ac;
  ctx->gal_R[0] = Rp;
  ctx->gal_R[1] = Rj;
  ctx->gal_Rv = Rv;
  ctx->gal_AP[0] = APp;
  ctx->gal_AP[1] = APj;
  ctx->gal_APv = APv;
  return RN_OK;
}

// ---------------------------------------------------------------------------
// valued pattern N = S^d C (Sec. 3.4 with the values of Eq. soc)
// ---------------------------------------------------------------------------
// C as CSR: row I holds (agg[I], 1).
__global__ __launch_bounds__(RN_BLOCK) void k_agg_csr(int32_t nn, const int32_t *__restrict__ agg,
                                                     int32_t *__restrict__ Cp, int32_t *__restrict__ Cj,
                                                     double *__restrict__ Cv) {
  const int I = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (I > nn) return;
  Cp[I] = I;
  if (I < nn) {
    Cj[I] = agg[I];
    Cv[I] = 1.0;
  }
}

extern "C" rn_status rn_pattern_values(rn_ctx *ctx, int32_t nn, const int32_t *S_rowptr, const int32_t *S_colind,
                                       const double *S_vals, int64_t nnz_S, const int32_t *agg, int32_t n_agg,
                                       int32_t degree, int32_t *Nn_rowptr, int32_t *Nn_colind, double *Nn_vals,
                                       int64_t *nnz_Nn) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (nn < 0 || n_agg < 0 || degree < 0 || nnz_S < 0 || !nnz_Nn || !Nn_rowptr)
    return rn_fail(ctx, RN_EINVAL, "rn_pattern_values: bad argument");
  if ((nn > 0 && (!S_rowptr || !agg)) || (nnz_S > 0 && (!S_colind || !S_vals)))
    return rn_fail(ctx, RN_EINVAL, "rn_pattern_values: null argument");
  if (nnz_S >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_pattern_values: nnz_S >= 2^31");
  rn_status st = RN_OK;
  if (Nn_colind) {  // phase 2: copy out the last level phase 1 left
    if (ctx->pv_nn != nn || !ctx->pv_j) return rn_fail(ctx, RN_EINVAL, "rn_pattern_values: phase 2 without phase 1");
    if (ctx->pv_nnz > 0) {
      HIP_TRY(ctx, hipMemcpyAsync(Nn_colind, ctx->pv_j, (size_t)ctx->pv_nnz * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, ctx->stream));
      if (Nn_vals)
        HIP_TRY(ctx, hipMemcpyAsync(Nn_vals, ctx->pv_v, (size_t)ctx->pv_nnz * sizeof(double),
                                    hipMemcpyDeviceToDevice, ctx->stream));
    }
    *nnz_Nn = ctx->pv_nnz;
    ctx->pv_nn = -1;
    return RN_OK;
  }
  int32_t *guard = rn_guard_begin(ctx, &st);
  if (!guard) return st;
  RnChecks v{};
  v.csr[0] = {nn, nn, nnz_S, S_rowptr, S_colind, GUARD_S};
  v.ncsr = 1;
  v.range[0] = {nn, agg, 0, n_agg, GUARD_AGG};
  v.nrange = 1;
  RN_TRY(rn_validate(ctx, v, guard));
  // X_0 = C, then X_t = S X_(t-1) in alternating scratch slots
  int32_t *Xp = (int32_t *)rn_scratch(ctx, SLOT_GAL_RP, (size_t)(nn + 1) * sizeof(int32_t), &st);
  int32_t *Xj = (int32_t *)rn_scratch(ctx, SLOT_GAL_RJ, (size_t)(nn + 1) * sizeof(int32_t), &st);
  double *Xv = (double *)rn_scratch(ctx, SLOT_GAL_RV, (size_t)(nn + 1) * sizeof(double), &st);
  if (!Xp || !Xj || !Xv) return st;
  hipLaunchKernelGGL(k_agg_csr, dim3(rn_div_up(nn + 1, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, nn, agg, Xp, Xj,
                     Xv);
  LAUNCH_CHECK(ctx);
  int64_t nnzX = nn;
  const int slots[2][3] = {{SLOT_GAL_APP, SLOT_GAL_APJ, SLOT_GAL_APV}, {SLOT_GAL_RP, SLOT_GAL_RJ, SLOT_GAL_RV}};
  for (int t = 0; t < degree; ++t) {
    const int *sl = slots[t % 2];
    int32_t *Yp = nullptr, *Yj = nullptr;
    double *Yv = nullptr;
    int64_t nnzY = 0;
    RN_TRY(sg_full(ctx, nn, nnz_S, S_rowptr, S_colind, S_vals, Xp, Xj, Xv, sl[0], sl[1], sl[2], &Yp, &Yj, &Yv,
                   &nnzY, guard, "rn_pattern_values"));
    Xp = Yp;
    Xj = Yj;
    Xv = Yv;
    nnzX = nnzY;
  }
  if (degree == 0) RN_TRY(rn_check_guard(ctx, guard, "rn_pattern_values"));
  if (nnzX >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_pattern_values: pattern nnz reaches 2^31");
  if (nn >= 0)
    HIP_TRY(ctx, hipMemcpyAsync(Nn_rowptr, Xp, (size_t)(nn + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                ctx->stream));
  ctx->pv_nn = nn;
  ctx->pv_nnz = nnzX;
  ctx->pv_j = Xj;
  ctx->pv_v = Xv;
  *nnz_Nn = nnzX;
  return RN_OK;
}

// ---------------------------------------------------------------------------
// helpers for the normal-equation minimisation (rn_emin.hip)
// ---------------------------------------------------------------------------
rn_status rn_sg_pattern(rn_ctx *ctx, int32_t rows, int64_t nnzX, const int32_t *Xp, const int32_t *Xj,
                        const int32_t *Yp, const int32_t *Yj, int slot_p, int slot_j, int32_t **Cp, int32_t **Cj,
                        int64_t *nnz, int32_t *guard, const char *what) {
  return sg_full(ctx, rows, nnzX, Xp, Xj, nullptr, Yp, Yj, nullptr, slot_p, slot_j, -1, Cp, Cj, nullptr, nnz, guard,
                 what);
}

rn_status rn_sg_values(rn_ctx *ctx, int32_t rows, int64_t nnzC, const int32_t *Xp, const int32_t *Xj,
                       const double *Xv, const int32_t *Yp, const int32_t *Yj, const double *Yv, const int32_t *Cp,
                       const int32_t *Cj, double *Cv, const int32_t *guard) {
  return sg_numeric(ctx, rows, nnzC, Xp, Xj, Xv, Yp, Yj, Yv, Cp, Cj, Cv, guard);
}

rn_status rn_scalar_view(rn_ctx *ctx, const rn_matrix *A, const int32_t **Sp_out, const int32_t **Sj_out,
                         const double **Sv_out, int32_t *guard) {
  if (A->block_m == 1) {
    *Sp_out = A->rowptr;
    *Sj_out = A->colind;
    *Sv_out = A->vals;
    return RN_OK;
  }
  rn_status st = RN_OK;
  const int32_t n = A->n, nn = n / 2;
  int32_t *cnt = (int32_t *)rn_scratch(ctx, SLOT_PRD_CNT, (size_t)(n + 1) * sizeof(int32_t), &st);
  int32_t *p = (int32_t *)rn_scratch(ctx, SLOT_GAL_ASP, (size_t)(n + 1) * sizeof(int32_t), &st);
  int32_t *j = (int32_t *)rn_scratch(ctx, SLOT_GAL_ASJ, (size_t)(A->nnz * 4 + 1) * sizeof(int32_t), &st);
  double *x = (double *)rn_scratch(ctx, SLOT_GAL_ASV, (size_t)(A->nnz * 4 + 1) * sizeof(double), &st);
  if (!cnt || !p || !j || !x) return st;
  if (nn > 0) {
    hipLaunchKernelGGL(k_bsr2_rows, dim3(rn_div_up(nn, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, nn, A->rowptr,
                       cnt);
    LAUNCH_CHECK(ctx);
  }
  RN_TRY(rn_scan_counts(ctx, cnt, p, n, nullptr));
  if (nn > 0) {
    hipLaunchKernelGGL(k_bsr2_fill, dim3(rn_div_up(nn, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, nn, A->rowptr,
                       A->colind, A->vals, p, j, x, guard);
    LAUNCH_CHECK(ctx);
  }
  *Sp_out = p;
  *Sj_out = j;
  *Sv_out = x;
  return RN_OK;
}
