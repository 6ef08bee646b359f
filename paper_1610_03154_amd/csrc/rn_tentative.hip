// rn_tentative.hip -- inject (Sec. 3.6): coarse candidates by injection at
// the root DOFs, the root-node tentative operator of Eq. root-nodeform, and
// the minimum-norm row update of Eq. Tproj for candidates beyond the first m.
#include <cmath>
#include <cstring>
#include "rn_gram.h"
#include "rn_internal.h"

// One thread per aggregate a: the injected rows Bc[m*a + c, :] = B[m*root + c, :]
// (c < m) and the inverse of the m x m root block of the first m candidates
// (m <= 2 here); a zero or singular root block raises flag bit 0.
__global__ __launch_bounds__(RN_BLOCK) void k_inject_root(int n_agg, int m, int nB,
                                                         const int32_t *__restrict__ roots,
                                                         const double *__restrict__ B, double *__restrict__ Bc,
                                                         double *__restrict__ binv, int32_t *__restrict__ flags,
                                                         const int32_t *__restrict__ guard) {
  const int a = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (a >= n_agg || *guard) return;
  const int64_t r0 = (int64_t)m * roots[a];
  for (int c = 0; c < m; ++c)
    for (int k = 0; k < nB; ++k) Bc[((int64_t)m * a + c) * nB + k] = B[(r0 + c) * nB + k];
  if (m == 1) {
    const double b = B[r0 * nB];
    if (b == 0.0) atomicOr(flags, 1);
    binv[a] = b != 0.0 ? 1.0 / b : 0.0;
  } else {
    const double b00 = B[r0 * nB], b01 = B[r0 * nB + 1];
    const double b10 = B[(r0 + 1) * nB], b11 = B[(r0 + 1) * nB + 1];
    const double det = b00 * b11 - b01 * b10;
    if (det == 0.0) atomicOr(flags, 1);
    const double id = det != 0.0 ? 1.0 / det : 0.0;
    binv[4 * a + 0] = b11 * id;
    binv[4 * a + 1] = -b01 * id;
    binv[4 * a + 2] = -b10 * id;
    binv[4 * a + 3] = b00 * id;
  }
}

// T on the pattern: root rows = identity row; F row i of aggregate a holds
// B[i, 0:m] inv(root block) at columns m*a .. m*a+m-1, zero elsewhere.
// W lanes per row (entries s + l, s + l + W, ...).
template <int W, int M>
__global__ __launch_bounds__(RN_BLOCK) void k_tent_T(int n, int nB, const int32_t *__restrict__ Np,
                                                    const int32_t *__restrict__ Nj,
                                                    const uint8_t *__restrict__ is_root,
                                                    const int32_t *__restrict__ agg, const double *__restrict__ B,
                                                    const double *__restrict__ binv, double *__restrict__ T,
                                                    const int32_t *__restrict__ guard) {
  const int64_t gid = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x;
  const int i = (int)(gid / W), l = (int)(gid % W);
  if (i >= n || *guard) return;
  const int a = agg[i / M], c = i % M;
  const bool root = is_root[i];
  for (int p = Np[i] + l; p < Np[i + 1]; p += W) {
    const int j = Nj[p];
    double t = 0.0;
    if (root) {
      t = (j == M * a + c) ? 1.0 : 0.0;
    } else if (j / M == a) {
      const int cc = j % M;
      for (int r = 0; r < M; ++r) t += B[(int64_t)i * nB + r] * binv[(int64_t)a * M * M + r * M + cc];
    }
    T[p] = t;
  }
}

// Eq. Tproj on F rows: t <- t + (B_i - t B_J) G^+ B_J^T, G = B_J^T B_J, one
// thread per row; gp (nullable) receives each row's G^+ packed as the plan
// keeps it (upper triangle, root rows zero).
template <int NB>
__global__ __launch_bounds__(RN_BLOCK) void k_tproj(int n, const int32_t *__restrict__ Np,
                                                   const int32_t *__restrict__ Nj,
                                                   const uint8_t *__restrict__ is_root,
                                                   const double *__restrict__ B, const double *__restrict__ Bc,
                                                   double *__restrict__ T, double *__restrict__ gp,
                                                   int32_t *__restrict__ rank_def,
                                                   const int32_t *__restrict__ guard) {
  constexpr int NP = NB * (NB + 1) / 2;
  const int i = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (i >= n || *guard) return;
  if (is_root[i]) {
    if (gp)
#pragma unroll
      for (int k = 0; k < NP; ++k) gp[(int64_t)i * NP + k] = 0.0;
    return;
  }
  double Gp[NB * NB], rr[NB], y[NB], ts[NB], G[NB * NB];
  const int s = Np[i], e = Np[i + 1];
  // r = B_i - t B_J and G = B_J^T B_J in one pass over the row (each sum in
  // row order)
#pragma unroll
  for (int q = 0; q < NB; ++q) ts[q] = 0.0;
#pragma unroll
  for (int q = 0; q < NB * NB; ++q) G[q] = 0.0;
  rn_row_each<NB>(Nj, s, e, Bc, [&](int p, const double *b) {
    const double t = T[p];
#pragma unroll
    for (int q = 0; q < NB; ++q) ts[q] += t * b[q];
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int r = 0; r < NB; ++r) G[q * NB + r] += b[q] * b[r];
  });
#pragma unroll
  for (int q = 0; q < NB; ++q) rr[q] = B[(int64_t)i * NB + q] - ts[q];
  if (rn_row_pinv_g<NB>(Nj, s, e, Bc, G, Gp)) atomicAdd(rank_def, 1);
  if (gp)
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int r = q; r < NB; ++r) gp[(int64_t)i * NP + rn_pk(NB, q, r)] = Gp[q * NB + r];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    double v = 0.0;
#pragma unroll
    for (int r = 0; r < NB; ++r) v += Gp[q * NB + r] * rr[r];
    y[q] = v;
  }
  rn_row_each<NB>(Nj, s, e, Bc, [&](int p, const double *b) {
    double u = 0.0;
#pragma unroll
    for (int q = 0; q < NB; ++q) u += b[q] * y[q];
    T[p] += u;
  });
}

// Eq. Tproj on every F row (nB = 1..4)
static void launch_tproj(hipStream_t st, int n, int nB, const int32_t *Np, const int32_t *Nj, const uint8_t *is_root,
                         const double *B, const double *Bc, double *T, double *gp, int32_t *rank_def,
                         const int32_t *guard) {
  const dim3 g(rn_div_up(n, RN_BLOCK)), b(RN_BLOCK);
  switch (nB) {
    case 1: hipLaunchKernelGGL(k_tproj<1>, g, b, 0, st, n, Np, Nj, is_root, B, Bc, T, gp, rank_def, guard); break;
    case 2: hipLaunchKernelGGL(k_tproj<2>, g, b, 0, st, n, Np, Nj, is_root, B, Bc, T, gp, rank_def, guard); break;
    case 3: hipLaunchKernelGGL(k_tproj<3>, g, b, 0, st, n, Np, Nj, is_root, B, Bc, T, gp, rank_def, guard); break;
    case 4: hipLaunchKernelGGL(k_tproj<4>, g, b, 0, st, n, Np, Nj, is_root, B, Bc, T, gp, rank_def, guard); break;
  }
}

// Everything of rn_tentative up to its synchronisation: validation into
// guard (not reset here; skipped when the caller made N, agg and roots
// itself and checked them) and the kernels; *flags receives the device
// flags (singular root block, rank-deficient rows), which sit in the guard
// slot.
rn_status rn_tentative_launch(rn_ctx *ctx, int32_t n, int32_t m, const int32_t *Np, const int32_t *Nj,
                              int64_t nnz_N, const uint8_t *is_root, const int32_t *agg, const int32_t *roots,
                              int32_t n_agg, const double *B, int32_t nB, double *T, double *Bc, int32_t *guard,
                              const int32_t **flags_out, bool validate, double *gp_out) {
  if ((m != 1 && m != 2) || n < 0 || n % m || n_agg < 0 || nnz_N < 0 || nB < m || nB > RN_NBMAX)
    return rn_fail(ctx, RN_EINVAL, "rn_tentative: bad sizes (n %d, m %d, n_agg %d, nB %d; need m <= nB <= %d)", n,
                   m, n_agg, nB, RN_NBMAX);
  if (n > 0 && (!Np || !Nj || !is_root || !agg || !B || !T)) return rn_fail(ctx, RN_EINVAL, "rn_tentative: null argument");
  if (n_agg > 0 && (!roots || !Bc)) return rn_fail(ctx, RN_EINVAL, "rn_tentative: null argument");
  if (nnz_N >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_tentative: nnz_N >= 2^31");
  rn_status st = RN_OK;
  const int nn = n / m, nc = m * n_agg;
  double *binv = (double *)rn_scratch(ctx, SLOT_TEN_BINV, (size_t)(n_agg + 1) * m * m * sizeof(double), &st);
  if (!binv) return st;
  int32_t *flags = guard + GS_TFLAGS;  // zeroed with the guard
  if (validate) {
    RnChecks v{};
    v.csr[0] = {n, nc, nnz_N, Np, Nj, GUARD_N};
    v.ncsr = 1;
    v.range[0] = {nn, agg, 0, n_agg, GUARD_AGG};
    v.range[1] = {n_agg, roots, 0, nn, GUARD_ROOTS};
    v.nrange = 2;
    RN_TRY(rn_validate(ctx, v, guard));
  }
  if (nc > 0) {
    hipLaunchKernelGGL(k_inject_root, dim3(rn_div_up(n_agg, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, n_agg, m,
                       nB, roots, B, Bc, binv, flags, guard);
    LAUNCH_CHECK(ctx);
  }
  if (n > 0) {
    // (block_m a template argument: its divisions are shifts)
    const bool wide = rn_row_group(nnz_N, n) == 16;
    const dim3 gt(rn_div_up((int64_t)n * (wide ? 16 : 4), RN_BLOCK)), bt(RN_BLOCK);
    if (wide && m == 2)
      hipLaunchKernelGGL((k_tent_T<16, 2>), gt, bt, 0, ctx->stream, n, nB, Np, Nj, is_root, agg, B, binv, T, guard);
    else if (wide)
      hipLaunchKernelGGL((k_tent_T<16, 1>), gt, bt, 0, ctx->stream, n, nB, Np, Nj, is_root, agg, B, binv, T, guard);
    else if (m == 2)
      hipLaunchKernelGGL((k_tent_T<4, 2>), gt, bt, 0, ctx->stream, n, nB, Np, Nj, is_root, agg, B, binv, T, guard);
    else
      hipLaunchKernelGGL((k_tent_T<4, 1>), gt, bt, 0, ctx->stream, n, nB, Np, Nj, is_root, agg, B, binv, T, guard);
    LAUNCH_CHECK(ctx);
    if (nB > m) {
      launch_tproj(ctx->stream, n, nB, Np, Nj, is_root, B, Bc, T, gp_out, flags + 1, guard);
      LAUNCH_CHECK(ctx);
    }
  }
  *flags_out = flags;
  return RN_OK;
}

// The tentative's flags as read back: a singular root block is an error.
rn_status rn_tentative_flags(rn_ctx *ctx, const int32_t hf[2], int32_t *rank_deficient) {
  if (hf[0]) return rn_fail(ctx, RN_ESINGULAR, "rn_tentative: singular root block of B");
  if (rank_deficient) *rank_deficient = hf[1];
  return RN_OK;
}

extern "C" rn_status rn_tentative(rn_ctx *ctx, int32_t n, int32_t m, const int32_t *Np, const int32_t *Nj,
                                  int64_t nnz_N, const uint8_t *is_root, const int32_t *agg, const int32_t *roots,
                                  int32_t n_agg, const double *B, int32_t nB, double *T, double *Bc,
                                  int32_t *rank_deficient) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  rn_status st = RN_OK;
  int32_t *guard = rn_guard_begin(ctx, &st);
  if (!guard) return st;
  const int32_t *flags = nullptr;
  RN_TRY(rn_tentative_launch(ctx, n, m, Np, Nj, nnz_N, is_root, agg, roots, n_agg, B, nB, T, Bc, guard, &flags,
                             true, nullptr));
  // one synchronisation: guard and the two flags
  const RnFetch it[2] = {{guard, 4}, {flags, 2 * sizeof(int32_t)}};
  const unsigned char *hb = nullptr;
  size_t off[2];
  RN_TRY(rn_fetch(ctx, 2, it, &hb, off));
  int32_t gword = 0, hf[2] = {0, 0};
  memcpy(&gword, hb + off[0], 4);
  memcpy(hf, hb + off[1], 8);
  RN_TRY(rn_guard_status(ctx, gword, "rn_tentative"));
  return rn_tentative_flags(ctx, hf, rank_deficient);
}

// enforce (Sec. 3.7): Eq. Tproj on every F row of the caller's values.
extern "C" rn_status rn_enforce(rn_ctx *ctx, int32_t n, int32_t n_cols, const int32_t *N_rowptr,
                                const int32_t *N_colind, int64_t nnz_N, const uint8_t *is_root, const double *Bc,
                                const double *B, int32_t nB, double *vals, int32_t *rank_deficient) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (n < 0 || n_cols < 0 || nnz_N < 0 || nB < 1 || nB > RN_NBMAX)
    return rn_fail(ctx, RN_EINVAL, "rn_enforce: bad sizes (n %d, n_cols %d, nB %d; need 1 <= nB <= %d)", n, n_cols,
                   nB, RN_NBMAX);
  if (nnz_N >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_enforce: nnz_N >= 2^31");
  if (n > 0 && (!N_rowptr || !is_root || !B)) return rn_fail(ctx, RN_EINVAL, "rn_enforce: null argument");
  if (nnz_N > 0 && (!N_colind || !vals || !Bc)) return rn_fail(ctx, RN_EINVAL, "rn_enforce: null argument");
  rn_status st = RN_OK;
  int32_t *guard = rn_guard_begin(ctx, &st);
  if (!guard) return st;
  int32_t *flags = guard + GS_TFLAGS;  // flags[1]: rank-deficient rows (zeroed with the guard)
  RnChecks v{};
  v.csr[0] = {n, n_cols, nnz_N, N_rowptr, N_colind, GUARD_N};
  v.ncsr = 1;
  RN_TRY(rn_validate(ctx, v, guard));
  if (n > 0) {
    launch_tproj(ctx->stream, n, nB, N_rowptr, N_colind, is_root, B, Bc, vals, nullptr, flags + 1, guard);
    LAUNCH_CHECK(ctx);
  }
  const RnFetch it[2] = {{guard, 4}, {flags, 2 * sizeof(int32_t)}};
  const unsigned char *hb = nullptr;
  size_t off[2];
  RN_TRY(rn_fetch(ctx, 2, it, &hb, off));
  int32_t gword = 0, hf[2] = {0, 0};
  memcpy(&gword, hb + off[0], 4);
  memcpy(hf, hb + off[1], 8);
  RN_TRY(rn_guard_status(ctx, gword, "rn_enforce"));
  if (rank_deficient) *rank_deficient = hf[1];
  return RN_OK;
}

// ---------------------------------------------------------------------------
// candidate smoothing: damped Jacobi on A B = 0
// ---------------------------------------------------------------------------
// One thread per DOF row: Bn = Bs - omega (A Bs)_i / a_ii for every column,
// the row sum in the order of A's row (blocks in order, their columns in
// order for M = 2); a zero diagonal raises flag[0].
template <int M>
__global__ __launch_bounds__(RN_BLOCK) void k_jacobi_sweep(int n, int nB, const int32_t *__restrict__ Ap,
                                                          const int32_t *__restrict__ Aj,
                                                          const double *__restrict__ Ax, double omega,
                                                          const double *__restrict__ Bs, double *__restrict__ Bn,
                                                          int32_t *__restrict__ flag,
                                                          const int32_t *__restrict__ guard) {
  const int i = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (i >= n || *guard) return;
  const int I = i / M, r = i % M;
  double d = 0.0;
  for (int p = Ap[I]; p < Ap[I + 1]; ++p)
    if (Aj[p] == I) d = Ax[(int64_t)p * M * M + r * M + r];
  if (d == 0.0) atomicOr(flag, 1);
  for (int q = 0; q < nB; ++q) {
    double y = 0.0;
    for (int p = Ap[I]; p < Ap[I + 1]; ++p) {
      const int J = Aj[p];
#pragma unroll
      for (int c = 0; c < M; ++c) y += Ax[(int64_t)p * M * M + r * M + c] * Bs[((int64_t)M * J + c) * nB + q];
    }
    Bn[(int64_t)i * nB + q] = Bs[(int64_t)i * nB + q] - omega * (y / d);
  }
}

extern "C" rn_status rn_smooth_candidates(rn_ctx *ctx, const rn_matrix *A, double *B, int32_t nB, int32_t sweeps,
                                          double omega) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (!A || nB < 1 || sweeps < 0 || !std::isfinite(omega) || (A->block_m != 1 && A->block_m != 2) || A->n < 0 ||
      A->n % A->block_m || A->nnz < 0)
    return rn_fail(ctx, RN_EINVAL, "rn_smooth_candidates: bad argument");
  if (A->n > 0 && (!A->rowptr || !B || (A->nnz > 0 && (!A->colind || !A->vals))))
    return rn_fail(ctx, RN_EINVAL, "rn_smooth_candidates: null argument");
  if (A->nnz >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_smooth_candidates: nnz >= 2^31");
  if (sweeps == 0 || A->n == 0) return RN_OK;
  const int m = A->block_m, n = A->n, nn = n / m;
  rn_status st = RN_OK;
  int32_t *guard = rn_guard_begin(ctx, &st);
  if (!guard) return st;
  double *tmp = (double *)rn_scratch(ctx, SLOT_MISC, (size_t)n * nB * sizeof(double), &st);
  if (!tmp) return st;
  int32_t *flag = guard + GS_TFLAGS;  // zeroed with the guard
  RnChecks v{};
  v.csr[0] = {nn, nn, A->nnz, A->rowptr, A->colind, GUARD_A};
  v.ncsr = 1;
  RN_TRY(rn_validate(ctx, v, guard));
  double *src = B, *dst = tmp;
  for (int s = 0; s < sweeps; ++s) {
    if (m == 1)
      hipLaunchKernelGGL(k_jacobi_sweep<1>, dim3(rn_div_up(n, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, n, nB,
                         A->rowptr, A->colind, A->vals, omega, src, dst, flag, guard);
    else
      hipLaunchKernelGGL(k_jacobi_sweep<2>, dim3(rn_div_up(n, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, n, nB,
                         A->rowptr, A->colind, A->vals, omega, src, dst, flag, guard);
    LAUNCH_CHECK(ctx);
    double *t = src;
    src = dst;
    dst = t;
  }
  if (src != B)
    HIP_TRY(ctx, hipMemcpyAsync(B, src, (size_t)n * nB * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  const RnFetch it[2] = {{guard, 4}, {flag, 4}};
  const unsigned char *hb = nullptr;
  size_t off[2];
  RN_TRY(rn_fetch(ctx, 2, it, &hb, off));
  int32_t gword = 0, fl = 0;
  memcpy(&gword, hb + off[0], 4);
  memcpy(&fl, hb + off[1], 4);
  RN_TRY(rn_guard_status(ctx, gword, "rn_smooth_candidates"));
  if (fl) return rn_fail(ctx, RN_ESINGULAR, "rn_smooth_candidates: a diagonal entry of A is zero");
  return RN_OK;
}
