// rn_setup.hip -- one-shot set-up of one level (Alg. root_node_setup): the
// stage entry points run back to back inside the library, their outputs in
// device memory owned by the returned handle (drawn from the context's
// allocation cache, so repeated set-ups allocate nothing new).
#include <cstdlib>
#include <cstring>
#include <new>

#include "rn_emin.h"

struct rn_setup_out {
  rn_ctx *ctx = nullptr;
  rn_setup_view v{};
  rn_plan *plan = nullptr, *plan_T = nullptr;
  int32_t *AT_rowptr = nullptr, *AT_colind = nullptr;
  double *AT_vals = nullptr;
  void *bufs[24] = {};
  int nbuf = 0;
};

static void *setup_alloc(rn_setup_out *s, size_t bytes) {
  void *p = rn_dev_alloc(s->ctx, bytes ? bytes : 16);
  if (p) s->bufs[s->nbuf++] = p;
  return p;
}

extern "C" void rn_setup_destroy(rn_setup_out *s) {
  if (!s) return;
  if (s->plan) rn_plan_destroy(s->plan);
  if (s->plan_T) rn_plan_destroy(s->plan_T);
  for (int i = 0; i < s->nbuf; ++i) rn_dev_free(s->ctx, s->bufs[i]);
  delete s;
}

extern "C" rn_status rn_setup_view_get(const rn_setup_out *s, rn_setup_view *view) {
  if (!s || !view) return RN_EINVAL;
  *view = s->v;
  return RN_OK;
}

extern "C" rn_status rn_setup(rn_ctx *ctx, const rn_matrix *A, const int32_t *agg, const int32_t *roots,
                              int32_t n_agg, const double *B, const double *Bhat, int32_t nB, int32_t degree,
                              int32_t iters, double theta, rn_method method, rn_precision precision,
                              rn_setup_out **out, rn_emin_stats *stats, rn_emin_stats *stats_RT) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (!out || !A || !B || (A->n > 0 && (!agg || !A->vals)) || (n_agg > 0 && !roots))
    return rn_fail(ctx, RN_EINVAL, "rn_setup: null argument");
  *out = nullptr;
  const int m = A->block_m;
  if ((m != 1 && m != 2) || A->n < 0 || A->n % m) return rn_fail(ctx, RN_EINVAL, "rn_setup: bad matrix descriptor");
  if (Bhat && m != 1) return rn_fail(ctx, RN_EINVAL, "rn_setup: R^T on A^T needs a scalar CSR operator");
  rn_setup_out *s = new (std::nothrow) rn_setup_out();
  if (!s) return rn_fail(ctx, RN_ENOMEM, "rn_setup: host allocation");
  s->ctx = ctx;
  rn_setup_view &v = s->v;
  const int nn = A->n / m, n = A->n, nc = m * n_agg;
  v.n = n;
  v.n_cols = nc;
  v.nB = nB;
  rn_status st = RN_OK;
  auto fail = [&](rn_status e) {
    rn_setup_destroy(s);
    return e;
  };
  auto nomem = [&]() { return fail(rn_fail(ctx, RN_ENOMEM, "rn_setup: device allocation")); };
  // a1-a4: strength and pattern.  First with one synchronisation for both
  // (S filled into room for nnz(A) + n/m entries on the assumption of a
  // structurally symmetric A); otherwise the two-phase stage calls.
  int32_t *Sp = (int32_t *)setup_alloc(s, (size_t)(nn + 1) * 4);
  int32_t *Sj = (int32_t *)setup_alloc(s, (size_t)(A->nnz + nn + 1) * 4);
  int32_t *Np = (int32_t *)setup_alloc(s, (size_t)(n + 1) * 4);
  uint8_t *is_root = (uint8_t *)setup_alloc(s, (size_t)n + 1);
  if (!Sp || !Sj || !Np || !is_root) return nomem();
  int64_t nnzS = 0, nnzN = 0;
  bool done = false;
  if (ctx->opt[RN_OPT_FUSED_SETUP] &&  // 0: the stage calls only
      (st = rn_strength_pattern(ctx, A, theta, Sp, Sj, agg, roots, n_agg, degree, Np, is_root, &nnzS, &nnzN,
                                &done)) != RN_OK)
    return fail(st);
  if (!done) {
    if ((st = rn_strength(ctx, A, theta, Sp, nullptr, &nnzS)) != RN_OK) return fail(st);
    if (nnzS > A->nnz + nn && !(Sj = (int32_t *)setup_alloc(s, (size_t)nnzS * 4))) return nomem();
    if ((st = rn_strength(ctx, A, theta, Sp, Sj, &nnzS)) != RN_OK) return fail(st);
    if ((st = rn_pattern(ctx, nn, Sp, Sj, agg, roots, n_agg, degree, m, Np, nullptr, is_root, &nnzN)) != RN_OK)
      return fail(st);
  }
  v.S_rowptr = Sp;
  v.S_colind = Sj;
  v.nnz_S = nnzS;
  int32_t *Nj = (int32_t *)setup_alloc(s, (size_t)nnzN * 4);
  if (!Nj) return nomem();
  if ((st = rn_pattern(ctx, nn, Sp, Sj, agg, roots, n_agg, degree, m, Np, Nj, is_root, &nnzN)) != RN_OK)
    return fail(st);
  v.N_rowptr = Np;
  v.N_colind = Nj;
  v.is_root = is_root;
  v.nnz_N = nnzN;
  // a5/a6: T and Bc
  double *T = (double *)setup_alloc(s, (size_t)nnzN * 8);
  double *Bc = (double *)setup_alloc(s, (size_t)nc * nB * 8);
  double *P = (double *)setup_alloc(s, (size_t)nnzN * 8);
  if (!T || !Bc || !P) return nomem();
  // the tentative's checks are read at the plan's synchronisation (one
  // guard word for both stages); A, agg and roots were checked by the first
  // stage and N was made here, so neither stage validates again
  int32_t *guard = rn_guard_begin(ctx, &st);
  if (!guard) return fail(st);
  // with candidates beyond the first m, Eq. Tproj forms every F row's G^+;
  // the plan's projection takes that array instead of forming it again
  const int NP = nB * (nB + 1) / 2;
  double *gp = nB > m ? (double *)setup_alloc(s, (size_t)(n + 1) * NP * 8) : nullptr;
  if (nB > m && !gp) return nomem();
  const int32_t *tflags = nullptr;
  if ((st = rn_tentative_launch(ctx, n, m, Np, Nj, nnzN, is_root, agg, roots, n_agg, B, nB, T, Bc, guard,
                                &tflags, false, gp)) != RN_OK)
    return fail(st);
  v.T = T;
  v.Bc = Bc;
  // a7-a11: plan and energy minimisation of P
  int32_t hf[2] = {0, 0};
  const RnFetch fl = {tflags, sizeof hf};
  if ((st = rn_plan_create_ex(ctx, A, nc, Np, Nj, nnzN, is_root, Bc, nB, &s->plan, guard, &fl,
                              (unsigned char *)hf, false, gp)) != RN_OK)
    return fail(st);
  if ((st = rn_tentative_flags(ctx, hf, &v.rank_deficient)) != RN_OK) return fail(st);
  if (gp) s->plan->rank_def = v.rank_deficient;  // the same rows, counted by Eq. Tproj
  if ((st = rn_energy_min(ctx, s->plan, A->vals, 1, T, method, iters, precision, P, nullptr, stats, nullptr)) !=
      RN_OK)
    return fail(st);
  v.P = P;
  v.plan = s->plan;
  if (stats && ctx->opt[RN_OPT_METRICS] &&
      (st = rn_constraint_residual(ctx, n, nc, Np, Nj, nnzN, P, Bc, B, nB, &stats->constraint_residual)) != RN_OK)
    return fail(st);
  if (Bhat) {
    // a10: R^T by the same minimisation on A^T with T-hat from B-hat
    s->AT_rowptr = (int32_t *)setup_alloc(s, (size_t)(n + 1) * 4);
    s->AT_colind = (int32_t *)setup_alloc(s, (size_t)A->nnz * 4);
    s->AT_vals = (double *)setup_alloc(s, (size_t)A->nnz * 8);
    double *That = (double *)setup_alloc(s, (size_t)nnzN * 8);
    double *Bch = (double *)setup_alloc(s, (size_t)nc * nB * 8);
    double *RT = (double *)setup_alloc(s, (size_t)nnzN * 8);
    if (!s->AT_rowptr || !s->AT_colind || !s->AT_vals || !That || !Bch || !RT) return nomem();
    if ((st = rn_transpose(ctx, A, s->AT_rowptr, s->AT_colind, s->AT_vals, nullptr)) != RN_OK) return fail(st);
    const rn_matrix AT = {n, 1, A->nnz, s->AT_rowptr, s->AT_colind, s->AT_vals};
    int32_t *g2 = rn_guard_begin(ctx, &st);
    if (!g2) return fail(st);
    double *gph = nB > m ? (double *)setup_alloc(s, (size_t)(n + 1) * NP * 8) : nullptr;
    if (nB > m && !gph) return nomem();
    if ((st = rn_tentative_launch(ctx, n, m, Np, Nj, nnzN, is_root, agg, roots, n_agg, Bhat, nB, That, Bch, g2,
                                  &tflags, false, gph)) != RN_OK)
      return fail(st);
    const RnFetch fl2 = {tflags, sizeof hf};
    if ((st = rn_plan_create_ex(ctx, &AT, nc, Np, Nj, nnzN, is_root, Bch, nB, &s->plan_T, g2, &fl2,
                                (unsigned char *)hf, false, gph)) != RN_OK)
      return fail(st);
    int32_t rd_hat = 0;
    if ((st = rn_tentative_flags(ctx, hf, &rd_hat)) != RN_OK) return fail(st);
    if (gph) s->plan_T->rank_def = rd_hat;
    if ((st = rn_energy_min(ctx, s->plan_T, s->AT_vals, 1, That, method, iters, precision, RT, nullptr, stats_RT,
                            nullptr)) != RN_OK)
      return fail(st);
    if (stats_RT && ctx->opt[RN_OPT_METRICS] &&
        (st = rn_constraint_residual(ctx, n, nc, Np, Nj, nnzN, RT, Bch, Bhat, nB,
                                     &stats_RT->constraint_residual)) != RN_OK)
      return fail(st);
    v.That = That;
    v.Bchat = Bch;
    v.RT = RT;
    v.plan_T = s->plan_T;
  }
  *out = s;
  return RN_OK;
}
