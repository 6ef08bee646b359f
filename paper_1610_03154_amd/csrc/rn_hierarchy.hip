// rn_hierarchy.hip -- the multilevel set-up: Alg. root_node_setup applied
// level by level, each coarse operator the Galerkin product of the level
// above (Sec. 3.8).  Orchestration of the stage calls only: strength on the
// device, the host aggregation, the one-call set-up of the level, the
// Galerkin product; every array of a coarse level lives in device memory
// owned by the hierarchy.
#include <cstring>
#include <new>
#include <vector>

#include "rn_emin.h"

struct rn_hierarchy {
  rn_ctx *ctx = nullptr;
  struct Level {
    rn_matrix A{};
    const double *B = nullptr;
    int32_t nB = 0, n_agg = 0;
    int32_t *agg = nullptr, *roots = nullptr;
    rn_setup_out *s = nullptr;
    rn_emin_stats stats{}, stats_RT{};
  };
  std::vector<Level> lv;
  std::vector<void *> bufs;  // device memory of the coarse levels
};

extern "C" void rn_hierarchy_destroy(rn_hierarchy *h) {
  if (!h) return;
  for (auto &l : h->lv)
    if (l.s) rn_setup_destroy(l.s);
  for (void *p : h->bufs) rn_dev_free(h->ctx, p);
  delete h;
}

extern "C" int32_t rn_hierarchy_levels(const rn_hierarchy *h) { return h ? (int32_t)h->lv.size() : 0; }

extern "C" rn_status rn_hierarchy_level(const rn_hierarchy *h, int32_t level, rn_level_view *v) {
  if (!h || !v || level < 0 || level >= (int32_t)h->lv.size()) return RN_EINVAL;
  const rn_hierarchy::Level &l = h->lv[level];
  memset(v, 0, sizeof *v);
  v->n = l.A.n;
  v->block_m = l.A.block_m;
  v->nnz_A = l.A.nnz;
  v->A_rowptr = l.A.rowptr;
  v->A_colind = l.A.colind;
  v->A_vals = l.A.vals;
  v->B = l.B;
  v->nB = l.nB;
  v->n_agg = l.n_agg;
  v->agg = l.agg;
  v->roots = l.roots;
  v->setup = l.s;
  v->stats = l.stats;
  v->stats_RT = l.stats_RT;
  return RN_OK;
}

extern "C" rn_status rn_hierarchy_build(rn_ctx *ctx, const rn_matrix *A, const double *B, int32_t nB,
                                        int32_t max_levels, int32_t min_coarse, double theta, int32_t degree,
                                        int32_t iters, rn_method method, rn_precision precision,
                                        rn_hierarchy **out) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (!A || !B || !out) return rn_fail(ctx, RN_EINVAL, "rn_hierarchy_build: null argument");
  *out = nullptr;
  if (max_levels < 1 || min_coarse < 0 || nB < 1)
    return rn_fail(ctx, RN_EINVAL, "rn_hierarchy_build: max_levels >= 1, min_coarse >= 0 and nB >= 1");
  if (method != RN_CG && method != RN_GMRES)
    return rn_fail(ctx, RN_EINVAL, "rn_hierarchy_build: method RN_CG or RN_GMRES");
  if (method == RN_GMRES && A->block_m != 1)
    return rn_fail(ctx, RN_EINVAL, "rn_hierarchy_build: R^T on A^T needs a scalar CSR operator");
  rn_hierarchy *h = new (std::nothrow) rn_hierarchy();
  if (!h) return rn_fail(ctx, RN_ENOMEM, "rn_hierarchy_build: host allocation");
  h->ctx = ctx;
  rn_status st = RN_OK;
  auto fail = [&](rn_status e) {
    rn_hierarchy_destroy(h);
    return e;
  };
  auto dev = [&](size_t bytes) -> void * {
    void *p = rn_dev_alloc(ctx, bytes ? bytes : 16);
    if (p) {
      try {
        h->bufs.push_back(p);
      } catch (...) {
        rn_dev_free(ctx, p);
        return nullptr;
      }
    }
    return p;
  };
  auto nomem = [&]() { return fail(rn_fail(ctx, RN_ENOMEM, "rn_hierarchy_build: device allocation")); };
  rn_matrix Al = *A;
  const double *Bl = B;
  try {
    for (;;) {
      h->lv.push_back(rn_hierarchy::Level());
      rn_hierarchy::Level &L = h->lv.back();
      L.A = Al;
      L.B = Bl;
      L.nB = nB;
      const int m = Al.block_m, nn = Al.n / (m > 0 ? m : 1);
      if ((int32_t)h->lv.size() >= max_levels || Al.n <= min_coarse) break;
      // strength on the device, aggregation on the host (the same rules as
      // rn_aggregate_host's stage call)
      int64_t nnzS = 0;
      int32_t *Sp = (int32_t *)rn_dev_alloc(ctx, (size_t)(nn + 1) * 4);
      if (!Sp) return nomem();
      if ((st = rn_strength(ctx, &Al, theta, Sp, nullptr, &nnzS)) != RN_OK) {
        rn_dev_free(ctx, Sp);
        return fail(st);
      }
      int32_t *Sj = (int32_t *)rn_dev_alloc(ctx, (size_t)(nnzS + 1) * 4);
      if (!Sj) {
        rn_dev_free(ctx, Sp);
        return nomem();
      }
      if ((st = rn_strength(ctx, &Al, theta, Sp, Sj, &nnzS)) != RN_OK) {
        rn_dev_free(ctx, Sp);
        rn_dev_free(ctx, Sj);
        return fail(st);
      }
      std::vector<int32_t> hSp((size_t)nn + 1), hSj((size_t)nnzS + 1), hagg((size_t)nn + 1), hroots((size_t)nn + 1);
      hipError_t e = hipMemcpyAsync(hSp.data(), Sp, (size_t)(nn + 1) * 4, hipMemcpyDeviceToHost, ctx->stream);
      if (e == hipSuccess && nnzS > 0)
        e = hipMemcpyAsync(hSj.data(), Sj, (size_t)nnzS * 4, hipMemcpyDeviceToHost, ctx->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
      rn_dev_free(ctx, Sp);
      rn_dev_free(ctx, Sj);
      if (e != hipSuccess) return fail(rn_fail(ctx, RN_EHIP, "rn_hierarchy_build: %s", hipGetErrorString(e)));
      int32_t n_agg = 0;
      if ((st = rn_aggregate_host(nn, hSp.data(), hSj.data(), hagg.data(), hroots.data(), &n_agg)) != RN_OK)
        return fail(st);
      const int32_t nc = m * n_agg;
      if (n_agg == 0 || nc >= Al.n) break;  // this level does not coarsen: it is the coarsest
      L.agg = (int32_t *)dev((size_t)nn * 4);
      L.roots = (int32_t *)dev((size_t)n_agg * 4);
      if (!L.agg || !L.roots) return nomem();
      L.n_agg = n_agg;
      e = hipMemcpyAsync(L.agg, hagg.data(), (size_t)nn * 4, hipMemcpyHostToDevice, ctx->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(L.roots, hroots.data(), (size_t)n_agg * 4, hipMemcpyHostToDevice, ctx->stream);
      // (the host vectors must outlive the copies)
      if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
      if (e != hipSuccess) return fail(rn_fail(ctx, RN_EHIP, "rn_hierarchy_build: %s", hipGetErrorString(e)));
      // the level's set-up and its Galerkin product
      if ((st = rn_setup(ctx, &Al, L.agg, L.roots, n_agg, Bl, method == RN_GMRES ? Bl : nullptr, nB, degree, iters,
                         theta, method, precision, &L.s, &L.stats, &L.stats_RT)) != RN_OK)
        return fail(st);
      rn_setup_view sv;
      rn_setup_view_get(L.s, &sv);
      int32_t *Acp = (int32_t *)dev((size_t)(nc + 1) * 4);
      if (!Acp) return nomem();
      int64_t nnzAc = 0;
      const double *RT = method == RN_GMRES ? sv.RT : nullptr;
      if ((st = rn_galerkin(ctx, &Al, nc, sv.N_rowptr, sv.N_colind, sv.nnz_N, sv.P, RT, Acp, nullptr, nullptr,
                            &nnzAc)) != RN_OK)
        return fail(st);
      int32_t *Acj = (int32_t *)dev((size_t)(nnzAc + 1) * 4);
      double *Acv = (double *)dev((size_t)(nnzAc + 1) * 8);
      if (!Acj || !Acv) return nomem();
      if ((st = rn_galerkin(ctx, &Al, nc, sv.N_rowptr, sv.N_colind, sv.nnz_N, sv.P, RT, Acp, Acj, Acv, &nnzAc)) !=
          RN_OK)
        return fail(st);
      Al = rn_matrix{nc, 1, nnzAc, Acp, Acj, Acv};
      Bl = sv.Bc;
    }
  } catch (...) {
    return fail(rn_fail(ctx, RN_ENOMEM, "rn_hierarchy_build: host allocation"));
  }
  *out = h;
  return RN_OK;
}
