// rn_spgemm.hip -- the masked product Z = Pi(M(A X)) of the energy
// minimisation (Sec. 3.6: the product A P whose fill outside the pattern is
// dropped, then the projection onto U Bc = 0 with root rows fixed).
//
// One lane per pattern entry (per 2x2 block of node entries when A is
// node-blocked); a block owns the rows whose first entry lies in its chunk,
// so it holds <= 256 entries and whole rows.  The per-block header (row,
// entry and A ranges) is the only load the rest depends on: row metadata,
// the block's slice of A with the first pattern entry of each neighbour row,
// each lane's position codes (fixed stride per entry), its column, its own
// Krylov value and the projection data of the row it reduces all load in one
// round; X is gathered in the next.  Terms are added one at a time in the
// order of A's row.  Per-row sums of the projection go through LDS in
// pattern order.  Krylov dot products are fused into the epilogue as
// per-block partials (no inter-block synchronisation).
#include <cstring>
#include <type_traits>

#include "rn_emin.h"

template <int M, int NB, bool MIXED>
struct SpgSmem {
  using TV = typename std::conditional<MIXED, float, double>::type;
  static constexpr int NO = M * M;
  static constexpr size_t P1 = SPG_ACAP * sizeof(int) * M + SPG_ACAP * NO * sizeof(TV);
  static constexpr size_t P2 = (size_t)M * NB * (M * RN_BLOCK + RN_BLOCK) * sizeof(double);
  static constexpr size_t BYTES = P1 > P2 ? P1 : P2;
};

// Local row of entry t: the largest rr < nrows with s_rp[rr] <= t (rows are
// never empty, so s_rp is strictly increasing).
__device__ inline int spg_row_of(const int *s_rp, int nrows, int t) {
  int lo = 0, hi = nrows;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (s_rp[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

template <int M, int NB, int MODE, bool MIXED>
__global__ __launch_bounds__(RN_BLOCK) void k_spgemm(const SpgParams p) {
  using SM = SpgSmem<M, NB, MIXED>;
  using TV = typename SM::TV;
  constexpr int NP = NB * (NB + 1) / 2;
  constexpr int NO = M * M;
  __shared__ int s_rp[RN_BLOCK + 1];   // row starts, relative to the block's first entry
  __shared__ int s_ap[RN_BLOCK + 1];   // row starts in A, relative to the block's first A entry
  __shared__ int s_np0[M == 2 ? RN_BLOCK : 1], s_np1[M == 2 ? RN_BLOCK : 1];
  __shared__ uint8_t s_root[RN_BLOCK];
  __shared__ double s_w[8];
  __shared__ __align__(16) unsigned char s_buf[SM::BYTES];
  // phase 1 view: neighbour row starts and A values
  int *s_x0 = (int *)s_buf;
  int *s_x1 = s_x0 + SPG_ACAP;  // block_m = 2 only
  TV *s_ax = (TV *)(s_buf + SPG_ACAP * sizeof(int) * M);
  // phase 2 view: projection sums
  double(*s_red)[NB][M * RN_BLOCK] = (double(*)[NB][M * RN_BLOCK])s_buf;
  double(*s_y)[NB][RN_BLOCK] = (double(*)[NB][RN_BLOCK])(s_buf + (size_t)M * NB * M * RN_BLOCK * sizeof(double));

  const int blk = rn_xcd_block(blockIdx.x, p.nblk);
  if (blk < 0) return;
  const int b = blockIdx.y;
  const int32_t *st = p.st + (int64_t)b * ST_STRIDE;
  const double *sc = p.scal + (int64_t)b * p.scal_stride;
  if (MODE == MODE_CG_STEP || MODE == MODE_GM_STEP)
    if (st[ST_STATUS] || st[ST_DONE]) return;

  const int4 h0 = ((const int4 *)p.blk_hdr)[2 * blk];
  const int4 h1 = ((const int4 *)p.blk_hdr)[2 * blk + 1];
  const int r0 = h0.x, nrows = h0.y - h0.x, e0 = h0.z, ne = h0.w - h0.z;
  const int aB = h1.x, naB = h1.y - h1.x;
  const bool staged = naB <= SPG_ACAP;
  const TV *Ax = (const TV *)p.Ax + (int64_t)b * p.strideA;
  const TV *X = (const TV *)p.X + (int64_t)b * p.strideX;
  const int64_t zb = (int64_t)b * p.strideZ;
  const int32_t *rp = (M == 1) ? p.Np : p.nodeptr;
  const int t = threadIdx.x;
  const bool valid = t < ne;
  const bool proj = (MODE != MODE_PRODUCT) || p.project;

  // ---- one round of loads that depend on the header only ----
  // Straight-line code with clamped, always in-bounds indices, so every load
  // is issued before the first wait (a block has >= 1 entry and >= 1 row).
  // the lane's column (node column for block_m = 2), codes and own value;
  // the code array carries 16 bytes of slack, so three words are always
  // readable
  const int nw = p.cstride >> 2;
  const int te = valid ? t : 0;
  const uint32_t *cwp = (const uint32_t *)(p.codes + (int64_t)(e0 + t) * p.cstride);
  const uint32_t *cwq = (const uint32_t *)(p.codes + (int64_t)(e0 + te) * p.cstride);
  const int jc0 = (M == 1) ? p.Nj[e0 + te] : p.ncol[e0 + te];
  const uint32_t cw0 = cwq[0], cw1 = nw > 1 ? cwq[1] : 0xffffffffu, cw2 = nw > 2 ? cwq[2] : 0xffffffffu;
  double ownv[NO];
#pragma unroll
  for (int o = 0; o < NO; ++o) ownv[o] = 0.0;
  if constexpr (M == 1)
    if (MODE == MODE_CG_STEP) ownv[0] = p.Xown[zb + e0 + te];
  // row metadata: thread rr holds row rr (rows <= 256; row 256's start is
  // read separately below)
  const int rq = t < nrows ? t : nrows - 1;
  const int v_rp = rp[r0 + t < r0 + nrows ? r0 + t : r0 + nrows];
  const int v_ap = p.Ap[r0 + t < r0 + nrows ? r0 + t : r0 + nrows];
  const uint8_t v_root = p.is_root[(M == 1) ? r0 + rq : 2 * (r0 + rq)];
  int v_np0 = 0, v_np1 = 0;
  if constexpr (M == 2) {
    v_np0 = p.Np[2 * (r0 + rq)];
    v_np1 = p.Np[2 * (r0 + rq) + 1];
  }
  // projection data of the row this thread reduces in the first pass
  double gpre[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) gpre[q] = 0.0;
  if (proj) {
    const int tg = t < nrows * M ? t : 0;
    const int grow = (M == 1) ? r0 + tg : 2 * (r0 + tg / M) + tg % M;
#pragma unroll
    for (int q = 0; q < NP; ++q) gpre[q] = p.gp[(int64_t)grow * NP + q];
  }
  // the block's slice of A: at most SPG_ACAP / RN_BLOCK entries per thread
  constexpr int NIT = SPG_ACAP / RN_BLOCK;
  int v_x0[NIT], v_x1[NIT];
  TV v_ax[NIT][NO];
  if (staged && naB > 0) {
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      v_x0[it] = 0;
      v_x1[it] = 0;
#pragma unroll
      for (int o = 0; o < NO; ++o) v_ax[it][o] = 0;
      if (it * RN_BLOCK < naB) {  // uniform
        const int q = aB + (t + it * RN_BLOCK < naB ? t + it * RN_BLOCK : naB - 1);
        if constexpr (M == 1) {
          v_x0[it] = p.xoff[q];
        } else {
          v_x0[it] = p.xoff[2 * q];
          v_x1[it] = p.xoff[2 * q + 1];
        }
#pragma unroll
        for (int o = 0; o < NO; ++o) v_ax[it][o] = Ax[(int64_t)q * NO + o];
      }
    }
  }
  // LDS stores once everything is in flight
  if (t <= nrows) {
    s_rp[t] = v_rp - e0;
    s_ap[t] = v_ap - aB;
  }
  if (t < nrows) {
    s_root[t] = v_root;
    if constexpr (M == 2) {
      s_np0[t] = v_np0;
      s_np1[t] = v_np1;
    }
  }
  if (nrows == RN_BLOCK && t == 0) {
    s_rp[RN_BLOCK] = rp[r0 + RN_BLOCK] - e0;
    s_ap[RN_BLOCK] = p.Ap[r0 + RN_BLOCK] - aB;
  }
  if (staged && naB > 0) {
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int q = t + it * RN_BLOCK;
      if (q < naB) {
        s_x0[q] = v_x0[it];
        if constexpr (M == 2) s_x1[q] = v_x1[it];
#pragma unroll
        for (int o = 0; o < NO; ++o) s_ax[q * NO + o] = v_ax[it][o];
      }
    }
  }
  __syncthreads();

  // ---- the product: X gathered in the second round ----
  double bc[M][NB];
  int jc[M];
#pragma unroll
  for (int c = 0; c < M; ++c) {
    jc[c] = M * jc0 + c;
#pragma unroll
    for (int q = 0; q < NB; ++q) bc[c][q] = 0.0;
  }
  double z[NO];
  int64_t zi[NO];
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    z[o] = 0.0;
    zi[o] = -1;
  }
  int lrow = 0;
  bool froot = true;
  if (valid) {
    lrow = spg_row_of(s_rp, nrows, t);
    froot = s_root[lrow];
    const int la = s_ap[lrow], na = s_ap[lrow + 1] - la;
    const int r = t - s_rp[lrow];
    if (proj)  // root lanes load too (their column is in range): no branch
#pragma unroll
      for (int c = 0; c < M; ++c)
#pragma unroll
        for (int q = 0; q < NB; ++q) bc[c][q] = p.Bc[(int64_t)jc[c] * NB + q];
    if constexpr (M == 1) {
      zi[0] = e0 + t;
      if (!froot && staged && nw <= 3) {
        // every X load of the row issued before the first multiply-add:
        // straight-line code, a miss (codes past the row's length are
        // CODE_NONE) loads X[0]
        TV xv[12], av[12];
        bool hit[12];
#pragma unroll
        for (int u = 0; u < 12; ++u) {
          const uint32_t w = u < 4 ? cw0 : (u < 8 ? cw1 : cw2);
          const uint32_t c = (w >> (8 * (u & 3))) & 0xffu;
          hit[u] = c != CODE_NONE;
          const int q = la + (hit[u] ? u : 0);
          av[u] = s_ax[q];
          xv[u] = X[hit[u] ? s_x0[q] + (int)c : 0];
        }
        TV acc = 0;
#pragma unroll
        for (int u = 0; u < 12; ++u) acc += hit[u] ? av[u] * xv[u] : TV(0);
        z[0] = (double)acc;
      } else if (!froot) {
        TV acc = 0;
        for (int t0 = 0; t0 < na; t0 += 4) {
          const uint32_t w = cwp[t0 >> 2];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int tt = t0 + u;
            if (tt < na) {
              const uint32_t c = (w >> (8 * u)) & 0xffu;
              const bool hit = c != CODE_NONE;
              const TV a = staged ? s_ax[la + tt] : Ax[aB + la + tt];
              TV x = 0;
              if (hit) x = X[(staged ? s_x0[la + tt] : p.xoff[aB + la + tt]) + (int)c];
              acc += hit ? a * x : TV(0);
            }
          }
        }
        z[0] = (double)acc;
      }
    } else {
      const int s0 = s_np0[lrow], s1 = s_np1[lrow];
      if (froot) {
        zi[0] = s0;
        zi[M] = s1;
      } else {
        zi[0] = s0 + 2 * r;
        zi[1] = s0 + 2 * r + 1;
        zi[M] = s1 + 2 * r;
        zi[M + 1] = s1 + 2 * r + 1;
      }
      if (MODE == MODE_CG_STEP)
#pragma unroll
        for (int o = 0; o < NO; ++o)
          if (zi[o] >= 0) ownv[o] = p.Xown[zb + zi[o]];
      if (!froot) {
        TV z00 = 0, z01 = 0, z10 = 0, z11 = 0;
        for (int t0 = 0; t0 < na; t0 += 4) {
          const uint32_t w = nw <= 3 ? (t0 == 0 ? cw0 : (t0 == 4 ? cw1 : cw2)) : cwp[t0 >> 2];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t c = (w >> (8 * u)) & 0xffu;
            if (c == CODE_NONE) continue;  // also every padding code
            const int tt = t0 + u;
            int x0, x1;
            const TV *a;
            if (staged) {
              x0 = s_x0[la + tt];
              x1 = s_x1[la + tt];
              a = s_ax + (la + tt) * NO;
            } else {
              x0 = p.xoff[2 * (aB + la + tt)];
              x1 = p.xoff[2 * (aB + la + tt) + 1];
              a = Ax + (int64_t)(aB + la + tt) * NO;
            }
            TV x00, x01, x10, x11;
            if (c == CODE_ROOT) {
              x00 = X[x0];
              x11 = X[x1];
              x01 = 0;
              x10 = 0;
            } else {
              x00 = X[x0 + 2 * (int)c];
              x01 = X[x0 + 2 * (int)c + 1];
              x10 = X[x1 + 2 * (int)c];
              x11 = X[x1 + 2 * (int)c + 1];
            }
            // one term at a time, in the order of the scalar row (2K, 2K+1)
            z00 += a[0] * x00;
            z00 += a[1] * x10;
            z01 += a[0] * x01;
            z01 += a[1] * x11;
            z10 += a[2] * x00;
            z10 += a[3] * x10;
            z11 += a[2] * x01;
            z11 += a[3] * x11;
          }
        }
        z[0] = (double)z00;
        z[1] = (double)z01;
        z[M] = (double)z10;
        z[M + 1] = (double)z11;
      }
    }
  }
  if (MODE == MODE_GM_STEP) {
    const double xs = sc[GmLayout(p.K).s + p.k];
#pragma unroll
    for (int o = 0; o < NO; ++o) z[o] *= xs;
  }
  __syncthreads();  // phase 1 LDS (A staging) is reused below

  // ---- projection Pi_B on F rows (root rows stay zero) ----
  if (proj) {
    if (valid) {
#pragma unroll
      for (int c = 0; c < M; ++c)
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
          for (int cc = 0; cc < M; ++cc) s_red[c][q][M * t + cc] = froot ? 0.0 : z[c * M + cc] * bc[cc][q];
    }
    __syncthreads();
    for (int w = threadIdx.x; w < nrows * M; w += RN_BLOCK) {
      const int lr = w / M, c = w % M;
      const int row = (M == 1) ? r0 + lr : 2 * (r0 + lr) + c;
      double sv[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) sv[q] = 0.0;
      // the row's entries in pattern order, summed one at a time
      const int s = M * s_rp[lr], e = M * s_rp[lr + 1];
      for (int u = s; u < e; ++u)
#pragma unroll
        for (int q = 0; q < NB; ++q) sv[q] += s_red[c][q][u];
      double g[NP];
#pragma unroll
      for (int q = 0; q < NP; ++q) g[q] = gpre[q];
      if (w != t)
#pragma unroll
        for (int q = 0; q < NP; ++q) g[q] = p.gp[(int64_t)row * NP + q];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        double y = 0.0;
#pragma unroll
        for (int r = 0; r < NB; ++r) y += g[rn_pk(NB, q, r)] * sv[r];
        s_y[c][q][lr] = y;
      }
    }
    __syncthreads();
    if (valid && !froot) {
#pragma unroll
      for (int c = 0; c < M; ++c)
#pragma unroll
        for (int cc = 0; cc < M; ++cc) {
          double u = 0.0;
#pragma unroll
          for (int q = 0; q < NB; ++q) u += bc[cc][q] * s_y[c][q][lrow];
          z[c * M + cc] -= u;
        }
    }
  }

  // ---- epilogues: outputs and per-block partials of the fused dots ----
  double *part = p.part + (int64_t)b * RN_MAXDOT * p.nblk;
  if (MODE == MODE_PRODUCT) {
#pragma unroll
    for (int o = 0; o < NO; ++o)
      if (zi[o] >= 0) p.Z[zb + zi[o]] = z[o];
    return;
  }
  if (MODE == MODE_CG_INIT || MODE == MODE_GM_INIT) {
    RnAcc d;
#pragma unroll
    for (int o = 0; o < NO; ++o)
      if (zi[o] >= 0) {
        const double v = -z[o];
        p.Z[zb + zi[o]] = v;
        if (p.Z2) p.Z2[zb + zi[o]] = v;
        d.add(v * v);
      }
    const double S = rn_block_sum2(d.hi, d.lo, s_w);
    if (threadIdx.x == 0) part[blk] = S;
    return;
  }
  if (MODE == MODE_CG_STEP) {
    RnAcc d;
#pragma unroll
    for (int o = 0; o < NO; ++o)
      if (zi[o] >= 0) {
        p.Z[zb + zi[o]] = z[o];
        d.add(ownv[o] * z[o]);
      }
    const double S = rn_block_sum2(d.hi, d.lo, s_w);
    if (threadIdx.x == 0) part[blk] = S;
    return;
  }
  if (MODE == MODE_GM_STEP) {
#pragma unroll
    for (int o = 0; o < NO; ++o)
      if (zi[o] >= 0) p.Z[zb + zi[o]] = z[o];
    const double *U = p.U + (int64_t)b * p.Ubatch;
    for (int j = 0; j <= p.k; ++j) {
      const double *Uj = U + (int64_t)j * p.nnzN;
      RnAcc d;
#pragma unroll
      for (int o = 0; o < NO; ++o)
        if (zi[o] >= 0) d.add(Uj[zi[o]] * z[o]);
      const double S = rn_block_sum2(d.hi, d.lo, s_w);
      if (threadIdx.x == 0) part[(int64_t)j * p.nblk + blk] = S;
    }
  }
}

template <int M, int NB, int MODE>
static void launch_m(const SpgParams &p, int batch, bool mixed, hipStream_t s) {
  const dim3 grid(rn_xcd_grid((unsigned)p.nblk), (unsigned)batch), block(RN_BLOCK);
  if (mixed) hipLaunchKernelGGL((k_spgemm<M, NB, MODE, true>), grid, block, 0, s, p);
  else hipLaunchKernelGGL((k_spgemm<M, NB, MODE, false>), grid, block, 0, s, p);
}

template <int MODE>
static rn_status launch_mode(rn_ctx *ctx, const rn_plan *pl, const SpgParams &p, int batch, bool mixed) {
  hipStream_t s = ctx->stream;
  if (pl->m == 1) {
    switch (pl->nB) {
      case 1: launch_m<1, 1, MODE>(p, batch, mixed, s); break;
      case 2: launch_m<1, 2, MODE>(p, batch, mixed, s); break;
      case 3: launch_m<1, 3, MODE>(p, batch, mixed, s); break;
      case 4: launch_m<1, 4, MODE>(p, batch, mixed, s); break;
      default: return rn_fail(ctx, RN_EINVAL, "nB out of range");
    }
  } else {
    switch (pl->nB) {
      case 2: launch_m<2, 2, MODE>(p, batch, mixed, s); break;
      case 3: launch_m<2, 3, MODE>(p, batch, mixed, s); break;
      case 4: launch_m<2, 4, MODE>(p, batch, mixed, s); break;
      default: return rn_fail(ctx, RN_EINVAL, "nB out of range for block_m = 2");
    }
  }
  LAUNCH_CHECK(ctx);
  return RN_OK;
}

rn_status rn_launch_spgemm(rn_ctx *ctx, const rn_plan *pl, int mode, const SpgParams &p, int batch, bool mixed) {
  if (p.nblk == 0) return RN_OK;
  switch (mode) {
    case MODE_PRODUCT: return launch_mode<MODE_PRODUCT>(ctx, pl, p, batch, mixed);
    case MODE_CG_INIT: return launch_mode<MODE_CG_INIT>(ctx, pl, p, batch, mixed);
    case MODE_CG_STEP: return launch_mode<MODE_CG_STEP>(ctx, pl, p, batch, mixed);
    case MODE_GM_INIT: return launch_mode<MODE_GM_INIT>(ctx, pl, p, batch, mixed);
    case MODE_GM_STEP: return launch_mode<MODE_GM_STEP>(ctx, pl, p, batch, mixed);
  }
  return rn_fail(ctx, RN_EINVAL, "bad product mode");
}

SpgParams rn_spg_params(const rn_plan *pl) {
  SpgParams p;
  memset(&p, 0, sizeof p);
  p.n = pl->n;
  p.nr = pl->nr;
  p.nblk = pl->nblk;
  p.nnzN = pl->nnzN;
  p.Ap = pl->Ap;
  p.Aj = pl->Aj;
  p.Np = pl->Np;
  p.Nj = pl->Nj;
  p.cstride = pl->cstride;
  p.ncol = pl->ncol;
  p.nodeptr = pl->nodeptr;
  p.blk_row = pl->blk_row;
  p.blk_hdr = pl->blk_hdr;
  p.xoff = pl->xoff;
  p.codes = pl->codes;
  p.is_root = pl->is_root;
  p.Bc = pl->Bc;
  p.gp = pl->gp;
  p.strideZ = pl->nnzN;
  p.strideX = pl->nnzN;
  p.strideA = pl->nnzA * pl->m * pl->m;
  return p;
}
