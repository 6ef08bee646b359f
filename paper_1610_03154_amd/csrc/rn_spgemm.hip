// rn_spgemm.hip -- the masked product Z = Pi(M(A X)) of the energy
// minimisation (Sec. 3.6: the product A P whose fill outside the pattern is
// dropped, then the projection onto U Bc = 0 with root rows fixed).
//
// One lane per pattern entry (per 2x2 block of node entries when A is
// node-blocked); a block owns the rows whose first entry lies in its chunk,
// so it holds <= 256 entries and whole rows.  The plan supplies, per block,
// a header (row, entry and A ranges) and, per stored A entry, the first
// pattern entry of the neighbour row, so a block stages its rows' metadata
// and its slice of A in LDS with one level of coalesced loads.  Each lane
// then reads its one-byte position codes four at a time and gathers X;
// terms are added one at a time in the order of A's row.  Per-row sums of
// the projection go through LDS in pattern order.  Krylov dot products are
// fused into the epilogue as per-block partials (no inter-block
// synchronisation).
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

template <int M, int NB, int MODE, bool MIXED>
__global__ __launch_bounds__(RN_BLOCK) void k_spgemm(const SpgParams p) {
  using SM = SpgSmem<M, NB, MIXED>;
  using TV = typename SM::TV;
  constexpr int NP = NB * (NB + 1) / 2;
  constexpr int NO = M * M;
  __shared__ int s_rp[RN_BLOCK + 1];   // row starts, relative to the block's first entry
  __shared__ int s_ap[RN_BLOCK + 1];   // row starts in A, relative to the block's first A entry
  __shared__ int s_cp[RN_BLOCK];       // code offsets
  __shared__ int s_np0[M == 2 ? RN_BLOCK : 1], s_np1[M == 2 ? RN_BLOCK : 1];
  __shared__ uint8_t s_root[RN_BLOCK];
  __shared__ uint8_t s_row[RN_BLOCK];
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
  const int32_t *rp = (M == 1) ? p.Np : p.nodeptr;
  const int t = threadIdx.x;
  const bool valid = t < ne;

  // ---- stage row metadata and the block's slice of A (one load level) ----
  for (int rr = t; rr <= nrows; rr += RN_BLOCK) {
    s_rp[rr] = rp[r0 + rr] - e0;
    s_ap[rr] = p.Ap[r0 + rr] - aB;
    if (rr < nrows) {
      s_cp[rr] = p.code_ptr[r0 + rr];
      if constexpr (M == 1) {
        s_root[rr] = p.is_root[r0 + rr];
      } else {
        s_root[rr] = p.is_root[2 * (r0 + rr)];
        s_np0[rr] = p.Np[2 * (r0 + rr)];
        s_np1[rr] = p.Np[2 * (r0 + rr) + 1];
      }
    }
  }
  if (staged) {
    for (int q = t; q < naB; q += RN_BLOCK) {
      if constexpr (M == 1) {
        s_x0[q] = p.xoff[aB + q];
      } else {
        s_x0[q] = p.xoff[2 * (aB + q)];
        s_x1[q] = p.xoff[2 * (aB + q) + 1];
      }
#pragma unroll
      for (int o = 0; o < NO; ++o) s_ax[q * NO + o] = Ax[(int64_t)(aB + q) * NO + o];
    }
  }
  // the lane's own column and candidates (block_m = 1) load meanwhile
  const bool proj = (MODE != MODE_PRODUCT) || p.project;
  double bc[M][NB];
  int jc[M];
#pragma unroll
  for (int c = 0; c < M; ++c) {
    jc[c] = 0;
#pragma unroll
    for (int q = 0; q < NB; ++q) bc[c][q] = 0.0;
  }
  if constexpr (M == 1) {
    if (valid) {
      jc[0] = p.Nj[e0 + t];
      if (proj)
#pragma unroll
        for (int q = 0; q < NB; ++q) bc[0][q] = p.Bc[(int64_t)jc[0] * NB + q];
    }
  }
  __syncthreads();
  for (int rr = t; rr < nrows; rr += RN_BLOCK)
    for (int q = s_rp[rr]; q < s_rp[rr + 1]; ++q) s_row[q] = (uint8_t)rr;
  __syncthreads();

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
    lrow = s_row[t];
    froot = s_root[lrow];
    const int la = s_ap[lrow], na = s_ap[lrow + 1] - la, na4 = (na + 3) & ~3;
    const int r = t - s_rp[lrow];
    if constexpr (M == 1) {
      zi[0] = e0 + t;
      if (!froot && na <= 12) {
        // fast path: every code, A value and X load of the row issued before
        // the first multiply-add (one memory latency per lane)
        const uint32_t *cw = (const uint32_t *)(p.codes + s_cp[lrow] + r * na4);
        const uint32_t w0 = cw[0];
        const uint32_t w1 = na > 4 ? cw[1] : 0xffffffffu;
        const uint32_t w2 = na > 8 ? cw[2] : 0xffffffffu;
        TV av[12], xv[12];
        bool hit[12];
#pragma unroll
        for (int u = 0; u < 12; ++u) {
          const uint32_t w = u < 4 ? w0 : (u < 8 ? w1 : w2);
          const uint32_t c = (w >> (8 * (u & 3))) & 0xffu;
          hit[u] = u < na && c != CODE_NONE;
          av[u] = 0;
          xv[u] = 0;
          if (u < na) {
            const int xo = staged ? s_x0[la + u] : p.xoff[aB + la + u];
            av[u] = staged ? s_ax[la + u] : Ax[aB + la + u];
            // safe index for a miss: the neighbour row's first entry
            xv[u] = X[xo + (hit[u] ? (int)c : 0)];
          }
        }
        TV acc = 0;
#pragma unroll
        for (int u = 0; u < 12; ++u) acc += hit[u] ? av[u] * xv[u] : TV(0);
        z[0] = (double)acc;
      } else if (!froot) {
        const uint32_t *cw = (const uint32_t *)(p.codes + s_cp[lrow] + r * na4);
        TV acc = 0;
        for (int t0 = 0; t0 < na; t0 += 4) {
          const uint32_t w = cw[t0 >> 2];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int tt = t0 + u;
            if (tt < na) {
              const uint32_t c = (w >> (8 * u)) & 0xffu;
              const bool hit = c != CODE_NONE;
              const int xo = staged ? s_x0[la + tt] : p.xoff[aB + la + tt];
              const TV a = staged ? s_ax[la + tt] : Ax[aB + la + tt];
              // safe index for a miss: the neighbour row's first entry
              const TV x = X[xo + (hit ? (int)c : 0)];
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
        jc[0] = p.Nj[s0 + 2 * r];
        jc[1] = jc[0] + 1;
        const uint32_t *cw = (const uint32_t *)(p.codes + s_cp[lrow] + r * na4);
        TV z00 = 0, z01 = 0, z10 = 0, z11 = 0;
        for (int t0 = 0; t0 < na; t0 += 4) {
          const uint32_t w = cw[t0 >> 2];
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
        if (proj)
#pragma unroll
          for (int cc = 0; cc < M; ++cc)
#pragma unroll
            for (int q = 0; q < NB; ++q) bc[cc][q] = p.Bc[(int64_t)jc[cc] * NB + q];
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
      const double *g = p.gp + (int64_t)row * NP;
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
  const int64_t zb = (int64_t)b * p.strideZ;
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
    const double *own = p.Xown + zb;
    RnAcc d;
#pragma unroll
    for (int o = 0; o < NO; ++o)
      if (zi[o] >= 0) {
        p.Z[zb + zi[o]] = z[o];
        d.add(own[zi[o]] * z[o]);
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
  p.code_ptr = pl->code_ptr;
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
