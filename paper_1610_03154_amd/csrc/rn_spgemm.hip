// rn_spgemm.hip -- the masked product Z = Pi(M(A X)) of the energy
// minimisation (Sec. 3.6: the product A P whose fill outside the pattern is
// dropped, then the projection onto U Bc = 0 with root rows fixed).
//
// One lane per pattern entry (per 2x2 block of node entries when A is
// node-blocked); a block owns the rows whose first entry lies in its chunk,
// so it holds <= 256 entries and whole rows.  The per-block header (row,
// entry and A ranges) is the only load the rest depends on: row metadata,
// the block's slice of A with the first pattern entry of each neighbour row,
// each lane's record (position codes and its row within the block, fixed
// stride per entry), its column and its own Krylov value all load in one
// round; X and the row's projection data are gathered in the next.  Terms are added one at a time in the
// order of A's row.  Per-row sums of the projection go through LDS in
// pattern order.  Krylov dot products are fused into the epilogue as
// per-block partials (no inter-block synchronisation).
#include <cstring>
#include <type_traits>

#include "rn_emin.h"

// Byte offsets from a uniform base are formed in 32 bits (the plan keeps
// every array of the product below 2^29 elements), so each load is one
// scalar-base + vector-offset instruction with no 64-bit address arithmetic.
template <class T>
__device__ inline T spg_ld(const T *base, uint32_t i) {
  return *(const T *)((const char *)base + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ inline void spg_st(T *base, uint32_t i, T v) {
  *(T *)((char *)base + i * (uint32_t)sizeof(T)) = v;
}

template <int M, int NB, bool MIXED, int BS>
struct SpgShape {
  using TV = typename std::conditional<MIXED, float, double>::type;
  static constexpr int NO = M * M;
  static constexpr int ACAP = (M == 1 ? SPG_ACAP : SPG_ACAP / 2) * BS / RN_BLOCK;  // staged A entries
  static constexpr int NIT = ACAP / BS;                                          // staging loads per thread
  static constexpr size_t P1 = (size_t)ACAP * (sizeof(int) * M + NO * sizeof(TV));
  static constexpr size_t P2 = (size_t)M * NB * M * BS * sizeof(double);
  // + 128 bytes: the register path reads up to 15 entries past a row's start
  static constexpr size_t BYTES = (P1 > P2 ? P1 : P2) + 128;
};

template <int M, int NB, int MODE, bool MIXED, int BS>
__global__ __launch_bounds__(BS) void k_spgemm(const SpgParams p) {
  using SH = SpgShape<M, NB, MIXED, BS>;
  using TV = typename SH::TV;
  constexpr int NP = NB * (NB + 1) / 2;
  constexpr int NO = M * M;
  constexpr int ACAP = SH::ACAP, NIT = SH::NIT;
  constexpr int UMAX = 15;  // terms of the register path (records of <= 16 bytes)
  __shared__ int s_rp[BS + 1];   // row starts, relative to the block's first entry
  __shared__ int s_ap[BS + 1];   // row starts in A, relative to the block's first A entry
  __shared__ int s_np0[M == 2 ? BS : 1], s_np1[M == 2 ? BS : 1];
  __shared__ uint8_t s_root[BS];
  __shared__ double s_w[8];
  __shared__ __align__(16) unsigned char s_buf[SH::BYTES];
  // phase 1 view: neighbour row starts and A values
  int *s_x0 = (int *)s_buf;
  int *s_x1 = s_x0 + ACAP;  // block_m = 2 only
  TV *s_ax = (TV *)(s_buf + (size_t)ACAP * sizeof(int) * M);
  // phase 2 view: per-entry projection terms
  double(*s_red)[NB][M * BS] = (double(*)[NB][M * BS])s_buf;

  const int blk = rn_xcd_block(blockIdx.x, p.nblk);
  if (blk < 0) return;
  const int b = blockIdx.y;
  const int32_t *st = p.st + (int64_t)b * ST_STRIDE;
  const double *sc = p.scal + (int64_t)b * p.scal_stride;
  if (MODE == MODE_CG_STEP || MODE == MODE_GM_STEP)
    if (st[ST_STATUS] || st[ST_DONE]) return;
  if (p.kact >= 0 && st[ST_ITERS] <= p.kact) return;

  const int4 h0 = ((const int4 *)p.blk_hdr)[2 * blk];
  const int4 h1 = ((const int4 *)p.blk_hdr)[2 * blk + 1];
  const int r0 = h0.x, nrows = h0.y - h0.x, e0 = h0.z, ne = h0.w - h0.z;
  const int aB = h1.x, naB = h1.y - h1.x, namax = h1.z;
  const bool staged = naB <= ACAP;
  const TV *Ax = (const TV *)p.Ax + (int64_t)b * p.strideA;
  const TV *X = (const TV *)p.X + (int64_t)b * p.strideX;
  const int64_t zb = (int64_t)b * p.strideZ;
  double *Z = p.Z + zb;
  const int32_t *rp = (M == 1) ? p.Np : p.nodeptr;
  const int t = threadIdx.x;
  const bool valid = t < ne;
  const bool proj = (MODE != MODE_PRODUCT) || p.project;
  const uint32_t *codes = (const uint32_t *)p.codes;

  // ---- one round of loads that depend on the header only ----
  // Straight-line code with clamped, always in-bounds indices, so every load
  // is issued before the first wait (a block has >= 1 entry and >= 1 row).
  // The lane's record: its codes, then CODE_NONE padding, and in the last
  // byte its row within the block; the code array carries 16 bytes of slack.
  const int nw = p.cstride >> 2;
  const int te = valid ? t : 0;
  const uint32_t rec = (uint32_t)(e0 + te) * (uint32_t)nw;
  // records of up to 12 bytes load as one vector (one cache access per line)
  uint32_t w0, w1, w2, w3;
  if (nw <= 3) {
    const uint3 r3 = *(const uint3 *)((const char *)codes + rec * 4u);  // 4-byte aligned
    w0 = r3.x;
    w1 = r3.y;
    w2 = r3.z;
    w3 = 0xffffffffu;
  } else {
    w0 = spg_ld(codes, rec);
    w1 = spg_ld(codes, rec + 1);
    w2 = spg_ld(codes, rec + 2);
    w3 = spg_ld(codes, rec + 3);
  }
  const uint32_t wl = nw == 1 ? w0 : nw == 2 ? w1 : nw == 3 ? w2 : nw == 4 ? w3 : spg_ld(codes, rec + nw - 1);
  int jc0 = 0;
  if (proj) jc0 = (M == 1) ? spg_ld(p.Nj, (uint32_t)(e0 + te)) : spg_ld(p.ncol, (uint32_t)(e0 + te));
  double ownv[NO];
#pragma unroll
  for (int o = 0; o < NO; ++o) ownv[o] = 0.0;
  if constexpr (M == 1)
    if (MODE == MODE_CG_STEP) ownv[0] = spg_ld(p.Xown + zb, (uint32_t)(e0 + te));
  // row metadata: thread rr holds row rr (row 256's start is read below)
  const int rq = t < nrows ? t : nrows - 1;
  const int rt = t < nrows ? t : nrows;
  const int v_rp = spg_ld(rp, (uint32_t)(r0 + rt));
  const int v_ap = spg_ld(p.Ap, (uint32_t)(r0 + rt));
  const uint8_t v_root = spg_ld(p.is_root, (uint32_t)((M == 1) ? r0 + rq : 2 * (r0 + rq)));
  int v_np0 = 0, v_np1 = 0;
  if constexpr (M == 2) {
    v_np0 = spg_ld(p.Np, (uint32_t)(2 * (r0 + rq)));
    v_np1 = spg_ld(p.Np, (uint32_t)(2 * (r0 + rq) + 1));
  }
  // the block's slice of A
  int v_x0[NIT], v_x1[NIT];
  TV v_ax[NIT][NO];
  if (staged && naB > 0) {
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      v_x0[it] = 0;
      v_x1[it] = 0;
#pragma unroll
      for (int o = 0; o < NO; ++o) v_ax[it][o] = 0;
      if (it * BS < naB) {  // uniform
        const uint32_t q = (uint32_t)(aB + (t + it * BS < naB ? t + it * BS : naB - 1));
        if constexpr (M == 1) {
          v_x0[it] = spg_ld(p.xoff, q);
        } else {
          v_x0[it] = spg_ld(p.xoff, 2 * q);
          v_x1[it] = spg_ld(p.xoff, 2 * q + 1);
        }
#pragma unroll
        for (int o = 0; o < NO; ++o) v_ax[it][o] = spg_ld(Ax, q * NO + o);
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
  if (nrows == BS && t == 0) {
    s_rp[BS] = rp[r0 + BS] - e0;
    s_ap[BS] = p.Ap[r0 + BS] - aB;
  }
  if (staged && naB > 0) {
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int q = t + it * BS;
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
  double bc[M][NB], gq[M][NP];
#pragma unroll
  for (int c = 0; c < M; ++c) {
#pragma unroll
    for (int q = 0; q < NB; ++q) bc[c][q] = 0.0;
#pragma unroll
    for (int q = 0; q < NP; ++q) gq[c][q] = 0.0;
  }
  double z[NO];
  int zi[NO];
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    z[o] = 0.0;
    zi[o] = -1;
  }
  const int lrow = valid ? (int)(wl >> 24) : 0;
  const bool froot = !valid || s_root[lrow];
  if (valid) {
    const int la = s_ap[lrow];
    const int r = t - s_rp[lrow];
    if (proj) {  // root lanes load too (their row and column are in range): no branch
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const uint32_t grow = (M == 1) ? (uint32_t)(r0 + lrow) : (uint32_t)(2 * (r0 + lrow) + c);
#pragma unroll
        for (int q = 0; q < NP; ++q) gq[c][q] = spg_ld(p.gp, grow * NP + q);
#pragma unroll
        for (int q = 0; q < NB; ++q) bc[c][q] = spg_ld(p.Bc, (uint32_t)(M * jc0 + c) * NB + q);
      }
    }
    if constexpr (M == 1) {
      zi[0] = e0 + t;
      if (!froot && staged && nw <= 4) {
        // every X load of the row issued before the first multiply-add; the
        // term count is the block's longest row (uniform), a miss (codes past
        // a row's length are CODE_NONE) loads X[0]
        TV xv[UMAX];
        uint32_t hitm = 0;
#pragma unroll
        for (int u = 0; u < UMAX; ++u) {
          xv[u] = 0;
          if (u < namax) {  // uniform
            const uint32_t w = u < 4 ? w0 : (u < 8 ? w1 : (u < 12 ? w2 : w3));
            const uint32_t c = __builtin_amdgcn_ubfe(w, 8 * (u & 3), 8);
            const bool hit = c != CODE_NONE;
            hitm |= (uint32_t)hit << u;
            xv[u] = spg_ld(X, hit ? (uint32_t)s_x0[la + u] + c : 0u);
          }
        }
        TV acc = 0;
#pragma unroll
        for (int u = 0; u < UMAX; ++u)
          if (u < namax) acc += ((hitm >> u) & 1u) ? s_ax[la + u] * xv[u] : TV(0);
        z[0] = (double)acc;
      } else if (!froot) {
        const int na = s_ap[lrow + 1] - la;
        TV acc = 0;
        for (int t0 = 0; t0 < na; t0 += 4) {
          const uint32_t w = spg_ld(codes, rec + (t0 >> 2));
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
          if (zi[o] >= 0) ownv[o] = spg_ld(p.Xown + zb, (uint32_t)zi[o]);
      if (!froot) {
        const int na = s_ap[lrow + 1] - la;
        TV z00 = 0, z01 = 0, z10 = 0, z11 = 0;
        for (int t0 = 0; t0 < na; t0 += 4) {
          const uint32_t w = nw <= 4 ? (t0 == 0 ? w0 : (t0 == 4 ? w1 : (t0 == 8 ? w2 : w3)))
                                     : spg_ld(codes, rec + (t0 >> 2));
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int tt = t0 + u;
            const uint32_t c = (w >> (8 * u)) & 0xffu;
            if (tt >= na || c == CODE_NONE) continue;  // the record's last byte is no code
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
              x00 = spg_ld(X, (uint32_t)x0);
              x11 = spg_ld(X, (uint32_t)x1);
              x01 = 0;
              x10 = 0;
            } else {
              x00 = spg_ld(X, (uint32_t)(x0 + 2 * (int)c));
              x01 = spg_ld(X, (uint32_t)(x0 + 2 * (int)c + 1));
              x10 = spg_ld(X, (uint32_t)(x1 + 2 * (int)c));
              x11 = spg_ld(X, (uint32_t)(x1 + 2 * (int)c + 1));
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

  // ---- projection Pi_B on F rows (root rows stay zero): every lane sums
  // its row's terms in pattern order and applies the row's G^+ itself ----
  if (proj) {
    __syncthreads();  // phase 1 LDS (A staging) is reused
    if (valid) {
#pragma unroll
      for (int c = 0; c < M; ++c)
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
          for (int cc = 0; cc < M; ++cc) s_red[c][q][M * t + cc] = froot ? 0.0 : z[c * M + cc] * bc[cc][q];
    }
    __syncthreads();
    if (!froot) {
      const int s = M * s_rp[lrow], e = M * s_rp[lrow + 1];
#pragma unroll
      for (int c = 0; c < M; ++c) {
        double sv[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) sv[q] = 0.0;
        for (int u = s; u < e; ++u)
#pragma unroll
          for (int q = 0; q < NB; ++q) sv[q] += s_red[c][q][u];
        double y[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          y[q] = 0.0;
#pragma unroll
          for (int r2 = 0; r2 < NB; ++r2) y[q] += gq[c][rn_pk(NB, q, r2)] * sv[r2];
        }
#pragma unroll
        for (int cc = 0; cc < M; ++cc) {
          double u = 0.0;
#pragma unroll
          for (int q = 0; q < NB; ++q) u += bc[cc][q] * y[q];
          z[c * M + cc] -= u;
        }
      }
    }
  }

  // ---- epilogues: outputs and per-block partials of the fused dots ----
  double *part = p.part + (int64_t)b * RN_MAXDOT * p.nblk;
  if (MODE == MODE_PRODUCT) {
#pragma unroll
    for (int o = 0; o < NO; ++o)
      if (zi[o] >= 0) spg_st(Z, (uint32_t)zi[o], p.accum ? spg_ld((const double *)Z, (uint32_t)zi[o]) + z[o] : z[o]);
    return;
  }
  if (MODE == MODE_CG_INIT || MODE == MODE_GM_INIT) {
    RnAcc d;
#pragma unroll
    for (int o = 0; o < NO; ++o)
      if (zi[o] >= 0) {
        const double v = -z[o];
        spg_st(Z, (uint32_t)zi[o], v);
        if (p.Z2) spg_st(p.Z2 + zb, (uint32_t)zi[o], v);
        d.add(v * v);
      }
    const double S = rn_block_sum2_w<BS / RN_WAVE>(d.hi, d.lo, s_w);
    if (threadIdx.x == 0) part[blk] = S;
    return;
  }
  if (MODE == MODE_CG_STEP) {
    RnAcc d;
#pragma unroll
    for (int o = 0; o < NO; ++o)
      if (zi[o] >= 0) {
        spg_st(Z, (uint32_t)zi[o], z[o]);
        d.add(ownv[o] * z[o]);
      }
    const double S = rn_block_sum2_w<BS / RN_WAVE>(d.hi, d.lo, s_w);
    if (threadIdx.x == 0) part[blk] = S;
    return;
  }
  if (MODE == MODE_GM_STEP) {
#pragma unroll
    for (int o = 0; o < NO; ++o)
      if (zi[o] >= 0) spg_st(Z, (uint32_t)zi[o], z[o]);
    const double *U = p.U + (int64_t)b * p.Ubatch;
    for (int j = 0; j <= p.k; ++j) {
      const double *Uj = U + (int64_t)j * p.nnzN;
      RnAcc d;
#pragma unroll
      for (int o = 0; o < NO; ++o)
        if (zi[o] >= 0) d.add(spg_ld(Uj, (uint32_t)zi[o]) * z[o]);
      const double S = rn_block_sum2_w<BS / RN_WAVE>(d.hi, d.lo, s_w);
      if (threadIdx.x == 0) part[(int64_t)j * p.nblk + blk] = S;
    }
  }
}

template <int M, int NB, int MODE>
static void launch_m(const SpgParams &p, int batch, bool mixed, hipStream_t s) {
  const dim3 grid(rn_xcd_grid((unsigned)p.nblk), (unsigned)batch);
  if (M == 1 && p.bs == 128) {
    if (mixed) hipLaunchKernelGGL((k_spgemm<M, NB, MODE, true, 128>), grid, dim3(128), 0, s, p);
    else hipLaunchKernelGGL((k_spgemm<M, NB, MODE, false, 128>), grid, dim3(128), 0, s, p);
  } else if (M == 1 && p.bs == 64) {
    if (mixed) hipLaunchKernelGGL((k_spgemm<M, NB, MODE, true, 64>), grid, dim3(64), 0, s, p);
    else hipLaunchKernelGGL((k_spgemm<M, NB, MODE, false, 64>), grid, dim3(64), 0, s, p);
  } else {
    if (mixed) hipLaunchKernelGGL((k_spgemm<M, NB, MODE, true, RN_BLOCK>), grid, dim3(RN_BLOCK), 0, s, p);
    else hipLaunchKernelGGL((k_spgemm<M, NB, MODE, false, RN_BLOCK>), grid, dim3(RN_BLOCK), 0, s, p);
  }
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
  p.bs = pl->bs;
  p.kact = -1;
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
