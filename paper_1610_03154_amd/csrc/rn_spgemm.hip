// rn_spgemm.hip -- the masked product Z = Pi(M(A X)) of the energy
// minimisation (Sec. 3.6: the product A P whose fill outside the pattern is
// dropped, then the projection onto U Bc = 0 with root rows fixed).
//
// One lane per pattern entry (per 2x2 block of node entries when A is
// node-blocked); a product block owns the rows whose first entry lies in its
// chunk, so it holds <= bs entries and whole rows.  The block's header (row,
// entry and A ranges) is the only load the rest depends on.  Terms are added
// one at a time in the order of A's row.  Per-row sums of the projection go
// through LDS in pattern order.  The CG dot products are fused into the
// epilogue as per-block partials (no inter-block synchronisation); the GMRES
// step only scales and stores its vector (its Gram-Schmidt dots run in their
// own streaming passes).
//
// k_spgemm (every operator): one product block per workgroup; the block's
// slice of A and the neighbour offsets are staged in LDS, X is gathered from
// global memory (from the block's X window in LDS when the plan built one).
// k_spgemm_p (scalar operators, n_B <= 2, records of <= 12 bytes):
// persistent workgroups that stage each block's X window, A slice, Bc rows
// and G^+ in one round of contiguous loads and prefetch the next block while
// computing the current one from LDS.
#include <cstdlib>
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

// two adjacent elements at element index i (i even, base aligned to the pair)
template <class T>
__device__ inline typename std::conditional<sizeof(T) == 8, double2, float2>::type spg_ld2(const T *base,
                                                                                           uint32_t i) {
  using T2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
  return *(const T2 *)((const char *)base + i * (uint32_t)sizeof(T));
}

template <int M, int NB, bool MIXED, int BS>
struct SpgShape {
  using TV = typename std::conditional<MIXED, float, double>::type;
  static constexpr int NO = M * M;
  static constexpr int ACAP = M == 1 ? SPG_ACAP_M1(BS) : SPG_ACAP / 2 * BS / RN_BLOCK;  // staged A entries
  static constexpr int NIT = (ACAP + BS - 1) / BS;                                    // staging loads per thread
  static constexpr int XCAP = M == 1 ? SPG_XCAP_M1(BS) : 0;                           // X window elements
  // block_m = 1, n_B <= 2: the rows' G^+ (read before the projection reuses the buffer)
  static constexpr size_t PG = (M == 1 && NB <= 2) ? (size_t)BS * (NB * (NB + 1) / 2) * sizeof(double) : 0;
  static constexpr size_t P1 =
      (size_t)ACAP * (sizeof(int) * M + NO * sizeof(TV)) + (size_t)XCAP * sizeof(TV) + PG;
  static constexpr size_t P2 = (size_t)M * NB * M * BS * sizeof(double);
  // block_m = 2: + 128 bytes, the term loop reads up to 15 entries past a row's
  // start (block_m = 1 over-reads land in the next region of the buffer)
  static constexpr size_t BYTES = (P1 > P2 ? P1 : P2) + (M == 2 ? 128 : 0);
};

template <int M, int NB, int MODE, bool MIXED, int BS>
__global__ __launch_bounds__(BS) void k_spgemm(const SpgParams p) {
  using SH = SpgShape<M, NB, MIXED, BS>;
  using TV = typename SH::TV;
  constexpr int NP = NB * (NB + 1) / 2;
  constexpr int NO = M * M;
  constexpr int ACAP = SH::ACAP, NIT = SH::NIT;
  constexpr int UMAX = 11;  // terms of the register path (records of <= 12 bytes)
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
  TV *s_xw = s_ax + ACAP * NO;  // block_m = 1: the X window
  double *s_gp = (double *)(s_xw + SH::XCAP);  // block_m = 1, n_B <= 2: the rows' G^+
  // phase 2 view: per-entry projection terms
  double(*s_red)[NB][M * BS] = (double(*)[NB][M * BS])s_buf;

  // block_m = 1 with n_B <= 2: each entry's Bc row comes from the plan and
  // the rows' G^+ are staged with the rest, so the projection data load in
  // the first round with everything else
  constexpr bool PRE = M == 1 && NB <= 2;
  // block_m = 1: A values and the X window as 32-bit words (contiguous 32-bit
  // loads cost the vector L1 about a third of 64-bit ones per byte); chunk c
  // of 64 words holds one window unit of doubles or two of floats
  constexpr int DPE = sizeof(TV) / 4;
  constexpr int NITD = M == 1 ? (ACAP * DPE + BS - 1) / BS : 1;
  constexpr int XIT = M == 1 ? SH::XCAP * DPE / BS : 1;
  constexpr int NUW = M == 1 ? (DPE == 2 ? XIT : 2 * XIT) : 1;

  const int blk = rn_xcd_block(blockIdx.x, p.nblk);
  if (blk < 0) return;
  const int b = blockIdx.y;
  const int t = threadIdx.x;
  // the header and the window's unit starts depend on the block index only:
  // they load together, before anything else
  const int4 h0 = ((const int4 *)p.blk_hdr)[2 * blk];
  const int4 h1 = ((const int4 *)p.blk_hdr)[2 * blk + 1];
  const int wv = __builtin_amdgcn_readfirstlane(t / RN_WAVE);
  int uwv[NUW];
  if constexpr (M == 1) {
    const int32_t *uw = p.xwin + (int64_t)blk * (SH::XCAP / XW_UNIT);
#pragma unroll
    for (int i = 0; i < XIT; ++i) {
      const int c = wv + i * (BS / RN_WAVE);
      if (DPE == 2) {
        uwv[i] = uw[c];
      } else {
        uwv[2 * i] = uw[2 * c];
        uwv[2 * i + 1] = uw[2 * c + 1];
      }
    }
  }
  const int32_t *st = p.st + (int64_t)b * ST_STRIDE;
  const double *sc = p.scal + (int64_t)b * p.scal_stride;
  const int st_stop = (MODE == MODE_CG_STEP || MODE == MODE_GM_STEP) ? (st[ST_STATUS] | st[ST_DONE]) : 0;
  const int st_iters = st[ST_ITERS];
  {
    // all of these arrive before the exit test (one wait for the lot)
    int all = h0.x | h1.w | st_stop | st_iters;
#pragma unroll
    for (int i = 0; i < NUW; ++i) all |= M == 1 ? uwv[i] : 0;
    asm volatile("" ::"s"(all));
  }
  if (st_stop) return;
  if (p.kact >= 0 && st_iters <= p.kact) return;
  const int r0 = h0.x, nrows = h0.y - h0.x, e0 = h0.z, ne = h0.w - h0.z;
  const int aB = h1.x, naB = h1.y - h1.x, namax = h1.z;
  const bool staged = naB <= ACAP;
  const int nunit = M == 1 ? h1.w : 0;  // X window units (the plan keeps naB <= ACAP for these)
  const bool win = nunit > 0;
  const TV *Ax = (const TV *)p.Ax + (int64_t)b * p.strideA;
  const TV *X = (const TV *)p.X + (int64_t)b * p.strideX;
  const int64_t zb = (int64_t)b * p.strideZ;
  double *Z = p.Z + zb;
  const int32_t *rp = (M == 1) ? p.Np : p.nodeptr;
  const bool valid = t < ne;
  const bool proj = (MODE != MODE_PRODUCT) || p.project;
  const uint32_t *codes = (const uint32_t *)p.codes;

  // ---- one round of loads that depend on the header only ----
  // Straight-line code with clamped, always in-bounds indices, so every load
  // is issued before the first wait (a block has >= 1 entry and >= 1 row).
  // The lane's record: byte 0 its row within the block, code u in byte u + 1,
  // CODE_NONE padding.  Words 0..2 load as one vector whatever the stride
  // (the code array carries 16 bytes of slack); longer records read the rest
  // in the term loop.
  const int nw = p.cstride >> 2;
  const int te = valid ? t : 0;
  const uint32_t rec = (uint32_t)(e0 + te) * (uint32_t)nw;
  const uint3 r3 = *(const uint3 *)((const char *)codes + rec * 4u);  // 4-byte aligned
  const uint32_t w0 = r3.x, w1 = r3.y, w2 = r3.z;
  int jc0 = 0;
  double bcv[PRE ? NB : 1], v_gp[PRE ? NP : 1];
  if (PRE) {
    if (proj) {
#pragma unroll
      for (int q = 0; q < NB; ++q) bcv[q] = spg_ld(p.bce, (uint32_t)(e0 + te) * NB + q);
    }
  } else if (proj) {
    jc0 = (M == 1) ? spg_ld(p.Nj, (uint32_t)(e0 + te)) : spg_ld(p.ncol, (uint32_t)(e0 + te));
  }
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
  if (PRE && proj) {
#pragma unroll
    for (int q = 0; q < NP; ++q) v_gp[q] = spg_ld(p.gp, (uint32_t)(r0 + rq) * NP + q);
  }
  int v_np0 = 0, v_np1 = 0;
  if constexpr (M == 2) {
    v_np0 = spg_ld(p.Np, (uint32_t)(2 * (r0 + rq)));
    v_np1 = spg_ld(p.Np, (uint32_t)(2 * (r0 + rq) + 1));
  }
  // the block's slice of A
  int v_x0[NIT], v_x1[NIT];
  TV v_ax[NIT][NO];
  uint32_t v_ad[NITD], v_xw[XIT];
  if (M == 1 && staged && naB > 0) {
    const int32_t *xsrc = win ? p.xl : p.xoff;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      v_x0[it] = 0;
      if (it * BS < naB) v_x0[it] = spg_ld(xsrc, (uint32_t)(aB + (t + it * BS < naB ? t + it * BS : naB - 1)));
    }
    const uint32_t *Axd = (const uint32_t *)Ax;
    const int nd = naB * DPE;
#pragma unroll
    for (int it = 0; it < NITD; ++it) {
      v_ad[it] = 0;
      if (it * BS < nd) v_ad[it] = spg_ld(Axd, (uint32_t)(aB * DPE + (t + it * BS < nd ? t + it * BS : nd - 1)));
    }
    if (win) {
      const int lane = t & (RN_WAVE - 1);
      const uint32_t *Xd = (const uint32_t *)X;
#pragma unroll
      for (int i = 0; i < XIT; ++i) {
        const int c = wv + i * (BS / RN_WAVE);
        v_xw[i] = 0;
        if (DPE == 2) {
          if (c < nunit) v_xw[i] = spg_ld(Xd, (uint32_t)(2 * uwv[i] + lane));
        } else if (2 * c < nunit) {
          const int u0 = uwv[2 * i], u1 = 2 * c + 1 < nunit ? uwv[2 * i + 1] : u0;
          v_xw[i] = spg_ld(Xd, (uint32_t)((lane < 32 ? u0 : u1) + (lane & 31)));
        }
      }
    }
  } else if (staged && naB > 0) {
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
    if (PRE && proj)
#pragma unroll
      for (int q = 0; q < NP; ++q) s_gp[t * NP + q] = v_gp[q];
    if constexpr (M == 2) {
      s_np0[t] = v_np0;
      s_np1[t] = v_np1;
    }
  }
  if (nrows == BS && t == 0) {  // the end of the last row is in the header
    s_rp[BS] = ne;
    s_ap[BS] = naB;
  }
  if (M == 1 && staged && naB > 0) {
#pragma unroll
    for (int it = 0; it < NIT; ++it)
      if (t + it * BS < naB) s_x0[t + it * BS] = v_x0[it];
    uint32_t *s_ad = (uint32_t *)s_ax;
#pragma unroll
    for (int it = 0; it < NITD; ++it)
      if (t + it * BS < naB * DPE) s_ad[t + it * BS] = v_ad[it];
    if (win) {
      uint32_t *s_xd = (uint32_t *)s_xw;
      const int wv = t / RN_WAVE, lane = t & (RN_WAVE - 1);
#pragma unroll
      for (int i = 0; i < XIT; ++i) {
        const int c = wv + i * (BS / RN_WAVE);
        if (c * 64 < nunit * XW_UNIT * DPE) s_xd[c * 64 + lane] = v_xw[i];
      }
    }
  } else if (staged && naB > 0) {
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
  const int lrow = valid ? (int)(w0 & 0xffu) : 0;
  const bool froot = !valid || s_root[lrow];
  if (valid) {
    const int la = s_ap[lrow];
    const int r = t - s_rp[lrow];
    if (PRE && proj) {
#pragma unroll
      for (int q = 0; q < NP; ++q) gq[0][q] = s_gp[lrow * NP + q];
#pragma unroll
      for (int q = 0; q < NB; ++q) bc[0][q] = bcv[q];
    } else if (proj && M == 1) {  // root lanes load too (their row and column are in range): no branch
#pragma unroll
      for (int q = 0; q < NP; ++q) gq[0][q] = spg_ld(p.gp, (uint32_t)(r0 + lrow) * NP + q);
#pragma unroll
      for (int q = 0; q < NB; ++q) bc[0][q] = spg_ld(p.Bc, (uint32_t)jc0 * NB + q);
    }
    if constexpr (M == 1) {
      zi[0] = e0 + t;
      if (!froot && staged && nw <= 3) {
        // every X load of the row issued before the first multiply-add; the
        // term count is the block's longest row (uniform), a miss (codes past
        // a row's length are CODE_NONE) loads X[0]
        // Branch-free within the three code words (terms 0-2, 3-6, 7-10; a
        // word is skipped when the block's rows are shorter): all index reads,
        // then all X reads, then the multiply-adds in the order of A's row.
        // A miss (or a term past the row) reads element 0 and adds nothing.
        TV xv[UMAX], av[UMAX];
        uint32_t xi[UMAX];
        uint32_t hitm = 0;
        const bool g1 = namax > 3, g2 = namax > 7;
        auto index = [&](const int lo, const int hi, const uint32_t w) {
#pragma unroll
          for (int u = lo; u < hi; ++u) {
            const uint32_t c = __builtin_amdgcn_ubfe(w, 8 * ((u + 1) & 3), 8);
            const uint32_t hm = (c != CODE_NONE && u < namax) ? 0xffffffffu : 0u;
            hitm |= hm & (1u << u);
            av[u] = s_ax[la + u];
            xi[u] = ((uint32_t)s_x0[la + u] + c) & hm;
          }
        };
        auto gather = [&](const int lo, const int hi) {
#pragma unroll
          for (int u = lo; u < hi; ++u) xv[u] = win ? s_xw[xi[u]] : spg_ld(X, xi[u]);
        };
#pragma unroll
        for (int u = 0; u < UMAX; ++u) {
          xv[u] = 0;
          av[u] = 0;
        }
        index(0, 3, w0);
        if (g1) index(3, 7, w1);
        if (g2) index(7, 11, w2);
        if (win) {  // uniform: X from the block's window in LDS, or from global memory
          gather(0, 3);
          if (g1) gather(3, 7);
          if (g2) gather(7, 11);
        } else {
          gather(0, 3);
          if (g1) gather(3, 7);
          if (g2) gather(7, 11);
        }
        TV acc = 0;
#pragma unroll
        for (int u = 0; u < UMAX; ++u) {
          const TV pr = av[u] * xv[u];
          acc += ((hitm >> u) & 1u) ? pr : TV(0);
        }
        z[0] = (double)acc;
      } else if (!froot) {
        const int na = s_ap[lrow + 1] - la;
        TV acc = 0;
        uint32_t w = w0;
        for (int tt = 0; tt < na; ++tt) {
          const int pb = tt + 1;  // byte of the code in the record
          if ((pb & 3) == 0) w = pb == 4 ? w1 : (pb == 8 ? w2 : spg_ld(codes, rec + (pb >> 2)));
          const uint32_t c = (w >> (8 * (pb & 3))) & 0xffu;
          const bool hit = c != CODE_NONE;
          const TV a = staged ? s_ax[la + tt] : Ax[aB + la + tt];
          TV x = 0;
          if (hit)
            x = win ? s_xw[s_x0[la + tt] + (int)c] : X[(staged ? s_x0[la + tt] : p.xoff[aB + la + tt]) + (int)c];
          acc += hit ? a * x : TV(0);
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
        uint32_t w = w0;
        // Every node's DOF rows start at an even pattern offset: a non-root
        // node's two rows hold the same even number of entries, a root
        // node's one each (the plan checks both).  So a non-root neighbour's
        // pair (2c, 2c + 1) of either row is one aligned two-element load,
        // and a root neighbour's two entries are the pair at its first row
        // (x1 = x0 + 1), whenever X itself is aligned to a pair.
        const bool xpair = ((uintptr_t)X & (2 * sizeof(TV) - 1)) == 0;
        if (staged && xpair) {
          // three terms at a time: their loads, then their multiply-adds in
          // the order of A's row; a term past the row or without a code
          // loads the pair at 0 and adds nothing (+0 leaves the sums as
          // they are: they start at +0 and never become -0)
          using TV2 = typename std::conditional<MIXED, float2, double2>::type;
          constexpr int U2 = 3;
          for (int t0 = 0; t0 < na; t0 += U2) {
            TV2 va[U2], vb[U2];
            TV av4[U2][NO];
            bool hit[U2], rootk[U2];
#pragma unroll
            for (int u = 0; u < U2; ++u) {
              const int tt = t0 + u;
              const bool live = tt < na;
              const int tq = live ? tt : 0;
              const int pb = tq + 1, wi = pb >> 2;
              const uint32_t wd = wi == 0 ? w0 : (wi == 1 ? w1 : (wi == 2 ? w2 : spg_ld(codes, rec + wi)));
              const uint32_t c = live ? (wd >> (8 * (pb & 3))) & 0xffu : (uint32_t)CODE_NONE;
              const int x0 = s_x0[la + tq], x1 = s_x1[la + tq];
              hit[u] = c != CODE_NONE;
              rootk[u] = c == CODE_ROOT;
              const uint32_t ia = !hit[u] ? 0u : (uint32_t)(rootk[u] ? x0 : x0 + 2 * (int)c);
              const uint32_t ib = !hit[u] ? 0u : (uint32_t)(rootk[u] ? x0 : x1 + 2 * (int)c);
              va[u] = spg_ld2(X, ia);
              vb[u] = spg_ld2(X, ib);
#pragma unroll
              for (int o = 0; o < NO; ++o) av4[u][o] = s_ax[(la + tq) * NO + o];
            }
#pragma unroll
            for (int u = 0; u < U2; ++u) {
              const TV x00 = va[u].x, x01 = rootk[u] ? TV(0) : va[u].y, x10 = rootk[u] ? TV(0) : vb[u].x,
                       x11 = rootk[u] ? va[u].y : vb[u].y;
              const TV *a = av4[u];
              const bool h = hit[u];
              z00 += h ? a[0] * x00 : TV(0);
              z00 += h ? a[1] * x10 : TV(0);
              z01 += h ? a[0] * x01 : TV(0);
              z01 += h ? a[1] * x11 : TV(0);
              z10 += h ? a[2] * x00 : TV(0);
              z10 += h ? a[3] * x10 : TV(0);
              z11 += h ? a[2] * x01 : TV(0);
              z11 += h ? a[3] * x11 : TV(0);
            }
          }
        } else
        for (int tt = 0; tt < na; ++tt) {
          const int pb = tt + 1;  // byte of the code in the record
          if ((pb & 3) == 0) w = pb == 4 ? w1 : (pb == 8 ? w2 : spg_ld(codes, rec + (pb >> 2)));
          {
            const uint32_t c = (w >> (8 * (pb & 3))) & 0xffu;
            if (c == CODE_NONE) continue;
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
            } else if (xpair && ((x0 | x1) & 1) == 0) {
              const auto xa = spg_ld2(X, (uint32_t)(x0 + 2 * (int)c));
              const auto xb = spg_ld2(X, (uint32_t)(x1 + 2 * (int)c));
              x00 = xa.x;
              x01 = xa.y;
              x10 = xb.x;
              x11 = xb.y;
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
      // the projection data of both DOF rows load after the term loop (held
      // across it they would cost a workgroup per compute unit)
      if (proj) {
#pragma unroll
        for (int c = 0; c < M; ++c) {
          const uint32_t grow = (uint32_t)(2 * (r0 + lrow) + c);
#pragma unroll
          for (int q = 0; q < NP; ++q) gq[c][q] = spg_ld(p.gp, grow * NP + q);
#pragma unroll
          for (int q = 0; q < NB; ++q) bc[c][q] = spg_ld(p.Bc, (uint32_t)(M * jc0 + c) * NB + q);
        }
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
  }
}

// ---------------------------------------------------------------------------
// Persistent form for scalar operators (block_m = 1, n_B <= 2, plans with
// compact 8-byte records: at most 11 A terms per row and neighbour pattern
// rows of at most 30 entries).  G resident workgroups (a multiple of 8) walk the product
// blocks of their XCD's range with stride G/8.  While one block is computed
// from LDS, the header, window table and first-round loads of the next block
// are in flight, so a block costs its LDS work instead of its chain of memory
// round trips, and the grid drains in one generation.  Same arithmetic, same
// order and same per-block partials as k_spgemm.
// ---------------------------------------------------------------------------
template <int NB, int MODE, bool MIXED, int BS>
__global__ __launch_bounds__(BS) void k_spgemm_p(const SpgParams p, const int G) {
  using SH = SpgShape<1, NB, MIXED, BS>;
  using TV = typename SH::TV;
  constexpr int NP = NB * (NB + 1) / 2;
  constexpr int ACAP = SH::ACAP, NIT = SH::NIT, XCAP = SH::XCAP;
  constexpr int DPE = sizeof(TV) / 4;
  constexpr int NITD = (ACAP * DPE + BS - 1) / BS;
  constexpr int XIT = XCAP * DPE / BS;
  constexpr int NUW = DPE == 2 ? XIT : 2 * XIT;
  constexpr int NU = XCAP / XW_UNIT;
  constexpr int NWV = BS / RN_WAVE;
  constexpr int UMAX = 11;
  // CG step with the direction formed in the staging: X is D_{k-1} (FP64 in
  // both precisions) and each window element is R + beta D_{k-1}, loaded as
  // whole doubles, two units (one per half wave) per load, and in the mixed
  // form rounded to FP32 once formed (the separate direction pass's FP32
  // shadow of D_k, bit for bit)
  constexpr bool FUSE = MODE == MODE_CG_FSTEP;
  constexpr bool CGS = MODE == MODE_CG_STEP || FUSE;
  constexpr int XF = FUSE ? NUW / 2 : 1;
  // (256 lanes: the partials of beta are summed in the order the separate
  // direction pass uses)
  static_assert(!FUSE || (NUW % 2 == 0 && BS == RN_BLOCK), "fused step: units in pairs");
  static_assert(NIT * BS == ACAP && NITD * BS == ACAP * DPE, "staging covers the capacity exactly");
  // row starts double-buffered (the projection of one block reads them while
  // the next block is staged); the projection terms have their own buffer:
  // two barriers per block
  __shared__ int s_rp2[2][BS + 1];
  __shared__ int s_ap[BS + 1];
  __shared__ double s_red[NB][BS];
  __shared__ double s_w[8];
  __shared__ __align__(16) unsigned char s_buf[SH::BYTES];
  int *s_x0 = (int *)s_buf;
  TV *s_ax = (TV *)(s_buf + (size_t)ACAP * sizeof(int));
  TV *s_xw = s_ax + ACAP;
  double *s_gp = (double *)(s_xw + XCAP);

  const int b = blockIdx.y, t = threadIdx.x, lane = t & (RN_WAVE - 1);
  const int wv = __builtin_amdgcn_readfirstlane(t / RN_WAVE);
  const int32_t *st = p.st + (int64_t)b * ST_STRIDE;
  const double *sc = p.scal + (int64_t)b * p.scal_stride;
  if (CGS || MODE == MODE_GM_STEP)
    if (st[ST_STATUS] || st[ST_DONE]) return;
  if (p.kact >= 0 && st[ST_ITERS] <= p.kact) return;
  const int per = (p.nblk + 7) >> 3, Gx = G >> 3;
  const int xcd = blockIdx.x & 7;
  const int hiB = min(p.nblk, (xcd + 1) * per);
  int blk = xcd * per + (int)(blockIdx.x >> 3);
  // single-dot modes: one partial per workgroup (slot blockIdx.x)
  double *pcw = p.part + (int64_t)b * RN_MAXDOT * p.nblk;
  if (blk >= hiB) {
    if ((MODE == MODE_CG_INIT || MODE == MODE_GM_INIT || CGS) && t == 0) pcw[blockIdx.x] = 0.0;
    return;
  }

  const bool proj = (MODE != MODE_PRODUCT) || p.project;
  const TV *Ax = (const TV *)p.Ax + (int64_t)b * p.strideA;
  const TV *X = (const TV *)p.X + (int64_t)b * p.strideX;
  const double *Rr = FUSE ? p.Rres + (int64_t)b * p.strideX : nullptr;
  const double *Dp = FUSE ? (const double *)p.X + (int64_t)b * p.strideX : nullptr;  // fused step: D_{k-1}
  double be = 0.0;  // fused step: beta_{k-1}, set before the first staging
  const int64_t zb = (int64_t)b * p.strideZ;
  double *Z = p.Z + zb;
  double *part = p.part + (int64_t)b * RN_MAXDOT * p.nblk;

  // ---- a block's header and window unit starts: loaded (as uniform vector
  // loads) two blocks ahead, read into scalars once they have arrived ----
  // lane i < 8 holds header word i, lane i < NUW the i-th unit start this
  // wave uses (two registers, read out with readlane)
  struct HdV {
    int h, u;
  };
  struct Hd {
    int r0, nrows, e0, ne, aB, naB, namax, nunit;
    int uw[NUW];
  };
  // buffer loads: always vector-memory instructions (a plain load may become
  // a scalar one where no store precedes it, and the wait counts of the
  // pipeline then differ between the first iteration and the others)
  const __amdgpu_buffer_rsrc_t rs_h =
      __builtin_amdgcn_make_buffer_rsrc((void *)p.blk_hdr, (short)0, (p.nblk + 1) * 32, 0x00020000);
  const __amdgpu_buffer_rsrc_t rs_u =
      __builtin_amdgcn_make_buffer_rsrc((void *)p.xwin, (short)0, (p.nblk + 1) * NU * 4, 0x00020000);
  const int ul = lane < NUW ? lane : 0;
  const int uidx = DPE == 2 ? wv + ul * NWV : 2 * (wv + (ul >> 1) * NWV) + (ul & 1);  // < NU
  auto load_hdv = [&](const int bb, HdV &v) {
    v.h = (int)__builtin_amdgcn_raw_buffer_load_b32(rs_h, (lane & 7) * 4, bb * 32, 0);
    v.u = (int)__builtin_amdgcn_raw_buffer_load_b32(rs_u, uidx * 4, bb * NU * 4, 0);
  };
  auto to_hd = [&](const HdV &v, Hd &h) {
    const int r0 = __builtin_amdgcn_readlane(v.h, 0), r1 = __builtin_amdgcn_readlane(v.h, 1);
    const int e0 = __builtin_amdgcn_readlane(v.h, 2), e1 = __builtin_amdgcn_readlane(v.h, 3);
    const int a0 = __builtin_amdgcn_readlane(v.h, 4), a1 = __builtin_amdgcn_readlane(v.h, 5);
    h.r0 = r0;
    h.nrows = r1 - r0;
    h.e0 = e0;
    h.ne = e1 - e0;
    h.aB = a0;
    h.naB = a1 - a0;
    h.namax = __builtin_amdgcn_readlane(v.h, 6);
    h.nunit = __builtin_amdgcn_readlane(v.h, 7);
#pragma unroll
    for (int i = 0; i < NUW; ++i) h.uw[i] = __builtin_amdgcn_readlane(v.u, i);
  };
  // ---- a block's first round of vector loads (registers) ----
  struct Rd {
    uint32_t w0, w1;  // compact record (row, 5-bit codes)
    double bcv[NB], gp[NP], own, ownr;
    int rp, ap;
    int x0[NIT];
    uint32_t ad[NITD], xw[XIT];
    double fr[XF], fd[XF];  // fused step: the window's R and D_{k-1}
  };
  auto load_rd = [&](const Hd &h, Rd &r) {
    const int te = t < h.ne ? t : 0;
    const uint32_t e = (uint32_t)(h.e0 + te);
    const uint2 r2 = *(const uint2 *)((const char *)p.ccodes + e * 8u);  // compact record
    r.w0 = r2.x;
    r.w1 = r2.y;
    r.own = r.ownr = 0.0;
    if (MODE == MODE_CG_STEP) r.own = spg_ld(p.Xown + zb, e);
    if (FUSE) {  // this lane's R and D_{k-1} (D_k is formed in the epilogue)
      r.ownr = spg_ld(Rr, e);
      r.own = spg_ld(Dp, e);
    }
    const int rq = t < h.nrows ? t : h.nrows - 1, rt = t < h.nrows ? t : h.nrows;
    r.rp = spg_ld(p.Np, (uint32_t)(h.r0 + rt));
    r.ap = spg_ld(p.Ap, (uint32_t)(h.r0 + rt));
#pragma unroll
    for (int q = 0; q < NB; ++q) r.bcv[q] = 0.0;
#pragma unroll
    for (int q = 0; q < NP; ++q) r.gp[q] = 0.0;
    if (proj) {
      // Bc = 1: every lane reads the same first row (no traffic) and uses 1
#pragma unroll
      for (int q = 0; q < NB; ++q) r.bcv[q] = spg_ld(p.bce, p.unit_bc ? (uint32_t)q : e * NB + q);
      if (p.unit_bc)
#pragma unroll
        for (int q = 0; q < NB; ++q) r.bcv[q] = 1.0;
#pragma unroll
      for (int q = 0; q < NP; ++q) r.gp[q] = spg_ld(p.gp, (uint32_t)(h.r0 + rq) * NP + q);
    }
    // Branch-free: every load is issued whatever the block's sizes (indices
    // clamped into the block's slice; the plan writes every window-table
    // entry, unused ones point at element 0), so no register of an earlier
    // round is waited for while this one is issued.
    {
      // a block without A entries reads the last one
      const int nA = h.naB > 0 ? h.naB : 1;
      const int a0 = h.naB > 0 ? h.aB : (int)p.strideA - 1;
      const int32_t *xsrc = h.nunit > 0 ? p.xl : p.xoff;
#pragma unroll
      for (int it = 0; it < NIT; ++it) r.x0[it] = spg_ld(xsrc, (uint32_t)(a0 + min(t + it * BS, nA - 1)));
      const uint32_t *Axd = (const uint32_t *)Ax;
      const int nd = nA * DPE;
#pragma unroll
      for (int it = 0; it < NITD; ++it)
        r.ad[it] = spg_ld(Axd, (uint32_t)(a0 * DPE + min(t + it * BS, nd - 1)));
      const uint32_t *Xd = (const uint32_t *)X;
      if (FUSE) {
#pragma unroll
        for (int j = 0; j < XF; ++j) {
          const uint32_t xi = (uint32_t)((lane < 32 ? h.uw[2 * j] : h.uw[2 * j + 1]) + (lane & 31));
          r.fr[j] = spg_ld(Rr, xi);
          r.fd[j] = spg_ld(Dp, xi);
        }
      }
#pragma unroll
      for (int i = 0; i < (FUSE ? 0 : XIT); ++i) {
        if (DPE == 2) {
          r.xw[i] = spg_ld(Xd, (uint32_t)(2 * h.uw[i] + lane));
        } else {
          r.xw[i] = spg_ld(Xd, (uint32_t)((lane < 32 ? h.uw[2 * i] : h.uw[2 * i + 1]) + (lane & 31)));
        }
      }
    }
  };
  // ---- registers -> LDS (every position written is inside its region) ----
  auto stage = [&](const Hd &h, const Rd &r, int *s_rp) {
    if (t <= h.nrows) {
      s_rp[t] = r.rp - h.e0;
      s_ap[t] = r.ap - h.aB;
    }
    if (h.nrows == BS && t == 0) {  // the end of the last row is in the header
      s_rp[BS] = h.ne;
      s_ap[BS] = h.naB;
    }
    if (proj && t < h.nrows)
#pragma unroll
      for (int q = 0; q < NP; ++q) s_gp[t * NP + q] = r.gp[q];
    if (h.naB <= ACAP && h.naB > 0) {
#pragma unroll
      for (int it = 0; it < NIT; ++it) s_x0[t + it * BS] = r.x0[it];
      uint32_t *s_ad = (uint32_t *)s_ax;
#pragma unroll
      for (int it = 0; it < NITD; ++it) s_ad[t + it * BS] = r.ad[it];
      if (h.nunit > 0) {
        if (FUSE) {
          // the same rounding as the separate direction pass (no
          // contraction); FP64: unit wv + i NWV at element (wv + i NWV)
          // XW_UNIT; FP32: units 2 (wv + j NWV) and the next at word
          // (wv + j NWV) 64, one per half wave
#pragma unroll
          for (int j = 0; j < XF; ++j) {
            const double dk = r.fr[j] + be * r.fd[j];
            if (MIXED) s_xw[(wv + j * NWV) * 64 + lane] = (TV)dk;
            else ((double *)s_xw)[(wv + (2 * j + (lane >> 5)) * NWV) * XW_UNIT + (lane & 31)] = dk;
          }
        } else {
          uint32_t *s_xd = (uint32_t *)s_xw;
#pragma unroll
          for (int i = 0; i < XIT; ++i) s_xd[(wv + i * NWV) * 64 + lane] = r.xw[i];
        }
      }
    }
  };

  // pipeline: at the top of an iteration the block's first round (R) and the
  // next block's header (V1) are in flight; after staging R the next block's
  // first round (Rn) and then the header after that (V2) are issued, so a
  // wait for an Rn register never waits for V2
  Hd H;
  Rd R;
  HdV V1;
  {
    HdV V0;
    load_hdv(blk, V0);
    to_hd(V0, H);
  }
  load_rd(H, R);  // same issue order as in the loop: first round, then the next header
  // (unconditional, clamped: the wait counts then agree on every path)
  load_hdv(min(blk + Gx, hiB - 1), V1);
  if (FUSE) {
    // beta_{k-1} = gamma_k / gamma_{k-1} from the update's <R,R> partials,
    // loaded behind the first round (one wait for both): every workgroup
    // sums them in the same fixed order, so all get the same gamma_k and
    // take the same stopping decision; workgroup 0 stores the scalars and
    // the test.  The window is combined with beta at the first staging.
    const CgLayout L(p.K);
    const double gam = sc[L.gam + p.k - 1], gam0 = sc[SC_GAMMA0];
    const double g = rn_reduce_part_w<BS>(p.part_rr + (int64_t)b * p.pstride_rr, p.np_rr, s_w);
    if (blockIdx.x == 0 && t == 0)
      rn_cg_beta_fin(g, gam, gam0, p.scal + (int64_t)b * p.scal_stride, p.st + (int64_t)b * ST_STRIDE,
                     p.hist ? p.hist + (int64_t)b * p.hist_stride : nullptr, p.K, p.k - 1);
    if (!isfinite(g) || g <= RN_CG_STOP * gam0) return;  // stopped: no D_k, no product
    be = g / gam;
  }
  // single-dot modes: every lane adds its terms over all of this workgroup's
  // blocks, in block order; one compensated block sum at the end
  RnAcc dacc;
  int par = 0;
  for (;;) {
    const int nxt = blk + Gx;
    const bool more = nxt < hiB;
    int *s_rp = s_rp2[par];
    stage(H, R, s_rp);
    __syncthreads();
    Hd Hn;
    Rd Rn;
    HdV V2;
    if (more) {
      to_hd(V1, Hn);
      load_rd(Hn, Rn);  // in flight while this block is computed
      load_hdv(min(nxt + Gx, hiB - 1), V2);
    }

    // ---- the product from LDS (root rows: every code is CODE_NONE, z = 0) ----
    const bool valid = t < H.ne;
    const bool staged = H.naB <= ACAP, win = H.nunit > 0;
    const int lrow = valid ? (int)(R.w0 & 0xffu) : 0;
    double z = 0.0;
    double gq[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) gq[q] = 0.0;
    if (valid) {
      const int la = s_ap[lrow];
      if (proj)
#pragma unroll
        for (int q = 0; q < NP; ++q) gq[q] = s_gp[lrow * NP + q];
      const bool g1 = H.namax > 3, g2 = H.namax > 5, g3 = H.namax > 7, g4 = H.namax > 9;
      TV acc = 0;
      // one group of terms (lo..hi-1): offsets, then A and X, then the
      // multiply-adds in the order of A's row; A past the block's slice and X
      // element 0 only meet masked terms.  Separate paths keep every LDS
      // access an LDS instruction (a generic access would also wait for the
      // next block's loads in flight).
      const uint64_t rec = (uint64_t)R.w0 | ((uint64_t)R.w1 << 32);
      auto group = [&](const int lo, const int hi, const int path) {
        uint32_t xi[4], hm[4];
        TV av[4], xv[4];
#pragma unroll
        for (int u = lo; u < hi; ++u) {
          const uint32_t c = (uint32_t)(rec >> (8 + 5 * u)) & CCODE_NONE;
          hm[u - lo] = (c != CCODE_NONE && u < H.namax) ? 0xffffffffu : 0u;
          const uint32_t xo =
              path < 2 ? (uint32_t)s_x0[la + u] : (uint32_t)p.xoff[H.aB + min(la + u, H.naB - 1)];
          xi[u - lo] = (xo + c) & hm[u - lo];
        }
#pragma unroll
        for (int u = lo; u < hi; ++u) {
          if (path < 2) av[u - lo] = s_ax[la + u];
          else av[u - lo] = Ax[H.aB + min(la + u, H.naB - 1)];
          if (path == 0) xv[u - lo] = s_xw[xi[u - lo]];
          else if (FUSE) xv[u - lo] = (TV)(spg_ld(Rr, xi[u - lo]) + be * spg_ld(Dp, xi[u - lo]));
          else xv[u - lo] = spg_ld(X, xi[u - lo]);
        }
#pragma unroll
        for (int u = lo; u < hi; ++u) {
          const TV pr = av[u - lo] * xv[u - lo];
          acc += hm[u - lo] ? pr : TV(0);
        }
      };
      // terms in groups of 3, 2, 2, 2 and 2 (groups past the block's longest
      // A row skipped): rows of 5, 7 or 9 A entries take no masked term
      if (staged && win) {
        group(0, 3, 0);
        if (g1) group(3, 5, 0);
        if (g2) group(5, 7, 0);
        if (g3) group(7, 9, 0);
        if (g4) group(9, 11, 0);
      } else if (staged) {
        group(0, 3, 1);
        if (g1) group(3, 5, 1);
        if (g2) group(5, 7, 1);
        if (g3) group(7, 9, 1);
        if (g4) group(9, 11, 1);
      } else {
        group(0, 3, 2);
        if (g1) group(3, 5, 2);
        if (g2) group(5, 7, 2);
        if (g3) group(7, 9, 2);
        if (g4) group(9, 11, 2);
      }
      z = (double)acc;
      if (MODE == MODE_GM_STEP) z *= sc[GmLayout(p.K).s + p.k];
    }

    // ---- projection: every lane sums its row's terms in pattern order ----
    if (proj) {
      if (valid)
#pragma unroll
        for (int q = 0; q < NB; ++q) s_red[q][t] = z * R.bcv[q];
      __syncthreads();
      if (valid) {
        const int rs = s_rp[lrow], re = s_rp[lrow + 1];
        double sv[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) sv[q] = 0.0;
        for (int u = rs; u < re; ++u)
#pragma unroll
          for (int q = 0; q < NB; ++q) sv[q] += s_red[q][u];
        double y[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          y[q] = 0.0;
#pragma unroll
          for (int r2 = 0; r2 < NB; ++r2) y[q] += gq[rn_pk(NB, q, r2)] * sv[r2];
        }
        double u = 0.0;
#pragma unroll
        for (int q = 0; q < NB; ++q) u += R.bcv[q] * y[q];
        z -= u;
      }
    }

    // ---- epilogue: output and this block's partials ----
    const uint32_t e = (uint32_t)(H.e0 + t);
    if (MODE == MODE_PRODUCT) {
      if (valid) spg_st(Z, e, p.accum ? spg_ld((const double *)Z, e) + z : z);
    } else if (MODE == MODE_CG_INIT || MODE == MODE_GM_INIT) {
      if (valid) {
        const double v = -z;
        spg_st(Z, e, v);
        if (p.Z2) spg_st(p.Z2 + zb, e, v);
        dacc.add(v * v);
      }
    } else if (MODE == MODE_CG_STEP) {
      if (valid) {
        spg_st(Z, e, z);
        dacc.add(R.own * z);
      }
    } else if (FUSE) {
      if (valid) {
        const double dk = R.ownr + be * R.own;
        spg_st(p.Dnew + zb, e, dk);
        spg_st(Z, e, z);
        dacc.add(dk * z);
      }
    } else if (MODE == MODE_GM_STEP) {
      if (valid) spg_st(Z, e, z);
    }
    if (!more) break;
    // without the projection no barrier separates this block's LDS reads from
    // the next staging
    if (!proj) __syncthreads();
    par ^= 1;
    blk = nxt;
    H = Hn;
    R = Rn;
    V1 = V2;
  }
  if (MODE == MODE_CG_INIT || MODE == MODE_GM_INIT || CGS) {
    const double S = rn_block_sum2_w<NWV>(dacc.hi, dacc.lo, s_w);
    if (t == 0) pcw[blockIdx.x] = S;
  }
}

// resident workgroups of one persistent launch: the occupancy of the kernel
// times the number of compute units, split over the batch, a multiple of 8
template <int NB, int MODE, bool MIXED, int BS>
static int persist_grid(int nblk, int batch) {
  static int cap = -1;
  if (cap < 0) {
    int per_cu = 0, dev = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_spgemm_p<NB, MODE, MIXED, BS>, BS, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      per_cu = 0;
    cap = per_cu * ncu;
  }
  int g = cap / (batch > 0 ? batch : 1);
  g = g / 8 * 8;
  const int full = (int)rn_xcd_grid((unsigned)nblk);
  if (g > full) g = full;
  return g;
}

// the grid of the persistent launch, or 0 when it cannot run
template <int NB, int MODE, int BS>
static int launch_p(const SpgParams &p, int batch, bool mixed, hipStream_t s) {
  const int G = p.grid > 0 ? p.grid
                           : mixed ? persist_grid<NB, MODE, true, BS>(p.nblk, batch)
                                   : persist_grid<NB, MODE, false, BS>(p.nblk, batch);
  if (G < 8) return 0;
  const dim3 grid((unsigned)G, (unsigned)batch);
  if (mixed) hipLaunchKernelGGL((k_spgemm_p<NB, MODE, true, BS>), grid, dim3(BS), 0, s, p, G);
  else hipLaunchKernelGGL((k_spgemm_p<NB, MODE, false, BS>), grid, dim3(BS), 0, s, p, G);
  return G;
}

// the fused CG step runs only as the persistent FP64 product of 256 lanes
static bool fused_plan(const SpgParams &p) {
  return p.ccodes && p.nnzN >= 64 && p.strideA >= 1 && p.persist && p.bs == RN_BLOCK;
}

// the number of per-workgroup partials a single-dot mode leaves (0: the
// fused step cannot run)
template <int M, int NB, int MODE>
static int launch_m(const SpgParams &p, int batch, bool mixed, hipStream_t s) {
  if constexpr (MODE == MODE_CG_FSTEP) {
    if constexpr (M == 1 && NB <= 2) {
      if (!fused_plan(p)) return 0;
      const int G = p.grid > 0 ? p.grid
                               : mixed ? persist_grid<NB, MODE, true, RN_BLOCK>(p.nblk, batch)
                                       : persist_grid<NB, MODE, false, RN_BLOCK>(p.nblk, batch);
      if (G < 8) return 0;
      const dim3 grid((unsigned)G, (unsigned)batch);
      if (mixed) hipLaunchKernelGGL((k_spgemm_p<NB, MODE, true, RN_BLOCK>), grid, dim3(RN_BLOCK), 0, s, p, G);
      else hipLaunchKernelGGL((k_spgemm_p<NB, MODE, false, RN_BLOCK>), grid, dim3(RN_BLOCK), 0, s, p, G);
      return G;
    }
    return 0;
  } else {
    if constexpr (M == 1 && NB <= 2) {
      // the persistent form serves scalar operators with n_B <= 2 and compact
      // records, unless the plan was made with RN_OPT_PERSISTENT_PRODUCT = 0
      // (the branch-free first round reads 32 elements of X and one of A whatever the block)
      if (p.ccodes && p.nnzN >= 64 && p.strideA >= 1 && p.persist) {
        int G = 0;
        if (p.bs == 128 && (G = launch_p<NB, MODE, 128>(p, batch, mixed, s)) > 0) return G;
        if (p.bs == RN_BLOCK && (G = launch_p<NB, MODE, RN_BLOCK>(p, batch, mixed, s)) > 0) return G;
      }
    }
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
    return p.nblk;
  }
}

template <int MODE>
static rn_status launch_mode(rn_ctx *ctx, const rn_plan *pl, const SpgParams &p, int batch, bool mixed, int *np) {
  hipStream_t s = ctx->stream;
  if (pl->m == 1) {
    switch (pl->nB) {
      case 1: *np = launch_m<1, 1, MODE>(p, batch, mixed, s); break;
      case 2: *np = launch_m<1, 2, MODE>(p, batch, mixed, s); break;
      case 3: *np = launch_m<1, 3, MODE>(p, batch, mixed, s); break;
      case 4: *np = launch_m<1, 4, MODE>(p, batch, mixed, s); break;
      default: return rn_fail(ctx, RN_EINVAL, "nB out of range");
    }
  } else {
    switch (pl->nB) {
      case 2: *np = launch_m<2, 2, MODE>(p, batch, mixed, s); break;
      case 3: *np = launch_m<2, 3, MODE>(p, batch, mixed, s); break;
      case 4: *np = launch_m<2, 4, MODE>(p, batch, mixed, s); break;
      default: return rn_fail(ctx, RN_EINVAL, "nB out of range for block_m = 2");
    }
  }
  if (MODE == MODE_CG_FSTEP && *np == 0)
    return rn_fail(ctx, RN_EINVAL, "fused CG step requested for a plan the persistent product cannot serve");
  LAUNCH_CHECK(ctx);
  return RN_OK;
}

int rn_spgemm_fused_grid(const rn_plan *pl, int batch, bool mixed) {
  const SpgParams p = rn_spg_params(pl);
  if (pl->m != 1 || pl->nB > 2 || p.nblk <= 0 || !fused_plan(p)) return 0;
  int G;
  if (mixed)
    G = pl->nB == 1 ? persist_grid<1, MODE_CG_FSTEP, true, RN_BLOCK>(p.nblk, batch)
                    : persist_grid<2, MODE_CG_FSTEP, true, RN_BLOCK>(p.nblk, batch);
  else
    G = pl->nB == 1 ? persist_grid<1, MODE_CG_FSTEP, false, RN_BLOCK>(p.nblk, batch)
                    : persist_grid<2, MODE_CG_FSTEP, false, RN_BLOCK>(p.nblk, batch);
  return G >= 8 ? G : 0;
}

rn_status rn_launch_spgemm(rn_ctx *ctx, const rn_plan *pl, int mode, const SpgParams &p, int batch, bool mixed,
                           int *npart) {
  int np = 0;
  rn_status st = RN_OK;
  if (p.nblk > 0) {
    switch (mode) {
      case MODE_PRODUCT: st = launch_mode<MODE_PRODUCT>(ctx, pl, p, batch, mixed, &np); break;
      case MODE_CG_INIT: st = launch_mode<MODE_CG_INIT>(ctx, pl, p, batch, mixed, &np); break;
      case MODE_CG_STEP: st = launch_mode<MODE_CG_STEP>(ctx, pl, p, batch, mixed, &np); break;
      case MODE_GM_INIT: st = launch_mode<MODE_GM_INIT>(ctx, pl, p, batch, mixed, &np); break;
      case MODE_GM_STEP: st = launch_mode<MODE_GM_STEP>(ctx, pl, p, batch, mixed, &np); break;
      case MODE_CG_FSTEP: st = launch_mode<MODE_CG_FSTEP>(ctx, pl, p, batch, mixed, &np); break;
      default: return rn_fail(ctx, RN_EINVAL, "bad product mode");
    }
  }
  if (npart) *npart = np;
  return st;
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
  p.xl = pl->xl;
  p.bce = pl->bce;
  p.xwin = pl->xwin;
  p.codes = pl->codes;
  p.ccodes = pl->ccodes;
  p.is_root = pl->is_root;
  p.Bc = pl->Bc;
  p.gp = pl->gp;
  p.strideZ = pl->nnzN;
  p.strideX = pl->nnzN;
  p.strideA = pl->nnzA * pl->m * pl->m;
  p.unit_bc = pl->unit_bc ? 1 : 0;
  p.persist = pl->persist ? 1 : 0;
  return p;
}
