// rn_plan.hip -- symbolic part of the energy minimisation (Sec. 3.6): the
// position codes of the masked product, the per-row least-squares data of the
// constraint projection and the block partition of the product.
#include <climits>
#include <cstdlib>
#include <cstring>
#include <new>

#include "rn_emin.h"

void *rn_plan_ws(rn_plan *pl, int slot, size_t bytes, rn_status *st) {
  RnScratch &s = pl->ws[slot];
  if (bytes == 0) bytes = 16;
  if (pl->arena) {  // allocation-free call: consecutive 256-byte aligned pieces of the arena
    const size_t off = (pl->arena_used + 255) & ~(size_t)255;
    if (off > pl->arena_cap || bytes > pl->arena_cap - off) {
      *st = rn_fail(pl->ctx, RN_ELIMIT, "workspace of %zu bytes beyond the allocation-free scratch", bytes);
      return nullptr;
    }
    pl->arena_used = off + bytes;
    return pl->arena + off;
  }
  if (s.cap >= bytes) return s.ptr;
  if (!pl->ctx) {
    *st = RN_EINVAL;
    return nullptr;
  }
  rn_dev_free(pl->ctx, s.ptr);  // stream-ordered reuse: no synchronisation needed
  s.ptr = nullptr;
  s.cap = 0;
  const size_t cap = bytes + bytes / 8 + 256;
  s.ptr = rn_dev_alloc(pl->ctx, cap);
  if (!s.ptr) {
    *st = rn_fail(pl->ctx, RN_ENOMEM, "plan workspace allocation of %zu bytes failed", cap);
    return nullptr;
  }
  s.cap = cap;
  return s.ptr;
}

template <class T>
static bool plan_alloc(rn_plan *pl, T **p, size_t bytes) {
  *p = (T *)rn_dev_alloc(pl->ctx, bytes);
  return *p != nullptr;
}

static __device__ inline int pad4(int x) { return (x + 3) & ~3; }

// Block-wide maximum / sum of one int per thread, written by thread 0 to
// out[blockIdx.x] (no atomics on a shared address: thousands of waves
// updating one word serialise in the memory system).  Every thread calls it.
template <bool MAX>
static __device__ inline void block_to_slot(int v, int32_t *out) {
  __shared__ int s[RN_BLOCK / RN_WAVE];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int o = __shfl_xor(v, off, RN_WAVE);
    v = MAX ? max(v, o) : v + o;
  }
  __syncthreads();
  if ((threadIdx.x & (RN_WAVE - 1)) == 0) s[threadIdx.x / RN_WAVE] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int r = s[0];
    for (int w = 1; w < (int)(blockDim.x / RN_WAVE); ++w) r = MAX ? max(r, s[w]) : r + s[w];
    out[blockIdx.x] = r;
  }
}

// one block: out = max or sum of in[0..n); with a second pair (in2, out2)
// a second block does the same for it
template <bool MAX, typename TO>
__global__ __launch_bounds__(RN_BLOCK) void k_finish_slots(const int32_t *__restrict__ in, int n,
                                                          TO *__restrict__ out, const int32_t *__restrict__ in2 = nullptr,
                                                          TO *__restrict__ out2 = nullptr) {
  if (blockIdx.x == 1) {
    in = in2;
    out = out2;
  }
  __shared__ long long s[RN_BLOCK];
  long long v = 0;
  for (int q = threadIdx.x; q < n; q += RN_BLOCK) v = MAX ? (v > in[q] ? v : in[q]) : v + in[q];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int w = RN_BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] = MAX ? (s[threadIdx.x] > s[threadIdx.x + w] ? s[threadIdx.x] : s[threadIdx.x + w])
                                               : s[threadIdx.x] + s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = (TO)s[0];
}

// ---- sizes: longest pattern row and longest A row of a non-root row
// (block_m = 1: DOF rows, 2: node rows), as per-block maxima ---------------
// (and *bcflag = 1 where an entry of Bc differs from 1: with Bc = 1 the
// product needs no per-entry Bc rows)
__global__ __launch_bounds__(RN_BLOCK) void k_plan_count_m1(int n, const int32_t *__restrict__ Ap,
                                                           const int32_t *__restrict__ Np,
                                                           const uint8_t *__restrict__ is_root,
                                                           int32_t *__restrict__ maxlen, int32_t *__restrict__ maxna,
                                                           int32_t *__restrict__ guard, const double *__restrict__ Bc,
                                                           int64_t nbcv, int32_t *__restrict__ bcflag) {
  const int i = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (*guard) return;
  bool other = false;
  for (int64_t q = i; q < nbcv; q += (int64_t)gridDim.x * RN_BLOCK) other = other || Bc[q] != 1.0;
  if (other) *bcflag = 1;  // every writer stores the same value
  int len = 0, na = 0;
  if (i < n) {
    len = Np[i + 1] - Np[i];
    if (len > CODE_MAXLEN) atomicOr(guard, GUARD_LIMIT);
    if (len == 0 || (is_root[i] && len != 1)) atomicOr(guard, GUARD_N);
    na = is_root[i] ? 0 : Ap[i + 1] - Ap[i];
  }
  block_to_slot<true>(len, maxlen);  // finished by k_finish_slots
  block_to_slot<true>(na, maxna);
}

__global__ __launch_bounds__(RN_BLOCK) void k_plan_count_m2(int nr, const int32_t *__restrict__ Ap,
                                                           const int32_t *__restrict__ Np,
                                                           const uint8_t *__restrict__ is_root,
                                                           int32_t *__restrict__ ncnt, int32_t *__restrict__ maxlen,
                                                           int32_t *__restrict__ maxna,
                                                           int32_t *__restrict__ guard) {
  const int I = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (*guard) {
    if (I < nr) ncnt[I] = 0;
    return;
  }
  int len = 0, na = 0;
  if (I < nr) {
    const bool root = is_root[2 * I];
    const int l0 = Np[2 * I + 1] - Np[2 * I], l1 = Np[2 * I + 2] - Np[2 * I + 1];
    if (root != (bool)is_root[2 * I + 1]) atomicOr(guard, GUARD_N);
    if (root) {
      if (l0 != 1 || l1 != 1) atomicOr(guard, GUARD_N);
      ncnt[I] = 1;
      len = 1;
    } else {
      if (l0 != l1 || (l0 & 1) || l0 == 0) atomicOr(guard, GUARD_N);
      len = l0 / 2;
      if (len > CODE_MAXLEN) atomicOr(guard, GUARD_LIMIT);
      ncnt[I] = len;
      na = Ap[I + 1] - Ap[I];
    }
  }
  block_to_slot<true>(len, maxlen);  // finished by k_finish_slots
  block_to_slot<true>(na, maxna);
}

// G^+ of every F row (zero for root rows), one thread per row; per-block
// counts of rows that took the pseudo-inverse fallback
template <int NB>
__global__ __launch_bounds__(RN_BLOCK) void k_plan_gram(int n, const int32_t *__restrict__ Np,
                                                       const int32_t *__restrict__ Nj,
                                                       const uint8_t *__restrict__ is_root,
                                                       const double *__restrict__ Bc, double *__restrict__ gp,
                                                       int32_t *__restrict__ rank_def,
                                                       const int32_t *__restrict__ guard) {
  constexpr int NP = NB * (NB + 1) / 2;
  const int i = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (*guard) return;
  int bad = 0;
  if (i < n) {
    double *out = gp + (int64_t)i * NP;
    if (is_root[i]) {
      for (int q = 0; q < NP; ++q) out[q] = 0.0;
    } else {
      double Gp[NB * NB];
      bad = rn_row_pinv<NB>(Nj, Np[i], Np[i + 1], Bc, Gp);
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int r = q; r < NB; ++r) out[rn_pk(NB, q, r)] = Gp[q * NB + r];
    }
  }
  block_to_slot<false>(bad, rank_def);  // per-block counts
}

// ---- one element-wise launch for two per-entry tables: the Bc row of each
// pattern entry's column (block_m = 1, n_B <= 2; bce may be NULL) and the
// first pattern entry of each stored A entry's neighbour row (xoff) ----------
__global__ __launch_bounds__(RN_BLOCK) void k_plan_bce_xoff(int64_t nnzN, int nB, const int32_t *__restrict__ Nj,
                                                           const double *__restrict__ Bc, double *__restrict__ bce,
                                                           int64_t nnzA, int m, const int32_t *__restrict__ Aj,
                                                           const int32_t *__restrict__ Np,
                                                           int32_t *__restrict__ xoff) {
  const int64_t s = (int64_t)gridDim.x * RN_BLOCK, q0 = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x;
  if (bce)
    for (int64_t e = q0; e < nnzN; e += s)
      for (int q = 0; q < nB; ++q) bce[e * nB + q] = Bc[(int64_t)Nj[e] * nB + q];
  for (int64_t q = q0; q < nnzA; q += s) {
    const int k = Aj[q];
    if (m == 1) {
      xoff[q] = Np[k];
    } else {
      xoff[2 * q] = Np[2 * k];
      xoff[2 * q + 1] = Np[2 * k + 1];
    }
  }
}

// ---- block partition: rows whose first entry lies in [b*chunk, (b+1)*chunk)
// belong to block b; header = r0, r1, e0, e1, a0, a1 (A entries/blocks) and
// (filled in by k_plan_codes) the longest A row of the block's non-root rows ----
// Row-parallel: thread r is the first row of every block b with
// rp[r-1] < b*chunk <= rp[r] (the lower bound of b*chunk) and so also the
// end row of block b-1; thread nr closes the last block.
__global__ __launch_bounds__(RN_BLOCK) void k_plan_blocks_rows(int nr, const int32_t *__restrict__ rp,
                                                              const int32_t *__restrict__ Ap, int nblk, int chunk,
                                                              int32_t *__restrict__ blk_row,
                                                              int32_t *__restrict__ hdr) {
  const int r = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (r > nr) return;
  const int64_t hi = rp[r];
  const int64_t lo = r > 0 ? (int64_t)rp[r - 1] : -1;
  const int a = Ap[r];
  if (r == nr) {
    blk_row[nblk] = nr;
    if (nblk > 0) {
      int32_t *h = hdr + 8 * (int64_t)(nblk - 1);
      h[1] = nr;
      h[3] = (int32_t)hi;
      h[5] = a;
    }
  }
  // blocks b in (lo / chunk, hi / chunk] (b = 0 for r = 0), below nblk
  const int64_t b0 = lo < 0 ? 0 : lo / chunk + 1;
  for (int64_t b = b0; b * chunk <= hi && b < nblk; ++b) {
    blk_row[b] = r;
    int32_t *h = hdr + 8 * b;
    h[0] = r;
    h[2] = (int32_t)hi;
    h[4] = a;
    h[6] = 0;
    h[7] = 0;
    if (b > 0) {
      h[-8 + 1] = r;
      h[-8 + 3] = (int32_t)hi;
      h[-8 + 5] = a;
    }
  }
}

// ---- X windows (block_m = 1): one block per product block --------------------
// The distinct columns k of the block's A rows are marked in an LDS bitmap
// over [kmin, kmin + XW_SPAN) and listed in ascending order; the pattern rows
// k form runs of consecutive pattern entries (runs closer than XW_GAP merge);
// each run is padded to a multiple of XW_UNIT entries and the runs are laid
// out one after another.  Outputs: the window's unit starts (global index of
// the first element of every unit, 0 where unused), for each A entry of the
// block the offset of its neighbour row inside the window, and the unit count
// in the header (0 when the block has too many A entries or runs, its columns
// span XW_SPAN or more, or the window does not fit).
#define XW_SPAN 8192
// Exclusive prefix of a per-thread count over the block (wave shuffles, then
// the wave totals through LDS); total = the sum over the block.
template <int BSZ>
__device__ inline int xw_scan(int v, int *s_cnt, int &total) {
  const int t = threadIdx.x, lane = t & (RN_WAVE - 1), w = t / RN_WAVE;
  int inc = v;
#pragma unroll
  for (int off = 1; off < RN_WAVE; off <<= 1) {
    const int o = __shfl_up(inc, off, RN_WAVE);
    if (lane >= off) inc += o;
  }
  if (lane == RN_WAVE - 1) s_cnt[w] = inc;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int ww = 0; ww < BSZ / RN_WAVE; ++ww) {
    const int c = s_cnt[ww];
    off += ww < w ? c : 0;
    tot += c;
  }
  __syncthreads();
  total = tot;
  return off + inc - v;
}

template <int BSZ>
__global__ __launch_bounds__(BSZ) void k_plan_xwin(int32_t *__restrict__ hdr, const int32_t *__restrict__ Aj,
                                                  const int32_t *__restrict__ Np, int64_t nnzN,
                                                  int32_t *__restrict__ xl, int32_t *__restrict__ xwin) {
  constexpr int ACAP = SPG_ACAP_M1(BSZ), XCAP = SPG_XCAP_M1(BSZ), NU = XCAP / XW_UNIT;
  constexpr int NWORD = XW_SPAN / 32, WPT = NWORD / BSZ;  // bitmap words, per thread
  static_assert(NWORD % BSZ == 0, "bitmap words split evenly");
  __shared__ uint32_t s_bits[NWORD];
  __shared__ int s_v[ACAP];  // distinct columns, ascending
  __shared__ int s_r[ACAP];  // run of each distinct column
  __shared__ int s_np0[ACAP], s_np1[ACAP];  // first and end pattern entry of each distinct column's row
  __shared__ int s_cnt[BSZ / RN_WAVE];
  __shared__ int s_mm[2 * (BSZ / RN_WAVE)];
  __shared__ int s_xs[XW_RUNMAX + 1], s_xe[XW_RUNMAX + 1], s_dst[XW_RUNMAX + 1];
  __shared__ int s_ok;
  const int t = threadIdx.x, lane = t & (RN_WAVE - 1), w = t / RN_WAVE;
  int32_t *h = hdr + 8 * (int64_t)blockIdx.x;
  const int a0 = h[4], na = h[5] - h[4];
  int32_t *uw = xwin + (int64_t)blockIdx.x * NU;
  auto none = [&]() {
    if (t == 0) h[7] = 0;
    for (int u = t; u < NU; u += BSZ) uw[u] = 0;
  };
  if (na <= 0 || na > ACAP) {  // uniform
    none();
    return;
  }
  // the block's A columns, loaded once (na <= ACAP = KPT * BSZ)
  constexpr int KPT = ACAP / BSZ;
  int kr[KPT];
#pragma unroll
  for (int i = 0; i < KPT; ++i) kr[i] = t + i * BSZ < na ? Aj[a0 + t + i * BSZ] : -1;
  // column range of the block
  int kmin = INT_MAX, kmax = -1;
#pragma unroll
  for (int i = 0; i < KPT; ++i)
    if (kr[i] >= 0) {
      kmin = min(kmin, kr[i]);
      kmax = max(kmax, kr[i]);
    }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    kmin = min(kmin, __shfl_xor(kmin, off, RN_WAVE));
    kmax = max(kmax, __shfl_xor(kmax, off, RN_WAVE));
  }
  if (lane == 0) {
    s_mm[w] = kmin;
    s_mm[BSZ / RN_WAVE + w] = kmax;
  }
#pragma unroll
  for (int i = 0; i < WPT; ++i) s_bits[t * WPT + i] = 0u;
  __syncthreads();
#pragma unroll
  for (int ww = 0; ww < BSZ / RN_WAVE; ++ww) {
    kmin = min(kmin, s_mm[ww]);
    kmax = max(kmax, s_mm[BSZ / RN_WAVE + ww]);
  }
  if (kmax - kmin >= XW_SPAN) {  // uniform
    none();
    return;
  }
#pragma unroll
  for (int i = 0; i < KPT; ++i)
    if (kr[i] >= 0) {
      const int k = kr[i] - kmin;
      atomicOr(&s_bits[k >> 5], 1u << (k & 31));
    }
  __syncthreads();
  // distinct columns in ascending order: thread t owns words t*WPT ..
  uint32_t wd[WPT];
  int c = 0;
#pragma unroll
  for (int i = 0; i < WPT; ++i) {
    wd[i] = s_bits[t * WPT + i];
    c += __popc(wd[i]);
  }
  int nu;
  int pos = xw_scan<BSZ>(c, s_cnt, nu);
#pragma unroll
  for (int i = 0; i < WPT; ++i) {
    uint32_t m = wd[i];
    while (m) {
      const int bit = __ffs(m) - 1;
      m &= m - 1u;
      s_v[pos++] = kmin + (t * WPT + i) * 32 + bit;
    }
  }
  __syncthreads();
  for (int i = t; i < nu; i += BSZ) {
    s_np0[i] = Np[s_v[i]];
    s_np1[i] = Np[s_v[i] + 1];
  }
  __syncthreads();
  // runs of the neighbour rows' entries
  int nrun = 0;
  for (int i0 = 0; i0 < nu; i0 += BSZ) {
    const int i = i0 + t;
    bool f = false;
    if (i < nu) f = i == 0 || (int64_t)s_np0[i] - s_np1[i - 1] > XW_GAP;
    int tot;
    const int pre = xw_scan<BSZ>(f ? 1 : 0, s_cnt, tot);
    // run id of position i: starts at or before i, minus one
    if (i < nu) {
      const int rid = nrun + pre + (f ? 1 : 0) - 1;
      s_r[i] = rid;
      if (rid <= XW_RUNMAX - 1) {
        if (f) s_xs[rid] = s_np0[i];
        // the last column of its run: the next position starts a run or ends the list
        const bool last = i == nu - 1 || (int64_t)s_np0[i + 1] - s_np1[i] > XW_GAP;
        if (last) s_xe[rid] = s_np1[i];
      }
    }
    nrun += tot;
  }
  __syncthreads();
  if (t == 0) {
    bool ok = nrun <= XW_RUNMAX;
    int dst = 0;
    for (int r = 0; ok && r < nrun; ++r) {
      const int len = s_xe[r] - s_xs[r];
      const int lp = (len + XW_UNIT - 1) / XW_UNIT * XW_UNIT;
      int64_t xs = s_xs[r];
      if (xs + lp > nnzN) xs = nnzN - lp;  // keep the padding inside X
      if (xs < 0) ok = false;
      s_xs[r] = (int)xs;
      s_dst[r] = dst;
      dst += lp;
    }
    if (dst > XCAP) ok = false;
    s_ok = ok ? dst / XW_UNIT : 0;
    h[7] = s_ok;
  }
  __syncthreads();
  const int nunit = s_ok;
  if (nunit == 0) {
    for (int u = t; u < NU; u += BSZ) uw[u] = 0;
    return;
  }
  for (int u = t; u < NU; u += BSZ) {
    int r = 0;
    for (int rr = 1; rr < nrun; ++rr)
      if (s_dst[rr] <= u * XW_UNIT) r = rr;
    uw[u] = u < nunit ? s_xs[r] + u * XW_UNIT - s_dst[r] : 0;
  }
#pragma unroll
  for (int i = 0; i < KPT; ++i)
    if (kr[i] >= 0) {
      const int idx = rn_lower_bound(s_v, nu, kr[i]);
      const int r = s_r[idx];
      xl[a0 + t + i * BSZ] = s_dst[r] + s_np0[idx] - s_xs[r];
    }
}

// ---- position codes: one lane per pattern entry (node entry for block_m = 2),
// one block per product block.  The column of the entry is searched in every
// neighbour row; the searches of one record word run in lockstep so their loads overlap.
// Root entries get CODE_NONE throughout; the record's first byte is the
// entry's row within the block, code u is byte u + 1. ------------------------
// Blocks with an X window (block_m = 1, the window built by k_plan_xwin)
// search in LDS: the window's column indices, and per A entry of the block
// the window offset and length of its row of N, are staged first.
template <int M>
__global__ __launch_bounds__(RN_BLOCK) void k_plan_codes(int nblk, int32_t *__restrict__ hdr,
                                                        const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ Ap,
                                                        const int32_t *__restrict__ Aj,
                                                        const int32_t *__restrict__ Np,
                                                        const int32_t *__restrict__ Nj,
                                                        const uint8_t *__restrict__ is_root, int cstride,
                                                        uint8_t *__restrict__ codes, int32_t *__restrict__ ncol,
                                                        int32_t *__restrict__ terms, const int32_t *__restrict__ xl,
                                                        const int32_t *__restrict__ xwin, int nu_stride, int acap,
                                                        int nit, uint64_t *__restrict__ ccodes) {
  constexpr int WCAP = SPG_XCAP_M1(RN_BLOCK), ACAPX = SPG_ACAP_M1(RN_BLOCK);
  __shared__ uint8_t s_row[RN_BLOCK];
  __shared__ int s_na[RN_BLOCK / RN_WAVE];
  __shared__ int32_t s_nw[M == 1 ? WCAP : 1];
  __shared__ int32_t s_xl[M == 1 ? ACAPX : 1], s_len[M == 1 ? ACAPX : 1];
  const int t = threadIdx.x;
  int32_t *h = (int32_t *)hdr + 8 * (int64_t)blockIdx.x;
  const int r0 = h[0], e0 = h[2], ne = h[3] - h[2], nrows = h[1] - h[0];
  const int a0b = h[4], nab = h[5] - h[4];
  const int nunit = M == 1 && xl ? h[7] : 0;
  const bool win = M == 1 && nunit > 0 && nab <= acap && nunit * XW_UNIT <= WCAP && nab <= ACAPX;  // uniform
  if (win) {
    const int32_t *uw = xwin + (int64_t)blockIdx.x * nu_stride;
    for (int q = t; q < nunit * XW_UNIT; q += blockDim.x) s_nw[q] = Nj[uw[q / XW_UNIT] + q % XW_UNIT];
    for (int q = t; q < nab; q += blockDim.x) {
      const int k = Aj[a0b + q];
      s_xl[q] = xl[a0b + q];
      s_len[q] = Np[k + 1] - Np[k];
    }
  }
  // per row of the block: its A range and root flag, staged with the row map
  // (the lanes then read them from LDS instead of waiting on more loads)
  __shared__ int32_t s_ra[RN_BLOCK], s_rn[RN_BLOCK];
  __shared__ uint8_t s_rr[RN_BLOCK];
  const int jpre = (M == 1 && t < ne) ? Nj[e0 + t] : 0;  // block_m = 1: the entry's column
  int na_max = 0;
  for (int rr = t; rr < nrows; rr += blockDim.x) {
    for (int q = rp[r0 + rr] - e0; q < rp[r0 + rr + 1] - e0; ++q) s_row[q] = (uint8_t)rr;
    const int a = Ap[r0 + rr], an = Ap[r0 + rr + 1] - a;
    const uint8_t rt = is_root[M * (r0 + rr)];
    s_ra[rr] = a;
    s_rn[rr] = an;
    s_rr[rr] = rt;
    if (!rt) na_max = max(na_max, an);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) na_max = max(na_max, __shfl_xor(na_max, off, RN_WAVE));
  if ((t & (RN_WAVE - 1)) == 0) s_na[t / RN_WAVE] = na_max;
  __syncthreads();
  if (t == 0) {
    int mx = s_na[0];
    for (int w = 1; w < (int)(blockDim.x / RN_WAVE); ++w) mx = max(mx, s_na[w]);
    h[6] = mx;
  }
  int hit = 0;
  if (t < ne) {
    const int lr = s_row[t];
    const int i = r0 + lr;
    uint32_t *cw = (uint32_t *)(codes + (int64_t)(e0 + t) * cstride);
    const int nw = cstride >> 2;
    uint64_t cc = (uint64_t)lr | ~(uint64_t)0xff;  // compact record: every code "none" so far
    if (s_rr[lr]) {
      cw[0] = 0xffffff00u | (uint32_t)lr;
      for (int w = 1; w < nw; ++w) cw[w] = 0xffffffffu;
      if (M == 2) ncol[e0 + t] = Nj[Np[2 * i]] / 2;
    } else {
      const int a0 = s_ra[lr], na = s_rn[lr];
      const int j = M == 1 ? jpre : Nj[Np[2 * i] + 2 * (e0 + t - rp[i])] / 2;
      if (M == 2) ncol[e0 + t] = j;
      // one record word at a time: byte b of word w holds code u = 4w + b - 1
      // (byte 0 of word 0 is the row); its four searches run in lockstep
      for (int w = 0; w < nw; ++w) {
        constexpr int U = 4;
        int ks[U], lo[U], hi[U], len[U];
        bool live[U], kroot[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
          const int u = 4 * w + q - 1;
          live[q] = u >= 0 && u < na;
          if (win) {
            const int x = live[q] ? a0 - a0b + u : 0;
            ks[q] = s_xl[x];
            len[q] = live[q] ? s_len[x] : 0;
            kroot[q] = false;
          } else {
            const int k = live[q] ? Aj[a0 + u] : 0;
            ks[q] = Np[M * k];
            len[q] = live[q] ? (Np[M * k + 1] - ks[q]) / M : 0;
            kroot[q] = live[q] && M == 2 && is_root[2 * k];
          }
          lo[q] = 0;
          hi[q] = len[q];
        }
        if (win) {
          // in LDS: nit halvings cover every row (len <= maxlen < 2^nit),
          // branch-free with clamped reads
          const int wl = nunit * XW_UNIT - 1;
          for (int it = 0; it < nit; ++it) {
#pragma unroll
            for (int q = 0; q < U; ++q) {
              const int mid = (lo[q] + hi[q]) >> 1;
              const bool lt = s_nw[min(ks[q] + mid, wl)] < j, go = lo[q] < hi[q];
              lo[q] = (go && lt) ? mid + 1 : lo[q];
              hi[q] = (go && !lt) ? mid : hi[q];
            }
          }
        } else {
          // lockstep binary search for j among the (node) columns of each row
          bool more = true;
          while (more) {
            more = false;
#pragma unroll
            for (int q = 0; q < U; ++q) {
              if (!kroot[q] && lo[q] < hi[q]) {
                const int mid = (lo[q] + hi[q]) >> 1;
                const int c = M == 1 ? Nj[ks[q] + mid] : Nj[ks[q] + 2 * mid] / 2;
                if (c < j) lo[q] = mid + 1; else hi[q] = mid;
                more = more || lo[q] < hi[q];
              }
            }
          }
        }
        uint32_t word = w == 0 ? (uint32_t)lr : 0u;
#pragma unroll
        for (int q = 0; q < U; ++q) {
          uint32_t code = CODE_NONE;
          if (win) {
            const bool f = live[q] && lo[q] < len[q] && s_nw[min(ks[q] + lo[q], nunit * XW_UNIT - 1)] == j;
            code = f ? (uint32_t)lo[q] : CODE_NONE;
          } else if (live[q]) {
            if (kroot[q]) {
              code = (Nj[ks[q]] / 2 == j) ? CODE_ROOT : CODE_NONE;
            } else if (lo[q] < len[q]) {
              const int c = M == 1 ? Nj[ks[q] + lo[q]] : Nj[ks[q] + 2 * lo[q]] / 2;
              if (c == j) code = (uint32_t)lo[q];
            }
          }
          hit += live[q] && code != CODE_NONE;
          if (w > 0 || q > 0) word |= code << (8 * q);
          const int u = 4 * w + q - 1;
          if (u >= 0 && u < CCODE_MAXNA && code != CODE_NONE)
            cc &= ~((uint64_t)(CCODE_NONE - code) << (8 + 5 * u));
        }
        cw[w] = word;
      }
    }
    if (M == 1 && ccodes) ccodes[e0 + t] = cc;
  }
  block_to_slot<false>(hit, terms);  // per-workgroup term counts
}

extern "C" rn_status rn_plan_create(rn_ctx *ctx, const rn_matrix *A, int32_t n_cols, const int32_t *Np,
                                    const int32_t *Nj, int64_t nnz_N, const uint8_t *is_root, const double *Bc,
                                    int32_t nB, rn_plan **out) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  return rn_plan_create_ex(ctx, A, n_cols, Np, Nj, nnz_N, is_root, Bc, nB, out, nullptr, nullptr, nullptr, true);
}

rn_status rn_plan_create_ex(rn_ctx *ctx, const rn_matrix *A, int32_t n_cols, const int32_t *Np, const int32_t *Nj,
                            int64_t nnz_N, const uint8_t *is_root, const double *Bc, int32_t nB, rn_plan **out,
                            int32_t *guard_in, const RnFetch *extra, unsigned char *extra_out, bool validate,
                            const double *gp_in) {
  if (!A || !out) return rn_fail(ctx, RN_EINVAL, "rn_plan_create: null argument");
  *out = nullptr;
  const int m = A->block_m;
  if ((m != 1 && m != 2) || A->n < 0 || A->n % m || A->nnz < 0 || n_cols < 0 || nnz_N < 0)
    return rn_fail(ctx, RN_EINVAL, "rn_plan_create: bad sizes");
  if (nB < 1 || nB > RN_NBMAX || (m == 2 && nB < 2))
    return rn_fail(ctx, RN_ELIMIT, "rn_plan_create: nB = %d outside the supported range", nB);
  if (A->n > 0 && (!A->rowptr || !Np || !is_root || !Bc || (A->nnz && !A->colind) || (nnz_N && !Nj)))
    return rn_fail(ctx, RN_EINVAL, "rn_plan_create: null argument");
  if (A->nnz >= ((int64_t)1 << 30) || nnz_N >= ((int64_t)1 << 31))
    return rn_fail(ctx, RN_ELIMIT, "rn_plan_create: counts reach 2^31");
  rn_plan *pl = new (std::nothrow) rn_plan();
  if (!pl) return rn_fail(ctx, RN_ENOMEM, "rn_plan_create: host allocation");
  pl->ctx = ctx;
  pl->n = A->n;
  pl->nc = n_cols;
  pl->m = m;
  pl->nB = nB;
  pl->nr = A->n / m;
  pl->nnzN = nnz_N;
  pl->nnzA = A->nnz;
  pl->Ap = A->rowptr;
  pl->Aj = A->colind;
  pl->Np = Np;
  pl->Nj = Nj;
  pl->is_root = is_root;
  pl->Bc = Bc;
  rn_status st = RN_OK;
  auto fail = [&](rn_status s) {
    rn_plan_destroy(pl);
    return s;
  };
  const int n = pl->n, nr = pl->nr;
  const int NP = nB * (nB + 1) / 2;
  int32_t *guard = guard_in ? guard_in : rn_guard_begin(ctx, &st);
  if (!guard) return fail(st);
  if (validate) {
    RnChecks v{};
    v.csr[0] = {nr, nr, A->nnz, A->rowptr, A->colind, GUARD_A};
    v.csr[1] = {n, n_cols, nnz_N, Np, Nj, GUARD_N};
    v.ncsr = 2;
    if (rn_validate(ctx, v, guard) != RN_OK) return fail(RN_EHIP);
  }
  // scratch: [0] maxlen, [1] rank_def, [2] longest A row of a non-root row,
  // [8..9] node-entry total (int64); written by the finishing kernels below
  // (zeroed here only when there are none)
  int32_t *misc = (int32_t *)rn_scratch(ctx, SLOT_MISC, 64, &st);
  if (!misc) return fail(st);
  if (nr == 0 && hipMemsetAsync(misc, 0, 64, ctx->stream) != hipSuccess)
    return fail(rn_fail(ctx, RN_EHIP, "memset"));
  if (gp_in) {
    pl->gp = (double *)gp_in;
    pl->gp_ext = true;
  }
  if ((!gp_in && !plan_alloc(pl, &pl->gp, (size_t)(n + 1) * NP * sizeof(double))) || !plan_alloc(pl, &pl->d_terms, 16) ||
      !plan_alloc(pl, &pl->xoff, (size_t)(A->nnz + 1) * m * sizeof(int32_t)))
    return fail(rn_fail(ctx, RN_ENOMEM, "rn_plan_create: device allocation"));
  if (m == 2 && !plan_alloc(pl, &pl->nodeptr, (size_t)(nr + 1) * sizeof(int32_t)))
    return fail(rn_fail(ctx, RN_ENOMEM, "rn_plan_create: device allocation"));
  pl->fixed_bytes = (size_t)(nr + 1) * 4 * (m == 2 ? 1 : 0) + (gp_in ? 0 : (size_t)(n + 1) * NP * 8) +
                    (size_t)(A->nnz + 1) * m * 4;
  // per-block partial results of the counting kernels
  const int nbn = (int)rn_div_up(n > 0 ? n : 1, RN_BLOCK);
  int32_t *blk_max = (int32_t *)rn_scratch(ctx, SLOT_BLK0, (size_t)(nbn + 1) * sizeof(int32_t), &st);
  int32_t *blk_na = (int32_t *)rn_scratch(ctx, SLOT_PAT_CNT, (size_t)(nbn + 1) * sizeof(int32_t), &st);
  if (!blk_max || !blk_na) return fail(st);
  if (nr > 0) {
    int nbc;
    if (m == 1) {
      nbc = (int)rn_div_up(n, RN_BLOCK);
      hipLaunchKernelGGL(k_plan_count_m1, dim3(nbc), dim3(RN_BLOCK), 0, ctx->stream, n, A->rowptr, Np, is_root,
                         blk_max, blk_na, guard, Bc, (int64_t)n_cols * nB, guard + GS_BCNU);
    } else {
      int32_t *ncnt = (int32_t *)rn_scratch(ctx, SLOT_STR_CNT, (size_t)(nr + 1) * sizeof(int32_t), &st);
      if (!ncnt) return fail(st);
      nbc = (int)rn_div_up(nr, RN_BLOCK);
      hipLaunchKernelGGL(k_plan_count_m2, dim3(nbc), dim3(RN_BLOCK), 0, ctx->stream, nr, A->rowptr, Np, is_root, ncnt,
                         blk_max, blk_na, guard);
      if (hipGetLastError() != hipSuccess) return fail(rn_fail(ctx, RN_EHIP, "launch"));
      if (rn_scan_counts(ctx, ncnt, pl->nodeptr, nr, nullptr) != RN_OK) return fail(RN_EHIP);
      if (hipMemcpyAsync(misc + 8, ctx->slot[SLOT_SCAN_TOTAL].ptr, 8, hipMemcpyDeviceToDevice, ctx->stream) !=
          hipSuccess)
        return fail(rn_fail(ctx, RN_EHIP, "copy"));
    }
    if (hipGetLastError() != hipSuccess) return fail(rn_fail(ctx, RN_EHIP, "launch"));
    hipLaunchKernelGGL((k_finish_slots<true, int32_t>), dim3(2), dim3(RN_BLOCK), 0, ctx->stream, blk_max, nbc, misc,
                       (const int32_t *)blk_na, misc + 2);
    // the Gram data (or none: the caller's, and a zero count)
    const int nbg = gp_in ? 0 : nbn;
    int32_t *blk_bad = (int32_t *)rn_scratch(ctx, SLOT_BLK1, (size_t)(nbg + 1) * sizeof(int32_t), &st);
    if (!blk_bad) return fail(st);
    if (!gp_in) {
      const dim3 g(nbg), bl(RN_BLOCK);
      switch (nB) {
        case 1: hipLaunchKernelGGL(k_plan_gram<1>, g, bl, 0, ctx->stream, n, Np, Nj, is_root, Bc, pl->gp, blk_bad, guard); break;
        case 2: hipLaunchKernelGGL(k_plan_gram<2>, g, bl, 0, ctx->stream, n, Np, Nj, is_root, Bc, pl->gp, blk_bad, guard); break;
        case 3: hipLaunchKernelGGL(k_plan_gram<3>, g, bl, 0, ctx->stream, n, Np, Nj, is_root, Bc, pl->gp, blk_bad, guard); break;
        case 4: hipLaunchKernelGGL(k_plan_gram<4>, g, bl, 0, ctx->stream, n, Np, Nj, is_root, Bc, pl->gp, blk_bad, guard); break;
      }
    }
    hipLaunchKernelGGL((k_finish_slots<false, int32_t>), dim3(1), dim3(RN_BLOCK), 0, ctx->stream, blk_bad, nbg,
                       misc + 1);
    if (hipGetLastError() != hipSuccess) return fail(rn_fail(ctx, RN_EHIP, "launch"));
  }
  // one synchronisation: guard, maxlen, rank_def, longest A row, node-entry total
  // (and the caller's extra item, read at the same synchronisation)
  const RnFetch it[4] = {{misc, 16}, {misc + 8, 8}, {guard, 4 * (GS_BCNU + 1)}, extra ? *extra : RnFetch{nullptr, 0}};
  const unsigned char *hb = nullptr;
  size_t off[4];
  st = rn_fetch(ctx, extra ? 4 : 3, it, &hb, off);
  if (st != RN_OK) return fail(st);
  if (extra) memcpy(extra_out, hb + off[3], extra->bytes);
  int64_t hp[5];
  int32_t gword = 0, bcnu = 1;
  memcpy(hp + 2, hb + off[0], 16);
  memcpy(hp + 4, hb + off[1], 8);
  memcpy(&gword, hb + off[2], 4);
  memcpy(&bcnu, hb + off[2] + 4 * GS_BCNU, 4);
  pl->unit_bc = m == 1 && nr > 0 && bcnu == 0;
  st = rn_guard_status(ctx, gword, "rn_plan_create");
  if (st != RN_OK) {
    if (st == RN_ELIMIT)
      rn_fail(ctx, RN_ELIMIT, "rn_plan_create: a pattern row holds more than %d entries", CODE_MAXLEN);
    return fail(st);
  }
  pl->maxlen = ((const int32_t *)(hp + 2))[0];
  pl->rank_def = ((const int32_t *)(hp + 2))[1];
  const int maxna = ((const int32_t *)(hp + 2))[2];
  pl->nnzN_node = m == 1 ? nnz_N : hp[4];
  if (maxna > CODE_MAXLEN)
    return fail(rn_fail(ctx, RN_ELIMIT, "rn_plan_create: an A row holds more than %d entries", CODE_MAXLEN));
  // record: the codes, then the row byte
  pl->cstride = 4 * ((maxna + 1 + 3) / 4);
  const int64_t ncodes = pl->nnzN_node * pl->cstride;
  pl->ncodes = ncodes;
  // the product forms element offsets in 32 bits
  const int64_t lim = (int64_t)1 << 29;
  if (ncodes >= ((int64_t)1 << 31) || nnz_N * nB >= lim || A->nnz * m * m >= lim || (int64_t)(n + 1) * NP >= lim ||
      (int64_t)n_cols * nB >= lim)
    return fail(rn_fail(ctx, RN_ELIMIT, "rn_plan_create: pattern or operator too large for 32-bit offsets"));
  // product blocks: every block holds at most 256 entries (node entries for
  // block_m = 2): rows starting in a chunk of 257 - maxlen entries
  const int ml = pl->maxlen < 1 ? 1 : pl->maxlen;
  // 64- and 128-lane blocks for scalar operators with short pattern rows
  // (RN_OPT_PRODUCT_LANES)
  const int lanes = ctx->opt[RN_OPT_PRODUCT_LANES];
  pl->bs = (m == 1 && (lanes == 64 || lanes == 128) && ml <= lanes / 4) ? lanes : RN_BLOCK;
  pl->persist = ctx->opt[RN_OPT_PERSISTENT_PRODUCT] != 0;
  pl->chunk = pl->bs + 1 - ml;
  pl->nblk = (int)((pl->nnzN_node + pl->chunk - 1) / pl->chunk);
  if ((m == 2 && !plan_alloc(pl, &pl->ncol, (size_t)(pl->nnzN_node + 1) * sizeof(int32_t))) ||
      !plan_alloc(pl, &pl->codes, (size_t)ncodes + 16) ||
      !plan_alloc(pl, &pl->blk_row, (size_t)(pl->nblk + 1) * sizeof(int32_t)) ||
      !plan_alloc(pl, &pl->blk_hdr, (size_t)(pl->nblk + 1) * 8 * sizeof(int32_t)))
    return fail(rn_fail(ctx, RN_ENOMEM, "rn_plan_create: code allocation (%lld bytes)", (long long)ncodes));
  pl->fixed_bytes += (size_t)ncodes + (size_t)(pl->nblk + 1) * 36 + (m == 2 ? (size_t)(pl->nnzN_node + 1) * 4 : 0);
  const int nunit_max = SPG_XCAP_M1(pl->bs) / XW_UNIT;
  if (m == 1 && (!plan_alloc(pl, &pl->xl, (size_t)(A->nnz + 1) * sizeof(int32_t)) ||
                 !plan_alloc(pl, &pl->xwin, (size_t)(pl->nblk + 1) * nunit_max * sizeof(int32_t))))
    return fail(rn_fail(ctx, RN_ENOMEM, "rn_plan_create: device allocation"));
  if (m == 1) pl->fixed_bytes += (size_t)(A->nnz + 1) * 4 + (size_t)(pl->nblk + 1) * nunit_max * 4;
  // compact records where every code fits 5 bits and a row's codes 56 bits
  if (m == 1 && maxna <= CCODE_MAXNA && pl->maxlen <= CCODE_MAXLEN && nnz_N > 0) {
    if (!plan_alloc(pl, &pl->ccodes, (size_t)(nnz_N + 1) * sizeof(uint64_t)))
      return fail(rn_fail(ctx, RN_ENOMEM, "rn_plan_create: device allocation"));
    pl->fixed_bytes += (size_t)(nnz_N + 1) * 8;
  }
  if (m == 1 && nB <= 2) {
    if (!plan_alloc(pl, &pl->bce, (size_t)(nnz_N + 1) * nB * sizeof(double)))
      return fail(rn_fail(ctx, RN_ENOMEM, "rn_plan_create: device allocation"));
    pl->fixed_bytes += (size_t)(nnz_N + 1) * nB * 8;
  }
  const int32_t *rp = m == 1 ? Np : pl->nodeptr;
  hipLaunchKernelGGL(k_plan_blocks_rows, dim3(rn_div_up(nr + 1, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, nr, rp,
                     A->rowptr, pl->nblk, pl->chunk, pl->blk_row, pl->blk_hdr);
  if (hipGetLastError() != hipSuccess) return fail(rn_fail(ctx, RN_EHIP, "launch"));
  const int64_t n_bce = pl->bce ? nnz_N : 0;
  if (A->nnz > 0 || n_bce > 0) {
    unsigned g = rn_div_up(A->nnz > n_bce ? A->nnz : n_bce, RN_BLOCK);
    hipLaunchKernelGGL(k_plan_bce_xoff, dim3(g > 8192 ? 8192 : g), dim3(RN_BLOCK), 0, ctx->stream, n_bce, nB, Nj, Bc,
                       pl->bce, A->nnz, m, A->colind, Np, pl->xoff);
    if (hipGetLastError() != hipSuccess) return fail(rn_fail(ctx, RN_EHIP, "launch"));
  }
  if (pl->nblk > 0) {
    int32_t *blk_hit = (int32_t *)rn_scratch(ctx, SLOT_BLK2, (size_t)(pl->nblk + 1) * sizeof(int32_t), &st);
    if (!blk_hit) return fail(st);
    const dim3 gc(pl->nblk), bc(pl->bs);  // one thread per entry slot of a product block
    const int nb = pl->nblk;
    // X windows first: the codes of a block with a window are searched in LDS
    if (m == 1) {
      switch (pl->bs) {
        case 64:
          hipLaunchKernelGGL(k_plan_xwin<64>, gc, dim3(64), 0, ctx->stream, pl->blk_hdr, A->colind, Np, nnz_N, pl->xl,
                             pl->xwin);
          break;
        case 128:
          hipLaunchKernelGGL(k_plan_xwin<128>, gc, dim3(128), 0, ctx->stream, pl->blk_hdr, A->colind, Np, nnz_N,
                             pl->xl, pl->xwin);
          break;
        default:
          hipLaunchKernelGGL(k_plan_xwin<RN_BLOCK>, gc, dim3(RN_BLOCK), 0, ctx->stream, pl->blk_hdr, A->colind, Np,
                             nnz_N, pl->xl, pl->xwin);
      }
    }
    const int nu_stride = SPG_XCAP_M1(pl->bs) / XW_UNIT, acap = SPG_ACAP_M1(pl->bs);
    if (m == 1)
      hipLaunchKernelGGL((k_plan_codes<1>), gc, bc, 0, ctx->stream, nb, pl->blk_hdr, rp, A->rowptr, A->colind, Np,
                         Nj, is_root, pl->cstride, pl->codes, pl->ncol, blk_hit, pl->xl, pl->xwin, nu_stride, acap,
                         32 - __builtin_clz((unsigned)(pl->maxlen > 0 ? pl->maxlen : 1)), pl->ccodes);
    else
      hipLaunchKernelGGL((k_plan_codes<2>), gc, bc, 0, ctx->stream, nb, pl->blk_hdr, rp, A->rowptr, A->colind, Np,
                         Nj, is_root, pl->cstride, pl->codes, pl->ncol, blk_hit, (const int32_t *)nullptr,
                         (const int32_t *)nullptr, 0, 0, 0, (uint64_t *)nullptr);
    hipLaunchKernelGGL((k_finish_slots<false, unsigned long long>), dim3(1), dim3(RN_BLOCK), 0, ctx->stream, blk_hit,
                       pl->nblk, pl->d_terms);
    if (hipGetLastError() != hipSuccess) return fail(rn_fail(ctx, RN_EHIP, "launch"));
  } else if (hipMemsetAsync(pl->d_terms, 0, 16, ctx->stream) != hipSuccess) {  // no blocks: no terms
    return fail(rn_fail(ctx, RN_EHIP, "memset"));
  }
  try {
    ctx->plans.push_back(pl);
  } catch (...) {
    return fail(rn_fail(ctx, RN_ENOMEM, "rn_plan_create: host allocation"));
  }
  *out = pl;
  return RN_OK;
}

// The plan's device memory back to its context (stream-ordered reuse, no
// wait); the plan keeps only its host object.
void rn_plan_release(rn_plan *pl) {
  if (!pl->ctx) return;
  if (pl->gp_ext) pl->gp = nullptr;
  void **bufs[] = {(void **)&pl->codes,   (void **)&pl->ncol,    (void **)&pl->nodeptr, (void **)&pl->gp,
                   (void **)&pl->d_terms, (void **)&pl->blk_row, (void **)&pl->blk_hdr, (void **)&pl->xoff,
                   (void **)&pl->xl,      (void **)&pl->xwin,    (void **)&pl->bce,     (void **)&pl->ccodes};
  for (void **b : bufs) {
    rn_dev_free(pl->ctx, *b);
    *b = nullptr;
  }
  for (int s = 0; s < WS_COUNT; ++s) {
    rn_dev_free(pl->ctx, pl->ws[s].ptr);
    pl->ws[s].ptr = nullptr;
    pl->ws[s].cap = 0;
  }
  pl->ctx = nullptr;
}

extern "C" void rn_plan_destroy(rn_plan *pl) {
  if (!pl) return;
  if (pl->ctx) {  // (a plan whose context was destroyed first holds no device memory)
    auto &v = pl->ctx->plans;
    for (size_t q = 0; q < v.size(); ++q)
      if (v[q] == pl) {
        v[q] = v.back();
        v.pop_back();
        break;
      }
    rn_plan_release(pl);
  }
  delete pl;
}

extern "C" size_t rn_plan_bytes(const rn_plan *pl) {
  if (!pl) return 0;
  size_t b = pl->fixed_bytes;
  for (int s = 0; s < WS_COUNT; ++s) b += pl->ws[s].cap;
  return b;
}
