// rn_plan.hip -- symbolic part of the energy minimisation (Sec. 3.6): the
// position codes of the masked product, the per-row least-squares data of the
// constraint projection and the block partition of the product.
#include <cstring>
#include <new>

#include "rn_emin.h"

void *rn_plan_ws(rn_plan *pl, int slot, size_t bytes, rn_status *st) {
  RnScratch &s = pl->ws[slot];
  if (bytes == 0) bytes = 16;
  if (s.cap >= bytes) return s.ptr;
  if (s.ptr) {
    (void)hipStreamSynchronize(pl->ctx->stream);
    (void)hipFree(s.ptr);
    s.ptr = nullptr;
    s.cap = 0;
  }
  const size_t cap = bytes + bytes / 8 + 256;
  if (hipMalloc(&s.ptr, cap) != hipSuccess) {
    s.ptr = nullptr;
    *st = rn_fail(pl->ctx, RN_ENOMEM, "plan workspace allocation of %zu bytes failed", cap);
    return nullptr;
  }
  s.cap = cap;
  return s.ptr;
}

static __device__ inline int pad4(int x) { return (x + 3) & ~3; }

// ---- block_m = 1 ----------------------------------------------------------
__global__ __launch_bounds__(RN_BLOCK) void k_plan_count_m1(int n, const int32_t *__restrict__ Ap,
                                                           const int32_t *__restrict__ Np,
                                                           const uint8_t *__restrict__ is_root,
                                                           int32_t *__restrict__ ccnt, int32_t *__restrict__ maxlen,
                                                           int32_t *__restrict__ guard) {
  const int i = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (i >= n) return;
  if (*guard) {
    ccnt[i] = 0;
    return;
  }
  const int len = Np[i + 1] - Np[i];
  if (len > CODE_MAXLEN) atomicOr(guard, GUARD_LIMIT);
  if (len == 0 || (is_root[i] && len != 1)) atomicOr(guard, GUARD_N);
  atomicMax(maxlen, len);
  ccnt[i] = is_root[i] ? 0 : len * pad4(Ap[i + 1] - Ap[i]);
}

__global__ __launch_bounds__(RN_BLOCK) void k_plan_codes_m1(int n, const int32_t *__restrict__ Ap,
                                                           const int32_t *__restrict__ Aj,
                                                           const int32_t *__restrict__ Np,
                                                           const int32_t *__restrict__ Nj,
                                                           const uint8_t *__restrict__ is_root,
                                                           const int32_t *__restrict__ code_ptr,
                                                           uint8_t *__restrict__ codes,
                                                           unsigned long long *__restrict__ terms,
                                                           const int32_t *__restrict__ guard) {
  const int i = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (i >= n || *guard || is_root[i]) return;
  const int s = Np[i], len = Np[i + 1] - s;
  const int a0 = Ap[i], na = Ap[i + 1] - a0, na4 = pad4(na);
  uint8_t *cw = codes + code_ptr[i];
  unsigned long long hit = 0;
  for (int t = 0; t < na; ++t) {
    const int k = Aj[a0 + t], ks = Np[k], ke = Np[k + 1];
    int u = ks;
    for (int r = 0; r < len; ++r) {
      const int j = Nj[s + r];
      while (u < ke && Nj[u] < j) ++u;
      const bool f = u < ke && Nj[u] == j;
      cw[r * na4 + t] = f ? (uint8_t)(u - ks) : (uint8_t)CODE_NONE;
      hit += f;
    }
  }
  for (int r = 0; r < len; ++r)
    for (int t = na; t < na4; ++t) cw[r * na4 + t] = CODE_NONE;
  atomicAdd(terms, hit);
}

// ---- block_m = 2 (node rows) --------------------------------------------------
__global__ __launch_bounds__(RN_BLOCK) void k_plan_count_m2(int nr, const int32_t *__restrict__ Ap,
                                                           const int32_t *__restrict__ Np,
                                                           const uint8_t *__restrict__ is_root,
                                                           int32_t *__restrict__ ncnt, int32_t *__restrict__ ccnt,
                                                           int32_t *__restrict__ maxlen,
                                                           int32_t *__restrict__ guard) {
  const int I = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (I >= nr) return;
  if (*guard) {
    ncnt[I] = 0;
    ccnt[I] = 0;
    return;
  }
  const bool root = is_root[2 * I];
  const int l0 = Np[2 * I + 1] - Np[2 * I], l1 = Np[2 * I + 2] - Np[2 * I + 1];
  if (root != (bool)is_root[2 * I + 1]) atomicOr(guard, GUARD_N);
  if (root) {
    if (l0 != 1 || l1 != 1) atomicOr(guard, GUARD_N);
    ncnt[I] = 1;
    ccnt[I] = 0;
    return;
  }
  if (l0 != l1 || (l0 & 1) || l0 == 0) atomicOr(guard, GUARD_N);
  const int len = l0 / 2;
  if (len > CODE_MAXLEN) atomicOr(guard, GUARD_LIMIT);
  atomicMax(maxlen, len);
  ncnt[I] = len;
  ccnt[I] = len * pad4(Ap[I + 1] - Ap[I]);
}

__global__ __launch_bounds__(RN_BLOCK) void k_plan_codes_m2(int nr, const int32_t *__restrict__ Ap,
                                                           const int32_t *__restrict__ Aj,
                                                           const int32_t *__restrict__ Np,
                                                           const int32_t *__restrict__ Nj,
                                                           const uint8_t *__restrict__ is_root,
                                                           const int32_t *__restrict__ code_ptr,
                                                           uint8_t *__restrict__ codes,
                                                           unsigned long long *__restrict__ terms,
                                                           const int32_t *__restrict__ guard) {
  const int I = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (I >= nr || *guard || is_root[2 * I]) return;
  const int s = Np[2 * I], len = (Np[2 * I + 1] - s) / 2;
  const int a0 = Ap[I], na = Ap[I + 1] - a0, na4 = pad4(na);
  uint8_t *cw = codes + code_ptr[I];
  unsigned long long hit = 0;
  for (int t = 0; t < na; ++t) {
    const int K = Aj[a0 + t], ks = Np[2 * K];
    if (is_root[2 * K]) {
      const int aK = Nj[ks] / 2;
      for (int r = 0; r < len; ++r) {
        const bool f = Nj[s + 2 * r] / 2 == aK;
        cw[r * na4 + t] = f ? (uint8_t)CODE_ROOT : (uint8_t)CODE_NONE;
        hit += f;
      }
    } else {
      const int lk = (Np[2 * K + 1] - ks) / 2;
      int u = 0;
      for (int r = 0; r < len; ++r) {
        const int a = Nj[s + 2 * r] / 2;
        while (u < lk && Nj[ks + 2 * u] / 2 < a) ++u;
        const bool f = u < lk && Nj[ks + 2 * u] / 2 == a;
        cw[r * na4 + t] = f ? (uint8_t)u : (uint8_t)CODE_NONE;
        hit += f;
      }
    }
  }
  for (int r = 0; r < len; ++r)
    for (int t = na; t < na4; ++t) cw[r * na4 + t] = CODE_NONE;
  atomicAdd(terms, hit);
}

template <int NB>
__global__ __launch_bounds__(RN_BLOCK) void k_plan_gram(int n, const int32_t *__restrict__ Np,
                                                       const int32_t *__restrict__ Nj,
                                                       const uint8_t *__restrict__ is_root,
                                                       const double *__restrict__ Bc, double *__restrict__ gp,
                                                       int32_t *__restrict__ rank_def,
                                                       const int32_t *__restrict__ guard) {
  constexpr int NP = NB * (NB + 1) / 2;
  const int i = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (i >= n || *guard) return;
  double *out = gp + (int64_t)i * NP;
  if (is_root[i]) {
    for (int q = 0; q < NP; ++q) out[q] = 0.0;
    return;
  }
  double Gp[NB * NB];
  if (rn_row_pinv<NB>(Nj, Np[i], Np[i + 1], Bc, Gp)) atomicAdd(rank_def, 1);
#pragma unroll
  for (int q = 0; q < NB; ++q)
#pragma unroll
    for (int r = q; r < NB; ++r) out[rn_pk(NB, q, r)] = Gp[q * NB + r];
}

// first row of each product block: rows whose first entry falls in
// [b*chunk, (b+1)*chunk) belong to block b
__global__ __launch_bounds__(RN_BLOCK) void k_plan_blocks(int nr, const int32_t *__restrict__ rp, int nblk,
                                                         int chunk, int32_t *__restrict__ blk_row) {
  const int b = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (b > nblk) return;
  blk_row[b] = b == nblk ? nr : rn_lower_bound(rp, nr, (int64_t)b * chunk);
}

extern "C" rn_status rn_plan_create(rn_ctx *ctx, const rn_matrix *A, int32_t n_cols, const int32_t *Np,
                                    const int32_t *Nj, int64_t nnz_N, const uint8_t *is_root, const double *Bc,
                                    int32_t nB, rn_plan **out) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (!A || !out) return rn_fail(ctx, RN_EINVAL, "rn_plan_create: null argument");
  *out = nullptr;
  const int m = A->block_m;
  if ((m != 1 && m != 2) || A->n < 0 || A->n % m || A->nnz < 0 || n_cols < 0 || nnz_N < 0)
    return rn_fail(ctx, RN_EINVAL, "rn_plan_create: bad sizes");
  if (nB < 1 || nB > RN_NBMAX || (m == 2 && nB < 2))
    return rn_fail(ctx, RN_ELIMIT, "rn_plan_create: nB = %d outside the supported range", nB);
  if (A->n > 0 && (!A->rowptr || !Np || !is_root || !Bc || (A->nnz && !A->colind) || (nnz_N && !Nj)))
    return rn_fail(ctx, RN_EINVAL, "rn_plan_create: null argument");
  if (A->nnz >= ((int64_t)1 << 31) || nnz_N >= ((int64_t)1 << 31))
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
  int32_t *guard = rn_guard_begin(ctx, &st);
  if (!guard) return fail(st);
  if (rn_validate_csr(ctx, nr, nr, A->nnz, A->rowptr, A->colind, guard, GUARD_A) != RN_OK ||
      rn_validate_csr(ctx, n, n_cols, nnz_N, Np, Nj, guard, GUARD_N) != RN_OK)
    return fail(RN_EHIP);
  // scratch: [0] maxlen, [1] rank_def, [8..9] node-entry total (int64)
  int32_t *misc = (int32_t *)rn_scratch(ctx, SLOT_MISC, 64, &st);
  if (!misc) return fail(st);
  if (hipMemsetAsync(misc, 0, 64, ctx->stream) != hipSuccess) return fail(rn_fail(ctx, RN_EHIP, "memset"));
  int32_t *ccnt = (int32_t *)rn_scratch(ctx, SLOT_PAT_CNT, (size_t)(nr + 1) * sizeof(int32_t), &st);
  if (!ccnt) return fail(st);
  if (hipMalloc(&pl->code_ptr, (size_t)(nr + 1) * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&pl->gp, (size_t)(n + 1) * NP * sizeof(double)) != hipSuccess ||
      hipMalloc(&pl->d_terms, 16) != hipSuccess)
    return fail(rn_fail(ctx, RN_ENOMEM, "rn_plan_create: device allocation"));
  if (m == 2 && hipMalloc(&pl->nodeptr, (size_t)(nr + 1) * sizeof(int32_t)) != hipSuccess)
    return fail(rn_fail(ctx, RN_ENOMEM, "rn_plan_create: device allocation"));
  pl->fixed_bytes = (size_t)(nr + 1) * 4 * (m == 2 ? 2 : 1) + (size_t)(n + 1) * NP * 8;
  if (hipMemsetAsync(pl->d_terms, 0, 16, ctx->stream) != hipSuccess) return fail(rn_fail(ctx, RN_EHIP, "memset"));
  if (nr > 0) {
    if (m == 1) {
      hipLaunchKernelGGL(k_plan_count_m1, dim3(rn_div_up(n, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, n, A->rowptr,
                         Np, is_root, ccnt, misc, guard);
    } else {
      int32_t *ncnt = (int32_t *)rn_scratch(ctx, SLOT_STR_CNT, (size_t)(nr + 1) * sizeof(int32_t), &st);
      if (!ncnt) return fail(st);
      hipLaunchKernelGGL(k_plan_count_m2, dim3(rn_div_up(nr, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, nr,
                         A->rowptr, Np, is_root, ncnt, ccnt, misc, guard);
      if (hipGetLastError() != hipSuccess) return fail(rn_fail(ctx, RN_EHIP, "launch"));
      if (rn_scan_counts(ctx, ncnt, pl->nodeptr, nr, nullptr) != RN_OK) return fail(RN_EHIP);
      if (hipMemcpyAsync(misc + 8, ctx->slot[SLOT_SCAN_TOTAL].ptr, 8, hipMemcpyDeviceToDevice, ctx->stream) !=
          hipSuccess)
        return fail(rn_fail(ctx, RN_EHIP, "copy"));
    }
    if (hipGetLastError() != hipSuccess) return fail(rn_fail(ctx, RN_EHIP, "launch"));
    const dim3 g(rn_div_up(n, RN_BLOCK)), bl(RN_BLOCK);
    switch (nB) {
      case 1: hipLaunchKernelGGL(k_plan_gram<1>, g, bl, 0, ctx->stream, n, Np, Nj, is_root, Bc, pl->gp, misc + 1, guard); break;
      case 2: hipLaunchKernelGGL(k_plan_gram<2>, g, bl, 0, ctx->stream, n, Np, Nj, is_root, Bc, pl->gp, misc + 1, guard); break;
      case 3: hipLaunchKernelGGL(k_plan_gram<3>, g, bl, 0, ctx->stream, n, Np, Nj, is_root, Bc, pl->gp, misc + 1, guard); break;
      case 4: hipLaunchKernelGGL(k_plan_gram<4>, g, bl, 0, ctx->stream, n, Np, Nj, is_root, Bc, pl->gp, misc + 1, guard); break;
    }
    if (hipGetLastError() != hipSuccess) return fail(rn_fail(ctx, RN_EHIP, "launch"));
  }
  if (rn_scan_counts(ctx, ccnt, pl->code_ptr, nr, nullptr) != RN_OK) return fail(RN_EHIP);
  // one synchronisation: guard, code total, maxlen, rank_def, node-entry total
  int64_t *hp = ctx->pinned;
  if (hipMemcpyAsync(hp + 1, ctx->slot[SLOT_SCAN_TOTAL].ptr, 8, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipMemcpyAsync(hp + 2, misc, 8, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipMemcpyAsync(hp + 4, misc + 8, 8, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess)
    return fail(rn_fail(ctx, RN_EHIP, "copy"));
  st = rn_check_guard(ctx, guard, "rn_plan_create");
  if (st != RN_OK) {
    if (st == RN_ELIMIT)
      rn_fail(ctx, RN_ELIMIT, "rn_plan_create: a pattern row holds more than %d entries", CODE_MAXLEN);
    return fail(st);
  }
  const int64_t ncodes = hp[1];
  pl->maxlen = ((const int32_t *)(hp + 2))[0];
  pl->rank_def = ((const int32_t *)(hp + 2))[1];
  pl->nnzN_node = m == 1 ? nnz_N : hp[4];
  if (ncodes >= ((int64_t)1 << 31)) return fail(rn_fail(ctx, RN_ELIMIT, "rn_plan_create: plan codes reach 2^31"));
  pl->ncodes = ncodes;
  if (hipMalloc(&pl->codes, (size_t)ncodes + 16) != hipSuccess)
    return fail(rn_fail(ctx, RN_ENOMEM, "rn_plan_create: code allocation (%lld bytes)", (long long)ncodes));
  pl->fixed_bytes += (size_t)ncodes;
  if (nr > 0) {
    if (m == 1)
      hipLaunchKernelGGL(k_plan_codes_m1, dim3(rn_div_up(n, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, n, A->rowptr,
                         A->colind, Np, Nj, is_root, pl->code_ptr, pl->codes, pl->d_terms, guard);
    else
      hipLaunchKernelGGL(k_plan_codes_m2, dim3(rn_div_up(nr, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, nr,
                         A->rowptr, A->colind, Np, Nj, is_root, pl->code_ptr, pl->codes, pl->d_terms, guard);
    if (hipGetLastError() != hipSuccess) return fail(rn_fail(ctx, RN_EHIP, "launch"));
  }
  // product blocks: every block holds at most 256 entries (node entries for
  // block_m = 2): rows starting in a chunk of 257 - maxlen entries
  const int ml = pl->maxlen < 1 ? 1 : pl->maxlen;
  pl->chunk = RN_BLOCK + 1 - ml;
  pl->nblk = (int)((pl->nnzN_node + pl->chunk - 1) / pl->chunk);
  if (hipMalloc(&pl->blk_row, (size_t)(pl->nblk + 1) * sizeof(int32_t)) != hipSuccess)
    return fail(rn_fail(ctx, RN_ENOMEM, "rn_plan_create: device allocation"));
  pl->fixed_bytes += (size_t)(pl->nblk + 1) * 4;
  hipLaunchKernelGGL(k_plan_blocks, dim3(rn_div_up(pl->nblk + 1, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, nr,
                     m == 1 ? Np : pl->nodeptr, pl->nblk, pl->chunk, pl->blk_row);
  if (hipGetLastError() != hipSuccess) return fail(rn_fail(ctx, RN_EHIP, "launch"));
  *out = pl;
  return RN_OK;
}

extern "C" void rn_plan_destroy(rn_plan *pl) {
  if (!pl) return;
  if (pl->ctx) (void)hipStreamSynchronize(pl->ctx->stream);
  void *bufs[] = {pl->code_ptr, pl->codes, pl->nodeptr, pl->gp, pl->d_terms, pl->blk_row};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  for (int s = 0; s < WS_COUNT; ++s)
    if (pl->ws[s].ptr) (void)hipFree(pl->ws[s].ptr);
  delete pl;
}

extern "C" size_t rn_plan_bytes(const rn_plan *pl) {
  if (!pl) return 0;
  size_t b = pl->fixed_bytes;
  for (int s = 0; s < WS_COUNT; ++s) b += pl->ws[s].cap;
  return b;
}
