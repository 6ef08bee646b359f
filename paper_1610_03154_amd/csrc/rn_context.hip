// rn_context.hip -- context, scratch, scan and CSR transpose.
#include "rn_internal.h"

#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

rn_status rn_fail(rn_ctx *ctx, rn_status st, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

#define RN_CACHE_MAX ((size_t)8 << 30)  // bytes a context keeps for reuse

static void cache_release(rn_ctx *ctx, size_t keep) {
  while (ctx->cached_bytes > keep && !ctx->cache.empty()) {
    const rn_ctx::Block b = ctx->cache.front();  // oldest first
    ctx->cache.erase(ctx->cache.begin());
    ctx->cached_bytes -= b.cap;
    (void)hipFree(b.p);
  }
}

void *rn_dev_alloc(rn_ctx *ctx, size_t bytes) {
  bytes = bytes == 0 ? 256 : (bytes + 255) & ~(size_t)255;
  try {
    if (ctx->alloc_fn) {
      void *p = ctx->alloc_fn(bytes, ctx->alloc_user);
      if (!p) return nullptr;
      ctx->live[p] = bytes;
      return p;
    }
    // the smallest cached block that fits and wastes at most half of itself
    int best = -1;
    for (int i = 0; i < (int)ctx->cache.size(); ++i) {
      const size_t c = ctx->cache[i].cap;
      if (c >= bytes && c <= 2 * bytes + 4096 && (best < 0 || c < ctx->cache[best].cap)) best = i;
    }
    if (best >= 0) {
      const rn_ctx::Block b = ctx->cache[best];
      ctx->cache.erase(ctx->cache.begin() + best);
      ctx->cached_bytes -= b.cap;
      ctx->live[b.p] = b.cap;
      return b.p;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipStreamSynchronize(ctx->stream);
      cache_release(ctx, 0);
      if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    ctx->live[p] = bytes;
    return p;
  } catch (...) {
    return nullptr;
  }
}

void rn_dev_free(rn_ctx *ctx, void *p) {
  if (!p) return;
  if (!ctx) {
    (void)hipFree(p);
    return;
  }
  auto it = ctx->live.find(p);
  if (it == ctx->live.end()) {
    (void)hipFree(p);
    return;
  }
  if (ctx->free_fn) {  // stream-ordered reuse is the caller's allocator's business
    ctx->live.erase(it);
    ctx->free_fn(p, ctx->alloc_user);
    return;
  }
  try {
    ctx->cache.push_back({p, it->second});
    ctx->cached_bytes += it->second;
    ctx->live.erase(it);
    if (ctx->cached_bytes > RN_CACHE_MAX) {
      (void)hipStreamSynchronize(ctx->stream);
      cache_release(ctx, RN_CACHE_MAX / 2);
    }
  } catch (...) {
    ctx->live.erase(p);
    (void)hipFree(p);
  }
}

void *rn_scratch(rn_ctx *ctx, int slot, size_t bytes, rn_status *st) {
  RnScratch &s = ctx->slot[slot];
  if (bytes == 0) bytes = 16;
  if (s.cap >= bytes) return s.ptr;
  if (s.ptr) {
    if (ctx->free_fn) {
      ctx->free_fn(s.ptr, ctx->alloc_user);
    } else {
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipFree(s.ptr);
    }
    s.ptr = nullptr;
    s.cap = 0;
  }
  size_t cap = bytes + bytes / 4 + 256;
  if (ctx->alloc_fn) {
    s.ptr = ctx->alloc_fn(cap, ctx->alloc_user);
  } else if (hipMalloc(&s.ptr, cap) != hipSuccess) {
    (void)hipGetLastError();
    s.ptr = nullptr;
  }
  if (!s.ptr) {
    *st = rn_fail(ctx, RN_ENOMEM, "scratch allocation of %zu bytes failed", cap);
    return nullptr;
  }
  s.cap = cap;
  return s.ptr;
}

// (Re)allocate the pinned read-back area with room for cap bytes.
static rn_status readback_reserve(rn_ctx *ctx, size_t cap) {
  if (ctx->rb_host) {
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    (void)hipHostFree(ctx->rb_host);
    ctx->rb_host = nullptr;
    ctx->rb_dev = nullptr;
    ctx->rb_cap = 0;
  }
  if (cap < 4096) cap = 4096;
  if (hipHostMalloc((void **)&ctx->rb_host, cap, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    (void)hipGetLastError();
    ctx->rb_host = nullptr;
    return rn_fail(ctx, RN_ENOMEM, "rn_fetch: pinned read-back area of %zu bytes", cap);
  }
  ctx->rb_cap = cap;
  void *d = nullptr;
  if (hipHostGetDevicePointer(&d, ctx->rb_host, 0) != hipSuccess) {
    (void)hipGetLastError();
    d = nullptr;
  }
  ctx->rb_dev = d;
  return RN_OK;
}

struct FetchArgs {
  const uint32_t *src[RN_FETCH_MAX];
  int32_t words[RN_FETCH_MAX];
  int32_t off[RN_FETCH_MAX];  // in 4-byte words
  int n;
};

__global__ __launch_bounds__(RN_BLOCK) void k_fetch(const FetchArgs a, uint32_t *__restrict__ dst) {
  for (int i = 0; i < a.n; ++i)
    for (int q = threadIdx.x; q < a.words[i]; q += RN_BLOCK) dst[a.off[i] + q] = a.src[i][q];
}

rn_status rn_fetch(rn_ctx *ctx, int n, const RnFetch *items, const unsigned char **host, size_t *off) {
  if (n < 0 || n > RN_FETCH_MAX) return rn_fail(ctx, RN_EINVAL, "rn_fetch: %d items", n);
  size_t total = 0;
  for (int i = 0; i < n; ++i) {
    if (((uintptr_t)items[i].src & 3) || (items[i].bytes & 3) || items[i].bytes >= ((size_t)1 << 31))
      return rn_fail(ctx, RN_EINVAL, "rn_fetch: misaligned item");
    off[i] = total;
    total += (items[i].bytes + 7) & ~(size_t)7;
  }
  if (total > ctx->rb_cap) RN_TRY(readback_reserve(ctx, total + total / 2));
  if (ctx->rb_dev) {
    FetchArgs a{};
    a.n = n;
    for (int i = 0; i < n; ++i) {
      a.src[i] = (const uint32_t *)items[i].src;
      a.words[i] = (int32_t)(items[i].bytes / 4);
      a.off[i] = (int32_t)(off[i] / 4);
    }
    if (n > 0) {
      hipLaunchKernelGGL(k_fetch, dim3(1), dim3(RN_BLOCK), 0, ctx->stream, a, (uint32_t *)ctx->rb_dev);
      LAUNCH_CHECK(ctx);
    }
  } else {
    for (int i = 0; i < n; ++i)
      if (items[i].bytes)
        HIP_TRY(ctx, hipMemcpyAsync(ctx->rb_host + off[i], items[i].src, items[i].bytes, hipMemcpyDeviceToHost,
                                    ctx->stream));
  }
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  *host = ctx->rb_host;
  return RN_OK;
}

rn_status rn_read_i64(rn_ctx *ctx, const void *dev, int64_t *out) {
  const RnFetch it[1] = {{dev, sizeof(int64_t)}};
  const unsigned char *h = nullptr;
  size_t off[1];
  RN_TRY(rn_fetch(ctx, 1, it, &h, off));
  memcpy(out, h + off[0], sizeof(int64_t));
  return RN_OK;
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 counts: per-block totals, one-block scan of the
// totals (int64, sequential over chunks of 1024), then the add-back pass.
// ---------------------------------------------------------------------------
#define SCAN_ITEMS 4
#define SCAN_TILE (RN_BLOCK * SCAN_ITEMS)

__global__ __launch_bounds__(RN_BLOCK) void k_scan_tiles(const int32_t *__restrict__ cnt, int64_t n,
                                                        int64_t *__restrict__ bsum) {
  __shared__ int64_t lds[RN_BLOCK];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t s = 0;
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; ++q)
    if (base + q < n) s += cnt[base + q];
  lds[threadIdx.x] = s;
  __syncthreads();
  for (int w = RN_BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = lds[0];
}

__global__ __launch_bounds__(1024) void k_scan_bsum(int64_t *__restrict__ bsum, int64_t nb,
                                                   int64_t *__restrict__ total) {
  __shared__ int64_t lds[1024];
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
    const int64_t i = c0 + threadIdx.x;
    const int64_t v = i < nb ? bsum[i] : 0;
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // Hillis-Steele inclusive
      int64_t t = threadIdx.x >= (unsigned)off ? lds[threadIdx.x - off] : 0;
      __syncthreads();
      lds[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nb) bsum[i] = carry + lds[threadIdx.x] - v;  // exclusive prefix
    carry += lds[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(RN_BLOCK) void k_scan_apply(const int32_t *__restrict__ cnt, int64_t n,
                                                        const int64_t *__restrict__ bpre,
                                                        const int64_t *__restrict__ total,
                                                        int32_t *__restrict__ out) {
  __shared__ int64_t lds[RN_BLOCK];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS];
  int64_t s = 0;
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; ++q) {
    v[q] = base + q < n ? cnt[base + q] : 0;
    s += v[q];
  }
  lds[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < RN_BLOCK; off <<= 1) {
    int64_t t = threadIdx.x >= (unsigned)off ? lds[threadIdx.x - off] : 0;
    __syncthreads();
    lds[threadIdx.x] += t;
    __syncthreads();
  }
  int64_t run = bpre[blockIdx.x] + lds[threadIdx.x] - s;
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; ++q) {
    if (base + q < n) out[base + q] = (int32_t)run;
    run += v[q];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = (int32_t)*total;
}

// Tile scan with the prefix of the preceding tiles summed by each block
// itself (for up to SCAN_FUSED_TILES tiles: two launches instead of three);
// the last block writes the total.
#define SCAN_FUSED_TILES 4096
__global__ __launch_bounds__(RN_BLOCK) void k_scan_apply_pre(const int32_t *__restrict__ cnt, int64_t n,
                                                            const int64_t *__restrict__ bsum,
                                                            int64_t *__restrict__ total,
                                                            int32_t *__restrict__ out) {
  __shared__ int64_t lds[RN_BLOCK];
  __shared__ int64_t s_pre;
  int64_t p = 0;
  for (int64_t q = threadIdx.x; q < blockIdx.x; q += RN_BLOCK) p += bsum[q];
  lds[threadIdx.x] = p;
  __syncthreads();
  for (int w = RN_BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) s_pre = lds[0];
  __syncthreads();
  const int64_t pre = s_pre;
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS];
  int64_t s = 0;
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; ++q) {
    v[q] = base + q < n ? cnt[base + q] : 0;
    s += v[q];
  }
  lds[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < RN_BLOCK; off <<= 1) {
    int64_t t = threadIdx.x >= (unsigned)off ? lds[threadIdx.x - off] : 0;
    __syncthreads();
    lds[threadIdx.x] += t;
    __syncthreads();
  }
  int64_t run = pre + lds[threadIdx.x] - s;
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; ++q) {
    if (base + q < n) out[base + q] = (int32_t)run;
    run += v[q];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == RN_BLOCK - 1) {
    *total = run;
    out[n] = (int32_t)run;
  }
}

rn_status rn_scan_counts(rn_ctx *ctx, const int32_t *counts, int32_t *out, int64_t n,
                         int64_t *total_host) {
  rn_status st = RN_OK;
  const int64_t nb = n > 0 ? (n + SCAN_TILE - 1) / SCAN_TILE : 1;
  int64_t *bsum = (int64_t *)rn_scratch(ctx, SLOT_SCAN_BSUM, (size_t)nb * sizeof(int64_t), &st);
  if (!bsum) return st;
  int64_t *total = (int64_t *)rn_scratch(ctx, SLOT_SCAN_TOTAL, sizeof(int64_t), &st);
  if (!total) return st;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nb), dim3(RN_BLOCK), 0, ctx->stream, counts, n, bsum);
  LAUNCH_CHECK(ctx);
  if (nb <= SCAN_FUSED_TILES) {
    hipLaunchKernelGGL(k_scan_apply_pre, dim3((unsigned)nb), dim3(RN_BLOCK), 0, ctx->stream, counts, n, bsum,
                       total, out);
  } else {
    hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(1024), 0, ctx->stream, bsum, nb, total);
    LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(RN_BLOCK), 0, ctx->stream, counts, n, bsum,
                       total, out);
  }
  LAUNCH_CHECK(ctx);
  if (total_host) {
    RN_TRY(rn_read_i64(ctx, total, total_host));
    if (*total_host >= ((int64_t)1 << 31))
      return rn_fail(ctx, RN_ELIMIT, "count %lld reaches 2^31", (long long)*total_host);
  }
  return RN_OK;
}

// ---------------------------------------------------------------------------
// CSR transpose: count columns, scan, scatter with atomics, then sort each
// row of the transpose by its (unique) column so the result is canonical.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RN_BLOCK) void k_tr_count(const int32_t *__restrict__ Aj, int64_t nnz,
                                                      int32_t *__restrict__ cnt, const int32_t *__restrict__ guard) {
  if (*guard) return;
  for (int64_t p = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * RN_BLOCK)
    atomicAdd(&cnt[Aj[p]], 1);
}

__global__ __launch_bounds__(RN_BLOCK) void k_tr_scatter(int32_t rows, const int32_t *__restrict__ Ap,
                                                        const int32_t *__restrict__ Aj,
                                                        int32_t *__restrict__ cursor,
                                                        int32_t *__restrict__ trow,
                                                        int32_t *__restrict__ tperm,
                                                        const int32_t *__restrict__ guard) {
  const int i = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (i >= rows || *guard) return;
  for (int p = Ap[i]; p < Ap[i + 1]; ++p) {
    const int q = atomicAdd(&cursor[Aj[p]], 1);
    trow[q] = i;
    tperm[q] = p;
  }
}

__global__ __launch_bounds__(RN_BLOCK) void k_tr_sort(int32_t cols, const int32_t *__restrict__ Tp,
                                                     const int32_t *__restrict__ trow,
                                                     const int32_t *__restrict__ tperm,
                                                     int32_t *__restrict__ Tj, int32_t *__restrict__ perm,
                                                     const int32_t *__restrict__ guard) {
  const int j = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (j >= cols || *guard) return;
  const int s = Tp[j], e = Tp[j + 1];
  for (int q = s; q < e; ++q) {
    const int key = trow[q];
    int rank = 0;
    for (int u = s; u < e; ++u) rank += trow[u] < key;
    Tj[s + rank] = key;
    if (perm) perm[s + rank] = tperm[q];
  }
}

rn_status rn_transpose_structure(rn_ctx *ctx, int32_t rows, int32_t cols, int64_t nnz,
                                 const int32_t *Ap, const int32_t *Aj, int32_t *Tp, int32_t *Tj,
                                 int32_t *perm, const int32_t *guard) {
  rn_status st = RN_OK;
  int32_t *cnt = (int32_t *)rn_scratch(ctx, SLOT_TR_CNT, (size_t)(cols + 1) * sizeof(int32_t), &st);
  if (!cnt) return st;
  int32_t *trow = (int32_t *)rn_scratch(ctx, SLOT_TR_ROW, (size_t)(nnz + 1) * sizeof(int32_t), &st);
  if (!trow) return st;
  int32_t *tperm = (int32_t *)rn_scratch(ctx, SLOT_TR_PERM, (size_t)(nnz + 1) * sizeof(int32_t), &st);
  if (!tperm) return st;
  HIP_TRY(ctx, hipMemsetAsync(cnt, 0, (size_t)(cols + 1) * sizeof(int32_t), ctx->stream));
  unsigned g = rn_div_up(nnz, RN_BLOCK);
  if (g > 4096) g = 4096;
  if (g == 0) g = 1;
  hipLaunchKernelGGL(k_tr_count, dim3(g), dim3(RN_BLOCK), 0, ctx->stream, Aj, nnz, cnt, guard);
  LAUNCH_CHECK(ctx);
  RN_TRY(rn_scan_counts(ctx, cnt, Tp, cols, nullptr));
  HIP_TRY(ctx, hipMemcpyAsync(cnt, Tp, (size_t)cols * sizeof(int32_t), hipMemcpyDeviceToDevice, ctx->stream));
  if (rows > 0) {
    hipLaunchKernelGGL(k_tr_scatter, dim3(rn_div_up(rows, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, rows,
                       Ap, Aj, cnt, trow, tperm, guard);
    LAUNCH_CHECK(ctx);
  }
  if (cols > 0) {
    hipLaunchKernelGGL(k_tr_sort, dim3(rn_div_up(cols, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, cols, Tp,
                       trow, tperm, Tj, perm, guard);
    LAUNCH_CHECK(ctx);
  }
  return RN_OK;
}

// ---------------------------------------------------------------------------
// public: context
// ---------------------------------------------------------------------------
// The scratch array of the allocation-free entry point (rn_energy_min_noalloc).
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address on each GPU comes from hipGetSymbolAddress, looked up once
// per device (the first rn_create with that device current) and kept below.
static __device__ __align__(256) unsigned char scratch[RN_NOALLOC_SCRATCH_BYTES];

#define RN_MAX_DEVICES 64
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[RN_MAX_DEVICES];
static bool g_scratch_tried[RN_MAX_DEVICES];

static void *noalloc_scratch_lookup(int device) {
  if (device < 0 || device >= RN_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_tried[device]) {
    g_scratch_tried[device] = true;
    void *ptr = nullptr;
    if (hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)) == hipSuccess) {
      g_scratch_ptr[device] = ptr;
    } else {
      (void)hipGetLastError();
      g_scratch_ptr[device] = nullptr;
    }
  }
  return g_scratch_ptr[device];
}

extern "C" rn_status rn_create(rn_ctx **out, void *stream) {
  if (!out) return RN_EINVAL;
  *out = nullptr;
  rn_ctx *ctx = new (std::nothrow) rn_ctx();
  if (!ctx) return RN_ENOMEM;
  ctx->stream = (hipStream_t)stream;
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    return RN_EHIP;
  }
  // set-up for the allocation-free entry point: this device's scratch array
  // and a read-back area large enough that it never has to grow there (a
  // failure here only disables that entry point)
  ctx->noalloc_scratch = noalloc_scratch_lookup(ctx->device);
  if (readback_reserve(ctx, RN_READBACK_RESERVE) != RN_OK) ctx->err.clear();
  *out = ctx;
  return RN_OK;
}

extern "C" void rn_destroy(rn_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  // plans and tapes still alive give their device memory back now
  for (rn_plan *pl : ctx->plans) rn_plan_release(pl);
  ctx->plans.clear();
  for (rn_tape *t : ctx->tapes) rn_tape_release(t);
  ctx->tapes.clear();
  cache_release(ctx, 0);
  for (int s = 0; s < SLOT_COUNT; ++s)
    if (ctx->slot[s].ptr) {
      if (ctx->free_fn) ctx->free_fn(ctx->slot[s].ptr, ctx->alloc_user);
      else (void)hipFree(ctx->slot[s].ptr);
    }
  if (ctx->rb_host) (void)hipHostFree(ctx->rb_host);
  delete ctx;
}

extern "C" rn_status rn_set_allocator(rn_ctx *ctx, void *(*alloc)(size_t bytes, void *user),
                                      void (*release)(void *ptr, void *user), void *user) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if ((alloc == nullptr) != (release == nullptr))
    return rn_fail(ctx, RN_EINVAL, "rn_set_allocator: give both functions or neither");
  bool holds = !ctx->live.empty() || !ctx->cache.empty();
  for (int s = 0; s < SLOT_COUNT; ++s) holds = holds || ctx->slot[s].ptr != nullptr;
  if (holds)
    return rn_fail(ctx, RN_EINVAL, "rn_set_allocator: the context already holds device memory (set the allocator "
                                   "before the first call that allocates)");
  ctx->alloc_fn = alloc;
  ctx->free_fn = release;
  ctx->alloc_user = user;
  return RN_OK;
}

extern "C" rn_status rn_set_option(rn_ctx *ctx, rn_option opt, int32_t value) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  switch (opt) {
    case RN_OPT_PERSISTENT_PRODUCT:
    case RN_OPT_PADDED_PATTERN:
    case RN_OPT_FUSED_SETUP:
    case RN_OPT_METRICS:
    case RN_OPT_FUSED_CG:
      if (value != 0 && value != 1) return rn_fail(ctx, RN_EINVAL, "rn_set_option: value must be 0 or 1");
      break;
    case RN_OPT_PRODUCT_LANES:
      if (value != 64 && value != 128 && value != 256)
        return rn_fail(ctx, RN_EINVAL, "rn_set_option: product lanes must be 64, 128 or 256");
      break;
    case RN_OPT_TAPE_INTERVAL:
      if (value < 0) return rn_fail(ctx, RN_EINVAL, "rn_set_option: the tape interval must be >= 0");
      break;
    default:
      return rn_fail(ctx, RN_EINVAL, "rn_set_option: unknown option %d", (int)opt);
  }
  ctx->opt[opt] = value;
  return RN_OK;
}

extern "C" rn_status rn_set_stream(rn_ctx *ctx, void *stream) {
  if (!ctx) return RN_EINVAL;
  // cached blocks and scratch may still be read by work on the old stream
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  ctx->stream = (hipStream_t)stream;
  return RN_OK;
}

extern "C" const char *rn_last_error(const rn_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" const char *rn_version(void) { return "rnamg 0.1 gfx950"; }

extern "C" rn_status rn_transpose(rn_ctx *ctx, const rn_matrix *A, int32_t *ATp, int32_t *ATj, double *ATx,
                                  int32_t *perm) {
  if (!ctx || !A) return RN_EINVAL;
  ctx->err.clear();
  if (A->block_m != 1) return rn_fail(ctx, RN_EINVAL, "rn_transpose: scalar CSR only (block_m = 1)");
  if (A->n < 0 || A->nnz < 0 || !A->rowptr || (A->nnz && !A->colind) || !ATp || (A->nnz && !ATj))
    return rn_fail(ctx, RN_EINVAL, "rn_transpose: null or negative argument");
  if (A->nnz >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_transpose: nnz >= 2^31");
  if (ATx && !A->vals) return rn_fail(ctx, RN_EINVAL, "rn_transpose: AT_vals requested but A->vals is NULL");
  rn_status st = RN_OK;
  int32_t *pm = perm;
  if (!pm && ATx) {
    pm = (int32_t *)rn_scratch(ctx, SLOT_MISC, (size_t)(A->nnz + 1) * sizeof(int32_t), &st);
    if (!pm) return st;
  }
  int32_t *guard = rn_guard_begin(ctx, &st);
  if (!guard) return st;
  RN_TRY(rn_validate_csr(ctx, A->n, A->n, A->nnz, A->rowptr, A->colind, guard, GUARD_A));
  RN_TRY(rn_transpose_structure(ctx, A->n, A->n, A->nnz, A->rowptr, A->colind, ATp, ATj, pm, guard));
  if (ATx) RN_TRY(rn_gather_values(ctx, A->vals, pm, A->nnz, ATx));
  return rn_check_guard(ctx, guard, "rn_transpose");
}

__global__ __launch_bounds__(RN_BLOCK) void k_gather(const double *__restrict__ src,
                                                    const int32_t *__restrict__ idx, int64_t n,
                                                    double *__restrict__ dst) {
  for (int64_t q = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; q < n; q += (int64_t)gridDim.x * RN_BLOCK)
    dst[q] = src[idx[q]];
}

rn_status rn_gather_values(rn_ctx *ctx, const double *src, const int32_t *idx, int64_t n, double *dst) {
  if (n == 0) return RN_OK;
  unsigned g = rn_div_up(n, RN_BLOCK);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_gather, dim3(g), dim3(RN_BLOCK), 0, ctx->stream, src, idx, n, dst);
  LAUNCH_CHECK(ctx);
  return RN_OK;
}

// ---------------------------------------------------------------------------
// input validation
// ---------------------------------------------------------------------------
int32_t *rn_guard_begin(rn_ctx *ctx, rn_status *st) {
  int32_t *g = (int32_t *)rn_scratch(ctx, SLOT_GUARD, 64, st);
  if (!g) return nullptr;
  // the whole slot: the guard word and the stage flags beside it
  if (hipMemsetAsync(g, 0, 64, ctx->stream) != hipSuccess) {
    *st = rn_fail(ctx, RN_EHIP, "guard reset failed");
    return nullptr;
  }
  return g;
}

__global__ __launch_bounds__(RN_BLOCK) void k_validate_csr(int32_t rows, int32_t cols, int64_t nnz,
                                                          const int32_t *__restrict__ Ap,
                                                          const int32_t *__restrict__ Aj,
                                                          int32_t *__restrict__ guard, int32_t bit) {
  const int i = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (i > rows) return;
  if (nnz < 0) nnz = Ap[rows];  // structure sized by its own last row pointer
  const int64_t s = Ap[i];
  bool bad = (i == 0 && s != 0) || (i == rows && s != nnz) || s < 0 || s > nnz;
  if (!bad && i < rows) {
    const int64_t e = Ap[i + 1];
    if (e < s || e > nnz) {
      bad = true;
    } else {
      int prev = -1;
      for (int64_t p = s; p < e; ++p) {
        const int j = Aj[p];
        if (j <= prev || j >= cols) { bad = true; break; }
        prev = j;
      }
    }
  }
  if (bad) atomicOr(guard, bit);
}

__global__ __launch_bounds__(RN_BLOCK) void k_validate_range(int64_t n, const int32_t *__restrict__ a, int32_t lo,
                                                            int32_t hi, int32_t *__restrict__ guard, int32_t bit) {
  bool bad = false;
  for (int64_t q = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; q < n; q += (int64_t)gridDim.x * RN_BLOCK)
    bad |= (a[q] < lo || a[q] >= hi);
  if (bad) atomicOr(guard, bit);
}

rn_status rn_validate_csr(rn_ctx *ctx, int32_t rows, int32_t cols, int64_t nnz, const int32_t *Ap,
                          const int32_t *Aj, int32_t *guard, int32_t bit) {
  hipLaunchKernelGGL(k_validate_csr, dim3(rn_div_up((int64_t)rows + 1, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream,
                     rows, cols, nnz, Ap, Aj, guard, bit);
  LAUNCH_CHECK(ctx);
  return RN_OK;
}

rn_status rn_validate_range(rn_ctx *ctx, int64_t n, const int32_t *a, int32_t lo, int32_t hi, int32_t *guard,
                            int32_t bit) {
  if (n <= 0) return RN_OK;
  unsigned g = rn_div_up(n, RN_BLOCK);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_validate_range, dim3(g), dim3(RN_BLOCK), 0, ctx->stream, n, a, lo, hi, guard, bit);
  LAUNCH_CHECK(ctx);
  return RN_OK;
}

// Several checks in one launch: thread i takes row i of each CSR structure
// and element i of each index array.
__global__ __launch_bounds__(RN_BLOCK) void k_validate_all(const RnChecks v, int32_t *__restrict__ guard) {
  const int64_t i = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x;
  int32_t bad = 0;
  for (int q = 0; q < v.ncsr; ++q) {
    const RnCsrCheck &c = v.csr[q];
    if (i > c.rows) continue;
    const int64_t nnz = c.nnz < 0 ? c.Ap[c.rows] : c.nnz;
    const int64_t s = c.Ap[i];
    bool b = (i == 0 && s != 0) || (i == c.rows && s != nnz) || s < 0 || s > nnz;
    if (!b && i < c.rows) {
      const int64_t e = c.Ap[i + 1];
      if (e < s || e > nnz) {
        b = true;
      } else {
        int prev = -1;
        for (int64_t p = s; p < e; ++p) {
          const int j = c.Aj[p];
          if (j <= prev || j >= c.cols) { b = true; break; }
          prev = j;
        }
      }
    }
    if (b) bad |= c.bit;
  }
  for (int q = 0; q < v.nrange; ++q) {
    const RnRangeCheck &r = v.range[q];
    if (i < r.n && (r.a[i] < r.lo || r.a[i] >= r.hi)) bad |= r.bit;
  }
  if (bad) atomicOr(guard, bad);
}

rn_status rn_validate(rn_ctx *ctx, const RnChecks &v, int32_t *guard) {
  int64_t m = 0;
  for (int q = 0; q < v.ncsr; ++q) m = v.csr[q].rows + 1 > m ? v.csr[q].rows + 1 : m;
  for (int q = 0; q < v.nrange; ++q) m = v.range[q].n > m ? v.range[q].n : m;
  if (m <= 0) return RN_OK;
  if (m >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_validate: %lld elements", (long long)m);
  hipLaunchKernelGGL(k_validate_all, dim3(rn_div_up(m, RN_BLOCK)), dim3(RN_BLOCK), 0, ctx->stream, v, guard);
  LAUNCH_CHECK(ctx);
  return RN_OK;
}

static rn_status guard_message(rn_ctx *ctx, int32_t g, const char *what) {
  if (!g) return RN_OK;
  if (g & GUARD_LIMIT) return rn_fail(ctx, RN_ELIMIT, "%s: a documented size limit was exceeded", what);
  return rn_fail(ctx, RN_EINVAL, "%s: malformed input (%s%s%s%s%s)", what, (g & GUARD_A) ? "A " : "",
                 (g & GUARD_S) ? "S " : "", (g & GUARD_N) ? "N " : "", (g & GUARD_AGG) ? "agg " : "",
                 (g & GUARD_ROOTS) ? "roots" : "");
}

rn_status rn_guard_status(rn_ctx *ctx, int32_t g, const char *what) { return guard_message(ctx, g, what); }

rn_status rn_check_guard(rn_ctx *ctx, const int32_t *guard, const char *what) {
  const RnFetch it[1] = {{guard, sizeof(int32_t)}};
  const unsigned char *h = nullptr;
  size_t off[1];
  RN_TRY(rn_fetch(ctx, 1, it, &h, off));
  int32_t g;
  memcpy(&g, h + off[0], sizeof(g));
  return guard_message(ctx, g, what);
}

rn_status rn_read_guard_i64(rn_ctx *ctx, const int32_t *guard, const void *dev, int64_t *out, const char *what) {
  const RnFetch it[2] = {{dev, sizeof(int64_t)}, {guard, sizeof(int32_t)}};
  const unsigned char *h = nullptr;
  size_t off[2];
  RN_TRY(rn_fetch(ctx, 2, it, &h, off));
  memcpy(out, h + off[0], sizeof(int64_t));
  int32_t g;
  memcpy(&g, h + off[1], sizeof(g));
  return guard_message(ctx, g, what);
}
