// rn_internal.h -- shared internals of librnamg (context, scratch, launch
// checks, deterministic block reductions).  gfx950 only: wave64.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <unordered_map>
#include <vector>

#include "rnamg.h"

#define RN_WAVE 64
#define RN_BLOCK 256

// ---------------------------------------------------------------------------
// scratch slots owned by a context (grow-only)
// ---------------------------------------------------------------------------
enum RnSlot {
  SLOT_SCAN_BSUM = 0,
  SLOT_SCAN_TOTAL,
  SLOT_STR_DIAG,
  SLOT_STR_MASK,
  SLOT_STR_TP,
  SLOT_STR_TJ,
  SLOT_STR_TPERM,
  SLOT_STR_TMASK,
  SLOT_STR_CNT,
  SLOT_STR_SJ,
  SLOT_TR_CNT,
  SLOT_TR_ROW,
  SLOT_TR_PERM,
  SLOT_PAT_XP0,
  SLOT_PAT_XJ0,
  SLOT_PAT_XP1,
  SLOT_PAT_XJ1,
  SLOT_PAT_CNT,
  SLOT_PAT_OVF,
  SLOT_TEN_BINV,
  SLOT_MISC,
  SLOT_GUARD,
  SLOT_BLK0,
  SLOT_BLK1,
  SLOT_BLK2,
  SLOT_FLT_KEEP,
  SLOT_FLT_CNT,
  SLOT_PRD_CNT,
  SLOT_PRD_CUR,
  SLOT_GAL_ASP,
  SLOT_GAL_ASJ,
  SLOT_GAL_ASV,
  SLOT_GAL_APP,
  SLOT_GAL_APJ,
  SLOT_GAL_APV,
  SLOT_GAL_RP,
  SLOT_GAL_RJ,
  SLOT_GAL_RV,
  SLOT_GAL_PERM,
  SLOT_NRM_TP,
  SLOT_NRM_TJ,
  SLOT_NRM_TV,
  SLOT_NRM_PERM,
  SLOT_NRM_WP,
  SLOT_NRM_WJ,
  SLOT_NRM_WV,
  SLOT_COUNT
};

struct RnScratch {
  void *ptr = nullptr;
  size_t cap = 0;
};

// One level of the pattern expansion: CSR (row pointers p) or padded (row J
// at J * stride, its length in c[J], or 1 when c is NULL).
struct XRows {
  const int32_t *p;
  const int32_t *v;
  const int32_t *c;
  int stride;
};

// Context options (rn_set_option), indexed by rn_option.
#define RN_OPT_COUNT 7

struct rn_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  int32_t opt[RN_OPT_COUNT] = {1, 1, 1, RN_BLOCK, 0, 1, 0};
  // device allocator of the caller (rn_set_allocator); NULL: hipMalloc/hipFree
  void *(*alloc_fn)(size_t, void *) = nullptr;
  void (*free_fn)(void *, void *) = nullptr;
  void *alloc_user = nullptr;
  // device address of this GPU's allocation-free scratch array (looked up by
  // rn_create; NULL when the lookup failed)
  void *noalloc_scratch = nullptr;
  // live tapes made on this context (rn_destroy releases their device memory)
  std::vector<rn_tape *> tapes;
  RnScratch slot[SLOT_COUNT];
  // read-back area (rn_fetch): host-coherent pinned memory the device writes
  // directly (rb_dev = its device address, NULL when it cannot be mapped)
  unsigned char *rb_host = nullptr;
  void *rb_dev = nullptr;
  size_t rb_cap = 0;
  // two-phase caches
  int64_t str_nnz = -1;
  int32_t str_nodes = -1;
  bool str_direct = false;     // phase 2 of the strength fills S from the kept-entry mask
  int64_t pat_nnz = -1;        // nnz of the DOF pattern
  int32_t pat_n = -1;          // rows of the DOF pattern
  XRows pat_x{};               // the final nodal level (read by phase 2)
  int32_t pat_m = 1;
  int32_t flt_n = -1;          // rn_filter: rows and input entries of phase 1, kept count
  int64_t flt_nnz_in = -1, flt_nnz = -1;
  int32_t prd_rows = -1;       // rn_spgemm: rows and nnz of phase 1
  int64_t prd_nnz = -1;
  int32_t gal_n = -1, gal_nc = -1;  // rn_galerkin: phase 1's sizes and intermediates (scratch)
  int64_t gal_nnz = -1;
  const int32_t *gal_R[2] = {nullptr, nullptr}, *gal_AP[2] = {nullptr, nullptr};
  const double *gal_Rv = nullptr, *gal_APv = nullptr;
  int32_t pv_nn = -1;          // rn_pattern_values: phase 1's last level (scratch)
  int64_t pv_nnz = -1;
  const int32_t *pv_j = nullptr;
  const double *pv_v = nullptr;
  // live plans made on this context: rn_destroy detaches them, so a plan
  // destroyed after its context frees its memory without touching the context
  std::vector<rn_plan *> plans;
  // caching device allocator (rn_dev_alloc / rn_dev_free)
  struct Block {
    void *p;
    size_t cap;
  };
  std::vector<Block> cache;                  // freed blocks, reusable
  std::unordered_map<void *, size_t> live;   // blocks handed out
  size_t cached_bytes = 0;
};

// Bytes of the pinned read-back area rn_create reserves (rn_fetch grows it
// on demand; the allocation-free entry point must fit in it).
#define RN_READBACK_RESERVE ((size_t)64 << 10)

// Error helpers -------------------------------------------------------------
rn_status rn_fail(rn_ctx *ctx, rn_status st, const char *fmt, ...);

#define RN_TRY(expr)                   \
  do {                                 \
    rn_status _s = (expr);             \
    if (_s != RN_OK) return _s;        \
  } while (0)

#define HIP_TRY(ctx, expr)                                                       \
  do {                                                                           \
    hipError_t _e = (expr);                                                      \
    if (_e != hipSuccess)                                                        \
      return rn_fail((ctx), RN_EHIP, "%s:%d %s: %s", __FILE__, __LINE__, #expr,  \
                     hipGetErrorString(_e));                                     \
  } while (0)

#define LAUNCH_CHECK(ctx) HIP_TRY(ctx, hipGetLastError())

// Device memory for objects made on a context (plans and their workspaces):
// freed blocks stay with the context and serve later requests of a similar
// size, so repeated set-ups do not call hipMalloc / hipFree.  Reuse is
// ordered by the context's stream (a block is handed out again only to work
// queued after the work that used it).  rn_dev_free with ctx = NULL frees
// the block outright.  rn_dev_alloc returns NULL when the device is full.
// With a caller's allocator (rn_set_allocator) blocks come from it and go
// straight back to it (it does its own caching).
void *rn_dev_alloc(rn_ctx *ctx, size_t bytes);
void rn_dev_free(rn_ctx *ctx, void *p);
// Device memory of a plan or tape goes back to its context when the context is
// destroyed first (the later destroy call then frees only the host object).
void rn_plan_release(rn_plan *pl);
void rn_tape_release(rn_tape *tape);

// Read-back of small device values at a synchronisation point: n <= 6 items
// (device address, size in bytes, both multiples of 4) copied by one kernel
// into the context's host read-back area, then the stream is synchronised.
// Item i lands at (*host) + off[i]; offsets are 8-byte aligned and in order.
// The area is valid until the next rn_fetch on the context.
#define RN_FETCH_MAX 6
struct RnFetch {
  const void *src;
  size_t bytes;
};
rn_status rn_fetch(rn_ctx *ctx, int n, const RnFetch *items, const unsigned char **host, size_t *off);

// rn_strength and phase 1 of rn_pattern with one synchronisation (rn_setup);
// Sj has room for nnz(A) + n/block_m entries.  *done false: run the stage
// calls instead (A not structurally symmetric, or a pattern row too long for
// the padded levels).
rn_status rn_strength_pattern(rn_ctx *ctx, const rn_matrix *A, double theta, int32_t *Sp, int32_t *Sj,
                              const int32_t *agg, const int32_t *roots, int32_t n_agg, int32_t degree, int32_t *Np,
                              uint8_t *is_root, int64_t *nnz_S, int64_t *nnz_N, bool *done);

// The error of a guard word read back from the device (RN_OK when 0).
rn_status rn_guard_status(rn_ctx *ctx, int32_t g, const char *what);

// Grow-only scratch; contents are not preserved on growth.
void *rn_scratch(rn_ctx *ctx, int slot, size_t bytes, rn_status *st);

// Device exclusive scan of n int32 counts into out[0..n] (out[n] = total).
// The total is also left in device memory at *total_dev (int64) and, when
// total_host != NULL, copied to the host (synchronising the stream).
// RN_ELIMIT when the total reaches 2^31.
rn_status rn_scan_counts(rn_ctx *ctx, const int32_t *counts, int32_t *out,
                         int64_t n, int64_t *total_host);

// Read one int64 from device memory (synchronises the stream).
rn_status rn_read_i64(rn_ctx *ctx, const void *dev, int64_t *out);

// Input guard of one public call.  Validation kernels set bits in a device
// int32; every kernel that indexes memory with caller data reads the guard
// first and does nothing when it is set, so malformed input cannot fault.
// The host reads the guard at the call's next synchronisation.
enum RnGuardBits { GUARD_A = 1, GUARD_S = 2, GUARD_N = 4, GUARD_AGG = 8, GUARD_ROOTS = 16, GUARD_LIMIT = 32 };
// rn_guard_begin zeroes 64 bytes: the guard word and, beside it, the stage
// flags (so they need no reset of their own): strength asymmetry, padded
// pattern overflow, the tentative's two flags, an entry of Bc other than 1.
enum RnGuardSlot { GS_ASYM = 1, GS_PFLAG = 2, GS_TFLAGS = 4, GS_BCNU = 8, GS_POW0 = 10 };
// the pattern expansion's wide-row counters of its first GS_NPOW powers sit in
// guard slots GS_POW0 .. GS_POW0 + GS_NPOW - 1 (zeroed with the guard)
#define GS_NPOW 6
int32_t *rn_guard_begin(rn_ctx *ctx, rn_status *st);
// rows x cols CSR: rowptr[0] = 0, non-decreasing, rowptr[rows] = nnz,
// columns in [0, cols) and strictly increasing within a row.
// Up to two CSR structures and two index arrays checked in one launch (the
// same tests as rn_validate_csr / rn_validate_range).
struct RnCsrCheck {
  int32_t rows, cols;
  int64_t nnz;  // < 0: the structure's own last row pointer
  const int32_t *Ap, *Aj;
  int32_t bit;
};
struct RnRangeCheck {
  int64_t n;
  const int32_t *a;
  int32_t lo, hi, bit;
};
struct RnChecks {
  RnCsrCheck csr[2];
  RnRangeCheck range[2];
  int ncsr, nrange;
};
rn_status rn_validate(rn_ctx *ctx, const RnChecks &v, int32_t *guard);
rn_status rn_validate_csr(rn_ctx *ctx, int32_t rows, int32_t cols, int64_t nnz, const int32_t *Ap,
                          const int32_t *Aj, int32_t *guard, int32_t bit);
// every a[q] in [lo, hi)
rn_status rn_validate_range(rn_ctx *ctx, int64_t n, const int32_t *a, int32_t lo, int32_t hi, int32_t *guard,
                            int32_t bit);
// Reads the guard (synchronises); RN_EINVAL naming the failed input.
rn_status rn_check_guard(rn_ctx *ctx, const int32_t *guard, const char *what);
// Reads the guard and one int64 with a single synchronisation.
rn_status rn_read_guard_i64(rn_ctx *ctx, const int32_t *guard, const void *dev, int64_t *out, const char *what);
rn_status rn_gather_values(rn_ctx *ctx, const double *src, const int32_t *idx, int64_t n, double *dst);

// General sparse product pieces (rn_product.hip).  rn_sg_pattern: the
// structure of C = X Y into two scratch slots (one synchronisation, guard
// read with it); rn_sg_values: C's values on a given pattern of C, each the
// sum over X's row in its order (asynchronous).  rn_scalar_view: the scalar
// CSR of A (block_m = 2: built into scratch).
rn_status rn_sg_pattern(rn_ctx *ctx, int32_t rows, int64_t nnzX, const int32_t *Xp, const int32_t *Xj,
                        const int32_t *Yp, const int32_t *Yj, int slot_p, int slot_j, int32_t **Cp, int32_t **Cj,
                        int64_t *nnz, int32_t *guard, const char *what);
rn_status rn_sg_values(rn_ctx *ctx, int32_t rows, int64_t nnzC, const int32_t *Xp, const int32_t *Xj,
                       const double *Xv, const int32_t *Yp, const int32_t *Yj, const double *Yv, const int32_t *Cp,
                       const int32_t *Cj, double *Cv, const int32_t *guard);
rn_status rn_scalar_view(rn_ctx *ctx, const rn_matrix *A, const int32_t **Sp, const int32_t **Sj, const double **Sv,
                         int32_t *guard);

// Internal transpose of a CSR structure with a permutation (used by the
// strength symmetrisation and by rn_transpose).  rows x cols -> cols x rows.
rn_status rn_transpose_structure(rn_ctx *ctx, int32_t rows, int32_t cols,
                                 int64_t nnz, const int32_t *Ap,
                                 const int32_t *Aj, int32_t *Tp, int32_t *Tj,
                                 int32_t *perm, const int32_t *guard);

static inline unsigned rn_div_up(int64_t a, int64_t b) {
  return (unsigned)((a + b - 1) / b);
}

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
// Error-free transformation a + b = s + e (Knuth's TwoSum).
__device__ inline void rn_two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Compensated running sum: hi carries the sum, lo the accumulated rounding.
struct RnAcc {
  double hi = 0.0, lo = 0.0;
  __device__ inline void add(double v) {
    double s, e;
    rn_two_sum(hi, v, s, e);
    hi = s;
    lo += e;
  }
};

// Deterministic compensated block sum (NW waves; blockDim.x == 64 NW <= 256):
// a fixed shuffle tree within each wave and a fixed-order combination of the waves, each
// addition done with TwoSum so the result is accurate to a few ulp whatever
// the number of terms.  lds8 holds 8 doubles.  Every thread gets the result.
template <int NW>
__device__ inline double rn_block_sum2_w(double hi, double lo, double *lds8) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double oh = __shfl_down(hi, off, RN_WAVE), ol = __shfl_down(lo, off, RN_WAVE);
    double s, e;
    rn_two_sum(hi, oh, s, e);
    hi = s;
    lo = lo + ol + e;
  }
  const int lane = threadIdx.x & (RN_WAVE - 1), wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    lds8[wid] = hi;
    lds8[4 + wid] = lo;
  }
  __syncthreads();
  double h = lds8[0], l = lds8[4];
#pragma unroll
  for (int w = 1; w < NW; ++w) {
    double s, e;
    rn_two_sum(h, lds8[w], s, e);
    h = s;
    l = l + lds8[4 + w] + e;
  }
  __syncthreads();
  return h + l;
}
__device__ inline double rn_block_sum2(double hi, double lo, double *lds8) { return rn_block_sum2_w<4>(hi, lo, lds8); }

// NJ compensated block sums at once, each with the arithmetic of
// rn_block_sum2_w (the same shuffle tree per wave, the waves combined in
// order), one barrier for all: thread j < nd writes total j to out[j * ostride].
// lds holds 2 * NJ * NW doubles.
template <int NW, int NJ>
__device__ inline void rn_block_sum2_multi(const double (&hi0)[NJ], const double (&lo0)[NJ], int nd, double *lds,
                                           double *out, int64_t ostride) {
  const int lane = threadIdx.x & (RN_WAVE - 1), wid = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    double hi = hi0[j], lo = lo0[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double oh = __shfl_down(hi, off, RN_WAVE), ol = __shfl_down(lo, off, RN_WAVE);
      double s, e;
      rn_two_sum(hi, oh, s, e);
      hi = s;
      lo = lo + ol + e;
    }
    if (lane == 0) {
      lds[(j * NW + wid) * 2] = hi;
      lds[(j * NW + wid) * 2 + 1] = lo;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nd && (int)threadIdx.x < NJ) {
    const int j = threadIdx.x;
    double h = lds[(j * NW) * 2], l = lds[(j * NW) * 2 + 1];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      double s, e;
      rn_two_sum(h, lds[(j * NW + w) * 2], s, e);
      h = s;
      l = l + lds[(j * NW + w) * 2 + 1] + e;
    }
    out[j * ostride] = h + l;
  }
}
__device__ inline double rn_block_sum(double v, double *lds8) { return rn_block_sum2(v, 0.0, lds8); }

// First index i in [0, n] with a[i] >= x (a non-decreasing, a[n] exists).
__device__ inline int rn_lower_bound(const int32_t *a, int n, int64_t x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if ((int64_t)a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// XCD-aware block order: hardware dispatches consecutive workgroups to the
// 8 XCDs round-robin; remap so each XCD walks one contiguous range of the
// logical blocks (keeps neighbouring rows in one L2).  Grid must be padded
// to a multiple of 8; returns -1 for padding blocks.
__device__ inline int rn_xcd_block(int hw, int nlogical) {
  const int per = (nlogical + 7) >> 3;
  const int lb = (hw & 7) * per + (hw >> 3);
  return lb < nlogical ? lb : -1;
}
static inline unsigned rn_xcd_grid(unsigned nlogical) {
  unsigned per = (nlogical + 7u) / 8u;
  return per * 8u;
}
