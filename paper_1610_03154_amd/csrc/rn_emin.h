// rn_emin.h -- plan object and kernel parameter blocks of the energy
// minimisation (Sec. 3.6 improve).  Internal.
#pragma once
#include "rn_gram.h"
#include "rn_internal.h"

// Position codes: for pattern entry r of row i and the t-th stored entry
// A(i,k), the position of column j_r in row k of the pattern (0..252), or
// CODE_ROOT (k is a root node, block_m = 2: its two DOF rows hold one entry
// each), or CODE_NONE.  Layout: one record per (node) entry with one stride
// for every entry (the longest A row of a non-root row plus one byte, rounded
// up to 4 bytes): the entry's row within its product block in byte 0, then
// the codes, then CODE_NONE padding.  A lane finds its record from its entry
// index alone and reads it as 32-bit words.
#define CODE_NONE 255
#define CODE_ROOT 254
#define CODE_MAXLEN 253
// Compact record (block_m = 1, at most 11 A entries per row, rows of N of at
// most 31 entries): one 64-bit word, the row in bits 0-7 and code u in bits
// 8 + 5u .. 12 + 5u, CCODE_NONE where there is none.  The persistent product
// reads these; the 12-byte records stay for the other kernels.
#define CCODE_NONE 31u
#define CCODE_MAXLEN 31
#define CCODE_MAXNA 11

// Block-row A entries staged in LDS by the product kernel (larger blocks read
// A from global memory directly).
#define SPG_ACAP 1024
// Scalar operators: A entries staged per block of bs lanes, and the capacity
// (elements) of the block's X window.  The window holds the pattern entries
// of every neighbour row the block's rows touch, as runs of consecutive rows
// padded to XW_UNIT elements, so the product reads X from LDS after loading
// it with contiguous 32-bit loads.  Per block the plan stores, for each
// XW_UNIT-element unit of the window, the global index of its first element.
#define SPG_ACAP_M1(bs) (3 * (bs))
#define SPG_XCAP_M1(bs) (4 * (bs))
#define XW_UNIT 32
#define XW_GAP 16     // runs closer than this many elements are merged
#define XW_RUNMAX 15  // more runs: the block reads X from global memory

// per-batch integer state
// per batch entry: status, converged flag, steps done, GMRES basis size
// (ST_PREC: the Jacobi preconditioner met a diagonal entry that is not positive)
enum { ST_STATUS = 0, ST_DONE = 1, ST_ITERS = 2, ST_KD = 3, ST_PREC = 4, ST_STRIDE = 8 };

// per-batch double scalars
enum { SC_GAMMA0 = 0, SC_BETA0, SC_BASE = 4 };
// CG: gamma[K+1], delta[K], alpha[K], beta[K] after SC_BASE
struct CgLayout {
  int gam, del, alp, bet, total;
  __host__ __device__ CgLayout(int K) {
    gam = SC_BASE;
    del = gam + K + 1;
    alp = del + K;
    bet = alp + K;
    total = bet + K;
  }
};
// GMRES: scales, Hessenberg, Givens, residual vector, y, two GS passes
struct GmLayout {
  int s, H, cs, sn, g, y, h1, h2, total;
  __host__ __device__ GmLayout(int K) {
    s = SC_BASE;
    H = s + (K + 1);
    cs = H + (K + 1) * K;
    sn = cs + K;
    g = sn + K;
    y = g + (K + 1);
    h1 = y + K;
    h2 = h1 + (K + 1);
    total = h2 + (K + 1);
  }
};

// MODE_CG_FSTEP: CG step k >= 1 that first finishes beta_{k-1} from the
// <R,R> partials of the previous update and forms D_k = R + beta_{k-1}
// D_{k-1} (X = D_{k-1}, Rres = R, Dnew = D_k) as it stages X
enum { MODE_PRODUCT = 0, MODE_CG_INIT, MODE_CG_STEP, MODE_GM_INIT, MODE_GM_STEP, MODE_CG_FSTEP };

#define RN_MAXDOT 65  // GMRES iterations <= 64

enum RnWs {
  WS_R = 0, WS_D, WS_Z, WS_D32, WS_A32, WS_T32, WS_U, WS_U32, WS_PART, WS_SCAL, WS_ST, WS_CNT,
  WS_TAPE_TMP0, WS_TAPE_TMP1, WS_TAPE_TMP2, WS_TAPE_TMP3, WS_Y, WS_DIAG, WS_D2, WS_COUNT
};

struct rn_plan {
  rn_ctx *ctx = nullptr;
  int32_t n = 0, nc = 0, m = 1, nB = 1, nr = 0;
  int64_t nnzN = 0, nnzA = 0, nnzN_node = 0;
  const int32_t *Ap = nullptr, *Aj = nullptr, *Np = nullptr, *Nj = nullptr;
  const uint8_t *is_root = nullptr;
  const double *Bc = nullptr;
  uint8_t *codes = nullptr;     // [entries][cstride]
  uint64_t *ccodes = nullptr;   // [entries] compact records, or NULL
  int64_t ncodes = 0;
  int32_t cstride = 4;          // code bytes per (node) entry, multiple of 4
  int32_t *nodeptr = nullptr;   // block_m = 2: node-entry row pointer
  int32_t *ncol = nullptr;      // block_m = 2: node column of each node entry
  int32_t *blk_row = nullptr;   // product blocks: first row of block b, b = 0..nblk
  int32_t *blk_hdr = nullptr;   // per block: r0, r1, e0, e1, a0, a1, longest A row,
                                // X window units (0: no window) -- 8 ints
  int32_t *xoff = nullptr;      // per stored A entry: first pattern entry of the
                                // neighbour row (block_m = 2: of rows 2K, 2K+1)
  int32_t *xl = nullptr;        // block_m = 1, per stored A entry of a block with
                                // an X window: the neighbour row's offset in it
  int32_t *xwin = nullptr;      // block_m = 1, per block: bs/8 unit starts
  double *bce = nullptr;        // block_m = 1, n_B <= 2: Bc row of each entry's column
  bool unit_bc = false;         // block_m = 1 and every entry of Bc is 1
  double *gp = nullptr;         // packed Gram pseudo-inverse per DOF row
  int32_t rank_def = 0, maxlen = 0, chunk = 1, nblk = 0;
  int32_t bs = RN_BLOCK;        // lanes per product block (block_m = 1: 64, 128 or 256)
  bool persist = true;          // the persistent product may serve this plan
  bool gp_ext = false;          // gp is the caller's array (not freed with the plan)
  unsigned long long *d_terms = nullptr;  // multiply-add terms of one product
  size_t fixed_bytes = 0;
  RnScratch ws[WS_COUNT];
  // While set, workspace requests are carved from this caller-provided area
  // (the allocation-free scratch array) instead of the slots above.
  unsigned char *arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
};

void *rn_plan_ws(rn_plan *pl, int slot, size_t bytes, rn_status *st);

// Parameters of one masked-product launch (passed by value).
struct SpgParams {
  int32_t n, nr, nblk, k, K, hist_stride, project, scal_stride, cstride, bs;
  int32_t accum;  // MODE_PRODUCT: Z += result instead of Z = result
  int32_t kact;   // >= 0: batch entries whose st[ST_ITERS] <= kact do nothing
  int32_t unit_bc;  // every entry of Bc is 1: the projection's Bc rows are 1 (no per-entry loads)
  int32_t persist;  // the persistent product may serve the launch
  int32_t grid;     // > 0: the persistent launch's workgroups per batch entry (a multiple of 8)
  int64_t nnzN, strideA, strideX, strideZ;
  const int32_t *Ap, *Aj, *Np, *Nj, *nodeptr, *ncol, *blk_row, *blk_hdr, *xoff, *xl, *xwin;
  const uint8_t *codes, *is_root;
  const uint64_t *ccodes;  // compact records (the persistent product's condition)
  const double *Bc, *gp, *bce;
  const void *Ax;      // double or float, [batch][strideA]
  const void *X;       // double or float, [batch][strideX]
  const double *Xown;  // FP64 own-entry values for the CG dot (D)
  double *Z, *Z2;
  double *part;        // [batch][RN_MAXDOT][nblk]
  double *scal;        // [batch][scal_stride]
  int32_t *st;         // [batch][ST_STRIDE]
  // MODE_CG_FSTEP: the residual R_k, the direction written (D_k), the
  // update's <R,R> partials (np_rr per batch entry, pstride_rr apart) and
  // the history (nullable, hist_stride per batch entry)
  const double *Rres;
  double *Dnew;
  const double *part_rr;
  int32_t np_rr;
  int64_t pstride_rr;
  double *hist;
};

// Launch the masked product in one of the modes (rn_spgemm.hip).  Single-dot
// modes (CG_INIT, CG_STEP, GM_INIT) leave per-workgroup partials at the start
// of each batch entry's partial row; *npart (when given) receives their
// number (the grid of the persistent form, else one per product block).
rn_status rn_launch_spgemm(rn_ctx *ctx, const rn_plan *pl, int mode, const SpgParams &p, int batch, bool mixed,
                           int *npart = nullptr);
SpgParams rn_spg_params(const rn_plan *pl);
// Workgroups per batch entry of the persistent MODE_CG_FSTEP launch for this
// plan (FP64 or FP32-mixed), or 0 when it cannot run.  CG passes it as
// SpgParams::grid to every step product (MODE_CG_STEP too), so the
// <D, Pi(A D)> partials are grouped alike whichever path forms the direction.
int rn_spgemm_fused_grid(const rn_plan *pl, int batch, bool mixed = false);

// rn_plan_create on the caller's guard word (not reset; NULL: a fresh one),
// with one extra device item (nullable) read back at the plan's
// synchronisation into extra_out (host, extra->bytes).
// validate = false: A and N were checked (or made) by the caller.
// gp_in (nullable): every row's G^+ as Eq. Tproj formed it (packed, root
// rows zero, the same row group as the plan's own Gram kernel); the plan
// uses that array in place of computing its own (the caller keeps it alive
// for the plan's lifetime) and reports no rank-deficient rows itself.
rn_status rn_plan_create_ex(rn_ctx *ctx, const rn_matrix *A, int32_t n_cols, const int32_t *Np, const int32_t *Nj,
                            int64_t nnz_N, const uint8_t *is_root, const double *Bc, int32_t nB, rn_plan **out,
                            int32_t *guard_in, const RnFetch *extra, unsigned char *extra_out, bool validate,
                            const double *gp_in = nullptr);
// rn_tentative without its synchronisation: kernels queued on guard, the
// device flags (singular root block, rank-deficient rows) in *flags; then
// rn_tentative_flags on the flags as read back.
rn_status rn_tentative_launch(rn_ctx *ctx, int32_t n, int32_t m, const int32_t *Np, const int32_t *Nj,
                              int64_t nnz_N, const uint8_t *is_root, const int32_t *agg, const int32_t *roots,
                              int32_t n_agg, const double *B, int32_t nB, double *T, double *Bc, int32_t *guard,
                              const int32_t **flags, bool validate, double *gp_out);
rn_status rn_tentative_flags(rn_ctx *ctx, const int32_t hf[2], int32_t *rank_deficient);

// tape hooks called by rn_energy_min (CG, FP64) -- implemented with the adjoint
rn_status rn_tape_record_begin(rn_ctx *ctx, rn_plan *pl, rn_tape *tape, int32_t batch, int32_t iters,
                               rn_method method, rn_precision prec, const double *T);
// the tape's checkpoint slot of R_k and of D_k, each [batch][nnzN], when k
// is a checkpoint step (a multiple of the tape's interval below K), else
// NULL: the CG kernels write R_k and D_k there as they produce them
double *rn_tape_R(rn_tape *tape, int k);
double *rn_tape_D(rn_tape *tape, int k);
// after the last step: the per-batch scalars and status
rn_status rn_tape_record_end(rn_ctx *ctx, rn_tape *tape, const double *scal, const int32_t *st, int32_t batch);

// Deterministic sum of nb partials by a block of NT threads (fixed
// assignment of partials to threads, compensated, fixed tree).
template <int NT>
__device__ inline double rn_reduce_part_w(const double *part, int nb, double *lds8) {
  RnAcc a;
  // up to eight loads in flight per thread (predicated, so a short tail is
  // not loaded one round trip at a time), then the additions in index order
  for (int q = threadIdx.x; q < nb; q += 8 * NT) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = q + k * NT < nb ? part[q + k * NT] : 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (q + k * NT < nb) a.add(v[k]);
  }
  return rn_block_sum2_w<NT / RN_WAVE>(a.hi, a.lo, lds8);
}
__device__ inline double rn_reduce_part(const double *part, int nb, double *lds8) {
  return rn_reduce_part_w<RN_BLOCK>(part, nb, lds8);
}

// Krylov stopping rules (converged to round-off): CG once <R,R> <= 1e-24
// <R0,R0>, GMRES once the residual estimate is <= 1e-12 ||R0||.
#define RN_CG_STOP 1e-24
#define RN_GM_STOP 1e-12

// Scalar steps of one batch entry (one thread), from the step's reduced dot:
// gamma_0 = <R_0,R_0> (Sec. 4.1): stop at once when it is zero
__device__ inline void rn_cg_init_fin(double g, double *sc, int32_t *st, double *hist, int K) {
  const CgLayout L(K);
  sc[SC_GAMMA0] = g;
  sc[L.gam] = g;
  if (hist) hist[0] = g;
  if (!isfinite(g)) st[ST_STATUS] = RN_ENONFINITE;
  else if (g == 0.0) st[ST_DONE] = 1;
}
// delta_k = <D_k, Pi(A D_k)> and alpha_k = gamma_k / delta_k; breakdown when
// the curvature is not positive
// (gam = gamma_k, read by the caller together with its other loads)
__device__ inline void rn_cg_alpha_fin(double dl, double gam, double *sc, int32_t *st, double *hist, int K, int k) {
  const CgLayout L(K);
  sc[L.del + k] = dl;
  if (hist) hist[1 + K + k] = dl;
  if (!isfinite(dl)) {
    st[ST_STATUS] = RN_ENONFINITE;
    return;
  }
  if (dl <= 0.0) {
    st[ST_STATUS] = RN_EBREAKDOWN;
    return;
  }
  const double al = gam / dl;
  sc[L.alp + k] = al;
  if (hist) hist[1 + 2 * K + k] = al;
}
// gamma_{k+1} = <R_{k+1}, R_{k+1}>, beta_k = gamma_{k+1} / gamma_k, the step
// count and the stopping test
// (gam = gamma_k and gam0 = gamma_0, read by the caller with its other loads)
__device__ inline double rn_cg_beta_fin(double g, double gam, double gam0, double *sc, int32_t *st, double *hist,
                                        int K, int k) {
  const CgLayout L(K);
  const double be = g / gam;
  sc[L.gam + k + 1] = g;
  sc[L.bet + k] = be;
  if (hist) hist[k + 1] = g;
  st[ST_ITERS] = k + 1;
  if (!isfinite(g)) st[ST_STATUS] = RN_ENONFINITE;
  else if (g <= RN_CG_STOP * gam0) st[ST_DONE] = 1;
  return be;
}
// GMRES: beta_0 = ||R_0|| and the scale of the first basis vector
__device__ inline void rn_gm_init_fin(double tot, double *sc, int32_t *st, double *hist, int K) {
  const GmLayout L(K);
  const double beta = sqrt(tot);
  sc[SC_BETA0] = beta;
  sc[L.g] = beta;
  if (hist) hist[0] = beta;
  if (!isfinite(beta)) st[ST_STATUS] = RN_ENONFINITE;
  else if (beta == 0.0) st[ST_DONE] = 1;
  else sc[L.s] = 1.0 / beta;
}
