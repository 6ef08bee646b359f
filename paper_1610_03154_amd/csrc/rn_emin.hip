// rn_emin.hip -- energy minimisation of the interpolation operator
// (Sec. 3.6 improve; Sec. 4.1 CG form, Sec. 4.2 GMRES form).
//
// CG step k:   product (Z = Pi(A D), partials of <D,Z>)
//              -> alpha: one block per batch entry sums the <D,Z> partials
//              -> update: P += alpha D, R -= alpha Z, partials of <R,R>
//              -> direction: every block sums the <R,R> partials, beta,
//                 D = R + beta D.
// No inter-block synchronisation and no host round trip inside the loop; the
// scalars of step k are kept per step so no kernel overwrites a value another
// block of the same kernel still reads.
// GMRES step k: product W = A V_k, then three streaming passes (partials of
// <W, V_j>; classical Gram-Schmidt twice), each followed by a kernel that
// sums the partials; the Hessenberg column, Givens rotations and the
// stopping test run on the device.
// (Each finishing step is its own small kernel: a last-workgroup finish
// inside the producing kernel needs a device-scope release per workgroup,
// which writes back the compute die's L2 and made those kernels several
// times slower.)
#include <cmath>
#include <cstring>
#include <new>

#include <algorithm>

#include "rn_emin.h"

// ---------------------------------------------------------------------------
// CG
// ---------------------------------------------------------------------------
// (part: np partials per batch entry, batch entries pstride apart)
__global__ __launch_bounds__(RN_BLOCK) void k_cg_fin_init(int np, int64_t pstride, const double *__restrict__ part,
                                                         double *__restrict__ scal, int scal_stride, int K,
                                                         int32_t *__restrict__ stv, double *__restrict__ histv,
                                                         int hist_stride) {
  __shared__ double s_w[8];
  const int b = blockIdx.x;
  const double g = rn_reduce_part(part + (int64_t)b * pstride, np, s_w);
  if (threadIdx.x != 0) return;
  rn_cg_init_fin(g, scal + (int64_t)b * scal_stride, stv + (int64_t)b * ST_STRIDE,
                 histv ? histv + (int64_t)b * hist_stride : nullptr, K);
}

// Elements per lane whose loads the CG element-wise kernels issue together
// (one memory round trip for up to U * grid * RN_BLOCK elements); each lane
// still visits its elements in the order e, e + grid, e + 2 grid, ...  The
// update holds four vectors per element: five elements keep it at four
// workgroups per compute unit, so all 1024 of its workgroups are resident.
#define CG_UPD_U 5
#define CG_DIR_U 8

// delta_k = <D, Pi(A D)> from the product's per-workgroup partials: every
// block sums them in the same fixed order (compensated), so all blocks get
// the same delta_k and alpha_k; block 0 stores them with the breakdown and
// finiteness tests.  Then P += alpha D, R -= alpha Z and partials of <R,R>.
__global__ __launch_bounds__(RN_BLOCK) void k_cg_update(int64_t nnz, int64_t stride, int K, int k, int np,
                                                       int64_t pstride, const double *__restrict__ part_spg,
                                                       double *__restrict__ P, double *__restrict__ R,
                                                       const double *__restrict__ D, const double *__restrict__ Z,
                                                       double *__restrict__ part_ew, double *__restrict__ scal,
                                                       int scal_stride, int32_t *__restrict__ stv,
                                                       double *__restrict__ histv, int hist_stride,
                                                       double *__restrict__ Rrec) {
  __shared__ double s_w[8];
  const int b = blockIdx.y;
  int32_t *st = stv + (int64_t)b * ST_STRIDE;
  double *sc = scal + (int64_t)b * scal_stride;
  const int64_t off = (int64_t)b * stride, gs = (int64_t)gridDim.x * RN_BLOCK;
  const int64_t e0 = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x;
  double p[CG_UPD_U], d[CG_UPD_U], r[CG_UPD_U], z[CG_UPD_U];
  auto load = [&](int64_t base) {
#pragma unroll
    for (int u = 0; u < CG_UPD_U; ++u) {
      const int64_t e = base + u * gs;
      p[u] = d[u] = r[u] = z[u] = 0.0;
      if (e < nnz) {
        p[u] = P[off + e];
        d[u] = D[off + e];
        r[u] = R[off + e];
        z[u] = Z[off + e];
      }
    }
  };
  // the partials' loads go out first, then the first round of elements: the
  // partials are summed (and delta_k, alpha_k formed) while the element loads
  // are still in flight.  The additions are rn_reduce_part's, in its order.
  // A stopped entry's loads are made and not used.
  const double *pp = part_spg + (int64_t)b * pstride;
  constexpr int PQ = 8;
  double pv[PQ];
  const bool pfew = np <= PQ * RN_BLOCK;
#pragma unroll
  for (int q = 0; q < PQ; ++q) {
    const int i = threadIdx.x + q * RN_BLOCK;
    pv[q] = pfew && i < np ? pp[i] : 0.0;
  }
  load(e0);
  const int32_t s0 = st[ST_STATUS], s1 = st[ST_DONE];
  const double gam = sc[CgLayout(K).gam + k];
  double dl;
  if (pfew) {
    RnAcc a;
#pragma unroll
    for (int q = 0; q < PQ; ++q)
      if (threadIdx.x + q * RN_BLOCK < np) a.add(pv[q]);
    dl = rn_block_sum2(a.hi, a.lo, s_w);
  } else {
    dl = rn_reduce_part(pp, np, s_w);
  }
  if (s0 || s1) return;
  // (another block may read the status before or after block 0 sets a
  // breakdown here; either way it stops on the same delta_k)
  if (blockIdx.x == 0 && threadIdx.x == 0)
    rn_cg_alpha_fin(dl, gam, sc, st, histv ? histv + (int64_t)b * hist_stride : nullptr, K, k);
  if (!isfinite(dl) || dl <= 0.0) return;  // breakdown: nothing is updated
  const double al = gam / dl;
  RnAcc s;
  for (int64_t base = e0; base < nnz; base += CG_UPD_U * gs) {
    if (base != e0) load(base);
#pragma unroll
    for (int u = 0; u < CG_UPD_U; ++u) {
      const int64_t e = base + u * gs;
      if (e < nnz) {
        P[off + e] = p[u] + al * d[u];
        const double rr = r[u] - al * z[u];
        R[off + e] = rr;
        if (Rrec) Rrec[off + e] = rr;
        s.add(rr * rr);
      }
    }
  }
  const double S = rn_block_sum2(s.hi, s.lo, s_w);
  if (threadIdx.x == 0) part_ew[(int64_t)b * RN_MAXDOT * gridDim.x + blockIdx.x] = S;
}

// Every block sums the <R,R> partials (same fixed order, same scalars), block
// 0 stores gamma_{k+1}, beta_k and the stopping test; D = R + beta_k D (and
// its FP32 shadow).
template <bool MIXED>
__global__ __launch_bounds__(RN_BLOCK) void k_cg_dir(int64_t nnz, int64_t stride, int K, int k, int nb_ew,
                                                    const double *__restrict__ R, double *__restrict__ D,
                                                    float *__restrict__ D32, const double *__restrict__ part_ew,
                                                    double *__restrict__ scal, int scal_stride,
                                                    int32_t *__restrict__ stv, double *__restrict__ histv,
                                                    int hist_stride, double *__restrict__ Drec) {
  __shared__ double s_w[8];
  const int b = blockIdx.y;
  int32_t *st = stv + (int64_t)b * ST_STRIDE;
  double *sc = scal + (int64_t)b * scal_stride;
  const CgLayout L(K);
  const int64_t off = (int64_t)b * stride, gs = (int64_t)gridDim.x * RN_BLOCK;
  const int64_t e0 = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x;
  double r[CG_DIR_U], d[CG_DIR_U];
  auto load = [&](int64_t base) {
#pragma unroll
    for (int u = 0; u < CG_DIR_U; ++u) {
      const int64_t e = base + u * gs;
      r[u] = d[u] = 0.0;
      if (e < nnz) {
        r[u] = R[off + e];
        d[u] = D[off + e];
      }
    }
  };
  // status, gamma_k, gamma_0, the partials and the first round go out
  // together (one memory round trip)
  load(e0);
  const int32_t s0 = st[ST_STATUS], s1 = st[ST_DONE];
  const double gam = sc[L.gam + k], gam0 = sc[SC_GAMMA0];
  const double g = rn_reduce_part(part_ew + (int64_t)b * RN_MAXDOT * nb_ew, nb_ew, s_w);
  if (s0 || s1) return;
  const double be = g / gam;
  // (a block that reads the stop flag block 0 sets here skips its part of
  // D_{k+1}, which no later step reads once the iteration has stopped)
  if (blockIdx.x == 0 && threadIdx.x == 0)
    rn_cg_beta_fin(g, gam, gam0, sc, st, histv ? histv + (int64_t)b * hist_stride : nullptr, K, k);
  if (!isfinite(g)) return;
  for (int64_t base = e0; base < nnz; base += CG_DIR_U * gs) {
    if (base != e0) load(base);
#pragma unroll
    for (int u = 0; u < CG_DIR_U; ++u) {
      const int64_t e = base + u * gs;
      if (e < nnz) {
        const double dd = r[u] + be * d[u];
        D[off + e] = dd;
        if (Drec) Drec[off + e] = dd;
        if (MIXED) D32[off + e] = (float)dd;
      }
    }
  }
}

// After the last fused step: gamma_K, beta_{K-1}, the step count and the
// stopping test from the last update's <R,R> partials (one block per batch
// entry; the direction D_K is not formed)
__global__ __launch_bounds__(RN_BLOCK) void k_cg_last(int nb_ew, const double *__restrict__ part_ew, int K,
                                                     double *__restrict__ scal, int scal_stride,
                                                     int32_t *__restrict__ stv, double *__restrict__ histv,
                                                     int hist_stride) {
  __shared__ double s_w[8];
  const int b = blockIdx.x;
  int32_t *st = stv + (int64_t)b * ST_STRIDE;
  double *sc = scal + (int64_t)b * scal_stride;
  const CgLayout L(K);
  const int32_t s0 = st[ST_STATUS], s1 = st[ST_DONE];
  const double gam = sc[L.gam + K - 1], gam0 = sc[SC_GAMMA0];
  const double g = rn_reduce_part(part_ew + (int64_t)b * RN_MAXDOT * nb_ew, nb_ew, s_w);
  if (s0 || s1 || threadIdx.x != 0) return;
  rn_cg_beta_fin(g, gam, gam0, sc, st, histv ? histv + (int64_t)b * hist_stride : nullptr, K, K - 1);
}

// ---------------------------------------------------------------------------
// GMRES
// ---------------------------------------------------------------------------
// Sums partial rows and finishes the scalars of one stage (one block per
// batch entry).  STAGE 0: beta0 after the initial product; 1: first-pass
// coefficients h1_j = s_j <W, U_j>; 2: second-pass h2_j; 3: ||W||, column k
// of H, Givens rotation, residual estimate, next scale, stopping test.
template <int STAGE>
__global__ __launch_bounds__(RN_BLOCK) void k_gm_fin(int nb, int64_t pstride, const double *__restrict__ part, int K,
                                                    int k,
                                                    double *__restrict__ scal, int scal_stride,
                                                    int32_t *__restrict__ stv, double *__restrict__ histv,
                                                    int hist_stride) {
  __shared__ double s_w[8];
  // stages 1 and 2: one workgroup per coefficient j (blockIdx.x) and batch entry
  const int b = (STAGE == 1 || STAGE == 2) ? blockIdx.y : blockIdx.x;
  int32_t *st = stv + (int64_t)b * ST_STRIDE;
  if (STAGE > 0 && (st[ST_STATUS] || st[ST_DONE])) return;
  double *sc = scal + (int64_t)b * scal_stride;
  const GmLayout L(K);
  const double *pb = part + (int64_t)b * pstride;
  double *hist = histv ? histv + (int64_t)b * hist_stride : nullptr;
  if (STAGE == 1 || STAGE == 2) {
    const int j = blockIdx.x;
    const double tot = rn_reduce_part(pb + (int64_t)j * nb, nb, s_w);
    if (threadIdx.x == 0) sc[(STAGE == 1 ? L.h1 : L.h2) + j] = sc[L.s + j] * tot;
    return;
  }
  const double tot = rn_reduce_part(pb, nb, s_w);
  if (threadIdx.x != 0) return;
  if (STAGE == 0) {
    rn_gm_init_fin(tot, sc, st, hist, K);
    return;
  }
  double *H = sc + L.H;
  const double hn = sqrt(tot);
  for (int j = 0; j <= k; ++j) H[j * K + k] = sc[L.h1 + j] + sc[L.h2 + j];
  H[(k + 1) * K + k] = hn;
  if (!isfinite(hn)) {
    st[ST_STATUS] = RN_ENONFINITE;
    return;
  }
  for (int j = 0; j < k; ++j) {
    const double a = H[j * K + k], bb = H[(j + 1) * K + k];
    H[j * K + k] = sc[L.cs + j] * a + sc[L.sn + j] * bb;
    H[(j + 1) * K + k] = -sc[L.sn + j] * a + sc[L.cs + j] * bb;
  }
  const double a = H[k * K + k], bb = H[(k + 1) * K + k];
  const double r = hypot(a, bb);
  sc[L.cs + k] = a / r;
  sc[L.sn + k] = bb / r;
  H[k * K + k] = r;
  H[(k + 1) * K + k] = 0.0;
  sc[L.g + k + 1] = -sc[L.sn + k] * sc[L.g + k];
  sc[L.g + k] = sc[L.cs + k] * sc[L.g + k];
  if (hist) hist[k + 1] = fabs(sc[L.g + k + 1]);
  st[ST_KD] = k + 1;
  st[ST_ITERS] = k + 1;
  if (hn == 0.0 || fabs(sc[L.g + k + 1]) <= RN_GM_STOP * sc[SC_BETA0]) st[ST_DONE] = 1;
  else sc[L.s + k + 1] = 1.0 / hn;
}

// Gram-Schmidt passes on the new vector W = U_{k+1} (classical, twice):
// pass 0: partials of <W, U_j> (W untouched)
// pass 1: W -= sum_j h1_j V_j, partials of <W, U_j>
// pass 2: W -= sum_j h2_j V_j, partials of ||W||^2 (and the FP32 shadow)
template <int NJ, int PASS, bool MIXED>
__global__ __launch_bounds__(RN_BLOCK) void k_gm_orth(int64_t nnz, int64_t ubatch, int K, int k,
                                                     double *__restrict__ Uall, float *__restrict__ U32all,
                                                     double *__restrict__ part, const double *__restrict__ scal,
                                                     int scal_stride, const int32_t *__restrict__ stv) {
  __shared__ double s_w[8];
  const int b = blockIdx.y;
  const int32_t *st = stv + (int64_t)b * ST_STRIDE;
  if (st[ST_STATUS] || st[ST_DONE]) return;
  const double *sc = scal + (int64_t)b * scal_stride;
  const GmLayout L(K);
  double *U = Uall + (int64_t)b * ubatch;
  double *W = U + (int64_t)(k + 1) * nnz;
  double coef[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) coef[j] = (PASS > 0 && j <= k) ? sc[(PASS == 1 ? L.h1 : L.h2) + j] * sc[L.s + j] : 0.0;
  RnAcc acc[NJ];
  for (int64_t e = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * RN_BLOCK) {
    double w = W[e];
    if (PASS > 0) {
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        if (j <= k) w -= coef[j] * U[(int64_t)j * nnz + e];
      W[e] = w;
    }
    if (PASS <= 1) {
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        if (j <= k) acc[j].add(w * U[(int64_t)j * nnz + e]);
    } else {
      acc[0].add(w * w);
      if (MIXED) U32all[(int64_t)b * ubatch + (int64_t)(k + 1) * nnz + e] = (float)w;
    }
  }
  double *pb = part + (int64_t)b * RN_MAXDOT * gridDim.x;
  const int nd = PASS <= 1 ? k + 1 : 1;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    if (j >= nd) break;
    const double S = rn_block_sum2(acc[j].hi, acc[j].lo, s_w);
    if (threadIdx.x == 0) pb[(int64_t)j * gridDim.x + blockIdx.x] = S;
  }
}

// The same pass with the number of basis vectors KP = k + 1 fixed at compile
// time: every load of an element's KP basis values is issued before its
// first use, and the KP partials of a block come from one reduction.  Same
// arithmetic and order as k_gm_orth.
template <int KP, int PASS, bool MIXED>
__global__ __launch_bounds__(RN_BLOCK) void k_gm_orth_k(int64_t nnz, int64_t ubatch, int K, int k,
                                                       double *__restrict__ Uall, float *__restrict__ U32all,
                                                       double *__restrict__ part, const double *__restrict__ scal,
                                                       int scal_stride, const int32_t *__restrict__ stv) {
  constexpr int ND = PASS <= 1 ? KP : 1;
  __shared__ double s_r[2 * ND * (RN_BLOCK / RN_WAVE)];
  const int b = blockIdx.y;
  const int32_t *st = stv + (int64_t)b * ST_STRIDE;
  if (st[ST_STATUS] || st[ST_DONE]) return;
  const double *sc = scal + (int64_t)b * scal_stride;
  const GmLayout L(K);
  double *U = Uall + (int64_t)b * ubatch;
  double *W = U + (int64_t)(k + 1) * nnz;
  double coef[KP];
#pragma unroll
  for (int j = 0; j < KP; ++j) coef[j] = PASS > 0 ? sc[(PASS == 1 ? L.h1 : L.h2) + j] * sc[L.s + j] : 0.0;
  RnAcc acc[ND];
  for (int64_t e = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * RN_BLOCK) {
    double u[KP];
#pragma unroll
    for (int j = 0; j < KP; ++j) u[j] = U[(int64_t)j * nnz + e];
    double w = W[e];
    if (PASS > 0) {
#pragma unroll
      for (int j = 0; j < KP; ++j) w -= coef[j] * u[j];
      W[e] = w;
    }
    if (PASS <= 1) {
#pragma unroll
      for (int j = 0; j < KP; ++j) acc[j].add(w * u[j]);
    } else {
      acc[0].add(w * w);
      if (MIXED) U32all[(int64_t)b * ubatch + (int64_t)(k + 1) * nnz + e] = (float)w;
    }
  }
  double hi[ND], lo[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) {
    hi[j] = acc[j].hi;
    lo[j] = acc[j].lo;
  }
  double *pb = part + (int64_t)b * RN_MAXDOT * gridDim.x;
  rn_block_sum2_multi<RN_BLOCK / RN_WAVE, ND>(hi, lo, ND, s_r, pb + blockIdx.x, gridDim.x);
}

template <int PASS, bool MIXED>
static void gm_orth_k(int kp, dim3 g, dim3 bl, hipStream_t s, int64_t nz, int64_t ub, int K, int k, double *U,
                      float *U32, double *part, double *scal, int scal_stride, int32_t *st) {
#define GM_K(KP)                                                                                                   \
  case KP:                                                                                                         \
    hipLaunchKernelGGL((k_gm_orth_k<KP, PASS, MIXED>), g, bl, 0, s, nz, ub, K, k, U, U32, part, scal, scal_stride, \
                       st);                                                                                        \
    break;
  switch (kp) {
    GM_K(1) GM_K(2) GM_K(3) GM_K(4) GM_K(5) GM_K(6) GM_K(7) GM_K(8)
    GM_K(9) GM_K(10) GM_K(11) GM_K(12) GM_K(13) GM_K(14) GM_K(15) GM_K(16)
  }
#undef GM_K
}

__global__ void k_gm_solve(int K, double *__restrict__ scal, int scal_stride, const int32_t *__restrict__ stv) {
  const int b = blockIdx.x;
  if (threadIdx.x != 0) return;
  const int32_t *st = stv + (int64_t)b * ST_STRIDE;
  double *sc = scal + (int64_t)b * scal_stride;
  const GmLayout L(K);
  const int kd = st[ST_KD];
  const double *H = sc + L.H;
  for (int j = kd - 1; j >= 0; --j) {
    double v = sc[L.g + j];
    for (int l = j + 1; l < kd; ++l) v -= H[j * K + l] * sc[L.y + l];
    sc[L.y + j] = v / H[j * K + j];
  }
}

template <int NJ>
__global__ __launch_bounds__(RN_BLOCK) void k_gm_combine(int64_t nnz, int64_t ubatch, int K,
                                                        const double *__restrict__ T, const double *__restrict__ Uall,
                                                        double *__restrict__ P, const double *__restrict__ scal,
                                                        int scal_stride, const int32_t *__restrict__ stv) {
  const int b = blockIdx.y;
  const int32_t *st = stv + (int64_t)b * ST_STRIDE;
  const double *sc = scal + (int64_t)b * scal_stride;
  const GmLayout L(K);
  const int kd = st[ST_STATUS] ? 0 : st[ST_KD];
  double c[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) c[j] = j < kd ? sc[L.y + j] * sc[L.s + j] : 0.0;
  const double *U = Uall + (int64_t)b * ubatch;
  double *Pb = P + (int64_t)b * nnz;
  for (int64_t e = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * RN_BLOCK) {
    double v = T[e];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
      if (j < kd) v += c[j] * U[(int64_t)j * nnz + e];
    Pb[e] = v;
  }
}

// The same combination with K fixed at compile time: vector j is read for
// every j < K (the index clamped to the last vector the solve used, whose
// coefficient is zero beyond it), so the K loads of an element are all in
// flight before the first multiply-add.  Same arithmetic and order.
template <int KP>
__global__ __launch_bounds__(RN_BLOCK) void k_gm_combine_k(int64_t nnz, int64_t ubatch, const double *__restrict__ T,
                                                          const double *__restrict__ Uall, double *__restrict__ P,
                                                          const double *__restrict__ scal, int scal_stride,
                                                          const int32_t *__restrict__ stv) {
  const int b = blockIdx.y;
  const int32_t *st = stv + (int64_t)b * ST_STRIDE;
  const double *sc = scal + (int64_t)b * scal_stride;
  const GmLayout L(KP);
  const int kd = st[ST_STATUS] ? 0 : st[ST_KD];
  double *Pb = P + (int64_t)b * nnz;
  if (kd <= 0) {
    for (int64_t e = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * RN_BLOCK)
      Pb[e] = T[e];
    return;
  }
  const double *U = Uall + (int64_t)b * ubatch;
  double c[KP];
  const double *Uj[KP];
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    c[j] = j < kd ? sc[L.y + j] * sc[L.s + j] : 0.0;
    Uj[j] = U + (int64_t)(j < kd ? j : kd - 1) * nnz;
  }
  for (int64_t e = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * RN_BLOCK) {
    double u[KP];
#pragma unroll
    for (int j = 0; j < KP; ++j) u[j] = Uj[j][e];
    double v = T[e];
#pragma unroll
    for (int j = 0; j < KP; ++j) v += c[j] * u[j];
    Pb[e] = v;
  }
}

__global__ __launch_bounds__(RN_BLOCK) void k_zero3(int32_t *__restrict__ a, int64_t na, double *__restrict__ b,
                                                   int64_t nb, double *__restrict__ c, int64_t nc) {
  const int64_t s = (int64_t)gridDim.x * RN_BLOCK;
  for (int64_t q = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; q < na; q += s) a[q] = 0;
  for (int64_t q = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; q < nb; q += s) b[q] = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; q < nc; q += s) c[q] = 0.0;
}

__global__ __launch_bounds__(RN_BLOCK) void k_to_f32(const double *__restrict__ src, int64_t n,
                                                    float *__restrict__ dst) {
  for (int64_t q = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; q < n; q += (int64_t)gridDim.x * RN_BLOCK)
    dst[q] = (float)src[q];
}

// P = T for every batch entry (grid.y), and, by the blocks of entry 0, the
// status, scalar and history blocks zeroed: the CG set-up in one launch
__global__ __launch_bounds__(RN_BLOCK) void k_cg_start(const double *__restrict__ src, int64_t n, int64_t stride,
                                                      double *__restrict__ dst, int32_t *__restrict__ za, int64_t na,
                                                      double *__restrict__ zb, int64_t nb, double *__restrict__ zc,
                                                      int64_t nc) {
  const int b = blockIdx.y;
  const int64_t s = (int64_t)gridDim.x * RN_BLOCK, q0 = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x;
  if (b == 0) {
    for (int64_t q = q0; q < na; q += s) za[q] = 0;
    for (int64_t q = q0; q < nb; q += s) zb[q] = 0.0;
    for (int64_t q = q0; q < nc; q += s) zc[q] = 0.0;
  }
  for (int64_t q = q0; q < n; q += s) dst[(int64_t)b * stride + q] = src[q];
}

// ---------------------------------------------------------------------------
// preconditioned and normal-equation CG: row-wise projection passes
// ---------------------------------------------------------------------------
// Diagonal of A per DOF row and batch entry (M x M blocks), for the Jacobi
// preconditioner; a diagonal entry that is not positive raises st[ST_PREC].
template <int M>
__global__ __launch_bounds__(RN_BLOCK) void k_row_diag(int n, const int32_t *__restrict__ Ap,
                                                      const int32_t *__restrict__ Aj, const double *__restrict__ Ax,
                                                      int64_t strideA, double *__restrict__ dg,
                                                      int32_t *__restrict__ stv) {
  const int i = blockIdx.x * RN_BLOCK + threadIdx.x, b = blockIdx.y;
  if (i >= n) return;
  const int I = i / M, c = i % M;
  double d = 0.0;
  for (int p = Ap[I]; p < Ap[I + 1]; ++p)
    if (Aj[p] == I) d = Ax[(int64_t)b * strideA + (int64_t)p * M * M + c * M + c];
  dg[(int64_t)b * n + i] = d;
  if (!(d > 0.0)) stv[(int64_t)b * ST_STRIDE + ST_PREC] = 1;
}

enum { RP_PREC = 0, RP_PLAIN = 1, RP_INIT = 2 };

// One thread per DOF row (grid-stride over rows, grid.y = batch entry): the
// row of X (RP_PREC: scaled by 1 / a_ii) projected, Pi (Sec. 3.6: root rows
// zero, the least-squares component along Bc_J removed), into Y, with
// per-block compensated partials of one inner product:
//   RP_PREC  Y = Pi(D^-1 X), partial of <X, Y>    (Jacobi preconditioner)
//   RP_PLAIN Y = Pi(X),      partial of <V, Y>    (Y may be X)
//   RP_INIT  Y = Y2 = -Pi(X), partial of <Y, Y>.
// With check set, a stopped batch entry does nothing (the test is uniform per
// block).
template <int NB, int MODE>
__global__ __launch_bounds__(RN_BLOCK) void k_row_proj(int n, int64_t nnz, const int32_t *__restrict__ Np,
                                                      const int32_t *__restrict__ Nj,
                                                      const uint8_t *__restrict__ is_root,
                                                      const double *__restrict__ Bc, const double *__restrict__ gp,
                                                      const double *__restrict__ dg, const double *X,
                                                      double *Y, double *__restrict__ Y2,
                                                      const double *__restrict__ V, double *__restrict__ part,
                                                      int64_t pstride, const int32_t *__restrict__ stv, int check) {
  constexpr int NP = NB * (NB + 1) / 2;
  __shared__ double s_w[8];
  const int b = blockIdx.y;
  if (check) {
    const int32_t *st = stv + (int64_t)b * ST_STRIDE;
    if (st[ST_STATUS] || st[ST_DONE]) return;
  }
  const int64_t off = (int64_t)b * nnz;
  RnAcc acc;
  for (int i = blockIdx.x * RN_BLOCK + threadIdx.x; i < n; i += gridDim.x * RN_BLOCK) {
    const int s = Np[i], e = Np[i + 1];
    if (is_root[i]) {
      for (int p = s; p < e; ++p) {
        Y[off + p] = 0.0;
        if (MODE == RP_INIT) Y2[off + p] = 0.0;
      }
      continue;
    }
    const double d = MODE == RP_PREC ? dg[(int64_t)b * n + i] : 1.0;
    double sv[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) sv[q] = 0.0;
    for (int p = s; p < e; ++p) {
      const double x = MODE == RP_PREC ? X[off + p] / d : X[off + p];
      const double *bc = Bc + (int64_t)Nj[p] * NB;
#pragma unroll
      for (int q = 0; q < NB; ++q) sv[q] += x * bc[q];
    }
    double y[NB];
    const double *g = gp + (int64_t)i * NP;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      double t = 0.0;
#pragma unroll
      for (int r = 0; r < NB; ++r) t += g[rn_pk(NB, q, r)] * sv[r];
      y[q] = t;
    }
    for (int p = s; p < e; ++p) {
      const double xr = X[off + p];
      const double x = MODE == RP_PREC ? xr / d : xr;
      const double *bc = Bc + (int64_t)Nj[p] * NB;
      double u = 0.0;
#pragma unroll
      for (int q = 0; q < NB; ++q) u += bc[q] * y[q];
      const double z = x - u;
      if (MODE == RP_PREC) {
        Y[off + p] = z;
        acc.add(xr * z);
      } else if (MODE == RP_PLAIN) {
        const double v = V[off + p];
        Y[off + p] = z;
        acc.add(v * z);
      } else {
        Y[off + p] = -z;
        Y2[off + p] = -z;
        acc.add(z * z);
      }
    }
  }
  const double S = rn_block_sum2(acc.hi, acc.lo, s_w);
  if (threadIdx.x == 0) part[(int64_t)b * pstride + blockIdx.x] = S;
}

template <int MODE>
static void row_proj(int nB, dim3 g, hipStream_t stream, const rn_plan *pl, const double *dg, const double *X,
                     double *Y, double *Y2, const double *V, double *part, int64_t pstride, const int32_t *st,
                     int check) {
  const dim3 blk(RN_BLOCK);
  switch (nB) {
#define RP_CASE(NB)                                                                                                   \
  case NB:                                                                                                            \
    hipLaunchKernelGGL((k_row_proj<NB, MODE>), g, blk, 0, stream, pl->n, pl->nnzN, pl->Np, pl->Nj, pl->is_root,    \
                       pl->Bc, pl->gp, dg, X, Y, Y2, V, part, pstride, st, check);                                   \
    break;
    RP_CASE(1) RP_CASE(2) RP_CASE(3) RP_CASE(4)
#undef RP_CASE
  }
}

// ---------------------------------------------------------------------------
// metrics: inner products and the constraint residual
// ---------------------------------------------------------------------------
// Per-block compensated partials of <x, y> (grid-stride).
__global__ __launch_bounds__(RN_BLOCK) void k_dot_part(int64_t n, const double *__restrict__ x,
                                                      const double *__restrict__ y, double *__restrict__ part) {
  __shared__ double s_w[8];
  RnAcc a;
  for (int64_t q = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; q < n; q += (int64_t)gridDim.x * RN_BLOCK)
    a.add(x[q] * y[q]);
  const double S = rn_block_sum2(a.hi, a.lo, s_w);
  if (threadIdx.x == 0) part[blockIdx.x] = S;
}

// Per-block maxima of |(V Bc)_iq - ref_iq| with ref = B when given, else
// (T Bc)_iq (then (V - T) Bc is formed entry by entry); one thread per row.
template <int NB>
__global__ __launch_bounds__(RN_BLOCK) void k_cres_part(int n, const int32_t *__restrict__ Np,
                                                       const int32_t *__restrict__ Nj, const double *__restrict__ V,
                                                       const double *__restrict__ T, const double *__restrict__ Bc,
                                                       const double *__restrict__ B, double *__restrict__ part) {
  __shared__ double s_m[RN_BLOCK / RN_WAVE];
  double mx = 0.0;
  for (int i = blockIdx.x * RN_BLOCK + threadIdx.x; i < n; i += gridDim.x * RN_BLOCK) {
    double s[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) s[q] = 0.0;
    for (int p = Np[i]; p < Np[i + 1]; ++p) {
      const double v = T ? V[p] - T[p] : V[p];
      const double *bc = Bc + (int64_t)Nj[p] * NB;
#pragma unroll
      for (int q = 0; q < NB; ++q) s[q] += v * bc[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) mx = fmax(mx, fabs(B ? s[q] - B[(int64_t)i * NB + q] : s[q]));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, RN_WAVE));
  if ((threadIdx.x & (RN_WAVE - 1)) == 0) s_m[threadIdx.x / RN_WAVE] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = s_m[0];
    for (int w = 1; w < RN_BLOCK / RN_WAVE; ++w) m = fmax(m, s_m[w]);
    part[blockIdx.x] = m;
  }
}

// (A P) at the one entry of each root row (the masked product leaves root
// rows at zero): a thread per DOF row, the terms in the order of A's row (M x M
// blocks), P_kj found by binary search in row k of N.
template <int M>
__global__ __launch_bounds__(RN_BLOCK) void k_root_ap(int n, const int32_t *__restrict__ Ap,
                                                     const int32_t *__restrict__ Aj, const double *__restrict__ Ax,
                                                     const int32_t *__restrict__ Np, const int32_t *__restrict__ Nj,
                                                     const uint8_t *__restrict__ is_root,
                                                     const double *__restrict__ P, double *__restrict__ Y) {
  const int i = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (i >= n || !is_root[i] || Np[i + 1] == Np[i]) return;
  const int I = i / M, c = i % M, p0 = Np[i], j = Nj[p0];
  double s = 0.0;
  for (int b = Ap[I]; b < Ap[I + 1]; ++b) {
    const int J = Aj[b];
#pragma unroll
    for (int cc = 0; cc < M; ++cc) {
      const int k = M * J + cc;
      int lo = Np[k], hi = Np[k + 1];
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (Nj[mid] < j) lo = mid + 1; else hi = mid;
      }
      if (lo < Np[k + 1] && Nj[lo] == j) s += Ax[(int64_t)b * M * M + c * M + cc] * P[lo];
    }
  }
  Y[p0] = s;
}

// One block: out[0] = the sum (MAX = false) or the maximum of np partials.
template <bool MAX>
__global__ __launch_bounds__(RN_BLOCK) void k_fin_part(int np, const double *__restrict__ part,
                                                      double *__restrict__ out) {
  __shared__ double s_w[8];
  if (MAX) {
    double m = 0.0;
    for (int q = threadIdx.x; q < np; q += RN_BLOCK) m = fmax(m, part[q]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, RN_WAVE));
    if ((threadIdx.x & (RN_WAVE - 1)) == 0) s_w[threadIdx.x / RN_WAVE] = m;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = fmax(fmax(s_w[0], s_w[1]), fmax(s_w[2], s_w[3]));
  } else {
    const double S = rn_reduce_part(part, np, s_w);
    if (threadIdx.x == 0) out[0] = S;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// element-wise passes: two elements per lane and up to 1024 workgroups (4
// per compute unit), enough loads in flight to stream HBM; every dot leaves
// one partial per workgroup, which the next step sums in every workgroup or
// in a one-block finisher (2048 workgroups took the upwind1024 set-up 3 %
// longer, 256 were slower again)
static unsigned ew_grid(int64_t n) {
  unsigned g = rn_div_up(n, RN_BLOCK * 2);
  if (g < 1) g = 1;
  if (g > 1024) g = 1024;
  return g;
}

// Algorithmic bytes / flops of one masked product: A values + indices + row
// pointers, pattern indices + row pointers, X read once, Z written once, the
// root flags, the coarse candidates and the stored Gram data of the F rows.
static void product_cost(const rn_plan *pl, bool mixed, unsigned long long terms, double *bytes, double *flops) {
  const double val = mixed ? 4.0 : 8.0;
  const double mm = (double)pl->m * pl->m;
  double b = (4.0 + val * mm) * (double)pl->nnzA + 4.0 * (pl->nr + 1);  // A
  b += 4.0 * (double)pl->nnzN + 4.0 * (pl->n + 1);                      // N
  b += val * (double)pl->nnzN + 8.0 * (double)pl->nnzN;                 // X in, Z out
  b += (double)pl->n;                                                   // root flags
  const double nF = (double)pl->n - (double)pl->nc;
  b += 8.0 * (double)pl->nc * pl->nB + 8.0 * nF * (pl->nB * (pl->nB + 1) / 2);
  *bytes = b;
  // one term is a scalar multiply-add (block_m = 1) or a 2x2 block product
  // (8 multiply-adds, block_m = 2)
  *flops = 2.0 * (double)terms * (pl->m == 1 ? 1.0 : 8.0);
}

static rn_status common_ws(rn_plan *pl, int batch, int scal_stride, unsigned gew, SpgParams &p) {
  rn_status st = RN_OK;
  p.st = (int32_t *)rn_plan_ws(pl, WS_ST, (size_t)batch * ST_STRIDE * 4, &st);
  p.scal = (double *)rn_plan_ws(pl, WS_SCAL, (size_t)batch * scal_stride * 8, &st);
  // product partials [batch][RN_MAXDOT][nblk] then element-wise partials
  p.part = (double *)rn_plan_ws(pl, WS_PART, (size_t)batch * RN_MAXDOT * ((size_t)pl->nblk + gew + 2) * 8, &st);
  if (!p.st || !p.scal || !p.part) return st;
  p.scal_stride = scal_stride;
  return RN_OK;
}

static constexpr unsigned METRIC_GRID = 512;

// Constraint residual of V (one problem) against B, or against T Bc when B is
// NULL, into out (device double); res (device, 2 * METRIC_GRID doubles) holds
// the partials.
static rn_status cres_launch(rn_ctx *ctx, int32_t n, const int32_t *Np, const int32_t *Nj, const double *V,
                             const double *T, const double *Bc, const double *B, int nB, double *part, double *out) {
  const dim3 g(METRIC_GRID), blk(RN_BLOCK);
  switch (nB) {
    case 1: hipLaunchKernelGGL(k_cres_part<1>, g, blk, 0, ctx->stream, n, Np, Nj, V, T, Bc, B, part); break;
    case 2: hipLaunchKernelGGL(k_cres_part<2>, g, blk, 0, ctx->stream, n, Np, Nj, V, T, Bc, B, part); break;
    case 3: hipLaunchKernelGGL(k_cres_part<3>, g, blk, 0, ctx->stream, n, Np, Nj, V, T, Bc, B, part); break;
    case 4: hipLaunchKernelGGL(k_cres_part<4>, g, blk, 0, ctx->stream, n, Np, Nj, V, T, Bc, B, part); break;
    default: return rn_fail(ctx, RN_EINVAL, "constraint residual: nB %d", nB);
  }
  LAUNCH_CHECK(ctx);
  hipLaunchKernelGGL(k_fin_part<true>, dim3(1), blk, 0, ctx->stream, (int)METRIC_GRID, part, out);
  LAUNCH_CHECK(ctx);
  return RN_OK;
}

// E(P) = <P, A P> over N (root rows included) and <Y, Pi(Y)> = ||Pi(Y)||^2
// for Y = A P kept to N into out[0], out[1] (device); Y in the plan's Z
// workspace (projected in place).
static rn_status energy_launch(rn_ctx *ctx, rn_plan *pl, const double *A_vals, const double *P, double *part,
                               double *out) {
  rn_status st = RN_OK;
  double *Y = (double *)rn_plan_ws(pl, WS_Z, (size_t)pl->nnzN * 8, &st);
  if (!Y) return st;
  SpgParams q = rn_spg_params(pl);
  RN_TRY(common_ws(pl, 1, SC_BASE, 1, q));
  q.project = 0;
  q.Z = Y;
  q.Ax = A_vals;
  q.X = P;
  RN_TRY(rn_launch_spgemm(ctx, pl, MODE_PRODUCT, q, 1, false));
  const dim3 g(METRIC_GRID), blk(RN_BLOCK);
  if (pl->n > 0) {
    if (pl->m == 1)
      hipLaunchKernelGGL(k_root_ap<1>, dim3(rn_div_up(pl->n, RN_BLOCK)), blk, 0, ctx->stream, pl->n, pl->Ap, pl->Aj,
                         A_vals, pl->Np, pl->Nj, pl->is_root, P, Y);
    else
      hipLaunchKernelGGL(k_root_ap<2>, dim3(rn_div_up(pl->n, RN_BLOCK)), blk, 0, ctx->stream, pl->n, pl->Ap, pl->Aj,
                         A_vals, pl->Np, pl->Nj, pl->is_root, P, Y);
    LAUNCH_CHECK(ctx);
  }
  hipLaunchKernelGGL(k_dot_part, g, blk, 0, ctx->stream, pl->nnzN, P, Y, part);
  LAUNCH_CHECK(ctx);
  hipLaunchKernelGGL(k_fin_part<false>, dim3(1), blk, 0, ctx->stream, (int)METRIC_GRID, part, out);
  LAUNCH_CHECK(ctx);
  // the status block must read "running" for the projection pass
  row_proj<RP_PLAIN>(pl->nB, dim3(METRIC_GRID), ctx->stream, pl, nullptr, Y, Y, nullptr, Y, part + METRIC_GRID,
                     0, q.st, 0);
  LAUNCH_CHECK(ctx);
  hipLaunchKernelGGL(k_fin_part<false>, dim3(1), blk, 0, ctx->stream, (int)METRIC_GRID, part + METRIC_GRID, out + 1);
  LAUNCH_CHECK(ctx);
  return RN_OK;
}

extern "C" rn_status rn_energy(rn_ctx *ctx, rn_plan *pl, const double *A_vals, const double *P, double *energy,
                               double *proj_residual) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (!pl || !A_vals || !P) return rn_fail(ctx, RN_EINVAL, "rn_energy: null argument");
  rn_status st = RN_OK;
  double *part = (double *)rn_scratch(ctx, SLOT_MISC, (2 * METRIC_GRID + 4) * sizeof(double), &st);
  if (!part) return st;
  double *out = part + 2 * METRIC_GRID;
  RN_TRY(energy_launch(ctx, pl, A_vals, P, part, out));
  const RnFetch it[1] = {{out, 2 * sizeof(double)}};
  const unsigned char *hb = nullptr;
  size_t off[1];
  RN_TRY(rn_fetch(ctx, 1, it, &hb, off));
  double v[2];
  memcpy(v, hb + off[0], sizeof v);
  if (energy) *energy = v[0];
  if (proj_residual) *proj_residual = sqrt(fmax(v[1], 0.0));
  return RN_OK;
}

extern "C" rn_status rn_constraint_residual(rn_ctx *ctx, int32_t n, int32_t n_cols, const int32_t *Np,
                                            const int32_t *Nj, int64_t nnz_N, const double *vals, const double *Bc,
                                            const double *B, int32_t nB, double *res) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (!res || n < 0 || n_cols < 0 || nnz_N < 0 || nB < 1 || nB > RN_NBMAX || (n > 0 && (!Np || !B)) ||
      (nnz_N > 0 && (!Nj || !vals || !Bc)))
    return rn_fail(ctx, RN_EINVAL, "rn_constraint_residual: bad argument");
  if (nnz_N >= ((int64_t)1 << 31)) return rn_fail(ctx, RN_ELIMIT, "rn_constraint_residual: nnz_N >= 2^31");
  rn_status st = RN_OK;
  int32_t *guard = rn_guard_begin(ctx, &st);
  if (!guard) return st;
  double *part = (double *)rn_scratch(ctx, SLOT_MISC, (2 * METRIC_GRID + 4) * sizeof(double), &st);
  if (!part) return st;
  RnChecks v{};
  v.csr[0] = {n, n_cols, nnz_N, Np, Nj, GUARD_N};
  v.ncsr = 1;
  RN_TRY(rn_validate(ctx, v, guard));
  // kernels run only on a valid pattern: read the guard first
  RN_TRY(rn_check_guard(ctx, guard, "rn_constraint_residual"));
  double *out = part + 2 * METRIC_GRID;
  RN_TRY(cres_launch(ctx, n, Np, Nj, vals, nullptr, Bc, B, nB, part, out));
  const RnFetch it[1] = {{out, sizeof(double)}};
  const unsigned char *hb = nullptr;
  size_t off[1];
  RN_TRY(rn_fetch(ctx, 1, it, &hb, off));
  memcpy(res, hb + off[0], sizeof(double));
  return RN_OK;
}

extern "C" rn_status rn_masked_product(rn_ctx *ctx, rn_plan *pl, const double *A_vals, int32_t batch,
                                       const double *X, int32_t project, rn_precision prec, double *Z) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (!pl || !A_vals || !X || !Z || batch < 1) return rn_fail(ctx, RN_EINVAL, "rn_masked_product: bad argument");
  if (prec != RN_FP64 && prec != RN_FP32_MIXED) return rn_fail(ctx, RN_EINVAL, "rn_masked_product: bad precision");
  const bool mixed = prec == RN_FP32_MIXED;
  SpgParams p = rn_spg_params(pl);
  RN_TRY(common_ws(pl, batch, SC_BASE, 1, p));
  p.project = project != 0;
  p.Z = Z;
  p.Ax = A_vals;
  p.X = X;
  if (mixed) {
    rn_status st = RN_OK;
    const int64_t na = (int64_t)batch * p.strideA, nx = (int64_t)batch * pl->nnzN;
    float *A32 = (float *)rn_plan_ws(pl, WS_A32, (size_t)na * 4, &st);
    float *X32 = (float *)rn_plan_ws(pl, WS_D32, (size_t)nx * 4, &st);
    if (!A32 || !X32) return st;
    hipLaunchKernelGGL(k_to_f32, dim3(ew_grid(na)), dim3(RN_BLOCK), 0, ctx->stream, A_vals, na, A32);
    hipLaunchKernelGGL(k_to_f32, dim3(ew_grid(nx)), dim3(RN_BLOCK), 0, ctx->stream, X, nx, X32);
    LAUNCH_CHECK(ctx);
    p.Ax = A32;
    p.X = X32;
  }
  return rn_launch_spgemm(ctx, pl, MODE_PRODUCT, p, batch, mixed);
}

// Arguments of rn_energy_min checked on the host.
static rn_status emin_check(rn_ctx *ctx, rn_plan *pl, const double *A_vals, int32_t batch, const double *T,
                            rn_method method, int32_t iters, rn_precision prec, double *P) {
  if (!pl || !A_vals || !T || !P || batch < 1 || iters < 0)
    return rn_fail(ctx, RN_EINVAL, "rn_energy_min: bad argument");
  if (method != RN_CG && method != RN_GMRES && method != RN_PCG_JACOBI && method != RN_CGNR)
    return rn_fail(ctx, RN_EINVAL, "rn_energy_min: bad method");
  if (prec != RN_FP64 && prec != RN_FP32_MIXED) return rn_fail(ctx, RN_EINVAL, "rn_energy_min: bad precision");
  if ((method == RN_PCG_JACOBI || method == RN_CGNR) && prec != RN_FP64)
    return rn_fail(ctx, RN_EINVAL, "rn_energy_min: the preconditioned and normal-equation forms run in FP64");
  if (method == RN_CGNR && batch != 1) return rn_fail(ctx, RN_EINVAL, "rn_energy_min: CGNR takes one problem");
  if (method == RN_GMRES && iters > RN_MAXDOT - 1)
    return rn_fail(ctx, RN_ELIMIT, "rn_energy_min: GMRES supports at most %d iterations", RN_MAXDOT - 1);
  return RN_OK;
}

static rn_status emin_run(rn_ctx *ctx, rn_plan *pl, const double *A_vals, int32_t batch, const double *T,
                          rn_method method, int32_t iters, rn_precision prec, double *P, double *hist,
                          rn_emin_stats *stats, rn_tape *tape);

extern "C" rn_status rn_energy_min(rn_ctx *ctx, rn_plan *pl, const double *A_vals, int32_t batch, const double *T,
                                   rn_method method, int32_t iters, rn_precision prec, double *P, double *hist,
                                   rn_emin_stats *stats, rn_tape *tape) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  RN_TRY(emin_check(ctx, pl, A_vals, batch, T, method, iters, prec, P));
  if (tape && method != RN_CG) return rn_fail(ctx, RN_EINVAL, "rn_energy_min: a tape records CG only");
  if (tape) RN_TRY(rn_tape_record_begin(ctx, pl, tape, batch, iters, method, prec, T));
  return emin_run(ctx, pl, A_vals, batch, T, method, iters, prec, P, hist, stats, tape);
}

// Workspace bytes emin_run requests (each piece rounded to 256 bytes, as the
// arena carves them), and the bytes of its one read-back.
// the tape's Z_k slot at a checkpoint step (rn_adjoint.hip), else NULL
double *rn_tape_Z(rn_tape *tape, int k);

// CG (FP64 with or without a tape, or FP32-mixed) forms each direction inside
// the next product when the context allows it and the persistent product
// serves the plan
static bool cg_fused(const rn_ctx *ctx, const rn_plan *pl, int32_t batch, rn_method method, rn_precision prec) {
  return ctx->opt[RN_OPT_FUSED_CG] && method == RN_CG && (prec == RN_FP64 || prec == RN_FP32_MIXED) &&
         rn_spgemm_fused_grid(pl, batch, prec == RN_FP32_MIXED) > 0;
}

static size_t emin_ws_need(const rn_plan *pl, int32_t batch, bool gm, bool pcg, int K, bool mixed, bool fused,
                           size_t *fetch) {
  auto r = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const int64_t nz = pl->nnzN, nzb = (int64_t)batch * nz;
  const unsigned gew = gm ? ew_grid(nz) : std::min(ew_grid(nz), 1024u);
  const int scal_stride = gm ? GmLayout(K).total : CgLayout(K).total;
  const SpgParams p = rn_spg_params(pl);
  size_t need = r((size_t)batch * ST_STRIDE * 4) + r((size_t)batch * scal_stride * 8) +
                r((size_t)batch * RN_MAXDOT * ((size_t)pl->nblk + gew + 2) * 8);
  if (mixed) need += r((size_t)batch * p.strideA * 4) + r((size_t)nz * 4);
  if (!gm) {
    need += (fused ? 4 : 3) * r((size_t)nzb * 8) + (mixed ? r((size_t)nzb * 4) : 0);
    if (pcg) need += r((size_t)nzb * 8) + r((size_t)batch * (pl->n + 1) * 8);
  } else {
    const size_t ub = (size_t)(K + 1) * nz;
    need += r((size_t)batch * ub * 8) + (mixed ? r((size_t)batch * ub * 4) : 0);
  }
  auto a8 = [](size_t b) { return (b + 7) & ~(size_t)7; };
  *fetch = a8((size_t)batch * ST_STRIDE * 4) + a8((size_t)scal_stride * 8) + 8;
  return need;
}

extern "C" rn_status rn_energy_min_noalloc(rn_ctx *ctx, rn_plan *pl, const double *A_vals, int32_t batch,
                                           const double *T, rn_method method, int32_t iters, rn_precision prec,
                                           double *P, double *hist, rn_emin_stats *stats) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  RN_TRY(emin_check(ctx, pl, A_vals, batch, T, method, iters, prec, P));
  if (method == RN_CGNR)
    return rn_fail(ctx, RN_EINVAL, "rn_energy_min_noalloc: CGNR builds the pattern of A N and needs allocation");
  if (!ctx->noalloc_scratch)
    return rn_fail(ctx, RN_EHIP, "rn_energy_min_noalloc: no device address for the scratch array on device %d",
                   ctx->device);
  if (!ctx->rb_host) return rn_fail(ctx, RN_ENOMEM, "rn_energy_min_noalloc: no read-back area");
  size_t fetch = 0;
  const size_t need = emin_ws_need(pl, batch, method == RN_GMRES, method == RN_PCG_JACOBI, iters,
                                   prec == RN_FP32_MIXED, cg_fused(ctx, pl, batch, method, prec), &fetch);
  if (need > RN_NOALLOC_SCRATCH_BYTES)
    return rn_fail(ctx, RN_ELIMIT,
                   "rn_energy_min_noalloc: the call needs %zu bytes of scratch, the allocation-free limit is %zu",
                   need, (size_t)RN_NOALLOC_SCRATCH_BYTES);
  if (fetch > ctx->rb_cap)
    return rn_fail(ctx, RN_ELIMIT, "rn_energy_min_noalloc: read-back of %zu bytes beyond the reserved %zu", fetch,
                   ctx->rb_cap);
  // the plan's workspace requests are carved from the scratch array for the
  // duration of this call
  struct ArenaScope {
    rn_plan *pl;
    ArenaScope(rn_plan *p, void *base) : pl(p) {
      pl->arena = (unsigned char *)base;
      pl->arena_cap = RN_NOALLOC_SCRATCH_BYTES;
      pl->arena_used = 0;
    }
    ~ArenaScope() {
      pl->arena = nullptr;
      pl->arena_cap = pl->arena_used = 0;
    }
  } scope(pl, ctx->noalloc_scratch);
  return emin_run(ctx, pl, A_vals, batch, T, method, iters, prec, P, hist, stats, nullptr);
}

static rn_status emin_run(rn_ctx *ctx, rn_plan *pl, const double *A_vals, int32_t batch, const double *T,
                          rn_method method, int32_t iters, rn_precision prec, double *P, double *hist,
                          rn_emin_stats *stats, rn_tape *tape) {
  const bool mixed = prec == RN_FP32_MIXED;
  const bool gm = method == RN_GMRES;
  const bool fuse = cg_fused(ctx, pl, batch, method, prec);
  const int K = iters;
  const int64_t nz = pl->nnzN, nzb = (int64_t)batch * nz;
  rn_status st = RN_OK;
  // CG: at most 1024 workgroups for its element-wise kernels (every block of
  // the update and direction kernels sums the previous kernel's partials)
  const unsigned gew = gm ? ew_grid(nz) : std::min(ew_grid(nz), 1024u);
  const int scal_stride = gm ? GmLayout(K).total : CgLayout(K).total;
  const int hist_stride = 3 * K + 1;
  SpgParams p = rn_spg_params(pl);
  RN_TRY(common_ws(pl, batch, scal_stride, gew, p));
  p.K = K;
  double *part_spg = p.part;
  double *part_ew = p.part + (int64_t)batch * RN_MAXDOT * pl->nblk;
  const int64_t pstride_spg = (int64_t)RN_MAXDOT * pl->nblk, pstride_ew = (int64_t)RN_MAXDOT * gew;
  // status, scalars and history start at zero (one launch for the three;
  // for CG the launch that sets P = T does it)
  const int64_t n_st = (int64_t)batch * ST_STRIDE, n_sc = (int64_t)batch * scal_stride,
                n_hist = hist ? (int64_t)batch * hist_stride : 0;
  if (gm) {
    hipLaunchKernelGGL(k_zero3, dim3(64), dim3(RN_BLOCK), 0, ctx->stream, p.st, n_st, p.scal, n_sc, hist, n_hist);
    LAUNCH_CHECK(ctx);
  }
  const float *A32 = nullptr, *T32 = nullptr;
  if (mixed) {
    const int64_t na = (int64_t)batch * p.strideA;
    float *a32 = (float *)rn_plan_ws(pl, WS_A32, (size_t)na * 4, &st);
    float *t32 = (float *)rn_plan_ws(pl, WS_T32, (size_t)nz * 4, &st);
    if (!a32 || !t32) return st;
    hipLaunchKernelGGL(k_to_f32, dim3(ew_grid(na)), dim3(RN_BLOCK), 0, ctx->stream, A_vals, na, a32);
    hipLaunchKernelGGL(k_to_f32, dim3(ew_grid(nz)), dim3(RN_BLOCK), 0, ctx->stream, T, nz, t32);
    LAUNCH_CHECK(ctx);
    A32 = a32;
    T32 = t32;
  }
  const void *Aop = mixed ? (const void *)A32 : (const void *)A_vals;
  const void *Top = mixed ? (const void *)T32 : (const void *)T;
  const dim3 g2(gew, (unsigned)batch), blk(RN_BLOCK);
  const int64_t pstride_row = (int64_t)RN_MAXDOT * gew;  // partials of the row passes, per batch entry
  if (method == RN_PCG_JACOBI) {
    // Jacobi-preconditioned CG: Y = Pi(D^-1 R) replaces R in gamma = <R, Y>
    // and in the direction D = Y + beta D; products and updates as for CG
    double *R = (double *)rn_plan_ws(pl, WS_R, (size_t)nzb * 8, &st);
    double *D = (double *)rn_plan_ws(pl, WS_D, (size_t)nzb * 8, &st);
    double *Z = (double *)rn_plan_ws(pl, WS_Z, (size_t)nzb * 8, &st);
    double *Y = (double *)rn_plan_ws(pl, WS_Y, (size_t)nzb * 8, &st);
    double *dg = (double *)rn_plan_ws(pl, WS_DIAG, (size_t)batch * (pl->n + 1) * 8, &st);
    if (!R || !D || !Z || !Y || !dg) return st;
    hipLaunchKernelGGL(k_cg_start, g2, blk, 0, ctx->stream, T, nz, nz, P, p.st, n_st, p.scal, n_sc, hist, n_hist);
    LAUNCH_CHECK(ctx);
    if (pl->n > 0) {
      const dim3 gd(rn_div_up(pl->n, RN_BLOCK), (unsigned)batch);
      if (pl->m == 1)
        hipLaunchKernelGGL(k_row_diag<1>, gd, blk, 0, ctx->stream, pl->n, pl->Ap, pl->Aj, A_vals, p.strideA, dg,
                           p.st);
      else
        hipLaunchKernelGGL(k_row_diag<2>, gd, blk, 0, ctx->stream, pl->n, pl->Ap, pl->Aj, A_vals, p.strideA, dg,
                           p.st);
      LAUNCH_CHECK(ctx);
    }
    // R_0 = -Pi(A T), D_0 = Y_0 = Pi(D^-1 R_0), gamma_0 = <R_0, Y_0>
    SpgParams q = p;
    q.Ax = A_vals;
    q.X = T;
    q.strideX = 0;
    q.Z = R;
    q.Z2 = D;
    RN_TRY(rn_launch_spgemm(ctx, pl, MODE_CG_INIT, q, batch, false));
    row_proj<RP_PREC>(pl->nB, g2, ctx->stream, pl, dg, R, D, nullptr, nullptr, part_ew, pstride_row, p.st, 0);
    LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_cg_fin_init, dim3(batch), blk, 0, ctx->stream, (int)gew, pstride_row, part_ew, p.scal,
                       scal_stride, K, p.st, hist, hist_stride);
    LAUNCH_CHECK(ctx);
    for (int k = 0; k < K; ++k) {
      SpgParams s = p;
      s.k = k;
      s.Ax = A_vals;
      s.X = D;
      s.Xown = D;
      s.Z = Z;
      int np = 0;
      RN_TRY(rn_launch_spgemm(ctx, pl, MODE_CG_STEP, s, batch, false, &np));
      hipLaunchKernelGGL(k_cg_update, g2, blk, 0, ctx->stream, nz, nz, K, k, np, pstride_spg, part_spg, P, R, D, Z,
                         part_ew, p.scal, scal_stride, p.st, hist, hist_stride, (double *)nullptr);
      LAUNCH_CHECK(ctx);
      row_proj<RP_PREC>(pl->nB, g2, ctx->stream, pl, dg, R, Y, nullptr, nullptr, part_ew, pstride_row, p.st, 1);
      LAUNCH_CHECK(ctx);
      hipLaunchKernelGGL(k_cg_dir<false>, g2, blk, 0, ctx->stream, nz, nz, K, k, (int)gew, Y, D, (float *)nullptr,
                         part_ew, p.scal, scal_stride, p.st, hist, hist_stride, (double *)nullptr);
      LAUNCH_CHECK(ctx);
    }
  } else if (method == RN_CGNR) {
    // CGNR (one problem): W = A X on the pattern of A N, Pi(A^T W) kept to N
    int32_t *guard = rn_guard_begin(ctx, &st);
    if (!guard) return st;
    const rn_matrix Am = {pl->n, pl->m, pl->nnzA, pl->Ap, pl->Aj, A_vals};
    const int32_t *Sp = nullptr, *Sj = nullptr;
    const double *Sv = nullptr;
    RN_TRY(rn_scalar_view(ctx, &Am, &Sp, &Sj, &Sv, guard));
    const int64_t nzA = pl->nnzA * pl->m * pl->m;
    const int32_t n = pl->n;
    int32_t *ATp = (int32_t *)rn_scratch(ctx, SLOT_NRM_TP, (size_t)(n + 1) * 4, &st);
    int32_t *ATj = (int32_t *)rn_scratch(ctx, SLOT_NRM_TJ, (size_t)(nzA + 1) * 4, &st);
    double *ATv = (double *)rn_scratch(ctx, SLOT_NRM_TV, (size_t)(nzA + 1) * 8, &st);
    int32_t *perm = (int32_t *)rn_scratch(ctx, SLOT_NRM_PERM, (size_t)(nzA + 1) * 4, &st);
    if (!ATp || !ATj || !ATv || !perm) return st;
    RN_TRY(rn_transpose_structure(ctx, n, n, nzA, Sp, Sj, ATp, ATj, perm, guard));
    RN_TRY(rn_gather_values(ctx, Sv, perm, nzA, ATv));
    int32_t *Wp = nullptr, *Wj = nullptr;
    int64_t nzW = 0;
    RN_TRY(rn_sg_pattern(ctx, n, nzA, Sp, Sj, pl->Np, pl->Nj, SLOT_NRM_WP, SLOT_NRM_WJ, &Wp, &Wj, &nzW, guard,
                         "rn_energy_min (CGNR)"));
    double *Wv = (double *)rn_scratch(ctx, SLOT_NRM_WV, (size_t)(nzW + 1) * 8, &st);
    double *R = (double *)rn_plan_ws(pl, WS_R, (size_t)nz * 8, &st);
    double *D = (double *)rn_plan_ws(pl, WS_D, (size_t)nz * 8, &st);
    double *Z = (double *)rn_plan_ws(pl, WS_Z, (size_t)nz * 8, &st);
    if (!Wv || !R || !D || !Z) return st;
    hipLaunchKernelGGL(k_cg_start, g2, blk, 0, ctx->stream, T, nz, nz, P, p.st, n_st, p.scal, n_sc, hist, n_hist);
    LAUNCH_CHECK(ctx);
    // R_0 = D_0 = -Pi(A^T (A T)), gamma_0 = <R_0, R_0>
    RN_TRY(rn_sg_values(ctx, n, nzW, Sp, Sj, Sv, pl->Np, pl->Nj, T, Wp, Wj, Wv, guard));
    RN_TRY(rn_sg_values(ctx, n, nz, ATp, ATj, ATv, Wp, Wj, Wv, pl->Np, pl->Nj, Z, guard));
    row_proj<RP_INIT>(pl->nB, g2, ctx->stream, pl, nullptr, Z, R, D, nullptr, part_ew, pstride_row, p.st, 0);
    LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_cg_fin_init, dim3(1), blk, 0, ctx->stream, (int)gew, pstride_row, part_ew, p.scal,
                       scal_stride, K, p.st, hist, hist_stride);
    LAUNCH_CHECK(ctx);
    double *part_dz = part_ew + gew;  // <D, Z> partials (the update writes <R, R> at part_ew)
    for (int k = 0; k < K; ++k) {
      RN_TRY(rn_sg_values(ctx, n, nzW, Sp, Sj, Sv, pl->Np, pl->Nj, D, Wp, Wj, Wv, guard));
      RN_TRY(rn_sg_values(ctx, n, nz, ATp, ATj, ATv, Wp, Wj, Wv, pl->Np, pl->Nj, Z, guard));
      row_proj<RP_PLAIN>(pl->nB, g2, ctx->stream, pl, nullptr, Z, Z, nullptr, D, part_dz, pstride_row, p.st, 1);
      LAUNCH_CHECK(ctx);
      hipLaunchKernelGGL(k_cg_update, g2, blk, 0, ctx->stream, nz, nz, K, k, (int)gew, pstride_row, part_dz, P, R,
                         D, Z, part_ew, p.scal, scal_stride, p.st, hist, hist_stride, (double *)nullptr);
      LAUNCH_CHECK(ctx);
      hipLaunchKernelGGL(k_cg_dir<false>, g2, blk, 0, ctx->stream, nz, nz, K, k, (int)gew, R, D, (float *)nullptr,
                         part_ew, p.scal, scal_stride, p.st, hist, hist_stride, (double *)nullptr);
      LAUNCH_CHECK(ctx);
    }
  } else if (!gm) {
    // fused: D_k alternates between D and D2 (product k reads D_{k-1} from
    // one and writes D_k to the other while other workgroups still read)
    double *R = (double *)rn_plan_ws(pl, WS_R, (size_t)nzb * 8, &st);
    double *D = (double *)rn_plan_ws(pl, WS_D, (size_t)nzb * 8, &st);
    double *Z = (double *)rn_plan_ws(pl, WS_Z, (size_t)nzb * 8, &st);
    float *D32 = mixed ? (float *)rn_plan_ws(pl, WS_D32, (size_t)nzb * 4, &st) : nullptr;
    double *D2 = fuse ? (double *)rn_plan_ws(pl, WS_D2, (size_t)nzb * 8, &st) : nullptr;
    if (!R || !D || !Z || (mixed && !D32) || (fuse && !D2)) return st;
    hipLaunchKernelGGL(k_cg_start, g2, blk, 0, ctx->stream, T, nz, nz, P, p.st, n_st, p.scal, n_sc, hist, n_hist);
    LAUNCH_CHECK(ctx);
    // R_0 = D_0 = -Pi(A T), gamma_0
    SpgParams q = p;
    q.Ax = Aop;
    q.X = Top;
    q.strideX = 0;
    q.Z = R;
    q.Z2 = D;
    int np = 0;
    RN_TRY(rn_launch_spgemm(ctx, pl, MODE_CG_INIT, q, batch, mixed, &np));
    hipLaunchKernelGGL(k_cg_fin_init, dim3(batch), blk, 0, ctx->stream, np, pstride_spg, part_spg, p.scal,
                       scal_stride, K, p.st, hist, hist_stride);
    LAUNCH_CHECK(ctx);
    if (mixed) {
      hipLaunchKernelGGL(k_to_f32, dim3(ew_grid(nzb)), blk, 0, ctx->stream, D, nzb, D32);
      LAUNCH_CHECK(ctx);
    }
    if (tape) {  // R_0 = D_0 into slot 0; later iterates are written by the kernels
      HIP_TRY(ctx, hipMemcpyAsync(rn_tape_R(tape, 0), R, (size_t)nzb * 8, hipMemcpyDeviceToDevice, ctx->stream));
      HIP_TRY(ctx, hipMemcpyAsync(rn_tape_D(tape, 0), D, (size_t)nzb * 8, hipMemcpyDeviceToDevice, ctx->stream));
    }
    // every step product on the fused kernel's grid (the same grouping of
    // the <D, Z> partials with or without fusion and tape)
    const int step_grid = rn_spgemm_fused_grid(pl, batch, mixed);
    for (int k = 0; k < K; ++k) {
      SpgParams s = p;
      s.k = k;
      s.Ax = Aop;
      // a tape keeps Z_k at its checkpoint steps: the product writes it there
      double *Zs = tape ? rn_tape_Z(tape, k) : nullptr;
      double *Zk = Zs ? Zs : Z;
      s.Z = Zk;
      s.grid = step_grid;
      double *Dk = (fuse && (k & 1)) ? D2 : D;
      int np = 0;
      if (fuse && k > 0) {
        // beta_{k-1}, the stopping test and D_k in the product's staging
        s.X = (k & 1) ? D : D2;
        s.Rres = R;
        s.Dnew = Dk;
        s.part_rr = part_ew;
        s.np_rr = (int)gew;
        s.pstride_rr = pstride_ew;
        s.hist = hist;
        s.hist_stride = hist_stride;
        RN_TRY(rn_launch_spgemm(ctx, pl, MODE_CG_FSTEP, s, batch, mixed, &np));
        // a checkpoint step keeps the D_k the product just formed (a batch
        // entry that stopped leaves its slot unread: the reverse sweep skips
        // the steps it did not take)
        if (double *dt = tape ? rn_tape_D(tape, k) : nullptr)
          HIP_TRY(ctx, hipMemcpyAsync(dt, Dk, (size_t)nzb * 8, hipMemcpyDeviceToDevice, ctx->stream));
      } else {
        s.X = mixed ? (const void *)D32 : (const void *)D;
        s.Xown = D;
        RN_TRY(rn_launch_spgemm(ctx, pl, MODE_CG_STEP, s, batch, mixed, &np));
      }
      hipLaunchKernelGGL(k_cg_update, g2, blk, 0, ctx->stream, nz, nz, K, k, np, pstride_spg, part_spg, P, R, Dk, Zk,
                         part_ew, p.scal, scal_stride, p.st, hist, hist_stride,
                         tape ? rn_tape_R(tape, k + 1) : nullptr);
      LAUNCH_CHECK(ctx);
      if (fuse) continue;
      if (mixed)
        hipLaunchKernelGGL(k_cg_dir<true>, g2, blk, 0, ctx->stream, nz, nz, K, k, (int)gew, R, D, D32, part_ew, p.scal,
                           scal_stride, p.st, hist, hist_stride, (double *)nullptr);
      else
        hipLaunchKernelGGL(k_cg_dir<false>, g2, blk, 0, ctx->stream, nz, nz, K, k, (int)gew, R, D, (float *)nullptr,
                           part_ew, p.scal, scal_stride, p.st, hist, hist_stride,
                           tape ? rn_tape_D(tape, k + 1) : nullptr);
      LAUNCH_CHECK(ctx);
    }
    if (fuse && K > 0) {
      hipLaunchKernelGGL(k_cg_last, dim3(batch), blk, 0, ctx->stream, (int)gew, part_ew, K, p.scal, scal_stride, p.st,
                         hist, hist_stride);
      LAUNCH_CHECK(ctx);
    }
    if (tape) RN_TRY(rn_tape_record_end(ctx, tape, p.scal, p.st, batch));
  } else {
    const int64_t ub = (int64_t)(K + 1) * nz;
    double *U = (double *)rn_plan_ws(pl, WS_U, (size_t)batch * ub * 8, &st);
    float *U32 = mixed ? (float *)rn_plan_ws(pl, WS_U32, (size_t)batch * ub * 4, &st) : nullptr;
    if (!U || (mixed && !U32)) return st;
    SpgParams q = p;
    q.Ax = Aop;
    q.X = Top;
    q.strideX = 0;
    q.Z = U;
    q.strideZ = ub;
    int np = 0;
    RN_TRY(rn_launch_spgemm(ctx, pl, MODE_GM_INIT, q, batch, mixed, &np));
    hipLaunchKernelGGL(k_gm_fin<0>, dim3(batch), blk, 0, ctx->stream, np, pstride_spg, part_spg, K, 0, p.scal,
                       scal_stride, p.st, hist, hist_stride);
    LAUNCH_CHECK(ctx);
    if (mixed) {
      for (int b = 0; b < batch; ++b)
        hipLaunchKernelGGL(k_to_f32, dim3(ew_grid(nz)), blk, 0, ctx->stream, U + (int64_t)b * ub, nz,
                           U32 + (int64_t)b * ub);
      LAUNCH_CHECK(ctx);
    }
    for (int k = 0; k < K; ++k) {
      SpgParams s = p;
      s.k = k;
      s.Ax = Aop;
      s.X = mixed ? (const void *)(U32 + (int64_t)k * nz) : (const void *)(U + (int64_t)k * nz);
      s.strideX = ub;
      s.Z = U + (int64_t)(k + 1) * nz;
      s.strideZ = ub;
      RN_TRY(rn_launch_spgemm(ctx, pl, MODE_GM_STEP, s, batch, mixed));
#define GM_ORTH(NJ, PASS)                                                                                       \
  if (mixed)                                                                                                    \
    hipLaunchKernelGGL((k_gm_orth<NJ, PASS, true>), g2, blk, 0, ctx->stream, nz, ub, K, k, U, U32, part_ew,      \
                       p.scal, scal_stride, p.st);                                                              \
  else                                                                                                          \
    hipLaunchKernelGGL((k_gm_orth<NJ, PASS, false>), g2, blk, 0, ctx->stream, nz, ub, K, k, U, U32, part_ew,     \
                       p.scal, scal_stride, p.st);                                                              \
  LAUNCH_CHECK(ctx);
      if (k + 1 <= 16) {
        gm_orth_k<0, false>(k + 1, g2, blk, ctx->stream, nz, ub, K, k, U, U32, part_ew, p.scal, scal_stride, p.st);
        LAUNCH_CHECK(ctx);
      } else {
        GM_ORTH(65, 0);
      }
      hipLaunchKernelGGL(k_gm_fin<1>, dim3(k + 1, batch), blk, 0, ctx->stream, (int)gew, pstride_ew, part_ew, K, k,
                         p.scal, scal_stride, p.st, hist, hist_stride);
      LAUNCH_CHECK(ctx);
      if (k + 1 <= 16) {
        if (mixed) gm_orth_k<1, true>(k + 1, g2, blk, ctx->stream, nz, ub, K, k, U, U32, part_ew, p.scal, scal_stride, p.st);
        else gm_orth_k<1, false>(k + 1, g2, blk, ctx->stream, nz, ub, K, k, U, U32, part_ew, p.scal, scal_stride, p.st);
        LAUNCH_CHECK(ctx);
      } else {
        GM_ORTH(65, 1);
      }
      hipLaunchKernelGGL(k_gm_fin<2>, dim3(k + 1, batch), blk, 0, ctx->stream, (int)gew, pstride_ew, part_ew, K, k,
                         p.scal, scal_stride, p.st, hist, hist_stride);
      LAUNCH_CHECK(ctx);
      if (k + 1 <= 16) {
        if (mixed) gm_orth_k<2, true>(k + 1, g2, blk, ctx->stream, nz, ub, K, k, U, U32, part_ew, p.scal, scal_stride, p.st);
        else gm_orth_k<2, false>(k + 1, g2, blk, ctx->stream, nz, ub, K, k, U, U32, part_ew, p.scal, scal_stride, p.st);
        LAUNCH_CHECK(ctx);
      } else {
        GM_ORTH(65, 2);
      }
#undef GM_ORTH
      hipLaunchKernelGGL(k_gm_fin<3>, dim3(batch), blk, 0, ctx->stream, (int)gew, pstride_ew, part_ew, K, k, p.scal,
                         scal_stride, p.st, hist, hist_stride);
      LAUNCH_CHECK(ctx);
    }
    hipLaunchKernelGGL(k_gm_solve, dim3(batch), dim3(64), 0, ctx->stream, K, p.scal, scal_stride, p.st);
    LAUNCH_CHECK(ctx);
    switch (K) {
#define GM_C(KP)                                                                                                \
  case KP:                                                                                                      \
    hipLaunchKernelGGL(k_gm_combine_k<KP>, g2, blk, 0, ctx->stream, nz, ub, T, U, P, p.scal, scal_stride, p.st); \
    break;
      GM_C(1) GM_C(2) GM_C(3) GM_C(4) GM_C(5) GM_C(6) GM_C(7) GM_C(8)
      GM_C(9) GM_C(10) GM_C(11) GM_C(12) GM_C(13) GM_C(14) GM_C(15) GM_C(16)
#undef GM_C
      default:
        hipLaunchKernelGGL(k_gm_combine<65>, g2, blk, 0, ctx->stream, nz, ub, K, T, U, P, p.scal, scal_stride, p.st);
    }
    LAUNCH_CHECK(ctx);
  }
  // read back the device status of every batch entry and batch 0's scalars
  const size_t stb = (size_t)batch * ST_STRIDE * 4;
  const RnFetch it[3] = {{p.st, stb}, {p.scal, (size_t)scal_stride * 8}, {pl->d_terms, 8}};
  const unsigned char *hb = nullptr;
  size_t off[3];
  RN_TRY(rn_fetch(ctx, 3, it, &hb, off));
  const int32_t *hst = (const int32_t *)(hb + off[0]);
  const double *hsc = (const double *)(hb + off[1]);
  const unsigned long long *hterms = (const unsigned long long *)(hb + off[2]);
  rn_status res = RN_OK;
  int bad = -1;
  for (int b = 0; b < batch; ++b) {
    if (method == RN_PCG_JACOBI && hst[b * ST_STRIDE + ST_PREC]) {
      res = RN_ESINGULAR;
      bad = b;
      break;
    }
    if (hst[b * ST_STRIDE + ST_STATUS]) {
      res = (rn_status)hst[b * ST_STRIDE + ST_STATUS];
      bad = b;
      break;
    }
  }
  if (stats) {
    stats->energy = stats->proj_residual = stats->constraint_residual = NAN;
    stats->iters_done = hst[gm ? ST_KD : ST_ITERS];
    stats->rank_deficient_rows = pl->rank_def;
    stats->fused_cg = fuse ? 1 : 0;
    stats->status_code = hst[ST_STATUS];
    if (gm) {
      const GmLayout L(K);
      stats->first = hsc[SC_BETA0];
      stats->last = fabs(hsc[L.g + hst[ST_KD]]);
    } else {
      const CgLayout L(K);
      stats->first = hsc[SC_GAMMA0];
      stats->last = hsc[L.gam + hst[ST_ITERS]];
    }
    product_cost(pl, mixed, *hterms, &stats->spgemm_bytes, &stats->spgemm_flops);
    const double nprod = (double)(stats->iters_done + 1) * (method == RN_CGNR ? 2.0 : 1.0);
    stats->work_units = nprod * stats->spgemm_flops / (2.0 * (double)pl->nnzA * pl->m * pl->m);
  }
  // (not in an allocation-free call: the metrics use the context's scratch)
  if (stats && res == RN_OK && ctx->opt[RN_OPT_METRICS] && !pl->arena) {
    // E(P), ||Pi(A P)|| and max |(P - T) Bc| of batch entry 0 (one more
    // product, one synchronisation)
    double *part = (double *)rn_scratch(ctx, SLOT_MISC, (2 * METRIC_GRID + 4) * sizeof(double), &st);
    if (!part) return st;
    double *out = part + 2 * METRIC_GRID;
    RN_TRY(energy_launch(ctx, pl, A_vals, P, part, out));
    RN_TRY(cres_launch(ctx, pl->n, pl->Np, pl->Nj, P, T, pl->Bc, nullptr, pl->nB, part, out + 2));
    const RnFetch it2[1] = {{out, 3 * sizeof(double)}};
    const unsigned char *hb2 = nullptr;
    size_t off2[1];
    RN_TRY(rn_fetch(ctx, 1, it2, &hb2, off2));
    double v[3];
    memcpy(v, hb2 + off2[0], sizeof v);
    stats->energy = v[0];
    stats->proj_residual = sqrt(fmax(v[1], 0.0));
    stats->constraint_residual = v[2];
    stats->work_units += stats->spgemm_flops / (2.0 * (double)pl->nnzA * pl->m * pl->m);
  }
  if (res == RN_ESINGULAR)
    return rn_fail(ctx, res, "rn_energy_min: Jacobi preconditioner: a diagonal entry of A is not positive (batch "
                             "entry %d)", bad);
  if (res == RN_EBREAKDOWN)
    return rn_fail(ctx, res, "rn_energy_min: CG curvature <D, Pi(A D)> <= 0 (batch entry %d)", bad);
  if (res != RN_OK) return rn_fail(ctx, res, "rn_energy_min: non-finite Krylov scalar (batch entry %d)", bad);
  return RN_OK;
}
