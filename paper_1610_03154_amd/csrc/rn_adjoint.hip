// rn_adjoint.hip -- reverse mode of the CG energy minimisation: the map from
// the stored values of A to P after K CG steps (Sec. 3.6 improve, in the CG
// form of Sec. 4.1), differentiated through the recurrences with every
// stored a_ik an independent variable and pattern, T and Bc held fixed.
//
// Forward, with Q(X) = Pi(M(A X)):
//   R_0 = D_0 = -Q(T), gamma_0 = <R_0,R_0>; step k:
//   Z_k = Q(D_k), delta_k = <D_k,Z_k>, alpha_k = gamma_k/delta_k,
//   P_{k+1} = P_k + alpha_k D_k, R_{k+1} = R_k - alpha_k Z_k,
//   gamma_{k+1} = <R_{k+1},R_{k+1}>, beta_k = gamma_{k+1}/gamma_k,
//   D_{k+1} = R_{k+1} + beta_k D_k.
// Reverse step k (bars are adjoints, Pbar is the same at every step):
//   betabar_k  = <Dbar, D_k>,  gammabar_{k+1} += betabar_k / gamma_k,
//   Rbar      += Dbar + 2 gammabar_{k+1} R_{k+1},
//   alphabar_k = <Pbar, D_k> - <Rbar, Z_k>,
//   deltabar_k = -alphabar_k alpha_k / delta_k,
//   gammabar_k = alphabar_k / delta_k - betabar_k gamma_{k+1} / gamma_k^2,
//   Zbar       = deltabar_k D_k - alpha_k Rbar,
//   Dbar       = beta_k Dbar + alpha_k Pbar + deltabar_k Z_k + Q^T(Zbar),
//   Abar      += d<Zbar, Q(D_k)>/dA;
// and at the start: Abar += d<Ybar, Q(T)>/dA with
//   Ybar = -(Rbar + Dbar + 2 gammabar_0 R_0).
// Pi is an orthogonal projector row by row, so Q^T(Y) = M(A^T Pi(Y)) (the
// masked product on a plan of A^T, same pattern, no output projection), and
// d<Y, Q(X)>/dA_ik = sum over the pattern of row i of Pi(Y)_ij X_kj, which
// the product's position codes give directly.  The tape keeps R_k and D_k at
// the checkpoint steps k = 0, c, 2c, ... only, with Z_k = Q(D_k) there (the
// forward's product writes it into the tape); reverse step k recomputes
// from the checkpoint k0 <= k, with the recorded alpha_j and beta_j, Z_j =
// Q(D_j) (j > k0), R_{j+1} = R_j - alpha_j Z_j and D_{j+1} = R_{j+1} +
// beta_j D_j for j = k0..k (the forward's own expressions, so the same
// bits), which yields D_k, Z_k and R_{k+1}.
#include <cstring>
#include <new>
#include <type_traits>

#include "rn_emin.h"

struct rn_tape {
  rn_ctx *ctx = nullptr;  // owner of the device memory (NULL once released)
  const rn_plan *pl = nullptr;
  int32_t batch = 0, K = 0, scal_stride = 0;
  int32_t c = 1, ncp = 0;             // checkpoint interval and count (steps 0, c, ... < K)
  int64_t nz = 0, nzb = 0;
  double *R = nullptr, *D = nullptr;  // [ncp][batch][nz]
  double *Z = nullptr;                // [ncp][batch][nz]: Z_k = Q(D_k) at the checkpoints k < K
  double *W = nullptr;                // [4][batch][nz]: recomputed R and D, two of each
  double *T = nullptr;                // [nz]
  double *scal = nullptr;             // [batch][scal_stride], the forward CG scalars
  int32_t *st = nullptr;              // [batch][ST_STRIDE]
  // reverse-sweep workspace
  double *Rb = nullptr, *Db = nullptr, *Zk = nullptr, *Yb = nullptr, *Yh = nullptr;  // [batch][nz]
  double *gbar = nullptr;             // [batch][K+1]
  double *part = nullptr;             // [batch][RN_MAXDOT][ew blocks]
  double *ATv = nullptr;              // [batch][nnz(A)]
  int64_t nnzA = 0;
  bool recorded = false;
};

static unsigned adj_grid(int64_t n) {
  int64_t g = (n + 8 * RN_BLOCK - 1) / (8 * RN_BLOCK);
  if (g < 1) g = 1;
  if (g > 512) g = 512;
  return (unsigned)g;
}

// The tape's device memory back to its context (stream-ordered reuse: work
// queued on the context's stream that still reads it runs first).
void rn_tape_release(rn_tape *t) {
  if (!t->ctx) return;
  void **bufs[] = {(void **)&t->R,  (void **)&t->D,  (void **)&t->Z,  (void **)&t->W,  (void **)&t->T,  (void **)&t->scal, (void **)&t->st,
                   (void **)&t->Rb, (void **)&t->Db, (void **)&t->Zk, (void **)&t->Yb,   (void **)&t->Yh,
                   (void **)&t->gbar, (void **)&t->part, (void **)&t->ATv};
  for (void **b : bufs) {
    rn_dev_free(t->ctx, *b);
    *b = nullptr;
  }
  t->ctx = nullptr;
  t->recorded = false;
}

extern "C" void rn_tape_destroy(rn_tape *tape) {
  if (!tape) return;
  if (tape->ctx) {  // (a tape whose context was destroyed first holds no device memory)
    auto &v = tape->ctx->tapes;
    for (size_t q = 0; q < v.size(); ++q)
      if (v[q] == tape) {
        v[q] = v.back();
        v.pop_back();
        break;
      }
    rn_tape_release(tape);
  }
  delete tape;
}

extern "C" rn_status rn_tape_create(rn_ctx *ctx, rn_plan *pl, int32_t batch, int32_t iters, rn_tape **out) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (!out) return rn_fail(ctx, RN_EINVAL, "rn_tape_create: null argument");
  *out = nullptr;
  if (!pl || batch < 1 || iters < 0) return rn_fail(ctx, RN_EINVAL, "rn_tape_create: bad argument");
  if (pl->m != 1) return rn_fail(ctx, RN_EINVAL, "rn_tape_create: the adjoint takes scalar CSR operators (block_m = 1)");
  rn_tape *t = new (std::nothrow) rn_tape();
  if (!t) return rn_fail(ctx, RN_ENOMEM, "rn_tape_create: host allocation");
  try {
    ctx->tapes.push_back(t);
  } catch (...) {
    delete t;
    return rn_fail(ctx, RN_ENOMEM, "rn_tape_create: host allocation");
  }
  t->ctx = ctx;
  t->pl = pl;
  t->batch = batch;
  t->K = iters;
  t->nz = pl->nnzN;
  t->nzb = (int64_t)batch * pl->nnzN;
  t->nnzA = pl->nnzA;
  t->scal_stride = CgLayout(iters).total;
  int c = ctx->opt[RN_OPT_TAPE_INTERVAL];
  if (c <= 0)
    for (c = 1; c * c < iters; ++c) {
    }
  t->c = c;
  t->ncp = iters > 0 ? (iters + c - 1) / c : 1;
  const size_t v = (size_t)(t->nzb + 1) * 8;
  const size_t slots = (size_t)t->ncp * v;
  auto get = [&](auto **p, size_t bytes) {
    *p = (std::remove_reference_t<decltype(**p)> *)rn_dev_alloc(ctx, bytes);
    return *p != nullptr;
  };
  bool ok = get(&t->R, slots) && get(&t->D, slots) && get(&t->Z, slots) && get(&t->W, 4 * v) && get(&t->T, (size_t)(t->nz + 1) * 8) &&
            get(&t->scal, (size_t)batch * t->scal_stride * 8) && get(&t->st, (size_t)batch * ST_STRIDE * 4) &&
            get(&t->Rb, v) && get(&t->Db, v) && get(&t->Zk, v) && get(&t->Yb, v) && get(&t->Yh, v) &&
            get(&t->gbar, (size_t)batch * (iters + 1) * 8) &&
            get(&t->part, (size_t)batch * RN_MAXDOT * (adj_grid(t->nz) + 2) * 8) &&
            get(&t->ATv, (size_t)batch * (pl->nnzA + 1) * 8);
  if (!ok) {
    rn_tape_destroy(t);
    return rn_fail(ctx, RN_ENOMEM, "rn_tape_create: device allocation (%zu bytes of iterates)", 3 * slots);
  }
  *out = t;
  return RN_OK;
}

rn_status rn_tape_record_begin(rn_ctx *ctx, rn_plan *pl, rn_tape *tape, int32_t batch, int32_t iters,
                               rn_method method, rn_precision prec, const double *T) {
  if (method != RN_CG || prec != RN_FP64)
    return rn_fail(ctx, RN_EINVAL, "rn_energy_min: a tape records the FP64 CG form only");
  if (!tape->ctx) return rn_fail(ctx, RN_EINVAL, "rn_energy_min: the tape's context was destroyed");
  if (tape->pl != pl || tape->batch != batch || tape->K != iters)
    return rn_fail(ctx, RN_EINVAL, "rn_energy_min: tape made for another plan, batch or iteration count");
  tape->recorded = false;
  HIP_TRY(ctx, hipMemcpyAsync(tape->T, T, (size_t)tape->nz * 8, hipMemcpyDeviceToDevice, ctx->stream));
  return RN_OK;
}

double *rn_tape_R(rn_tape *tape, int k) {
  return (k % tape->c == 0 && (k < tape->K || k == 0)) ? tape->R + (int64_t)(k / tape->c) * tape->nzb : nullptr;
}
double *rn_tape_D(rn_tape *tape, int k) {
  return (k % tape->c == 0 && (k < tape->K || k == 0)) ? tape->D + (int64_t)(k / tape->c) * tape->nzb : nullptr;
}
double *rn_tape_Z(rn_tape *tape, int k) {
  return (k % tape->c == 0 && k < tape->K) ? tape->Z + (int64_t)(k / tape->c) * tape->nzb : nullptr;
}

rn_status rn_tape_record_end(rn_ctx *ctx, rn_tape *tape, const double *scal, const int32_t *st, int32_t batch) {
  HIP_TRY(ctx, hipMemcpyAsync(tape->scal, scal, (size_t)batch * tape->scal_stride * 8, hipMemcpyDeviceToDevice,
                              ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(tape->st, st, (size_t)batch * ST_STRIDE * 4, hipMemcpyDeviceToDevice, ctx->stream));
  tape->recorded = true;
  return RN_OK;
}

// ---------------------------------------------------------------------------
// reverse-sweep kernels; grid.y = batch entry, a batch entry whose forward
// stopped before step k skips step k
// ---------------------------------------------------------------------------
__device__ inline bool adj_active(const int32_t *tst, int b, int k) {
  const int32_t *st = tst + (int64_t)b * ST_STRIDE;
  return st[ST_STATUS] == 0 && k < st[ST_ITERS];
}

// The last recomputation step of reverse step k: R_{k+1} = R_k - alpha_k Z_k
// (the forward's expression), and over the same entries the partials of
// <Dbar,D_k>, <Pbar,D_k>, <Rbar,Z_k>, <Dbar,Z_k>, <R_{k+1},Z_k>
__global__ __launch_bounds__(RN_BLOCK) void k_adj_refwd_dots(int64_t nz, int K, int k,
                                                            const double *__restrict__ Rk,
                                                            const double *__restrict__ Dk,
                                                            const double *__restrict__ Zk, double *__restrict__ R1,
                                                            const double *__restrict__ tscal, int scal_stride,
                                                            const double *__restrict__ Db,
                                                            const double *__restrict__ Pb,
                                                            const double *__restrict__ Rb, double *__restrict__ part,
                                                            const int32_t *__restrict__ tst) {
  __shared__ double s_w[8];
  const int b = blockIdx.y;
  if (!adj_active(tst, b, k)) return;
  const CgLayout L(K);
  const double al = tscal[(int64_t)b * scal_stride + L.alp + k];
  const int64_t off = (int64_t)b * nz;
  RnAcc a[5];
  for (int64_t e = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; e < nz; e += (int64_t)gridDim.x * RN_BLOCK) {
    const double db = Db[off + e], dk = Dk[off + e], z = Zk[off + e];
    const double rr = Rk[off + e] - al * z;
    R1[off + e] = rr;
    a[0].add(db * dk);
    a[1].add(Pb[off + e] * dk);
    a[2].add(Rb[off + e] * z);
    a[3].add(db * z);
    a[4].add(rr * z);
  }
  double *pb = part + (int64_t)b * RN_MAXDOT * gridDim.x;
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const double S = rn_block_sum2(a[j].hi, a[j].lo, s_w);
    if (threadIdx.x == 0) pb[(int64_t)j * gridDim.x + blockIdx.x] = S;
  }
}

// Every block sums the partials itself (same fixed order, same scalars),
// block 0 stores gammabar_k; then the element-wise updates of Rbar, Zbar
// (into Yb) and the first part of Dbar.
__global__ __launch_bounds__(RN_BLOCK) void k_adj_update(int64_t nz, int K, int k, int nb,
                                                        const double *__restrict__ part,
                                                        const double *__restrict__ tscal, int scal_stride,
                                                        const int32_t *__restrict__ tst, double *__restrict__ gbar,
                                                        double *__restrict__ Rb, double *__restrict__ Db,
                                                        const double *__restrict__ Pb,
                                                        const double *__restrict__ R1, const double *__restrict__ Dk,
                                                        const double *__restrict__ Zk, double *__restrict__ Yb) {
  __shared__ double s_w[8];
  const int b = blockIdx.y;
  if (!adj_active(tst, b, k)) return;
  const double *pb = part + (int64_t)b * RN_MAXDOT * nb;
  double d[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) d[j] = rn_reduce_part(pb + (int64_t)j * nb, nb, s_w);
  const double *sc = tscal + (int64_t)b * scal_stride;
  const CgLayout L(K);
  const double gk = sc[L.gam + k], gk1 = sc[L.gam + k + 1], dl = sc[L.del + k], al = sc[L.alp + k],
               be = sc[L.bet + k];
  double *gb = gbar + (int64_t)b * (K + 1);
  const double betabar = d[0];
  const double gb1 = gb[k + 1] + betabar / gk;  // final gammabar_{k+1}
  const double c = 2.0 * gb1;
  const double rz = d[2] + d[3] + c * d[4];     // <Rbar + Dbar + c R_{k+1}, Z_k>
  const double alphabar = d[1] - rz;
  const double deltabar = -alphabar * al / dl;
  if (blockIdx.x == 0 && threadIdx.x == 0) gb[k] = alphabar / dl - betabar * gk1 / (gk * gk);
  const int64_t off = (int64_t)b * nz;
  for (int64_t e = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; e < nz; e += (int64_t)gridDim.x * RN_BLOCK) {
    const double db = Db[off + e], dk = Dk[off + e];
    const double rb = Rb[off + e] + db + c * R1[off + e];
    Rb[off + e] = rb;
    Yb[off + e] = deltabar * dk - al * rb;
    Db[off + e] = be * db + al * Pb[off + e] + deltabar * Zk[off + e];
  }
}

// Ybar = -(Rbar + Dbar + 2 gammabar_0 R_0): the adjoint of R_0 = -Q(T) (every
// batch entry, also those whose forward did no step)
__global__ __launch_bounds__(RN_BLOCK) void k_adj_init(int64_t nz, int K, const double *__restrict__ gbar,
                                                      const double *__restrict__ Rb, const double *__restrict__ Db,
                                                      const double *__restrict__ R0, double *__restrict__ Yb,
                                                      const int32_t *__restrict__ tst) {
  const int b = blockIdx.y;
  const int64_t off = (int64_t)b * nz;
  if (tst[(int64_t)b * ST_STRIDE + ST_STATUS]) return;
  const double c = 2.0 * gbar[(int64_t)b * (K + 1)];
  for (int64_t e = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; e < nz; e += (int64_t)gridDim.x * RN_BLOCK)
    Yb[off + e] = -(Rb[off + e] + Db[off + e] + c * R0[off + e]);
}

// One forward step of the recomputation from a checkpoint: R_{j+1} = R_j -
// alpha_j Z_j and D_{j+1} = R_{j+1} + beta_j D_j, with the recorded scalars
// and the forward kernels' expressions
__global__ __launch_bounds__(RN_BLOCK) void k_adj_refwd(int64_t nz, int K, int j,
                                                       const double *__restrict__ Rj, const double *__restrict__ Dj,
                                                       const double *__restrict__ Zj, double *__restrict__ Rn,
                                                       double *__restrict__ Dn, const double *__restrict__ tscal,
                                                       int scal_stride, const int32_t *__restrict__ tst) {
  const int b = blockIdx.y;
  if (!adj_active(tst, b, j)) return;
  const CgLayout L(K);
  const double *sc = tscal + (int64_t)b * scal_stride;
  const double al = sc[L.alp + j], be = sc[L.bet + j];
  const int64_t off = (int64_t)b * nz;
  for (int64_t e = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; e < nz; e += (int64_t)gridDim.x * RN_BLOCK) {
    const double rr = Rj[off + e] - al * Zj[off + e];
    Rn[off + e] = rr;
    Dn[off + e] = rr + be * Dj[off + e];
  }
}

// Yh = Pi(Yb): one thread per DOF row, the same arithmetic as the product's
// projection (row sums in pattern order, then the packed G^+); root rows 0.
template <int NB>
__global__ __launch_bounds__(RN_BLOCK) void k_adj_project(int n, int64_t nz, int k, const int32_t *__restrict__ Np,
                                                         const int32_t *__restrict__ Nj,
                                                         const uint8_t *__restrict__ is_root,
                                                         const double *__restrict__ Bc, const double *__restrict__ gp,
                                                         const double *__restrict__ Yb, double *__restrict__ Yh,
                                                         const int32_t *__restrict__ tst) {
  constexpr int NP = NB * (NB + 1) / 2;
  const int b = blockIdx.y;
  if (k >= 0 && !adj_active(tst, b, k)) return;
  if (k < 0 && tst[(int64_t)b * ST_STRIDE + ST_STATUS]) return;
  const int i = blockIdx.x * RN_BLOCK + threadIdx.x;
  if (i >= n) return;
  const int64_t off = (int64_t)b * nz;
  const int s = Np[i], e = Np[i + 1];
  if (is_root[i]) {
    for (int r = s; r < e; ++r) Yh[off + r] = 0.0;
    return;
  }
  double sv[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) sv[q] = 0.0;
  for (int r = s; r < e; ++r) {
    const double y = Yb[off + r];
#pragma unroll
    for (int q = 0; q < NB; ++q) sv[q] += y * Bc[(int64_t)Nj[r] * NB + q];
  }
  double w[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    w[q] = 0.0;
#pragma unroll
    for (int r2 = 0; r2 < NB; ++r2) w[q] += gp[(int64_t)i * NP + rn_pk(NB, q, r2)] * sv[r2];
  }
  for (int r = s; r < e; ++r) {
    double u = 0.0;
#pragma unroll
    for (int q = 0; q < NB; ++q) u += Bc[(int64_t)Nj[r] * NB + q] * w[q];
    Yh[off + r] = Yb[off + r] - u;
  }
}

// The same projection entry-parallel over the product's blocks (scalar
// operators, n_B <= 2, the plan's per-entry Bc rows): one lane per pattern
// entry; the products y_r Bc[j_r] go through LDS and every lane sums its row's
// in pattern order, exactly as k_adj_project does.
template <int NB>
__global__ __launch_bounds__(RN_BLOCK) void k_adj_project_b(int nblk, int64_t nz, int k, const int32_t *__restrict__ hdr,
                                                           const int32_t *__restrict__ Np,
                                                           const uint8_t *__restrict__ is_root,
                                                           const uint8_t *__restrict__ codes, int cstride,
                                                           const double *__restrict__ bce,
                                                           const double *__restrict__ gp,
                                                           const double *__restrict__ Yb, double *__restrict__ Yh,
                                                           const int32_t *__restrict__ tst) {
  constexpr int NP = NB * (NB + 1) / 2;
  __shared__ int s_rp[RN_BLOCK + 1];
  __shared__ uint8_t s_root[RN_BLOCK];
  __shared__ double s_red[NB][RN_BLOCK];
  const int b = blockIdx.y, t = threadIdx.x;
  if (k >= 0 && !adj_active(tst, b, k)) return;
  if (k < 0 && tst[(int64_t)b * ST_STRIDE + ST_STATUS]) return;
  const int blk = rn_xcd_block(blockIdx.x, nblk);
  if (blk < 0) return;
  const int4 h0 = ((const int4 *)hdr)[2 * blk];
  const int r0 = h0.x, nrows = h0.y - h0.x, e0 = h0.z, ne = h0.w - h0.z;
  const int64_t off = (int64_t)b * nz;
  const bool valid = t < ne;
  const int e = valid ? e0 + t : (ne > 0 ? e0 : 0);  // idle lanes read a valid entry
  const double y = Yb[off + e];
  const int lrow = valid ? codes[(int64_t)e * cstride] : 0;  // record byte 0: the row within the block
  double bc[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) bc[q] = bce[(int64_t)e * NB + q];
  if (t <= nrows) s_rp[t] = Np[r0 + t] - e0;
  if (t < nrows) s_root[t] = is_root[r0 + t];
  if (nrows == RN_BLOCK && t == 0) s_rp[RN_BLOCK] = ne;
  if (valid)
#pragma unroll
    for (int q = 0; q < NB; ++q) s_red[q][t] = y * bc[q];
  __syncthreads();
  if (!valid) return;
  const int i = r0 + lrow;
  if (s_root[lrow]) {
    Yh[off + e] = 0.0;
    return;
  }
  double sv[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) sv[q] = 0.0;
  for (int r = s_rp[lrow]; r < s_rp[lrow + 1]; ++r)
#pragma unroll
    for (int q = 0; q < NB; ++q) sv[q] += s_red[q][r];
  double w[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    w[q] = 0.0;
#pragma unroll
    for (int r2 = 0; r2 < NB; ++r2) w[q] += gp[(int64_t)i * NP + rn_pk(NB, q, r2)] * sv[r2];
  }
  double u = 0.0;
#pragma unroll
  for (int q = 0; q < NB; ++q) u += bc[q] * w[q];
  Yh[off + e] = y - u;
}

// Abar_ik += sum over the pattern entries r of row i of Yh_r X[k, j_r]
// (X = D_k, or T for the start term).  Organised by the product's blocks:
// block b owns the stored A entries of its rows, one thread per entry; the
// entry's row comes from the block's A row starts in LDS, and the position
// codes of the row's pattern entries locate j_r in row k.  Root rows get no
// contribution (Q is zero there).
__global__ __launch_bounds__(RN_BLOCK) void k_adj_sddmm(int nblk, int64_t nz, int64_t nnzA, int64_t strideX, int k,
                                                       const int32_t *__restrict__ hdr,
                                                       const int32_t *__restrict__ Ap,
                                                       const int32_t *__restrict__ Np,
                                                       const uint8_t *__restrict__ is_root,
                                                       const uint8_t *__restrict__ codes, int cstride,
                                                       const int32_t *__restrict__ xoff,
                                                       const double *__restrict__ Yh, const double *__restrict__ X,
                                                       double *__restrict__ Abar, const int32_t *__restrict__ tst) {
  __shared__ int s_ap[RN_BLOCK + 1];
  const int b = blockIdx.y;
  if (k >= 0 && !adj_active(tst, b, k)) return;
  if (k < 0 && tst[(int64_t)b * ST_STRIDE + ST_STATUS]) return;
  const int blk = rn_xcd_block(blockIdx.x, nblk);
  if (blk < 0) return;
  const int4 h0 = ((const int4 *)hdr)[2 * blk];
  const int4 h1 = ((const int4 *)hdr)[2 * blk + 1];
  const int r0 = h0.x, nrows = h0.y - h0.x, a0 = h1.x, na = h1.y - h1.x;
  for (int rr = threadIdx.x; rr <= nrows; rr += RN_BLOCK) s_ap[rr] = Ap[r0 + rr] - a0;
  __syncthreads();
  const double *y = Yh + (int64_t)b * nz;
  const double *x = X + (int64_t)b * strideX;
  double *ab = Abar + (int64_t)b * nnzA;
  for (int q = threadIdx.x; q < na; q += RN_BLOCK) {
    int lo = 0, hi = nrows;  // row: the largest rr with s_ap[rr] <= q
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_ap[mid] <= q) lo = mid; else hi = mid;
    }
    const int i = r0 + lo;
    if (is_root[i]) continue;
    const int u = q - s_ap[lo];
    const int xo = xoff[a0 + q];
    double acc = 0.0;
    for (int r = Np[i]; r < Np[i + 1]; ++r) {
      const uint32_t c = codes[(int64_t)r * cstride + 1 + u];  // byte 0 is the row
      if (c != CODE_NONE) acc += y[r] * x[xo + (int)c];
    }
    ab[a0 + q] += acc;
  }
}

// The same sum for scalar operators with records of at most 16 bytes, with
// the block's data staged in LDS by contiguous loads: the pattern values Yh
// and position records of its entries, its row starts, and the block's X
// window (the neighbour rows' pattern entries; blocks without a window read X
// from global memory).  Each A entry then reads only LDS; the sum runs over
// the row's pattern entries in the same order as k_adj_sddmm.
#define SD_REC 4  // record words staged per entry
__global__ __launch_bounds__(RN_BLOCK) void k_adj_sddmm_w(int nblk, int64_t nz, int64_t nnzA, int64_t strideX, int k,
                                                         const int32_t *__restrict__ hdr,
                                                         const int32_t *__restrict__ Ap,
                                                         const int32_t *__restrict__ Np,
                                                         const uint8_t *__restrict__ is_root,
                                                         const uint8_t *__restrict__ codes, int cstride,
                                                         const int32_t *__restrict__ xoff,
                                                         const int32_t *__restrict__ xl,
                                                         const int32_t *__restrict__ xwin, int nu,
                                                         const double *__restrict__ Yh, const double *__restrict__ X,
                                                         double *__restrict__ Abar, const int32_t *__restrict__ tst) {
  __shared__ int s_ap[RN_BLOCK + 1];
  __shared__ int s_rp[RN_BLOCK + 1];
  __shared__ uint8_t s_root[RN_BLOCK];
  __shared__ double s_y[RN_BLOCK];
  __shared__ uint32_t s_rec[RN_BLOCK * SD_REC];
  __shared__ double s_xw[SPG_XCAP_M1(RN_BLOCK)];
  __shared__ uint8_t s_arow[SPG_ACAP_M1(RN_BLOCK)];  // row of each staged A entry
  const int b = blockIdx.y, t = threadIdx.x;
  if (k >= 0 && !adj_active(tst, b, k)) return;
  if (k < 0 && tst[(int64_t)b * ST_STRIDE + ST_STATUS]) return;
  const int blk = rn_xcd_block(blockIdx.x, nblk);
  if (blk < 0) return;
  // the window's unit starts depend on the block alone: they load with the header
  const int32_t *uw = xwin + (int64_t)blk * nu;
  int uwv[SPG_XCAP_M1(RN_BLOCK) / RN_BLOCK];
#pragma unroll
  for (int i = 0; i < SPG_XCAP_M1(RN_BLOCK) / RN_BLOCK; ++i) uwv[i] = uw[(t + i * RN_BLOCK) / XW_UNIT];
  const int4 h0 = ((const int4 *)hdr)[2 * blk];
  const int4 h1 = ((const int4 *)hdr)[2 * blk + 1];
  const int r0 = h0.x, nrows = h0.y - h0.x, e0 = h0.z, ne = h0.w - h0.z, a0 = h1.x, na = h1.y - h1.x;
  const int nunit = h1.w;
  const bool byrow = na <= SPG_ACAP_M1(RN_BLOCK);  // uniform: A entries find their row in LDS
  const double *y = Yh + (int64_t)b * nz;
  const double *x = X + (int64_t)b * strideX;
  double *ab = Abar + (int64_t)b * nnzA;
  const int nw = cstride >> 2;
  // one round of loads that depend on the header only (row starts and root
  // flags, the entries' Yh and records, the window, and for this lane's A
  // entries their neighbour-row offsets and the Abar values they add to),
  // then the LDS stores
  constexpr int NAQ = SPG_ACAP_M1(RN_BLOCK) / RN_BLOCK;  // A entries per lane when they find their row in LDS
  const int tr = t < nrows ? t : nrows;
  const int v_ap = Ap[r0 + tr] - a0, v_rp = Np[r0 + tr] - e0;
  const uint8_t v_root = t < nrows ? is_root[r0 + t] : (uint8_t)0;
  int v_ap2 = 0, v_rp2 = 0;
  if (t == 0 && nrows == RN_BLOCK) {  // the end of the last row
    v_ap2 = Ap[r0 + RN_BLOCK] - a0;
    v_rp2 = Np[r0 + RN_BLOCK] - e0;
  }
  const double v_y = t < ne ? y[e0 + t] : 0.0;
  const uint32_t *cw = (const uint32_t *)codes + (int64_t)e0 * nw;
  uint32_t v_rec[SD_REC];
#pragma unroll
  for (int i = 0; i < SD_REC; ++i) {
    const int q = t + i * RN_BLOCK;
    v_rec[i] = q < ne * nw ? cw[q] : 0u;
  }
  double v_xw[SPG_XCAP_M1(RN_BLOCK) / RN_BLOCK];
#pragma unroll
  for (int i = 0; i < SPG_XCAP_M1(RN_BLOCK) / RN_BLOCK; ++i) {
    const int q = t + i * RN_BLOCK;
    v_xw[i] = (nunit > 0 && q < nunit * XW_UNIT) ? x[uwv[i] + q % XW_UNIT] : 0.0;
  }
  int v_xo[NAQ];
  double v_ab[NAQ];
#pragma unroll
  for (int i = 0; i < NAQ; ++i) {
    const int q = t + i * RN_BLOCK;
    v_xo[i] = 0;
    v_ab[i] = 0.0;
    if (q < na) {
      v_xo[i] = nunit > 0 ? xl[a0 + q] : xoff[a0 + q];
      v_ab[i] = ab[a0 + q];
    }
  }
  if (t <= nrows) {
    s_ap[t] = v_ap;
    s_rp[t] = v_rp;
  }
  if (t < nrows) s_root[t] = v_root;
  if (t == 0 && nrows == RN_BLOCK) {
    s_ap[RN_BLOCK] = v_ap2;
    s_rp[RN_BLOCK] = v_rp2;
  }
  if (t < ne) s_y[t] = v_y;
#pragma unroll
  for (int i = 0; i < SD_REC; ++i) {
    const int q = t + i * RN_BLOCK;
    if (q < ne * nw) s_rec[(q / nw) * SD_REC + q % nw] = v_rec[i];
  }
  if (nunit > 0) {
#pragma unroll
    for (int i = 0; i < SPG_XCAP_M1(RN_BLOCK) / RN_BLOCK; ++i) {
      const int q = t + i * RN_BLOCK;
      if (q < nunit * XW_UNIT) s_xw[q] = v_xw[i];
    }
  }
  __syncthreads();
  if (byrow)
    for (int rr = t; rr < nrows; rr += RN_BLOCK)
      for (int q = s_ap[rr]; q < s_ap[rr + 1]; ++q) s_arow[q] = (uint8_t)rr;
  __syncthreads();
  // the block row of A entry q
  auto row_of = [&](const int q) -> int {
    if (byrow) return s_arow[q];
    int lo = 0, hi = nrows;  // the largest rr with s_ap[rr] <= q
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_ap[mid] <= q) lo = mid; else hi = mid;
    }
    return lo;
  };
  // the sum of A entry q (in row lo) over the row's pattern entries, in pattern order
  auto entry = [&](const int q, const int lo, const int xo) -> double {
    const int u = q - s_ap[lo];
    const int pb = u + 1;  // byte of the code in each record
    const uint32_t *rec = s_rec + (pb >> 2);
    const int sh = 8 * (pb & 3);
    double acc = 0.0;
    if (nunit > 0) {
      for (int r = s_rp[lo]; r < s_rp[lo + 1]; ++r) {
        const uint32_t c = (rec[r * SD_REC] >> sh) & 0xffu;
        if (c != CODE_NONE) acc += s_y[r] * s_xw[xo + (int)c];
      }
    } else {
      for (int r = s_rp[lo]; r < s_rp[lo + 1]; ++r) {
        const uint32_t c = (rec[r * SD_REC] >> sh) & 0xffu;
        if (c != CODE_NONE) acc += s_y[r] * x[xo + (int)c];
      }
    }
    return acc;
  };
  // root rows get no contribution: their Abar entries are not written
#pragma unroll
  for (int i = 0; i < NAQ; ++i) {
    const int q = t + i * RN_BLOCK;
    if (q < na) {
      const int lo = row_of(q);
      if (!s_root[lo]) ab[a0 + q] = v_ab[i] + entry(q, lo, v_xo[i]);
    }
  }
  // blocks with more A entries than that: the rest one at a time
  for (int q = t + NAQ * RN_BLOCK; q < na; q += RN_BLOCK) {
    const int lo = row_of(q);
    if (s_root[lo]) continue;
    const double acc = entry(q, lo, nunit > 0 ? xl[a0 + q] : xoff[a0 + q]);
    ab[a0 + q] += acc;
  }
}

__global__ __launch_bounds__(RN_BLOCK) void k_adj_gather(const double *__restrict__ src, const int32_t *__restrict__ perm,
                                                        int64_t n, double *__restrict__ dst) {
  const int b = blockIdx.y;
  for (int64_t q = (int64_t)blockIdx.x * RN_BLOCK + threadIdx.x; q < n; q += (int64_t)gridDim.x * RN_BLOCK)
    dst[(int64_t)b * n + q] = src[(int64_t)b * n + perm[q]];
}

static rn_status adj_project(rn_ctx *ctx, const rn_plan *pl, int k, rn_tape *t) {
  if (pl->m == 1 && pl->bs == RN_BLOCK && pl->bce && pl->nB <= 2) {
    if (pl->nblk == 0) return RN_OK;
    const dim3 gb(rn_xcd_grid((unsigned)pl->nblk), (unsigned)t->batch), bb(RN_BLOCK);
    if (pl->nB == 1)
      hipLaunchKernelGGL(k_adj_project_b<1>, gb, bb, 0, ctx->stream, pl->nblk, t->nz, k, pl->blk_hdr, pl->Np,
                         pl->is_root, pl->codes, pl->cstride, pl->bce, pl->gp, t->Yb, t->Yh, t->st);
    else
      hipLaunchKernelGGL(k_adj_project_b<2>, gb, bb, 0, ctx->stream, pl->nblk, t->nz, k, pl->blk_hdr, pl->Np,
                         pl->is_root, pl->codes, pl->cstride, pl->bce, pl->gp, t->Yb, t->Yh, t->st);
    LAUNCH_CHECK(ctx);
    return RN_OK;
  }
  const dim3 g(rn_div_up(pl->n > 0 ? pl->n : 1, RN_BLOCK), (unsigned)t->batch), bl(RN_BLOCK);
  switch (pl->nB) {
    case 1: hipLaunchKernelGGL(k_adj_project<1>, g, bl, 0, ctx->stream, pl->n, t->nz, k, pl->Np, pl->Nj, pl->is_root, pl->Bc, pl->gp, t->Yb, t->Yh, t->st); break;
    case 2: hipLaunchKernelGGL(k_adj_project<2>, g, bl, 0, ctx->stream, pl->n, t->nz, k, pl->Np, pl->Nj, pl->is_root, pl->Bc, pl->gp, t->Yb, t->Yh, t->st); break;
    case 3: hipLaunchKernelGGL(k_adj_project<3>, g, bl, 0, ctx->stream, pl->n, t->nz, k, pl->Np, pl->Nj, pl->is_root, pl->Bc, pl->gp, t->Yb, t->Yh, t->st); break;
    case 4: hipLaunchKernelGGL(k_adj_project<4>, g, bl, 0, ctx->stream, pl->n, t->nz, k, pl->Np, pl->Nj, pl->is_root, pl->Bc, pl->gp, t->Yb, t->Yh, t->st); break;
    default: return rn_fail(ctx, RN_EINVAL, "nB out of range");
  }
  LAUNCH_CHECK(ctx);
  return RN_OK;
}

static rn_status adj_sddmm(rn_ctx *ctx, const rn_plan *pl, int k, rn_tape *t, const double *X, int64_t strideX,
                           double *A_bar) {
  if (pl->nblk == 0) return RN_OK;
  const dim3 g(rn_xcd_grid((unsigned)pl->nblk), (unsigned)t->batch), bl(RN_BLOCK);
  if (pl->m == 1 && pl->bs == RN_BLOCK && pl->cstride <= 4 * SD_REC && pl->xl && pl->xwin)
    hipLaunchKernelGGL(k_adj_sddmm_w, g, bl, 0, ctx->stream, pl->nblk, t->nz, pl->nnzA, strideX, k, pl->blk_hdr,
                       pl->Ap, pl->Np, pl->is_root, pl->codes, pl->cstride, pl->xoff, pl->xl, pl->xwin,
                       SPG_XCAP_M1(RN_BLOCK) / XW_UNIT, t->Yh, X, A_bar, t->st);
  else
    hipLaunchKernelGGL(k_adj_sddmm, g, bl, 0, ctx->stream, pl->nblk, t->nz, pl->nnzA, strideX, k, pl->blk_hdr,
                       pl->Ap, pl->Np, pl->is_root, pl->codes, pl->cstride, pl->xoff, t->Yh, X, A_bar, t->st);
  LAUNCH_CHECK(ctx);
  return RN_OK;
}

extern "C" rn_status rn_energy_min_bwd(rn_ctx *ctx, rn_plan *pl, rn_plan *plT, const int32_t *perm, rn_tape *t,
                                       const double *A_vals, const double *P_bar, double *A_bar) {
  if (!ctx) return RN_EINVAL;
  ctx->err.clear();
  if (!pl || !plT || !t || !A_vals || !P_bar || !A_bar || (pl->nnzA > 0 && !perm))
    return rn_fail(ctx, RN_EINVAL, "rn_energy_min_bwd: null argument");
  if (!t->recorded || t->pl != pl)
    return rn_fail(ctx, RN_EINVAL, "rn_energy_min_bwd: the tape holds no forward run of this plan");
  if (pl->m != 1 || plT->m != 1 || plT->n != pl->n || plT->nnzN != pl->nnzN || plT->nnzA != pl->nnzA ||
      plT->nB != pl->nB)
    return rn_fail(ctx, RN_EINVAL, "rn_energy_min_bwd: plan_T does not match plan (A^T with the same pattern)");
  const int B = t->batch, K = t->K;
  const int64_t nz = t->nz;
  // the forward's status and step count of every batch entry
  const size_t stb = (size_t)B * ST_STRIDE * 4;
  const RnFetch it[1] = {{t->st, stb}};
  const unsigned char *hb = nullptr;
  size_t off[1];
  RN_TRY(rn_fetch(ctx, 1, it, &hb, off));
  const void *hbuf = hb + off[0];
  int kmax = 0, bad = -1;
  for (int b = 0; b < B; ++b) {
    const int32_t *s = (const int32_t *)hbuf + b * ST_STRIDE;
    if (s[ST_STATUS]) bad = b;
    kmax = s[ST_ITERS] > kmax ? s[ST_ITERS] : kmax;
  }
  if (bad >= 0) return rn_fail(ctx, RN_EINVAL, "rn_energy_min_bwd: the forward run failed (batch entry %d)", bad);
  const size_t vb = (size_t)t->nzb * 8;
  HIP_TRY(ctx, hipMemsetAsync(t->Rb, 0, vb, ctx->stream));
  HIP_TRY(ctx, hipMemsetAsync(t->Db, 0, vb, ctx->stream));
  HIP_TRY(ctx, hipMemsetAsync(t->gbar, 0, (size_t)B * (K + 1) * 8, ctx->stream));
  HIP_TRY(ctx, hipMemsetAsync(A_bar, 0, (size_t)B * pl->nnzA * 8, ctx->stream));
  const unsigned ge = adj_grid(nz);
  const dim3 g2(ge, (unsigned)B), bl(RN_BLOCK);
  if (pl->nnzA > 0) {
    hipLaunchKernelGGL(k_adj_gather, dim3(adj_grid(pl->nnzA), (unsigned)B), bl, 0, ctx->stream, A_vals, perm,
                       pl->nnzA, t->ATv);
    LAUNCH_CHECK(ctx);
  }
  double *Wv[4];
  for (int i = 0; i < 4; ++i) Wv[i] = t->W + (int64_t)i * t->nzb;
  for (int k = kmax - 1; k >= 0; --k) {
    // D_k, Z_k = Q(D_k) and R_{k+1} from the checkpoint k0 <= k (a batch
    // entry that stopped before step j skips it, as in every kernel below)
    const int k0 = (k / t->c) * t->c;
    const double *Dj = rn_tape_D(t, k0), *Rj = rn_tape_R(t, k0);
    const double *Dk = nullptr, *R1 = nullptr, *Zk = nullptr;
    for (int j = k0; j <= k; ++j) {
      const double *Zj = t->Zk;
      if (j == k0) {
        Zj = rn_tape_Z(t, k0);  // the forward's own Z_{k0}
      } else {
        SpgParams q = rn_spg_params(pl);
        q.Ax = A_vals;
        q.X = Dj;
        q.Z = t->Zk;
        q.project = 1;
        q.st = t->st;
        q.kact = j;
        RN_TRY(rn_launch_spgemm(ctx, pl, MODE_PRODUCT, q, B, false));
      }
      // next iterates into the work vectors not holding R_j, D_j; the last
      // step (R_{k+1} only) also leaves the partials of step k's five dots
      double *Rn = Wv[2 * ((j - k0) & 1)], *Dn = Wv[2 * ((j - k0) & 1) + 1];
      if (j < k)
        hipLaunchKernelGGL(k_adj_refwd, g2, bl, 0, ctx->stream, nz, K, j, Rj, Dj, Zj, Rn, Dn, t->scal,
                           t->scal_stride, t->st);
      else
        hipLaunchKernelGGL(k_adj_refwd_dots, g2, bl, 0, ctx->stream, nz, K, k, Rj, Dj, Zj, Rn, t->scal,
                           t->scal_stride, t->Db, P_bar, t->Rb, t->part, t->st);
      LAUNCH_CHECK(ctx);
      if (j == k) {
        Dk = Dj;
        R1 = Rn;
        Zk = Zj;
      } else {
        Rj = Rn;
        Dj = Dn;
      }
    }
    hipLaunchKernelGGL(k_adj_update, g2, bl, 0, ctx->stream, nz, K, k, (int)ge, t->part, t->scal, t->scal_stride,
                       t->st, t->gbar, t->Rb, t->Db, P_bar, R1, Dk, Zk, t->Yb);
    LAUNCH_CHECK(ctx);
    RN_TRY(adj_project(ctx, pl, k, t));
    // Dbar += M(A^T Pi(Zbar))
    SpgParams r = rn_spg_params(plT);
    r.Ax = t->ATv;
    r.X = t->Yh;
    r.Z = t->Db;
    r.project = 0;
    r.accum = 1;
    r.st = t->st;
    r.kact = k;
    RN_TRY(rn_launch_spgemm(ctx, plT, MODE_PRODUCT, r, B, false));
    RN_TRY(adj_sddmm(ctx, pl, k, t, Dk, nz, A_bar));
  }
  hipLaunchKernelGGL(k_adj_init, g2, bl, 0, ctx->stream, nz, K, t->gbar, t->Rb, t->Db, rn_tape_R(t, 0), t->Yb, t->st);
  LAUNCH_CHECK(ctx);
  RN_TRY(adj_project(ctx, pl, -1, t));
  RN_TRY(adj_sddmm(ctx, pl, -1, t, t->T, 0, A_bar));
  return RN_OK;
}
