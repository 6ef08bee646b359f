// rn_gram.h -- per-row Gram pseudo-inverse used by Eq. Tproj and by the
// constraint projection Pi_B (Sec. 3.6).  nB <= RN_NBMAX.
//
// Decision rule of the least-squares solve: when every Cholesky pivot of
// G = B_J^T B_J exceeds 1e-12 * max(diag G), G^+ = G^-1 is formed from a
// backward-stable QR of B_J (CholeskyQR2); otherwise the pseudo-inverse comes
// from a cyclic Jacobi eigen-decomposition of G keeping eigenvalues above
// 1e-12 * lambda_max.
#pragma once
#include <hip/hip_runtime.h>

#define RN_NBMAX 4

// Lanes per row of the kernels that write T row by row: 16 where pattern
// rows hold more than 8 entries on average, else 4.
static inline int rn_row_group(int64_t nnz, int n) { return (n > 0 && nnz > 8 * (int64_t)n) ? 16 : 4; }

// index of (q, r), q <= r, in the packed upper triangle of an nB x nB matrix
__host__ __device__ inline int rn_pk(int nB, int q, int r) {
  if (q > r) { const int t = q; q = r; r = t; }
  return q * nB - (q * (q - 1)) / 2 + (r - q);
}

__device__ inline void rn_gram_pinv_eig(int nB, const double *G, double *Gp);

// The entries of one pattern row in rounds of RN_ROW_CHUNK: the column
// indices of a round are loaded together, then their Bc rows together, so a
// pass over a short row costs two memory round trips, not two per entry;
// f(p, b) sees the entries in row order (the sums keep that order).
#define RN_ROW_CHUNK 8
template <int NB, class F>
__device__ inline void rn_row_each(const int32_t *__restrict__ J, int s, int e, const double *__restrict__ Bc, F &&f) {
  for (int p0 = s; p0 < e; p0 += RN_ROW_CHUNK) {
    int j[RN_ROW_CHUNK];
#pragma unroll
    for (int k = 0; k < RN_ROW_CHUNK; ++k) j[k] = p0 + k < e ? J[p0 + k] : 0;
    double b[RN_ROW_CHUNK][NB];
#pragma unroll
    for (int k = 0; k < RN_ROW_CHUNK; ++k)
#pragma unroll
      for (int q = 0; q < NB; ++q) b[k][q] = p0 + k < e ? Bc[(int64_t)j[k] * NB + q] : 0.0;
#pragma unroll
    for (int k = 0; k < RN_ROW_CHUNK; ++k)
      if (p0 + k < e) f(p0 + k, b[k]);
  }
}

// Least-squares data of one pattern row: Gp = pinv(B_J^T B_J) where the rows
// of B_J are Bc[J[p]], p in [s, e).  Formed by CholeskyQR2 over the row's
// entries (two streaming passes, no storage of B_J): G = B_J^T B_J = R1^T R1,
// then Q1 = B_J R1^-1 and Q1^T Q1 = R2^T R2, R = R2 R1, Gp = R^-1 R^-T.  The
// result is backward stable (error ~ cond(B_J) eps instead of cond(B_J)^2 eps
// for inverting G directly).  Rank rule: every pivot of the first Cholesky
// must exceed 1e-12 max(diag G); otherwise the eigen pseudo-inverse of G.
// Returns 1 when the fallback was taken.
// rn_row_pinv_g: the same from the row's G = B_J^T B_J, summed by the caller
// in row order (with other sums of the same pass).
template <int NB>
__device__ inline int rn_row_pinv_g(const int32_t *__restrict__ J, int s, int e, const double *__restrict__ Bc,
                                    const double *G, double *Gp);
template <int NB>
__device__ inline int rn_row_pinv(const int32_t *__restrict__ J, int s, int e, const double *__restrict__ Bc,
                                  double *Gp) {
  double G[NB * NB];
#pragma unroll
  for (int q = 0; q < NB * NB; ++q) G[q] = 0.0;
  rn_row_each<NB>(J, s, e, Bc, [&](int, const double *b) {
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int r = 0; r < NB; ++r) G[q * NB + r] += b[q] * b[r];
  });
  return rn_row_pinv_g<NB>(J, s, e, Bc, G, Gp);
}
template <int NB>
__device__ inline int rn_row_pinv_g(const int32_t *__restrict__ J, int s, int e, const double *__restrict__ Bc,
                                    const double *G, double *Gp) {
  double dmax = 0.0;
#pragma unroll
  for (int q = 0; q < NB; ++q) dmax = fmax(dmax, G[q * NB + q]);
  // Cholesky G = R1^T R1, R1 upper triangular
  double R1[NB * NB];
#pragma unroll
  for (int q = 0; q < NB * NB; ++q) R1[q] = 0.0;
  bool ok = dmax > 0.0 && (e - s) >= NB;
  for (int k = 0; k < NB && ok; ++k) {
    double d = G[k * NB + k];
    for (int t = 0; t < k; ++t) d -= R1[t * NB + k] * R1[t * NB + k];
    if (!(d > 1e-12 * dmax)) {
      ok = false;
      break;
    }
    const double rk = sqrt(d);
    R1[k * NB + k] = rk;
    for (int j = k + 1; j < NB; ++j) {
      double v = G[k * NB + j];
      for (int t = 0; t < k; ++t) v -= R1[t * NB + k] * R1[t * NB + j];
      R1[k * NB + j] = v / rk;
    }
  }
  if (!ok) {
    rn_gram_pinv_eig(NB, G, Gp);
    return 1;
  }
  // second pass: G2 = sum q q^T with q = b R1^-1 (forward substitution)
  double G2[NB * NB];
#pragma unroll
  for (int q = 0; q < NB * NB; ++q) G2[q] = 0.0;
  rn_row_each<NB>(J, s, e, Bc, [&](int, const double *b) {
    double qv[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      double v = b[k];
#pragma unroll
      for (int t = 0; t < k; ++t) v -= R1[t * NB + k] * qv[t];
      qv[k] = v / R1[k * NB + k];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int r = 0; r < NB; ++r) G2[q * NB + r] += qv[q] * qv[r];
  });
  double R2[NB * NB];
#pragma unroll
  for (int q = 0; q < NB * NB; ++q) R2[q] = 0.0;
  for (int k = 0; k < NB; ++k) {
    double d = G2[k * NB + k];
    for (int t = 0; t < k; ++t) d -= R2[t * NB + k] * R2[t * NB + k];
    if (!(d > 0.0)) {
      rn_gram_pinv_eig(NB, G, Gp);
      return 1;
    }
    const double rk = sqrt(d);
    R2[k * NB + k] = rk;
    for (int j = k + 1; j < NB; ++j) {
      double v = G2[k * NB + j];
      for (int t = 0; t < k; ++t) v -= R2[t * NB + k] * R2[t * NB + j];
      R2[k * NB + j] = v / rk;
    }
  }
  // R = R2 R1 (upper), Ri = R^-1, Gp = Ri Ri^T
  double R[NB * NB], Ri[NB * NB];
#pragma unroll
  for (int q = 0; q < NB; ++q)
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      double v = 0.0;
      for (int t = q; t <= r; ++t) v += R2[q * NB + t] * R1[t * NB + r];
      R[q * NB + r] = r >= q ? v : 0.0;
      Ri[q * NB + r] = 0.0;
    }
  for (int c = 0; c < NB; ++c) {
    Ri[c * NB + c] = 1.0 / R[c * NB + c];
    for (int r = c - 1; r >= 0; --r) {
      double v = 0.0;
      for (int t = r + 1; t <= c; ++t) v += R[r * NB + t] * Ri[t * NB + c];
      Ri[r * NB + c] = -v / R[r * NB + r];
    }
  }
#pragma unroll
  for (int q = 0; q < NB; ++q)
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      double v = 0.0;
#pragma unroll
      for (int t = 0; t < NB; ++t) v += Ri[q * NB + t] * Ri[r * NB + t];
      Gp[q * NB + r] = v;
    }
  return 0;
}

// Eigen pseudo-inverse of a symmetric nB x nB Gram matrix (cyclic Jacobi):
// eigenvalues above 1e-12 lambda_max are inverted, the rest dropped.
__device__ inline void rn_gram_pinv_eig(int nB, const double *G, double *Gp) {
  // cyclic Jacobi eigen-decomposition of G
  double w[RN_NBMAX][RN_NBMAX], v[RN_NBMAX][RN_NBMAX];
  for (int q = 0; q < nB; ++q)
    for (int r = 0; r < nB; ++r) {
      w[q][r] = G[q * nB + r];
      v[q][r] = (q == r) ? 1.0 : 0.0;
    }
  // converged once the off-diagonal sum of squares is below 1e-36 of the
  // diagonal's (rank-deficient G often never reaches an exact zero; rotations
  // then only move round-off); at most 40 sweeps
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dn = 0.0;
    for (int q = 0; q < nB; ++q) {
      dn += w[q][q] * w[q][q];
      for (int r = q + 1; r < nB; ++r) off += w[q][r] * w[q][r];
    }
    if (off <= 1e-36 * dn) break;
    for (int q = 0; q < nB; ++q)
      for (int r = q + 1; r < nB; ++r) {
        const double wqr = w[q][r];
        if (wqr == 0.0) continue;
        const double th = (w[r][r] - w[q][q]) / (2.0 * wqr);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < nB; ++k) {  // columns q, r
          const double x = w[k][q], y = w[k][r];
          w[k][q] = c * x - s * y;
          w[k][r] = s * x + c * y;
        }
        for (int k = 0; k < nB; ++k) {  // rows q, r
          const double x = w[q][k], y = w[r][k];
          w[q][k] = c * x - s * y;
          w[r][k] = s * x + c * y;
        }
        for (int k = 0; k < nB; ++k) {
          const double x = v[k][q], y = v[k][r];
          v[k][q] = c * x - s * y;
          v[k][r] = s * x + c * y;
        }
      }
  }
  double lmax = 0.0;
  for (int q = 0; q < nB; ++q) lmax = fmax(lmax, w[q][q]);
  for (int q = 0; q < nB * nB; ++q) Gp[q] = 0.0;
  for (int e = 0; e < nB; ++e) {
    const double lam = w[e][e];
    if (!(lam > 1e-12 * lmax) || lam <= 0.0) continue;
    for (int q = 0; q < nB; ++q)
      for (int r = 0; r < nB; ++r) Gp[q * nB + r] += v[q][e] * v[r][e] / lam;
  }
}
