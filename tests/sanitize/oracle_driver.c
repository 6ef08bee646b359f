/* Drives every oracle routine on small generated problems, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py).
 * Exit status 0 when every call returns normally and the results pass basic
 * checks; the sanitizers abort on a memory or undefined-behaviour error. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      return 1;                                               \
    }                                                         \
  } while (0)

/* 5-point Laplacian on nx x nx, scalar (m = 1), or each entry times the 2x2
 * block [[2, -0.5], [-0.5, 2]] scaled (m = 2, interleaved DOFs) */
static int grid(int nx, int m, int **Ap, int **Aj, double **Ax) {
  const int nn = nx * nx, n = nn * m;
  *Ap = malloc((n + 1) * sizeof(int));
  *Aj = malloc(5 * m * n * sizeof(int));
  *Ax = malloc(5 * m * n * sizeof(double));
  int w = 0;
  (*Ap)[0] = 0;
  for (int i = 0; i < n; ++i) {
    const int I = i / m, c = i % m, x = I % nx, y = I / nx;
    const int nb[5] = {y > 0 ? I - nx : -1, x > 0 ? I - 1 : -1, I, x < nx - 1 ? I + 1 : -1, y < nx - 1 ? I + nx : -1};
    for (int k = 0; k < 5; ++k) {
      if (nb[k] < 0) continue;
      const double s = nb[k] == I ? 4.0 : -1.0;
      for (int cc = 0; cc < m; ++cc) {
        const double b = m == 1 ? 1.0 : (c == cc ? 2.0 : -0.5);
        (*Aj)[w] = m * nb[k] + cc;
        (*Ax)[w] = s * b;
        ++w;
      }
    }
    (*Ap)[i + 1] = w;
  }
  return n;
}

static int run(int nx, int m, int nB) {
  int *Ap, *Aj;
  double *Ax;
  const int n = grid(nx, m, &Ap, &Aj, &Ax), nn = n / m;
  const int cap = 2 * Ap[n] + nn;
  int *Sp = malloc((nn + 1) * sizeof(int)), *Sj = malloc(cap * sizeof(int));
  const int nS = orc_strength(n, Ap, Aj, Ax, m, 0.1, Sp, Sj, cap);
  CHECK(nS > 0);
  double *Sx = malloc(nS * sizeof(double));
  CHECK(orc_strength_values(n, Ap, Aj, Ax, m, 0.1, Sp, Sj, Sx) == ORC_OK);
  int *agg = malloc(nn * sizeof(int)), *roots = malloc(nn * sizeof(int));
  const int na = orc_aggregate(nn, Sp, Sj, agg, roots);
  CHECK(na > 0);
  const int ncap = nn * na;
  int *Npn = malloc((nn + 1) * sizeof(int)), *Njn = malloc(ncap * sizeof(int));
  const int nnzn = orc_pattern_nodes(nn, Sp, Sj, agg, na, 2, Npn, Njn, ncap);
  CHECK(nnzn > 0);
  const int dcap = nnzn * m * m + n;
  int *Np = malloc((n + 1) * sizeof(int)), *Nj = malloc(dcap * sizeof(int));
  unsigned char *is_root = malloc(n);
  const int nz = orc_pattern_dofs(nn, m, Npn, Njn, agg, roots, na, Np, Nj, dcap, is_root);
  CHECK(nz > 0);
  const int nc = m * na;
  double *B = malloc(n * nB * sizeof(double)), *Bc = malloc(nc * nB * sizeof(double));
  for (int i = 0; i < n; ++i)
    for (int q = 0; q < nB; ++q) B[i * nB + q] = q < m ? (i % m == q) : 1.0 + 0.1 * q * ((i / m) % nx);
  double *T = malloc(nz * sizeof(double)), *P = malloc(nz * sizeof(double)), *Q = malloc(nz * sizeof(double));
  int rd = 0;
  CHECK(orc_tentative(n, m, Np, Nj, is_root, agg, roots, na, B, nB, T, Bc, &rd) == ORC_OK);
  double gam[9], del[8], alp[8], res[9];
  int it = 0;
  CHECK(orc_emin_cg(n, nc, Ap, Aj, Ax, Np, Nj, is_root, Bc, nB, T, 8, P, gam, del, alp, &it) == ORC_OK);
  CHECK(orc_constraint_residual(n, Np, Nj, P, Bc, B, nB) < 1e-8 || rd > 0);
  CHECK(isfinite(orc_energy(n, nc, Ap, Aj, Ax, Np, Nj, P)));
  CHECK(orc_emin_pcg(n, nc, Ap, Aj, Ax, Np, Nj, is_root, Bc, nB, T, 8, Q, gam, del, alp, &it) == ORC_OK);
  CHECK(orc_emin_cgnr(n, nc, Ap, Aj, Ax, Np, Nj, is_root, Bc, nB, T, 4, Q, gam, del, alp, &it) == ORC_OK);
  CHECK(orc_emin_gmres(n, nc, Ap, Aj, Ax, Np, Nj, is_root, Bc, nB, T, 8, Q, res, &it) == ORC_OK);
  double *dA = malloc(Ap[n] * sizeof(double));
  for (int p = 0; p < Ap[n]; ++p) dA[p] = 0.01 * (p % 7);
  CHECK(orc_emin_cg_jvp(n, nc, Ap, Aj, Ax, dA, Np, Nj, is_root, Bc, nB, T, 4, Q, P) == ORC_OK);
  unsigned char *keep = malloc(nz);
  CHECK(orc_filter(n, m, Np, Nj, Q, is_root, agg, 2, 0.2, keep) == ORC_OK);
  int *Fp = malloc((n + 1) * sizeof(int)), *Fj = malloc(nz * sizeof(int));
  double *Fv = malloc(nz * sizeof(double));
  const int nf = orc_compact(n, Np, Nj, Q, keep, Fp, Fj, Fv);
  CHECK(nf > 0 && nf <= nz);
  CHECK(orc_enforce(n, Fp, Fj, is_root, Bc, nB, B, Fv) >= 0);
  int *Tp = malloc((n + 1) * sizeof(int)), *Tj = malloc(Ap[n] * sizeof(int));
  double *Tx = malloc(Ap[n] * sizeof(double));
  orc_transpose(n, n, Ap, Aj, Ax, Tp, Tj, Tx);
  const long ccap = (long)Ap[n] * 40;
  int *Cp = malloc((n + 1) * sizeof(int)), *Cj = malloc(ccap * sizeof(int));
  double *Cx = malloc(ccap * sizeof(double));
  CHECK(orc_spgemm(n, n, nc, Ap, Aj, Ax, Np, Nj, P, Cp, Cj, Cx, ccap) > 0);
  CHECK(orc_spgemm(n, n, nc, Ap, Aj, Ax, Np, Nj, P, Cp, Cj, Cx, 3) == ORC_ECAP);
  double *Bs = malloc(n * nB * sizeof(double));
  for (int i = 0; i < n * nB; ++i) Bs[i] = B[i];
  CHECK(orc_smooth_candidates(n, Ap, Aj, Ax, Bs, nB, 3, 2.0 / 3.0) == ORC_OK);
  double G[4] = {2.0, 1.0, 1.0, 0.5}, Gp[4];
  orc_gram_pinv(2, G, Gp);
  free(Ap); free(Aj); free(Ax); free(Sp); free(Sj); free(Sx); free(agg); free(roots); free(Npn); free(Njn);
  free(Np); free(Nj); free(is_root); free(B); free(Bc); free(T); free(P); free(Q); free(dA); free(keep);
  free(Fp); free(Fj); free(Fv); free(Tp); free(Tj); free(Tx); free(Cp); free(Cj); free(Cx); free(Bs);
  return 0;
}

int main(void) {
  orc_set_threads(2);
  if (run(12, 1, 1) || run(12, 1, 3) || run(7, 2, 2) || run(7, 2, 3)) return 1;
  printf("oracle driver ok\n");
  return 0;
}
