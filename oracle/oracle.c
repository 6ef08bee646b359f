/*
 * oracle.c -- plain FP64 CPU reference of root-node AMG interpolation setup.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written from the paper's
 * description, step by step, with no blocking, fusion or reordering: each
 * function states the passage it follows.  Built with -O2 -ffp-contract=off
 * so that every product and sum is rounded as written.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NBMAX 8

/* Threads: the loops over rows and over entries that are independent run
 * under OpenMP with a static schedule; every sum is split into fixed chunks
 * whose boundaries do not depend on the thread count, so results are
 * identical for any number of threads. */
void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* small helpers                                                             */
/* ------------------------------------------------------------------------ */
static int cmp_ll(const void *a, const void *b) {
  long long x = *(const long long *)a, y = *(const long long *)b;
  return (x > y) - (x < y);
}
static int cmp_int(const void *a, const void *b) {
  int x = *(const int *)a, y = *(const int *)b;
  return (x > y) - (x < y);
}
/* Frobenius inner product <X, Y> = sum over the pattern of X_ij Y_ij.
 * Evaluated with compensated (Neumaier) summation: a plain running sum of
 * 10^6 terms carries a relative error of ~1e-12 into P, which is larger than
 * the FP64 parity tolerance, while the compensated sum is accurate to a few
 * units in the last place whatever the length. */
#define DOT_CHUNK 4096
/* add v to the compensated pair (s, c) (Neumaier) */
static void comp_add(double *s, double *c, double v) {
  const double t = *s + v;
  *c += (fabs(*s) >= fabs(v)) ? (*s - t) + v : (v - t) + *s;
  *s = t;
}
/* Chunks of DOT_CHUNK terms are summed on their own, then the chunk sums (and
 * their corrections) in chunk order. */
static double dot(long len, const double *x, const double *y) {
  const long nch = (len + DOT_CHUNK - 1) / DOT_CHUNK;
  double *cs = (double *)malloc((size_t)(nch > 0 ? nch : 1) * 2 * sizeof(double));
#pragma omp parallel for schedule(static)
  for (long ch = 0; ch < nch; ++ch) {
    double s = 0.0, c = 0.0;
    const long e = (ch + 1) * DOT_CHUNK < len ? (ch + 1) * DOT_CHUNK : len;
    for (long p = ch * DOT_CHUNK; p < e; ++p) comp_add(&s, &c, x[p] * y[p]);
    cs[2 * ch] = s;
    cs[2 * ch + 1] = c;
  }
  double s = 0.0, c = 0.0;
  for (long ch = 0; ch < nch; ++ch) {
    comp_add(&s, &c, cs[2 * ch]);
    c += cs[2 * ch + 1];
  }
  free(cs);
  return s + c;
}

/* Stopping rules for iterations that have converged to round-off: CG stops
 * once <R,R> <= CG_STOP <R0,R0> (the residual has dropped by 1e12), GMRES
 * once its residual estimate is <= GM_STOP ||R0||.  Past that point both
 * methods would only iterate on rounding noise. */
#define CG_STOP 1e-24
#define GM_STOP 1e-12

/* ------------------------------------------------------------------------ */
/* Strength of connection, Sec. 3.2.  Symmetric measure: entry (i,j) is     */
/* strong when |a_ij| >= theta sqrt(|a_ii a_jj|), evaluated squared.  For   */
/* vector problems the amalgamate step collapses each m x m block to one    */
/* node entry; a block is strong when any of its DOF entries is.            */
/* ------------------------------------------------------------------------ */
int orc_strength(int n, const int *Ap, const int *Aj, const double *Ax, int m,
                 double theta, int *Sp, int *Sj, int cap) {
  if (m < 1 || n % m) return ORC_EINVAL;
  int nn = n / m;
  double *diag = (double *)calloc((size_t)n, sizeof(double));
  for (int i = 0; i < n; ++i)
    for (int p = Ap[i]; p < Ap[i + 1]; ++p)
      if (Aj[p] == i) diag[i] = Ax[p];
  long maxk = 2L * Ap[n] + nn;
  long long *key = (long long *)malloc((size_t)maxk * sizeof(long long));
  long cnt = 0;
  for (int I = 0; I < nn; ++I) key[cnt++] = (long long)I * nn + I;
  double th2 = theta * theta;
  for (int i = 0; i < n; ++i) {
    for (int p = Ap[i]; p < Ap[i + 1]; ++p) {
      int j = Aj[p];
      double lhs = Ax[p] * Ax[p];
      double rhs = th2 * fabs(diag[i] * diag[j]);
      if (i == j || lhs >= rhs) {
        int I = i / m, J = j / m;
        key[cnt++] = (long long)I * nn + J;  /* S            */
        key[cnt++] = (long long)J * nn + I;  /* S^T: S u S^T */
      }
    }
  }
  qsort(key, (size_t)cnt, sizeof(long long), cmp_ll);
  long u = 0;
  for (long q = 0; q < cnt; ++q)
    if (q == 0 || key[q] != key[q - 1]) key[u++] = key[q];
  int rc = (int)u;
  if (u > cap) {
    rc = ORC_ECAP;
  } else {
    for (int I = 0; I <= nn; ++I) Sp[I] = 0;
    for (long q = 0; q < u; ++q) {
      Sp[key[q] / nn + 1]++;
      Sj[q] = (int)(key[q] % nn);
    }
    for (int I = 0; I < nn; ++I) Sp[I + 1] += Sp[I];
  }
  free(key);
  free(diag);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Aggregation, Sec. 3.3: the classical greedy scheme.  An unaggregated     */
/* node whose strong neighbours are all unaggregated becomes a root and     */
/* collects those neighbours.  Left-over nodes then join a neighbouring     */
/* aggregate formed in that first sweep; nodes still left form new          */
/* aggregates with their unaggregated neighbours, rooted at themselves.     */
/* ------------------------------------------------------------------------ */
int orc_aggregate(int nn, const int *Sp, const int *Sj, int *agg, int *roots) {
  int na = 0;
  for (int i = 0; i < nn; ++i) agg[i] = -1;
  /* sweep 1 */
  for (int i = 0; i < nn; ++i) {
    if (agg[i] >= 0) continue;
    int free_nb = 1;
    for (int p = Sp[i]; p < Sp[i + 1]; ++p)
      if (Sj[p] != i && agg[Sj[p]] >= 0) { free_nb = 0; break; }
    if (!free_nb) continue;
    roots[na] = i;
    agg[i] = na;
    for (int p = Sp[i]; p < Sp[i + 1]; ++p) agg[Sj[p]] = na;
    ++na;
  }
  /* sweep 2: join the lowest-index neighbour aggregated in sweep 1 */
  int *snap = (int *)malloc((size_t)(nn > 0 ? nn : 1) * sizeof(int));
  memcpy(snap, agg, (size_t)nn * sizeof(int));
  for (int i = 0; i < nn; ++i) {
    if (agg[i] >= 0) continue;
    for (int p = Sp[i]; p < Sp[i + 1]; ++p) {
      int j = Sj[p];
      if (j != i && snap[j] >= 0) { agg[i] = snap[j]; break; }
    }
  }
  free(snap);
  /* sweep 3 */
  for (int i = 0; i < nn; ++i) {
    if (agg[i] >= 0) continue;
    roots[na] = i;
    agg[i] = na;
    for (int p = Sp[i]; p < Sp[i + 1]; ++p)
      if (agg[Sj[p]] < 0) agg[Sj[p]] = na;
    ++na;
  }
  return na;
}

/* ------------------------------------------------------------------------ */
/* Pattern N = S^d C, Sec. 3.4, as d boolean sparse products: X_0 = C and   */
/* X_{t+1} = S X_t.  A marker array gives the union of each row.            */
/* ------------------------------------------------------------------------ */
int orc_pattern_nodes(int nn, const int *Sp, const int *Sj, const int *agg,
                      int n_agg, int d, int *Np, int *Nj, int cap) {
  if (d < 0) return ORC_EINVAL;
  int *Xp = (int *)malloc((size_t)(nn + 1) * sizeof(int));
  int *Xj = (int *)malloc((size_t)(nn > 0 ? nn : 1) * sizeof(int));
  for (int I = 0; I <= nn; ++I) Xp[I] = I;
  for (int I = 0; I < nn; ++I) Xj[I] = agg[I];
  int *mark = (int *)malloc((size_t)(n_agg > 0 ? n_agg : 1) * sizeof(int));
  for (int t = 0; t < d; ++t) {
    for (int a = 0; a < n_agg; ++a) mark[a] = -1;
    int *Yp = (int *)malloc((size_t)(nn + 1) * sizeof(int));
    Yp[0] = 0;
    for (int I = 0; I < nn; ++I) {
      int c = 0;
      for (int p = Sp[I]; p < Sp[I + 1]; ++p) {
        int J = Sj[p];
        for (int q = Xp[J]; q < Xp[J + 1]; ++q)
          if (mark[Xj[q]] != I) { mark[Xj[q]] = I; ++c; }
      }
      Yp[I + 1] = Yp[I] + c;
    }
    int *Yj = (int *)malloc((size_t)(Yp[nn] > 0 ? Yp[nn] : 1) * sizeof(int));
    for (int a = 0; a < n_agg; ++a) mark[a] = -1;
    for (int I = 0; I < nn; ++I) {
      int w = Yp[I];
      for (int p = Sp[I]; p < Sp[I + 1]; ++p) {
        int J = Sj[p];
        for (int q = Xp[J]; q < Xp[J + 1]; ++q)
          if (mark[Xj[q]] != I) { mark[Xj[q]] = I; Yj[w++] = Xj[q]; }
      }
      qsort(Yj + Yp[I], (size_t)(Yp[I + 1] - Yp[I]), sizeof(int), cmp_int);
    }
    free(Xp);
    free(Xj);
    Xp = Yp;
    Xj = Yj;
  }
  int rc = Xp[nn];
  if (rc > cap) {
    rc = ORC_ECAP;
  } else {
    memcpy(Np, Xp, (size_t)(nn + 1) * sizeof(int));
    memcpy(Nj, Xj, (size_t)Xp[nn] * sizeof(int));
  }
  free(mark);
  free(Xp);
  free(Xj);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* unamalgamate and root_node_pattern, Sec. 3.4: DOF entry (i,j) exists when */
/* nodal entry (floor(i/m), floor(j/m)) does; each root DOF row becomes the  */
/* identity row of its coarse DOF.                                           */
/* ------------------------------------------------------------------------ */
int orc_pattern_dofs(int nn, int m, const int *Npn, const int *Njn,
                     const int *agg, const int *roots, int n_agg,
                     int *Np, int *Nj, int cap, unsigned char *is_root) {
  (void)n_agg;
  int n = nn * m;
  long w = 0;
  Np[0] = 0;
  for (int i = 0; i < n; ++i) {
    int I = i / m, c = i % m, a = agg[I];
    int root = (roots[a] == I);
    is_root[i] = (unsigned char)root;
    if (root) {
      if (w + 1 > cap) return ORC_ECAP;
      Nj[w++] = m * a + c;
    } else {
      long len = (long)(Npn[I + 1] - Npn[I]) * m;
      if (w + len > cap) return ORC_ECAP;
      for (int p = Npn[I]; p < Npn[I + 1]; ++p)
        for (int cc = 0; cc < m; ++cc) Nj[w++] = m * Njn[p] + cc;
    }
    Np[i + 1] = (int)w;
  }
  return (int)w;
}

/* ------------------------------------------------------------------------ */
/* Pseudo-inverse of a small SPD(-ish) Gram matrix.                          */
/* ------------------------------------------------------------------------ */
static void jacobi_eig(int k, double *a, double *v) {
  /* cyclic Jacobi on the symmetric k x k matrix a; eigenvalues end up on the
   * diagonal of a, eigenvectors in the columns of v */
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) v[i * k + j] = (i == j);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < k; ++i)
      for (int j = i + 1; j < k; ++j) off += a[i * k + j] * a[i * k + j];
    if (off == 0.0) break;
    for (int p = 0; p < k; ++p) {
      for (int q = p + 1; q < k; ++q) {
        double apq = a[p * k + q];
        if (apq == 0.0) continue;
        double theta = (a[q * k + q] - a[p * k + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) /
                   (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < k; ++r) {
          double arp = a[r * k + p], arq = a[r * k + q];
          a[r * k + p] = c * arp - s * arq;
          a[r * k + q] = s * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) {
          double apr = a[p * k + r], aqr = a[q * k + r];
          a[p * k + r] = c * apr - s * aqr;
          a[q * k + r] = s * apr + c * aqr;
        }
        for (int r = 0; r < k; ++r) {
          double vrp = v[r * k + p], vrq = v[r * k + q];
          v[r * k + p] = c * vrp - s * vrq;
          v[r * k + q] = s * vrp + c * vrq;
        }
      }
    }
  }
}

/* Eigen pseudo-inverse of a symmetric Gram matrix: eigenvalues above
 * 1e-12 lambda_max are inverted, the rest dropped. */
static void orc_gram_pinv_eig(int nB, const double *G, double *Gp) {
  double a[NBMAX * NBMAX], v[NBMAX * NBMAX];
  memcpy(a, G, sizeof(double) * (size_t)(nB * nB));
  jacobi_eig(nB, a, v);
  double lmax = 0.0;
  for (int i = 0; i < nB; ++i) lmax = fmax(lmax, a[i * nB + i]);
  for (int i = 0; i < nB * nB; ++i) Gp[i] = 0.0;
  for (int l = 0; l < nB; ++l) {
    double lam = a[l * nB + l];
    if (!(lam > 1e-12 * lmax) || lam <= 0.0) continue;
    for (int i = 0; i < nB; ++i)
      for (int j = 0; j < nB; ++j) Gp[i * nB + j] += v[i * nB + l] * v[j * nB + l] / lam;
  }
}

int orc_gram_pinv(int nB, const double *G, double *Gp) {
  if (nB <= 0) return 0;
  double L[NBMAX * NBMAX], D[NBMAX], maxd = 0.0;
  for (int i = 0; i < nB; ++i) maxd = fmax(maxd, G[i * nB + i]);
  int ok = maxd > 0.0;
  for (int k = 0; k < nB && ok; ++k) {
    double dk = G[k * nB + k];
    for (int l = 0; l < k; ++l) dk -= L[k * nB + l] * L[k * nB + l] * D[l];
    if (!(dk > 1e-12 * maxd)) { ok = 0; break; }
    D[k] = dk;
    L[k * nB + k] = 1.0;
    for (int i = k + 1; i < nB; ++i) {
      double s = G[i * nB + k];
      for (int l = 0; l < k; ++l) s -= L[i * nB + l] * L[k * nB + l] * D[l];
      L[i * nB + k] = s / dk;
    }
  }
  if (ok) {
    /* Linv: inverse of unit lower-triangular L */
    double Li[NBMAX * NBMAX];
    for (int j = 0; j < nB; ++j) {
      for (int i = 0; i < nB; ++i) Li[i * nB + j] = (i == j);
      for (int i = j + 1; i < nB; ++i) {
        double s = 0.0;
        for (int l = j; l < i; ++l) s += L[i * nB + l] * Li[l * nB + j];
        Li[i * nB + j] = -s;
      }
    }
    /* G^-1 = Li^T D^-1 Li */
    for (int i = 0; i < nB; ++i)
      for (int j = 0; j < nB; ++j) {
        double s = 0.0;
        for (int l = 0; l < nB; ++l) s += Li[l * nB + i] * Li[l * nB + j] / D[l];
        Gp[i * nB + j] = s;
      }
    return 0;
  }
  orc_gram_pinv_eig(nB, G, Gp);
  return 1;
}

/* Least-squares data of one F row i: G^+ for G = B_J^T B_J, where B_J is the
 * len x nB matrix of the coarse candidates at the row's pattern columns.
 * Formed through a Householder QR, B_J = Q R, as G^+ = R^-1 R^-T: its
 * rounding error grows like cond(B_J) rather than cond(B_J)^2 for the normal
 * equations (cond(G) ~ 1e5 for rigid-body modes, where forming G^-1 from G
 * alone was measured to move P by 2e-11).  Rank test: every R_kk^2 must
 * exceed 1e-12 max_q ||B_J e_q||^2 (in exact arithmetic R_kk^2 are the
 * pivots of G's LDL^T and the column norms its diagonal); otherwise the
 * eigen pseudo-inverse of G = R^T R is used.  W: scratch of len * nB.
 * Returns 1 when the fallback was taken. */
static int row_pinv(int len, const int *J, const double *Bc, int nB, double *W, double *Gp) {
  double R[NBMAX * NBMAX], cmax = 0.0;
  for (int r = 0; r < len; ++r)
    for (int q = 0; q < nB; ++q) W[(long)r * nB + q] = Bc[(long)J[r] * nB + q];
  for (int q = 0; q < nB; ++q) {
    double s = 0.0;
    for (int r = 0; r < len; ++r) s += W[(long)r * nB + q] * W[(long)r * nB + q];
    cmax = fmax(cmax, s);
  }
  for (int q = 0; q < nB * nB; ++q) R[q] = 0.0;
  for (int k = 0; k < nB && k < len; ++k) {
    /* Householder reflector zeroing column k below row k */
    double nx = 0.0;
    for (int r = k; r < len; ++r) nx += W[(long)r * nB + k] * W[(long)r * nB + k];
    nx = sqrt(nx);
    const double x0 = W[(long)k * nB + k];
    const double alpha = x0 >= 0.0 ? -nx : nx;
    double vv = 0.0;
    W[(long)k * nB + k] = x0 - alpha; /* v stored in place, column k rows k.. */
    for (int r = k; r < len; ++r) vv += W[(long)r * nB + k] * W[(long)r * nB + k];
    for (int j = k + 1; j < nB; ++j) {
      if (vv == 0.0) break;
      double w = 0.0;
      for (int r = k; r < len; ++r) w += W[(long)r * nB + k] * W[(long)r * nB + j];
      const double f = 2.0 * w / vv;
      for (int r = k; r < len; ++r) W[(long)r * nB + j] -= f * W[(long)r * nB + k];
    }
    R[k * nB + k] = alpha;
    for (int j = k + 1; j < nB; ++j) R[k * nB + j] = W[(long)k * nB + j];
  }
  int ok = cmax > 0.0 && len >= nB;
  for (int k = 0; k < nB && ok; ++k)
    if (!(R[k * nB + k] * R[k * nB + k] > 1e-12 * cmax)) ok = 0;
  if (ok) {
    /* Ri = R^-1 (upper triangular), G^+ = Ri Ri^T */
    double Ri[NBMAX * NBMAX];
    for (int q = 0; q < nB * nB; ++q) Ri[q] = 0.0;
    for (int c = 0; c < nB; ++c) {
      Ri[c * nB + c] = 1.0 / R[c * nB + c];
      for (int r = c - 1; r >= 0; --r) {
        double s = 0.0;
        for (int l = r + 1; l <= c; ++l) s += R[r * nB + l] * Ri[l * nB + c];
        Ri[r * nB + c] = -s / R[r * nB + r];
      }
    }
    for (int q = 0; q < nB; ++q)
      for (int r = 0; r < nB; ++r) {
        double s = 0.0;
        for (int l = 0; l < nB; ++l) s += Ri[q * nB + l] * Ri[r * nB + l];
        Gp[q * nB + r] = s;
      }
    return 0;
  }
  double G[NBMAX * NBMAX];
  for (int q = 0; q < nB; ++q)
    for (int r = 0; r < nB; ++r) {
      double s = 0.0;
      for (int l = 0; l < nB; ++l) s += R[l * nB + q] * R[l * nB + r];
      G[q * nB + r] = s;
    }
  orc_gram_pinv_eig(nB, G, Gp);
  return 1;
}

int orc_gram_rows(int n, const int *Np, const int *Nj,
                  const unsigned char *is_root, const double *Bc, int nB,
                  double *Gp) {
  int bad = 0, maxlen = 1;
  for (int i = 0; i < n; ++i) maxlen = Np[i + 1] - Np[i] > maxlen ? Np[i + 1] - Np[i] : maxlen;
#pragma omp parallel reduction(+ : bad)
  {
    double *W = (double *)malloc((size_t)maxlen * (nB > 0 ? nB : 1) * sizeof(double));
#pragma omp for schedule(static)
    for (int i = 0; i < n; ++i) {
      double *gi = Gp + (long)i * nB * nB;
      for (int q = 0; q < nB * nB; ++q) gi[q] = 0.0;
      if (is_root[i] || nB == 0) continue;
      bad += row_pinv(Np[i + 1] - Np[i], Nj + Np[i], Bc, nB, W, gi);
    }
    free(W);
  }
  return bad;
}

/* ------------------------------------------------------------------------ */
/* Projection onto the constraint space (Sec. 3.6: updates U must satisfy   */
/* U Bc = 0 on the pattern, with root rows fixed): zero the root rows; on   */
/* each F row remove the least-squares component x B_J G^+ B_J^T.           */
/* ------------------------------------------------------------------------ */
void orc_project(int n, const int *Np, const int *Nj,
                 const unsigned char *is_root, const double *Bc, int nB,
                 const double *Gp, double *X) {
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    double s[NBMAX], y[NBMAX];
    if (is_root[i]) {
      for (int p = Np[i]; p < Np[i + 1]; ++p) X[p] = 0.0;
      continue;
    }
    if (nB == 0) continue;
    const double *gi = Gp + (long)i * nB * nB;
    for (int q = 0; q < nB; ++q) s[q] = 0.0;
    for (int p = Np[i]; p < Np[i + 1]; ++p)
      for (int q = 0; q < nB; ++q) s[q] += X[p] * Bc[(long)Nj[p] * nB + q];
    for (int q = 0; q < nB; ++q) {
      y[q] = 0.0;
      for (int r = 0; r < nB; ++r) y[q] += gi[q * nB + r] * s[r];
    }
    for (int p = Np[i]; p < Np[i + 1]; ++p) {
      double u = 0.0;
      for (int q = 0; q < nB; ++q) u += Bc[(long)Nj[p] * nB + q] * y[q];
      X[p] -= u;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Product A X kept to the pattern (Sec. 3.6: the smoothing product whose   */
/* fill is dropped outside N).  Row-by-row Gustavson product with a dense   */
/* accumulator, contributions summed in the order of A's row.               */
/* ------------------------------------------------------------------------ */
void orc_masked_product(int n, int nc, const int *Ap, const int *Aj,
                        const double *Ax, const int *Np, const int *Nj,
                        const double *X, double *Z) {
#pragma omp parallel
  {
    double *acc = (double *)calloc((size_t)(nc > 0 ? nc : 1), sizeof(double));
#pragma omp for schedule(static)
    for (int i = 0; i < n; ++i) {
      for (int t = Ap[i]; t < Ap[i + 1]; ++t) {
        int k = Aj[t];
        for (int q = Np[k]; q < Np[k + 1]; ++q) acc[Nj[q]] += Ax[t] * X[q];
      }
      for (int p = Np[i]; p < Np[i + 1]; ++p) Z[p] = acc[Nj[p]];
      for (int t = Ap[i]; t < Ap[i + 1]; ++t) {
        int k = Aj[t];
        for (int q = Np[k]; q < Np[k + 1]; ++q) acc[Nj[q]] = 0.0;
      }
    }
    free(acc);
  }
}

/* ------------------------------------------------------------------------ */
/* inject, Sec. 3.6: coarse candidates by injection at the root DOFs; T     */
/* from the first m candidates normalised so that coarse DOFs inject to the */
/* roots (Eq. root-nodeform); further candidates by the minimum-norm row    */
/* update of Eq. Tproj.                                                     */
/* ------------------------------------------------------------------------ */
static int invert_small(int m, const double *a, double *ai) {
  double w[NBMAX * 2 * NBMAX];
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < 2 * m; ++j)
      w[i * 2 * m + j] = j < m ? a[i * m + j] : (double)(j - m == i);
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int r = c + 1; r < m; ++r)
      if (fabs(w[r * 2 * m + c]) > fabs(w[piv * 2 * m + c])) piv = r;
    if (w[piv * 2 * m + c] == 0.0) return ORC_ESINGULAR;
    if (piv != c)
      for (int j = 0; j < 2 * m; ++j) {
        double t = w[c * 2 * m + j];
        w[c * 2 * m + j] = w[piv * 2 * m + j];
        w[piv * 2 * m + j] = t;
      }
    double d = w[c * 2 * m + c];
    for (int j = 0; j < 2 * m; ++j) w[c * 2 * m + j] /= d;
    for (int r = 0; r < m; ++r) {
      if (r == c) continue;
      double f = w[r * 2 * m + c];
      for (int j = 0; j < 2 * m; ++j) w[r * 2 * m + j] -= f * w[c * 2 * m + j];
    }
  }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) ai[i * m + j] = w[i * 2 * m + m + j];
  return ORC_OK;
}

int orc_tentative(int n, int m, const int *Np, const int *Nj,
                  const unsigned char *is_root, const int *agg,
                  const int *roots, int n_agg, const double *B, int nB,
                  double *T, double *Bc, int *rank_def) {
  if (m < 1 || nB < m || m > NBMAX || nB > NBMAX) return ORC_EINVAL;
  int nc = m * n_agg;
  for (int a = 0; a < n_agg; ++a)
    for (int c = 0; c < m; ++c)
      for (int q = 0; q < nB; ++q)
        Bc[(long)(m * a + c) * nB + q] = B[(long)(m * roots[a] + c) * nB + q];
  double *binv = (double *)malloc((size_t)(n_agg > 0 ? n_agg : 1) * m * m * sizeof(double));
  for (int a = 0; a < n_agg; ++a) {
    double blk[NBMAX * NBMAX];
    for (int r = 0; r < m; ++r)
      for (int c = 0; c < m; ++c) blk[r * m + c] = B[(long)(m * roots[a] + r) * nB + c];
    if (invert_small(m, blk, binv + (long)a * m * m) != ORC_OK) {
      free(binv);
      return ORC_ESINGULAR;
    }
  }
  for (int i = 0; i < n; ++i) {
    int a = agg[i / m];
    for (int p = Np[i]; p < Np[i + 1]; ++p) {
      int j = Nj[p];
      if (is_root[i]) {
        T[p] = (j == m * a + i % m) ? 1.0 : 0.0;
      } else if (j / m == a) {
        int cc = j % m;
        double s = 0.0;
        for (int r = 0; r < m; ++r) s += B[(long)i * nB + r] * binv[(long)a * m * m + r * m + cc];
        T[p] = s;
      } else {
        T[p] = 0.0;
      }
    }
  }
  free(binv);
  int bad = 0;
  if (nB > m) bad = orc_enforce(n, Np, Nj, is_root, Bc, nB, B, T);
  (void)nc;
  if (rank_def) *rank_def = bad;
  return ORC_OK;
}

/* Eq. Tproj on every F row: the minimum-norm update u of the row's entries
 * t (on its pattern J) such that (t + u) Bc_J = B_i, u = (B_i - t Bc_J) G^+
 * Bc_J^T with G = Bc_J^T Bc_J.  Root rows are left alone.  Used by inject
 * for the candidates beyond the first m, and as enforce after a post-filter
 * (Sec. 3.7).  Returns the number of rows that took the pseudo-inverse. */
int orc_enforce(int n, const int *Np, const int *Nj, const unsigned char *is_root,
                const double *Bc, int nB, const double *B, double *V) {
  if (nB < 1 || nB > NBMAX) return ORC_EINVAL;
  double Gp[NBMAX * NBMAX], r[NBMAX], y[NBMAX];
  int maxlen = 1, bad = 0;
  for (int i = 0; i < n; ++i) maxlen = Np[i + 1] - Np[i] > maxlen ? Np[i + 1] - Np[i] : maxlen;
  double *W = (double *)malloc((size_t)maxlen * nB * sizeof(double));
  for (int i = 0; i < n; ++i) {
    if (is_root[i]) continue;
    bad += row_pinv(Np[i + 1] - Np[i], Nj + Np[i], Bc, nB, W, Gp);
    for (int q = 0; q < nB; ++q) {
      double s = 0.0;
      for (int p = Np[i]; p < Np[i + 1]; ++p) s += V[p] * Bc[(long)Nj[p] * nB + q];
      r[q] = B[(long)i * nB + q] - s;
    }
    for (int q = 0; q < nB; ++q) {
      y[q] = 0.0;
      for (int u = 0; u < nB; ++u) y[q] += Gp[q * nB + u] * r[u];
    }
    for (int p = Np[i]; p < Np[i + 1]; ++p) {
      double u = 0.0;
      for (int q = 0; q < nB; ++q) u += Bc[(long)Nj[p] * nB + q] * y[q];
      V[p] += u;
    }
  }
  free(W);
  return bad;
}

/* ------------------------------------------------------------------------ */
/* filter, Alg. filter (Sec. 3.5 pre-filter of N, Sec. 3.7 post-filter of   */
/* P).  The rows of an n x (m n_agg) matrix G stored on a pattern whose DOF */
/* rows m I + c (c < m) share the node structure of node row I.  Each node  */
/* entry (I, a) has the magnitude g = max |G| over its m x m block.  The    */
/* entry in the row's own aggregate (a = agg[I]) plays the diagonal: it is  */
/* always kept and is not an "off-diagonal" entry.  With k > 0, off entries */
/* below the k-th largest off magnitude of the row are dropped; with        */
/* theta > 0, off entries below theta times the largest off magnitude.      */
/* Ties are kept.  Rows flagged in is_root (nullable) keep everything.      */
/* keep[p] is written for every stored DOF entry.                           */
/* ------------------------------------------------------------------------ */
static int cmp_desc(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x < y) - (x > y);
}

int orc_filter(int n, int m, const int *Np, const int *Nj, const double *G,
               const unsigned char *is_root, const int *agg, int k, double theta,
               unsigned char *keep) {
  if (m < 1 || n % m || k < 0 || !(theta >= 0.0)) return ORC_EINVAL;
  int maxlen = 1;
  for (int i = 0; i < n; ++i) maxlen = Np[i + 1] - Np[i] > maxlen ? Np[i + 1] - Np[i] : maxlen;
  double *g = (double *)malloc((size_t)maxlen * sizeof(double));
  double *srt = (double *)malloc((size_t)maxlen * sizeof(double));
  for (int I = 0; I < n / m; ++I) {
    const int i0 = m * I;
    const int len = (Np[i0 + 1] - Np[i0]) / m;  /* node entries of row I */
    int root = 0;
    for (int c = 0; c < m; ++c) root |= is_root ? is_root[i0 + c] : 0;
    if (root) {
      for (int c = 0; c < m; ++c)
        for (int p = Np[i0 + c]; p < Np[i0 + c + 1]; ++p) keep[p] = 1;
      continue;
    }
    int noff = 0;
    for (int q = 0; q < len; ++q) {
      double v = 0.0;
      for (int c = 0; c < m; ++c)
        for (int cc = 0; cc < m; ++cc) v = fmax(v, fabs(G[Np[i0 + c] + m * q + cc]));
      g[q] = v;
      if (Nj[Np[i0] + m * q] / m != agg[I]) srt[noff++] = v;
    }
    qsort(srt, (size_t)noff, sizeof(double), cmp_desc);
    for (int q = 0; q < len; ++q) {
      int kp = 1;
      if (Nj[Np[i0] + m * q] / m != agg[I]) {
        if (k > 0 && noff >= k && g[q] < srt[k - 1]) kp = 0;
        if (theta > 0.0 && noff > 0 && g[q] < theta * srt[0]) kp = 0;
      }
      for (int c = 0; c < m; ++c)
        for (int cc = 0; cc < m; ++cc) keep[Np[i0 + c] + m * q + cc] = (unsigned char)kp;
    }
  }
  free(g);
  free(srt);
  return ORC_OK;
}

/* The entries of (Np, Nj, V) with keep[p] set, in order: the compacted
 * pattern and values.  Returns the kept count. */
int orc_compact(int n, const int *Np, const int *Nj, const double *V,
                const unsigned char *keep, int *Np2, int *Nj2, double *V2) {
  int w = 0;
  Np2[0] = 0;
  for (int i = 0; i < n; ++i) {
    for (int p = Np[i]; p < Np[i + 1]; ++p)
      if (keep[p]) {
        Nj2[w] = Nj[p];
        if (V2) V2[w] = V ? V[p] : 0.0;
        ++w;
      }
    Np2[i + 1] = w;
  }
  return w;
}

/* ------------------------------------------------------------------------ */
/* improve by conjugate gradients, Sec. 3.6 and Sec. 4.1 (Lemma th:cg):     */
/* minimise E(P) = trace(P^T A P) over P in T + V, V = {U on N, zero root   */
/* rows, U Bc = 0}.  The gradient direction is -Pi(A P); the operator is    */
/* Pi A Pi restricted to V.                                                 */
/* ------------------------------------------------------------------------ */
int orc_emin_cg(int n, int nc, const int *Ap, const int *Aj, const double *Ax,
                const int *Np, const int *Nj, const unsigned char *is_root,
                const double *Bc, int nB, const double *T, int K, double *P,
                double *gam, double *del, double *alp, int *iters) {
  long nz = Np[n];
  size_t sz = (size_t)(nz > 0 ? nz : 1) * sizeof(double);
  double *R = (double *)malloc(sz), *D = (double *)malloc(sz), *Z = (double *)malloc(sz);
  double *Gp = (double *)malloc((size_t)n * (nB > 0 ? nB * nB : 1) * sizeof(double));
  orc_gram_rows(n, Np, Nj, is_root, Bc, nB, Gp);
  memcpy(P, T, (size_t)nz * sizeof(double));
  orc_masked_product(n, nc, Ap, Aj, Ax, Np, Nj, P, Z);
  orc_project(n, Np, Nj, is_root, Bc, nB, Gp, Z);
  for (long p = 0; p < nz; ++p) { R[p] = -Z[p]; D[p] = R[p]; }
  double g = dot(nz, R, R);
  const double g0 = g;
  if (gam) gam[0] = g;
  int rc = ORC_OK, it = 0;
  if (!isfinite(g)) rc = ORC_ENONFINITE;
  for (int k = 0; k < K && rc == ORC_OK; ++k) {
    if (g <= CG_STOP * g0) break;
    orc_masked_product(n, nc, Ap, Aj, Ax, Np, Nj, D, Z);
    orc_project(n, Np, Nj, is_root, Bc, nB, Gp, Z);
    double dl = dot(nz, D, Z);
    if (del) del[k] = dl;
    if (!isfinite(dl)) { rc = ORC_ENONFINITE; break; }
    if (dl <= 0.0) { rc = ORC_EBREAKDOWN; break; }
    double al = g / dl;
    if (alp) alp[k] = al;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < nz; ++p) {
      P[p] += al * D[p];
      R[p] -= al * Z[p];
    }
    double gn = dot(nz, R, R);
    if (gam) gam[k + 1] = gn;
    if (!isfinite(gn)) { rc = ORC_ENONFINITE; break; }
    double be = gn / g;
    g = gn;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < nz; ++p) D[p] = R[p] + be * D[p];
    ++it;
  }
  if (iters) *iters = it;
  free(R); free(D); free(Z); free(Gp);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Tangent-linear model of orc_emin_cg: every statement above differentiated */
/* in direction dA (A's stored values), pattern and T held fixed.            */
/* ------------------------------------------------------------------------ */
int orc_emin_cg_jvp(int n, int nc, const int *Ap, const int *Aj,
                    const double *Ax, const double *dAx, const int *Np,
                    const int *Nj, const unsigned char *is_root,
                    const double *Bc, int nB, const double *T, int K,
                    double *P, double *dP) {
  long nz = Np[n];
  size_t sz = (size_t)(nz > 0 ? nz : 1) * sizeof(double);
  double *R = (double *)malloc(sz), *D = (double *)malloc(sz), *Z = (double *)malloc(sz);
  double *dR = (double *)malloc(sz), *dD = (double *)malloc(sz), *dZ = (double *)malloc(sz);
  double *tmp = (double *)malloc(sz);
  double *Gp = (double *)malloc((size_t)n * (nB > 0 ? nB * nB : 1) * sizeof(double));
  orc_gram_rows(n, Np, Nj, is_root, Bc, nB, Gp);
  memcpy(P, T, (size_t)nz * sizeof(double));
  for (long p = 0; p < nz; ++p) dP[p] = 0.0;
  /* R = -Pi(A P), dR = -Pi(dA P) */
  orc_masked_product(n, nc, Ap, Aj, Ax, Np, Nj, P, Z);
  orc_project(n, Np, Nj, is_root, Bc, nB, Gp, Z);
  orc_masked_product(n, nc, Ap, Aj, dAx, Np, Nj, P, dZ);
  orc_project(n, Np, Nj, is_root, Bc, nB, Gp, dZ);
  for (long p = 0; p < nz; ++p) {
    R[p] = -Z[p]; D[p] = R[p];
    dR[p] = -dZ[p]; dD[p] = dR[p];
  }
  double g = dot(nz, R, R), dg = 2.0 * dot(nz, R, dR);
  const double g0 = g;
  int rc = isfinite(g) ? ORC_OK : ORC_ENONFINITE;
  for (int k = 0; k < K && rc == ORC_OK; ++k) {
    if (g <= CG_STOP * g0) break;
    /* Z = Pi(A D), dZ = Pi(dA D + A dD) */
    orc_masked_product(n, nc, Ap, Aj, Ax, Np, Nj, D, Z);
    orc_project(n, Np, Nj, is_root, Bc, nB, Gp, Z);
    orc_masked_product(n, nc, Ap, Aj, dAx, Np, Nj, D, dZ);
    orc_masked_product(n, nc, Ap, Aj, Ax, Np, Nj, dD, tmp);
    for (long p = 0; p < nz; ++p) dZ[p] += tmp[p];
    orc_project(n, Np, Nj, is_root, Bc, nB, Gp, dZ);
    double dl = dot(nz, D, Z);
    double ddl = dot(nz, dD, Z) + dot(nz, D, dZ);
    if (!isfinite(dl)) { rc = ORC_ENONFINITE; break; }
    if (dl <= 0.0) { rc = ORC_EBREAKDOWN; break; }
    double al = g / dl;
    double dal = (dg * dl - g * ddl) / (dl * dl);
    for (long p = 0; p < nz; ++p) {
      dP[p] += dal * D[p] + al * dD[p];
      P[p] += al * D[p];
      dR[p] -= dal * Z[p] + al * dZ[p];
      R[p] -= al * Z[p];
    }
    double gn = dot(nz, R, R), dgn = 2.0 * dot(nz, R, dR);
    double be = gn / g;
    double dbe = (dgn * g - gn * dg) / (g * g);
    g = gn;
    dg = dgn;
    for (long p = 0; p < nz; ++p) {
      dD[p] = dR[p] + dbe * D[p] + be * dD[p];
      D[p] = R[p] + be * D[p];
    }
  }
  free(R); free(D); free(Z); free(dR); free(dD); free(dZ); free(tmp); free(Gp);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* improve by GMRES, Sec. 3.6 and Sec. 4.2 (non-symmetric A): minimise      */
/* ||Pi(A P)||_F over T plus the Krylov space of Pi A Pi from               */
/* R_0 = -Pi(A T).  Unrestarted, modified Gram-Schmidt in the Frobenius     */
/* inner product on N, Givens rotations for the small least-squares problem.*/
/* ------------------------------------------------------------------------ */
int orc_emin_gmres(int n, int nc, const int *Ap, const int *Aj,
                   const double *Ax, const int *Np, const int *Nj,
                   const unsigned char *is_root, const double *Bc, int nB,
                   const double *T, int K, double *P, double *resid,
                   int *iters) {
  long nz = Np[n];
  size_t sz = (size_t)(nz > 0 ? nz : 1) * sizeof(double);
  double **V = (double **)malloc((size_t)(K + 1) * sizeof(double *));
  for (int k = 0; k <= K; ++k) V[k] = (double *)malloc(sz);
  double *W = (double *)malloc(sz);
  double *H = (double *)calloc((size_t)(K + 1) * (K > 0 ? K : 1), sizeof(double));
#define HH(i, j) H[(long)(i) * (K > 0 ? K : 1) + (j)]
  double *cs = (double *)calloc((size_t)(K + 1), sizeof(double));
  double *sn = (double *)calloc((size_t)(K + 1), sizeof(double));
  double *gv = (double *)calloc((size_t)(K + 2), sizeof(double));
  double *Gp = (double *)malloc((size_t)n * (nB > 0 ? nB * nB : 1) * sizeof(double));
  orc_gram_rows(n, Np, Nj, is_root, Bc, nB, Gp);
  memcpy(P, T, (size_t)nz * sizeof(double));
  orc_masked_product(n, nc, Ap, Aj, Ax, Np, Nj, P, W);
  orc_project(n, Np, Nj, is_root, Bc, nB, Gp, W);
  for (long p = 0; p < nz; ++p) V[0][p] = -W[p];
  double beta = sqrt(dot(nz, V[0], V[0]));
  if (resid) resid[0] = beta;
  int rc = isfinite(beta) ? ORC_OK : ORC_ENONFINITE;
  int kd = 0;
  if (rc == ORC_OK && beta > 0.0) {
    for (long p = 0; p < nz; ++p) V[0][p] /= beta;
    gv[0] = beta;
    for (int k = 0; k < K; ++k) {
      orc_masked_product(n, nc, Ap, Aj, Ax, Np, Nj, V[k], W);
      orc_project(n, Np, Nj, is_root, Bc, nB, Gp, W);
      for (int j = 0; j <= k; ++j) {
        double h = dot(nz, W, V[j]);
        HH(j, k) = h;
        const double *Vj = V[j];
#pragma omp parallel for schedule(static)
        for (long p = 0; p < nz; ++p) W[p] -= h * Vj[p];
      }
      double hn = sqrt(dot(nz, W, W));
      if (!isfinite(hn)) { rc = ORC_ENONFINITE; break; }
      HH(k + 1, k) = hn;
      /* apply earlier rotations to column k, then a new one */
      for (int j = 0; j < k; ++j) {
        double a = HH(j, k), b = HH(j + 1, k);
        HH(j, k) = cs[j] * a + sn[j] * b;
        HH(j + 1, k) = -sn[j] * a + cs[j] * b;
      }
      double a = HH(k, k), b = HH(k + 1, k);
      double r = hypot(a, b);
      cs[k] = a / r;
      sn[k] = b / r;
      HH(k, k) = r;
      HH(k + 1, k) = 0.0;
      gv[k + 1] = -sn[k] * gv[k];
      gv[k] = cs[k] * gv[k];
      if (resid) resid[k + 1] = fabs(gv[k + 1]);
      kd = k + 1;
      /* invariant Krylov space, or converged to round-off */
      if (hn == 0.0 || fabs(gv[k + 1]) <= GM_STOP * beta) break;
      double *Vn = V[k + 1];
#pragma omp parallel for schedule(static)
      for (long p = 0; p < nz; ++p) Vn[p] = W[p] / hn;
    }
    if (rc == ORC_OK) {
      double *y = (double *)calloc((size_t)(kd > 0 ? kd : 1), sizeof(double));
      for (int j = kd - 1; j >= 0; --j) {
        double s = gv[j];
        for (int l = j + 1; l < kd; ++l) s -= HH(j, l) * y[l];
        y[j] = s / HH(j, j);
      }
      for (int j = 0; j < kd; ++j) {
        const double yj = y[j], *Vj = V[j];
#pragma omp parallel for schedule(static)
        for (long p = 0; p < nz; ++p) P[p] += yj * Vj[p];
      }
      free(y);
    }
  }
#undef HH
  if (iters) *iters = kd;
  for (int k = 0; k <= K; ++k) free(V[k]);
  free(V); free(W); free(H); free(cs); free(sn); free(gv); free(Gp);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Metrics and utilities                                                    */
/* ------------------------------------------------------------------------ */
void orc_transpose(int n_rows, int n_cols, const int *Ap, const int *Aj,
                   const double *Ax, int *Tp, int *Tj, double *Tx) {
  for (int j = 0; j <= n_cols; ++j) Tp[j] = 0;
  for (int p = 0; p < Ap[n_rows]; ++p) Tp[Aj[p] + 1]++;
  for (int j = 0; j < n_cols; ++j) Tp[j + 1] += Tp[j];
  int *w = (int *)malloc((size_t)(n_cols > 0 ? n_cols : 1) * sizeof(int));
  for (int j = 0; j < n_cols; ++j) w[j] = Tp[j];
  for (int i = 0; i < n_rows; ++i)
    for (int p = Ap[i]; p < Ap[i + 1]; ++p) {
      int q = w[Aj[p]]++;
      Tj[q] = i;
      Tx[q] = Ax[p];
    }
  free(w);
}

double orc_energy(int n, int nc, const int *Ap, const int *Aj, const double *Ax,
                  const int *Np, const int *Nj, const double *P) {
  long nz = Np[n];
  double *Y = (double *)malloc((size_t)(nz > 0 ? nz : 1) * sizeof(double));
  orc_masked_product(n, nc, Ap, Aj, Ax, Np, Nj, P, Y);
  double e = dot(nz, P, Y);
  free(Y);
  return e;
}

double orc_constraint_residual(int n, const int *Np, const int *Nj,
                               const double *P, const double *Bc,
                               const double *B, int nB) {
  double mx = 0.0;
  for (int i = 0; i < n; ++i)
    for (int q = 0; q < nB; ++q) {
      double s = 0.0;
      for (int p = Np[i]; p < Np[i + 1]; ++p) s += P[p] * Bc[(long)Nj[p] * nB + q];
      mx = fmax(mx, fabs(s - B[(long)i * nB + q]));
    }
  return mx;
}

/* ------------------------------------------------------------------------ */
/* Sparse product C = X Y (Gustavson, row by row): the Galerkin product of  */
/* Sec. 3.8 as two such products, and the pattern powers of Sec. 3.4 with   */
/* values.  Each row of C holds the union of the columns of the rows of Y   */
/* that the row of X selects, sorted; each value is accumulated in the      */
/* order of X's row (terms of one column added in that order from 0).       */
/* Returns nnz(C), or ORC_ECAP when it exceeds cap (Cj, Cx not written past */
/* cap).  Xx, Yx, Cx nullable: structure only.                              */
/* ------------------------------------------------------------------------ */
int orc_spgemm(int rows, int inner, int cols, const int *Xp, const int *Xj,
               const double *Xx, const int *Yp, const int *Yj, const double *Yx,
               int *Cp, int *Cj, double *Cx, long cap) {
  (void)inner;
  int *mark = (int *)malloc((size_t)(cols > 0 ? cols : 1) * sizeof(int));
  double *acc = (double *)calloc((size_t)(cols > 0 ? cols : 1), sizeof(double));
  for (int j = 0; j < cols; ++j) mark[j] = -1;
  long w = 0;
  int rc = 0;
  Cp[0] = 0;
  for (int i = 0; i < rows; ++i) {
    const long r0 = w;
    for (int t = Xp[i]; t < Xp[i + 1]; ++t) {
      const int k = Xj[t];
      for (int q = Yp[k]; q < Yp[k + 1]; ++q) {
        const int j = Yj[q];
        if (mark[j] != i) {
          mark[j] = i;
          if (w < cap) Cj[w] = j;
          ++w;
        }
        if (Xx && Yx) acc[j] += Xx[t] * Yx[q];
      }
    }
    if (w <= cap) {
      qsort(Cj + r0, (size_t)(w - r0), sizeof(int), cmp_int);
      for (long p = r0; p < w; ++p) {
        if (Cx) Cx[p] = acc[Cj[p]];
        acc[Cj[p]] = 0.0;
      }
    } else {
      rc = ORC_ECAP;
      for (int j = 0; j < cols; ++j) acc[j] = 0.0;
    }
    Cp[i + 1] = (int)(w < cap ? w : cap);
  }
  free(mark);
  free(acc);
  return rc < 0 ? rc : (int)w;
}

/* ------------------------------------------------------------------------ */
/* Strength values normalised as Eq. soc (Sec. 3.2), on the node graph S   */
/* made by orc_strength with the same A, m and theta.  The value of node    */
/* entry (I, J), J != I, is the largest |a_ij| over the strong DOF entries  */
/* of block (I, J) and over those of block (J, I) (S u S^T taken as the     */
/* entry-wise maximum; amalgamation takes the block's largest entry).  Each */
/* row is then divided by its largest off-diagonal value and its diagonal   */
/* set to 1, so that both equal 1 (rows whose off values are all 0 keep 0). */
/* ------------------------------------------------------------------------ */
static int find_col(const int *Sj, int s, int e, int J) {
  for (int p = s; p < e; ++p)
    if (Sj[p] == J) return p;
  return -1;
}

int orc_strength_values(int n, const int *Ap, const int *Aj, const double *Ax, int m,
                        double theta, const int *Sp, const int *Sj, double *Sx) {
  if (m < 1 || n % m) return ORC_EINVAL;
  const int nn = n / m;
  double *diag = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  for (int i = 0; i < n; ++i)
    for (int p = Ap[i]; p < Ap[i + 1]; ++p)
      if (Aj[p] == i) diag[i] = Ax[p];
  for (long q = 0; q < Sp[nn]; ++q) Sx[q] = 0.0;
  const double th2 = theta * theta;
  for (int i = 0; i < n; ++i) {
    for (int p = Ap[i]; p < Ap[i + 1]; ++p) {
      const int j = Aj[p];
      const int I = i / m, J = j / m;
      if (I == J) continue;
      const double lhs = Ax[p] * Ax[p];
      const double rhs = th2 * fabs(diag[i] * diag[j]);
      if (!(lhs >= rhs)) continue;
      const double v = fabs(Ax[p]);
      const int q1 = find_col(Sj, Sp[I], Sp[I + 1], J), q2 = find_col(Sj, Sp[J], Sp[J + 1], I);
      if (q1 < 0 || q2 < 0) { free(diag); return ORC_EINVAL; }
      Sx[q1] = fmax(Sx[q1], v);
      Sx[q2] = fmax(Sx[q2], v);
    }
  }
  for (int I = 0; I < nn; ++I) {
    double mx = 0.0;
    for (int q = Sp[I]; q < Sp[I + 1]; ++q)
      if (Sj[q] != I) mx = fmax(mx, Sx[q]);
    for (int q = Sp[I]; q < Sp[I + 1]; ++q) {
      if (Sj[q] == I) Sx[q] = 1.0;
      else if (mx > 0.0) Sx[q] = Sx[q] / mx;
    }
  }
  free(diag);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Candidate smoothing, the smooth line of Alg. root_node_setup (Sec. 3.1): */
/* relaxation sweeps on A B = 0, here damped Jacobi (reading R28):          */
/* B <- B - omega D^-1 A B, all nB columns, the row sums of A B taken in    */
/* the order of A's row.  A is scalar CSR; D its diagonal.                  */
/* ------------------------------------------------------------------------ */
int orc_smooth_candidates(int n, const int *Ap, const int *Aj, const double *Ax,
                          double *B, int nB, int sweeps, double omega) {
  if (nB < 1 || sweeps < 0) return ORC_EINVAL;
  double *d = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double *Bn = (double *)malloc((size_t)(n > 0 ? n : 1) * nB * sizeof(double));
  for (int i = 0; i < n; ++i)
    for (int p = Ap[i]; p < Ap[i + 1]; ++p)
      if (Aj[p] == i) d[i] = Ax[p];
  for (int i = 0; i < n; ++i)
    if (d[i] == 0.0) { free(d); free(Bn); return ORC_ESINGULAR; }
  for (int sw = 0; sw < sweeps; ++sw) {
    for (int i = 0; i < n; ++i)
      for (int q = 0; q < nB; ++q) {
        double y = 0.0;
        for (int p = Ap[i]; p < Ap[i + 1]; ++p) y += Ax[p] * B[(long)Aj[p] * nB + q];
        Bn[(long)i * nB + q] = B[(long)i * nB + q] - omega * (y / d[i]);
      }
    memcpy(B, Bn, (size_t)n * nB * sizeof(double));
  }
  free(d);
  free(Bn);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* improve by Jacobi-preconditioned CG (reading R29): CG on the same energy */
/* with the preconditioner Y = Pi(D^-1 R), D = diag(A) scaling each row of  */
/* the residual (Pi D^-1 Pi is symmetric positive definite on V when A's    */
/* diagonal is positive, so the iteration minimises the same E(P) over the */
/* preconditioned Krylov space).  gam holds <R_k, Y_k>.                     */
/* ------------------------------------------------------------------------ */
static void precondition(int n, const int *Ap, const int *Aj, const double *Ax, const int *Np,
                         const int *Nj, const unsigned char *is_root, const double *Bc, int nB,
                         const double *Gp, const double *R, double *Y) {
  for (int i = 0; i < n; ++i) {
    double d = 0.0;
    for (int p = Ap[i]; p < Ap[i + 1]; ++p)
      if (Aj[p] == i) d = Ax[p];
    for (int p = Np[i]; p < Np[i + 1]; ++p) Y[p] = R[p] / d;
  }
  orc_project(n, Np, Nj, is_root, Bc, nB, Gp, Y);
}

int orc_emin_pcg(int n, int nc, const int *Ap, const int *Aj, const double *Ax,
                 const int *Np, const int *Nj, const unsigned char *is_root,
                 const double *Bc, int nB, const double *T, int K, double *P,
                 double *gam, double *del, double *alp, int *iters) {
  long nz = Np[n];
  size_t sz = (size_t)(nz > 0 ? nz : 1) * sizeof(double);
  double *R = (double *)malloc(sz), *D = (double *)malloc(sz), *Z = (double *)malloc(sz);
  double *Y = (double *)malloc(sz);
  double *Gp = (double *)malloc((size_t)n * (nB > 0 ? nB * nB : 1) * sizeof(double));
  orc_gram_rows(n, Np, Nj, is_root, Bc, nB, Gp);
  memcpy(P, T, (size_t)nz * sizeof(double));
  orc_masked_product(n, nc, Ap, Aj, Ax, Np, Nj, P, Z);
  orc_project(n, Np, Nj, is_root, Bc, nB, Gp, Z);
  for (long p = 0; p < nz; ++p) R[p] = -Z[p];
  precondition(n, Ap, Aj, Ax, Np, Nj, is_root, Bc, nB, Gp, R, Y);
  memcpy(D, Y, (size_t)nz * sizeof(double));
  double g = dot(nz, R, Y);
  const double g0 = g;
  if (gam) gam[0] = g;
  int rc = ORC_OK, it = 0;
  if (!isfinite(g)) rc = ORC_ENONFINITE;
  for (int k = 0; k < K && rc == ORC_OK; ++k) {
    if (g <= CG_STOP * g0) break;
    orc_masked_product(n, nc, Ap, Aj, Ax, Np, Nj, D, Z);
    orc_project(n, Np, Nj, is_root, Bc, nB, Gp, Z);
    double dl = dot(nz, D, Z);
    if (del) del[k] = dl;
    if (!isfinite(dl)) { rc = ORC_ENONFINITE; break; }
    if (dl <= 0.0) { rc = ORC_EBREAKDOWN; break; }
    double al = g / dl;
    if (alp) alp[k] = al;
    for (long p = 0; p < nz; ++p) {
      P[p] += al * D[p];
      R[p] -= al * Z[p];
    }
    precondition(n, Ap, Aj, Ax, Np, Nj, is_root, Bc, nB, Gp, R, Y);
    double gn = dot(nz, R, Y);
    if (gam) gam[k + 1] = gn;
    if (!isfinite(gn)) { rc = ORC_ENONFINITE; break; }
    double be = gn / g;
    g = gn;
    for (long p = 0; p < nz; ++p) D[p] = Y[p] + be * D[p];
    ++it;
  }
  if (iters) *iters = it;
  free(R); free(D); free(Z); free(Y); free(Gp);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* improve by CGNR (Sec. 4.2: energy minimisation in the A*A norm for a     */
/* non-symmetric A): minimise ||A P||_F^2 = trace(P^T A^T A P), the product */
/* A P taken whole (not kept to N), over P in T + V.  The gradient          */
/* direction is -Pi(A^T (A P)) kept to N; CG on Pi A^T A Pi.                */
/* ------------------------------------------------------------------------ */
/* Z = (A^T W) on the pattern N, W a CSR matrix on any pattern. */
static void masked_product_gen(int n, int nc, const int *Tp, const int *Tj, const double *Tx,
                               const int *Wp, const int *Wj, const double *Wx, const int *Np,
                               const int *Nj, double *Z) {
  double *acc = (double *)calloc((size_t)(nc > 0 ? nc : 1), sizeof(double));
  for (int i = 0; i < n; ++i) {
    for (int t = Tp[i]; t < Tp[i + 1]; ++t) {
      const int k = Tj[t];
      for (int q = Wp[k]; q < Wp[k + 1]; ++q) acc[Wj[q]] += Tx[t] * Wx[q];
    }
    for (int p = Np[i]; p < Np[i + 1]; ++p) Z[p] = acc[Nj[p]];
    for (int t = Tp[i]; t < Tp[i + 1]; ++t) {
      const int k = Tj[t];
      for (int q = Wp[k]; q < Wp[k + 1]; ++q) acc[Wj[q]] = 0.0;
    }
  }
  free(acc);
}

/* Z = Pi(A^T (A X)): the full product W = A X (orc_spgemm), then A^T W kept
 * to N, then the projection. */
static void normal_product(int n, int nc, const int *Ap, const int *Aj, const double *Ax,
                           const int *Tp, const int *Tj, const double *Tx, const int *Np,
                           const int *Nj, const unsigned char *is_root, const double *Bc, int nB,
                           const double *Gp, const double *X, int *Wp, int *Wj, double *Wx,
                           long wcap, double *Z) {
  orc_spgemm(n, n, nc, Ap, Aj, Ax, Np, Nj, X, Wp, Wj, Wx, wcap);
  masked_product_gen(n, nc, Tp, Tj, Tx, Wp, Wj, Wx, Np, Nj, Z);
  orc_project(n, Np, Nj, is_root, Bc, nB, Gp, Z);
}

int orc_emin_cgnr(int n, int nc, const int *Ap, const int *Aj, const double *Ax,
                  const int *Np, const int *Nj, const unsigned char *is_root,
                  const double *Bc, int nB, const double *T, int K, double *P,
                  double *gam, double *del, double *alp, int *iters) {
  long nz = Np[n];
  size_t sz = (size_t)(nz > 0 ? nz : 1) * sizeof(double);
  double *R = (double *)malloc(sz), *D = (double *)malloc(sz), *Z = (double *)malloc(sz);
  double *Gp = (double *)malloc((size_t)n * (nB > 0 ? nB * nB : 1) * sizeof(double));
  const long nzA = Ap[n];
  int *Tp = (int *)malloc((size_t)(n + 1) * sizeof(int));
  int *Tj = (int *)malloc((size_t)(nzA > 0 ? nzA : 1) * sizeof(int));
  double *Tx = (double *)malloc((size_t)(nzA > 0 ? nzA : 1) * sizeof(double));
  orc_transpose(n, n, Ap, Aj, Ax, Tp, Tj, Tx);
  /* the pattern of A X has at most nnz(A) max-row(N) entries per row sum */
  int maxr = 1;
  for (int i = 0; i < n; ++i) maxr = Np[i + 1] - Np[i] > maxr ? Np[i + 1] - Np[i] : maxr;
  const long wcap = nzA * (long)maxr + 1;
  int *Wp = (int *)malloc((size_t)(n + 1) * sizeof(int));
  int *Wj = (int *)malloc((size_t)wcap * sizeof(int));
  double *Wx = (double *)malloc((size_t)wcap * sizeof(double));
  orc_gram_rows(n, Np, Nj, is_root, Bc, nB, Gp);
  memcpy(P, T, (size_t)nz * sizeof(double));
  normal_product(n, nc, Ap, Aj, Ax, Tp, Tj, Tx, Np, Nj, is_root, Bc, nB, Gp, P, Wp, Wj, Wx, wcap, Z);
  for (long p = 0; p < nz; ++p) { R[p] = -Z[p]; D[p] = R[p]; }
  double g = dot(nz, R, R);
  const double g0 = g;
  if (gam) gam[0] = g;
  int rc = ORC_OK, it = 0;
  if (!isfinite(g)) rc = ORC_ENONFINITE;
  for (int k = 0; k < K && rc == ORC_OK; ++k) {
    if (g <= CG_STOP * g0) break;
    normal_product(n, nc, Ap, Aj, Ax, Tp, Tj, Tx, Np, Nj, is_root, Bc, nB, Gp, D, Wp, Wj, Wx, wcap, Z);
    double dl = dot(nz, D, Z);
    if (del) del[k] = dl;
    if (!isfinite(dl)) { rc = ORC_ENONFINITE; break; }
    if (dl <= 0.0) { rc = ORC_EBREAKDOWN; break; }
    double al = g / dl;
    if (alp) alp[k] = al;
    for (long p = 0; p < nz; ++p) {
      P[p] += al * D[p];
      R[p] -= al * Z[p];
    }
    double gn = dot(nz, R, R);
    if (gam) gam[k + 1] = gn;
    if (!isfinite(gn)) { rc = ORC_ENONFINITE; break; }
    double be = gn / g;
    g = gn;
    for (long p = 0; p < nz; ++p) D[p] = R[p] + be * D[p];
    ++it;
  }
  if (iters) *iters = it;
  free(R); free(D); free(Z); free(Gp); free(Tp); free(Tj); free(Tx); free(Wp); free(Wj); free(Wx);
  return rc;
}
