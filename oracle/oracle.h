/*
 * oracle.h -- plain, slow, obviously-correct FP64 CPU reference of the
 * root-node AMG interpolation setup (Manteuffel, Olson, Schroder, Southworth,
 * "A Root-Node Based Algebraic Multigrid Method").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library, and the HIP library never
 * calls it.
 *
 * Conventions: int indices (0-based), CSR with sorted unique column indices,
 * double values, host memory owned by the caller.  Functions that produce a
 * sparse structure take an output capacity and return the produced count, or
 * ORC_ECAP when the capacity is too small.  No function allocates memory that
 * outlives the call.
 *
 * Parity status of each function (see tests/test_oracle_*.py for the pins):
 *   orc_strength, orc_aggregate, orc_pattern_nodes, orc_pattern_dofs,
 *   orc_tentative, orc_gram_pinv, orc_project, orc_masked_product,
 *   orc_emin_cg, orc_emin_gmres, orc_transpose, orc_energy,
 *   orc_constraint_residual, orc_emin_cg_jvp            -- pinned.
 *   orc_set_threads, orc_threads: thread control, no arithmetic.
 */
#ifndef RN_ORACLE_H
#define RN_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK         0
#define ORC_ECAP      -1  /* output capacity too small                     */
#define ORC_ESINGULAR -2  /* singular root block of B (Eq. root-nodeform)  */
#define ORC_EBREAKDOWN -3 /* CG curvature <D, Pi(A D)> <= 0                */
#define ORC_ENONFINITE -4 /* NaN or Inf in a Krylov scalar                 */
#define ORC_EINVAL    -5  /* malformed input                               */

/* Threads of the loops over rows and entries (OpenMP); the results do not
 * depend on the number (fixed summation chunks). */
void orc_set_threads(int n);
int orc_threads(void);

/* Symmetric strength of connection (Sec. 3.2, Alg. root_node_setup strength
 * and amalgamate steps).  Keeps (i,i) and stored (i,j) with
 * a_ij^2 >= theta^2 |a_ii a_jj|.  For block size m > 1 the DOF-level result
 * is amalgamated to nodes by a boolean OR over each m x m block, then
 * symmetrised.  Sp has n/m + 1 entries.  Returns nnz(S) or ORC_ECAP. */
int orc_strength(int n, const int *Ap, const int *Aj, const double *Ax, int m,
                 double theta, int *Sp, int *Sj, int cap);

/* Standard greedy aggregation with root nodes (Sec. 3.3).  Returns n_agg.
 * agg has nn entries, roots must hold nn entries (only n_agg are used). */
int orc_aggregate(int nn, const int *Sp, const int *Sj, int *agg, int *roots);

/* Nodal pattern N = S^d C as a boolean product (Sec. 3.4).  Np: nn + 1.
 * Returns nnz or ORC_ECAP. */
int orc_pattern_nodes(int nn, const int *Sp, const int *Sj, const int *agg,
                      int n_agg, int d, int *Np, int *Nj, int cap);

/* unamalgamate + root_node_pattern (Sec. 3.4): DOF pattern n x (m n_agg),
 * root DOF rows replaced by the identity row.  Np: m*nn + 1, is_root: m*nn.
 * Returns nnz or ORC_ECAP. */
int orc_pattern_dofs(int nn, int m, const int *Npn, const int *Njn,
                     const int *agg, const int *roots, int n_agg,
                     int *Np, int *Nj, int cap, unsigned char *is_root);

/* inject (Sec. 3.6, Eq. root-nodeform, Eq. Tproj): coarse candidates Bc
 * (m*n_agg x nB, row-major) and tentative T on the pattern.  When nB > m the
 * remaining candidates are projected into T row by row (Eq. Tproj).
 * Returns ORC_OK or ORC_ESINGULAR; *rank_def counts rows whose Gram matrix
 * needed the pseudo-inverse fallback. */
int orc_tentative(int n, int m, const int *Np, const int *Nj,
                  const unsigned char *is_root, const int *agg,
                  const int *roots, int n_agg, const double *B, int nB,
                  double *T, double *Bc, int *rank_def);

/* Pseudo-inverse of a symmetric nB x nB Gram matrix (row-major).  LDL^T when
 * every pivot exceeds 1e-12 max(diag); otherwise a Jacobi eigen-decomposition
 * with cutoff 1e-12 lambda_max.  Returns 1 when the fallback was taken. */
int orc_gram_pinv(int nB, const double *G, double *Gp);

/* Per F row i: Gp_i = pinv(B_Ji^T B_Ji) (nB*nB doubles per row, zero on
 * root rows).  Returns the number of rows that took the fallback. */
int orc_gram_rows(int n, const int *Np, const int *Nj,
                  const unsigned char *is_root, const double *Bc, int nB,
                  double *Gp);

/* Pi = Pi_B o M in place: zero root rows; on F rows subtract the orthogonal
 * projection of x_i onto the row space of B_Ji^T.  Gp from orc_gram_rows. */
void orc_project(int n, const int *Np, const int *Nj,
                 const unsigned char *is_root, const double *Bc, int nB,
                 const double *Gp, double *X);

/* Z = (A X) restricted to the pattern N, all rows.  X, Z aligned with N. */
void orc_masked_product(int n, int nc, const int *Ap, const int *Aj,
                        const double *Ax, const int *Np, const int *Nj,
                        const double *X, double *Z);

/* Energy-minimisation by K steps of unpreconditioned CG (Sec. 3.6 improve,
 * Sec. 4.1 Lemma th:cg).  gam: K+1, del/alp: K (each nullable).  Returns
 * ORC_OK / ORC_EBREAKDOWN / ORC_ENONFINITE; *iters = steps taken. */
int orc_emin_cg(int n, int nc, const int *Ap, const int *Aj, const double *Ax,
                const int *Np, const int *Nj, const unsigned char *is_root,
                const double *Bc, int nB, const double *T, int K, double *P,
                double *gam, double *del, double *alp, int *iters);

/* Energy-minimisation by K steps of unrestarted GMRES with modified
 * Gram-Schmidt (Sec. 3.6 improve, Sec. 4.2).  resid: K+1 (nullable) holds
 * ||Pi(A P_k)||_F.  Returns ORC_OK / ORC_ENONFINITE. */
int orc_emin_gmres(int n, int nc, const int *Ap, const int *Aj,
                   const double *Ax, const int *Np, const int *Nj,
                   const unsigned char *is_root, const double *Bc, int nB,
                   const double *T, int K, double *P, double *resid,
                   int *iters);

/* Plain CSR transpose (n_rows x n_cols -> n_cols x n_rows). */
void orc_transpose(int n_rows, int n_cols, const int *Ap, const int *Aj,
                   const double *Ax, int *Tp, int *Tj, double *Tx);

/* E(P) = sum over N of P_ij (A P)_ij = trace(P^T A P). */
double orc_energy(int n, int nc, const int *Ap, const int *Aj, const double *Ax,
                  const int *Np, const int *Nj, const double *P);

/* max |P Bc - B| over all rows and candidates (Eq. mode_constraint). */
double orc_constraint_residual(int n, const int *Np, const int *Nj,
                               const double *P, const double *Bc,
                               const double *B, int nB);

/* Eq. Tproj as enforce (Sec. 3.7): on every F row of V (values on the
 * pattern Np/Nj), the minimum-norm update that restores V Bc = B.  Root rows
 * untouched.  Returns the count of rows whose Gram matrix took the eigen
 * pseudo-inverse, or ORC_EINVAL. */
int orc_enforce(int n, const int *Np, const int *Nj, const unsigned char *is_root,
                const double *Bc, int nB, const double *B, double *V);

/* Alg. filter on node blocks (Sec. 3.5 pre-filter, Sec. 3.7 post-filter):
 * keep[p] for every stored entry of G (n DOF rows, m DOFs per node, DOF rows
 * of one node sharing its node structure).  Block magnitude = max |G| over
 * the m x m block; the own-aggregate entry (node column agg[I]) is the row's
 * diagonal and always kept; off entries below the k-th largest off
 * magnitude (k > 0) or below theta times the largest (theta > 0) dropped;
 * rows with is_root set (nullable) kept whole. */
int orc_filter(int n, int m, const int *Np, const int *Nj, const double *G,
               const unsigned char *is_root, const int *agg, int k, double theta,
               unsigned char *keep);

/* Kept entries of a pattern and its values (V, V2 nullable); returns the
 * kept count. */
int orc_compact(int n, const int *Np, const int *Nj, const double *V,
                const unsigned char *keep, int *Np2, int *Nj2, double *V2);

/* C = X Y for CSR X (rows x inner) and Y (inner x cols): rows of C sorted,
 * values accumulated in the order of X's row (Sec. 3.8 Galerkin product,
 * Sec. 3.4 valued pattern powers).  Returns nnz(C) or ORC_ECAP (> cap). */
int orc_spgemm(int rows, int inner, int cols, const int *Xp, const int *Xj,
               const double *Xx, const int *Yp, const int *Yj, const double *Yx,
               int *Cp, int *Cj, double *Cx, long cap);

/* Eq. soc values on the node graph S of orc_strength (same A, m, theta):
 * off entry (I, J) = largest |a_ij| over strong DOF entries of blocks (I, J)
 * and (J, I); each row divided by its largest off value; diagonal 1. */
int orc_strength_values(int n, const int *Ap, const int *Aj, const double *Ax, int m,
                        double theta, const int *Sp, const int *Sj, double *Sx);

/* Candidate smoothing (the smooth line of Alg. root_node_setup): `sweeps`
 * damped Jacobi sweeps B <- B - omega D^-1 A B on A B = 0 (B: n x nB,
 * row-major, in place).  ORC_ESINGULAR for a zero diagonal entry. */
int orc_smooth_candidates(int n, const int *Ap, const int *Aj, const double *Ax,
                          double *B, int nB, int sweeps, double omega);

/* Jacobi-preconditioned CG energy minimisation: as orc_emin_cg with the
 * preconditioner Y = Pi(D^-1 R); gam holds <R_k, Y_k>. */
int orc_emin_pcg(int n, int nc, const int *Ap, const int *Aj, const double *Ax,
                 const int *Np, const int *Nj, const unsigned char *is_root,
                 const double *Bc, int nB, const double *T, int K, double *P,
                 double *gam, double *del, double *alp, int *iters);

/* CGNR energy minimisation (Sec. 4.2, A*A norm): minimises ||A P||_F^2 with
 * A P taken whole; direction -Pi(A^T (A P)) kept to N. */
int orc_emin_cgnr(int n, int nc, const int *Ap, const int *Aj, const double *Ax,
                  const int *Np, const int *Nj, const unsigned char *is_root,
                  const double *Bc, int nB, const double *T, int K, double *P,
                  double *gam, double *del, double *alp, int *iters);

/* Tangent-linear (forward-mode) derivative of orc_emin_cg with respect to
 * the stored values of A in direction dAx.  Pattern, T and Bc are constants.
 * Writes P (as orc_emin_cg) and dP.  Returns as orc_emin_cg. */
int orc_emin_cg_jvp(int n, int nc, const int *Ap, const int *Aj,
                    const double *Ax, const double *dAx, const int *Np,
                    const int *Nj, const unsigned char *is_root,
                    const double *Bc, int nB, const double *T, int K,
                    double *P, double *dP);

#ifdef __cplusplus
}
#endif
#endif
