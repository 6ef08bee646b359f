/*
 * rnamg.h -- C ABI of librnamg: the data-parallel hot path of root-node AMG
 * interpolation setup on AMD Instinct MI355X (gfx950).
 *
 * Method: Manteuffel, Olson, Schroder, Southworth, "A Root-Node Based
 * Algebraic Multigrid Method", Sec. 3 (Alg. root_node_setup) and Sec. 4.
 * Given a sparse operator A, its aggregates with root nodes, candidate
 * vectors B and a pattern degree d, the library forms the pattern
 * N = S^d C with root rows set to identity, the tentative T and coarse
 * candidates Bc, and runs K energy-minimisation iterations (CG for SPD A,
 * GMRES otherwise, and on A^T for R^T) that keep P on N with P Bc = B.
 *
 * General conventions (apply to every call):
 *   - Pointers are DEVICE pointers unless the parameter says "host".
 *   - Indices are int32, 0-based.  CSR column indices are sorted ascending
 *     and unique within each row.  Every count of stored entries must be
 *     below 2^31 (checked, RN_ELIMIT).
 *   - Inputs are owned by the caller, read-only, and must stay valid until
 *     the work queued on the context's stream has completed (and, for
 *     arrays captured by a plan, until rn_plan_destroy).
 *   - Outputs are allocated by the caller.  Calls whose output size is only
 *     known after the computation are TWO-PHASE: the first call (output
 *     index array NULL) computes the result into the context, writes the
 *     row pointer array and the host-side count; the second call (same
 *     context, same arguments, output array non-NULL) copies it out; no
 *     other call that computes into the context may come between the two.
 *   - All device work is queued on the context's HIP stream.  Calls that
 *     return a size, a status found on the device or host statistics read
 *     back from the device and therefore synchronise that stream.
 *   - Every call returns rn_status.  Arguments are validated on the host
 *     before any launch (RN_EINVAL).  Nothing aborts; no C++ exception
 *     crosses the ABI.  rn_last_error() gives a message for the last
 *     failure on the context.
 *   - One context per stream; contexts share no state.  Calls on one
 *     context must not overlap in time (the context owns scratch memory).
 */
#ifndef RNAMG_H
#define RNAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RN_OK = 0,
  RN_EINVAL = 1,      /* malformed argument, detected on the host          */
  RN_ENOMEM = 2,      /* device allocation of scratch memory failed        */
  RN_ESINGULAR = 3,   /* singular root block of B (cannot normalise T)     */
  RN_EBREAKDOWN = 4,  /* CG curvature <D, Pi(A D)> <= 0: A not SPD on V    */
  RN_ENONFINITE = 5,  /* NaN or Inf in a Krylov scalar                     */
  RN_EHIP = 6,        /* HIP runtime error                                 */
  RN_ELIMIT = 7       /* a documented size limit was exceeded              */
} rn_status;

/* RN_CG: conjugate gradients on the energy trace(P^T A P) (Sec. 4.1, SPD A).
 * RN_GMRES: unrestarted GMRES on ||Pi(A P)||_F (Sec. 4.2, non-symmetric A).
 * RN_PCG_JACOBI: RN_CG with the Jacobi preconditioner Y = Pi(D^-1 R), D the
 *   diagonal of A (positive; RN_ESINGULAR otherwise); FP64.
 * RN_CGNR: conjugate gradients on ||A P||_F^2 with A P taken whole (the A*A
 *   norm of Sec. 4.2, CGNR): direction -Pi(A^T (A P)) kept to N; FP64, one
 *   problem (batch 1); builds the pattern of A N and A^T in the context. */
typedef enum { RN_CG = 0, RN_GMRES = 1, RN_PCG_JACOBI = 2, RN_CGNR = 3 } rn_method;
typedef enum { RN_FP64 = 0, RN_FP32_MIXED = 1 } rn_precision;

typedef struct rn_ctx rn_ctx;
typedef struct rn_plan rn_plan;
typedef struct rn_tape rn_tape;

/* Sparse operator A (Sec. 3 input A_l).  block_m = 1: scalar CSR with n
 * rows; block_m = 2: node-blocked BSR (Sec. 5.5 elasticity) with n/2 node
 * rows, nnz stored 2x2 blocks, values row-major inside a block.  Scalar DOF
 * of node I and component c is 2*I + c. */
typedef struct {
  int32_t n;               /* scalar rows (= scalar columns)                */
  int32_t block_m;         /* 1 or 2                                        */
  int64_t nnz;             /* stored entries (m=1) or stored blocks (m=2)   */
  const int32_t *rowptr;   /* device, n/block_m + 1                         */
  const int32_t *colind;   /* device, nnz                                   */
  const double *vals;      /* device, nnz*block_m*block_m (may be NULL where
                              only the structure is used)                   */
} rn_matrix;

/* Statistics of one rn_energy_min call, for batch entry 0. */
typedef struct {
  int32_t iters_done;          /* Krylov steps completed                    */
  int32_t rank_deficient_rows; /* F rows whose Gram matrix took the
                                  pseudo-inverse fallback                   */
  int32_t status_code;         /* device-side status (an rn_status value)   */
  int32_t fused_cg;            /* 1: each CG direction was formed inside
                                  the next product (RN_OPT_FUSED_CG)        */
  double first;                /* CG: <R0,R0>; GMRES: ||Pi(A T)||_F         */
  double last;                 /* CG: last <R,R>; GMRES: last residual      */
  double spgemm_bytes;         /* algorithmic bytes of one masked product:
                                  A's indices and values, A's and N's row
                                  pointers, N's indices, X in, Z out (FP64),
                                  the Gram data when nB > block_m          */
  double spgemm_flops;         /* 2 x multiply-adds of one masked product   */
  /* work units of the call (Sec. 2.4, Table sc: cost in multiples of one
   * product with A, 2 nnz(A) flops): the masked products it ran times
   * spgemm_flops / (2 nnz(A)), scalar entries of A; CGNR's two products per
   * step are each counted as one masked product                            */
  double work_units;
  /* with RN_OPT_METRICS set (else NaN), for batch entry 0 of the result:
   * energy = E(P) = sum over N of P_ij (A P)_ij (trace(P^T A P), Sec. 4.1);
   * proj_residual = ||Pi(A P)||_F over N (what GMRES minimises, Sec. 4.2);
   * constraint_residual = max |P Bc - B| over rows and candidates (Eq.
   * mode_constraint); rn_energy_min, which has no B, takes T Bc for B (equal
   * to B for a T made by rn_tentative), rn_setup takes B itself            */
  double energy, proj_residual, constraint_residual;
} rn_emin_stats;

/* ---- context ----------------------------------------------------------- */
/* Create a context bound to hip_stream (a hipStream_t; NULL = the null
 * stream) on the current device.  The context owns grow-only scratch. */
rn_status rn_create(rn_ctx **ctx, void *hip_stream);
/* Free all device memory owned by the context, including that of plans and
 * tapes made on it that are still alive (their destroy calls then free only
 * the host object; such a plan or tape can no longer be used).  Set-ups
 * (rn_setup) made on it must be destroyed first. */
void rn_destroy(rn_ctx *ctx);
rn_status rn_set_stream(rn_ctx *ctx, void *hip_stream);
/* Device memory from the caller's allocator (for instance a framework's
 * caching allocator), for everything the context allocates: scratch, plans,
 * tapes, set-up results.  alloc(bytes, user) returns a device pointer usable
 * by work queued on the context's stream, or NULL (then RN_ENOMEM); release(
 * ptr, user) gives a block back while work queued before the call on that
 * stream may still read it (the allocator must order its reuse after that
 * work, as a stream-ordered caching allocator does).  Both NULL: hipMalloc /
 * hipFree with the context's own cache (the default).  RN_EINVAL when exactly
 * one is NULL, or when the context already holds device memory (set the
 * allocator before the first call that allocates).  The pinned host area used
 * to read results back is not device memory and still comes from HIP. */
rn_status rn_set_allocator(rn_ctx *ctx, void *(*alloc)(size_t bytes, void *user),
                           void (*release)(void *ptr, void *user), void *user);
/* Alternative kernel paths.  Every value computes the same result to the
 * stated tolerances; the options exist so that each path can be tested and
 * timed.  RN_EINVAL for an unknown option or value. */
typedef enum {
  /* 1 (default): products of plans for scalar operators with nB <= 2, at
   * most 11 A entries per row and pattern rows of at most 31 entries run as
   * persistent pipelined workgroups; 0: one workgroup per product block.
   * Read when a plan is made. */
  RN_OPT_PERSISTENT_PRODUCT = 0,
  /* 1 (default): the pattern expansion keeps each power in padded rows of 64
   * columns (no host round trip between powers; rows that outgrow it are
   * redone with exact CSR powers); 0: exact CSR powers throughout. */
  RN_OPT_PADDED_PATTERN = 1,
  /* 1 (default): rn_setup runs strength and the first phase of the pattern
   * with one synchronisation when A is structurally symmetric; 0: it chains
   * the two-phase stage calls. */
  RN_OPT_FUSED_SETUP = 2,
  /* 256 (default), 128 or 64: lanes (pattern entries) per product block for
   * plans of scalar operators whose pattern rows hold at most lanes/4
   * entries (other plans use 256).  Read when a plan is made. */
  RN_OPT_PRODUCT_LANES = 3,
  /* 0 (default) or 1: rn_energy_min and rn_setup also compute the energy,
   * the projected residual and the constraint residual of their result into
   * rn_emin_stats (one more product and two reductions per call). */
  RN_OPT_METRICS = 4,
  /* 1 (default): CG (RN_CG; FP64, with or without a tape, or FP32-mixed) on
   * plans whose products run as persistent workgroups of 256 lanes forms the
   * direction D = R + beta D in FP64 while the next product stages its X
   * window (rounded to FP32 there in the mixed form; two launches per step,
   * two D buffers); 0: a separate direction pass (three launches per step).
   * The two give the same result bit for bit. */
  RN_OPT_FUSED_CG = 5,
  /* 0 (default): tapes made by rn_tape_create keep the CG iterates R_k, D_k
   * and Z_k at every c-th step, c = ceil(sqrt(iters)); c >= 1: that
   * interval.  The reverse sweep recomputes the steps between checkpoints
   * from the tape's step lengths (the gradient is the same bit for bit for
   * every c; c = 1 stores every step and recomputes none).  Read when a tape
   * is made. */
  RN_OPT_TAPE_INTERVAL = 6
} rn_option;
rn_status rn_set_option(rn_ctx *ctx, rn_option opt, int32_t value);
/* Message of the last failure on ctx ("" if none).  Valid until the next
 * call on ctx. */
const char *rn_last_error(const rn_ctx *ctx);
/* Library version string. */
const char *rn_version(void);

/* ---- a1/a2: strength of connection (Sec. 3.2, strength and amalgamate
 * steps of Alg. root_node_setup) --------------------------------------- */
/* Symmetric measure: stored (i,j) is strong when a_ij^2 >= theta^2 |a_ii
 * a_jj| (no fused multiply-add); (i,i) is always strong.  For block_m = 2
 * a node pair is strong when any DOF entry of its block is (boolean
 * amalgamation).  The result is symmetrised, S <- S u S^T, and returned as
 * a boolean node graph (n/block_m node rows, diagonal included).
 * TWO-PHASE.  S_rowptr (n/block_m + 1) is written in phase 1 together with
 * *nnz_S (host); S_colind (nnz_S) in phase 2.  theta >= 0. */
rn_status rn_strength(rn_ctx *ctx, const rn_matrix *A, double theta,
                      int32_t *S_rowptr, int32_t *S_colind, int64_t *nnz_S);

/* Strength values normalised as Eq. soc (Sec. 3.2), for the pre-filter of
 * Sec. 3.5: on the node graph S that rn_strength made from the same A and
 * theta, S_vals[q] for node entry (I, J), J != I, is the largest |a_ij| over
 * the strong DOF entries of blocks (I, J) and (J, I) of A (S u S^T as the
 * entry-wise maximum, amalgamation by the block's largest entry); each row
 * is then divided by its largest off-diagonal value (left at 0 when that is
 * 0) and its diagonal set to 1.  Synchronises the stream. */
rn_status rn_strength_values(rn_ctx *ctx, const rn_matrix *A, double theta,
                             const int32_t *S_rowptr, const int32_t *S_colind,
                             int64_t nnz_S, double *S_vals);

/* ---- aggregation (Sec. 3.3), host helper --------------------------------
 * Standard greedy aggregation on the HOST (host pointers): sweep 1 makes a
 * node whose strong neighbours are all free the root of a new aggregate
 * holding them; sweep 2 attaches each left-over node to the aggregate of
 * its lowest-index neighbour aggregated in sweep 1; sweep 3 makes each node
 * still free the root of a new aggregate with its free neighbours.
 * agg: n_nodes, roots: room for n_nodes.  The GPU path takes agg/roots as
 * inputs; this helper is inherently sequential. */
rn_status rn_aggregate_host(int32_t n_nodes, const int32_t *S_rowptr_host,
                            const int32_t *S_colind_host, int32_t *agg_host,
                            int32_t *roots_host, int32_t *n_agg_host);

/* ---- a3/a4: interpolation pattern (Sec. 3.4) ----------------------------
 * Nodal pattern N_node = S^d C (boolean product, d >= 0, S with diagonal),
 * then unamalgamate (DOF (i,j) present when node entry (i/m, j/m) is) and
 * root_node_pattern (each root DOF row becomes the identity row of its
 * coarse DOF m*agg + c).  Output: DOF pattern, n = m*n_nodes rows, m*n_agg
 * columns, sorted rows; is_root[i] = 1 for root DOF rows.
 * TWO-PHASE.  Phase 1 writes N_rowptr (n+1), is_root (n) and *nnz_N;
 * phase 2 writes N_colind.  Limit: a nodal row may gather at most 6144
 * candidate entries in one expansion step (RN_ELIMIT). */
rn_status rn_pattern(rn_ctx *ctx, int32_t n_nodes, const int32_t *S_rowptr,
                     const int32_t *S_colind, const int32_t *agg,
                     const int32_t *roots, int32_t n_agg, int32_t degree,
                     int32_t block_m, int32_t *N_rowptr, int32_t *N_colind,
                     uint8_t *is_root, int64_t *nnz_N);

/* Valued nodal pattern N = S^d C (Sec. 3.4 with the values of Eq. soc, the
 * matrix the pre-filter of Sec. 3.5 reads): X_0 = C (row I holds 1 at
 * column agg[I]), X_t = S X_(t-1) as sparse products (rn_spgemm's order of
 * summation).  Node rows, n_agg columns, no root-row replacement.
 * TWO-PHASE: phase 1 writes Nn_rowptr (nn + 1) and *nnz_Nn, phase 2 (same
 * arguments) Nn_colind and Nn_vals (nullable). */
rn_status rn_pattern_values(rn_ctx *ctx, int32_t n_nodes,
                            const int32_t *S_rowptr, const int32_t *S_colind,
                            const double *S_vals, int64_t nnz_S,
                            const int32_t *agg, int32_t n_agg, int32_t degree,
                            int32_t *Nn_rowptr, int32_t *Nn_colind,
                            double *Nn_vals, int64_t *nnz_Nn);

/* DOF pattern of a given nodal pattern (the unamalgamate and
 * root_node_pattern lines of Alg. root_node_setup): as the second half of
 * rn_pattern, for a nodal pattern made elsewhere (for instance one that
 * rn_filter pre-filtered).  Nn: n_nodes x n_agg CSR.  TWO-PHASE as
 * rn_pattern: phase 1 writes N_rowptr, is_root and *nnz_N, phase 2 N_colind. */
rn_status rn_pattern_dofs(rn_ctx *ctx, int32_t n_nodes,
                          const int32_t *Nn_rowptr, const int32_t *Nn_colind,
                          int64_t nnz_Nn, const int32_t *agg,
                          const int32_t *roots, int32_t n_agg, int32_t block_m,
                          int32_t *N_rowptr, int32_t *N_colind,
                          uint8_t *is_root, int64_t *nnz_N);

/* ---- candidate smoothing (the smooth line of Alg. root_node_setup, Sec. 3.1)
 * `sweeps` damped Jacobi sweeps on A B = 0, in place on B (n x nB,
 * row-major, device): B <- B - omega D^-1 A B with D the diagonal of A (the
 * scalar diagonal for block_m = 2), the sums of A B in the order of A's
 * rows.  RN_ESINGULAR when a diagonal entry is zero.  Synchronises the
 * stream. */
rn_status rn_smooth_candidates(rn_ctx *ctx, const rn_matrix *A, double *B,
                               int32_t nB, int32_t sweeps, double omega);

/* ---- a5/a6: inject (Sec. 3.6, Eq. root-nodeform, Eq. Tproj) -------------
 * Bc[m*a + c, :] = B[m*roots[a] + c, :] (n_agg*m x nB, row-major).
 * T (aligned with N): root rows exactly 1; F row i in aggregate a gets
 * (B[i,0:m] inv(B[root block,0:m]))_c' at columns m*a + c', zero elsewhere.
 * When nB > m each F row then takes the minimum-norm update of Eq. Tproj so
 * that T Bc = B (least squares through the Gram pseudo-inverse where the
 * row's pattern cannot carry all candidates).  B is n x nB row-major,
 * m <= nB <= 4.  *rank_deficient (host, nullable) counts F rows whose Gram
 * matrix took the eigen pseudo-inverse (synchronises the stream).
 * RN_ESINGULAR if a root block of B is singular. */
rn_status rn_tentative(rn_ctx *ctx, int32_t n, int32_t block_m,
                       const int32_t *N_rowptr, const int32_t *N_colind,
                       int64_t nnz_N, const uint8_t *is_root,
                       const int32_t *agg, const int32_t *roots, int32_t n_agg,
                       const double *B, int32_t nB, double *T, double *Bc,
                       int32_t *rank_deficient);

/* ---- filter (Alg. filter; Sec. 3.5 pre-filter, Sec. 3.7 post-filter) ----
 * Drops small entries of a matrix G stored on a pattern (n DOF rows; for
 * block_m = 2 the two DOF rows of a node share its node structure, DOF
 * column 2a + c' in node column a).  A node entry's magnitude is the largest
 * |G| of its block_m x block_m block.  The entry of the row's own aggregate
 * (node column agg[I], agg: n/block_m node aggregates) plays the diagonal:
 * it is always kept and is not an off entry.  With k > 0, off entries below
 * the k-th largest off magnitude of the row are dropped; with theta > 0, off
 * entries below theta times the largest (both: either rule drops); ties
 * are kept.  Rows of nodes with is_root set are kept whole (is_root may be
 * NULL: no such rows, as for the nodal pattern of the pre-filter).
 * TWO-PHASE.  Phase 1 (F_colind NULL) writes F_rowptr (n+1) and *nnz_F
 * (host); phase 2 (same arguments, F_colind non-NULL) writes the kept
 * columns into F_colind and, when F_vals is non-NULL, their values, in
 * order.  k >= 0, theta >= 0.  RN_EINVAL for a malformed pattern or DOF
 * rows of one node with different structures. */
rn_status rn_filter(rn_ctx *ctx, int32_t n, int32_t block_m,
                    const int32_t *N_rowptr, const int32_t *N_colind,
                    int64_t nnz_N, const uint8_t *is_root, const int32_t *agg,
                    const double *vals, int32_t k, double theta,
                    int32_t *F_rowptr, int32_t *F_colind, double *F_vals,
                    int64_t *nnz_F);

/* ---- enforce (Sec. 3.7, Eq. Tproj) ---------------------------------------
 * In place on vals (values on the pattern N, n rows, n_cols columns): every
 * F row takes the minimum-norm update of its stored entries that restores
 * vals Bc = B (least squares through the Gram pseudo-inverse of Bc on the
 * row's columns where the row cannot carry every candidate); root rows are
 * untouched.  Bc: n_cols x nB, B: n x nB, row-major; 1 <= nB <= 4.
 * *rank_deficient (host, nullable) counts rows that took the eigen
 * pseudo-inverse.  Synchronises the stream. */
rn_status rn_enforce(rn_ctx *ctx, int32_t n, int32_t n_cols,
                     const int32_t *N_rowptr, const int32_t *N_colind,
                     int64_t nnz_N, const uint8_t *is_root, const double *Bc,
                     const double *B, int32_t nB, double *vals,
                     int32_t *rank_deficient);

/* ---- sparse product and Galerkin coarse operator (Sec. 3.8) ------------
 * C = X Y for CSR X (rows x inner) and Y (inner x cols): each row of C holds
 * the sorted union of the columns of the rows of Y that the row of X
 * selects (entries whose terms cancel stay, with value 0); C_ij is the sum
 * over the row of X, in its order, of X_it Y_(k_t) j.  TWO-PHASE: phase 1
 * (C_colind NULL) writes C_rowptr (rows+1) and *nnz_C; phase 2 (same
 * arguments) writes C_colind and, when C_vals is non-NULL, the values
 * (X_vals, Y_vals may be NULL when C_vals is). */
rn_status rn_spgemm(rn_ctx *ctx, int32_t rows, int32_t inner, int32_t cols,
                    const int32_t *X_rowptr, const int32_t *X_colind,
                    const double *X_vals, int64_t nnz_X,
                    const int32_t *Y_rowptr, const int32_t *Y_colind,
                    const double *Y_vals, int64_t nnz_Y, int32_t *C_rowptr,
                    int32_t *C_colind, double *C_vals, int64_t *nnz_C);
/* A_c = R A P (the last line of Alg. root_node_setup): P (n x n_cols) given
 * by its values on the pattern N; R = P^T when RT is NULL (symmetric A),
 * else R = (R^T)^T with R^T on the same pattern (non-symmetric A, Sec. 3.8).
 * A scalar CSR or node-blocked (its scalar entries are used).  Computed as
 * R (A P) with two rn_spgemm products.  TWO-PHASE as rn_spgemm: phase 1
 * writes Ac_rowptr (n_cols + 1) and *nnz_Ac and keeps A P and R in the
 * context; phase 2 (same arguments) writes Ac_colind and Ac_vals. */
rn_status rn_galerkin(rn_ctx *ctx, const rn_matrix *A, int32_t n_cols,
                      const int32_t *N_rowptr, const int32_t *N_colind,
                      int64_t nnz_N, const double *P, const double *RT,
                      int32_t *Ac_rowptr, int32_t *Ac_colind, double *Ac_vals,
                      int64_t *nnz_Ac);

/* ---- transpose (needed for R^T on A^T, Alg. root_node_setup non-symmetric
 * branch, and for the adjoint) ------------------------------------------
 * Scalar CSR only (block_m = 1).  AT_rowptr: n+1, AT_colind/AT_vals: nnz
 * (AT_vals may be NULL), perm (nullable): perm[q] = index in A of the q-th
 * entry of A^T, so that AT_vals[q] = A.vals[perm[q]]. */
rn_status rn_transpose(rn_ctx *ctx, const rn_matrix *A, int32_t *AT_rowptr,
                       int32_t *AT_colind, double *AT_vals, int32_t *perm);

/* ---- plan: the symbolic part of energy minimisation ---------------------
 * Binds the structure of A (values unused) to the pattern N and the coarse
 * candidates: per F row the Gram pseudo-inverse of B_J^T B_J (projection
 * Pi_B of Sec. 3.6), and for every pattern entry (i,j) and every stored
 * A(i,k) the position of j in N(k) (the intersection the masked product
 * needs).  The plan keeps the device pointers it was given (A->rowptr,
 * A->colind, N_rowptr, N_colind, is_root, Bc): they must stay valid until
 * rn_plan_destroy.  Limits (RN_ELIMIT): rows of N hold at most 253
 * entries (block_m = 1) or 253 nodal entries (block_m = 2); 1 <= nB <= 4;
 * block_m = 2 requires nB >= 2. */
rn_status rn_plan_create(rn_ctx *ctx, const rn_matrix *A, int32_t n_cols,
                         const int32_t *N_rowptr, const int32_t *N_colind,
                         int64_t nnz_N, const uint8_t *is_root,
                         const double *Bc, int32_t nB, rn_plan **plan);
/* Destroying a plan queues no wait: its memory is reused only by work queued
 * after the call on the context's stream. */
void rn_plan_destroy(rn_plan *plan);
/* Bytes of device memory held by the plan (codes, Gram data, workspace). */
size_t rn_plan_bytes(const rn_plan *plan);

/* ---- a7/a8: one masked product (Sec. 3.6: the smoothing product whose
 * fill outside N is dropped, followed by the constraint projection) -------
 * Z = M(A X): (A X)_ij for (i,j) in N on F rows, zero on root rows; when
 * project != 0, each F row then loses its least-squares component along
 * B_J (Pi_B).  A_vals: [batch][nnz(A) m m], X and Z: [batch][nnz_N].
 * RN_FP32_MIXED rounds A and X to FP32 and accumulates in FP32; the
 * projection runs in FP64 on the FP32 product.  Asynchronous (no stream
 * synchronisation). */
rn_status rn_masked_product(rn_ctx *ctx, rn_plan *plan, const double *A_vals,
                            int32_t batch, const double *X, int32_t project,
                            rn_precision precision, double *Z);

/* ---- a7-a11: energy minimisation (Sec. 3.6 improve, Sec. 4) -------------
 * P = T + U minimising trace(P^T A P) (RN_CG) or ||Pi(A P)||_F (RN_GMRES)
 * over U in the Krylov space of Pi A Pi started from -Pi(A T), after
 * `iters` steps; Pi zeroes root rows and removes, row by row, the
 * least-squares component along B_J (so U Bc = 0 and root rows stay 1).
 * A_vals: [batch][nnz(A) * m * m] values for the plan's structure (batch
 * entries share structure, T and Bc).  T: [nnz_N].  P: [batch][nnz_N].
 * RN_FP32_MIXED (RN_CG and RN_GMRES): the masked products read FP32 copies
 * of A and of the search direction (GMRES: of the basis vector) and
 * accumulate in FP32; projection, inner products, step lengths and the
 * iterates stay FP64.
 * hist (device, nullable): [batch][3*iters + 1] doubles: CG: gamma_0..K,
 * delta_0..K-1, alpha_0..K-1; GMRES: residual estimates 0..K then zeros.
 * stats (host, nullable).  The call synchronises the stream to read the
 * device status: RN_EBREAKDOWN / RN_ENONFINITE report the first failing
 * batch entry (its P holds the last good iterate).
 * hist for RN_PCG_JACOBI holds gamma_k = <R_k, Y_k>.
 * tape (nullable, RN_CG + RN_FP64 only): records what rn_energy_min_bwd
 * needs (scalars and the iterates R_k, D_k, Z_k at its checkpoints). */
rn_status rn_energy_min(rn_ctx *ctx, rn_plan *plan, const double *A_vals,
                        int32_t batch, const double *T, rn_method method,
                        int32_t iters, rn_precision precision, double *P,
                        double *hist, rn_emin_stats *stats, rn_tape *tape);

/* ---- the same minimisation without allocation ---------------------------
 * For callers that cannot allocate device memory during the call (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments, results and errors as rn_energy_min without
 * a tape; the Krylov vectors, scalars, partial sums and FP32 copies live in
 * one library-owned device array of RN_NOALLOC_SCRATCH_BYTES per GPU
 * (reserved when the library's code is loaded, held until the process ends)
 * instead of the plan's workspace.  The call allocates nothing: no hipMalloc,
 * no hipFree, no caller allocator, no pinned host memory (the read-back area
 * is reserved by rn_create).  RN_ELIMIT, before any launch, when the call
 * needs more than that array: CG needs about (3 + 1.5 [FP32-mixed]) x 8 x
 * batch x nnz_N bytes plus 520 x (product blocks + 1026) x batch, GMRES
 * (iters + 1) x (8 [+ 4]) x batch x nnz_N plus the same partials.  Every call
 * on one GPU, from any context, shares that GPU's array, and each call
 * overwrites it (its state is set at the start of the call): calls that
 * overlap in time on one GPU race and give wrong results.  RN_EHIP when
 * the array's device address could not be obtained when ctx was created. */
#define RN_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
rn_status rn_energy_min_noalloc(rn_ctx *ctx, rn_plan *plan,
                                const double *A_vals, int32_t batch,
                                const double *T, rn_method method,
                                int32_t iters, rn_precision precision,
                                double *P, double *hist,
                                rn_emin_stats *stats);

/* ---- metrics (Sec. 4.1 energy, Sec. 4.2 residual, Eq. mode_constraint) --
 * rn_energy: for values P on the plan's pattern (one problem), *energy =
 * sum over N of P_ij (A P)_ij and *proj_residual = ||Pi(M(A P))||_F (either
 * pointer, host, may be NULL).  rn_constraint_residual: *res = max over rows
 * i and candidates q of |(V Bc)_iq - B_iq|, V on the pattern N (n rows,
 * n_cols columns), Bc n_cols x nB, B n x nB.  Both synchronise the stream. */
rn_status rn_energy(rn_ctx *ctx, rn_plan *plan, const double *A_vals,
                    const double *P, double *energy, double *proj_residual);
rn_status rn_constraint_residual(rn_ctx *ctx, int32_t n, int32_t n_cols,
                                 const int32_t *N_rowptr, const int32_t *N_colind,
                                 int64_t nnz_N, const double *vals,
                                 const double *Bc, const double *B, int32_t nB,
                                 double *res);

/* ---- a12: adjoint of the CG energy minimisation (map A values -> P) -----
 * Tape for `batch` problems of `iters` CG steps on `plan`; holds the Krylov
 * scalars and the iterates R_k, D_k and Z_k = Pi(A D_k) at the checkpoints
 * k = 0, c, 2c, ... < iters (c from RN_OPT_TAPE_INTERVAL).  The reverse
 * sweep recomputes, from the checkpoint k0 at or before each step k, the
 * products Z_j = Pi(A D_j) for k0 < j <= k and the recurrences up to D_k,
 * Z_k and R_{k+1}: c(c-1)/2 products per checkpoint segment (none with
 * c = 1), 3 ceil(iters/c) + 4 iterate vectors per problem. */
rn_status rn_tape_create(rn_ctx *ctx, rn_plan *plan, int32_t batch,
                         int32_t iters, rn_tape **tape);
void rn_tape_destroy(rn_tape *tape);
/* Given P_bar [batch][nnz_N] (dL/dP), write A_bar [batch][nnz(A)]
 * = dL/dA_vals for the stored entries of A (each stored value an
 * independent variable).  plan_T is a plan on A^T (same N, is_root, Bc)
 * whose A^T structure came from rn_transpose with permutation perm
 * (nnz(A)).  Scalar CSR only. */
rn_status rn_energy_min_bwd(rn_ctx *ctx, rn_plan *plan, rn_plan *plan_T,
                            const int32_t *perm, rn_tape *tape,
                            const double *A_vals, const double *P_bar,
                            double *A_bar);

/* ---- one-shot set-up of one level (Alg. root_node_setup) ---------------
 * strength -> pattern -> tentative -> plan -> energy minimisation of P, and
 * with Bhat (nullable, scalar CSR only) the transpose of A and the same
 * minimisation of R^T on A^T from T-hat = inject(Bhat) (Sec. 4: R^T for a
 * non-symmetric A; without Bhat R = P^T is left to the caller).  Inputs as
 * for the stage calls: A (device, with values), agg (n/block_m) and roots
 * (n_agg) device arrays from the caller's aggregation, B and Bhat (n x nB,
 * row-major, device).  Every stage runs inside the library, one call; the
 * outputs are device arrays owned by *out until rn_setup_destroy, which
 * must come before rn_destroy of ctx.  A's arrays must stay valid while
 * *out lives (its plans keep them).  On failure *out is NULL and nothing is
 * kept.  stats / stats_RT (host, nullable) as for rn_energy_min. */
typedef struct rn_setup_out rn_setup_out;
typedef struct {
  int32_t n, n_cols, nB, rank_deficient;
  int64_t nnz_S, nnz_N;
  const int32_t *S_rowptr, *S_colind; /* node graph S (n/block_m rows)         */
  const int32_t *N_rowptr, *N_colind; /* pattern N (n rows, n_cols columns)   */
  const uint8_t *is_root;             /* n                                     */
  const double *T, *Bc, *P;           /* nnz_N, n_cols x nB, nnz_N             */
  const double *That, *Bchat, *RT;    /* as T, Bc, P for B-hat on A^T, or NULL */
  const rn_plan *plan, *plan_T;       /* plan_T NULL without Bhat              */
} rn_setup_view;
rn_status rn_setup(rn_ctx *ctx, const rn_matrix *A, const int32_t *agg,
                   const int32_t *roots, int32_t n_agg, const double *B,
                   const double *Bhat, int32_t nB, int32_t degree,
                   int32_t iters, double theta, rn_method method,
                   rn_precision precision, rn_setup_out **out,
                   rn_emin_stats *stats, rn_emin_stats *stats_RT);
/* Device pointers and sizes of the results (host struct). */
rn_status rn_setup_view_get(const rn_setup_out *s, rn_setup_view *view);
void rn_setup_destroy(rn_setup_out *s);

/* ---- F3: multilevel set-up (Alg. root_node_setup level by level; Sec. 3.8:
 * the next level's operator is the Galerkin product A_c = R A P) ------------
 * From A_0 = A and B_0 = B (n x nB, device, row-major): for each level l,
 * strength (theta), the host aggregation on S (rn_aggregate_host, same rules
 * as the stage call), rn_setup (pattern of the given degree, T, iters steps
 * of method; RN_GMRES also minimises R^T on A^T with B-hat = B_l), then
 * A_{l+1} = R A_l P (rn_galerkin; R = P^T for RN_CG, (R^T)^T for RN_GMRES)
 * and B_{l+1} = Bc.  Level 0 may be node-blocked (block_m = 2, RN_CG only);
 * the coarse levels are scalar CSR (m DOFs per aggregate of the level
 * above).  Stops after max_levels (>= 1) levels, at a level of at most
 * min_coarse rows, or where aggregation would not coarsen (every node its own
 * aggregate).  Every level's arrays are device memory owned by *out (level
 * 0's A and B stay the caller's and must stay valid while *out lives) until
 * rn_hierarchy_destroy, which must come before rn_destroy of ctx.  Host
 * synchronisations: one per level for the aggregation, plus rn_setup's and
 * rn_galerkin's.  Errors as for the stage calls; on failure *out is NULL. */
typedef struct rn_hierarchy rn_hierarchy;
typedef struct {
  int32_t n;              /* rows of A_l                                    */
  int32_t block_m;        /* 1, or 2 for a node-blocked level 0             */
  int64_t nnz_A;          /* stored entries (blocks for block_m = 2)        */
  const int32_t *A_rowptr, *A_colind; /* device                             */
  const double *A_vals;   /* device                                         */
  const double *B;        /* device, n x nB, the level's candidates         */
  int32_t nB;
  int32_t n_agg;          /* aggregates of this level (0 on the coarsest)   */
  const int32_t *agg, *roots; /* device, n/block_m and n_agg (NULL on the coarsest) */
  const rn_setup_out *setup; /* the level's set-up: rn_setup_view_get gives
                                S, N, T, Bc, P (and R^T); NULL on the coarsest */
  rn_emin_stats stats, stats_RT; /* of its energy minimisations           */
} rn_level_view;
rn_status rn_hierarchy_build(rn_ctx *ctx, const rn_matrix *A, const double *B,
                             int32_t nB, int32_t max_levels, int32_t min_coarse,
                             double theta, int32_t degree, int32_t iters,
                             rn_method method, rn_precision precision,
                             rn_hierarchy **out);
/* Number of levels (>= 1); 0 for NULL. */
int32_t rn_hierarchy_levels(const rn_hierarchy *h);
/* The level's pointers and sizes (host struct); RN_EINVAL out of range. */
rn_status rn_hierarchy_level(const rn_hierarchy *h, int32_t level,
                             rn_level_view *view);
void rn_hierarchy_destroy(rn_hierarchy *h);

#ifdef __cplusplus
}
#endif
#endif /* RNAMG_H */
