/*
 * chase.h -- C ABI of the MI355X (gfx950) ChASE library.
 *
 * ChASE (Chebyshev Accelerated Subspace iteration Eigensolver) computes the
 * nev lowest eigenpairs of a dense Hermitian (complex double) or symmetric
 * (real double) matrix H by subspace iteration on nev+nex vectors
 * (paper: Algorithm 1).  Each iteration filters the non-converged vectors
 * with a Chebyshev polynomial (three-term recurrence of Eq. (3)),
 * orthonormalises [locked | active] (QR), projects H onto the active part
 * (Rayleigh-Ritz), computes residuals, locks converged pairs and re-optimises
 * the per-vector polynomial degrees.
 *
 * Conventions shared by every entry point
 *  - All matrices are column-major (LAPACK layout) with a leading dimension
 *    (ld >= number of rows).  H is read in full (both triangles) and is never
 *    modified; the caller guarantees it is Hermitian.
 *  - Element type is fixed per handle: CHASE_C128 (interleaved re,im
 *    doubles) or CHASE_F64.  "void*" device pointers point to that type.
 *  - Pointers named *_dev are device (HBM) pointers owned by the caller;
 *    *_host are host pointers owned by the caller.  The library owns only the
 *    workspace inside the handle, allocated once in chase_create.
 *  - Every call is ordered on the given HIP stream (0 = null stream) and
 *    returns only after the results it writes to host memory are valid;
 *    device outputs are valid once the stream reaches the end of the call
 *    (the calls below synchronise the stream before returning).
 *  - Errors: a chase_status is returned; no exception crosses the ABI.  The
 *    message of the last error on the calling thread is available from
 *    chase_last_error().  On any error other than CHASE_ERR_NOCONV the
 *    outputs are unspecified.
 *  - A handle may be used by one thread at a time.
 */
#ifndef CHASE_MI355X_H
#define CHASE_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum chase_status {
  CHASE_OK = 0,
  CHASE_ERR_ARG = 1,      /* invalid argument (sizes, pointers, options)   */
  CHASE_ERR_NOMEM = 2,    /* workspace does not fit in free device memory  */
  CHASE_ERR_HIP = 3,      /* a HIP / rocSOLVER runtime call failed          */
  CHASE_ERR_NOCONV = 4,   /* max_iter reached; outputs hold the best pairs */
  CHASE_ERR_NUMERIC = 5   /* NaN/Inf or breakdown of every QR variant      */
} chase_status;

typedef enum chase_dtype { CHASE_C128 = 0, CHASE_F64 = 1 } chase_dtype;

/* Precision of the filter's matrix products (the rest of the method always
 * runs in FP64).  CHASE_PREC_FP32: complex64/float32 MFMA products with FP32
 * accumulation.  CHASE_PREC_BF16X3: split-BF16 products on the BF16 matrix
 * cores: each value x of H and of the block is carried as hi = bf16(x) and
 * lo = bf16(x - hi), a real product as hi*hi + hi*lo + lo*hi with FP32
 * accumulation (about 2^-16 relative per product); the handle keeps the
 * split of H (n*n*8 bytes complex, n*n*4 real, padded) and of the block.
 * CHASE_PREC_BF16X2: the same split of H, the block rounded to bf16 (its hi
 * part only): a real product is hi*hi + lo*hi, two MFMAs instead of three
 * (about 2^-9 relative per product; same memory as BF16X3).  In a solve it
 * is used for the defect-correction passes only (the start block's plain
 * pass runs with three terms): where the spectrum rather than precision
 * limits convergence it takes about as many matrix-vector products as
 * BF16X3 at two thirds of the MFMA work.
 * In all low-precision modes the start block is filtered with the plain
 * recurrence, Ritz vectors in the defect-correction form (see
 * chase_filter_ritz), whose rounding error shrinks with the residual; a
 * vector switches to the FP64 filter for good if its residual grows tenfold
 * in an iteration, or once it is below switch_tol (> 0).  H must be
 * Hermitian (the split stores conj(H) = H^T so that rows are contiguous). */
typedef enum chase_prec {
  CHASE_PREC_FP64 = 0,
  CHASE_PREC_FP32 = 1,
  CHASE_PREC_BF16X3 = 2,
  CHASE_PREC_BF16X2 = 3
} chase_prec;

typedef struct chase_opts {
  int max_deg;         /* cap of the optimised degree (default 36)           */
  int deg_extra;       /* margin added to the optimised degree (default 2)   */
  int optimize_degree; /* 1: per-vector degrees (Algorithm 1); 0: fixed deg   */
  int lanczos_steps;   /* length of each Lanczos run (default 25)            */
  int lanczos_vecs;    /* number of Lanczos runs, 1..8 (default 4)           */
  int max_iter;        /* subspace iterations before NOCONV (default 50)     */
  int filter_prec;     /* chase_prec (default CHASE_PREC_FP64)                */
  double switch_tol;   /* residual below which a vector leaves the low-
                          precision filter for FP64; <= 0: never             */
  int verbose;         /* 1: one line per iteration on stderr                */
  int initial_rr;      /* 1: Rayleigh-Ritz on the start block before the first
                          filter (warm starts from approximate eigenvectors:
                          converged pairs lock at once, the first degrees are
                          optimised, mixed modes use the defect form from the
                          start).  Not in Algorithm 1; default 0            */
  int fp64_tail;       /* mixed modes, start block's (plain) low-precision
                          pass: run its last fp64_tail steps with FP64
                          products, which damp the earlier steps' rounding
                          errors so the pass can reach FP64 residuals.
                          -1 (default): automatic, the steps that shrink a
                          rounding floor (2^-14 split-BF16, 2^-17
                          sqrt(max(1, n/3000)) FP32) to
                          tol at the growth rate of the density-of-states
                          estimate of the nev-th eigenvalue, used only if
                          fewer than the degree; 0: off; > 0: that many
                          (capped at the degree).  Ignored with initial_rr  */
  int seed;            /* start blocks the caller leaves NULL in chase_solve
                          (V0_dev, S_dev) are drawn from N(0, 1) by a
                          counter-based generator (SplitMix64 + Box-Muller)
                          with this seed: the same seed gives the same
                          blocks on every call and device (default 0)      */
  int debug;           /* 1 (or the environment variable CHASE_DEBUG=1 when
                          the handle is created): chase_solve checks that H
                          is Hermitian (max |H - H^H| <= 1e-12 max |H|,
                          else CHASE_ERR_ARG), the block after every QR step
                          (max |Q^H Q - I| <= 1e-8, else CHASE_ERR_NUMERIC)
                          and every phase's output for NaN/Inf; the measured
                          defects go to chase_stats.  Costs one extra pass
                          over H and one Gram product per iteration
                          (default 0)                                       */
  int adjoint_reserve; /* > 0: chase_create also allocates what the adjoints
                          need (the eigenvector adjoint's two n x (nev+nex)
                          blocks and a filter tape of adjoint_reserve steps
                          over nev+nex columns), so that chase_filter with
                          record_tape = 1 (degrees <= adjoint_reserve) and
                          chase_eigvec_adjoint allocate nothing; counted by
                          chase_workspace_bytes.  0 (default): they
                          allocate on first use                             */
  int eig_solver;      /* dense eigensolver of the Rayleigh-Ritz step
                          (chase_eig): CHASE_EIG_AUTO (default) runs the
                          library's own Jacobi eigensolver when the projected
                          matrix is already close to diagonal (off-diagonal
                          Frobenius norm <= 0.05 of the whole; the later
                          iterations of a solve) and the divide-and-conquer
                          solver of the ROCm library otherwise;
                          CHASE_EIG_LIBRARY / CHASE_EIG_JACOBI force one    */
  int fp64_emulation;  /* 0 (default): FP64 filter products on the FP64 matrix
                          cores.  8, 10, 12, 14 or 16: every FP64 filter
                          product (the FP64 mode's, the FP64 tail and FP64
                          ranks of the mixed modes) runs on the INT8 matrix
                          cores as an exact integer product modulo that many
                          moduli <= 256, recovered by Chinese remaindering
                          (Ozaki scheme II): rows of H and columns of the
                          block are rounded to integers of about
                          (log2 M - log2 n) / 2 bits, M the moduli's product
                          (14 moduli at n = 20000: 46-47 bits, the accuracy
                          class of FP64 products).  Rayleigh-Ritz's H Q,
                          from which the reported residuals come, runs on
                          INT8 only with 14 or 16 moduli (with 12 the
                          residuals were off by half of tol = 1e-10); fewer
                          moduli serve the filter alone, for looser
                          tolerances: with 12 the n = 20000 solve stalls at a
                          residual near 1e-10.  H must be
                          Hermitian and n <= 65535; the handle keeps 3N n^2
                          bytes of residues of H (complex; N n^2 real) and
                          15N n (nev+nex) bytes of per-step buffers         */
} chase_opts;

/* Dense Hermitian eigensolvers for the Rayleigh-Ritz step (chase_opts
 * eig_solver, chase_heev).  CHASE_EIG_JACOBI is block-cyclic two-sided
 * Jacobi on the GPU (blocks of 16 indices, round-robin order; every round
 * diagonalises the pairs of blocks in LDS and applies their rotations to the
 * matrix and the eigenvectors in one launch), converged when the
 * off-diagonal Frobenius norm is <= 1e-14 of the matrix's; it takes about
 * 8-10 sweeps on a dense random matrix and 2-4 on a nearly diagonal one.
 * CHASE_EIG_LIBRARY is rocSOLVER's divide and conquer (zheevd / dsyevd). */
typedef enum chase_eig {
  CHASE_EIG_AUTO = 0,
  CHASE_EIG_LIBRARY = 1,
  CHASE_EIG_JACOBI = 2
} chase_eig;

typedef struct chase_stats {
  int iterations;        /* subspace iterations performed                    */
  int locked;            /* converged (locked) pairs                         */
  int64_t matvecs_fp64;  /* filter matrix-vector products in FP64 (Matvecs)  */
  int64_t matvecs_low;   /* filter matrix-vector products in low precision   */
  double t_all;          /* seconds, whole solve (Table 2 columns)           */
  double t_lanczos, t_filter, t_qr, t_rr, t_resid;
  double t_filter_kernels; /* summed HIP-event time of the filter GEMMs       */
  int64_t filter_launches; /* number of filter GEMM launches                 */
  double filter_flops;     /* algorithmic filter FLOPs (8 n^2 per complex mv) */
  double b_sup, mu_1, mu_ne; /* final spectral bounds                         */
  int qr_shifted;          /* QR passes that needed the shifted variant      */
  int qr_householder;      /* QR calls that fell back to Householder         */
  double t_lanczos_gemv;   /* summed HIP-event time of the Lanczos block GEMVs */
  int64_t lanczos_gemv_launches; /* number of Lanczos block GEMV launches   */
  double lanczos_gemv_bytes; /* bytes of H read by them (one pass per launch) */
  double t_filter_kernels_low; /* the part of t_filter_kernels spent in
                                  low-precision filter GEMMs                */
  int64_t filter_launches_low; /* the low-precision ones of filter_launches */
  int fp64_tail;           /* FP64 steps at the end of the start block's
                              low-precision pass (0: none)                  */
  double debug_herm_defect; /* debug mode: max |H - H^H| / max |H| (else 0)  */
  double debug_orth_defect; /* debug mode: largest max |Q^H Q - I| after a QR
                               step of the solve (else 0)                   */
  double t_rr_eig;         /* summed HIP-event time of the dense eigensolves
                              of Rayleigh-Ritz (part of t_rr)               */
  int eig_jacobi_calls;    /* Rayleigh-Ritz eigensolves done by Jacobi       */
  int eig_jacobi_sweeps;   /* their Jacobi sweeps, summed                    */
} chase_stats;

typedef struct chase_handle_s* chase_handle_t;

/* Fill *opts with the defaults listed above. */
void chase_default_opts(chase_opts* opts);

/* Bytes of device workspace chase_create allocates for this problem
 * (one-GPU form of the paper's GPU memory estimate, Eq. (7), without the
 * caller-owned matrix).  Returns 0 for invalid sizes. */
size_t chase_workspace_bytes(chase_dtype dtype, int64_t n, int nev, int nex,
                             const chase_opts* opts);

/* Create a handle on the current HIP device and allocate its workspace
 * once (as the paper pre-allocates its library buffers, Section 2.3).
 * Requires 1 <= nev, 1 <= nex, nev+nex <= n.  opts may be NULL (defaults).
 * CHASE_ERR_NOMEM if the workspace exceeds the free device memory.  With
 * CHASE_PREC_FP32 the workspace includes a complex64 copy of H when it fits
 * (chase_workspace_bytes counts it); otherwise H is rounded on the fly.
 * With CHASE_PREC_BF16X3 the split copy of H, two split copies of the
 * block (a filter step's operand and the next step's, which the step writes
 * beside its FP64 result) and 64 MiB (32 MiB real) of partial tiles for the
 * product's split-K tail are required (NOMEM if they do not fit). */
chase_status chase_create(chase_handle_t* handle, chase_dtype dtype, int64_t n,
                          int nev, int nex, const chase_opts* opts);
void chase_destroy(chase_handle_t handle);

/* Algorithm 1.  Inputs: H_dev (n x n, ld ldh), tol > 0 (bound on
 * ||H v - lambda v||_2 relative to the largest Lanczos Ritz value in
 * magnitude, a lower bound of ||H||_2), degree >= 2
 * (initial degree, rounded up to even), V0_dev (n x (nev+nex), ld n: the
 * start block; NULL: drawn by the library, see chase_opts.seed), S_dev
 * (n x lanczos_vecs, ld n: Lanczos start vectors; NULL: drawn likewise).
 * Outputs: evals_host[nev] ascending, evecs_dev (n x nev, ld ldv),
 * resid_host[nev] (may be NULL), stats (may be NULL).
 * CHASE_ERR_NOCONV: max_iter reached; outputs hold the lowest nev current
 * Ritz pairs and stats->locked tells how many converged. */
chase_status chase_solve(chase_handle_t handle, const void* H_dev, int64_t ldh,
                         double tol, int degree, const void* V0_dev,
                         const void* S_dev, double* evals_host, void* evecs_dev,
                         int64_t ldv, double* resid_host, chase_stats* stats,
                         void* stream);

/* Spectral bounds by the Lanczos step of Algorithm 1 from the start vectors
 * S_dev (n x nvec, ld n, nvec <= lanczos_vecs) with `steps` steps each:
 * b_sup (upper bound of the spectrum), mu_1 (lowest Ritz value) and mu_ne
 * (DoS estimate of the (nev+nex)-th eigenvalue).  alpha_host/beta_host
 * (may be NULL) receive the tridiagonal entries, nvec x steps, run-major;
 * steps_host[nvec] (may be NULL) the length of each run. */
chase_status chase_lanczos(chase_handle_t handle, const void* H_dev, int64_t ldh,
                           const void* S_dev, int nvec, int steps, double* b_sup,
                           double* mu_1, double* mu_ne, double* alpha_host,
                           double* beta_host, int* steps_host, void* stream);

/* chase_lanczos without a handle and without allocating device memory, for
 * callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same computation and outputs as
 * chase_lanczos for an element type `dtype` and a problem with n_e = nev+nex
 * wanted columns (n_e sets the density-of-states estimate mu_ne); H_dev
 * (n x n, ld ldh) and S_dev (n x nvec, ld n) are the caller's, 1 <= nvec
 * <= 8, 1 <= steps <= min(200, n).  The work buffers (3 n nvec vectors,
 * the block GEMV's partial sums, the tridiagonals) live in a fixed device
 * array of 64 MiB that the library holds on every GPU it runs on until the
 * process ends; a problem that needs more is refused with CHASE_ERR_ARG
 * before any GPU work (complex, 25 steps: n <= 104000 at nvec = 8, n <= 262000
 * at nvec = 4; real: about twice that).  Every call on a GPU uses that GPU's one array: calls that
 * overlap on the same GPU (other threads, other streams) race and must be
 * serialised by the caller.  Calls no hipMalloc/hipFree and no allocating
 * library routine; host-side it keeps the small tridiagonals in host memory. */
chase_status chase_lanczos_noalloc(chase_dtype dtype, const void* H_dev, int64_t ldh,
                                   int64_t n, int n_e, const void* S_dev, int nvec, int steps,
                                   double* b_sup, double* mu_1, double* mu_ne,
                                   double* alpha_host, double* beta_host, int* steps_host,
                                   void* stream);

/* Chebyshev filter (Eq. (3), scaled so the polynomial is 1 at mu_1, damping
 * [mu_ne, b_sup]).  Column a of X_dev (n x k, ld ldx, in/out) is replaced by
 * p_{m_a}(H) x_a with m_a = degrees_host[a]: even, >= 2, non-decreasing in a.
 * prec: chase_prec (CHASE_PREC_BF16X3 needs a handle created with
 * filter_prec = CHASE_PREC_BF16X3, else CHASE_ERR_ARG; H_dev is split on
 * every call).  record_tape=1 keeps every intermediate block on the
 * device for chase_filter_adjoint (needs tape memory, (max degree + 1) n k
 * elements: reserved at creation by chase_opts.adjoint_reserve, else
 * allocated here; CHASE_ERR_NOMEM if it does not fit).  matvecs (may be
 * NULL) receives the matrix-vector count. */
chase_status chase_filter(chase_handle_t handle, const void* H_dev, int64_t ldh,
                          void* X_dev, int64_t ldx, int k, const int* degrees_host,
                          double b_sup, double mu_1, double mu_ne, int prec,
                          int record_tape, int64_t* matvecs, void* stream);

/* The same filter applied to Ritz vectors in defect-correction form:
 * V_dev (n x k, ld ldv, in/out) holds Ritz vectors v_a with Ritz values
 * theta_host[a] and R_dev (n x k, ld ldr) their residuals r_a = H v_a -
 * theta_a v_a.  Since (H - gamma I) v = (theta - gamma) v + r, p(H) v =
 * T_m(theta) v + D_m where D follows the three-term recurrence of Eq. (3)
 * started from D_0 = 0 with the extra term alpha_s T_{s-1}(theta) r_a; only
 * D is multiplied by H, so with a low-precision prec the rounding error is
 * relative to ||r|| rather than ||p(H) v||.  Degrees as in chase_filter.
 * matvecs (may be NULL) receives the number of column products (m_a - 1 per
 * column: the first step needs none). */
chase_status chase_filter_ritz(chase_handle_t handle, const void* H_dev, int64_t ldh,
                               void* V_dev, int64_t ldv, const void* R_dev, int64_t ldr,
                               const double* theta_host, int k, const int* degrees_host,
                               double b_sup, double mu_1, double mu_ne, int prec,
                               int64_t* matvecs, void* stream);

/* QR step of Algorithm 1: orthonormalise the n x k block X_dev (ld ldx)
 * in place, keeping its first `locked` columns (assumed orthonormal)
 * unchanged; the others become orthonormal and orthogonal to them with the
 * same span as [locked | rest] (a span that contains it if the block is
 * rank deficient).  Cholesky QR until two consecutive passes are clean;
 * a pass whose factor is ill conditioned is redone on the shifted Gram
 * matrix (at most 6 times); Householder QR (the paper's geqrf, Section 2.3)
 * if the Gram matrix has a zero or non-finite diagonal entry or the
 * shifted passes do not lead to clean ones.  shifted_passes and householder
 * (may be NULL) receive the number of shifted passes and 1 if the
 * Householder QR was used (else 0). */
chase_status chase_qr(chase_handle_t handle, void* X_dev, int64_t ldx, int k,
                      int locked, int* shifted_passes, int* householder, void* stream);

/* Rayleigh-Ritz + residual steps of Algorithm 1 on the orthonormal block
 * Q_dev (n x k, ld ldq, in/out): Q is replaced by the Ritz vectors,
 * ritz_host[k] receives the Ritz values ascending and resid_host[k]
 * (may be NULL) ||H v - theta v||_2 / norm_scale. */
chase_status chase_rayleigh_ritz(chase_handle_t handle, const void* H_dev,
                                 int64_t ldh, void* Q_dev, int64_t ldq, int k,
                                 double norm_scale, double* ritz_host,
                                 double* resid_host, void* stream);

/* Dense Hermitian eigensolve of the Rayleigh-Ritz step (Algorithm 1;
 * Section 2.3) on its own: G_dev (k x k, ld ldg, column-major, both
 * triangles, k <= nev+nex of the handle) is overwritten by the orthonormal
 * eigenvectors (columns), evals_host[k] receives the eigenvalues ascending.
 * method is a chase_eig value (CHASE_EIG_AUTO: the rule of
 * chase_opts.eig_solver); sweeps_host (may be NULL) receives the Jacobi
 * sweeps, 0 when the library's solver ran.  Uses the handle's workspace
 * (nothing is allocated).  CHASE_ERR_NUMERIC on non-finite entries or if
 * Jacobi does not converge in 60 sweeps. */
chase_status chase_heev(chase_handle_t handle, void* G_dev, int64_t ldg, int k,
                        int method, double* evals_host, int* sweeps_host,
                        void* stream);

/* Cholesky factorisation A = R^H R of a Hermitian positive definite matrix,
 * the factorisation inside chase_qr's Cholesky QR passes (this library's
 * reading of the QR step of Algorithm 1; Section 2.3 names Householder QR)
 * on its own.  A_dev (k x k, ld lda >= max(1, k), column-major, the handle's
 * element type): its upper triangle is read and overwritten by R (upper
 * triangular, positive real diagonal); the strict lower triangle is not
 * touched.  info_host receives 0, or the 1-based order of the first
 * leading minor that is not positive definite, as LAPACK's potrf; then A
 * holds partial results (not an error status: CHASE_OK is returned).
 * Non-finite pivots count as not positive.  k = 0 is a no-op (A_dev may
 * then be NULL).  Needs no workspace and allocates nothing; k is not
 * limited by the handle's sizes. */
chase_status chase_cholesky(chase_handle_t handle, void* A_dev, int64_t lda, int k,
                            int* info_host, void* stream);

/* Adjoint of the eigenvalue map: dH += V diag(g) V^H for V_dev (n x m,
 * ld ldv) orthonormal eigenvectors and g_host[m]; dH_dev (n x n, ld ldd)
 * is accumulated into (the gradient of sum_i g_i lambda_i w.r.t. Hermitian
 * H, torch's complex convention). */
chase_status chase_eigval_adjoint(chase_handle_t handle, const void* V_dev,
                                  int64_t ldv, int m, const double* g_host,
                                  void* dH_dev, int64_t ldd, void* stream);

/* Adjoint of the eigenvector map, for real losses of the lowest m
 * eigenvectors that do not depend on each vector's phase (for instance on
 * V V^H, or on |v_i^H b|).  Not in the paper: it completes the
 * differentiation of the solver's outputs.  Inputs: H_dev (n x n, ld ldh),
 * V_dev (n x m, ld ldv) orthonormal eigenvectors of the m lowest, simple
 * eigenvalues lambda_host[m] (as returned by chase_solve), G_dev (n x m, ld
 * ldg) the gradient of the loss w.r.t. V in torch's complex convention
 * (dL = Re tr(G^H dV)).  Accumulates into dH_dev (n x n, ld ldd) the
 * gradient w.r.t. Hermitian H, from first-order perturbation
 * dv_i = sum_{k != i} u_k (u_k^H dH v_i) / (lambda_i - mu_k):
 *   within span(V):  V E V^H, E = Hermitian part of (v_i^H g_j) / (lambda_j - lambda_i)
 *                    (0 on the diagonal and between equal eigenvalues),
 *   complement:      (X V^H + V X^H) / 2, (H - lambda_j I) x_j = -(I - V V^H) g_j,
 *                    x_j orthogonal to V.
 * The complement systems are positive definite (V spans the lowest
 * eigenvectors) and are solved together by conjugate gradients, one FP64
 * GEMM per iteration, until every column's residual is below tol times its
 * initial residual (checked every 10 iterations); iterations (may be NULL)
 * receives the count.  CHASE_ERR_NOCONV after max_iter iterations, with
 * dH_dev unchanged.  Uses the handle's workspace (1 <= m <= nev+nex) and
 * two more n x (nev+nex) blocks, reserved at creation by
 * chase_opts.adjoint_reserve, else allocated by the first call. */
chase_status chase_eigvec_adjoint(chase_handle_t handle, const void* H_dev, int64_t ldh,
                                  const void* V_dev, int64_t ldv, int m,
                                  const double* lambda_host, const void* G_dev, int64_t ldg,
                                  void* dH_dev, int64_t ldd, double tol, int max_iter,
                                  int* iterations, void* stream);

/* Adjoint of the last chase_filter call made with record_tape=1: given
 * gY_dev (n x k, ld ldg), the gradient of a real loss w.r.t. the filtered
 * block, accumulate into dH_dev (n x n, ld ldd) the gradient w.r.t. H
 * (recurrence replayed in reverse, rank-k updates, Hermitian part) and, if
 * gX_dev is not NULL, write the gradient w.r.t. the filter input (n x k,
 * ld ldg).  Degrees and bounds are those of the recorded call. */
chase_status chase_filter_adjoint(chase_handle_t handle, const void* H_dev,
                                  int64_t ldh, const void* gY_dev, int64_t ldg,
                                  void* dH_dev, int64_t ldd, void* gX_dev,
                                  void* stream);

/* Host-side steps of Algorithm 1 (no handle, no GPU): the scalar logic the
 * solver applies between its device steps, for callers that drive the steps
 * themselves (chase_lanczos, chase_filter, chase_qr, chase_rayleigh_ritz).
 *
 * chase_filter_coefficients: the m steps of the scaled Chebyshev recurrence
 * of Eq. (3) (normalised at mu_1, damping [mu_ne, b_sup]) used by
 * chase_filter: coef_host[3s], [3s+1], [3s+2] = alpha, gamma, beta of step
 * s+1, X_{s+1} = alpha (H - gamma I) X_s + beta X_{s-1}.  Requires 1 <= m
 * <= 1000 and mu_1 < mu_ne < b_sup.
 *
 * chase_spectral_bounds: b_sup (largest Ritz value of a run plus its last
 * |beta|, maximised over runs), mu_1 (smallest Ritz value) and mu_ne (the
 * density-of-states estimate of the n_e-th eigenvalue, clamped into
 * [mu_1, b_sup]) from Lanczos tridiagonals in the layout chase_lanczos
 * returns (alpha_host, beta_host: nvec x steps, run-major; a run ends at its
 * first beta <= 1e-14 max|alpha|).  steps_host[nvec] (may be NULL) receives
 * each run's length.  Requires 1 <= n_e <= n, beta >= 0.
 *
 * chase_degrees: the degree step of Algorithm 1 for k vectors with
 * residuals resid_host[k] (> 0, the solver's normalisation) and Ritz values
 * ritz_host[k]: with c = (b_sup + mu_ne)/2, e = (b_sup - mu_ne)/2,
 * t = (ritz - c)/e and rho = max|t +- sqrt(t^2 - 1)|, degrees_host[a] =
 * ceil(|ln(resid/tol)| / ln rho) + deg_extra, capped at max_deg (max_deg if
 * rho <= 1 + 1e-12), at least 2, rounded up to even; with optimize_degree 0
 * every degree is `degree` rounded up to even.  opts may be NULL. */
chase_status chase_filter_coefficients(int m, double b_sup, double mu_1, double mu_ne,
                                       double* coef_host);
chase_status chase_spectral_bounds(const double* alpha_host, const double* beta_host, int nvec,
                                   int steps, int64_t n, int n_e, double* b_sup, double* mu_1,
                                   double* mu_ne, int* steps_host);
chase_status chase_degrees(const double* resid_host, const double* ritz_host, int k, double b_sup,
                           double mu_ne, double tol, int degree, const chase_opts* opts,
                           int* degrees_host);

/* Message of the last error raised on the calling thread ("" if none). */
const char* chase_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CHASE_MI355X_H */
