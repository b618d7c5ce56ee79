/*
 * sdc.h -- C ABI of the MI355X (gfx950) inverse-free spectral split library.
 *
 * The library computes one step of the randomized spectral divide-and-conquer
 * of Ballard, Demmel and Dumitriu, "Minimizing Communication for
 * Eigenproblems and the Singular Value Decomposition" (arXiv 1011.3077):
 *
 *   - implicit repeated squaring (IRS, Alg. 3 of Sec. 3.1): repeated
 *     Householder QR of the stacked 2n x n matrix [B_j; -A_j] = Q [R_j; 0]
 *     and the updates A_{j+1} = Q12^T A_j, B_{j+1} = Q22^T B_j, until
 *     ||R_j - R_{j-1}||_1 <= tau ||R_{j-1}||_1;
 *   - the generalized randomized URV (GRURV, Alg. 2 on RURV, Alg. 1) that
 *     extracts an orthogonal basis of the right (and left) deflating subspace
 *     from (A_p + B_p)^{-1} A_p without inverses;
 *   - the block form and split-point choice of RGNEP (Alg. 4) and RSEP
 *     (Alg. 6): A_hat = Q_L^T A Q_R (and B_hat) with the block size k that
 *     minimizes ||E21||_1/||A||_1 (+ ||F21||_1/||B||_1).
 *
 * Conventions shared by every entry point
 *   - Matrices are real, COLUMN-MAJOR, with a leading dimension >= n.
 *   - Matrix pointers are DEVICE pointers (memory from hipMalloc or a torch
 *     CUDA/HIP tensor) on the handle's device.  Inputs are never modified;
 *     outputs are caller-allocated and written in full.
 *   - Inputs and outputs are always FP64.  SDC_FP32_REFINE (symmetric
 *     problems only; pencils return SDC_ERR_INVALID) runs the repeated
 *     squaring in FP32 with FP32 accumulation, keeps the convergence test,
 *     the rank decision, the block form and the split search in FP64, and
 *     adds an FP64 Newton refinement of the basis (not in the paper): X
 *     solving X A11 - A22 X = E21 by conjugate gradients, Q <- Q [I -X^T; X I]
 *     re-orthonormalized, up to 3 rounds, until ||E21||_1/||A||_1 <=
 *     split_tol.  The refinement needs the two eigenvalue groups separated by
 *     a point, so SDC_FP32_REFINE is accepted only with an SDC_HALFPLANE
 *     region (other kinds: SDC_ERR_INVALID).  A problem whose FP32 attempts all fail
 *     (any status other than SDC_OK and SDC_NO_SPLIT) is split again in FP64
 *     and info->fp64_fallback is set.
 *   - Eigenvalues of the pencil A - lambda B are the roots of
 *     det(A - lambda B) = 0.  The region's boundary is mapped to the unit
 *     circle (Sec. 3.3): a half plane Re z < shift with scale s becomes the
 *     pencil (A - (shift - s) B, A - (shift + s) B); a disk |z - c| < r
 *     becomes (A - c B, r B).
 *   - Ordering: the leading k_lead columns of Q (of Q_R) span the deflating
 *     subspace of the eigenvalues OUTSIDE the region (the range of
 *     (A_p + B_p)^{-1} A_p, Sec. 3.2), so A11 = A_hat[0:k, 0:k] holds the
 *     outside eigenvalues and A22 the n_inside = n - k_lead inside ones.
 *   - Negative status: outputs are undefined.  Positive status
 *     (NOT_CONVERGED, NO_SPLIT, RANK_AMBIGUOUS): outputs hold the best split
 *     found and *info is filled.
 *   - Calls are synchronous with respect to the host and run on the stream
 *     given to sdc_create.  A handle must not be used by two host threads at
 *     once; use one handle per stream.
 *   - Workspace is allocated by the library from device memory and kept in
 *     the handle, capped by hbm_budget_bytes (0 = no cap).  A call whose
 *     workspace would exceed the cap returns SDC_ERR_NOMEM.
 */
#ifndef SDC_H_
#define SDC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sdc_handle_s* sdc_handle_t;

typedef enum {
    SDC_OK = 0,
    SDC_NOT_CONVERGED = 1,   /* IRS hit maxit (Alg. 3 "until ... j > maxit") */
    SDC_NO_SPLIT = 2,        /* every eigenvalue lies on one side of the curve */
    SDC_RANK_AMBIGUOUS = 3,  /* retries exhausted without a split meeting split_tol */
    SDC_ERR_INVALID = -1,    /* bad argument */
    SDC_ERR_NOMEM = -2,      /* device allocation failed or budget exceeded */
    SDC_ERR_DEVICE = -3,     /* a HIP runtime call failed */
    SDC_ERR_NONFINITE = -4   /* NaN/Inf met in the iteration */
} sdc_status_t;

typedef enum { SDC_FP64 = 0, SDC_FP32_REFINE = 1 } sdc_prec_t;
typedef enum { SDC_UNIT_DISK = 0, SDC_DISK = 1, SDC_HALFPLANE = 2 } sdc_region_kind_t;

/* Splitting curve (Sec. 3.3): SDC_DISK |z - center| < radius;
 * SDC_HALFPLANE Re z < shift with Moebius scale `scale` (> 0). */
typedef struct {
    int kind;
    double center, radius;
    double shift, scale;
} sdc_region_t;

typedef struct {
    int prec;            /* sdc_prec_t */
    double tau;          /* IRS tolerance; <= 0 -> sqrt(eps) of the iterate precision */
    int maxit;           /* IRS iteration cap (Alg. 3); <= 0 -> 60 */
    uint64_t seed;       /* key of the Gaussian draw; attempt a uses seed + a */
    int max_retries;     /* extra GRURV draws after a failed split (default 2) */
    double split_tol;    /* accept a split when e(k) <= split_tol; <= 0 -> 1e-10 */
    const double* G;     /* optional DEVICE array of (max_retries+1)*2 column-major
                            n x n Gaussian matrices, index [attempt*2 + side]
                            (side 0 right, 1 left); NULL -> Philox4x32-10 draws */
    int diagnostics;     /* nonzero: also compute info->orth_err (one more GEMM) */
    int panel_width;     /* QR panel width, 32 or 64 columns; 0 -> the handle's table
                            (sdc_tune_set / sdc_autotune), which chooses per problem from its
                            own order, so a problem gives the same bits alone and in a batch */
} sdc_opts_t;

typedef struct {
    int n;
    int k_lead;          /* leading block size (eigenvalues outside); -1 (with n_inside -1)
                            when no draw split and a pencil's right and left sides
                            disagreed about every eigenvalue lying on one side */
    int n_inside;        /* n - k_lead: eigenvalues inside the region */
    int iters_right;     /* IRS iterations p on (A, B) */
    int iters_left;      /* IRS iterations p on (A^T, B^T) (pencils) */
    int attempts;        /* Gaussian draws used (1 + retries) */
    int refine_rounds;   /* FP64 refinement rounds (SDC_FP32_REFINE) */
    int k_rho;           /* rank read off the GRURV diagonals */
    double rconv_last;   /* last relative R change of the right-side IRS */
    double e21_rel;      /* minimized ||E21||_1/||A||_1 (+ ||F21||_1/||B||_1) */
    double orth_err;     /* ||Q^T Q - I||_F of Q (Q_R), if diagnostics (summed over blocks
                            atomically: its last bit may differ between runs) */
    double rank_gap;     /* ratio across the largest gap of the sorted diagonal ratios */
    double ms;           /* wall time of the call in milliseconds */
    int fp64_fallback;   /* SDC_FP32_REFINE: 1 if every FP32 attempt failed and the split
                            was redone in FP64 (the reported result is the FP64 one) */
} sdc_info_t;

/* Fill *opts with the defaults (FP64, tau = sqrt(eps), maxit 60, seed 0,
 * 2 retries, split_tol 1e-10, no caller Gaussian). */
void sdc_opts_default(sdc_opts_t* opts);

/* Create a handle bound to `device` and `stream` (a hipStream_t; NULL = the
 * null stream).  hbm_budget_bytes caps the workspace (0 = no cap).
 * Returns SDC_ERR_DEVICE if the device cannot be used. */
sdc_status_t sdc_create(sdc_handle_t* handle, int device, size_t hbm_budget_bytes, void* stream);

/* Free the handle and its workspace.  NULL is accepted. */
sdc_status_t sdc_destroy(sdc_handle_t handle);

/* Human-readable name of a status code (static string). */
const char* sdc_status_string(int status);

/* Implicit repeated squaring alone (Alg. 3) on the mapped pencil of
 * (A, B) for `region` (B == NULL means B = I).  With transpose != 0 it runs on
 * (A^T, B^T) (the left side of Alg. 4).  Writes A_p, B_p (n x n, FP64, ld ldo)
 * and, if R != NULL, the last R_j (n x n upper triangular, non-negative
 * diagonal, ld ldo).  *p receives the iteration count and *rconv the last
 * relative change ||R_j - R_{j-1}||_1/||R_{j-1}||_1.
 * Returns SDC_OK or SDC_NOT_CONVERGED. */
sdc_status_t sdc_irs(sdc_handle_t h, int n, const double* A, int lda, const double* B, int ldb,
                     int transpose, sdc_region_t region, const sdc_opts_t* opts,
                     double* Ap, double* Bp, double* R, int ldo, int* p, double* rconv);

/* One split of a symmetric A with B = I (RSEP, Alg. 6, with the map of
 * Sec. 3.3).  Q (n x n, orthogonal) and A_hat = sym(Q^T A Q) are written. */
sdc_status_t sdc_split_sym(sdc_handle_t h, int n, const double* A, int lda, sdc_region_t region,
                           const sdc_opts_t* opts, double* Q, int ldq, double* Ahat, int ldah,
                           sdc_info_t* info);

/* Largest order and device memory of sdc_split_sym_noalloc. */
#define SDC_NOALLOC_MAX_N 1024
#define SDC_NOALLOC_SCRATCH_MIB 112

/* sdc_split_sym without any device-memory allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments, layout, ownership, statuses
 * and results are those of sdc_split_sym (the same kernels in the same
 * order: the outputs are bitwise equal), with n <= SDC_NOALLOC_MAX_N
 * (SDC_ERR_INVALID beyond it).  The workspace is a static device array of
 * SDC_NOALLOC_SCRATCH_MIB MiB per device that the library holds from the
 * first sdc_create on that device until the process ends, and host-side
 * staging is static too; the handle's streams and events are made by
 * sdc_create.  Every call on one device shares that memory: calls that
 * overlap in time on one device (from several threads or handles) race and
 * must be serialized by the caller; consecutive calls are safe (each ends
 * with a synchronization of the handle's stream).  Profiling
 * (sdc_profile_enable) does not apply to this entry point. */
sdc_status_t sdc_split_sym_noalloc(sdc_handle_t h, int n, const double* A, int lda, sdc_region_t region,
                                   const sdc_opts_t* opts, double* Q, int ldq, double* Ahat, int ldah,
                                   sdc_info_t* info);

/* RNEP: one split step of a non-symmetric A (B = I; the paragraph after
 * Alg. 4).  The left deflating subspace equals the right one, so only the
 * right side runs: IRS of the mapped (A, I), GRURV(2, A_p + B_p, A_p, -1, 1)
 * giving Q, then Ahat = Q^T A Q (not symmetrized) and the split point that
 * minimizes ||E21||_1 / ||A||_1 (the backward error).  Arguments, layout,
 * ownership and statuses as for sdc_split_sym (any region kind); FP64 only
 * (SDC_FP32_REFINE gives SDC_ERR_INVALID).  Half the work of
 * sdc_split_pencil with B = I (whose Q_R it reproduces when both accept the
 * same draw). */
sdc_status_t sdc_split_nonsym(sdc_handle_t h, int n, const double* A, int lda, sdc_region_t region,
                              const sdc_opts_t* opts, double* Q, int ldq, double* Ahat, int ldah, sdc_info_t* info);

/* One split of a regular pencil (RGNEP, Alg. 4, with the map of Sec. 3.3).
 * Q_L, Q_R (n x n, orthogonal), A_hat = Q_L^T A Q_R and B_hat = Q_L^T B Q_R
 * are written; the split point minimizes ||E21||_1/||A||_1 + ||F21||_1/||B||_1. */
sdc_status_t sdc_split_pencil(sdc_handle_t h, int n, const double* A, int lda, const double* B,
                              int ldb, sdc_region_t region, const sdc_opts_t* opts, double* QL,
                              int ldql, double* QR, int ldqr, double* Ahat, int ldah, double* Bhat,
                              int ldbh, sdc_info_t* info);

/* `count` independent symmetric splits of possibly different sizes, run in
 * lockstep on the device (the problems are independent: Sec. 4.3 assigns
 * subproblems to disjoint processor sets).  n, lda, regions, infos and the
 * pointer arrays A, Q, Ahat are HOST arrays of length count whose elements are
 * device pointers.  opts applies to every problem; problem i draws its
 * Gaussians with seed opts->seed + i*1000003 so its result does not depend on
 * the batch it runs in.  opts->G must be NULL.  statuses[i] receives problem
 * i's status; the return value is SDC_OK unless an argument or device error
 * occurred. */
sdc_status_t sdc_split_sym_batched(sdc_handle_t h, int count, const int* n, const double* const* A,
                                   const int* lda, const sdc_region_t* regions,
                                   const sdc_opts_t* opts, double* const* Q, const int* ldq,
                                   double* const* Ahat, const int* ldah, sdc_info_t* infos,
                                   int* statuses);

/* Statistics of a divide-and-conquer run. */
typedef struct {
    int n;
    int nblocks;         /* diagonal blocks of the final block-triangular pair */
    int splits;          /* split steps attempted (every call of the split step) */
    int accepted;        /* split steps that divided a block */
    int extra_splits;    /* additional split points taken from accepted steps: every k'
                            besides the step's k with e(k') <= split_tol also divides the
                            block (more than two pieces, the remark after Alg. 4) */
    int levels;          /* recursion levels run (each level is one batched call) */
    int unsplit;         /* blocks larger than leaf_max given up on (every curve tried met
                            their pseudospectrum, Sec. 3.6) */
    int near_singular;   /* of those, blocks given up while no circle had yet split or bounded
                            them: every curve meets the pseudospectrum, the mark of a (nearly)
                            singular pencil (Sec. 3.5) */
    int iters_total;     /* sum of IRS iterations over all split steps and sides */
    double nominal_flops;/* sum over split steps of (40/3 (p_R + p_L) + 32) m^3 (pencil)
                            or (40/3 p + 16) m^3 (symmetric), the flop model of the
                            paper's cost analysis with LAPACK leading terms */
    double ms;
    double e21_max;      /* largest e21_rel (sdc_info_t) among the accepted splits:
                            the coupling blocks set to zero, relative to their
                            subproblem in the 1-norm */
} sdc_dc_info_t;

/* Bound on the eigenvalues of one diagonal block of sdc_eig_dc's result: the
 * eigenvalues mu of the block (mu = 1/lambda when `inverted`, lambda
 * otherwise) satisfy re_lo <= Re mu <= re_hi and |mu| <= radius, up to the
 * backward error of the splits.  Infinite entries mean no bound is known.
 * For a block given up on (`unsplit` = 1) this is the block Schur form's
 * bound on the block's pseudospectrum that Sec. 3.6 returns. */
typedef struct {
    double re_lo, re_hi, radius;
    int inverted;
    int unsplit;
} sdc_block_bound_t;

/* Randomized spectral divide-and-conquer to blocks of order <= leaf_max
 * (Sec. 3.3-3.5).  symmetric != 0: A symmetric, B ignored (B = I), splits at
 * a random point of the middle half of the current interval of each block,
 * starting from A's Gershgorin interval (Sec. 3.4).  Otherwise the pencil is
 * split first at the unit circle.  If every eigenvalue is inside, radii
 * 1/2, 1/4, 1/16, ... (2^{-2^k}) follow until a circle splits the spectrum or
 * finds it all outside; the last circle with everything inside bounds the
 * block, which continues with random vertical lines through the middle half
 * of that disk.  If every eigenvalue is outside, radii 2, 4, 16, ...
 * follow the same way, and the block continues on the swapped pair (B, A),
 * whose eigenvalues (the reciprocals) lie inside 1/r for the largest radius r
 * with everything outside (Sec. 3.5).  A block split at a circle of radius r
 * continues with lines inside r (its inside part) and, swapped, inside 1/r
 * (its outside part).  Lines are real, so a complex-conjugate pair is never
 * separated.  A circle that meets the pseudospectrum is retried at a
 * perturbed radius; after 3 failed circles with none that worked the block is
 * given up and counted in info->near_singular, after 8 failed lines it is
 * given up with the bound the search reached (info->unsplit counts both).
 * An accepted step divides its block at its split point k and at every other
 * k' whose coupling blocks are as small (e(k') <= opts->split_tol), so a
 * cluster of equal eigenvalues, which no curve separates, still falls apart
 * into blocks of order 1 once it is split off (info->extra_splits).
 * Outputs (device, column-major): T = Q_L^T A Q_R and, for pencils,
 * S = Q_L^T B Q_R, block upper triangular with the strictly-lower coupling
 * blocks set to zero; QL and QR (may be NULL) accumulate the transformations
 * (QL is unused for symmetric A, where QR = Q).  block_start (HOST, n + 1
 * ints) receives the first index of each diagonal block and n at position
 * *nblocks.  bounds (HOST, may be NULL; room for n entries) receives one
 * sdc_block_bound_t per block.  opts->prec SDC_FP32_REFINE is accepted for
 * symmetric A (every split is at a half plane).  Returns SDC_OK or a
 * negative error. */
sdc_status_t sdc_eig_dc(sdc_handle_t h, int n, const double* A, int lda, const double* B, int ldb,
                        int symmetric, int leaf_max, const sdc_opts_t* opts, double* T, int ldt,
                        double* S, int lds, double* QL, int ldql, double* QR, int ldqr,
                        int* nblocks, int* block_start, sdc_block_bound_t* bounds, sdc_dc_info_t* info);

/* RSVD split (the singular value problem of Sec. 3, through the symmetric
 * embedding E = [0 A; A^T 0] of order m + n, whose eigenvalues are the
 * singular values of A, their negatives and |m - n| zeros, with eigenvectors
 * [u; v] / sqrt(2)).  One symmetric split step (as sdc_split_sym) of E at
 * the half plane Re z < region.shift (kind SDC_HALFPLANE, shift >= 0; the
 * scale as for sdc_split_sym) separates the k = info->k_lead singular values
 * above the shift:
 *   U (m x min(m,n), ldu >= m): columns 0..k-1 an orthonormal basis of the
 *     left singular subspace of those values (sqrt(2) times E's Q rows 0..m-1);
 *   V (n x min(m,n), ldv >= n): the right one (E's Q rows m..m+n-1);
 *   S11 (min(m,n) x min(m,n), lds11 >= min(m,n)): leading k x k block
 *     U^T A V (symmetric; its eigenvalues are the k singular values), zero
 *     elsewhere; the columns of U and V after k are zero.
 * A, U, V, S11 are device pointers, column-major, caller-owned; the
 * library's workspace grows by 3 (m + n)^2 doubles.  m + n <= 16384.
 * Statuses as for sdc_split_sym (SDC_NO_SPLIT when no singular value, or
 * every one, lies above the shift); SDC_ERR_INVALID for bad arguments,
 * including a shift of 0 with m != n (E's |m - n| zero eigenvalues would lie
 * on the line). */
sdc_status_t sdc_split_svd(sdc_handle_t h, int m, int n, const double* A, int lda, sdc_region_t region,
                           const sdc_opts_t* opts, double* U, int ldu, double* V, int ldv, double* S11, int lds11,
                           sdc_info_t* info);

/* Eigenvalues of the diagonal blocks of a block upper-triangular T (and S)
 * as sdc_eig_dc returns them: the recursion of Sec. 3.3-3.5 stops at blocks
 * small enough for a standard dense method, and this is that method.
 *   symmetric != 0: each block of T of order <= 128 is symmetrized and
 *     diagonalized by cyclic Jacobi (rotations in round-robin order, to an
 *     off-diagonal norm of 1e-15 of the block's); its eigenvalues go to
 *     wr[start .. start + m) in ascending order, wi = 0.  S is not read.
 *   symmetric == 0: each block pair (T_bb, S_bb) of order 1 or 2 gives the
 *     roots of det(T_bb - lambda S_bb) = 0 in closed form (order 2: real
 *     roots ascending; a complex pair as (re, +im), (re, -im); an infinite
 *     eigenvalue, for a singular S_bb, as +-inf); a block of order 3 to 64
 *     gives the eigenvalues of S_bb^{-1} T_bb (or the inverted ones of
 *     T_bb^{-1} S_bb when S_bb is the worse conditioned; an eigenvalue that
 *     is infinite in exact arithmetic comes out very large) by the
 *     double-shift QR algorithm, ordered the same way (real ones ascending,
 *     then the complex pairs by real part); NaN for a block whose matrices
 *     are both exactly singular or whose iteration did not converge.
 *   Any other block (symmetric above order 128, pencil above order 64) gets
 *   NaN in wr and wi (sdc_eig_dc with a smaller leaf_max reduces it).
 * V (optional, symmetric only; n x n, ldv >= n): the diagonal block
 * V[start .. start + m, start .. start + m] receives the block's orthonormal
 * eigenvectors, column i for wr[start + i], for blocks of order <= 64 (NaN for
 * larger ones); entries outside the diagonal blocks are not written.  With
 * V block diagonal (zero elsewhere) and QR from sdc_eig_dc, QR V holds the
 * eigenvectors of A.
 * T, S, wr, wi, V are device pointers (column-major T and S with leading
 * dimensions ldt, lds >= n; wr, wi hold n doubles each, caller-owned);
 * block_start is a HOST array of nblocks + 1 increasing ints from 0 to n.
 * Returns SDC_OK, or SDC_ERR_INVALID for inconsistent arguments (nothing
 * written). */
sdc_status_t sdc_block_eigvals(sdc_handle_t h, int n, const double* T, int ldt, const double* S, int lds,
                               int nblocks, const int* block_start, int symmetric, double* wr, double* wi,
                               double* V, int ldv);

/* Eigenvectors of an upper-triangular matrix or pencil (TREVC, Sec. 5),
 * blocked as Alg. 8 with 32 x 32 blocks.  For upper-triangular T (and S;
 * S == NULL means S = I) with eigenvalues lambda_j = T_jj / S_jj, X (n x n)
 * receives the upper-triangular eigenvector matrix with unit diagonal:
 * T X = S X diag(lambda), i.e. column j solves (T - lambda_j S) x = 0 with
 * x_j = 1 and zeros below; X is written in full.  Only the upper triangles
 * of T and S are read.  The eigenvalues are assumed distinct (a real
 * spectrum: sdc_eig_dc with leaf_max = 1 on a pencil with real eigenvalues
 * gives such T and S, and Q_R X then holds the pencil's right
 * eigenvectors); a denominator T_ii - lambda_j S_ii smaller than
 * eps (|T_ii| + |lambda_j S_ii|) is replaced by that bound, as LAPACK's
 * TREVC guards it.  No scaling against overflow is done.  T, S, X are
 * device pointers, column-major, leading dimensions >= n, caller-owned.
 * Returns SDC_OK, or SDC_ERR_INVALID for bad arguments. */
sdc_status_t sdc_trevc(sdc_handle_t h, int n, const double* T, int ldt, const double* S, int lds, double* X,
                       int ldx);

/* Per-kernel timing (opt-in).  With profiling enabled every launch of the
 * hot kernels is bracketed by HIP events on the handle's stream and its
 * algorithmic work is recorded: kernel 0 = tree-level trailing update of the
 * QR (4 R nb ntr + 2 nb^2 ntr flops, 2 R ntr + R nb words for R rows, nb
 * panel columns, ntr trailing columns), 1 = panel factorization
 * (2 m nb^2 flops), 2 = GEMM (2 M N K flops), 3 = look-ahead update of the
 * next panel's columns (the kernel-0 figures with ntr = nb).  Events
 * serialize nothing but add a few microseconds per launch. */
typedef struct {
    long long launches;
    double ms;          /* summed event time */
    double flops;       /* summed algorithmic flops */
    double bytes;       /* summed algorithmic bytes */
} sdc_kernel_stats_t;

/* Replay the repeated-squaring iterations (Alg. 3) of sdc_split_sym,
 * sdc_split_pencil, sdc_split_nonsym, sdc_split_svd, the batched call and
 * the divide-and-conquer from a HIP graph (on != 0) instead of launching
 * their kernels one by one: one iteration of every problem of the call is
 * captured once (on a stream of the handle's own, after the descriptors are
 * resident on the device) and replayed per iteration; problems whose
 * convergence test has passed are switched off between replays.  Results
 * are bitwise the same either way.  Calls with a problem that takes the
 * two-stream look-ahead schedule (sdc_lookahead_set; by default none) keep
 * the direct launches (only one-stream QRs are captured).  Not used
 * while profiling is on, nor by the served form (its set of problems
 * changes every iteration).
 * SDC_ERR_INVALID for the no-allocation handle. */
sdc_status_t sdc_graphs_enable(sdc_handle_t h, int on);

/* QR schedule of the repeated squaring and the rank-revealing QRs (Alg. 3,
 * Alg. 1; the TSQR panel of Sec. 4.2): with on != 0 (the default), a
 * 32-column panel whose reduction tree has more than one level and that has
 * no look-ahead part (see sdc_lookahead_set; by default none) has the levels
 * above its leaves factored in the same launch as the leaves' trailing
 * update, which does not depend on them; with on == 0 the whole tree is
 * factored first.  Results are bitwise the same either way. */
sdc_status_t sdc_tree_overlap_enable(sdc_handle_t h, int on);

/* QR schedule: problems with at least min_cols factored columns (min_cols
 * > 0) take the two-stream look-ahead schedule (the trailing update of
 * panel k split so that the next panel's columns are updated first and
 * panel k + 1 is factored on a second stream beside the rest; Alg. 3's QRs
 * and the rank-revealing ones); min_cols <= 0 (the default) sends every
 * problem through the one-stream schedule, which measured faster at every
 * order up to 8192 once the panel's tree is factored beside its leaves'
 * update.  Results differ from the one-stream schedule's in rounding only
 * (the look-ahead columns are updated by another kernel); a problem's bits
 * depend on its own shape and this setting, not on the rest of a batch. */
sdc_status_t sdc_lookahead_set(sdc_handle_t h, int min_cols);

/* Enable (on != 0) or disable profiling; either way the totals are reset. */
sdc_status_t sdc_profile_enable(sdc_handle_t h, int on);
/* Totals of `kernel` (0 to 3 as above) since the last enable. */
sdc_status_t sdc_profile_read(sdc_handle_t h, int kernel, sdc_kernel_stats_t* out);

/* The Gaussian n x n matrix the library draws when opts->G is NULL:
 * Philox4x32-10 keyed by `seed`, counter (e mod 2^32, e div 2^32, tag, 0) for
 * the column-major element index e, then Box-Muller.  G is a device pointer. */
sdc_status_t sdc_gaussian(sdc_handle_t h, int n, uint64_t seed, int tag, double* G, int ldg);

/* ------------------------------------------------------------------------
 * Panel-width tuning of the repeated squaring's QR (the batched blocked
 * Householder QR of Alg. 3, costed with the communication-avoiding QR of
 * Sec. 4.2).  Panels are 32 or 64 columns wide; a problem with at least
 * nb64_min factored columns takes 64-column panels (per precision of the
 * iterates: FP64, and the FP32 iterates of SDC_FP32_REFINE).  The choice is
 * per problem, from its own order, so a problem gives the same bits alone
 * and in any batch on handles with the same table; opts->panel_width
 * overrides it for one call.
 * ---------------------------------------------------------------------- */
#define SDC_PANEL64_NEVER (-1)

/* Set the table: the smallest order that takes 64-column panels, for FP64
 * and for FP32 iterates; SDC_PANEL64_NEVER (any negative value) for none.
 * The default is SDC_PANEL64_NEVER for both (measured on MI355X: the
 * 32-column panels are faster at every order up to 8192). */
sdc_status_t sdc_tune_set(sdc_handle_t h, int nb64_min_fp64, int nb64_min_fp32);
sdc_status_t sdc_tune_get(sdc_handle_t h, int* nb64_min_fp64, int* nb64_min_fp32);

typedef struct {
    int n;               /* order timed */
    int prec;            /* SDC_FP64 or SDC_FP32_REFINE (FP32 iterates) */
    double ms_nb32;      /* one repeated-squaring iteration, 32-column panels (best of reps) */
    double ms_nb64;      /* the same with 64-column panels */
} sdc_tune_result_t;

/* Autotuner: for each of the `count` orders (1 .. 16384) and both iterate
 * precisions, time one repeated-squaring iteration (Alg. 3: the QR of the
 * stacked pair and the updates) of a Gaussian matrix with each panel width,
 * best of `reps` (>= 1) runs, and set the table: per precision, the
 * smallest timed order from which the 64-column panels win at every larger
 * timed order (SDC_PANEL64_NEVER if they do not win at the largest).
 * results (device-independent host memory, 2 * count entries, FP64 rows
 * first) receives the timings, or may be NULL.  Allocates device memory
 * for the test matrices (SDC_ERR_NOMEM if it cannot); results are
 * undefined on error.  Minutes at orders of several thousand. */
sdc_status_t sdc_autotune(sdc_handle_t h, const int* orders, int count, int reps, sdc_tune_result_t* results);

/* Write the table as JSON to `path` ({"nb64_min_fp64": .., "nb64_min_fp32": ..,
 * "arch": ..}), or read it back (keys missing from the file leave the table
 * as it is).  SDC_ERR_INVALID if the file cannot be written, read or
 * parsed. */
sdc_status_t sdc_tune_save(sdc_handle_t h, const char* path);
sdc_status_t sdc_tune_load(sdc_handle_t h, const char* path);

/* ------------------------------------------------------------------------
 * Served form: a request loop with continuous batching.
 *
 * Split requests (the independent subproblems of Sec. 4.3) are queued by
 * sdc_server_submit and run by one worker thread that owns its own HIP stream
 * on `device`.  Requests are admitted in arrival order while the sum of the
 * admitted requests' workspaces stays within hbm_budget_bytes (0 = 80% of the
 * device memory free at creation) and at most max_active run at once
 * (<= 0 = 64).  Admitted requests advance together, one repeated-squaring
 * iteration per tick (each at its own iteration count), and a request that
 * arrives while others run joins at the next tick; a request whose squaring
 * ends is finished (GRURV, block form, split search, refinement) in the tick
 * it ends, and its workspace is freed for the requests waiting.  A request's
 * result is the same as that of the single-problem entry point with the same
 * arguments, whichever requests share its ticks.
 *
 * Ownership: the request's input and output pointers are DEVICE pointers the
 * caller keeps valid (and does not write) until the request is reported done;
 * the inputs must be complete (their producer synchronized) before the call.
 * Outputs are complete when sdc_server_poll reports done or sdc_server_wait
 * returns.  A request whose workspace alone exceeds the budget finishes with
 * SDC_ERR_NOMEM.
 * ------------------------------------------------------------------------ */
typedef struct sdc_server_s* sdc_server_t;

typedef enum { SDC_REQ_SYM = 0, SDC_REQ_PENCIL = 1 } sdc_request_kind_t;

typedef struct {
    int kind;            /* sdc_request_kind_t */
    int n;
    const double* A; int lda;
    const double* B; int ldb;       /* pencils */
    sdc_region_t region;
    sdc_opts_t opts;
    double* Q; int ldq;             /* Q (symmetric) or Q_R */
    double* QL; int ldql;           /* pencils */
    double* Ahat; int ldah;
    double* Bhat; int ldbh;         /* pencils */
} sdc_request_t;

typedef struct {
    long long submitted, completed, failed;
    int active;          /* requests running now */
    int pending;         /* requests waiting for admission */
    int peak_active;     /* most requests that ran in one tick */
    long long ticks;
    double p50_ms, p99_ms, mean_ms, max_ms;   /* latency, submission to completion */
    double wall_ms;      /* first submission to last completion */
    double nominal_flops;/* sum over completed requests of the split flop model */
    size_t peak_bytes;   /* largest sum of admitted workspaces */
    size_t budget_bytes;
} sdc_server_stats_t;

/* Start a server (and its worker thread) on `device`. */
sdc_status_t sdc_server_create(sdc_server_t* server, int device, size_t hbm_budget_bytes, int max_active);
/* Queue a request; *ticket identifies it.  Validation as in sdc_split_sym /
 * sdc_split_pencil (SDC_ERR_INVALID, nothing queued). */
sdc_status_t sdc_server_submit(sdc_server_t server, const sdc_request_t* req, long long* ticket);
/* *done = 1 once the request finished; then *status and *info (may be NULL)
 * hold its result and the ticket is released.  SDC_ERR_INVALID for an unknown
 * or released ticket. */
sdc_status_t sdc_server_poll(sdc_server_t server, long long ticket, int* done, int* status, sdc_info_t* info);
/* Block until the request finished, then as sdc_server_poll with *done = 1.
 * A ticket's result goes to one caller: a second thread waiting on the same
 * ticket returns SDC_ERR_INVALID once the first has taken it. */
sdc_status_t sdc_server_wait(sdc_server_t server, long long ticket, int* status, sdc_info_t* info);
/* Latency percentiles, throughput counters, admission state. */
sdc_status_t sdc_server_stats(sdc_server_t server, sdc_server_stats_t* out);
/* Finish every queued request, stop the worker and free the server. */
sdc_status_t sdc_server_destroy(sdc_server_t server);

#ifdef __cplusplus
}
#endif
#endif /* SDC_H_ */
