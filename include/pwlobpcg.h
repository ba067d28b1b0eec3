/*
 * pwlobpcg.h -- C ABI of the MI355X (gfx950) plane-wave block-LOBPCG library.
 *
 * The library solves H c = eps c for the lowest bands of a plane-wave
 * Kohn-Sham Hamiltonian at one k-point with identity overlap (Bottin, Leroux,
 * Knyazev, Zerah, Comput. Mater. Sci. 2007 -- sec. 2.1: the wave-function is
 * expanded over plane waves e^{i(k+G).r} and the projected eigenproblem is
 * solved; with norm-conserving potentials the overlap operator is the
 * identity), or the generalized form H c = eps O c once an overlap operator
 * is set (pw_set_overlap).  The iteration is the block LOBPCG of sec. 3.2, Algorithm 1,
 * run multiband-by-multiband with each block orthogonal to the previous ones,
 * followed by a final Rayleigh-Ritz over all bands.
 *
 *   H = 1/2 |k+G|^2                                      kinetic diagonal
 *     + FFT^-1 . diag(V(r)) . FFT                        local potential (sec. 2.2 iii)
 *     + sum_p D_p |beta_p><beta_p|                       KB projectors (sec. 2.2 iv, 4.3)
 *
 * Conventions shared by every entry point:
 *  - Complex arrays are interleaved (re, im): double2 in FP64, float2 where a
 *    mixed-precision variant says so.  Block vectors are column-major
 *    [npw x nb] with a leading dimension ld >= npw; column j is band j.
 *  - The plane-wave order is the library's sphere order (pw_get_miller).
 *  - Every call returns pw_status; no exception or abort crosses the ABI.  On
 *    failure pw_last_error(ctx) describes the cause.
 *  - Device pointers must stay valid until the context stream has completed
 *    the call.  Calls that return host data synchronise the stream; the others
 *    are asynchronous on the context stream.
 *  - One context per host thread / stream.  Calls on one context are not
 *    thread-safe.
 *  - Ownership: the context owns its copies of the sphere tables, V(r) and the
 *    projector table; the caller owns X, Y, the workspace and every host array.
 *    The library never frees caller memory.
 */
#ifndef PWLOBPCG_H
#define PWLOBPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pw_ctx_s *pw_ctx;

typedef enum {
    PW_OK = 0,
    PW_ERR_ARG = 1,            /* invalid argument (null pointer, bad size, unsupported grid) */
    PW_ERR_STATE = 2,          /* call out of order (e.g. apply before init/potential/workspace) */
    PW_ERR_NOMEM = 3,          /* workspace too small or device allocation failed */
    PW_ERR_DEVICE = 4,         /* HIP runtime error */
    PW_ERR_NOT_CONVERGED = 5,  /* max_iter reached; best Ritz pairs and residuals still written */
    PW_ERR_NUMERIC = 6         /* NaN/Inf or a breakdown the solver could not recover from */
} pw_status;

/* Precision of the iteration.  PW_PREC_MIXED runs the block iteration on
 * complex64 blocks: the FFT apply, V(r) multiply, projector and Gram GEMMs in
 * FP32 (FP32 matrix cores, FP32 sums within a K chunk, chunk sums in FP64),
 * while the Gram results, Cholesky factors, Rayleigh-Ritz eigenproblems and
 * every reduction stay FP64.  Each block is iterated to a residual of
 * max(tol, 1e-5), then the FP64 iteration refines all bands from those
 * vectors to tol and runs the final Rayleigh-Ritz, so the returned
 * eigenpairs meet the same residual test as PW_PREC_FP64.
 * PW_PREC_MIXED_BF16 is the same iteration with the nonlocal projector
 * products on BF16 matrix cores (sec. 4.1's projector "zgemm"s, the largest
 * GEMMs of H X); PW_PREC_MIXED_BF16_GRAM also forms the Rayleigh-Ritz Gram
 * matrix Z^H (H Z) of the complex64 stage on BF16 matrix cores (the CholQR
 * Grams, constraint products and block updates stay FP32).  Both BF16 forms
 * refine in FP64 exactly like PW_PREC_MIXED.  PW_PREC_MIXED_FP32_RR is
 * PW_PREC_MIXED with the Householder reduction of the complex64 stage's
 * Rayleigh-Ritz eigenproblems (sizes up to 192) in FP32 on the FP64 Gram
 * rounded to float, and their eigenvalues bisected to FP32 width; inverse
 * iteration, orthogonalisation and back-transform stay FP64, and the FP64
 * stage is that of PW_PREC_MIXED. */
typedef enum {
    PW_PREC_FP64 = 0,          /* every step in complex128 / float64 */
    PW_PREC_MIXED = 1,         /* complex64 iteration, FP64 small dense steps and refinement */
    PW_PREC_MIXED_BF16 = 2,    /* PW_PREC_MIXED with the projector products (B^H X and
                                  B (D B^H X)) on BF16 matrix cores: complex64 operands
                                  split into hi + lo bf16 pairs, three products per real
                                  product, FP32 accumulation */
    PW_PREC_MIXED_BF16_GRAM = 3, /* PW_PREC_MIXED_BF16 with the Rayleigh-Ritz Gram of the
                                    complex64 stage on the same split-bf16 products */
    PW_PREC_MIXED_FP32_RR = 4    /* PW_PREC_MIXED with the complex64 stage's Rayleigh-Ritz
                                    tridiagonal reduction in FP32 */
} pw_precision;

/* Per-solve counters and phase times (milliseconds, measured with HIP events
 * on the context stream).  The five phase times are measured only while
 * pw_set_phase_timing is on (they read 0 otherwise); ms_total always is. */
typedef struct {
    int32_t iterations;        /* LOBPCG iterations summed over blocks */
    int32_t blocks;            /* number of blocks */
    int32_t h_applies;         /* number of H.X columns applied */
    int32_t p_restarts;        /* iterations where the P direction was dropped */
    double ms_total;           /* wall time of the solve on the stream */
    double ms_apply;           /* H.X (FFT apply + projectors) */
    double ms_gemm;            /* Gram, projection and block-update GEMMs */
    double ms_dense;           /* small dense FP64 steps (Cholesky, eigensolver) */
    double ms_vec;             /* residual / preconditioner / copies */
    double ms_final_rr;        /* final Rayleigh-Ritz over all bands */
    int32_t mixed_iterations;  /* mixed forms: iterations of the complex64 stage (included in
                                  iterations); 0 for PW_PREC_FP64 */
} pw_stats;

/* Create a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL = the legacy default stream). */
pw_status pw_create(int device, void *hip_stream, pw_ctx *out);
void pw_destroy(pw_ctx ctx);
/* Text of the last error on ctx (valid until the next call on ctx). */
const char *pw_last_error(pw_ctx ctx);

/* Plane-wave sphere S = { n in Z^3 : 1/2 |B (n + kfrac)|^2 <= ecut } (sec. 2.1),
 * B = 2 pi cell^-T.  cell: 3x3 row-major, rows = lattice vectors (bohr).
 * kfrac: k in reduced coordinates.  ecut: Ha.  fft_n: grid points per axis;
 * the grid must be cubic (n0 = n1 = n2), a supported size (see pw_fft_sizes)
 * and hold the sphere without collisions (n >= 2 nmax + 1).  Writes npw.
 * Sphere order: lexicographic in (n_x, n_y, n_z), so every z-column
 * ("stick") of the sphere is contiguous.  Resets potential, projectors and
 * workspace. */
pw_status pw_init_basis(pw_ctx ctx, const double cell[9], const double kfrac[3],
                        double ecut, const int32_t fft_n[3], int64_t *npw);
/* Supported FFT sizes: writes up to `cap` sizes to `sizes`, returns the count
 * in *count. */
pw_status pw_fft_sizes(int32_t *sizes, int32_t cap, int32_t *count);
/* Miller indices of the sphere, host int32 [npw][3], library order. */
pw_status pw_get_miller(pw_ctx ctx, int32_t *miller);
/* Kinetic diagonal 1/2 |k+G|^2 in Ha, host double [npw], library order. */
pw_status pw_get_kinetic(pw_ctx ctx, double *kin);

/* Local potential V(r_j) (Ha) on the grid, real, C order [j0][j1][j2] with
 * r_j = cell^T (j / N).  Host pointer (on_device = 0) or device pointer. The
 * context keeps its own permuted copy.  Non-finite values -> PW_ERR_NUMERIC. */
pw_status pw_set_local_potential(pw_ctx ctx, const double *v, int on_device);

/* Kleinman-Bylander projectors (sec. 2.2 iv, sec. 4.3): for atom a at pos[a]
 * (bohr, Cartesian) and each (l, m) in lm[nproj_per_atom][2] (l in {0, 1},
 * real harmonics Y00 = 1/(2 sqrt pi), (Y1-1, Y10, Y11) = sqrt(3/4pi)(y, z, x)/|q|),
 *   beta_{a,lm}(q) = Omega^-1/2 c exp(-|q|^2/2) Y_lm(q/|q|) exp(-i q.R_a),
 *   c = (32 pi^(5/2))^(1/2),  q = k + G,
 * and the term sum_{a,p} D[a*nproj_per_atom + p] |beta><beta| is added to H.
 * natom = 0 removes the projectors.  Host arrays. */
pw_status pw_set_projectors(pw_ctx ctx, int32_t natom, const double *pos,
                            int32_t nproj_per_atom, const int32_t *lm, const double *D);

/* Overlap operator of the generalized form H psi = eps O psi (sec. 2.1: the
 * right-hand side of the Kohn-Sham equations for ultrasoft / PAW
 * projectors; Algorithm 1 with R = H Psi - O Psi Upsilon):
 *   O = I + sum_p q[p] |beta_p><beta_p|
 * over the projectors of pw_set_projectors, in the same order as D.  q: host
 * double[nproj], finite and >= 0 (O >= I, positive definite), else
 * PW_ERR_ARG; q = NULL restores O = I.  Needs projectors (PW_ERR_STATE
 * otherwise); pw_set_projectors clears the overlap.  With an overlap set,
 * pw_lobpcg_solve solves the generalized problem and the workspace grows by
 * O Z and O X blocks: call pw_workspace_size after this call. */
pw_status pw_set_overlap(pw_ctx ctx, const double *q);

/* Device workspace the caller allocates: bytes needed by pw_lobpcg_solve for
 * (nbands, block) at precision prec, by pw_apply_H (which works in chunks
 * of `block` columns) and by pw_density of up to nbands bands (an N^3 grid of
 * doubles besides the stick buffer).  A workspace sized for a mixed form also serves
 * PW_PREC_FP64.  Also answers on a host-only context (device < 0), so a
 * caller can size device memory before touching the GPU. */
pw_status pw_workspace_size(pw_ctx ctx, int32_t nbands, int32_t block, pw_precision prec,
                            size_t *bytes);
/* Hand the workspace to the context (device pointer, 256-byte aligned).  The
 * plan of the last pw_workspace_size call must fit: else PW_ERR_NOMEM. */
pw_status pw_set_workspace(pw_ctx ctx, void *dptr, size_t bytes);

/* Y = H X on the context stream (rows a2-a7 of the hot path).  X, Y: device,
 * column-major [npw x nb], ldx, ldy >= npw, complex128 for PW_PREC_FP64 and
 * complex64 for the mixed forms (FFT, V(r) multiply and projector GEMMs then
 * run in FP32); X and Y must not overlap.  Needs basis, potential and a
 * workspace sized for prec.  Asynchronous. */
pw_status pw_apply_H(pw_ctx ctx, const void *X, int64_t ldx, void *Y, int64_t ldy,
                     int32_t nb, pw_precision prec);

/* Y_k = H_k X_k for the nk (1..16) contexts of one cell's k-points at once
 * (sec. 5.2: the k-points are the third level of parallelism; one GPU takes
 * them together).  The contexts share one device, one stream and one FFT
 * grid; their spheres, kinetic energies, projectors and stick buffers are
 * their own, and the local potential of ctxs[0] serves them all, as do its
 * launch parameters (pw_set_tuning: radix split, FFT tiling, split-K target).  Each of the three FFT passes is one launch over every (k-point,
 * band) work item; the projector products of each context follow on the same
 * stream.  X[k], Y[k]: device, column-major [npw_k x nb], ldx[k], ldy[k] >=
 * npw_k, complex128 for PW_PREC_FP64 and complex64 for the mixed forms, as in
 * pw_apply_H, whose result it gives for every context bitwise when the
 * contexts hold the same potential and launch parameters.  Every context
 * needs a workspace sized for prec; none may be in use elsewhere during the
 * call.  Errors (bad argument, mismatched contexts) are recorded on ctxs[0].
 * Only kernel launches go to the stream (no allocation, copy or
 * synchronisation once the contexts' mixed-form tables exist), so the call
 * can be recorded into a graph.  Asynchronous. */
pw_status pw_apply_H_batch(pw_ctx const *ctxs, int32_t nk, const void *const *X, const int64_t *ldx,
                           void *const *Y, const int64_t *ldy, int32_t nb, pw_precision prec);

/* Launch parameters of a context (0 = built-in default) and, from
 * pw_autotune, the timings behind the choice (ms per launch).  The sticks and
 * rows change the partition of the work only (the FFT results are bitwise the
 * same); the radix split changes the order of the FFT's operations and the
 * split-K target that of the Gram sums, so both may change the rounding. */
typedef struct {
    int32_t fft_sticks_per_block;   /* z passes: sticks per workgroup, 0 or 1..64 (default 16) */
    int32_t fft_plane_rows;         /* plane pass: row chunk, 0 or 1..128 (default 48, capped by LDS) */
    int32_t gemm_split_workgroups;  /* split-K TN target workgroups, 0 or 1..1024 (default 1024) */
    double apply_ms_default, apply_ms_tuned;   /* local H X of nb bands */
    double gemm_ms_default, gemm_ms_tuned;     /* 3m x 3m Gram over npw (+ projector overlaps) */
    int32_t fft_radix2;   /* radix split of the length-N FFTs: N = (N / R2) R2, both factors
                             products of 2, 3, 5 in [2, 16]; 0 = the default (R1 = 8 where
                             it fits, else the largest R2 <= sqrt(N)); the stored
                             potential follows the split's order */
} pw_tuning;

/* Autotuner for this context's shapes (batched k-points and served requests
 * differ in npw, grid and projector count): times the local H X of nb bands
 * (1 <= nb <= block of the workspace) for every radix split of the grid's FFT
 * length x sticks per block {16, 32, 64} x plane rows {16, 32, 48, 96}, and the Rayleigh-Ritz Gram (3 block x 3 block over
 * npw) plus the projector overlaps for split targets {384, 512, 768, 1024},
 * with HIP events on the context stream (mean of 5 after a warm-up); keeps
 * the fastest of each (or the default when nothing beats it) for later
 * calls on this context and reports it in *out.  Needs basis, potential,
 * projectors if any, and a workspace; overwrites workspace contents only.
 * Synchronises the stream. */
pw_status pw_autotune(pw_ctx ctx, int32_t nb, pw_tuning *out);
/* Set the three launch parameters (the timing fields are ignored); NULL
 * restores the defaults.  Out-of-range values -> PW_ERR_ARG.  Contexts given
 * the same parameters give bitwise the same results. */
pw_status pw_set_tuning(pw_ctx ctx, const pw_tuning *t);

/* Y = O X (the overlap of pw_set_overlap; PW_ERR_STATE if none is set), with
 * the same blocks, precisions, requirements and stream behaviour as
 * pw_apply_H: a copy of X plus the projector products B diag(q) B^H X. */
pw_status pw_apply_O(pw_ctx ctx, const void *X, int64_t ldx, void *Y, int64_t ldy,
                     int32_t nb, pw_precision prec);

/* Lowest `nbands` eigenpairs by block LOBPCG (sec. 3.2, Algorithm 1) in blocks
 * of `block` bands, each block kept orthogonal to the previous ones, then a
 * final Rayleigh-Ritz over all bands.  Convergence per block: every residual
 * ||H x - theta x||_2 (||x||_2 = 1) <= tol.  With an overlap set
 * (pw_set_overlap) the pencil (H, O) is solved instead: every orthogonality
 * is in the O inner product, theta = x^H H x / x^H O x and the residual is
 * ||H x - theta O x||_2 / (x^H O x)^1/2; X is returned O-orthonormal.  tol = 0 selects the fixed-sweep
 * mode of the paper's iteration count (sec. 3.2): every block runs exactly
 * max_iter iterations (a column whose residual is at the rounding floor,
 * 1e-10 max(1, Ecut), gets no new direction, and a block with every column
 * there stops and counts its remaining sweeps as done), the final
 * Rayleigh-Ritz follows and the call returns PW_OK (FP64 only).  X: device complex128
 * [npw x nbands], ldx >= npw, for both precisions; on entry a starting guess
 * if use_guess != 0 (columns of it with nothing independent left -- zero,
 * repeated, spanned by earlier bands -- or with non-finite entries are
 * replaced by random columns),
 * on exit the orthonormal eigenvectors.  prec: see
 * pw_precision (the workspace must be sized for it).  eig: host
 * double[nbands], ascending.
 * If every block converged but a residual exceeds tol after the final
 * Rayleigh-Ritz, the blocks are swept once more from the rotated vectors.
 * Limits: 1 <= block <= 64, nbands <= 1024 and nbands + 3 block <= npw (so
 * every block has room for its basis [X P W] beside the earlier bands);
 * else PW_ERR_ARG (also from pw_workspace_size).
 * Returns PW_ERR_NOT_CONVERGED (with the best pairs written) if a block hits
 * max_iter or a final residual still exceeds tol.  Synchronises the stream. */
pw_status pw_lobpcg_solve(pw_ctx ctx, int32_t nbands, int32_t block, double tol,
                          int32_t max_iter, pw_precision prec, void *X, int64_t ldx,
                          int32_t use_guess, double *eig);
/* Independent solves of n contexts run concurrently -- the k-points of one
 * cell, or any independent cells (sec. 5.2: k-points need no communication
 * inside the eigensolve).  Each context must be ready for pw_lobpcg_solve
 * (basis, potential, projectors, a workspace sized for (nbands, block, prec))
 * and bound to its own stream; contexts may have different plane-wave counts.
 * The library drives context i from its own host thread, so the kernels of
 * different contexts overlap on the device.  X[i], ldx[i], eig[i] are as in
 * pw_lobpcg_solve for context i; status[i] receives its result.  Returns
 * PW_OK if every solve succeeded, else the first error that is not
 * PW_ERR_NOT_CONVERGED, else PW_ERR_NOT_CONVERGED.  A context may appear
 * once.  Synchronises every context's stream. */
pw_status pw_lobpcg_solve_batch(pw_ctx *ctxs, int32_t n, int32_t nbands, int32_t block,
                                double tol, int32_t max_iter, pw_precision prec,
                                void *const *X, const int64_t *ldx, int32_t use_guess,
                                double *const *eig, pw_status *status);
/* Electron density of nb bands (sec. 4.1: the density is built from the bands
 * with the same FFTs as H.X): rho(r_j) = sum_n occ[n] |psi_n(r_j)|^2 with
 * psi_n(r) = Omega^-1/2 sum_G X[G, n] e^{i(k+G).r} on the grid points
 * r_j = cell^T (j / N).  X: device complex128 [npw x nb], ldx >= npw, library
 * sphere order; occ: host double[nb]; rho: device double [N][N][N], C order
 * [j0][j1][j2] (the layout of pw_set_local_potential).  Needs basis and a
 * workspace of at least block * N * (sticks rounded up to 16) * 16 + N^3 * 8 +
 * nb * 8 bytes (any workspace sized by pw_workspace_size for the same block
 * is enough for nb <= nbands).  Deterministic; synchronises the stream. */
pw_status pw_density(pw_ctx ctx, const void *X, int64_t ldx, int32_t nb, const double *occ,
                     void *rho);
/* Residual norms ||H x_j - theta_j x_j||_2 of the last solve, host double[nbands]. */
pw_status pw_get_residuals(pw_ctx ctx, double *res);
/* Counters and phase times of the last solve. */
pw_status pw_get_stats(pw_ctx ctx, pw_stats *stats);
/* Phase timing of the solves on ctx: on != 0 records a pair of HIP events
 * around every phase of every iteration (the ms_apply .. ms_final_rr of
 * pw_stats).  Each record is a marker packet between two kernels on the
 * stream; at the paper-scale cell (12 phases per iteration, ~600 iterations)
 * they lengthen a solve by ~5 %, so timing is off by default and the phase
 * times then read 0.  Applies to every later solve on ctx (pw_lobpcg_solve,
 * pw_lobpcg_solve_batch). */
pw_status pw_set_phase_timing(pw_ctx ctx, int32_t on);

/* ---- Building blocks of the iteration, exported for per-step parity tests ----
 * All pointers are device pointers; complex128 column-major; asynchronous on
 * the context stream; no workspace needed unless stated. */

/* Gram block C = A^H B (sec. 4.1: Gram blocks by zgemm over the plane-wave
 * coefficients; the Rayleigh-Ritz of sec. 3.2, Algorithm 1).  A [K x p], B [K x q], C [p x q].
 * Deterministic split-K reduction in the workspace: at least p q complex128
 * (PW_ERR_NOMEM otherwise); a workspace smaller than the split needs only
 * lowers the number of K chunks. */
pw_status pw_gram(pw_ctx ctx, const void *A, int64_t lda, const void *B, int64_t ldb,
                  int64_t K, int32_t p, int32_t q, void *C, int64_t ldc);
/* Block update Y = alpha A C + beta Y (the Ritz-vector update of sec. 3.2, Algorithm 1: Psi Delta +
 * W Lambda + P Gamma).  A [K x p], C [p x q], Y [K x q]; alpha, beta real.
 * Y must not overlap A unless q <= 64 and Y == A (in-place right multiply). */
pw_status pw_block_update(pw_ctx ctx, const void *A, int64_t lda, const void *C, int64_t ldc,
                          int64_t K, int32_t p, int32_t q, double alpha, double beta,
                          void *Y, int64_t ldy);
/* The same two products on complex64 blocks (the PW_PREC_MIXED iteration):
 * A, B, Y complex64; C complex128 (pw_gram_mixed: FP32 products and sums
 * within each K chunk, chunk partials summed in FP64; pw_block_update_mixed:
 * C rounded to complex64 as it is read, FP32 products and sums). */
pw_status pw_gram_mixed(pw_ctx ctx, const void *A, int64_t lda, const void *B, int64_t ldb,
                        int64_t K, int32_t p, int32_t q, void *C, int64_t ldc);
pw_status pw_block_update_mixed(pw_ctx ctx, const void *A, int64_t lda, const void *C,
                                int64_t ldc, int64_t K, int32_t p, int32_t q, double alpha,
                                double beta, void *Y, int64_t ldy);
/* CholQR factor of a block (row a11 of the hot path; the orthonormalisation
 * W <- W R^-1 of the LOBPCG iteration, sec. 3.2): for G = R^H R (device,
 * Hermitian positive definite n x n, ldg >= n; the Hermitian part of the
 * stored matrix is used) write R^-1 (upper triangular, zeros below the
 * diagonal, positive real diagonal) to Rinv (device, ldr >= n).  1 <= n <= 64.
 * A tiny diagonal shift (1e-15 n max_i G_ii) is added; a non-positive pivot
 * returns PW_ERR_NUMERIC.  Synchronises the stream. */
pw_status pw_chol_inv(pw_ctx ctx, const void *G, int64_t ldg, int32_t n, void *Rinv, int64_t ldr);
/* Lowest k eigenpairs of a Hermitian n x n matrix A (lda >= n) -- the small
 * dense Rayleigh-Ritz eigenproblem of sec. 3.2 (Algorithm 1) and of the final
 * Rayleigh-Ritz (sec. 3.2, sec. 4.2).  Householder tridiagonalisation,
 * bisection, inverse iteration, re-orthogonalisation, back-transform, FP64;
 * the reduction runs in one workgroup for n <= 192 and over many above.
 * w: device double[k] ascending; V: device [n x k], ldv >= n.
 * A is overwritten.  1 <= k <= n <= 1024.  Needs the workspace. */
pw_status pw_small_eigh(pw_ctx ctx, void *A, int64_t lda, int32_t n, int32_t k,
                        void *w, void *V, int64_t ldv);
/* pw_small_eigh without the workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same kernels, with their scratch in a fixed
 * 4 MiB array the library holds on every GPU it runs on until the process
 * ends.  Needs only a context on a device (no pw_init_basis, no workspace);
 * allocates nothing, and clears its status word with a kernel (no memset).
 * Limit: 256 + heev_scratch(n, k) <= 4 MiB, i.e. k = n up to n ~ 700 and
 * k = 64 up to n = 1024 (heev_scratch(n, k) = 8*256 + 16n + 16n + 8nk +
 * 16n(3 + ceil(n/64)) bytes); larger (n, k) return PW_ERR_ARG naming the limit.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (several streams or host threads)
 * race and must be serialised by the caller.  Synchronises the context
 * stream (to report PW_ERR_NUMERIC); A is overwritten as in pw_small_eigh. */
pw_status pw_small_eigh_noalloc(pw_ctx ctx, void *A, int64_t lda, int32_t n, int32_t k,
                                void *w, void *V, int64_t ldv);
/* Residuals and preconditioned residuals (Eq. (1) with O = I; the residual
 * and preconditioning of sec. 3.1-3.2): theta_j = Re(x_j^H Hx_j) (columns of X assumed unit norm),
 * R = HX - X diag(theta), res_j = ||R_j||_2, and W = K(R) with the
 * Teter-Payne-Allan factor K(x) = (27+18x+12x^2+8x^3)/(27+18x+12x^2+8x^3+16x^4),
 * x = T_g / max(E_kin,j, 1e-3), E_kin,j = sum_g T_g |x_gj|^2.
 * theta, res: device double[nb].  W may be NULL (residual norms only). */
pw_status pw_residuals(pw_ctx ctx, const void *X, int64_t ldx, const void *HX, int64_t ldhx,
                       int32_t nb, void *theta, void *res, void *W, int64_t ldw);

#ifdef __cplusplus
}
#endif
#endif /* PWLOBPCG_H */
