/*
 * ofrr.h -- C ABI of the MI355X (gfx950) orthogonalization-free
 * Rayleigh-Ritz library.
 *
 * Method: Xu, Zhang, Chen, Saad and Xi, "Mixed Precision
 * Orthogonalization-Free Projection Methods for Eigenvalue and Singular
 * Value Problems" (arXiv 2505.00281).  A few eigenpairs of a symmetric A
 * (or singular triplets of a rectangular A) are computed by subspace
 * iteration whose basis is built in reduced precision without inner
 * products (per-column scaling and the Hessenberg process, Sec. 4.2),
 * projected in higher precision (G = V^T V, H = V^T A V, eq. (geig)), and
 * extracted from the small generalized eigenproblem in FP64 (Sec. 3, the
 * mixed-precision plan at the end of Sec. 4).
 *
 * Conventions shared by every entry point
 *   - Dense matrices are column-major with a leading dimension (ld >= rows).
 *   - Every array argument is a DEVICE pointer on the context's device,
 *     owned by the caller, unless the comment says "host".  Inputs are
 *     read-only; outputs are overwritten.  Nothing is retained after a call
 *     returns.
 *   - Every call is enqueued on the context's HIP stream and returns once
 *     its outputs are ready (the call synchronises that stream).
 *   - A negative status is a failure: outputs are undefined and
 *     ofrr_last_error() describes it.  Arguments are validated before any
 *     device work; invalid ones give OFRR_ERR_INVALID_ARG and touch
 *     nothing.  No C++ exception crosses this boundary.
 *   - A context is used by one host thread at a time.
 */
#ifndef OFRR_H
#define OFRR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ofrr_ctx_s *ofrr_ctx;

typedef enum {
    OFRR_OK = 0,
    OFRR_NOT_CONVERGED = 1,     /* warning: outputs valid, fewer than k pairs met tol */
    OFRR_ERR_INVALID_ARG = -1,
    OFRR_ERR_UNSUPPORTED = -2,  /* valid but not implemented combination */
    OFRR_ERR_NO_DEVICE = -3,
    OFRR_ERR_OOM = -4,
    OFRR_ERR_HIP = -5,          /* a HIP runtime call failed */
    OFRR_ERR_NUMERIC = -6       /* NaN/Inf met, or every basis column dropped */
} ofrr_status;

typedef enum { OFRR_DENSE_COLMAJOR = 0, OFRR_CSR = 1 } ofrr_format;

typedef enum {
    OFRR_F64 = 0,
    OFRR_F32 = 1,
    OFRR_BF16 = 2,
    OFRR_F16 = 3,
    OFRR_F8E4M3 = 4   /* OCP e4m3fn with one power-of-two scale per 32 x 32 block */
} ofrr_dtype;

typedef enum { OFRR_LARGEST = 0, OFRR_SMALLEST = 1 } ofrr_which;
typedef enum { OFRR_POWER = 0, OFRR_CHEBYSHEV = 1 } ofrr_filter;
/* Products of the FP64 phase that ends a refined plan (dense A). */
typedef enum {
    OFRR_TAIL_F64 = 0,       /* FP64 arithmetic */
    OFRR_TAIL_I8_SLICED = 1  /* exact INT8 products of 7-bit digit planes: 6 of each row of
                                A (FP32 or FP64 stored) and 6 of each basis column, the 21
                                digit pairs with s + t <= 7 summed in int32; the result is
                                within about 2^-40 of |A||V| per entry (FP64 gives 2^-53 K) */
} ofrr_tail;

/* Accumulation of the projections G = V^T V, H = V^T W (the mixed-
 * precision plan at the end of Sec. 4 forms them in FP32 from reduced-
 * precision data).  The FP32 modes take FP32, BF16 or F16 blocks (FP64
 * blocks give OFRR_ERR_UNSUPPORTED) and use FP32 MFMA, whose products of
 * such values are rounded to FP32. */
typedef enum {
    OFRR_ACC_F32 = 0,             /* FP32 sums over each workgroup's row chunk (at least
                                     256 rows), chunk partials summed in FP32 */
    OFRR_ACC_F32_COMPENSATED = 1, /* FP32 sums over runs of 32 rows, the runs and the
                                     chunk partials summed in FP64: per entry the error
                                     of a 32-term FP32 sum, independent of n */
    OFRR_ACC_F64 = 2              /* FP64 sums (products of stored values are exact) */
} ofrr_accum;

/* Matrix descriptor.  Dense: values (rows x cols, column-major, ld).
 * CSR: 0-based row_ptr[rows+1] and col_idx[nnz] sorted within each row,
 * values[nnz].  values are FP64 or FP32 (dtype).  Symmetry of A is assumed
 * by the eigenvalue entry points, not checked. */
typedef struct {
    ofrr_format format;
    ofrr_dtype dtype;
    int64_t rows, cols, ld;
    const void *values;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    int64_t nnz;
} ofrr_matrix;

/* Precision plan and iteration controls.  Fill with ofrr_plan_default(). */
typedef struct {
    ofrr_dtype basis_dtype;  /* storage/compute type of the products and the basis in
                                the first phase: F64 gives the FP64 form of the method
                                (all FP64); F32, BF16, F16, F8E4M3 the mixed forms */
    ofrr_accum gram_accum;   /* accumulation of G and H in the first phase (later
                                phases and the FP64 form accumulate in FP64); see
                                gram_switch_t */
    int32_t refine;          /* 0: one phase in basis_dtype; 1: first phase until its
                                residual estimate stalls, then an FP64 tail; 2 (dense,
                                BF16): BF16 phase, then a phase with A and the basis as
                                two-term BF16 splits (about 16 significant bits each,
                                three MFMAs per fragment), then the FP64 tail; 2 (CSR,
                                F16 or BF16): the 16-bit phase, an FP32 phase, the FP64
                                tail */
    ofrr_filter filter;
    int32_t degree;          /* products per outer iteration (power steps or
                                Chebyshev degree), >= 1 */
    double lo, hi;           /* Chebyshev damping interval [lo, hi], lo < hi */
    double drop_tol;         /* Hessenberg column drop tolerance on |pivot| of a column
                                scaled to infinity-norm (1/2, 1]; 0 -> machine epsilon of
                                the arithmetic the sweep runs in (FP64 for the FP64 form,
                                FP32 for reduced-precision phases, whose sweep works on
                                the FP32 product before rounding; Sec. 5.2 ties the
                                tolerance to the working precision) */
    double tol;              /* stop when all k relative residuals <= tol; 0 -> run
                                exactly max_iters outer iterations */
    double anorm;            /* residual normaliser ||A||_2; 0 -> max |Ritz value| */
    int32_t max_iters;       /* outer iterations cap (>= 1) */
    int32_t stall_iters;     /* refine>=1: leave a reduced-precision phase once the
                                smallest largest-wanted-residual estimate of the last
                                stall_iters outer iterations is not 10% below the
                                smallest one before them */
    double switch_resid;     /* refine>=1: also leave it once the largest wanted residual
                                estimate is below this value (0 -> never by value) */
    int32_t b_split;         /* BF16/F16 products: 2 carries the basis block as a two-
                                term split (hi + lo) through the MFMA, 1 rounds it once */
    int32_t profile;         /* nonzero: time every kernel launch with HIP events */
    int32_t tail_product;    /* ofrr_tail: products of the FP64 phase after reduced-precision
                                phases (refine >= 1, dense A; ofrr_eig_partial,
                                ofrr_eig_general and ofrr_svd_partial); the FP64 form
                                (basis_dtype F64) always runs FP64 arithmetic */
    double gram_switch_t;    /* FP32 gram_accum: a projection is accumulated in FP64 instead
                                when the conditioning statistic of the previous iteration's
                                mass matrix, t(G) = sum_i G_ii (G^-1)_ii / b (t = 1 for a
                                diagonal G; t <= kappa of G scaled to unit diagonal), is
                                above this value, or when that G was not numerically
                                positive definite; 0 -> 1000 (an FP32 perturbation of
                                2^-24 per term of a 32-row run, scaled by t, stays below
                                about 1e-3 of G's smallest eigenvalue) */
    int32_t svd_form;        /* ofrr_svd_partial: 0 the augmented pencil [0 B; B^T 0] of
                                Sec. 3.2 (the paper's form); 1 the normal equations: the
                                eigen solver on the operator A^T A (each product A V then
                                A^T (A V)), s = sqrt(theta), u = A v / s.  The second
                                squares the condition of the singular values: s is found
                                to about u (s_1 / s)^2 relative (dense A, BF16/F16/F64
                                basis) */
    int32_t stab;            /* basis stabilisation: 0 the Hessenberg process (Sec. 4.2);
                                1 QR by MGS with re-orthogonalisation (the comparison of
                                Sec. 5.2) */
    int32_t projection;      /* 0 the orthogonalization-free pencil H y = theta G y
                                (Sec. 3.1); 1 the classical Rayleigh-Ritz projection,
                                which takes the basis as orthonormal (G = I) */
    int32_t qr_dtype;        /* stab 1: arithmetic of the QR (an ofrr_dtype: F64, F32, or F16
                                storage with FP32 arithmetic); -1 -> the phase's storage type.  A QR wider
                                than a reduced-precision phase's storage leaves its basis at
                                the phase's FP32 master precision (the products still read it
                                rounded to the storage type): the [MatVec]-[QR] precision
                                pairs of the Sec. 2 experiment */
    int32_t matvec_round;    /* reduced-precision phases: every product's result rounded to
                                this type, F16 or BF16, before use, the product itself
                                computed in the phase's arithmetic (an F32 phase: from A as
                                stored); -1 -> not rounded.  With stab 1 and qr_dtype this
                                gives the [MatVec]-[QR] pairs of the Sec. 2 experiment */
    int32_t tail_digits;     /* OFRR_TAIL_I8_SLICED: signed 7-bit digits per side of the
                                digit-plane products.  0: chosen per iteration from the
                                previous largest residual estimate r (4 while r > 1600
                                2^-28, 5 while r > 1600 2^-35, else 6); 4, 5 or 6: fixed.
                                S digits are exact to about 2^-7S of the row and column
                                scales of A and V.  The iteration stops at tol only after
                                an iteration whose products took six digits (eig_partial,
                                eig_general, svd_partial) */
} ofrr_plan;

typedef struct {
    int32_t iters;           /* outer iterations done */
    int32_t iters_low;       /* of which in the first (reduced-precision) phase */
    int32_t n_converged;     /* wanted pairs with final residual <= tol */
    int32_t basis_eff;       /* columns kept by the last Hessenberg sweep */
    int32_t products;        /* block products by A (or A^T) */
    double max_resid;        /* largest final residual among the k pairs */
    double seconds;          /* device time of the call (HIP events on the stream) */
    double gram_t_max;       /* largest t(G) seen while the FP32 gram_accum was in force
                                (0 if it never was) */
    int32_t grams_f64;       /* first-phase projections that t(G) sent to FP64 */
} ofrr_info;

/* --------------------------------------------------------------------- */
/* Context                                                                */
/* --------------------------------------------------------------------- */

/* Defaults: FP64 basis, FP64 accumulation, no refinement, power filter of
 * degree 1, drop_tol 0, tol 0, anorm 0, max_iters 20, stall_iters 3,
 * switch_resid 0, b_split 1, profile 0, tail_product F64, gram_switch_t 0,
 * svd_form 0, stab 0, projection 0, qr_dtype -1, matvec_round -1, tail_digits 0. */
void ofrr_plan_default(ofrr_plan *plan);

/* Creates a context bound to `device` and to `hip_stream` (a hipStream_t,
 * NULL = the default stream).  The context owns a workspace that grows to
 * the largest problem seen and is reused; it is freed by ofrr_destroy.
 * Errors: OFRR_ERR_NO_DEVICE if no HIP device `device` is visible. */
ofrr_status ofrr_create(ofrr_ctx *ctx, int device, void *hip_stream);
ofrr_status ofrr_destroy(ofrr_ctx ctx);

/* Message of the last failure on this context (or of the last failed
 * ofrr_create when ctx is NULL); valid until the next call. */
const char *ofrr_last_error(ofrr_ctx ctx);

/* Kernel timing (plan.profile != 0): number of launches and summed device
 * milliseconds of the kernel family `name` since the last reset, measured
 * with HIP events on the context's stream.  Families: "quantize",
 * "product_bf16", "product_bf16x2", "product_f16", "product_f8", "product_f64", "product_f32",
 * "product_i8x" (the digit-plane products; also by digits per side:
 * "product_i8x_d4", "product_i8x_d5", "product_i8x_d6"), "product_reduce"
 * (the fixed-order sum of split-K
 * partials), "spmm" (every CSR product; the solver's phases also by block
 * storage: "spmm_f16" for binary16/bfloat16, "spmm_f32", "spmm_f64"),
 * "scale", "hessenberg", "gram", "small_eig", "lift", "residual".
 * Returns OFRR_ERR_INVALID_ARG for an unknown name. */
ofrr_status ofrr_kernel_stats(ofrr_ctx ctx, const char *name, int64_t *launches /*host*/,
                              double *total_ms /*host*/);
ofrr_status ofrr_kernel_stats_reset(ofrr_ctx ctx);
/* Kernel timing for the step entry points (on != 0: every launch of a step
 * call is timed into the families above); the whole-method calls set it
 * from plan.profile. */
ofrr_status ofrr_set_profile(ofrr_ctx ctx, int32_t on);

/* --------------------------------------------------------------------- */
/* Whole-method entry points (Sec. 2-4)                                   */
/* --------------------------------------------------------------------- */

/* k eigenpairs of a symmetric A (rows == cols == n) by subspace iteration
 * with a basis of `basis` columns (k <= basis <= n), the filter of `plan`
 * (Alg. "Multiple Step Subspace Iteration" with restart from all Ritz
 * vectors), the Hessenberg process in place of QR (Sec. 4.2) and the
 * orthogonalization-free projection (Sec. 3.1, eq. (geig)).
 *   X0     n x basis start block, FP64, column-major (ld = n), or NULL for
 *          U(0,1) drawn on the device from a fixed seed.
 *   evals  k FP64, sorted by `which` (descending for LARGEST).
 *   evecs  n x k FP64 column-major (ld = n), unit 2-norm, the entry of
 *          largest magnitude (first on ties) positive.
 *   resid  k FP64: ||A x - lambda x||_2 / anorm, computed in FP64 from A as
 *          stored.
 *   info   host, may be NULL.
 * Returns OFRR_OK, OFRR_NOT_CONVERGED (tol > 0 and some resid > tol), or an
 * error. */
ofrr_status ofrr_eig_partial(ofrr_ctx ctx, const ofrr_matrix *A, int32_t k, int32_t basis,
                             ofrr_which which, const ofrr_plan *plan, const double *X0,
                             double *evals, double *evecs, double *resid, ofrr_info *info);

/* k largest singular triplets of a dense A (m x n, column-major) by
 * alternating subspace iteration U = A V, V = A^T U with the Hessenberg
 * process as stabiliser and the orthogonalization-free projection for the
 * SVD (Sec. 3.2): the positive eigenvalues of
 * [0 B; B^T 0] [y; z] = s blkdiag(U^T U, V^T V) [y; z], B = U^T A V, lifted
 * as sqrt(2) U Y and sqrt(2) V Z (Theorem of Sec. 3.2).
 *   V0     n x basis FP64 start block or NULL.
 *   sigma  k FP64 descending; U m x k and V n x k FP64 column-major;
 *   resid  k FP64 sqrt(||A v - s u||^2 + ||A^T u - s v||^2) / anorm.
 * plan.filter must be OFRR_POWER with degree 1; plan.gram_accum must be
 * OFRR_ACC_F64 (OFRR_ERR_UNSUPPORTED otherwise). */
ofrr_status ofrr_svd_partial(ofrr_ctx ctx, const ofrr_matrix *A, int32_t k, int32_t basis,
                             const ofrr_plan *plan, const double *V0, double *sigma,
                             double *U, double *V, double *resid, ofrr_info *info);

/* k eigenpairs of largest modulus of a real non-symmetric A (rows == cols
 * == n, dense or CSR) by the same subspace iteration: products A V, the
 * power filter, the Hessenberg process, and the orthogonalization-free
 * projection with complex Ritz values (Sec. 3.1: the Galerkin condition
 * on a basis that is not orthonormal gives the pencil V^T A V y =
 * lambda V^T V y, eq. (geig); Alg. "Orthogonalization-Free Rayleigh-Ritz
 * Projection").  The pencil is solved in FP64 on the GPU by Cholesky
 * reduction and a Francis double-shift QR iteration; the restart block is
 * the real basis of all Ritz vectors (a conjugate pair contributes the real
 * and imaginary parts of one member).
 *   X0        n x basis FP64 start block (column-major) or NULL.
 *   evals_re, evals_im  k FP64: modulus descending, then real part, then
 *             imaginary part descending (of a conjugate pair the member
 *             with positive imaginary part first).  A pair cut at k keeps
 *             its first member only.
 *   evecs_re, evecs_im  n x k FP64 column-major: the real and imaginary
 *             parts of unit-2-norm vectors whose entry of largest modulus
 *             (first on ties) is real and positive.
 *   resid     k FP64: ||A x - lambda x||_2 / anorm, in FP64 from A as
 *             stored (anorm = plan.anorm, or the largest Ritz modulus).
 * plan: basis_dtype F64, BF16 or F16 (refine as for ofrr_eig_partial: a
 * split-BF16 middle phase for refine 2 with dense A, an FP32 one for CSR,
 * and the FP64 tail), filter OFRR_POWER, stab Hessenberg, projection OFRR,
 * gram_accum F64, qr_dtype and matvec_round unset; OFRR_ERR_UNSUPPORTED
 * otherwise.  OFRR_ERR_NUMERIC if the projected mass matrix is not positive
 * definite or the small eigensolver does not converge. */
ofrr_status ofrr_eig_general(ofrr_ctx ctx, const ofrr_matrix *A, int32_t k, int32_t basis, const ofrr_plan *plan,
                             const double *X0, double *evals_re, double *evals_im, double *evecs_re,
                             double *evecs_im, double *resid, ofrr_info *info);

/* nprob independent symmetric eigenproblems (dense, each with its own n),
 * the same k, basis and plan.  As[p], X0s (may be NULL), evals[p],
 * evecs[p], resid[p] are per-problem pointers held in HOST arrays of length
 * nprob; the pointers themselves are device pointers.  infos: host array of
 * nprob or NULL. */
ofrr_status ofrr_eig_partial_batched(ofrr_ctx ctx, int32_t nprob, const ofrr_matrix *As,
                                     int32_t k, int32_t basis, ofrr_which which,
                                     const ofrr_plan *plan, const double *const *X0s,
                                     double *const *evals, double *const *evecs,
                                     double *const *resid, ofrr_info *infos);

/* What the last ofrr_eig_partial_batched call on this context ran (host
 * outputs, any may be NULL): *grouped = 1 if it took the grouped path (one
 * launch per step over all unconverged problems, iterations replayed from a
 * HIP graph: plans with degree 1, basis <= 32, refine <= 1, BF16/F16 or F64
 * basis, FP64 projections, dense A), else 0 (problems one after another);
 * *rows_red and *rows_f64 the row-tile heights of its reduced and FP64
 * grouped products, picked by timing each candidate (64, 128, 256 rows) on
 * the first call for a given problem set and cached in the context;
 * *replays the graph replays (outer iterations of the slowest problem,
 * rounded up to the readback interval); *first_product_ms the device time
 * (HIP events on the context's stream) of the call's first grouped product
 * A X0, which covers every problem in the first phase. */
ofrr_status ofrr_batched_last_config(ofrr_ctx ctx, int32_t *grouped, int32_t *rows_red, int32_t *rows_f64,
                                     int32_t *replays, double *first_product_ms);

/* The paper's Krylov method for sparse (or dense) symmetric A (Sec. 4.1,
 * Alg. "Computing non-orthogonal bases from the Krylov-Hessenberg
 * Process", with the orthogonalization-free projection of Sec. 3.1 and the
 * restart of the sparse experiments in Sec. 5.2): each cycle builds the
 * Krylov-Hessenberg basis of K_k(A, v) (v scaled by its largest entry,
 * then per step w = A v_j loses its entry at each earlier pivot row times
 * that basis vector, and is scaled by its new largest entry: no inner
 * products), projects G = V^T V and H = V^T A V in FP64, solves the pencil
 * in FP64, and restarts from the Ritz vector of the largest Ritz value;
 * `restarts` cycles follow the first.
 *   k          Krylov dimension, 2 <= k <= 512, k <= n.
 *   nev        wanted pairs (largest algebraic), 1 <= nev <= k.
 *   basis_dtype storage and arithmetic of the process: OFRR_F64, OFRR_F32,
 *              or OFRR_F16 (binary16 storage, FP32 arithmetic).
 *   v0         n FP64 start vector (device) or NULL for U(0,1).
 *   tol        > 0: info.n_converged counts resid <= tol (and the status is
 *              OFRR_NOT_CONVERGED if fewer than nev meet it); 0: no test.
 *   evals      nev FP64, descending; evecs n x nev FP64 column-major, unit
 *              2-norm, sign rule as ofrr_eig_partial.
 *   resid      nev FP64: ||A x - lambda x||_2 / |lambda|, from A as stored
 *              in FP64 (the paper's Krylov metric).
 * If the process meets an invariant subspace (w = 0) the basis stops there
 * (info.basis_eff < k) and the projection drops the missing directions. */
ofrr_status ofrr_krylov_eig(ofrr_ctx ctx, const ofrr_matrix *A, int32_t k, int32_t nev, int32_t restarts,
                            ofrr_dtype basis_dtype, const double *v0, double tol, double *evals,
                            double *evecs, double *resid, ofrr_info *info);

/* --------------------------------------------------------------------- */
/* Step entry points: one step of the method on caller buffers.  They run  */
/* the same kernels the whole-method calls use.                           */
/* --------------------------------------------------------------------- */

/* Round an FP32 array of `count` elements to `dst_dtype` (BF16 or F16 bits,
 * uint16 per element), round to nearest even.  Mixed-precision plan of
 * Sec. 4: the matrix and basis are stored in reduced precision. */
ofrr_status ofrr_quantize(ofrr_ctx ctx, ofrr_dtype dst_dtype, int64_t count,
                          const float *src, void *dst);

/* FP8 e4m3fn with one power-of-two scale per 32 x 32 block: A (rows x cols
 * FP32 column-major, lda) -> codes (rows x cols uint8, column-major, ld =
 * rows) and scales (ceil(rows/32) x ceil(cols/32) FP32, column-major).  The
 * block scale is 2^ceil(log2(amax/448)) (1 for an all-zero block); the code
 * is e4m3fn(A/scale), nearest even, saturating. */
ofrr_status ofrr_quantize_fp8_blocks(ofrr_ctx ctx, int64_t rows, int64_t cols, const float *A,
                                     int64_t lda, uint8_t *codes, float *scales);

/* Block product W = op(A) V (Sec. 2, the products X_{iter} = A^{iter} X_0).
 *   A         descriptor: dense F64/F32 (FP64 arithmetic, FP64 V and W), dense
 *             BF16/F16 (uint16 values; V BF16/F16 in the same type, W FP32;
 *             MFMA with FP32 accumulation), or CSR F32/F64 (V and W FP32 or
 *             FP64 per v_dtype).
 *   trans     0: W = A V; 1: W = A^T V (dense only).
 *   v_dtype   element type of V and W as described above.
 *   V         (op(A) cols) x b, row-major (ld = b); W (op rows) x b, row-major
 *             (ld = b). */
ofrr_status ofrr_block_product(ofrr_ctx ctx, const ofrr_matrix *A, int32_t trans, int32_t b,
                               ofrr_dtype v_dtype, const void *V, void *W);

/* FP64-class block product W = op(A) V from exact INT8 digit-plane products
 * (the OFRR_TAIL_I8_SLICED products of the final phase; Sec. 2 products).
 * A: dense F32/F64 descriptor; V: FP64 row-major (op(A) cols) x b (ld b);
 * W: FP64 row-major (op(A) rows) x b (ld b); digits: signed 7-bit digits per
 * side, 4, 5 or 6 (0 -> 6).  Per entry the error is below
 * 2^-7d (2^e_i sum_k |V_kj| + 2^f_j sum_k |op(A)_ik| + 1.02 (d - 1) K 2^(e_i+f_j))
 * plus FP64 rounding of the final sums, with d the digits, 2^e_i the
 * smallest power of two above max_k |op(A)_ik| and 2^f_j that above
 * max_k |V_kj| (d = 6: 2^-42 and 5.1 K). */
ofrr_status ofrr_block_product_sliced(ofrr_ctx ctx, const ofrr_matrix *A, int32_t trans, int32_t b,
                                      int32_t digits, const double *V, double *W);

/* FP8 block product W = op(A) V (trans 0: A V; 1: A^T V) for A given as
 * e4m3fn codes (rows x cols, column-major, ld = rows) with 32 x 32 block
 * scales as produced by ofrr_quantize_fp8_blocks.  V: FP32 row-major
 * (op(A) cols x b), quantised inside the call to e4m3fn with one
 * power-of-two scale per 32 consecutive rows of each column (the smallest
 * 2^k with amax / 2^k <= 448).  W: FP32 row-major (op(A) rows x b); both
 * operands' scales are applied inside the block-scaled MFMA, accumulation
 * in FP32. */
ofrr_status ofrr_block_product_fp8(ofrr_ctx ctx, int64_t rows, int64_t cols, const uint8_t *codes,
                                   const float *scales, int32_t trans, int32_t b, const float *V,
                                   float *W);

/* Right-looking Hessenberg process on an n x b block Y (Sec. 4.2) in FP64
 * (dtype F64) or FP32 (dtype F32), in place: for each column the first row
 * of largest magnitude is the pivot; a column whose pivot magnitude is
 * below tol is dropped (keep=0, piv=-1), otherwise it is divided by its
 * pivot and its multiple eliminates the pivot row from every later column
 * (one fused multiply-add per element).  piv, keep: int32[b].  Returns the
 * kept count in *kept (host).  The kept columns equal P^T L of the
 * row-pivoted LU factorisation of Y. */
ofrr_status ofrr_hessenberg(ofrr_ctx ctx, ofrr_dtype dtype, int64_t n, int32_t b, void *Y,
                            int64_t ldy, double tol, int32_t *piv, int32_t *keep,
                            int32_t *kept);

/* Allocation-free variant of ofrr_hessenberg, for callers that cannot
 * allocate device or pinned memory during a call: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and results (bit for bit) as ofrr_hessenberg; the
 * sweep's exchange words live in a fixed device array of the library
 * (526,336 64-bit words = 4 MiB + 16 KiB, one per GPU, whose address the
 * context takes at ofrr_create and which stays allocated until the process
 * ends) instead of the context's workspace, and the kept count is read
 * back through host stack memory.  Maximum size: the sweep needs
 * 1 + 2 G (w + 1) + 2 G b w words (G <= 256 row slices, w = 2 for F64 and 1
 * for F32), which covers every n with b <= 512; a larger need gives
 * OFRR_ERR_INVALID_ARG before any launch.  Every call on one GPU shares
 * that array (each call clears it before its sweep): calls that overlap on
 * one GPU (two streams, contexts or threads) race and must not be issued.
 * Kernel timing (plan.profile) is not recorded for this call. */
ofrr_status ofrr_hessenberg_noalloc(ofrr_ctx ctx, ofrr_dtype dtype, int64_t n, int32_t b, void *Y,
                                    int64_t ldy, double tol, int32_t *piv, int32_t *keep,
                                    int32_t *kept);

/* The basis-generation processes compared with the Hessenberg process
 * (Sec. 4.2, the comparison table of MGS, CGS and Hessenberg; timed in
 * Sec. 5.3, Table 3). */
typedef enum {
    OFRR_BASIS_MGS_L = 0,  /* left-looking MGS, no re-orthogonalisation: column j is
                              projected against q_0..q_{j-1} one at a time */
    OFRR_BASIS_MGS_R = 1,  /* right-looking MGS: q_i removed from all later columns */
    OFRR_BASIS_CGS = 2,    /* classical GS: r = Q^T a_j, v = a_j - Q r */
    OFRR_BASIS_CGS2 = 3,   /* CGS with one re-orthogonalisation */
    OFRR_BASIS_HESS_L = 4, /* Hessenberg process, left-looking (column j receives the
                              eliminations of the kept columns before it, in order) */
    OFRR_BASIS_HESS_R = 5, /* Hessenberg process, right-looking (Alg. "Computing
                              non-orthogonal bases from the Hessenberg Process") */
    OFRR_BASIS_MGS2 = 6    /* left-looking MGS with a second projection pass when the
                              first reduced the norm below sqrt(2)/2 of its value
                              (Sec. 5.1); the QR of the classical comparisons */
} ofrr_basis_method;

/* One basis-generation process on a column-major m x n block A (lda >= m,
 * n <= m, n <= 512, m < 2^31), in place, as one cooperative launch on the
 * context's stream:
 *   storage  OFRR_F64 (double), OFRR_F32 (float) or OFRR_F16 (binary16 bits,
 *            uint16 per entry, every result rounded to binary16, FP32
 *            arithmetic and FP32 inner products: the paper's FP16 runs).
 *   Gram-Schmidt methods: A becomes Q (orthonormal columns up to rounding);
 *            R (n x n FP64, column-major, upper triangle; NULL to skip) gets
 *            the coefficients, A_in = Q R.  No column is dropped, except by
 *            MGS2 with tol > 0: a column whose norm after its projections is
 *            at most tol times its norm before them is excluded (keep = 0,
 *            piv = -1, left unnormalised and not projected out of later
 *            columns; piv = j for a kept column); piv and keep may then be
 *            NULL (not returned).
 *   Hessenberg methods: the pivot of column j is its first row of largest
 *            magnitude, the column is divided by it and its multiple removed
 *            from later columns (one fused multiply-add per entry); columns
 *            whose pivot magnitude is below tol are dropped (keep = 0,
 *            piv = -1) and eliminate nothing.  The kept columns of A are
 *            then P^T L of the row-pivoted LU factorisation.  piv, keep:
 *            int32[n] device; R ignored.  The two forms give the same bits.
 *   kept     host, may be NULL: kept columns (n for Gram-Schmidt without
 *            exclusion).
 *   kernel_ms host, may be NULL: device time of the launch (HIP events).
 * A grid-barrier wait that times out gives OFRR_ERR_HIP. */
ofrr_status ofrr_basis_generate(ofrr_ctx ctx, ofrr_basis_method method, ofrr_dtype storage, int64_t m,
                                int32_t n, void *A, int64_t lda, double tol, double *R, int32_t *piv,
                                int32_t *keep, int32_t *kept, double *kernel_ms);

/* Projections G = V^T V and H = V^T W (Alg. "Orthogonalization-Free
 * Rayleigh-Ritz Projection", the products forming B and M), b x b FP64
 * outputs, column-major.  V: n x b in v_dtype (F64, F32, BF16, F16); W:
 * n x b in w_dtype (F64 or F32); both row-major with ld = b.  Accumulation
 * per `accum` (FP32 modes: no FP64 block; else OFRR_ERR_UNSUPPORTED). */
ofrr_status ofrr_project(ofrr_ctx ctx, int64_t n, int32_t b, ofrr_dtype v_dtype, const void *V,
                         ofrr_dtype w_dtype, const void *W, ofrr_accum accum, double *G,
                         double *H);

/* Symmetric definite pencil H y = theta G y (eq. (geig)) in FP64 on the
 * GPU: Cholesky G = L L^T, symmetric eigen-decomposition of L^{-1} H L^{-T}
 * by cyclic Jacobi, Y = L^{-T} Z.  theta: b, sorted by `which`; Y: b x b
 * with Y^T G Y = I.  If G is not positive definite the directions of G with
 * eigenvalues below 1e-14 * max are discarded first and the discarded
 * columns of Y are zero with theta = 0 placed last; *rank (host) receives
 * the number of retained directions. */
ofrr_status ofrr_pencil_eig(ofrr_ctx ctx, int32_t b, const double *H, const double *G,
                            ofrr_which which, double *theta, double *Y, int32_t *rank);

/* Non-symmetric pencil H y = theta G y (eq. (geig) for a real
 * non-symmetric A, Sec. 3.1), FP64 on the GPU: Cholesky G = L L^T,
 * C = L^{-1} H L^{-T}, Householder reduction of C to Hessenberg form,
 * Francis double-shift QR iteration to real Schur form, eigenvectors by
 * back substitution, y = L^{-T} z with unit z.  H, G: b x b column-major
 * (G symmetric positive definite; its symmetric part is used).
 *   theta_re, theta_im  b: the order of ofrr_eig_general.
 *   Y   b x b column-major, packed real: a real theta's column is y; a
 *       conjugate pair (slots j, j+1, theta_im[j] > 0) holds Re y and Im y
 *       of the member with positive imaginary part.  y^H G y = 1.
 * OFRR_ERR_NUMERIC if G is not positive definite or the iteration does not
 * converge (30 max(10, b) double-shift steps). */
ofrr_status ofrr_pencil_eig_general(ofrr_ctx ctx, int32_t b, const double *H, const double *G, double *theta_re,
                                    double *theta_im, double *Y);

/* The SVD pencil of Sec. 3.2 for B (k1 x k2), MU (k1 x k1), MV (k2 x k2):
 * sigma (min(k1,k2), descending, the positive eigenvalues), Y (k1 x
 * min(k1,k2)), Z (k2 x min(k1,k2)) normalised so that [y; z]^T blkdiag(MU,
 * MV) [y; z] = 1.  All device pointers, column-major, k1 + k2 <= 1024.
 * OFRR_ERR_NUMERIC if MU or MV is not positive definite (the message names
 * which); OFRR_ERR_HIP if a grid barrier of the multi-workgroup Jacobi
 * sweeps (k1, k2 <= 256) timed out. */
ofrr_status ofrr_svd_pencil(ofrr_ctx ctx, int32_t k1, int32_t k2, const double *B,
                            const double *MU, const double *MV, double *sigma, double *Y,
                            double *Z);

#ifdef __cplusplus
}
#endif

#endif /* OFRR_H */
