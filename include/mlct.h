/*
 * mlct.h - multilevel Chebyshev-Hutchinson trace estimation on gfx950.
 *
 * C ABI of libmlct.so.  The library estimates tr f(A) for a symmetric matrix
 * A (Section 1, eq. def:trace) by Hutchinson's estimator over Rademacher
 * probes (Section 2.1, eq. def:mcEstimate), with f replaced by its degree-n
 * Chebyshev interpolant on an interval [a, b] that contains the spectrum
 * (Section 2.2, eqs. eqn:recurrence and eqn:chebSeries), split into levels
 * (Section 3, eqs. def:qlevels and eqn:decomposition) and combined by the
 * multilevel estimator (Section 4, eq. eqn:multiEstimator).
 *
 * Conventions shared by every call:
 *  - Every function returns an mlct_status.  Arguments are validated before
 *    any device work is enqueued; on error the outputs are left untouched and
 *    mlct_last_error(ctx) describes the reason.  No C++ exception crosses
 *    this boundary.
 *  - Matrix and probe buffers passed in are DEVICE pointers owned by the
 *    caller; they are borrowed and must stay valid (and unmodified) while an
 *    operator handle that refers to them is in use.
 *  - Output arrays are HOST pointers unless the parameter name ends in _dev.
 *  - Device work is enqueued on the stream given to mlct_create.  A call that
 *    returns host results synchronises that stream before returning.
 *  - Calls on one context are not thread-safe; use one context per thread.
 *  - The library allocates its own device workspace (grow-only, owned by the
 *    context, freed by mlct_destroy).
 */
#ifndef MLCT_H
#define MLCT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MLCT_OK = 0,
  MLCT_EINVAL = 1,       /* invalid argument (shape, pointer, interval, CSR) */
  MLCT_ENOMEM = 2,       /* device workspace allocation failed or over cap  */
  MLCT_EDEVICE = 3,      /* a HIP runtime call failed                       */
  MLCT_ESPECTRUM = 4,    /* |mu_j| > |z|^2 (1 + 1e-3): spectrum outside [a,b] */
  MLCT_ERANGE = 5,       /* coefficients or result not representable        */
  MLCT_EUNSUPPORTED = 6  /* valid request this build does not implement     */
} mlct_status;

/* f in tr f(A) (Section 1: log-determinant, trace of inverse, Estrada
 * index, Schatten norms via A = X^T X; Section 5: sqrt, log, exp, x^3). */
typedef enum {
  MLCT_LOG = 0,   /* f(x) = log x      (needs a > 0)                  */
  MLCT_SQRT = 1,  /* f(x) = sqrt x     (needs a >= 0)                 */
  MLCT_EXP = 2,   /* f(x) = exp x      (result carries a log-scale)   */
  MLCT_CUBE = 3,  /* f(x) = x^3                                       */
  MLCT_INV = 4,   /* f(x) = 1/x        (needs 0 outside [a, b])       */
  MLCT_POW = 5    /* f(x) = x^power    (needs a >= 0)                 */
} mlct_func_kind;

typedef struct {
  int32_t kind;  /* mlct_func_kind */
  double power;  /* exponent for MLCT_POW, ignored otherwise */
} mlct_func;

/* Arithmetic of the recurrence.  FP32: FP32 vectors and matrix, FP32
 * products, FP64 moment accumulation.  FP64: everything FP64.  BF16X3: dense
 * operators only, A and V split into bf16 hi+lo parts, three bf16 MFMA
 * products (hi*hi + hi*lo + lo*hi) accumulated in FP32. */
typedef enum {
  MLCT_FP64 = 0,
  MLCT_FP32 = 1,
  MLCT_BF16X3 = 2
} mlct_prec;

/* How moments are formed (Section 2.2, Section 3.1).  DIRECT: n matvecs,
 * mu_j = z . T_j(A_hat) z.  DOUBLING: ceil(n/2) matvecs, mu_{2k} =
 * 2 v_k.v_k - mu_0 and mu_{2k+1} = 2 v_{k+1}.v_k - mu_1.  OR-ing
 * MLCT_LEVEL_INTERP into the mode of mlct_estimate gives every level its own
 * interpolant of degree l_k instead of truncating the top one. */
typedef enum {
  MLCT_DIRECT = 0,
  MLCT_DOUBLING = 1
} mlct_mode;
#define MLCT_LEVEL_INTERP 0x10
/* OR'ed into the mode of mlct_estimate / mlct_estimate_batch: the terms
 * j <= 2 leave the level variables and enter exactly as
 * sum_{j<=2} c_j tr T_j(A_hat), with tr T_0 = d, tr T_1 = alpha tr A + beta d
 * and tr T_2 = 2 ||A_hat||_F^2 - d (A symmetric), from tr A and ||A||_F^2
 * computed once per operator (the exactly computable low-degree traces
 * remarked on at the end of Section 5.4).  c_j are the top interpolant's. */
#define MLCT_EXACT_LOW 0x20
/* OR'ed into the mode of mlct_estimate_batch: after one launch for the first
 * step, run every later step of every probe block in one persistent launch
 * (per row-length class of the operators), with a barrier per probe block
 * between its steps, instead of one launch per step.  Same results bit for
 * bit.  EDEVICE if a barrier wait exceeds two seconds (the launch then ends
 * early; it cannot hang). */
#define MLCT_BATCH_PERSISTENT 0x40
/* OR'ed into the mode of mlct_estimate_batch: one launch per step.  With
 * neither flag the context's choice is used: one launch per step unless
 * mlct_autotune_batch found the persistent launch faster. */
#define MLCT_BATCH_LOCKSTEP 0x80

typedef enum {
  MLCT_DT_F32 = 0,
  MLCT_DT_F64 = 1,
  MLCT_DT_PATTERN = 2  /* CSR without values: every stored entry is 1 */
} mlct_dtype;

typedef enum {
  MLCT_PROBE_RADEMACHER = 0, /* counter-based, see mlct_probes              */
  MLCT_PROBE_EXPLICIT = 1    /* caller's int8 entries (e.g. Hadamard, e_i)  */
} mlct_probe_kind;

/* A set of m probe vectors z^(0..m-1) of length d.
 * RADEMACHER: z^(p) is probe id (first_id + p) of generator ``seed``:
 *   key = SplitMix64 output number id of a stream started at seed,
 *   word_c = SplitMix64 output number c of a stream started at key,
 *   z_i = +1 if bit (i mod 64) of word_{i/64} is 0, else -1
 *   (SplitMix64: Steele, Lea & Flood, OOPSLA 2014).
 * EXPLICIT: entries_dev is a device int8 array, row-major d x ld_entries;
 *   z^(p)_i = entries_dev[i * ld_entries + first_id + p]. */
typedef struct {
  int32_t kind;
  uint64_t seed;
  int64_t first_id;
  int64_t m;
  const int8_t* entries_dev;
  int64_t ld_entries;
} mlct_probes;

#define MLCT_MAX_LEVELS 32

/* Levels 0 <= degree[0] < ... < degree[L-1] = n and samples per level
 * (Section 3, eq. eqn:decomposition; Section 4, eq. eqn:multiEstimator). */
typedef struct {
  int32_t L;
  const int32_t* degree;  /* host, L entries */
  const int64_t* m;       /* host, L entries, each >= 1 */
} mlct_levels;

/* Result of an estimate.  value = Gamma (eq. eqn:multiEstimator);
 * estimate = value * exp(log_scale) (log_scale != 0 only for MLCT_EXP,
 * where exp((a+b)/2) is factored out of the coefficients). */
typedef struct {
  double estimate;
  double value;
  double log_scale;
  double est_var;                     /* sum_k s_k^2 / m_k, units of value */
  double level_mean[MLCT_MAX_LEVELS]; /* mean of Q_{l_{k-1} l_k}          */
  double level_var[MLCT_MAX_LEVELS];  /* unbiased sample variance s_k^2   */
  int64_t matvecs;                    /* probe-matvecs applied            */
  int64_t probe_degrees;              /* sum_k m_k * l_k                  */
  double max_moment_ratio;            /* max_j |mu_j| / mu_0 over probes  */
  double interval_a, interval_b;      /* the [a, b] the estimate used     */
  uint32_t flags;                     /* MLCT_FLAG_* bits                 */
} mlct_result;

#define MLCT_FLAG_FEW_SAMPLES 0x1u /* some m_k < 2: its variance is NaN    */
#define MLCT_FLAG_OVERFLOW 0x2u    /* estimate not finite (see log_scale)  */
#define MLCT_FLAG_BF16 0x4u        /* BF16X3 arithmetic was used           */

typedef struct mlct_ctx mlct_ctx;
typedef struct mlct_op mlct_op;

/* ---- context ------------------------------------------------------------ */

/* Create a context bound to HIP device ``device`` and stream ``hip_stream``
 * (a hipStream_t; NULL = the null stream).  tune_cache_path may be NULL. */
mlct_status mlct_create(int device, void* hip_stream, const char* tune_cache_path,
                        mlct_ctx** out);
mlct_status mlct_destroy(mlct_ctx* ctx);
/* Text of the last error on this context ("" if none).  Owned by ctx. */
const char* mlct_last_error(const mlct_ctx* ctx);
/* Cap on the context's device workspace in bytes (0 = no cap).  A call that
 * would exceed it fails with MLCT_ENOMEM before enqueuing any work. */
mlct_status mlct_set_workspace_limit(mlct_ctx* ctx, uint64_t bytes);

/* Context options.  MLCT_OPT_TWO_STEP (default 0): 1 runs two recurrence steps
 * per launch where the operator allows it (CSR, FP32, at most 5 entries per
 * row, no column farther from its row than 1/16 of the rows, Rademacher
 * probes, and a device whose eight XCDs all receive workgroups of a launch,
 * probed once per context); 0 runs one step per launch.  On the MI355X the
 * two-step launch is measured slower than two single steps (its second
 * step finds too little of the first step's output still in L2), so it is
 * off by default.  The probe vectors
 * are the same bit for bit either way, and so are the moments where one
 * step's workgroups take at most 512 rows each (up to 1,048,576 rows); on
 * larger operators the moments' FP64 sums are taken per 512-row tile
 * instead of per workgroup band, which moves them by rounding only (about
 * 1e-13 of |z|^2).  A two-step call whose
 * launch left an XCD's rows unprocessed fails with MLCT_EDEVICE.  Errors:
 * EINVAL (unknown option or value). */
#define MLCT_OPT_TWO_STEP 1
/* MLCT_OPT_WAIT_LIMIT_US (default 2,000,000): the longest a two-step launch
 * waits for a neighbouring tile before it gives up; a call whose launch gave
 * up fails with MLCT_EDEVICE (its outputs are then unspecified) and the
 * context stays usable.  0..60,000,000. */
#define MLCT_OPT_WAIT_LIMIT_US 2
/* Tuning knobs of the two-step launch with no effect on the vectors (0 = the
 * library's choice): MLCT_OPT_TWO_STEP_LAG, how many tiles the first step
 * runs ahead of the second beyond twice the operator's bandwidth (default
 * 64, 0..4096); MLCT_OPT_TWO_STEP_ROWS, rows per tile (default: the
 * single-step bands up to 512 rows, else 512; a multiple of 8 up to 8192;
 * sets the moments' summation order); MLCT_OPT_TWO_STEP_WGS, workgroups
 * per XCD (default 64, up to 512). */
#define MLCT_OPT_TWO_STEP_LAG 3
#define MLCT_OPT_TWO_STEP_ROWS 4
#define MLCT_OPT_TWO_STEP_WGS 5
/* MLCT_OPT_BATCH_SOLO_ROWS: the operator size (rows) from which an item of
 * mlct_estimate_batch runs as a single estimate instead of sharing launches
 * (0 = the default, 131,072); results are the same either way. */
#define MLCT_OPT_BATCH_SOLO_ROWS 6
mlct_status mlct_set_option(mlct_ctx* ctx, int32_t option, int64_t value);

/* Per-kernel device time of the library's own launches, measured with HIP
 * events recorded on the context stream around every launch of the kernel
 * families below while timing is enabled (used for roofline figures).
 * mlct_timing(ctx, 1) resets the counters and starts timing; (ctx, 0) stops.
 * mlct_timing_read returns the launches and summed milliseconds collected by
 * calls that completed since timing was enabled. */
typedef enum {
  MLCT_KERNEL_CSR_STEP = 0,   /* one recurrence step over a CSR operator   */
  MLCT_KERNEL_DENSE_STEP = 1, /* one recurrence step over a dense operator */
  MLCT_KERNEL_TRI_STEP = 2,   /* one integer triangle-moment SpMM          */
  MLCT_KERNEL_GRAM = 3,       /* Gram matrix formation                     */
  MLCT_KERNEL_BATCH_STEP = 4, /* one batched recurrence step (all blocks)  */
  MLCT_KERNEL_GRAM_CSR_STEP = 5, /* one step over X^T X + lambda I, X CSR:
                                    W = X V_k, then the recurrence over X^T W */
  MLCT_KERNEL_SLQ_SPMM = 6,   /* Lanczos product u = A w_j with the alpha dots */
  MLCT_KERNEL_SLQ_UPDATE = 7, /* Lanczos three-term update with the beta dots  */
  MLCT_KERNEL_CALLBACK_STEP = 8, /* recurrence update after a callback product */
  MLCT_KERNEL_CSR_STEP2 = 9,  /* two CSR recurrence steps in one launch; its
                                 count is of steps (two per launch, one for a
                                 trailing single step)                       */
  MLCT_NUM_KERNEL_IDS = 10
} mlct_kernel_id;
mlct_status mlct_timing(mlct_ctx* ctx, int32_t enable);
mlct_status mlct_timing_read(const mlct_ctx* ctx, int32_t kernel, int64_t* launches,
                             double* total_ms);

/* ---- operators (the only access to A, Section 2.1) ---------------------- */

/* Operators keep a pointer to their context: destroy every operator before
 * the context it was created on. */

/* Symmetric sparse A in CSR form: rowptr[d+1] and col[nnz] int32 (device),
 * values float32 (MLCT_DT_F32) or absent (val_dev = NULL, MLCT_DT_PATTERN).
 * Columns within a row need not be sorted; duplicates are summed.  The
 * structure is validated on the device at creation: rowptr[0] = 0,
 * non-decreasing, rowptr[d] = nnz, 0 <= col < d; violations give EINVAL. */
mlct_status mlct_op_csr(mlct_ctx* ctx, int64_t d, int64_t nnz, const int32_t* rowptr_dev,
                        const int32_t* col_dev, const void* val_dev, int32_t dtype,
                        mlct_op** out);
/* Symmetric dense A, row-major d x d with leading dimension lda >= d,
 * float64 (MLCT_DT_F64) or float32 (MLCT_DT_F32). */
mlct_status mlct_op_dense(mlct_ctx* ctx, int64_t d, const void* A_dev, int64_t lda,
                          int32_t dtype, mlct_op** out);
/* Sparse Gram operator A = X^T X + lambda I, applied matrix-free as two
 * sparse products per recurrence step (W = X V, then X^T W), for nuclear
 * norms (f = sqrt, lambda = 0) and regularised log-determinants of sparse or
 * rectangular X without forming X^T X (the Gram footnote of Section 1 and
 * the nuclear-norm experiments of Section 5).  X: device CSR, rows x cols
 * (rowptr int32[rows+1], col int32[nnz] in [0, cols), val float32[nnz] or
 * NULL for a 0/1 pattern), borrowed for the operator's lifetime.  X^T is
 * built at creation (a stable counting sort on the host, so every sum over
 * it has a fixed order) and owned.  The operator's dimension is cols;
 * precisions MLCT_FP32 and MLCT_FP64.  a = b = NaN in mlct_estimate finds
 * the interval by Lanczos through the two products.  Not usable with
 * mlct_triangles, mlct_estimate_batch or MLCT_EXACT_LOW (EINVAL /
 * EUNSUPPORTED).  Errors: EINVAL (shape, CSR structure, lambda < 0),
 * ENOMEM. */
mlct_status mlct_op_gram_csr(mlct_ctx* ctx, int64_t rows, int64_t cols, int64_t nnz,
                             const int32_t* rowptr_dev, const int32_t* col_dev,
                             const float* val_dev, double lambda, mlct_op** out);

/* A = X^T X for X row-major rows x cols (leading dimension ldx >= cols),
 * float32.  The Gram matrix (cols x cols) is formed once on the device, in
 * the arithmetic ``prec`` (MLCT_FP32 or MLCT_BF16X3), and owned by the op. */
mlct_status mlct_op_gram(mlct_ctx* ctx, int64_t rows, int64_t cols, const void* X_dev,
                         int64_t ldx, int32_t dtype, int32_t prec, mlct_op** out);
/* Matrix-free symmetric operator: the library touches A only through
 * products with blocks of probe vectors, which is all the estimator needs
 * (Section 2.1: each sample costs matrix-vector products; Section 3.1
 * counts cost in them).  Each recurrence step calls
 *   apply(user, V_dev, AV_dev, B, hip_stream)
 * which must enqueue AV = A V on hip_stream (the context's stream) and
 * return 0; V_dev and AV_dev are device float32 arrays, row-major d x B
 * (probe index fastest, leading dimension B; B = 64, columns past the
 * block's probes are zero), owned by the library and valid for the call
 * only; the function must not read or write outside them.  A non-zero
 * return fails the call with MLCT_EDEVICE.  Precision MLCT_FP32 (FP32
 * vectors, FP64 moment sums); mlct_moments, mlct_estimate (without
 * MLCT_EXACT_LOW), mlct_select_levels, mlct_estimate_auto and the learned
 * level accept it; the interval [a, b] must be given (no Lanczos on FP32
 * products): a = b = NaN, mlct_bounds, mlct_lanczos, mlct_autotune and the
 * CSR-only calls fail with MLCT_EUNSUPPORTED.  The function is called from
 * the thread that makes the library call.  Errors: EINVAL (d < 1, no
 * function). */
typedef int32_t (*mlct_apply_fn)(void* user, const float* V_dev, float* AV_dev, int64_t B,
                                 void* hip_stream);
mlct_status mlct_op_callback(mlct_ctx* ctx, int64_t d, mlct_apply_fn apply, void* user,
                             mlct_op** out);
mlct_status mlct_op_destroy(mlct_op* op);
/* Copy the d x d matrix of a dense or Gram operator to the host as float64,
 * row-major (out_host: d*d doubles).  EINVAL for CSR operators. */
mlct_status mlct_op_read_dense(mlct_ctx* ctx, const mlct_op* op, double* out_host);

/* ---- building blocks ---------------------------------------------------- */

/* Chebyshev coefficients c_0..c_n of f mapped from [a, b] to [-1, 1]: the
 * interpolant at x_k = cos(k pi / n) (Section 2.2), by a type-I DCT in FP64
 * on the device.  c_out: host, n+1 doubles.  log_scale_out (may be NULL):
 * (a+b)/2 for MLCT_EXP (coefficients are those of exp((b-a)/2 x)), else 0. */
mlct_status mlct_cheb_coeffs(mlct_ctx* ctx, mlct_func f, double a, double b, int32_t n,
                             double* c_out, double* log_scale_out);

/* Moments mu[p][j] = z^(p)T T_j(A_hat) z^(p), j = 0..n, p = 0..m-1, with
 * A_hat = 2/(b-a) A - (a+b)/(b-a) I (Section 2.2).  mu_out: host, m x (n+1)
 * row-major doubles.  mode: MLCT_DIRECT or MLCT_DOUBLING. */
mlct_status mlct_moments(mlct_ctx* ctx, const mlct_op* op, double a, double b, int32_t n,
                         const mlct_probes* probes, int32_t prec, int32_t mode,
                         double* mu_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * moments of mlct_moments, written to DEVICE memory and without allocating
 * anything.  CSR operators, MLCT_FP32 or MLCT_FP64, MLCT_DIRECT or
 * MLCT_DOUBLING; the same kernels as mlct_moments, so the results are the
 * same bit for bit.  mu_dev: device, m x (n+1) doubles, row-major, written
 * on the context stream; the call returns once the work is enqueued (no
 * synchronisation, no host copy).
 * Scratch: a fixed device array of MLCT_NOALLOC_SCRATCH_BYTES inside the
 * library, one per GPU, held until the process ends.  A request needs
 * 2 d 64 s bytes (two probe vectors, s = 4 or 8) + 1024 G (S + 1) (moment
 * partials; G workgroups per step, up to 2048; S steps) + 1024 (S + 1) + 64 s
 * per 256-entry chunk of the rows longer than 256 entries, each part rounded
 * up to 256; more than the array holds fails with MLCT_ENOMEM before any work
 * (about d <= 65,536 rows in FP32 at degree 200, symmetric form).  Every
 * buffer is written
 * before it is read, so nothing needs clearing between calls.  All calls on
 * one GPU share that GPU's array: calls that overlap in time on one GPU
 * (other streams, contexts or threads) race and give wrong results.
 * Errors: EINVAL, EUNSUPPORTED (not CSR, BF16X3), ENOMEM (scratch too
 * small), EDEVICE. */
#define MLCT_NOALLOC_SCRATCH_BYTES (64ull << 20)
mlct_status mlct_moments_noalloc(mlct_ctx* ctx, const mlct_op* op, double a, double b,
                                 int32_t n, const mlct_probes* probes, int32_t prec,
                                 int32_t mode, double* mu_dev);

/* Spectral interval by ``steps`` FP64 Lanczos steps with full
 * reorthogonalisation from Rademacher probe 0 of ``seed``: extreme Ritz values
 * widened by their residual bounds and by rel_margin * (width). */
mlct_status mlct_bounds(mlct_ctx* ctx, const mlct_op* op, int32_t steps, uint64_t seed,
                        double rel_margin, double* a_out, double* b_out);
/* The Lanczos tridiagonal behind mlct_bounds: alpha_out[0..k-1],
 * beta_out[0..k-1] (beta_out[k-1] = residual norm after the last step), the
 * number of steps k actually taken (fewer than ``steps`` after a breakdown),
 * and info_out[0..5] = theta_min, theta_max, r_min, r_max, a, b.  Any output
 * pointer may be NULL.  1 <= steps <= 128. */
mlct_status mlct_lanczos(mlct_ctx* ctx, const mlct_op* op, int32_t steps, uint64_t seed,
                         double rel_margin, double* alpha_out, double* beta_out,
                         int32_t* k_out, double* info_out);

/* ---- estimators ---------------------------------------------------------- */

/* Multilevel estimate of tr f(A) (Section 4, eq. eqn:multiEstimator).  Level
 * k uses Rademacher probe ids [off_k, off_k + m_k), off_k = sum_{k'<k} m_k',
 * so all samples are independent; Q uses the coefficients of the single
 * degree-n interpolant (eq. def:qlevels) unless MLCT_LEVEL_INTERP is set.
 * Returns MLCT_ESPECTRUM if some |mu_j| exceeds |z|^2 (1 + 1e-3).
 * If a and b are both NaN the interval is found first by mlct_bounds with
 * min(64, d) steps, margin 0.01 and seed (seed + 0x9E3779B97F4A7C15).
 * A CSR operator with fewer than 512 workgroups per step (about d < 131072),
 * no row longer than 256 entries, MLCT_FP32 and at least four probe blocks
 * runs as a one-item mlct_estimate_batch (all blocks in shared launches);
 * the result is the same bit for bit. */
mlct_status mlct_estimate(mlct_ctx* ctx, const mlct_op* op, mlct_func f, double a, double b,
                          const mlct_levels* levels, uint64_t seed, int32_t prec,
                          int32_t mode, mlct_result* out);

/* Stochastic Lanczos quadrature (the Lanczos-based alternative to
 * Chebyshev interpolation of the paper's introduction).  Per probe z, k
 * Lanczos steps from z/|z| (FP64, no reorthogonalisation; a probe whose
 * Krylov space is exhausted, |w_{j+1}| <= 1e-12 max|a_i|, stops early)
 * give the Jacobi matrix T_j, and Gauss quadrature gives
 * q = |z|^2 sum_i S_{1i}^2 f(theta_i) with T_j = S diag(theta) S^T (exact
 * for polynomials of degree <= 2j - 1).  CSR operators; 1 <= k <= 256;
 * probes in blocks of 64.  q_out: host, probes->m values.  EUNSUPPORTED for
 * dense or Gram operators. */
mlct_status mlct_slq_quadforms(mlct_ctx* ctx, const mlct_op* op, mlct_func f, int32_t k,
                               const mlct_probes* probes, double* q_out);

/* Two-level estimator with a Lanczos-quadrature fine level (Sections 2.3
 * and 4 with SLQ as the level-n approximator): level 0 = z^T p_l(A_hat) z
 * with the degree-l interpolant (l = cheb_degree, arithmetic prec / mode as
 * in mlct_estimate) on probe ids [0, m0); level 1 = q_SLQ,k - z^T p_l z on
 * ids [m0, m0 + m1).  Unbiased for E[q_SLQ,k].  out->level_mean/var hold the
 * two levels; matvecs counts both parts; a = b = NaN uses mlct_bounds. */
mlct_status mlct_estimate_slq(mlct_ctx* ctx, const mlct_op* op, mlct_func f, double a,
                              double b, int32_t cheb_degree, int64_t m0, int32_t k, int64_t m1,
                              uint64_t seed, int32_t prec, int32_t mode, mlct_result* out);

/* Automatic level selection (Section 3.2, Theorem thm:levels).
 *
 * From a pilot table of per-probe terms t_j = c_j z^T T_j(A_hat) z
 * (j = 0..n), the variance V_{l'l} of each level variable Q_{l'l}
 * (eq. def:qlevels) is the pilot sample variance of sum_{j=l'+1}^{l} t_j; a
 * sample of Q_{l'l} costs C(l) = l matvecs (MLCT_DIRECT) or ceil(l/2)
 * (MLCT_DOUBLING), Section 3.1.  The levels minimise
 * sum_k sqrt(V_{l_{k-1} l_k} C(l_k)) by the dynamic programme of Theorem
 * thm:levels (eq. eqn:costrecurrence), with the top level n chosen under the
 * condition of Section 3.2 that the allocation of eqs. eqn:optSamples /
 * eqn:optMu recommends at least min_top samples for it.  Ties go to the
 * smaller second-highest level; with no admissible choice the single level
 * {n} is returned.  The j = 0 term belongs to the first level (its variance
 * is zero for Rademacher probes).  Sample sizes are rounded up, at least 2.
 * A plan holds at most MLCT_MAX_LEVELS levels: when the optimum has more
 * (noisy pilots of slowly converging expansions can ask for dozens of
 * levels that each save little), the plan is the optimum over plans of at
 * most MLCT_MAX_LEVELS levels, by the same recurrence indexed by the number
 * of levels (its cost opt_total is then at least the unconstrained one).
 *
 * target_kind MLCT_TARGET_VARIANCE: target = eps^2, a variance of
 * mlct_result.value (the estimate without its exp log_scale factor);
 * MLCT_TARGET_BUDGET: target = total matvecs sum_k m_k C(l_k). */
#define MLCT_TARGET_VARIANCE 0
#define MLCT_TARGET_BUDGET 1
#define MLCT_MAX_PLAN_DEGREE 1024

typedef struct {
  int32_t L;                          /* levels chosen                     */
  int32_t degree[MLCT_MAX_LEVELS];    /* l_1 < ... < l_L = n               */
  int64_t m[MLCT_MAX_LEVELS];         /* recommended samples per level     */
  double var[MLCT_MAX_LEVELS];        /* pilot V_{l_{k-1} l_k}             */
  double cost[MLCT_MAX_LEVELS];       /* C(l_k), matvecs per sample        */
  double m_real[MLCT_MAX_LEVELS];     /* allocation before rounding        */
  double opt_total;                   /* sum_k sqrt(V_k C_k) of the plan   */
  double single_total;                /* sqrt(V_{0n} C(n)): single level   */
  double predicted_var;               /* sum_k var_k / m_k                 */
  double predicted_cost;              /* sum_k m_k cost_k                  */
} mlct_level_plan;

/* Plan from a given pilot term table.  terms: host, m_pilot x (n+1) FP64
 * row-major; 1 <= n <= MLCT_MAX_PLAN_DEGREE; m_pilot >= 2; target > 0;
 * mode MLCT_DIRECT or MLCT_DOUBLING (sets C(l)).  Errors: EINVAL for
 * arguments. */
mlct_status mlct_plan_levels(mlct_ctx* ctx, const double* terms, int64_t m_pilot, int32_t n,
                             int32_t mode, double target, int32_t target_kind,
                             int64_t min_top, mlct_level_plan* out);

/* Pilot and plan: m_pilot Rademacher probes (ids 0 .. m_pilot-1 of seed) at
 * degree n in arithmetic prec and form mode, then mlct_plan_levels with
 * min_top = m_pilot.  Use another seed for the estimate itself so that its
 * probes are independent of the pilot's.  a = b = NaN: the interval from
 * mlct_bounds as in mlct_estimate.  mu_out (host, may be NULL): the pilot
 * moments, m_pilot x (n+1). */
mlct_status mlct_select_levels(mlct_ctx* ctx, const mlct_op* op, mlct_func f, double a,
                               double b, int32_t n, int64_t m_pilot, uint64_t seed,
                               int32_t prec, int32_t mode, double target, int32_t target_kind,
                               mlct_level_plan* out, double* mu_out);

/* Pilot, automatic levels and the estimate in one call (Section 3.2: the
 * pilot samples are reused).  The pilot's m_pilot probes (ids 0 ..
 * m_pilot-1 of seed, degree n) are the first samples of the top level,
 * which is what the plan's condition (at least m_pilot samples at the top)
 * pays for; the top level takes max(m_L, m_pilot) samples, its remaining
 * probes and every lower level use fresh ids of the same seed, disjoint
 * across levels.  out->matvecs counts the pilot.  plan_out (may be NULL):
 * the plan, with the top level's m as used.  Other arguments and errors as
 * in mlct_select_levels and mlct_estimate. */
mlct_status mlct_estimate_auto(mlct_ctx* ctx, const mlct_op* op, mlct_func f, double a,
                               double b, int32_t n, int64_t m_pilot, uint64_t seed,
                               int32_t prec, int32_t mode, double target, int32_t target_kind,
                               mlct_level_plan* plan_out, mlct_result* out);

/* Autotuner: times the candidate launch shapes of the recurrence for this
 * operator on the device and keeps the fastest in the operator (CSR: the cap
 * on workgroups per step, 512 / 1024 / 2048 / 4096, FP32, 64 probes;
 * dense: 32 x 32, 64 x 64 or 128 x 128 square tiles or the skinny split-K
 * kernel (64 or 32 probes x 16 rows per workgroup) in arithmetic ``prec`` at
 * block width B_max; kept as 0, 2, 1 or 3).  Without tuning, blocks of at
 * most 64 probes take the skinny kernel and wider ones the largest square
 * tile that still fills the device.  With a cache file given to mlct_create the decision is written
 * there, keyed by the operator's shape (dense: and by precision and block
 * width); CSR operators of the same shape pick it up when they are created,
 * dense operators whenever a block of that precision and width runs.
 * Values in the file that the autotuner could not have chosen are ignored.
 * choice_out (may be NULL): the value kept. */
mlct_status mlct_autotune(mlct_ctx* ctx, mlct_op* op, int32_t B_max, int32_t prec,
                          int32_t* choice_out);

/* Many estimates in shared launches: every (item, level, block of 64
 * probes) of all items advances one recurrence step per launch, so the
 * number of launches is the largest step count, not the sum over items.
 * Items must use square CSR operators (valued or pattern, any sizes; not
 * sparse Gram operators); precision MLCT_FP32; mode MLCT_DIRECT or
 * MLCT_DOUBLING (optionally with MLCT_LEVEL_INTERP and / or MLCT_EXACT_LOW).
 * Items whose operator has 131,072 rows or more (MLCT_OPT_BATCH_SOLO_ROWS)
 * fill the device on their own and run as single estimates (then any size
 * is accepted); the others share launches.  Each item's result equals what mlct_estimate returns
 * for it, bit for bit (rows longer than 256 entries are summed in the same
 * 256-entry chunks).  outs: host, nitems results.  Fails with
 * MLCT_ESPECTRUM if any item's moments leave [-|z|^2, |z|^2] (every item's
 * result is still written). */
typedef struct {
  const mlct_op* op;
  mlct_func f;
  double a, b;
  mlct_levels levels;
  uint64_t seed;
} mlct_batch_item;

mlct_status mlct_estimate_batch(mlct_ctx* ctx, int32_t nitems, const mlct_batch_item* items,
                                int32_t prec, int32_t mode, mlct_result* outs);

/* Autotuner for batches: runs this batch (three times each, the first as a
 * warm-up) with one launch per step and with the persistent launch, timed
 * with events on the context stream, and keeps the faster as the context's
 * launch form for batches given neither MLCT_BATCH_PERSISTENT nor
 * MLCT_BATCH_LOCKSTEP.  choice_out (may be NULL): 1 = persistent, 0 = one
 * launch per step.  Arguments as mlct_estimate_batch. */
mlct_status mlct_autotune_batch(mlct_ctx* ctx, int32_t nitems, const mlct_batch_item* items,
                                int32_t prec, int32_t mode, int32_t* choice_out);

/* Triangle count tr(A^3)/6 of a 0/1 pattern CSR graph (Section 2.1 example,
 * Section 5.4): per probe, exact integer y = A z and w = A y with int64
 * w1 = z.y, w2 = y.y, w3 = y.w.  w_out (host, m x 3 int64, may be NULL).
 * z is held as one sign word per row and y as int16 with exact escapes
 * (results exact for every graph); at most 536,870,911 rows, else
 * MLCT_EUNSUPPORTED. */
typedef struct {
  int64_t sum_w3;
  double estimate;     /* sum w3 / (6 m) */
  double estimate_cv;  /* control-variate estimate (Section 5.4)           */
  double a1, a2;       /* regression coefficients of w3 on (w1, w2)        */
} mlct_tri_result;

mlct_status mlct_triangles(mlct_ctx* ctx, const mlct_op* op, int64_t m, uint64_t seed,
                           int64_t* w_out, mlct_tri_result* out);

/* ---- learned control-variate level (not in the paper) -------------------
 * g predicts a probe's fine-level value q = z^T p_{n_fine}(A_hat) z from its
 * cheap moments: the truncation q_c = sum_{j <= n_cheap} c_j mu_j plus a
 * correction of the standardised residual (q - q_c)/mu_0 in two stages, a
 * linear least-squares fit on the standardised inputs u_f (mu_f / mu_0 for
 * f = 1..n_cheap, centred and scaled over the training probes; the linear
 * control variate of Section 5.4) and a small MLP (F = n_cheap + 1 inputs,
 * two hidden tanh layers of 64 units, one output) trained on what the linear
 * fit leaves:  g = q_c + mu_0 (ybar + ysd (beta . u + net(u))).  It is
 * trained on pilot probes, then used as one more multilevel term (Section 2.3, eq.
 * eqn:telescope; the control-variate form of Section 5.4):
 *   Gamma = (1/M0) sum_{S0} g + (1/M1) sum_{S1} (q - g),
 * S0 at degree n_cheap, S1 at degree n_fine, probe sets disjoint from each
 * other and from the pilot, so Gamma is unbiased for tr p_{n_fine}(A_hat)
 * whatever g is.  Training is FP32 (Adam, full batch), inference BF16 (bf16
 * weights, inputs and hidden activations; FP32 accumulation), the same
 * function for both terms.  If on the held-out pilot probes var(q - g) is not
 * below var(q), the level falls back to the plain estimator. */
typedef struct mlct_mlp mlct_mlp;

typedef struct {
  int32_t epochs;         /* full-batch Adam steps (default 2000)            */
  float lr;               /* Adam learning rate (default 1e-3)               */
  double train_fraction;  /* pilot probes used for training (default 0.75)   */
  uint64_t init_seed;     /* weight initialisation stream (default seed^const) */
} mlct_mlp_cfg;

typedef struct {
  double var_q;       /* variance of q on the held-out pilot probes        */
  double var_resid;   /* variance of q - g on the same probes              */
  double mean_resid;  /* mean of q - g on the same probes                  */
  double var_g;       /* variance of g on the same probes                  */
  double ybar, ysd;   /* target standardisation (of q / mu_0)              */
  double final_loss;  /* training loss (standardised units) after training */
  int32_t fallback;   /* 1 if the learned level is not used                */
  int32_t n_features, n_cheap, n_fine;
  int64_t ntrain, nval, nparams;
  double x_mean[16];  /* input standardisation: u_f = (mu_f/mu_0 - x_mean_f) */
  double x_sd[16];    /*   / x_sd_f (0 for f = 0 and constant inputs)       */
  double lin[16];     /* linear stage beta_f (beta_0 = 0)                   */
} mlct_mlp_info;

#define MLCT_FLAG_LEARNED_FALLBACK 0x8u /* learned level disabled: plain used */

/* Pilot: Rademacher probes [0, m_pilot) of ``seed`` at degree n_fine
 * (symmetric moment form, arithmetic ``prec``), then training.  [a, b] as in
 * mlct_estimate (NaN, NaN = Lanczos).  1 <= n_cheap <= 15, n_cheap < n_fine,
 * m_pilot >= 8.  The first max(2, train_fraction * m_pilot) probes train the
 * network; the rest are held out (their moments are kept in the handle for
 * mlct_learned_plan) and there must be at least 2 of them, else EINVAL.
 * cfg may be NULL (defaults). */
mlct_status mlct_learned_fit(mlct_ctx* ctx, const mlct_op* op, mlct_func f, double a, double b,
                             int32_t n_fine, int32_t n_cheap, int64_t m_pilot, uint64_t seed,
                             int32_t prec, const mlct_mlp_cfg* cfg, mlct_mlp** out);
/* Estimate with the learned level: S0 = probe ids [0, M0), S1 = ids
 * [M0, M0 + M1) of ``seed`` (seed must differ from the fit seed).  In the
 * result, level_mean/var[0] describe g over S0 and [1] describe q - g over
 * S1 (plain fallback: [1] = q over S1, M0 unused).  max_moment_ratio covers
 * both sets; above 1 + 1e-3 the call fails with MLCT_ESPECTRUM, as
 * mlct_estimate does. */
mlct_status mlct_estimate_learned(mlct_ctx* ctx, const mlct_op* op, const mlct_mlp* mlp,
                                  int64_t M0, int64_t M1, uint64_t seed, mlct_result* out);

/* Per-probe values of the learned level on the given probes (arithmetic
 * and form of the fit): fine = 0 runs the recurrence to n_cheap and returns
 * g; fine = 1 runs it to n_fine and returns g (from the same probes' cheap
 * moments) and q = z^T p_{n_fine}(A_hat) z in q_out.  g_out: host,
 * probes->m doubles; q_out: host, probes->m doubles, or NULL (required
 * NULL when fine = 0).  The network is used whatever the fallback flag says.
 * Errors: EINVAL (arguments), ESPECTRUM as mlct_estimate. */
mlct_status mlct_learned_eval(mlct_ctx* ctx, const mlct_op* op, const mlct_mlp* mlp,
                              const mlct_probes* probes, int32_t fine, double* g_out,
                              double* q_out);

/* The learned level inside the multilevel estimator (Section 2.3, eq.
 * eqn:telescope; Section 4, eq. eqn:multiEstimator).  With
 * S(l) = z^T p^{(l)} z the truncation of the degree-n_fine interpolant to
 * degree l (eq. def:qlevels), except S(n_cheap) = g, and S(-1) = 0, level k
 * of levels {l_1 < ... < l_L = n_fine} is Q_k = S(l_k) - S(l_{k-1}) on its
 * own m_k probes (ids [off_k, off_k + m_k) of ``seed``, off_k the sum of the
 * earlier m).  The levels telescope to S(n_fine) = z^T p_{n_fine} z, so the
 * estimate is unbiased for tr p_{n_fine}(A_hat) whichever levels are used:
 * {n_cheap, n_fine} is mlct_estimate_learned's two-term estimator, any set
 * without n_cheap is the plain multilevel estimator, and a set with n_cheap
 * puts g in the chain with the Chebyshev levels above it (or below it).  A
 * sample of level k costs ceil(l_k / 2) matvecs.  The network is used
 * whatever the fallback flag says.  Result as mlct_estimate (level_mean/var
 * per level, max_moment_ratio, ESPECTRUM). */
mlct_status mlct_estimate_learned_ml(mlct_ctx* ctx, const mlct_op* op, const mlct_mlp* mlp,
                                     const mlct_levels* levels, uint64_t seed,
                                     mlct_result* out);

/* Levels and samples for mlct_estimate_learned_ml by the dynamic programme
 * of Theorem thm:levels (as mlct_plan_levels, min_top 0, symmetric-form
 * costs) on the fit's held-out pilot probes, with the per-probe terms
 * chosen so that their prefix sums are the S(l) above: the plan chooses
 * whether g enters the chain and which Chebyshev levels surround it.
 * target / target_kind as in mlct_plan_levels (a variance of the value, or
 * a matvec budget).  Errors: EINVAL (arguments, n_fine > 1024). */
mlct_status mlct_learned_plan(mlct_ctx* ctx, const mlct_mlp* mlp, double target,
                              int32_t target_kind, mlct_level_plan* out);
mlct_status mlct_mlp_info_get(const mlct_mlp* mlp, mlct_mlp_info* out);
/* Training loss after each epoch (standardised units): up to max values. */
mlct_status mlct_mlp_loss_history(const mlct_mlp* mlp, float* out, int32_t max, int32_t* n_out);
/* Read (get_out, nparams floats, may be NULL) and/or replace (set_in, may be
 * NULL) the FP32 weights; layout W1[64][F], b1[64], W2[64][64], b2[64],
 * w3[64], b3.  Replacing also refreshes the BF16 inference weights. */
mlct_status mlct_mlp_weights(mlct_ctx* ctx, mlct_mlp* mlp, float* get_out, const float* set_in);
/* Loss (1/N) sum (g(x_i) - y_i)^2 in standardised units and its gradient
 * (nparams floats) at the current FP32 weights, for host inputs X[N][F], y[N],
 * computed by the training kernels. */
mlct_status mlct_mlp_grad(mlct_ctx* ctx, const mlct_mlp* mlp, const float* X, const float* y,
                          int32_t N, float* grad_out, float* loss_out);
mlct_status mlct_mlp_destroy(mlct_mlp* mlp);

#ifdef __cplusplus
}
#endif
#endif /* MLCT_H */
