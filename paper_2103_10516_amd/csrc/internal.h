// Internal declarations of libmlct: context/operator objects and the
// launchers of the HIP kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mlct.h"

namespace mlct {

// Width of a probe block in the CSR recurrence: one probe per wavefront lane.
constexpr int kBlockProbes = 64;
// CSR rows with more entries than kHubLen are reduced in chunks of at most
// kHubChunk entries by a separate launch before each step.
constexpr int kHubLen = 256;
constexpr int kHubChunk = 256;

// OP_GRAM_CSR: A = X^T X + lambda I with X sparse rows x cols, applied as two
// SpMMs per step (X, then X^T).
// OP_CALLBACK: A applied by the caller's function (mlct_op_callback).
enum OpKind { OP_CSR = 0, OP_DENSE = 1, OP_GRAM = 2, OP_GRAM_CSR = 3, OP_CALLBACK = 4 };

// A CSR matrix as the step kernels see it (device arrays, borrowed or owned
// by the operator), with its hub table (rows longer than kHubLen).
struct CsrMat {
  const int32_t* rowptr = nullptr;
  const int32_t* col = nullptr;
  const float* val = nullptr;  // nullptr = 0/1 pattern
  int64_t nrows = 0, ncols = 0, nnz = 0;
  int max_row_nnz = 0;
  int bandwidth = -1;  // max |column - row|, found for rows of at most 5 entries (-1: unknown)
  int32_t* hub_rows = nullptr;  // [hub_n] sorted
  int32_t* hub_c0 = nullptr;    // [hub_n + 1]
  int32_t* hub_cs = nullptr;    // [hub_chunks] first entry of each chunk
  int32_t* hub_ce = nullptr;    // [hub_chunks] one past its last entry
  int hub_n = 0, hub_chunks = 0;
  // Row bands of equal work for matrices with very uneven rows (owned by the
  // operator): band[g] .. band[g + 1] - 1 are workgroup g's rows when a step
  // runs band_groups workgroups.
  const int32_t* band = nullptr;
  int band_groups = 0;
};
// Per-row cost of a band, in units of one entry's gather: the row pointer,
// the own-row read and the result write.
constexpr int kBandRowCost = 2;
// Rows uneven enough for equal-work bands: the longest row exceeds four times
// the mean plus eight.  Bands are used from kBandMinGroups workgroups per step
// on: below that a step's workgroups are short-lived and the extra dependent
// load of the band bounds costs more than the balance gains.
inline bool csr_uneven(const CsrMat& m) {
  return m.nrows > 0 && m.max_row_nnz > 4 * (m.nnz / m.nrows) + 8;
}
constexpr int kBandMinGroups = 0;

struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// The affine parts of the learned level (k_mlp.hip): target standardisation,
// input standardisation and the linear least-squares stage.
constexpr int kMlpStats = 2 + 3 * 16;  // doubles written by the training-set kernel
struct MlpAffine {
  double ybar = 0.0, ysd = 1.0;
  double xmean[16] = {}, xsd[16] = {}, lin[16] = {};
};

}  // namespace mlct

struct mlct_timed_launch {
  hipEvent_t start, stop;
  int kernel;
  int units;  // recurrence steps the launch ran (1, or 2 for a two-step launch)
};

// Rows from which a batch item runs as a single estimate (mlct_estimate_batch).
constexpr int64_t kBatchSoloRowsDefault = (int64_t)1 << 17;

struct mlct_ctx {
  int device = 0;
  // per-kernel timing (mlct_timing)
  bool timing = false;
  std::vector<hipEvent_t> event_pool;
  std::vector<mlct_timed_launch> pending;
  double kernel_ms[MLCT_NUM_KERNEL_IDS] = {};
  int64_t kernel_launches[MLCT_NUM_KERNEL_IDS] = {};
  hipStream_t stream = nullptr;
  std::string err;
  uint64_t ws_limit = 0;  // 0 = unlimited
  uint64_t ws_total = 0;  // bytes currently held in workspace slots
  std::vector<mlct::DevBuf> slots;  // grow-only named workspace slots
  void* host_pinned = nullptr;      // staging for small D2H results
  size_t host_pinned_bytes = 0;
  std::string tune_path;            // autotune cache file ("" = none)
  std::vector<std::string> tune_lines;  // cached decisions, one per operator shape
  int batch_persistent = 0;  // launch form of batches without an explicit flag (autotuned)
  int two_step = 0;          // two recurrence steps per launch where the operator allows (opt-in)
  int two_step_lag = 0;      // tiles sub-step 1 runs ahead beyond twice the window (0: default)
  int two_step_rows = 0;     // rows per tile of a two-step launch (0: default)
  int two_step_wgs = 0;      // workgroups per XCD of a two-step launch (0: default)
  int64_t batch_solo_rows = kBatchSoloRowsDefault;  // batch items this large run as single estimates
  int xcd_ok = -1;           // every XCD receives workgroups of a two-step launch (-1: not probed)
  int64_t wait_limit_us = 2000000;  // bound on a two-step launch's tile wait
  int* fused_abort = nullptr;  // device flag of the two-step launches since the last check
  bool fused_check = false;    // a two-step launch ran: check the flag at the next sync
};

// An operator refers to its context; destroy operators before the context.
struct mlct_op {
  mlct_ctx* ctx = nullptr;
  int device = 0;
  int kind = mlct::OP_CSR;
  int64_t d = 0;
  // CSR: the matrix (OP_CSR), or X^T (cols x rows) for OP_GRAM_CSR, the pass
  // that carries the recurrence; csrx = X (rows x cols) for OP_GRAM_CSR
  mlct::CsrMat csr, csrx;
  double gram_lambda = 0.0;    // OP_GRAM_CSR: the shift lambda
  void* hub_mem = nullptr;     // hub table of csr (one allocation)
  void* hubx_mem = nullptr;    // hub table of csrx
  void* gram_mem = nullptr;    // OP_GRAM_CSR: the X^T arrays (owned)
  void* band_mem = nullptr;    // equal-work row bands of csr and csrx (owned)
  // tr A and ||A||_F^2 (exact low-degree traces), computed on first use
  bool stats_ready = false;
  double tr_a = 0.0, fro2 = 0.0;
  int tuned_groups = 0;      // CSR: workgroup cap chosen by mlct_autotune (0 = default)
  int tuned_dense = -1;      // dense: 1 = 128x128, 2 = 64x64, 0 = 32x32 tiles, 3 = skinny, -1 = default rule
  // dense / Gram (row-major d x d)
  const void* A = nullptr;
  int64_t lda = 0;
  int dtype = MLCT_DT_F32;
  void* owned = nullptr;      // Gram matrix or other op-owned memory
  void* split_hi = nullptr;   // bf16 hi part of A (lazily built)
  void* split_lo = nullptr;   // bf16 lo part of A
  void* pack_hi = nullptr;    // the split packed for the skinny kernel (lazily built)
  void* pack_lo = nullptr;
  void* a32 = nullptr;        // FP32 copy of an FP64 dense A (lazily built)
  void* a64 = nullptr;        // FP64 copy of an FP32 dense A (lazily built)
  // callback operator: W = A V by the caller's function
  mlct_apply_fn cb_apply = nullptr;
  void* cb_user = nullptr;
};

// A trained learned level (mlct_learned_fit).  Device arrays are owned.
struct mlct_mlp {
  int device = 0;
  int F = 9, n_cheap = 8, n_fine = 256;
  int32_t func_kind = MLCT_LOG;
  double power = 1.0, a = 0.0, b = 1.0, log_scale = 0.0;
  int32_t prec = MLCT_FP32;
  uint64_t seed = 0;
  int64_t m_pilot = 0, ntrain = 0;
  float* theta = nullptr;  // FP32 weights (device)
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  void* wbf16 = nullptr;   // bf16 inference weights (device)
  double* coef = nullptr;  // c_0..c_{n_fine} (device)
  double ybar = 0.0, ysd = 1.0;
  mlct::MlpAffine aff;
  double var_q = 0.0, var_resid = 0.0, mean_resid = 0.0, var_g = 0.0;
  int fallback = 0;
  // moments of the held-out pilot probes, nval x (n_fine + 1) (device, owned)
  double* val_mu = nullptr;
  int64_t nval = 0;
  std::vector<float> loss_hist;
};

namespace mlct {

// Workspace slot indices (each slot grows independently).
enum Slot {
  WS_V0 = 0, WS_V1, WS_PART, WS_MU, WS_COEF, WS_QSTAT, WS_RESULT, WS_MISC,
  WS_TRI, WS_LANCZOS, WS_DENSE, WS_MLP, WS_MU2, WS_BATCH, WS_HUB, WS_PLAN, WS_STATS, WS_GRAMW, WS_SLQ, WS_SLQQ,
  WS_DPACK, WS_CBW, WS_FSYNC, WS_FABORT, WS_TRISIDE, WS_NSLOTS
};

// ---- probe-generation constants (SplitMix64) ------------------------------
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kMul1 = 0xBF58476D1CE4E5B9ull;
constexpr uint64_t kMul2 = 0x94D049BB133111EBull;

// Probe source descriptor passed by value to kernels.
struct ProbeSrc {
  uint64_t seed;
  int64_t first_id;      // id of column 0 of the current block
  const int8_t* entries; // non-null: explicit entries [d][ld]
  int64_t ld;
  int32_t active;        // columns in use in the current block (<= width)
};

// ---- launchers (k_common.hip) --------------------------------------------
hipError_t launch_cheb_dct(hipStream_t s, int kind, double power, double a, double b,
                           int n, double* c_dev, double* log_scale_dev);
hipError_t launch_csr_validate(hipStream_t s, const int32_t* rowptr, const int32_t* col,
                               int64_t nrows, int64_t ncols, int64_t nnz, int32_t* flags_dev);
hipError_t launch_reduce_partials(hipStream_t s, const double* part, int steps, int nslots,
                                  int ngroups, int width, double* dots);
hipError_t launch_assemble_moments(hipStream_t s, const double* dots, int steps, int width,
                                   int active, int mode, int n, double* mu, int64_t ldmu);
// Per level: Q per probe (into q_dev), mean, unbiased variance and the
// largest |mu_j|/mu_0; then the multilevel sum into result_dev.
struct LevelDesc {
  int32_t degree[MLCT_MAX_LEVELS];
  int64_t m[MLCT_MAX_LEVELS];
  int64_t off[MLCT_MAX_LEVELS];
  int32_t L;
  int32_t interp;     // separate interpolant per level
  int32_t coef_stride;
  int32_t jmin = 0;   // first degree in the level variables (3: j <= 2 exact)
  double low_tr[3] = {0.0, 0.0, 0.0};  // tr T_j(A_hat), j <= 2, when jmin = 3
};
// tr A and ||A||_F^2 of an operator (FP64, fixed-order sums) into out[0..1];
// partial: scratch of 2 * kStatsGroups doubles.
constexpr int kStatsGroups = 1024;
hipError_t launch_op_stats(hipStream_t s, const mlct_op* op, double* partial, double* out);
hipError_t launch_level_combine(hipStream_t s, const double* mu, int64_t ldmu,
                                const double* coef, const double* log_scale,
                                const LevelDesc& lv, double* q_dev, double* stats_dev,
                                mlct_result* result_dev);

// ---- CSR recurrence (k_csr.hip) -------------------------------------------
struct CsrStepPlan {
  int ngroups;        // workgroups per step (= partial-sum slots)
  int rows_per_group; // contiguous rows per workgroup (without bands)
  const int32_t* band = nullptr;  // [ngroups + 1] first row of each workgroup, or none
};
// Workgroups per step: one per 256 rows, a multiple of 8 (one band per XCD),
// at most max_groups (0 = the default cap of 2048; the autotuner's choice
// otherwise).
CsrStepPlan plan_csr(int64_t d, int max_groups = 0);
template <typename T>
hipError_t launch_probe_init(hipStream_t s, T* v0, int64_t d, ProbeSrc src,
                             const CsrStepPlan& plan, double* part0);
// One probe block of a batch (FP32, 64 probes) over one CSR operator.
struct BatchBlock {
  const int32_t* rowptr;
  const int32_t* col;
  const float* val;  // nullptr = pattern
  int64_t d, nnz;
  float* v0;
  float* v1;
  double* part;       // [steps + 1][2][ngroups][64]
  ProbeSrc src;
  double alpha, beta;
  int steps, ngroups, rows_per_group;
  const int32_t* band;  // the operator's row bands for ngroups, or nullptr
  int64_t group_base;  // first workgroup of this block in the launch grid
};
hipError_t launch_probe_init_batched(hipStream_t s, const BatchBlock* tab, int nblocks,
                                     int64_t total_groups);
// Placement of a batched step launch on the 8 XCDs (workgroup w runs on XCD
// w mod 8): XCD x takes slots 0 .. slots[x] - 1 (workgroups 8 slot + x),
// which belong to the entries first[x] .. first[x] + count[x] - 1 in that
// order; entry e is bands xg0[e], xg0[e] + 1, ... of block xblk[e], from
// slot xbase[e] on.  An entry is a whole block (its vectors gathered
// through one L2) or, for steps with fewer blocks than XCDs, an eighth of
// one.
struct XcdLaunch {
  int first[8];
  int count[8];
  int64_t slots[8];
};
// zmode 0 or 1 (regenerated probes); step >= 1; maxnz: the longest row of
// the blocks' operators (above 8: the generic loop for long rows); grid =
// 8 x max slots[x]
hipError_t launch_csr_step_batched(hipStream_t s, const BatchBlock* tab, const int32_t* xblk,
                                   const int32_t* xg0, const int64_t* xbase,
                                   const XcdLaunch& xl, int64_t grid, int step, bool pattern,
                                   int maxnz, int zmode);
// Steps 2 .. steps of a batch in one cooperative launch of 8 * per_xcd
// workgroups (per_xcd from csr_batch_persistent_per_xcd: the resident
// count), after step 1 ran as a batched launch; slots_at[s][x] = running
// slots of XCD x at step s (entries as in XcdLaunch, xl.slots unused); cnt:
// nblocks ints of scratch (zeroed here); abort_flag: one int, set if a
// block barrier's wait exceeded spin_ticks of the 100 MHz real-time clock.
// zmode: the moment form after the first step.
hipError_t launch_csr_batch_persistent(hipStream_t s, const BatchBlock* tab,
                                       const int32_t* xblk, const int32_t* xg0,
                                       const int64_t* xbase, const XcdLaunch& xl, int steps,
                                       const int64_t* slots_at, int* cnt, int nblocks,
                                       int* abort_flag, int per_xcd, bool pattern, int maxnz,
                                       int zmode, long long spin_ticks);
// Workgroups per XCD of the persistent kernel that can be resident at once
// on the current device (0 if the query fails).
int csr_batch_persistent_per_xcd(bool pattern, int maxnz, int zmode);
// zmode: 0 = dots with V_k (symmetric form), 1 = regenerated Rademacher z,
// 2 = explicit z entries.  has_prev = false for the first step (no V_prev).
// hub_part: workspace of op->hub_chunks x 64 elements of T (unused without
// hub rows); the step first launches the hub chunk reduction into it.
template <typename T>
hipError_t launch_csr_step(hipStream_t s, const CsrMat& m, const T* vk, T* vm, T ca, T cb,
                           bool has_prev, int zmode, ProbeSrc src, const CsrStepPlan& plan,
                           void* hub_part, double* part);
// Gram operator A = X^T X + lambda I, one step: W = X V_k (rows x 64), then
// V_new = ca X^T W + cb V_k [- V_prev] with the moments (cb includes
// ca * lambda).  plan_rows / plan_cols: bands over X's rows / columns.
template <typename T>
hipError_t launch_gram_csr_step(hipStream_t s, const CsrMat& X, const CsrMat& XT, const T* vk,
                                T* vm, T* W, T ca, T cb, bool has_prev, int zmode, ProbeSrc src,
                                const CsrStepPlan& plan_rows, const CsrStepPlan& plan_cols,
                                void* hubx_part, void* hubt_part, double* part);
// Rows longer than kHubLen as (row, start, end) triples, unordered; count is
// incremented once per such row (entries past cap are not written).
// Equal-work row bands: band[g] = the first row r with
// rowptr[r] + kBandRowCost * r >= g * (nnz + kBandRowCost * d) / ngroups,
// g = 0 .. ngroups (band[0] = 0, band[ngroups] = d).
hipError_t launch_csr_bands(hipStream_t s, const int32_t* rowptr, int64_t d, int ngroups,
                            int32_t* band);
hipError_t launch_hub_find(hipStream_t s, const int32_t* rowptr, int64_t d, int32_t* out,
                           int32_t* count, int cap);

// ---- two recurrence steps per launch (csr_fused2_kernel in k_csr.hip; the
// support kernels in k_fused.hip) ------------------------------------------------
// CSR operators with at most 5 entries per row, FP32, Rademacher probes:
// tiles of rows_per_tile rows (ntiles a multiple of 8), each XCD taking one
// eighth of them in order, sub-step 2 of a tile waiting on sub-step 1 of the
// tiles within `window` of it, issued `lag` (> 2 window) tiles ahead.  The
// vectors are bitwise those of launch_csr_step.  x holds V_{s-1} and
// receives V_{s+1}; y holds V_s and receives V_{s+2} (two = false: sub-step
// 1 only).  zm1 / zm2: moment form of each sub-step (0 symmetric, 1
// direct); part1 / part2: [2][ntiles][64] partials.  sync: 8 + ntiles ints
// (cleared here, after checking the previous launch's counters against
// prev_total when > 0); abort_flag: 1 if a wait exceeded spin_ticks of the
// 100 MHz clock, 2 if an XCD's tiles were left unprocessed.
hipError_t launch_csr_fused2(hipStream_t s, const CsrMat& m, float* x, float* y, float ca1,
                             float cb1, bool prev1, float ca2, float cb2, bool two, int zm1,
                             int zm2, ProbeSrc src, int rows_per_tile, int ntiles, int window,
                             double* part1, double* part2, int* sync, int* abort_flag,
                             int grid, int lag, int prev_total, long long spin_ticks);
// Clears sync[0 .. n-1] after the counter check described above (n = 0:
// the check of a block's last launch only).
hipError_t launch_fused_sync(hipStream_t s, int* sync, int64_t n, int prev_total,
                             int* abort_flag);
// out[w] = XCD of workgroup w of a grid-workgroup launch.
hipError_t launch_xcc_probe(hipStream_t s, int* out, int grid);
hipError_t launch_csr_bandwidth(hipStream_t s, const int32_t* rowptr, const int32_t* col,
                                int64_t d, int32_t* out);
// p[0 .. n-1] = 0 by a kernel (safe inside a captured graph).
hipError_t launch_fill_zero_i32(hipStream_t s, int* p, int64_t n);

// ---- matrix-free operator (k_callback.hip) ----------------------------------
// V_new = ca W + cb V_k (- V_prev) over the d x 64 block, W = A V_k from the
// caller, with the moment partials of the CSR step (zmode as there).
hipError_t launch_callback_step(hipStream_t s, const float* w, const float* vk, float* vm,
                                float ca, float cb, bool has_prev, int zmode, ProbeSrc src,
                                int64_t d, const CsrStepPlan& plan, double* part);

// ---- automatic level selection (k_levels.hip) ------------------------------
constexpr int kMaxPlanDegree = 1024;
struct LevelPlanDev {
  int L;  // number of levels (may exceed MLCT_MAX_LEVELS: then only L is set)
  int degree[MLCT_MAX_LEVELS];
  int64_t m[MLCT_MAX_LEVELS];
  double var[MLCT_MAX_LEVELS], cost[MLCT_MAX_LEVELS], m_real[MLCT_MAX_LEVELS];
  double opt_total, single_total;
};
// mu: pilot moments m x (n+1) (row stride ldmu); coef: c_0..c_n or null (the
// rows are the terms themselves).  Scratch S (m x (n+1)), mean (n+1),
// V ((n+2) x (n+1)), prevk (MLCT_MAX_LEVELS x (n+1) ints).  target: eps^2
// (budget = 0) or a matvec budget.
hipError_t launch_level_plan(hipStream_t s, const double* mu, int64_t ldmu, const double* coef,
                             int n, int64_t m, double* S, double* mean, double* V, int doubling,
                             double target, int budget, int64_t min_top, int* prevk,
                             LevelPlanDev* out);

// ---- stochastic Lanczos quadrature (k_slq.hip, slq_spmm in k_csr.hip) ------
constexpr int kSlqMaxSteps = 256;
// Per-block Lanczos state, lane = probe: the Jacobi matrices and scales.
struct SlqState {
  double alpha[kSlqMaxSteps * 64];        // a_j, j-major
  double beta[(kSlqMaxSteps + 1) * 64];   // b_j (j >= 1 couples j-1 and j)
  double s_cur[64], s_prev[64], b_cur[64], amax[64], znorm2[64];
  int kend[64];                           // diagonal entries kept per probe
};
hipError_t launch_slq_spmm(hipStream_t s, const CsrMat& m, const double* w, double* u,
                           const double* sdev, const CsrStepPlan& plan, void* hub_part,
                           double* part);
hipError_t launch_slq_update(hipStream_t s, double* U, const double* W1, const double* W0,
                             const SlqState* st, int j, int64_t d, const CsrStepPlan& plan,
                             double* part);
hipError_t launch_slq_init(hipStream_t s, const double* z2, int k, SlqState* st);
hipError_t launch_slq_alpha(hipStream_t s, const double* dots, int j, SlqState* st);
hipError_t launch_slq_beta(hipStream_t s, const double* dots, int j, int k, SlqState* st);
hipError_t launch_slq_quadrature(hipStream_t s, const SlqState* st, int kmax, int kind,
                                 double power, double log_scale, int active, double* scratch,
                                 double* out);
hipError_t launch_slq_combine(hipStream_t s, const double* mu, int64_t ldmu, const double* c,
                              int n, int64_t m0, int64_t m1, const double* qslq,
                              double log_scale, mlct_result* out);

// ---- integer triangle moments (k_tri.hip) ----------------------------------
// z of a probe block packed one 64-bit word per row (bit p: probe p is -1).
hipError_t launch_tri_init(hipStream_t s, const mlct_op* op, ProbeSrc src,
                           const CsrStepPlan& plan, uint64_t* zbits);
// Pass 1 gathers zbits and writes y = A z (int16 rows [d][64]; values past
// +-32767 as -32768 with the exact value in side[hub slot][64]); pass 2
// gathers y.  side: [hub_n][64] int32; hub_part: the hub chunk partials.
hipError_t launch_tri_step(hipStream_t s, const CsrMat& m, int pass, const CsrStepPlan& plan,
                           const uint64_t* zbits, int16_t* y, int32_t* side, void* hub_part,
                           long long* part);
hipError_t launch_tri_reduce(hipStream_t s, const long long* part, int ngroups, int active,
                             int pass, long long* w, int64_t p0);
hipError_t launch_tri_cv(hipStream_t s, const long long* w, int64_t m, int64_t nnz,
                         mlct_tri_result* out);

// ---- dense recurrence on MFMA (k_dense.hip) --------------------------------
// Probe blocks of the dense path are probe-major (V^T, bpad x d).
constexpr int64_t kDenseMaxBlock = 4096;
struct DenseStepArgs {
  const void* A0;  // matrix (FP64 / FP32) or its bf16 hi part
  const void* A1;  // bf16 lo part (BF16X3 only)
  int64_t lda, d, bpad;
  const void* vk;
  void* vm;
  double ca, cb;
  bool has_prev;
  int zmode;
  ProbeSrc src;
  double* part;  // [2][ntiles][bpad] for this step
  int tile_force;  // see dense_tile
  // BF16X3 skinny and 128 x 128 blocks: A and V_k packed in the MFMA lane layout
  // (launch_dense_pack_*), V_new packed by the epilogue; null = unpacked
  const void* pk_a_hi = nullptr;
  const void* pk_a_lo = nullptr;
  const void* pk_v_hi = nullptr;
  const void* pk_v_lo = nullptr;
  void* pk_o_hi = nullptr;
  void* pk_o_lo = nullptr;
};
struct DenseTile {
  bool large;
  bool skinny;  // split-K kernel: bm probes x 16 matrix rows per workgroup
  int bm, bn;
};
// force: -1 = default rule, 0 = 32 x 32, 1 = 128 x 128, 2 = 64 x 64 tiles,
// 3 = skinny (each when the block and the row alignment allow it)
DenseTile dense_tile(int prec, int64_t d, int64_t lda, int64_t bpad, int force = -1);
hipError_t launch_dense_step(hipStream_t s, int prec, const DenseStepArgs& a);
hipError_t launch_dense_probe_init(hipStream_t s, int prec, void* v0, int64_t d, int64_t bpad,
                                   ProbeSrc src, double* dots0);
// Packed operands of the skinny BF16X3 kernel: bytes of one part (hi or lo)
// for rows x d, and the packing of A's bf16 split (d x d, row-major) and of
// an FP32 probe block (rows x d, probe-major).
size_t dense_pack_bytes(int64_t rows, int64_t d);
hipError_t launch_dense_pack_a(hipStream_t s, const void* hi, const void* lo, int64_t d,
                               void* out_hi, void* out_lo);
hipError_t launch_dense_pack_v(hipStream_t s, const float* v, int64_t rows, int64_t d,
                               void* out_hi, void* out_lo);
hipError_t launch_dense_split(hipStream_t s, const void* a, int dtype, int64_t d, int64_t lda,
                              void* hi, void* lo);
hipError_t launch_dense_convert(hipStream_t s, const void* a, int src_dtype, int64_t d,
                                int64_t lda, void* out);
hipError_t launch_gram(hipStream_t s, const float* X, int64_t rows, int64_t cols, int64_t ldx,
                       float* G);

// ---- Lanczos spectral interval (k_lanczos.hip) -----------------------------
constexpr int kLanczosMaxSteps = 128;
struct LanczosState {
  double alpha[kLanczosMaxSteps];
  double beta[kLanczosMaxSteps];
  double work[3 * kLanczosMaxSteps];
  int k;        // steps completed
  int stopped;  // breakdown reached
};
// out[0..6] = a, b, theta_min, theta_max, r_min, r_max, k
hipError_t launch_lanczos(hipStream_t s, const mlct_op* op, const void* a64, int64_t lda,
                          int steps, uint64_t seed, double margin, double* Q, double* w,
                          double* h, double* part, LanczosState* st, double* out,
                          double* tmp,        // X-row scratch (OP_GRAM_CSR)
                          double* hub_part);  // chunk sums of long rows (hub_chunks doubles)

// ---- learned control-variate level (k_mlp.hip) -----------------------------
constexpr int kMlpHidden = 64;
constexpr int kMlpMaxFeatures = 16;
constexpr int kMlpWaves = 256;
int mlp_nparams(int F);
hipError_t launch_mlp_init(hipStream_t s, float* theta, float* m, float* v, int F, uint64_t seed);
hipError_t launch_mlp_grad(hipStream_t s, const float* theta, int F, const float* X,
                           const float* y, int N, int nwaves, float* part, float* loss_part);
hipError_t launch_mlp_gradsum(hipStream_t s, const float* part, int nwaves, int F,
                              const float* loss_part, int N, float* grad, float* loss);
hipError_t launch_mlp_adam(hipStream_t s, float* theta, float* m, float* v, const float* part,
                           int nwaves, int F, int t, float lr, const float* loss_part, int N,
                           float* loss_hist);
hipError_t launch_mlp_to_bf16(hipStream_t s, const float* theta, int F, void* w);
hipError_t launch_mlp_infer(hipStream_t s, const void* w, int F, const double* coef,
                            const double* mu, int64_t ldmu, int64_t rows, const MlpAffine& aff,
                            double* g);
hipError_t launch_qvals(hipStream_t s, const double* mu, int64_t ldmu, const double* c, int n,
                        int64_t rows, double* q);
hipError_t launch_mlp_prepare(hipStream_t s, const double* mu, int64_t ldmu, const double* q,
                              const double* coef, int F, int ntrain, float* X, float* y,
                              double* stats);
hipError_t launch_mlp_combine(hipStream_t s, const double* a, int64_t na, const double* b,
                              const double* a2, int64_t nb, double* out);
// Learned multilevel chain (S(l) = truncation to degree l, S(nc) = g,
// S(-1) = 0): q = S(hi) - S(lo) per row; the planner's per-probe terms
// (rows x (n+1), prefix sums = S); max_j |mu_j| / mu_0 over rows into out[0].
hipError_t launch_learned_level_q(hipStream_t s, const double* mu, int64_t ldmu, const double* c,
                                  int hi, int lo, int nc, const double* g, int64_t rows,
                                  double* q);
hipError_t launch_learned_terms(hipStream_t s, const double* mu, int64_t ldmu, const double* c,
                                int n, int nc, const double* g, int64_t rows, double* t);
hipError_t launch_moment_ratio(hipStream_t s, const double* mu, int64_t ldmu, int ncols,
                               int64_t rows, double* out);

}  // namespace mlct
