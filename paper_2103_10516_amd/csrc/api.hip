// Host side of libmlct: argument validation, workspace, planning and the
// C-ABI entry points declared in include/mlct.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <algorithm>
#include <array>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"

using namespace mlct;

// Fixed scratch of mlct_moments_noalloc: one array per GPU in the library's
// code object, held until the process ends.  Host code never names it in a
// launch or copy: it uses the device address hipGetSymbolAddress returns
// for each GPU, taken once per device by mlct_create (noalloc_scratch).
static __device__ __align__(256) unsigned char scratch[MLCT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// The address of this device's scratch array (device current), looked up on
// the first call for the device; nullptr if the lookup fails.
void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

mlct_status fail(mlct_ctx* ctx, mlct_status st, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

#define HIPCHK(ctx, expr)                                                               \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail((ctx), MLCT_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define CHECK(expr)                    \
  do {                                 \
    mlct_status st_ = (expr);          \
    if (st_ != MLCT_OK) return st_;    \
  } while (0)

// Grow-only workspace slot.  Growing frees the old buffer (hipFree waits for
// the device), so pointers from an earlier ws_get of the same slot become
// invalid; callers take all slots they need before enqueuing work.
mlct_status ws_get(mlct_ctx* ctx, int slot, size_t bytes, void** out) {
  if (bytes == 0) bytes = 256;
  DevBuf& b = ctx->slots[slot];
  if (b.bytes >= bytes) {
    *out = b.ptr;
    return MLCT_OK;
  }
  const uint64_t new_total = ctx->ws_total - b.bytes + bytes;
  if (ctx->ws_limit && new_total > ctx->ws_limit)
    return fail(ctx, MLCT_ENOMEM, "workspace of %llu bytes exceeds the limit of %llu",
                (unsigned long long)new_total, (unsigned long long)ctx->ws_limit);
  // a slot that grows again grows by at least half its size (2 MiB granules),
  // so a run of calls on ever larger operators reallocates a few times
  // rather than on every call; never past the limit
  size_t want = bytes;
  if (b.bytes) {
    want = std::max(bytes, b.bytes + b.bytes / 2);
    want = (want + ((size_t)1 << 21) - 1) & ~(((size_t)1 << 21) - 1);
    if (ctx->ws_limit && ctx->ws_total - b.bytes + want > ctx->ws_limit) want = bytes;
  }
  if (b.ptr) {
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipFree(b.ptr));
    ctx->ws_total -= b.bytes;
    b.ptr = nullptr;
    b.bytes = 0;
  }
  void* p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    if (want == bytes || hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, MLCT_ENOMEM, "hipMalloc(%zu) failed", bytes);
    }
    want = bytes;
  }
  b.ptr = p;
  b.bytes = want;
  ctx->ws_total += want;
  *out = p;
  return MLCT_OK;
}

// ---- kernel timing --------------------------------------------------------
hipEvent_t pool_event(mlct_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records a start event before a launch and a stop event after it when
// timing is enabled; durations are collected after the next synchronisation.
struct LaunchTimer {
  mlct_ctx* ctx;
  int kernel;
  hipEvent_t start = nullptr;
  LaunchTimer(mlct_ctx* c, int k) : ctx(c), kernel(k) {
    if (ctx->timing && (start = pool_event(ctx))) (void)hipEventRecord(start, ctx->stream);
  }
  void done() {
    if (!start) return;
    hipEvent_t stop = pool_event(ctx);
    if (!stop) {
      ctx->event_pool.push_back(start);
      return;
    }
    (void)hipEventRecord(stop, ctx->stream);
    ctx->pending.push_back({start, stop, kernel, units});
    start = nullptr;
  }
  void done(int n) {
    units = n;
    done();
  }
  int units = 1;
};

// Called after the context stream has been synchronised.
void collect_timing(mlct_ctx* ctx) {
  for (auto& t : ctx->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.start, t.stop) == hipSuccess) {
      ctx->kernel_ms[t.kernel] += ms;
      ctx->kernel_launches[t.kernel] += t.units;
    }
    ctx->event_pool.push_back(t.start);
    ctx->event_pool.push_back(t.stop);
  }
  ctx->pending.clear();
}

mlct_status sync_stream(mlct_ctx* ctx) {
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  collect_timing(ctx);
  if (ctx->fused_check) {
    ctx->fused_check = false;
    int32_t ab = 0;
    HIPCHK(ctx, hipMemcpy(&ab, ctx->fused_abort, sizeof ab, hipMemcpyDeviceToHost));
    if (ab == 1) return fail(ctx, MLCT_EDEVICE, "a two-step launch's tile wait timed out");
    if (ab) return fail(ctx, MLCT_EDEVICE, "a two-step launch left an XCD's tiles unprocessed");
  }
  return MLCT_OK;
}

// ---- autotune cache (plain text, one decision per line) -------------------
std::string tune_key(const mlct_op* op, int prec, int64_t bpad) {
  char buf[160];
  if (op->kind == OP_CSR || op->kind == OP_GRAM_CSR)
    snprintf(buf, sizeof buf, "%s d=%lld nnz=%lld maxrow=%d pattern=%d",
             op->kind == OP_CSR ? "csr" : "gramcsr", (long long)op->d, (long long)op->csr.nnz,
             op->csr.max_row_nnz, op->csr.val == nullptr ? 1 : 0);
  else
    snprintf(buf, sizeof buf, "dense d=%lld prec=%d bpad=%lld", (long long)op->d, prec,
             (long long)bpad);
  return buf;
}

// A cached decision, or -1 when there is none or the file holds a value the
// autotuner could not have chosen (a hand-edited or foreign cache).
int tune_lookup(const mlct_ctx* ctx, const std::string& key, const std::vector<int>& allowed) {
  for (const std::string& l : ctx->tune_lines)
    if (l.compare(0, key.size(), key) == 0 && l.size() > key.size() + 3 &&
        l.compare(key.size(), 3, " = ") == 0) {
      const int v = std::atoi(l.c_str() + key.size() + 3);
      for (int a : allowed)
        if (v == a) return v;
      return -1;
    }
  return -1;
}
// The autotuner's candidates: CSR workgroup caps and dense tile choices.
const std::vector<int> kCsrGroupCands = {512, 1024, 2048, 4096};
const std::vector<int> kDenseTileCands = {0, 2, 1, 3};

// Dense tile choice: the operator's own (mlct_autotune on it), else a
// cached decision for this shape, precision and block width, else the
// default rule (-1).
int dense_choice(const mlct_ctx* ctx, const mlct_op* op, int prec, int64_t bpad) {
  if (op->tuned_dense >= 0) return op->tuned_dense;
  if (ctx->tune_lines.empty()) return -1;
  return tune_lookup(ctx, tune_key(op, prec, bpad), kDenseTileCands);
}

void tune_store(mlct_ctx* ctx, const std::string& key, int value) {
  const std::string line = key + " = " + std::to_string(value);
  bool found = false;
  for (std::string& l : ctx->tune_lines)
    if (l.compare(0, key.size() + 3, key + " = ") == 0) {
      l = line;
      found = true;
    }
  if (!found) ctx->tune_lines.push_back(line);
  if (ctx->tune_path.empty()) return;
  FILE* fh = std::fopen(ctx->tune_path.c_str(), "w");
  if (!fh) return;
  std::fprintf(fh, "# mlct autotune cache (gfx950)\n");
  for (const std::string& l : ctx->tune_lines) std::fprintf(fh, "%s\n", l.c_str());
  std::fclose(fh);
}

void tune_load(mlct_ctx* ctx) {
  FILE* fh = std::fopen(ctx->tune_path.c_str(), "r");
  if (!fh) return;
  char buf[256];
  while (std::fgets(buf, sizeof buf, fh)) {
    std::string l(buf);
    while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
    if (!l.empty() && l[0] != '#') ctx->tune_lines.push_back(l);
  }
  std::fclose(fh);
}

mlct_status set_device(mlct_ctx* ctx) {
  HIPCHK(ctx, hipSetDevice(ctx->device));
  return MLCT_OK;
}

bool finite_interval(double a, double b) { return std::isfinite(a) && std::isfinite(b) && a < b; }

mlct_status check_func(mlct_ctx* ctx, mlct_func f, double a, double b) {
  if (!finite_interval(a, b)) return fail(ctx, MLCT_EINVAL, "need finite a < b (a=%g b=%g)", a, b);
  switch (f.kind) {
    case MLCT_LOG:
      if (a <= 0) return fail(ctx, MLCT_EINVAL, "log needs a > 0 (a=%g)", a);
      break;
    case MLCT_SQRT:
    case MLCT_POW:
      if (a < 0) return fail(ctx, MLCT_EINVAL, "sqrt/pow need a >= 0 (a=%g)", a);
      if (f.kind == MLCT_POW && !std::isfinite(f.power))
        return fail(ctx, MLCT_EINVAL, "pow needs a finite exponent");
      break;
    case MLCT_INV:
      if (a <= 0 && b >= 0) return fail(ctx, MLCT_EINVAL, "1/x needs 0 outside [a, b]");
      break;
    case MLCT_EXP:
      if ((b - a) / 2 > 700)
        return fail(ctx, MLCT_ERANGE, "exp on an interval of half-width %g overflows FP64", (b - a) / 2);
      break;
    case MLCT_CUBE:
      break;
    default:
      return fail(ctx, MLCT_EINVAL, "unknown function kind %d", f.kind);
  }
  return MLCT_OK;
}

constexpr int kMaxDegree = 4096;  // DCT samples and cosines live in 48 KB of LDS

mlct_status check_probes(mlct_ctx* ctx, const mlct_op* op, const mlct_probes* pr) {
  if (!pr) return fail(ctx, MLCT_EINVAL, "probes is NULL");
  if (pr->m < 1) return fail(ctx, MLCT_EINVAL, "need m >= 1 probes");
  if (pr->kind == MLCT_PROBE_RADEMACHER) {
    if (pr->first_id < 0) return fail(ctx, MLCT_EINVAL, "first_id must be >= 0");
    return MLCT_OK;
  }
  if (pr->kind == MLCT_PROBE_EXPLICIT) {
    if (!pr->entries_dev) return fail(ctx, MLCT_EINVAL, "explicit probes need entries_dev");
    if (pr->first_id < 0 || pr->ld_entries < pr->first_id + pr->m)
      return fail(ctx, MLCT_EINVAL, "explicit probes: need 0 <= first_id and first_id + m <= ld");
    (void)op;
    return MLCT_OK;
  }
  return fail(ctx, MLCT_EINVAL, "unknown probe kind %d", pr->kind);
}

// CSR steps with fewer workgroups than this leave the device partly idle
// (two 512-thread workgroups per CU on 256 CUs).
constexpr int kSmallGroups = 512;
constexpr int kSharedBlocks = 4;

// ---- one probe block through the recurrence ------------------------------
// Runs ``degree`` (direct) or ceil(degree/2) (symmetric form) steps on the
// ``src.active`` probes of one block and writes their moments mu_0..mu_n
// (n = degree) into mu_rows (device, row stride ldmu).
// Device buffers of one CSR probe block: the two vector buffers, the moment
// partials of every step, the reduced dots and the hub chunk sums.
struct CsrBlockBufs {
  void* v0 = nullptr;
  void* v1 = nullptr;
  double* part = nullptr;
  double* dots = nullptr;
  void* hub = nullptr;
  bool timed = true;  // record kernel timing events (these may allocate)
  int* fsync = nullptr;  // two-step launches: tickets, flags and abort flag (null: single steps)
};

// Bytes of each buffer for a block of degree ``degree`` in form ``mode``.
struct CsrBlockSizes {
  size_t v, part, dots, hub;
};
CsrBlockSizes csr_block_sizes(const mlct_op* op, size_t tsz, int mode, int degree) {
  const int S = (mode == MLCT_DOUBLING) ? (degree + 1) / 2 : degree;
  const CsrStepPlan plan = plan_csr(op->d, op->tuned_groups);
  CsrBlockSizes z;
  z.v = (size_t)op->d * kBlockProbes * tsz;
  z.part = (size_t)2 * plan.ngroups * kBlockProbes * (S + 1) * sizeof(double);
  z.dots = (size_t)(S + 1) * 2 * kBlockProbes * sizeof(double);
  z.hub = op->csr.hub_n > 0 ? (size_t)op->csr.hub_chunks * kBlockProbes * tsz : 0;
  return z;
}

// Launch shape of the two-step path (csr_fused2_kernel), or ok = false where
// it does not apply: FP32 CSR with at most 5 entries per row and a known
// bandwidth, no hub rows, Rademacher probes, and tiles enough that each
// XCD's range holds more than twice the window.
constexpr int kFusedRows = 512;  // default rows per tile
constexpr int kFusedWgs = 64;    // default workgroups per XCD (2 per CU, all resident)
constexpr int kFusedLag = 64;    // default lag beyond twice the window, in tiles
// Chunks of the per-launch partial reduction of a two-step block: one
// (the single-step association) up to 2048 tiles, else 64 (a divisor: the
// tile count is a multiple of 8, and rounded to one of 64 there).
int fused_chunks(int ntiles) { return ntiles <= 2048 ? 1 : 64; }
struct FusedPlan {
  bool ok = false;
  int rows, ntiles, window, lag, grid;
};
FusedPlan fused_plan(const mlct_ctx* ctx, const mlct_op* op, const ProbeSrc& src, size_t tsz) {
  FusedPlan f;
  if (!ctx->two_step || tsz != 4 || op->kind != OP_CSR || op->csr.max_row_nnz > 5 ||
      op->csr.bandwidth < 0 || op->csr.nnz < 1 || op->csr.hub_n > 0 || src.entries)
    return f;
  // tiles: the single-step bands where these are short (then the moment
  // sums are bitwise the single-step path's), else kFusedRows rows
  const CsrStepPlan bands = plan_csr(op->d, op->tuned_groups);
  int64_t nt;
  if (ctx->two_step_rows == 0 && bands.rows_per_group <= kFusedRows) {
    f.rows = bands.rows_per_group;
    nt = bands.ngroups;
  } else {
    f.rows = ctx->two_step_rows > 0 ? ctx->two_step_rows : kFusedRows;
    nt = ((op->d + f.rows - 1) / f.rows + 7) / 8 * 8;
    if (nt > 2048) nt = (nt + 63) / 64 * 64;  // whole chunks of the partial reduction
  }
  const int64_t w = ((int64_t)op->csr.bandwidth + f.rows - 1) / f.rows;
  if (nt > (int64_t)1 << 24 || nt / 8 <= 2 * w || nt < 64) return f;
  f.ntiles = (int)nt;
  f.window = (int)w;
  f.lag = 2 * f.window + 1 + (ctx->two_step_lag > 0 ? ctx->two_step_lag : kFusedLag);
  f.grid = 8 * (ctx->two_step_wgs > 0 ? ctx->two_step_wgs : kFusedWgs);
  f.ok = true;
  return f;
}

template <typename T>
mlct_status run_block_csr_in(mlct_ctx* ctx, const mlct_op* op, double alpha, double beta,
                             int degree, int mode, ProbeSrc src, double* mu_rows, int64_t ldmu,
                             const CsrBlockBufs& bb) {
  const int S = (mode == MLCT_DOUBLING) ? (degree + 1) / 2 : degree;
  const CsrStepPlan plan = plan_csr(op->d, op->tuned_groups);
  if (bb.fsync) {
    // two steps per launch: the single steps' vectors; the moment partials
    // per tile, reduced after every launch
    const FusedPlan f = fused_plan(ctx, op, src, sizeof(T));
    CsrStepPlan tp;
    tp.ngroups = f.ntiles;
    tp.rows_per_group = f.rows;
    float* x = static_cast<float*>(bb.v1);  // V_{s-1} -> V_{s+1}
    float* y = static_cast<float*>(bb.v0);  // V_s -> V_{s+2}
    const size_t pstep = (size_t)2 * f.ntiles * kBlockProbes;
    double* P = bb.part;
    hipStream_t s = ctx->stream;
    int* abort_flag = ctx->fused_abort;
    // After every launch its tile partials are summed, in a fixed order, into
    // C chunk sums per step (C = 1 where the tiles are few: then the sums
    // are the single-step path's), and the chunks of all steps at the end.
    const int C = fused_chunks(f.ntiles);
    double* Q = C > 1 ? P + 2 * pstep : bb.dots;  // [S+1][2][C][64]
    auto reduce_launch = [&](int step0, int nsteps) {
      return launch_reduce_partials(s, P, 1, nsteps * 2 * C, f.ntiles / C, kBlockProbes,
                                    Q + (size_t)step0 * 2 * C * kBlockProbes);
    };
    HIPCHK(ctx, launch_probe_init<float>(s, y, op->d, src, tp, P));
    HIPCHK(ctx, reduce_launch(0, 1));
    if (!ctx->fused_check) HIPCHK(ctx, launch_fill_zero_i32(s, abort_flag, 1));
    ctx->fused_check = true;
    int prev_total = 0;
    for (int k = 1; k <= S; k += 2) {
      const bool first = k == 1, two = k + 1 <= S;
      const float ca1 = (float)(first ? alpha : 2.0 * alpha), cb1 = (float)(first ? beta : 2.0 * beta);
      const int zm1 = (mode == MLCT_DOUBLING || first) ? 0 : 1;
      const int zm2 = mode == MLCT_DOUBLING ? 0 : 1;
      LaunchTimer tm(ctx, MLCT_KERNEL_CSR_STEP2);
      HIPCHK(ctx, launch_csr_fused2(s, op->csr, x, y, ca1, cb1, !first, (float)(2.0 * alpha),
                                    (float)(2.0 * beta), two, zm1, zm2, src, f.rows, f.ntiles,
                                    f.window, P, P + pstep, bb.fsync, abort_flag, f.grid, f.lag,
                                    prev_total, ctx->wait_limit_us * 100LL));
      tm.done(two ? 2 : 1);
      prev_total = two ? 2 * (f.ntiles / 8) : f.ntiles / 8;
      HIPCHK(ctx, reduce_launch(k, two ? 2 : 1));
    }
    HIPCHK(ctx, launch_fused_sync(s, bb.fsync, 0, prev_total, abort_flag));
    if (C > 1) HIPCHK(ctx, launch_reduce_partials(s, Q, S + 1, 2, C, kBlockProbes, bb.dots));
    HIPCHK(ctx, launch_assemble_moments(s, bb.dots, S + 1, kBlockProbes, src.active, mode, degree,
                                        mu_rows, ldmu));
    return MLCT_OK;
  }
  const size_t pstep = (size_t)2 * plan.ngroups * kBlockProbes;  // doubles per step
  T* buf[2] = {static_cast<T*>(bb.v0), static_cast<T*>(bb.v1)};
  double* P = bb.part;
  void* dots = bb.dots;
  void* hub = bb.hub;
  hipStream_t s = ctx->stream;
  HIPCHK(ctx, launch_probe_init<T>(s, buf[0], op->d, src, plan, P));
  const int zdirect = src.entries ? 2 : 1;
  for (int k = 1; k <= S; ++k) {
    // v_k = ca A v_{k-1} + cb v_{k-1} [- v_{k-2}], written over v_{k-2}
    const T* vk = buf[(k - 1) & 1];
    T* vm = buf[k & 1];
    const bool first = (k == 1);
    const T ca = (T)(first ? alpha : 2.0 * alpha);
    const T cb = (T)(first ? beta : 2.0 * beta);
    const int zmode = (mode == MLCT_DOUBLING || first) ? 0 : zdirect;
    if (bb.timed) {
      LaunchTimer tm(ctx, MLCT_KERNEL_CSR_STEP);
      HIPCHK(ctx, launch_csr_step<T>(s, op->csr, vk, vm, ca, cb, !first, zmode, src, plan, hub,
                                     P + pstep * k));
      tm.done();
    } else {
      HIPCHK(ctx, launch_csr_step<T>(s, op->csr, vk, vm, ca, cb, !first, zmode, src, plan, hub,
                                     P + pstep * k));
    }
  }
  HIPCHK(ctx, launch_reduce_partials(s, P, S + 1, 2, plan.ngroups, kBlockProbes,
                                     static_cast<double*>(dots)));
  HIPCHK(ctx, launch_assemble_moments(s, static_cast<double*>(dots), S + 1, kBlockProbes,
                                      src.active, mode, degree, mu_rows, ldmu));
  return MLCT_OK;
}

// Two-step launches give each XCD one eighth of the tiles, so they need
// every XCD to receive workgroups (true when the device dispatches
// workgroups to its XCDs in turn; not on a partition that holds one XCD).
// Checked once per context with a launch of the same grid.
mlct_status probe_xcds(mlct_ctx* ctx, int* buf, int grid) {
  HIPCHK(ctx, launch_xcc_probe(ctx->stream, buf, grid));
  std::vector<int> ids(grid);
  HIPCHK(ctx, hipMemcpyAsync(ids.data(), buf, grid * sizeof(int), hipMemcpyDeviceToHost,
                             ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  int count[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int v : ids) count[v & 7]++;
  ctx->xcd_ok = 1;
  for (int x = 0; x < 8; ++x)
    if (count[x] == 0) ctx->xcd_ok = 0;
  return MLCT_OK;
}

template <typename T>
mlct_status run_block_csr(mlct_ctx* ctx, const mlct_op* op, double alpha, double beta,
                          int degree, int mode, ProbeSrc src, double* mu_rows, int64_t ldmu) {
  const CsrBlockSizes z = csr_block_sizes(op, sizeof(T), mode, degree);
  CsrBlockBufs bb;
  void* part;
  void* dots;
  CHECK(ws_get(ctx, WS_V0, z.v, &bb.v0));
  CHECK(ws_get(ctx, WS_V1, z.v, &bb.v1));
  CHECK(ws_get(ctx, WS_PART, z.part, &part));
  CHECK(ws_get(ctx, WS_MISC, z.dots, &dots));
  if (z.hub) CHECK(ws_get(ctx, WS_HUB, z.hub, &bb.hub));
  bb.part = static_cast<double*>(part);
  bb.dots = static_cast<double*>(dots);
  const CsrStepPlan plan = plan_csr(op->d, op->tuned_groups);
  const FusedPlan f = fused_plan(ctx, op, src, sizeof(T));
  if (f.ok) {
    void *fs, *fa;
    const size_t nsync = std::max<size_t>(8 + (size_t)f.ntiles, (size_t)f.grid);
    CHECK(ws_get(ctx, WS_FSYNC, nsync * sizeof(int), &fs));
    CHECK(ws_get(ctx, WS_FABORT, 64, &fa));  // never grows: the address stays valid
    if (ctx->xcd_ok < 0) CHECK(probe_xcds(ctx, static_cast<int*>(fs), f.grid));
    if (ctx->xcd_ok > 0) {
      // partials of two steps at a time, per tile, then the chunk sums of
      // every step
      const int C = fused_chunks(f.ntiles);
      const int S = (mode == MLCT_DOUBLING) ? (degree + 1) / 2 : degree;
      const size_t fpart =
          ((size_t)2 * 2 * f.ntiles + (C > 1 ? (size_t)(S + 1) * 2 * C : 0)) * kBlockProbes *
          sizeof(double);
      if (fpart > z.part) {
        CHECK(ws_get(ctx, WS_PART, fpart, &part));
        bb.part = static_cast<double*>(part);
      }
      bb.fsync = static_cast<int*>(fs);
      ctx->fused_abort = static_cast<int*>(fa);
    }
  }
  return run_block_csr_in<T>(ctx, op, alpha, beta, degree, mode, src, mu_rows, ldmu, bb);
}

// One probe block through the sparse Gram operator A = X^T X + lambda I:
// per step W = X V_k (rows x 64 scratch), then the recurrence over X^T W
// (the shift enters cb as ca * lambda).
// One probe block of a callback operator: per step the caller's function
// writes W = A V_k, then the update kernel forms V_new and the partials.
mlct_status run_block_callback(mlct_ctx* ctx, const mlct_op* op, double alpha, double beta,
                               int degree, int mode, ProbeSrc src, double* mu_rows,
                               int64_t ldmu) {
  const int S = (mode == MLCT_DOUBLING) ? (degree + 1) / 2 : degree;
  const CsrStepPlan plan = plan_csr(op->d, 0);
  const size_t vb = (size_t)op->d * kBlockProbes * sizeof(float);
  const size_t pstep = (size_t)2 * plan.ngroups * kBlockProbes;
  void *v0, *v1, *w, *part, *dots;
  CHECK(ws_get(ctx, WS_V0, vb, &v0));
  CHECK(ws_get(ctx, WS_V1, vb, &v1));
  CHECK(ws_get(ctx, WS_CBW, vb, &w));
  CHECK(ws_get(ctx, WS_PART, pstep * (S + 1) * sizeof(double), &part));
  CHECK(ws_get(ctx, WS_MISC, (size_t)(S + 1) * 2 * kBlockProbes * sizeof(double), &dots));
  float* buf[2] = {static_cast<float*>(v0), static_cast<float*>(v1)};
  double* P = static_cast<double*>(part);
  hipStream_t s = ctx->stream;
  HIPCHK(ctx, launch_probe_init<float>(s, buf[0], op->d, src, plan, P));
  const int zdirect = src.entries ? 2 : 1;
  for (int k = 1; k <= S; ++k) {
    const float* vk = buf[(k - 1) & 1];
    float* vm = buf[k & 1];
    const bool first = (k == 1);
    const float ca = (float)(first ? alpha : 2.0 * alpha);
    const float cb = (float)(first ? beta : 2.0 * beta);
    const int zmode = (mode == MLCT_DOUBLING || first) ? 0 : zdirect;
    const int32_t rc = op->cb_apply(op->cb_user, vk, static_cast<float*>(w), kBlockProbes,
                                    static_cast<void*>(s));
    if (rc != 0) return fail(ctx, MLCT_EDEVICE, "the operator's apply function returned %d", rc);
    LaunchTimer tm(ctx, MLCT_KERNEL_CALLBACK_STEP);
    HIPCHK(ctx, launch_callback_step(s, static_cast<const float*>(w), vk, vm, ca, cb, !first,
                                     zmode, src, op->d, plan, P + pstep * k));
    tm.done();
  }
  HIPCHK(ctx, launch_reduce_partials(s, P, S + 1, 2, plan.ngroups, kBlockProbes,
                                     static_cast<double*>(dots)));
  HIPCHK(ctx, launch_assemble_moments(s, static_cast<double*>(dots), S + 1, kBlockProbes,
                                      src.active, mode, degree, mu_rows, ldmu));
  return MLCT_OK;
}

template <typename T>
mlct_status run_block_gram_csr(mlct_ctx* ctx, const mlct_op* op, double alpha, double beta,
                               int degree, int mode, ProbeSrc src, double* mu_rows,
                               int64_t ldmu) {
  const int S = (mode == MLCT_DOUBLING) ? (degree + 1) / 2 : degree;
  const CsrStepPlan plan = plan_csr(op->d, op->tuned_groups);
  const CsrStepPlan plan_r = plan_csr(op->csrx.nrows, op->tuned_groups);
  const size_t vbytes = (size_t)op->d * kBlockProbes * sizeof(T);
  const size_t pstep = (size_t)2 * plan.ngroups * kBlockProbes;
  void *v0, *v1, *part, *dots, *wb, *hubs = nullptr;
  CHECK(ws_get(ctx, WS_V0, vbytes, &v0));
  CHECK(ws_get(ctx, WS_V1, vbytes, &v1));
  CHECK(ws_get(ctx, WS_PART, pstep * (S + 1) * sizeof(double), &part));
  CHECK(ws_get(ctx, WS_MISC, (size_t)(S + 1) * 2 * kBlockProbes * sizeof(double), &dots));
  CHECK(ws_get(ctx, WS_GRAMW, (size_t)op->csrx.nrows * kBlockProbes * sizeof(T), &wb));
  const size_t hx = (size_t)op->csrx.hub_chunks * kBlockProbes, ht = (size_t)op->csr.hub_chunks * kBlockProbes;
  if (hx + ht > 0) CHECK(ws_get(ctx, WS_HUB, (hx + ht) * sizeof(T), &hubs));
  T* hubx = static_cast<T*>(hubs);
  T* hubt = hubx ? hubx + hx : nullptr;
  T* buf[2] = {static_cast<T*>(v0), static_cast<T*>(v1)};
  T* W = static_cast<T*>(wb);
  double* P = static_cast<double*>(part);
  hipStream_t s = ctx->stream;
  HIPCHK(ctx, launch_probe_init<T>(s, buf[0], op->d, src, plan, P));
  const int zdirect = src.entries ? 2 : 1;
  for (int k = 1; k <= S; ++k) {
    const T* vk = buf[(k - 1) & 1];
    T* vm = buf[k & 1];
    const bool first = (k == 1);
    const double ca = first ? alpha : 2.0 * alpha;
    const double cb = (first ? beta : 2.0 * beta) + ca * op->gram_lambda;
    const int zmode = (mode == MLCT_DOUBLING || first) ? 0 : zdirect;
    LaunchTimer tm(ctx, MLCT_KERNEL_GRAM_CSR_STEP);
    HIPCHK(ctx, launch_gram_csr_step<T>(s, op->csrx, op->csr, vk, vm, W, (T)ca, (T)cb, !first,
                                        zmode, src, plan_r, plan, hubx, hubt, P + pstep * k));
    tm.done();
  }
  HIPCHK(ctx, launch_reduce_partials(s, P, S + 1, 2, plan.ngroups, kBlockProbes,
                                     static_cast<double*>(dots)));
  HIPCHK(ctx, launch_assemble_moments(s, static_cast<double*>(dots), S + 1, kBlockProbes,
                                      src.active, mode, degree, mu_rows, ldmu));
  return MLCT_OK;
}

// Matrix operand of a dense operator in the arithmetic ``prec``: the
// caller's A when it already has that type, else a converted or bf16-split
// copy built once and owned by the operator.
// Hub table of a CSR operator (rows longer than kHubLen): found on the
// device, sorted by row on the host, cut into chunks of kHubChunk entries.
// At most nnz / (kHubLen + 1) rows qualify, which bounds the search output.
mlct_status build_hubs(mlct_ctx* ctx, mlct::CsrMat& mat, void** mem_out) {
  const int cap = (int)(mat.nnz / (kHubLen + 1) + 1);
  void* tmp;
  CHECK(ws_get(ctx, WS_HUB, (size_t)(3 * (int64_t)cap + 1) * sizeof(int32_t), &tmp));
  int32_t* trip = static_cast<int32_t*>(tmp);
  int32_t* count = trip + 3 * (int64_t)cap;
  hipStream_t s = ctx->stream;
  HIPCHK(ctx, hipMemsetAsync(count, 0, sizeof(int32_t), s));
  HIPCHK(ctx, launch_hub_find(s, mat.rowptr, mat.nrows, trip, count, cap));
  int32_t n = 0;
  HIPCHK(ctx, hipMemcpyAsync(&n, count, sizeof n, hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  if (n <= 0 || n > cap) return fail(ctx, MLCT_EDEVICE, "hub row search returned %d rows", n);
  std::vector<int32_t> h((size_t)3 * n);
  HIPCHK(ctx, hipMemcpyAsync(h.data(), trip, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return h[3 * x] < h[3 * y]; });
  std::vector<int32_t> rows(n), c0(n + 1), cs, ce;
  for (int k = 0; k < n; ++k) {
    const int32_t* t = &h[3 * (size_t)order[k]];
    rows[k] = t[0];
    c0[k] = (int32_t)cs.size();
    for (int32_t a = t[1]; a < t[2]; a += kHubChunk) {
      cs.push_back(a);
      ce.push_back(std::min<int32_t>(a + kHubChunk, t[2]));
    }
  }
  c0[n] = (int32_t)cs.size();
  const size_t nch = cs.size();
  const size_t words = (size_t)n + (n + 1) + 2 * nch;
  void* mem = nullptr;
  if (hipMalloc(&mem, words * sizeof(int32_t)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, MLCT_ENOMEM, "no memory for the hub table");
  }
  std::vector<int32_t> all;
  all.reserve(words);
  all.insert(all.end(), rows.begin(), rows.end());
  all.insert(all.end(), c0.begin(), c0.end());
  all.insert(all.end(), cs.begin(), cs.end());
  all.insert(all.end(), ce.begin(), ce.end());
  const hipError_t e = hipMemcpy(mem, all.data(), words * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(mem);
    return fail(ctx, MLCT_EDEVICE, "hub table upload: %s", hipGetErrorString(e));
  }
  int32_t* base = static_cast<int32_t*>(mem);
  *mem_out = mem;
  mat.hub_rows = base;
  mat.hub_c0 = base + n;
  mat.hub_cs = base + n + (n + 1);
  mat.hub_ce = mat.hub_cs + nch;
  mat.hub_n = n;
  mat.hub_chunks = (int)nch;
  return MLCT_OK;
}

// tr T_j(A_hat) for j = 0, 1, 2 with A_hat = alpha A + beta I (A symmetric):
// d, alpha tr A + beta d, 2 ||A_hat||_F^2 - d, from tr A and ||A||_F^2
// (computed once per operator on the device, then kept).
mlct_status low_traces(mlct_ctx* ctx, const mlct_op* cop, double alpha, double beta,
                       double t[3]) {
  mlct_op* op = const_cast<mlct_op*>(cop);
  if (!op->stats_ready) {
    void* w;
    CHECK(ws_get(ctx, WS_STATS, (2 * (size_t)kStatsGroups + 2) * sizeof(double), &w));
    double* part = static_cast<double*>(w);
    HIPCHK(ctx, launch_op_stats(ctx->stream, op, part, part + 2 * kStatsGroups));
    double h[2];
    HIPCHK(ctx, hipMemcpyAsync(h, part + 2 * kStatsGroups, sizeof h, hipMemcpyDeviceToHost,
                               ctx->stream));
    CHECK(sync_stream(ctx));
    op->tr_a = h[0];
    op->fro2 = h[1];
    op->stats_ready = true;
  }
  const double d = (double)op->d;
  const double fro_hat = alpha * alpha * op->fro2 + 2.0 * alpha * beta * op->tr_a + beta * beta * d;
  t[0] = d;
  t[1] = alpha * op->tr_a + beta * d;
  t[2] = 2.0 * fro_hat - d;
  return MLCT_OK;
}

mlct_status dense_operand(mlct_ctx* ctx, const mlct_op* cop, int prec, const void** a0,
                          const void** a1, int64_t* lda) {
  mlct_op* op = const_cast<mlct_op*>(cop);
  const int64_t d = op->d;
  *a1 = nullptr;
  if ((prec == MLCT_FP64 && op->dtype == MLCT_DT_F64) ||
      (prec == MLCT_FP32 && op->dtype == MLCT_DT_F32)) {
    *a0 = op->A;
    *lda = op->lda;
    return MLCT_OK;
  }
  *lda = d;
  if (prec == MLCT_BF16X3) {
    if (!op->split_hi) {
      void *hi = nullptr, *lo = nullptr;
      if (hipMalloc(&hi, (size_t)d * d * 2) != hipSuccess || hipMalloc(&lo, (size_t)d * d * 2) != hipSuccess) {
        (void)hipGetLastError();
        if (hi) (void)hipFree(hi);
        return fail(ctx, MLCT_ENOMEM, "no memory for the bf16 split of A");
      }
      HIPCHK(ctx, launch_dense_split(ctx->stream, op->A, op->dtype, d, op->lda, hi, lo));
      op->split_hi = hi;
      op->split_lo = lo;
    }
    *a0 = op->split_hi;
    *a1 = op->split_lo;
    return MLCT_OK;
  }
  void** slot = prec == MLCT_FP64 ? &op->a64 : &op->a32;
  if (!*slot) {
    void* p = nullptr;
    if (hipMalloc(&p, (size_t)d * d * (prec == MLCT_FP64 ? 8 : 4)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, MLCT_ENOMEM, "no memory for a converted copy of A");
    }
    HIPCHK(ctx, launch_dense_convert(ctx->stream, op->A, op->dtype, d, op->lda, p));
    *slot = p;
  }
  *a0 = *slot;
  return MLCT_OK;
}

int64_t dense_bpad(int64_t active) { return (active + 31) / 32 * 32; }

// The bf16 split of A packed for the skinny kernel (built once per operator).
mlct_status dense_packed_a(mlct_ctx* ctx, const mlct_op* cop, const void* hi, const void* lo,
                           const void** phi, const void** plo) {
  mlct_op* op = const_cast<mlct_op*>(cop);
  if (!op->pack_hi) {
    const size_t bytes = dense_pack_bytes(op->d, op->d);
    void *h = nullptr, *l = nullptr;
    if (hipMalloc(&h, bytes) != hipSuccess || hipMalloc(&l, bytes) != hipSuccess) {
      (void)hipGetLastError();
      if (h) (void)hipFree(h);
      return fail(ctx, MLCT_ENOMEM, "no memory for the packed bf16 split of A");
    }
    HIPCHK(ctx, launch_dense_pack_a(ctx->stream, hi, lo, op->d, h, l));
    op->pack_hi = h;
    op->pack_lo = l;
  }
  *phi = op->pack_hi;
  *plo = op->pack_lo;
  return MLCT_OK;
}

// Device workspace of one probe block (taken before any launch, so that
// growth never frees a buffer still in use).
mlct_status reserve_block_ws(mlct_ctx* ctx, const mlct_op* op, int prec, int mode, int degree,
                             int64_t block) {
  const int S = (mode == MLCT_DOUBLING) ? (degree + 1) / 2 : degree;
  void* tmp;
  if (op->kind == OP_CALLBACK) {
    const CsrStepPlan plan = plan_csr(op->d, 0);
    const size_t vb = (size_t)op->d * kBlockProbes * sizeof(float);
    CHECK(ws_get(ctx, WS_V0, vb, &tmp));
    CHECK(ws_get(ctx, WS_V1, vb, &tmp));
    CHECK(ws_get(ctx, WS_CBW, vb, &tmp));
    CHECK(ws_get(ctx, WS_PART, (size_t)2 * plan.ngroups * kBlockProbes * (S + 1) * sizeof(double), &tmp));
    CHECK(ws_get(ctx, WS_MISC, (size_t)(S + 1) * 2 * kBlockProbes * sizeof(double), &tmp));
    return MLCT_OK;
  }
  if (op->kind == OP_CSR || op->kind == OP_GRAM_CSR) {
    const CsrStepPlan plan = plan_csr(op->d, op->tuned_groups);
    const size_t tsz = prec == MLCT_FP64 ? 8 : 4;
    CHECK(ws_get(ctx, WS_V0, (size_t)op->d * kBlockProbes * tsz, &tmp));
    CHECK(ws_get(ctx, WS_V1, (size_t)op->d * kBlockProbes * tsz, &tmp));
    CHECK(ws_get(ctx, WS_PART, (size_t)2 * plan.ngroups * kBlockProbes * (S + 1) * sizeof(double), &tmp));
    CHECK(ws_get(ctx, WS_MISC, (size_t)(S + 1) * 2 * kBlockProbes * sizeof(double), &tmp));
    const size_t hubs = (size_t)op->csr.hub_chunks + (op->kind == OP_GRAM_CSR ? op->csrx.hub_chunks : 0);
    if (hubs > 0) CHECK(ws_get(ctx, WS_HUB, hubs * kBlockProbes * tsz, &tmp));
    if (op->kind == OP_GRAM_CSR)
      CHECK(ws_get(ctx, WS_GRAMW, (size_t)op->csrx.nrows * kBlockProbes * tsz, &tmp));
    return MLCT_OK;
  }
  const int64_t bpad = dense_bpad(block);
  const int64_t ntiles = (op->d + 15) / 16;  // the narrowest tile: an upper bound for any block
  const size_t tsz = prec == MLCT_FP64 ? 8 : 4;
  CHECK(ws_get(ctx, WS_V0, (size_t)bpad * op->d * tsz, &tmp));
  CHECK(ws_get(ctx, WS_V1, (size_t)bpad * op->d * tsz, &tmp));
  CHECK(ws_get(ctx, WS_PART, (size_t)2 * ntiles * bpad * (S + 1) * sizeof(double), &tmp));
  CHECK(ws_get(ctx, WS_MISC, (size_t)(S + 1) * 2 * bpad * sizeof(double), &tmp));
  const DenseTile tb = dense_tile(prec, op->d, op->d, bpad, dense_choice(ctx, op, prec, bpad));
  if (prec == MLCT_BF16X3 && (tb.skinny || tb.bm == 128))
    CHECK(ws_get(ctx, WS_DPACK, 4 * dense_pack_bytes(bpad, op->d), &tmp));
  return MLCT_OK;
}

mlct_status run_block_dense(mlct_ctx* ctx, const mlct_op* op, double alpha, double beta,
                            int degree, int mode, int prec, ProbeSrc src, double* mu_rows,
                            int64_t ldmu) {
  const int S = (mode == MLCT_DOUBLING) ? (degree + 1) / 2 : degree;
  const int64_t d = op->d, bpad = dense_bpad(src.active);
  const void *a0, *a1;
  int64_t lda;
  CHECK(dense_operand(ctx, op, prec, &a0, &a1, &lda));
  const int tile_choice = dense_choice(ctx, op, prec, bpad);
  const DenseTile t = dense_tile(prec, d, lda, bpad, tile_choice);
  const int64_t ntiles = (d + t.bn - 1) / t.bn;
  CHECK(reserve_block_ws(ctx, op, prec, mode, degree, src.active));
  const size_t tsz = prec == MLCT_FP64 ? 8 : 4;
  void *v0, *v1, *part, *dots;
  CHECK(ws_get(ctx, WS_V0, (size_t)bpad * d * tsz, &v0));
  CHECK(ws_get(ctx, WS_V1, (size_t)bpad * d * tsz, &v1));
  CHECK(ws_get(ctx, WS_PART, (size_t)2 * ntiles * bpad * (S + 1) * sizeof(double), &part));
  CHECK(ws_get(ctx, WS_MISC, (size_t)(S + 1) * 2 * bpad * sizeof(double), &dots));
  void* buf[2] = {v0, v1};
  double* P = static_cast<double*>(part);
  double* D = static_cast<double*>(dots);
  const size_t pstep = (size_t)2 * ntiles * bpad;
  hipStream_t s = ctx->stream;
  HIPCHK(ctx, launch_dense_probe_init(s, prec, buf[0], d, bpad, src, D));
  // BF16X3 skinny and 128-wide blocks read A and V_k packed; two packed V
  // blocks alternate
  // (V_0 packed here, V_new packed by each step's epilogue; their padding
  // stays zero)
  const bool packed = prec == MLCT_BF16X3 && (t.skinny || t.bm == 128);
  const void *pa_hi = nullptr, *pa_lo = nullptr;
  char* vpk[4] = {nullptr, nullptr, nullptr, nullptr};  // (hi, lo) of blocks 0 and 1
  if (packed) {
    CHECK(dense_packed_a(ctx, op, a0, a1, &pa_hi, &pa_lo));
    const size_t pb = dense_pack_bytes(bpad, d);
    void* w;
    CHECK(ws_get(ctx, WS_DPACK, 4 * pb, &w));
    for (int i = 0; i < 4; ++i) vpk[i] = static_cast<char*>(w) + i * pb;
    HIPCHK(ctx, launch_dense_pack_v(s, static_cast<const float*>(buf[0]), bpad, d, vpk[0],
                                    vpk[1]));
    HIPCHK(ctx, hipMemsetAsync(vpk[2], 0, 2 * pb, s));
  }
  const int zdirect = src.entries ? 2 : 1;
  for (int k = 1; k <= S; ++k) {
    const bool first = (k == 1);
    DenseStepArgs a;
    a.A0 = a0;
    a.A1 = a1;
    a.lda = lda;
    a.d = d;
    a.bpad = bpad;
    a.vk = buf[(k - 1) & 1];
    a.vm = buf[k & 1];
    a.ca = first ? alpha : 2.0 * alpha;
    a.cb = first ? beta : 2.0 * beta;
    a.has_prev = !first;
    a.zmode = (mode == MLCT_DOUBLING || first) ? 0 : zdirect;
    a.src = src;
    a.part = P + pstep * (k - 1);
    a.tile_force = tile_choice;
    if (packed) {
      const int in = (k - 1) & 1, out = k & 1;
      a.pk_a_hi = pa_hi;
      a.pk_a_lo = pa_lo;
      a.pk_v_hi = vpk[2 * in];
      a.pk_v_lo = vpk[2 * in + 1];
      a.pk_o_hi = vpk[2 * out];
      a.pk_o_lo = vpk[2 * out + 1];
    }
    LaunchTimer tm(ctx, MLCT_KERNEL_DENSE_STEP);
    HIPCHK(ctx, launch_dense_step(s, prec, a));
    tm.done();
  }
  if (S > 0)
    HIPCHK(ctx, launch_reduce_partials(s, P, S, 2, (int)ntiles, (int)bpad, D + 2 * bpad));
  HIPCHK(ctx, launch_assemble_moments(s, D, S + 1, (int)bpad, src.active, mode, degree, mu_rows,
                                      ldmu));
  return MLCT_OK;
}

mlct_status run_block(mlct_ctx* ctx, const mlct_op* op, double alpha, double beta, int degree,
                      int mode, int prec, ProbeSrc src, double* mu_rows, int64_t ldmu) {
  if (op->kind == OP_CSR) {
    if (prec == MLCT_FP32)
      return run_block_csr<float>(ctx, op, alpha, beta, degree, mode, src, mu_rows, ldmu);
    if (prec == MLCT_FP64)
      return run_block_csr<double>(ctx, op, alpha, beta, degree, mode, src, mu_rows, ldmu);
    return fail(ctx, MLCT_EUNSUPPORTED, "CSR operators support MLCT_FP32 and MLCT_FP64");
  }
  if (op->kind == OP_CALLBACK) {
    if (prec != MLCT_FP32)
      return fail(ctx, MLCT_EUNSUPPORTED, "callback operators run in MLCT_FP32");
    return run_block_callback(ctx, op, alpha, beta, degree, mode, src, mu_rows, ldmu);
  }
  if (op->kind == OP_GRAM_CSR) {
    if (prec == MLCT_FP32)
      return run_block_gram_csr<float>(ctx, op, alpha, beta, degree, mode, src, mu_rows, ldmu);
    if (prec == MLCT_FP64)
      return run_block_gram_csr<double>(ctx, op, alpha, beta, degree, mode, src, mu_rows, ldmu);
    return fail(ctx, MLCT_EUNSUPPORTED, "sparse Gram operators support MLCT_FP32 and MLCT_FP64");
  }
  return run_block_dense(ctx, op, alpha, beta, degree, mode, prec, src, mu_rows, ldmu);
}

// Moments of probes [0, m) of a probe set, in blocks of kBlockProbes.
mlct_status run_probe_set(mlct_ctx* ctx, const mlct_op* op, double alpha, double beta,
                          int degree, int mode, int prec, const mlct_probes* pr, double* mu_dev,
                          int64_t ldmu) {
  const bool sparse = op->kind == OP_CSR || op->kind == OP_GRAM_CSR || op->kind == OP_CALLBACK;
  const int64_t width = sparse ? kBlockProbes : kDenseMaxBlock;
  for (int64_t p0 = 0; p0 < pr->m; p0 += width) {
    ProbeSrc src;
    src.seed = pr->seed;
    src.first_id = pr->first_id + p0;
    src.entries = pr->kind == MLCT_PROBE_EXPLICIT ? pr->entries_dev : nullptr;
    src.ld = pr->ld_entries;
    src.active = (int32_t)((pr->m - p0) < width ? (pr->m - p0) : width);
    CHECK(run_block(ctx, op, alpha, beta, degree, mode, prec, src, mu_dev + p0 * ldmu, ldmu));
  }
  return MLCT_OK;
}

mlct_status check_mode_prec(mlct_ctx* ctx, int mode, int prec) {
  if (mode != MLCT_DIRECT && mode != MLCT_DOUBLING)
    return fail(ctx, MLCT_EINVAL, "unknown mode %d", mode);
  if (prec != MLCT_FP32 && prec != MLCT_FP64 && prec != MLCT_BF16X3)
    return fail(ctx, MLCT_EINVAL, "unknown precision %d", prec);
  return MLCT_OK;
}

// Equal-work row bands of the operator's CSR matrices for the workgroup count
// of its current plan; only matrices with very uneven rows get them.  Built
// on the context stream, so steps already enqueued keep the bands they read.
constexpr int kMaxBandGroups = 8192;

mlct_status refresh_bands(mlct_ctx* ctx, mlct_op* op) {
  CsrMat* mats[2] = {&op->csr, op->kind == OP_GRAM_CSR ? &op->csrx : nullptr};
  for (int k = 0; k < 2; ++k) {
    CsrMat* m = mats[k];
    if (!m) continue;
    const CsrStepPlan p = plan_csr(m->nrows, op->tuned_groups);
    if (!csr_uneven(*m) || p.ngroups < kBandMinGroups || p.ngroups > kMaxBandGroups) {
      m->band = nullptr;
      m->band_groups = 0;
      continue;
    }
    if (m->band && m->band_groups == p.ngroups) continue;
    if (!op->band_mem)
      HIPCHK(ctx, hipMalloc(&op->band_mem, 2 * (size_t)(kMaxBandGroups + 1) * sizeof(int32_t)));
    int32_t* band = static_cast<int32_t*>(op->band_mem) + k * (kMaxBandGroups + 1);
    HIPCHK(ctx, launch_csr_bands(ctx->stream, m->rowptr, m->nrows, p.ngroups, band));
    m->band = band;
    m->band_groups = p.ngroups;
  }
  return MLCT_OK;
}

}  // namespace

// =========================================================================
extern "C" {

mlct_status mlct_create(int device, void* hip_stream, const char* tune_cache_path,
                        mlct_ctx** out) {
  if (!out) return MLCT_EINVAL;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return MLCT_EDEVICE;
  }
  mlct_ctx* ctx = new (std::nothrow) mlct_ctx();
  if (!ctx) return MLCT_ENOMEM;
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  ctx->slots.resize(WS_NSLOTS);
  if (tune_cache_path && *tune_cache_path) {
    ctx->tune_path = tune_cache_path;
    tune_load(ctx);
  }
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return MLCT_EDEVICE;
  }
  if (device < kMaxScratchDevices && !noalloc_scratch(device)) {
    delete ctx;
    return MLCT_EDEVICE;
  }
  *out = ctx;
  return MLCT_OK;
}

mlct_status mlct_destroy(mlct_ctx* ctx) {
  if (!ctx) return MLCT_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& b : ctx->slots)
    if (b.ptr) (void)hipFree(b.ptr);
  for (auto& t : ctx->pending) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
  if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
  delete ctx;
  return MLCT_OK;
}

const char* mlct_last_error(const mlct_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

mlct_status mlct_timing(mlct_ctx* ctx, int32_t enable) {
  if (!ctx) return MLCT_EINVAL;
  if (enable) {
    for (int k = 0; k < MLCT_NUM_KERNEL_IDS; ++k) {
      ctx->kernel_ms[k] = 0.0;
      ctx->kernel_launches[k] = 0;
    }
  }
  ctx->timing = enable != 0;
  return MLCT_OK;
}

mlct_status mlct_timing_read(const mlct_ctx* ctx, int32_t kernel, int64_t* launches,
                             double* total_ms) {
  if (!ctx || kernel < 0 || kernel >= MLCT_NUM_KERNEL_IDS) return MLCT_EINVAL;
  if (launches) *launches = ctx->kernel_launches[kernel];
  if (total_ms) *total_ms = ctx->kernel_ms[kernel];
  return MLCT_OK;
}

mlct_status mlct_set_workspace_limit(mlct_ctx* ctx, uint64_t bytes) {
  if (!ctx) return MLCT_EINVAL;
  ctx->ws_limit = bytes;
  return MLCT_OK;
}

mlct_status mlct_set_option(mlct_ctx* ctx, int32_t option, int64_t value) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (option == MLCT_OPT_TWO_STEP) {
    if (value != 0 && value != 1) return fail(ctx, MLCT_EINVAL, "MLCT_OPT_TWO_STEP takes 0 or 1");
    ctx->two_step = (int)value;
    return MLCT_OK;
  }
  if (option == MLCT_OPT_TWO_STEP_LAG) {
    if (value < 0 || value > 4096) return fail(ctx, MLCT_EINVAL, "MLCT_OPT_TWO_STEP_LAG takes 0..4096");
    ctx->two_step_lag = (int)value;
    return MLCT_OK;
  }
  if (option == MLCT_OPT_TWO_STEP_ROWS) {
    if (value < 0 || value > 8192 || value % 8)
      return fail(ctx, MLCT_EINVAL, "MLCT_OPT_TWO_STEP_ROWS takes 0 or a multiple of 8 up to 8192");
    ctx->two_step_rows = (int)value;
    return MLCT_OK;
  }
  if (option == MLCT_OPT_TWO_STEP_WGS) {
    if (value < 0 || value > 512) return fail(ctx, MLCT_EINVAL, "MLCT_OPT_TWO_STEP_WGS takes 0..512");
    ctx->two_step_wgs = (int)value;
    return MLCT_OK;
  }
  if (option == MLCT_OPT_BATCH_SOLO_ROWS) {
    if (value < 0) return fail(ctx, MLCT_EINVAL, "MLCT_OPT_BATCH_SOLO_ROWS takes a row count >= 0");
    ctx->batch_solo_rows = value == 0 ? kBatchSoloRowsDefault : value;
    return MLCT_OK;
  }
  if (option == MLCT_OPT_WAIT_LIMIT_US) {
    if (value < 0 || value > 60000000) return fail(ctx, MLCT_EINVAL, "wait limit must be in [0, 6e7] us");
    ctx->wait_limit_us = value;
    return MLCT_OK;
  }
  return fail(ctx, MLCT_EINVAL, "unknown option %d", option);
}

mlct_status mlct_op_csr(mlct_ctx* ctx, int64_t d, int64_t nnz, const int32_t* rowptr_dev,
                        const int32_t* col_dev, const void* val_dev, int32_t dtype,
                        mlct_op** out) {
  if (!ctx || !out) return MLCT_EINVAL;
  ctx->err.clear();
  if (d < 1 || d > (int64_t)1 << 31) return fail(ctx, MLCT_EINVAL, "bad dimension d=%lld", (long long)d);
  if (nnz < 0 || nnz > INT32_MAX) return fail(ctx, MLCT_EINVAL, "bad nnz=%lld", (long long)nnz);
  if (!rowptr_dev || (nnz > 0 && !col_dev))
    return fail(ctx, MLCT_EINVAL, "rowptr/col must be device pointers");
  if (dtype == MLCT_DT_F32) {
    if (nnz > 0 && !val_dev) return fail(ctx, MLCT_EINVAL, "MLCT_DT_F32 needs values");
  } else if (dtype == MLCT_DT_PATTERN) {
    if (val_dev) return fail(ctx, MLCT_EINVAL, "MLCT_DT_PATTERN takes no values");
  } else {
    return fail(ctx, MLCT_EUNSUPPORTED, "CSR values must be float32 or a pattern");
  }
  CHECK(set_device(ctx));
  void* flags;
  CHECK(ws_get(ctx, WS_MISC, 64, &flags));
  HIPCHK(ctx, hipMemsetAsync(flags, 0, 2 * sizeof(int32_t), ctx->stream));
  HIPCHK(ctx, launch_csr_validate(ctx->stream, rowptr_dev, col_dev, d, d, nnz,
                                  static_cast<int32_t*>(flags)));
  int32_t hf[2] = {0, 0};
  HIPCHK(ctx, hipMemcpyAsync(hf, flags, sizeof hf, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (hf[0])
    return fail(ctx, MLCT_EINVAL, "invalid CSR structure (flags 0x%x: 1 rowptr[0]!=0, 2 decreasing rowptr, 4 rowptr[d]!=nnz, 8 column out of range)", hf[0]);
  mlct_op* op = new (std::nothrow) mlct_op();
  if (!op) return fail(ctx, MLCT_ENOMEM, "out of host memory");
  op->ctx = ctx;
  op->device = ctx->device;
  op->kind = OP_CSR;
  op->d = d;
  op->csr.nnz = nnz;
  op->csr.nrows = op->csr.ncols = d;
  op->csr.rowptr = rowptr_dev;
  op->csr.col = col_dev;
  op->csr.val = dtype == MLCT_DT_F32 ? static_cast<const float*>(val_dev) : nullptr;
  op->dtype = dtype;
  op->csr.max_row_nnz = hf[1];
  op->tuned_groups = std::max(0, tune_lookup(ctx, tune_key(op, MLCT_FP32, 64), kCsrGroupCands));
  mlct_status st = MLCT_OK;
  if (op->csr.max_row_nnz <= 5 && nnz > 0) {
    // the bandwidth decides whether two steps fit one launch
    hipError_t e = hipMemsetAsync(flags, 0, sizeof(int32_t), ctx->stream);
    if (e == hipSuccess)
      e = launch_csr_bandwidth(ctx->stream, rowptr_dev, col_dev, d, static_cast<int32_t*>(flags));
    int32_t bw = -1;
    if (e == hipSuccess) e = hipMemcpyAsync(&bw, flags, sizeof bw, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      mlct_op_destroy(op);
      return fail(ctx, MLCT_EDEVICE, "bandwidth: %s", hipGetErrorString(e));
    }
    op->csr.bandwidth = bw;
  }
  if (op->csr.max_row_nnz > kHubLen) st = build_hubs(ctx, op->csr, &op->hub_mem);
  if (st == MLCT_OK) st = refresh_bands(ctx, op);
  if (st != MLCT_OK) {
    mlct_op_destroy(op);
    return st;
  }
  *out = op;
  return MLCT_OK;
}

mlct_status mlct_op_gram_csr(mlct_ctx* ctx, int64_t rows, int64_t cols, int64_t nnz,
                             const int32_t* rowptr_dev, const int32_t* col_dev,
                             const float* val_dev, double lambda, mlct_op** out) {
  if (!ctx || !out) return MLCT_EINVAL;
  ctx->err.clear();
  if (rows < 1 || cols < 1 || rows > INT32_MAX || cols > INT32_MAX)
    return fail(ctx, MLCT_EINVAL, "bad shape %lld x %lld", (long long)rows, (long long)cols);
  if (nnz < 0 || nnz > INT32_MAX) return fail(ctx, MLCT_EINVAL, "bad nnz=%lld", (long long)nnz);
  if (!rowptr_dev || (nnz > 0 && !col_dev))
    return fail(ctx, MLCT_EINVAL, "rowptr/col must be device pointers");
  if (!(lambda >= 0.0) || !std::isfinite(lambda))
    return fail(ctx, MLCT_EINVAL, "lambda must be finite and >= 0");
  CHECK(set_device(ctx));
  hipStream_t s = ctx->stream;
  void* flags;
  CHECK(ws_get(ctx, WS_MISC, 64, &flags));
  HIPCHK(ctx, hipMemsetAsync(flags, 0, 2 * sizeof(int32_t), s));
  HIPCHK(ctx, launch_csr_validate(s, rowptr_dev, col_dev, rows, cols, nnz,
                                  static_cast<int32_t*>(flags)));
  int32_t hf[2] = {0, 0};
  HIPCHK(ctx, hipMemcpyAsync(hf, flags, sizeof hf, hipMemcpyDeviceToHost, s));
  CHECK(sync_stream(ctx));
  if (hf[0])
    return fail(ctx, MLCT_EINVAL, "invalid CSR structure of X (flags 0x%x)", hf[0]);
  // X^T by a stable counting sort on the host: entries of a column keep
  // their row order, so the transpose (and every sum over it) is fixed.
  std::vector<int32_t> rp(rows + 1), cl(nnz), rpt(cols + 1, 0), clt(nnz);
  std::vector<float> vl(val_dev ? nnz : 0), vlt(val_dev ? nnz : 0);
  HIPCHK(ctx, hipMemcpy(rp.data(), rowptr_dev, (rows + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (nnz > 0) {
    HIPCHK(ctx, hipMemcpy(cl.data(), col_dev, nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (val_dev)
      HIPCHK(ctx, hipMemcpy(vl.data(), val_dev, nnz * sizeof(float), hipMemcpyDeviceToHost));
  }
  for (int64_t e = 0; e < nnz; ++e) ++rpt[cl[e] + 1];
  int maxt = 0;
  for (int64_t j = 0; j < cols; ++j) {
    maxt = std::max(maxt, rpt[j + 1]);
    rpt[j + 1] += rpt[j];
  }
  {
    std::vector<int32_t> next(rpt.begin(), rpt.end() - 1);
    for (int64_t i = 0; i < rows; ++i)
      for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int32_t k = next[cl[e]]++;
        clt[k] = (int32_t)i;
        if (val_dev) vlt[k] = vl[e];
      }
  }
  const size_t words = (size_t)(cols + 1) + nnz + (val_dev ? nnz : 0);
  void* mem = nullptr;
  if (hipMalloc(&mem, words * 4) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, MLCT_ENOMEM, "no memory for X^T");
  }
  int32_t* base = static_cast<int32_t*>(mem);
  hipError_t e1 = hipMemcpy(base, rpt.data(), (cols + 1) * 4, hipMemcpyHostToDevice);
  if (e1 == hipSuccess && nnz > 0) e1 = hipMemcpy(base + cols + 1, clt.data(), nnz * 4, hipMemcpyHostToDevice);
  if (e1 == hipSuccess && val_dev && nnz > 0)
    e1 = hipMemcpy(base + cols + 1 + nnz, vlt.data(), nnz * 4, hipMemcpyHostToDevice);
  if (e1 != hipSuccess) {
    (void)hipFree(mem);
    return fail(ctx, MLCT_EDEVICE, "upload of X^T: %s", hipGetErrorString(e1));
  }
  mlct_op* op = new (std::nothrow) mlct_op();
  if (!op) {
    (void)hipFree(mem);
    return fail(ctx, MLCT_ENOMEM, "out of host memory");
  }
  op->ctx = ctx;
  op->device = ctx->device;
  op->kind = OP_GRAM_CSR;
  op->d = cols;
  op->dtype = val_dev ? MLCT_DT_F32 : MLCT_DT_PATTERN;
  op->gram_lambda = lambda;
  op->gram_mem = mem;
  op->csrx.rowptr = rowptr_dev;
  op->csrx.col = col_dev;
  op->csrx.val = val_dev;
  op->csrx.nrows = rows;
  op->csrx.ncols = cols;
  op->csrx.nnz = nnz;
  op->csrx.max_row_nnz = hf[1];
  op->csr.rowptr = base;
  op->csr.col = base + cols + 1;
  op->csr.val = val_dev ? reinterpret_cast<const float*>(base + cols + 1 + nnz) : nullptr;
  op->csr.nrows = cols;
  op->csr.ncols = rows;
  op->csr.nnz = nnz;
  op->csr.max_row_nnz = maxt;
  op->tuned_groups = std::max(0, tune_lookup(ctx, tune_key(op, MLCT_FP32, 64), kCsrGroupCands));
  mlct_status st = MLCT_OK;
  if (op->csrx.max_row_nnz > kHubLen) st = build_hubs(ctx, op->csrx, &op->hubx_mem);
  if (st == MLCT_OK && op->csr.max_row_nnz > kHubLen) st = build_hubs(ctx, op->csr, &op->hub_mem);
  if (st == MLCT_OK) st = refresh_bands(ctx, op);
  if (st != MLCT_OK) {
    mlct_op_destroy(op);
    return st;
  }
  *out = op;
  return MLCT_OK;
}

mlct_status mlct_op_destroy(mlct_op* op) {
  if (!op) return MLCT_EINVAL;
  (void)hipSetDevice(op->device);
  void* owned[] = {op->owned,   op->split_hi, op->split_lo, op->pack_hi, op->pack_lo,
                   op->a32,     op->a64,      op->hub_mem,  op->hubx_mem, op->gram_mem,
                   op->band_mem};
  for (void* p : owned)
    if (p) (void)hipFree(p);
  delete op;
  return MLCT_OK;
}

mlct_status mlct_cheb_coeffs(mlct_ctx* ctx, mlct_func f, double a, double b, int32_t n,
                             double* c_out, double* log_scale_out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!c_out) return fail(ctx, MLCT_EINVAL, "c_out is NULL");
  if (n < 1 || n > kMaxDegree) return fail(ctx, MLCT_EINVAL, "degree must be in [1, %d]", kMaxDegree);
  CHECK(check_func(ctx, f, a, b));
  CHECK(set_device(ctx));
  void* c;
  CHECK(ws_get(ctx, WS_COEF, (size_t)(n + 2) * sizeof(double), &c));
  double* cd = static_cast<double*>(c);
  HIPCHK(ctx, launch_cheb_dct(ctx->stream, f.kind, f.power, a, b, n, cd, cd + n + 1));
  std::vector<double> h(n + 2);
  HIPCHK(ctx, hipMemcpyAsync(h.data(), cd, (n + 2) * sizeof(double), hipMemcpyDeviceToHost,
                             ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  std::memcpy(c_out, h.data(), (n + 1) * sizeof(double));
  if (log_scale_out) *log_scale_out = h[n + 1];
  return MLCT_OK;
}

mlct_status mlct_moments(mlct_ctx* ctx, const mlct_op* op, double a, double b, int32_t n,
                         const mlct_probes* probes, int32_t prec, int32_t mode,
                         double* mu_out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!op || !mu_out) return fail(ctx, MLCT_EINVAL, "op and mu_out are required");
  if (!finite_interval(a, b)) return fail(ctx, MLCT_EINVAL, "need finite a < b");
  if (n < 0 || n > kMaxDegree) return fail(ctx, MLCT_EINVAL, "degree must be in [0, %d]", kMaxDegree);
  CHECK(check_mode_prec(ctx, mode, prec));
  CHECK(check_probes(ctx, op, probes));
  CHECK(set_device(ctx));
  const double alpha = 2.0 / (b - a), beta = -(a + b) / (b - a);
  const int64_t ldmu = n + 1;
  void* mu;
  CHECK(ws_get(ctx, WS_MU, (size_t)probes->m * ldmu * sizeof(double), &mu));
  CHECK(reserve_block_ws(ctx, op, prec, mode, n,
                         probes->m < kDenseMaxBlock ? probes->m : kDenseMaxBlock));
  CHECK(run_probe_set(ctx, op, alpha, beta, n, mode, prec, probes, static_cast<double*>(mu), ldmu));
  HIPCHK(ctx, hipMemcpyAsync(mu_out, mu, (size_t)probes->m * ldmu * sizeof(double),
                             hipMemcpyDeviceToHost, ctx->stream));
  CHECK(sync_stream(ctx));
  return MLCT_OK;
}

mlct_status mlct_moments_noalloc(mlct_ctx* ctx, const mlct_op* op, double a, double b,
                                 int32_t n, const mlct_probes* probes, int32_t prec,
                                 int32_t mode, double* mu_dev) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!op || !mu_dev) return fail(ctx, MLCT_EINVAL, "op and mu_dev are required");
  if (op->kind != OP_CSR) return fail(ctx, MLCT_EUNSUPPORTED, "only CSR operators");
  if (prec != MLCT_FP32 && prec != MLCT_FP64)
    return fail(ctx, MLCT_EUNSUPPORTED, "precision must be MLCT_FP32 or MLCT_FP64");
  if (!finite_interval(a, b)) return fail(ctx, MLCT_EINVAL, "need finite a < b");
  if (n < 0 || n > kMaxDegree) return fail(ctx, MLCT_EINVAL, "degree must be in [0, %d]", kMaxDegree);
  CHECK(check_mode_prec(ctx, mode, prec));
  CHECK(check_probes(ctx, op, probes));
  // carve the block buffers out of the fixed scratch (256-byte aligned)
  const size_t tsz = prec == MLCT_FP64 ? 8 : 4;
  const CsrBlockSizes z = csr_block_sizes(op, tsz, mode, n);
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t need = 2 * up(z.v) + up(z.part) + up(z.dots) + up(z.hub);
  if (need > (size_t)MLCT_NOALLOC_SCRATCH_BYTES)
    return fail(ctx, MLCT_ENOMEM,
                "needs %zu bytes of scratch, more than the fixed %llu (fewer rows or a lower degree)",
                need, (unsigned long long)MLCT_NOALLOC_SCRATCH_BYTES);
  CHECK(set_device(ctx));
  char* base = static_cast<char*>(noalloc_scratch(ctx->device));
  if (!base) return fail(ctx, MLCT_EDEVICE, "no scratch address for device %d", ctx->device);
  CsrBlockBufs bb;
  bb.timed = false;
  bb.v0 = base;
  bb.v1 = base + up(z.v);
  bb.part = reinterpret_cast<double*>(base + 2 * up(z.v));
  bb.dots = reinterpret_cast<double*>(base + 2 * up(z.v) + up(z.part));
  bb.hub = z.hub ? base + 2 * up(z.v) + up(z.part) + up(z.dots) : nullptr;
  const double alpha = 2.0 / (b - a), beta = -(a + b) / (b - a);
  const int64_t ldmu = n + 1;
  for (int64_t p0 = 0; p0 < probes->m; p0 += kBlockProbes) {
    ProbeSrc src;
    src.seed = probes->seed;
    src.first_id = probes->first_id + p0;
    src.entries = probes->kind == MLCT_PROBE_EXPLICIT ? probes->entries_dev : nullptr;
    src.ld = probes->ld_entries;
    src.active = (int32_t)std::min<int64_t>(probes->m - p0, kBlockProbes);
    if (prec == MLCT_FP32)
      CHECK(run_block_csr_in<float>(ctx, op, alpha, beta, n, mode, src, mu_dev + p0 * ldmu, ldmu, bb));
    else
      CHECK(run_block_csr_in<double>(ctx, op, alpha, beta, n, mode, src, mu_dev + p0 * ldmu, ldmu, bb));
  }
  return MLCT_OK;
}

mlct_status mlct_estimate(mlct_ctx* ctx, const mlct_op* op, mlct_func f, double a, double b,
                          const mlct_levels* levels, uint64_t seed, int32_t prec, int32_t mode,
                          mlct_result* out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!op || !levels || !out) return fail(ctx, MLCT_EINVAL, "op, levels and out are required");
  const int32_t mode_flags = mode;
  const int interp = (mode & MLCT_LEVEL_INTERP) ? 1 : 0;
  const int exact_low = (mode & MLCT_EXACT_LOW) ? 1 : 0;
  mode &= ~(MLCT_LEVEL_INTERP | MLCT_EXACT_LOW);
  CHECK(check_mode_prec(ctx, mode, prec));
  if (std::isnan(a) && std::isnan(b)) {
    const int steps = op->d < 64 ? (int)op->d : 64;
    CHECK(mlct_bounds(ctx, op, steps, seed + kGamma, 0.01, &a, &b));
  }
  // A CSR operator too small to fill the device with one probe block per
  // launch (fewer than kSmallGroups workgroups per step) and without rows
  // longer than kHubLen runs its probe blocks in shared launches (the
  // batched path, whose results equal this function's bit for bit) when
  // there are at least kSharedBlocks of them; fewer gain less than the
  // batched path's set-up costs.  (Only below the batch's solo threshold,
  // from which the batched path would hand the operator back here.)
  if (op->kind == OP_CSR && prec == MLCT_FP32 && op->csr.hub_n == 0 &&
      op->d < ctx->batch_solo_rows &&
      (mode == MLCT_DIRECT || mode == MLCT_DOUBLING) && levels->L >= 1 &&
      levels->L <= MLCT_MAX_LEVELS && levels->m &&
      (uint64_t)op->d * 64 * 4 <= 0xFFFFFFFFull &&
      plan_csr(op->d, op->tuned_groups).ngroups < kSmallGroups) {
    int64_t blocks = 0;
    for (int k = 0; k < levels->L; ++k) blocks += (levels->m[k] + kBlockProbes - 1) / kBlockProbes;
    if (blocks >= kSharedBlocks) {
      const mlct_batch_item it{op, f, a, b, *levels, seed};
      return mlct_estimate_batch(ctx, 1, &it, prec, mode_flags, out);
    }
  }
  CHECK(check_func(ctx, f, a, b));
  const int L = levels->L;
  if (L < 1 || L > MLCT_MAX_LEVELS || !levels->degree || !levels->m)
    return fail(ctx, MLCT_EINVAL, "need 1..%d levels", MLCT_MAX_LEVELS);
  LevelDesc lv{};
  lv.L = L;
  lv.interp = interp;
  int64_t total = 0, mv = 0, pd = 0;
  for (int k = 0; k < L; ++k) {
    const int dk = levels->degree[k];
    if (dk < 0 || dk > kMaxDegree) return fail(ctx, MLCT_EINVAL, "level degree %d out of range", dk);
    if (k && dk <= levels->degree[k - 1]) return fail(ctx, MLCT_EINVAL, "level degrees must increase");
    if (levels->m[k] < 1) return fail(ctx, MLCT_EINVAL, "each level needs m_k >= 1");
    if (interp && dk < 1) return fail(ctx, MLCT_EINVAL, "separate interpolants need degrees >= 1");
    lv.degree[k] = dk;
    lv.m[k] = levels->m[k];
    lv.off[k] = total;
    total += levels->m[k];
    mv += levels->m[k] * (int64_t)(mode == MLCT_DOUBLING ? (dk + 1) / 2 : dk);
    pd += levels->m[k] * (int64_t)dk;
  }
  const int n = lv.degree[L - 1];
  if (n < 1) return fail(ctx, MLCT_EINVAL, "top degree must be >= 1");
  CHECK(set_device(ctx));
  const double alpha = 2.0 / (b - a), beta = -(a + b) / (b - a);
  if (exact_low) {
    if (op->kind == OP_GRAM_CSR || op->kind == OP_CALLBACK)
      return fail(ctx, MLCT_EUNSUPPORTED,
                  "MLCT_EXACT_LOW needs tr A and ||A||_F, not available for this operator");
    lv.jmin = 3;
    CHECK(low_traces(ctx, op, alpha, beta, lv.low_tr));
  }
  const int64_t ldmu = n + 1;
  const int ncoef = interp ? L : 1;
  lv.coef_stride = n + 1;
  void *mu, *coef, *qstat, *res;
  CHECK(ws_get(ctx, WS_MU, (size_t)total * ldmu * sizeof(double), &mu));
  CHECK(ws_get(ctx, WS_COEF, ((size_t)ncoef * (n + 1) + 1) * sizeof(double), &coef));
  CHECK(ws_get(ctx, WS_QSTAT, ((size_t)total + 3 * MLCT_MAX_LEVELS) * sizeof(double), &qstat));
  CHECK(ws_get(ctx, WS_RESULT, sizeof(mlct_result), &res));
  // Block workspace is taken before any launch so that growth never frees a
  // buffer in use.
  {
    int64_t maxm = 0;
    for (int k = 0; k < L; ++k) maxm = lv.m[k] > maxm ? lv.m[k] : maxm;
    CHECK(reserve_block_ws(ctx, op, prec, mode, n, maxm < kDenseMaxBlock ? maxm : kDenseMaxBlock));
  }
  double* cd = static_cast<double*>(coef);
  double* ls = cd + (size_t)ncoef * (n + 1);
  hipStream_t s = ctx->stream;
  if (!interp) {
    HIPCHK(ctx, launch_cheb_dct(s, f.kind, f.power, a, b, n, cd, ls));
  } else {
    for (int k = 0; k < L; ++k)
      HIPCHK(ctx, launch_cheb_dct(s, f.kind, f.power, a, b, lv.degree[k], cd + (size_t)k * (n + 1), ls));
  }
  double* mud = static_cast<double*>(mu);
  for (int k = 0; k < L; ++k) {
    mlct_probes pr{};
    pr.kind = MLCT_PROBE_RADEMACHER;
    pr.seed = seed;
    pr.first_id = lv.off[k];
    pr.m = lv.m[k];
    CHECK(run_probe_set(ctx, op, alpha, beta, lv.degree[k], mode, prec, &pr,
                        mud + lv.off[k] * ldmu, ldmu));
  }
  double* q = static_cast<double*>(qstat);
  HIPCHK(ctx, launch_level_combine(s, mud, ldmu, cd, ls, lv, q, q + total,
                                   static_cast<mlct_result*>(res)));
  mlct_result h;
  HIPCHK(ctx, hipMemcpyAsync(&h, res, sizeof h, hipMemcpyDeviceToHost, s));
  CHECK(sync_stream(ctx));
  if (!(h.max_moment_ratio <= 1.0 + 1e-3))
    return fail(ctx, MLCT_ESPECTRUM,
                "max |mu_j|/|z|^2 = %g > 1: the spectrum is not inside [a, b] = [%g, %g]",
                h.max_moment_ratio, a, b);
  h.matvecs = mv;
  h.probe_degrees = pd;
  h.interval_a = a;
  h.interval_b = b;
  if (prec == MLCT_BF16X3) h.flags |= MLCT_FLAG_BF16;
  *out = h;
  return MLCT_OK;
}

mlct_status mlct_op_dense(mlct_ctx* ctx, int64_t d, const void* A_dev, int64_t lda,
                          int32_t dtype, mlct_op** out) {
  if (!ctx || !out) return MLCT_EINVAL;
  ctx->err.clear();
  if (d < 1 || d > (int64_t)1 << 20) return fail(ctx, MLCT_EINVAL, "bad dimension d=%lld", (long long)d);
  if (!A_dev || lda < d) return fail(ctx, MLCT_EINVAL, "need a device matrix with lda >= d");
  if (dtype != MLCT_DT_F32 && dtype != MLCT_DT_F64)
    return fail(ctx, MLCT_EINVAL, "dense values must be float32 or float64");
  mlct_op* op = new (std::nothrow) mlct_op();
  if (!op) return fail(ctx, MLCT_ENOMEM, "out of host memory");
  op->ctx = ctx;
  op->device = ctx->device;
  op->kind = OP_DENSE;
  op->d = d;
  op->A = A_dev;
  op->lda = lda;
  op->dtype = dtype;
  *out = op;
  return MLCT_OK;
}

mlct_status mlct_op_callback(mlct_ctx* ctx, int64_t d, mlct_apply_fn apply, void* user,
                             mlct_op** out) {
  if (!ctx || !out) return MLCT_EINVAL;
  ctx->err.clear();
  if (!apply) return fail(ctx, MLCT_EINVAL, "apply function is required");
  if (d < 1 || d > ((int64_t)1 << 31) - 1) return fail(ctx, MLCT_EINVAL, "need 1 <= d < 2^31");
  mlct_op* op = new (std::nothrow) mlct_op();
  if (!op) return fail(ctx, MLCT_ENOMEM, "out of host memory");
  op->ctx = ctx;
  op->device = ctx->device;
  op->kind = OP_CALLBACK;
  op->d = d;
  op->dtype = MLCT_DT_F32;
  op->cb_apply = apply;
  op->cb_user = user;
  *out = op;
  return MLCT_OK;
}

mlct_status mlct_op_read_dense(mlct_ctx* ctx, const mlct_op* op, double* out_host) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!op || !out_host || (op->kind != OP_DENSE && op->kind != OP_GRAM))
    return fail(ctx, MLCT_EINVAL, "need a dense or Gram operator and an output array");
  CHECK(set_device(ctx));
  const void *a0, *a1;
  int64_t lda;
  CHECK(dense_operand(ctx, op, MLCT_FP64, &a0, &a1, &lda));
  HIPCHK(ctx, hipMemcpy2DAsync(out_host, op->d * sizeof(double), a0, lda * sizeof(double),
                               op->d * sizeof(double), op->d, hipMemcpyDeviceToHost, ctx->stream));
  return sync_stream(ctx);
}

mlct_status mlct_op_gram(mlct_ctx* ctx, int64_t rows, int64_t cols, const void* X_dev,
                         int64_t ldx, int32_t dtype, int32_t prec, mlct_op** out) {
  if (!ctx || !out) return MLCT_EINVAL;
  ctx->err.clear();
  if (rows < 1 || cols < 1 || cols > (int64_t)1 << 20 || ldx < cols || !X_dev)
    return fail(ctx, MLCT_EINVAL, "need rows, cols >= 1, ldx >= cols and a device X");
  if (dtype != MLCT_DT_F32) return fail(ctx, MLCT_EINVAL, "X must be float32");
  if (prec != MLCT_FP32) return fail(ctx, MLCT_EUNSUPPORTED, "the Gram matrix is formed in FP32");
  CHECK(set_device(ctx));
  void* G = nullptr;
  if (hipMalloc(&G, (size_t)cols * cols * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, MLCT_ENOMEM, "no memory for the %lld x %lld Gram matrix", (long long)cols,
                (long long)cols);
  }
  {
    LaunchTimer tm(ctx, MLCT_KERNEL_GRAM);
    hipError_t e = launch_gram(ctx->stream, static_cast<const float*>(X_dev), rows, cols, ldx,
                               static_cast<float*>(G));
    tm.done();
    if (e != hipSuccess) {
      (void)hipFree(G);
      return fail(ctx, MLCT_EDEVICE, "Gram kernel launch failed: %s", hipGetErrorString(e));
    }
  }
  mlct_status st = sync_stream(ctx);
  if (st != MLCT_OK) {
    (void)hipFree(G);
    return st;
  }
  mlct_op* op = new (std::nothrow) mlct_op();
  if (!op) {
    (void)hipFree(G);
    return fail(ctx, MLCT_ENOMEM, "out of host memory");
  }
  op->ctx = ctx;
  op->device = ctx->device;
  op->kind = OP_GRAM;
  op->d = cols;
  op->A = G;
  op->owned = G;
  op->lda = cols;
  op->dtype = MLCT_DT_F32;
  *out = op;
  return MLCT_OK;
}

mlct_status mlct_lanczos(mlct_ctx* ctx, const mlct_op* op, int32_t steps, uint64_t seed,
                         double rel_margin, double* alpha_out, double* beta_out,
                         int32_t* k_out, double* info_out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!op) return fail(ctx, MLCT_EINVAL, "op is required");
  if (op->kind == OP_CALLBACK)
    return fail(ctx, MLCT_EUNSUPPORTED,
                "no FP64 products through a callback operator: give the interval [a, b]");
  if (steps < 1 || steps > kLanczosMaxSteps)
    return fail(ctx, MLCT_EINVAL, "steps must be in [1, %d]", kLanczosMaxSteps);
  if (!(rel_margin >= 0.0) || !std::isfinite(rel_margin))
    return fail(ctx, MLCT_EINVAL, "rel_margin must be finite and >= 0");
  CHECK(set_device(ctx));
  const int64_t d = op->d;
  const void* a64 = nullptr;
  const void* unused;
  int64_t lda = 0;
  if (op->kind != OP_CSR && op->kind != OP_GRAM_CSR)
    CHECK(dense_operand(ctx, op, MLCT_FP64, &a64, &unused, &lda));
  const int64_t nb = (d + 255) / 256 < 1024 ? (d + 255) / 256 : 1024;
  const int64_t xrows = op->kind == OP_GRAM_CSR ? op->csrx.nrows : 0;
  const int64_t hubc = std::max(op->csr.hub_chunks, op->csrx.hub_chunks);
  void *q, *misc;
  CHECK(ws_get(ctx, WS_LANCZOS, ((size_t)(steps + 2) * d + xrows + hubc) * sizeof(double), &q));
  const size_t misc_bytes = sizeof(LanczosState) + (size_t)(kLanczosMaxSteps + 1) * nb * 8 +
                            (kLanczosMaxSteps + 1) * 8 + 64 * 8;
  CHECK(ws_get(ctx, WS_DENSE, misc_bytes, &misc));
  double* Q = static_cast<double*>(q);
  double* w = Q + (size_t)(steps + 1) * d;
  LanczosState* st = static_cast<LanczosState*>(misc);
  double* part = reinterpret_cast<double*>(st + 1);
  double* h = part + (size_t)(kLanczosMaxSteps + 1) * nb;
  double* out = h + kLanczosMaxSteps + 1;
  HIPCHK(ctx, launch_lanczos(ctx->stream, op, a64, lda, steps, seed, rel_margin, Q, w, h, part,
                             st, out, xrows ? w + d : nullptr, w + d + xrows));
  LanczosState hs;
  double ho[8];
  HIPCHK(ctx, hipMemcpyAsync(&hs, st, sizeof hs, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipMemcpyAsync(ho, out, sizeof ho, hipMemcpyDeviceToHost, ctx->stream));
  CHECK(sync_stream(ctx));
  if (!(std::isfinite(ho[0]) && std::isfinite(ho[1])))
    return fail(ctx, MLCT_ERANGE, "Lanczos produced a non-finite interval");
  if (alpha_out) std::memcpy(alpha_out, hs.alpha, hs.k * sizeof(double));
  if (beta_out) std::memcpy(beta_out, hs.beta, hs.k * sizeof(double));
  if (k_out) *k_out = hs.k;
  if (info_out) {
    info_out[0] = ho[2];
    info_out[1] = ho[3];
    info_out[2] = ho[4];
    info_out[3] = ho[5];
    info_out[4] = ho[0];
    info_out[5] = ho[1];
  }
  return MLCT_OK;
}

mlct_status mlct_bounds(mlct_ctx* ctx, const mlct_op* op, int32_t steps, uint64_t seed,
                        double rel_margin, double* a_out, double* b_out) {
  if (!ctx) return MLCT_EINVAL;
  if (!a_out || !b_out) return fail(ctx, MLCT_EINVAL, "a_out and b_out are required");
  double info[6];
  CHECK(mlct_lanczos(ctx, op, steps, seed, rel_margin, nullptr, nullptr, nullptr, info));
  *a_out = info[4];
  *b_out = info[5];
  // Gram operators are known to be >= lambda I (lambda = 0 for X^T X)
  if (op->kind == OP_GRAM && *a_out < 0.0) *a_out = 0.0;
  if (op->kind == OP_GRAM_CSR && *a_out < op->gram_lambda) *a_out = op->gram_lambda;
  return MLCT_OK;
}

mlct_status mlct_triangles(mlct_ctx* ctx, const mlct_op* op, int64_t m, uint64_t seed,
                           int64_t* w_out, mlct_tri_result* out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!op || !out) return fail(ctx, MLCT_EINVAL, "op and out are required");
  if (op->kind != OP_CSR || op->csr.val != nullptr)
    return fail(ctx, MLCT_EINVAL, "triangle counting needs a 0/1 pattern CSR operator");
  if (m < 1) return fail(ctx, MLCT_EINVAL, "need m >= 1 probes");
  // the packed signs are gathered through a buffer resource of 32-bit size
  if ((uint64_t)op->d * sizeof(uint64_t) > 0xFFFFFFFFull)
    return fail(ctx, MLCT_EUNSUPPORTED, "triangle counting supports at most 536,870,911 rows");
  CHECK(set_device(ctx));
  const CsrStepPlan plan = plan_csr(op->d, op->tuned_groups);
  void *z, *y, *part, *w, *res, *side = nullptr;
  CHECK(ws_get(ctx, WS_V0, (size_t)op->d * sizeof(uint64_t), &z));        // packed signs
  CHECK(ws_get(ctx, WS_V1, (size_t)op->d * kBlockProbes * sizeof(int16_t), &y));
  if (op->csr.hub_n > 0)
    CHECK(ws_get(ctx, WS_TRISIDE, (size_t)op->csr.hub_n * kBlockProbes * sizeof(int32_t), &side));
  CHECK(ws_get(ctx, WS_PART, (size_t)2 * plan.ngroups * kBlockProbes * sizeof(long long), &part));
  CHECK(ws_get(ctx, WS_TRI, (size_t)m * 3 * sizeof(long long), &w));
  CHECK(ws_get(ctx, WS_RESULT, sizeof(mlct_tri_result), &res));
  void* hub = nullptr;
  if (op->csr.hub_n > 0)
    CHECK(ws_get(ctx, WS_HUB, (size_t)op->csr.hub_chunks * kBlockProbes * sizeof(int32_t), &hub));
  hipStream_t s = ctx->stream;
  long long* P = static_cast<long long*>(part);
  long long* W = static_cast<long long*>(w);
  for (int64_t p0 = 0; p0 < m; p0 += kBlockProbes) {
    ProbeSrc src{};
    src.seed = seed;
    src.first_id = p0;
    src.active = (int32_t)((m - p0) < kBlockProbes ? (m - p0) : kBlockProbes);
    HIPCHK(ctx, launch_tri_init(s, op, src, plan, static_cast<uint64_t*>(z)));
    {
      LaunchTimer tm(ctx, MLCT_KERNEL_TRI_STEP);
      HIPCHK(ctx, launch_tri_step(s, op->csr, 1, plan, static_cast<uint64_t*>(z),
                                  static_cast<int16_t*>(y), static_cast<int32_t*>(side), hub, P));
      tm.done();
    }
    HIPCHK(ctx, launch_tri_reduce(s, P, plan.ngroups, src.active, 1, W, p0));
    {
      LaunchTimer tm(ctx, MLCT_KERNEL_TRI_STEP);
      HIPCHK(ctx, launch_tri_step(s, op->csr, 2, plan, nullptr, static_cast<int16_t*>(y),
                                  static_cast<int32_t*>(side), hub, P));
      tm.done();
    }
    HIPCHK(ctx, launch_tri_reduce(s, P, plan.ngroups, src.active, 2, W, p0));
  }
  HIPCHK(ctx, launch_tri_cv(s, W, m, op->csr.nnz, static_cast<mlct_tri_result*>(res)));
  mlct_tri_result h;
  HIPCHK(ctx, hipMemcpyAsync(&h, res, sizeof h, hipMemcpyDeviceToHost, s));
  if (w_out)
    HIPCHK(ctx, hipMemcpyAsync(w_out, W, (size_t)m * 3 * sizeof(long long),
                               hipMemcpyDeviceToHost, s));
  CHECK(sync_stream(ctx));
  *out = h;
  return MLCT_OK;
}

}  // extern "C"

// ---- learned control-variate level ------------------------------------------
namespace {

constexpr uint64_t kMlpInitMix = 0xD1B54A32D192ED03ull;

size_t align8(size_t x) { return (x + 7) / 8 * 8; }

// Carves consecutive 8-byte-aligned regions out of one workspace slot.
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + off);
    off = align8(off + count * sizeof(T));
    return p;
  }
};

void mlp_free(mlct_mlp* m) {
  void* ps[] = {m->theta, m->adam_m, m->adam_v, m->wbf16, m->coef, m->val_mu};
  for (void* p : ps)
    if (p) (void)hipFree(p);
}

mlct_status mlp_malloc(mlct_ctx* ctx, void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(ctx, MLCT_ENOMEM, "hipMalloc(%zu) failed", bytes);
  }
  return MLCT_OK;
}

}  // namespace

extern "C" {

mlct_status mlct_learned_fit(mlct_ctx* ctx, const mlct_op* op, mlct_func f, double a, double b,
                             int32_t n_fine, int32_t n_cheap, int64_t m_pilot, uint64_t seed,
                             int32_t prec, const mlct_mlp_cfg* cfg, mlct_mlp** out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!op || !out) return fail(ctx, MLCT_EINVAL, "op and out are required");
  if (n_cheap < 1 || n_cheap >= kMlpMaxFeatures)
    return fail(ctx, MLCT_EINVAL, "n_cheap must be in [1, %d]", kMlpMaxFeatures - 1);
  if (n_fine <= n_cheap || n_fine > kMaxDegree)
    return fail(ctx, MLCT_EINVAL, "need n_cheap < n_fine <= %d", kMaxDegree);
  if (m_pilot < 8 || m_pilot > (1 << 24)) return fail(ctx, MLCT_EINVAL, "need 8 <= m_pilot <= 2^24");
  CHECK(check_mode_prec(ctx, MLCT_DOUBLING, prec));
  const int epochs = cfg && cfg->epochs > 0 ? cfg->epochs : 2000;
  const float lr = cfg && cfg->lr > 0 ? cfg->lr : 1e-3f;
  const double frac = cfg && cfg->train_fraction > 0 && cfg->train_fraction <= 1 ? cfg->train_fraction : 0.75;
  const uint64_t init_seed = cfg && cfg->init_seed ? cfg->init_seed : (seed ^ kMlpInitMix);
  if (epochs > (1 << 20)) return fail(ctx, MLCT_EINVAL, "too many epochs");
  CHECK(set_device(ctx));
  if (std::isnan(a) && std::isnan(b)) {
    const int steps = op->d < 64 ? (int)op->d : 64;
    CHECK(mlct_bounds(ctx, op, steps, seed + kGamma, 0.01, &a, &b));
  }
  CHECK(check_func(ctx, f, a, b));
  const int F = n_cheap + 1, P = mlp_nparams(F);
  const int64_t ldmu = n_fine + 1;
  const int64_t ntrain = std::max<int64_t>(2, (int64_t)(frac * m_pilot));
  const int64_t nval = m_pilot - ntrain;
  if (nval < 2)
    return fail(ctx, MLCT_EINVAL,
                "train_fraction %g of %lld pilot probes leaves %lld held out (need >= 2)", frac,
                (long long)m_pilot, (long long)nval);
  // workspace (all before the first launch)
  void *mu, *scratch;
  CHECK(ws_get(ctx, WS_MU, (size_t)m_pilot * ldmu * sizeof(double), &mu));
  CHECK(reserve_block_ws(ctx, op, prec, MLCT_DOUBLING, n_fine,
                         m_pilot < kDenseMaxBlock ? m_pilot : kDenseMaxBlock));
  const size_t sbytes = align8(m_pilot * 8) + align8(ntrain * F * 4) + align8(ntrain * 4) +
                        align8((size_t)kMlpWaves * P * 4) + align8(kMlpWaves * 4) +
                        align8((size_t)epochs * 4) + align8(kMlpStats * 8) + align8(nval * 8) + 128 + 256;
  CHECK(ws_get(ctx, WS_MLP, sbytes, &scratch));
  Carver cv{static_cast<char*>(scratch)};
  double* q = cv.take<double>(m_pilot);
  float* X = cv.take<float>(ntrain * F);
  float* y = cv.take<float>(ntrain);
  float* part = cv.take<float>((size_t)kMlpWaves * P);
  float* loss_part = cv.take<float>(kMlpWaves);
  float* loss_hist = cv.take<float>(epochs);
  double* stats = cv.take<double>(kMlpStats);
  double* gval = cv.take<double>(nval > 0 ? nval : 1);
  double* comb = cv.take<double>(8);

  mlct_mlp* m = new (std::nothrow) mlct_mlp();
  if (!m) return fail(ctx, MLCT_ENOMEM, "out of host memory");
  m->device = ctx->device;
  m->F = F;
  m->n_cheap = n_cheap;
  m->n_fine = n_fine;
  m->func_kind = f.kind;
  m->power = f.power;
  m->a = a;
  m->b = b;
  m->prec = prec;
  m->seed = seed;
  m->m_pilot = m_pilot;
  m->ntrain = ntrain;
  mlct_status st = MLCT_OK;
#define MLP_TRY(expr)          \
  do {                         \
    st = (expr);               \
    if (st != MLCT_OK) {       \
      mlp_free(m);             \
      delete m;                \
      return st;               \
    }                          \
  } while (0)
#define MLP_HIP(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      mlp_free(m);                                                                          \
      delete m;                                                                             \
      return fail(ctx, MLCT_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
    }                                                                                       \
  } while (0)
  MLP_TRY(mlp_malloc(ctx, (void**)&m->theta, (size_t)P * 4));
  MLP_TRY(mlp_malloc(ctx, (void**)&m->adam_m, (size_t)P * 4));
  MLP_TRY(mlp_malloc(ctx, (void**)&m->adam_v, (size_t)P * 4));
  MLP_TRY(mlp_malloc(ctx, &m->wbf16, (size_t)P * 2));
  MLP_TRY(mlp_malloc(ctx, (void**)&m->coef, (size_t)(n_fine + 2) * 8));
  MLP_TRY(mlp_malloc(ctx, (void**)&m->val_mu, (size_t)nval * ldmu * 8));
  m->nval = nval;
  hipStream_t s = ctx->stream;
  const double alpha = 2.0 / (b - a), beta = -(a + b) / (b - a);
  // pilot moments and fine-level values q
  mlct_probes pr{};
  pr.kind = MLCT_PROBE_RADEMACHER;
  pr.seed = seed;
  pr.first_id = 0;
  pr.m = m_pilot;
  MLP_TRY(run_probe_set(ctx, op, alpha, beta, n_fine, MLCT_DOUBLING, prec, &pr,
                        static_cast<double*>(mu), ldmu));
  MLP_HIP(launch_cheb_dct(s, f.kind, f.power, a, b, n_fine, m->coef, m->coef + n_fine + 1));
  MLP_HIP(launch_qvals(s, static_cast<double*>(mu), ldmu, m->coef, n_fine, m_pilot, q));
  // training set and training
  MLP_HIP(launch_mlp_prepare(s, static_cast<double*>(mu), ldmu, q, m->coef, F, (int)ntrain, X, y,
                             stats));
  MLP_HIP(launch_mlp_init(s, m->theta, m->adam_m, m->adam_v, F, init_seed));
  for (int t = 1; t <= epochs; ++t) {
    MLP_HIP(launch_mlp_grad(s, m->theta, F, X, y, (int)ntrain, kMlpWaves, part, loss_part));
    MLP_HIP(launch_mlp_adam(s, m->theta, m->adam_m, m->adam_v, part, kMlpWaves, F, t, lr,
                            loss_part, (int)ntrain, loss_hist));
  }
  MLP_HIP(launch_mlp_to_bf16(s, m->theta, F, m->wbf16));
  double hstats[kMlpStats];
  MLP_HIP(hipMemcpyAsync(hstats, stats, sizeof hstats, hipMemcpyDeviceToHost, s));
  MLP_TRY(sync_stream(ctx));
  m->ybar = hstats[0];
  m->ysd = hstats[1];
  m->aff.ybar = hstats[0];
  m->aff.ysd = hstats[1];
  for (int f = 0; f < 16; ++f) {
    m->aff.xmean[f] = hstats[2 + f];
    m->aff.xsd[f] = hstats[2 + 16 + f];
    m->aff.lin[f] = hstats[2 + 32 + f];
  }
  // held-out pilot probes: variance of q and of q - g; their moments stay
  // with the handle for the level planner
  {
    const double* muv = static_cast<double*>(mu) + ntrain * ldmu;
    MLP_HIP(hipMemcpyAsync(m->val_mu, muv, (size_t)nval * ldmu * 8, hipMemcpyDeviceToDevice, s));
    MLP_HIP(launch_mlp_infer(s, m->wbf16, F, m->coef, muv, ldmu, nval, m->aff, gval));
    MLP_HIP(launch_mlp_combine(s, q + ntrain, nval, q + ntrain, gval, nval, comb));
    MLP_HIP(launch_mlp_combine(s, gval, nval, gval, nullptr, 0, comb + 4));
    double hc[8];
    MLP_HIP(hipMemcpyAsync(hc, comb, sizeof hc, hipMemcpyDeviceToHost, s));
    MLP_TRY(sync_stream(ctx));
    m->var_g = hc[5];
    m->var_q = hc[1];
    m->var_resid = hc[3];
    m->mean_resid = hc[2];
    m->fallback = !(hc[3] < hc[1]);
  }
  m->loss_hist.resize(epochs);
  MLP_HIP(hipMemcpyAsync(m->loss_hist.data(), loss_hist, (size_t)epochs * 4,
                         hipMemcpyDeviceToHost, s));
  MLP_TRY(sync_stream(ctx));
  double ls = 0.0;
  MLP_HIP(hipMemcpy(&ls, m->coef + n_fine + 1, 8, hipMemcpyDeviceToHost));
  m->log_scale = ls;
#undef MLP_TRY
#undef MLP_HIP
  *out = m;
  return MLCT_OK;
}

}  // extern "C"

namespace {

// The learned multilevel chain: level k of L holds S(deg[k]) - S(deg[k-1])
// over its own probes (ids off_k .. off_k + m_k - 1 of seed), where
// S(l) = z^T p^{(l)} z (the truncation of the degree-n_fine interpolant),
// S(n_cheap) = g and S(-1) = 0.  The levels telescope to S(n_fine).
mlct_status learned_chain(mlct_ctx* ctx, const mlct_op* op, const mlct_mlp* m, int L,
                          const int32_t* deg, const int64_t* mk, uint64_t seed,
                          mlct_result* out) {
  if (!op || !m || !out || !deg || !mk) return fail(ctx, MLCT_EINVAL, "op, mlp, levels and out are required");
  if (L < 1 || L > MLCT_MAX_LEVELS) return fail(ctx, MLCT_EINVAL, "need 1 <= L <= %d", MLCT_MAX_LEVELS);
  if (seed == m->seed) return fail(ctx, MLCT_EINVAL, "use a seed different from the pilot's");
  if (op->d <= 0) return fail(ctx, MLCT_EINVAL, "empty operator");
  const int nc = m->n_cheap, n = m->n_fine, F = m->F;
  int64_t mmax = 0, rows_deg = 0;
  for (int k = 0; k < L; ++k) {
    if (deg[k] < 0 || (k && deg[k] <= deg[k - 1]))
      return fail(ctx, MLCT_EINVAL, "level degrees must increase from 0");
    if (mk[k] < 1 || mk[k] > ((int64_t)1 << 32)) return fail(ctx, MLCT_EINVAL, "level %d: need 1 <= m <= 2^32", k);
    mmax = std::max(mmax, mk[k]);
    rows_deg = std::max(rows_deg, mk[k] * (deg[k] + 1));
  }
  if (deg[L - 1] != n) return fail(ctx, MLCT_EINVAL, "the top level must be the fit's n_fine = %d", n);
  CHECK(set_device(ctx));
  const double alpha = 2.0 / (m->b - m->a), beta = -(m->a + m->b) / (m->b - m->a);
  void *mu, *scratch;
  CHECK(ws_get(ctx, WS_MU, (size_t)rows_deg * 8, &mu));
  CHECK(reserve_block_ws(ctx, op, m->prec, MLCT_DOUBLING, n, mmax < kDenseMaxBlock ? mmax : kDenseMaxBlock));
  CHECK(ws_get(ctx, WS_MLP, 2 * align8(mmax * 8) + align8((size_t)5 * L * 8) + 64, &scratch));
  Carver cv{static_cast<char*>(scratch)};
  double* g = cv.take<double>(mmax);
  double* q = cv.take<double>(mmax);
  double* st = cv.take<double>((size_t)5 * L);  // per level: 4 combine outputs + ratio
  hipStream_t s = ctx->stream;
  double* mud = static_cast<double*>(mu);
  int64_t off = 0;
  for (int k = 0; k < L; ++k) {
    const int hi = deg[k], lo = k ? deg[k - 1] : -1;
    mlct_probes pr{};
    pr.kind = MLCT_PROBE_RADEMACHER;
    pr.seed = seed;
    pr.first_id = off;
    pr.m = mk[k];
    CHECK(run_probe_set(ctx, op, alpha, beta, hi, MLCT_DOUBLING, m->prec, &pr, mud, hi + 1));
    const bool with_g = hi == nc || lo == nc;  // hi >= nc then, so mu holds F columns
    if (with_g) HIPCHK(ctx, launch_mlp_infer(s, m->wbf16, F, m->coef, mud, hi + 1, mk[k], m->aff, g));
    HIPCHK(ctx, launch_learned_level_q(s, mud, hi + 1, m->coef, hi, lo, nc, with_g ? g : nullptr,
                                       mk[k], q));
    HIPCHK(ctx, launch_mlp_combine(s, nullptr, 0, q, nullptr, mk[k], st + 4 * k));
    HIPCHK(ctx, launch_moment_ratio(s, mud, hi + 1, hi + 1, mk[k], st + 4 * L + k));
    off += mk[k];
  }
  std::vector<double> h((size_t)5 * L);
  HIPCHK(ctx, hipMemcpyAsync(h.data(), st, h.size() * 8, hipMemcpyDeviceToHost, s));
  CHECK(sync_stream(ctx));
  mlct_result r{};
  double mr = 0.0;
  for (int k = 0; k < L; ++k) {
    r.value += h[4 * k + 2];
    r.level_mean[k] = h[4 * k + 2];
    r.level_var[k] = h[4 * k + 3];
    if (mk[k] > 1) r.est_var += h[4 * k + 3] / (double)mk[k];
    else r.flags |= MLCT_FLAG_FEW_SAMPLES;
    r.matvecs += mk[k] * ((deg[k] + 1) / 2);
    r.probe_degrees += mk[k] * deg[k];
    mr = std::max(mr, h[4 * L + k]);
  }
  if (r.flags & MLCT_FLAG_FEW_SAMPLES) r.est_var = NAN;
  if (!(mr <= 1.0 + 1e-3))
    return fail(ctx, MLCT_ESPECTRUM,
                "max |mu_j|/|z|^2 = %g > 1: the spectrum is not inside [a, b] = [%g, %g]", mr,
                m->a, m->b);
  r.max_moment_ratio = mr;
  r.log_scale = m->log_scale;
  r.estimate = r.value * std::exp(r.log_scale);
  r.interval_a = m->a;
  r.interval_b = m->b;
  if (m->prec == MLCT_BF16X3) r.flags |= MLCT_FLAG_BF16;
  if (!std::isfinite(r.estimate)) r.flags |= MLCT_FLAG_OVERFLOW;
  *out = r;
  return MLCT_OK;
}

}  // namespace

extern "C" {

mlct_status mlct_estimate_learned(mlct_ctx* ctx, const mlct_op* op, const mlct_mlp* m,
                                  int64_t M0, int64_t M1, uint64_t seed, mlct_result* out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!op || !m || !out) return fail(ctx, MLCT_EINVAL, "op, mlp and out are required");
  const bool learned = !m->fallback;
  if (M1 < 2 || (learned && M0 < 2)) return fail(ctx, MLCT_EINVAL, "need M0, M1 >= 2");
  if (learned) {
    const int32_t deg[2] = {m->n_cheap, m->n_fine};
    const int64_t mk[2] = {M0, M1};
    return learned_chain(ctx, op, m, 2, deg, mk, seed, out);
  }
  // plain fallback: q over ids [0, M1), reported as level 1
  const int32_t deg[1] = {m->n_fine};
  const int64_t mk[1] = {M1};
  mlct_result r;
  CHECK(learned_chain(ctx, op, m, 1, deg, mk, seed, &r));
  r.level_mean[1] = r.level_mean[0];
  r.level_var[1] = r.level_var[0];
  r.level_mean[0] = r.level_var[0] = 0.0;
  r.flags |= MLCT_FLAG_LEARNED_FALLBACK;
  *out = r;
  return MLCT_OK;
}

mlct_status mlct_estimate_learned_ml(mlct_ctx* ctx, const mlct_op* op, const mlct_mlp* m,
                                     const mlct_levels* levels, uint64_t seed,
                                     mlct_result* out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!levels) return fail(ctx, MLCT_EINVAL, "levels are required");
  return learned_chain(ctx, op, m, levels->L, levels->degree, levels->m, seed, out);
}

mlct_status mlct_learned_eval(mlct_ctx* ctx, const mlct_op* op, const mlct_mlp* m,
                              const mlct_probes* probes, int32_t fine, double* g_out,
                              double* q_out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!op || !m || !probes || !g_out) return fail(ctx, MLCT_EINVAL, "op, mlp, probes and g_out are required");
  if (fine != 0 && fine != 1) return fail(ctx, MLCT_EINVAL, "fine must be 0 or 1");
  if (!fine && q_out) return fail(ctx, MLCT_EINVAL, "q_out needs fine = 1");
  CHECK(check_probes(ctx, op, probes));
  CHECK(set_device(ctx));
  const int deg = fine ? m->n_fine : m->n_cheap;
  const int64_t rows = probes->m, ld = deg + 1;
  const double alpha = 2.0 / (m->b - m->a), beta = -(m->a + m->b) / (m->b - m->a);
  void *mu, *scratch;
  CHECK(ws_get(ctx, WS_MU, (size_t)rows * ld * 8, &mu));
  CHECK(reserve_block_ws(ctx, op, m->prec, MLCT_DOUBLING, deg, rows < kDenseMaxBlock ? rows : kDenseMaxBlock));
  CHECK(ws_get(ctx, WS_MLP, 2 * align8(rows * 8) + 64, &scratch));
  Carver cv{static_cast<char*>(scratch)};
  double* g = cv.take<double>(rows);
  double* q = cv.take<double>(rows);
  double* ratio = cv.take<double>(1);
  hipStream_t s = ctx->stream;
  double* mud = static_cast<double*>(mu);
  CHECK(run_probe_set(ctx, op, alpha, beta, deg, MLCT_DOUBLING, m->prec, probes, mud, ld));
  HIPCHK(ctx, launch_mlp_infer(s, m->wbf16, m->F, m->coef, mud, ld, rows, m->aff, g));
  if (fine) HIPCHK(ctx, launch_qvals(s, mud, ld, m->coef, deg, rows, q));
  HIPCHK(ctx, launch_moment_ratio(s, mud, ld, deg + 1, rows, ratio));
  double mr = 0.0;
  HIPCHK(ctx, hipMemcpyAsync(&mr, ratio, 8, hipMemcpyDeviceToHost, s));
  CHECK(sync_stream(ctx));
  if (!(mr <= 1.0 + 1e-3))
    return fail(ctx, MLCT_ESPECTRUM,
                "max |mu_j|/|z|^2 = %g > 1: the spectrum is not inside [a, b] = [%g, %g]", mr,
                m->a, m->b);
  HIPCHK(ctx, hipMemcpy(g_out, g, (size_t)rows * 8, hipMemcpyDeviceToHost));
  if (q_out) HIPCHK(ctx, hipMemcpy(q_out, q, (size_t)rows * 8, hipMemcpyDeviceToHost));
  return MLCT_OK;
}

mlct_status mlct_mlp_info_get(const mlct_mlp* m, mlct_mlp_info* out) {
  if (!m || !out) return MLCT_EINVAL;
  out->var_q = m->var_q;
  out->var_resid = m->var_resid;
  out->mean_resid = m->mean_resid;
  out->var_g = m->var_g;
  out->ybar = m->ybar;
  out->ysd = m->ysd;
  for (int f = 0; f < 16; ++f) {
    out->x_mean[f] = m->aff.xmean[f];
    out->x_sd[f] = m->aff.xsd[f];
    out->lin[f] = m->aff.lin[f];
  }
  out->final_loss = m->loss_hist.empty() ? NAN : m->loss_hist.back();
  out->fallback = m->fallback;
  out->n_features = m->F;
  out->n_cheap = m->n_cheap;
  out->n_fine = m->n_fine;
  out->ntrain = m->ntrain;
  out->nval = m->m_pilot - m->ntrain;
  out->nparams = mlp_nparams(m->F);
  return MLCT_OK;
}

mlct_status mlct_mlp_loss_history(const mlct_mlp* m, float* out, int32_t max, int32_t* n_out) {
  if (!m || (!out && max > 0)) return MLCT_EINVAL;
  const int32_t n = std::min<int32_t>(max, (int32_t)m->loss_hist.size());
  if (n > 0) std::memcpy(out, m->loss_hist.data(), (size_t)n * 4);
  if (n_out) *n_out = (int32_t)m->loss_hist.size();
  return MLCT_OK;
}

mlct_status mlct_mlp_weights(mlct_ctx* ctx, mlct_mlp* m, float* get_out, const float* set_in) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!m) return fail(ctx, MLCT_EINVAL, "mlp is required");
  CHECK(set_device(ctx));
  const int P = mlp_nparams(m->F);
  if (set_in) {
    HIPCHK(ctx, hipMemcpyAsync(m->theta, set_in, (size_t)P * 4, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, launch_mlp_to_bf16(ctx->stream, m->theta, m->F, m->wbf16));
  }
  if (get_out)
    HIPCHK(ctx, hipMemcpyAsync(get_out, m->theta, (size_t)P * 4, hipMemcpyDeviceToHost, ctx->stream));
  return sync_stream(ctx);
}

mlct_status mlct_mlp_grad(mlct_ctx* ctx, const mlct_mlp* m, const float* X, const float* y,
                          int32_t N, float* grad_out, float* loss_out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!m || !X || !y || !grad_out || N < 1) return fail(ctx, MLCT_EINVAL, "bad arguments");
  CHECK(set_device(ctx));
  const int F = m->F, P = mlp_nparams(F);
  void* scratch;
  CHECK(ws_get(ctx, WS_MLP, align8((size_t)N * F * 4) + align8((size_t)N * 4) +
                                align8((size_t)kMlpWaves * P * 4) + align8(kMlpWaves * 4) +
                                align8((size_t)P * 4) + 64, &scratch));
  Carver cv{static_cast<char*>(scratch)};
  float* dX = cv.take<float>((size_t)N * F);
  float* dy = cv.take<float>(N);
  float* part = cv.take<float>((size_t)kMlpWaves * P);
  float* lp = cv.take<float>(kMlpWaves);
  float* g = cv.take<float>(P);
  float* loss = cv.take<float>(2);
  hipStream_t s = ctx->stream;
  HIPCHK(ctx, hipMemcpyAsync(dX, X, (size_t)N * F * 4, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemcpyAsync(dy, y, (size_t)N * 4, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, launch_mlp_grad(s, m->theta, F, dX, dy, N, kMlpWaves, part, lp));
  HIPCHK(ctx, launch_mlp_gradsum(s, part, kMlpWaves, F, lp, N, g, loss));
  HIPCHK(ctx, hipMemcpyAsync(grad_out, g, (size_t)P * 4, hipMemcpyDeviceToHost, s));
  float hl = 0.f;
  HIPCHK(ctx, hipMemcpyAsync(&hl, loss, 4, hipMemcpyDeviceToHost, s));
  CHECK(sync_stream(ctx));
  if (loss_out) *loss_out = hl;
  return MLCT_OK;
}

mlct_status mlct_mlp_destroy(mlct_mlp* m) {
  if (!m) return MLCT_EINVAL;
  (void)hipSetDevice(m->device);
  mlp_free(m);
  delete m;
  return MLCT_OK;
}

}  // extern "C"

// ---- batched estimates --------------------------------------------------------
namespace {

struct HostBlock {
  int item, level;
  int64_t first_id;
  int active, degree, steps;
  int variant;  // index into the variant list
};

}  // namespace

extern "C" mlct_status mlct_estimate_batch(mlct_ctx* ctx, int32_t nitems,
                                           const mlct_batch_item* items, int32_t prec,
                                           int32_t mode, mlct_result* outs) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (nitems < 1 || !items || !outs) return fail(ctx, MLCT_EINVAL, "need items and outs");
  const int interp = (mode & MLCT_LEVEL_INTERP) ? 1 : 0;
  const int exact_low = (mode & MLCT_EXACT_LOW) ? 1 : 0;
  if ((mode & MLCT_BATCH_PERSISTENT) && (mode & MLCT_BATCH_LOCKSTEP))
    return fail(ctx, MLCT_EINVAL, "MLCT_BATCH_PERSISTENT and MLCT_BATCH_LOCKSTEP exclude each other");
  const int persistent = (mode & MLCT_BATCH_PERSISTENT) ? 1
                         : (mode & MLCT_BATCH_LOCKSTEP) ? 0
                                                        : ctx->batch_persistent;
  const int32_t item_mode = mode & ~(MLCT_BATCH_PERSISTENT | MLCT_BATCH_LOCKSTEP);
  const int32_t batch_mode = mode;
  mode &= ~(MLCT_LEVEL_INTERP | MLCT_EXACT_LOW | MLCT_BATCH_PERSISTENT | MLCT_BATCH_LOCKSTEP);
  if (prec != MLCT_FP32) return fail(ctx, MLCT_EUNSUPPORTED, "batched estimates run in MLCT_FP32");
  CHECK(check_mode_prec(ctx, mode, prec));
  // Operators with batch_solo_rows rows or more fill the device on their
  // own with the tuned single-matrix step kernel: they run as single
  // estimates, the others share launches.  The results are those of single
  // calls either way.
  {
    std::vector<int> solo, rest;
    for (int i = 0; i < nitems; ++i)
      (items[i].op && items[i].op->kind == OP_CSR && items[i].op->d >= ctx->batch_solo_rows ? solo
                                                                                            : rest)
          .push_back(i);
    if (!solo.empty()) {
      // an item whose moments leave the spectrum's range still gets its
      // result, and the call reports MLCT_ESPECTRUM after all items ran
      std::string spectrum_msg;
      for (int i : solo) {
        const mlct_batch_item& it = items[i];
        const mlct_status st = mlct_estimate(ctx, it.op, it.f, it.a, it.b, &it.levels, it.seed,
                                             prec, item_mode, &outs[i]);
        if (st == MLCT_ESPECTRUM && spectrum_msg.empty()) {
          spectrum_msg = "item " + std::to_string(i) + ": " + ctx->err;
        } else if (st != MLCT_OK && st != MLCT_ESPECTRUM) {
          const std::string msg = ctx->err;
          return fail(ctx, st, "item %d: %s", i, msg.c_str());
        }
      }
      if (!rest.empty()) {
        std::vector<mlct_batch_item> sub;
        for (int i : rest) sub.push_back(items[i]);
        std::vector<mlct_result> subo(rest.size());
        const mlct_status st = mlct_estimate_batch(ctx, (int32_t)sub.size(), sub.data(), prec,
                                                   batch_mode, subo.data());
        if (st != MLCT_OK && st != MLCT_ESPECTRUM) return st;
        for (size_t k = 0; k < rest.size(); ++k) outs[rest[k]] = subo[k];
        if (st == MLCT_ESPECTRUM && spectrum_msg.empty()) spectrum_msg = ctx->err;
      }
      if (!spectrum_msg.empty()) return fail(ctx, MLCT_ESPECTRUM, "%s", spectrum_msg.c_str());
      ctx->err.clear();
      return MLCT_OK;
    }
  }
  // ---- validate items, build level descriptors and blocks ----
  std::vector<LevelDesc> lvs(nitems);
  std::vector<int64_t> totals(nitems);
  std::vector<int> top(nitems);
  std::vector<HostBlock> blocks;
  std::vector<std::pair<bool, int>> variants;  // (pattern, maxnz class)
  for (int i = 0; i < nitems; ++i) {
    const mlct_batch_item& it = items[i];
    if (!it.op || it.op->kind != OP_CSR) return fail(ctx, MLCT_EINVAL, "item %d: need a CSR operator", i);
    if ((uint64_t)it.op->d * 64 * 4 > 0xFFFFFFFFull)
      return fail(ctx, MLCT_EUNSUPPORTED, "item %d: operator too large for a batch", i);
    CHECK(check_func(ctx, it.f, it.a, it.b));
    const int L = it.levels.L;
    if (L < 1 || L > MLCT_MAX_LEVELS || !it.levels.degree || !it.levels.m)
      return fail(ctx, MLCT_EINVAL, "item %d: need 1..%d levels", i, MLCT_MAX_LEVELS);
    LevelDesc& lv = lvs[i];
    lv = LevelDesc{};
    lv.L = L;
    lv.interp = interp;
    int64_t tot = 0;
    for (int k = 0; k < L; ++k) {
      const int dk = it.levels.degree[k];
      if (dk < 0 || dk > kMaxDegree || (k && dk <= it.levels.degree[k - 1]) || it.levels.m[k] < 1 ||
          (interp && dk < 1))
        return fail(ctx, MLCT_EINVAL, "item %d: bad levels", i);
      lv.degree[k] = dk;
      lv.m[k] = it.levels.m[k];
      lv.off[k] = tot;
      tot += it.levels.m[k];
    }
    totals[i] = tot;
    top[i] = lv.degree[L - 1];
    if (top[i] < 1) return fail(ctx, MLCT_EINVAL, "item %d: top degree must be >= 1", i);
    lv.coef_stride = top[i] + 1;
    if (exact_low) {
      CHECK(set_device(ctx));
      lv.jmin = 3;
      const double al = 2.0 / (it.b - it.a), be = -(it.a + it.b) / (it.b - it.a);
      CHECK(low_traces(ctx, it.op, al, be, lv.low_tr));
    }
    const bool pat = it.op->csr.val == nullptr;
    // row-length class: straight-line gathers up to 4 / 5 / 8 entries, or
    // 9 = longer rows present (the generic loop)
    const int mxr = it.op->csr.max_row_nnz;
    const int mz = mxr <= 4 ? 4 : mxr <= 5 ? 5 : mxr <= 8 ? 8 : 9;
    int var = -1;
    for (size_t v = 0; v < variants.size(); ++v)
      if (variants[v] == std::make_pair(pat, mz)) var = (int)v;
    if (var < 0) {
      variants.push_back({pat, mz});
      var = (int)variants.size() - 1;
    }
    for (int k = 0; k < L; ++k)
      for (int64_t p0 = 0; p0 < lv.m[k]; p0 += kBlockProbes) {
        HostBlock hb;
        hb.item = i;
        hb.level = k;
        hb.first_id = lv.off[k] + p0;
        hb.active = (int)std::min<int64_t>(kBlockProbes, lv.m[k] - p0);
        hb.degree = lv.degree[k];
        hb.steps = mode == MLCT_DOUBLING ? (hb.degree + 1) / 2 : hb.degree;
        hb.variant = var;
        blocks.push_back(hb);
      }
  }
  // variant-major, then by steps descending: the blocks still running at
  // step s are a prefix of their variant's table
  std::stable_sort(blocks.begin(), blocks.end(), [](const HostBlock& x, const HostBlock& y) {
    return x.variant != y.variant ? x.variant < y.variant : x.steps > y.steps;
  });
  CHECK(set_device(ctx));
  // ---- workspace sizes ----
  const size_t nb = blocks.size();
  size_t bytes = align8(nb * sizeof(BatchBlock)) + 256;
  for (const HostBlock& hb : blocks) {
    const int64_t d = items[hb.item].op->d;
    const CsrStepPlan plan = plan_csr(d, items[hb.item].op->tuned_groups);
    bytes += 2 * align8((size_t)d * 64 * 4);
    bytes += align8((size_t)(hb.steps + 1) * 2 * plan.ngroups * 64 * 8);
    bytes += align8((size_t)(hb.steps + 1) * 2 * 64 * 8);
  }
  for (int i = 0; i < nitems; ++i) {
    const int ncoef = interp ? lvs[i].L : 1;
    bytes += align8((size_t)totals[i] * (top[i] + 1) * 8);           // moment table
    bytes += align8(((size_t)ncoef * (top[i] + 1) + 1) * 8);         // coefficients + log-scale
    bytes += align8(((size_t)totals[i] + 3 * MLCT_MAX_LEVELS) * 8);  // Q and level stats
  }
  bytes += align8((size_t)nitems * sizeof(mlct_result));
  bytes += 2 * align8(8 * nb * sizeof(int32_t)) + align8(8 * nb * sizeof(int64_t));  // XCD layout
  int max_steps = 0;
  for (const HostBlock& hb : blocks) max_steps = std::max(max_steps, hb.steps);
  // persistent launch: running slots per (step, XCD) of every variant, the
  // blocks' barrier counters and the abort flag
  bytes += align8((size_t)variants.size() * (max_steps + 1) * 8 * sizeof(int64_t)) +
           align8((nb + 1) * sizeof(int32_t)) + 64;
  void* ws;
  CHECK(ws_get(ctx, WS_BATCH, bytes, &ws));
  Carver cv{static_cast<char*>(ws)};
  BatchBlock* dtab = cv.take<BatchBlock>(nb);
  std::vector<BatchBlock> tab(nb);
  std::vector<double*> dots(nb);
  for (size_t bi = 0; bi < nb; ++bi) {
    const HostBlock& hb = blocks[bi];
    const mlct_op* op = items[hb.item].op;
    const CsrStepPlan plan = plan_csr(op->d, op->tuned_groups);
    BatchBlock& B = tab[bi];
    B.rowptr = op->csr.rowptr;
    B.col = op->csr.col;
    B.val = op->csr.val;
    B.d = op->d;
    B.nnz = op->csr.nnz;
    B.v0 = cv.take<float>((size_t)op->d * 64);
    B.v1 = cv.take<float>((size_t)op->d * 64);
    B.part = cv.take<double>((size_t)(hb.steps + 1) * 2 * plan.ngroups * 64);
    dots[bi] = cv.take<double>((size_t)(hb.steps + 1) * 2 * 64);
    B.src = ProbeSrc{items[hb.item].seed, hb.first_id, nullptr, 0, hb.active};
    const double a = items[hb.item].a, b = items[hb.item].b;
    B.alpha = 2.0 / (b - a);
    B.beta = -(a + b) / (b - a);
    B.steps = hb.steps;
    B.ngroups = plan.ngroups;
    B.rows_per_group = plan.rows_per_group;
    B.band = op->csr.band && op->csr.band_groups == plan.ngroups ? op->csr.band : nullptr;
  }
  std::vector<double*> mu(nitems), coef(nitems), qst(nitems);
  for (int i = 0; i < nitems; ++i) {
    const int ncoef = interp ? lvs[i].L : 1;
    mu[i] = cv.take<double>((size_t)totals[i] * (top[i] + 1));
    coef[i] = cv.take<double>((size_t)ncoef * (top[i] + 1) + 1);
    qst[i] = cv.take<double>((size_t)totals[i] + 3 * MLCT_MAX_LEVELS);
  }
  mlct_result* dres = cv.take<mlct_result>(nitems);
  int32_t* dxblk = cv.take<int32_t>(8 * nb);
  int32_t* dxg0 = cv.take<int32_t>(8 * nb);
  int64_t* dxbase = cv.take<int64_t>(8 * nb);
  int64_t* dslots = cv.take<int64_t>(variants.size() * (max_steps + 1) * 8);
  int32_t* dcnt = cv.take<int32_t>(nb + 1);
  int32_t* dabort = cv.take<int32_t>(2);
  // group bases per variant table (each variant's blocks are contiguous)
  std::vector<size_t> vstart(variants.size() + 1, nb);
  for (size_t bi = nb; bi-- > 0;) vstart[blocks[bi].variant] = bi;
  vstart[variants.size()] = nb;
  for (size_t v = 0; v < variants.size(); ++v) {
    int64_t base = 0;
    for (size_t bi = vstart[v]; bi < vstart[v + 1]; ++bi) {
      tab[bi].group_base = base;
      base += tab[bi].ngroups;
    }
  }
  // XCD layout of each variant's blocks for the step launches: blocks go
  // whole to one XCD, tier by tier (a tier = blocks with the same step
  // count, larger first), each to the XCD with the least work so far, so
  // the blocks running at any step are balanced and a prefix of each XCD's
  // list.  A tier with fewer than four blocks per XCD has each block cut
  // into eight pieces of ngroups / 8 bands, one per XCD, so that the XCDs
  // stay evenly loaded.  Work of a block = nnz + kBandRowCost d.  Entries
  // of variant v sit at 8 vstart[v] onwards (at most eight per block).
  struct XEntry {
    int32_t blk, g0, cnt;
  };
  std::vector<int32_t> xblk(8 * nb), xg0(8 * nb), xcnt(8 * nb);
  std::vector<int64_t> xbase(8 * nb);
  std::vector<std::array<size_t, 9>> xoff(variants.size());
  std::vector<std::vector<int>> xsteps(variants.size());  // step count of each entry
  for (size_t v = 0; v < variants.size(); ++v) {
    const size_t b0 = vstart[v], b1 = vstart[v + 1];
    std::vector<XEntry> lists[8];
    double load[8] = {};
    auto work = [&](size_t bi) { return (double)tab[bi].nnz + kBandRowCost * (double)tab[bi].d; };
    for (size_t i = b0; i < b1;) {
      size_t j = i;
      while (j < b1 && tab[j].steps == tab[i].steps) ++j;
      if (j - i < 32) {
        for (size_t bi = i; bi < j; ++bi) {
          const int32_t per = tab[bi].ngroups / 8;
          for (int x = 0; x < 8; ++x) {
            lists[x].push_back({(int32_t)(bi - b0), x * per, per});
            load[x] += work(bi) / 8;
          }
        }
      } else {
        std::vector<size_t> ord;
        for (size_t bi = i; bi < j; ++bi) ord.push_back(bi);
        std::stable_sort(ord.begin(), ord.end(),
                         [&](size_t a, size_t b) { return work(a) > work(b); });
        for (size_t bi : ord) {
          const int x = (int)(std::min_element(load, load + 8) - load);
          lists[x].push_back({(int32_t)(bi - b0), 0, tab[bi].ngroups});
          load[x] += work(bi);
        }
      }
      i = j;
    }
    size_t pos = 8 * b0;
    for (int x = 0; x < 8; ++x) {
      xoff[v][x] = pos - 8 * b0;
      int64_t sb = 0;
      for (const XEntry& e : lists[x]) {
        xblk[pos] = e.blk;
        xg0[pos] = e.g0;
        xcnt[pos] = e.cnt;
        xbase[pos] = sb;
        xsteps[v].push_back(tab[b0 + e.blk].steps);
        sb += e.cnt;
        ++pos;
      }
    }
    xoff[v][8] = pos - 8 * b0;
  }
  hipStream_t s = ctx->stream;
  HIPCHK(ctx, hipMemcpyAsync(dtab, tab.data(), nb * sizeof(BatchBlock), hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemcpyAsync(dxblk, xblk.data(), 8 * nb * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemcpyAsync(dxg0, xg0.data(), 8 * nb * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemcpyAsync(dxbase, xbase.data(), 8 * nb * sizeof(int64_t), hipMemcpyHostToDevice, s));
  // ---- coefficients ----
  for (int i = 0; i < nitems; ++i) {
    const int n = top[i];
    double* ls = coef[i] + (size_t)(interp ? lvs[i].L : 1) * (n + 1);
    if (!interp) {
      HIPCHK(ctx, launch_cheb_dct(s, items[i].f.kind, items[i].f.power, items[i].a, items[i].b, n,
                                  coef[i], ls));
    } else {
      for (int k = 0; k < lvs[i].L; ++k)
        HIPCHK(ctx, launch_cheb_dct(s, items[i].f.kind, items[i].f.power, items[i].a, items[i].b,
                                    lvs[i].degree[k], coef[i] + (size_t)k * (n + 1), ls));
    }
  }
  // ---- probes, steps ----
  for (size_t v = 0; v < variants.size(); ++v) {
    const size_t b0 = vstart[v], cnt = vstart[v + 1] - b0;
    if (!cnt) continue;
    const int64_t groups = tab[b0 + cnt - 1].group_base + tab[b0 + cnt - 1].ngroups;
    HIPCHK(ctx, launch_probe_init_batched(s, dtab + b0, (int)cnt, groups));
  }
  // running slots of XCD x at step st (the running entries are a prefix of
  // each XCD's list)
  auto running = [&](size_t v, int st, XcdLaunch& xl) {
    const size_t x0 = 8 * vstart[v];
    int64_t most = 0;
    for (int x = 0; x < 8; ++x) {
      const size_t e0 = xoff[v][x], e1 = xoff[v][x + 1];
      size_t e = e0;
      while (e < e1 && xsteps[v][e] >= st) ++e;
      xl.first[x] = (int)e0;
      xl.count[x] = (int)(e - e0);
      xl.slots[x] = e > e0 ? xbase[x0 + e - 1] + xcnt[x0 + e - 1] : 0;
      most = std::max(most, xl.slots[x]);
    }
    return most;
  };
  if (persistent) {
    // step 1 as a batched launch, then steps 2 .. S in one cooperative
    // launch per row-length variant; the grid is what can be resident at
    // once, so every block barrier's wait ends
    for (size_t v = 0; v < variants.size(); ++v) {
      XcdLaunch xl;
      const int64_t most = running(v, 1, xl);
      if (!most) continue;
      const size_t x0 = 8 * vstart[v];
      LaunchTimer tm(ctx, MLCT_KERNEL_BATCH_STEP);
      HIPCHK(ctx, launch_csr_step_batched(s, dtab + vstart[v], dxblk + x0, dxg0 + x0,
                                          dxbase + x0, xl, 8 * most, 1, variants[v].first,
                                          variants[v].second, 0));
      tm.done();
    }
    std::vector<int64_t> hslots(variants.size() * (max_steps + 1) * 8, 0);
    std::vector<int> per(variants.size(), 0);
    for (size_t v = 0; v < variants.size(); ++v) {
      per[v] = csr_batch_persistent_per_xcd(variants[v].first, variants[v].second,
                                            mode == MLCT_DOUBLING ? 0 : 1);
      if (per[v] < 1) return fail(ctx, MLCT_EDEVICE, "no resident grid for the persistent batch");
      for (int st = 1; st <= max_steps; ++st) {
        XcdLaunch xl;
        running(v, st, xl);
        for (int x = 0; x < 8; ++x) hslots[(v * (max_steps + 1) + st) * 8 + x] = xl.slots[x];
      }
    }
    HIPCHK(ctx, hipMemcpyAsync(dslots, hslots.data(), hslots.size() * sizeof(int64_t),
                               hipMemcpyHostToDevice, s));
    for (size_t v = 0; v < variants.size(); ++v) {
      const size_t b0 = vstart[v], x0 = 8 * b0, cnt = vstart[v + 1] - b0;
      if (!cnt) continue;
      XcdLaunch xl;
      for (int x = 0; x < 8; ++x) {
        xl.first[x] = (int)xoff[v][x];
        xl.count[x] = (int)(xoff[v][x + 1] - xoff[v][x]);
        xl.slots[x] = 0;
      }
      int vsteps = 0;
      for (size_t bi = b0; bi < b0 + cnt; ++bi) vsteps = std::max(vsteps, tab[bi].steps);
      if (vsteps < 2) continue;
      LaunchTimer tm(ctx, MLCT_KERNEL_BATCH_STEP);
      HIPCHK(ctx, launch_csr_batch_persistent(
                      s, dtab + b0, dxblk + x0, dxg0 + x0, dxbase + x0, xl, vsteps,
                      dslots + v * (max_steps + 1) * 8, dcnt, (int)cnt, dabort, per[v],
                      variants[v].first, variants[v].second, mode == MLCT_DOUBLING ? 0 : 1,
                      200000000LL));
      tm.done();
    }
  }
  for (int st = 1; st <= max_steps && !persistent; ++st) {
    for (size_t v = 0; v < variants.size(); ++v) {
      const size_t b0 = vstart[v];
      XcdLaunch xl;
      int64_t most = 0;
      const size_t x0 = 8 * b0;  // this variant's entries
      for (int x = 0; x < 8; ++x) {
        const size_t e0 = xoff[v][x], e1 = xoff[v][x + 1];
        size_t e = e0;
        while (e < e1 && xsteps[v][e] >= st) ++e;
        xl.first[x] = (int)e0;
        xl.count[x] = (int)(e - e0);
        // slots of the running entries: up to the end of the last of them
        const int64_t slots = e > e0 ? xbase[x0 + e - 1] + xcnt[x0 + e - 1] : 0;
        xl.slots[x] = slots;
        most = std::max(most, slots);
      }
      if (!most) continue;
      const int zmode = (st == 1 || mode == MLCT_DOUBLING) ? 0 : 1;
      LaunchTimer tm(ctx, MLCT_KERNEL_BATCH_STEP);
      HIPCHK(ctx, launch_csr_step_batched(s, dtab + b0, dxblk + x0, dxg0 + x0, dxbase + x0, xl,
                                          8 * most, st, variants[v].first, variants[v].second,
                                          zmode));
      tm.done();
    }
  }
  // ---- moments, levels ----
  for (size_t bi = 0; bi < nb; ++bi) {
    const HostBlock& hb = blocks[bi];
    HIPCHK(ctx, launch_reduce_partials(s, tab[bi].part, hb.steps + 1, 2, tab[bi].ngroups, 64,
                                       dots[bi]));
    HIPCHK(ctx, launch_assemble_moments(s, dots[bi], hb.steps + 1, 64, hb.active, mode, hb.degree,
                                        mu[hb.item] + hb.first_id * (top[hb.item] + 1),
                                        top[hb.item] + 1));
  }
  for (int i = 0; i < nitems; ++i) {
    const int n = top[i];
    double* ls = coef[i] + (size_t)(interp ? lvs[i].L : 1) * (n + 1);
    HIPCHK(ctx, launch_level_combine(s, mu[i], n + 1, coef[i], ls, lvs[i], qst[i],
                                     qst[i] + totals[i], dres + i));
  }
  std::vector<mlct_result> h(nitems);
  HIPCHK(ctx, hipMemcpyAsync(h.data(), dres, nitems * sizeof(mlct_result), hipMemcpyDeviceToHost, s));
  int32_t aborted = 0;
  if (persistent)
    HIPCHK(ctx, hipMemcpyAsync(&aborted, dabort, sizeof aborted, hipMemcpyDeviceToHost, s));
  CHECK(sync_stream(ctx));
  if (aborted)
    return fail(ctx, MLCT_EDEVICE, "a block barrier of the persistent batch timed out");
  bool escaped = false;
  for (int i = 0; i < nitems; ++i) {
    int64_t mv = 0, pd = 0;
    for (int k = 0; k < lvs[i].L; ++k) {
      const int dk = lvs[i].degree[k];
      mv += lvs[i].m[k] * (int64_t)(mode == MLCT_DOUBLING ? (dk + 1) / 2 : dk);
      pd += lvs[i].m[k] * (int64_t)dk;
    }
    h[i].matvecs = mv;
    h[i].probe_degrees = pd;
    h[i].interval_a = items[i].a;
    h[i].interval_b = items[i].b;
    if (!(h[i].max_moment_ratio <= 1.0 + 1e-3)) escaped = true;
    outs[i] = h[i];
  }
  if (escaped) return fail(ctx, MLCT_ESPECTRUM, "an item's spectrum is not inside its [a, b]");
  return MLCT_OK;
}

// Autotuner for batches: times the two launch forms on the caller's batch
// and keeps the faster for later batches of this context.
extern "C" mlct_status mlct_autotune_batch(mlct_ctx* ctx, int32_t nitems,
                                           const mlct_batch_item* items, int32_t prec,
                                           int32_t mode, int32_t* choice_out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (nitems < 1 || !items) return fail(ctx, MLCT_EINVAL, "need items");
  mode &= ~(MLCT_BATCH_PERSISTENT | MLCT_BATCH_LOCKSTEP);
  std::vector<mlct_result> outs(nitems);
  CHECK(set_device(ctx));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  struct Ev {
    hipEvent_t* a;
    hipEvent_t* b;
    ~Ev() {
      if (*a) (void)hipEventDestroy(*a);
      if (*b) (void)hipEventDestroy(*b);
    }
  } ev{&e0, &e1};
  HIPCHK(ctx, hipEventCreate(&e0));
  HIPCHK(ctx, hipEventCreate(&e1));
  float best[2] = {1e30f, 1e30f};
  const int32_t flag[2] = {MLCT_BATCH_LOCKSTEP, MLCT_BATCH_PERSISTENT};
  for (int rep = 0; rep < 3; ++rep)
    for (int f = 0; f < 2; ++f) {
      HIPCHK(ctx, hipEventRecord(e0, ctx->stream));
      CHECK(mlct_estimate_batch(ctx, nitems, items, prec, mode | flag[f], outs.data()));
      HIPCHK(ctx, hipEventRecord(e1, ctx->stream));
      HIPCHK(ctx, hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(ctx, hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) best[f] = std::min(best[f], ms);  // the first round warms up
    }
  ctx->batch_persistent = best[1] < best[0] ? 1 : 0;
  if (choice_out) *choice_out = ctx->batch_persistent;
  return MLCT_OK;
}

// ---- stochastic Lanczos quadrature -------------------------------------------
namespace {

// SLQ values of the src.active probes of one block (CSR operators, FP64),
// into q_dev[0..active).
mlct_status run_block_slq(mlct_ctx* ctx, const mlct_op* op, int k, mlct_func f,
                          double log_scale, ProbeSrc src, double* q_dev) {
  const CsrStepPlan plan = plan_csr(op->d, op->tuned_groups);
  const size_t vbytes = (size_t)op->d * kBlockProbes * sizeof(double);
  void *w0, *w1, *w, *part, *dots, *hub = nullptr;
  CHECK(ws_get(ctx, WS_V0, vbytes, &w0));
  CHECK(ws_get(ctx, WS_V1, vbytes, &w1));
  const size_t state_off = (vbytes + 255) & ~(size_t)255;
  const size_t scratch_off = (state_off + sizeof(SlqState) + 255) & ~(size_t)255;
  CHECK(ws_get(ctx, WS_SLQ, scratch_off + (size_t)3 * k * 64 * sizeof(double), &w));
  CHECK(ws_get(ctx, WS_PART, (size_t)2 * plan.ngroups * kBlockProbes * sizeof(double), &part));
  CHECK(ws_get(ctx, WS_MISC, (size_t)2 * kBlockProbes * sizeof(double), &dots));
  if (op->csr.hub_n > 0)
    CHECK(ws_get(ctx, WS_HUB, (size_t)op->csr.hub_chunks * kBlockProbes * sizeof(double), &hub));
  double* W0 = static_cast<double*>(w0);
  double* W1 = static_cast<double*>(w1);
  double* U = static_cast<double*>(w);
  SlqState* st = reinterpret_cast<SlqState*>(static_cast<char*>(w) + state_off);
  double* scratch = reinterpret_cast<double*>(static_cast<char*>(w) + scratch_off);
  double* P = static_cast<double*>(part);
  double* D = static_cast<double*>(dots);
  hipStream_t s = ctx->stream;
  HIPCHK(ctx, launch_probe_init<double>(s, W1, op->d, src, plan, P));
  HIPCHK(ctx, launch_reduce_partials(s, P, 1, 2, plan.ngroups, kBlockProbes, D));
  HIPCHK(ctx, hipMemsetAsync(W0, 0, vbytes, s));
  HIPCHK(ctx, launch_slq_init(s, D, k, st));
  for (int j = 0; j < k; ++j) {
    LaunchTimer tm(ctx, MLCT_KERNEL_SLQ_SPMM);
    HIPCHK(ctx, launch_slq_spmm(s, op->csr, W1, U, st->s_cur, plan, hub, P));
    tm.done();
    HIPCHK(ctx, launch_reduce_partials(s, P, 1, 2, plan.ngroups, kBlockProbes, D));
    HIPCHK(ctx, launch_slq_alpha(s, D, j, st));
    LaunchTimer tu(ctx, MLCT_KERNEL_SLQ_UPDATE);
    HIPCHK(ctx, launch_slq_update(s, U, W1, W0, st, j, op->d, plan, P));
    tu.done();
    HIPCHK(ctx, launch_reduce_partials(s, P, 1, 2, plan.ngroups, kBlockProbes, D));
    HIPCHK(ctx, launch_slq_beta(s, D, j, k, st));
    double* t = W0;  // rotate: w_{j-1} <- w_j <- w_{j+1}
    W0 = W1;
    W1 = U;
    U = t;
  }
  HIPCHK(ctx, launch_slq_quadrature(s, st, k, f.kind, f.power, log_scale, src.active, scratch,
                                    q_dev));
  return MLCT_OK;
}

mlct_status check_slq_args(mlct_ctx* ctx, const mlct_op* op, int k) {
  if (!op) return fail(ctx, MLCT_EINVAL, "op is required");
  if (op->kind != OP_CSR)
    return fail(ctx, MLCT_EUNSUPPORTED, "Lanczos quadrature runs on CSR operators");
  if (k < 1 || k > kSlqMaxSteps)
    return fail(ctx, MLCT_EINVAL, "Lanczos steps must be in [1, %d]", kSlqMaxSteps);
  return MLCT_OK;
}

}  // namespace

extern "C" mlct_status mlct_slq_quadforms(mlct_ctx* ctx, const mlct_op* op, mlct_func f,
                                          int32_t k, const mlct_probes* probes,
                                          double* q_out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  CHECK(check_slq_args(ctx, op, k));
  if (!q_out) return fail(ctx, MLCT_EINVAL, "q_out is required");
  if (f.kind < MLCT_LOG || f.kind > MLCT_POW) return fail(ctx, MLCT_EINVAL, "unknown function");
  CHECK(check_probes(ctx, op, probes));
  CHECK(set_device(ctx));
  void* q;
  CHECK(ws_get(ctx, WS_SLQQ, (size_t)probes->m * sizeof(double), &q));
  double* qd = static_cast<double*>(q);
  for (int64_t p0 = 0; p0 < probes->m; p0 += kBlockProbes) {
    ProbeSrc src;
    src.seed = probes->seed;
    src.first_id = probes->first_id + p0;
    src.entries = probes->kind == MLCT_PROBE_EXPLICIT ? probes->entries_dev : nullptr;
    src.ld = probes->ld_entries;
    src.active = (int32_t)std::min<int64_t>(kBlockProbes, probes->m - p0);
    CHECK(run_block_slq(ctx, op, k, f, 0.0, src, qd + p0));
  }
  HIPCHK(ctx, hipMemcpyAsync(q_out, qd, (size_t)probes->m * sizeof(double),
                             hipMemcpyDeviceToHost, ctx->stream));
  return sync_stream(ctx);
}

extern "C" mlct_status mlct_estimate_slq(mlct_ctx* ctx, const mlct_op* op, mlct_func f, double a,
                                         double b, int32_t cheb_degree, int64_t m0, int32_t k,
                                         int64_t m1, uint64_t seed, int32_t prec, int32_t mode,
                                         mlct_result* out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  CHECK(check_slq_args(ctx, op, k));
  if (!out) return fail(ctx, MLCT_EINVAL, "out is required");
  if (m0 < 1 || m1 < 1) return fail(ctx, MLCT_EINVAL, "both levels need samples");
  if (cheb_degree < 1 || cheb_degree > kMaxDegree)
    return fail(ctx, MLCT_EINVAL, "Chebyshev degree must be in [1, %d]", kMaxDegree);
  CHECK(check_mode_prec(ctx, mode, prec));
  if (std::isnan(a) && std::isnan(b)) {
    const int steps = op->d < 64 ? (int)op->d : 64;
    CHECK(mlct_bounds(ctx, op, steps, seed + kGamma, 0.01, &a, &b));
  }
  CHECK(check_func(ctx, f, a, b));
  CHECK(set_device(ctx));
  const int n = cheb_degree;
  const int64_t ldmu = n + 1, total = m0 + m1;
  void *mu, *coef, *q, *res;
  CHECK(ws_get(ctx, WS_MU, (size_t)total * ldmu * sizeof(double), &mu));
  CHECK(ws_get(ctx, WS_COEF, (size_t)(n + 2) * sizeof(double), &coef));
  CHECK(ws_get(ctx, WS_SLQQ, (size_t)m1 * sizeof(double), &q));
  CHECK(ws_get(ctx, WS_RESULT, sizeof(mlct_result), &res));
  CHECK(reserve_block_ws(ctx, op, prec, mode, n, kBlockProbes));
  double* cd = static_cast<double*>(coef);
  hipStream_t s = ctx->stream;
  HIPCHK(ctx, launch_cheb_dct(s, f.kind, f.power, a, b, n, cd, cd + n + 1));
  const double alpha = 2.0 / (b - a), beta = -(a + b) / (b - a);
  const double ls = f.kind == MLCT_EXP ? 0.5 * (a + b) : 0.0;
  mlct_probes pr{};
  pr.kind = MLCT_PROBE_RADEMACHER;
  pr.seed = seed;
  pr.first_id = 0;
  pr.m = total;
  double* mud = static_cast<double*>(mu);
  CHECK(run_probe_set(ctx, op, alpha, beta, n, mode, prec, &pr, mud, ldmu));
  double* qd = static_cast<double*>(q);
  for (int64_t p0 = 0; p0 < m1; p0 += kBlockProbes) {
    ProbeSrc src{};
    src.seed = seed;
    src.first_id = m0 + p0;
    src.active = (int32_t)std::min<int64_t>(kBlockProbes, m1 - p0);
    CHECK(run_block_slq(ctx, op, k, f, ls, src, qd + p0));
  }
  HIPCHK(ctx, launch_slq_combine(s, mud, ldmu, cd, n, m0, m1, qd, ls,
                                 static_cast<mlct_result*>(res)));
  mlct_result h;
  HIPCHK(ctx, hipMemcpyAsync(&h, res, sizeof h, hipMemcpyDeviceToHost, s));
  CHECK(sync_stream(ctx));
  if (!(h.max_moment_ratio <= 1.0 + 1e-3))
    return fail(ctx, MLCT_ESPECTRUM,
                "max |mu_j|/|z|^2 = %g > 1: the spectrum is not inside [a, b] = [%g, %g]",
                h.max_moment_ratio, a, b);
  h.matvecs = total * (int64_t)(mode == MLCT_DOUBLING ? (n + 1) / 2 : n) + m1 * (int64_t)k;
  h.probe_degrees = total * (int64_t)n + m1 * (int64_t)k;
  h.interval_a = a;
  h.interval_b = b;
  *out = h;
  return MLCT_OK;
}

// ---- automatic level selection ----------------------------------------------
namespace {

// V, DP and plan on the device for a pilot table already on the device
// (mu rows of n+1 values, multiplied by coef when given).
mlct_status plan_on_device(mlct_ctx* ctx, const double* mu, int64_t ldmu, const double* coef,
                           int64_t m, int n, int mode, double target, int target_kind,
                           int64_t min_top, mlct_level_plan* out) {
  const size_t nS = (size_t)m * (n + 1), nV = (size_t)(n + 2) * (n + 1);
  void* w;
  const size_t nP = (size_t)MLCT_MAX_LEVELS * (n + 1);
  CHECK(ws_get(ctx, WS_PLAN,
               (nS + (n + 1) + nV) * sizeof(double) + sizeof(LevelPlanDev) + 256 +
                   nP * sizeof(int),
               &w));
  double* S = static_cast<double*>(w);
  double* mean = S + nS;
  double* V = mean + (n + 1);
  LevelPlanDev* pd = reinterpret_cast<LevelPlanDev*>(
      (reinterpret_cast<uintptr_t>(V + nV) + 255) & ~(uintptr_t)255);
  int* prevk = reinterpret_cast<int*>(pd + 1);
  hipStream_t s = ctx->stream;
  HIPCHK(ctx, launch_level_plan(s, mu, ldmu, coef, n, m, S, mean, V, mode == MLCT_DOUBLING ? 1 : 0,
                                target, target_kind == MLCT_TARGET_BUDGET ? 1 : 0, min_top, prevk,
                                pd));
  LevelPlanDev h;
  HIPCHK(ctx, hipMemcpyAsync(&h, pd, sizeof h, hipMemcpyDeviceToHost, s));
  CHECK(sync_stream(ctx));
  if (h.L > MLCT_MAX_LEVELS)
    return fail(ctx, MLCT_ERANGE, "the optimal plan has %d levels (at most %d are supported)", h.L,
                MLCT_MAX_LEVELS);
  mlct_level_plan r{};
  r.L = h.L;
  r.opt_total = h.opt_total;
  r.single_total = h.single_total;
  for (int k = 0; k < h.L; ++k) {
    r.degree[k] = h.degree[k];
    r.m[k] = h.m[k];
    r.var[k] = h.var[k];
    r.cost[k] = h.cost[k];
    r.m_real[k] = h.m_real[k];
    r.predicted_var += h.var[k] / (double)h.m[k];
    r.predicted_cost += (double)h.m[k] * h.cost[k];
  }
  *out = r;
  return MLCT_OK;
}

mlct_status check_plan_args(mlct_ctx* ctx, int64_t m, int n, int mode, double target, int kind,
                            const void* out) {
  if (!out) return fail(ctx, MLCT_EINVAL, "out is required");
  if (n < 1 || n > kMaxPlanDegree)
    return fail(ctx, MLCT_EINVAL, "plan degree must be in [1, %d]", kMaxPlanDegree);
  if (m < 2) return fail(ctx, MLCT_EINVAL, "a pilot needs at least 2 probes");
  if (mode != MLCT_DIRECT && mode != MLCT_DOUBLING)
    return fail(ctx, MLCT_EINVAL, "mode must be MLCT_DIRECT or MLCT_DOUBLING");
  if (kind != MLCT_TARGET_VARIANCE && kind != MLCT_TARGET_BUDGET)
    return fail(ctx, MLCT_EINVAL, "unknown target kind %d", kind);
  if (!(target > 0.0) || !std::isfinite(target))
    return fail(ctx, MLCT_EINVAL, "target must be positive and finite");
  return MLCT_OK;
}

}  // namespace

extern "C" mlct_status mlct_plan_levels(mlct_ctx* ctx, const double* terms, int64_t m_pilot,
                                        int32_t n, int32_t mode, double target,
                                        int32_t target_kind, int64_t min_top,
                                        mlct_level_plan* out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!terms) return fail(ctx, MLCT_EINVAL, "terms is required");
  CHECK(check_plan_args(ctx, m_pilot, n, mode, target, target_kind, out));
  CHECK(set_device(ctx));
  void* t;
  CHECK(ws_get(ctx, WS_MU, (size_t)m_pilot * (n + 1) * sizeof(double), &t));
  HIPCHK(ctx, hipMemcpyAsync(t, terms, (size_t)m_pilot * (n + 1) * sizeof(double),
                             hipMemcpyHostToDevice, ctx->stream));
  return plan_on_device(ctx, static_cast<const double*>(t), n + 1, nullptr, m_pilot, n, mode,
                        target, target_kind, min_top, out);
}

extern "C" mlct_status mlct_learned_plan(mlct_ctx* ctx, const mlct_mlp* m, double target,
                                         int32_t target_kind, mlct_level_plan* out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!m) return fail(ctx, MLCT_EINVAL, "mlp is required");
  const int n = m->n_fine;
  CHECK(check_plan_args(ctx, m->nval, n, MLCT_DOUBLING, target, target_kind, out));
  CHECK(set_device(ctx));
  void *t, *scratch;
  CHECK(ws_get(ctx, WS_MU, (size_t)m->nval * (n + 1) * sizeof(double), &t));
  CHECK(ws_get(ctx, WS_MLP, align8(m->nval * 8) + 64, &scratch));
  double* g = static_cast<double*>(scratch);
  hipStream_t s = ctx->stream;
  HIPCHK(ctx, launch_mlp_infer(s, m->wbf16, m->F, m->coef, m->val_mu, n + 1, m->nval, m->aff, g));
  HIPCHK(ctx, launch_learned_terms(s, m->val_mu, n + 1, m->coef, n, m->n_cheap, g, m->nval,
                                   static_cast<double*>(t)));
  return plan_on_device(ctx, static_cast<const double*>(t), n + 1, nullptr, m->nval, n,
                        MLCT_DOUBLING, target, target_kind, 0, out);
}

extern "C" mlct_status mlct_select_levels(mlct_ctx* ctx, const mlct_op* op, mlct_func f, double a,
                                          double b, int32_t n, int64_t m_pilot, uint64_t seed,
                                          int32_t prec, int32_t mode, double target,
                                          int32_t target_kind, mlct_level_plan* out,
                                          double* mu_out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!op) return fail(ctx, MLCT_EINVAL, "op is required");
  CHECK(check_plan_args(ctx, m_pilot, n, mode, target, target_kind, out));
  CHECK(check_mode_prec(ctx, mode, prec));
  if (std::isnan(a) && std::isnan(b)) {
    const int steps = op->d < 64 ? (int)op->d : 64;
    CHECK(mlct_bounds(ctx, op, steps, seed + kGamma, 0.01, &a, &b));
  }
  CHECK(check_func(ctx, f, a, b));
  CHECK(set_device(ctx));
  void *mu, *coef;
  CHECK(ws_get(ctx, WS_MU, (size_t)m_pilot * (n + 1) * sizeof(double), &mu));
  CHECK(ws_get(ctx, WS_COEF, (size_t)(n + 2) * sizeof(double), &coef));
  CHECK(reserve_block_ws(ctx, op, prec, mode, n, m_pilot < kDenseMaxBlock ? m_pilot : kDenseMaxBlock));
  double* cd = static_cast<double*>(coef);
  hipStream_t s = ctx->stream;
  HIPCHK(ctx, launch_cheb_dct(s, f.kind, f.power, a, b, n, cd, cd + n + 1));
  const double alpha = 2.0 / (b - a), beta = -(a + b) / (b - a);
  mlct_probes pr{};
  pr.kind = MLCT_PROBE_RADEMACHER;
  pr.seed = seed;
  pr.first_id = 0;
  pr.m = m_pilot;
  double* mud = static_cast<double*>(mu);
  CHECK(run_probe_set(ctx, op, alpha, beta, n, mode, prec, &pr, mud, n + 1));
  if (mu_out)
    HIPCHK(ctx, hipMemcpyAsync(mu_out, mud, (size_t)m_pilot * (n + 1) * sizeof(double),
                               hipMemcpyDeviceToHost, s));
  return plan_on_device(ctx, mud, n + 1, cd, m_pilot, n, mode, target, target_kind, m_pilot, out);
}

extern "C" mlct_status mlct_estimate_auto(mlct_ctx* ctx, const mlct_op* op, mlct_func f, double a,
                                          double b, int32_t n, int64_t m_pilot, uint64_t seed,
                                          int32_t prec, int32_t mode, double target,
                                          int32_t target_kind, mlct_level_plan* plan_out,
                                          mlct_result* out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!op || !out) return fail(ctx, MLCT_EINVAL, "op and out are required");
  mlct_level_plan plan{};
  CHECK(check_plan_args(ctx, m_pilot, n, mode, target, target_kind, &plan));
  CHECK(check_mode_prec(ctx, mode, prec));
  if (std::isnan(a) && std::isnan(b)) {
    const int steps = op->d < 64 ? (int)op->d : 64;
    CHECK(mlct_bounds(ctx, op, steps, seed + kGamma, 0.01, &a, &b));
  }
  CHECK(check_func(ctx, f, a, b));
  CHECK(set_device(ctx));
  const int64_t ldmu = n + 1;
  void *pil, *coef, *res;
  CHECK(ws_get(ctx, WS_MU2, (size_t)m_pilot * ldmu * sizeof(double), &pil));
  CHECK(ws_get(ctx, WS_COEF, (size_t)(n + 2) * sizeof(double), &coef));
  CHECK(ws_get(ctx, WS_RESULT, sizeof(mlct_result), &res));
  CHECK(reserve_block_ws(ctx, op, prec, mode, n, kDenseMaxBlock));
  double* cd = static_cast<double*>(coef);
  hipStream_t s = ctx->stream;
  HIPCHK(ctx, launch_cheb_dct(s, f.kind, f.power, a, b, n, cd, cd + n + 1));
  const double alpha = 2.0 / (b - a), beta = -(a + b) / (b - a);
  auto run = [&](int64_t first, int64_t m, int degree, double* rows) -> mlct_status {
    mlct_probes pr{};
    pr.kind = MLCT_PROBE_RADEMACHER;
    pr.seed = seed;
    pr.first_id = first;
    pr.m = m;
    return run_probe_set(ctx, op, alpha, beta, degree, mode, prec, &pr, rows, ldmu);
  };
  double* pd = static_cast<double*>(pil);
  CHECK(run(0, m_pilot, n, pd));
  CHECK(plan_on_device(ctx, pd, ldmu, cd, m_pilot, n, mode, target, target_kind, m_pilot, &plan));
  // Row layout of the moment table: the top level first (its first m_pilot
  // rows are the pilot's, probe ids = row index), then the lower levels.
  const int L = plan.L;
  LevelDesc lv{};
  lv.L = L;
  lv.coef_stride = n + 1;
  const int64_t mtop = plan.m[L - 1] > m_pilot ? plan.m[L - 1] : m_pilot;
  int64_t total = mtop, mv = 0, pdeg = 0;
  for (int k = 0; k < L; ++k) {
    lv.degree[k] = plan.degree[k];
    lv.m[k] = k == L - 1 ? mtop : plan.m[k];
    if (k < L - 1) {
      lv.off[k] = total;
      total += lv.m[k];
    } else {
      lv.off[k] = 0;
    }
    mv += lv.m[k] * (int64_t)(mode == MLCT_DOUBLING ? (lv.degree[k] + 1) / 2 : lv.degree[k]);
    pdeg += lv.m[k] * (int64_t)lv.degree[k];
  }
  void *mu, *qstat;
  CHECK(ws_get(ctx, WS_MU, (size_t)total * ldmu * sizeof(double), &mu));
  CHECK(ws_get(ctx, WS_QSTAT, ((size_t)total + 3 * MLCT_MAX_LEVELS) * sizeof(double), &qstat));
  double* mud = static_cast<double*>(mu);
  HIPCHK(ctx, hipMemcpyAsync(mud, pd, (size_t)m_pilot * ldmu * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
  if (mtop > m_pilot) CHECK(run(m_pilot, mtop - m_pilot, n, mud + m_pilot * ldmu));
  for (int k = 0; k < L - 1; ++k) CHECK(run(lv.off[k], lv.m[k], lv.degree[k], mud + lv.off[k] * ldmu));
  double* q = static_cast<double*>(qstat);
  HIPCHK(ctx, launch_level_combine(s, mud, ldmu, cd, cd + n + 1, lv, q, q + total,
                                   static_cast<mlct_result*>(res)));
  mlct_result h;
  HIPCHK(ctx, hipMemcpyAsync(&h, res, sizeof h, hipMemcpyDeviceToHost, s));
  CHECK(sync_stream(ctx));
  if (!(h.max_moment_ratio <= 1.0 + 1e-3))
    return fail(ctx, MLCT_ESPECTRUM,
                "max |mu_j|/|z|^2 = %g > 1: the spectrum is not inside [a, b] = [%g, %g]",
                h.max_moment_ratio, a, b);
  h.matvecs = mv;
  h.probe_degrees = pdeg;
  h.interval_a = a;
  h.interval_b = b;
  if (prec == MLCT_BF16X3) h.flags |= MLCT_FLAG_BF16;
  plan.m[L - 1] = mtop;
  if (plan_out) *plan_out = plan;
  *out = h;
  return MLCT_OK;
}

extern "C" mlct_status mlct_autotune(mlct_ctx* ctx, mlct_op* op, int32_t B_max, int32_t prec,
                                     int32_t* choice_out) {
  if (!ctx) return MLCT_EINVAL;
  ctx->err.clear();
  if (!op) return fail(ctx, MLCT_EINVAL, "op is required");
  if (op->kind == OP_CALLBACK)
    return fail(ctx, MLCT_EUNSUPPORTED, "callback operators have no launch shapes to tune");
  CHECK(set_device(ctx));
  const bool csr = op->kind == OP_CSR || op->kind == OP_GRAM_CSR;
  if (csr) prec = MLCT_FP32;
  CHECK(check_mode_prec(ctx, MLCT_DIRECT, prec));
  const int64_t block = csr ? kBlockProbes : std::max<int64_t>(32, std::min<int64_t>(B_max, kDenseMaxBlock));
  const int degree = 8;
  std::vector<int> cands;
  if (csr) cands = kCsrGroupCands;
  else cands = kDenseTileCands;
  // workspace for the largest candidate
  const int saved_g = op->tuned_groups, saved_t = op->tuned_dense;
  // on every early return the operator keeps the launch shape it had
  struct Guard {
    mlct_ctx* ctx;
    mlct_op* op;
    int g, t;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool restore = true;
    ~Guard() {
      if (restore) {
        op->tuned_groups = g;
        op->tuned_dense = t;
        (void)refresh_bands(ctx, op);
      }
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } guard{ctx, op, saved_g, saved_t};
  op->tuned_groups = 4096;
  void* mu;
  CHECK(ws_get(ctx, WS_MU, (size_t)block * (degree + 1) * 8, &mu));
  CHECK(reserve_block_ws(ctx, op, prec, MLCT_DIRECT, degree, block));
  op->tuned_groups = saved_g;
  HIPCHK(ctx, hipEventCreate(&guard.e0));
  HIPCHK(ctx, hipEventCreate(&guard.e1));
  hipEvent_t e0 = guard.e0, e1 = guard.e1;
  ProbeSrc src{0x5EEDull, 0, nullptr, 0, (int32_t)block};
  float best = 1e30f;
  int choice = csr ? 2048 : -1;
  for (int c : cands) {
    if (!csr && c == 1 && dense_bpad(block) % 128) continue;  // 128-tiles need bpad % 128 == 0
    if (!csr && c == 2 && dense_bpad(block) % 64) continue;
    if (csr) {
      op->tuned_groups = c;
      CHECK(refresh_bands(ctx, op));
    } else {
      op->tuned_dense = c;
    }
    float tmin = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      HIPCHK(ctx, hipEventRecord(e0, ctx->stream));
      CHECK(run_block(ctx, op, 0.1, 0.0, degree, MLCT_DIRECT, prec, src, static_cast<double*>(mu),
                      degree + 1));
      HIPCHK(ctx, hipEventRecord(e1, ctx->stream));
      HIPCHK(ctx, hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(ctx, hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) tmin = std::min(tmin, ms);
    }
    if (tmin < best) {
      best = tmin;
      choice = c;
    }
  }
  guard.restore = false;
  if (csr) {
    op->tuned_groups = choice;
    op->tuned_dense = saved_t;
    CHECK(refresh_bands(ctx, op));
  } else {
    op->tuned_dense = choice;
    op->tuned_groups = saved_g;
  }
  tune_store(ctx, tune_key(op, prec, csr ? 64 : dense_bpad(block)), choice);
  if (choice_out) *choice_out = choice;
  return MLCT_OK;
}
