// Block Chebyshev recurrence over a CSR operator (Section 2.2, eq.
// eqn:recurrence in matrix form) with the per-probe moments fused in.
//
// Layout: a probe block V is row-major d x 64 (probe index fastest), so the
// gather of row j of V is one 256-byte (FP32) or 512-byte (FP64) contiguous
// read by a whole wavefront, lane = probe.  One step computes
//     V_new = ca * (A V_k) + cb * V_k  [- V_prev]
// in place over V_prev (each element is read and then written by the same
// lane), and accumulates per lane, in FP64 with exact FP64 products,
//     ZMODE 0: V_k[i].V_new[i] and V_new[i].V_new[i]   (symmetric form)
//     ZMODE 1: z[i].V_new[i], z regenerated from SplitMix64 (direct form)
//     ZMODE 2: z[i].V_new[i], z read from explicit int8 entries.
// Each workgroup owns a contiguous band of rows and writes one partial sum
// per probe and slot; partials are reduced later in a fixed order, so the
// moments are bitwise reproducible.
//
// Operators whose rows all have at most 8 entries take a wide form of the
// same step (csr_step_wide_kernel, ZMODE 0 and 1): a lane holds 16 bytes of
// probes and a wave instruction moves several rows, with the same row sums,
// update and moment summation order as the lane = probe body.
//
// The same row machinery runs the integer passes of triangle counting
// (T = int32, pattern rows, int64 partials): only the per-row epilogue
// differs, so it is a policy type (RecEpi, TriEpi).
//
// Long rows (more than kHubLen entries, the hubs of power-law graphs) would
// leave one wave walking tens of thousands of gathers while the rest of the
// device idles.  Their entries are cut into chunks of kHubChunk that a
// separate launch (csr_hub_kernel) reduces first, one wave per chunk; the
// step kernel then sums a hub row's chunk partials in chunk order.
#include <algorithm>
#include <climits>
#include <type_traits>

#include "device.hpp"

namespace mlct {

namespace {

constexpr int kWaves = 8;
constexpr int kThreads = kWaves * 64;

// What a step kernel does with rows the straight-line path cannot take.
constexpr int kTailNone = 0;  // nothing: no row is longer than MAXNZ
constexpr int kTailGen = 1;   // the generic loop
constexpr int kTailHubs = 2;  // the generic loop, and hub partials past kHubLen

template <typename P>
__device__ __forceinline__ void store_partials(P a1, P a2, int g, int ngroups,
                                               P* __restrict__ part) {
  __shared__ P sh[2][kWaves][64];
  const int lane = lane_id(), wave = wave_id();
  sh[0][wave][lane] = a1;
  sh[1][wave][lane] = a2;
  __syncthreads();
  if (wave == 0) {
    P s1 = sh[0][0][lane], s2 = sh[1][0][lane];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) {
      s1 += sh[0][w][lane];
      s2 += sh[1][w][lane];
    }
    part[(size_t)g * 64 + lane] = s1;
    part[((size_t)ngroups + g) * 64 + lane] = s2;
  }
}

template <typename T>
__device__ __forceinline__ void probe_init_wg(T* __restrict__ v0, int64_t d, const ProbeSrc& src,
                                              int rows_per_group, int ngroups,
                                              double* __restrict__ part, int bid) {
  const int lane = lane_id(), wave = wave_id();
  const int g = xcd_band(bid, ngroups);
  const int64_t r0 = (int64_t)g * rows_per_group;
  const int64_t r1 = min<int64_t>(r0 + rows_per_group, d);
  const bool act = lane < src.active;
  const uint64_t key = sm_output(src.seed, (uint64_t)(src.first_id + lane));
  int64_t cached = -1;
  uint64_t word = 0;
  double acc = 0.0;
  for (int64_t i = r0 + wave; i < r1; i += kWaves) {
    T z = T(0);
    if (act) {
      if (src.entries) {
        z = (T)src.entries[i * src.ld + src.first_id + lane];
      } else {
        const int64_t c = i >> 6;
        if (c != cached) {
          word = sm_output(key, (uint64_t)c);
          cached = c;
        }
        z = sign_from_word<T>(word, i);
      }
    }
    v0[i * 64 + lane] = z;
    acc += (double)z * (double)z;
  }
  store_partials<double>(acc, 0.0, g, ngroups, part);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void probe_init_kernel(T* __restrict__ v0, int64_t d,
                                                              ProbeSrc src, int rows_per_group,
                                                              int ngroups,
                                                              double* __restrict__ part) {
  probe_init_wg<T>(v0, d, src, rows_per_group, ngroups, part, blockIdx.x);
}

// Per-row epilogue of the recurrence: V_new = ca*acc + cb*V_k[i] (- V_prev[i]),
// written over V_prev (with a non-temporal store unless KEEP: a vector
// gathered again soon is stored normally, to stay in the caches), and the
// lane's moment partials (FP64).  With CLS = 4 (FP32, ZMODE 0 or 1,
// operators whose rows all fit the straight-line path) the partials are kept per row
// class (the row's index in its group, mod 4) and the classes added in
// order at the end: the summation order of the wide step kernel, whose lane
// quads take one class each, so both kernels give the same bits.
template <typename T, int ZMODE, bool HAS_PREV, bool KEEP = false, int CLS = 1>
struct RecEpi {
  using Part = double;
  static constexpr bool kOwn = true;    // needs V_k[i] of its own row
  static constexpr bool kParts = true;  // writes moment partials
  static constexpr int kCls = (ZMODE <= 1 && sizeof(T) == 4) ? CLS : 1;
  T ca, cb;
  T* vm;
  ProbeSrc src;
  bool act;
  uint64_t key = 0;
  int64_t cached = -1;
  uint64_t word = 0;
  double a1[kCls] = {}, a2[kCls] = {};
  __device__ RecEpi(T ca_, T cb_, T* vm_, const ProbeSrc& s) : ca(ca_), cb(cb_), vm(vm_), src(s) {
    const int lane = lane_id();
    act = lane < src.active;
    if (ZMODE == 1) key = sm_output(src.seed, (uint64_t)(src.first_id + lane));
  }
  __device__ __forceinline__ T prev(int64_t i) const {
    return HAS_PREV ? __builtin_nontemporal_load(vm + i * 64 + lane_id()) : T(0);
  }
  // r: the row's index in its group (a compile-time constant at every call)
  __device__ __forceinline__ void finish(int64_t i, T acc, T xi, T xp, int r) {
    const int lane = lane_id();
    const int c = r % kCls;
    // one explicit contraction, so every kernel that shares this update
    // (the two-step and wide kernels included) rounds it the same way
    T vn = fma(ca, acc, cb * xi);
    if (HAS_PREV) vn -= xp;
    if (KEEP)
      vm[i * 64 + lane] = vn;
    else
      __builtin_nontemporal_store(vn, vm + i * 64 + lane);
    if (ZMODE == 0) {
      a1[c] += (double)xi * (double)vn;
      a2[c] += (double)vn * (double)vn;
    } else if (ZMODE == 1) {
      const int64_t cw = i >> 6;
      if (cw != cached) {
        word = sm_output(key, (uint64_t)cw);
        cached = cw;
      }
      a1[c] += sign_from_word<double>(word, i) * (double)vn;
    } else {
      const double z = act ? (double)src.entries[i * src.ld + src.first_id + lane] : 0.0;
      a1[c] += z * (double)vn;
    }
  }
  __device__ __forceinline__ double part1() const { return class_sum(a1); }
  __device__ __forceinline__ double part2() const { return class_sum(a2); }
  static __device__ __forceinline__ double class_sum(const double (&a)[kCls]) {
    double s = a[0];
#pragma unroll
    for (int k = 1; k < kCls; ++k) s += a[k];
    return s;
  }
};

// The int16 form of y (triangle passes): a value outside [-32767, 32767]
// is stored as this sentinel, its exact value in the row of its hub (rows
// longer than kHubLen, the only ones that can hold such a value) in a side
// table.
constexpr int32_t kY16Sentinel = -32768;
struct HubSide {
  const int32_t* rows;  // sorted hub row ids
  int n;
  int32_t* side;        // [n][64] exact values of the sentinel entries
  __device__ __forceinline__ int slot(int64_t i) const {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (rows[mid] < i) lo = mid + 1; else hi = mid;
    }
    return lo;
  }
};

// Per-row epilogue of the triangle passes (exact int64 sums):
//   PASS 1: y = A z stored as int16 rows (a value beyond +-32767 as the
//           sentinel, exact in the hub side table: see Y16Reader),
//           slot 0 = z.y, slot 1 = y.y
//   PASS 2: w = A y not stored, slot 0 = y.w.
// |y_i| <= deg(i) and |w_i| <= nnz < 2^31, so int32 holds every sum.
template <int PASS>
struct TriEpi {
  using Part = long long;
  static constexpr bool kOwn = true;
  static constexpr bool kParts = true;
  int16_t* vout;
  HubSide hs;
  long long a1 = 0, a2 = 0;
  __device__ TriEpi(int16_t* v, const HubSide& h) : vout(v), hs(h) {}
  __device__ __forceinline__ int32_t prev(int64_t) const { return 0; }
  __device__ __forceinline__ long long part1() const { return a1; }
  __device__ __forceinline__ long long part2() const { return a2; }
  __device__ __forceinline__ void finish(int64_t i, int32_t acc, int32_t own, int32_t, int) {
    const int lane = lane_id();
    if (PASS == 1) {
      int16_t st = (int16_t)acc;
      if (__builtin_expect(acc < -32767 || acc > 32767, 0)) {
        st = (int16_t)kY16Sentinel;
        hs.side[(int64_t)hs.slot(i) * 64 + lane] = acc;
      }
      __builtin_nontemporal_store(st, vout + i * 64 + lane);
      a1 += (long long)own * acc;
      a2 += (long long)acc * acc;
    } else {
      if (__builtin_expect(own == kY16Sentinel, 0)) own = hs.side[(int64_t)hs.slot(i) * 64 + lane];
      a1 += (long long)own * acc;
    }
  }
};

// First product of a Gram step: the row sums are stored (W = X V_k), no
// recurrence, no partials.
template <typename T>
struct StoreEpi {
  using Part = double;
  static constexpr bool kOwn = false;
  static constexpr bool kParts = false;
  T* out;
  double a1 = 0.0, a2 = 0.0;
  __device__ explicit StoreEpi(T* o) : out(o) {}
  __device__ __forceinline__ T prev(int64_t) const { return T(0); }
  __device__ __forceinline__ double part1() const { return a1; }
  __device__ __forceinline__ double part2() const { return a2; }
  __device__ __forceinline__ void finish(int64_t i, T acc, T, T, int) { out[i * 64 + lane_id()] = acc; }
};

// SpMM of a Lanczos step (FP64, lane = probe): u = s (A w_j) stored, with
// s = 1 / |w_j| per probe, and partials of (s w_j) . u (the Jacobi diagonal).
struct SlqEpi {
  using Part = double;
  static constexpr bool kOwn = true;
  static constexpr bool kParts = true;
  double* out;
  double s;
  double a1 = 0.0, a2 = 0.0;
  __device__ SlqEpi(double* o, const double* sdev) : out(o), s(sdev[lane_id()]) {}
  __device__ __forceinline__ double prev(int64_t) const { return 0.0; }
  __device__ __forceinline__ double part1() const { return a1; }
  __device__ __forceinline__ double part2() const { return a2; }
  __device__ __forceinline__ void finish(int64_t i, double acc, double xi, double, int) {
    const double u = s * acc;
    out[i * 64 + lane_id()] = u;
    a1 += (s * xi) * u;
  }
};

// One gathered entry into a row sum: weight w (ignored for patterns) times x,
// or nothing when on is false.
template <typename T, bool PATTERN>
__device__ __forceinline__ T accum(T acc, float w, bool on, T x) {
  if constexpr (std::is_integral<T>::value) {
    return acc + (on ? x : T(0));
  } else {
    const float onf = on ? 1.f : 0.f;
    const float ww = PATTERN ? onf : w * onf;
    return fma((T)ww, x, acc);
  }
}

// Gathers of block rows.  With OFF32 (block under 4 GiB, FP32) they are
// buffer loads: the block base sits in a scalar resource, the row offset
// j * 256 in a scalar register and lane * 4 in one VGPR shared by every
// gather, so a gather costs no address registers.  Out-of-range offsets read
// as 0 (the resource's size is the block's size).
template <typename T, bool OFF32>
struct RowReader {
  using Elem = T;  // element type of the gathered block
  using Val = T;   // type of a gathered value
  const T* base;
  __amdgpu_buffer_rsrc_t rsrc;
  uint32_t lane_off;
  __device__ __forceinline__ RowReader(const T* b, int64_t d, int lane) : base(b) {
    if (OFF32) {
      rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(b), (short)0,
                                               (int)(uint32_t)(d * 64 * sizeof(T)), 0x00020000);
      lane_off = (uint32_t)lane * sizeof(T);
    }
  }
  __device__ __forceinline__ T operator()(int64_t j, int lane) const {
    if constexpr (OFF32) {
      static_assert(sizeof(T) == 4, "32-bit offsets are for 4-byte elements");
      const uint32_t bits = __builtin_amdgcn_raw_buffer_load_b32(
          rsrc, lane_off, (int)((uint32_t)j * (uint32_t)(64 * sizeof(T))), 0);
      if constexpr (std::is_integral<T>::value) return (T)bits;
      else return __uint_as_float(bits);
    } else {
      return base[j * 64 + lane];
    }
  }
  // a gathered value as the row sum takes it (the raw value here)
  static constexpr bool kFix = false;
  __device__ __forceinline__ T fix(int64_t, T x) const { return x; }
  // gathers by a byte offset precomputed as column * kRowBytes (buffer form)
  // (raw load, then conversion: the sequence form issues every load of a
  // batch before it converts the first)
  static constexpr bool kScaled = OFF32 && sizeof(T) == 4;
  static constexpr uint32_t kRowBytes = 64 * sizeof(T);
  using Raw = uint32_t;
  __device__ __forceinline__ uint32_t raw(uint32_t soff) const {
    if constexpr (kScaled) return __builtin_amdgcn_raw_buffer_load_b32(rsrc, lane_off, (int)soff, 0);
    else return 0u;
  }
  __device__ __forceinline__ T cvt(uint32_t bits) const {
    if constexpr (std::is_integral<T>::value) return (T)bits;
    else return __uint_as_float(bits);
  }
};

// Triangle pass 1 gathers only Rademacher signs: one 64-bit word per row,
// bit p set where probe p is -1.  Every lane of a wave gathers the same row:
// lanes 0-31 load its low 32 bits and lanes 32-63 its high 32 bits by a
// vector buffer load from a scalar row offset (one 8-byte request; vector
// loads keep many more gathers in flight than scalar loads would).
struct SignBitsReader {
  using Elem = uint64_t;
  using Val = int32_t;
  __amdgpu_buffer_rsrc_t rsrc;
  uint32_t half_off;
  int shift;
  __device__ __forceinline__ SignBitsReader(const uint64_t* b, int64_t d, int lane) {
    rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint64_t*>(b), (short)0,
                                             (int)(uint32_t)(d * sizeof(uint64_t)), 0x00020000);
    half_off = (uint32_t)(lane >> 5) * 4;
    shift = lane & 31;
  }
  __device__ __forceinline__ int32_t operator()(int64_t j, int) const {
    return cvt(raw((uint32_t)j * (uint32_t)sizeof(uint64_t)));
  }
  static constexpr bool kScaled = true;
  static constexpr uint32_t kRowBytes = sizeof(uint64_t);
  using Raw = uint32_t;
  __device__ __forceinline__ uint32_t raw(uint32_t soff) const {
    return __builtin_amdgcn_raw_buffer_load_b32(rsrc, half_off, (int)soff, 0);
  }
  __device__ __forceinline__ int32_t cvt(uint32_t w) const {
    return 1 - 2 * (int32_t)__builtin_amdgcn_ubfe(w, (uint32_t)shift, 1u);
  }
  static constexpr bool kFix = false;
  __device__ __forceinline__ int32_t fix(int64_t, int32_t x) const { return x; }
};

// Rows of 64 int16 values (triangle pass 2 gathers y = A z, |y_i| <= the
// degree of row i).  A value outside [-32767, 32767], possible only on rows
// longer than kHubLen (the hub rows), is stored as the sentinel -32768 with
// the exact int32 value in that hub's row of a side table; fix() takes it
// from there.  It is applied when the value is summed, after every gather
// of the group was issued, so the check does not stall the gathers.
template <bool OFF32>
struct Y16Reader {
  using Elem = int16_t;
  using Val = int32_t;
  const int16_t* base;
  __amdgpu_buffer_rsrc_t rsrc;
  uint32_t lane_off;
  HubSide hs;
  __device__ __forceinline__ Y16Reader(const int16_t* y, int64_t d, int lane, const HubSide& h)
      : base(y), hs(h) {
    if (OFF32) {
      rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<int16_t*>(y), (short)0,
                                               (int)(uint32_t)(d * 64 * sizeof(int16_t)),
                                               0x00020000);
      lane_off = (uint32_t)lane * sizeof(int16_t);
    }
  }
  __device__ __forceinline__ int32_t operator()(int64_t j, int lane) const {
    if constexpr (OFF32) {
      return cvt(raw((uint32_t)j * kRowBytes));
    } else {
      return base[j * 64 + lane];
    }
  }
  static constexpr bool kScaled = OFF32;
  static constexpr uint32_t kRowBytes = 64 * sizeof(int16_t);
  using Raw = uint16_t;
  __device__ __forceinline__ uint16_t raw(uint32_t soff) const {
    if constexpr (OFF32) return __builtin_amdgcn_raw_buffer_load_b16(rsrc, lane_off, (int)soff, 0);
    else return 0;
  }
  __device__ __forceinline__ int32_t cvt(uint16_t bits) const { return (int32_t)(int16_t)bits; }
  static constexpr bool kFix = true;
  __device__ __forceinline__ int32_t fix(int64_t j, int32_t x) const {
    if (__builtin_expect(x == kY16Sentinel, 0)) x = hs.side[(int64_t)hs.slot(j) * 64 + lane_id()];
    return x;
  }
};

// Applies rd.fix to n gathered values (x[u] from column col(u)) with one
// test per batch: the sentinel is the smallest int16, so a batch holds one
// only if its minimum equals it (rare: only hub rows' extreme sums).
template <class RD, int N, class X, class C>
__device__ __forceinline__ void fix_batch(const RD& rd, X* x, C col) {
  if constexpr (RD::kFix) {
    int32_t m = x[0];
#pragma unroll
    for (int u = 1; u < N; ++u) m = min(m, (int32_t)x[u]);
    if (__builtin_expect(m == kY16Sentinel, 0)) {
#pragma unroll
      for (int u = 0; u < N; ++u) x[u] = rd.fix(col(u), x[u]);
    }
  }
}

// Generic row: 64-entry chunks of the row's columns, each loaded in one
// coalesced read, then gathered 16 at a time (all 16 in flight before the
// first is consumed; slots past the end gather the chunk's last row with
// weight 0).
constexpr int kGen = 16;
// Gathers in flight per wave in the sequence form of a group (below).  16
// for FP32 lowers the batched kernel's registers to four waves per SIMD but
// measured 3x slower on the 64-graph Chung-Lu batch (more workgroups in
// flight over a multi-GB gather working set); single-matrix steps time the
// same with either.
template <typename T>
constexpr int kFlatOf = sizeof(T) == 8 ? 16 : 32;

template <typename T, bool PATTERN, class RD>
__device__ __forceinline__ T row_dot_generic(const int32_t* __restrict__ col,
                                             const float* __restrict__ val, const RD& rd,
                                             int64_t s, int64_t e) {
  const int lane = lane_id();
  T acc = T(0);
  for (int64_t base = s; base < e; base += 64) {
    const int c = (int)min<int64_t>(64, e - base);
    const int64_t ce = base + min(lane, c - 1);
    const int cj = col[ce];
    const float av = PATTERN ? 1.f : val[ce];
    for (int t = 0; t < c; t += kGen) {
      T x[kGen];
#pragma unroll
      for (int u = 0; u < kGen; ++u) x[u] = rd(read_lane(cj, min(t + u, c - 1)), lane);
      fix_batch<RD, kGen>(rd, x, [&](int u) { return read_lane(cj, min(t + u, c - 1)); });
#pragma unroll
      for (int u = 0; u < kGen; ++u)
        acc = accum<T, PATTERN>(acc, PATTERN ? 1.f : read_lane(av, min(t + u, c - 1)),
                                t + u < c, x[u]);
    }
  }
  return acc;
}

// A row as consecutive chunks of kHubChunk entries, each reduced on its own
// and the chunk sums added in order: the association the hub path uses, so a
// row's sum is bitwise the same whether or not its chunks ran as a hub.
template <typename T, bool PATTERN, class RD>
__device__ __forceinline__ T row_dot_chunked(const int32_t* __restrict__ col,
                                             const float* __restrict__ val, const RD& rd,
                                             int64_t s, int64_t e) {
  T acc = T(0);
  for (int64_t c0 = s; c0 < e; c0 += kHubChunk)
    acc += row_dot_generic<T, PATTERN>(col, val, rd, c0, min<int64_t>(c0 + kHubChunk, e));
  return acc;
}

// Hub rows: sorted row ids, the first chunk of each (hub_c0[k] .. hub_c0[k+1]),
// and the chunk partials of the current step (chunk-major, 64 lanes each).
struct HubView {
  const int32_t* rows;
  const int32_t* c0;
  int n;
  const void* part;
};

template <typename T>
__device__ __forceinline__ T hub_sum(const HubView& h, int64_t i) {
  int lo = 0, hi = h.n - 1;  // the row is in the table
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (h.rows[mid] < i) lo = mid + 1; else hi = mid;
  }
  const int c0 = h.c0[lo], c1 = h.c0[lo + 1];
  const T* p = static_cast<const T*>(h.part);
  T acc = T(0);
  for (int c = c0; c < c1; ++c) acc += p[(int64_t)c * 64 + lane_id()];
  return acc;
}

// Extent of one group of up to ROWS consecutive rows.  The group's rows sit
// in lanes q .. q+ROWS-1 of a batch: rs = start of the row's columns,
// rlen = its length (0 for lanes past the end of the matrix).
template <int ROWS>
struct GroupExt {
  int gs, cnt, nr, maxlen;
  int off[ROWS], len[ROWS];
};

template <int ROWS>
__device__ __forceinline__ GroupExt<ROWS> group_extent(int rs, int rlen, int q, int nr) {
  GroupExt<ROWS> e;
  e.nr = nr;
  e.gs = read_lane(rs, q);
  e.maxlen = 0;
  e.cnt = 0;
#pragma unroll
  for (int r = 0; r < ROWS; ++r) {
    const bool in = r < nr;
    e.off[r] = in ? read_lane(rs, q + r) - e.gs : 0;
    e.len[r] = in ? read_lane(rlen, q + r) : 0;
    e.maxlen = max(e.maxlen, e.len[r]);
    if (in) e.cnt = e.off[r] + e.len[r];  // static indices only
  }
  return e;
}

// Work split: a workgroup owns a contiguous band of rows (equal row counts,
// or the plan's equal-work bands) cut into groups of ROWS rows; wave w takes
// groups w, w + kWaves, w + 2 kWaves, ..., so the waves of a workgroup sweep
// the band side by side.  A wave fetches the row extents of its next 64/ROWS
// groups in one load (a "batch", prefetched one batch ahead) and the column
// indices and values of a group in one coalesced load, issued while the
// previous group's gathers are in flight.  When every row of a group has at
// most MAXNZ entries its gathers are straight-line code (unused slots gather
// some valid row with weight 0), all in flight before the first is consumed.
// Other groups (TAIL kTailGen / kTailHubs) are gathered as one sequence of
// entries when no row exceeds kHubChunk, else row by row, rows longer than
// kHubLen through their chunk partials (kTailHubs).  With kTailNone the
// caller guarantees that no row is longer than MAXNZ (and ROWS * MAXNZ <=
// 64), so every group is straight-line.
//
// d: rows processed; dv: rows of the gathered block vk.  SEP: the own-row
// value V_k[i] the epilogue needs comes from vown instead of vk (the second
// product of a Gram step gathers from W but recurs on V_k).
template <typename T, bool PATTERN, int MAXNZ, bool OFF32, int TAIL, bool SEP, class Epi,
          class RD = RowReader<T, OFF32>>
__device__ __forceinline__ void csr_step_wg(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, int64_t d, int64_t dv, int64_t nnz, const RD& rd,
    const T* __restrict__ vown, Epi& epi, const HubView& hub, const CsrStepPlan& plan,
    typename Epi::Part* __restrict__ part, int bid) {
  constexpr int ROWS = MAXNZ <= 5 ? 8 : 4;
  constexpr int GPB = 64 / ROWS;  // groups per batch
  constexpr bool HUBS = TAIL == kTailHubs;
  constexpr int kFlat = kFlatOf<T>;
  const int lane = lane_id(), wave = wave_id();
  const int ngroups = plan.ngroups;
  const int g = xcd_band(bid, ngroups);
  const int64_t r0 = plan.band ? (int64_t)plan.band[g] : (int64_t)g * plan.rows_per_group;
  const int64_t r1 = plan.band ? (int64_t)plan.band[g + 1]
                               : min<int64_t>(r0 + plan.rows_per_group, d);

  const int64_t ngrp = r1 > r0 ? (r1 - r0 + ROWS - 1) / ROWS : 0;  // groups in the band
  const int64_t nk = ngrp > wave ? (ngrp - wave + kWaves - 1) / kWaves : 0;  // this wave's
  auto own = [&](int64_t i) -> T {
    if constexpr (!Epi::kOwn) return T(0);
    else if constexpr (SEP) return vown[i * 64 + lane];
    else return rd(i, lane);
  };
  // first row of this wave's k-th group, and its number of rows
  auto grp_row0 = [&](int64_t k) { return r0 + (k * kWaves + wave) * ROWS; };
  auto grp_rows = [&](int64_t k) { return (int)min<int64_t>(ROWS, r1 - grp_row0(k)); };

  if (nk > 0) {
    auto load_batch = [&](int64_t j, int& rs, int& rlen) {
      const int64_t k = j * GPB + lane / ROWS;
      const int64_t row = grp_row0(k) + lane % ROWS;
      const bool ok = k < nk && row < r1;
      const int64_t rr = ok ? row : r0;
      rs = rowptr[rr];
      rlen = ok ? rowptr[rr + 1] - rs : 0;
    };
    auto load_cols = [&](const GroupExt<ROWS>& e, int& cj, float& av) {
      const int64_t ce = min<int64_t>((int64_t)e.gs + lane, nnz - 1);
      cj = col[ce];
      av = PATTERN ? 1.f : val[ce];
    };
    const int64_t nbatch = (nk + GPB - 1) / GPB;
    int64_t j = 0;
    int rs, rlen, rs_n = 0, rlen_n = 0;
    load_batch(0, rs, rlen);
    if (nbatch > 1) load_batch(1, rs_n, rlen_n);
    int64_t k = 0;
    GroupExt<ROWS> cur = group_extent<ROWS>(rs, rlen, 0, grp_rows(0));
    int cj = 0;
    float av = 0.f;
    if (nnz > 0) load_cols(cur, cj, av);

    while (true) {
      const int64_t row0 = grp_row0(k);
      const bool fast =
          TAIL == kTailNone || (nnz > 0 && cur.maxlen <= MAXNZ && cur.cnt <= 64);
      T x[ROWS][MAXNZ > 0 ? MAXNZ : 1];
      T xi[ROWS], xp[ROWS];
      if (fast) {
        // all gathers of the group before anything else is issued
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
          const int64_t i = row0 + min(r, cur.nr - 1);
#pragma unroll
          for (int t = 0; t < MAXNZ; ++t) x[r][t] = rd(read_lane(cj, min(cur.off[r] + t, 63)), lane);
          xi[r] = own(i);
          xp[r] = epi.prev(i);
        }
      }
      // next group: extent and column prefetch
      const int64_t kn = k + 1;
      const bool has_next = kn < nk;
      const bool new_batch = has_next && (kn % GPB) == 0;
      GroupExt<ROWS> nxt = cur;
      int cjn = 0;
      float avn = 0.f;
      if (has_next) {
        const int qn = (int)(kn % GPB) * ROWS;
        nxt = new_batch ? group_extent<ROWS>(rs_n, rlen_n, 0, grp_rows(kn))
                        : group_extent<ROWS>(rs, rlen, qn, grp_rows(kn));
        if (nnz > 0) load_cols(nxt, cjn, avn);
      }
      if (fast) {
        if constexpr (RD::kFix) {
#pragma unroll
          for (int r = 0; r < ROWS; ++r)
            fix_batch<RD, (MAXNZ > 0 ? MAXNZ : 1)>(
                rd, x[r], [&](int t) { return read_lane(cj, min(cur.off[r] + t, 63)); });
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
          T acc = T(0);
#pragma unroll
          for (int t = 0; t < MAXNZ; ++t)
            acc = accum<T, PATTERN>(acc, PATTERN ? 1.f : read_lane(av, min(cur.off[r] + t, 63)),
                                    t < cur.len[r], x[r][t]);
          if (r < cur.nr) epi.finish(row0 + r, acc, xi[r], xp[r], r);
        }
      } else if constexpr (TAIL != kTailNone) {
        if (cur.maxlen <= kHubChunk) {
          // the group's entries as one sequence: 64-entry chunks of column
          // indices (the first already loaded), gathered kFlat at a time and
          // summed in column order into a running sum that is handed to its
          // row's accumulator at the row's last entry (rows are contiguous)
          T acc[ROWS];
#pragma unroll
          for (int r = 0; r < ROWS; ++r) {
            const int64_t i = row0 + min(r, cur.nr - 1);
            acc[r] = T(0);
            xi[r] = own(i);
            xp[r] = epi.prev(i);
          }
          // per-group tables in lanes 0 .. ROWS: the position of row r's
          // last entry (INT_MAX past the rows, so it is never reached) and
          // the next row after r that has entries (ROWS: none); the current
          // row rc and its end rend are uniform
          int end_v = INT_MAX, nxt_v = ROWS;
          int first = ROWS;
#pragma unroll
          for (int r = ROWS - 1; r >= 0; --r) {
            if (lane == r) {
              end_v = cur.len[r] > 0 ? cur.off[r] + cur.len[r] - 1 : INT_MAX;
              nxt_v = first;
            }
            if (cur.len[r] > 0) first = r;
          }
          int rc = first;
          int rend = read_lane(end_v, rc);
          T run = T(0);
          for (int base = 0; base < cur.cnt; base += 64) {
            int cjc = cj;
            float avc = av;
            if (base > 0) {
              const int64_t ce = min<int64_t>((int64_t)cur.gs + base + lane, nnz - 1);
              cjc = col[ce];
              avc = PATTERN ? 1.f : val[ce];
            }
            const int c = min(64, cur.cnt - base);
            // lanes past the chunk's end repeat its last column (a valid row,
            // not summed), and the reader's row offsets are formed once per
            // chunk, so a gather is one lane read and one load
            const int cl = lane < c ? cjc : read_lane(cjc, c - 1);
            const int off = (int)((uint32_t)cl * RD::kRowBytes);
#pragma unroll
            for (int h = 0; h < 64 / kFlat; ++h) {
              const int t = h * kFlat;
              if (t >= c) break;
              T xg[kFlat];
              if constexpr (RD::kScaled) {
                typename RD::Raw xr[kFlat];
#pragma unroll
                for (int u = 0; u < kFlat; ++u) xr[u] = rd.raw((uint32_t)read_lane(off, t + u));
                // every load of the batch is in flight before the first is used
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < kFlat; ++u) xg[u] = rd.cvt(xr[u]);
              } else {
#pragma unroll
                for (int u = 0; u < kFlat; ++u) xg[u] = rd(read_lane(cl, t + u), lane);
              }
              fix_batch<RD, kFlat>(rd, xg, [&](int u) { return read_lane(cl, t + u); });
              const int lim = c - t;         // entries of this batch in the group
              int rloc = rend - (base + t);  // batch position of the current row's end
              // summed in column order; at a row's last entry its sum goes to
              // the row's accumulator and the next row begins
              auto sum_batch = [&](auto full) {
#pragma unroll
                for (int u = 0; u < kFlat; ++u) {
                  if (!decltype(full)::value && u >= lim) break;
                  const float w = PATTERN ? 1.f : read_lane(avc, t + u);
                  run = accum<T, PATTERN>(run, w, true, xg[u]);
                  if (u == rloc) {
#pragma unroll
                    for (int r = 0; r < ROWS; ++r)
                      if (r == rc) acc[r] = run;
                    run = T(0);
                    rc = read_lane(nxt_v, rc);
                    rend = read_lane(end_v, rc);
                    rloc = rend - (base + t);
                  }
                }
              };
              if (lim >= kFlat)
                sum_batch(std::true_type());
              else
                sum_batch(std::false_type());
            }
          }
#pragma unroll
          for (int r = 0; r < ROWS; ++r)
            if (r < cur.nr) epi.finish(row0 + r, acc[r], xi[r], xp[r], r);
        } else {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {  // static indices: cur stays in registers
          if (r < cur.nr) {
            const int64_t i = row0 + r;
            const int64_t s0 = (int64_t)cur.gs + cur.off[r];
            T acc;
            if (HUBS && cur.len[r] > kHubLen)
              acc = hub_sum<T>(hub, i);
            else
              acc = row_dot_chunked<T, PATTERN>(col, val, rd, s0, s0 + cur.len[r]);
            epi.finish(i, acc, own(i), epi.prev(i), r);
          }
        }
        }
      }
      if (!has_next) break;
      if (new_batch) {
        rs = rs_n;
        rlen = rlen_n;
        ++j;
        if (j + 1 < nbatch) load_batch(j + 1, rs_n, rlen_n);
      }
      k = kn;
      cur = nxt;
      cj = cjn;
      av = avn;
    }
  }
  if constexpr (Epi::kParts)
    store_partials<typename Epi::Part>(epi.part1(), epi.part2(), g, ngroups, part);
}

template <typename T, bool PATTERN, int ZMODE, bool HAS_PREV, int MAXNZ, bool OFF32, int TAIL>
__global__ __launch_bounds__(kThreads) void csr_step_kernel(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, int64_t d, int64_t nnz, const T* __restrict__ vk,
    T* __restrict__ vm, T ca, T cb, ProbeSrc src, HubView hub, CsrStepPlan plan,
    double* __restrict__ part) {
  RecEpi<T, ZMODE, HAS_PREV, false, TAIL == kTailNone ? 4 : 1> epi(ca, cb, vm, src);
  csr_step_wg<T, PATTERN, MAXNZ, OFF32, TAIL, false>(rowptr, col, val, d, d, nnz,
                                                     RowReader<T, OFF32>(vk, d, lane_id()),
                                                     nullptr, epi, hub, plan, part, blockIdx.x);
}

// ---- wide form of the step ------------------------------------------------------
// For operators whose rows all fit the straight-line path (no tail) and
// moments of the symmetric form (ZMODE 0) or the direct form with
// regenerated Rademacher probes (ZMODE 1), the same step with a lane
// holding PPL = 16 / sizeof(T) probes (4 in FP32, 2 in FP64): every access
// is 16 bytes, so one wave instruction moves PPL rows (lane group q, of
// 64 / PPL lanes, on the group's rows q, q + PPL, ...) and a step issues
// 1 / PPL of the memory instructions of the lane = probe body.  The work
// split (bands, groups of ROWS rows, wave w on groups w, w + 8, ...), the
// column prefetch, the row sums (entry order, one fma per entry, unused
// slots weighted 0) and the update are those of csr_step_wg with RecEpi; a
// lane's row offset and length are picked from the group's extent by its
// lane group, and its column indices and values come from the group's
// coalesced load by a lane permute.  The moment partials are kept per row
// class (row index in the group mod PPL, one class per lane group) and the
// classes added in order; in FP32 that is the order of RecEpi with CLS = 4,
// so this kernel and the lane = probe body give the same bits.  With SLQ
// the rows are the product of a Lanczos step instead (the SlqEpi epilogue:
// u = s (A w) stored, partials of (s w) . u; FP64, no recurrence).
template <typename T>
struct WideVec;
template <>
struct WideVec<float> {
  typedef float V __attribute__((ext_vector_type(4)));
};
template <>
struct WideVec<double> {
  typedef double V __attribute__((ext_vector_type(2)));
};

template <typename T, bool OFF32>
struct WideRows {
  using V = typename WideVec<T>::V;
  const T* base;
  __amdgpu_buffer_rsrc_t rsrc;
  uint32_t lane_off;
  __device__ __forceinline__ WideRows(const T* b, int64_t d, int sub) : base(b) {
    if (OFF32)
      rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(b), (short)0,
                                               (int)(uint32_t)(d * 64 * sizeof(T)), 0x00020000);
    lane_off = (uint32_t)sub * 16;
  }
  // the lane's probes of block row j
  __device__ __forceinline__ V operator()(int64_t j) const {
    if constexpr (OFF32)
      return __builtin_bit_cast(
          V, __builtin_amdgcn_raw_buffer_load_b128(
                 rsrc, (uint32_t)j * (uint32_t)(64 * sizeof(T)) + lane_off, 0, 0));
    else
      return *reinterpret_cast<const V*>(base + j * 64 + lane_off / sizeof(T));
  }
};

__device__ __forceinline__ int permute_lane(int v, int src) {
  return __builtin_amdgcn_ds_bpermute(src << 2, v);
}

template <typename T>
using WidePartials = double[2][kWaves][16 / sizeof(T)][64];

// Band g of the wide step: its rows, then its moment partials (sh: the
// workgroup's LDS for the partials).
template <typename T, bool PATTERN, int ZMODE, bool HAS_PREV, int MAXNZ, bool OFF32,
          bool SLQ = false>
__device__ __forceinline__ void wide_band(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, int64_t d, int64_t nnz, const T* __restrict__ vk,
    T* __restrict__ vm, T ca, T cb, const ProbeSrc& src, const CsrStepPlan& plan,
    double* __restrict__ part, int g, WidePartials<T>& sh, const double* sdev = nullptr) {
  static_assert(ZMODE == 0 || ZMODE == 1, "symmetric or regenerated direct moments");
  static_assert(!SLQ || (ZMODE == 0 && !HAS_PREV), "the Lanczos product has no recurrence");
  using V = typename WideVec<T>::V;
  constexpr int PPL = 16 / (int)sizeof(T);  // probes per lane = rows per wave instruction
  constexpr int LPR = 64 / PPL;             // lanes per row
  constexpr int ROWS = MAXNZ <= 5 ? 8 : 4;
  constexpr int H = ROWS / PPL;   // wave instructions per group
  constexpr int GPB = 64 / ROWS;  // groups per batch of row extents
  static_assert(ROWS * MAXNZ <= 64, "a group's entries fit one coalesced load");
  static_assert(ROWS % PPL == 0, "whole wave instructions per group");
  const int lane = lane_id(), wave = wave_id();
  const int q = lane / LPR, sub = lane % LPR;
  const int ngroups = plan.ngroups;
  const int64_t r0 = plan.band ? (int64_t)plan.band[g] : (int64_t)g * plan.rows_per_group;
  const int64_t r1 = plan.band ? (int64_t)plan.band[g + 1]
                               : min<int64_t>(r0 + plan.rows_per_group, d);
  const int64_t ngrp = r1 > r0 ? (r1 - r0 + ROWS - 1) / ROWS : 0;
  const int64_t nk = ngrp > wave ? (ngrp - wave + kWaves - 1) / kWaves : 0;
  const WideRows<T, OFF32> rd(vk, d, sub);
  T* vm_l = vm + sub * PPL;
  // moment partials of probes PPL sub + e, row class q
  double m1[PPL], m2[PPL];
#pragma unroll
  for (int e = 0; e < PPL; ++e) m1[e] = m2[e] = 0.0;
  // SLQ: the lane's probe scales
  double sc[PPL];
  if constexpr (SLQ) {
#pragma unroll
    for (int e = 0; e < PPL; ++e) sc[e] = sdev[PPL * sub + e];
  }
  // ZMODE 1: the key of probe PPL sub + q and the sign words of the lane's
  // probes for the 64-row chunk `cached` (uniform)
  uint64_t word[PPL], keyq = 0;
  int64_t cached = -1;
  if constexpr (ZMODE == 1) {
#pragma unroll
    for (int e = 0; e < PPL; ++e) word[e] = 0;
    keyq = sm_output(src.seed, (uint64_t)(src.first_id + PPL * sub + q));
  }
  auto grp_row0 = [&](int64_t k) { return r0 + (k * kWaves + wave) * ROWS; };
  auto grp_rows = [&](int64_t k) { return (int)min<int64_t>(ROWS, r1 - grp_row0(k)); };

  if (nk > 0) {
    auto load_batch = [&](int64_t j, int& rs, int& rlen) {
      const int64_t k = j * GPB + lane / ROWS;
      const int64_t row = grp_row0(k) + lane % ROWS;
      const bool ok = k < nk && row < r1;
      const int64_t rr = ok ? row : r0;
      rs = rowptr[rr];
      rlen = ok ? rowptr[rr + 1] - rs : 0;
    };
    auto load_cols = [&](const GroupExt<ROWS>& e, int& cj, float& av) {
      const int64_t ce = min<int64_t>((int64_t)e.gs + lane, nnz - 1);
      cj = col[ce];
      av = PATTERN ? 1.f : val[ce];
    };
    const int64_t nbatch = (nk + GPB - 1) / GPB;
    int64_t j = 0;
    int rs, rlen, rs_n = 0, rlen_n = 0;
    load_batch(0, rs, rlen);
    if (nbatch > 1) load_batch(1, rs_n, rlen_n);
    int64_t k = 0;
    GroupExt<ROWS> cur = group_extent<ROWS>(rs, rlen, 0, grp_rows(0));
    int cj = 0;
    float av = 0.f;
    load_cols(cur, cj, av);

    while (true) {
      const int64_t row0 = grp_row0(k);
      V x[H][MAXNZ], xi[H], xp[H];
      float w[H][MAXNZ];
      int len[H];
      int64_t row[H];
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int rr = PPL * h + q;  // this lane's row in the group
        // its offset and length, selected with static indices (the extent
        // stays in registers)
        int off = cur.off[PPL * h];
        len[h] = cur.len[PPL * h];
#pragma unroll
        for (int r = 1; r < PPL; ++r) {
          off = q == r ? cur.off[PPL * h + r] : off;
          len[h] = q == r ? cur.len[PPL * h + r] : len[h];
        }
        row[h] = row0 + min(rr, cur.nr - 1);
#pragma unroll
        for (int t = 0; t < MAXNZ; ++t) {
          const int src = min(off + t, 63);
          x[h][t] = rd(permute_lane(cj, src));
          w[h][t] = PATTERN ? 1.f : __int_as_float(permute_lane(__float_as_int(av), src));
        }
        xi[h] = rd(row[h]);
        if constexpr (HAS_PREV)
          xp[h] = __builtin_nontemporal_load(reinterpret_cast<const V*>(vm_l + row[h] * 64));
        else
          xp[h] = V{};
      }
      // next group: extent and column prefetch
      const int64_t kn = k + 1;
      const bool has_next = kn < nk;
      const bool new_batch = has_next && (kn % GPB) == 0;
      GroupExt<ROWS> nxt = cur;
      int cjn = 0;
      float avn = 0.f;
      if (has_next) {
        const int qn = (int)(kn % GPB) * ROWS;
        nxt = new_batch ? group_extent<ROWS>(rs_n, rlen_n, 0, grp_rows(kn))
                        : group_extent<ROWS>(rs, rlen, qn, grp_rows(kn));
        load_cols(nxt, cjn, avn);
      }
      // ZMODE 1, a group inside one 64-row chunk: each lane hashes the word
      // of one probe, the lane groups exchange them (one hash per lane per
      // chunk, as in the lane = probe body); a group across two chunks
      // hashes per row below
      bool one_chunk = true;
      if constexpr (ZMODE == 1) {
        const int64_t c0 = row0 >> 6;
        one_chunk = ((row0 + ROWS - 1) >> 6) == c0;
        if (one_chunk && c0 != cached) {
          const uint64_t mine = sm_output(keyq, (uint64_t)c0);
          const int lo = (int)(uint32_t)mine, hi = (int)(uint32_t)(mine >> 32);
#pragma unroll
          for (int e = 0; e < PPL; ++e) {
            const int from = e * LPR + sub;  // lane group e holds probe PPL sub + e
            word[e] = (uint64_t)(uint32_t)permute_lane(lo, from) |
                      ((uint64_t)(uint32_t)permute_lane(hi, from) << 32);
          }
          cached = c0;
        }
      }
#pragma unroll
      for (int h = 0; h < H; ++h) {
        T acc[PPL];
#pragma unroll
        for (int e = 0; e < PPL; ++e) acc[e] = T(0);
#pragma unroll
        for (int t = 0; t < MAXNZ; ++t) {
          const float onf = t < len[h] ? 1.f : 0.f;
          const T ww = (T)(PATTERN ? onf : w[h][t] * onf);
#pragma unroll
          for (int e = 0; e < PPL; ++e) acc[e] = fma(ww, x[h][t][e], acc[e]);
        }
        if (SLQ && PPL * h + q < cur.nr) {
          if constexpr (SLQ) {
            V u;
#pragma unroll
            for (int e = 0; e < PPL; ++e) {
              u[e] = sc[e] * acc[e];
              m1[e] += (sc[e] * xi[h][e]) * u[e];
            }
            __builtin_nontemporal_store(u, reinterpret_cast<V*>(vm_l + row[h] * 64));
          }
        } else if (PPL * h + q < cur.nr) {
          V vn;
#pragma unroll
          for (int e = 0; e < PPL; ++e) {
            T v = fma(ca, acc[e], cb * xi[h][e]);
            if (HAS_PREV) v -= xp[h][e];
            vn[e] = v;
          }
          __builtin_nontemporal_store(vn, reinterpret_cast<V*>(vm_l + row[h] * 64));
          if constexpr (ZMODE == 0) {
#pragma unroll
            for (int e = 0; e < PPL; ++e) {
              m1[e] += (double)xi[h][e] * (double)vn[e];
              m2[e] += (double)vn[e] * (double)vn[e];
            }
          } else {
            // (a group across two chunks: the lane's own keys, rehashed)
            uint64_t wd[PPL];
#pragma unroll
            for (int e = 0; e < PPL; ++e)
              wd[e] = one_chunk ? word[e]
                                : sm_output(sm_output(src.seed, (uint64_t)(src.first_id + PPL * sub + e)),
                                            (uint64_t)(row[h] >> 6));
#pragma unroll
            for (int e = 0; e < PPL; ++e)
              m1[e] += sign_from_word<double>(wd[e], row[h]) * (double)vn[e];
          }
        }
      }
      if (!has_next) break;
      if (new_batch) {
        rs = rs_n;
        rlen = rlen_n;
        ++j;
        if (j + 1 < nbatch) load_batch(j + 1, rs_n, rlen_n);
      }
      k = kn;
      cur = nxt;
      cj = cjn;
      av = avn;
    }
  }
  // per probe: each wave's classes in class order, then the waves in order
#pragma unroll
  for (int e = 0; e < PPL; ++e) {
    sh[0][wave][q][PPL * sub + e] = m1[e];
    sh[1][wave][q][PPL * sub + e] = m2[e];
  }
  __syncthreads();
  if (wave == 0) {
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      double t1 = sh[0][w][0][lane], t2 = sh[1][w][0][lane];
#pragma unroll
      for (int c = 1; c < PPL; ++c) {
        t1 += sh[0][w][c][lane];
        t2 += sh[1][w][c][lane];
      }
      if (w == 0) {
        s1 = t1;
        s2 = t2;
      } else {
        s1 += t1;
        s2 += t2;
      }
    }
    part[(size_t)g * 64 + lane] = s1;
    part[((size_t)ngroups + g) * 64 + lane] = s2;
  }
}

// FP32 direct form with 32-bit gather offsets: at least 4 waves per SIMD
// (128 VGPRs; it otherwise takes 132 and drops to 3: 0.729 against 0.673 ms
// per step on the 2D Laplacian 2048^2; the same bound costs the symmetric
// form 2 % and makes the 64-bit-offset form spill)
template <typename T, bool PATTERN, int ZMODE, bool HAS_PREV, int MAXNZ, bool OFF32>
__global__ __launch_bounds__(kThreads, sizeof(T) == 4 && ZMODE == 1 && OFF32 ? 4 : 1) void
csr_step_wide_kernel(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, int64_t d, int64_t nnz, const T* __restrict__ vk,
    T* __restrict__ vm, T ca, T cb, ProbeSrc src, CsrStepPlan plan, double* __restrict__ part) {
  __shared__ WidePartials<T> sh;
  wide_band<T, PATTERN, ZMODE, HAS_PREV, MAXNZ, OFF32>(rowptr, col, val, d, nnz, vk, vm, ca, cb,
                                                        src, plan, part,
                                                        xcd_band(blockIdx.x, plan.ngroups), sh);
}

// Gram step, first product: W = X V_k over X's rows (V_k has dv = X's
// column count rows).
template <typename T, bool PATTERN, int MAXNZ, bool OFF32, int TAIL>
__global__ __launch_bounds__(kThreads) void gram_pass1_kernel(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, int64_t d, int64_t dv, int64_t nnz, const T* __restrict__ vk,
    T* __restrict__ W, HubView hub, CsrStepPlan plan) {
  StoreEpi<T> epi(W);
  csr_step_wg<T, PATTERN, MAXNZ, OFF32, TAIL, false>(rowptr, col, val, d, dv, nnz,
                                                     RowReader<T, OFF32>(vk, dv, lane_id()),
                                                     nullptr, epi, hub, plan, nullptr, blockIdx.x);
}

// Gram step, second product with the recurrence: V_new = ca X^T W + cb V_k
// [- V_prev] over X^T's rows, gathering from W, own rows from V_k.
template <typename T, bool PATTERN, int ZMODE, bool HAS_PREV, int MAXNZ, bool OFF32, int TAIL>
__global__ __launch_bounds__(kThreads) void gram_pass2_kernel(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, int64_t d, int64_t dv, int64_t nnz, const T* __restrict__ W,
    const T* __restrict__ vk, T* __restrict__ vm, T ca, T cb, ProbeSrc src, HubView hub,
    CsrStepPlan plan, double* __restrict__ part) {
  RecEpi<T, ZMODE, HAS_PREV> epi(ca, cb, vm, src);
  csr_step_wg<T, PATTERN, MAXNZ, OFF32, TAIL, true>(rowptr, col, val, d, dv, nnz,
                                                    RowReader<T, OFF32>(W, dv, lane_id()), vk,
                                                    epi, hub, plan, part, blockIdx.x);
}

template <bool PATTERN, int MAXNZ, int TAIL>
__global__ __launch_bounds__(kThreads) void slq_spmm_kernel(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, int64_t d, int64_t nnz, const double* __restrict__ w,
    double* __restrict__ u, const double* __restrict__ sdev, HubView hub, CsrStepPlan plan,
    double* __restrict__ part) {
  if constexpr (TAIL == kTailNone) {
    // rows within the straight-line capacity: the wide form, 2 probes per lane
    __shared__ WidePartials<double> sh;
    wide_band<double, PATTERN, 0, false, MAXNZ, false, true>(
        rowptr, col, val, d, nnz, w, u, 0.0, 0.0, ProbeSrc{}, plan, part,
        xcd_band(blockIdx.x, plan.ngroups), sh, sdev);
  } else {
    SlqEpi epi(u, sdev);
    csr_step_wg<double, PATTERN, MAXNZ, false, TAIL, false>(
        rowptr, col, val, d, d, nnz, RowReader<double, false>(w, d, lane_id()), nullptr, epi,
        hub, plan, part, blockIdx.x);
  }
}

// Integer pass of triangle counting over a pattern CSR: PASS 1 gathers the
// packed signs of z (y = A z written to yout), PASS 2 gathers y (int16).
template <int PASS, int MAXNZ, int TAIL, bool OFF32>
__global__ __launch_bounds__(kThreads) void tri_step_kernel(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col, int64_t d, int64_t nnz,
    const uint64_t* __restrict__ zbits, const int16_t* __restrict__ yin,
    int16_t* __restrict__ yout, HubSide hs, HubView hub, CsrStepPlan plan,
    long long* __restrict__ part) {
  TriEpi<PASS> epi(yout, hs);
  if constexpr (PASS == 1)
    csr_step_wg<int32_t, true, MAXNZ, false, TAIL, false>(
        rowptr, col, nullptr, d, d, nnz, SignBitsReader(zbits, d, lane_id()), nullptr, epi, hub,
        plan, part, blockIdx.x);
  else
    csr_step_wg<int32_t, true, MAXNZ, false, TAIL, false>(
        rowptr, col, nullptr, d, d, nnz, Y16Reader<OFF32>(yin, d, lane_id(), hs), nullptr, epi,
        hub, plan, part, blockIdx.x);
}

// Chunk partials of the hub rows for the triangle passes (as csr_hub_kernel).
template <int PASS, bool OFF32>
__global__ __launch_bounds__(256) void tri_hub_kernel(const int32_t* __restrict__ col, int64_t d,
                                                      const uint64_t* __restrict__ zbits,
                                                      const int16_t* __restrict__ yin,
                                                      HubSide hs, const int32_t* __restrict__ cs,
                                                      const int32_t* __restrict__ ce,
                                                      int nchunks, int32_t* __restrict__ out) {
  const int c = blockIdx.x * 4 + wave_id();
  if (c >= nchunks) return;
  const int lane = lane_id();
  int32_t v;
  if constexpr (PASS == 1)
    v = row_dot_generic<int32_t, true>(col, nullptr, SignBitsReader(zbits, d, lane), cs[c], ce[c]);
  else
    v = row_dot_generic<int32_t, true>(col, nullptr, Y16Reader<OFF32>(yin, d, lane, hs), cs[c],
                                       ce[c]);
  out[(int64_t)c * 64 + lane] = v;
}

// Chunk partials of the hub rows: one wave per chunk of at most kHubChunk
// entries, sum over the chunk of A[i][j] V_k[j] (exact for int32).
template <typename T, bool PATTERN, bool OFF32>
__global__ __launch_bounds__(256) void csr_hub_kernel(const int32_t* __restrict__ col,
                                                      const float* __restrict__ val, int64_t d,
                                                      const T* __restrict__ vk,
                                                      const int32_t* __restrict__ cs,
                                                      const int32_t* __restrict__ ce,
                                                      int nchunks, T* __restrict__ out) {
  const int c = blockIdx.x * 4 + wave_id();
  if (c >= nchunks) return;
  const int lane = lane_id();
  const RowReader<T, OFF32> rd(vk, d, lane);
  out[(int64_t)c * 64 + lane] = row_dot_generic<T, PATTERN>(col, val, rd, cs[c], ce[c]);
}

// Equal-work row bands by binary search on rowptr[r] + kBandRowCost * r.
__global__ __launch_bounds__(256) void csr_band_kernel(const int32_t* __restrict__ rowptr,
                                                       int64_t d, int ngroups,
                                                       int32_t* __restrict__ band) {
  const int g = blockIdx.x * 256 + threadIdx.x;
  if (g > ngroups) return;
  const int64_t base = rowptr[0];
  const int64_t work = (int64_t)rowptr[d] - base + kBandRowCost * d;
  const int64_t target = work * g / ngroups;
  int64_t lo = 0, hi = d;  // f(d) = work >= target
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)rowptr[mid] - base + kBandRowCost * mid >= target) hi = mid;
    else lo = mid + 1;
  }
  band[g] = (int32_t)lo;
}

// Rows longer than kHubLen: (row, start, end) triples in any order; the host
// sorts them by row.
__global__ __launch_bounds__(256) void hub_find_kernel(const int32_t* __restrict__ rowptr,
                                                       int64_t d, int32_t* __restrict__ out,
                                                       int32_t* __restrict__ count, int cap) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < d;
       i += (int64_t)gridDim.x * 256) {
    const int32_t s = rowptr[i], e = rowptr[i + 1];
    if (e - s > kHubLen) {
      const int slot = atomicAdd(count, 1);
      if (slot < cap) {
        out[3 * (int64_t)slot] = (int32_t)i;
        out[3 * (int64_t)slot + 1] = s;
        out[3 * (int64_t)slot + 2] = e;
      }
    }
  }
}

// ---- batches of probe blocks over many operators -----------------------------
// One launch covers step s of every block in a table (blocks sorted by their
// number of steps, so the blocks still running at step s are a prefix).  Each
// block's workgroups are a contiguous, 8-aligned range of the grid; a
// workgroup finds its block by binary search over the ranges' starts.
__device__ __forceinline__ int find_block(const BatchBlock* __restrict__ tab, int n, int64_t bid) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].group_base <= bid) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <bool PATTERN, int ZMODE, bool HAS_PREV, int MAXNZ, int TAIL>
__global__ __launch_bounds__(kThreads) void csr_step_batched_kernel(
    const BatchBlock* __restrict__ tab, const int32_t* __restrict__ xblk,
    const int32_t* __restrict__ xg0, const int64_t* __restrict__ xbase, XcdLaunch xl, int s) {
  const int x = blockIdx.x & 7;
  const int64_t slot = blockIdx.x >> 3;
  if (slot >= xl.slots[x]) return;  // this XCD has no more work in the launch
  int lo = xl.first[x], hi = xl.first[x] + xl.count[x] - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (xbase[mid] <= slot) lo = mid; else hi = mid - 1;
  }
  const int bi = __builtin_amdgcn_readfirstlane(xblk[lo]);
  const BatchBlock& B = tab[bi];
  // band g of the block; bid is the index whose xcd_band is g
  const int g = xg0[lo] + (int)(slot - xbase[lo]);
  const int per = B.ngroups >> 3;
  const int bid = (g % per) * 8 + g / per;
  const float* vk = (s - 1) & 1 ? B.v1 : B.v0;
  float* vm = s & 1 ? B.v1 : B.v0;
  const float ca = (float)(HAS_PREV ? 2.0 * B.alpha : B.alpha);
  const float cb = (float)(HAS_PREV ? 2.0 * B.beta : B.beta);
  const CsrStepPlan plan{B.ngroups, B.rows_per_group, B.band};
  double* part = B.part + (size_t)s * 2 * B.ngroups * 64;
  if constexpr (ZMODE <= 1 && TAIL == kTailNone) {
    // the single-operator step's wide form (same bits)
    __shared__ WidePartials<float> sh;
    wide_band<float, PATTERN, ZMODE, HAS_PREV, MAXNZ, true>(B.rowptr, B.col, B.val, B.d, B.nnz, vk,
                                                             vm, ca, cb, B.src, plan, part, g, sh);
  } else {
    RecEpi<float, ZMODE, HAS_PREV, false, TAIL == kTailNone ? 4 : 1> epi(ca, cb, vm, B.src);
    const HubView nohub{nullptr, nullptr, 0, nullptr};
    csr_step_wg<float, PATTERN, MAXNZ, true, TAIL, false>(
        B.rowptr, B.col, B.val, B.d, B.d, B.nnz, RowReader<float, true>(vk, B.d, lane_id()),
        nullptr, epi, nohub, plan, part, bid);
  }
}

// ---- one persistent launch for the steps of a batch ---------------------------
// Step 1 of every block runs as a plain batched launch; steps 2 .. S run in
// one launch whose grid is sized to be resident all at once (cooperative
// launch).  The workgroups of XCD x share that XCD's slot list (the layout
// of the batched launches): at step s, slots 0 .. slots_at[s][x] - 1 belong
// to the blocks still running, and workgroup j of the XCD takes slots j,
// j + P_x, ... .  Before a band of block b starts step s, every band of b
// must have finished step s - 1 (its vector is gathered from all rows); a
// band's arrival is counted in cnt[b] after its writes are released at
// device scope, and the wait acquires them.  A workgroup finishes all its
// step-(s - 1) slots before any step-s slot, so every wait ends once all
// workgroups are resident.  A wait longer than spin_ticks of the 100 MHz
// real-time clock (or a raised abort flag) sets the flag and ends the
// kernel, so no wave can wait forever.
struct PersistLaunch {
  int first[8];            // the XCD's first entry
  int count[8];            // its entries
  int per_xcd;             // workgroups per XCD in the grid
  int steps;               // largest step count
  const int64_t* slots_at; // [steps + 1][8] running slots per XCD and step
  int* cnt;                // [nblocks] band arrivals from step 2 on, zero at launch
  int* abort_flag;         // set on a wait that timed out
  long long spin_ticks;
};

__device__ __forceinline__ bool persist_wait(const PersistLaunch& pl, int blk, int target) {
  __shared__ int ok;
  if (threadIdx.x == 0) {
    const long long t0 = (long long)__builtin_amdgcn_s_memrealtime();
    ok = 1;
    while (__hip_atomic_load(pl.cnt + blk, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(pl.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
          (long long)__builtin_amdgcn_s_memrealtime() - t0 > pl.spin_ticks) {
        __hip_atomic_store(pl.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();
  return ok != 0;
}

// ZMODE: the moment form of steps 2 .. S (0 symmetric, 1 direct).  A
// workgroup's consecutive slots of one block share one wait and one
// release (its arrivals are added together before it waits on another
// block or leaves the step).
template <bool PATTERN, int ZMODE, int MAXNZ, int TAIL>
__global__ __launch_bounds__(kThreads) void csr_batch_persistent_kernel(
    const BatchBlock* __restrict__ tab, const int32_t* __restrict__ xblk,
    const int32_t* __restrict__ xg0, const int64_t* __restrict__ xbase, PersistLaunch pl) {
  const int x = blockIdx.x & 7;
  const int j = blockIdx.x >> 3;
  auto release = [&](int blk, int n) {
    __syncthreads();  // every wave's rows and partials are written
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(pl.cnt + blk, n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  };
  for (int s = 2; s <= pl.steps; ++s) {
    const int64_t nslots = pl.slots_at[(size_t)s * 8 + x];
    int held = -1, pending = 0;  // block whose barrier this step has passed; arrivals owed
    for (int64_t slot = j; slot < nslots; slot += pl.per_xcd) {
      int lo = pl.first[x], hi = pl.first[x] + pl.count[x] - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (xbase[mid] <= slot) lo = mid; else hi = mid - 1;
      }
      const int bi = __builtin_amdgcn_readfirstlane(xblk[lo]);
      const BatchBlock& B = tab[bi];
      const int g = xg0[lo] + (int)(slot - xbase[lo]);
      const int per = B.ngroups >> 3;
      const int bid = (g % per) * 8 + g / per;
      if (bi != held) {
        if (pending) release(held, pending);
        pending = 0;
        if (s > 2 && !persist_wait(pl, bi, (s - 2) * B.ngroups)) return;
        held = bi;
      }
      const float* vk = (s - 1) & 1 ? B.v1 : B.v0;
      float* vm = s & 1 ? B.v1 : B.v0;
      const float ca = (float)(2.0 * B.alpha), cb = (float)(2.0 * B.beta);
      const CsrStepPlan plan{B.ngroups, B.rows_per_group, B.band};
      double* part = B.part + (size_t)s * 2 * B.ngroups * 64;
      if constexpr (ZMODE <= 1 && TAIL == kTailNone) {
        __shared__ WidePartials<float> sh;
        wide_band<float, PATTERN, ZMODE, true, MAXNZ, true>(B.rowptr, B.col, B.val, B.d, B.nnz, vk,
                                                             vm, ca, cb, B.src, plan, part, g, sh);
      } else {
        RecEpi<float, ZMODE, true, false, TAIL == kTailNone ? 4 : 1> epi(ca, cb, vm, B.src);
        const HubView nohub{nullptr, nullptr, 0, nullptr};
        csr_step_wg<float, PATTERN, MAXNZ, true, TAIL, false>(
            B.rowptr, B.col, B.val, B.d, B.d, B.nnz, RowReader<float, true>(vk, B.d, lane_id()),
            nullptr, epi, nohub, plan, part, bid);
      }
      __syncthreads();  // the step body's shared partial buffer is reused
      ++pending;
    }
    if (pending) release(held, pending);
  }
}

__global__ void fill_zero_i32_kernel(int* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ __launch_bounds__(kThreads) void probe_init_batched_kernel(
    const BatchBlock* __restrict__ tab, int nblocks) {
  const int bi = __builtin_amdgcn_readfirstlane(find_block(tab, nblocks, blockIdx.x));
  const BatchBlock& B = tab[bi];
  const int bid = (int)(blockIdx.x - B.group_base);
  probe_init_wg<float>(B.v0, B.d, B.src, B.rows_per_group, B.ngroups, B.part, bid);
}

// The plan with the matrix's equal-work row bands when they were built for
// this number of workgroups, else with equal row counts.
CsrStepPlan banded(const CsrMat& m, CsrStepPlan p) {
  p.band = (m.band != nullptr && m.band_groups == p.ngroups) ? m.band : nullptr;
  return p;
}

template <typename T, bool PATTERN, int ZMODE, int MAXNZ, bool OFF32, int TAIL>
hipError_t launch_step_t(hipStream_t s, const CsrMat& m, const T* vk, T* vm, T ca, T cb,
                         bool has_prev, ProbeSrc src, const CsrStepPlan& plan, const HubView& hub,
                         double* part) {
  const dim3 grid(plan.ngroups), block(kThreads);
  if constexpr (ZMODE <= 1 && TAIL == kTailNone) {
    if (has_prev)
      csr_step_wide_kernel<T, PATTERN, ZMODE, true, MAXNZ, OFF32><<<grid, block, 0, s>>>(
          m.rowptr, m.col, m.val, m.nrows, m.nnz, vk, vm, ca, cb, src, banded(m, plan), part);
    else
      csr_step_wide_kernel<T, PATTERN, ZMODE, false, MAXNZ, OFF32><<<grid, block, 0, s>>>(
          m.rowptr, m.col, m.val, m.nrows, m.nnz, vk, vm, ca, cb, src, banded(m, plan), part);
  } else {
    if (has_prev)
      csr_step_kernel<T, PATTERN, ZMODE, true, MAXNZ, OFF32, TAIL><<<grid, block, 0, s>>>(
          m.rowptr, m.col, m.val, m.nrows, m.nnz, vk, vm, ca, cb, src, hub, banded(m, plan), part);
    else
      csr_step_kernel<T, PATTERN, ZMODE, false, MAXNZ, OFF32, TAIL><<<grid, block, 0, s>>>(
          m.rowptr, m.col, m.val, m.nrows, m.nnz, vk, vm, ca, cb, src, hub, banded(m, plan), part);
  }
  return hipGetLastError();
}

// Whether gathers from a block of dv rows can use 32-bit offsets (4-byte
// elements, block under 4 GiB).
template <typename T>
bool block_off32(int64_t dv) {
  return sizeof(T) == 4 && (uint64_t)dv * 64 * sizeof(T) <= 0xFFFFFFFFull;
}

HubView hub_view(const CsrMat& m, void* hub_part) {
  return HubView{m.hub_rows, m.hub_c0, m.hub_n, hub_part};
}

// Hub chunk partials of the gathered block v (dv rows) for this step (a
// no-op without hub rows).
template <typename T, bool PATTERN>
hipError_t launch_hubs(hipStream_t s, const CsrMat& m, const T* v, int64_t dv, void* hub_part) {
  if (m.hub_n == 0) return hipSuccess;
  const int grid = (m.hub_chunks + 3) / 4;
  T* out = static_cast<T*>(hub_part);
  if constexpr (sizeof(T) == 4) {
    if (block_off32<T>(dv)) {
      csr_hub_kernel<T, PATTERN, true><<<grid, 256, 0, s>>>(m.col, m.val, dv, v, m.hub_cs,
                                                           m.hub_ce, m.hub_chunks, out);
      return hipGetLastError();
    }
  }
  csr_hub_kernel<T, PATTERN, false><<<grid, 256, 0, s>>>(m.col, m.val, dv, v, m.hub_cs, m.hub_ce,
                                                        m.hub_chunks, out);
  return hipGetLastError();
}

// Row capacity of the straight-line path: the smallest of {4, 5, 8} that
// holds the longest row.  When one does, every group takes the straight-line
// path and the generic loop is not compiled in (kTailNone: it would hold
// registers the straight-line path can use); else MAXNZ = 8 and longer rows
// take the generic loop (kTailGen), and rows past kHubLen the hub partials
// (kTailHubs).  FP32 blocks under 4 GiB use 32-bit gather offsets; FP64 (a
// verification precision) uses one general instantiation.
// F(MAXNZ, OFF32, TAIL) launches one instantiation.
template <typename T, class F>
hipError_t dispatch_shape(const CsrMat& m, int64_t dv, F&& f) {
  using I4 = std::integral_constant<int, 4>;
  using I5 = std::integral_constant<int, 5>;
  using I8 = std::integral_constant<int, 8>;
  using None = std::integral_constant<int, kTailNone>;
  using Gen = std::integral_constant<int, kTailGen>;
  using Hubs = std::integral_constant<int, kTailHubs>;
  if constexpr (sizeof(T) == 4) {
    if (block_off32<T>(dv)) {
      if (m.hub_n > 0) return f(I8(), std::true_type(), Hubs());
      if (m.nnz > 0 && m.max_row_nnz <= 4) return f(I4(), std::true_type(), None());
      if (m.nnz > 0 && m.max_row_nnz <= 5) return f(I5(), std::true_type(), None());
      if (m.nnz > 0 && m.max_row_nnz <= 8) return f(I8(), std::true_type(), None());
      return f(I8(), std::true_type(), Gen());
    }
  }
  if (m.hub_n > 0) return f(I8(), std::false_type(), Hubs());
  if (m.nnz > 0 && m.max_row_nnz <= 4) return f(I4(), std::false_type(), None());
  if (m.nnz > 0 && m.max_row_nnz <= 5) return f(I5(), std::false_type(), None());
  if (m.nnz > 0 && m.max_row_nnz <= 8) return f(I8(), std::false_type(), None());
  return f(I8(), std::false_type(), Gen());
}

template <typename T, bool PATTERN, int ZMODE>
hipError_t launch_step_nz(hipStream_t s, const CsrMat& m, const T* vk, T* vm, T ca, T cb,
                          bool has_prev, ProbeSrc src, const CsrStepPlan& plan, void* hub_part,
                          double* part) {
  const HubView hub = hub_view(m, hub_part);
  if (m.hub_n > 0) {
    const hipError_t e = launch_hubs<T, PATTERN>(s, m, vk, m.ncols, hub_part);
    if (e != hipSuccess) return e;
  }
  return dispatch_shape<T>(m, m.ncols, [&](auto mz, auto off32, auto tail) {
    return launch_step_t<T, PATTERN, ZMODE, decltype(mz)::value, decltype(off32)::value,
                         decltype(tail)::value>(s, m, vk, vm, ca, cb, has_prev, src, plan, hub,
                                                part);
  });
}

template <typename T>
hipError_t launch_step_any(hipStream_t s, const CsrMat& m, const T* vk, T* vm, T ca, T cb,
                           bool has_prev, int zmode, ProbeSrc src, const CsrStepPlan& plan,
                           void* hub_part, double* part) {
  const bool pat = m.val == nullptr;
  if (pat) {
    if (zmode == 0) return launch_step_nz<T, true, 0>(s, m, vk, vm, ca, cb, has_prev, src, plan, hub_part, part);
    if (zmode == 1) return launch_step_nz<T, true, 1>(s, m, vk, vm, ca, cb, has_prev, src, plan, hub_part, part);
    return launch_step_nz<T, true, 2>(s, m, vk, vm, ca, cb, has_prev, src, plan, hub_part, part);
  }
  if (zmode == 0) return launch_step_nz<T, false, 0>(s, m, vk, vm, ca, cb, has_prev, src, plan, hub_part, part);
  if (zmode == 1) return launch_step_nz<T, false, 1>(s, m, vk, vm, ca, cb, has_prev, src, plan, hub_part, part);
  return launch_step_nz<T, false, 2>(s, m, vk, vm, ca, cb, has_prev, src, plan, hub_part, part);
}

template <int PASS, bool OFF32>
hipError_t launch_tri_pass(hipStream_t s, const CsrMat& m, const CsrStepPlan& plan,
                           const uint64_t* zbits, const int16_t* yin, int16_t* yout,
                           const HubSide& hs, const HubView& hub, long long* part) {
  const dim3 grid(plan.ngroups), block(kThreads);
#define MLCT_TRI(M, H)                                                                      \
  tri_step_kernel<PASS, M, H, OFF32><<<grid, block, 0, s>>>(m.rowptr, m.col, m.nrows, m.nnz, \
                                                            zbits, yin, yout, hs, hub,      \
                                                            banded(m, plan), part)
  if (m.hub_n > 0) MLCT_TRI(8, kTailHubs);
  else if (m.nnz > 0 && m.max_row_nnz <= 4) MLCT_TRI(4, kTailNone);
  else if (m.nnz > 0 && m.max_row_nnz <= 5) MLCT_TRI(5, kTailNone);
  else if (m.nnz > 0 && m.max_row_nnz <= 8) MLCT_TRI(8, kTailNone);
  else MLCT_TRI(8, kTailGen);
#undef MLCT_TRI
  return hipGetLastError();
}

// The two products of a Gram step for one pattern/valued and z-mode choice.
template <typename T, bool PATTERN, int ZMODE>
hipError_t launch_gram_z(hipStream_t s, const CsrMat& X, const CsrMat& XT, const T* vk, T* vm,
                         T* W, T ca, T cb, bool has_prev, ProbeSrc src,
                         const CsrStepPlan& pr, const CsrStepPlan& pc, void* hubx_part,
                         void* hubt_part, double* part) {
  hipError_t e = launch_hubs<T, PATTERN>(s, X, vk, X.ncols, hubx_part);
  if (e != hipSuccess) return e;
  const HubView hx = hub_view(X, hubx_part), ht = hub_view(XT, hubt_part);
  e = dispatch_shape<T>(X, X.ncols, [&](auto mz, auto off32, auto tail) {
    gram_pass1_kernel<T, PATTERN, decltype(mz)::value, decltype(off32)::value,
                      decltype(tail)::value><<<pr.ngroups, kThreads, 0, s>>>(
        X.rowptr, X.col, X.val, X.nrows, X.ncols, X.nnz, vk, W, hx, banded(X, pr));
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  e = launch_hubs<T, PATTERN>(s, XT, W, XT.ncols, hubt_part);
  if (e != hipSuccess) return e;
  return dispatch_shape<T>(XT, XT.ncols, [&](auto mz, auto off32, auto tail) {
    if (has_prev)
      gram_pass2_kernel<T, PATTERN, ZMODE, true, decltype(mz)::value, decltype(off32)::value,
                        decltype(tail)::value><<<pc.ngroups, kThreads, 0, s>>>(
          XT.rowptr, XT.col, XT.val, XT.nrows, XT.ncols, XT.nnz, W, vk, vm, ca, cb, src, ht,
          banded(XT, pc), part);
    else
      gram_pass2_kernel<T, PATTERN, ZMODE, false, decltype(mz)::value, decltype(off32)::value,
                        decltype(tail)::value><<<pc.ngroups, kThreads, 0, s>>>(
          XT.rowptr, XT.col, XT.val, XT.nrows, XT.ncols, XT.nnz, W, vk, vm, ca, cb, src, ht,
          banded(XT, pc), part);
    return hipGetLastError();
  });
}


// ---- two recurrence steps per launch ------------------------------------------
// For operators whose rows have at most 5 entries and whose columns lie
// within a bandwidth of the row (every column of a row in tile j lies in
// tiles j - w .. j + w), one launch applies the recurrence (Section 2.2, eq.
// eqn:recurrence) twice:
//   sub-step 1 on tile j: V_{s+1} = ca1 A V_s + cb1 V_s (- V_{s-1}) over V_{s-1}
//   sub-step 2 on tile j: V_{s+2} = ca2 A V_{s+1} + cb2 V_{s+1} - V_s  over V_s
// each tile through csr_step_wg, the single-step kernel's body, so every
// vector entry is bitwise the single-step path's (only the association of
// the FP64 moment sums follows the tiles).
//
// Work order: the tiles are split into eight contiguous ranges, one per XCD
// (read from the hardware XCC_ID register), and the workgroups of an XCD
// take tickets from that XCD's counter: sub-step 1 of its first L tiles,
// then alternately one sub-step 2 and the sub-step 1 L tiles ahead; the
// sub-steps 2 run from the range's tile w upward and its first w tiles come
// last.  With L > 2 w every sub-step 2 of the range was issued after the
// sub-steps 1 it gathers from inside the range; the first w tiles, which
// also gather from the top of the range below, wait for it at the end.
// Sub-steps 1 never wait, so every wait ends whether or not all workgroups
// are resident; waits are bounded by the real-time clock and an abort flag
// besides.  The lag L (chosen > 2 w + 64) leaves a tile's neighbours time to
// finish before its sub-step 2 claims them; V_{s+1} and V_s are then still
// in the memory-side cache, so the block vectors cross HBM about four times
// per two steps instead of six.
//
// Coherence: within an XCD a writer's stores complete (to the XCD's L2)
// before its tile flag is set, and a waiter polls the flags past its L1 and
// invalidates its L1 before gathering.  Tiles read by another XCD (the
// first and last w of a range) are released and acquired at device scope.
struct Fused2Args {
  const int32_t* rowptr;
  const int32_t* col;
  const float* val;
  int64_t d, nnz;
  float* x;  // V_{s-1} in, V_{s+1} out
  float* y;  // V_s in, V_{s+2} out
  float ca1, cb1, ca2, cb2;
  ProbeSrc src;
  int rows_per_tile, ntiles, window, lag;
  int two;        // 1: both sub-steps; 0: sub-step 1 only
  double* part1;  // [2][ntiles][64] partials of sub-step 1
  double* part2;  // [2][ntiles][64] partials of sub-step 2
  int* tickets;   // [8] ticket counters, zero at launch
  int* done;      // [ntiles] sub-step 1 completion flags, zero at launch
  int* abort_flag;
  long long spin_ticks;
};

// Ticket k of an XCD's range of per tiles -> (sub-step, tile in the range).
__device__ __forceinline__ void fused_ticket(int k, int per, int lag, int w, int two, int& sub,
                                             int& t) {
  if (!two) {
    sub = 1;
    t = k;
    return;
  }
  const int L = min(lag, per);
  if (k < L) {
    sub = 1;
    t = k;
    return;
  }
  const int m = k - L;
  const int pairs = per - L;
  int j;
  if (m < 2 * pairs) {
    if (m & 1) {
      sub = 1;
      t = (m >> 1) + L;
      return;
    }
    j = m >> 1;
  } else {
    j = pairs + (m - 2 * pairs);
  }
  sub = 2;
  t = j + w < per ? j + w : j + w - per;
}

// Thread 0 waits for the flags of tiles t0 .. t1; far: some lie in another
// XCD's range (acquire at device scope), else the L1 is invalidated.
__device__ __forceinline__ bool fused_wait(const Fused2Args& a, int t0, int t1, bool far) {
  __shared__ int ok;
  if (threadIdx.x == 0) {
    ok = 1;
    const long long c0 = (long long)__builtin_amdgcn_s_memrealtime();
    for (int t = t0; t <= t1 && ok; ++t) {
      while (__hip_atomic_load(a.done + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        if (__hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
            (long long)__builtin_amdgcn_s_memrealtime() - c0 > a.spin_ticks) {
          __hip_atomic_store(a.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    if (far)
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    else
      asm volatile("buffer_inv sc0" ::: "memory");
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(ok) != 0;
}

template <bool PATTERN, int Z1, int Z2, bool PREV1, int MAXNZ, bool OFF32>
__global__ __launch_bounds__(kThreads) void csr_fused2_kernel(Fused2Args a) {
  __shared__ int tk;
  const int xcd = xcc_of_wg();
  const int per = a.ntiles >> 3;
  const int base = xcd * per;
  const int total = a.two ? 2 * per : per;
  const int w = a.window;
  CsrStepPlan plan;
  plan.ngroups = a.ntiles;
  plan.rows_per_group = a.rows_per_tile;
  plan.band = nullptr;
  const HubView hub{nullptr, nullptr, 0, nullptr};
  // Thread 0 sets the flag of the sub-step-1 tile just done and claims the
  // next ticket in one block at the loop head, and the ticket is made
  // wave-uniform: the loop's control flow is then uniform, so no lane of
  // wave 0 can be split off into a loop of its own (two adjacent thread-0
  // blocks let the compiler send the other lanes straight back to the
  // barrier, where they re-read the old ticket).
  int pending = -1;
  bool pending_far = false;
  while (true) {
    if (threadIdx.x == 0) {
      if (pending >= 0) {
        if (pending_far)
          __hip_atomic_store(a.done + pending, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        else
          __hip_atomic_store(a.done + pending, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      tk = atomicAdd(a.tickets + xcd, 1);
    }
    __syncthreads();
    const int k = __builtin_amdgcn_readfirstlane(tk);
    __syncthreads();  // tk is rewritten by the next claim
    if (k >= total) break;
    int sub, t;
    fused_ticket(k, per, a.lag, w, a.two, sub, t);
    const int bid = t * 8 + xcd;  // the workgroup index whose band is tile base + t
    if (sub == 1) {
      RecEpi<float, Z1, PREV1, true, 4> epi(a.ca1, a.cb1, a.x, a.src);
      csr_step_wg<float, PATTERN, MAXNZ, OFF32, kTailNone, false>(
          a.rowptr, a.col, a.val, a.d, a.d, a.nnz, RowReader<float, OFF32>(a.y, a.d, lane_id()),
          nullptr, epi, hub, plan, a.part1, bid);
      // every wave's stores complete (in L2) before the flag is set
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
      pending = base + t;
      pending_far = t < w || t >= per - w;
    } else {
      pending = -1;
      const int tile = base + t;
      const int t0 = max(0, tile - w), t1 = min(a.ntiles - 1, tile + w);
      if (!fused_wait(a, t0, t1, t0 < base || t1 >= base + per)) break;
      RecEpi<float, Z2, true, false, 4> epi(a.ca2, a.cb2, a.y, a.src);
      csr_step_wg<float, PATTERN, MAXNZ, OFF32, kTailNone, false>(
          a.rowptr, a.col, a.val, a.d, a.d, a.nnz, RowReader<float, OFF32>(a.x, a.d, lane_id()),
          nullptr, epi, hub, plan, a.part2, bid);
    }
  }
}

}  // namespace

CsrStepPlan plan_csr(int64_t d, int max_groups) {
  // the cap is a multiple of 8 so that every XCD band gets whole workgroups
  const int64_t cap = max_groups > 0 ? std::max<int64_t>(8, max_groups / 8 * 8) : 2048;
  int64_t g = (d + 255) / 256;
  g = (g + 7) / 8 * 8;
  if (g > cap) g = cap;
  if (g < 8) g = 8;
  CsrStepPlan p;
  p.ngroups = (int)g;
  p.rows_per_group = (int)((d + g - 1) / g);
  return p;
}

template <typename T>
hipError_t launch_probe_init(hipStream_t s, T* v0, int64_t d, ProbeSrc src,
                             const CsrStepPlan& plan, double* part0) {
  probe_init_kernel<T><<<dim3(plan.ngroups), dim3(kThreads), 0, s>>>(
      v0, d, src, plan.rows_per_group, plan.ngroups, part0);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_csr_step(hipStream_t s, const CsrMat& m, const T* vk, T* vm, T ca, T cb,
                           bool has_prev, int zmode, ProbeSrc src, const CsrStepPlan& plan,
                           void* hub_part, double* part) {
  return launch_step_any<T>(s, m, vk, vm, ca, cb, has_prev, zmode, src, plan, hub_part, part);
}

template <typename T>
hipError_t launch_gram_csr_step(hipStream_t s, const CsrMat& X, const CsrMat& XT, const T* vk,
                                T* vm, T* W, T ca, T cb, bool has_prev, int zmode, ProbeSrc src,
                                const CsrStepPlan& plan_rows, const CsrStepPlan& plan_cols,
                                void* hubx_part, void* hubt_part, double* part) {
#define MLCT_GZ(P, Z)                                                                       \
  return launch_gram_z<T, P, Z>(s, X, XT, vk, vm, W, ca, cb, has_prev, src, plan_rows,      \
                                plan_cols, hubx_part, hubt_part, part)
  if (X.val == nullptr) {
    if (zmode == 0) MLCT_GZ(true, 0);
    if (zmode == 1) MLCT_GZ(true, 1);
    MLCT_GZ(true, 2);
  }
  if (zmode == 0) MLCT_GZ(false, 0);
  if (zmode == 1) MLCT_GZ(false, 1);
  MLCT_GZ(false, 2);
#undef MLCT_GZ
}

hipError_t launch_tri_step(hipStream_t s, const CsrMat& m, int pass, const CsrStepPlan& plan,
                           const uint64_t* zbits, int16_t* y, int32_t* side, void* hub_part,
                           long long* part) {
  const HubView hub = hub_view(m, hub_part);
  const HubSide hs{m.hub_rows, m.hub_n, side};
  const bool off32 = (uint64_t)m.ncols * 64 * sizeof(int16_t) <= 0xFFFFFFFFull;
  if (m.hub_n > 0) {
    const int grid = (m.hub_chunks + 3) / 4;
    int32_t* out = static_cast<int32_t*>(hub_part);
#define MLCT_TH(P, O)                                                                          \
  tri_hub_kernel<P, O><<<grid, 256, 0, s>>>(m.col, m.ncols, zbits, y, hs, m.hub_cs, m.hub_ce, \
                                            m.hub_chunks, out)
    if (pass == 1) MLCT_TH(1, true);
    else if (off32) MLCT_TH(2, true);
    else MLCT_TH(2, false);
#undef MLCT_TH
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (pass == 1) return launch_tri_pass<1, true>(s, m, plan, zbits, nullptr, y, hs, hub, part);
  return off32 ? launch_tri_pass<2, true>(s, m, plan, nullptr, y, nullptr, hs, hub, part)
               : launch_tri_pass<2, false>(s, m, plan, nullptr, y, nullptr, hs, hub, part);
}

hipError_t launch_slq_spmm(hipStream_t s, const CsrMat& m, const double* w, double* u,
                           const double* sdev, const CsrStepPlan& plan, void* hub_part,
                           double* part) {
  const bool pat = m.val == nullptr;
  if (m.hub_n > 0) {
    const hipError_t e = pat ? launch_hubs<double, true>(s, m, w, m.ncols, hub_part)
                             : launch_hubs<double, false>(s, m, w, m.ncols, hub_part);
    if (e != hipSuccess) return e;
  }
  const HubView hub = hub_view(m, hub_part);
  return dispatch_shape<double>(m, m.ncols, [&](auto mz, auto, auto tail) {
    constexpr int MZ = decltype(mz)::value, TL = decltype(tail)::value;
    if (pat)
      slq_spmm_kernel<true, MZ, TL><<<plan.ngroups, kThreads, 0, s>>>(
          m.rowptr, m.col, m.val, m.nrows, m.nnz, w, u, sdev, hub, banded(m, plan), part);
    else
      slq_spmm_kernel<false, MZ, TL><<<plan.ngroups, kThreads, 0, s>>>(
          m.rowptr, m.col, m.val, m.nrows, m.nnz, w, u, sdev, hub, banded(m, plan), part);
    return hipGetLastError();
  });
}

hipError_t launch_csr_bands(hipStream_t s, const int32_t* rowptr, int64_t d, int ngroups,
                            int32_t* band) {
  csr_band_kernel<<<(ngroups + 1 + 255) / 256, 256, 0, s>>>(rowptr, d, ngroups, band);
  return hipGetLastError();
}

hipError_t launch_hub_find(hipStream_t s, const int32_t* rowptr, int64_t d, int32_t* out,
                           int32_t* count, int cap) {
  const int64_t blocks = std::min<int64_t>((d + 255) / 256, 4096);
  hub_find_kernel<<<(int)blocks, 256, 0, s>>>(rowptr, d, out, count, cap);
  return hipGetLastError();
}

hipError_t launch_probe_init_batched(hipStream_t s, const BatchBlock* tab, int nblocks,
                                     int64_t total_groups) {
  probe_init_batched_kernel<<<(unsigned)total_groups, kThreads, 0, s>>>(tab, nblocks);
  return hipGetLastError();
}

hipError_t launch_csr_step_batched(hipStream_t s, const BatchBlock* tab, const int32_t* xblk,
                                   const int32_t* xg0, const int64_t* xbase,
                                   const XcdLaunch& xl, int64_t groups, int step, bool pattern,
                                   int maxnz, int zmode) {
  const bool hp = step > 1;
  const unsigned grid = (unsigned)groups;
#define MLCT_BATCH(P, Z, H, M, T) \
  csr_step_batched_kernel<P, Z, H, M, T><<<grid, kThreads, 0, s>>>(tab, xblk, xg0, xbase, xl, step)
#define MLCT_BATCH_M(P, Z, H)                                                       \
  if (maxnz <= 4) MLCT_BATCH(P, Z, H, 4, kTailNone);                                \
  else if (maxnz <= 5) MLCT_BATCH(P, Z, H, 5, kTailNone);                           \
  else if (maxnz <= 8) MLCT_BATCH(P, Z, H, 8, kTailNone);                           \
  else MLCT_BATCH(P, Z, H, 8, kTailGen)
#define MLCT_BATCH_H(P, Z) \
  if (hp) { MLCT_BATCH_M(P, Z, true); } else { MLCT_BATCH_M(P, Z, false); }
#define MLCT_BATCH_Z(P) \
  if (zmode == 0) { MLCT_BATCH_H(P, 0); } else { MLCT_BATCH_H(P, 1); }
  if (pattern) { MLCT_BATCH_Z(true); } else { MLCT_BATCH_Z(false); }
#undef MLCT_BATCH_Z
#undef MLCT_BATCH_H
#undef MLCT_BATCH_M
#undef MLCT_BATCH
  return hipGetLastError();
}

hipError_t launch_csr_batch_persistent(hipStream_t s, const BatchBlock* tab,
                                       const int32_t* xblk, const int32_t* xg0,
                                       const int64_t* xbase, const XcdLaunch& xl, int steps,
                                       const int64_t* slots_at, int* cnt, int nblocks,
                                       int* abort_flag, int per_xcd, bool pattern, int maxnz,
                                       int zmode, long long spin_ticks) {
  const int64_t nz = nblocks + 1;
  fill_zero_i32_kernel<<<(unsigned)((nz + 255) / 256), 256, 0, s>>>(cnt, nblocks);
  fill_zero_i32_kernel<<<1, 64, 0, s>>>(abort_flag, 1);
  PersistLaunch pl;
  for (int x = 0; x < 8; ++x) {
    pl.first[x] = xl.first[x];
    pl.count[x] = xl.count[x];
  }
  pl.per_xcd = per_xcd;
  pl.steps = steps;
  pl.slots_at = slots_at;
  pl.cnt = cnt;
  pl.abort_flag = abort_flag;
  pl.spin_ticks = spin_ticks;
  void* args[] = {(void*)&tab, (void*)&xblk, (void*)&xg0, (void*)&xbase, (void*)&pl};
  const dim3 grid((unsigned)(8 * per_xcd)), block(kThreads);
#define MLCT_PERSIST(P, Z, M, T)                                                          \
  return hipLaunchCooperativeKernel((const void*)csr_batch_persistent_kernel<P, Z, M, T>, \
                                    grid, block, args, 0, s)
#define MLCT_PERSIST_M(P, Z)                              \
  if (maxnz <= 4) MLCT_PERSIST(P, Z, 4, kTailNone);       \
  else if (maxnz <= 5) MLCT_PERSIST(P, Z, 5, kTailNone);  \
  else if (maxnz <= 8) MLCT_PERSIST(P, Z, 8, kTailNone);  \
  else MLCT_PERSIST(P, Z, 8, kTailGen)
#define MLCT_PERSIST_Z(P) \
  if (zmode == 0) { MLCT_PERSIST_M(P, 0); } else { MLCT_PERSIST_M(P, 1); }
  if (pattern) { MLCT_PERSIST_Z(true); } else { MLCT_PERSIST_Z(false); }
#undef MLCT_PERSIST_Z
#undef MLCT_PERSIST_M
#undef MLCT_PERSIST
}

int csr_batch_persistent_per_xcd(bool pattern, int maxnz, int zmode) {
  int per_cu = 0;
  hipError_t e = hipSuccess;
#define MLCT_OCC(P, Z, M, T)                                                                \
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(                                         \
      &per_cu, (const void*)csr_batch_persistent_kernel<P, Z, M, T>, kThreads, 0)
#define MLCT_OCC_M(P, Z)                              \
  if (maxnz <= 4) MLCT_OCC(P, Z, 4, kTailNone);       \
  else if (maxnz <= 5) MLCT_OCC(P, Z, 5, kTailNone);  \
  else if (maxnz <= 8) MLCT_OCC(P, Z, 8, kTailNone);  \
  else MLCT_OCC(P, Z, 8, kTailGen)
#define MLCT_OCC_Z(P) \
  if (zmode == 0) { MLCT_OCC_M(P, 0); } else { MLCT_OCC_M(P, 1); }
  if (pattern) { MLCT_OCC_Z(true); } else { MLCT_OCC_Z(false); }
#undef MLCT_OCC_Z
#undef MLCT_OCC_M
#undef MLCT_OCC
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return per_cu * cus / 8;
}


hipError_t launch_csr_fused2(hipStream_t s, const CsrMat& m, float* x, float* y, float ca1,
                             float cb1, bool prev1, float ca2, float cb2, bool two, int zm1,
                             int zm2, ProbeSrc src, int rows_per_tile, int ntiles, int window,
                             double* part1, double* part2, int* sync, int* abort_flag,
                             int grid, int lag, int prev_total, long long spin_ticks) {
  // sync: [8] tickets, [ntiles] flags, cleared for every launch (after the
  // previous launch's counters are checked)
  hipError_t e = launch_fused_sync(s, sync, 8 + (int64_t)ntiles, prev_total, abort_flag);
  if (e != hipSuccess) return e;
  Fused2Args a;
  a.rowptr = m.rowptr;
  a.col = m.col;
  a.val = m.val;
  a.d = m.nrows;
  a.nnz = m.nnz;
  a.x = x;
  a.y = y;
  a.ca1 = ca1;
  a.cb1 = cb1;
  a.ca2 = ca2;
  a.cb2 = cb2;
  a.src = src;
  a.rows_per_tile = rows_per_tile;
  a.ntiles = ntiles;
  a.window = window;
  a.lag = lag;
  a.two = two ? 1 : 0;
  a.part1 = part1;
  a.part2 = part2;
  a.tickets = sync;
  a.done = sync + 8;
  a.abort_flag = abort_flag;
  a.spin_ticks = spin_ticks;
  const bool pat = m.val == nullptr;
  const bool off32 = block_off32<float>(m.ncols);
  const int mz = m.max_row_nnz <= 4 ? 4 : 5;
  const dim3 g(grid), b(kThreads);
#define MLCT_F(P, Z1, Z2, PV, M, O) csr_fused2_kernel<P, Z1, Z2, PV, M, O><<<g, b, 0, s>>>(a)
#define MLCT_F_O(P, Z1, Z2, PV, M) \
  if (off32) { MLCT_F(P, Z1, Z2, PV, M, true); } else { MLCT_F(P, Z1, Z2, PV, M, false); }
#define MLCT_F_M(P, Z1, Z2, PV) \
  if (mz == 4) { MLCT_F_O(P, Z1, Z2, PV, 4) } else { MLCT_F_O(P, Z1, Z2, PV, 5) }
#define MLCT_F_PV(P, Z1, Z2) \
  if (prev1) { MLCT_F_M(P, Z1, Z2, true) } else { MLCT_F_M(P, Z1, Z2, false) }
#define MLCT_F_Z(P)                                            \
  if (zm1 == 0 && zm2 == 0) { MLCT_F_PV(P, 0, 0) }             \
  else if (zm1 == 0) { MLCT_F_PV(P, 0, 1) }                    \
  else { MLCT_F_PV(P, 1, 1) }
  if (pat) { MLCT_F_Z(true) } else { MLCT_F_Z(false) }
#undef MLCT_F_Z
#undef MLCT_F_PV
#undef MLCT_F_M
#undef MLCT_F_O
#undef MLCT_F
  return hipGetLastError();
}

template hipError_t launch_probe_init<float>(hipStream_t, float*, int64_t, ProbeSrc,
                                             const CsrStepPlan&, double*);
template hipError_t launch_probe_init<double>(hipStream_t, double*, int64_t, ProbeSrc,
                                              const CsrStepPlan&, double*);
template hipError_t launch_csr_step<float>(hipStream_t, const CsrMat&, const float*, float*,
                                           float, float, bool, int, ProbeSrc,
                                           const CsrStepPlan&, void*, double*);
template hipError_t launch_csr_step<double>(hipStream_t, const CsrMat&, const double*,
                                            double*, double, double, bool, int, ProbeSrc,
                                            const CsrStepPlan&, void*, double*);
template hipError_t launch_gram_csr_step<float>(hipStream_t, const CsrMat&, const CsrMat&,
                                                const float*, float*, float*, float, float, bool,
                                                int, ProbeSrc, const CsrStepPlan&,
                                                const CsrStepPlan&, void*, void*, double*);
template hipError_t launch_gram_csr_step<double>(hipStream_t, const CsrMat&, const CsrMat&,
                                                 const double*, double*, double*, double, double,
                                                 bool, int, ProbeSrc, const CsrStepPlan&,
                                                 const CsrStepPlan&, void*, void*, double*);

}  // namespace mlct
