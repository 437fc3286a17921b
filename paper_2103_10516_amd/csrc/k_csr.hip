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
#include "device.hpp"

namespace mlct {

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = kWaves * 64;

template <typename T>
__device__ __forceinline__ void store_partials(double a1, double a2, int g, int ngroups,
                                               double* __restrict__ part) {
  __shared__ double sh[2][kWaves][64];
  const int lane = lane_id(), wave = wave_id();
  sh[0][wave][lane] = a1;
  sh[1][wave][lane] = a2;
  __syncthreads();
  if (wave == 0) {
    double s1 = sh[0][0][lane], s2 = sh[1][0][lane];
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
__global__ __launch_bounds__(kThreads) void probe_init_kernel(T* __restrict__ v0, int64_t d,
                                                              ProbeSrc src, int rows_per_group,
                                                              int ngroups,
                                                              double* __restrict__ part) {
  const int lane = lane_id(), wave = wave_id();
  const int g = xcd_band(blockIdx.x, ngroups);
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
  store_partials<T>(acc, 0.0, g, ngroups, part);
}

// Per-row epilogue: V_new = ca*acc + cb*V_k[i] (- V_prev[i]), written over
// V_prev with a non-temporal store, and the lane's moment partials.
template <typename T, int ZMODE, bool HAS_PREV>
__device__ __forceinline__ void finish_row(int64_t i, T acc, T xi, T xp, T ca, T cb,
                                           T* __restrict__ vm, const ProbeSrc& src, bool act,
                                           uint64_t key, int64_t& cached, uint64_t& word,
                                           double& acc1, double& acc2) {
  const int lane = lane_id();
  T vn = ca * acc + cb * xi;
  if (HAS_PREV) vn -= xp;
  __builtin_nontemporal_store(vn, vm + i * 64 + lane);
  if (ZMODE == 0) {
    acc1 += (double)xi * (double)vn;
    acc2 += (double)vn * (double)vn;
  } else if (ZMODE == 1) {
    const int64_t c = i >> 6;
    if (c != cached) {
      word = sm_output(key, (uint64_t)c);
      cached = c;
    }
    acc1 += sign_from_word<double>(word, i) * (double)vn;
  } else {
    const double z = act ? (double)src.entries[i * src.ld + src.first_id + lane] : 0.0;
    acc1 += z * (double)vn;
  }
}

// Generic row: loop over 64-entry chunks of the row's columns.
template <typename T, bool PATTERN>
__device__ __forceinline__ T row_dot_generic(const int32_t* __restrict__ col,
                                             const float* __restrict__ val,
                                             const T* __restrict__ vk, int s, int e) {
  const int lane = lane_id();
  T acc = T(0);
  for (int base = s; base < e; base += 64) {
    const int c = min(64, e - base);
    int cj = 0;
    float av = 0.f;
    if (lane < c) {
      cj = col[base + lane];
      if (!PATTERN) av = val[base + lane];
    }
    int t = 0;
    for (; t + 4 <= c; t += 4) {
      const T x0 = vk[(int64_t)read_lane(cj, t) * 64 + lane];
      const T x1 = vk[(int64_t)read_lane(cj, t + 1) * 64 + lane];
      const T x2 = vk[(int64_t)read_lane(cj, t + 2) * 64 + lane];
      const T x3 = vk[(int64_t)read_lane(cj, t + 3) * 64 + lane];
      if (PATTERN) {
        acc += (x0 + x1) + (x2 + x3);
      } else {
        acc = fma((T)read_lane(av, t), x0, acc);
        acc = fma((T)read_lane(av, t + 1), x1, acc);
        acc = fma((T)read_lane(av, t + 2), x2, acc);
        acc = fma((T)read_lane(av, t + 3), x3, acc);
      }
    }
    for (; t < c; ++t) {
      const T x = vk[(int64_t)read_lane(cj, t) * 64 + lane];
      if (PATTERN)
        acc += x;
      else
        acc = fma((T)read_lane(av, t), x, acc);
    }
  }
  return acc;
}

// Rows are taken in batches of 64 per wave (lane l holds the extent of row
// b0 + l), and within a batch in groups of kGroupRows rows whose column
// indices arrive in one coalesced load.  When every row of a group has at
// most MAXNZ entries, the group's gathers are issued as straight-line code
// (unused slots gather the row itself with weight 0), so all of them are in
// flight before the first is consumed.  Other groups take the generic loop.
constexpr int kGroupRows = 4;

template <typename T, bool PATTERN, int ZMODE, bool HAS_PREV, int MAXNZ>
__global__ __launch_bounds__(kThreads) void csr_step_kernel(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, int64_t d, int64_t nnz, const T* __restrict__ vk,
    T* __restrict__ vm, T ca, T cb, ProbeSrc src, int rows_per_group, int ngroups,
    double* __restrict__ part) {
  const int lane = lane_id(), wave = wave_id();
  const int g = xcd_band(blockIdx.x, ngroups);
  const int64_t r0 = (int64_t)g * rows_per_group;
  const int64_t r1 = min<int64_t>(r0 + rows_per_group, d);
  const bool act = lane < src.active;
  uint64_t key = 0;
  if (ZMODE == 1) key = sm_output(src.seed, (uint64_t)(src.first_id + lane));
  int64_t cached = -1;
  uint64_t word = 0;
  double acc1 = 0.0, acc2 = 0.0;

  for (int64_t b0 = r0 + (int64_t)wave * 64; b0 < r1; b0 += kWaves * 64) {
    const int nb = (int)min<int64_t>(64, r1 - b0);
    const int64_t rl = b0 + min(lane, nb - 1);
    const int rs = rowptr[rl];
    const int rlen = (lane < nb) ? rowptr[rl + 1] - rs : 0;
    for (int q = 0; q < nb; q += kGroupRows) {
      const int nr = min(kGroupRows, nb - q);
      int off[kGroupRows], len[kGroupRows];
      const int gs = read_lane(rs, q);
      int maxlen = 0;
#pragma unroll
      for (int r = 0; r < kGroupRows; ++r) {
        const int rr = min(q + r, nb - 1);
        off[r] = read_lane(rs, rr) - gs;
        len[r] = (r < nr) ? read_lane(rlen, rr) : 0;
        maxlen = max(maxlen, len[r]);
      }
      const int cnt = off[nr - 1] + len[nr - 1];
      if (MAXNZ > 0 && maxlen <= MAXNZ && cnt <= 64 && nnz > 0) {
        // one coalesced load of the group's columns (clamped, always in bounds)
        const int64_t ce = min<int64_t>((int64_t)gs + lane, nnz - 1);
        const int cj = col[ce];
        const float av = PATTERN ? 1.f : val[ce];
        T x[kGroupRows][MAXNZ > 0 ? MAXNZ : 1];
        T xi[kGroupRows], xp[kGroupRows];
#pragma unroll
        for (int r = 0; r < kGroupRows; ++r) {
          const int64_t i = b0 + min(q + r, nb - 1);
#pragma unroll
          for (int t = 0; t < MAXNZ; ++t) {
            const int slot = min(off[r] + t, 63);
            const int j = (t < len[r]) ? read_lane(cj, slot) : (int)i;
            x[r][t] = vk[(int64_t)j * 64 + lane];
          }
          xi[r] = vk[i * 64 + lane];
          xp[r] = HAS_PREV ? __builtin_nontemporal_load(vm + i * 64 + lane) : T(0);
        }
#pragma unroll
        for (int r = 0; r < kGroupRows; ++r) {
          T acc = T(0);
#pragma unroll
          for (int t = 0; t < MAXNZ; ++t) {
            const int slot = min(off[r] + t, 63);
            const float w = (t < len[r]) ? (PATTERN ? 1.f : read_lane(av, slot)) : 0.f;
            acc = fma((T)w, x[r][t], acc);
          }
          if (r < nr)
            finish_row<T, ZMODE, HAS_PREV>(b0 + q + r, acc, xi[r], xp[r], ca, cb, vm, src,
                                           act, key, cached, word, acc1, acc2);
        }
      } else {
        for (int r = 0; r < nr; ++r) {
          const int64_t i = b0 + q + r;
          const int s = gs + off[r];
          const T acc = row_dot_generic<T, PATTERN>(col, val, vk, s, s + len[r]);
          const T xi = vk[i * 64 + lane];
          const T xp = HAS_PREV ? __builtin_nontemporal_load(vm + i * 64 + lane) : T(0);
          finish_row<T, ZMODE, HAS_PREV>(i, acc, xi, xp, ca, cb, vm, src, act, key, cached,
                                         word, acc1, acc2);
        }
      }
    }
  }
  store_partials<T>(acc1, acc2, g, ngroups, part);
}

template <typename T, bool PATTERN, int ZMODE, int MAXNZ>
hipError_t launch_step_t(hipStream_t s, const mlct_op* op, const T* vk, T* vm, T ca, T cb,
                         bool has_prev, ProbeSrc src, const CsrStepPlan& plan, double* part) {
  const dim3 grid(plan.ngroups), block(kThreads);
  const float* val = static_cast<const float*>(op->val);
  if (has_prev)
    csr_step_kernel<T, PATTERN, ZMODE, true, MAXNZ><<<grid, block, 0, s>>>(
        op->rowptr, op->col, val, op->d, op->nnz, vk, vm, ca, cb, src, plan.rows_per_group,
        plan.ngroups, part);
  else
    csr_step_kernel<T, PATTERN, ZMODE, false, MAXNZ><<<grid, block, 0, s>>>(
        op->rowptr, op->col, val, op->d, op->nnz, vk, vm, ca, cb, src, plan.rows_per_group,
        plan.ngroups, part);
  return hipGetLastError();
}

// Row capacity of the straight-line path: the smallest of {4, 8} that holds
// the longest row, else 8 (long rows then take the generic loop).
template <typename T, bool PATTERN, int ZMODE>
hipError_t launch_step_nz(hipStream_t s, const mlct_op* op, const T* vk, T* vm, T ca, T cb,
                          bool has_prev, ProbeSrc src, const CsrStepPlan& plan, double* part) {
  if (op->max_row_nnz <= 4)
    return launch_step_t<T, PATTERN, ZMODE, 4>(s, op, vk, vm, ca, cb, has_prev, src, plan, part);
  return launch_step_t<T, PATTERN, ZMODE, 8>(s, op, vk, vm, ca, cb, has_prev, src, plan, part);
}

template <typename T>
hipError_t launch_step_any(hipStream_t s, const mlct_op* op, const T* vk, T* vm, T ca, T cb,
                           bool has_prev, int zmode, ProbeSrc src, const CsrStepPlan& plan,
                           double* part) {
  const bool pat = op->val == nullptr;
  if (pat) {
    if (zmode == 0) return launch_step_nz<T, true, 0>(s, op, vk, vm, ca, cb, has_prev, src, plan, part);
    if (zmode == 1) return launch_step_nz<T, true, 1>(s, op, vk, vm, ca, cb, has_prev, src, plan, part);
    return launch_step_nz<T, true, 2>(s, op, vk, vm, ca, cb, has_prev, src, plan, part);
  }
  if (zmode == 0) return launch_step_nz<T, false, 0>(s, op, vk, vm, ca, cb, has_prev, src, plan, part);
  if (zmode == 1) return launch_step_nz<T, false, 1>(s, op, vk, vm, ca, cb, has_prev, src, plan, part);
  return launch_step_nz<T, false, 2>(s, op, vk, vm, ca, cb, has_prev, src, plan, part);
}

}  // namespace

CsrStepPlan plan_csr(int64_t d) {
  int64_t g = (d + 255) / 256;
  g = (g + 7) / 8 * 8;
  if (g > 2048) g = 2048;
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
hipError_t launch_csr_step(hipStream_t s, const mlct_op* op, const T* vk, T* vm, T ca, T cb,
                           bool has_prev, int zmode, ProbeSrc src, const CsrStepPlan& plan,
                           double* part) {
  return launch_step_any<T>(s, op, vk, vm, ca, cb, has_prev, zmode, src, plan, part);
}

template hipError_t launch_probe_init<float>(hipStream_t, float*, int64_t, ProbeSrc,
                                             const CsrStepPlan&, double*);
template hipError_t launch_probe_init<double>(hipStream_t, double*, int64_t, ProbeSrc,
                                              const CsrStepPlan&, double*);
template hipError_t launch_csr_step<float>(hipStream_t, const mlct_op*, const float*, float*,
                                           float, float, bool, int, ProbeSrc,
                                           const CsrStepPlan&, double*);
template hipError_t launch_csr_step<double>(hipStream_t, const mlct_op*, const double*,
                                            double*, double, double, bool, int, ProbeSrc,
                                            const CsrStepPlan&, double*);

}  // namespace mlct
