// Recurrence step of a matrix-free operator (mlct_op_callback): the
// caller's function has written W = A V_k for the probe block; this kernel
// finishes the three-term recurrence of Section 2.2 (eq. eqn:recurrence),
//   V_new = ca W + cb V_k (- V_prev),   ca = 2 alpha, cb = 2 beta,
// written over V_prev, with the per-probe moment partials of the CSR step
// (symmetric form: V_k . V_new and V_new . V_new; direct form: z . V_new).
// Layout as the CSR path: V row-major d x 64, probe index fastest, so one
// wavefront moves one 256-byte row segment per load (lane = probe).
#include "device.hpp"

namespace mlct {

namespace {

constexpr int kCbWaves = 8;
constexpr int kCbThreads = kCbWaves * 64;

template <int ZMODE, bool HAS_PREV>
__global__ __launch_bounds__(kCbThreads) void callback_step_kernel(
    const float* __restrict__ w, const float* __restrict__ vk, float* __restrict__ vm, float ca,
    float cb, ProbeSrc src, int64_t d, int rows_per_group, int ngroups,
    double* __restrict__ part) {
  __shared__ double sh[2][kCbWaves][64];
  const int lane = lane_id(), wave = wave_id();
  const int g = xcd_band(blockIdx.x, ngroups);
  const int64_t r0 = (int64_t)g * rows_per_group;
  const int64_t r1 = min<int64_t>(r0 + rows_per_group, d);
  const bool act = lane < src.active;
  uint64_t key = 0, word = 0;
  int64_t cached = -1;
  if (ZMODE == 1) key = sm_output(src.seed, (uint64_t)(src.first_id + lane));
  double a1 = 0.0, a2 = 0.0;
  for (int64_t i = r0 + wave; i < r1; i += kCbWaves) {
    const int64_t e = i * 64 + lane;
    const float xi = vk[e];
    float vn = fmaf(ca, __builtin_nontemporal_load(w + e), cb * xi);
    if (HAS_PREV) vn -= __builtin_nontemporal_load(vm + e);
    __builtin_nontemporal_store(vn, vm + e);
    if (ZMODE == 0) {
      a1 += (double)xi * (double)vn;
      a2 += (double)vn * (double)vn;
    } else if (ZMODE == 1) {
      const int64_t c = i >> 6;
      if (c != cached) {
        word = sm_output(key, (uint64_t)c);
        cached = c;
      }
      a1 += sign_from_word<double>(word, i) * (double)vn;
    } else {
      const double z = act ? (double)src.entries[i * src.ld + src.first_id + lane] : 0.0;
      a1 += z * (double)vn;
    }
  }
  // per-workgroup partials, the waves summed in a fixed order
  sh[0][wave][lane] = a1;
  sh[1][wave][lane] = a2;
  __syncthreads();
  if (wave == 0) {
    double s1 = sh[0][0][lane], s2 = sh[1][0][lane];
#pragma unroll
    for (int k = 1; k < kCbWaves; ++k) {
      s1 += sh[0][k][lane];
      s2 += sh[1][k][lane];
    }
    part[(size_t)g * 64 + lane] = s1;
    part[((size_t)ngroups + g) * 64 + lane] = s2;
  }
}

template <int ZMODE>
hipError_t launch_cb(hipStream_t s, const float* w, const float* vk, float* vm, float ca, float cb,
                     bool has_prev, ProbeSrc src, int64_t d, const CsrStepPlan& plan,
                     double* part) {
  if (has_prev)
    callback_step_kernel<ZMODE, true><<<plan.ngroups, kCbThreads, 0, s>>>(
        w, vk, vm, ca, cb, src, d, plan.rows_per_group, plan.ngroups, part);
  else
    callback_step_kernel<ZMODE, false><<<plan.ngroups, kCbThreads, 0, s>>>(
        w, vk, vm, ca, cb, src, d, plan.rows_per_group, plan.ngroups, part);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_callback_step(hipStream_t s, const float* w, const float* vk, float* vm,
                                float ca, float cb, bool has_prev, int zmode, ProbeSrc src,
                                int64_t d, const CsrStepPlan& plan, double* part) {
  if (zmode == 0) return launch_cb<0>(s, w, vk, vm, ca, cb, has_prev, src, d, plan, part);
  if (zmode == 1) return launch_cb<1>(s, w, vk, vm, ca, cb, has_prev, src, d, plan, part);
  return launch_cb<2>(s, w, vk, vm, ca, cb, has_prev, src, d, plan, part);
}

}  // namespace mlct
