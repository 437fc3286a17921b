// Exact triangle-count moments over a 0/1 pattern CSR (Section 2.1 example
// and footnote, Section 5.4).  Per probe z, two integer SpMMs:
//   pass 1: y = A z   (int32, stored), w1 += z_i y_i, w2 += y_i^2   (int64)
//   pass 2: w = A y   (int32, never stored), w3 += y_i w_i           (int64)
// The passes run on the CSR step machinery (k_csr.hip, launch_tri_step);
// this file holds the probe fill, the reduction of the int64 partials and
// the control-variate fit.
// Layout as in the FP recurrence: blocks are row-major d x 64, lane = probe.
#include "device.hpp"

namespace mlct {

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = kWaves * 64;

__global__ __launch_bounds__(kThreads) void tri_init_kernel(uint64_t* __restrict__ zbits,
                                                            int64_t d, ProbeSrc src,
                                                            int rows_per_group, int ngroups) {
  // z packed one word per row: bit p set where probe p is -1 (lane p finds
  // its sign, a ballot gathers the wave's 64 bits); probes past src.active
  // get +1, which only their own, discarded, sums see
  const int lane = lane_id(), wave = wave_id();
  const int g = xcd_band(blockIdx.x, ngroups);
  const int64_t r0 = (int64_t)g * rows_per_group;
  const int64_t r1 = min<int64_t>(r0 + rows_per_group, d);
  const bool act = lane < src.active;
  const uint64_t key = sm_output(src.seed, (uint64_t)(src.first_id + lane));
  int64_t cached = -1;
  uint64_t word = 0;
  for (int64_t i = r0 + wave; i < r1; i += kWaves) {
    bool neg = false;
    if (act) {
      const int64_t c = i >> 6;
      if (c != cached) {
        word = sm_output(key, (uint64_t)c);
        cached = c;
      }
      neg = sign_from_word<int32_t>(word, i) < 0;
    }
    const uint64_t bits = __ballot(neg);
    if (lane == 0) zbits[i] = bits;
  }
}

// w[(p0 + p) * 3 + slot_out] = sum over groups of the partials: one
// workgroup per (probe, slot), a strided sum per thread and a tree in LDS
// (int64, exact in any order).
constexpr int kRedThreads = 256;

__global__ __launch_bounds__(kRedThreads) void tri_reduce_kernel(
    const long long* __restrict__ part, int ngroups, int active, int pass,
    long long* __restrict__ w, int64_t p0) {
  __shared__ long long sh[kRedThreads];
  const int p = blockIdx.x >> 1, slot = blockIdx.x & 1;
  if (pass == 2 && slot == 1) return;
  long long acc = 0;
  for (int g = threadIdx.x; g < ngroups; g += kRedThreads)
    acc += part[((size_t)slot * ngroups + g) * 64 + p];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int st = kRedThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) w[(p0 + p) * 3 + (pass == 1 ? slot : 2)] = sh[0];
}

// Control variates of Section 5.4: ordinary least squares of w3 on
// [1, w1, w2] (centred normal equations), then
// T_cv = (mean(w3 - a1 w1 - a2 w2) + a1 tr(A) + a2 nnz) / 6 with tr(A) = 0.
// If the centred 2x2 system is singular no control variate is used.
// One workgroup, fixed-order sums.
constexpr int kCvThreads = 256;

__device__ double cv_block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int st = kCvThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ long long cv_block_sum_i(long long v, long long* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int st = kCvThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  const long long r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kCvThreads) void tri_cv_kernel(const long long* __restrict__ w,
                                                            int64_t m, int64_t nnz,
                                                            mlct_tri_result* __restrict__ out) {
  __shared__ double sh[kCvThreads];
  __shared__ long long shi[kCvThreads];
  long long t1 = 0, t2 = 0, t3 = 0;
  for (int64_t p = threadIdx.x; p < m; p += kCvThreads) {
    t1 += w[p * 3];
    t2 += w[p * 3 + 1];
    t3 += w[p * 3 + 2];
  }
  const long long s1 = cv_block_sum_i(t1, shi), s2 = cv_block_sum_i(t2, shi);
  const long long s3 = cv_block_sum_i(t3, shi);
  const double m1 = (double)s1 / m, m2 = (double)s2 / m, m3 = (double)s3 / m;
  double c11 = 0, c12 = 0, c22 = 0, c13 = 0, c23 = 0;
  for (int64_t p = threadIdx.x; p < m; p += kCvThreads) {
    const double x1 = (double)w[p * 3] - m1, x2 = (double)w[p * 3 + 1] - m2;
    const double x3 = (double)w[p * 3 + 2] - m3;
    c11 += x1 * x1;
    c12 += x1 * x2;
    c22 += x2 * x2;
    c13 += x1 * x3;
    c23 += x2 * x3;
  }
  c11 = cv_block_sum(c11, sh);
  c12 = cv_block_sum(c12, sh);
  c22 = cv_block_sum(c22, sh);
  c13 = cv_block_sum(c13, sh);
  c23 = cv_block_sum(c23, sh);
  if (threadIdx.x == 0) {
    double a1 = 0.0, a2 = 0.0;
    const double det = c11 * c22 - c12 * c12;
    if (m >= 3 && det > 1e-12 * c11 * c22 && c11 > 0 && c22 > 0) {
      a1 = (c22 * c13 - c12 * c23) / det;
      a2 = (c11 * c23 - c12 * c13) / det;
    }
    out->sum_w3 = s3;
    out->estimate = (double)s3 / (6.0 * (double)m);
    out->estimate_cv = (m3 - a1 * m1 - a2 * m2 + a2 * (double)nnz) / 6.0;
    out->a1 = a1;
    out->a2 = a2;
  }
}

}  // namespace

hipError_t launch_tri_init(hipStream_t s, const mlct_op* op, ProbeSrc src,
                           const CsrStepPlan& plan, uint64_t* zbits) {
  tri_init_kernel<<<plan.ngroups, kThreads, 0, s>>>(zbits, op->d, src, plan.rows_per_group,
                                                    plan.ngroups);
  return hipGetLastError();
}

hipError_t launch_tri_reduce(hipStream_t s, const long long* part, int ngroups, int active,
                             int pass, long long* w, int64_t p0) {
  if (active <= 0) return hipSuccess;
  tri_reduce_kernel<<<2 * active, kRedThreads, 0, s>>>(part, ngroups, active, pass, w, p0);
  return hipGetLastError();
}

hipError_t launch_tri_cv(hipStream_t s, const long long* w, int64_t m, int64_t nnz,
                         mlct_tri_result* out) {
  tri_cv_kernel<<<1, kCvThreads, 0, s>>>(w, m, nnz, out);
  return hipGetLastError();
}

}  // namespace mlct
