// Stochastic Lanczos quadrature as a level approximator (the Lanczos-based
// alternative to Chebyshev interpolation named in the paper's
// introduction), inside the multilevel estimator of Sections 2.3 and 4.
//
// A block of 64 probes runs the Lanczos three-term recurrence side by side
// (lane = probe, FP64, no reorthogonalisation), with unnormalised vectors
// w_j and a per-probe scale s_j = 1 / |w_j|:
//   u       = s_j A w_j                     (CSR SpMM, slq_spmm_kernel)
//   a_j     = (s_j w_j) . u
//   w_{j+1} = u - a_j s_j w_j - b_j s_{j-1} w_{j-1},   b_{j+1} = |w_{j+1}|
// A probe whose b_{j+1} falls to 1e-12 max|a| (its Krylov space is
// exhausted) stops with j + 1 diagonal entries.  The Jacobi matrix of each
// probe then goes through the implicit symmetric QR algorithm with
// Wilkinson shifts (Golub & Van Loan, Algorithm 8.3.2), tracking only the
// first row of the eigenvector matrix, and Gauss quadrature gives
// z^T f(A) z ~ |z|^2 sum_i S_{1i}^2 f(theta_i).
#include <cfloat>

#include "device.hpp"

namespace mlct {

namespace {

constexpr int kUT = 256;

// w_{j+1} = u - a s w_j - b s_prev w_{j-1} in place over u, and partials of
// |w_{j+1}|^2 per (workgroup band, probe); slot 1 of the partials is zero.
__global__ __launch_bounds__(kUT) void slq_update_kernel(double* __restrict__ U,
                                                         const double* __restrict__ W1,
                                                         const double* __restrict__ W0,
                                                         const SlqState* __restrict__ st,
                                                         int j, int64_t d, int rows_per_group,
                                                         int ngroups, double* __restrict__ part) {
  __shared__ double sh[kUT / 64][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = xcd_band(blockIdx.x, ngroups);
  const int64_t r0 = (int64_t)g * rows_per_group;
  const int64_t r1 = min<int64_t>(r0 + rows_per_group, d);
  const double a = st->alpha[(int64_t)j * 64 + lane];
  const double c1 = a * st->s_cur[lane];
  const double c0 = st->b_cur[lane] * st->s_prev[lane];
  double acc = 0.0;
  for (int64_t i = r0 + wave; i < r1; i += kUT / 64) {
    const int64_t e = i * 64 + lane;
    const double w = U[e] - c1 * W1[e] - c0 * W0[e];
    U[e] = w;
    acc += w * w;
  }
  sh[wave][lane] = acc;
  __syncthreads();
  if (wave == 0) {
    double t = sh[0][lane];
    for (int w = 1; w < kUT / 64; ++w) t += sh[w][lane];
    part[(int64_t)g * 64 + lane] = t;
    part[((int64_t)ngroups + g) * 64 + lane] = 0.0;
  }
}

// Lane = probe.  init: |z|^2 from the probe fill's partial sums.
__global__ void slq_init_kernel(const double* __restrict__ z2, int k, SlqState* __restrict__ st) {
  const int p = threadIdx.x;
  st->znorm2[p] = z2[p];
  st->s_cur[p] = z2[p] > 0.0 ? 1.0 / sqrt(z2[p]) : 0.0;
  st->s_prev[p] = 0.0;
  st->b_cur[p] = 0.0;
  st->amax[p] = 0.0;
  st->kend[p] = z2[p] > 0.0 ? k : 0;
}

__global__ void slq_alpha_kernel(const double* __restrict__ dots, int j,
                                 SlqState* __restrict__ st) {
  const int p = threadIdx.x;
  const double a = dots[p];
  st->alpha[(int64_t)j * 64 + p] = a;
  if (j < st->kend[p]) st->amax[p] = fmax(st->amax[p], fabs(a));
}

__global__ void slq_beta_kernel(const double* __restrict__ dots, int j, int k,
                                SlqState* __restrict__ st) {
  const int p = threadIdx.x;
  const double b = sqrt(fmax(dots[p], 0.0));
  double s_next = 0.0;
  if (j < st->kend[p]) {
    if (j == k - 1 || b <= 1e-12 * fmax(st->amax[p], DBL_MIN)) {
      st->kend[p] = j + 1;
    } else {
      st->beta[(int64_t)(j + 1) * 64 + p] = b;
      s_next = 1.0 / b;
    }
  }
  st->s_prev[p] = st->s_cur[p];
  st->s_cur[p] = s_next;
  st->b_cur[p] = b;
}

// Eigenvalues (into a) and squared first components of the eigenvectors
// (q^2, q = first row of the eigenvector matrix) of the symmetric
// tridiagonal matrix with diagonal a[0..n) and off-diagonal b[0..n-1)
// (b[i] couples i and i+1), by implicit QR steps with Wilkinson shifts.
__device__ void tridiag_gauss(double* a, double* b, double* q, int n) {
  for (int i = 0; i < n; ++i) q[i] = i == 0 ? 1.0 : 0.0;
  auto small = [&](int i) {  // b[i] negligible against its diagonal neighbours
    return fabs(b[i]) <= DBL_EPSILON * (fabs(a[i]) + fabs(a[i + 1])) || fabs(b[i]) < DBL_MIN;
  };
  int hi = n - 1, iter = 0;
  while (hi > 0) {
    if (small(hi - 1) || iter > 100) {
      b[hi - 1] = 0.0;
      --hi;
      iter = 0;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && !small(lo - 1)) --lo;
    if (lo > 0) b[lo - 1] = 0.0;
    ++iter;
    const double dd = 0.5 * (a[hi - 1] - a[hi]), e = b[hi - 1];
    const double den = dd + (dd >= 0.0 ? 1.0 : -1.0) * hypot(dd, e);
    const double mu = a[hi] - e * e / den;
    double x = a[lo] - mu, z = b[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = hypot(x, z);
      const double c = r > 0.0 ? x / r : 1.0, s = r > 0.0 ? -z / r : 0.0;
      if (k > lo) b[k - 1] = r;
      const double ak = a[k], ak1 = a[k + 1], bk = b[k];
      a[k] = c * c * ak - 2.0 * c * s * bk + s * s * ak1;
      a[k + 1] = s * s * ak + 2.0 * c * s * bk + c * c * ak1;
      b[k] = c * s * (ak - ak1) + (c * c - s * s) * bk;
      const double qk = q[k], qk1 = q[k + 1];
      q[k] = c * qk - s * qk1;
      q[k + 1] = s * qk + c * qk1;
      if (k + 1 < hi) {
        z = -s * b[k + 1];
        b[k + 1] = c * b[k + 1];
        x = b[k];
      }
    }
  }
}

// Lane = probe: q_p = |z|^2 sum_i S_{1i}^2 f(theta_i) * exp(-log_scale);
// scratch: 3 * kmax doubles per probe.
__global__ void slq_quadrature_kernel(const SlqState* __restrict__ st, int kmax, int kind,
                                      double power, double log_scale, int active,
                                      double* __restrict__ scratch, double* __restrict__ out) {
  const int p = threadIdx.x;
  if (p >= active) return;
  const int n = st->kend[p];
  double* a = scratch + (int64_t)p * 3 * kmax;
  double* b = a + kmax;
  double* q = b + kmax;
  for (int i = 0; i < n; ++i) a[i] = st->alpha[(int64_t)i * 64 + p];
  for (int i = 0; i + 1 < n; ++i) b[i] = st->beta[(int64_t)(i + 1) * 64 + p];
  double v = 0.0;
  if (n > 0) {
    tridiag_gauss(a, b, q, n);
    for (int i = 0; i < n; ++i) v += q[i] * q[i] * eval_f(kind, power, a[i]);
  }
  out[p] = st->znorm2[p] * v * exp(-log_scale);
}

// Two-level combination: level 0 = q_cheb on rows [0, m0), level 1 =
// q_slq - q_cheb on rows [m0, m0 + m1); one workgroup, fixed-order sums.
constexpr int kCT = 256;

__device__ double block_sum_cf(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kCT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kCT) void slq_combine_kernel(const double* __restrict__ mu,
                                                          int64_t ldmu, const double* __restrict__ c,
                                                          int n, int64_t m0, int64_t m1,
                                                          const double* __restrict__ qslq,
                                                          double log_scale,
                                                          mlct_result* __restrict__ out) {
  __shared__ double sh[kCT];
  auto qc = [&](int64_t r) {
    double s = 0.0;
    for (int j = 0; j <= n; ++j) s += c[j] * mu[r * ldmu + j];
    return s;
  };
  double mean[2], var[2], mr = 0.0;
  const int64_t mk[2] = {m0, m1};
  for (int lv = 0; lv < 2; ++lv) {
    double s = 0.0;
    for (int64_t p = threadIdx.x; p < mk[lv]; p += kCT) {
      const int64_t r = lv ? m0 + p : p;
      s += lv ? qslq[p] - qc(r) : qc(r);
      for (int j = 0; j <= n; ++j) mr = fmax(mr, fabs(mu[r * ldmu + j]) / mu[r * ldmu]);
    }
    mean[lv] = block_sum_cf(s, sh) / (double)mk[lv];
    double ss = 0.0;
    for (int64_t p = threadIdx.x; p < mk[lv]; p += kCT) {
      const int64_t r = lv ? m0 + p : p;
      const double x = (lv ? qslq[p] - qc(r) : qc(r)) - mean[lv];
      ss += x * x;
    }
    var[lv] = mk[lv] > 1 ? block_sum_cf(ss, sh) / (double)(mk[lv] - 1) : NAN;
  }
  sh[threadIdx.x] = mr;
  __syncthreads();
  for (int s = kCT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double v = mean[0] + mean[1];
    out->value = v;
    out->log_scale = log_scale;
    out->estimate = v * exp(log_scale);
    out->est_var = var[0] / (double)m0 + var[1] / (double)m1;
    for (int k = 0; k < MLCT_MAX_LEVELS; ++k) {
      out->level_mean[k] = k < 2 ? mean[k] : 0.0;
      out->level_var[k] = k < 2 ? var[k] : 0.0;
    }
    out->max_moment_ratio = sh[0];
    uint32_t flags = 0;
    if (m0 < 2 || m1 < 2) flags |= MLCT_FLAG_FEW_SAMPLES;
    if (!isfinite(out->estimate)) flags |= MLCT_FLAG_OVERFLOW;
    out->flags = flags;
  }
}

}  // namespace

hipError_t launch_slq_update(hipStream_t s, double* U, const double* W1, const double* W0,
                             const SlqState* st, int j, int64_t d, const CsrStepPlan& plan,
                             double* part) {
  slq_update_kernel<<<plan.ngroups, kUT, 0, s>>>(U, W1, W0, st, j, d, plan.rows_per_group,
                                                 plan.ngroups, part);
  return hipGetLastError();
}

hipError_t launch_slq_init(hipStream_t s, const double* z2, int k, SlqState* st) {
  slq_init_kernel<<<1, 64, 0, s>>>(z2, k, st);
  return hipGetLastError();
}

hipError_t launch_slq_alpha(hipStream_t s, const double* dots, int j, SlqState* st) {
  slq_alpha_kernel<<<1, 64, 0, s>>>(dots, j, st);
  return hipGetLastError();
}

hipError_t launch_slq_beta(hipStream_t s, const double* dots, int j, int k, SlqState* st) {
  slq_beta_kernel<<<1, 64, 0, s>>>(dots, j, k, st);
  return hipGetLastError();
}

hipError_t launch_slq_quadrature(hipStream_t s, const SlqState* st, int kmax, int kind,
                                 double power, double log_scale, int active, double* scratch,
                                 double* out) {
  slq_quadrature_kernel<<<1, 64, 0, s>>>(st, kmax, kind, power, log_scale, active, scratch, out);
  return hipGetLastError();
}

hipError_t launch_slq_combine(hipStream_t s, const double* mu, int64_t ldmu, const double* c,
                              int n, int64_t m0, int64_t m1, const double* qslq,
                              double log_scale, mlct_result* out) {
  slq_combine_kernel<<<1, kCT, 0, s>>>(mu, ldmu, c, n, m0, m1, qslq, log_scale, out);
  return hipGetLastError();
}

}  // namespace mlct
