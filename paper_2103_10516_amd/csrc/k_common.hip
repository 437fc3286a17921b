// Small FP64 kernels of libmlct: Chebyshev coefficients (type-I DCT),
// CSR structure validation, fixed-order reduction of moment partials,
// assembly of the moment table, and the multilevel level combination.
#include <cmath>

#include "device.hpp"

namespace mlct {

namespace {

// Coefficients of the degree-n interpolant at x_k = cos(k pi / n)
// (Section 2.2): c_j = (2/n) sum''_k f~(x_k) cos(pi (j k mod 2n) / n), with
// the end terms of the sum and c_0, c_n halved.  For exp the factor
// exp((a+b)/2) is returned separately as a log-scale.  The angle index
// r = j k mod 2n is folded to [0, n/2] (cos(2 pi - t) = cos t,
// cos(pi - t) = -cos t), so each workgroup evaluates n/2 + 1 cosines once
// into LDS; workgroup w computes c_j for j = 256 w .. 256 w + 255, each as
// one sequential sum over k with the index advanced by additions.
__global__ __launch_bounds__(256) void cheb_dct_kernel(int kind, double power, double a,
                                                       double b, int n, double* __restrict__ c,
                                                       double* __restrict__ log_scale) {
  extern __shared__ double lds[];
  double* fk = lds;              // n + 1 samples
  double* cs = lds + (n + 1);    // cos(pi r / n), r = 0 .. n/2
  const double half = 0.5 * (b - a), mid = 0.5 * (a + b);
  const int nh = n / 2;
  for (int k = threadIdx.x; k <= n; k += blockDim.x) {
    const double x = cos(M_PI * (double)k / (double)n);
    fk[k] = (kind == MLCT_EXP) ? exp(half * x) : eval_f(kind, power, half * x + mid);
  }
  for (int r = threadIdx.x; r <= nh; r += blockDim.x) cs[r] = cos(M_PI * (double)r / (double)n);
  __syncthreads();
  const int two_n = 2 * n;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j <= n) {
    double s = 0.0;
    int jk = 0;  // j k mod 2n, advanced by j each step (j <= n < 2n)
    for (int k = 0; k <= n; ++k) {
      const int r = jk > n ? two_n - jk : jk;
      jk += j;
      if (jk >= two_n) jk -= two_n;
      const double cr = (r <= nh) ? cs[r] : -cs[n - r];
      const double w = (k == 0 || k == n) ? 0.5 : 1.0;
      s += w * fk[k] * cr;
    }
    s *= 2.0 / (double)n;
    if (j == 0 || j == n) s *= 0.5;
    c[j] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && log_scale) *log_scale = (kind == MLCT_EXP) ? mid : 0.0;
}

// flags[0]: bit0 rowptr[0] != 0, bit1 decreasing rowptr, bit2 rowptr[d] != nnz,
// bit3 column out of range.  flags[1]: longest row.
__global__ void csr_validate_kernel(const int32_t* __restrict__ rowptr,
                                    const int32_t* __restrict__ col, int64_t d, int64_t ncols,
                                    int64_t nnz, int32_t* __restrict__ flags) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int bad = 0, longest = 0;
  for (int64_t i = tid; i < d; i += stride) {
    const int32_t s = rowptr[i], e = rowptr[i + 1];
    if (e < s) bad |= 2;
    else longest = max(longest, e - s);
  }
  if (tid == 0) {
    if (rowptr[0] != 0) bad |= 1;
    if ((int64_t)rowptr[d] != nnz) bad |= 4;
  }
  for (int64_t t = tid; t < nnz; t += stride) {
    const int32_t j = col[t];
    if (j < 0 || (int64_t)j >= ncols) bad |= 8;
  }
  if (bad) atomicOr(&flags[0], bad);
  if (longest) atomicMax(&flags[1], longest);
}

// dots[s][slot][p] = sum_{g = 0..ngroups-1} part[s][slot][g][p].  One
// workgroup per (s, slot) row and chunk of 64 probes; wave w sums the
// groups g = w, w + 4, w + 8, ... with four interleaved accumulators, and
// the partial sums are combined in a fixed order, so the result does not
// depend on timing.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double* __restrict__ part,
                                                              int ngroups, int width,
                                                              double* __restrict__ dots) {
  __shared__ double sh[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t row = blockIdx.x;
  const int p = blockIdx.y * 64 + lane;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (p < width) {
    const double* src = part + row * ngroups * width + p;
    int g = wave;
    for (; g + 12 < ngroups; g += 16) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += src[(int64_t)(g + 4 * u) * width];
    }
    for (; g < ngroups; g += 4) acc[0] += src[(int64_t)g * width];
  }
  sh[wave][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (wave == 0 && p < width)
    dots[row * width + p] = (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
}

// Moment table rows from the per-step dot products.
// Direct form: mu_0 = z.z, mu_j = z.v_j.
// Symmetric form: mu_1 = v_1.v_0, mu_2 = 2 v_1.v_1 - mu_0,
// mu_{2s-1} = 2 v_s.v_{s-1} - mu_1 and mu_{2s} = 2 v_s.v_s - mu_0 for s >= 2.
__global__ void assemble_moments_kernel(const double* __restrict__ dots, int steps, int width,
                                        int active, int mode, int n, double* __restrict__ mu,
                                        int64_t ldmu) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= active) return;
  auto D = [&](int s, int slot) { return dots[((int64_t)s * 2 + slot) * width + p]; };
  double* row = mu + (int64_t)p * ldmu;
  const double mu0 = D(0, 0);
  row[0] = mu0;
  if (mode == MLCT_DIRECT) {
    for (int j = 1; j <= n; ++j) row[j] = D(j, 0);
    return;
  }
  if (n < 1) return;
  const double mu1 = D(1, 0);
  row[1] = mu1;
  if (n >= 2) row[2] = 2.0 * D(1, 1) - mu0;
  for (int s = 2; s < steps; ++s) {
    if (2 * s - 1 <= n) row[2 * s - 1] = 2.0 * D(s, 0) - mu1;
    if (2 * s <= n) row[2 * s] = 2.0 * D(s, 1) - mu0;
  }
}

constexpr int kCombThreads = 256;

__device__ double block_sum_fixed(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int st = kCombThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ double block_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int st = kCombThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + st]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// One workgroup per level k (eq. def:qlevels):
//   Q^{(p)} = sum_{j = l_{k-1}+1}^{l_k} c_j mu_j^{(p)}   (truncation), or
//   Q^{(p)} = z^T p_{l_k} z - z^T p_{l_{k-1}} z          (separate interpolants),
// then the level mean and the unbiased sample variance, and max |mu_j| / mu_0.
__global__ __launch_bounds__(kCombThreads) void level_stats_kernel(
    const double* __restrict__ mu, int64_t ldmu, const double* __restrict__ coef, LevelDesc lv,
    double* __restrict__ q, double* __restrict__ stats) {
  __shared__ double sh[kCombThreads];
  const int k = blockIdx.x;
  const int hi = lv.degree[k];
  const int lo = k ? lv.degree[k - 1] : -1;
  const int64_t mk = lv.m[k], o = lv.off[k];
  const double* ch = lv.interp ? coef + (int64_t)k * lv.coef_stride : coef;
  const double* cl = (lv.interp && k) ? coef + (int64_t)(k - 1) * lv.coef_stride : nullptr;
  double s = 0.0, mr = 0.0;
  for (int64_t p = threadIdx.x; p < mk; p += kCombThreads) {
    const double* r = mu + (o + p) * ldmu;
    double qv = 0.0;
    if (!lv.interp) {
      for (int j = max(lo + 1, lv.jmin); j <= hi; ++j) qv += ch[j] * r[j];
    } else {
      for (int j = lv.jmin; j <= hi; ++j) qv += ch[j] * r[j];
      if (cl) {
        double ql = 0.0;
        for (int j = lv.jmin; j <= lo; ++j) ql += cl[j] * r[j];
        qv -= ql;
      }
    }
    q[o + p] = qv;
    s += qv;
    const double inv0 = 1.0 / r[0];
    for (int j = 0; j <= hi; ++j) mr = fmax(mr, fabs(r[j]) * inv0);
  }
  const double mean = block_sum_fixed(s, sh) / (double)mk;
  double ss = 0.0;
  for (int64_t p = threadIdx.x; p < mk; p += kCombThreads) {
    const double dlt = q[o + p] - mean;
    ss += dlt * dlt;
  }
  ss = block_sum_fixed(ss, sh);
  mr = block_max(mr, sh);
  if (threadIdx.x == 0) {
    stats[3 * k + 0] = mean;
    stats[3 * k + 1] = mk > 1 ? ss / (double)(mk - 1) : NAN;
    stats[3 * k + 2] = mr;
  }
}

// Multilevel estimator (eq. eqn:multiEstimator): Gamma = sum_k mean_k and
// its variance estimate sum_k s_k^2 / m_k, summed over k in order.
__global__ void level_finalize_kernel(const double* __restrict__ stats, LevelDesc lv,
                                      const double* __restrict__ coef,
                                      const double* __restrict__ log_scale,
                                      mlct_result* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double v = 0.0, var = 0.0, mr = 0.0;
  uint32_t flags = 0;
  // exact low-degree terms with the top interpolant's coefficients
  const int n = lv.degree[lv.L - 1];
  const double* ctop = lv.interp ? coef + (int64_t)(lv.L - 1) * lv.coef_stride : coef;
  for (int j = 0; j < lv.jmin && j <= n; ++j) v += ctop[j] * lv.low_tr[j];
  for (int k = 0; k < lv.L; ++k) {
    v += stats[3 * k];
    if (lv.m[k] > 1) var += stats[3 * k + 1] / (double)lv.m[k];
    else flags |= MLCT_FLAG_FEW_SAMPLES;
    mr = fmax(mr, stats[3 * k + 2]);
    out->level_mean[k] = stats[3 * k];
    out->level_var[k] = stats[3 * k + 1];
  }
  for (int k = lv.L; k < MLCT_MAX_LEVELS; ++k) {
    out->level_mean[k] = 0.0;
    out->level_var[k] = 0.0;
  }
  const double ls = *log_scale;
  const double est = v * exp(ls);
  if (!isfinite(est)) flags |= MLCT_FLAG_OVERFLOW;
  if (flags & MLCT_FLAG_FEW_SAMPLES) var = NAN;
  out->value = v;
  out->log_scale = ls;
  out->estimate = est;
  out->est_var = var;
  out->max_moment_ratio = mr;
  out->flags = flags;
}

}  // namespace

hipError_t launch_cheb_dct(hipStream_t s, int kind, double power, double a, double b, int n,
                           double* c_dev, double* log_scale_dev) {
  const size_t lds = (size_t)(n + 1 + n / 2 + 1) * sizeof(double);
  cheb_dct_kernel<<<(n + 256) / 256, 256, lds, s>>>(kind, power, a, b, n, c_dev, log_scale_dev);
  return hipGetLastError();
}

hipError_t launch_csr_validate(hipStream_t s, const int32_t* rowptr, const int32_t* col,
                               int64_t d, int64_t ncols, int64_t nnz, int32_t* flags_dev) {
  const int64_t work = d > nnz ? d : nnz;
  int64_t blocks = (work + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  csr_validate_kernel<<<(int)blocks, 256, 0, s>>>(rowptr, col, d, ncols, nnz, flags_dev);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(hipStream_t s, const double* part, int steps, int nslots,
                                  int ngroups, int width, double* dots) {
  const dim3 grid(steps * nslots, (width + 63) / 64);
  reduce_partials_kernel<<<grid, 256, 0, s>>>(part, ngroups, width, dots);
  return hipGetLastError();
}

hipError_t launch_assemble_moments(hipStream_t s, const double* dots, int steps, int width,
                                   int active, int mode, int n, double* mu, int64_t ldmu) {
  assemble_moments_kernel<<<(active + 63) / 64, 64, 0, s>>>(dots, steps, width, active, mode,
                                                             n, mu, ldmu);
  return hipGetLastError();
}

hipError_t launch_level_combine(hipStream_t s, const double* mu, int64_t ldmu,
                                const double* coef, const double* log_scale,
                                const LevelDesc& lv, double* q_dev, double* stats_dev,
                                mlct_result* result_dev) {
  level_stats_kernel<<<lv.L, kCombThreads, 0, s>>>(mu, ldmu, coef, lv, q_dev, stats_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  level_finalize_kernel<<<1, 64, 0, s>>>(stats_dev, lv, coef, log_scale, result_dev);
  return hipGetLastError();
}

namespace {

constexpr int kST = 256;

// Per-workgroup partial sums of diag(A) and of A_ij^2 over rows g, g + G, ...
// of one workgroup per row block (one thread per row, FP64).
__global__ __launch_bounds__(kST) void op_stats_kernel(const int32_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ col,
                                                       const float* __restrict__ val,
                                                       const void* __restrict__ A, int dtype,
                                                       int64_t lda, int64_t d,
                                                       double* __restrict__ partial) {
  __shared__ double s1[kST], s2[kST];
  double tr = 0.0, fr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kST + threadIdx.x; i < d;
       i += (int64_t)gridDim.x * kST) {
    if (rowptr) {
      for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        const double a = val ? (double)val[e] : 1.0;
        if (col[e] == i) tr += a;
        fr += a * a;
      }
    } else {
      for (int64_t j = 0; j < d; ++j) {
        const double a = dtype == MLCT_DT_F64 ? static_cast<const double*>(A)[i * lda + j]
                                              : (double)static_cast<const float*>(A)[i * lda + j];
        if (j == i) tr += a;
        fr += a * a;
      }
    }
  }
  s1[threadIdx.x] = tr;
  s2[threadIdx.x] = fr;
  __syncthreads();
  for (int st = kST / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      s1[threadIdx.x] += s1[threadIdx.x + st];
      s2[threadIdx.x] += s2[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s1[0];
    partial[2 * blockIdx.x + 1] = s2[0];
  }
}

__global__ void op_stats_reduce_kernel(const double* __restrict__ partial, int g,
                                       double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double tr = 0.0, fr = 0.0;
  for (int b = 0; b < g; ++b) {
    tr += partial[2 * b];
    fr += partial[2 * b + 1];
  }
  out[0] = tr;
  out[1] = fr;
}

}  // namespace

hipError_t launch_op_stats(hipStream_t s, const mlct_op* op, double* partial, double* out) {
  const int64_t want = (op->d + kST - 1) / kST;
  const int g = (int)(want < kStatsGroups ? want : kStatsGroups);
  const bool csr = op->kind == OP_CSR;
  op_stats_kernel<<<g, kST, 0, s>>>(csr ? op->csr.rowptr : nullptr, csr ? op->csr.col : nullptr,
                                    csr ? op->csr.val : nullptr, csr ? nullptr : op->A, op->dtype,
                                    op->lda, op->d, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  op_stats_reduce_kernel<<<1, 64, 0, s>>>(partial, g, out);
  return hipGetLastError();
}

}  // namespace mlct
