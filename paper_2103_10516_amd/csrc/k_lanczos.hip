// Spectral interval [a, b] for the affine map of Section 2.2 by the Lanczos
// process in FP64 (the paper needs only "a rough estimate" of the extreme
// eigenvalues and gives no procedure; this is the library's choice).
//
// Step j (basis Q = [q_0 .. q_j], q_0 = z / |z| for a Rademacher z):
//   w = A q_j;  h = Q^T w;  w -= Q h;  h' = Q^T w;  w -= Q h'  (classical
//   Gram-Schmidt twice: full reorthogonalisation);
//   alpha_j = h_j + h'_j;  beta_j = |w|;  q_{j+1} = w / beta_j.
// All scalars stay on the device; a step after a breakdown (beta_j tiny) is
// a no-op.  The extreme eigenvalues of the tridiagonal T_k are found by
// Sturm-sequence bisection and the last entries of their eigenvectors by
// inverse iteration, giving the residual bounds |beta_k s_k|.
#include <cmath>

#include "device.hpp"

namespace mlct {

namespace {

constexpr int kT = 256;

__device__ double block_sum256(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int st = kT / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// q_0 = z / |z| with z = Rademacher probe 0 of the seed: |z| = sqrt(d).
__global__ void lz_start_kernel(double* __restrict__ q0, int64_t d, uint64_t seed,
                                LanczosState* st) {
  const uint64_t key = sm_output(seed, 0);
  const double inv = 1.0 / sqrt((double)d);
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < d;
       n += (int64_t)gridDim.x * blockDim.x)
    q0[n] = sign_from_word<double>(sm_output(key, (uint64_t)(n >> 6)), n) * inv;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->k = 0;
    st->stopped = 0;
  }
}

// Sums over the chunks of the rows longer than kHubLen (the matrix's hub
// table): one wave per chunk of at most kHubChunk entries, FP64.
__global__ __launch_bounds__(256) void lz_hub_chunk_kernel(const int32_t* __restrict__ col,
                                                           const float* __restrict__ val,
                                                           const int32_t* __restrict__ cs,
                                                           const int32_t* __restrict__ ce,
                                                           int nchunks,
                                                           const double* __restrict__ q,
                                                           double* __restrict__ out,
                                                           const LanczosState* st) {
  if (st->stopped) return;
  const int c = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (c >= nchunks) return;
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int t = cs[c] + lane; t < ce[c]; t += 64) s += (val ? (double)val[t] : 1.0) * q[col[t]];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) out[c] = s;
}

// w = A q (+ shift * qs when qs is given), CSR, FP64 arithmetic on FP32 or
// implicit-1 values: 16 lanes per row (4 rows per wave), the row's entries
// strided over its lanes (coalesced index and value loads) and added in a
// fixed shuffle tree; a row longer than kHubLen adds its chunk sums
// (lz_hub_chunk_kernel) in chunk order.
__global__ __launch_bounds__(kT) void lz_spmv_kernel(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, int64_t d, const double* __restrict__ q,
    double* __restrict__ w, double shift, const double* __restrict__ qs,
    const int32_t* __restrict__ hub_rows, const int32_t* __restrict__ hub_c0, int hub_n,
    const double* __restrict__ hub_part, const LanczosState* st) {
  if (st->stopped) return;
  const int lane = threadIdx.x & 63, sub = lane & 15;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i0 = wave * 4; i0 < d; i0 += nw * 4) {  // uniform over the wave
    const int64_t i = i0 + (lane >> 4);
    double s = 0.0;
    bool hub = false;
    if (i < d) {
      const int t0 = rowptr[i], t1 = rowptr[i + 1];
      hub = hub_n > 0 && t1 - t0 > kHubLen;
      if (!hub)
        for (int t = t0 + sub; t < t1; t += 16) s += (val ? (double)val[t] : 1.0) * q[col[t]];
    }
    for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);  // within the 16 lanes
    if (sub == 0 && i < d) {
      if (hub) {
        int lo = 0, hi = hub_n - 1;  // the row is in the table
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (hub_rows[mid] < i) lo = mid + 1; else hi = mid;
        }
        s = 0.0;
        for (int c = hub_c0[lo]; c < hub_c0[lo + 1]; ++c) s += hub_part[c];
      }
      if (qs) s += shift * qs[i];
      w[i] = s;
    }
  }
}

// w = M q (+ shift * qs) for one CSR matrix M, long rows through the chunks.
void lz_csr_product(hipStream_t s, const CsrMat& m, int grid, const double* q, double* w,
                    double shift, const double* qs, double* hub_part, const LanczosState* st) {
  if (m.hub_n > 0)
    lz_hub_chunk_kernel<<<(m.hub_chunks + 3) / 4, 256, 0, s>>>(m.col, m.val, m.hub_cs, m.hub_ce,
                                                               m.hub_chunks, q, hub_part, st);
  lz_spmv_kernel<<<grid, kT, 0, s>>>(m.rowptr, m.col, m.val, m.nrows, q, w, shift, qs,
                                     m.hub_rows, m.hub_c0, m.hub_n, hub_part, st);
}

// w = A q (dense FP64, row-major): one wave per row.
__global__ void lz_gemv_kernel(const double* __restrict__ A, int64_t lda, int64_t d,
                               const double* __restrict__ q, double* __restrict__ w,
                               const LanczosState* st) {
  if (st->stopped) return;
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < d; i += nw) {
    double s = 0.0;
    for (int64_t k = lane; k < d; k += 64) s += A[i * lda + k] * q[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) w[i] = s;
  }
}

// part[c][b] = sum over block b's slice of Q[c] . w, for c = 0..ncols-1.
__global__ __launch_bounds__(kT) void lz_dots_kernel(const double* __restrict__ Q, int64_t d,
                                                     const double* __restrict__ w, int ncols,
                                                     double* __restrict__ part,
                                                     const LanczosState* st) {
  __shared__ double sh[kT];
  if (st->stopped) return;
  const int c = blockIdx.y;
  if (c >= ncols) return;
  const double* qc = Q + (int64_t)c * d;
  double s = 0.0;
  for (int64_t n = (int64_t)blockIdx.x * kT + threadIdx.x; n < d; n += (int64_t)gridDim.x * kT)
    s += qc[n] * w[n];
  s = block_sum256(s, sh);
  if (threadIdx.x == 0) part[(int64_t)c * gridDim.x + blockIdx.x] = s;
}

// Sum of part[0 .. nb) by one wave in a fixed order: lane l adds entries
// l, l + 64, ..., then a shuffle tree.  Every lane returns the total.
__device__ double wave_sum_fixed(const double* __restrict__ part, int nb) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int b = lane; b < nb; b += 64) s += part[b];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  return s;
}

// h[c] = sum_b part[c][b], one wave (workgroup) per column c.  mode 0: first
// pass (alpha_j = h_j); mode 1: second pass (alpha_j += h_j).
__global__ __launch_bounds__(64) void lz_dots_reduce_kernel(const double* __restrict__ part,
                                                            int nb, int ncols,
                                                            double* __restrict__ h, int mode,
                                                            int j, LanczosState* st) {
  if (st->stopped) return;
  const int c = blockIdx.x;
  if (c >= ncols) return;
  const double s = wave_sum_fixed(part + (int64_t)c * nb, nb);
  if (threadIdx.x == 0) {
    h[c] = s;
    if (c == j) st->alpha[j] = (mode == 0) ? s : st->alpha[j] + s;
  }
}

// w -= sum_c h[c] Q[c]
__global__ void lz_update_kernel(const double* __restrict__ Q, int64_t d, int ncols,
                                 const double* __restrict__ h, double* __restrict__ w,
                                 const LanczosState* st) {
  if (st->stopped) return;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < d;
       n += (int64_t)gridDim.x * blockDim.x) {
    double s = w[n];
    for (int c = 0; c < ncols; ++c) s -= h[c] * Q[(int64_t)c * d + n];
    w[n] = s;
  }
}

// beta_j = |w| from the partials of w.w; q_{j+1} = w / beta_j, or stop.
__global__ __launch_bounds__(64) void lz_norm_reduce_kernel(const double* __restrict__ part,
                                                            int nb, int j, LanczosState* st) {
  if (st->stopped) return;
  const double s = wave_sum_fixed(part, nb);
  if (threadIdx.x != 0) return;
  const double beta = sqrt(s);
  st->beta[j] = beta;
  st->k = j + 1;
  if (!(beta > 1e-12 * fmax(1.0, fabs(st->alpha[j])))) st->stopped = 1;
}

__global__ void lz_next_kernel(const double* __restrict__ w, int64_t d, int j,
                               double* __restrict__ qn, const LanczosState* st) {
  if (st->stopped) return;
  const double inv = 1.0 / st->beta[j];
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < d;
       n += (int64_t)gridDim.x * blockDim.x)
    qn[n] = w[n] * inv;
}

__device__ int sturm_count(const double* al, const double* be, int k, double x) {
  int cnt = 0;
  double dd = 1.0;
  for (int i = 0; i < k; ++i) {
    const double off = i ? be[i - 1] * be[i - 1] / dd : 0.0;
    dd = al[i] - x - off;
    if (dd == 0.0) dd = -1e-300;
    if (dd < 0) ++cnt;
  }
  return cnt;
}

__device__ double bisect(const double* al, const double* be, int k, int index) {
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < k; ++i) {
    const double r = (i ? fabs(be[i - 1]) : 0.0) + (i + 1 < k ? fabs(be[i]) : 0.0);
    lo = fmin(lo, al[i] - r);
    hi = fmax(hi, al[i] + r);
  }
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(al, be, k, mid) > index)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

// |last entry| of the unit eigenvector of T for eigenvalue theta, by three
// steps of inverse iteration with the tridiagonal (Thomas) solver.
__device__ double last_component(const double* al, const double* be, int k, double theta,
                                 double* x, double* cp, double* dp) {
  const double scale = fmax(fabs(theta), 1e-300);
  for (int i = 0; i < k; ++i) x[i] = 1.0;
  for (int it = 0; it < 3; ++it) {
    // solve (T - theta I) y = x
    for (int i = 0; i < k; ++i) {
      const double sub = i ? be[i - 1] : 0.0;
      double piv = al[i] - theta - (i ? sub * cp[i - 1] : 0.0);
      if (fabs(piv) < 1e-15 * scale) piv = (piv < 0 ? -1e-15 : 1e-15) * scale;
      cp[i] = (i + 1 < k) ? be[i] / piv : 0.0;
      dp[i] = (x[i] - (i ? sub * dp[i - 1] : 0.0)) / piv;
    }
    for (int i = k - 1; i >= 0; --i) x[i] = dp[i] - (i + 1 < k ? cp[i] * x[i + 1] : 0.0);
    double nrm = 0.0;
    for (int i = 0; i < k; ++i) nrm += x[i] * x[i];
    nrm = sqrt(nrm);
    for (int i = 0; i < k; ++i) x[i] /= nrm;
  }
  return fabs(x[k - 1]);
}

__global__ void lz_interval_kernel(LanczosState* st, double margin, double* out) {
  if (threadIdx.x != 0) return;
  const int k = st->k;
  double* x = st->work;
  double* cp = st->work + kLanczosMaxSteps;
  double* dp = st->work + 2 * kLanczosMaxSteps;
  const double tmin = bisect(st->alpha, st->beta, k, 0);
  const double tmax = bisect(st->alpha, st->beta, k, k - 1);
  const double bk = st->beta[k - 1];
  const double rmin = fabs(bk) * last_component(st->alpha, st->beta, k, tmin, x, cp, dp);
  const double rmax = fabs(bk) * last_component(st->alpha, st->beta, k, tmax, x, cp, dp);
  const double w = tmax - tmin;
  out[0] = tmin - rmin - margin * w;
  out[1] = tmax + rmax + margin * w;
  out[2] = tmin;
  out[3] = tmax;
  out[4] = rmin;
  out[5] = rmax;
  out[6] = (double)k;
}

}  // namespace

hipError_t launch_lanczos(hipStream_t s, const mlct_op* op, const void* a64, int64_t lda,
                          int steps, uint64_t seed, double margin, double* Q, double* w,
                          double* h, double* part, LanczosState* st, double* out, double* tmp,
                          double* hub_part) {
  const int64_t d = op->d;
  const int nb = (int)((d + kT - 1) / kT < 1024 ? (d + kT - 1) / kT : 1024);
  const int grid = nb;
  lz_start_kernel<<<grid, kT, 0, s>>>(Q, d, seed, st);
  for (int j = 0; j < steps; ++j) {
    const double* qj = Q + (int64_t)j * d;
    if (op->kind == OP_CSR) {
      lz_csr_product(s, op->csr, grid, qj, w, 0.0, nullptr, hub_part, st);
    } else if (op->kind == OP_GRAM_CSR) {  // w = X^T (X q) + lambda q
      lz_csr_product(s, op->csrx, grid, qj, tmp, 0.0, nullptr, hub_part, st);
      lz_csr_product(s, op->csr, grid, tmp, w, op->gram_lambda, qj, hub_part, st);
    } else
      lz_gemv_kernel<<<grid, kT, 0, s>>>(static_cast<const double*>(a64), lda, d, qj, w, st);
    for (int pass = 0; pass < 2; ++pass) {
      lz_dots_kernel<<<dim3(nb, j + 1), kT, 0, s>>>(Q, d, w, j + 1, part, st);
      lz_dots_reduce_kernel<<<j + 1, 64, 0, s>>>(part, nb, j + 1, h, pass, j, st);
      lz_update_kernel<<<grid, kT, 0, s>>>(Q, d, j + 1, h, w, st);
    }
    lz_dots_kernel<<<dim3(nb, 1), kT, 0, s>>>(w, d, w, 1, part, st);
    lz_norm_reduce_kernel<<<1, 64, 0, s>>>(part, nb, j, st);
    lz_next_kernel<<<grid, kT, 0, s>>>(w, d, j, Q + (int64_t)(j + 1) * d, st);
  }
  lz_interval_kernel<<<1, 64, 0, s>>>(st, margin, out);
  return hipGetLastError();
}

}  // namespace mlct
