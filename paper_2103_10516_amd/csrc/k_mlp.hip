// Learned control-variate level: the cheap truncation of the fine-level
// quadratic form plus a learned correction,
//     g = q_c + mu_0 (ybar + ysd (beta . u + net(u))),
// u = the probe's cheap moments mu_f / mu_0 (f = 1..F-1) standardised over
// the training probes, beta the least-squares fit of the standardised
// target on u (the linear control variate of Section 5.4), and
// net(u) = w3 . tanh(W2 tanh(W1 u + b1) + b2) + b3 (64 hidden units per
// layer) trained on what the linear fit leaves; used as an extra multilevel
// term in the sense of Section 2.3.  Standardising matters: the moments of
// different probes differ by ~1/sqrt(d) relative, far below bf16's
// resolution, so raw inputs would be rounded to constants at inference.
//
// Training (FP32): one wavefront per slice of samples, lane = hidden unit.
// Each lane keeps its row of W1, its row AND column of W2 in registers, so
// the forward pass (h2_l = sum_k W2[l][k] h1_k) and the backward pass
// (dL/dh1_k = sum_l W2[l][k] dL/da2_l) both read the other lanes' values as
// uniform scalars (v_readlane), with no LDS traffic.  Gradients leave each
// wave as one partial per parameter; the Adam kernel sums them in a fixed
// order, so training is deterministic.
// Inference (BF16): weights rounded to bf16 once; inputs and hidden
// activations rounded to bf16 between layers, products accumulated in FP32.
// The same function is used for every probe of both estimator terms.
#include <cmath>

#include "device.hpp"

namespace mlct {

namespace {

constexpr int H = kMlpHidden;
constexpr int FMAX = kMlpMaxFeatures;

struct Off {
  int W1, b1, W2, b2, w3, b3, P;
  __host__ __device__ explicit Off(int F) {
    W1 = 0;
    b1 = H * F;
    W2 = b1 + H;
    b2 = W2 + H * H;
    w3 = b2 + H;
    b3 = w3 + H;
    P = b3 + 1;
  }
};

__device__ __forceinline__ float wave_sum_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(64) void mlp_grad_kernel(const float* __restrict__ theta, int F,
                                                      const float* __restrict__ X,
                                                      const float* __restrict__ y, int N,
                                                      int per_wave, float* __restrict__ part,
                                                      float* __restrict__ loss_part) {
  const Off o(F);
  const int l = threadIdx.x;
  float w1[FMAX], gW1[FMAX];
#pragma unroll
  for (int f = 0; f < FMAX; ++f) {
    w1[f] = f < F ? theta[o.W1 + l * F + f] : 0.f;
    gW1[f] = 0.f;
  }
  float w2r[H], w2c[H], gW2[H];
#pragma unroll
  for (int k = 0; k < H; ++k) {
    w2r[k] = theta[o.W2 + l * H + k];
    w2c[k] = theta[o.W2 + k * H + l];
    gW2[k] = 0.f;
  }
  const float b1 = theta[o.b1 + l], b2 = theta[o.b2 + l], w3 = theta[o.w3 + l];
  const float b3 = theta[o.b3];
  float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, loss = 0.f;
  const int i0 = blockIdx.x * per_wave, i1 = min(N, i0 + per_wave);
  const float scale = 2.f / (float)N;
  for (int i = i0; i < i1; ++i) {
    float x[FMAX];
    float a1 = b1;
#pragma unroll
    for (int f = 0; f < FMAX; ++f) {
      x[f] = f < F ? X[(int64_t)i * F + f] : 0.f;
      a1 = fmaf(w1[f], x[f], a1);
    }
    const float h1 = tanhf(a1);
    float a2 = b2;
#pragma unroll
    for (int k = 0; k < H; ++k) a2 = fmaf(w2r[k], read_lane(h1, k), a2);
    const float h2 = tanhf(a2);
    const float out = wave_sum_f(w3 * h2) + b3;
    const float r = out - y[i];
    loss += r * r;
    const float go = scale * r;
    gw3 = fmaf(go, h2, gw3);
    gb3 += go;
    const float ga2 = go * w3 * (1.f - h2 * h2);
#pragma unroll
    for (int k = 0; k < H; ++k) gW2[k] = fmaf(ga2, read_lane(h1, k), gW2[k]);
    gb2 += ga2;
    float gh1 = 0.f;
#pragma unroll
    for (int m = 0; m < H; ++m) gh1 = fmaf(w2c[m], read_lane(ga2, m), gh1);
    const float ga1 = gh1 * (1.f - h1 * h1);
#pragma unroll
    for (int f = 0; f < FMAX; ++f) gW1[f] = fmaf(ga1, x[f], gW1[f]);
    gb1 += ga1;
  }
  float* p = part + (int64_t)blockIdx.x * o.P;
#pragma unroll
  for (int f = 0; f < FMAX; ++f)
    if (f < F) p[o.W1 + l * F + f] = gW1[f];
#pragma unroll
  for (int k = 0; k < H; ++k) p[o.W2 + l * H + k] = gW2[k];
  p[o.b1 + l] = gb1;
  p[o.b2 + l] = gb2;
  p[o.w3 + l] = gw3;
  if (l == 0) {
    p[o.b3] = gb3;
    loss_part[blockIdx.x] = loss;
  }
}

// Adam (Kingma & Ba) with bias correction; the gradient is the fixed-order
// sum of the per-wave partials: a workgroup takes 64 parameters, its eight
// waves sum the partials b = c, c + 8, c + 16, ... (wave c) of each, and
// the eight sums are added in wave order.  Wave 1 of workgroup 0 also
// records the epoch's loss.
constexpr int kAdamChunks = 8;
__global__ __launch_bounds__(64 * kAdamChunks) void mlp_adam_kernel(
    float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
    const float* __restrict__ part, int nparts, int P, int t, float lr, float beta1, float beta2,
    float eps, const float* __restrict__ loss_part, int N, float* __restrict__ loss_hist) {
  __shared__ float sh[kAdamChunks][64];
  const int q = threadIdx.x & 63, c = threadIdx.x >> 6;
  const int p = blockIdx.x * 64 + q;
  float g = 0.f;
  if (p < P) {
#pragma unroll 8
    for (int b = c; b < nparts; b += kAdamChunks) g += part[(int64_t)b * P + p];
  }
  sh[c][q] = g;
  if (blockIdx.x == 0 && c == 1) {
    float s = 0.f;
    for (int b = q; b < nparts; b += 64) s += loss_part[b];
    s = wave_sum_f(s);
    if (q == 0) loss_hist[t - 1] = s / (float)N;
  }
  __syncthreads();
  if (c != 0 || p >= P) return;
  g = sh[0][q];
#pragma unroll
  for (int k = 1; k < kAdamChunks; ++k) g += sh[k][q];
  const float mm = beta1 * m[p] + (1.f - beta1) * g;
  const float vv = beta2 * v[p] + (1.f - beta2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const float mhat = mm / (1.f - powf(beta1, (float)t));
  const float vhat = vv / (1.f - powf(beta2, (float)t));
  theta[p] -= lr * mhat / (sqrtf(vhat) + eps);
}

// Glorot-uniform weights from a counter-based stream (SplitMix64 output p of
// the seed gives parameter p), zero biases.
__global__ void mlp_init_kernel(float* __restrict__ theta, float* __restrict__ m,
                                float* __restrict__ v, int F, uint64_t seed) {
  const Off o(F);
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= o.P) return;
  float lim = 0.f;
  if (p < o.b1) lim = sqrtf(6.f / (float)(F + H));
  else if (p >= o.W2 && p < o.b2) lim = sqrtf(6.f / (float)(H + H));
  else if (p >= o.w3 && p < o.b3) lim = sqrtf(6.f / (float)(H + 1));
  const uint64_t r = sm_output(seed, (uint64_t)p);
  const double u01 = (double)(r >> 11) * (1.0 / 9007199254740992.0);
  theta[p] = (float)((2.0 * u01 - 1.0) * lim);
  m[p] = 0.f;
  v[p] = 0.f;
}

__global__ void mlp_to_bf16_kernel(const float* __restrict__ theta, int P, __bf16* __restrict__ w) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) w[p] = (__bf16)theta[p];
}

__device__ __forceinline__ float bf(float x) { return (float)(__bf16)x; }

// g for rows of a moment table: the cheap truncation q_c = sum_{f<F} c_f mu_f
// plus the network's correction, g = q_c + mu_0 (ybar + ysd * out), with
// inputs x_f = mu_f / mu_0.  One wave per 64-row slice.
__global__ __launch_bounds__(64) void mlp_infer_kernel(const __bf16* __restrict__ w, int F,
                                                       const double* __restrict__ coef,
                                                       const double* __restrict__ mu,
                                                       int64_t ldmu, int64_t rows, MlpAffine aff,
                                                       double* __restrict__ g) {
  const Off o(F);
  const int l = threadIdx.x;
  float w1[FMAX], w2r[H];
#pragma unroll
  for (int f = 0; f < FMAX; ++f) w1[f] = f < F ? (float)w[o.W1 + l * F + f] : 0.f;
#pragma unroll
  for (int k = 0; k < H; ++k) w2r[k] = (float)w[o.W2 + l * H + k];
  const float b1 = (float)w[o.b1 + l], b2 = (float)w[o.b2 + l], w3 = (float)w[o.w3 + l];
  const float b3 = (float)w[o.b3];
  const int64_t i0 = (int64_t)blockIdx.x * 64, i1 = min<int64_t>(rows, i0 + 64);
  for (int64_t i = i0; i < i1; ++i) {
    const double* r = mu + i * ldmu;
    const double inv0 = 1.0 / r[0];
    float a1 = b1;
    double lin = 0.0;
#pragma unroll
    for (int f = 0; f < FMAX; ++f)
      if (f < F) {
        const double sd = aff.xsd[f];
        const double u = sd > 0.0 ? (r[f] * inv0 - aff.xmean[f]) / sd : 0.0;
        lin += aff.lin[f] * u;
        a1 = fmaf(w1[f], bf((float)u), a1);
      }
    const float h1 = bf(tanhf(a1));
    float a2 = b2;
#pragma unroll
    for (int k = 0; k < H; ++k) a2 = fmaf(w2r[k], read_lane(h1, k), a2);
    const float h2 = bf(tanhf(a2));
    const float out = wave_sum_f(w3 * h2) + b3;
    if (l == 0) {
      double qc = 0.0;
      for (int f = 0; f < F; ++f) qc += coef[f] * r[f];
      g[i] = qc + r[0] * (aff.ybar + aff.ysd * (lin + (double)out));
    }
  }
}

// q = sum_j c_j mu_j (j = 0..n) for each row.
__global__ void qvals_kernel(const double* __restrict__ mu, int64_t ldmu,
                             const double* __restrict__ c, int n, int64_t rows,
                             double* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  const double* r = mu + i * ldmu;
  double s = 0.0;
  for (int j = 0; j <= n; ++j) s += c[j] * r[j];
  q[i] = s;
}

constexpr int kRT = 256;

// Prefix values of the learned multilevel chain: S(l) = sum_{j<=l} c_j mu_j,
// except S(nc) = g and S(-1) = 0.  q[p] = S(hi) - S(lo) of row p.
__device__ __forceinline__ double chain_value(const double* r, const double* c, int l, int nc,
                                              double g) {
  if (l < 0) return 0.0;
  if (l == nc) return g;
  double s = 0.0;
  for (int j = 0; j <= l; ++j) s += c[j] * r[j];
  return s;
}

__global__ void learned_level_q_kernel(const double* __restrict__ mu, int64_t ldmu,
                                       const double* __restrict__ c, int hi, int lo, int nc,
                                       const double* __restrict__ g, int64_t rows,
                                       double* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  const double* r = mu + i * ldmu;
  const double gi = g ? g[i] : 0.0;
  q[i] = chain_value(r, c, hi, nc, gi) - chain_value(r, c, lo, nc, gi);
}

// Per-probe terms whose prefix sums are the chain values above (the pilot
// table of the level planner): t_j = c_j mu_j, then t_nc = g - S(nc - 1) and
// t_{nc+1} = S(nc + 1) - g.
__global__ void learned_terms_kernel(const double* __restrict__ mu, int64_t ldmu,
                                     const double* __restrict__ c, int n, int nc,
                                     const double* __restrict__ g, int64_t rows,
                                     double* __restrict__ t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  const double* r = mu + i * ldmu;
  double* o = t + i * (int64_t)(n + 1);
  double below = 0.0;  // S(nc - 1)
  for (int j = 0; j <= n; ++j) {
    o[j] = c[j] * r[j];
    if (j < nc) below += o[j];
  }
  const double at = below + o[nc];  // S(nc) of the plain truncation
  o[nc] = g[i] - below;
  o[nc + 1] = (at + o[nc + 1]) - g[i];
}

// out[0] = max over rows and j <= ncols - 1 of |mu_j| / mu_0.  One workgroup.
__global__ __launch_bounds__(kRT) void moment_ratio_kernel(const double* __restrict__ mu,
                                                           int64_t ldmu, int ncols, int64_t rows,
                                                           double* __restrict__ out) {
  __shared__ double sh[kRT];
  double mr = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += kRT) {
    const double* r = mu + i * ldmu;
    const double inv0 = 1.0 / r[0];
    for (int j = 0; j < ncols; ++j) mr = fmax(mr, fabs(r[j]) * inv0);
  }
  sh[threadIdx.x] = mr;
  __syncthreads();
  for (int st = kRT / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

__device__ double rsum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int st = kRT / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Training set from the pilot.  Target t = ((q - q_c) / mu_0 - ybar) / ysd,
// the standardised residual of the cheap truncation q_c = sum_{f<F} c_f mu_f;
// inputs u_f = (mu_f / mu_0 - xmean_f) / xsd_f for f >= 1 (0 for f = 0 and
// for constant features), means and unbiased standard deviations over the
// training rows.  beta = argmin |t - U beta|^2 from the normal equations
// (Cholesky, ridge 1e-12 trace / K), and y = t - U beta, what the network
// learns.  X = u (float), y (float); stats: [0] ybar, [1] ysd, [2 + f]
// xmean, [2 + FMAX + f] xsd, [2 + 2 FMAX + f] beta.  One workgroup, FP64,
// fixed-order sums.
__device__ __forceinline__ double resid_target(const double* r, double q, const double* c, int F) {
  double qc = 0.0;
  for (int f = 0; f < F; ++f) qc += c[f] * r[f];
  return (q - qc) / r[0];
}

__global__ __launch_bounds__(kRT) void mlp_prepare_kernel(const double* __restrict__ mu,
                                                          int64_t ldmu,
                                                          const double* __restrict__ q,
                                                          const double* __restrict__ coef, int F,
                                                          int ntrain, float* __restrict__ X,
                                                          float* __restrict__ y,
                                                          double* __restrict__ stats) {
  __shared__ double sh[kRT];
  __shared__ double xm[FMAX], xs[FMAX], beta[FMAX], G[FMAX][FMAX], rhs[FMAX];
  const int tid = threadIdx.x;
  const double den = ntrain > 1 ? ntrain - 1 : 1;
  double s = 0.0;
  for (int i = tid; i < ntrain; i += kRT) s += resid_target(mu + (int64_t)i * ldmu, q[i], coef, F);
  const double mean = rsum(s, sh) / ntrain;
  double ss = 0.0;
  for (int i = tid; i < ntrain; i += kRT) {
    const double t = resid_target(mu + (int64_t)i * ldmu, q[i], coef, F) - mean;
    ss += t * t;
  }
  double sd = sqrt(rsum(ss, sh) / den);
  if (!(sd > 0.0)) sd = 1.0;
  auto xf = [&](int i, int f) {
    const double* r = mu + (int64_t)i * ldmu;
    return r[f] / r[0];
  };
  if (tid < FMAX) xm[tid] = xs[tid] = beta[tid] = 0.0;
  __syncthreads();
  for (int f = 1; f < F; ++f) {
    double a = 0.0;
    for (int i = tid; i < ntrain; i += kRT) a += xf(i, f);
    const double m = rsum(a, sh) / ntrain;
    double b = 0.0;
    for (int i = tid; i < ntrain; i += kRT) {
      const double e = xf(i, f) - m;
      b += e * e;
    }
    const double v = sqrt(rsum(b, sh) / den);
    if (tid == 0) {
      xm[f] = m;
      xs[f] = v > 0.0 ? v : 0.0;
    }
    __syncthreads();
  }
  auto u = [&](int i, int f) { return xs[f] > 0.0 ? (xf(i, f) - xm[f]) / xs[f] : 0.0; };
  auto tgt = [&](int i) {
    return (resid_target(mu + (int64_t)i * ldmu, q[i], coef, F) - mean) / sd;
  };
  // normal equations over f = 1..F-1
  const int K = F - 1;
  for (int a = 1; a < F; ++a) {
    for (int b = a; b < F; ++b) {
      double acc = 0.0;
      for (int i = tid; i < ntrain; i += kRT) acc += u(i, a) * u(i, b);
      const double v = rsum(acc, sh);
      if (tid == 0) G[a][b] = G[b][a] = v;
    }
    double acc = 0.0;
    for (int i = tid; i < ntrain; i += kRT) acc += u(i, a) * tgt(i);
    const double v = rsum(acc, sh);
    if (tid == 0) rhs[a] = v;
  }
  __syncthreads();
  if (tid == 0 && K > 0) {
    double tr = 0.0;
    for (int a = 1; a < F; ++a) tr += G[a][a];
    const double ridge = 1e-12 * tr / K + 1e-300;
    for (int a = 1; a < F; ++a) G[a][a] += ridge;
    // Cholesky G = L L^T in place (lower triangle), then two triangular solves
    for (int j = 1; j < F; ++j) {
      double d = G[j][j];
      for (int k = 1; k < j; ++k) d -= G[j][k] * G[j][k];
      d = sqrt(d > 0.0 ? d : 1e-300);
      G[j][j] = d;
      for (int i = j + 1; i < F; ++i) {
        double e = G[i][j];
        for (int k = 1; k < j; ++k) e -= G[i][k] * G[j][k];
        G[i][j] = e / d;
      }
    }
    double z[FMAX];
    for (int i = 1; i < F; ++i) {
      double e = rhs[i];
      for (int k = 1; k < i; ++k) e -= G[i][k] * z[k];
      z[i] = e / G[i][i];
    }
    for (int i = F - 1; i >= 1; --i) {
      double e = z[i];
      for (int k = i + 1; k < F; ++k) e -= G[k][i] * beta[k];
      beta[i] = e / G[i][i];
    }
  }
  __syncthreads();
  for (int i = tid; i < ntrain; i += kRT) {
    double lin = 0.0;
    X[(int64_t)i * F] = 0.f;
    for (int f = 1; f < F; ++f) {
      const double uf = u(i, f);
      X[(int64_t)i * F + f] = (float)uf;
      lin += beta[f] * uf;
    }
    y[i] = (float)(tgt(i) - lin);
  }
  if (tid == 0) {
    stats[0] = mean;
    stats[1] = sd;
  }
  if (tid < FMAX) {
    stats[2 + tid] = xm[tid];
    stats[2 + FMAX + tid] = xs[tid];
    stats[2 + 2 * FMAX + tid] = beta[tid];
  }
}

// out[0..3] = mean(a), var(a) (unbiased), mean(b - a2), var(b - a2); a or b
// may be empty.  One workgroup, fixed-order sums.
__global__ __launch_bounds__(kRT) void mlp_combine_kernel(const double* __restrict__ a,
                                                          int64_t na,
                                                          const double* __restrict__ b,
                                                          const double* __restrict__ a2,
                                                          int64_t nb, double* __restrict__ out) {
  __shared__ double sh[kRT];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < na; i += kRT) s += a[i];
  const double ma = na ? rsum(s, sh) / na : (rsum(0.0, sh), 0.0);
  s = 0.0;
  for (int64_t i = threadIdx.x; i < na; i += kRT) s += (a[i] - ma) * (a[i] - ma);
  const double va = na > 1 ? rsum(s, sh) / (na - 1) : (rsum(0.0, sh), NAN);
  s = 0.0;
  for (int64_t i = threadIdx.x; i < nb; i += kRT) s += b[i] - (a2 ? a2[i] : 0.0);
  const double mb = nb ? rsum(s, sh) / nb : (rsum(0.0, sh), 0.0);
  s = 0.0;
  for (int64_t i = threadIdx.x; i < nb; i += kRT) {
    const double t = b[i] - (a2 ? a2[i] : 0.0) - mb;
    s += t * t;
  }
  const double vb = nb > 1 ? rsum(s, sh) / (nb - 1) : (rsum(0.0, sh), NAN);
  if (threadIdx.x == 0) {
    out[0] = ma;
    out[1] = va;
    out[2] = mb;
    out[3] = vb;
  }
}

// grad[p] = sum over waves of the partials (fixed order); loss = mean.
__global__ void mlp_gradsum_kernel(const float* __restrict__ part, int nparts, int P,
                                   const float* __restrict__ loss_part, int N,
                                   float* __restrict__ grad, float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0) {
    float s = 0.f;
    for (int b = 0; b < nparts; ++b) s += loss_part[b];
    *loss = s / (float)N;
  }
  if (p >= P) return;
  float g = 0.f;
  for (int b = 0; b < nparts; ++b) g += part[(int64_t)b * P + p];
  grad[p] = g;
}

}  // namespace

int mlp_nparams(int F) { return Off(F).P; }

hipError_t launch_mlp_gradsum(hipStream_t s, const float* part, int nwaves, int F,
                              const float* loss_part, int N, float* grad, float* loss) {
  const int P = Off(F).P;
  mlp_gradsum_kernel<<<(P + 255) / 256, 256, 0, s>>>(part, nwaves, P, loss_part, N, grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_init(hipStream_t s, float* theta, float* m, float* v, int F, uint64_t seed) {
  const int P = Off(F).P;
  mlp_init_kernel<<<(P + 255) / 256, 256, 0, s>>>(theta, m, v, F, seed);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(hipStream_t s, const float* theta, int F, const float* X,
                           const float* y, int N, int nwaves, float* part, float* loss_part) {
  const int per = (N + nwaves - 1) / nwaves;
  mlp_grad_kernel<<<nwaves, 64, 0, s>>>(theta, F, X, y, N, per, part, loss_part);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(hipStream_t s, float* theta, float* m, float* v, const float* part,
                           int nwaves, int F, int t, float lr, const float* loss_part, int N,
                           float* loss_hist) {
  const int P = Off(F).P;
  mlp_adam_kernel<<<(P + 63) / 64, 64 * kAdamChunks, 0, s>>>(theta, m, v, part, nwaves, P, t, lr,
                                                             0.9f, 0.999f, 1e-8f, loss_part, N,
                                                             loss_hist);
  return hipGetLastError();
}

hipError_t launch_mlp_to_bf16(hipStream_t s, const float* theta, int F, void* w) {
  const int P = Off(F).P;
  mlp_to_bf16_kernel<<<(P + 255) / 256, 256, 0, s>>>(theta, P, static_cast<__bf16*>(w));
  return hipGetLastError();
}

hipError_t launch_mlp_infer(hipStream_t s, const void* w, int F, const double* coef,
                            const double* mu, int64_t ldmu, int64_t rows, const MlpAffine& aff,
                            double* g) {
  if (rows <= 0) return hipSuccess;
  mlp_infer_kernel<<<(int)((rows + 63) / 64), 64, 0, s>>>(static_cast<const __bf16*>(w), F, coef,
                                                          mu, ldmu, rows, aff, g);
  return hipGetLastError();
}

hipError_t launch_qvals(hipStream_t s, const double* mu, int64_t ldmu, const double* c, int n,
                        int64_t rows, double* q) {
  if (rows <= 0) return hipSuccess;
  qvals_kernel<<<(int)((rows + 255) / 256), 256, 0, s>>>(mu, ldmu, c, n, rows, q);
  return hipGetLastError();
}

hipError_t launch_mlp_prepare(hipStream_t s, const double* mu, int64_t ldmu, const double* q,
                              const double* coef, int F, int ntrain, float* X, float* y,
                              double* stats) {
  mlp_prepare_kernel<<<1, kRT, 0, s>>>(mu, ldmu, q, coef, F, ntrain, X, y, stats);
  return hipGetLastError();
}

hipError_t launch_learned_level_q(hipStream_t s, const double* mu, int64_t ldmu, const double* c,
                                  int hi, int lo, int nc, const double* g, int64_t rows,
                                  double* q) {
  if (rows <= 0) return hipSuccess;
  learned_level_q_kernel<<<(int)((rows + 255) / 256), 256, 0, s>>>(mu, ldmu, c, hi, lo, nc, g,
                                                                    rows, q);
  return hipGetLastError();
}

hipError_t launch_learned_terms(hipStream_t s, const double* mu, int64_t ldmu, const double* c,
                                int n, int nc, const double* g, int64_t rows, double* t) {
  if (rows <= 0) return hipSuccess;
  learned_terms_kernel<<<(int)((rows + 255) / 256), 256, 0, s>>>(mu, ldmu, c, n, nc, g, rows, t);
  return hipGetLastError();
}

hipError_t launch_moment_ratio(hipStream_t s, const double* mu, int64_t ldmu, int ncols,
                               int64_t rows, double* out) {
  moment_ratio_kernel<<<1, kRT, 0, s>>>(mu, ldmu, ncols, rows, out);
  return hipGetLastError();
}

hipError_t launch_mlp_combine(hipStream_t s, const double* a, int64_t na, const double* b,
                              const double* a2, int64_t nb, double* out) {
  mlp_combine_kernel<<<1, kRT, 0, s>>>(a, na, b, a2, nb, out);
  return hipGetLastError();
}

}  // namespace mlct
