// Automatic level selection (Section 3.2, Theorem thm:levels, eqs.
// eqn:levelCost and eqn:costrecurrence) from a pilot sample.
//
// Pilot terms t_j = c_j z^T T_j(A_hat) z (one row per probe) give prefix
// sums S_l = sum_{j<=l} t_j, and the variance of the level variable
// Q_{l'l} = S_l - S_{l'} (eq. def:qlevels) is its sample variance over the
// pilot.  The dynamic programme of Theorem thm:levels then runs in one wave;
// the top level takes the extra condition of Section 3.2 (the allocation of
// eqs. eqn:optSamples / eqn:optMu must recommend at least min_top samples
// for it).  Readings: ties go to the smaller l'; with no admissible l' the
// single level {n} is used; sample sizes are rounded up and at least 2.
// A plan holds at most MLCT_MAX_LEVELS levels: when the optimum has more,
// the recurrence is run again indexed by the number of levels,
// H_k(l) = min_{l' < l} H_{k-1}(l') + sqrt(V_{l'l} C(l)) with H_k(0) = 0 and
// H_0(l > 0) = inf (the least cost of at most k levels topped by l), and the
// top level is chosen over H_{MLCT_MAX_LEVELS - 1} with the same condition.
// All arithmetic is FP64 with sums in a fixed order.
#include <cfloat>

#include "device.hpp"

namespace mlct {

namespace {

constexpr int kPT = 256;

// S[p][l] = sum_{j<=l} c_j mu[p][j] (c_j = 1 when coef is null), in order of j.
__global__ __launch_bounds__(kPT) void level_prefix_kernel(const double* __restrict__ mu,
                                                           int64_t ldmu,
                                                           const double* __restrict__ coef,
                                                           int n, int64_t m,
                                                           double* __restrict__ S) {
  const int64_t p = (int64_t)blockIdx.x * kPT + threadIdx.x;
  if (p >= m) return;
  double s = 0.0;
  for (int j = 0; j <= n; ++j) {
    s += (coef ? coef[j] : 1.0) * mu[p * ldmu + j];
    S[p * (n + 1) + j] = s;
  }
}

// mean[l] = (1/m) sum_p S[p][l]: one workgroup per column, strided partial
// sums then a tree in LDS (fixed order).
__global__ __launch_bounds__(kPT) void level_mean_kernel(const double* __restrict__ S, int n,
                                                         int64_t m, double* __restrict__ mean) {
  __shared__ double sh[kPT];
  const int l = blockIdx.x;
  double acc = 0.0;
  for (int64_t p = threadIdx.x; p < m; p += kPT) acc += S[p * (n + 1) + l];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int st = kPT / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) mean[l] = sh[0] / (double)m;
}

// V[r][l] (r = l' + 1, 0 <= r <= l <= n) = sum_p ((S_l - mean_l) -
// (S_{r-1} - mean_{r-1}))^2 / (m - 1), with S_{-1} = 0.  One thread per pair;
// pair index q = l (l + 1) / 2 + r.
__global__ __launch_bounds__(kPT) void level_var_kernel(const double* __restrict__ S,
                                                        const double* __restrict__ mean, int n,
                                                        int64_t m, double* __restrict__ V) {
  const int64_t q = (int64_t)blockIdx.x * kPT + threadIdx.x;
  const int64_t npairs = (int64_t)(n + 1) * (n + 2) / 2;
  if (q >= npairs) return;
  int64_t l = (int64_t)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
  while (l * (l + 1) / 2 > q) --l;
  while ((l + 1) * (l + 2) / 2 <= q) ++l;
  const int r = (int)(q - l * (l + 1) / 2);
  const double ml = mean[l], mr = r ? mean[r - 1] : 0.0;
  double acc = 0.0;
  for (int64_t p = 0; p < m; ++p) {
    const double* row = S + p * (n + 1);
    const double x = (row[l] - ml) - (r ? row[r - 1] - mr : 0.0);
    acc += x * x;
  }
  V[(int64_t)r * (n + 1) + l] = acc / (double)(m - 1);
}

__device__ __forceinline__ double level_c(int l, int doubling) {
  return (double)(doubling ? (l + 1) / 2 : l);
}

// (value, index) minimum over the wave; ties go to the smaller index.
__device__ __forceinline__ void wave_argmin(double& v, int& i) {
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o, 64);
    const int oi = __shfl_xor(i, o, 64);
    if (ov < v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
}

// Second-highest level over h (cbar, or H of the capped recurrence) with
// the top-level condition: (arg, total), arg = INT32_MAX when none qualifies.
template <class VF>
__device__ void top_level(const double* h, VF Vat, int n, int doubling, double target,
                          int budget, int64_t min_top, int& arg, double& best) {
  const int lane = threadIdx.x;
  const double cn = level_c(n, doubling);
  best = DBL_MAX;
  arg = INT32_MAX;
  for (int lp = lane; lp < n; lp += 64) {
    const double vt = Vat(lp, n);
    const double tot = h[lp] + sqrt(vt * cn);
    if (!(tot > 0.0)) continue;
    const double mL = budget ? target * sqrt(vt / cn) / tot : tot * sqrt(vt / cn) / target;
    if (mL >= (double)min_top && tot < best) {
      best = tot;
      arg = lp;
    }
  }
  wave_argmin(best, arg);
}

// The dynamic programme and the plan; one wave.  prevk: scratch of
// MLCT_MAX_LEVELS * (n + 1) ints for the capped recurrence.
__global__ __launch_bounds__(64) void level_dp_kernel(const double* __restrict__ V, int n,
                                                      int doubling, double target, int budget,
                                                      int64_t min_top, int* __restrict__ prevk,
                                                      LevelPlanDev* __restrict__ out) {
  __shared__ double cbar[kMaxPlanDegree + 1];
  __shared__ double hcur[kMaxPlanDegree + 1];
  __shared__ int prev[kMaxPlanDegree + 1];
  __shared__ int chain[kMaxPlanDegree + 1];
  __shared__ int nlev;
  const int lane = threadIdx.x;
  auto Vat = [&](int lp, int l) { return fmax(V[(int64_t)(lp + 1) * (n + 1) + l], 0.0); };
  if (lane == 0) {
    cbar[0] = 0.0;
    prev[0] = 0;
  }
  __syncthreads();
  for (int l = 1; l < n; ++l) {
    const double cl = level_c(l, doubling);
    double best = DBL_MAX;
    int arg = INT32_MAX;
    for (int lp = lane; lp < l; lp += 64) {
      const double v = cbar[lp] + sqrt(Vat(lp, l) * cl);
      if (v < best) {
        best = v;
        arg = lp;
      }
    }
    wave_argmin(best, arg);
    if (lane == 0) {
      cbar[l] = best;
      prev[l] = arg;
    }
    __syncthreads();
  }
  const double cn = level_c(n, doubling);
  const double single = sqrt(Vat(0, n) * cn);
  double best;
  int arg;
  top_level(cbar, Vat, n, doubling, target, budget, min_top, arg, best);
  int chosen = arg;
  double total = best;
  if (arg == INT32_MAX) {
    chosen = 0;
    total = single;
  }
  // levels from the top down, then reversed
  if (lane == 0) {
    int L = 0;
    chain[L++] = n;
    for (int lp = chosen; lp > 0; lp = prev[lp]) chain[L++] = lp;
    nlev = L;
  }
  __syncthreads();
  if (nlev > MLCT_MAX_LEVELS) {
    // at most K + 1 levels: H_K over the l' below the top
    constexpr int K = MLCT_MAX_LEVELS - 1;
    double* hp = cbar;
    double* hc = hcur;
    for (int l = lane; l < n; l += 64) hp[l] = l == 0 ? 0.0 : __builtin_inf();
    __syncthreads();
    for (int k = 1; k <= K; ++k) {
      if (lane == 0) hc[0] = 0.0;
      for (int l = 1; l < n; ++l) {
        const double cl = level_c(l, doubling);
        double b = __builtin_inf();
        int a = INT32_MAX;
        for (int lp = lane; lp < l; lp += 64) {
          const double h = hp[lp];
          if (h == __builtin_inf()) continue;
          const double v = h + sqrt(Vat(lp, l) * cl);
          if (v < b) {
            b = v;
            a = lp;
          }
        }
        wave_argmin(b, a);
        if (lane == 0) {
          hc[l] = b;
          prevk[(int64_t)k * (n + 1) + l] = a == INT32_MAX ? 0 : a;
        }
      }
      __syncthreads();
      double* t = hp;
      hp = hc;
      hc = t;
    }
    top_level(hp, Vat, n, doubling, target, budget, min_top, arg, best);
    chosen = arg;
    total = best;
    if (arg == INT32_MAX) {
      chosen = 0;
      total = single;
    }
    if (lane == 0) {
      int L = 0;
      chain[L++] = n;
      for (int lp = chosen, k = K; lp > 0; --k) {
        chain[L++] = lp;
        lp = prevk[(int64_t)k * (n + 1) + lp];
      }
      nlev = L;
    }
  }
  if (lane != 0) return;
  const int L = nlev;
  out->L = L;
  out->opt_total = total;
  out->single_total = single;
  if (L > MLCT_MAX_LEVELS) return;  // the host reports it
  double s = 0.0;
  for (int k = 0; k < L; ++k) {
    const int hi = chain[L - 1 - k], lo = k ? chain[L - k] : 0;
    const double v = Vat(lo, hi), c = level_c(hi, doubling);
    out->degree[k] = hi;
    out->var[k] = v;
    out->cost[k] = c;
    s += sqrt(v * c);
  }
  const double mu = s > 0.0 ? (budget ? target / s : s / target) : 0.0;
  for (int k = 0; k < L; ++k) {
    const double mr = out->cost[k] > 0.0 ? mu * sqrt(out->var[k] / out->cost[k]) : 0.0;
    out->m_real[k] = mr;
    const double mc = ceil(mr);
    out->m[k] = mc < 2.0 ? 2 : (int64_t)mc;
  }
}

}  // namespace

hipError_t launch_level_plan(hipStream_t s, const double* mu, int64_t ldmu, const double* coef,
                             int n, int64_t m, double* S, double* mean, double* V, int doubling,
                             double target, int budget, int64_t min_top, int* prevk,
                             LevelPlanDev* out) {
  level_prefix_kernel<<<(int)((m + kPT - 1) / kPT), kPT, 0, s>>>(mu, ldmu, coef, n, m, S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  level_mean_kernel<<<n + 1, kPT, 0, s>>>(S, n, m, mean);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t npairs = (int64_t)(n + 1) * (n + 2) / 2;
  level_var_kernel<<<(int)((npairs + kPT - 1) / kPT), kPT, 0, s>>>(S, mean, n, m, V);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  level_dp_kernel<<<1, 64, 0, s>>>(V, n, doubling, target, budget, min_top, prevk, out);
  return hipGetLastError();
}

}  // namespace mlct
