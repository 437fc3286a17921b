// Block Chebyshev recurrence over a dense symmetric operator on the matrix
// cores (Section 2.2, eq. eqn:recurrence in matrix form), with the
// per-probe moments fused into the epilogue.
//
// Probe blocks are kept probe-major: V^T is B x d, row j = probe j.  Because
// A is symmetric, (A V)^T = V^T A, and the product is
//     C[j][n] = sum_k V^T[j][k] * A[n][k],
// so both MFMA operands are read along contiguous k (row j of V^T and row n
// of A).  The workgroup tile is BM probes x BN matrix rows; the epilogue
// forms  V_new^T = ca * C + cb * V_k^T  [- V_prev^T]  in place over V_prev^T
// and the per-probe dot products (FP64, exact products of the stored
// values), reduced over the tile's rows in a fixed order.
//
// Precisions (16x16 MFMA tiles):
//   PREC 0  FP64   v_mfma_f64_16x16x4f64
//   PREC 1  FP32   v_mfma_f32_16x16x4f32
//   PREC 2  BF16X3 v_mfma_f32_16x16x32_bf16 three times per tile:
//                  V_hi A_hi + V_hi A_lo + V_lo A_hi, FP32 accumulation;
//                  A is split once (A_hi = bf16(A), A_lo = bf16(A - A_hi)),
//                  V is split on the way into LDS.
#include "device.hpp"

namespace mlct {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Packed bf16 operands of the skinny BF16x3 kernel.  A (rows x d) is cut
// into tiles of 16 rows and k blocks of 32 columns; block (t, kb) holds the
// 64 lanes' operands of one 16x16x32 MFMA in lane order, 8 values per lane:
// lane l = (row % 16) + 16 g carries columns kb*32 + 8 g .. + 7.  Rows and
// columns past the matrix are zero.  The same layout serves a probe block
// (rows = probes) and the matrix (rows = matrix rows).
__host__ __device__ inline int64_t pk_kblocks(int64_t d) { return (d + 31) / 32; }
__host__ __device__ inline int64_t pk_index(int64_t row, int64_t k, int64_t kblocks) {
  const int64_t lane = (row & 15) + 16 * ((k & 31) >> 3);
  return (((row >> 4) * kblocks + (k >> 5)) * 64 + lane) * 8 + (k & 7);
}
struct PackedOps {
  const bf8* a_hi;  // matrix, packed
  const bf8* a_lo;
  const bf8* v_hi;  // V_k, packed
  const bf8* v_lo;
  __bf16* o_hi;     // V_new, packed (written by the epilogue)
  __bf16* o_lo;
};

template <int PREC>
struct Prec;
template <>
struct Prec<0> {
  using V = double;   // probe-block element
  using M = double;   // matrix element in LDS
  using Acc = d4;
  static constexpr int KM = 4;  // K of one MFMA
};
template <>
struct Prec<1> {
  using V = float;
  using M = float;
  using Acc = f4;
  static constexpr int KM = 4;
};
template <>
struct Prec<2> {
  using V = float;
  using M = __bf16;
  using Acc = f4;
  static constexpr int KM = 32;
};

// Row (within a 16x16 tile) of accumulator value r of lane l.
template <int PREC>
__device__ __forceinline__ int acc_row(int l, int r) {
  return PREC == 0 ? (l >> 4) + 4 * r : (l >> 4) * 4 + r;
}

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

template <int PREC, int WM, int WN, int TM, int TN, int BK, int ZMODE, bool HAS_PREV>
__global__ __launch_bounds__(64 * WM * WN) void dense_step_kernel(
    const void* __restrict__ A0, const void* __restrict__ A1, int64_t lda, int64_t d,
    const typename Prec<PREC>::V* __restrict__ vk, typename Prec<PREC>::V* __restrict__ vm,
    typename Prec<PREC>::V ca, typename Prec<PREC>::V cb, ProbeSrc src, int mtiles, int ntiles,
    double* __restrict__ part) {
  using P = Prec<PREC>;
  using VT = typename P::V;
  using MT = typename P::M;
  using AccT = typename P::Acc;
  constexpr int NT = 64 * WM * WN;
  constexpr int BM = WM * TM * 16, BN = WN * TN * 16;
  constexpr int PAD = PREC == 2 ? 8 : (PREC == 1 ? 4 : 2);
  constexpr int LK = BK + PAD;  // LDS row length in elements
  constexpr int NSPLIT = PREC == 2 ? 2 : 1;

  __shared__ MT sV[NSPLIT][BM][LK];
  __shared__ MT sA[NSPLIT][BN][LK];
  __shared__ double sred[WN][2][BM];

  // tile of this workgroup; workgroups of one XCD share matrix row tiles
  const int total = mtiles * ntiles;
  const int tiles8 = (total + 7) / 8 * 8;
  const int L = xcd_band(blockIdx.x, tiles8);
  if (L >= total) return;
  const int mt = L % mtiles, nt = L / mtiles;
  const int64_t m0 = (int64_t)mt * BM, n0 = (int64_t)nt * BN;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t ldv = d;

  AccT acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = AccT{};

  // ---- k loop: 16-byte global loads of the next tile into registers while
  // the current tile is in LDS and on the matrix cores ---------------------
  constexpr int GV = 16 / sizeof(VT);                     // V elements per load
  constexpr int GA = PREC == 2 ? 8 : 16 / (int)sizeof(MT);  // A elements per load
  constexpr int NV = BM * BK / GV / NT;                   // V loads per thread
  constexpr int NA = BN * BK / GA / NT;                   // A loads per thread (per part)
  static_assert(NV * GV * NT == BM * BK && NA * GA * NT == BN * BK, "tile/thread mismatch");
  typedef VT vvec __attribute__((ext_vector_type(GV)));
  typedef MT avec __attribute__((ext_vector_type(GA)));
  vvec rv[NV];
  avec ra[NSPLIT][NA];
  const bool dvec_ok = (d % GV == 0) && (lda % GA == 0);
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int e = (tid + u * NT) * GV, r = e / BK, c = e % BK;
      const int64_t k = k0 + c;
      const VT* src = vk + (m0 + r) * ldv + k;
      if (dvec_ok && k + GV <= d) {
        rv[u] = *reinterpret_cast<const vvec*>(src);
      } else {
#pragma unroll
        for (int q = 0; q < GV; ++q) rv[u][q] = (k + q < d) ? src[q] : VT(0);
      }
    }
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = (tid + u * NT) * GA, r = e / BK, c = e % BK;
      const int64_t k = k0 + c, n = n0 + r;
#pragma unroll
      for (int h = 0; h < NSPLIT; ++h) {
        const MT* src = static_cast<const MT*>(h ? A1 : A0) + (n < d ? n : 0) * lda + k;
        if (n < d && dvec_ok && k + GA <= d) {
          ra[h][u] = *reinterpret_cast<const avec*>(src);
        } else {
#pragma unroll
          for (int q = 0; q < GA; ++q) ra[h][u][q] = (n < d && k + q < d) ? src[q] : MT(0.f);
        }
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int e = (tid + u * NT) * GV, r = e / BK, c = e % BK;
      if constexpr (PREC == 2) {
#pragma unroll
        for (int q = 0; q < GV; ++q) {
          __bf16 hi, lo;
          split_bf16((float)rv[u][q], hi, lo);
          sV[0][r][c + q] = hi;
          sV[NSPLIT - 1][r][c + q] = lo;
        }
      } else {
        *reinterpret_cast<vvec*>(&sV[0][r][c]) = rv[u];
      }
    }
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = (tid + u * NT) * GA, r = e / BK, c = e % BK;
#pragma unroll
      for (int h = 0; h < NSPLIT; ++h) *reinterpret_cast<avec*>(&sA[h][r][c]) = ra[h][u];
    }
  };

  fetch(0);
  for (int64_t k0 = 0; k0 < d; k0 += BK) {
    stash();
    __syncthreads();
    if (k0 + BK < d) fetch(k0 + BK);
    // ---- MFMA ---------------------------------------------------------------
#pragma unroll
    for (int kk = 0; kk < BK; kk += P::KM) {
      if constexpr (PREC == 2) {
        bf8 ah[TM], al[TM], bh[TN], bl[TN];
        const int kc = kk + (lane >> 4) * 8;
#pragma unroll
        for (int a = 0; a < TM; ++a) {
          const int r = wm * TM * 16 + a * 16 + (lane & 15);
          ah[a] = *reinterpret_cast<const bf8*>(&sV[0][r][kc]);
          al[a] = *reinterpret_cast<const bf8*>(&sV[1][r][kc]);
        }
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          const int r = wn * TN * 16 + b * 16 + (lane & 15);
          bh[b] = *reinterpret_cast<const bf8*>(&sA[0][r][kc]);
          bl[b] = *reinterpret_cast<const bf8*>(&sA[1][r][kc]);
        }
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
          }
      } else {
        MT av[TM], bv[TN];
        const int kc = kk + (lane >> 4);
#pragma unroll
        for (int a = 0; a < TM; ++a) av[a] = sV[0][wm * TM * 16 + a * 16 + (lane & 15)][kc];
#pragma unroll
        for (int b = 0; b < TN; ++b) bv[b] = sA[0][wn * TN * 16 + b * 16 + (lane & 15)][kc];
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b) {
            if constexpr (PREC == 0)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
            else
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
          }
      }
    }
    __syncthreads();
  }

  // ---- epilogue: recurrence, in-place store, moment partials --------------
  double p1[TM][4], p2[TM][4];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) p1[a][r] = p2[a][r] = 0.0;
#pragma unroll
  for (int a = 0; a < TM; ++a) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t j = m0 + wm * TM * 16 + a * 16 + acc_row<PREC>(lane, r);
      const bool jact = j < src.active;
      uint64_t key = 0;
      if (ZMODE == 1) key = sm_output(src.seed, (uint64_t)(src.first_id + j));
      int64_t cached = -1;
      uint64_t word = 0;
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int64_t n = n0 + wn * TN * 16 + b * 16 + (lane & 15);
        if (n >= d) continue;
        const int64_t idx = j * ldv + n;
        const VT xk = vk[idx];
        VT vn = ca * (VT)acc[a][b][r] + cb * xk;
        if (HAS_PREV) vn -= vm[idx];
        vm[idx] = vn;
        if (ZMODE == 0) {
          p1[a][r] += (double)xk * (double)vn;
          p2[a][r] += (double)vn * (double)vn;
        } else if (ZMODE == 1) {
          const int64_t c = n >> 6;
          if (c != cached) {
            word = sm_output(key, (uint64_t)c);
            cached = c;
          }
          p1[a][r] += sign_from_word<double>(word, n) * (double)vn;
        } else {
          const double z = jact ? (double)src.entries[n * src.ld + src.first_id + j] : 0.0;
          p1[a][r] += z * (double)vn;
        }
      }
    }
  }
  // reduce over the 16 lanes that hold the same probe rows (fixed order)
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        p1[a][r] += __shfl_xor(p1[a][r], o, 64);
        p2[a][r] += __shfl_xor(p2[a][r], o, 64);
      }
  if ((lane & 15) == 0) {
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int jl = wm * TM * 16 + a * 16 + acc_row<PREC>(lane, r);
        sred[wn][0][jl] = p1[a][r];
        sred[wn][1][jl] = p2[a][r];
      }
  }
  __syncthreads();
  for (int e = tid; e < 2 * BM; e += NT) {
    const int slot = e / BM, jl = e % BM;
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < WN; ++w) s += sred[w][slot][jl];
    part[((int64_t)slot * ntiles + nt) * ((int64_t)mtiles * BM) + m0 + jl] = s;
  }
}

// Wide BF16x3 blocks (a multiple of 128 probes) on packed operands: a
// workgroup owns 128 probes x 128 matrix rows, its four waves 64 x 64 each
// (4 x 4 MFMA tiles, one accumulator per tile, hi*hi + hi*lo + lo*hi).  Each
// k block of 32 columns is staged in LDS exactly in the packed lane layout
// (8 V tiles and 8 A tiles, hi and lo, 1 KB each), so the stage is a
// contiguous 32 KB copy and every operand read is one conflict-free 16-byte
// LDS load per lane.  Two LDS stages and two register sets: block k + 2
// streams from global memory into registers while block k is on the matrix
// cores, and block k + 1 (already in registers) goes into the other stage;
// one barrier per block.  The 48 MFMAs of a block are issued product by
// product (all hi*hi, then hi*lo, then lo*hi) so that consecutive ones are
// independent.  Epilogue as in dense_step_kernel, plus the packed V_new for
// the next step.
template <int ZMODE, bool HAS_PREV>
__global__ __launch_bounds__(256) void dense_pk_gemm_kernel(
    int64_t d, const float* __restrict__ vk, float* __restrict__ vm, float ca, float cb,
    ProbeSrc src, int mtiles, int ntiles, double* __restrict__ part, PackedOps pk) {
  constexpr int BM = 128, BN = 128, TM = 4, TN = 4, WN = 2;
  // stage layout: [which (0 V, 1 A)][part (0 hi, 1 lo)][tile 0..7][lane] of bf8
  __shared__ bf8 st[2][2][2][8][64];
  __shared__ double sred[WN][2][BM];
  const int total = mtiles * ntiles;
  const int L = xcd_band(blockIdx.x, (total + 7) / 8 * 8);
  if (L >= total) return;
  const int mt = L % mtiles, nt = L / mtiles;
  const int64_t m0 = (int64_t)mt * BM, n0 = (int64_t)nt * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t KB = pk_kblocks(d);
  // this thread's 8 pieces of a stage: piece e = tid + 256 u, decoded as
  // (which, part, tile, lane) in the order of the stage layout
  const bf8* src_of[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int e = tid + 256 * u;
    const int l = e & 63, t = (e >> 6) & 7, prt = (e >> 9) & 1, which = e >> 10;
    const bf8* base = which == 0 ? (prt ? pk.v_lo : pk.v_hi) : (prt ? pk.a_lo : pk.a_hi);
    const int64_t tile = which == 0 ? m0 / 16 + t : n0 / 16 + t;
    src_of[u] = base + tile * KB * 64 + l;
  }
  bf8 ra[8];
  auto fetch = [&](int64_t kb, bf8 (&rg)[8]) {
#pragma unroll
    for (int u = 0; u < 8; ++u) rg[u] = src_of[u][kb * 64];
  };
  auto stash = [&](int s, const bf8 (&rg)[8]) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = tid + 256 * u;
      (&st[s][0][0][0][0])[e] = rg[u];
    }
  };
  f4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

  auto block = [&](int s) {
    bf8 vh[TM], vl[TM], ah[TN], al[TN];
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      vh[a] = st[s][0][0][wm * TM + a][lane];
      vl[a] = st[s][0][1][wm * TM + a][lane];
    }
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      ah[b] = st[s][1][0][wn * TN + b][lane];
      al[b] = st[s][1][1][wn * TN + b][lane];
    }
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vh[a], ah[b], acc[a][b], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vh[a], al[b], acc[a][b], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vl[a], ah[b], acc[a][b], 0, 0, 0);
  };
  fetch(0, ra);
  stash(0, ra);
  __syncthreads();
  for (int64_t kb = 0; kb < KB; ++kb) {
    const int s = (int)(kb & 1);
    if (kb + 1 < KB) fetch(kb + 1, ra);
    block(s);
    if (kb + 1 < KB) stash(s ^ 1, ra);
    __syncthreads();
  }

  // ---- epilogue: recurrence in place, packed V_new, moment partials -------
  double p1[TM][4], p2[TM][4];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) p1[a][r] = p2[a][r] = 0.0;
#pragma unroll
  for (int a = 0; a < TM; ++a) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t j = m0 + wm * TM * 16 + a * 16 + acc_row<2>(lane, r);
      const bool jact = j < src.active;
      uint64_t key = 0;
      if (ZMODE == 1) key = sm_output(src.seed, (uint64_t)(src.first_id + j));
      int64_t cached = -1;
      uint64_t word = 0;
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int64_t n = n0 + wn * TN * 16 + b * 16 + (lane & 15);
        if (n >= d) continue;
        const int64_t idx = j * d + n;
        const float xk = vk[idx];
        float vn = ca * acc[a][b][r] + cb * xk;
        if (HAS_PREV) vn -= vm[idx];
        vm[idx] = vn;
        __bf16 h, lo;
        split_bf16(vn, h, lo);
        const int64_t q = pk_index(j, n, KB);
        pk.o_hi[q] = h;
        pk.o_lo[q] = lo;
        if (ZMODE == 0) {
          p1[a][r] += (double)xk * (double)vn;
          p2[a][r] += (double)vn * (double)vn;
        } else if (ZMODE == 1) {
          const int64_t c = n >> 6;
          if (c != cached) {
            word = sm_output(key, (uint64_t)c);
            cached = c;
          }
          p1[a][r] += sign_from_word<double>(word, n) * (double)vn;
        } else {
          const double z = jact ? (double)src.entries[n * src.ld + src.first_id + j] : 0.0;
          p1[a][r] += z * (double)vn;
        }
      }
    }
  }
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        p1[a][r] += __shfl_xor(p1[a][r], o, 64);
        p2[a][r] += __shfl_xor(p2[a][r], o, 64);
      }
  if ((lane & 15) == 0) {
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int jl = wm * TM * 16 + a * 16 + acc_row<2>(lane, r);
        sred[wn][0][jl] = p1[a][r];
        sred[wn][1][jl] = p2[a][r];
      }
  }
  __syncthreads();
  for (int e = tid; e < 2 * BM; e += 256) {
    const int slot = e / BM, jl = e % BM;
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < WN; ++w) sum += sred[w][slot][jl];
    part[((int64_t)slot * ntiles + nt) * ((int64_t)mtiles * BM) + m0 + jl] = sum;
  }
}

// Skinny blocks (32 or 64 probes per tile).  A block-square tile would give
// a few hundred single-wave workgroups that each walk the whole k range with
// one load in flight, so the step would be latency-bound.  Here a workgroup
// owns all BM probes of its tile against only 16 matrix rows, and its four
// waves split the k range between them (split-K inside the workgroup):
// wave w takes chunks w, w+4, ... of KC = 4E columns, each lane loading E
// columns of its row (64 bytes of V), the next chunks prefetched into
// registers while the current one is on the matrix cores.  No LDS staging: the MFMA
// operands come straight from the registers the loads filled, since the
// assignment of columns to an MFMA's k slots only has to agree between the
// two operands.  The four partial accumulators are summed through LDS in a
// fixed wave order, and wave a runs the epilogue of probe tile a.
//
// PK (BF16x3 only): both operands come pre-split and pre-packed in the lane
// layout of the 16x16x32 bf16 MFMA (see the packed layout below), so each
// 16-byte load of a wave covers 1 KB of contiguous memory instead of 16
// rows' worth of scattered pieces; the epilogue writes V_new packed for the
// next step as well.  The number of distinct cache lines per load, not the
// bytes, bounds the unpacked form.
template <int PREC, int TM, int W, int ZMODE, bool HAS_PREV, bool PK = false>
__global__ __launch_bounds__(64 * W) void dense_skinny_kernel(
    const void* __restrict__ A0, const void* __restrict__ A1, int64_t lda, int64_t d,
    const typename Prec<PREC>::V* __restrict__ vk, typename Prec<PREC>::V* __restrict__ vm,
    typename Prec<PREC>::V ca, typename Prec<PREC>::V cb, ProbeSrc src, int mtiles, int ntiles,
    double* __restrict__ part, PackedOps pk) {
  using P = Prec<PREC>;
  using VT = typename P::V;
  using MT = typename P::M;
  using AccT = typename P::Acc;
  constexpr int BM = TM * 16;
  constexpr int E = PREC == 0 ? 8 : 16;  // columns per lane per chunk
  constexpr int KC = 4 * E;              // columns per chunk
  // Lane group g = lane / 16 loads columns [g E, g E + E) of each chunk, as
  // 16-byte pieces (QA elements of A, QV of V): element e of a lane is the
  // same column in A and in V, which is all the MFMA k-slot assignment needs.
  constexpr int QA = 16 / (int)sizeof(MT), QV = 16 / (int)sizeof(VT);
  constexpr int NA = E / QA, NV = E / QV;  // pieces per lane per chunk
  constexpr int NSPLIT = PREC == 2 ? 2 : 1;
  typedef MT aq __attribute__((ext_vector_type(QA)));
  typedef VT vq __attribute__((ext_vector_type(QV)));
  static_assert(TM <= W, "one epilogue tile per wave");

  __shared__ AccT red[W][TM][64];

  const int total = mtiles * ntiles;
  const int L = xcd_band(blockIdx.x, (total + 7) / 8 * 8);
  if (L >= total) return;
  const int mt = L % mtiles, nt = L / mtiles;
  const int64_t m0 = (int64_t)mt * BM, n0 = (int64_t)nt * 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, rl = lane & 15;

  // Rows past d read row 0: column n of the product depends on row n of A
  // only, and the epilogue drops columns n >= d.
  const int64_t nrow = n0 + rl < d ? n0 + rl : 0;
  const MT* arow[NSPLIT];
#pragma unroll
  for (int h = 0; h < NSPLIT; ++h) arow[h] = static_cast<const MT*>(h ? A1 : A0) + nrow * lda;
  const VT* vrow[TM];
#pragma unroll
  for (int a = 0; a < TM; ++a) vrow[a] = vk + (m0 + a * 16 + rl) * d;

  // NS accumulators per probe tile, so that consecutive MFMAs of one wave
  // are independent (a chain of dependent MFMAs issues at a fraction of the
  // matrix-core rate): bf16x3 keeps one per product (hi*hi, hi*lo, lo*hi),
  // FP32 and FP64 one per k slot modulo NS.  Summed in a fixed order.
  constexpr int NS = PREC == 2 ? 3 : (PREC == 1 ? 2 : 1);
  AccT acc[TM][NS];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int q = 0; q < NS; ++q) acc[a][q] = AccT{};

  aq ra[NSPLIT][NA], xa[NSPLIT][NA];
  vq rv[TM][NV], xv[TM][NV];
  auto load = [&](int64_t c, aq (&ta)[NSPLIT][NA], vq (&tv)[TM][NV]) {
    const int64_t k = c * KC + g * E;
#pragma unroll
    for (int h = 0; h < NSPLIT; ++h)
#pragma unroll
      for (int p = 0; p < NA; ++p) ta[h][p] = *reinterpret_cast<const aq*>(arow[h] + k + p * QA);
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int p = 0; p < NV; ++p) tv[a][p] = *reinterpret_cast<const vq*>(vrow[a] + k + p * QV);
  };
  auto compute = [&](const aq (&ta)[NSPLIT][NA], const vq (&tv)[TM][NV]) {
    if constexpr (PREC == 2) {
#pragma unroll
      for (int t = 0; t < E / 8; ++t) {
        const bf8 bh = ta[0][t], bl = ta[1][t];
#pragma unroll
        for (int a = 0; a < TM; ++a) {
          bf8 vh, vl;
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            __bf16 hi, lo;
            split_bf16(tv[a][(8 * t + q) / QV][(8 * t + q) % QV], hi, lo);
            vh[q] = hi;
            vl[q] = lo;
          }
          acc[a][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vh, bh, acc[a][0], 0, 0, 0);
          acc[a][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vh, bl, acc[a][1], 0, 0, 0);
          acc[a][2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vl, bh, acc[a][2], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < E; ++t) {
        const MT b = ta[0][t / QA][t % QA];
#pragma unroll
        for (int a = 0; a < TM; ++a) {
          const VT x = tv[a][t / QV][t % QV];
          if constexpr (PREC == 0)
            acc[a][t % NS] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, b, acc[a][t % NS], 0, 0, 0);
          else
            acc[a][t % NS] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, b, acc[a][t % NS], 0, 0, 0);
        }
      }
    }
  };

  // Two register buffers in turn: chunk i + 1 streams into one while chunk
  // i is on the matrix cores from the other.  After each load group, an
  // empty asm with a memory clobber keeps the compiler from merging the
  // loads that feed a loop-carried buffer into one load at the top of the
  // loop, and a scheduling barrier keeps the instruction scheduler from
  // sinking the loads down to their uses (either would turn the prefetch
  // back into load-then-use).  Past the last chunk a load re-reads that
  // chunk (a cache hit), so every load in the loop is unconditional.
  if constexpr (PK) {
    static_assert(PREC == 2, "packed operands are bf16 hi / lo");
    // k blocks of 32: wave w takes blocks w, w + W, ...; two register sets
    // in turn, as below.  Padding (k >= d, rows >= d) is zero in both.
    const int64_t KB = pk_kblocks(d);
    const bf8* ph = pk.a_hi + ((int64_t)nt * KB) * 64 + lane;
    const bf8* pl = pk.a_lo + ((int64_t)nt * KB) * 64 + lane;
    const bf8* qh = pk.v_hi + ((int64_t)(m0 / 16) * KB) * 64 + lane;
    const bf8* ql = pk.v_lo + ((int64_t)(m0 / 16) * KB) * 64 + lane;
    const int64_t nk = KB > wave ? (KB - wave + W - 1) / W : 0;
    auto kbof = [&](int64_t i) { return (int64_t)wave + (i < nk ? i : nk - 1) * W; };
    bf8 b0h, b0l, b1h, b1l, x0h[TM], x0l[TM], x1h[TM], x1l[TM];
    auto ld = [&](int64_t kb, bf8& bh, bf8& bl, bf8 (&xh)[TM], bf8 (&xl)[TM]) {
      bh = ph[kb * 64];
      bl = pl[kb * 64];
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        xh[a] = qh[(a * KB + kb) * 64];
        xl[a] = ql[(a * KB + kb) * 64];
      }
    };
    auto mm = [&](const bf8& bh, const bf8& bl, const bf8 (&xh)[TM], const bf8 (&xl)[TM]) {
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        acc[a][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[a], bh, acc[a][0], 0, 0, 0);
        acc[a][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[a], bl, acc[a][1], 0, 0, 0);
        acc[a][2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl[a], bh, acc[a][2], 0, 0, 0);
      }
    };
    if (nk > 0) {
      ld(kbof(0), b0h, b0l, x0h, x0l);
      asm volatile("" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
      int64_t i = 0;
      for (; i + 2 <= nk; i += 2) {
        ld(kbof(i + 1), b1h, b1l, x1h, x1l);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        mm(b0h, b0l, x0h, x0l);
        ld(kbof(i + 2), b0h, b0l, x0h, x0l);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        mm(b1h, b1l, x1h, x1l);
      }
      if (i < nk) mm(b0h, b0l, x0h, x0l);
    }
  } else {
  const int64_t nfull = d / KC;
  const int64_t mine = wave < nfull ? (nfull - wave + W - 1) / W : 0;  // chunks of this wave
  auto chunk = [&](int64_t i) { return (int64_t)wave + (i < mine ? i : mine - 1) * W; };
  if (mine > 0) {
    load(chunk(0), ra, rv);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    int64_t i = 0;
    for (; i + 2 <= mine; i += 2) {
      load(chunk(i + 1), xa, xv);
      asm volatile("" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
      compute(ra, rv);
      load(chunk(i + 2), ra, rv);
      asm volatile("" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
      compute(xa, xv);
    }
    if (i < mine) compute(ra, rv);
  }
  // ragged tail [nfull * KC, d): element loads, zero past d in both operands
  if (nfull * KC < d && wave == (int)(nfull % W)) {
    const int64_t k0 = nfull * KC + g * E;
#pragma unroll
    for (int h = 0; h < NSPLIT; ++h)
#pragma unroll
      for (int p = 0; p < NA; ++p)
#pragma unroll
        for (int q = 0; q < QA; ++q) {
          const int64_t k = k0 + p * QA + q;
          ra[h][p][q] = k < d ? arow[h][k] : MT(0.f);
        }
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int p = 0; p < NV; ++p)
#pragma unroll
        for (int q = 0; q < QV; ++q) {
          const int64_t k = k0 + p * QV + q;
          rv[a][p][q] = k < d ? vrow[a][k] : VT(0);
        }
    compute(ra, rv);
  }
  }  // unpacked operands

#pragma unroll
  for (int a = 0; a < TM; ++a) {
    AccT t = acc[a][0];
#pragma unroll
    for (int q = 1; q < NS; ++q) t += acc[a][q];
    red[wave][a][lane] = t;
  }
  __syncthreads();
  if (wave >= TM) return;

  // ---- epilogue of probe tile a = wave: recurrence in place, partials ----
  const int a = wave;
  AccT sum = red[0][a][lane];
#pragma unroll
  for (int w = 1; w < W; ++w) sum += red[w][a][lane];
  const int64_t n = n0 + rl;
  double p1[4], p2[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    p1[r] = p2[r] = 0.0;
    const int64_t j = m0 + a * 16 + acc_row<PREC>(lane, r);
    if (n >= d) continue;
    const int64_t idx = j * d + n;
    const VT x = vk[idx];
    VT vn = ca * (VT)sum[r] + cb * x;
    if (HAS_PREV) vn -= vm[idx];
    vm[idx] = vn;
    if constexpr (PK) {
      __bf16 h, lo;
      split_bf16((float)vn, h, lo);
      const int64_t q = pk_index(j, n, pk_kblocks(d));
      pk.o_hi[q] = h;
      pk.o_lo[q] = lo;
    }
    if (ZMODE == 0) {
      p1[r] = (double)x * (double)vn;
      p2[r] = (double)vn * (double)vn;
    } else if (ZMODE == 1) {
      const uint64_t key = sm_output(src.seed, (uint64_t)(src.first_id + j));
      p1[r] = sign_from_word<double>(sm_output(key, (uint64_t)(n >> 6)), n) * (double)vn;
    } else {
      const double z = j < src.active ? (double)src.entries[n * src.ld + src.first_id + j] : 0.0;
      p1[r] = z * (double)vn;
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      p1[r] += __shfl_xor(p1[r], o, 64);
      p2[r] += __shfl_xor(p2[r], o, 64);
    }
  if (rl == 0) {
    const int64_t width = (int64_t)mtiles * BM;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t j = m0 + a * 16 + acc_row<PREC>(lane, r);
      part[(int64_t)nt * width + j] = p1[r];
      part[((int64_t)ntiles + nt) * width + j] = p2[r];
    }
  }
}

// V0^T[j][n] = z_n^(j) for j < active (0 for padding rows) and the moment
// mu_0 = z.z per probe (one workgroup per probe row, fixed-order sum).
template <typename VT>
__global__ __launch_bounds__(256) void dense_probe_init_kernel(VT* __restrict__ v0, int64_t d,
                                                               ProbeSrc src,
                                                               double* __restrict__ dots0) {
  __shared__ double sh[256];
  const int64_t j = blockIdx.x;
  const bool act = j < src.active;
  const uint64_t key = sm_output(src.seed, (uint64_t)(src.first_id + j));
  double s = 0.0;
  for (int64_t n = threadIdx.x; n < d; n += 256) {
    VT z = VT(0);
    if (act) {
      if (src.entries)
        z = (VT)src.entries[n * src.ld + src.first_id + j];
      else
        z = sign_from_word<VT>(sm_output(key, (uint64_t)(n >> 6)), n);
    }
    v0[j * d + n] = z;
    s += (double)z * (double)z;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) dots0[j] = sh[0];
}

// A_hi = bf16(A), A_lo = bf16(A - A_hi), from FP32 or FP64 A (row-major).
// Pack rows x d values (row stride ld; FP32 split into bf16 hi / lo, or
// bf16 hi and lo given apart) into the packed lane layout, zero past the
// rows and columns (all of rp x ceil(d / 32) * 32, rp a multiple of 16).
template <typename ST>
__global__ __launch_bounds__(256) void pack_kernel(const ST* __restrict__ hi_or_val,
                                                   const ST* __restrict__ lo, int64_t rows,
                                                   int64_t rp, int64_t d, int64_t ld,
                                                   __bf16* __restrict__ out_hi,
                                                   __bf16* __restrict__ out_lo) {
  const int64_t KB = pk_kblocks(d);
  const int64_t cols = KB * 32;
  const int64_t total = rp * cols;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * 256) {
    const int64_t r = t / cols, k = t % cols;
    __bf16 h = (__bf16)0.f, l = (__bf16)0.f;
    if (r < rows && k < d) {
      if constexpr (std::is_same<ST, float>::value) {
        split_bf16(hi_or_val[r * ld + k], h, l);
      } else {
        h = hi_or_val[r * ld + k];
        l = lo[r * ld + k];
      }
    }
    const int64_t q = pk_index(r, k, KB);
    out_hi[q] = h;
    out_lo[q] = l;
  }
}

template <typename ST>
__global__ void split_kernel(const ST* __restrict__ a, int64_t d, int64_t lda,
                             __bf16* __restrict__ hi, __bf16* __restrict__ lo) {
  const int64_t total = d * d;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / d, c = e % d;
    __bf16 h, l;
    split_bf16((float)a[r * lda + c], h, l);
    hi[e] = h;
    lo[e] = l;
  }
}

template <typename ST, typename DT>
__global__ void convert_kernel(const ST* __restrict__ a, int64_t d, int64_t lda,
                               DT* __restrict__ out) {
  const int64_t total = d * d;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / d, c = e % d;
    out[e] = (DT)a[r * lda + c];
  }
}

// Gram matrix G = X^T X (X row-major rows x cols, FP32) on FP32 MFMA.  Only
// tiles with nt >= mt are computed; each writes G[i][j] and G[j][i] from the
// same accumulator, so G is exactly symmetric.  Slices of BK rows of both
// column panels go through two LDS stages: the next slice's global loads
// (16-byte when VEC: cols and ldx multiples of 4, X 16-byte aligned) are in
// flight in registers while the current slice is on the matrix cores.
template <int WM, int WN, int TM, int TN, int BK, bool VEC>
__global__ __launch_bounds__(64 * WM * WN) void gram_kernel(const float* __restrict__ X,
                                                            int64_t rows, int64_t cols,
                                                            int64_t ldx, float* __restrict__ G,
                                                            int tiles) {
  constexpr int NT = 64 * WM * WN;
  constexpr int BM = WM * TM * 16, BN = WN * TN * 16;
  static_assert(BM == BN, "square tiles");
  constexpr int PER = BK * BM / NT;  // elements of each panel per thread per slice
  static_assert(PER % 4 == 0, "slices in 4-element pieces");
  __shared__ float sX[2][2][BK][BM + 4];  // [stage][panel]
  // upper-triangular tile pair (mt <= nt) from the linear index
  int L = blockIdx.x, mt = 0;
  while (L >= tiles - mt) {
    L -= tiles - mt;
    ++mt;
  }
  const int nt = mt + L;
  const int64_t i0 = (int64_t)mt * BM, j0 = (int64_t)nt * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  f4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = f4{};
  // thread piece q covers slice element e = (q NT + tid) 4 .. +3 of a panel
  float ra[PER], rb[PER];
  auto gload = [&](int64_t r0) {
#pragma unroll
    for (int q = 0; q < PER / 4; ++q) {
      const int e = (q * NT + tid) * 4;
      const int k = e / BM, c = e % BM;
      const int64_t r = r0 + k;
      if constexpr (VEC) {
        float4 va = {0.f, 0.f, 0.f, 0.f}, vb = {0.f, 0.f, 0.f, 0.f};
        if (r < rows && i0 + c < cols) va = *reinterpret_cast<const float4*>(X + r * ldx + i0 + c);
        if (r < rows && j0 + c < cols) vb = *reinterpret_cast<const float4*>(X + r * ldx + j0 + c);
        ra[4 * q] = va.x; ra[4 * q + 1] = va.y; ra[4 * q + 2] = va.z; ra[4 * q + 3] = va.w;
        rb[4 * q] = vb.x; rb[4 * q + 1] = vb.y; rb[4 * q + 2] = vb.z; rb[4 * q + 3] = vb.w;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ra[4 * q + u] = (r < rows && i0 + c + u < cols) ? X[r * ldx + i0 + c + u] : 0.f;
          rb[4 * q + u] = (r < rows && j0 + c + u < cols) ? X[r * ldx + j0 + c + u] : 0.f;
        }
      }
    }
  };
  auto sstore = [&](int st) {
#pragma unroll
    for (int q = 0; q < PER / 4; ++q) {
      const int e = (q * NT + tid) * 4;
      const int k = e / BM, c = e % BM;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        sX[st][0][k][c + u] = ra[4 * q + u];
        sX[st][1][k][c + u] = rb[4 * q + u];
      }
    }
  };
  const int64_t nit = (rows + BK - 1) / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int64_t it = 0; it < nit; ++it) {
    const int st = (int)(it & 1);
    if (it + 1 < nit) gload((it + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      float av[TM], bv[TN];
      const int k = kk + (lane >> 4);
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = sX[st][0][k][wm * TM * 16 + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < TN; ++b) bv[b] = sX[st][1][k][wn * TN * 16 + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    // the other stage was last read in the previous iteration, before the
    // barrier that ended it
    if (it + 1 < nit) sstore(st ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wm * TM * 16 + a * 16 + (lane >> 4) * 4 + r;
        const int64_t j = j0 + wn * TN * 16 + b * 16 + (lane & 15);
        if (i < cols && j < cols) {
          G[i * cols + j] = acc[a][b][r];
          G[j * cols + i] = acc[a][b][r];
        }
      }
}

template <int PREC, int WM, int WN, int TM, int TN, int BK>
hipError_t launch_dense_cfg(hipStream_t s, const DenseStepArgs& a) {
  using VT = typename Prec<PREC>::V;
  constexpr int BM = WM * TM * 16, BN = WN * TN * 16;
  const int mtiles = (int)(a.bpad / BM);
  const int ntiles = (int)((a.d + BN - 1) / BN);
  const int grid = (mtiles * ntiles + 7) / 8 * 8;
  const VT ca = (VT)a.ca, cb = (VT)a.cb;
  const VT* vk = static_cast<const VT*>(a.vk);
  VT* vm = static_cast<VT*>(a.vm);
#define MLCT_DENSE_LAUNCH(Z, HP)                                                           \
  dense_step_kernel<PREC, WM, WN, TM, TN, BK, Z, HP><<<grid, 64 * WM * WN, 0, s>>>(        \
      a.A0, a.A1, a.lda, a.d, vk, vm, ca, cb, a.src, mtiles, ntiles, a.part)
  if (a.has_prev) {
    if (a.zmode == 0) MLCT_DENSE_LAUNCH(0, true);
    else if (a.zmode == 1) MLCT_DENSE_LAUNCH(1, true);
    else MLCT_DENSE_LAUNCH(2, true);
  } else {
    if (a.zmode == 0) MLCT_DENSE_LAUNCH(0, false);
    else if (a.zmode == 1) MLCT_DENSE_LAUNCH(1, false);
    else MLCT_DENSE_LAUNCH(2, false);
  }
#undef MLCT_DENSE_LAUNCH
  return hipGetLastError();
}

template <int PREC, int TM, int W>
hipError_t launch_skinny_cfg(hipStream_t s, const DenseStepArgs& a) {
  using VT = typename Prec<PREC>::V;
  const int mtiles = (int)(a.bpad / (TM * 16));
  const int ntiles = (int)((a.d + 15) / 16);
  const int grid = (mtiles * ntiles + 7) / 8 * 8;
  const VT ca = (VT)a.ca, cb = (VT)a.cb;
  const VT* vk = static_cast<const VT*>(a.vk);
  VT* vm = static_cast<VT*>(a.vm);
  const PackedOps pk{static_cast<const bf8*>(a.pk_a_hi), static_cast<const bf8*>(a.pk_a_lo),
                     static_cast<const bf8*>(a.pk_v_hi), static_cast<const bf8*>(a.pk_v_lo),
                     static_cast<__bf16*>(a.pk_o_hi), static_cast<__bf16*>(a.pk_o_lo)};
  const bool packed = PREC == 2 && a.pk_a_hi != nullptr;
#define MLCT_SKINNY_LAUNCH(Z, HP)                                                             \
  if (packed)                                                                                 \
    dense_skinny_kernel<PREC, TM, W, Z, HP, PREC == 2><<<grid, 64 * W, 0, s>>>(                \
        a.A0, a.A1, a.lda, a.d, vk, vm, ca, cb, a.src, mtiles, ntiles, a.part, pk);            \
  else                                                                                        \
    dense_skinny_kernel<PREC, TM, W, Z, HP><<<grid, 64 * W, 0, s>>>(                           \
        a.A0, a.A1, a.lda, a.d, vk, vm, ca, cb, a.src, mtiles, ntiles, a.part, pk)
  if (a.has_prev) {
    if (a.zmode == 0) MLCT_SKINNY_LAUNCH(0, true);
    else if (a.zmode == 1) MLCT_SKINNY_LAUNCH(1, true);
    else MLCT_SKINNY_LAUNCH(2, true);
  } else {
    if (a.zmode == 0) MLCT_SKINNY_LAUNCH(0, false);
    else if (a.zmode == 1) MLCT_SKINNY_LAUNCH(1, false);
    else MLCT_SKINNY_LAUNCH(2, false);
  }
#undef MLCT_SKINNY_LAUNCH
  return hipGetLastError();
}

// The packed wide kernel for BF16x3 blocks of 128-probe tiles.
hipError_t launch_pk_gemm(hipStream_t s, const DenseStepArgs& a) {
  const int mtiles = (int)(a.bpad / 128), ntiles = (int)((a.d + 127) / 128);
  const int grid = (mtiles * ntiles + 7) / 8 * 8;
  const PackedOps pk{static_cast<const bf8*>(a.pk_a_hi), static_cast<const bf8*>(a.pk_a_lo),
                     static_cast<const bf8*>(a.pk_v_hi), static_cast<const bf8*>(a.pk_v_lo),
                     static_cast<__bf16*>(a.pk_o_hi), static_cast<__bf16*>(a.pk_o_lo)};
  const float* vk = static_cast<const float*>(a.vk);
  float* vm = static_cast<float*>(a.vm);
  const float ca = (float)a.ca, cb = (float)a.cb;
#define MLCT_PKG(Z, HP)                                                                    \
  dense_pk_gemm_kernel<Z, HP><<<grid, 256, 0, s>>>(a.d, vk, vm, ca, cb, a.src, mtiles, ntiles, \
                                                   a.part, pk)
  if (a.has_prev) {
    if (a.zmode == 0) MLCT_PKG(0, true);
    else if (a.zmode == 1) MLCT_PKG(1, true);
    else MLCT_PKG(2, true);
  } else {
    if (a.zmode == 0) MLCT_PKG(0, false);
    else if (a.zmode == 1) MLCT_PKG(1, false);
    else MLCT_PKG(2, false);
  }
#undef MLCT_PKG
  return hipGetLastError();
}

}  // namespace

DenseTile dense_tile(int prec, int64_t d, int64_t lda, int64_t bpad, int force) {
  // Blocks of at most 64 probes (512 for BF16x3) take the skinny split-K
  // kernel (16-row tiles) when rows are 16-byte aligned.  Otherwise the largest square tile
  // that still gives a few hundred workgroups: 128 x 128, then 64 x 64; a
  // problem too small for either takes the skinny kernel over several probe
  // tiles (it splits k over four waves: FP64 d = 512, 256 probes, degree 64
  // in 0.61 ms against 1.52 ms on 32 x 32 tiles, d = 2048 2.8 vs 5.2 ms),
  // else 32 x 32.
  // force: 0 = 32, 1 = 128, 2 = 64, 3 = skinny (when the block allows it).
  // the skinny kernel's 16-byte loads need 16-byte aligned rows of V and A
  const int qv = prec == MLCT_FP64 ? 2 : 4, qa = prec == MLCT_FP64 ? 2 : (prec == MLCT_FP32 ? 4 : 8);
  const bool skinny_ok = d % qv == 0 && lda % qa == 0;
  const int64_t n128 = (bpad / 128) * ((d + 127) / 128);
  const int64_t n64 = (bpad / 64) * ((d + 63) / 64);
  DenseTile t;
  t.skinny = false;
  int size = 32;
  if (force == 3 && skinny_ok) t.skinny = true;
  else if (force == 1 && bpad % 128 == 0) size = 128;
  else if (force == 2 && bpad % 64 == 0) size = 64;
  else if (force < 0) {
    // BF16x3 reads packed operands on the skinny kernel, which beats square
    // tiles up to 512 probes (d = 4096: 69 vs 124 us at 320, 108 vs 119 at
    // 512); FP64 and FP32 read row-major arrays and keep it to 64
    const int64_t skinny_max = prec == MLCT_BF16X3 ? 512 : 64;
    if (bpad <= skinny_max && skinny_ok) t.skinny = true;
    else if (bpad % 128 == 0 && n128 >= 256) size = 128;
    else if (bpad % 64 == 0 && n64 >= 256) size = 64;
    else if (skinny_ok) t.skinny = true;
  }
  if (t.skinny) {
    t.large = false;
    t.bm = bpad % 64 == 0 ? 64 : 32;
    t.bn = 16;
    return t;
  }
  t.large = size == 128;
  t.bm = t.bn = size;
  return t;
}

hipError_t launch_dense_step(hipStream_t s, int prec, const DenseStepArgs& a) {
  const DenseTile t = dense_tile(prec, a.d, a.lda, a.bpad, a.tile_force);
  if (t.skinny) {
    constexpr int W = 4;
    if (prec == MLCT_FP64)
      return t.bm == 64 ? launch_skinny_cfg<0, 4, W>(s, a) : launch_skinny_cfg<0, 2, W>(s, a);
    if (prec == MLCT_FP32)
      return t.bm == 64 ? launch_skinny_cfg<1, 4, W>(s, a) : launch_skinny_cfg<1, 2, W>(s, a);
    return t.bm == 64 ? launch_skinny_cfg<2, 4, W>(s, a) : launch_skinny_cfg<2, 2, W>(s, a);
  }
  if (prec == MLCT_FP64) {
    if (t.bm == 128) return launch_dense_cfg<0, 2, 2, 4, 4, 16>(s, a);
    if (t.bm == 64) return launch_dense_cfg<0, 2, 2, 2, 2, 16>(s, a);
    return launch_dense_cfg<0, 1, 1, 2, 2, 16>(s, a);
  }
  if (prec == MLCT_FP32) {
    if (t.bm == 128) return launch_dense_cfg<1, 2, 2, 4, 4, 16>(s, a);
    if (t.bm == 64) return launch_dense_cfg<1, 2, 2, 2, 2, 16>(s, a);
    return launch_dense_cfg<1, 1, 1, 2, 2, 16>(s, a);
  }
  if (t.bm == 128) {
    if (a.pk_a_hi) return launch_pk_gemm(s, a);
    return launch_dense_cfg<2, 2, 2, 4, 4, 64>(s, a);
  }
  if (t.bm == 64) return launch_dense_cfg<2, 2, 2, 2, 2, 64>(s, a);
  return launch_dense_cfg<2, 1, 1, 2, 2, 32>(s, a);
}

hipError_t launch_dense_probe_init(hipStream_t s, int prec, void* v0, int64_t d, int64_t bpad,
                                   ProbeSrc src, double* dots0) {
  if (prec == MLCT_FP64)
    dense_probe_init_kernel<double><<<(int)bpad, 256, 0, s>>>(static_cast<double*>(v0), d, src, dots0);
  else
    dense_probe_init_kernel<float><<<(int)bpad, 256, 0, s>>>(static_cast<float*>(v0), d, src, dots0);
  return hipGetLastError();
}

hipError_t launch_dense_split(hipStream_t s, const void* a, int dtype, int64_t d, int64_t lda,
                              void* hi, void* lo) {
  if (dtype == MLCT_DT_F64)
    split_kernel<double><<<2048, 256, 0, s>>>(static_cast<const double*>(a), d, lda,
                                               static_cast<__bf16*>(hi), static_cast<__bf16*>(lo));
  else
    split_kernel<float><<<2048, 256, 0, s>>>(static_cast<const float*>(a), d, lda,
                                              static_cast<__bf16*>(hi), static_cast<__bf16*>(lo));
  return hipGetLastError();
}

// Packed rows are padded to a multiple of 128 (the wide kernel's tile).
static int64_t pk_rows(int64_t rows) { return (rows + 127) / 128 * 128; }

size_t dense_pack_bytes(int64_t rows, int64_t d) {
  return (size_t)(pk_rows(rows) / 16) * (size_t)pk_kblocks(d) * 64 * 8 * sizeof(__bf16);
}

hipError_t launch_dense_pack_a(hipStream_t s, const void* hi, const void* lo, int64_t d,
                               void* out_hi, void* out_lo) {
  pack_kernel<__bf16><<<2048, 256, 0, s>>>(static_cast<const __bf16*>(hi),
                                           static_cast<const __bf16*>(lo), d, pk_rows(d), d, d,
                                           static_cast<__bf16*>(out_hi),
                                           static_cast<__bf16*>(out_lo));
  return hipGetLastError();
}

hipError_t launch_dense_pack_v(hipStream_t s, const float* v, int64_t rows, int64_t d,
                               void* out_hi, void* out_lo) {
  pack_kernel<float><<<512, 256, 0, s>>>(v, nullptr, rows, pk_rows(rows), d, d,
                                         static_cast<__bf16*>(out_hi),
                                         static_cast<__bf16*>(out_lo));
  return hipGetLastError();
}

hipError_t launch_dense_convert(hipStream_t s, const void* a, int src_dtype, int64_t d,
                                int64_t lda, void* out) {
  if (src_dtype == MLCT_DT_F64)
    convert_kernel<double, float><<<2048, 256, 0, s>>>(static_cast<const double*>(a), d, lda,
                                                       static_cast<float*>(out));
  else
    convert_kernel<float, double><<<2048, 256, 0, s>>>(static_cast<const float*>(a), d, lda,
                                                       static_cast<double*>(out));
  return hipGetLastError();
}

hipError_t launch_gram(hipStream_t s, const float* X, int64_t rows, int64_t cols, int64_t ldx,
                       float* G) {
  constexpr int T = 128;
  const int tiles = (int)((cols + T - 1) / T);
  const int grid = tiles * (tiles + 1) / 2;
  const bool vec = cols % 4 == 0 && ldx % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0;
  if (vec) gram_kernel<2, 2, 4, 4, 16, true><<<grid, 256, 0, s>>>(X, rows, cols, ldx, G, tiles);
  else gram_kernel<2, 2, 4, 4, 16, false><<<grid, 256, 0, s>>>(X, rows, cols, ldx, G, tiles);
  return hipGetLastError();
}

}  // namespace mlct
