// Device-side helpers shared by the HIP kernels of libmlct.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace mlct {

// SplitMix64 output function (Steele, Lea & Flood 2014).
__device__ __forceinline__ uint64_t sm_mix(uint64_t x) {
  x = (x ^ (x >> 30)) * kMul1;
  x = (x ^ (x >> 27)) * kMul2;
  return x ^ (x >> 31);
}

// Output number k (0-based) of SplitMix64 started at state s.
__device__ __forceinline__ uint64_t sm_output(uint64_t s, uint64_t k) {
  return sm_mix(s + (k + 1) * kGamma);
}

// Rademacher entry from the 64-bit word that holds row i's sign bit.
template <typename T>
__device__ __forceinline__ T sign_from_word(uint64_t word, int64_t i) {
  return ((word >> (i & 63)) & 1ull) ? T(-1) : T(1);
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b % 8).  Map b to a chunk index so that each XCD walks one contiguous
// band of chunks, which keeps neighbouring rows in the same L2.
// ngroups must be a multiple of 8.
__device__ __forceinline__ int xcd_band(int b, int ngroups) {
  const int per = ngroups >> 3;
  return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// XCD (XCC) that executes the calling workgroup, from the hardware register.
__device__ __forceinline__ int xcc_of_wg() {
  unsigned v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(v));
  return (int)(v & 7u);
}

// The functions f of tr f(A) (mlct_func_kind).
__device__ __forceinline__ double eval_f(int kind, double power, double t) {
  switch (kind) {
    case MLCT_LOG: return log(t);
    case MLCT_SQRT: return sqrt(t);
    case MLCT_EXP: return exp(t);
    case MLCT_CUBE: return t * t * t;
    case MLCT_INV: return 1.0 / t;
    default: return pow(t, power);
  }
}

template <typename T>
__device__ __forceinline__ T read_lane(T v, int l);

template <>
__device__ __forceinline__ int read_lane<int>(int v, int l) {
  return __builtin_amdgcn_readlane(v, l);
}
template <>
__device__ __forceinline__ float read_lane<float>(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

}  // namespace mlct
