// Support kernels of the two-steps-per-launch CSR path (csr_fused2_kernel in
// k_csr.hip): the operator's bandwidth, which decides whether two steps fit
// one launch; the clearing of a launch's tickets and flags, with a check
// that the previous launch's tickets were all taken; and the XCD probe that
// tells whether every XCD receives workgroups of a launch.
#include "device.hpp"

namespace mlct {

namespace {

// Clears p[0 .. n-1]; first, when the previous launch issued prev_total
// tickets per XCD, marks (abort value 2) an XCD whose counter stayed short
// of it: that XCD's range of tiles was not processed.
__global__ void fused_sync_kernel(int* __restrict__ p, int64_t n, int prev_total,
                                  int* __restrict__ abort_flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 8 && prev_total > 0 && p[i] < prev_total) atomicMax(abort_flag, 2);
  if (i < n) p[i] = 0;
}

// XCD of each workgroup of a launch.
__global__ void xcc_probe_kernel(int* __restrict__ out) {
  if (threadIdx.x == 0) out[blockIdx.x] = xcc_of_wg();
}

// out[0] = max over entries of |column - row| (atomic maximum).
__global__ __launch_bounds__(256) void csr_bandwidth_kernel(const int32_t* __restrict__ rowptr,
                                                            const int32_t* __restrict__ col,
                                                            int64_t d, int32_t* __restrict__ out) {
  int64_t best = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d;
       i += (int64_t)gridDim.x * blockDim.x) {
    for (int t = rowptr[i]; t < rowptr[i + 1]; ++t) {
      const int64_t o = (int64_t)col[t] - i;
      best = max(best, o < 0 ? -o : o);
    }
  }
  if (best) atomicMax(out, (int32_t)min<int64_t>(best, 0x7fffffff));
}

}  // namespace

hipError_t launch_fused_sync(hipStream_t s, int* sync, int64_t n, int prev_total,
                             int* abort_flag) {
  const int64_t threads = std::max<int64_t>(n, 8);
  fused_sync_kernel<<<(unsigned)((threads + 255) / 256), 256, 0, s>>>(sync, n, prev_total,
                                                                      abort_flag);
  return hipGetLastError();
}

hipError_t launch_fill_zero_i32(hipStream_t s, int* p, int64_t n) {
  if (n <= 0) return hipSuccess;
  return launch_fused_sync(s, p, n, 0, nullptr);
}

hipError_t launch_xcc_probe(hipStream_t s, int* out, int grid) {
  xcc_probe_kernel<<<grid, 64, 0, s>>>(out);
  return hipGetLastError();
}

hipError_t launch_csr_bandwidth(hipStream_t s, const int32_t* rowptr, const int32_t* col,
                                int64_t d, int32_t* out) {
  int64_t blocks = (d + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  csr_bandwidth_kernel<<<(unsigned)blocks, 256, 0, s>>>(rowptr, col, d, out);
  return hipGetLastError();
}

}  // namespace mlct
