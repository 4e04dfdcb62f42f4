// Kernels without a storage type: the fixed-order reduction of per-block
// partials, the time-counter set, and the streaming copy of the bandwidth
// reference.
#include "runtime.hpp"

namespace lbm {

// Reduce per-block partials (single workgroup, fixed order: deterministic).
// opmask holds 2 bits per entry: 0 sum, 1 max, 2 min.
__global__ __launch_bounds__(BLOCK) void k_finalize(const double* part, int nblk, int n, uint32_t opmask, double* out) {
  __shared__ double sh[BLOCK];
  for (int k = 0; k < n; ++k) {
    const int op = (int)((opmask >> (2 * k)) & 3u);
    double r = op == 0 ? 0.0 : (op == 1 ? -1e300 : 1e300);
    for (int i = threadIdx.x; i < nblk; i += BLOCK) {
      const double v = part[(size_t)i * n + k];
      r = op == 0 ? r + v : (op == 1 ? fmax(r, v) : fmin(r, v));
    }
    sh[threadIdx.x] = r;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        const double a = sh[threadIdx.x], c2 = sh[threadIdx.x + s];
        sh[threadIdx.x] = op == 0 ? a + c2 : (op == 1 ? fmax(a, c2) : fmin(a, c2));
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sh[0];
    __syncthreads();
  }
}

// Set the time counter slot of parity t & 1 to t (one work-item).
__global__ void k_set_time(uint32_t* tc, uint32_t t) {
  if (blockIdx.x == 0 && threadIdx.x == 0) tc[t & 1u] = t;
}

// Plain streaming copy (16-byte vectors), the achievable-bandwidth reference.
__global__ __launch_bounds__(BLOCK) void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
  size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * BLOCK;
  for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace lbm

namespace lbmrt {

void launch_finalize(hipStream_t s, const double* part, int nparts, int n, uint32_t ops, double* out) {
  hipLaunchKernelGGL(lbm::k_finalize, dim3(1), dim3(BLOCK), 0, s, part, nparts, n, ops, out);
}

void launch_set_time(hipStream_t s, uint32_t* tc, uint32_t t) {
  hipLaunchKernelGGL(lbm::k_set_time, dim3(1), dim3(64), 0, s, tc, t);
}

void launch_copy(hipStream_t s, const void* src, void* dst, size_t n16, unsigned blocks) {
  hipLaunchKernelGGL(lbm::k_copy, dim3(blocks), dim3(BLOCK), 0, s, (const uint4*)src, (uint4*)dst, n16);
}

}  // namespace lbmrt
