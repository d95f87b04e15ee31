// Bandwidth probes that ground the rooflines of the evaluation kernels in
// measured rather than published peaks: HBM (a streaming copy) and LDS (a
// conflict-free ds_read_b128 stream per workgroup).
#include <hip/hip_runtime.h>

#include "bl_internal.h"

namespace bl {

namespace {

// dst = src, n16 16-byte words, grid-stride.
__global__ __launch_bounds__(256) void k_peak_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                   size_t n16) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

constexpr int kPeakLdsWords = 2048;  // uint4 words: 32 KB per workgroup

// Each lane reads 16 bytes per step from LDS, consecutive lanes consecutive
// words (no bank conflicts), `steps` steps; the XOR of what it read goes to
// out so that the reads stay.
__global__ __launch_bounds__(256) void k_peak_lds(uint32_t steps, uint32_t *out) {
  __shared__ uint4 buf[kPeakLdsWords];
  for (int i = threadIdx.x; i < kPeakLdsWords; i += blockDim.x)
    buf[i] = uint4{(uint32_t)i, (uint32_t)i * 3u, (uint32_t)i * 5u, (uint32_t)i * 7u};
  __syncthreads();
  uint4 acc{0u, 0u, 0u, 0u};
  uint32_t idx = threadIdx.x;
#pragma unroll 8
  for (uint32_t s = 0; s < steps; ++s) {
    const uint4 v = buf[idx];
    acc.x ^= v.x;
    acc.y ^= v.y;
    acc.z ^= v.z;
    acc.w ^= v.w;
    idx = (idx + blockDim.x) & (kPeakLdsWords - 1);
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

}  // namespace

hipError_t launch_peak_copy(const void *src, void *dst, size_t bytes, int n_cu, hipStream_t s) {
  hipLaunchKernelGGL(k_peak_copy, dim3(n_cu * 8), dim3(256), 0, s, reinterpret_cast<const uint4 *>(src),
                     reinterpret_cast<uint4 *>(dst), bytes / 16);
  return hipGetLastError();
}

size_t peak_lds_blocks(int n_cu) { return (size_t)n_cu * 4; }

hipError_t launch_peak_lds(uint32_t steps, uint32_t *out, int n_cu, hipStream_t s) {
  hipLaunchKernelGGL(k_peak_lds, dim3((unsigned)peak_lds_blocks(n_cu)), dim3(256), 0, s, steps, out);
  return hipGetLastError();
}

}  // namespace bl
