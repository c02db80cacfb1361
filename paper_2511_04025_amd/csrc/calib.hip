// A plain streaming copy, the reference stream for the measurements: its
// duration gives the read+write rate the GPU sustains, and its hardware
// traffic counters calibrate those of the solver's kernels (a copy of B bytes
// moves exactly B bytes in and B bytes out of HBM when B is far above the
// 256 MB last-level cache).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "shellhom.h"

namespace {

// 16-byte vector loads and stores, four in flight per thread, grid-stride.
__global__ __launch_bounds__(256) void stream_copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                          uint64_t n16) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n16; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" int32_t shh_stream_copy(const void *d_src, void *d_dst, size_t bytes, void *hip_stream) {
  if (!d_src || !d_dst || bytes == 0 || bytes % 16 != 0 || ((uintptr_t)d_src | (uintptr_t)d_dst) % 16 != 0)
    return SHH_INVALID_ARG;
  const uint64_t n16 = bytes / 16;
  uint64_t blocks = (n16 + 255) / 256;
  if (blocks > 8192) blocks = 8192;  // 32 workgroups per CU, grid-stride beyond
  hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream,
                     (const uint4 *)d_src, (uint4 *)d_dst, n16);
  if (hipGetLastError() != hipSuccess) return SHH_HIP_ERROR;
  return SHH_OK;
}
