// Bandwidth probe beside the product library: a plain device copy, one
// 16-byte load and store per work item. The benchmark quotes the step
// kernel's HBM traffic against what this streaming copy reaches on the same
// device, and the byte counters are calibrated on it. Not part of libdugks.

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace {

__global__ __launch_bounds__(256) void k_copy16(const uint4* __restrict__ src,
                                                uint4* __restrict__ dst, long long n16) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n16) dst[i] = src[i];
}

}  // namespace

// Copy `bytes` (a positive multiple of 16) from device buffer src to device
// buffer dst (both 16-byte aligned, not overlapping) on `stream` (a
// hipStream_t; NULL = null stream), asynchronously. Returns 0, -1 for bad
// arguments, -3 if the launch fails.
extern "C" int copy_probe(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src || bytes == 0 || bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(dst) & 15) ||
      (reinterpret_cast<uintptr_t>(src) & 15))
    return -1;
  const char* a = static_cast<const char*>(src);
  const char* b = static_cast<const char*>(dst);
  if (a < b + bytes && b < a + bytes) return -1;
  const long long n16 = (long long)(bytes / 16);
  const long long blocks = (n16 + 255) / 256;
  if (blocks > 0x7fffffffLL) return -1;
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}
