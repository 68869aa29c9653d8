// hpm_probe.hip -- a device-memory read probe for the benchmark (not part of
// the matcher): the rate at which one kernel can stream a buffer from HBM,
// the ceiling the arc scan is compared against.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Every block streams a contiguous range of 16-byte words with non-temporal
// loads, four in flight per thread and step, and folds them with XOR; the
// block's XOR goes to sink[block] so that no load is dead.
__global__ __launch_bounds__(256) void k_read_probe(const v4u* __restrict__ buf, uint64_t words,
                                                    uint32_t* __restrict__ sink) {
  const uint64_t per = (words + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * per;
  const uint64_t b1 = b0 + per < words ? b0 + per : words;
  v4u acc = {0u, 0u, 0u, 0u};
  uint64_t i = b0 + threadIdx.x;
  for (; i + 3 * 256 < b1; i += 4 * 256) {
    const v4u a = __builtin_nontemporal_load(buf + i);
    const v4u b = __builtin_nontemporal_load(buf + i + 256);
    const v4u c = __builtin_nontemporal_load(buf + i + 512);
    const v4u d = __builtin_nontemporal_load(buf + i + 768);
    acc ^= a ^ b ^ c ^ d;
  }
  for (; i < b1; i += 256) acc ^= __builtin_nontemporal_load(buf + i);
  uint32_t x = acc.x ^ acc.y ^ acc.z ^ acc.w;
  for (int o = 32; o > 0; o >>= 1) x ^= __shfl_xor(x, o);
  __shared__ uint32_t s[4];
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) sink[blockIdx.x] = s[0] ^ s[1] ^ s[2] ^ s[3];
}

}  // namespace

extern "C" {

// Streams `bytes` (a multiple of 16) from device buffer `buf` with `blocks`
// blocks of 256 threads on `stream` (a hipStream_t); sink: device uint32[blocks].
// Returns a hipError_t value (0 on success).
int hpm_probe_read(const void* buf, uint64_t bytes, int32_t blocks, void* stream,
                   uint32_t* sink) {
  if (!buf || !sink || blocks <= 0 || bytes % 16) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_read_probe, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                     (const v4u*)buf, bytes / 16, sink);
  return (int)hipGetLastError();
}

}  // extern "C"
