// Dependent random-gather probe: the load rate the sampling kernels' memory roofline is
// measured against.  Built as its own library (libmoss_probe.so); see moss_probe.h.
#include <hip/hip_runtime.h>

#include "moss_probe.h"

namespace {

__device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256) k_probe_fill(uint64_t* __restrict__ buf, uint64_t words, uint64_t seed) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
    buf[i] = splitmix64(seed + i);
}

// Lane t follows C chains side by side: chain c starts at a place given by (t, c) and
// each step loads x = buf[j_c] and moves to j_c = floor((x ^ salt_c) * words / 2^64), so a
// lane has C independent loads in flight and each of them depends on its chain's last.
template <int C>
__global__ void __launch_bounds__(256) k_probe_gather(const uint64_t* __restrict__ buf, uint64_t words,
                                                      uint32_t steps, uint64_t* __restrict__ out) {
  const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  uint64_t j[C], salt[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const uint64_t id = t * C + c;
    salt[c] = splitmix64(~id) | 1;
    j[c] = __umul64hi(splitmix64(id), words);  // < words
  }
  uint64_t acc = 0;
  for (uint32_t s = 0; s < steps; ++s) {
    uint64_t x[C];
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = buf[j[c]];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      acc += x[c];
      j[c] = __umul64hi(x[c] ^ salt[c], words);  // < words
    }
  }
  out[t] = acc;
}

}  // namespace

extern "C" int moss_probe_fill(uint64_t* buf, uint64_t words, uint64_t seed, void* stream) {
  if (!buf || words == 0) return -1;
  const uint64_t want = (words + 255) / 256;
  const uint32_t blocks = (uint32_t)(want < 8192 ? want : 8192);
  hipLaunchKernelGGL(k_probe_fill, dim3(blocks), dim3(256), 0, (hipStream_t)stream, buf, words, seed);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

extern "C" int moss_probe_gather(const uint64_t* buf, uint64_t words, uint32_t blocks, uint32_t steps,
                                 uint32_t chains, uint64_t* out, void* stream) {
  if (!buf || !out || words == 0 || blocks == 0 || blocks > (1u << 20) || steps == 0 || steps > (1u << 20))
    return -1;
  hipStream_t s = (hipStream_t)stream;
  switch (chains) {
    case 1: hipLaunchKernelGGL(k_probe_gather<1>, dim3(blocks), dim3(256), 0, s, buf, words, steps, out); break;
    case 2: hipLaunchKernelGGL(k_probe_gather<2>, dim3(blocks), dim3(256), 0, s, buf, words, steps, out); break;
    case 4: hipLaunchKernelGGL(k_probe_gather<4>, dim3(blocks), dim3(256), 0, s, buf, words, steps, out); break;
    case 8: hipLaunchKernelGGL(k_probe_gather<8>, dim3(blocks), dim3(256), 0, s, buf, words, steps, out); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}
