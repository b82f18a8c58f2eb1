// Measurement hook, not on the hashing path: the device's rate of
// v_mad_u64_u32, the 32x32->64 multiply-add that the level-1 sums of Eq. (1)
// are built from (Sec. 6). The batch kernel is compared with this rate as its
// multiply roofline.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pmp {

// Every lane runs 8 independent chains of v_mad_u64_u32, `iters` rounds
// each; the sums are stored so that nothing is optimised away.
__global__ __launch_bounds__(256) void mad_probe(uint64_t* out, uint32_t iters, uint32_t seed) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t acc[8];
  uint32_t x[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    acc[u] = t + u;
    x[u] = seed * (t + 1u) + 0x9e3779b9u * (uint32_t)u;
  }
  for (uint32_t r = 0; r < iters; ++r) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      uint64_t c;
      asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc[u]), "=s"(c) : "v"(x[u]), "v"(x[(u + 1) & 7]));
    }
  }
  uint64_t s = 0;
#pragma unroll
  for (int u = 0; u < 8; ++u) s ^= acc[u];
  out[t] = s;
}

// `blocks` blocks of 256 threads; out holds one word per thread
hipError_t launch_mad_probe(uint64_t* out, int blocks, uint32_t iters, hipStream_t s) {
  hipLaunchKernelGGL(mad_probe, dim3(blocks), dim3(256), 0, s, out, iters, 0x2545f491u);
  return hipGetLastError();
}

}  // namespace pmp
