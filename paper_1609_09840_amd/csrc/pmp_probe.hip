// Measurement hooks, not on the hashing path: the device's rate of
// v_mad_u64_u32, the 32x32->64 multiply-add that the level-1 sums of Eq. (1)
// are built from (Sec. 6), and the read bandwidth a plain streaming kernel
// reaches. The kernels are compared with these as their achievable
// rooflines, beside the published peaks.
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

// Workgroups take chunks of 2048 16-byte pieces (32 KiB) in turn: chunk c
// of workgroup w is w + c * gridDim; thread t reads pieces t, t + 256, ...,
// t + 1792 of it (eight in flight, each wave 1 KiB contiguous per load) and
// folds them into one word, stored per thread so that no load is optimised
// away.
__global__ __launch_bounds__(256) void read_probe(const uint4* p, uint64_t n, uint32_t* out) {
  constexpr uint64_t CH = 2048;
  uint32_t acc = 0;
  for (uint64_t c = blockIdx.x; c * CH < n; c += gridDim.x) {
    const uint64_t base = c * CH + threadIdx.x;
    if (c * CH + CH <= n) {
      uint4 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = p[base + 256 * u];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    } else {
      for (uint64_t i = base; i < n; i += 256) {
        const uint4 a = p[i];
        acc ^= a.x ^ a.y ^ a.z ^ a.w;
      }
    }
  }
  out[(uint64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// `blocks` blocks of 256 threads over n 16-byte pieces; out holds one word
// per thread
hipError_t launch_read_probe(const void* buf, uint64_t n16, uint32_t* out, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(read_probe, dim3(blocks), dim3(256), 0, s, (const uint4*)buf, n16, out);
  return hipGetLastError();
}

}  // namespace pmp
