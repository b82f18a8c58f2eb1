// pmp_hash_mixed_noalloc: the batch launch of pmp_hash_mixed for callers that
// cannot allocate device memory (code under stream capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// The batch kernel's node accumulators (16 bytes per 128-word block of
// buffer, for strings of more than one level-2 node) live in a file-scope
// device array of fixed size instead of a plan's workspace. Each device that
// runs the call holds its own copy of the array until the process ends; its
// device address is looked up once per device with hipGetSymbolAddress
// (the array's name in host code is only a stand-in for the symbol). A call
// first clears the accumulators it will use and the caller's status word
// with a fill kernel (no hipMemsetAsync, so the call may be captured), then
// launches the batch kernel on them. Calls that overlap on one device share
// the array and race; calls on one stream are ordered.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pmp.h"
#include "pmp_batch.h"
#include "pmp_internal.h"

namespace {

constexpr uint64_t SCRATCH_BYTES = PMP_NOALLOC_SCRATCH_BYTES;
static_assert(SCRATCH_BYTES % sizeof(pmp::Slot) == 0, "whole accumulators");

static __device__ __align__(256) uint8_t scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
struct DeviceScratch {
  bool ready = false;
  pmp::Slot* slots = nullptr;  // the device address of `scratch` on that device
  int cus = 0;
};
std::mutex g_mu;
DeviceScratch g_dev[MAX_DEVICES];

// Zero n 16-byte accumulators and the status word.
__global__ void clear_scratch(uint4* p, uint64_t n, int32_t* status) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x == 0) *status = 0;
}

// The current device's scratch address and CU count, looked up on the
// device's first call.
int device_scratch(DeviceScratch* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return pmp::set_error(PMP_E_HIP, "hipGetDevice failed");
  if (dev < 0 || dev >= MAX_DEVICES) return pmp::set_error(PMP_E_INVALID_ARG, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceScratch& d = g_dev[dev];
  if (!d.ready) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return pmp::set_error(PMP_E_HIP, "hipGetSymbolAddress of the static scratch failed");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return pmp::set_error(PMP_E_HIP, "hipGetDeviceProperties failed");
    d.slots = (pmp::Slot*)ptr;
    d.cus = prop.multiProcessorCount;
    d.ready = true;
  }
  *out = d;
  return PMP_OK;
}

uint64_t slots_needed(const pmp_batch* b) {
  if (!b || b->count <= 0) return 0;
  const uint64_t blk = b->wide ? 1024 : 512;  // 128 words of 8 or 4 bytes
  return (b->buf_bytes + blk - 1) / blk + 2;
}

}  // namespace

extern "C" int pmp_hash_mixed_noalloc(const pmp_batch* b0, const pmp_batch* b1, int32_t* d_status,
                                      pmp_stream_t stream) {
  if (!d_status) return pmp::set_error(PMP_E_INVALID_ARG, "d_status is NULL");
  const uint64_t cap = SCRATCH_BYTES / sizeof(pmp::Slot);
  const uint64_t need = slots_needed(b0) + slots_needed(b1);
  if (need > cap)
    return pmp::set_error(PMP_E_NOMEM, "the batches need more node accumulators than the static scratch "
                                       "holds (16 bytes per 128-word block of buffer)");
  DeviceScratch d;
  int r = device_scratch(&d);
  if (r) return r;
  hipStream_t s = (hipStream_t)stream;
  const uint64_t n = need ? need : 1;
  int grid = (int)((n + 255) / 256);
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(clear_scratch, dim3(grid), dim3(256), 0, s, (uint4*)d.slots, need, d_status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return pmp::set_error(PMP_E_HIP, "scratch clear launch failed");
  const pmp_batch* l[2] = {b0, b1};
  return pmp::run_static(l, 2, d.slots, cap, d_status, d.cus, s);
}
