// Structures of the batch kernel shared with the host side of libpmp (not
// part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pmp.h"

namespace pmp {

constexpr uint32_t FLAG_NO_MIX = 1u;
constexpr uint32_t FLAG_OUT_FIELD = 2u;

constexpr int32_t STATUS_OFFSETS = 1;   // an offsets pair was out of order or out of range
constexpr int32_t STATUS_INTERNAL = 2;  // a node accumulator fell outside the workspace

// Accumulator of one tree node (level >= 2), all zero between launches.
// PM+32: w0 = (weight received << 56) | sum of field elements (< 2^40).
// PM+64: w0 = low 64 bits of the sum, w1 = (weight << 32) | high bits.
struct Slot {
  uint64_t w0;
  uint64_t w1;
};

// One batch as the kernel sees it.
struct BatchArgs {
  const uint8_t* buf;
  uint64_t buf_bytes;
  const int64_t* offsets;
  int64_t count;
  const void* keys;  // uint32[1032] (PM+32) or uint64[1032] (PM+64)
  void* out;
  uint32_t flags;
  uint32_t wide;
  Slot* slots;  // ceil(buf_bytes / (128 W)) + 2 node accumulators
  uint64_t nslots;
  uint64_t work0;  // work of the batches before this one
  uint64_t work;   // alpha * count + buf_bytes (count when split by count)
};

// The work of a launch is the sum over batches of alpha * count + buf_bytes:
// string i of a batch starts at work position work0 + alpha * i + offsets[i]
// (a byte of buffer and a string each count as work). With alpha =
// PMP_ALPHA_BY_COUNT a string is one unit of work whatever its length, and
// string i starts at work0 + i. The work is cut into
// per_wave * total_waves shares of `share` units; wave w takes shares w,
// w + total_waves, w + 2 total_waves, ...
struct KArgs {
  BatchArgs b[2];              // up to two batches travel in the arguments...
  const BatchArgs* batches;    // ...more come as a device array (else null)
  uint32_t nbatch;
  uint32_t alpha;        // per-string work in byte equivalents (PMP_ALPHA_BY_COUNT: strings only)
  int32_t* status;       // device status word (STATUS_* bits)
  uint32_t total_waves;  // waves sharing the work
  uint32_t per_wave;     // shares per wave
  uint64_t total;        // work of all batches
  uint64_t share;        // work per share
};

}  // namespace pmp
