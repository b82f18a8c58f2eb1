// Structures shared by the host side of libpmp and its kernels (not part of
// the public ABI).
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
  uint64_t work;   // alpha * count + buf_bytes
};

// The work of a launch is the sum over batches of alpha * count + buf_bytes:
// string i of a batch starts at work position work0 + alpha * i + offsets[i]
// (a byte of buffer and a string each count as work). The work is cut into
// per_wave * total_waves shares of `share` units; wave w takes shares w,
// w + total_waves, w + 2 total_waves, ...
struct KArgs {
  BatchArgs b[2];              // up to two batches travel in the arguments...
  const BatchArgs* batches;    // ...more come as a device array (else null)
  uint32_t nbatch;
  uint32_t alpha;        // per-string work in byte equivalents
  int32_t* status;       // device status word (STATUS_* bits)
  uint32_t total_waves;  // waves sharing the work
  uint32_t per_wave;     // shares per wave
  uint64_t total;        // work of all batches
  uint64_t share;        // work per share
};

// Incremental hashing of one string delivered in pieces (the streaming form
// of Algorithm 1: one open node per level, Sec. 4). Device-resident; all
// zero after creation and reset.
//   part[j] (j = 2..8): exact sum sum_i a_{j,i} z_i over the level-(j-1)
//     values z already produced for the open level-j node (b_j not added);
//     3 words (PM+32: lo, hi, 0; PM+64: w0, w1, w2), the fourth unused.
//   carry: the bytes of the open level-1 block (fewer than 128 W).
struct IncrState {
  uint64_t part[9][4];
  uint32_t carry[(1024 + 16) / 4];
};

// One append that completes at least one level-1 block. The piece's bytes
// follow the t carried bytes; blocks s1 .. s1 + k - 1 (numbered from the
// string's start) are completed by it; r_new bytes are carried afterwards.
// Workgroup w of the first launch takes segment s1 / 32 + w (32 blocks, a
// quarter of a level-2 node). Per level-2 node touched (numbered from node
// s1 / 128): an accumulator Slot for its segments (0 between launches).
constexpr int INCR_SEG = 32;
struct IncrArgs {
  const uint8_t* piece;
  int64_t n;
  uint64_t s1;
  uint64_t k;
  uint32_t t;
  uint32_t r_new;
  uint32_t nwg;
  uint32_t pad_;
  const void* keys;
  IncrState* st;
  uint4* za;        // level outputs, ping-pong: each `cap` entries
  uint4* zb;
  Slot* slots;      // per node touched
  uint64_t* sums;   // sums of the first and last level-2 nodes, when open (2 x 4 words)
};

// host side (pmp_api.cpp)
int set_error(int code, const char* msg);  // sets the message pmp_last_error returns
int run_batches(pmp_plan* plan, const pmp_batch* const* in, int n_in, hipStream_t stream);

// kernels/launchers (pmp_kernels.hip)
hipError_t launch_batch(const KArgs& a, int grid, int g32, int g64, hipStream_t s);
int batch_blocks_per_cu(int g32, int g64);       // resident 256-thread blocks per CU
bool batch_tiles_supported(int g32, int g64);    // compiled lanes-per-block pairs
int batch_tile_pairs(int (*pairs)[2], int max);  // list them; returns how many
hipError_t launch_plain_string(int wide, const uint8_t* buf, uint64_t buf_bytes, int64_t o0, int64_t len,
                               const void* keys, void* out, int64_t index, uint32_t flags, uint4* scratch,
                               uint64_t scratch_slots, hipStream_t s);
hipError_t launch_incr_append(int wide, const IncrArgs& a, hipStream_t s);
hipError_t launch_incr_carry(IncrState* st, uint32_t t, const uint8_t* piece, int64_t n, hipStream_t s);
hipError_t launch_incr_digest(int wide, const IncrState* st, uint32_t t, const uint64_t* nodes, const void* keys,
                              void* out, uint32_t flags, hipStream_t s);
hipError_t launch_incr_reset(IncrState* st, hipStream_t s);
// exclusive scan of m uint32 counts into start[0..m] (start[m] = total);
// bsum: excl_scan_work_bytes(m) bytes of device scratch
uint64_t excl_scan_work_bytes(uint64_t m);
hipError_t launch_excl_scan_u32(const uint32_t* cnt, uint64_t m, int64_t* start, uint64_t* bsum, hipStream_t s);
uint64_t table_work_bytes(uint64_t m);
hipError_t launch_table_build(const void* h, uint32_t wide, int64_t n, uint64_t m, int64_t* start, int64_t* entries,
                              void* work, hipStream_t s);
hipError_t launch_table_probe(const uint8_t* qbuf, const int64_t* qoff, int64_t nq, const void* qh, const uint8_t* kbuf,
                              const int64_t* koff, const void* kh, uint32_t wide, uint64_t m, const int64_t* start,
                              const int64_t* entries, int64_t* result, hipStream_t s);
uint64_t pm128_scratch_bytes(int64_t count, uint64_t buf_bytes);
hipError_t launch_pm128(const uint8_t* buf, uint64_t buf_bytes, const int64_t* offsets, int64_t count,
                        const uint64_t* keys, void* out, uint32_t flags, void* scratch, hipStream_t s);
hipError_t launch_debug_fold(int wide, const void* w0, const void* w1, const uint32_t* w2, void* z, int64_t n,
                             hipStream_t s);

}  // namespace pmp
