// Structures shared by the host side of libpmp and its kernels (not part of
// the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pmp.h"
#include "pmp_batch.h"
#include "pmp_incr.h"

namespace pmp {

// host side (pmp_api.cpp)
int set_error(int code, const char* msg);  // sets the message pmp_last_error returns
int run_batches(pmp_plan* plan, const pmp_batch* const* in, int n_in, hipStream_t stream);
// at most two batches, on caller-given node accumulators and status word, no allocation
int run_static(const pmp_batch* const* in, int n_in, Slot* slots, uint64_t nslots, int32_t* status, int cus,
               hipStream_t stream);
// a plan's device status word, and a clear of it and of the plan's node
// accumulators ordered on `stream` (after a launch that flagged an error)
int32_t* plan_status_word(pmp_plan* plan);
int plan_clear_async(pmp_plan* plan, hipStream_t stream);

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
hipError_t launch_incr_flush(int wide, IncrState* st, const void* keys, const IncrTree& t, hipStream_t s);
hipError_t launch_incr_digest(int wide, IncrState* st, uint32_t t, const uint64_t* nodes, const void* keys,
                              void* out, uint32_t flags, uint32_t pending, const IncrTree& prev, hipStream_t s);
hipError_t launch_incr_reset(IncrState* st, hipStream_t s);
// exclusive scan of m uint32 counts into start[0..m] (start[m] = total);
// bsum: excl_scan_work_bytes(m) bytes of device scratch
uint64_t excl_scan_work_bytes(uint64_t m);
hipError_t launch_excl_scan_u32(const uint32_t* cnt, uint64_t m, int64_t* start, uint64_t* bsum, hipStream_t s);
uint64_t table_work_bytes(uint64_t m);
hipError_t launch_table_build(const void* h, uint32_t wide, int64_t n, uint64_t m, const int64_t* koff,
                              int64_t* start, pmp_table_entry* entries, void* work, hipStream_t s);
hipError_t launch_table_probe(const uint8_t* qbuf, const int64_t* qoff, int64_t nq, const void* qh, const uint8_t* kbuf,
                              uint32_t wide, uint64_t m, const int64_t* start, const pmp_table_entry* entries,
                              int64_t* result, hipStream_t s);
uint64_t pm128_scratch_bytes(int64_t count, uint64_t buf_bytes);
hipError_t launch_pm128(const uint8_t* buf, uint64_t buf_bytes, const int64_t* offsets, int64_t count,
                        const uint64_t* keys, void* out, uint32_t flags, void* scratch, hipStream_t s);
hipError_t launch_debug_fold(int wide, const void* w0, const void* w1, const uint32_t* w2, void* z, int64_t n,
                             hipStream_t s);

}  // namespace pmp
