// Wave-level helpers shared by the batch kernels (gfx950, wave64): uniform
// values, DPP prefix scans, counter waits, and the staging of a tile's short
// strings in LDS.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pmp {

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}
__device__ __forceinline__ int64_t uni64s(int64_t v) { return (int64_t)uni64((uint64_t)v); }
// lane l's value of v (l uniform)
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  return uni64(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l)) |
               ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l) << 32));
}

// Inclusive prefix over the wave with DPP moves only (no LDS): steps of
// 1, 2, 4 and 8 lanes within each row of 16, then the last lane of row 0
// into row 1 and of row 2 into row 3 (row_bcast:15), then the last lane of
// row 1 into rows 2 and 3 (row_bcast:31). OP: 0 sum, 1 max.
template <int OP>
__device__ __forceinline__ uint32_t wave_incl(uint32_t v) {
  auto op = [](uint32_t a, uint32_t b) { return OP == 0 ? a + b : (a > b ? a : b); };
  uint32_t x = v;
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true));  // row_shr:1
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true));  // row_shr:2
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true));  // row_shr:4
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true));  // row_shr:8
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false));  // row_bcast:15
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return x;
}
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl<1>(v), 63);
}
// exclusive prefix sum over the wave of values whose total stays below
// 2^32; *total receives the sum (uniform)
__device__ __forceinline__ uint64_t wave_excl_scan(uint64_t v, uint64_t* total) {
  const uint32_t x = wave_incl<0>((uint32_t)v);
  *total = (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
  return x - (uint32_t)v;
}

// s_waitcnt through the builtin, so that the compiler's own wait insertion
// knows that every outstanding load (direct-to-LDS ones included) is done.
// gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8.
__device__ __forceinline__ void wait_vm0() { __builtin_amdgcn_s_waitcnt(0x0F70); }
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}
__device__ __forceinline__ void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(0xC07F); }
// A per-lane address in global memory as a pointer the compiler knows to be
// global: loads through it are global loads (counted by vmcnt alone), not
// flat ones, whose waits would also drain every outstanding flat load
// whenever the LDS is read.
__device__ __forceinline__ const uint8_t* gaddr(uint64_t a) {
  return (const uint8_t*)(const __attribute__((address_space(1))) uint8_t*)(uintptr_t)a;
}

// Software pipelining over `steps` steps with D buffers: the loads of step
// n + D - 1 are issued (fill) before step n is used, so that D - 1 steps are
// in flight while one is computed. The buffers are used in turn by a loop
// unrolled D times, so that none is ever copied (a copy costs a move per
// register and waits for its loads). fill may be called for steps past the
// last; it must then read harmless memory.
template <int D, typename Buf, typename Fill, typename Use>
__device__ __forceinline__ void pipelined(uint32_t steps, Fill fill, Use use) {
  Buf b[D];
#pragma unroll
  for (int q = 0; q + 1 < D; ++q) fill(b[q], (uint32_t)q);
  for (uint32_t st = 0; st < steps; st += D) {
#pragma unroll
    for (int q = 0; q < D; ++q) {
      fill(b[(q + D - 1) % D], st + (uint32_t)(q + D - 1));
      use(b[q], st + (uint32_t)q);
      if (st + (uint32_t)q + 1 >= steps) return;
    }
  }
}

// ---------------------------------------------------------------------------
// Short strings of a tile, one per lane, staged in LDS.
//
// Per-lane loads of 64 unrelated strings are slow (64 cache lines per load
// instruction, and few in flight per lane), so the wave first copies the
// 16-byte chunks that hold its strings into its LDS stage with direct-to-LDS
// loads. The strings of a tile lie back to back in the buffer: when the
// chunks from the first one's to the last one's fit in the stage, they are
// copied as one run (64 consecutive chunks per load). Otherwise each lane
// reserves a slot per chunk of its string, in lane order, and writes the
// numbers of its chunks, relative to the first string's chunk, into a slot
// table; load instruction k then fills slots 64k .. 64k + 63, and since
// consecutive slots mostly belong to one string those loads are coalesced
// too. Lanes that do not fit go in a further pass.
constexpr uint32_t STAGE_CHUNKS = 768;             // 12 KiB of string bytes per wave
constexpr uint32_t STAGE_BYTES = 16 * STAGE_CHUNKS;
constexpr uint32_t STAGE_SLACK = 512;              // reads past a lane's chunks stay in the wave's region

// Stages the strings of the lanes in `act` (ulen bytes at buf + o0; at most
// STAGE_BYTES - 15 bytes each, so that any one string fits the stage) and
// calls hash(in, p0, sh) once per pass, right after
// the pass's loads are issued: a lane in `in` finds its string from byte
// p0 + sh of `stage` on (p0 4-aligned, sh = the string's start mod 4). hash
// must wait for the loads (wait_vm0) before it reads the stage; its reads
// may run up to STAGE_SLACK bytes past the stage. `table` holds
// STAGE_CHUNKS entries.
template <typename Hash>
__device__ __forceinline__ void stage_strings(const uint8_t* buf, bool act, int64_t o0, uint32_t ulen, uint8_t* stage,
                                              uint32_t* table, Hash&& hash) {
  uint64_t todo = __ballot(act);
  if (!todo) return;
  const int lane = lane_id();
  const uint8_t* s = buf + (act ? o0 : 0);
  const uint32_t lead = (uint32_t)((uintptr_t)s & 15u);
  const uint64_t a16 = (uint64_t)(uintptr_t)(s - lead);
  const uint32_t sh = lead & 3u;
  // chunks [a16, a16 + 16 nl) hold the string (none for an empty one: its
  // buffer may be empty)
  const uint32_t nl = act && ulen > 0 ? (lead + ulen + 15) / 16 : 0u;
  const auto* lds1 = (__attribute__((address_space(3))) uint8_t*)stage;
  {
    // one run of chunks, from the first string's to the end of the last one's
    const uint64_t tb = readlane64(a16, __ffsll((unsigned long long)todo) - 1);
    const uint64_t rend = act ? ((a16 - tb) >> 4) + nl : 0;  // (huge when a16 < tb)
    const uint32_t tp = wave_max(rend <= STAGE_CHUNKS ? (uint32_t)rend : STAGE_CHUNKS + 1);
    if (!__ballot(act && a16 < tb) && tp <= STAGE_CHUNKS) {
      wait_lgkm0();  // the stage's previous readers are done
      for (uint32_t k = 0; 64 * k < tp; ++k) {
        const uint32_t j = 64 * k + (uint32_t)lane;
        if (j < tp)
          __builtin_amdgcn_global_load_lds((const void*)(uintptr_t)(tb + 16ull * j),
                                           (__attribute__((address_space(3))) void*)(lds1 + 1024 * k), 16, 0, 0);
      }
      hash(act, act ? (uint32_t)(a16 - tb) + (lead & ~3u) : 0u, sh);
      return;
    }
  }
  uint64_t total = 0;
  const uint32_t c0 = (uint32_t)wave_excl_scan(nl, &total);
  uint32_t base = 0;  // first slot number of this pass
  while (todo) {
    const bool mine = (todo >> lane) & 1ull;
    // chunk numbers are kept relative to the pass's first string, in 32 bits
    const uint64_t tb = readlane64(a16, __ffsll((unsigned long long)todo) - 1);
    const uint64_t rel = (a16 - tb) >> 4;
    const bool fits = c0 + nl - base <= STAGE_CHUNKS && rel + nl < (1ull << 32);
    // the pass takes its lanes up to the first one that does not fit, so
    // that every slot below tp is written (the first lane always fits: its
    // chunks fit the stage and its rel is 0); offsets that decrease
    // somewhere can leave a later string in front of the first one
    const uint64_t stop = __ballot(mine && !fits);
    const bool in = mine && fits && (stop == 0 || lane < __ffsll((unsigned long long)stop) - 1);
    const uint64_t pm = __ballot(in);
    const uint32_t tp = wave_max(in ? c0 + nl - base : 0u);  // slots used by this pass
    wait_lgkm0();  // the previous pass is done reading the stage
    // (also written with inline asm, so that the compiler does not wait for
    // the previous tile's output stores before each entry)
    if (in) {
      const uint32_t ta = lds_addr(table) + 4 * (c0 - base);
      // two entries per write
      for (uint32_t t = 0; t + 1 < nl; t += 2)
        asm volatile("ds_write2_b32 %0, %1, %2 offset1:1" ::"v"(ta + 4 * t), "v"((uint32_t)rel + t),
                     "v"((uint32_t)rel + t + 1)
                     : "memory");
      if (nl & 1u) asm volatile("ds_write_b32 %0, %1" ::"v"(ta + 4 * (nl - 1)), "v"((uint32_t)rel + nl - 1) : "memory");
    }
    // Four table entries per read: the table is read with inline asm (its
    // wait included) because the compiler would otherwise wait for every
    // outstanding direct-to-LDS load before each LDS read.
    for (uint32_t k0 = 0; k0 * 64 < tp; k0 += 4) {
      const uint32_t ta = lds_addr(table) + 4 * (k0 * 64 + (uint32_t)lane);
      uint32_t e[4];
      asm volatile(
          "ds_read_b32 %0, %4\n\tds_read_b32 %1, %4 offset:256\n\tds_read_b32 %2, %4 offset:512\n\t"
          "ds_read_b32 %3, %4 offset:768\n\ts_waitcnt lgkmcnt(0)"
          : "=&v"(e[0]), "=&v"(e[1]), "=&v"(e[2]), "=&v"(e[3])
          : "v"(ta)
          : "memory");
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) {
        const uint32_t k = k0 + u;
        if (k * 64 >= tp) break;  // uniform
        const uint32_t j = k * 64 + (uint32_t)lane;
        if (j < tp)
          __builtin_amdgcn_global_load_lds((const void*)(uintptr_t)(tb + 16ull * e[u]),
                                           (__attribute__((address_space(3))) void*)(lds1 + 1024 * k), 16, 0, 0);
      }
    }
    hash(in, in ? 16 * (c0 - base) + (lead & ~3u) : 0u, sh);
    todo &= ~pm;
    base += tp;
  }
}

}  // namespace pmp
