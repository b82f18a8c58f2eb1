// Hash table of variable-length keys on PM+ outputs (the use that motivates
// the paper, Sec. 1 and Sec. 3: the bucket of key i is h_i mod M, which keeps
// the family almost universal and regular by Lemma 1 and Lemma 8).
//
// Build (after the keys are hashed by the batch kernel): count the keys of
// each bucket with atomics, an exclusive scan of the counts gives the CSR
// bucket starts, and a scatter with per-bucket atomic cursors places each
// key's record in its bucket. The order inside a bucket is whatever the
// atomics give; the probe does not depend on it.
//
// Each entry is a 32-byte record (key index, hash, offset, length), so that
// a probe reads one record per candidate.
//
// Probe (after the queries are hashed): one lane per query walks its bucket
// for the smallest key with the query's full n-bit hash and length, then
// compares that key's bytes, 64 at a time from 16-byte loads; only when a
// full-hash collision has different bytes does the lane go on to the next
// such key. The result is the smallest equal key index, or -1.
#include "pmp_device.hpp"
#include "pmp_internal.h"

namespace pmp {

namespace {

constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = 256 * SCAN_ITEMS;  // counts per scan workgroup

__device__ __forceinline__ uint64_t hash_at(const void* h, uint32_t wide, int64_t i) {
  return wide ? ((const uint64_t*)h)[i] : (uint64_t)((const uint32_t*)h)[i];
}

__global__ void tab_zero(uint32_t* a, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    a[i] = 0;
}

__global__ void tab_count(const void* h, uint32_t wide, int64_t n, uint64_t m, uint32_t* cnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(cnt + hash_at(h, wide, i) % m, 1u);
}

// exclusive scan of the 256 thread values of a workgroup; *total gets the sum
__device__ uint64_t block_excl_scan(uint64_t v, uint64_t* total) {
  __shared__ uint64_t ws[4];
  const int lane = (int)(threadIdx.x & 63u), wave = (int)(threadIdx.x >> 6);
  uint64_t x = v;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)x, d, 64);
    const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(x >> 32), d, 64);
    if (lane >= d) x += ((uint64_t)hi << 32) | lo;
  }
  if (lane == 63) ws[wave] = x;
  __syncthreads();
  uint64_t before = 0, all = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < wave) before += ws[w];
    all += ws[w];
  }
  __syncthreads();  // ws may be reused by the next call
  *total = all;
  return before + x - v;
}

// Phase 1: each workgroup scans SCAN_TILE counts into start[] (relative to
// its tile) and leaves the tile's total in bsum[].
__global__ void tab_scan_tiles(const uint32_t* cnt, uint64_t m, int64_t* start, uint64_t* bsum) {
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  uint64_t s = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = base + k < m ? cnt[base + k] : 0u;
    s += v[k];
  }
  uint64_t total;
  uint64_t run = block_excl_scan(s, &total);
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < m) start[base + k] = (int64_t)run;
    run += v[k];
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Phase 2 (one workgroup): exclusive scan of the tile totals, in place;
// start[m] = the number of keys.
__global__ void tab_scan_totals(uint64_t* bsum, uint64_t nb, int64_t* start, uint64_t m) {
  uint64_t carry = 0;
  for (uint64_t b0 = 0; b0 < nb; b0 += 256) {
    const uint64_t i = b0 + threadIdx.x;
    const uint64_t v = i < nb ? bsum[i] : 0;
    uint64_t total;
    const uint64_t x = block_excl_scan(v, &total);
    if (i < nb) bsum[i] = carry + x;
    carry += total;
  }
  if (threadIdx.x == 0) start[m] = (int64_t)carry;
}

// Phase 3: add each tile's offset; with `clear`, the counts are set back to
// zero on the way (the scatter's cursors), which saves a launch.
__global__ void tab_scan_add(int64_t* start, uint64_t m, const uint64_t* bsum, uint32_t* clear) {
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
  const int64_t add = (int64_t)bsum[blockIdx.x];
  for (int k = threadIdx.x; k < SCAN_TILE; k += 256)
    if (base + k < m) {
      start[base + k] += add;
      if (clear) clear[base + k] = 0;
    }
}

// Each key's record (index, hash, offset, length) goes to its bucket: a
// probe then reads one 32-byte record per candidate instead of the entry,
// the key's hash and its offsets from three places.
__global__ void tab_scatter(const void* h, uint32_t wide, int64_t n, uint64_t m, const int64_t* koff,
                            const int64_t* start, uint32_t* fill, pmp_table_entry* entries) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t hi = hash_at(h, wide, i);
    const int64_t o0 = koff[i], o1 = koff[i + 1];
    const uint64_t b = hi % m;
    pmp_table_entry r;
    r.key = i;
    r.hash = hi;
    r.offset = o0;
    r.length = o1 - o0;
    entries[start[b] + atomicAdd(fill + b, 1u)] = r;
  }
}

__device__ __forceinline__ const uint32_t* gdw(uint64_t a) {
  return (const uint32_t*)(const __attribute__((address_space(1))) uint32_t*)(uintptr_t)a;
}

// Records read per round of the bucket walk, and bytes compared per round:
// a wave waits for its slowest lane, so each round issues all of its loads
// before it uses any. At load factor 1 a bucket rarely holds more than a few
// keys; wider compare steps cost registers (occupancy) for fewer rounds.
constexpr int RECS = 2;
constexpr int STEP = 64;

// Bytes [o, o + STEP) of a string at p as STEP / 4 little-endian dwords
// (r = bytes of the string left from o, r > 0; dwords past its end hold
// anything). The 16-byte chunks of the aligned region around those bytes are
// loaded, every chunk that holds a byte of the string from its own address
// (such a chunk lies in the string's memory page) and any other one from the
// first chunk's, so that no load is conditional; then the chunks are shifted
// down by the string's offset in its first chunk: whole dwords with two
// rounds of byte permutes, then bytes with alignbyte.
__device__ __forceinline__ void load_step(const uint8_t* p, int64_t o, int64_t r, uint32_t* x) {
  constexpr int NC = STEP / 16 + 1;  // chunks that can hold the bytes
  const uint64_t a = (uint64_t)(uintptr_t)p + (uint64_t)o;
  const uint32_t lead = (uint32_t)(a & 15u);
  const uint64_t base = a - lead;
  const uint32_t lim = lead + (uint32_t)(r < STEP ? r : STEP);  // chunk c holds a wanted byte iff 16c < lim
  uint32_t d[4 * NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const uint4 q = *(const uint4*)gdw(16u * c < lim ? base + 16u * c : base);
    d[4 * c] = q.x;
    d[4 * c + 1] = q.y;
    d[4 * c + 2] = q.z;
    d[4 * c + 3] = q.w;
  }
  // v_perm_b32 picks bytes 4..7 (its first operand) or 0..3 (its second):
  // written as selects, the shifts would become an indexed copy in scratch
  const uint32_t s2 = (lead & 8u) ? 0x07060504u : 0x03020100u;
  const uint32_t s1 = (lead & 4u) ? 0x07060504u : 0x03020100u;
#pragma unroll
  for (int k = 0; k + 2 < 4 * NC; ++k) d[k] = __builtin_amdgcn_perm(d[k + 2], d[k], s2);
#pragma unroll
  for (int k = 0; k + 1 < 4 * NC; ++k) d[k] = __builtin_amdgcn_perm(d[k + 1], d[k], s1);
#pragma unroll
  for (int k = 0; k < STEP / 4; ++k) x[k] = __builtin_amdgcn_alignbyte(d[k + 1], d[k], lead & 3u);
}

// STEP bytes per round, both strings' loads issued before the comparison;
// the differences are masked to the bytes of the strings
__device__ __forceinline__ bool bytes_equal(const uint8_t* a, const uint8_t* b, int64_t len) {
  for (int64_t o = 0; o < len; o += STEP) {
    const int64_t r = len - o;
    uint32_t xa[STEP / 4], xb[STEP / 4];
    load_step(a, o, r, xa);
    load_step(b, o, r, xb);
    const uint32_t rr = (uint32_t)(r < STEP ? r : STEP);
    uint32_t diff = 0;
#pragma unroll
    for (int k = 0; k < STEP / 4; ++k) {
      const uint32_t v = xa[k] ^ xb[k];
      // bytes 4k .. 4k + 3 of the step that lie inside the string
      const uint32_t keep = 4u * k + 4 <= rr ? ~0u : (4u * k < rr ? (1u << (8 * (rr - 4u * k))) - 1u : 0u);
      diff |= v & keep;
    }
    if (diff) return false;
  }
  return true;
}

__global__ void __launch_bounds__(256)
    tab_probe(const uint8_t* qbuf, const int64_t* qoff, int64_t nq, const void* qh, const uint8_t* kbuf, uint32_t wide,
              uint64_t m, const int64_t* start, const pmp_table_entry* entries, int64_t* result) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q0 = qoff[q], len = qoff[q + 1] - q0;
    const uint64_t hq = hash_at(qh, wide, q);
    const uint64_t b = hq % m;
    const int64_t e0 = start[b], e1 = start[b + 1];
    // Candidates in increasing key order: the smallest key above `lo` with
    // the query's hash and length (every equal key has both), then its bytes.
    // The first candidate is nearly always the answer or there is none; a
    // full-hash collision with different bytes sends the lane round again.
    int64_t best = -1, lo = -1;
    for (;;) {
      int64_t cand = -1, coff = 0;
      for (int64_t e = e0; e < e1; e += RECS) {
        // records past the bucket's end are read from its first one, unused
        pmp_table_entry r[RECS];
#pragma unroll
        for (int u = 0; u < RECS; ++u) r[u] = entries[e + u < e1 ? e + u : e];
#pragma unroll
        for (int u = 0; u < RECS; ++u)
          if (e + u < e1 && r[u].hash == hq && r[u].length == len && r[u].key > lo && (cand < 0 || r[u].key < cand)) {
            cand = r[u].key;
            coff = r[u].offset;
          }
      }
      if (cand < 0) break;
      if (bytes_equal(qbuf + q0, kbuf + coff, len)) {
        best = cand;
        break;
      }
      lo = cand;
    }
    result[q] = best;
  }
}

unsigned grid_for(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

}  // namespace

uint64_t table_work_bytes(uint64_t m) {
  const uint64_t nb = (m + SCAN_TILE - 1) / SCAN_TILE;
  return ((4 * m + 7) & ~7ull) + 8 * (nb + 1);
}

uint64_t excl_scan_work_bytes(uint64_t m) { return 8 * ((m + SCAN_TILE - 1) / SCAN_TILE + 1); }

// Exclusive scan of m counts into start[0..m] (start[m] = the total); with
// `clear`, the counts (at `clear`, the same array as cnt) are zeroed after
// they are read.
static hipError_t excl_scan(const uint32_t* cnt, uint64_t m, int64_t* start, uint64_t* bsum, uint32_t* clear,
                            hipStream_t s) {
  const uint64_t nb = (m + SCAN_TILE - 1) / SCAN_TILE;
  if (nb) hipLaunchKernelGGL(tab_scan_tiles, dim3((unsigned)nb), dim3(256), 0, s, cnt, m, start, bsum);
  hipLaunchKernelGGL(tab_scan_totals, dim3(1), dim3(256), 0, s, bsum, nb, start, m);
  if (nb) hipLaunchKernelGGL(tab_scan_add, dim3((unsigned)nb), dim3(256), 0, s, start, m, bsum, clear);
  return hipGetLastError();
}

hipError_t launch_excl_scan_u32(const uint32_t* cnt, uint64_t m, int64_t* start, uint64_t* bsum, hipStream_t s) {
  return excl_scan(cnt, m, start, bsum, nullptr, s);
}

hipError_t launch_table_build(const void* h, uint32_t wide, int64_t n, uint64_t m, const int64_t* koff,
                              int64_t* start, pmp_table_entry* entries, void* work, hipStream_t s) {
  uint32_t* cnt = (uint32_t*)work;
  uint64_t* bsum = (uint64_t*)((char*)work + ((4 * m + 7) & ~7ull));
  hipLaunchKernelGGL(tab_zero, dim3(grid_for((int64_t)m)), dim3(256), 0, s, cnt, m);
  if (n > 0) hipLaunchKernelGGL(tab_count, dim3(grid_for(n)), dim3(256), 0, s, h, wide, n, m, cnt);
  // the scan zeroes the counts for the scatter's cursors
  hipError_t e = excl_scan(cnt, m, start, bsum, n > 0 ? cnt : nullptr, s);
  if (e != hipSuccess) return e;
  if (n > 0)
    hipLaunchKernelGGL(tab_scatter, dim3(grid_for(n)), dim3(256), 0, s, h, wide, n, m, koff, start, cnt, entries);
  return hipGetLastError();
}

hipError_t launch_table_probe(const uint8_t* qbuf, const int64_t* qoff, int64_t nq, const void* qh, const uint8_t* kbuf,
                              uint32_t wide, uint64_t m, const int64_t* start, const pmp_table_entry* entries,
                              int64_t* result, hipStream_t s) {
  if (nq > 0)
    hipLaunchKernelGGL(tab_probe, dim3(grid_for(nq)), dim3(256), 0, s, qbuf, qoff, nq, qh, kbuf, wide, m, start,
                       entries, result);
  return hipGetLastError();
}

}  // namespace pmp
