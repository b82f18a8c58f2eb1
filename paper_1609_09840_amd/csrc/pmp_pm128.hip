// PM+128: the PM+ construction over p = 2^128 + 51 (the smallest prime above
// 2^128, Table "smallestprimes") with 128-bit words, for batches of ragged
// strings. The paper gives only the prime for n = 128; words, Eq. (1), the
// tree of Algorithm 1 and the output h mod 2^128 (Sec. 5) follow the PM+32 /
// PM+64 construction, with keys a in [1, 2^128 - 50] (kappa = 2 (k - 1) =
// 100) and no Sec. 7 mixer.
//
// Arithmetic: a 128 x 128 product is four 64 x 64 -> 128 products; a block
// sum (at most 128 products plus b, below 2^264) is kept exactly in five
// 64-bit limbs and reduced once per block with 2^128 = -51 (mod p):
//   S = s0 + 2^128 s1 + 2^256 s2 == s0 + 51 (2^128 - s1) + 2601 (1 + s2)
// (adding 51 p keeps every term non-negative), which is below 53 * 2^128;
// one more step v0 - 51 v1 (plus p when negative) lands in [0, p).
//
// Launches: (1) the number of units of each string of more than one block
// (a unit is a quarter of a level-2 node: 32 blocks) and an exclusive scan
// of those counts; (2) strings of one block, two lanes each; (3) one wave
// per unit, 8 lanes per block and 8 blocks at a time: each block's exact sum
// is reduced over its 8 lanes and folded, and the unit's share of its node,
// sum a_{2,i} z_i reduced mod p, is stored; (4) one wave
// per string of more than one block adds each node's units and b_2 and
// climbs the levels above 2 in place.
#include <atomic>

#include "pmp_device.hpp"
#include "pmp_internal.h"
#include "pmp_stage.hpp"

namespace pmp {

namespace {

constexpr uint64_t K128 = 51;
constexpr int W16 = 16;                      // bytes per word
constexpr uint64_t BLK_BYTES = BLOCK * W16;  // 2 KiB per level-1 block
constexpr int QB = 32;                       // blocks per unit: a quarter of a level-2 node
constexpr int UPN = BLOCK / QB;              // units per level-2 node

struct A5 {
  uint64_t w[5];
};
struct F128 {  // a field element lo + 2^64 hi + 2^128 top, below p
  uint64_t lo, hi;
  uint32_t top;
};

__device__ __forceinline__ void zero(A5& s) {
#pragma unroll
  for (int i = 0; i < 5; ++i) s.w[i] = 0;
}

// s += v * 2^(64 k), k <= 2
__device__ __forceinline__ void add_at(A5& s, u128 v, int k) {
  u128 t = (u128)s.w[k] + (uint64_t)v;
  s.w[k] = (uint64_t)t;
  t = (u128)s.w[k + 1] + (uint64_t)(v >> 64) + (uint64_t)(t >> 64);
  s.w[k + 1] = (uint64_t)t;
  uint64_t c = (uint64_t)(t >> 64);
  for (int i = k + 2; i < 5; ++i) {
    t = (u128)s.w[i] + c;
    s.w[i] = (uint64_t)t;
    c = (uint64_t)(t >> 64);
  }
}

__device__ __forceinline__ void add(A5& s, const A5& t) {
  uint64_t c = 0;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const u128 x = (u128)s.w[i] + t.w[i] + c;
    s.w[i] = (uint64_t)x;
    c = (uint64_t)(x >> 64);
  }
}

// s += a * x, a and x 128-bit
__device__ __forceinline__ void mac(A5& s, uint64_t a0, uint64_t a1, uint64_t x0, uint64_t x1) {
  add_at(s, (u128)a0 * x0, 0);
  add_at(s, (u128)a0 * x1, 1);
  add_at(s, (u128)a1 * x0, 1);
  add_at(s, (u128)a1 * x1, 2);
}

// s += a * z, z a field element
__device__ __forceinline__ void mac_fe(A5& s, uint64_t a0, uint64_t a1, const F128& z) {
  mac(s, a0, a1, z.lo, z.hi);
  if (z.top) add_at(s, (u128)a0 | ((u128)a1 << 64), 2);
}

// S mod p for S below 2^264 (see the header)
__device__ F128 fold(const A5& S) {
  const u128 s0 = (u128)S.w[0] | ((u128)S.w[1] << 64);
  const u128 s1 = (u128)S.w[2] | ((u128)S.w[3] << 64);
  const uint64_t s2 = S.w[4];
  // V = s0 + 51 (2^128 - s1) + 2601 (1 + s2) as v0 + 2^128 v1
  A5 V;
  zero(V);
  add_at(V, s0, 0);
  if (s1 == 0) {
    V.w[2] += K128;
  } else {
    const u128 m1 = (u128)0 - s1;  // 2^128 - s1
    add_at(V, (u128)(uint64_t)m1 * K128, 0);
    add_at(V, (u128)(uint64_t)(m1 >> 64) * K128, 1);
  }
  add_at(V, (u128)(K128 * K128) * (1 + s2), 0);
  const u128 v0 = (u128)V.w[0] | ((u128)V.w[1] << 64);
  const uint64_t v1 = V.w[2];  // at most 52
  F128 z;
  if (v0 >= (u128)(K128 * v1)) {
    const u128 r = v0 - K128 * v1;
    z.lo = (uint64_t)r;
    z.hi = (uint64_t)(r >> 64);
    z.top = 0;
  } else {
    // v0 < 51 v1 is small: r = v0 - 51 v1 + p = 2^128 + d
    const int64_t d = (int64_t)(uint64_t)v0 + (int64_t)K128 - (int64_t)(K128 * v1);
    if (d >= 0) {
      z.lo = (uint64_t)d;
      z.hi = 0;
      z.top = 1;
    } else {
      const u128 r = (u128)0 - (u128)(uint64_t)(-d);
      z.lo = (uint64_t)r;
      z.hi = (uint64_t)(r >> 64);
      z.top = 0;
    }
  }
  return z;
}


__device__ __forceinline__ const uint8_t* gp16(uint64_t a) {
  return (const uint8_t*)(const __attribute__((address_space(1))) uint8_t*)(uintptr_t)a;
}

__device__ __forceinline__ uint64_t shx64(uint64_t v, int m) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ void wave_sum(A5& s) {
  for (int m = 1; m < 64; m <<= 1) {
    A5 t;
#pragma unroll
    for (int i = 0; i < 5; ++i) t.w[i] = shx64(s.w[i], m);
    add(s, t);
  }
}

// key i of level j (1-based) and b_j: entries of two uint64 (lo, hi)
__device__ __forceinline__ void key_a(const uint64_t* keys, int j, uint32_t i, uint64_t* a0, uint64_t* a1) {
  const uint64_t* k = keys + 2 * ((uint64_t)(j - 1) * BLOCK + i);
  *a0 = k[0];
  *a1 = k[1];
}
__device__ __forceinline__ void add_b(A5& s, const uint64_t* keys, int j) {
  const uint64_t* k = keys + 2 * (LMAX * BLOCK + (j - 1));
  add_at(s, (u128)k[0] | ((u128)k[1] << 64), 0);
}

// word w of a string (start s, len bytes), padded (end of Sec. 4), as two
// 64-bit halves; reads stay inside [lo, hi)
__device__ __forceinline__ void word128(const uint8_t* s, int64_t len, int64_t w, const uint8_t* lo, const uint8_t* hi,
                                        uint64_t* x0, uint64_t* x1) {
  const int64_t r = len - W16 * w;
  uint32_t x[4] = {0, 0, 0, 0};
  if (r >= 0) {
    const uint8_t* p = s + W16 * w;
    const uint32_t sh = (uint32_t)((uintptr_t)p & 3u);
    const uint8_t* a4 = p - sh;
    const Q q = load16_guarded(a4, lo, hi);
    const uint32_t d4 = sh ? load4_guarded(a4 + 16, lo, hi) : 0u;
    const uint32_t d[5] = {q.d[0], q.d[1], q.d[2], q.d[3], d4};
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = tail_word32(align_bytes(d[u + 1], d[u], sh), r - 4 * u);
  }
  *x0 = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
  *x1 = (uint64_t)x[2] | ((uint64_t)x[3] << 32);
}

__device__ __forceinline__ int64_t blocks_of(int64_t len) { return (len / W16 + 1 + BLOCK - 1) / BLOCK; }
// units of the node kernel: parts of level-2 nodes (QB blocks); strings
// of one block have none (the short-string kernel takes them)
__device__ __forceinline__ int64_t units_of(int64_t len) {
  const int64_t n1 = blocks_of(len);
  return n1 == 1 ? 0 : (n1 + QB - 1) / QB;
}

__device__ __forceinline__ int64_t str_len(const int64_t* off, int64_t i, uint64_t buf_bytes) {
  const int64_t o0 = off[i], o1 = off[i + 1];
  // offsets out of order or past the buffer: the string is taken as empty
  return (o0 < 0 || o1 < o0 || (uint64_t)o1 > buf_bytes) ? 0 : o1 - o0;
}

__device__ __forceinline__ void store128(void* out, uint32_t flags, int64_t i, const F128& z) {
  uint64_t* o = (uint64_t*)out;
  if (flags & PMP_OUT_FIELD) {
    o[3 * i] = z.lo;
    o[3 * i + 1] = z.hi;
    o[3 * i + 2] = z.top;
  } else {  // h mod 2^128
    o[2 * i] = z.lo;
    o[2 * i + 1] = z.hi;
  }
}

struct P128Args {
  const uint8_t* buf;
  uint64_t buf_bytes;
  const int64_t* off;
  int64_t count;
  const uint64_t* keys;
  void* out;
  uint32_t flags;
  uint32_t* tcnt;         // units of each tile of 64 strings
  const int64_t* tstart;  // tiles + 1: first unit of each tile (the last entry is the total)
  F128* z2;               // level-2 values of strings with more than one node, at start(s) + k
  uint64_t zcap;          // entries of z2 (only offsets that decrease can ask for more)
};
constexpr int64_t TILE = 64;  // strings per tile
__device__ __forceinline__ int64_t tiles_of(int64_t count) { return (count + TILE - 1) / TILE; }

// Unit g: part k of string s, whose first unit is start (the units of a
// string are numbered after those of the strings before it). The tile by a
// 64-ary search over the tile starts, then the string by a wave scan of its
// tile's unit counts.
struct UnitPos {
  int64_t s, k, start;
};
__device__ UnitPos unit_at(const P128Args& A, int64_t g, int lane) {
  int64_t lo = 0, hi = tiles_of(A.count);
  while (hi - lo > 1) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t idx = lo + (int64_t)lane * step;
    const bool le = idx < hi && A.tstart[idx] <= g;
    const uint64_t mask = __ballot(le);
    const int last = 63 - __clzll((long long)mask);
    lo = lo + (int64_t)last * step;
    hi = lo + step < hi ? lo + step : hi;
  }
  const int64_t i = lo * TILE + lane;
  const uint32_t u = i < A.count ? (uint32_t)units_of(str_len(A.off, i, A.buf_bytes)) : 0u;
  uint64_t tot = 0;
  const int64_t ex = (int64_t)wave_excl_scan(u, &tot);
  const int64_t r = g - A.tstart[lo];  // the unit's rank in its tile
  const uint64_t own = __ballot(u > 0 && ex <= r && r < ex + (int64_t)u);
  const int l = own ? __ffsll((unsigned long long)own) - 1 : 0;
  const int64_t exl = (int64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)ex, l);
  return UnitPos{lo * TILE + l, r - exl, A.tstart[lo] + exl};
}

// ---------------------------------------------------------------------------
// Exact sums of 128 x 128 products from 32 x 32 -> 64 partial products:
// with a = sum a_i 2^(32 i) and x = sum x_j 2^(32 j), a x = sum over the
// diagonals d = i + j of (sum a_i x_j) 2^(32 d); diagonal d is kept as
// acc[d] + 2^64 cnt[d] (v_mad_u64_u32 with its carry counted), and turned
// into five 64-bit limbs once per block.
template <int ND>
struct Dg {
  uint64_t acc[ND];
  uint32_t cnt[ND];
};
using D7 = Dg<7>;  // a 128 x 128 product sum
template <int ND>
__device__ __forceinline__ void zero(Dg<ND>& s) {
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    s.acc[d] = 0;
    s.cnt[d] = 0;
  }
}
// (for each limb a_i the four multiply-adds, on four different diagonals,
// are issued before their four carry adds: a carry read right after it is
// written holds the wave up)
template <int ND>
__device__ __forceinline__ void mac128(Dg<ND>& s, const uint32_t* a, const uint32_t* x) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    uint64_t k0, k1, k2, k3;
    asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(s.acc[i]), "=s"(k0) : "v"(a[i]), "v"(x[0]));
    asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(s.acc[i + 1]), "=s"(k1) : "v"(a[i]), "v"(x[1]));
    asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(s.acc[i + 2]), "=s"(k2) : "v"(a[i]), "v"(x[2]));
    asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(s.acc[i + 3]), "=s"(k3) : "v"(a[i]), "v"(x[3]));
    asm("v_addc_co_u32_e64 %0, %1, 0, %0, %1" : "+v"(s.cnt[i]), "+s"(k0));
    asm("v_addc_co_u32_e64 %0, %1, 0, %0, %1" : "+v"(s.cnt[i + 1]), "+s"(k1));
    asm("v_addc_co_u32_e64 %0, %1, 0, %0, %1" : "+v"(s.cnt[i + 2]), "+s"(k2));
    asm("v_addc_co_u32_e64 %0, %1, 0, %0, %1" : "+v"(s.cnt[i + 3]), "+s"(k3));
  }
}
// s += v at 64-bit limb k (k <= 4), carries up to limb 4
__device__ __forceinline__ void add_limb(A5& s, uint64_t v, int k) {
  uint64_t c = v;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    if (i < k) continue;
    const uint64_t t = s.w[i] + c;
    c = t < c ? 1u : 0u;
    s.w[i] = t;
  }
}
// the diagonals as five 64-bit limbs (the sum must lie below 2^320)
template <int ND>
__device__ __forceinline__ A5 collapse(const Dg<ND>& s) {
  A5 r;
  zero(r);
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const int m = d >> 1;
    if ((d & 1) == 0) {
      add_limb(r, s.acc[d], m);
      if (m + 1 < 5) add_limb(r, s.cnt[d], m + 1);
    } else {
      add_limb(r, s.acc[d] << 32, m);
      add_limb(r, (s.acc[d] >> 32) | ((uint64_t)s.cnt[d] << 32), m + 1);
    }
  }
  return r;
}

template <int CTRL>
__device__ __forceinline__ A5 dpp5(const A5& s) {
  A5 r;
#pragma unroll
  for (int i = 0; i < 5; ++i) r.w[i] = dpp<CTRL>(s.w[i]);
  return r;
}

constexpr uint32_t OUTSIDE = 0x80000000u;  // past every buffer resource's end

// Word w (its four dwords realigned by sh, then masked to the padded string
// of Sec. 4: r = string bytes from the word's start) from the five dwords
// d[] read at its 4-aligned start.
__device__ __forceinline__ void word_dwords(const uint32_t* d, uint32_t sh, bool tail, int64_t r, uint32_t* x) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    x[u] = align_bytes(d[u + 1], d[u], sh);
    if (tail) x[u] = tail_word32(x[u], r - 4 * u);
  }
}

// Unit g: part k of string s's level-2 nodes (blocks QB k .. QB k + 31). The
// wave takes 8 blocks at a time, 8 lanes per block: lane j of a group holds
// words j, j + 8, ..., j + 120 of its block, all sixteen read at once through
// a buffer resource over the unit's bytes (range-checked per dword by the
// hardware: reads past the string's last dword are zeros, nothing is
// fetched for them), with the level-1 keys from LDS. The group adds its
// eight sums, folds, and multiplies by the block's level-2 key; the unit's
// share of its node is reduced and stored. (Eight lanes per block spread a
// step's fold and level-2 product over 16 KiB; at 168 VGPRs three waves per
// SIMD stay resident.)
constexpr int GW = 8;               // lanes per block
constexpr int WPL = BLOCK / GW;     // words per lane and block
constexpr int BPS = 64 / GW;        // blocks per wave step
constexpr int SPLIT = 1;            // load rounds per step
constexpr int WPR = WPL / SPLIT;    // words per lane and round
static_assert(WPL % SPLIT == 0, "whole rounds");
// sum over aligned groups of GW lanes, every lane of a group ends with it
__device__ __forceinline__ void group_sum(A5& s) {
  add(s, dpp5<0xB1>(s));
  add(s, dpp5<0x4E>(s));
  if constexpr (GW >= 8) add(s, dpp5<0x141>(s));
  if constexpr (GW >= 16) add(s, dpp5<0x140>(s));
}
__device__ void node_unit(const P128Args& A, const uint32_t* lk, int64_t g, int lane) {
  const UnitPos up = unit_at(A, g, lane);
  const int64_t s = up.s, k = up.k;
  const int64_t len = str_len(A.off, s, A.buf_bytes);
  const uint8_t* str = A.buf + (len ? A.off[s] : 0);
  const int64_t n1 = blocks_of(len);
  const int grp = lane / GW, j = lane % GW;
  const uint32_t sh = (uint32_t)((uintptr_t)str & 3u);
  const int64_t c0 = k * QB;
  const int64_t c1 = c0 + QB < n1 ? c0 + QB : n1;
  // the unit's bytes: from its first block (4-aligned) to the dword holding
  // the string's last byte (which lies in the buffer's pages)
  const uint64_t ubase = ((uint64_t)(uintptr_t)str - sh) + (uint64_t)c0 * BLK_BYTES;
  const uint64_t span = (((uint64_t)sh + (uint64_t)len + 3) & ~3ull) - (uint64_t)c0 * BLK_BYTES;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(uintptr_t)uni64(ubase), (short)0, (int)(span < 0x7fffffffull ? span : 0x7fffffffull), 0x00020000);
  A5 node;  // this group's blocks' share of the node (its lane 0)
  zero(node);
  for (int64_t cb = c0; cb < c1; cb += BPS) {
    const int64_t c = cb + grp;
    const bool act = c < c1;
    const bool tail = __ballot(act && c * (int64_t)BLK_BYTES + (int64_t)BLK_BYTES > len) != 0;
    D7 acc;
    zero(acc);
#pragma unroll
    for (int h = 0; h < SPLIT; ++h) {
      uint32_t d[WPR][5];
#pragma unroll
      for (int t = 0; t < WPR; ++t) {
        const uint32_t o =
            act ? (uint32_t)(c - c0) * (uint32_t)BLK_BYTES + 16u * (uint32_t)(j + GW * (WPR * h + t)) : OUTSIDE;
        const auto q = __builtin_amdgcn_raw_buffer_load_b128(rs, o, 0, 0);
        d[t][0] = q[0];
        d[t][1] = q[1];
        d[t][2] = q[2];
        d[t][3] = q[3];
        d[t][4] = __builtin_amdgcn_raw_buffer_load_b32(rs, o + 16u, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);  // every load of the round is issued before any is used
#pragma unroll
      for (int t = 0; t < WPR; ++t) {
        const int w = j + GW * (WPR * h + t);
        uint32_t x[4];
        word_dwords(d[t], sh, tail, len - W16 * (c * BLOCK + w), x);
        const uint4 kv = *(const uint4*)(lk + 4 * w);  // a_{1,w} as four 32-bit limbs
        const uint32_t a[4] = {kv.x, kv.y, kv.z, kv.w};
        mac128(acc, a, x);
      }
    }
    A5 sum = collapse(acc);
    group_sum(sum);
    if (act && j == 0) {
      add_b(sum, A.keys, 1);
      const F128 z1 = fold(sum);
      uint64_t a0, a1;
      key_a(A.keys, 2, (uint32_t)(c % BLOCK), &a0, &a1);
      mac_fe(node, a0, a1, z1);
    }
  }
  // the groups' shares (held by lanes 0, 16, 32, 48; zero elsewhere)
  for (int m = GW; m < 64; m <<= 1) {
    A5 o;
#pragma unroll
    for (int i = 0; i < 5; ++i) o.w[i] = shx64(node.w[i], m);
    add(node, o);
  }
  // the unit's share of its node, reduced (b_2 is added with the node)
  if (lane == 0 && (uint64_t)(up.start + k) < A.zcap) A.z2[up.start + k] = fold(node);
}

// Level-1 keys of the batch in LDS, a_{1,w} as four 32-bit limbs.
__device__ __forceinline__ void stage_keys(const uint64_t* keys, uint32_t* lk) {
  for (int i = (int)threadIdx.x; i < BLOCK; i += (int)blockDim.x) {
    const uint64_t lo = keys[2 * i], hi = keys[2 * i + 1];
    lk[4 * i] = (uint32_t)lo;
    lk[4 * i + 1] = (uint32_t)(lo >> 32);
    lk[4 * i + 2] = (uint32_t)hi;
    lk[4 * i + 3] = (uint32_t)(hi >> 32);
  }
  __syncthreads();
}

// Persistent waves over the units (their number is the last tile start).
__global__ __launch_bounds__(256, 3) void p128_nodes(P128Args A) {
  __shared__ __attribute__((aligned(16))) uint32_t lk[4 * BLOCK];
  const int64_t units = A.tstart[tiles_of(A.count)];
  if (units == 0) return;  // (the whole workgroup)
  stage_keys(A.keys, lk);
  const int lane = (int)(threadIdx.x & 63u);
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64; g < units; g += nw)
    node_unit(A, lk, g, lane);
}

// Strings of one block (at most 127 data words) longer than the tiny ones,
// four lanes per string: lane j holds words j, j + 4, ..., four at a time,
// read at once through a buffer resource over the wave's strings' bytes
// (range-checked per dword: past the buffer's last dword the reads are
// zeros) and masked to the padded string (Sec. 4); the four sums are added,
// folded and stored (the root is level 1). A wave whose strings span 2 GiB or
// more (a long string between them) reads word by word with guarded loads
// instead. Lanes with `mine` hold string s (lane j of its four).
constexpr int SG = 4;   // lanes per string
constexpr int SWL = 4;  // words per lane and round
__device__ void short4(const P128Args& A, const uint32_t* lk, bool mine, int64_t s, int j) {
  const int64_t len = mine ? str_len(A.off, s, A.buf_bytes) : 0;
  const int64_t o0 = len ? A.off[s] : 0;
  const uint8_t* str = A.buf + o0;
  const uint32_t sh = (uint32_t)((uintptr_t)str & 3u);
  const int64_t nw = mine ? len / W16 + 1 : 0;  // words, the pad's included
  // the wave's window: from its first string's dword to the buffer's end
  const uint64_t lo4 = (uint64_t)(uintptr_t)A.buf & ~3ull;
  const uint64_t hi4 = ((uint64_t)(uintptr_t)A.buf + A.buf_bytes + 3) & ~3ull;
  uint64_t wlo = mine ? (uint64_t)(uintptr_t)str - sh : ~0ull;
  uint64_t whi = mine ? (uint64_t)(uintptr_t)str - sh + 16 * (uint64_t)nw + 4 : 0ull;
  for (int m = 1; m < 64; m <<= 1) {
    const uint64_t a = (uint64_t)__shfl_xor((long long)wlo, m, 64), b = (uint64_t)__shfl_xor((long long)whi, m, 64);
    wlo = a < wlo ? a : wlo;
    whi = b > whi ? b : whi;
  }
  wlo = uni64(wlo < lo4 ? lo4 : wlo);
  whi = uni64(whi);
  const bool windowed = whi <= wlo || whi - wlo < 0x7fffffffull;
  A5 sum;
  zero(sum);
  if (windowed) {
    const uint64_t nrec = hi4 > wlo ? (hi4 - wlo < 0x7fffffffull ? hi4 - wlo : 0x7fffffffull) : 0;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)(uintptr_t)wlo, (short)0, (int)nrec, 0x00020000);
    const uint32_t sbase = mine ? (uint32_t)((uint64_t)(uintptr_t)str - sh - wlo) : 0u;
    int64_t rounds = (nw + SG * SWL - 1) / (SG * SWL);
    for (int m = 1; m < 64; m <<= 1) {
      const int64_t o = __shfl_xor((long long)rounds, m, 64);
      rounds = o > rounds ? o : rounds;
    }
    for (int64_t r0 = 0; r0 < rounds; ++r0) {
      uint32_t d[SWL][5];
#pragma unroll
      for (int q = 0; q < SWL; ++q) {
        const int64_t w = r0 * SG * SWL + j + SG * q;
        const uint32_t o = w < nw ? sbase + 16u * (uint32_t)w : OUTSIDE;
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, o, 0, 0);
        d[q][0] = v[0];
        d[q][1] = v[1];
        d[q][2] = v[2];
        d[q][3] = v[3];
        d[q][4] = __builtin_amdgcn_raw_buffer_load_b32(rs, o + 16u, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
      D7 acc;
      zero(acc);
#pragma unroll
      for (int q = 0; q < SWL; ++q) {
        const int64_t w = r0 * SG * SWL + j + SG * q;
        uint32_t x[4];
        word_dwords(d[q], sh, true, w < nw ? len - W16 * w : -64, x);
        const uint4 kv = *(const uint4*)(lk + 4 * (w < BLOCK ? w : 0));
        const uint32_t a[4] = {kv.x, kv.y, kv.z, kv.w};
        mac128(acc, a, x);
      }
      add(sum, collapse(acc));
    }
  } else if (mine) {
    for (int64_t w = j; w < nw; w += SG) {
      uint64_t x0, x1, a0, a1;
      word128(str, len, w, A.buf, A.buf + A.buf_bytes, &x0, &x1);
      key_a(A.keys, 1, (uint32_t)w, &a0, &a1);
      mac(sum, a0, a1, x0, x1);
    }
  }
  // the four lanes' sums (every lane takes part in the moves)
  add(sum, dpp5<0xB1>(sum));
  add(sum, dpp5<0x4E>(sum));
  if (mine && j == 0) {
    add_b(sum, A.keys, 1);
    store128(A.out, A.flags, s, fold(sum));
  }
}

// Tiny strings (at most TINY_BYTES, 17 words), one lane each, out of the
// wave's LDS stage (stage_strings): every word but the last lies wholly
// inside the string, the last one is masked to the padded string (Sec. 4);
// one word's LDS reads are issued before the word ahead of it is summed.
constexpr int64_t TINY_BYTES = 271;
__device__ __forceinline__ void hash_staged128(const P128Args& A, const uint32_t* lk, const uint8_t* stage, int64_t i,
                                               bool in, uint32_t p0, uint32_t sh, uint32_t ulen) {
  wait_vm0();
  const uint32_t nw = in ? ulen / W16 + 1 : 0u;  // words, the pad's included
  const uint32_t maxw = wave_max(nw);
  D7 acc;
  zero(acc);
  struct Wd {
    uint32_t d[5];
    uint4 k;
  };
  pipelined<2, Wd>(
      maxw > 0 ? maxw - 1 : 0u,
      [&](Wd& r, uint32_t w) {
        const uint32_t* q = (const uint32_t*)(stage + p0 + 16 * w);
#pragma unroll
        for (int u = 0; u < 5; ++u) r.d[u] = q[u];
        r.k = *(const uint4*)(lk + 4 * w);  // a_{1,w} as four 32-bit limbs
      },
      [&](const Wd& r, uint32_t w) {
        if (w + 1 >= nw) return;  // lanes past their full words sit out
        uint32_t x[4];
        word_dwords(r.d, sh, false, 0, x);
        const uint32_t a[4] = {r.k.x, r.k.y, r.k.z, r.k.w};
        mac128(acc, a, x);
      });
  if (!in) return;
  const uint32_t wl = nw - 1;  // the word that holds the end
  const uint32_t* q = (const uint32_t*)(stage + p0 + 16 * wl);
  uint32_t d[5];
#pragma unroll
  for (int u = 0; u < 5; ++u) d[u] = q[u];
  const uint4 kv = *(const uint4*)(lk + 4 * wl);
  const uint32_t a[4] = {kv.x, kv.y, kv.z, kv.w};
  uint32_t x[4];
  word_dwords(d, sh, true, (int64_t)ulen - W16 * (int64_t)wl, x);
  mac128(acc, a, x);
  A5 sum = collapse(acc);
  add_b(sum, A.keys, 1);
  store128(A.out, A.flags, i, fold(sum));
}

// Strings of one block in tiles of 64 consecutive strings, persistent waves
// (wave w takes tiles w, w + W, ...): tiny strings one lane each, the other
// strings of one block four lanes each, sixteen at a time. Each tile's units
// (parts of level-2 nodes of its longer strings) are counted for the node
// kernels.
__global__ __launch_bounds__(256, 2) void p128_tiles(P128Args A) {
  __shared__ __attribute__((aligned(16))) uint32_t lk[4 * BLOCK];
  __shared__ __attribute__((aligned(16))) uint8_t stages[4][STAGE_BYTES + STAGE_SLACK];
  __shared__ __attribute__((aligned(16))) uint32_t tables[4][STAGE_CHUNKS];
  stage_keys(A.keys, lk);
  const int lane = lane_id();
  const int wv = (int)(threadIdx.x / 64);
  uint8_t* stage = stages[wv];
  uint32_t* table = tables[wv];
  const int64_t nt = tiles_of(A.count);
  const int64_t nwv = (int64_t)gridDim.x * 4;
  for (int64_t t = (int64_t)blockIdx.x * 4 + wv; t < nt; t += nwv) {
    const int64_t i = t * TILE + lane;
    const bool act = i < A.count;
    const int64_t len = act ? str_len(A.off, i, A.buf_bytes) : 0;
    const int64_t o0 = len ? A.off[i] : 0;
    uint64_t tot = 0;
    (void)wave_excl_scan(act ? (uint32_t)units_of(len) : 0u, &tot);
    if (lane == 0) A.tcnt[t] = (uint32_t)tot;
    const bool tiny = act && len <= TINY_BYTES;
    stage_strings(A.buf, tiny, o0, (uint32_t)len, stage, table, [&](bool in, uint32_t p0, uint32_t sh) {
      hash_staged128(A, lk, stage, i, in, p0, sh, (uint32_t)len);
    });
    uint64_t rest = __ballot(act && !tiny && blocks_of(len) == 1);
    while (rest) {
      // the lanes of the next sixteen such strings, in lane order
      const uint32_t rank =
          __builtin_amdgcn_mbcnt_hi((uint32_t)(rest >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)rest, 0u));
      const bool pick = ((rest >> lane) & 1ull) && rank < 64 / SG;
      wait_lgkm0();  // earlier readers of the table are done
      if (pick) table[rank] = (uint32_t)lane;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const uint64_t picked = __ballot(pick);
      const int g = lane / SG;
      const bool have = g < __popcll(picked);
      const int src = have ? (int)table[g] : lane;
      short4(A, lk, have, t * TILE + src, lane % SG);
      rest &= ~picked;
    }
  }
}

__device__ __forceinline__ void add_fe(A5& s, const F128& z) {
  add_at(s, (u128)z.lo | ((u128)z.hi << 64), 0);
  if (z.top) add_at(s, (u128)1, 2);
}

// A string of more than one block, by one wave: its level-2 nodes from their
// units (node k = the sum of units UPN k .. UPN k + UPN - 1 plus b_2), then levels
// 3 and up. Each step writes its values over the previous ones: value q goes
// to index q, at or below its first input; a wave's loads of a step are done
// before its stores, and steps are ordered by a fence.
__device__ void climb_string(const P128Args& A, int64_t s, int64_t start, int lane) {
  const int64_t len = str_len(A.off, s, A.buf_bytes);
  const int64_t n1 = blocks_of(len);
  if (n1 == 1) return;
  const int64_t nq = (n1 + QB - 1) / QB;  // unit values
  if ((uint64_t)(start + nq) > A.zcap) return;
  F128* v = A.z2 + start;
  int64_t n = (n1 + BLOCK - 1) / BLOCK;  // level-2 values
  for (int64_t k0 = 0; k0 < n; k0 += 64) {
    const int64_t k = k0 + lane;
    A5 sum;
    zero(sum);
    if (k < n) {
      for (int64_t u = UPN * k; u < UPN * k + UPN && u < nq; ++u) add_fe(sum, v[u]);
      add_b(sum, A.keys, 2);
    }
    __threadfence();  // every lane has read its units
    if (k < n) v[k] = fold(sum);
    __threadfence();
  }
  for (int j = 3; n > 1 && j <= LMAX; ++j) {
    const int64_t nout = (n + BLOCK - 1) / BLOCK;
    for (int64_t q = 0; q < nout; ++q) {
      A5 sum;
      zero(sum);
      for (int u = 0; u < 2; ++u) {
        const int64_t i = q * BLOCK + 2 * lane + u;
        if (i < n) {
          uint64_t a0, a1;
          key_a(A.keys, j, (uint32_t)(i % BLOCK), &a0, &a1);
          mac_fe(sum, a0, a1, v[i]);
        }
      }
      wave_sum(sum);
      if (lane == 0) {
        add_b(sum, A.keys, j);
        v[q] = fold(sum);
      }
      __threadfence();  // node q's value is visible before any lane reads it
    }
    n = nout;
  }
  if (lane == 0) store128(A.out, A.flags, s, v[0]);
}

// Persistent waves over the units; a string's first unit climbs it.
__global__ __launch_bounds__(256) void p128_upper(P128Args A) {
  const int lane = (int)(threadIdx.x & 63u);
  const int64_t units = A.tstart[tiles_of(A.count)];
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64; g < units; g += nw) {
    const UnitPos up = unit_at(A, g, lane);
    if (up.k == 0) climb_string(A, up.s, up.start, lane);
  }
}

unsigned grid_for(int64_t threads) {
  const int64_t g = (threads + 255) / 256;
  return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

// scratch: unit counts (4 per tile of 64 strings, rounded to 8), tile starts
// (8 per tile and one), the scan's tile totals, then 32 bytes per possible
// unit
uint64_t pm128_scratch_bytes(int64_t count, uint64_t buf_bytes) {
  const uint64_t n = (uint64_t)count;
  const uint64_t nt = (n + TILE - 1) / TILE;
  const uint64_t units = 2 * n + buf_bytes / (BLK_BYTES * QB) + 2;
  return ((4 * nt + 7) & ~7ull) + 8 * (nt + 1) + excl_scan_work_bytes(nt) + sizeof(F128) * units;
}

hipError_t launch_pm128(const uint8_t* buf, uint64_t buf_bytes, const int64_t* offsets, int64_t count,
                        const uint64_t* keys, void* out, uint32_t flags, void* scratch, hipStream_t st) {
  const uint64_t n = (uint64_t)count;
  const uint64_t nt = (n + TILE - 1) / TILE;
  char* p = (char*)scratch;
  uint32_t* tcnt = (uint32_t*)p;
  p += (4 * nt + 7) & ~7ull;
  int64_t* tstart = (int64_t*)p;
  p += 8 * (nt + 1);
  uint64_t* bsum = (uint64_t*)p;
  p += excl_scan_work_bytes(nt);
  F128* z2 = (F128*)p;
  const uint64_t units_bound = 2 * n + buf_bytes / (BLK_BYTES * QB) + 2;
  P128Args a{buf, buf_bytes, offsets, count, keys, out, flags, tcnt, tstart, z2, units_bound};
  // the tile kernel: persistent, two workgroups of four waves per CU
  static std::atomic<int> cus_of[64];  // CUs per device, looked up once
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  int cus = cus_of[dev].load(std::memory_order_relaxed);
  if (!cus) {
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      return hipErrorInvalidDevice;
    cus_of[dev].store(cus, std::memory_order_relaxed);
  }
  const uint64_t tgrid = (nt + 3) / 4 < 2 * (uint64_t)cus ? (nt + 3) / 4 : 2 * (uint64_t)cus;
  if (nt) hipLaunchKernelGGL(p128_tiles, dim3((unsigned)tgrid), dim3(256), 0, st, a);
  hipError_t e = launch_excl_scan_u32(tcnt, nt, tstart, bsum, st);
  if (e != hipSuccess) return e;
  // persistent grids: at most 8192 waves, fewer when the units are fewer
  const int64_t waves = units_bound < 8192 ? (int64_t)units_bound : 8192;
  hipLaunchKernelGGL(p128_nodes, dim3(grid_for(waves * 64)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(p128_upper, dim3(grid_for(waves * 64)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace pmp
