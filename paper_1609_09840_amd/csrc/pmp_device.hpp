// Device-side arithmetic for PM+32 / PM+64 on gfx950 (wave64).
//
// Exact integer work on the vector ALU: 32x32->64 multiply-adds with the carry
// kept in a counter (deferred reduction: one modular reduction per 128-word
// block, as the paper's Sec. 6 does), the three-word fold of Sec. 6.2 and the
// canonicalisation of Algorithm 2 (with its last case as the prose states it),
// and the Sec. 7 mixers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pmp.h"

namespace pmp {

typedef unsigned __int128 u128;

constexpr uint32_t K32 = 15;  // p = 2^32 + 15 (Table "smallestprimes")
constexpr uint64_t K64 = 13;  // p = 2^64 + 13
constexpr int BLOCK = 128;    // m (Table "parameters")
constexpr int LMAX = 8;       // L (Table "parameters")

// ---------------------------------------------------------------------------
// acc + 2^64 * cnt += a * x   (one v_mad_u64_u32 whose carry-out feeds a
// 32-bit counter; the compiler does not expose the mad's carry by itself)
__device__ __forceinline__ void mac_vv(uint64_t& acc, uint32_t& cnt, uint32_t a, uint32_t x) {
  uint64_t c, d;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc), "=s"(c) : "v"(a), "v"(x));
  asm("v_addc_co_u32_e64 %0, %1, 0, %0, %2" : "+v"(cnt), "=s"(d) : "s"(c));
}
// same with a wave-uniform first factor held in an SGPR
__device__ __forceinline__ void mac_sv(uint64_t& acc, uint32_t& cnt, uint32_t a, uint32_t x) {
  uint64_t c, d;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc), "=s"(c) : "s"(a), "v"(x));
  asm("v_addc_co_u32_e64 %0, %1, 0, %0, %2" : "+v"(cnt), "=s"(d) : "s"(c));
}

// Four sums of that form, word u of a 16-byte group going to sum u. The four
// multiply-adds are issued before their carry adds, each carry in its own
// register pair: a carry read right after it is written holds the wave up,
// and four independent sums keep the multiply-adds from waiting on each other.
struct Acc4 {
  uint64_t lo[4];
  uint32_t hi[4];
};
__device__ __forceinline__ void zero(Acc4& s) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    s.lo[u] = 0;
    s.hi[u] = 0;
  }
}
__device__ __forceinline__ void mac4(Acc4& s, const uint32_t (&a)[4], const uint32_t (&x)[4]) {
  uint64_t k0, k1, k2, k3;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(s.lo[0]), "=s"(k0) : "v"(a[0]), "v"(x[0]));
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(s.lo[1]), "=s"(k1) : "v"(a[1]), "v"(x[1]));
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(s.lo[2]), "=s"(k2) : "v"(a[2]), "v"(x[2]));
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(s.lo[3]), "=s"(k3) : "v"(a[3]), "v"(x[3]));
  asm("v_addc_co_u32_e64 %0, %1, 0, %0, %1" : "+v"(s.hi[0]), "+s"(k0));
  asm("v_addc_co_u32_e64 %0, %1, 0, %0, %1" : "+v"(s.hi[1]), "+s"(k1));
  asm("v_addc_co_u32_e64 %0, %1, 0, %0, %1" : "+v"(s.hi[2]), "+s"(k2));
  asm("v_addc_co_u32_e64 %0, %1, 0, %0, %1" : "+v"(s.hi[3]), "+s"(k3));
}

// ---------------------------------------------------------------------------
// Block sums.
// PM+32: S = lo + 2^64 * hi  (a block sum is below 129 * 2^64)
struct S32 {
  uint64_t lo;
  uint32_t hi;
};
// PM+64: S = w0 + 2^64 * w1 + 2^128 * w2  (a block sum is below 129 * 2^128)
struct S64 {
  uint64_t w0, w1;
  uint32_t w2;
};
// PM+64 per-lane partial products of a 64x64 product split in 32-bit halves:
// value = p0 + 2^64 c0 + 2^32 (p1 + 2^64 c1) + 2^64 (p2 + 2^64 c2)
struct P64 {
  uint64_t p0, p1, p2;
  uint32_t c0, c1, c2;
};

__device__ __forceinline__ void zero(S32& s) { s.lo = 0; s.hi = 0; }
__device__ __forceinline__ void zero(S64& s) { s.w0 = 0; s.w1 = 0; s.w2 = 0; }
__device__ __forceinline__ void zero(P64& s) { s.p0 = s.p1 = s.p2 = 0; s.c0 = s.c1 = s.c2 = 0; }

__device__ __forceinline__ void add(S32& s, const S32& t) {
  uint64_t lo = s.lo + t.lo;
  s.hi = s.hi + t.hi + (lo < s.lo ? 1u : 0u);
  s.lo = lo;
}
__device__ __forceinline__ void add(S64& s, const S64& t) {
  u128 a = (u128)s.w0 + t.w0;
  u128 b = (u128)s.w1 + t.w1 + (uint64_t)(a >> 64);
  s.w0 = (uint64_t)a;
  s.w1 = (uint64_t)b;
  s.w2 = s.w2 + t.w2 + (uint32_t)(b >> 64);
}
// the exact total of four sums (each below 129 * 2^64 in a block sum)
__device__ __forceinline__ S32 sum4(const Acc4& q) {
  const u128 t = (u128)q.lo[0] + q.lo[1] + q.lo[2] + q.lo[3];
  return S32{(uint64_t)t, q.hi[0] + q.hi[1] + q.hi[2] + q.hi[3] + (uint32_t)(t >> 64)};
}
__device__ __forceinline__ void add_word(S32& s, uint64_t b) {
  uint64_t lo = s.lo + b;
  s.hi += (lo < s.lo ? 1u : 0u);
  s.lo = lo;
}
__device__ __forceinline__ void add_word(S64& s, uint64_t b) {
  u128 a = (u128)s.w0 + b;
  u128 c = (u128)s.w1 + (uint64_t)(a >> 64);
  s.w0 = (uint64_t)a;
  s.w1 = (uint64_t)c;
  s.w2 += (uint32_t)(c >> 64);
}

// PM+64 word x = (x0, x1), key a = (a0, a1): add a * x to the partial sums.
// The four multiply-adds go first and their carry adds after, each carry in
// its own register pair, so that no carry is read right after it is written
// (which would cost wait states).
__device__ __forceinline__ void mac64_vv(P64& s, uint64_t a, uint32_t x0, uint32_t x1) {
  uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  uint64_t k0, k1, k2, k3;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(s.p0), "=s"(k0) : "v"(a0), "v"(x0));
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(s.p1), "=s"(k1) : "v"(a0), "v"(x1));
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(s.p2), "=s"(k2) : "v"(a1), "v"(x1));
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(s.p1), "=s"(k3) : "v"(a1), "v"(x0));
  asm("v_addc_co_u32_e64 %0, %1, 0, %0, %1" : "+v"(s.c0), "+s"(k0));
  asm("v_addc_co_u32_e64 %0, %1, 0, %0, %1" : "+v"(s.c1), "+s"(k1));
  asm("v_addc_co_u32_e64 %0, %1, 0, %0, %1" : "+v"(s.c2), "+s"(k2));
  asm("v_addc_co_u32_e64 %0, %1, 0, %0, %1" : "+v"(s.c1), "+s"(k3));
}

// collapse the partial sums into three words
__device__ __forceinline__ S64 collapse(const P64& s) {
  u128 lo = (u128)s.p0 + ((u128)s.p1 << 32);  // p0 + 2^32 p1, below 2^97
  u128 mid = (u128)s.c0 + ((u128)s.c1 << 32) + s.p2 + (uint64_t)(lo >> 64);
  S64 r;
  r.w0 = (uint64_t)lo;
  r.w1 = (uint64_t)mid;
  r.w2 = s.c2 + (uint32_t)(mid >> 64);
  return r;
}

// ---------------------------------------------------------------------------
// Field elements z in [0, p) as lo + 2^n * hi, hi in {0, 1}.
struct Fe {
  uint64_t lo;
  uint32_t hi;
};

// Sec. 6.2 fold then Algorithm 2 (PM+32): S = w0 + 2^32 w1 + 2^64 w2 with
// w2 <= 128. With k*w1 = u1*2^32 + u0, S == (w0 + k^2 w2 + k u1) +
// (2^32 + k - u0) = v0 + 2^32 v1 (mod p), v1 <= 2. Then: if k v1 <= v0 the
// residue is v0 - k v1; if v1 = 1 (so v0 < k) it is v0 + 2^32; otherwise
// v1 = 2, v0 < 2k and it is 2^32 - k + v0 (since 2 * 2^32 == 2^32 - k).
__device__ __forceinline__ Fe fold32(uint32_t w0, uint32_t w1, uint32_t w2) {
  uint64_t kw1 = (uint64_t)w1 * K32;
  uint32_t u0 = (uint32_t)kw1, u1 = (uint32_t)(kw1 >> 32);
  uint64_t v = (uint64_t)w0 + (uint64_t)(K32 * K32) * w2 + (uint64_t)K32 * u1 + ((1ull << 32) + K32 - u0);
  uint32_t v0 = (uint32_t)v, v1 = (uint32_t)(v >> 32);
  // Algorithm 2 (corrected), without branches: v1 <= 2, so the result is
  // v0 - k v1 when that is not negative, else 2^32 + v0 (v1 = 1) or
  // 2^32 - k + v0 (v1 = 2)
  const uint32_t kv1 = K32 * v1;
  const bool ge = kv1 <= v0;
  const uint64_t wrap = (1ull << 32) + (uint64_t)v0 - (v1 == 1 ? 0u : K32);
  const uint64_t z = ge ? (uint64_t)(v0 - kv1) : wrap;
  Fe r;
  r.lo = (uint32_t)z;
  r.hi = (uint32_t)(z >> 32);
  return r;
}
__device__ __forceinline__ Fe reduce(const S32& s) { return fold32((uint32_t)s.lo, (uint32_t)(s.lo >> 32), s.hi); }

// Same for PM+64 with k = 13: S = w0 + 2^64 w1 + 2^128 w2, w2 <= 128.
__device__ __forceinline__ Fe fold64(uint64_t w0, uint64_t w1, uint32_t w2) {
  u128 kw1 = (u128)w1 * K64;
  uint64_t u0 = (uint64_t)kw1, u1 = (uint64_t)(kw1 >> 64);
  u128 v = (u128)w0 + (u128)(K64 * K64) * w2 + (u128)K64 * u1 + (((u128)1 << 64) + K64 - u0);
  uint64_t v0 = (uint64_t)v;
  uint32_t v1 = (uint32_t)(v >> 64);
  // Algorithm 2 (corrected), without branches (v1 <= 2): v0 - k v1 when that
  // is not negative, else 2^64 + v0 (v1 = 1) or 2^64 - k + v0 (v1 = 2)
  const uint64_t kv1 = K64 * (uint64_t)v1;
  const bool ge = kv1 <= v0;
  const uint64_t sub = v1 == 1 ? 0ull : K64;
  // 2^64 + v0 - sub: below 2^65; its high word is 0 when v0 < sub
  const uint64_t wlo = v0 - sub;
  const uint32_t whi = v0 >= sub ? 1u : 0u;
  Fe r;
  r.lo = ge ? v0 - kv1 : wlo;
  r.hi = ge ? 0u : whi;
  return r;
}
__device__ __forceinline__ Fe reduce(const S64& s) { return fold64(s.w0, s.w1, s.w2); }

// Upper levels: acc += a * z for a field element z = lo + 2^n hi.
__device__ __forceinline__ void mac_fe(S32& s, uint32_t a, const Fe& z) {
  mac_vv(s.lo, s.hi, a, (uint32_t)z.lo);
  if (z.hi) add(s, S32{(uint64_t)a << 32, 0u});
}
__device__ __forceinline__ void mac_fe(S64& s, uint64_t a, const Fe& z) {
  u128 pr = (u128)a * z.lo;
  S64 t;
  t.w0 = (uint64_t)pr;
  t.w1 = (uint64_t)(pr >> 64);
  t.w2 = 0;
  add(s, t);
  if (z.hi) add(s, S64{0, a, 0});
}

// ---------------------------------------------------------------------------
// Sec. 7 mixers (n-bit wraparound arithmetic).
__device__ __forceinline__ uint32_t mix32(uint32_t z) {
  z ^= z >> 13;
  z *= 0xab3be54fu;
  z ^= z >> 16;
  return z;
}
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 33;
  z *= 0xc4ceb9fe1a85ec53ull;
  z ^= z >> 33;
  return z;
}

// ---------------------------------------------------------------------------
// The two variants: key and block-sum types, word size W in bytes.
template <bool WIDE>
struct Tr;
template <>
struct Tr<false> {
  using key_t = uint32_t;
  using Sum = S32;
  static constexpr int W = 4;
};
template <>
struct Tr<true> {
  using key_t = uint64_t;
  using Sum = S64;
  static constexpr int W = 8;
};

// Output i (Sec. 5: h mod 2^n; the Sec. 7 mixer unless PMP_NO_MIX; or, with
// PMP_OUT_FIELD, the field value itself)
template <bool WIDE>
__device__ __forceinline__ void store_value(void* out, uint32_t flags, int64_t i, const Fe& z) {
  if (flags & PMP_OUT_FIELD) {
    uint64_t* o = (uint64_t*)out;
    if (WIDE) {
      o[2 * i] = z.lo;
      o[2 * i + 1] = z.hi;
    } else {
      o[i] = z.lo | ((uint64_t)z.hi << 32);
    }
  } else if (WIDE) {
    uint64_t r = z.lo;
    ((uint64_t*)out)[i] = (flags & PMP_NO_MIX) ? r : mix64(r);
  } else {
    uint32_t r = (uint32_t)z.lo;
    ((uint32_t*)out)[i] = (flags & PMP_NO_MIX) ? r : mix32(r);
  }
}

// ---------------------------------------------------------------------------
// Wave64 reductions (xor butterflies; every lane of a group ends with the sum)
__device__ __forceinline__ uint32_t shx(uint32_t v, int m) { return (uint32_t)__shfl_xor((int)v, m, 64); }
__device__ __forceinline__ uint64_t shx(uint64_t v, int m) {
  uint32_t lo = shx((uint32_t)v, m), hi = shx((uint32_t)(v >> 32), m);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ S32 shx(const S32& s, int m) { return S32{shx(s.lo, m), shx(s.hi, m)}; }
__device__ __forceinline__ S64 shx(const S64& s, int m) { return S64{shx(s.w0, m), shx(s.w1, m), shx(s.w2, m)}; }

// DPP lane moves within a row of 16 lanes (no LDS traffic):
//   0xB1 quad_perm [1,0,3,2] (lane ^ 1), 0x4E quad_perm [2,3,0,1] (lane ^ 2),
//   0x141 row_half_mirror (i -> 7 - i in each 8), 0x140 row_mirror (i -> 15 - i)
template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp(uint64_t v) {
  return ((uint64_t)dpp<CTRL>((uint32_t)(v >> 32)) << 32) | dpp<CTRL>((uint32_t)v);
}
template <int CTRL>
__device__ __forceinline__ S32 dpp(const S32& s) {
  return S32{dpp<CTRL>(s.lo), dpp<CTRL>(s.hi)};
}
template <int CTRL>
__device__ __forceinline__ S64 dpp(const S64& s) {
  return S64{dpp<CTRL>(s.w0), dpp<CTRL>(s.w1), dpp<CTRL>(s.w2)};
}
// Sum over aligned groups of G lanes (G = 1, 2, 4, 8, 16); every lane of a
// group ends with the group's sum. After the two quad steps each quad holds
// its sum, so mirroring within 8 (then 16) lanes pairs each lane with the
// other half.
template <int G, class S>
__device__ __forceinline__ void group_sum(S& s) {
  if constexpr (G >= 2) add(s, dpp<0xB1>(s));
  if constexpr (G >= 4) add(s, dpp<0x4E>(s));
  if constexpr (G >= 8) add(s, dpp<0x141>(s));
  if constexpr (G >= 16) add(s, dpp<0x140>(s));
}

template <class S>
__device__ __forceinline__ void reduce_lanes(S& s, int from, int to) {
  for (int m = from; m < to; m <<= 1) {
    S t = shx(s, m);
    add(s, t);
  }
}

// ---------------------------------------------------------------------------
// Word formation (end of Sec. 4): word w of a string of `len` bytes is the
// little-endian value of bytes [W w, W w + W) of bytes || 0x01 || 0...
// r = len - W w is the number of string bytes from the word's start.
__device__ __forceinline__ uint32_t tail_word32(uint32_t x, int64_t r) {
  if (r >= 4) return x;
  if (r < 0) return 0;
  uint32_t m = 1u << (8 * (uint32_t)r);
  return (x & (m - 1u)) | m;
}
__device__ __forceinline__ void tail_word64(uint32_t& x0, uint32_t& x1, int64_t r) {
  if (r >= 8) return;
  if (r < 0) {
    x0 = 0;
    x1 = 0;
    return;
  }
  if (r < 4) {
    uint32_t m = 1u << (8 * (uint32_t)r);
    x0 = (x0 & (m - 1u)) | m;
    x1 = 0;
  } else {
    uint32_t m = 1u << (8 * (uint32_t)(r - 4));
    x1 = (x1 & (m - 1u)) | m;
  }
}

// (hi:lo) >> (8 * sh), sh in [0, 3]
__device__ __forceinline__ uint32_t align_bytes(uint32_t hi, uint32_t lo, uint32_t sh) {
  return __builtin_amdgcn_alignbyte(hi, lo, sh);
}

// 16 bytes at a 4-byte-aligned address inside [lo, hi): one dwordx4 load.
// Anything not wholly inside is assembled byte by byte, zero outside.
struct Q {
  uint32_t d[4];
};
__device__ __forceinline__ Q load16(const uint8_t* a) {
  Q q;
  __builtin_memcpy(q.d, __builtin_assume_aligned(a, 4), 16);
  return q;
}
__device__ __forceinline__ Q load16_slow(const uint8_t* a, const uint8_t* lo, const uint8_t* hi) {
  Q q = {{0, 0, 0, 0}};
#pragma unroll 1
  for (int t = 0; t < 16; ++t) {
    const uint8_t* p = a + t;
    const uint32_t byte = (p >= lo && p < hi) ? (uint32_t)*p : 0u;
    q.d[t >> 2] |= byte << (8 * (t & 3));
  }
  return q;
}
__device__ __forceinline__ Q load16_guarded(const uint8_t* a, const uint8_t* lo, const uint8_t* hi) {
  if (a >= lo && a + 16 <= hi) return load16(a);
  return load16_slow(a, lo, hi);
}
__device__ __forceinline__ uint32_t load4_guarded(const uint8_t* a, const uint8_t* lo, const uint8_t* hi) {
  if (a >= lo && a + 4 <= hi) return *(const uint32_t*)__builtin_assume_aligned(a, 4);
  uint32_t v = 0;
#pragma unroll 1
  for (int t = 0; t < 4; ++t) {
    const uint8_t* p = a + t;
    v |= ((p >= lo && p < hi) ? (uint32_t)*p : 0u) << (8 * t);
  }
  return v;
}

}  // namespace pmp
