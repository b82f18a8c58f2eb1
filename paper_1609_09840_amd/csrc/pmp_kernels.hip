// PM+32 / PM+64 batch hashing kernels for gfx950 (wave64).
//
// One launch hashes a ragged batch (or two batches, one per variant). The
// work of a batch is the sum over strings of (alpha + bytes); wave w of the
// grid takes the w-th equal share of it, located by a 64-way search over the
// offsets, so every wave gets the same amount of work whatever the length
// mix, and no wave waits for another. Within its share a wave walks the
// strings 64 at a time:
//
//  - strings of one 128-word block (Algorithm 1 is then one Eq. (1)
//    evaluation) are hashed one per lane: the lane walks its string in
//    16-byte groups, the group's keys are wave-uniform scalar loads, and the
//    products are summed exactly with v_mad_u64_u32 plus a carry counter
//    (deferred reduction: one fold per block, Sec. 6);
//  - longer strings are hashed by the whole wave, G lanes per block (a lane
//    owns 128/G consecutive words of the block and keeps their level-1 keys
//    in registers); each block is reduced over its G lanes, folded into a
//    field element and multiplied straight into its level-2 node's sum.
//
// Tree levels >= 2 are finished without barriers: a level-2 node whose
// blocks all lie in one wave's share is computed by that wave; a node split
// between waves, and every node of level >= 3, has an accumulator slot that
// receives field elements by atomic adds with a weight counter (release /
// acquire at agent scope); the contribution that completes the weight
// computes the node, returns the slot to zero and climbs on.
#include "pmp_device.hpp"
#include "pmp_internal.h"

namespace pmp {

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

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}
__device__ __forceinline__ int64_t uni64s(int64_t v) { return (int64_t)uni64((uint64_t)v); }

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
  for (int m = 1; m < 64; m <<= 1) {
    uint32_t t = shx(v, m);
    v = t > v ? t : v;
  }
  return uni(v);
}
// exclusive prefix sum over the wave; *total receives the sum (uniform)
__device__ __forceinline__ uint64_t wave_excl_scan(uint64_t v, uint64_t* total) {
  const int lane = lane_id();
  uint64_t x = v;
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)x, d, 64);
    uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(x >> 32), d, 64);
    uint64_t y = ((uint64_t)hi << 32) | lo;
    if (lane >= d) x += y;
  }
  uint32_t tlo = (uint32_t)__shfl((int)(uint32_t)x, 63, 64);
  uint32_t thi = (uint32_t)__shfl((int)(uint32_t)(x >> 32), 63, 64);
  *total = uni64(((uint64_t)thi << 32) | tlo);
  return x - v;
}

// ---------------------------------------------------------------------------
// Output (Sec. 5: h mod 2^n; Sec. 7 mixer unless NO_MIX; or the field value)
template <bool WIDE>
__device__ __forceinline__ void store_out(const BatchArgs& B, int64_t i, const Fe& z) {
  if (B.flags & FLAG_OUT_FIELD) {
    uint64_t* o = (uint64_t*)B.out;
    if (WIDE) {
      o[2 * i] = z.lo;
      o[2 * i + 1] = z.hi;
    } else {
      o[i] = z.lo | ((uint64_t)z.hi << 32);
    }
  } else if (WIDE) {
    uint64_t r = z.lo;
    ((uint64_t*)B.out)[i] = (B.flags & FLAG_NO_MIX) ? r : mix64(r);
  } else {
    uint32_t r = (uint32_t)z.lo;
    ((uint32_t*)B.out)[i] = (B.flags & FLAG_NO_MIX) ? r : mix32(r);
  }
}

// ---------------------------------------------------------------------------
// Strings of one block, one per lane. `act` marks lanes with such a string.
template <bool WIDE>
__device__ void short_strings(const BatchArgs& B, int64_t i, bool act, int64_t o0, int64_t len) {
  using T = Tr<WIDE>;
  constexpr int W = T::W;
  constexpr int WPG = 16 / W;  // words per 16-byte group
  const uint8_t* lo = B.buf;
  const uint8_t* hi = B.buf + B.buf_bytes;
  const uint8_t* s = B.buf + (act ? o0 : 0);
  const uint32_t sh = (uint32_t)((uintptr_t)s & 3u);
  const uint8_t* a4 = s - sh;
  const int64_t nw = act ? len / W + 1 : 0;
  const uint32_t ng = (uint32_t)((nw + WPG - 1) / WPG);
  const uint32_t maxg = wave_max(ng);
  if (maxg == 0) return;
  const typename T::key_t* __restrict__ keys = (const typename T::key_t*)B.keys;

  typename T::Sum acc;
  zero(acc);
  P64 p;
  zero(p);
  Q cur = {{0, 0, 0, 0}};
  if (act) cur = load16_guarded(a4, lo, hi);
  for (uint32_t g = 0; g < maxg; ++g) {
    if (g < ng) {
      const uint8_t* nxa = a4 + 16 * (int64_t)(g + 1);
      Q nxt = {{0, 0, 0, 0}};
      if (g + 1 < ng) nxt = load16_guarded(nxa, lo, hi);
      else if (sh) nxt.d[0] = load4_guarded(nxa, lo, hi);
      uint32_t d[5] = {cur.d[0], cur.d[1], cur.d[2], cur.d[3], nxt.d[0]};
      uint32_t x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = align_bytes(d[u + 1], d[u], sh);
      if (g + 1 == ng) {
        const int64_t r0 = len - 16 * (int64_t)g;
        if constexpr (WIDE) {
          tail_word64(x[0], x[1], r0);
          tail_word64(x[2], x[3], r0 - 8);
        } else {
#pragma unroll
          for (int u = 0; u < 4; ++u) x[u] = tail_word32(x[u], r0 - 4 * u);
        }
      }
      if constexpr (WIDE) {
        const uint64_t* k = keys + 2 * g;
        mac64_sv(p, k[0], x[0], x[1]);
        mac64_sv(p, k[1], x[2], x[3]);
      } else {
        const uint32_t* k = keys + 4 * g;
#pragma unroll
        for (int u = 0; u < 4; ++u) mac_sv(acc.lo, acc.hi, k[u], x[u]);
      }
      cur = nxt;
    }
  }
  if (act) {
    typename T::Sum tot;
    if constexpr (WIDE) tot = collapse(p);
    else tot = acc;
    add_word(tot, (uint64_t)keys[8 * BLOCK]);  // b_1
    store_out<WIDE>(B, i, reduce(tot));
  }
}

// ---------------------------------------------------------------------------
// Tree shape of a string with C1 level-1 blocks (Algorithm 1): level j
// produces n[j] values, n[j+1] = ceil(n[j] / 128), until one value remains.
// Every node of level >= 2 owns one accumulator slot; the string's slots
// start at ceil(o0 / (128 W)) and are laid out level by level.
struct Levels {
  int L;
  uint64_t n[LMAX + 2];
  uint64_t off[LMAX + 2];  // slot offset of level j (j >= 2)
};
__device__ __forceinline__ Levels levels_of(uint64_t C1) {
  Levels t;
  t.n[1] = C1;
  int L = 1;
  while (t.n[L] > 1 && L <= LMAX) {
    t.n[L + 1] = (t.n[L] + BLOCK - 1) / BLOCK;
    ++L;
  }
  t.L = L;
  uint64_t o = 0;
  for (int j = 2; j <= L; ++j) {
    t.off[j] = o;
    o += t.n[j];
  }
  return t;
}

// A field element z as a number lo + 2^64 hi.
template <bool WIDE>
__device__ __forceinline__ uint64_t fe_lo(const Fe& z) {
  return WIDE ? z.lo : (z.lo | ((uint64_t)z.hi << 32));
}
template <bool WIDE>
__device__ __forceinline__ uint32_t fe_hi(const Fe& z) {
  return WIDE ? z.hi : 0u;
}

// Add a field element (< p) with weight `weight` to a node accumulator. The
// call that brings the weight to `target` gets true and the node's total
// (a sum of at most 128 field elements) in *tot, and returns the slot to
// zero for the next launch. Called by lane 0 only.
__device__ __forceinline__ bool contribute(Slot* sl, uint64_t clo, uint32_t chi, uint32_t weight, uint32_t target,
                                           uint64_t* tlo, uint32_t* thi) {
  const uint64_t old = __hip_atomic_fetch_add(&sl->lo, clo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t carry = (old + clo < old) ? 1u : 0u;
  if (carry + chi) __hip_atomic_fetch_add(&sl->hi, carry + chi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t before = __hip_atomic_fetch_add(&sl->cnt, weight, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
  if (before + weight != target) return false;
  *tlo = __hip_atomic_load(&sl->lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  *thi = __hip_atomic_load(&sl->hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&sl->lo, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&sl->hi, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&sl->cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

template <bool WIDE>
__device__ __forceinline__ Fe reduce_total(uint64_t lo, uint32_t hi, uint64_t b) {
  typename Tr<WIDE>::Sum s;
  zero(s);
  if constexpr (WIDE) {
    s.w0 = lo;
    s.w1 = hi;
  } else {
    s.lo = lo;
    s.hi = hi;
  }
  add_word(s, b);
  return reduce(s);
}

// A node value v at level j (index k) of string i is known: move up the tree.
// The parent's accumulator receives (a_{j+1, k mod 128} * v) mod p; whoever
// completes a parent computes it (adding b_{j+1}) and carries on. The root
// is written to the output. Wave-uniform arguments.
template <bool WIDE>
__device__ void climb(const KArgs& A, const BatchArgs& B, int64_t i, uint64_t sbase, const Levels& t, int j,
                      uint64_t k, Fe v) {
  using T = Tr<WIDE>;
  const typename T::key_t* keys = (const typename T::key_t*)B.keys;
  while (true) {
    if (j == t.L) {
      if (lane_id() == 0) store_out<WIDE>(B, i, v);
      return;
    }
    const uint64_t parent = k / BLOCK;
    const uint64_t nch = t.n[j] - parent * BLOCK < (uint64_t)BLOCK ? t.n[j] - parent * BLOCK : (uint64_t)BLOCK;
    typename T::Sum pr;
    zero(pr);
    mac_fe(pr, keys[(uint64_t)j * BLOCK + (k - parent * BLOCK)], v);  // level j+1 keys
    const Fe c = reduce(pr);
    const uint64_t si = sbase + t.off[j + 1] + parent;
    uint32_t done = 0;
    uint64_t tlo = 0;
    uint32_t thi = 0;
    if (lane_id() == 0) {
      if (si < B.nslots)
        done = contribute((Slot*)B.slots + si, fe_lo<WIDE>(c), fe_hi<WIDE>(c), 1u, (uint32_t)nch, &tlo, &thi) ? 1u : 0u;
      else __hip_atomic_fetch_or(A.status, STATUS_INTERNAL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!uni(done)) return;
    v = reduce_total<WIDE>(uni64(tlo), uni(thi), (uint64_t)keys[8 * BLOCK + j]);
    ++j;
    k = parent;
  }
}

// Exact sum over blocks c in [bl, bh) of level-2 node `node` of
// a_{2, c - 128 node} * f_1(block c), for a string of len bytes at s with C1
// blocks. G lanes per block: lane j of a group owns words [j*128/G,
// (j+1)*128/G) of its block, with those level-1 keys in registers. Every lane
// returns the whole wave's sum.
template <bool WIDE, int G>
__device__ typename Tr<WIDE>::Sum node_blocks(const BatchArgs& B, const uint8_t* s, int64_t len, int64_t C1,
                                              int64_t node, int64_t bl, int64_t bh) {
  using T = Tr<WIDE>;
  using key_t = typename T::key_t;
  using Sum = typename T::Sum;
  constexpr int W = T::W;
  constexpr int WPL = BLOCK / G;  // words per lane per block
  constexpr int BPL = WPL * W;    // bytes per lane per block
  constexpr int NL = BPL / 16;    // 16-byte loads per lane per block
  constexpr int ND = BPL / 4;     // dwords per lane per block
  constexpr int CPS = 64 / G;     // blocks per wave step
  static_assert(NL >= 1, "tile too wide");
  const int lane = lane_id();
  const int g = lane / G, j = lane % G;
  const uint8_t* lo = B.buf;
  const uint8_t* hi = B.buf + B.buf_bytes;
  const uint32_t sh = uni((uint32_t)((uintptr_t)s & 3u));
  const uint8_t* a4 = s - sh;
  const key_t* __restrict__ keys = (const key_t*)B.keys;
  const int64_t nb = node * BLOCK;

  key_t kr[WPL];
#pragma unroll
  for (int u = 0; u < WPL; ++u) kr[u] = keys[j * WPL + u];
  const key_t b1 = keys[8 * BLOCK];

  Sum acc2;
  zero(acc2);
  for (int64_t c0 = bl; c0 < bh; c0 += CPS) {
    const int64_t c = c0 + g;
    const bool act = c < bh;
    const int64_t off = c * (int64_t)(BLOCK * W) + (int64_t)j * BPL;
    const uint8_t* step_lo = a4 + c0 * (int64_t)(BLOCK * W);
    const uint8_t* step_hi = a4 + (c0 + CPS) * (int64_t)(BLOCK * W) + 4;
    const bool edge = (c0 + CPS >= bh) || step_lo < lo || step_hi > hi;  // uniform
    uint32_t d[ND + 1];
    if (!edge) {
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        Q q = load16(a4 + off + 16 * l);
        d[4 * l] = q.d[0];
        d[4 * l + 1] = q.d[1];
        d[4 * l + 2] = q.d[2];
        d[4 * l + 3] = q.d[3];
      }
      d[ND] = sh ? *(const uint32_t*)__builtin_assume_aligned(a4 + off + BPL, 4) : 0u;
    } else {
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        Q q = {{0, 0, 0, 0}};
        // bytes from the string end on are masked below, so skip such loads
        if (act && off + 16 * l < len + 4) q = load16_guarded(a4 + off + 16 * l, lo, hi);
        d[4 * l] = q.d[0];
        d[4 * l + 1] = q.d[1];
        d[4 * l + 2] = q.d[2];
        d[4 * l + 3] = q.d[3];
      }
      d[ND] = (act && sh && off + BPL < len + 4) ? load4_guarded(a4 + off + BPL, lo, hi) : 0u;
    }
    uint32_t x[ND];
#pragma unroll
    for (int u = 0; u < ND; ++u) x[u] = align_bytes(d[u + 1], d[u], sh);
    if (edge) {
      const int64_t w0 = c * BLOCK + (int64_t)j * WPL;  // first word of this lane
#pragma unroll
      for (int u = 0; u < WPL; ++u) {
        const int64_t r = act ? len - (int64_t)W * (w0 + u) : -1;
        if constexpr (WIDE) tail_word64(x[2 * u], x[2 * u + 1], r);
        else x[u] = tail_word32(x[u], r);
      }
    }
    Sum blk;
    if constexpr (WIDE) {
      P64 p;
      zero(p);
#pragma unroll
      for (int u = 0; u < WPL; ++u) mac64_vv(p, kr[u], x[2 * u], x[2 * u + 1]);
      blk = collapse(p);
    } else {
      zero(blk);
#pragma unroll
      for (int u = 0; u < WPL; ++u) mac_vv(blk.lo, blk.hi, kr[u], x[u]);
    }
    reduce_lanes(blk, 1, G);
    add_word(blk, (uint64_t)b1);
    const Fe z = reduce(blk);
    if (act) mac_fe(acc2, keys[BLOCK + (c - nb)], z);
  }
  reduce_lanes(acc2, G, 64);
  return acc2;
}

// Blocks [lo_c, hi_c) of one string with C1 >= 2 blocks, by the whole wave.
template <bool WIDE, int G>
__device__ void long_string(const KArgs& A, const BatchArgs& B, int64_t i, int64_t o0, int64_t len, int64_t C1,
                            int64_t lo_c, int64_t hi_c) {
  using T = Tr<WIDE>;
  constexpr int W = T::W;
  const typename T::key_t* keys = (const typename T::key_t*)B.keys;
  const uint8_t* s = B.buf + o0;
  const Levels t = levels_of((uint64_t)C1);
  if (t.L > LMAX) {  // more than 8 levels (over 2^56 words)
    if (lane_id() == 0) __hip_atomic_fetch_or(A.status, STATUS_OFFSETS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  const uint64_t sbase = ((uint64_t)o0 + BLOCK * W - 1) / (BLOCK * W);
  const uint64_t b2 = (uint64_t)keys[8 * BLOCK + 1];
  for (int64_t n = lo_c / BLOCK; n * BLOCK < hi_c; ++n) {
    const int64_t nlo = n * BLOCK;
    const int64_t nhi = (C1 < nlo + BLOCK) ? C1 : nlo + BLOCK;
    const int64_t bl = lo_c > nlo ? lo_c : nlo;
    const int64_t bh = hi_c < nhi ? hi_c : nhi;
    typename T::Sum part = node_blocks<WIDE, G>(B, s, len, C1, n, bl, bh);
    Fe v;
    if (bl == nlo && bh == nhi) {  // the whole node is here
      add_word(part, b2);
      v = reduce(part);
    } else {  // pieces of this node are hashed by neighbouring waves too
      const Fe c = reduce(part);
      const uint64_t si = sbase + t.off[2] + (uint64_t)n;
      uint32_t done = 0;
      uint64_t tlo = 0;
      uint32_t thi = 0;
      if (lane_id() == 0) {
        if (si < B.nslots)
          done = contribute((Slot*)B.slots + si, fe_lo<WIDE>(c), fe_hi<WIDE>(c), (uint32_t)(bh - bl),
                            (uint32_t)(nhi - nlo), &tlo, &thi)
                     ? 1u
                     : 0u;
        else __hip_atomic_fetch_or(A.status, STATUS_INTERNAL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (!uni(done)) continue;
      v = reduce_total<WIDE>(uni64(tlo), uni(thi), b2);
    }
    climb<WIDE>(A, B, i, sbase, t, 2, (uint64_t)n, v);
  }
}

// ---------------------------------------------------------------------------
// Static partition of a batch: the work of string i is alpha + len_i (a
// per-string cost plus its bytes). Positions (i, c) name level-1 block c of
// string i; pos(i, 0) = f(i) and pos(i, c) = f(i) + alpha + 128 W c for c > 0,
// with f(i) = alpha i + offsets[i] - offsets[0]. locate(x) is the first
// (i, c) with pos(i, c) >= x, so consecutive waves cover consecutive blocks.
struct Pos {
  int64_t i, c;
};
__device__ __forceinline__ uint64_t fpos(const int64_t* off, int64_t base, uint32_t alpha, int64_t i) {
  return (uint64_t)alpha * (uint64_t)i + (uint64_t)(off[i] - base);
}
template <int W>
__device__ Pos locate(const BatchArgs& B, uint32_t alpha, uint64_t x) {
  const int64_t* off = B.offsets;
  const int64_t n = B.count;
  const int64_t base = off[0];
  const int lane = lane_id();
  if (x == 0) return Pos{0, 0};
  if (x >= fpos(off, base, alpha, n)) return Pos{n, 0};
  int64_t lo = 0, hi = n;  // invariant: f(lo) <= x
  while (hi - lo >= 64) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t p = lo + (int64_t)lane * step;
    const bool ok = p <= hi && fpos(off, base, alpha, p) <= x;
    const uint64_t m = __ballot(ok) | 1ull;
    const int l = 63 - __clzll((long long)m);
    const int64_t nlo = lo + (int64_t)l * step;
    const int64_t nhi = nlo + step - 1;
    lo = nlo;
    hi = nhi < hi ? nhi : hi;
  }
  {
    const int64_t p = lo + lane;
    const bool ok = p <= hi && fpos(off, base, alpha, p) <= x;
    const uint64_t m = __ballot(ok) | 1ull;
    lo += 63 - __clzll((long long)m);
  }
  const int64_t i = uni64s(lo);
  if (i >= n) return Pos{n, 0};
  const uint64_t fi = fpos(off, base, alpha, i);
  if (x <= fi) return Pos{i, 0};
  const uint64_t y = x - fi;
  const int64_t len = off[i + 1] - off[i];
  const int64_t C1 = ((len / W + 1) + BLOCK - 1) / BLOCK;
  int64_t c = 1;
  if (y > alpha) c = (int64_t)((y - alpha + BLOCK * W - 1) / (BLOCK * W));
  if (c < 1) c = 1;
  if (c >= C1) return Pos{i + 1, 0};
  return Pos{i, c};
}

// All blocks in [ps, pe) of one batch, 64 strings at a time.
template <bool WIDE, int G>
__device__ void run_range(const KArgs& A, const BatchArgs& B, Pos ps, Pos pe) {
  using T = Tr<WIDE>;
  constexpr int W = T::W;
  const int lane = lane_id();
  if (pe.i < ps.i || (pe.i == ps.i && pe.c < ps.c)) {  // only possible when offsets decrease somewhere
    if (lane == 0) __hip_atomic_fetch_or(A.status, STATUS_OFFSETS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  const int64_t last = pe.c > 0 ? pe.i : pe.i - 1;  // last string with blocks here
  for (int64_t t0 = ps.i; t0 <= last; t0 += 64) {
    const int64_t i = t0 + lane;
    const bool in = i <= last && i < B.count;
    int64_t o0 = 0, o1 = 0;
    if (in) {
      o0 = B.offsets[i];
      o1 = B.offsets[i + 1];
    }
    const bool bad = in && !(o0 >= 0 && o0 <= o1 && (uint64_t)o1 <= B.buf_bytes);
    if (__ballot(bad) && lane == 0)
      __hip_atomic_fetch_or(A.status, STATUS_OFFSETS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool ok = in && !bad;
    const int64_t len = ok ? o1 - o0 : 0;
    const int64_t C1 = ((len / W + 1) + BLOCK - 1) / BLOCK;
    const int64_t lo_c = (i == ps.i) ? ps.c : 0;
    const int64_t hi_c = (i == pe.i) ? pe.c : C1;
    const bool shrt = ok && C1 == 1 && lo_c == 0 && hi_c >= 1;
    const bool lng = ok && C1 > 1 && lo_c < hi_c;

    short_strings<WIDE>(B, i, shrt, o0, len);

    uint64_t m = __ballot(lng);
    while (m) {
      const int l = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      const int64_t si = uni64s(__shfl((long long)i, l, 64));
      const int64_t so = uni64s(__shfl((long long)o0, l, 64));
      const int64_t sl = uni64s(__shfl((long long)len, l, 64));
      const int64_t sc = uni64s(__shfl((long long)C1, l, 64));
      const int64_t slo = uni64s(__shfl((long long)lo_c, l, 64));
      const int64_t shi = uni64s(__shfl((long long)hi_c, l, 64));
      long_string<WIDE, G>(A, B, si, so, sl, sc, slo, shi);
    }
  }
}

template <int G32, int G64>
__global__ __launch_bounds__(256) void batch_kernel(KArgs A) {
  const uint64_t w = (uint64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (w >= A.total_waves) return;
  uint64_t work[2] = {0, 0};
  for (uint32_t b = 0; b < A.nbatch; ++b) {
    const BatchArgs& B = A.b[b];
    if (B.count > 0) {
      const int64_t span = B.offsets[B.count] - B.offsets[0];
      work[b] = (uint64_t)A.alpha * (uint64_t)B.count + (uint64_t)(span > 0 ? span : 0);
    }
  }
  const uint64_t total = work[0] + work[1];
  const uint64_t x0 = (uint64_t)(((u128)total * w) / A.total_waves);
  const uint64_t x1 = (uint64_t)(((u128)total * (w + 1)) / A.total_waves);
  uint64_t bstart = 0;
  for (uint32_t b = 0; b < A.nbatch; ++b) {
    const uint64_t bend = bstart + work[b];
    const uint64_t lo = x0 > bstart ? x0 : bstart;
    const uint64_t hi = x1 < bend ? x1 : bend;
    if (lo < hi) {
      const BatchArgs& B = A.b[b];
      if (B.wide) {
        const Pos ps = locate<8>(B, A.alpha, lo - bstart), pe = locate<8>(B, A.alpha, hi - bstart);
        run_range<true, G64>(A, B, ps, pe);
      } else {
        const Pos ps = locate<4>(B, A.alpha, lo - bstart), pe = locate<4>(B, A.alpha, hi - bstart);
        run_range<false, G32>(A, B, ps, pe);
      }
    }
    bstart = bend;
  }
}

bool batch_tile_supported(int g) { return g == 4 || g == 8 || g == 16; }

template <int G32, int G64>
static hipError_t launch_t(const KArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((batch_kernel<G32, G64>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_batch(const KArgs& a, int grid, int g32, int g64, hipStream_t s) {
#define PMP_CASE(X, Y) \
  if (g32 == X && g64 == Y) return launch_t<X, Y>(a, grid, s);
  PMP_CASE(8, 8)
  PMP_CASE(4, 4)
  PMP_CASE(4, 8)
  PMP_CASE(8, 4)
  PMP_CASE(16, 8)
  PMP_CASE(8, 16)
  PMP_CASE(16, 16)
  PMP_CASE(4, 16)
  PMP_CASE(16, 4)
#undef PMP_CASE
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Plain GPU form (baseline): one string, one launch per tree level, one
// thread per block. Values are kept as 16-byte slots {lo, hi}.
template <bool WIDE>
__global__ void plain_level1(const uint8_t* buf, uint64_t buf_bytes, int64_t o0, int64_t len, const void* keysv,
                             uint4* vals, int64_t C1) {
  using T = Tr<WIDE>;
  constexpr int W = T::W;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C1) return;
  const typename T::key_t* keys = (const typename T::key_t*)keysv;
  const uint8_t* lo = buf;
  const uint8_t* hi = buf + buf_bytes;
  const uint8_t* s = buf + o0;
  const uint32_t sh = (uint32_t)((uintptr_t)s & 3u);
  const uint8_t* a4 = s - sh;
  typename T::Sum acc;
  zero(acc);
  P64 p;
  zero(p);
  for (int grp = 0; grp < BLOCK * W / 16; ++grp) {
    const int64_t boff = c * BLOCK * W + 16 * grp;
    uint32_t d[5] = {0, 0, 0, 0, 0};
    if (boff < len + 4) {
      Q q = load16_guarded(a4 + boff, lo, hi);
      for (int u = 0; u < 4; ++u) d[u] = q.d[u];
      d[4] = load4_guarded(a4 + boff + 16, lo, hi);
    }
    uint32_t x[4];
    for (int u = 0; u < 4; ++u) x[u] = align_bytes(d[u + 1], d[u], sh);
    const int64_t r0 = len - boff;
    if constexpr (WIDE) {
      tail_word64(x[0], x[1], r0);
      tail_word64(x[2], x[3], r0 - 8);
      const uint64_t* k = keys + 2 * grp;
      mac64_vv(p, k[0], x[0], x[1]);
      mac64_vv(p, k[1], x[2], x[3]);
    } else {
      const uint32_t* k = keys + 4 * grp;
      for (int u = 0; u < 4; ++u) mac_vv(acc.lo, acc.hi, k[u], tail_word32(x[u], r0 - 4 * u));
    }
  }
  typename T::Sum tot;
  if constexpr (WIDE) tot = collapse(p);
  else tot = acc;
  add_word(tot, (uint64_t)keys[8 * BLOCK]);
  Fe z = reduce(tot);
  vals[c] = make_uint4((uint32_t)z.lo, (uint32_t)(z.lo >> 32), z.hi, 0u);
}

template <bool WIDE>
__global__ void plain_upper(const uint4* in, uint64_t n_in, const void* keysv, int level0, uint4* outv) {
  using T = Tr<WIDE>;
  const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nout = (n_in + BLOCK - 1) / BLOCK;
  if (c >= nout) return;
  const typename T::key_t* keys = (const typename T::key_t*)keysv;
  typename T::Sum acc;
  zero(acc);
  for (int k = 0; k < BLOCK; ++k) {
    const uint64_t q = c * BLOCK + k;
    if (q >= n_in) break;
    const uint4 v = in[q];
    Fe z;
    z.lo = (uint64_t)v.x | ((uint64_t)v.y << 32);
    z.hi = v.z;
    mac_fe(acc, keys[(uint64_t)level0 * BLOCK + k], z);
  }
  add_word(acc, (uint64_t)keys[8 * BLOCK + level0]);
  Fe z = reduce(acc);
  outv[c] = make_uint4((uint32_t)z.lo, (uint32_t)(z.lo >> 32), z.hi, 0u);
}

template <bool WIDE>
__global__ void plain_store(const uint4* v, BatchArgs B, int64_t i) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    Fe z;
    z.lo = (uint64_t)v->x | ((uint64_t)v->y << 32);
    z.hi = v->z;
    store_out<WIDE>(B, i, z);
  }
}

template <bool WIDE>
static hipError_t plain_t(const uint8_t* buf, uint64_t buf_bytes, int64_t o0, int64_t len, const void* keys,
                          void* out, int64_t index, uint32_t flags, uint4* scratch, uint64_t slots, hipStream_t s) {
  constexpr int W = Tr<WIDE>::W;
  const int64_t nw = len / W + 1;
  uint64_t n = (uint64_t)((nw + BLOCK - 1) / BLOCK);
  uint64_t n2 = (n + BLOCK - 1) / BLOCK;
  if (n + n2 > slots) return hipErrorInvalidValue;
  uint4* a = scratch;
  uint4* b = scratch + n;
  hipLaunchKernelGGL(plain_level1<WIDE>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, buf, buf_bytes, o0,
                     len, keys, a, (int64_t)n);
  int level0 = 1;
  while (n > 1) {
    const uint64_t nout = (n + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(plain_upper<WIDE>, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, s, a, n, keys,
                       level0, b);
    uint4* t = a;
    a = b;
    b = t;
    n = nout;
    ++level0;
  }
  BatchArgs B{};
  B.out = out;
  B.flags = flags;
  B.wide = WIDE;
  hipLaunchKernelGGL(plain_store<WIDE>, dim3(1), dim3(64), 0, s, a, B, index);
  return hipGetLastError();
}

hipError_t launch_plain_string(int wide, const uint8_t* buf, uint64_t buf_bytes, int64_t o0, int64_t len,
                               const void* keys, void* out, int64_t index, uint32_t flags, uint4* scratch,
                               uint64_t scratch_slots, hipStream_t s) {
  return wide ? plain_t<true>(buf, buf_bytes, o0, len, keys, out, index, flags, scratch, scratch_slots, s)
              : plain_t<false>(buf, buf_bytes, o0, len, keys, out, index, flags, scratch, scratch_slots, s);
}

// ---------------------------------------------------------------------------
// Field reduction test hook
__global__ void debug_fold32(const uint32_t* w0, const uint32_t* w1, const uint32_t* w2, uint64_t* z, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (w2[i] > BLOCK) {
    z[i] = ~0ull;
    return;
  }
  Fe r = fold32(w0[i], w1[i], w2[i]);
  z[i] = r.lo | ((uint64_t)r.hi << 32);
}
__global__ void debug_fold64(const uint64_t* w0, const uint64_t* w1, const uint32_t* w2, uint64_t* z, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (w2[i] > BLOCK) {
    z[2 * i] = ~0ull;
    z[2 * i + 1] = ~0ull;
    return;
  }
  Fe r = fold64(w0[i], w1[i], w2[i]);
  z[2 * i] = r.lo;
  z[2 * i + 1] = r.hi;
}

hipError_t launch_debug_fold(int wide, const void* w0, const void* w1, const uint32_t* w2, void* z, int64_t n,
                             hipStream_t s) {
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (wide)
    hipLaunchKernelGGL(debug_fold64, dim3(grid), dim3(256), 0, s, (const uint64_t*)w0, (const uint64_t*)w1, w2,
                       (uint64_t*)z, n);
  else
    hipLaunchKernelGGL(debug_fold32, dim3(grid), dim3(256), 0, s, (const uint32_t*)w0, (const uint32_t*)w1, w2,
                       (uint64_t*)z, n);
  return hipGetLastError();
}

}  // namespace pmp
