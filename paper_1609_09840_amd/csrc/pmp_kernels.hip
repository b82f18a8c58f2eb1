// PM+32 / PM+64 batch hashing kernels for gfx950 (wave64).
//
// One launch hashes any number of ragged batches of either variant. The work
// of a batch is alpha per string plus its buffer bytes; wave w of the grid
// takes the w-th equal share of the launch's work and finds its first and
// last (string, block) positions by two 64-ary searches over the offsets run
// in lockstep, so no wave waits for another and no host pass is needed.
// Within its share a wave walks the strings 64 at a time:
//
//  - strings of at most 17 groups of 16 bytes are hashed one per lane out of
//    the wave's LDS stage, which direct-to-LDS loads fill with their chunks
//    (coalesced), Algorithm 1 being a single Eq. (1) evaluation for them;
//  - strings of up to 32 128-word blocks that lie wholly in the share: their
//    blocks form one task list shared out over the groups of G lanes, the
//    field elements go to LDS and level 2 is summed by all lanes together;
//  - longer strings by the whole wave, G lanes per block (a lane owns the
//    16-byte pieces j, j + G, ... of its block); each block is reduced over
//    its G lanes, folded into a field element (Sec. 6.2, Algorithm 2) and
//    multiplied straight into its level-2 node's sum.
//
// Products are summed exactly (v_mad_u64_u32 with a counted carry) and
// reduced once per block (deferred reduction). Tree levels >= 2 need no
// barrier: a level-2 node whose blocks all lie in one wave's share is
// computed by that wave; otherwise each contribution is added into the
// node's accumulator slot with relaxed device atomics together with its
// weight, and the contribution that completes the weight reads the sum back
// (its own atomic's result carries the data dependency), computes the node,
// returns the slot to zero and climbs on.
#include "pmp_device.hpp"
#include "pmp_batch.h"
#include "pmp_stage.hpp"

namespace pmp {

// ---------------------------------------------------------------------------
template <bool WIDE>
__device__ __forceinline__ void store_out(const BatchArgs& B, int64_t i, const Fe& z) {
  store_value<WIDE>(B.out, B.flags, i, z);
}

// ---------------------------------------------------------------------------
// Loads that are issued together. A piece whose bytes are not all inside
// [lo, hi) reads 16 bytes at `safe` instead (any readable address; the key
// table serves) so that every lane's load can be in flight at once; such
// pieces are zeroed, and the rare ones that straddle lo or hi are read again
// byte by byte afterwards.
__device__ __forceinline__ bool inside(const uint8_t* a, int n, const uint8_t* lo, const uint8_t* hi) {
  return a >= lo && a + n <= hi;
}

// Word u (0..3) of a 16-byte group held in dwords d[0..4], realigned by sh
// bytes, masked to the padded string (Sec. 4): r = string bytes from the
// start of the group's first word (negative: past the padded end).
template <bool WIDE>
__device__ __forceinline__ void group_words(const uint32_t* d, uint32_t sh, int64_t r, uint32_t* x) {
#pragma unroll
  for (int u = 0; u < 4; ++u) x[u] = align_bytes(d[u + 1], d[u], sh);
  if constexpr (WIDE) {
    tail_word64(x[0], x[1], r);
    tail_word64(x[2], x[3], r < 0 ? r : r - 8);
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = tail_word32(x[u], r < 0 ? r : r - 4 * u);
  }
}

// ---------------------------------------------------------------------------
// Length classes within a tile of 64 strings: "tiny" strings (at most
// TINY_GROUPS 16-byte groups of padded string) are hashed one per lane, all
// their loads in one batch; "medium" strings (the rest of those with at most
// MEDIUM_BLOCKS blocks, wholly in this wave's share) one per G-lane group;
// longer strings, or strings cut by the share's ends, by the whole wave.
constexpr uint32_t TINY_GROUPS = 17;  // strings of up to 271 bytes
constexpr int64_t MEDIUM_BLOCKS = 32;
static_assert(MEDIUM_BLOCKS <= BLOCK, "a medium string is one level-2 node");

// Dword u (string bytes 4u .. 4u + 3 from the group's start) of the group
// holding a string's end, rem = string bytes from the group's start: kept
// whole, cut at the end with the pad byte 0x01 after it, or zero (Sec. 4).
__device__ __forceinline__ uint32_t tail_dword(uint32_t x, int32_t r) {
  if (r >= 4) return x;
  if (r < 0) return 0u;
  const uint32_t b = 8u * (uint32_t)r;
  return (x & ((1u << b) - 1u)) | (1u << b);
}

// The sums of the tiny strings of the lanes in `in`, whose padded strings
// start p0 bytes into the stage (4-aligned, sh bytes before the string),
// once their chunks have been copied: b_1 + sum of key times word, folded.
template <bool WIDE>
__device__ __forceinline__ void hash_staged(const BatchArgs& B, const uint64_t* lk, const uint8_t* stage, int64_t i,
                                            bool in, uint32_t p0, uint32_t sh, uint32_t ulen, uint32_t ng) {
  using T = Tr<WIDE>;
  constexpr int KPG = WIDE ? 2 : 4;  // keys per group
  wait_vm0();
  const uint32_t maxg = wave_max(in ? ng : 0u);
  Acc4 acc;
  zero(acc);
  P64 p;
  zero(p);
  auto mac = [&](const uint32_t (&x)[4], const uint64_t (&k)[KPG]) {
    if constexpr (WIDE) {
      mac64_vv(p, k[0], x[0], x[1]);
      mac64_vv(p, k[1], x[2], x[3]);
    } else {
      const uint32_t k32[4] = {(uint32_t)k[0], (uint32_t)k[1], (uint32_t)k[2], (uint32_t)k[3]};
      mac4(acc, k32, x);
    }
  };
  // every group but the last: a group's LDS reads are issued before the one
  // ahead of it is summed (reads past a lane's string stay in the stage or its
  // slack; lanes past their full groups sit out)
  struct Grp {
    uint32_t d[5];
    uint64_t k[KPG];
  };
  pipelined<2, Grp>(
      maxg > 0 ? maxg - 1 : 0u,
      [&](Grp& r, uint32_t g) {
        const uint32_t* q = (const uint32_t*)(stage + p0 + 16 * g);
#pragma unroll
        for (int u = 0; u < 5; ++u) r.d[u] = q[u];
#pragma unroll
        for (int u = 0; u < KPG; ++u) r.k[u] = lk[KPG * g + u];  // level-1 keys, staged in LDS
      },
      [&](const Grp& r, uint32_t g) {
        if (g + 1 >= ng) return;
        uint32_t x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = align_bytes(r.d[u + 1], r.d[u], sh);
        mac(x, r.k);
      });
  if (!in) return;
  // the last group, masked to the padded string
  const uint32_t gl = ng - 1;
  const uint32_t* q = (const uint32_t*)(stage + p0 + 16 * gl);
  uint32_t d[5];
  uint64_t k[KPG];
#pragma unroll
  for (int u = 0; u < 5; ++u) d[u] = q[u];
#pragma unroll
  for (int u = 0; u < KPG; ++u) k[u] = lk[KPG * gl + u];
  const int32_t rem = (int32_t)ulen - 16 * (int32_t)gl;
  uint32_t x[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) x[u] = tail_dword(align_bytes(d[u + 1], d[u], sh), rem - 4 * u);
  mac(x, k);
  typename T::Sum tot;
  if constexpr (WIDE) tot = collapse(p);
  else tot = sum4(acc);
  add_word(tot, (uint64_t)((const typename T::key_t*)B.keys)[8 * BLOCK]);  // b_1
  store_out<WIDE>(B, i, reduce(tot));
}

// Tiny strings, one per lane out of the wave's LDS stage (stage_strings):
// each lane walks its string's groups, the level-1 keys being broadcast LDS
// reads; every group but the last lies wholly inside the string, and the
// last one, which holds the end, is masked to the padded string (Sec. 4: the
// bytes, a byte 0x01, zeros) in registers. The products are summed exactly
// with v_mad_u64_u32 plus carry counters (one fold per string).
template <bool WIDE>
__device__ void short_strings(const BatchArgs& B, const uint64_t* lk, uint8_t* stage, uint32_t* table, int64_t i,
                              bool act, int64_t o0, int64_t len) {
  using T = Tr<WIDE>;
  constexpr int W = T::W;
  const uint32_t ulen = act ? (uint32_t)len : 0u;  // < 272 here
  const uint32_t ng = act ? ((ulen / W + 1) * W + 15) / 16 : 0u;  // groups of the padded string
  stage_strings(B.buf, act, o0, ulen, stage, table, [&](bool in, uint32_t p0, uint32_t sh) {
    hash_staged<WIDE>(B, lk, stage, i, in, p0, sh, ulen, ng);
  });
}

// ---------------------------------------------------------------------------
// Node accumulators. Each node of level >= 2 that is not finished by a single
// wave owns one Slot; a string's slots start at ceil(o0 / (128 W)), level by
// level (level 2 first). Contributions are field elements; the call that
// brings the received weight to `target` gets the node's total (a sum of at
// most 128 field elements, lo + 2^64 hi), leaves the slot zeroed for the next
// launch and returns true. Only atomic read-modify-writes touch a slot, and a
// wave issues its second one only after the first has returned (its operand
// depends on the result), so no fence is needed: the completing wave's final
// exchange comes after every contribution in each word's order. Lane 0 only.
template <bool WIDE>
__device__ __forceinline__ bool contribute(Slot* sl, const Fe& c, uint32_t weight, uint32_t target, uint64_t* tlo,
                                           uint32_t* thi) {
  if constexpr (!WIDE) {
    constexpr uint64_t M56 = (1ull << 56) - 1;
    const uint64_t v = c.lo | ((uint64_t)c.hi << 32);  // < 2^33
    const uint64_t old =
        __hip_atomic_fetch_add(&sl->w0, ((uint64_t)weight << 56) + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((uint32_t)(old >> 56) + weight != target) return false;
    __hip_atomic_store(&sl->w0, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *tlo = (old & M56) + v;
    *thi = 0;
    return true;
  } else {
    const uint64_t old0 = __hip_atomic_fetch_add(&sl->w0, c.lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t carry = (old0 + c.lo < old0) ? 1u : 0u;
    const uint64_t add1 = ((uint64_t)weight << 32) | (uint64_t)(c.hi + carry);
    const uint64_t old1 = __hip_atomic_fetch_add(&sl->w1, add1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((uint32_t)(old1 >> 32) + weight != target) return false;
    *tlo = __hip_atomic_exchange(&sl->w0, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&sl->w1, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *thi = (uint32_t)old1 + c.hi + carry;
    return true;
  }
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

__device__ __forceinline__ uint64_t up(uint64_t n) { return (n + BLOCK - 1) / BLOCK; }

// Levels of a string with C1 blocks (Algorithm 1): n_1 = C1, n_{j+1} =
// ceil(n_j / 128), down to one value.
__device__ __forceinline__ int levels_of(uint64_t C1) {
  int L = 1;
  for (uint64_t n = C1; n > 1; n = up(n)) ++L;
  return L;
}

// The value v of node k on level 2 of string i is known; n2 = number of
// level-2 nodes. Move up the tree: the parent's accumulator receives
// (a_{j+1, k mod 128} * v) mod p; the wave that completes a parent computes
// it (adding b_{j+1}) and carries on; the root goes to the output.
template <bool WIDE>
__device__ void climb(const KArgs& A, const BatchArgs& B, int64_t i, uint64_t sbase, uint64_t n2, uint64_t k, Fe v) {
  using T = Tr<WIDE>;
  const typename T::key_t* keys = (const typename T::key_t*)B.keys;
  int j = 2;
  uint64_t nj = n2;    // values on level j
  uint64_t offj = 0;   // first slot of level j
  while (true) {
    if (nj == 1) {  // level j is the root
      if (lane_id() == 0) store_out<WIDE>(B, i, v);
      return;
    }
    const uint64_t parent = k / BLOCK;
    const uint64_t nch = nj - parent * BLOCK < (uint64_t)BLOCK ? nj - parent * BLOCK : (uint64_t)BLOCK;
    typename T::Sum pr;
    zero(pr);
    mac_fe(pr, keys[(uint64_t)j * BLOCK + (k - parent * BLOCK)], v);  // level j+1 keys
    const Fe c = reduce(pr);
    const uint64_t si = sbase + offj + nj + parent;  // slot of the parent on level j+1
    uint32_t done = 0;
    uint64_t tlo = 0;
    uint32_t thi = 0;
    if (lane_id() == 0) {
      if (si < B.nslots) done = contribute<WIDE>(B.slots + si, c, 1u, (uint32_t)nch, &tlo, &thi) ? 1u : 0u;
      else __hip_atomic_fetch_or(A.status, STATUS_INTERNAL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!uni(done)) return;
    v = reduce_total<WIDE>(uni64(tlo), uni(thi), (uint64_t)keys[8 * BLOCK + j]);
    offj += nj;
    nj = up(nj);
    ++j;
    k = parent;
  }
}

// Partial block sum of one lane: lane j of a G-lane group owns the 16-byte
// pieces j, j + G, j + 2G, ... of its block, so for each load the G lanes of
// a group read 16 G contiguous bytes. blk is the block start moved back by sh
// (4-aligned); piece P is bytes [16 P, 16 P + 16) of the block, read as
// dwords D0..D4 at blk + 16 P and realigned by sh bytes. block_loads issues
// all of a lane's loads at once (the caller guarantees that every byte read
// lies inside readable memory); block_sum turns them into the exact sum of
// key times word. lk holds the level-1 keys in LDS (as 64-bit words). TAIL:
// the block may be inactive (act) or run past the string end (rem = string
// bytes from the block start); its words are masked to the padded string of
// Sec. 4.

template <bool WIDE, int G>
struct Pieces {
  static constexpr int NL = BLOCK * Tr<WIDE>::W / 16 / G;  // pieces per lane
  uint32_t d[NL][5];
  uint32_t b[2];  // the dword pair that holds the string's end, when the block has it
};

// Byte offset, from a block's 4-aligned start, of the dword pair that holds
// the first byte past the string (rem = string bytes from the block's start;
// 0 when the string goes on past the block)
__device__ __forceinline__ uint32_t end_dword(int64_t rem, int64_t bw) {
  return rem >= 0 && rem < bw ? (uint32_t)rem & ~3u : 0u;
}

// The pieces of lane j of a group, read from the block at blk (4-aligned;
// rem = string bytes from its start). A piece that starts at or past the
// string's end is masked whole by block_sum, so it is read from the block's
// first piece instead (already on its way for the group's lane 0): the tail
// of a string's last block is not fetched from memory.
template <bool WIDE, int G>
__device__ __forceinline__ void block_loads(Pieces<WIDE, G>& P, const uint8_t* blk, int j, uint32_t sh,
                                            uint32_t eoff, int64_t rem) {
  const uint8_t* gb = gaddr((uint64_t)(uintptr_t)blk);  // global loads, whatever the pointer's origin
  constexpr int32_t BW = BLOCK * Tr<WIDE>::W;
  const int32_t rc = rem > BW ? BW : (rem < 0 ? 0 : (int32_t)rem);  // string bytes in the block
#pragma unroll
  for (int t = 0; t < Pieces<WIDE, G>::NL; ++t) {
    const int32_t o = 16 * (t * G + j);
    const uint8_t* pa = gb + (o < rc ? o : 0);
    Q q = load16(pa);
    P.d[t][0] = q.d[0];
    P.d[t][1] = q.d[1];
    P.d[t][2] = q.d[2];
    P.d[t][3] = q.d[3];
    // (loaded even when sh = 0, when it is not needed: a load under a
    // condition would make the compiler drain every load before its use)
    P.d[t][4] = *(const uint32_t*)__builtin_assume_aligned(pa + 16, 4);
  }
  // (eoff < 128 W, so these 8 bytes lie within the block's 128 W + 4)
  P.b[0] = *(const uint32_t*)__builtin_assume_aligned(gb + eoff, 4);
  P.b[1] = *(const uint32_t*)__builtin_assume_aligned(gb + eoff + 4, 4);
}

// A TAIL block may hold the string's end: a dword is summed only when all of
// its bytes are string bytes, and the dword that holds the first byte past
// the string (its own last bytes, the pad byte 0x01 and zeros: Sec. 4) is
// added once, by the lane whose piece holds it, from the pair P.b that
// block_loads read for it. Dwords past it are zero (padded string) and dropped.
template <bool WIDE, int G, bool TAIL>
__device__ __forceinline__ typename Tr<WIDE>::Sum block_sum(const Pieces<WIDE, G>& P, int j, uint32_t sh,
                                                            const uint64_t* lk, bool act, int64_t rem) {
  using T = Tr<WIDE>;
  constexpr int W = T::W;
  constexpr int WPP = 16 / W;  // words per piece
  constexpr int NL = Pieces<WIDE, G>::NL;
  constexpr int32_t BW = BLOCK * W;
  typename T::Sum acc;
  Acc4 q;
  P64 p;
  zero(q);
  zero(p);
  // string bytes from the block's start, clamped (inactive: every dword dropped)
  const int32_t rr = !TAIL ? BW : !act ? -16 : rem < -16 ? -16 : rem > BW ? BW : (int32_t)rem;
  const int32_t rj = rr - 16 * j - 4;  // dword u of piece t is kept when 16 G t + 4 u <= rj
#pragma unroll
  for (int t = 0; t < NL; ++t) {
    uint32_t x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[u] = align_bytes(P.d[t][u + 1], P.d[t][u], sh);
      if constexpr (TAIL) x[u] = 16 * G * t + 4 * u <= rj ? x[u] : 0u;
    }
    const uint64_t* kp = lk + WPP * (t * G + j);
    if constexpr (WIDE) {
      mac64_vv(p, kp[0], x[0], x[1]);
      mac64_vv(p, kp[1], x[2], x[3]);
    } else {
      const uint32_t k[4] = {(uint32_t)kp[0], (uint32_t)kp[1], (uint32_t)kp[2], (uint32_t)kp[3]};
      mac4(q, k, x);
    }
  }
  if constexpr (TAIL) {
    if (rr >= 0 && rr < BW && ((rr >> 4) % G) == j) {
      const uint32_t qb = (uint32_t)rr & 3u;  // string bytes in the end dword
      const uint32_t xb = align_bytes(P.b[1], P.b[0], sh);
      const uint32_t v = (xb & ((1u << (8 * qb)) - 1u)) | (1u << (8 * qb));
      const int32_t bd = rr >> 2;  // its dword in the block
      if constexpr (WIDE) {
        const bool high = bd & 1;
        mac64_vv(p, lk[bd >> 1], high ? 0u : v, high ? v : 0u);
      } else {
        mac_vv(q.lo[0], q.hi[0], (uint32_t)lk[bd], v);
      }
    }
  }
  if constexpr (WIDE) acc = collapse(p);
  else acc = sum4(q);
  return acc;
}

// The same for a step that touches the buffer edges (only possible at the
// very start or end of the buffer): one piece at a time, every byte checked.
template <bool WIDE, int G>
__device__ typename Tr<WIDE>::Sum block_guarded(const uint8_t* blk, int j, uint32_t sh, const uint64_t* lk, bool act,
                                                int64_t rem, const uint8_t* lo, const uint8_t* hi) {
  using T = Tr<WIDE>;
  constexpr int W = T::W;
  constexpr int WPP = 16 / W;
  constexpr int NL = BLOCK * W / 16 / G;
  const int64_t r = act ? rem : -(int64_t)(BLOCK * W) - 64;
  typename T::Sum acc;
  P64 p;
  zero(acc);
  zero(p);
#pragma unroll 1
  for (int t = 0; t < NL; ++t) {
    const int P = t * G + j;
    const int64_t rp = r - 16 * (int64_t)P;
    if (rp < 0) continue;  // the piece lies past the padded string
    const uint8_t* pa = gaddr((uint64_t)(uintptr_t)(blk + 16 * P));
    const Q q = load16_guarded(pa, lo, hi);
    const uint32_t d[5] = {q.d[0], q.d[1], q.d[2], q.d[3], sh ? load4_guarded(pa + 16, lo, hi) : 0u};
    uint32_t x[4];
    group_words<WIDE>(d, sh, rp, x);
    const uint64_t* kp = lk + WPP * P;
    if constexpr (WIDE) {
      mac64_vv(p, kp[0], x[0], x[1]);
      mac64_vv(p, kp[1], x[2], x[3]);
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) mac_vv(acc.lo, acc.hi, (uint32_t)kp[u], x[u]);
    }
  }
  if constexpr (WIDE) acc = collapse(p);
  return acc;
}

// Exact sum over blocks c in [bl, bh) of level-2 node `node` of
// a_{2, c - 128 node} * f_1(block c), for a string of len bytes at s, G lanes
// per block, 64 / G blocks per step. The loads of step n + 1 are issued
// before step n is summed (software pipelining: one step in flight while the
// other is computed); a step that touches the buffer's edges is read piece
// by piece instead. Every lane returns the whole wave's sum.
template <bool WIDE, int G>
__device__ typename Tr<WIDE>::Sum node_blocks(const BatchArgs& B, const uint64_t* lk, const uint8_t* s, int64_t len,
                                              int64_t node, int64_t bl, int64_t bh) {
  using T = Tr<WIDE>;
  using Sum = typename T::Sum;
  constexpr int W = T::W;
  constexpr int CPS = 64 / G;  // blocks per wave step
  static_assert(Pieces<WIDE, G>::NL >= 1, "tile too wide");
  const int lane = lane_id();
  const int g = lane / G, j = lane % G;
  const uint8_t* lo = B.buf;
  const uint8_t* hi = B.buf + B.buf_bytes;
  const uint8_t* safe = (const uint8_t*)B.keys;  // readable: 128 W + 16 bytes and more
  const uint32_t sh = uni((uint32_t)((uintptr_t)s & 3u));
  const uint8_t* a4 = s - sh;
  const int64_t nb = node * BLOCK;
  const uint64_t b1 = (uint64_t)((const typename T::key_t*)B.keys)[8 * BLOCK];
  // a step is read with plain loads when all of its bytes lie in the buffer
  auto plain = [&](int64_t c0) {
    const uint8_t* step_lo = a4 + c0 * (int64_t)(BLOCK * W);
    const uint8_t* step_hi = a4 + (c0 + CPS) * (int64_t)(BLOCK * W) + 4;
    return c0 < bh && step_lo >= lo && step_hi <= hi;  // uniform
  };

  Sum acc2;
  zero(acc2);
  // one step: blocks c0 .. c0 + CPS - 1, held in `cur` (read plainly) or
  // read piece by piece at the buffer's edges
  auto step = [&](const Pieces<WIDE, G>& cur, bool cur_loaded, int64_t c0) {
    // keys stay in LDS: reading them again each step keeps registers free
    asm volatile("" ::: "memory");
    const int64_t c = c0 + g;
    const bool act = c < bh;
    const uint8_t* blk = a4 + c * (int64_t)(BLOCK * W);
    const bool tail = c0 + CPS >= bh;  // uniform
    const int64_t rem = len - c * (int64_t)(BLOCK * W);
    Sum blk_sum;
    if (!cur_loaded) blk_sum = block_guarded<WIDE, G>(blk, j, sh, lk, act, rem, lo, hi);
    else if (tail) blk_sum = block_sum<WIDE, G, true>(cur, j, sh, lk, act, rem);
    else blk_sum = block_sum<WIDE, G, false>(cur, j, sh, lk, true, 0);
    group_sum<G>(blk_sum);
    add_word(blk_sum, b1);
    const Fe z = reduce(blk_sum);
    if (act) mac_fe(acc2, (typename T::key_t)lk[BLOCK + (c - nb)], z);
  };
  // the loads of step c0 (and where they came from)
  auto fill = [&](Pieces<WIDE, G>& P, bool& h, int64_t c0) {
    h = plain(c0);
    block_loads<WIDE, G>(P, h ? a4 + (c0 + g) * (int64_t)(BLOCK * W) : safe, j, sh,
                         end_dword(len - (c0 + g) * (int64_t)(BLOCK * W), BLOCK * W),
                         len - (c0 + g) * (int64_t)(BLOCK * W));
  };
  // two buffers used in turn, the loop unrolled twice so that neither is
  // ever copied (a copy costs a move per register and waits for the loads):
  // the next step's loads are issued before this one is summed
  Pieces<WIDE, G> pa, pb;
  bool ha, hb;
  fill(pa, ha, bl);
  for (int64_t c0 = bl; c0 < bh; c0 += 2 * CPS) {
    fill(pb, hb, c0 + CPS);
    step(pa, ha, c0);
    if (c0 + CPS >= bh) break;
    fill(pa, ha, c0 + 2 * CPS);
    step(pb, hb, c0 + CPS);
  }
  reduce_lanes(acc2, G, 64);
  return acc2;
}

// Blocks [lo_c, hi_c) of one string with C1 >= 2 blocks, by the whole wave.
template <bool WIDE, int G>
__device__ void long_string(const KArgs& A, const BatchArgs& B, const uint64_t* lk, int64_t i, int64_t o0,
                            int64_t len, int64_t C1, int64_t lo_c, int64_t hi_c) {
  using T = Tr<WIDE>;
  constexpr int W = T::W;
  const typename T::key_t* keys = (const typename T::key_t*)B.keys;
  const uint8_t* s = B.buf + o0;
  if (levels_of((uint64_t)C1) > LMAX) {  // more than 8 levels (over 2^56 words)
    if (lane_id() == 0) __hip_atomic_fetch_or(A.status, STATUS_OFFSETS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  const uint64_t n2 = up((uint64_t)C1);
  const uint64_t sbase = ((uint64_t)o0 + BLOCK * W - 1) / (BLOCK * W);
  const uint64_t b2 = (uint64_t)keys[8 * BLOCK + 1];
  for (int64_t n = lo_c / BLOCK; n * BLOCK < hi_c; ++n) {
    const int64_t nlo = n * BLOCK;
    const int64_t nhi = (C1 < nlo + BLOCK) ? C1 : nlo + BLOCK;
    const int64_t bl = lo_c > nlo ? lo_c : nlo;
    const int64_t bh = hi_c < nhi ? hi_c : nhi;
    typename T::Sum part = node_blocks<WIDE, G>(B, lk, s, len, n, bl, bh);
    Fe v;
    if (bl == nlo && bh == nhi) {  // the whole node is here
      add_word(part, b2);
      v = reduce(part);
    } else {  // pieces of this node are hashed by neighbouring waves too
      const Fe c = reduce(part);
      const uint64_t si = sbase + (uint64_t)n;
      uint32_t done = 0;
      uint64_t tlo = 0;
      uint32_t thi = 0;
      if (lane_id() == 0) {
        if (si < B.nslots)
          done = contribute<WIDE>(B.slots + si, c, (uint32_t)(bh - bl), (uint32_t)(nhi - nlo), &tlo, &thi) ? 1u : 0u;
        else __hip_atomic_fetch_or(A.status, STATUS_INTERNAL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (!uni(done)) continue;
      v = reduce_total<WIDE>(uni64(tlo), uni(thi), b2);
    }
    climb<WIDE>(A, B, i, sbase, n2, (uint64_t)n, v);
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
// Work position of the start of string i: alpha per string before it plus
// its byte offset.
__device__ __forceinline__ uint64_t fpos(const int64_t* off, uint32_t alpha, int64_t i) {
  return (uint64_t)alpha * (uint64_t)i + (uint64_t)off[i];
}
// The (string, block) positions of work offsets x0 <= x1 within a batch:
// the first block starting at or after each. Block 0 of string i starts at
// fpos(i); block c >= 1 at fpos(i) + alpha + (c - 1) * 128 W. Both 64-ary
// searches run in lockstep so that their loads share the round trips.
template <int W>
__device__ void locate2(const BatchArgs& B, uint32_t alpha, uint64_t x0, uint64_t x1, Pos& p0, Pos& p1) {
  const int64_t* off = B.offsets;
  const int64_t n = B.count;
  const int lane = lane_id();
  const uint64_t fn = fpos(off, alpha, n);
  // invariant: fpos(lo) <= x (or lo = 0)
  int64_t lo0 = 0, hi0 = n, lo1 = 0, hi1 = n;
  while (hi0 - lo0 >= 64 || hi1 - lo1 >= 64) {
    const int64_t st0 = (hi0 - lo0 + 63) / 64, st1 = (hi1 - lo1 + 63) / 64;
    const int64_t q0 = lo0 + (int64_t)lane * st0, q1 = lo1 + (int64_t)lane * st1;
    const bool a0 = hi0 - lo0 >= 64 && q0 <= hi0, a1 = hi1 - lo1 >= 64 && q1 <= hi1;
    const uint64_t f0 = a0 ? fpos(off, alpha, q0) : 0, f1 = a1 ? fpos(off, alpha, q1) : 0;
    if (hi0 - lo0 >= 64) {
      const uint64_t m = __ballot(a0 && f0 <= x0) | 1ull;
      const int64_t nlo = lo0 + (int64_t)(63 - __clzll((long long)m)) * st0, nhi = nlo + st0 - 1;
      lo0 = nlo;
      hi0 = nhi < hi0 ? nhi : hi0;
    }
    if (hi1 - lo1 >= 64) {
      const uint64_t m = __ballot(a1 && f1 <= x1) | 1ull;
      const int64_t nlo = lo1 + (int64_t)(63 - __clzll((long long)m)) * st1, nhi = nlo + st1 - 1;
      lo1 = nlo;
      hi1 = nhi < hi1 ? nhi : hi1;
    }
  }
  {
    const int64_t q0 = lo0 + lane, q1 = lo1 + lane;
    const bool a0 = q0 <= hi0, a1 = q1 <= hi1;
    const uint64_t f0 = a0 ? fpos(off, alpha, q0) : 0, f1 = a1 ? fpos(off, alpha, q1) : 0;
    lo0 += 63 - __clzll((long long)(__ballot(a0 && f0 <= x0) | 1ull));
    lo1 += 63 - __clzll((long long)(__ballot(a1 && f1 <= x1) | 1ull));
  }
  const int64_t i0 = uni64s(lo0), i1 = uni64s(lo1);
  // string i0 / i1 and the next offsets, loaded together
  const int64_t j = lane == 0 ? i0 : i1;
  const bool ld = lane < 2 && j < n;
  const int64_t oa = ld ? off[j] : 0, ob = ld ? off[j + 1] : 0;
  auto finish = [&](uint64_t x, int64_t i, int l) -> Pos {
    if (x == 0) return Pos{0, 0};
    if (x >= fn || i >= n) return Pos{n, 0};
    const int64_t o0 = uni64s((int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)oa, l)) |
                                        ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)oa >> 32), l) << 32)));
    const int64_t o1 = uni64s((int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)ob, l)) |
                                        ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)ob >> 32), l) << 32)));
    const uint64_t fi = (uint64_t)alpha * (uint64_t)i + (uint64_t)o0;
    if (x <= fi) return Pos{i, 0};
    const uint64_t y = x - fi;
    const int64_t len = o1 - o0;
    const int64_t C1 = ((len / W + 1) + BLOCK - 1) / BLOCK;
    int64_t c = 1;
    if (y > alpha) c = (int64_t)((y - alpha + BLOCK * W - 1) / (BLOCK * W));
    if (c < 1) c = 1;
    if (c >= C1) return Pos{i + 1, 0};
    return Pos{i, c};
  };
  p0 = finish(x0, i0, 0);
  p1 = finish(x1, i1, 1);
}

// Medium strings (2..MEDIUM_BLOCKS blocks, or one block of more than
// TINY_GROUPS groups). Their blocks form one task list: first every block but
// the last of each string (all of them full, summed without masks), then the
// last blocks (masked to the padded string of Sec. 4). Task t goes to G-lane
// group t mod (64 / G) at step t / (64 / G), so every group has the same
// number of blocks whatever the lengths. A block is summed by its group as in
// block_sum and folded (Sec. 6.2, Algorithm 2); its field element goes to
// LDS with its string's lane and block. The next step's block is loaded while
// the current one is summed. Then all lanes share the level-2 products
// a_{2,c} z_c (Eq. (1) on level 2) and each string's lane adds b_2 and folds.
// Strings whose tasks do not fit the LDS take a further round. `med` marks lanes whose string (i, o0, len, C1) is
// medium; `zbuf` and `tab` are the wave's stage and table.
constexpr uint32_t MEDIUM_TASKS = STAGE_BYTES / 16;  // field elements held at once
static_assert(64 * 4 * 8 <= 4 * STAGE_CHUNKS, "the level-2 limb sums of 64 strings fit the task table");

template <bool WIDE, int G>
__device__ void medium_strings(const BatchArgs& B, const uint64_t* lk, uint8_t* zbuf, uint32_t* tab, bool med,
                               int64_t i, int64_t o0, int64_t len, int64_t C1) {
  using T = Tr<WIDE>;
  using Sum = typename T::Sum;
  constexpr int W = T::W;
  constexpr int CPS = 64 / G;
  constexpr int64_t BW = BLOCK * W;
  uint64_t todo = __ballot(med);
  if (!todo) return;
  const int lane = lane_id();
  const int g = lane / G, j = lane % G;
  const uint8_t* lo = B.buf;
  const uint8_t* hi = B.buf + B.buf_bytes;
  const uint8_t* safe = (const uint8_t*)B.keys;  // readable: 128 W + 16 bytes and more
  const uint64_t b1 = (uint64_t)((const typename T::key_t*)B.keys)[8 * BLOCK];
  const uint64_t b2 = (uint64_t)((const typename T::key_t*)B.keys)[8 * BLOCK + 1];
  uint64_t ntask = 0;
  (void)wave_excl_scan(med ? (uint64_t)C1 : 0ull, &ntask);
  const uint32_t nmed = (uint32_t)__popcll(todo);
  if (ntask == nmed && nmed <= (uint32_t)CPS) {
    // a few single-block strings: one per group, no task list to build
    const uint32_t rank =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(todo >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)todo, 0u));
    if (med) tab[rank] = (uint32_t)lane;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const bool act = (uint32_t)g < nmed;
    const int src = act ? (int)tab[g] : lane;  // every lane takes part in the shuffles
    const int64_t si = __shfl((long long)i, src, 64);
    const int64_t so = __shfl((long long)o0, src, 64);
    const int64_t sl = __shfl((long long)len, src, 64);
    const uint8_t* sp = B.buf + (act ? so : 0);
    const uint32_t ssh = (uint32_t)((uintptr_t)sp & 3u);
    const uint8_t* blk = act ? sp - ssh : safe;
    Sum bs;
    if (__ballot(act && !inside(blk, BW + 4, lo, hi))) {
      bs = block_guarded<WIDE, G>(blk, j, ssh, lk, act, sl, lo, hi);
    } else {
      Pieces<WIDE, G> P;
      block_loads<WIDE, G>(P, blk, j, ssh, end_dword(act ? sl : -1, BW), act ? sl : -1);
      bs = block_sum<WIDE, G, true>(P, j, ssh, lk, act, sl);
    }
    group_sum<G>(bs);
    add_word(bs, b1);
    const Fe z = reduce(bs);
    if (act && j == 0) store_out<WIDE>(B, si, z);
    __builtin_amdgcn_wave_barrier();  // the table is read before it is used again
    return;
  }
  uint64_t* zl = (uint64_t*)zbuf;  // task t: z.lo at 2t, z.hi at 2t + 1
  const uint32_t nc = med ? (uint32_t)C1 : 0u;
  uint64_t tot = 0;
  const uint32_t c0 = (uint32_t)wave_excl_scan(nc, &tot);  // tasks before this lane's string
  uint32_t base = 0;
  const uint8_t* s = B.buf + (med ? o0 : 0);
  const uint32_t sh = (uint32_t)((uintptr_t)s & 3u);
  const uint8_t* a4 = s - sh;
  while (todo) {
    const bool in = ((todo >> lane) & 1ull) && c0 + nc - base <= MEDIUM_TASKS;
    const uint64_t pm = __ballot(in);
    uint64_t nfull = 0, nlast = 0;
    const uint32_t f0 = (uint32_t)wave_excl_scan(in ? nc - 1 : 0u, &nfull);  // this string's full blocks
    const uint32_t l0 = (uint32_t)wave_excl_scan(in ? 1u : 0u, &nlast);       // ... and its last one
    const uint32_t nf = (uint32_t)nfull;
    const uint32_t tr = nf + (uint32_t)nlast;  // tasks of this round
    const uint32_t tlast = nf + l0;            // task of this string's last block
    if (in) {
      for (uint32_t c = 0; c + 1 < nc; ++c) tab[f0 + c] = (uint32_t)lane;
      tab[tlast] = (uint32_t)lane;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the block of task t, for this lane's group (every lane takes part in
    // the shuffles: ds_bpermute reads 0 from a disabled source lane)
    auto task = [&](uint32_t t, const uint8_t*& blk, uint32_t& bsh, int64_t& rem, uint32_t& own) {
      const bool v = t < tr;
      const int src = v ? (int)tab[t] : lane;
      const uint64_t sa = (uint64_t)__shfl((long long)(uint64_t)(uintptr_t)a4, src, 64);
      const uint32_t ssh = (uint32_t)__shfl((int)sh, src, 64);
      const int64_t sl = __shfl((long long)len, src, 64);
      const uint32_t sf = (uint32_t)__shfl((int)f0, src, 64);
      const uint32_t sn = (uint32_t)__shfl((int)nc, src, 64);
      const uint32_t bc = t < nf ? t - sf : sn - 1;  // block of its string
      blk = v ? gaddr(sa + (uint64_t)bc * BW) : safe;
      bsh = v ? ssh : 0u;
      rem = v ? sl - (int64_t)bc * BW : -(int64_t)BW - 64;  // invalid: everything masked
      own = (uint32_t)src | (bc << 8);                       // its string's lane and block
    };
    const uint32_t steps = (tr + CPS - 1) / CPS;
    // a task's block, where it was read from, and its loads
    struct Tk {
      const uint8_t* blk;
      uint32_t sh;
      int64_t rem;
      uint32_t own;  // lane of its string | block << 8
      bool have;     // read with plain loads
    };
    auto issue = [&](Pieces<WIDE, G>& P, uint32_t t, Tk& k) {
      task(t, k.blk, k.sh, k.rem, k.own);
      k.have = t < tr && inside(k.blk, BW + 4, lo, hi);
      block_loads<WIDE, G>(P, k.have ? k.blk : safe, j, k.sh, end_dword(k.rem, BW), k.rem);
    };
    // the group's task of step st: sum, fold, field element to LDS
    auto compute = [&](const Pieces<WIDE, G>& P, const Tk& k, uint32_t st) {
      asm volatile("" ::: "memory");  // keys stay in LDS
      const uint32_t t = st * CPS + (uint32_t)g;
      const bool act = t < tr;
      const bool full = (st + 1) * CPS <= nf;  // uniform: every block of this step is full
      Sum bs;
      if (__ballot(act && !k.have)) bs = block_guarded<WIDE, G>(k.blk, j, k.sh, lk, act, k.rem, lo, hi);
      else if (full) bs = block_sum<WIDE, G, false>(P, j, k.sh, lk, true, 0);
      else bs = block_sum<WIDE, G, true>(P, j, k.sh, lk, act, k.rem);
      group_sum<G>(bs);
      add_word(bs, b1);
      const Fe z = reduce(bs);
      if (act && j == 0) {
        zl[2 * t] = z.lo;
        zl[2 * t + 1] = z.hi | ((uint64_t)k.own << 32);
      }
    };
    // two buffers used in turn (unrolled twice: neither is ever copied); the
    // next step's blocks are loaded while this one is summed
    Pieces<WIDE, G> pa, pb;
    Tk ka, kb;
    issue(pa, (uint32_t)g, ka);
    for (uint32_t st = 0; st < steps; st += 2) {
      issue(pb, (st + 1) * CPS + (uint32_t)g, kb);
      compute(pa, ka, st);
      if (st + 1 >= steps) break;
      issue(pa, (st + 2) * CPS + (uint32_t)g, ka);
      compute(pb, kb, st + 1);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // Level 2: b_2 + sum_c a_{2,c} z_c per string. The lanes share the
    // tasks (lane l takes tasks l, l + 64, ...) and add a_{2,c} z_c into the
    // string's sums in LDS (the task table is free now) as 32-bit limbs,
    // each summed in 64 bits (at most 32 terms of < 2^33: no overflow); then
    // the string's lane joins the limbs exactly and folds the total.
    constexpr int NLIMB = WIDE ? 4 : 2;
    using L2 = __attribute__((address_space(3))) uint64_t;
    L2* l2 = (L2*)(uintptr_t)lds_addr(tab);  // 64 strings x NLIMB sums
#pragma unroll
    for (int q = 0; q < NLIMB; ++q) l2[NLIMB * lane + q] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t t = (uint32_t)lane; t < tr; t += 64) {
      const uint64_t zlo = zl[2 * t];
      const uint64_t zhw = zl[2 * t + 1];
      const uint32_t own = (uint32_t)(zhw >> 32);
      const bool zh = zhw & 1u;
      const uint32_t sl = own & 63u;
      const uint64_t a = (uint64_t)(typename T::key_t)lk[BLOCK + (own >> 8)];
      uint64_t limb[NLIMB];
      if constexpr (WIDE) {
        const u128 pr = (u128)a * zlo;  // a z = a zlo + 2^64 a zh
        limb[0] = (uint32_t)pr;
        limb[1] = (uint32_t)(pr >> 32);
        limb[2] = (uint64_t)(uint32_t)(pr >> 64) + (zh ? (uint32_t)a : 0u);
        limb[3] = (uint64_t)(uint32_t)(pr >> 96) + (zh ? (uint32_t)(a >> 32) : 0u);
      } else {
        const uint64_t pr = a * zlo;  // a z = a zlo + 2^32 a zh
        limb[0] = (uint32_t)pr;
        limb[1] = (pr >> 32) + (zh ? a : 0u);
      }
#pragma unroll
      for (int q = 0; q < NLIMB; ++q)
        __hip_atomic_fetch_add(&l2[NLIMB * sl + q], limb[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (in) {
      Fe res;
      if (nc > 1) {
        Sum acc2;
        if constexpr (WIDE) {
          const u128 lo = (u128)l2[NLIMB * lane] + ((u128)l2[NLIMB * lane + 1] << 32);
          const u128 hi = (u128)l2[NLIMB * lane + 2] + ((u128)l2[NLIMB * lane + 3] << 32) + (uint64_t)(lo >> 64);
          acc2.w0 = (uint64_t)lo;
          acc2.w1 = (uint64_t)hi;
          acc2.w2 = (uint32_t)(hi >> 64);
        } else {
          const u128 v = (u128)l2[NLIMB * lane] + ((u128)l2[NLIMB * lane + 1] << 32);
          acc2.lo = (uint64_t)v;
          acc2.hi = (uint32_t)(v >> 64);
        }
        add_word(acc2, b2);
        res = reduce(acc2);
      } else {  // one block: its element is the hash
        res = Fe{zl[2 * tlast], (uint32_t)(zl[2 * tlast + 1] & 1u)};
      }
      store_out<WIDE>(B, i, res);
    }
    __builtin_amdgcn_wave_barrier();  // the table and the elements are read before the next round
    todo &= ~pm;
    base += tr;
  }
}

// All blocks in [ps, pe) of one batch, 64 strings at a time.
template <bool WIDE, int G>
__device__ void run_range(const KArgs& A, const BatchArgs& B, uint64_t* lk, uint8_t* stage, uint32_t* table,
                          Pos ps, Pos pe, bool restage, const uint64_t (&kv)[4]) {
  using T = Tr<WIDE>;
  constexpr int W = T::W;
  constexpr int WPG = 16 / W;
  const int lane = lane_id();
  const int64_t last = pe.c > 0 ? pe.i : pe.i - 1;  // last string with blocks here
  // each tile's offsets are loaded while the tile before it is hashed
  int64_t n0 = 0, n1 = 0;
  auto tile_offsets = [&](int64_t t0) {
    const int64_t q = t0 + lane;
    n0 = 0;
    n1 = 0;
    if (q <= last && q < B.count) {
      n0 = B.offsets[q];
      n1 = B.offsets[q + 1];
    }
  };
  tile_offsets(ps.i);
  // the batch's keys (loaded by the caller) go to LDS once the first tile's
  // offsets are on their way
  if (restage) {
    __builtin_amdgcn_wave_barrier();  // all lanes done with the previous keys
#pragma unroll
    for (int q = 0; q < 4; ++q) lk[lane + 64 * q] = kv[q];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // (the keys are staged even for an empty range: the caller counts on them)
  if (pe.i < ps.i || (pe.i == ps.i && pe.c < ps.c)) {  // only possible when offsets decrease somewhere
    if (lane == 0) __hip_atomic_fetch_or(A.status, STATUS_OFFSETS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  for (int64_t t0 = ps.i; t0 <= last; t0 += 64) {
    const int64_t i = t0 + lane;
    const bool in = i <= last && i < B.count;
    const int64_t o0 = n0, o1 = n1;
    if (t0 + 64 <= last) tile_offsets(t0 + 64);
    const bool bad = in && !(o0 >= 0 && o0 <= o1 && (uint64_t)o1 <= B.buf_bytes);
    if (__ballot(bad) && lane == 0)
      __hip_atomic_fetch_or(A.status, STATUS_OFFSETS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool ok = in && !bad;
    const int64_t len = ok ? o1 - o0 : 0;
    const int64_t nw = len / W + 1;
    const int64_t C1 = (nw + BLOCK - 1) / BLOCK;
    const int64_t lo_c = (i == ps.i) ? ps.c : 0;
    const int64_t hi_c = (i == pe.i) ? pe.c : C1;
    const bool whole = ok && lo_c == 0 && hi_c == C1;
    const bool tiny = whole && (nw + WPG - 1) / WPG <= TINY_GROUPS;
    const bool med = whole && !tiny && C1 <= MEDIUM_BLOCKS;
    const bool lng = ok && !tiny && !med && lo_c < hi_c;

    short_strings<WIDE>(B, lk, stage, table, i, tiny, o0, len);
    medium_strings<WIDE, G>(B, lk, stage, table, med, i, o0, len, C1);

    // the long strings, one at a time by the whole wave
    uint64_t m = __ballot(lng);
    while (m) {
      const int l = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      const int64_t si = t0 + l;
      const int64_t so = (int64_t)uni64(__builtin_amdgcn_readlane((int)(uint32_t)o0, l) |
                                        ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(o0 >> 32), l) << 32));
      const int64_t sl = (int64_t)uni64(__builtin_amdgcn_readlane((int)(uint32_t)len, l) |
                                        ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(len >> 32), l) << 32));
      const int64_t sc = ((sl / W + 1) + BLOCK - 1) / BLOCK;
      const int64_t slo = (si == ps.i) ? ps.c : 0;
      const int64_t shi = (si == pe.i) ? pe.c : sc;
      long_string<WIDE, G>(A, B, lk, si, so, sl, sc, slo, shi);
    }
  }
}

// A wave-uniform pointer to global memory, marked as such.
template <typename T>
__device__ __forceinline__ T* gptr(T* p) {
  using G = __attribute__((address_space(1))) T;
  return (T*)(G*)(uintptr_t)uni64((uint64_t)(uintptr_t)p);
}

// Batch b of the launch (b uniform). The argument copies of the first two
// batches are read by selection, never by a dynamic index, which would move
// the whole argument block to scratch.
__device__ __forceinline__ BatchArgs batch_at(const KArgs& A, uint32_t b) {
  BatchArgs B = A.batches ? gptr(A.batches)[b] : (b ? A.b[1] : A.b[0]);
  // a descriptor read from global memory is wave-uniform, but the compiler
  // cannot tell: keep its fields in scalar registers so that addresses built
  // from them (key tables above all) use scalar loads. The pointers are
  // rebuilt as global-memory pointers so that accesses through them stay
  // global loads and stores (generic ones would also count as LDS accesses).
  B.buf = gptr(B.buf);
  B.buf_bytes = uni64(B.buf_bytes);
  B.offsets = gptr(B.offsets);
  B.count = uni64s(B.count);
  B.keys = gptr(B.keys);
  B.out = gptr(B.out);
  B.flags = uni(B.flags);
  B.wide = uni(B.wide);
  B.slots = gptr(B.slots);
  B.nslots = uni64(B.nslots);
  B.work0 = uni64(B.work0);
  B.work = uni64(B.work);
  return B;
}

template <int G32, int G64>
__global__ __launch_bounds__(256, 2) void batch_kernel(KArgs A) {
  // each wave keeps the level-1 and level-2 keys of the batch it works on in
  // its own LDS region, as 64-bit words
  __shared__ uint64_t lkeys[4][2 * BLOCK];
  // the direct-to-LDS loads write only `stages`: the compiler then waits for
  // them before reads of `stages` alone, not before those of the tables
  __shared__ __attribute__((aligned(16))) uint8_t stages[4][STAGE_BYTES + STAGE_SLACK];
  __shared__ __attribute__((aligned(16))) uint32_t tables[4][STAGE_CHUNKS];
  const int lane = lane_id();
  uint64_t* lk = lkeys[threadIdx.x / 64];
  uint8_t* stage = stages[threadIdx.x / 64];
  uint32_t* table = tables[threadIdx.x / 64];
  const uint64_t w = (uint64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (w >= A.total_waves) return;
  const uint32_t nb = A.nbatch;
  const void* staged = nullptr;  // key table now in lk
  uint32_t staged_wide = 0;
  // shares w, w + W, w + 2W, ... (W waves): a wave's work is spread over the
  // launch, which evens out regions that cost more per unit of work
  for (uint32_t k = 0; k < A.per_wave; ++k) {
    const uint64_t sx = w + (uint64_t)k * A.total_waves;
    const uint64_t x0 = sx * A.share < A.total ? sx * A.share : A.total;
    const uint64_t x1 = x0 + A.share < A.total ? x0 + A.share : A.total;
    if (x0 >= x1) break;  // later shares lie further on
    // the batches that overlap [x0, x1), in order, 64 descriptors at a time
    for (uint32_t base = 0; base < nb; base += 64) {
      const uint32_t b = base + (uint32_t)lane;
      uint64_t s0 = 0, sw = 0;
      if (b < nb) {
        if (A.batches) {
          s0 = gptr(A.batches)[b].work0;
          sw = gptr(A.batches)[b].work;
        } else {
          s0 = b ? A.b[1].work0 : A.b[0].work0;
          sw = b ? A.b[1].work : A.b[0].work;
        }
      }
      uint64_t m = __ballot(b < nb && sw > 0 && s0 < x1 && s0 + sw > x0);
      const bool past = __ballot(b < nb && s0 >= x1) != 0;  // later chunks start past x1 too
      while (m) {
        const int l = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const BatchArgs B = batch_at(A, base + (uint32_t)l);
        const uint64_t lo = x0 > B.work0 ? x0 - B.work0 : 0;
        const uint64_t hi = x1 < B.work0 + B.work ? x1 - B.work0 : B.work;
        // this batch's keys go to the wave's LDS region; their loads are
        // issued before the share's search, so that the two overlap
        const bool restage = B.keys != staged || B.wide != staged_wide;  // uniform
        uint64_t kv[4] = {0, 0, 0, 0};
        if (restage) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int e = lane + 64 * q;
            kv[q] = B.wide ? ((const uint64_t*)B.keys)[e] : ((const uint32_t*)B.keys)[e];
          }
        }
        Pos ps, pe;
        if (A.alpha == PMP_ALPHA_BY_COUNT) {  // the work of a string is 1: [lo, hi) are its strings
          ps = Pos{(int64_t)lo, 0};
          pe = Pos{(int64_t)hi, 0};
        } else if (B.wide) {
          locate2<8>(B, A.alpha, lo, hi, ps, pe);
        } else {
          locate2<4>(B, A.alpha, lo, hi, ps, pe);
        }
        if (B.wide) run_range<true, G64>(A, B, lk, stage, table, ps, pe, restage, kv);
        else run_range<false, G32>(A, B, lk, stage, table, ps, pe, restage, kv);
        if (restage) {
          staged = B.keys;
          staged_wide = B.wide;
        }
      }
      if (past) break;
    }
  }
}

template <int G32, int G64>
static hipError_t launch_t(const KArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((batch_kernel<G32, G64>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int G32, int G64>
static int occupancy_t() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<G32, G64>, 256, 0) != hipSuccess) return 0;
  return n;
}

#define PMP_TILES(X) X(8, 16) X(8, 8) X(16, 16) X(4, 16) X(16, 8) X(4, 8)

hipError_t launch_batch(const KArgs& a, int grid, int g32, int g64, hipStream_t s) {
#define PMP_CASE(X, Y) \
  if (g32 == X && g64 == Y) return launch_t<X, Y>(a, grid, s);
  PMP_TILES(PMP_CASE)
#undef PMP_CASE
  return hipErrorInvalidValue;
}

int batch_blocks_per_cu(int g32, int g64) {
#define PMP_CASE(X, Y) \
  if (g32 == X && g64 == Y) return occupancy_t<X, Y>();
  PMP_TILES(PMP_CASE)
#undef PMP_CASE
  return 0;
}

int batch_tile_pairs(int (*pairs)[2], int max) {
  int n = 0;
#define PMP_CASE(X, Y)  \
  if (n < max) {        \
    pairs[n][0] = X;    \
    pairs[n][1] = Y;    \
  }                     \
  ++n;
  PMP_TILES(PMP_CASE)
#undef PMP_CASE
  return n < max ? n : max;
}

bool batch_tiles_supported(int g32, int g64) {
#define PMP_CASE(X, Y) \
  if (g32 == X && g64 == Y) return true;
  PMP_TILES(PMP_CASE)
#undef PMP_CASE
  return false;
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
