// Incremental hashing of one string that arrives in pieces (Sec. 4: the tree
// of Algorithm 1 needs only one open node per level when its words arrive in
// order, so a string of any length is hashed in bounded memory).
//
// The state (IncrState) keeps the bytes of the open level-1 block and, for
// each level j >= 2, the exact sum over the values already produced for the
// open level-j node. Because Eq. (1) is a sum of products, the values need not
// be kept: each is multiplied by its key as soon as it exists.
//
// An append that completes level-1 blocks is one launch. Workgroup w takes
// the w-th segment of 32 blocks (aligned to the string's start) that the
// piece touches: 32 groups of 8 lanes, one block per group, each lane loading
// the 16-byte pieces j, j + 8, ... of its block at once. A block is summed
// exactly over its 8 lanes, folded into a field element (Sec. 6.2 and
// Algorithm 2) and multiplied by its level-2 key; the workgroup adds its 32
// products and, when other segments share the node, adds the reduced sum
// into the node's accumulator with relaxed atomics (no fences: a
// device-scope release writes back the whole L2). The segment that completes
// a node finishes it if all its blocks lie in the piece. Workgroup 0 also
// stages the block that begins in the carried bytes and stores the bytes
// carried to the next piece. The append's tree step (its first and last
// level-2 nodes with the state's open sums, then levels 3 and up, at most
// 1/128 of the level-2 values, one wave per node) needs every workgroup's
// results, so it runs at the start of the next launch on the string:
// workgroup 0 of the next append, or the digest. Level outputs and boundary
// sums alternate between two buffers, so that an append's tree step reads
// what the next append does not write.
//
// A digest pads the open block (end of Sec. 4), hashes it and climbs through
// the open nodes to the root: the do-while of Algorithm 1 stops at the first
// level with a single node. It reads the state without changing it, so more
// pieces may follow.
#include "pmp_device.hpp"
#include "pmp_incr.h"

namespace pmp {

namespace {

constexpr int GL = 8;  // lanes per level-1 block

__device__ __forceinline__ const uint8_t* gp(uint64_t a) {
  return (const uint8_t*)(const __attribute__((address_space(1))) uint8_t*)(uintptr_t)a;
}

__device__ __forceinline__ void to_words(const S32& s, uint64_t* w) {
  w[0] = s.lo;
  w[1] = s.hi;
  w[2] = 0;
}
__device__ __forceinline__ void to_words(const S64& s, uint64_t* w) {
  w[0] = s.w0;
  w[1] = s.w1;
  w[2] = s.w2;
}
__device__ __forceinline__ void from_words(S32& s, const uint64_t* w) {
  s.lo = w[0];
  s.hi = (uint32_t)w[1];
}
__device__ __forceinline__ void from_words(S64& s, const uint64_t* w) {
  s.w0 = w[0];
  s.w1 = w[1];
  s.w2 = (uint32_t)w[2];
}
__device__ __forceinline__ uint4 pack(const Fe& z) {
  return make_uint4((uint32_t)z.lo, (uint32_t)(z.lo >> 32), z.hi, 0u);
}
__device__ __forceinline__ Fe unpack(const uint4& v) {
  Fe z;
  z.lo = (uint64_t)v.x | ((uint64_t)v.y << 32);
  z.hi = v.z;
  return z;
}

// Level j >= 2 node value from its exact sum: add b_j, reduce (Eq. (1)).
template <bool WIDE>
__device__ __forceinline__ Fe finish(typename Tr<WIDE>::Sum S, const typename Tr<WIDE>::key_t* keys, int j) {
  add_word(S, (uint64_t)keys[LMAX * BLOCK + (j - 1)]);
  return reduce(S);
}

// One climb step inside a workgroup, one wave per node: the n_in new
// level-(j-1) values in[], numbered s_in .. s_in + n_in - 1 within their
// level, go into the level-j nodes; complete nodes are written to out[] in
// order, the open one (if any) goes to part[j]. Returns the number written.
template <bool WIDE>
__device__ uint64_t climb(IncrState* st, const typename Tr<WIDE>::key_t* keys, int j, const uint4* in,
                          uint64_t n_in, uint64_t s_in, uint4* out, uint64_t* pend) {
  using S = typename Tr<WIDE>::Sum;
  const uint64_t q0 = s_in / BLOCK, q1 = (s_in + n_in - 1) / BLOCK;
  const bool start_open = s_in % BLOCK != 0;
  const bool end_open = (s_in + n_in) % BLOCK != 0;
  const int lane = (int)(threadIdx.x & 63u), wave = (int)(threadIdx.x >> 6), nw = (int)(blockDim.x >> 6);
  S old;
  from_words(old, st->part[j]);
  const typename Tr<WIDE>::key_t* a = keys + (j - 1) * BLOCK;
  for (uint64_t q = q0 + wave; q <= q1; q += nw) {
    const uint64_t lo = q * BLOCK > s_in ? q * BLOCK : s_in;
    const uint64_t hi = q * BLOCK + BLOCK < s_in + n_in ? q * BLOCK + BLOCK : s_in + n_in;
    S acc;
    zero(acc);
    for (uint64_t c = lo + lane; c < hi; c += 64) mac_fe(acc, a[c % BLOCK], unpack(in[c - s_in]));
    reduce_lanes(acc, 1, 64);
    if (lane == 0) {
      if (q == q0 && start_open) add(acc, old);
      if (hi == q * BLOCK + BLOCK) out[q - q0] = pack(finish<WIDE>(acc, keys, j));
      else to_words(acc, pend);  // the last node, still open
    }
  }
  __syncthreads();  // every reader of part[j] is done
  if (threadIdx.x == 0) {
    uint64_t* p = st->part[j];
    if (end_open) {
      p[0] = pend[0];
      p[1] = pend[1];
      p[2] = pend[2];
    } else {
      p[0] = p[1] = p[2] = 0;
    }
  }
  __syncthreads();  // out[] and part[j] are visible to the whole workgroup
  return (s_in + n_in) / BLOCK - q0;
}

// The tree step of an append (one workgroup, all threads): the level-2 nodes
// that its piece shares with the string before or after it, then the levels
// above 2.
template <bool WIDE>
__device__ void tree_step(IncrState* st, const typename Tr<WIDE>::key_t* keys, const IncrTree& T, uint64_t* pend) {
  using S = typename Tr<WIDE>::Sum;
  if (threadIdx.x == 0) {
    const bool start_open = T.s1 % BLOCK != 0;
    const bool end_open = (T.s1 + T.k) % BLOCK != 0;
    const bool one = T.s1 / BLOCK == (T.s1 + T.k - 1) / BLOCK;
    uint64_t np[3] = {0, 0, 0};
    if (start_open || (one && end_open)) {
      S x;
      from_words(x, T.sums);
      if (start_open) {
        S o;
        from_words(o, st->part[2]);
        add(x, o);
      }
      if (!(one && end_open)) T.za[0] = pack(finish<WIDE>(x, keys, 2));
      else to_words(x, np);
    }
    if (!one && end_open) {
      np[0] = T.sums[4];
      np[1] = T.sums[5];
      np[2] = T.sums[6];
    }
    st->part[2][0] = np[0];
    st->part[2][1] = np[1];
    st->part[2][2] = np[2];
  }
  __syncthreads();

  uint64_t n_in = (T.s1 + T.k) / BLOCK - T.s1 / BLOCK;  // complete level-2 nodes
  uint64_t s_in = T.s1 / BLOCK;                         // level-2 values before that piece
  uint4* in = T.za;
  uint4* out = T.zb;
  for (int lvl = 3; lvl <= LMAX && n_in > 0; ++lvl) {
    const uint64_t n_out = climb<WIDE>(st, keys, lvl, in, n_in, s_in, out, pend);
    s_in /= BLOCK;
    n_in = n_out;
    uint4* t = in;
    in = out;
    out = t;
  }
}

// A pending tree step on its own (before the workspace that holds its values
// is replaced).
template <bool WIDE>
__global__ __launch_bounds__(256) void incr_flush(IncrState* st, const void* keys, IncrTree T) {
  __shared__ uint64_t pend[3];
  tree_step<WIDE>(st, (const typename Tr<WIDE>::key_t*)keys, T, pend);
}

// Add field element v, with weight 1, into a node accumulator whose
// segments in this launch number `target`; the call that brings the weight
// to `target` gets the total (lo + 2^64 hi, at most four field elements) and
// returns the accumulator to zero. Relaxed device-scope atomics only: the
// completing call's own atomics come after every other contribution in each
// word's order (the second atomic of a call is issued after the first has
// returned), so no fence is needed.
template <bool WIDE>
__device__ __forceinline__ bool add_to_node(Slot* sl, const Fe& v, uint32_t target, uint64_t* lo, uint32_t* hi) {
  if constexpr (!WIDE) {
    constexpr uint64_t M56 = (1ull << 56) - 1;
    const uint64_t x = v.lo | ((uint64_t)v.hi << 32);
    const uint64_t old = __hip_atomic_fetch_add(&sl->w0, (1ull << 56) + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((uint32_t)(old >> 56) + 1 != target) return false;
    __hip_atomic_store(&sl->w0, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *lo = (old & M56) + x;
    *hi = 0;
    return true;
  } else {
    const uint64_t o0 = __hip_atomic_fetch_add(&sl->w0, v.lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t cy = o0 + v.lo < o0 ? 1u : 0u;
    const uint64_t o1 =
        __hip_atomic_fetch_add(&sl->w1, (1ull << 32) | (uint64_t)(v.hi + cy), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((uint32_t)(o1 >> 32) + 1 != target) return false;
    *lo = __hip_atomic_exchange(&sl->w0, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&sl->w1, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *hi = (uint32_t)o1 + v.hi + cy;
    return true;
  }
}

template <bool WIDE>
__global__ __launch_bounds__(256) void incr_blocks(IncrArgs A) {
  using T = Tr<WIDE>;
  using S = typename T::Sum;
  using K = typename T::key_t;
  constexpr int W = T::W;
  constexpr int C = BLOCK * W;        // bytes per level-1 block
  constexpr int NG = C / (16 * GL);   // 16-byte pieces per lane and block
  constexpr int KPG = 16 / W;         // words per 16-byte piece
  constexpr int SPN = BLOCK / INCR_SEG;  // segments per level-2 node
  static_assert(256 / GL == INCR_SEG, "one block per group of lanes");
  __shared__ uint32_t stg[C / 4];     // the block that begins in the carried bytes
  __shared__ uint64_t red[INCR_SEG][3];
  __shared__ uint64_t pend[3];

  const K* keys = (const K*)A.keys;
  const int tid = (int)threadIdx.x, g = tid / GL, j = tid % GL;
  if (blockIdx.x == 0 && A.pending) tree_step<WIDE>(A.st, keys, A.prev, pend);
  const uint64_t sg0 = A.s1 / INCR_SEG, sg1 = (A.s1 + A.k - 1) / INCR_SEG;
  const uint64_t sg = sg0 + blockIdx.x;  // this workgroup's segment
  const uint64_t c = sg * INCR_SEG + g;  // this group's block
  const bool act = c >= A.s1 && c < A.s1 + A.k;
  const uint64_t i = c - A.s1;           // block index within the piece
  const bool staged = blockIdx.x == 0 && A.t > 0;

  if (staged) {  // carried bytes, then the piece's first bytes
    uint8_t* s8 = (uint8_t*)stg;
    const uint8_t* cb = (const uint8_t*)A.st->carry;
    for (int p = tid; p < C; p += 256) s8[p] = p < (int)A.t ? cb[p] : A.piece[p - (int)A.t];
    __syncthreads();
  }
  if (blockIdx.x == 0) {  // the bytes carried to the next piece (the old ones are staged)
    uint8_t* cb = (uint8_t*)A.st->carry;
    const uint8_t* src = A.piece + (A.n - (int64_t)A.r_new);
    for (uint32_t p = (uint32_t)tid; p < A.r_new; p += 256) cb[p] = src[p];
  }

  // this lane's pieces of the block: all loads first
  uint32_t d[NG][5];
  const uint64_t base = (uint64_t)(uintptr_t)A.piece - A.t;  // every block shares its misalignment
  const uint32_t sh = (uint32_t)(base & 3u);
  uint32_t s_eff = sh;
  if (act) {
    if (staged && i == 0) {
#pragma unroll
      for (int u = 0; u < NG; ++u) {
        const uint32_t* p = stg + 4 * (GL * u + j);
#pragma unroll
        for (int v = 0; v < 4; ++v) d[u][v] = p[v];
        d[u][4] = 0;
      }
      s_eff = 0;
    } else {
      // the aligned dwords that hold the block; the one past its end only
      // when the block is misaligned (it then holds the block's last bytes)
      const uint64_t a4 = (base + i * C) & ~3ull;
#pragma unroll
      for (int u = 0; u < NG; ++u) {
        const uint8_t* p = gp(a4 + 16 * (uint64_t)(GL * u + j));
        Q x = load16(p);
#pragma unroll
        for (int v = 0; v < 4; ++v) d[u][v] = x.d[v];
        d[u][4] = sh ? *(const uint32_t*)__builtin_assume_aligned(p + 16, 4) : 0u;
      }
    }
  }
  // level-1 keys of this lane's pieces: word KPG (GL u + j) + v
  K kk[NG * KPG];
#pragma unroll
  for (int u = 0; u < NG; ++u)
#pragma unroll
    for (int v = 0; v < KPG; ++v) kk[KPG * u + v] = keys[KPG * (GL * u + j) + v];

  S node;
  zero(node);
  if (act) {
    S s;
    if constexpr (WIDE) {
      P64 p;
      zero(p);
#pragma unroll
      for (int u = 0; u < NG; ++u) {
        uint32_t x[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) x[v] = align_bytes(d[u][v + 1], d[u][v], s_eff);
        mac64_vv(p, kk[2 * u], x[0], x[1]);
        mac64_vv(p, kk[2 * u + 1], x[2], x[3]);
      }
      s = collapse(p);
    } else {
      zero(s);
#pragma unroll
      for (int u = 0; u < NG; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) mac_vv(s.lo, s.hi, kk[4 * u + v], align_bytes(d[u][v + 1], d[u][v], s_eff));
    }
    group_sum<GL>(s);  // the block's exact sum, in every lane of the group
    add_word(s, (uint64_t)keys[LMAX * BLOCK]);
    mac_fe(node, keys[BLOCK + c % BLOCK], reduce(s));
  }
  if (j == 0) to_words(node, red[g]);
  __syncthreads();
  if (tid != 0) return;

  S tot;
  zero(tot);
  for (int h = 0; h < INCR_SEG; ++h) {
    S x;
    from_words(x, red[h]);
    add(tot, x);
  }
  // the segments of this node that the piece touches
  const uint64_t q = sg / SPN, q0 = A.s1 / BLOCK, slot = q - q0;
  const uint64_t f = sg0 > q * SPN ? sg0 : q * SPN, l = sg1 < q * SPN + SPN - 1 ? sg1 : q * SPN + SPN - 1;
  const uint32_t nseg = (uint32_t)(l - f + 1);
  if (nseg > 1) {
    // this segment's share of the node, reduced (a sum of at most 32
    // products, well inside the fold's range)
    uint64_t lo;
    uint32_t hi;
    if (!add_to_node<WIDE>(A.slots + slot, reduce(tot), nseg, &lo, &hi)) return;
    zero(tot);
    if constexpr (WIDE) {
      tot.w0 = lo;
      tot.w1 = hi;
    } else {
      tot.lo = lo;
    }
  }
  const uint64_t c_lo = q * BLOCK > A.s1 ? q * BLOCK : A.s1;
  const uint64_t c_hi = q * BLOCK + BLOCK < A.s1 + A.k ? q * BLOCK + BLOCK : A.s1 + A.k;
  if (c_lo == q * BLOCK && c_hi == q * BLOCK + BLOCK) A.za[slot] = pack(finish<WIDE>(tot, keys, 2));
  else to_words(tot, A.sums + 4 * (slot == 0 ? 0 : 1));  // first or last node, open
}

// An append that completes no block: its bytes join the carried ones.
__global__ void incr_carry(IncrState* st, uint32_t t, const uint8_t* piece, int64_t n) {
  uint8_t* cb = (uint8_t*)st->carry;
  for (int64_t p = threadIdx.x; p < n; p += blockDim.x) cb[t + p] = piece[p];
}

// Digest: the pending tree step (all threads), then one wave: lane l forms
// words 2l and 2l + 1 of the padded open block (t carried bytes, a byte 0x01,
// zeros), then the climb. nodes[j] is the number of level-j nodes of the
// whole string (level 1: blocks).
struct Nodes {
  uint64_t n[LMAX + 1];
};
template <bool WIDE>
__global__ __launch_bounds__(256) void incr_digest(IncrState* st, uint32_t t, Nodes N, const void* keysv, void* out,
                                                   uint32_t flags, uint32_t pending, IncrTree prev) {
  using T = Tr<WIDE>;
  using S = typename T::Sum;
  using K = typename T::key_t;
  __shared__ uint64_t pend[3];
  const K* keys = (const K*)keysv;
  if (pending) tree_step<WIDE>(st, keys, prev, pend);  // the last append's levels >= 2
  if (threadIdx.x >= 64) return;
  const int lane = (int)threadIdx.x;
  S s;
  zero(s);
  if constexpr (WIDE) {
    P64 p;
    zero(p);
    for (int v = 0; v < 2; ++v) {
      const int w = 2 * lane + v;
      uint32_t x0 = st->carry[2 * w], x1 = st->carry[2 * w + 1];
      tail_word64(x0, x1, (int64_t)t - 8 * w);
      mac64_vv(p, keys[w], x0, x1);
    }
    s = collapse(p);
  } else {
    for (int v = 0; v < 2; ++v) {
      const int w = 2 * lane + v;
      mac_vv(s.lo, s.hi, keys[w], tail_word32(st->carry[w], (int64_t)t - 4 * w));
    }
  }
  reduce_lanes(s, 1, 64);
  if (lane != 0) return;
  add_word(s, (uint64_t)keys[LMAX * BLOCK]);
  Fe z = reduce(s);
  for (int j = 1; j < LMAX && N.n[j] > 1; ++j) {
    S acc;
    from_words(acc, st->part[j + 1]);
    mac_fe(acc, keys[j * BLOCK + (N.n[j] - 1) % BLOCK], z);
    z = finish<WIDE>(acc, keys, j + 1);
  }
  store_value<WIDE>(out, flags, 0, z);
}

__global__ void incr_reset(IncrState* st) {
  uint64_t* w = (uint64_t*)st;
  for (uint32_t i = threadIdx.x; i < sizeof(IncrState) / 8; i += blockDim.x) w[i] = 0;
}

}  // namespace

hipError_t launch_incr_append(int wide, const IncrArgs& a, hipStream_t s) {
  if (wide) hipLaunchKernelGGL(incr_blocks<true>, dim3(a.nwg), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(incr_blocks<false>, dim3(a.nwg), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_incr_flush(int wide, IncrState* st, const void* keys, const IncrTree& t, hipStream_t s) {
  if (wide) hipLaunchKernelGGL(incr_flush<true>, dim3(1), dim3(256), 0, s, st, keys, t);
  else hipLaunchKernelGGL(incr_flush<false>, dim3(1), dim3(256), 0, s, st, keys, t);
  return hipGetLastError();
}

hipError_t launch_incr_carry(IncrState* st, uint32_t t, const uint8_t* piece, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(incr_carry, dim3(1), dim3(256), 0, s, st, t, piece, n);
  return hipGetLastError();
}

hipError_t launch_incr_digest(int wide, IncrState* st, uint32_t t, const uint64_t* nodes, const void* keys,
                              void* out, uint32_t flags, uint32_t pending, const IncrTree& prev, hipStream_t s) {
  Nodes N;
  for (int j = 0; j <= LMAX; ++j) N.n[j] = nodes[j];
  if (wide)
    hipLaunchKernelGGL(incr_digest<true>, dim3(1), dim3(256), 0, s, st, t, N, keys, out, flags, pending, prev);
  else
    hipLaunchKernelGGL(incr_digest<false>, dim3(1), dim3(256), 0, s, st, t, N, keys, out, flags, pending, prev);
  return hipGetLastError();
}

hipError_t launch_incr_reset(IncrState* st, hipStream_t s) {
  hipLaunchKernelGGL(incr_reset, dim3(1), dim3(256), 0, s, st);
  return hipGetLastError();
}

}  // namespace pmp
