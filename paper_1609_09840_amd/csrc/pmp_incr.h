// Structures of the incremental-hashing kernels shared with the host side
// of libpmp (not part of the public ABI).
#pragma once
#include "pmp_batch.h"

namespace pmp {

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

// The tree step of an append that completed blocks s1 .. s1 + k - 1: its
// first and last level-2 nodes with the open sums, and the levels above 2.
// It runs at the start of the next launch on the string (next append or
// digest), so an append is one launch.
struct IncrTree {
  uint64_t s1;
  uint64_t k;
  uint4* za;        // that append's level-2 values, then level outputs (ping-pong with zb)
  uint4* zb;
  uint64_t* sums;   // its first and last level-2 node sums, when open (2 x 4 words)
};

// One append that completes at least one level-1 block. The piece's bytes
// follow the t carried bytes; blocks s1 .. s1 + k - 1 (numbered from the
// string's start) are completed by it; r_new bytes are carried afterwards.
// Workgroup w takes segment s1 / 32 + w (32 blocks, a quarter of a level-2
// node). Per level-2 node touched (numbered from node s1 / 128): an
// accumulator Slot for its segments (0 between launches). Workgroup 0 first
// runs the previous append's tree step when `pending`.
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
  uint32_t pending; // prev holds a tree step still to run
  IncrTree prev;
};

}  // namespace pmp
