/*
 * Test oracle for the PM+ hash families (PM+32, PM+64) of Ivanchykhin,
 * Ignatchenko and Lemire, "Regular and almost universal hashing: an efficient
 * implementation" (arXiv 1609.09840).
 *
 * THIS IS TEST INFRASTRUCTURE. It is a plain, slow CPU implementation written
 * from the paper's definitions so that the GPU library can be checked against
 * it. Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it. It shares no code, header or constant table with the GPU path.
 *
 * Arithmetic is exact: unsigned __int128 and the C remainder operator. The
 * paper's fast three-word fold (Sec. 6.2) and its Algorithm 2 are deliberately
 * NOT used here; this file computes every residue with a plain `%`.
 *
 * What is computed (citations are to the paper):
 *  - Field: p = 2^32 + 15 (PM+32) or p = 2^64 + 13 (PM+64), the smallest primes
 *    above 2^32 and 2^64 (Table "smallestprimes", Sec. 5).
 *  - Compression function, Eq. (1): f_j(s) = (b_j + sum_i a_{j,i} s_i) mod p,
 *    with b_j in [0, 2^n) and a_{j,i} in (0, p - kappa), kappa = 28 / 24
 *    (Table "parameters", Sec. 6.1). m = 128 words per block, at most L = 8
 *    levels.
 *  - Tree, Algorithm 1 (Sec. 4): append the value 1, then repeatedly zero-pad
 *    to a multiple of m and replace each block of m values by f_j of it, with
 *    j = 1 for the leaves, until one value remains.
 *  - Byte strings (end of Sec. 4): words are n-bit machine words; the appended
 *    1 is a byte 0x01 followed by zero bytes up to the next word boundary.
 *  - Output (Sec. 5, after Lemma 9): h mod 2^n, then the avalanche mixer of
 *    Sec. 7 (constants as printed there).
 *
 * Readings of the paper taken here (each is listed with its reason in the
 * design notes of the repository):
 *  R1 words are little-endian; R2 the 0x01 byte is always appended, so a
 *  length that is a multiple of the word size gains a whole word equal to 1;
 *  R3 leaves always use the level-1 keys (Algorithm 1 and Fig. 1); R4 at
 *  least one level is applied, even when the padded string is a single word;
 *  R5 key table layout a[8][128] (row-major, level-major) then b[8], drawn
 *  from splitmix64 with rejection of out-of-range a candidates.
 *
 * Parity status of each function is given in its comment. Pins live in the
 * CPU test suite (tests/test_oracle_*.py).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

typedef unsigned __int128 u128;

#define OR_MIXED 0 /* mixer(h mod 2^n)   */
#define OR_RAW 1   /* h mod 2^n          */
#define OR_FIELD 2 /* h in [0, p)        */

#define OR_OK 0
#define OR_E_ARG -1
#define OR_E_KEY -2
#define OR_E_LONG -3
#define OR_E_MEM -4

/* ---------------------------------------------------------------------- */
/* splitmix64 (Steele, Lea and Flood, OOPSLA 2014; the "mix64" finalizer of
 * the published SplittableRandom): state advances by the golden gamma and
 * each output is the finalizer of the new state. Pinned by its published
 * first output for seed 0. */
static uint64_t sm64_next(uint64_t* state) {
  uint64_t z = (*state += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

void oracle_splitmix64_stream(uint64_t seed, uint64_t* out, uint64_t n) {
  uint64_t s = seed;
  for (uint64_t i = 0; i < n; ++i) out[i] = sm64_next(&s);
}

/* Key table (reading R5). a candidates outside [1, p - kappa - 1] are
 * redrawn; the upper end p - kappa - 1 equals 2^32 - 14 (PM+32) and
 * 2^64 - 12 (PM+64), the open interval (0, p - kappa) of Sec. 6.1. */
int oracle_expand_keys32(uint64_t seed, uint32_t* keys) {
  uint64_t s = seed;
  const uint64_t amax = 4294967296ULL + 15 - 28 - 1; /* 2^32 - 14 */
  for (int i = 0; i < 8 * 128; ++i) {
    uint64_t c;
    do { c = sm64_next(&s) >> 32; } while (c < 1 || c > amax);
    keys[i] = (uint32_t)c;
  }
  for (int j = 0; j < 8; ++j) keys[8 * 128 + j] = (uint32_t)(sm64_next(&s) >> 32);
  return OR_OK;
}

int oracle_expand_keys64(uint64_t seed, uint64_t* keys) {
  uint64_t s = seed;
  const u128 amax = ((u128)1 << 64) + 13 - 24 - 1; /* 2^64 - 12 */
  for (int i = 0; i < 8 * 128; ++i) {
    uint64_t c;
    do { c = sm64_next(&s); } while (c < 1 || (u128)c > amax);
    keys[i] = c;
  }
  for (int j = 0; j < 8; ++j) keys[8 * 128 + j] = sm64_next(&s);
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Avalanche mixers, Sec. 7, n-bit unsigned arithmetic with wraparound. */
uint32_t oracle_mix32(uint32_t z) {
  z = z ^ (z >> 13);
  z = z * 0xab3be54fu;
  z = z ^ (z >> 16);
  return z;
}
uint64_t oracle_mix64(uint64_t z) {
  z = z ^ (z >> 33);
  z = z * 0xc4ceb9fe1a85ec53ULL;
  z = z ^ (z >> 33);
  return z;
}

/* ---------------------------------------------------------------------- */
/* Algorithm 1 over a word string sigma that already carries the appended 1
 * (reading R4: the loop body runs at least once). a is the level-major key
 * matrix a[lmax][m], b the per-level constants. The working string is held
 * as exact field elements. Returns the number of levels applied, or an
 * error. Keys are checked against the range of Eq. (1) with kappa as given. */
static int tree_generic(u128* sig, uint64_t len, int m, int lmax, u128 p, u128 amax,
                        const void* akeys, const void* bkeys, int wide, u128* h) {
  if (m < 2 || lmax < 1 || len < 1) return OR_E_ARG;
  u128* cur = (u128*)malloc((size_t)len * sizeof(u128));
  if (!cur) return OR_E_MEM;
  memcpy(cur, sig, (size_t)len * sizeof(u128));
  int j = 0;
  do {
    if (j >= lmax) { free(cur); return OR_E_LONG; }
    uint64_t blocks = (len + (uint64_t)m - 1) / (uint64_t)m;
    u128* next = (u128*)malloc((size_t)blocks * sizeof(u128));
    if (!next) { free(cur); return OR_E_MEM; }
    for (uint64_t c = 0; c < blocks; ++c) {
      u128 b = wide ? (u128)((const uint64_t*)bkeys)[j] : (u128)((const uint32_t*)bkeys)[j];
      u128 acc = b % p;
      for (int i = 0; i < m; ++i) {
        uint64_t idx = c * (uint64_t)m + (uint64_t)i;
        u128 s = idx < len ? cur[idx] : 0; /* zero padding of the last block */
        u128 a = wide ? (u128)((const uint64_t*)akeys)[(uint64_t)j * m + i]
                      : (u128)((const uint32_t*)akeys)[(uint64_t)j * m + i];
        if (a > amax) { free(cur); free(next); return OR_E_KEY; }
        /* a <= p - kappa - 1 and s <= p - 1, so a * s < 2^(2n) <= 2^128. */
        acc = (acc + (a * s) % p) % p;
      }
      next[c] = acc;
    }
    free(cur);
    cur = next;
    len = blocks;
    ++j;
  } while (len > 1);
  *h = cur[0];
  free(cur);
  return j;
}

/* Word-level entry points with a free block length m and level cap lmax,
 * used to check the tree shape against the paper's worked example (Fig. 1,
 * m = 4). sigma[] is the word string after the appended 1; field elements
 * are returned. */
int oracle_pm32_words(const uint64_t* sigma, uint64_t len, const uint32_t* a, const uint32_t* b,
                      int m, int lmax, uint64_t* h_out) {
  u128* sig = (u128*)malloc((size_t)(len ? len : 1) * sizeof(u128));
  if (!sig) return OR_E_MEM;
  for (uint64_t i = 0; i < len; ++i) sig[i] = sigma[i];
  u128 p = ((u128)1 << 32) + 15, h = 0;
  int r = tree_generic(sig, len, m, lmax, p, p - 28 - 1, a, b, 0, &h);
  free(sig);
  if (r > 0) *h_out = (uint64_t)h;
  return r;
}

int oracle_pm64_words(const uint64_t* sigma, uint64_t len, const uint64_t* a, const uint64_t* b,
                      int m, int lmax, uint64_t* h_out /* [lo, hi] */) {
  u128* sig = (u128*)malloc((size_t)(len ? len : 1) * sizeof(u128));
  if (!sig) return OR_E_MEM;
  for (uint64_t i = 0; i < len; ++i) sig[i] = sigma[i];
  u128 p = ((u128)1 << 64) + 13, h = 0;
  int r = tree_generic(sig, len, m, lmax, p, p - 24 - 1, a, b, 1, &h);
  free(sig);
  if (r > 0) {
    h_out[0] = (uint64_t)h;
    h_out[1] = (uint64_t)(h >> 64);
  }
  return r;
}

/* ---------------------------------------------------------------------- */
/* Byte string -> padded word string (end of Sec. 4, readings R1, R2):
 * y = bytes || 0x01 || zeros up to a multiple of W bytes; word i is the
 * little-endian value of y[W i .. W i + W). N' = floor(len / W) + 1. */
static u128* pad_words(const uint8_t* bytes, uint64_t len, int W, uint64_t* nwords) {
  uint64_t n = len / (uint64_t)W + 1;
  u128* sig = (u128*)calloc((size_t)n, sizeof(u128));
  if (!sig) return NULL;
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t v = 0;
    for (int t = 0; t < W; ++t) {
      uint64_t pos = i * (uint64_t)W + (uint64_t)t;
      uint64_t byte = pos < len ? bytes[pos] : (pos == len ? 1u : 0u);
      v |= byte << (8 * t);
    }
    sig[i] = v;
  }
  *nwords = n;
  return sig;
}

/* PM+32 of one byte string with the 1032-entry key table (a[8][128], b[8]).
 * mode: OR_MIXED -> out[0] = mix32(h mod 2^32); OR_RAW -> h mod 2^32;
 * OR_FIELD -> out[0] = h (< 2^32 + 15). Returns levels used or an error. */
int oracle_pm32(const uint8_t* bytes, uint64_t len, const uint32_t* keys, int mode, uint64_t* out) {
  uint64_t n = 0;
  u128* sig = pad_words(bytes, len, 4, &n);
  if (!sig) return OR_E_MEM;
  u128 p = ((u128)1 << 32) + 15, h = 0;
  int r = tree_generic(sig, n, 128, 8, p, p - 28 - 1, keys, keys + 8 * 128, 0, &h);
  free(sig);
  if (r < 0) return r;
  uint32_t low = (uint32_t)h; /* h mod 2^32 */
  if (mode == OR_FIELD) out[0] = (uint64_t)h;
  else if (mode == OR_RAW) out[0] = low;
  else out[0] = oracle_mix32(low);
  return r;
}

/* PM+64 of one byte string. OR_FIELD -> out[0..1] = (h mod 2^64, h >> 64). */
int oracle_pm64(const uint8_t* bytes, uint64_t len, const uint64_t* keys, int mode, uint64_t* out) {
  uint64_t n = 0;
  u128* sig = pad_words(bytes, len, 8, &n);
  if (!sig) return OR_E_MEM;
  u128 p = ((u128)1 << 64) + 13, h = 0;
  int r = tree_generic(sig, n, 128, 8, p, p - 24 - 1, keys, keys + 8 * 128, 1, &h);
  free(sig);
  if (r < 0) return r;
  uint64_t low = (uint64_t)h; /* h mod 2^64 */
  if (mode == OR_FIELD) {
    out[0] = low;
    out[1] = (uint64_t)(h >> 64);
  } else if (mode == OR_RAW) out[0] = low;
  else out[0] = oracle_mix64(low);
  return r;
}

/* ---------------------------------------------------------------------- */
/* Batch over a concatenated buffer with CSR offsets: string i is
 * buf[offsets[i] .. offsets[i+1]). Output stride: 1 word per string, or 2
 * for PM+64 field output. Strings are split over nthreads plain threads. */
typedef struct {
  const uint8_t* buf;
  const int64_t* off;
  int64_t lo, hi;
  const void* keys;
  int wide, mode;
  uint64_t* out;
  int err;
} job_t;

static void* run_job(void* arg) {
  job_t* jb = (job_t*)arg;
  int stride = (jb->wide && jb->mode == OR_FIELD) ? 2 : 1;
  for (int64_t i = jb->lo; i < jb->hi; ++i) {
    const uint8_t* s = jb->buf + jb->off[i];
    uint64_t len = (uint64_t)(jb->off[i + 1] - jb->off[i]);
    int r = jb->wide ? oracle_pm64(s, len, (const uint64_t*)jb->keys, jb->mode, jb->out + stride * i)
                     : oracle_pm32(s, len, (const uint32_t*)jb->keys, jb->mode, jb->out + stride * i);
    if (r < 0) { jb->err = r; return NULL; }
  }
  return NULL;
}

int oracle_batch(int wide, const uint8_t* buf, const int64_t* offsets, int64_t count, const void* keys,
                 int mode, uint64_t* out, int nthreads) {
  if (count < 0 || nthreads < 1) return OR_E_ARG;
  for (int64_t i = 0; i < count; ++i)
    if (offsets[i + 1] < offsets[i] || offsets[i] < 0) return OR_E_ARG;
  if (nthreads > 256) nthreads = 256;
  job_t jobs[256];
  pthread_t th[256];
  /* balance by bytes: thread t takes strings whose start lies in its share */
  int64_t total = count ? offsets[count] - offsets[0] : 0;
  int64_t i0 = 0;
  for (int t = 0; t < nthreads; ++t) {
    int64_t target = offsets[0] + (total * (t + 1)) / nthreads;
    int64_t i1 = i0;
    if (t == nthreads - 1) i1 = count;
    else while (i1 < count && offsets[i1] < target) ++i1;
    jobs[t] = (job_t){buf, offsets, i0, i1, keys, wide, mode, out, 0};
    i0 = i1;
  }
  for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, run_job, &jobs[t]);
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  for (int t = 0; t < nthreads; ++t)
    if (jobs[t].err) return jobs[t].err;
  return OR_OK;
}
